"""GPU parity of the PTA slow-time step with junction nodes
(dd_pta_step_junction_nodes) against the oracle's driver (oracle/pta.py with
oracle/junction_nodes.py): the same decisions (fast steps, convergence,
jumps, re-run chunks), the same topology, junction-node state and fast
clocks bit for bit, and averages, rates and positions within 1e-10 (FP64).
Volumes: mobile loops beside forests of sessile lines
(workloads.junction_forest) with slots for 4 junctions each."""
import numpy as np
import pytest
import torch

from oracle import junction_nodes as JN
from oracle import pta
from paper_2005_02498_amd import workloads as W
import paper_2005_02498_amd as dd

from gpu_util import MAT, batch_dev

pytestmark = pytest.mark.gpu

DELTA = 1e-8
K = 4
TOL = 1e-10


def _case(seeds=(1, 2, 3)):
    insts = [W.with_junction_slots(W.junction_forest(s), K) for s in seeds]
    rates = np.array([[0, 0, 4e15, 0, 0, 0], [0, 0, 0, 0, 0, 3e15], [1e15, 0, 3e15, 0, 0, 0]], float)[:len(insts)]
    fr = np.random.default_rng(9).uniform(0.0, 1.0, (len(insts), 3))
    return insts, rates, fr


def _run(insts, rates, fr, t, kw, fast0, rc=10.0, a=3 * W.DT, lmin=2.0):
    bt = W.pack(insts)
    d = batch_dev(bt)
    dev = d["x"].device
    st = dd.junction_node_state(int(bt.node_off[-1]), int(bt.seg_off[-1]), bt.n_inst, dev)
    fast = np.array(fast0, np.int64)
    P = dd.PTAParams(dt=W.DT, delta=DELTA, **kw)
    J = {"state": st, "fractions": torch.tensor(fr, device=dev), "capture_radius": rc, "max_break_time": a,
         "min_length": lmin, "n_slots": K, "fast_steps": fast}
    got = dd.dd_pta_step_junction_nodes(bt.node_off, bt.seg_off, d["x"], d["seg_nodes"], d["burgers"], d["normal"],
                                        d["pinned"], d["volume"], rates, t, P, MAT, J, 2, dd.DD_FP64)
    torch.cuda.synchronize()
    g = {k: v.cpu().numpy() for k, v in d.items() if torch.is_tensor(v)}
    g.update({k: v.cpu().numpy() for k, v in st.items()})
    OP = pta.PTAParams(dt=W.DT, delta=DELTA, chunk=kw["chunk_steps"], max_chunks=kw["max_chunks"],
                       lpdot_max=kw.get("lpdot_max", 0.05), max_jumps=kw.get("max_jumps", 2))
    Pj = JN.Params(rc, a, lmin, K)
    n_formed = 0
    for i, inst in enumerate(insts):
        jn = pta.JunctionNodes(Pj, JN.new_state(inst.n_nodes, inst.n_segs, fr[i]), np.array(inst.seg_nodes),
                               np.array(inst.burgers), np.array(inst.normal), int(fast0[i]))
        ref = pta.pta_step(inst, t[i], rates[i], W.material(), 2, OP, jn)
        R = ref["jn"]
        print(f"volume {i}: steps {got['steps_a'][i]}/{got['steps_b'][i]} (oracle {ref['steps_a']}/{ref['steps_b']}), "
              f"jumps {got['jumps'][i]}, rerun {got['rerun_chunks'][i]}, junctions {R.state['count']}")
        for k in ("steps_a", "steps_b", "jumps", "rerun_chunks", "conv_a", "conv_b"):
            assert got[k][i] == ref[k], k
        n0, n1 = bt.node_off[i], bt.node_off[i + 1]
        s0, s1 = bt.seg_off[i], bt.seg_off[i + 1]
        assert np.array_equal(g["seg_nodes"][:, s0:s1], R.seg_nodes), f"volume {i}: topology"
        assert np.array_equal(g["burgers"][:, s0:s1], R.burgers) and np.array_equal(g["normal"][:, s0:s1], R.normal)
        ses = np.where(R.state["ses"] >= 0, R.state["ses"] + s0, -1)
        assert np.array_equal(g["ses"][n0:n1], ses), f"volume {i}: junction nodes"
        act = R.state["ses"] >= 0
        assert np.array_equal(g["release"][n0:n1][act], R.state["release"][act])
        assert np.array_equal(g["ignore"][s0:s1].astype(bool), R.state["ignore"])
        kept = R.state["ignore"]
        assert np.array_equal(g["point"][:, s0:s1][:, kept], R.state["point"][:, kept])
        assert g["count"][i] == R.state["count"] and g["missed"][i] == R.state["missed"]
        assert fast[i] == R.fast
        for k in ("g_a", "g_b", "lp_a", "lp_b"):
            r = np.asarray(ref[k])
            assert np.abs(got[k][i] - r).max() <= TOL * max(np.abs(r).max(), 1e-300), k
        for k in ("rho_a", "rho_b", "h"):
            assert got[k][i] == pytest.approx(ref[k], rel=TOL, abs=1e-300), k
        disp_g, disp_o = g["x"][:, n0:n1] - inst.x, ref["x"] - inst.x
        assert np.abs(disp_g - disp_o).max() <= TOL * max(np.abs(disp_o).max(), 1e-300)
        n_formed += R.state["count"]
    return got, n_formed


def test_pta_junction_nodes_plain():
    insts, rates, fr = _case()
    got, n = _run(insts, rates, fr, [5e-8] * 3, dict(chunk_steps=2, max_chunks=3, lpdot_max=np.inf), [0, 11, 3])
    assert n >= 3


def test_pta_junction_nodes_jumps_and_rerun():
    """t < delta/2: the t - delta load is the larger, so step 5 continues the
    t - delta run from its own end (topology and node state restored around
    it); every check a jump, one restart: the saved states of steps 1 and 2
    are taken and put back several times."""
    insts, rates, fr = _case((4, 5))
    got, n = _run(insts, rates, fr, [0.2 * DELTA] * 2,
                  dict(chunk_steps=2, max_chunks=3, lpdot_max=0.0, max_jumps=1), [5, 0])
    assert (got["jumps"] == 1).all() and (got["rerun_chunks"] > 0).any()
    assert n >= 2
