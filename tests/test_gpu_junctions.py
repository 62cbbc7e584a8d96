"""GPU parity of bursts with junctions (dd_burst_batch_junctions) against the
oracle (oracle/junctions.py): the same captures, holds and releases (state
arrays equal, release times bit for bit) and the same trajectories and
slip rates to FP64 tolerance."""
import numpy as np
import pytest
import torch

from oracle import junctions as OJ
from paper_2005_02498_amd import workloads as W
import paper_2005_02498_amd as dd

from gpu_util import MAT, batch_dev, normwise

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def _state_dev(nn):
    return {"junction": torch.full((nn,), -1, dtype=torch.int32, device=DEV),
            "release": torch.zeros(nn, dtype=torch.float64, device=DEV),
            "ignore": torch.full((nn,), -1, dtype=torch.int32, device=DEV),
            "count": torch.zeros(nn, dtype=torch.int32, device=DEV)}


def _run(insts, n_steps, r_c, a, t0, fractions, calls=1):
    bt = W.pack(insts)
    d = batch_dev(bt)
    st = _state_dev(bt.node_off[-1])
    fr = torch.tensor(fractions, dtype=torch.float64, device=DEV)
    rates = []
    for c in range(calls):
        r = dd.dd_burst_batch_junctions(bt.node_off, bt.seg_off, d["x"], d["seg_nodes"], d["burgers"],
                                        d["normal"], d["pinned"], d["sigma_app"], d["volume"], MAT, st, fr,
                                        r_c, a, t0 + c * n_steps * W.DT, 2, dd.DD_FP64, 20.0, n_steps, W.DT)
        rates.append(r.cpu().numpy())
    torch.cuda.synchronize()
    # oracle, instance by instance, with the same calls
    for i, inst in enumerate(insts):
        n0, n1 = bt.node_off[i], bt.node_off[i + 1]
        s0 = bt.seg_off[i]
        ost = OJ.new_state(inst.n_nodes)
        x = inst
        for c in range(calls):
            xo, ro = OJ.burst(x, MAT, 2, n_steps, W.DT, r_c, a, t0 + c * n_steps * W.DT, fractions[n0:n1], ost)
            x = W.Instance(xo, inst.seg_nodes, inst.burgers, inst.normal, inst.pinned, inst.sigma_app, inst.volume, {})
            assert np.abs(rates[c][i] - ro).max() <= 1e-10 * max(np.abs(ro).max(), 1e-300)
        xg = d["x"].cpu().numpy()[:, n0:n1]
        assert normwise(xg - inst.x, xo - inst.x) < 1e-10
        jg = st["junction"].cpu().numpy()[n0:n1].astype(np.int64)
        ig = st["ignore"].cpu().numpy()[n0:n1].astype(np.int64)
        jo, io = ost["junction"], ost["ignore"]
        assert np.array_equal(np.where(jg >= 0, jg - s0, -1), jo)
        assert np.array_equal(np.where(ig >= 0, ig - s0, -1), io)
        assert np.array_equal(st["count"].cpu().numpy()[n0:n1], ost["count"])
        held = jo >= 0
        assert np.array_equal(st["release"].cpu().numpy()[n0:n1][held], ost["release"][held])
        yield i, ost


def _pair_of_loops():
    ang = np.arange(8) * np.pi / 4
    mob = np.stack([50 * np.cos(ang), 50 * np.sin(ang), np.zeros(8)])
    ses = np.array([[53.0, 53.0, 53.0, 53.0], [0.0, 0.0, 40.0, 40.0], [-20.0, 20.0, 20.0, -20.0]])
    x = np.concatenate([mob, ses], axis=1)
    sn = np.array([list(range(8)) + [8, 9, 10, 11], [1, 2, 3, 4, 5, 6, 7, 0, 9, 10, 11, 8]], np.int32)
    b = np.zeros((3, 12)); b[0, :8] = 1.0; b[1, 8:] = 1.0
    nrm = np.zeros((3, 12)); nrm[2, :8] = 1.0; nrm[0, 8:] = 1.0
    pinned = np.zeros(12, np.uint8); pinned[8:] = 1
    return W.Instance(x, sn, b, nrm, pinned, np.array([0, 0, 0, 0, 80e6, 0.0]), 2000.0 ** 3, {})


def test_hand_case_capture_hold_release():
    inst = _pair_of_loops()
    fr = np.full((12, 3), 0.9)
    fr[0, 0] = 0.5
    results = list(_run([inst], 8, 5.0, 5 * W.DT, 1e-9, fr))
    _, ost = results[0]
    assert ost["count"][0] == 1 and ost["junction"][0] == -1 and ost["ignore"][0] == 8


def _min_capture_distance(inst):
    ses = [s for s in range(inst.seg_nodes.shape[1])
           if inst.pinned[inst.seg_nodes[0, s]] and inst.pinned[inst.seg_nodes[1, s]]]
    best = np.inf
    for n in np.nonzero(inst.pinned == 0)[0]:
        for s in ses:
            best = min(best, OJ._dist2(inst.x[:, n], inst.x[:, inst.seg_nodes[0, s]],
                                       inst.x[:, inst.seg_nodes[1, s]]))
    return float(np.sqrt(best))


def test_batch_with_captures_over_two_calls():
    """Three burst volumes; the capture radius is 1.5 times the closest
    mobile-node to sessile-segment distance of the batch, and junctions break
    within a few steps, so captures, holds, releases and recaptures all
    happen; the state carries over from the first call to the second."""
    insts = []
    for i, nl in enumerate((4, 3, 5)):
        inst = W.subset(W.burst_instance(1_000_030 + i), nl)
        inst.pinned[:] = 0
        inst.pinned[64:] = 1          # loops 3 and later are sessile
        insts.append(inst)
    r_c = 1.5 * min(_min_capture_distance(inst) for inst in insts)
    nn = sum(inst.n_nodes for inst in insts)
    fr = np.random.default_rng(11).uniform(0.0, 1.0, (nn, 4))
    counts = [ost["count"].sum() for _, ost in _run(insts, 6, r_c, 3 * W.DT, 0.0, fr, calls=2)]
    print(f"capture radius {r_c:.2f} b, junctions formed per volume {counts}")
    assert sum(counts) > 0


def test_zero_radius_is_the_plain_burst():
    """A zero capture radius: bit for bit the plain burst of the same step
    graph (the persistent launch of small FP64 bursts sums in another order)."""
    insts = [W.subset(W.burst_instance(1_000_040 + i), nl) for i, nl in enumerate((2, 3))]
    bt = W.pack(insts)
    d1, d2 = batch_dev(bt), batch_dev(bt)
    prev = dd.dd_set_burst_mode(dd.BURST_GRAPH)
    try:
        r1, _ = dd.dd_burst_batch(bt.node_off, bt.seg_off, d1["x"], d1["seg_nodes"], d1["burgers"], d1["normal"],
                                  d1["pinned"], d1["sigma_app"], d1["volume"], MAT, 2, dd.DD_FP64, 20.0, 5, W.DT)
    finally:
        dd.dd_set_burst_mode(prev)
    st = _state_dev(bt.node_off[-1])
    fr = torch.full((bt.node_off[-1], 1), 0.5, dtype=torch.float64, device=DEV)
    r2 = dd.dd_burst_batch_junctions(bt.node_off, bt.seg_off, d2["x"], d2["seg_nodes"], d2["burgers"],
                                     d2["normal"], d2["pinned"], d2["sigma_app"], d2["volume"], MAT, st, fr,
                                     0.0, 1e-12, 0.0, 2, dd.DD_FP64, 20.0, 5, W.DT)
    torch.cuda.synchronize()
    assert torch.equal(d1["x"], d2["x"]) and torch.equal(r1, r2)
    assert int(st["count"].sum()) == 0


def test_invalid_junction_parameters():
    insts = [W.subset(W.burst_instance(1_000_050), 2)]
    bt = W.pack(insts)
    d = batch_dev(bt)
    st = _state_dev(bt.node_off[-1])
    fr = torch.full((bt.node_off[-1], 1), 0.5, dtype=torch.float64, device=DEV)
    for r_c, a, t0 in ((-1.0, 1e-12, 0.0), (1.0, -1.0, 0.0), (1.0, 1e-12, float("nan"))):
        with pytest.raises(dd.DDError):
            dd.dd_burst_batch_junctions(bt.node_off, bt.seg_off, d["x"], d["seg_nodes"], d["burgers"],
                                        d["normal"], d["pinned"], d["sigma_app"], d["volume"], MAT, st, fr,
                                        r_c, a, t0, 2, dd.DD_FP64, 20.0, 2, W.DT)


# ------------------------------------------------------ PTA with junctions --
from oracle import pta   # noqa: E402

DELTA = 1e-8


def _pta_volumes():
    insts = []
    for i, nl in enumerate((4, 3, 5)):
        inst = W.subset(W.burst_instance(1_000_030 + i), nl)
        inst.pinned[:] = 0
        inst.pinned[64:] = 1
        insts.append(inst)
    rates = np.array([[0, 0, 1e15, 0, 0, 0], [2e14, -1e14, 0, 3e14, 0, 1e14], [0, 0, 0, 0, 0, 8e14]], float)
    return insts, rates


def _pta_compare(insts, rates, ts, kw, fast0, calls=1, tol=1e-10, r_c=None):
    """dd_pta_step_junctions against oracle/pta.py with junctions over
    `calls` consecutive slow steps (times ts[c]); the junction state, fast
    clocks and microstructure carry over between calls on both sides."""
    bt = W.pack(insts)
    d = batch_dev(bt)
    nn = bt.node_off[-1]
    st = _state_dev(nn)
    if r_c is None:
        r_c = 1.5 * min(_min_capture_distance(inst) for inst in insts)
    a = 3 * W.DT
    fr = np.random.default_rng(17).uniform(0.0, 1.0, (nn, 4))
    fast = np.array(fast0, np.int64)
    J = {"state": st, "fractions": torch.tensor(fr, device=DEV), "capture_radius": r_c, "max_break_time": a,
         "fast_steps": fast}
    P = dd.PTAParams(dt=W.DT, delta=DELTA, **kw)
    OP = pta.PTAParams(dt=W.DT, delta=DELTA, chunk=kw["chunk_steps"], max_chunks=kw["max_chunks"],
                       lpdot_max=kw.get("lpdot_max", 0.05), max_jumps=kw.get("max_jumps", 2))
    ojn = [pta.Junctions(r_c, a, fr[bt.node_off[i]:bt.node_off[i + 1]], OJ.new_state(inst.n_nodes), int(fast0[i]))
           for i, inst in enumerate(insts)]
    cur = list(insts)
    outs = []
    for c in range(calls):
        got = dd.dd_pta_step(bt.node_off, bt.seg_off, d["x"], d["seg_nodes"], d["burgers"], d["normal"],
                             d["pinned"], d["volume"], rates, ts[c], P, MAT, 2, dd.DD_FP64, junctions=J)
        torch.cuda.synchronize()
        xg = d["x"].cpu().numpy()
        for i, inst in enumerate(cur):
            ref = pta.pta_step(inst, ts[c][i], rates[i], W.material(), 2, OP, ojn[i])
            print(f"call {c} volume {i}: steps {got['steps_a'][i]}/{got['steps_b'][i]}, jumps {got['jumps'][i]}, "
                  f"rerun {got['rerun_chunks'][i]}, fast clock {fast[i]} (oracle {ref['jn'].fast}), "
                  f"junctions {int(ref['jn'].state['count'].sum())}")
            for k in ("steps_a", "steps_b", "jumps", "rerun_chunks", "conv_a", "conv_b"):
                assert got[k][i] == ref[k], k
            for k in ("g_a", "g_b", "lp_a", "lp_b"):
                r = np.asarray(ref[k])
                assert np.abs(got[k][i] - r).max() <= tol * max(np.abs(r).max(), 1e-300), k
            n0, n1 = bt.node_off[i], bt.node_off[i + 1]
            disp_g, disp_o = xg[:, n0:n1] - insts[i].x, ref["x"] - insts[i].x
            assert np.abs(disp_g - disp_o).max() <= tol * max(np.abs(disp_o).max(), 1e-300)
            assert fast[i] == ref["jn"].fast
            s0 = bt.seg_off[i]
            os_ = ref["jn"].state
            jg = st["junction"].cpu().numpy()[n0:n1].astype(np.int64)
            ig = st["ignore"].cpu().numpy()[n0:n1].astype(np.int64)
            assert np.array_equal(np.where(jg >= 0, jg - s0, -1), os_["junction"])
            assert np.array_equal(np.where(ig >= 0, ig - s0, -1), os_["ignore"])
            assert np.array_equal(st["count"].cpu().numpy()[n0:n1], os_["count"])
            held = os_["junction"] >= 0
            assert np.array_equal(st["release"].cpu().numpy()[n0:n1][held], os_["release"][held])
            ojn[i] = ref["jn"]
            cur[i] = W.Instance(ref["x"], inst.seg_nodes, inst.burgers, inst.normal, inst.pinned, inst.sigma_app,
                                inst.volume, {})
        outs.append(got)
    return outs, [int(j.state["count"].sum()) for j in ojn]


def test_pta_junctions_two_slow_steps():
    insts, rates = _pta_volumes()
    ts = [np.array([5e-8, 3e-8, 4e-8]), np.array([6e-8, 4e-8, 5e-8])]
    _, counts = _pta_compare(insts, rates, ts, dict(chunk_steps=3, max_chunks=3, lpdot_max=np.inf), [0, 17, 5],
                             calls=2)
    assert sum(counts) > 0


def test_pta_junctions_jumps():
    insts, rates = _pta_volumes()
    outs, counts = _pta_compare(insts, rates, [np.array([5e-8, 3e-8, 4e-8])],
                                dict(chunk_steps=2, max_chunks=3, lpdot_max=0.0, max_jumps=2), [3, 0, 9])
    assert (outs[0]["jumps"] == 2).all() and sum(counts) > 0


def test_pta_junctions_rerun_restores_state():
    """t < delta/2: step 5 continues the t - delta run, with the junction
    state and clock of its own end; the t run's are carried on."""
    insts = []
    for seed in (1_000_072, 1_000_071):
        inst = W.subset(W.burst_instance(seed), 2)
        inst.pinned[:] = 0
        inst.pinned[32:] = 1            # the second loop is sessile
        insts.append(inst)
    rates = np.array([[0, 0, 1e15, 0, 0, 0], [0, 0, 0, 0, 0, 8e14]], float)
    # with this radius the second volume forms junctions and still takes step 5
    outs, counts = _pta_compare(insts, rates, [np.array([0.1, 0.1]) * DELTA],
                                dict(chunk_steps=2, max_chunks=3, lpdot_max=np.inf), [0, 4], r_c=421.0)
    assert outs[0]["rerun_chunks"][1] > 0 and counts[1] > 0


def test_pta_junctions_zero_radius_is_the_plain_step():
    insts, rates = _pta_volumes()
    bt = W.pack(insts)
    t = np.array([5e-8, 3e-8, 4e-8])
    P = dd.PTAParams(dt=W.DT, delta=DELTA, chunk_steps=2, max_chunks=2, lpdot_max=np.inf)
    d1, d2 = batch_dev(bt), batch_dev(bt)
    r1 = dd.dd_pta_step(bt.node_off, bt.seg_off, d1["x"], d1["seg_nodes"], d1["burgers"], d1["normal"],
                        d1["pinned"], d1["volume"], rates, t, P, MAT, 2, dd.DD_FP64)
    nn = bt.node_off[-1]
    fast = np.zeros(3, np.int64)
    J = {"state": _state_dev(nn), "fractions": torch.full((nn, 1), 0.5, dtype=torch.float64, device=DEV),
         "capture_radius": 0.0, "max_break_time": 1e-12, "fast_steps": fast}
    r2 = dd.dd_pta_step(bt.node_off, bt.seg_off, d2["x"], d2["seg_nodes"], d2["burgers"], d2["normal"],
                        d2["pinned"], d2["volume"], rates, t, P, MAT, 2, dd.DD_FP64, junctions=J)
    torch.cuda.synchronize()
    assert torch.equal(d1["x"], d2["x"])
    for k in r1:
        assert np.array_equal(r1[k], r2[k]), k
    assert (fast == r1["steps_a"] - 2 * r1["rerun_chunks"] + r1["steps_b"]).all()


def test_pta_junctions_invalid():
    insts, rates = _pta_volumes()
    bt = W.pack(insts)
    d = batch_dev(bt)
    nn = bt.node_off[-1]
    P = dd.PTAParams(dt=W.DT, delta=DELTA, chunk_steps=2, max_chunks=2, lpdot_max=np.inf)
    base = {"state": _state_dev(nn), "fractions": torch.full((nn, 1), 0.5, dtype=torch.float64, device=DEV),
            "capture_radius": 1.0, "max_break_time": 1e-12}
    for fs, r_c in ((np.array([0, -1, 0], np.int64), 1.0), (np.zeros(3, np.int64), -1.0)):
        with pytest.raises(dd.DDError):
            dd.dd_pta_step(bt.node_off, bt.seg_off, d["x"], d["seg_nodes"], d["burgers"], d["normal"],
                           d["pinned"], d["volume"], rates, np.array([5e-8] * 3), P, MAT, 2, dd.DD_FP64,
                           junctions=dict(base, fast_steps=fs, capture_radius=r_c))
