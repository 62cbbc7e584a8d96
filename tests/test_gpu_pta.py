"""GPU parity of the PTA slow-time step (dd_pta_step) against the oracle's
plain-Python driver (oracle/pta.py) on the same seeded volumes: the same
decisions (fast steps taken, convergence, jumps, re-run chunks) and the same
running averages, rates and final microstructure to FP64 tolerance."""
import numpy as np
import pytest
import torch

from oracle import pta
from paper_2005_02498_amd import workloads as W
import paper_2005_02498_amd as dd

from gpu_util import MAT, batch_dev

pytestmark = pytest.mark.gpu

DELTA = 1e-8


def _volumes():
    insts = [W.subset(W.burst_instance(1_000_010 + i), nl) for i, nl in enumerate((2, 3, 1))]
    insts[1].pinned[:] = 0
    insts[1].pinned[64:] = 1            # one sessile loop
    rates = np.array([[0, 0, 1e15, 0, 0, 0], [2e14, -1e14, 0, 3e14, 0, 1e14], [0, 0, 0, 0, 0, 8e14]], float)
    return insts, rates


def _compare(insts, rates, t, kw, tol=1e-10):
    bt = W.pack(insts)
    d = batch_dev(bt)
    P = dd.PTAParams(dt=W.DT, delta=DELTA, **kw)
    got = dd.dd_pta_step(bt.node_off, bt.seg_off, d["x"], d["seg_nodes"], d["burgers"], d["normal"],
                         d["pinned"], d["volume"], rates, t, P, MAT, 2, dd.DD_FP64)
    torch.cuda.synchronize()
    xg = d["x"].cpu().numpy()
    OP = pta.PTAParams(dt=W.DT, delta=DELTA, chunk=kw["chunk_steps"], max_chunks=kw["max_chunks"],
                       lpdot_max=kw.get("lpdot_max", 0.05), max_jumps=kw.get("max_jumps", 2),
                       h_max=kw.get("h_max", 1.0))
    for i, inst in enumerate(insts):
        ref = pta.pta_step(inst, t[i], rates[i], W.material(), 2, OP)
        print(f"volume {i}: steps {got['steps_a'][i]}/{got['steps_b'][i]} (oracle {ref['steps_a']}/{ref['steps_b']}), "
              f"jumps {got['jumps'][i]}, rerun {got['rerun_chunks'][i]}, h {got['h'][i]:.3e}")
        assert got["steps_a"][i] == ref["steps_a"] and got["steps_b"][i] == ref["steps_b"]
        assert got["jumps"][i] == ref["jumps"] and got["rerun_chunks"][i] == ref["rerun_chunks"]
        assert got["conv_a"][i] == ref["conv_a"] and got["conv_b"][i] == ref["conv_b"]
        for k in ("rho_a", "rho_b", "h"):
            assert got[k][i] == pytest.approx(ref[k], rel=tol, abs=1e-300), k
        for k in ("g_a", "g_b", "lp_a", "lp_b"):
            r = np.asarray(ref[k])
            assert np.abs(got[k][i] - r).max() <= tol * max(np.abs(r).max(), 1e-300), k
        # the rates are differences of nearly equal averages: compare on the scale of the averages
        assert abs(got["rhodot"][i] - ref["rhodot"]) <= tol * abs(ref["rho_b"]) / DELTA
        lp_scale = max(np.abs(ref["lp_a"]).max(), np.abs(ref["lp_b"]).max(), 1e-300)
        assert np.abs(got["lpdot"][i] - ref["lpdot"]).max() <= tol * lp_scale / DELTA
        s0, s1 = bt.node_off[i], bt.node_off[i + 1]
        disp_g, disp_o = xg[:, s0:s1] - inst.x, ref["x"] - inst.x
        assert np.abs(disp_g - disp_o).max() <= tol * max(np.abs(disp_o).max(), 1e-300)
    return got


def test_pta_step_no_jumps():
    insts, rates = _volumes()
    got = _compare(insts, rates, np.array([5e-8, 3e-8, 4e-8]),
                   dict(chunk_steps=3, max_chunks=4, lpdot_max=np.inf))
    assert (got["jumps"] == 0).all()


def test_pta_step_every_check_a_jump():
    insts, rates = _volumes()
    got = _compare(insts, rates, np.array([5e-8, 3e-8, 4e-8]),
                   dict(chunk_steps=2, max_chunks=3, lpdot_max=0.0, max_jumps=2))
    assert (got["jumps"] == 2).all()


def test_pta_step_rerun_rule():
    """t < delta/2: the t - delta load is the larger one, so step 5 runs."""
    insts, rates = _volumes()
    got = _compare(insts, rates, np.array([0.2 * DELTA, 0.3 * DELTA, 0.1 * DELTA]),
                   dict(chunk_steps=2, max_chunks=3, lpdot_max=np.inf))
    assert got["rerun_chunks"].max() > 0


def test_pta_step_mixed_close_to_fp64():
    insts, rates = _volumes()
    bt = W.pack(insts)
    t = np.array([5e-8, 3e-8, 4e-8])
    P = dd.PTAParams(dt=W.DT, delta=DELTA, chunk_steps=3, max_chunks=2, lpdot_max=np.inf)
    res = []
    for prec in (dd.DD_FP64, dd.DD_MIXED):
        d = batch_dev(bt)
        res.append(dd.dd_pta_step(bt.node_off, bt.seg_off, d["x"], d["seg_nodes"], d["burgers"], d["normal"],
                                  d["pinned"], d["volume"], rates, t, P, MAT, 2, prec))
    for k in ("lp_a", "lp_b"):
        a, b = res[0][k], res[1][k]
        assert np.abs(a - b).max() <= 1e-4 * np.abs(a).max()


def test_pta_invalid_parameters():
    insts, rates = _volumes()
    bt = W.pack(insts)
    d = batch_dev(bt)
    for bad in (dict(chunk_steps=0), dict(max_chunks=1), dict(delta=0.0), dict(tol_rho=-1.0)):
        kw = dict(dt=W.DT, delta=DELTA)
        kw.update(bad)
        with pytest.raises(dd.DDError):
            dd.dd_pta_step(bt.node_off, bt.seg_off, d["x"], d["seg_nodes"], d["burgers"], d["normal"],
                           d["pinned"], d["volume"], rates, np.zeros(3), dd.PTAParams(**kw), MAT, 2, dd.DD_FP64)


def test_pta_full_batch_of_512_sampled():
    """The benchmark's PTA workload (all 512 burst volumes in one call, chunks
    of 20 steps, at most 10 checks, l(t) = each volume's stress at t = 1e-7 s,
    delta = 1e-8 s), here in FP64: the four smallest volumes and the smallest
    one of at least 512 segments against the oracle driver, with the same
    decisions and values to 1e-10."""
    insts = W.config2(512)
    bt = W.pack(insts)
    d = batch_dev(bt)
    rates = np.asarray(bt.sigma_app) / 1e-7
    t = np.full(bt.n_inst, 1e-7)
    P = dd.PTAParams(dt=W.DT, chunk_steps=20, max_chunks=10, delta=1e-8, lpdot_max=float("inf"))
    got = dd.dd_pta_step(bt.node_off, bt.seg_off, d["x"], d["seg_nodes"], d["burgers"], d["normal"],
                         d["pinned"], d["volume"], rates, t, P, MAT, 2, dd.DD_FP64)
    torch.cuda.synchronize()
    xg = d["x"].cpu().numpy()
    ns = np.diff(bt.seg_off)
    order = np.argsort(ns, kind="stable")
    sample = [int(i) for i in order[:4]] + [int(next(i for i in order if ns[i] >= 512))]
    OP = pta.PTAParams(dt=W.DT, chunk=20, max_chunks=10, delta=1e-8, lpdot_max=np.inf)
    tol = 1e-10
    for i in sample:
        ref = pta.pta_step(insts[i], 1e-7, rates[i], W.material(), 2, OP)
        print(f"volume {i} ({ns[i]} segments): steps {got['steps_a'][i]}/{got['steps_b'][i]} "
              f"(oracle {ref['steps_a']}/{ref['steps_b']}), rerun {got['rerun_chunks'][i]}")
        for k in ("steps_a", "steps_b", "jumps", "rerun_chunks", "conv_a", "conv_b"):
            assert got[k][i] == ref[k], k
        for k in ("g_a", "g_b", "lp_a", "lp_b"):
            r = np.asarray(ref[k])
            assert np.abs(got[k][i] - r).max() <= tol * max(np.abs(r).max(), 1e-300), k
        n0, n1 = bt.node_off[i], bt.node_off[i + 1]
        disp_g, disp_o = xg[:, n0:n1] - insts[i].x, ref["x"] - insts[i].x
        assert np.abs(disp_g - disp_o).max() <= tol * max(np.abs(disp_o).max(), 1e-300)
