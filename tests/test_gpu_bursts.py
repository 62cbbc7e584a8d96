"""GPU parity of batched bursts (dd_burst_batch) against the FP64 oracle."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_2005_02498_amd import workloads as W
import paper_2005_02498_amd as dd

from gpu_util import MAT, batch_dev, normwise

pytestmark = pytest.mark.gpu


def _gpu_burst(bt, n_steps, prec=dd.DD_FP64, Q=2, features=True):
    d = batch_dev(bt)
    rate, feat = dd.dd_burst_batch(bt.node_off, bt.seg_off, d["x"], d["seg_nodes"], d["burgers"],
                                   d["normal"], d["pinned"], d["sigma_app"], d["volume"], MAT,
                                   Q, prec, 20.0, n_steps, W.DT, want_features=features)
    torch.cuda.synchronize()
    return (d["x"].cpu().numpy(), rate.cpu().numpy(),
            feat.cpu().numpy() if feat is not None else None)


def _small_batch():
    insts = []
    for i, nl in enumerate((1, 3, 2, 4)):
        insts.append(W.subset(W.burst_instance(1_000_000 + i), nl))
    # make sure the batch has mobile and pinned loops
    insts[1].pinned[:] = 0
    insts[1].pinned[64:] = 1
    insts[3].pinned[:] = 0
    insts[3].pinned[96:] = 1
    return W.pack(insts)


def test_config0_burst_100_steps_fp64():
    inst = W.config0()
    bt = W.pack([inst])
    xg, rg, fg = _gpu_burst(bt, 100)
    xo, ro, fo = O.burst(inst, W.material(), 2, 100, W.DT)
    e_disp = normwise(xg - inst.x, xo - inst.x)
    e_rate = np.abs(rg[0] - ro).max() / np.abs(ro).max()
    print(f"config0 100 steps: displacement err {e_disp:.2e}, rate err {e_rate:.2e}, "
          f"max displacement {np.linalg.norm(xo - inst.x, axis=0).max():.3f} b")
    assert e_disp < 1e-9
    assert e_rate < 1e-9
    np.testing.assert_allclose(fg[0], fo, rtol=1e-12, atol=0)


def test_small_batch_fp64_vs_oracle():
    bt = _small_batch()
    xg, rg, fg = _gpu_burst(bt, 5)
    xo, ro, fo = O.burst_batch(bt, W.material(), 2, 5, W.DT)
    assert normwise(xg - bt.x, xo - bt.x) < 1e-10
    assert np.abs(rg - ro).max() / np.abs(ro).max() < 1e-10
    np.testing.assert_allclose(fg, fo, rtol=1e-12, atol=0)
    assert np.count_nonzero(ro) > 0


def test_small_batch_mixed_vs_oracle():
    bt = _small_batch()
    xg, rg, _ = _gpu_burst(bt, 5, dd.DD_MIXED)
    xo, ro, _ = O.burst_batch(bt, W.material(), 2, 5, W.DT)
    assert normwise(xg - bt.x, xo - bt.x) < 1e-4
    assert np.abs(rg - ro).max() / np.abs(ro).max() < 1e-4


@pytest.mark.parametrize("variant", [0, 1, 2])
def test_small_batch_mixed_each_variant(variant):
    bt = _small_batch()
    dd.dd_set_plan(0, variant)
    try:
        xg, rg, _ = _gpu_burst(bt, 5, dd.DD_MIXED)
        assert dd.dd_last_plan()[2] == variant
    finally:
        dd.dd_set_plan(-1)
    xo, ro, _ = O.burst_batch(bt, W.material(), 2, 5, W.DT)
    assert normwise(xg - bt.x, xo - bt.x) < 1e-4
    assert np.abs(rg - ro).max() / np.abs(ro).max() < 1e-4


def test_batched_equals_single_calls():
    bt = _small_batch()
    xb, rb, fb = _gpu_burst(bt, 4)
    for i in range(bt.n_inst):
        n0, n1 = bt.node_off[i], bt.node_off[i + 1]
        s0, s1 = bt.seg_off[i], bt.seg_off[i + 1]
        one = W.Batch(np.array([0, n1 - n0]), np.array([0, s1 - s0]), bt.x[:, n0:n1].copy(),
                      bt.seg_nodes[:, s0:s1].copy(), bt.burgers[:, s0:s1].copy(),
                      bt.normal[:, s0:s1].copy(), bt.pinned[n0:n1].copy(),
                      bt.sigma_app[i:i + 1].copy(), bt.volume[i:i + 1].copy())
        x1, r1, f1 = _gpu_burst(one, 4)
        np.testing.assert_allclose(r1[0], rb[i], rtol=1e-13, atol=1e-13 * np.abs(rb[i]).max())
        np.testing.assert_allclose(x1, xb[:, n0:n1], rtol=0, atol=1e-11)
        np.testing.assert_array_equal(f1[0], fb[i])


def test_resume_equals_single_run():
    bt = _small_batch()
    x6, r6, _ = _gpu_burst(bt, 6, features=False)
    d = batch_dev(bt)
    r1, _ = dd.dd_burst_batch(bt.node_off, bt.seg_off, d["x"], d["seg_nodes"], d["burgers"],
                              d["normal"], d["pinned"], d["sigma_app"], d["volume"], MAT, 2,
                              dd.DD_FP64, 20.0, 3, W.DT)
    r1 = r1.cpu().numpy().copy()
    r2, _ = dd.dd_burst_batch(bt.node_off, bt.seg_off, d["x"], d["seg_nodes"], d["burgers"],
                              d["normal"], d["pinned"], d["sigma_app"], d["volume"], MAT, 2,
                              dd.DD_FP64, 20.0, 3, W.DT)
    np.testing.assert_array_equal(d["x"].cpu().numpy(), x6)
    np.testing.assert_allclose(0.5 * (r1 + r2.cpu().numpy()), r6, rtol=1e-14,
                               atol=1e-14 * np.abs(r6).max())


def test_zero_steps_and_empty_instances():
    insts = [W.subset(W.burst_instance(1_000_010), 1), W.subset(W.burst_instance(1_000_011), 2)]
    bt = W.pack(insts)
    xg, rg, fg = _gpu_burst(bt, 0)
    np.testing.assert_array_equal(xg, bt.x)
    assert np.all(rg == 0)
    _, _, fo = O.burst_batch(bt, W.material(), 2, 0, W.DT)
    np.testing.assert_allclose(fg, fo, rtol=1e-12, atol=0)
    # an instance with no nodes and no segments in the middle of the batch
    e = W.Instance(np.zeros((3, 0)), np.zeros((2, 0), np.int32), np.zeros((3, 0)),
                   np.zeros((3, 0)), np.zeros(0, np.uint8), np.zeros(6), 1.0)
    bt = W.pack([insts[0], e, insts[1]])
    xg, rg, _ = _gpu_burst(bt, 2)
    xo, ro, _ = O.burst_batch(bt, W.material(), 2, 2, W.DT)
    assert np.all(rg[1] == 0)
    assert normwise(xg - bt.x, xo - bt.x) < 1e-10


@pytest.mark.parametrize("prec,steps,tol", [(dd.DD_FP64, 2, 1e-10), (dd.DD_MIXED, 3, 1e-4)])
def test_full_batch_of_512_sampled(prec, steps, tol):
    """The benchmark's launch configuration: all 512 burst volumes (256-4096
    segments each) in one call; eight sampled volumes (the four smallest, two
    of median size and the two largest of at most 2048 segments, so that the
    oracle stays fast) against the oracle burst, volume by volume."""
    insts = W.config2(512)
    bt = W.pack(insts)
    xg, rg, _ = _gpu_burst(bt, steps, prec, features=False)
    ns = np.diff(bt.seg_off)
    order = np.argsort(ns, kind="stable")
    small = list(order[:4])
    mid = list(order[len(order) // 2:len(order) // 2 + 2])
    big = [i for i in order[::-1] if ns[i] <= 2048][:2]
    for i in small + mid + big:
        i = int(i)
        one = W.pack([insts[i]])
        xo, ro, _ = O.burst_batch(one, W.material(), 2, steps, W.DT)
        n0, n1 = bt.node_off[i], bt.node_off[i + 1]
        e_x = normwise(xg[:, n0:n1] - insts[i].x, xo - insts[i].x)
        e_r = np.abs(rg[i] - ro[0]).max() / max(np.abs(ro[0]).max(), 1e-300)
        print(f"volume {i} ({ns[i]} segments): displacement err {e_x:.2e}, rate err {e_r:.2e}")
        assert e_x < tol and e_r < tol


def test_async_two_calls_one_sync():
    """With validation off, dd_burst_batch is asynchronous once its instance
    tables, work split and step graph are cached.  Two calls enqueued back to
    back on one output (the second relaunches the first's cached graph, and
    resumes from its end state), a clone of the rates enqueued between them,
    and one synchronisation: the same rates and positions, bit for bit, as the
    same two calls made with validation on; the stream is still busy when the
    second call returns."""
    insts = [W.subset(W.burst_instance(1_000_020 + i), 32) for i in range(8)]
    bt = W.pack(insts)
    ref = batch_dev(bt)
    out = []
    for _ in range(2):
        r, _ = dd.dd_burst_batch(bt.node_off, bt.seg_off, ref["x"], ref["seg_nodes"], ref["burgers"],
                                 ref["normal"], ref["pinned"], ref["sigma_app"], ref["volume"], MAT, 2,
                                 dd.DD_MIXED, 20.0, 100, W.DT)
        out.append(r.cpu().numpy())
    d = batch_dev(bt)
    rate = torch.empty((bt.n_inst, 12), dtype=torch.float64, device="cuda:0")
    args = (bt.node_off, bt.seg_off, d["x"], d["seg_nodes"], d["burgers"], d["normal"], d["pinned"],
            d["sigma_app"], d["volume"], MAT, 2, dd.DD_MIXED, 20.0, 100, W.DT)
    prev = dd.dd_set_validation(False)
    try:
        # one call to cache tables and graph for this argument set
        dd.dd_burst_batch(*args, rate_avg_out=rate)
        torch.cuda.synchronize()
        d["x"].copy_(torch.tensor(bt.x, device="cuda:0"))
        torch.cuda.synchronize()
        dd.dd_burst_batch(*args, rate_avg_out=rate)
        first = rate.clone()
        dd.dd_burst_batch(*args, rate_avg_out=rate)
        busy = not torch.cuda.current_stream().query()
        torch.cuda.synchronize()
    finally:
        dd.dd_set_validation(prev)
    print(f"stream busy after the second call returned: {busy}")
    assert busy
    np.testing.assert_array_equal(first.cpu().numpy(), out[0])
    np.testing.assert_array_equal(rate.cpu().numpy(), out[1])
    np.testing.assert_array_equal(d["x"].cpu().numpy(), ref["x"].cpu().numpy())
    dd.dd_check()


def _in_mode(mode, fn):
    prev = dd.dd_set_burst_mode(mode)
    try:
        return fn()
    finally:
        dd.dd_set_burst_mode(prev)


def test_persistent_config0_against_graph_and_oracle():
    """The 256-segment volume, 100 FP64 steps: the persistent launch (128
    workgroups, and one workgroup) against the step graph and the oracle.
    The split does not change the positions (bit for bit); the slip rates
    differ between splits only in the order of the workgroups' sums."""
    inst = W.config0()
    bt = W.pack([inst])
    xa, ra, fa = _in_mode(dd.BURST_AUTO, lambda: _gpu_burst(bt, 100))
    x1, r1, _ = _in_mode(dd.BURST_PERSISTENT_ONE, lambda: _gpu_burst(bt, 100, features=False))
    xg, rg, fg = _in_mode(dd.BURST_GRAPH, lambda: _gpu_burst(bt, 100))
    xo, ro, fo = O.burst(inst, W.material(), 2, 100, W.DT)
    np.testing.assert_array_equal(xa, x1)
    np.testing.assert_allclose(ra, r1, rtol=1e-13, atol=1e-13 * np.abs(ra).max())
    e_graph = normwise(xa - inst.x, xg - inst.x)
    e_disp = normwise(xa - inst.x, xo - inst.x)
    e_rate = np.abs(ra[0] - ro).max() / np.abs(ro).max()
    print(f"persistent config0: vs graph {e_graph:.2e}, vs oracle displacement {e_disp:.2e}, rate {e_rate:.2e}")
    assert e_graph < 1e-12
    assert e_disp < 1e-9 and e_rate < 1e-9
    np.testing.assert_array_equal(fa, fg)


@pytest.mark.parametrize("Q", [1, 4])
def test_persistent_batch_against_oracle(Q):
    """A batch with an empty instance, instances of 1 to 4 loops with mobile
    and pinned loops, an odd number of steps (the positions end in the second
    buffer), Q = 1 and 4: against the oracle, and the same positions with one
    workgroup per instance."""
    insts = [W.subset(W.burst_instance(1_000_030 + i), nl) for i, nl in enumerate((2, 1, 4, 3))]
    insts[2].pinned[:] = 0
    insts[2].pinned[64:] = 1
    e = W.Instance(np.zeros((3, 0)), np.zeros((2, 0), np.int32), np.zeros((3, 0)), np.zeros((3, 0)),
                   np.zeros(0, np.uint8), np.zeros(6), 1.0)
    bt = W.pack(insts[:2] + [e] + insts[2:])
    xa, ra, _ = _in_mode(dd.BURST_AUTO, lambda: _gpu_burst(bt, 7, Q=Q, features=False))
    x1, _, _ = _in_mode(dd.BURST_PERSISTENT_ONE, lambda: _gpu_burst(bt, 7, Q=Q, features=False))
    xo, ro, _ = O.burst_batch(bt, W.material(), Q, 7, W.DT)
    np.testing.assert_array_equal(xa, x1)
    assert normwise(xa - bt.x, xo - bt.x) < 1e-10
    assert np.abs(ra - ro).max() / np.abs(ro).max() < 1e-10
    assert np.all(ra[2] == 0)
