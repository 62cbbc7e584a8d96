"""Pins of the junction oracle (oracle/junctions.py) on the CPU: with no
capture it is the plain burst, bit for bit; on a hand-built pair of loops a
mobile node next to a sessile segment is captured at the first step, held
fixed until t0 + f a, then released and not captured again by the same
segment while it stays within twice the capture radius."""
import numpy as np
import pytest

import oracle as O
from oracle import junctions as OJ
from paper_2005_02498_amd import workloads as W

MAT = W.material()


def _pair_of_loops():
    """A mobile octagon (radius 50 b, plane z = 0, node 0 at (50, 0, 0)) and a
    sessile square in the plane x = 53 whose first segment runs 3 b from node 0."""
    ang = np.arange(8) * np.pi / 4
    mob = np.stack([50 * np.cos(ang), 50 * np.sin(ang), np.zeros(8)])
    ses = np.array([[53.0, 53.0, 53.0, 53.0], [0.0, 0.0, 40.0, 40.0], [-20.0, 20.0, 20.0, -20.0]])
    x = np.concatenate([mob, ses], axis=1) * 1.0
    sn = np.array([list(range(8)) + [8, 9, 10, 11], [1, 2, 3, 4, 5, 6, 7, 0, 9, 10, 11, 8]], np.int32)
    b = np.zeros((3, 12))
    b[0, :8] = 1.0
    b[1, 8:] = 1.0
    nrm = np.zeros((3, 12))
    nrm[2, :8] = 1.0
    nrm[0, 8:] = 1.0
    pinned = np.zeros(12, np.uint8)
    pinned[8:] = 1
    sig = np.array([0, 0, 0, 0, 80e6, 0.0])   # xz shear: the edge loop expands
    return W.Instance(x, sn, b, nrm, pinned, sig, 2000.0 ** 3, {})


def test_no_capture_is_the_plain_burst():
    inst = W.subset(W.burst_instance(1_000_020), 2)
    fr = np.full((inst.n_nodes, 2), 0.5)
    st = OJ.new_state(inst.n_nodes)
    x, rate = OJ.burst(inst, MAT, 2, 4, W.DT, 0.0, 1e-12, 0.0, fr, st)
    x0, r0, _ = O.burst(inst, MAT, 2, 4, W.DT)
    assert np.array_equal(x, x0)
    assert np.array_equal(rate, r0)
    assert (st["junction"] == -1).all() and (st["count"] == 0).all()


def test_capture_hold_release_and_no_recapture():
    inst = _pair_of_loops()
    dt = W.DT
    a = 5 * dt
    fr = np.full((12, 3), 0.9)
    fr[0, 0] = 0.5                      # node 0's first junction: t_b = 2.5 dt
    st = OJ.new_state(12)
    t0 = 1e-9
    x1, _ = OJ.burst(inst, MAT, 2, 1, dt, 5.0, a, t0, fr, st)
    assert st["junction"][0] == 8 and st["count"][0] == 1
    assert st["release"][0] == t0 + 0.5 * a
    assert np.array_equal(x1[:, 0], inst.x[:, 0])          # held
    assert np.abs(x1[:, 1:8] - inst.x[:, 1:8]).max() > 0    # the rest of the loop moves
    assert (st["junction"][1:8] == -1).all()
    # steps 1 and 2 (t < release): still held; step 3 (t0 + 3 dt >= t0 + 2.5 dt): released
    s2 = W.Instance(x1, inst.seg_nodes, inst.burgers, inst.normal, inst.pinned, inst.sigma_app, inst.volume, {})
    x3, _ = OJ.burst(s2, MAT, 2, 2, dt, 5.0, a, t0 + dt, fr, st)
    assert np.array_equal(x3[:, 0], inst.x[:, 0]) and st["junction"][0] == 8
    s3 = W.Instance(x3, inst.seg_nodes, inst.burgers, inst.normal, inst.pinned, inst.sigma_app, inst.volume, {})
    x4, _ = OJ.burst(s3, MAT, 2, 1, dt, 5.0, a, t0 + 3 * dt, fr, st)
    assert st["junction"][0] == -1 and st["ignore"][0] == 8 and st["count"][0] == 1
    assert np.abs(x4[:, 0] - x3[:, 0]).max() > 0            # free again
    # within 2 r_c of segment 8 it is not captured again
    x5, _ = OJ.burst(W.Instance(x4, inst.seg_nodes, inst.burgers, inst.normal, inst.pinned, inst.sigma_app,
                                inst.volume, {}), MAT, 2, 3, dt, 5.0, a, t0 + 4 * dt, fr, st)
    assert st["junction"][0] == -1 and st["count"][0] == 1


def test_distance_rule():
    a, b = np.array([0.0, 0.0, 0.0]), np.array([10.0, 0.0, 0.0])
    assert OJ._dist2(np.array([5.0, 3.0, 4.0]), a, b) == pytest.approx(25.0)
    assert OJ._dist2(np.array([-3.0, 4.0, 0.0]), a, b) == pytest.approx(25.0)   # beyond the first end
    assert OJ._dist2(np.array([13.0, 0.0, 4.0]), a, b) == pytest.approx(25.0)   # beyond the second end
