"""Pins of the junction-node oracle (oracle/junction_nodes.py; Sec. "Thermal
activation", Eq. tb) on hand-built crossings whose junction point, timings and
topology are known in closed form, and against brute force (CPU only)."""
import numpy as np
import pytest

import oracle as O
from oracle import junction_nodes as JN
from paper_2005_02498_amd import workloads as W


def _brute(p, p2, q, q2, n=2001):
    u = np.linspace(0.0, 1.0, n)
    A = p[:, None] + u[None, :] * (p2 - p)[:, None]
    B = q[:, None] + u[None, :] * (q2 - q)[:, None]
    d2 = ((A[:, :, None] - B[:, None, :]) ** 2).sum(0)
    i, j = np.unravel_index(np.argmin(d2), d2.shape)
    return d2[i, j], u[i]


def test_closest_approach_closed_form_and_brute_force():
    # perpendicular crossing at height 3: distance 3, at the middle of the first
    d2, u = JN.segment_closest(np.array([30.0, -50, 3]), np.array([30.0, 50, 3]),
                               np.array([-100.0, 0, 0]), np.array([100.0, 0, 0]))
    assert d2 == 9.0 and u == 0.5
    # parallel, overlapping: distance 2, u = 0 by the rule for parallel lines
    d2, u = JN.segment_closest(np.array([0.0, 2, 0]), np.array([10.0, 2, 0]),
                               np.array([-5.0, 0, 0]), np.array([5.0, 0, 0]))
    assert d2 == pytest.approx(4.0) and u == 0.0
    # end to end on one line: the gap
    d2, u = JN.segment_closest(np.array([0.0, 0, 0]), np.array([1.0, 0, 0]),
                               np.array([3.0, 0, 0]), np.array([7.0, 0, 0]))
    assert d2 == pytest.approx(4.0) and u == 1.0
    rng = np.random.default_rng(5)
    for _ in range(60):
        p, p2, q, q2 = (rng.uniform(-10, 10, 3) for _ in range(4))
        d2, u = JN.segment_closest(p, p2, q, q2)
        b2, _ = _brute(p, p2, q, q2)
        # the exact minimum is at most the sampled one and close to it
        assert d2 <= b2 + 1e-9 and b2 - d2 < 5e-3 * (1 + b2)


def crossing(d=3.0, K=2, shift=0.0, cx=30.0, continued=False):
    """A pinned sessile segment on the x axis (nodes 0, 1; with `continued` a
    second one from x = 100 to 300, node 6) and a mobile chain along y at
    x = cx, height d (nodes 2-5, ends pinned): its middle segment (3 -> 4)
    passes over the sessile line at y = shift."""
    x = np.array([[-100.0, 100.0, cx, cx, cx, cx],
                  [0.0, 0.0, -150.0 + shift, -50.0 + shift, 50.0 + shift, 150.0 + shift],
                  [0.0, 0.0, d, d, d, d]])
    sn = np.array([[0, 2, 3, 4], [1, 3, 4, 5]], np.int32)
    b = np.array([[1.0, 0.0, 0.0, 0.0], [0.0, 1.0, 1.0, 1.0], [0.0, 0.0, 0.0, 0.0]])
    pinned = np.array([1, 1, 1, 0, 0, 1], np.uint8)
    if continued:
        x = np.concatenate([x, [[300.0], [0.0], [0.0]]], axis=1)
        sn = np.concatenate([sn, [[1], [6]]], axis=1).astype(np.int32)
        b = np.concatenate([b, [[1.0], [0.0], [0.0]]], axis=1)
        pinned = np.concatenate([pinned, [1]]).astype(np.uint8)
    nrm = np.tile(np.array([[0.0], [0.0], [1.0]]), (1, sn.shape[1]))
    inst = W.Instance(x=x, seg_nodes=sn, burgers=b, normal=nrm, pinned=pinned, sigma_app=np.zeros(6),
                      volume=1e9)
    return W.with_junction_slots(inst, K)


def _state(inst):
    return JN.new_state(inst.n_nodes, inst.n_segs, [0.25, 0.5, 0.75])


def test_crossing_capture_release_merge_and_ignore():
    inst = crossing()
    P = JN.Params(capture_radius=5.0, max_break_time=8.0, l_min=1.0, n_slots=2)
    x, sn, bu, nr = (np.array(a) for a in (inst.x, inst.seg_nodes, inst.burgers, inst.normal))
    st = _state(inst)
    made = JN.topology_step(x, sn, bu, nr, inst.pinned, 0.0, P, st)
    # segment 2 (3 -> 4) is split at its closest point (30, 0, 3) by the first
    # node slot (6) and the first segment slot (4)
    assert made == [(2, 0, 6, 4)]
    assert list(x[:, 6]) == [30.0, 0.0, 3.0]
    assert list(sn[:, 2]) == [3, 6] and list(sn[:, 4]) == [6, 4]
    assert list(bu[:, 4]) == list(bu[:, 2]) and list(nr[:, 4]) == list(nr[:, 2])
    assert st["release"][6] == 0.0 + 0.25 * 8.0 and st["ses"][6] == 0 and st["count"] == 1
    # both halves keep the junction point: never captured while the node holds them
    assert st["ignore"][2] and st["ignore"][4] and list(st["point"][:, 4]) == [30.0, 0.0, 3.0]
    # held until t = 2 (the other segments are farther than r_c: no capture)
    assert JN.topology_step(x, sn, bu, nr, inst.pinned, 1.5, P, st) == []
    assert list(sn[:, 2]) == [3, 6]
    # released at t = 2: the in-segment takes the out-segment's end, the slot is free again
    assert JN.topology_step(x, sn, bu, nr, inst.pinned, 2.0, P, st) == []
    assert list(sn[:, 2]) == [3, 4] and list(sn[:, 4]) == [8, 9] and not bu[:, 4].any()
    assert st["ses"][6] == -1 and st["ignore"][2] and not st["ignore"][4]
    # still within r_c, but the segment keeps the point of the junction it broke from
    assert JN.topology_step(x, sn, bu, nr, inst.pinned, 3.0, P, st) == []
    # moved to z = 8 (5 from the point, within 2 r_c): kept; to z = 14 (11, beyond): forgotten
    x[2, 2:6] = 8.0
    JN.topology_step(x, sn, bu, nr, inst.pinned, 4.0, P, st)
    assert st["ignore"][2]
    x[2, 2:6] = 14.0
    JN.topology_step(x, sn, bu, nr, inst.pinned, 5.0, P, st)
    assert not st["ignore"][2]
    # back within r_c: captured again, with the next fraction
    x[2, 2:6] = 3.0
    assert JN.topology_step(x, sn, bu, nr, inst.pinned, 6.0, P, st) == [(2, 0, 6, 4)]
    assert st["release"][6] == 6.0 + 0.5 * 8.0 and st["count"] == 2


def test_junction_point_clamped_near_an_end_and_short_segments():
    # the crossing 0.5 b before node 3: the point is clamped to l_min = 2 from it
    inst = crossing(shift=50.5)
    P = JN.Params(capture_radius=5.0, max_break_time=8.0, l_min=2.0, n_slots=2)
    x, sn, bu, nr = (np.array(a) for a in (inst.x, inst.seg_nodes, inst.burgers, inst.normal))
    made = JN.topology_step(x, sn, bu, nr, inst.pinned, 0.0, P, _state(inst))
    # segment 1 (2 -> 3, y -99.5 .. 0.5) passes over the crossing at 0.995 of its
    # length: clamped to 1 - 2/100; segment 2 (3 -> 4) at its start: clamped to 2/100
    assert [m[0] for m in made] == [1, 2]
    j1, j2 = made[0][2], made[1][2]
    assert x[1, j1] == pytest.approx(0.5 - 2.0) and x[1, j2] == pytest.approx(0.5 + 2.0)
    # a segment no longer than 2 l_min forms no junction
    P2 = JN.Params(capture_radius=5.0, max_break_time=8.0, l_min=50.0, n_slots=2)
    x, sn, bu, nr = (np.array(a) for a in (inst.x, inst.seg_nodes, inst.burgers, inst.normal))
    assert JN.topology_step(x, sn, bu, nr, inst.pinned, 0.0, P2, _state(inst)) == []


def test_adjacent_sessile_segment_does_not_recapture():
    """The crossing at x = 97, 3 b from the shared node of two sessile
    segments of one line: the first in index order forms the junction, and
    the halves of the split segment are not captured by the second while the
    node holds them."""
    inst = crossing(cx=97.0, continued=True)
    P = JN.Params(capture_radius=8.0, max_break_time=8.0, l_min=1.0, n_slots=2)
    x, sn, bu, nr = (np.array(a) for a in (inst.x, inst.seg_nodes, inst.burgers, inst.normal))
    st = _state(inst)
    assert [m[:2] for m in JN.topology_step(x, sn, bu, nr, inst.pinned, 0.0, P, st)] == [(2, 0)]
    # the second sessile segment (4) is within r_c of both halves
    for s_half in (2, 5):
        a, b = x[:, sn[0, s_half]], x[:, sn[1, s_half]]
        assert JN.segment_closest(a, b, x[:, 1], x[:, 6])[0] < 64.0
    for t in (0.5, 1.0, 1.5):
        assert JN.topology_step(x, sn, bu, nr, inst.pinned, t, P, st) == []


def test_no_free_slot_means_no_junction():
    inst = crossing(shift=50.5, K=1)
    P = JN.Params(capture_radius=5.0, max_break_time=8.0, l_min=2.0, n_slots=1)
    x, sn, bu, nr = (np.array(a) for a in (inst.x, inst.seg_nodes, inst.burgers, inst.normal))
    st = _state(inst)
    made = JN.topology_step(x, sn, bu, nr, inst.pinned, 0.0, P, st)
    assert [m[0] for m in made] == [1] and st["missed"] == 1


def test_free_slots_change_nothing():
    """With a zero capture radius the burst of the slotted volume equals the
    plain burst of the volume: free slot segments add exactly zero."""
    base = W.subset(W.burst_instance(1_000_010), 2)
    inst = W.with_junction_slots(base, 3)
    P = JN.Params(capture_radius=0.0, max_break_time=1e-9, l_min=1.0, n_slots=3)
    xj, sn, _, _, rj, log = JN.burst(inst, W.material(), 2, 3, W.DT, P, _state(inst))
    xo, ro, _ = O.burst(base, W.material(), 2, 3, W.DT)
    assert log == []
    assert np.array_equal(xj[:, :base.n_nodes], xo) and np.array_equal(rj, ro)


def test_held_node_stays_put_and_line_bows():
    """A burst of the crossing under stress: the junction node does not move
    while held, and the two halves of the split segment stay attached to it."""
    inst = crossing(d=2.0)
    inst.sigma_app = np.array([0.0, 0.0, 0.0, 3e8, 0.0, 0.0])   # sigma_yz: glide of the screw chain along x
    P = JN.Params(capture_radius=5.0, max_break_time=1.0, l_min=1.0, n_slots=2)
    st = _state(inst)
    x, sn, _, _, r, log = JN.burst(inst, W.material(), 2, 6, W.DT, P, st)
    assert log and log[0][:4] == (0, 2, 0, 6)
    assert list(x[:, 6]) == [30.0, 0.0, 2.0]
    assert sn[1, 2] == 6 and sn[0, 4] == 6
    assert np.abs(x[:, 3] - inst.x[:, 3]).max() > 0.0   # the free nodes moved
