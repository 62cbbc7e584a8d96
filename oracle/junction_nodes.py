"""FP64 oracle of bursts with junction nodes -- TEST INFRASTRUCTURE ONLY
(imported by tests/, never by the product library).

Sec. "Thermal activation": a mobile dislocation that meets a sessile one forms
a junction at their intersection, which holds it until the junction breaks
after t_b = f a (Eq. tb, f uniform in [0, 1), a the maximum breaking time);
meanwhile the mobile line bows around the junction point.  Readings taken
here (the paper states the rule, not the DD code's mechanics):
  * the junction point is the mobile segment's point of closest approach to
    a sessile segment (both of its nodes pinned, of the same volume), when
    the two segments come closer than the capture radius r_c; a pinned node
    is inserted there, splitting the mobile segment a -> b into a -> j and
    j -> b (same Burgers vector and slip plane);
  * the inserted node keeps at least l_min from both ends (its parameter on
    the segment is clamped to [l_min / L, 1 - l_min / L]); a segment no longer
    than 2 l_min forms no junction;
  * a segment forms no junction while it is within 2 r_c of the point of its
    last junction (point-to-segment distance): both halves of a split get the
    junction point, so they are never captured while the node holds them
    (junctions do not nest), and at release the node is removed (its
    in-segment takes the out-segment's end node) and the merged segment keeps
    the point until it has moved 2 r_c away from it;
  * every step, at time t_k = t0 + k dt, in this order: releases (node slots
    in index order, t_k >= release time), then captures found on the
    positions at the start of the step (one per mobile segment, the first
    sessile segment in index order), applied in
    segment index order; a capture needs a free node slot and a free segment
    slot (the lowest of each); without one it is not made and counted as
    missed;
  * f = fractions[count mod K], count = the volume's number of junctions so
    far.
Slots.  A volume with K junction slots has, after its own nodes and
segments, K node slots and two dummy nodes D1, D2 (all pinned), and K segment
slots; a free segment slot is D1 -> D2 with Burgers vector 0 (it adds no
stress, feels no force and belongs to no slip system).  Distances and the
junction point are computed in the order written, without fused multiply-
adds, so that the GPU path can take the same decisions.
"""
from __future__ import annotations

import copy
import math

import numpy as np

import oracle as O


def segment_closest(p, p2, q, q2):
    """Closest approach of the segments p -> p2 and q -> q2: (squared
    distance, parameter u on the first).  Clamped closest points of two
    lines: with d1 = p2 - p, d2 = q2 - q, r = p - q, the unclamped parameter
    on the first line is (b f - c e) / (a e - b^2) (a = d1.d1, b = d1.d2,
    c = d1.r, e = d2.d2, f = d2.r); it is clamped to [0, 1], the second
    parameter v = (b u + f) / e follows, and when v leaves [0, 1] it is
    clamped and u recomputed for that end of the second segment."""
    d10, d11, d12 = p2[0] - p[0], p2[1] - p[1], p2[2] - p[2]
    d20, d21, d22 = q2[0] - q[0], q2[1] - q[1], q2[2] - q[2]
    r0, r1, r2 = p[0] - q[0], p[1] - q[1], p[2] - q[2]
    a = d10 * d10 + d11 * d11 + d12 * d12
    e = d20 * d20 + d21 * d21 + d22 * d22
    f = d20 * r0 + d21 * r1 + d22 * r2
    c = d10 * r0 + d11 * r1 + d12 * r2
    b = d10 * d20 + d11 * d21 + d12 * d22
    den = a * e - b * b
    u = min(max((b * f - c * e) / den, 0.0), 1.0) if den > 0.0 else 0.0
    v = (b * u + f) / e
    if v < 0.0:
        v = 0.0
        u = min(max(-c / a, 0.0), 1.0)
    elif v > 1.0:
        v = 1.0
        u = min(max((b - c) / a, 0.0), 1.0)
    w0 = (p[0] + u * d10) - (q[0] + v * d20)
    w1 = (p[1] + u * d11) - (q[1] + v * d21)
    w2 = (p[2] + u * d12) - (q[2] + v * d22)
    return w0 * w0 + w1 * w1 + w2 * w2, u


class Params:
    def __init__(self, capture_radius, max_break_time, l_min, n_slots, t0=0.0):
        self.rc, self.a, self.l_min, self.K, self.t0 = capture_radius, max_break_time, l_min, n_slots, t0


def point_segment_d2(p, a, b):
    """Squared distance from p to the segment a -> b (the clamped projection)."""
    d0, d1, d2 = b[0] - a[0], b[1] - a[1], b[2] - a[2]
    w0, w1, w2 = p[0] - a[0], p[1] - a[1], p[2] - a[2]
    dd = d0 * d0 + d1 * d1 + d2 * d2
    t = min(max((w0 * d0 + w1 * d1 + w2 * d2) / dd, 0.0), 1.0)
    e0 = p[0] - (a[0] + t * d0)
    e1 = p[1] - (a[1] + t * d1)
    e2 = p[2] - (a[2] + t * d2)
    return e0 * e0 + e1 * e1 + e2 * e2


def new_state(nn, ns, fractions):
    """Per node: release time and the sessile segment of an active junction
    node (-1: none); per segment: whether it keeps a junction point and the
    point [3][ns]; the volume's junction count and missed captures; its
    fractions [Kf]."""
    return {"release": np.zeros(nn), "ses": np.full(nn, -1, np.int64), "ignore": np.zeros(ns, bool),
            "point": np.zeros((3, ns)), "count": 0, "missed": 0, "fractions": np.asarray(fractions, float)}


def _layout(nn, ns, K):
    return nn - K - 2, nn - 2, nn - 1, ns - K   # first node slot, D1, D2, first segment slot


def topology_step(x, sn, bur, nrm, pinned, t, P: Params, st):
    """Releases and captures of one volume at time t (arrays changed in
    place: x [3][nn], sn [2][ns] local node indices, bur, nrm [3][ns]).
    Returns the list of captures made, (segment, sessile, node, new segment)."""
    nn, ns = x.shape[1], sn.shape[1]
    n0, d1, d2, s0 = _layout(nn, ns, P.K)
    rc2, rf2 = P.rc * P.rc, (2.0 * P.rc) * (2.0 * P.rc)
    # releases, node slots in index order
    for j in range(n0, n0 + P.K):
        if st["ses"][j] >= 0 and t >= st["release"][j]:
            s_in = int(np.nonzero(sn[1] == j)[0][0])
            s_out = int(np.nonzero(sn[0] == j)[0][0])
            sn[1, s_in] = sn[1, s_out]
            sn[0, s_out], sn[1, s_out] = d1, d2
            bur[:, s_out] = 0.0
            nrm[:, s_out] = (0.0, 0.0, 1.0)
            st["ignore"][s_in] = True
            st["point"][:, s_in] = x[:, j]
            st["ignore"][s_out] = False
            st["ses"][j] = -1
    # candidates on the positions at the start of the step
    def free_seg(s):
        return sn[0, s] == d1 and sn[1, s] == d2

    def sessile(s):
        a, b = sn[0, s], sn[1, s]
        return s < s0 and a < n0 and b < n0 and bool(pinned[a]) and bool(pinned[b])

    ses = [s for s in range(ns) if sessile(s)]
    cand = []
    for s in range(ns):
        if free_seg(s) or sessile(s):
            continue
        p, p2 = x[:, sn[0, s]], x[:, sn[1, s]]
        if st["ignore"][s]:
            if point_segment_d2(st["point"][:, s], p, p2) > rf2:
                st["ignore"][s] = False
            else:
                continue
        for k in ses:
            dd2, u = segment_closest(p, p2, x[:, sn[0, k]], x[:, sn[1, k]])
            if dd2 < rc2:
                cand.append((s, k, u))
                break
    # captures, in segment index order
    made = []
    for s, k, u in cand:
        a, b = int(sn[0, s]), int(sn[1, s])
        e0, e1, e2 = x[0, b] - x[0, a], x[1, b] - x[1, a], x[2, b] - x[2, a]
        L = math.sqrt(e0 * e0 + e1 * e1 + e2 * e2)
        if not (L > 2.0 * P.l_min):
            continue
        u = min(max(u, P.l_min / L), 1.0 - P.l_min / L)
        free_n = [j for j in range(n0, n0 + P.K) if st["ses"][j] < 0]
        free_s = [q for q in range(s0, ns) if free_seg(q)]
        if not free_n or not free_s:
            st["missed"] += 1
            continue
        j, s2 = free_n[0], free_s[0]
        x[0, j] = x[0, a] + u * e0
        x[1, j] = x[1, a] + u * e1
        x[2, j] = x[2, a] + u * e2
        sn[1, s] = j
        sn[0, s2], sn[1, s2] = j, b
        bur[:, s2] = bur[:, s]
        nrm[:, s2] = nrm[:, s]
        st["ignore"][s] = True
        st["ignore"][s2] = True
        st["point"][:, s] = x[:, j]
        st["point"][:, s2] = x[:, j]
        c = int(st["count"])
        st["release"][j] = t + st["fractions"][c % len(st["fractions"])] * P.a
        st["ses"][j] = k
        st["count"] = c + 1
        made.append((s, k, j, s2))
    return made


def burst(inst, mat, Q, n_steps, dt, P: Params, st):
    """A burst of one volume with junction nodes: per step the topology step,
    then one glide step of the oracle's plain burst routine on the current
    topology.  The instance's arrays are not changed; returns (x, seg_nodes,
    burgers, normal, rate_avg[12], captures [(step, s, k, j, s2)])."""
    x = np.array(inst.x, float)
    sn = np.array(inst.seg_nodes, np.int32)
    bur = np.array(inst.burgers, float)
    nrm = np.array(inst.normal, float)
    acc = np.zeros(12)
    log = []
    for k in range(n_steps):
        t = P.t0 + k * dt
        for c in topology_step(x, sn, bur, nrm, inst.pinned, t, P, st):
            log.append((k,) + c)
        s = copy.copy(inst)
        s.x, s.seg_nodes, s.burgers, s.normal = x, sn, bur, nrm
        x, rate, _ = O.burst(s, mat, Q, 1, dt)
        acc += rate
    return x, sn, bur, nrm, acc / max(n_steps, 1), log
