"""FP64 oracle of bursts with junctions and their thermally activated
breaking -- TEST INFRASTRUCTURE ONLY (imported by tests/, never by the product
library).

Sec. "Thermal activation": mobile dislocations that meet sessile ones form
junctions, which hold them until they break; the breaking time is t_b = f a
(Eq. tb) with f uniform in [0, 1) and a the maximum breaking time.  Readings
taken here (the paper gives the rule, not the DD code's mechanics):
  * a junction forms when a mobile node (not pinned) comes closer than the
    capture radius r_c to a sessile segment (both its nodes pinned) of its own
    volume; the node is then held fixed, no node is inserted;
  * the checks run at the start of every step, at time t_k = t0 + k dt, in
    this order: a held node whose release time has come is released (and
    does not look for a new junction in that step); a free node first forgets
    the segment it last broke from once it is farther than 2 r_c from it, then
    takes the first sessile segment in index order, other than that one,
    closer than r_c;
  * at formation release = t_k + f a with f = fractions[node, count mod K]
    (the caller's uniform numbers, K per node) and count = the node's number
    of junctions so far.
The per-node state (junction segment or -1, release time, ignored segment or
-1, count) is carried in and out.  Distances are computed in this order of
operations (no fused multiply-adds) so that decisions are reproducible.
"""
from __future__ import annotations

import copy

import numpy as np

import oracle as O


def _dist2(p, a, b):
    d0, d1, d2 = b[0] - a[0], b[1] - a[1], b[2] - a[2]
    w0, w1, w2 = p[0] - a[0], p[1] - a[1], p[2] - a[2]
    dd = d0 * d0 + d1 * d1 + d2 * d2
    t = (w0 * d0 + w1 * d1 + w2 * d2) / dd
    t = min(max(t, 0.0), 1.0)
    e0 = p[0] - (a[0] + t * d0)
    e1 = p[1] - (a[1] + t * d1)
    e2 = p[2] - (a[2] + t * d2)
    return e0 * e0 + e1 * e1 + e2 * e2


def update(x, seg_nodes, pinned, t, r_c, a_max, fractions, state):
    """Junction checks of one volume at time t (positions x [3][nn]).  Returns
    the held-node mask; `state` (dict of arrays junction, release, ignore,
    count, per node) is updated in place."""
    nn = x.shape[1]
    ns = seg_nodes.shape[1]
    K = fractions.shape[1]
    sessile = [bool(pinned[seg_nodes[0, s]]) and bool(pinned[seg_nodes[1, s]]) for s in range(ns)]
    held = np.zeros(nn, np.uint8)
    rc2, rf2 = r_c * r_c, (2.0 * r_c) * (2.0 * r_c)
    for n in range(nn):
        if pinned[n]:
            continue
        js = int(state["junction"][n])
        if js >= 0:
            if t >= state["release"][n]:
                state["ignore"][n] = js
                state["junction"][n] = -1
            else:
                held[n] = 1
            continue
        p = x[:, n]
        ig = int(state["ignore"][n])
        if ig >= 0 and _dist2(p, x[:, seg_nodes[0, ig]], x[:, seg_nodes[1, ig]]) > rf2:
            ig = -1
            state["ignore"][n] = -1
        for s in range(ns):
            if not sessile[s] or s == ig:
                continue
            if _dist2(p, x[:, seg_nodes[0, s]], x[:, seg_nodes[1, s]]) < rc2:
                c = int(state["count"][n])
                f = float(fractions[n, c % K])
                state["junction"][n] = s
                state["release"][n] = t + f * a_max
                state["count"][n] = c + 1
                held[n] = 1
                break
    return held


def new_state(nn):
    return {"junction": np.full(nn, -1, np.int64), "release": np.zeros(nn),
            "ignore": np.full(nn, -1, np.int64), "count": np.zeros(nn, np.int64)}


def burst(inst, mat, Q, n_steps, dt, r_c, a_max, t0, fractions, state):
    """A burst of one volume with junctions: per step the junction checks,
    then one glide step with the held nodes fixed (the oracle's plain burst
    routine with them added to the pinned set).  Returns (x, rate_avg[12])."""
    x = np.array(inst.x, float)
    acc = np.zeros(12)
    for k in range(n_steps):
        t = t0 + k * dt
        held = update(x, inst.seg_nodes, inst.pinned, t, r_c, a_max, fractions, state)
        s = copy.copy(inst)
        s.x = x
        s.pinned = np.maximum(np.asarray(inst.pinned, np.uint8), held)
        x, rate, _ = O.burst(s, mat, Q, 1, dt)
        acc += rate
    return x, acc / max(n_steps, 1)
