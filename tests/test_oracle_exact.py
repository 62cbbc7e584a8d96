"""Pins of the oracle's exact target integral (oracle.pair_exact) and of the
exact band in its force routines, on the CPU.

The exact integral of a pair is the Q -> infinity limit of the Gauss rule
along the target.  It is pinned against an independent brute-force rule
(uniform composite 16-point Gauss-Legendre, 400 panels, written here in
NumPy), against the mathematics (a closed loop whose pair integrals are all
exact exerts no net force on itself: its energy does not change under a
rigid translation), and against the plain Q-point routine where the band
selects no pair."""
import numpy as np
import pytest

import oracle as O
from paper_2005_02498_amd import workloads as W

MAT = W.material()
MU, NU, A = MAT["mu"], MAT["nu"], MAT["a"]


def _brute(xa, xb, bj, y1, y2, bi, panels=400, n=16):
    s, w = O.gauss_legendre(n)
    d = xb - xa
    L = np.linalg.norm(d)
    t = d / L
    F1 = np.zeros(3)
    F2 = np.zeros(3)
    for p in range(panels):
        for g in range(n):
            u = (p + s[g]) / panels
            f = np.cross(O.segment_stress(xa + u * d, y1, y2, bi, MU, NU, A) @ bj, t)
            F1 += w[g] / panels * (1.0 - u) * L * f
            F2 += w[g] / panels * u * L * f
    return F1, F2


XA = np.array([0.0, 0.0, 0.0])
XB = np.array([50.0, 0.0, 0.0])
BJ = np.array([1.0, 1.0, 0.0]) / np.sqrt(2.0)
BI = np.array([0.0, 1.0, 1.0]) / np.sqrt(2.0)
PAIRS = {
    "adjacent": (XB, np.array([80.0, 30.0, 5.0])),
    "near_crossing": (np.array([20.0, -10.0, 1.5]), np.array([25.0, 10.0, 1.0])),
    "parallel_close": (np.array([-10.0, 3.0, 0.0]), np.array([70.0, 3.0, 0.0])),
    "far": (np.array([300.0, 200.0, 50.0]), np.array([330.0, 210.0, 40.0])),
}


@pytest.mark.parametrize("name", sorted(PAIRS))
def test_pair_exact_matches_brute_force(name):
    y1, y2 = PAIRS[name]
    F1, F2 = O.pair_exact(XA, XB, BJ, y1, y2, BI, MU, NU, A)
    B1, B2 = _brute(XA, XB, BJ, y1, y2, BI)
    scale = max(np.abs(B1).max(), np.abs(B2).max())
    assert scale > 0
    assert np.abs(F1 - B1).max() <= 1e-13 * scale
    assert np.abs(F2 - B2).max() <= 1e-13 * scale


def test_far_pair_exact_equals_16_point_rule():
    """Far from the source the integrand is a low-order polynomial to rounding:
    the 16-point Gauss rule alone is already exact."""
    y1, y2 = PAIRS["far"]
    F1, F2 = O.pair_exact(XA, XB, BJ, y1, y2, BI, MU, NU, A)
    G1, G2 = _brute(XA, XB, BJ, y1, y2, BI, panels=1)
    scale = max(np.abs(G1).max(), np.abs(G2).max())
    assert np.abs(F1 - G1).max() <= 1e-14 * scale
    assert np.abs(F2 - G2).max() <= 1e-14 * scale


def test_straight_segment_exerts_no_net_force_on_itself():
    F1, F2 = O.pair_exact(XA, XB, BJ, XA, XB, BJ, MU, NU, A)
    assert np.abs(F1).max() > 0
    assert np.abs(F1 + F2).max() <= 1e-12 * np.abs(F1).max()


def _random_loop(seed=3, n=32):
    rng = np.random.default_rng(seed)
    ang = np.sort(rng.uniform(0, 2 * np.pi, n))
    R = 300 * (1 + 0.3 * rng.uniform(-1, 1, n))
    x = np.stack([R * np.cos(ang), R * np.sin(ang), 0.2 * R * np.cos(ang) + rng.uniform(-5, 5, n)])
    sn = np.stack([np.arange(n), (np.arange(n) + 1) % n]).astype(np.int32)
    b = np.tile((np.array([1.0, 1.0, 0.0]) / np.sqrt(2.0))[:, None], (1, n))
    return x, sn, b


@pytest.mark.parametrize("include_self", [False, True])
def test_closed_loop_net_self_force_vanishes_when_every_pair_is_exact(include_self):
    """Translation invariance: a closed loop exerts no net force on itself.
    The 2-point rule misses this by several per cent on an irregular loop;
    exact pair integrals restore it to rounding."""
    x, sn, b = _random_loop()
    F_q = O.nodal_forces(x, sn, b, np.zeros(6), MU, NU, A, 2, include_self=include_self)
    with O.exact_band(1e6):
        F_e = O.nodal_forces(x, sn, b, np.zeros(6), MU, NU, A, 2, include_self=include_self)
    ref = np.abs(F_e).sum(1).max()
    assert np.abs(F_q.sum(1)).max() > 1e-2 * np.abs(F_q).sum(1).max()
    assert np.abs(F_e.sum(1)).max() <= 1e-13 * ref


def test_band_selecting_no_pair_is_the_gauss_rule():
    inst = W.config0()
    args = (inst.x, inst.seg_nodes, inst.burgers, inst.sigma_app, MU, NU, A, 2)
    F0 = O.nodal_forces(*args)
    with O.exact_band(1e-6):
        F1 = O.nodal_forces(*args)
    assert np.array_equal(F0, F1)


def test_near_rule_threshold():
    """Two segments: near exactly when their midpoints are closer than
    eta sqrt((L_i^2 + L_j^2) / 2)."""
    L1, L2 = 40.0, 30.0
    x = np.array([[0.0, L1, 100.0, 100.0],
                  [0.0, 0.0, 20.0, 20.0 + L2],
                  [0.0, 0.0, 5.0, 5.0]])
    sn = np.array([[0, 2], [1, 3]], np.int32)
    b = np.tile(BJ[:, None], (1, 2))
    m1 = 0.5 * (x[:, 0] + x[:, 1])
    m2 = 0.5 * (x[:, 2] + x[:, 3])
    eta0 = np.linalg.norm(m1 - m2) / np.sqrt(0.5 * (L1 ** 2 + L2 ** 2))
    args = (x, sn, b, np.zeros(6), MU, NU, A, 2)
    F_q = O.nodal_forces(*args)
    with O.exact_band(1e6):
        F_e = O.nodal_forces(*args)
    assert np.abs(F_e - F_q).max() > 1e-6 * np.abs(F_e).max()
    with O.exact_band(eta0 * (1 - 1e-9)):
        assert np.array_equal(O.nodal_forces(*args), F_q)
    with O.exact_band(eta0 * (1 + 1e-9)):
        assert np.array_equal(O.nodal_forces(*args), F_e)


def test_segment_end_forces_assemble_to_nodal_forces_with_band():
    inst = W.config0()
    with O.exact_band(2.0):
        F = O.nodal_forces(inst.x, inst.seg_nodes, inst.burgers, inst.sigma_app, MU, NU, A, 2)
        E = O.segment_end_forces(inst.x, inst.seg_nodes, inst.burgers, inst.sigma_app, MU, NU, A, 2,
                                 0, inst.n_segs)
    G = np.zeros_like(F)
    for s in range(inst.n_segs):
        G[:, inst.seg_nodes[0, s]] += E[s, 0]
        G[:, inst.seg_nodes[1, s]] += E[s, 1]
    assert np.abs(G - F).max() <= 1e-12 * np.abs(F).max()


def test_band_moves_forces_towards_the_all_exact_result():
    x, sn, b = _random_loop(seed=5)
    args = (x, sn, b, np.zeros(6), MU, NU, A, 2)
    F_q = O.nodal_forces(*args)
    with O.exact_band(2.0):
        F_b = O.nodal_forces(*args)
    with O.exact_band(1e6):
        F_e = O.nodal_forces(*args)
    assert np.abs(F_b - F_e).max() < 0.1 * np.abs(F_q - F_e).max()


def test_invalid_band_rejected():
    for bad in (-1.0, float("nan"), float("inf")):
        with pytest.raises(ValueError):
            O.set_exact_band(bad)
