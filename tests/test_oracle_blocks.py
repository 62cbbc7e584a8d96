"""Pins of the block-coupling oracle (oracle/blocks.py) on the CPU: block
averages, the L2 projection onto the block mesh with its two-level
interpolation, and the non-negative-dissipation fix, against closed forms,
invariants and brute force."""
import numpy as np
import pytest

from oracle import blocks as OB


def _trilinear(c, P):
    x, y, z = P[..., 0], P[..., 1], P[..., 2]
    return (c[0] + c[1] * x + c[2] * y + c[3] * z + c[4] * x * y + c[5] * x * z + c[6] * y * z
            + c[7] * x * y * z)


@pytest.mark.parametrize("n,m", [(1, 1), (2, 3), (3, 2)])
def test_average_of_linear_field_is_its_value_at_the_block_centre(n, m):
    B, h = 2.5, 0.7
    P = OB.gauss_points(n, m, B, h)
    f = np.stack([1.0 + 2.0 * P[:, 0] - 3.0 * P[:, 1] + 0.5 * P[:, 2], np.full(len(P), 4.0)], axis=1)
    avg = OB.block_average(f, n, m, B, h)
    for by in range(n):
        for bx in range(n):
            cx, cy, cz = (bx + 0.5) * B, (by + 0.5) * B, 0.5 * h
            np.testing.assert_allclose(avg[by * n + bx], [1 + 2 * cx - 3 * cy + 0.5 * cz, 4.0], rtol=1e-13)


def test_block_averages_integrate_a_quadratic_exactly():
    n, m, B, h = 3, 4, 1.5, 0.4
    P = OB.gauss_points(n, m, B, h)
    avg = OB.block_average((P[:, 0] ** 2)[:, None], n, m, B, h)
    Lx = n * B
    assert avg.sum() * B * B * h == pytest.approx(Lx ** 3 / 3 * Lx * h, rel=1e-13)


def test_two_block_projection_closed_form():
    """Blocks varying in x only: the projection is the 1D L2 projection of a
    two-piece constant onto hat functions.  With 1D mass matrix (B/6)
    [[2,1,0],[1,4,1],[0,1,2]] and load (B/2)[v0, v0+v1, v1] it is
    a0 = (5 v0 - v1)/4, a1 = (v0 + v1)/2, a2 = (5 v1 - v0)/4 (hand solved)."""
    n, B, h = 2, 3.0, 0.5
    v0, v1 = 1.7, -0.4
    f = np.array([[v0], [v1], [v0], [v1]])
    A = OB.l2_projection(f, n, B, h)[:, 0].reshape(2, n + 1, n + 1)   # [k][j][i]
    expect = np.array([(5 * v0 - v1) / 4, (v0 + v1) / 2, (5 * v1 - v0) / 4])
    for k in range(2):
        for j in range(n + 1):
            np.testing.assert_allclose(A[k, j], expect, rtol=1e-13, atol=1e-14)


def test_constant_blocks_project_to_the_constant():
    n, m, B, h = 4, 3, 1.0, 0.3
    f = np.tile([[2.0, -1.0, 0.25]], (n * n, 1))
    g = OB.block_to_gauss(f, n, m, B, h)
    np.testing.assert_allclose(g, np.tile(f[:1], (len(g), 1)), rtol=1e-13)


def test_projection_conserves_the_integral_and_is_z_independent():
    n, B, h = 4, 2.0, 0.5
    rng = np.random.default_rng(1)
    f = rng.normal(size=(n * n, 2))
    A = OB.l2_projection(f, n, B, h)
    nn, conn = OB._block_mesh(n, B, h)
    integral = sum(B * B * h / 8 * A[conn[r]].sum(0) for r in range(n * n))
    np.testing.assert_allclose(integral, f.sum(0) * B * B * h, rtol=1e-12)
    half = (n + 1) * (n + 1)
    np.testing.assert_allclose(A[:half], A[half:], rtol=1e-12, atol=1e-14)


def test_projection_minimises_the_l2_distance():
    n, B, h = 3, 1.0, 1.0
    rng = np.random.default_rng(2)
    f = rng.normal(size=(n * n, 1))
    A = OB.l2_projection(f, n, B, h)
    _, conn = OB._block_mesh(n, B, h)

    def dist(Av):
        tot = 0.0
        for r in range(n * n):
            for gz in range(2):
                for gy in range(2):
                    for gx in range(2):
                        N = OB._shape((2 * gx - 1) * OB.GP, (2 * gy - 1) * OB.GP, (2 * gz - 1) * OB.GP)
                        tot += (B / 2) ** 2 * (h / 2) * (N @ Av[conn[r], 0] - f[r, 0]) ** 2
        return tot

    d0 = dist(A)
    for _ in range(20):
        assert dist(A + 1e-3 * rng.normal(size=A.shape)) > d0


@pytest.mark.parametrize("n,m", [(1, 3), (2, 2), (3, 4)])
def test_two_level_interpolation_reproduces_trilinear_fields(n, m):
    B, h = 1.3, 0.6
    c = np.array([0.3, -1.1, 0.7, 2.0, 0.4, -0.6, 0.9, 0.25])
    nn, _ = OB._block_mesh(n, B, h)
    idx = np.arange(nn)
    i = idx % (n + 1)
    j = (idx // (n + 1)) % (n + 1)
    k = idx // ((n + 1) * (n + 1))
    nodes = np.stack([i * B, j * B, k * h], axis=1)
    g = OB.interpolate(_trilinear(c, nodes)[:, None], n, m, B, h)[:, 0]
    np.testing.assert_allclose(g, _trilinear(c, OB.gauss_points(n, m, B, h)), rtol=1e-12, atol=1e-12)


def _levi_civita():
    e = np.zeros((3, 3, 3))
    e[0, 1, 2] = e[1, 2, 0] = e[2, 0, 1] = 1
    e[0, 2, 1] = e[2, 1, 0] = e[1, 0, 2] = -1
    return e


def test_dissipation_fix_is_the_closest_non_negative_point():
    rng = np.random.default_rng(3)
    ng = 200
    T = rng.normal(size=(ng, 9))
    Lp = rng.normal(size=(ng, 9))
    alpha = rng.normal(size=(ng, 9))
    V = rng.normal(size=(ng, 3))
    L2, V2 = OB.dissipation_fix(T, alpha, Lp, V)
    eps = _levi_civita()
    for g in range(ng):
        Tg, ag = T[g].reshape(3, 3), alpha[g].reshape(3, 3)
        d = np.sum(Tg * Lp[g].reshape(3, 3))
        w = np.einsum("ijk,jr,rk->i", eps, Tg, ag)
        beta = V[g] @ w
        if d >= 0:
            assert np.array_equal(L2[g], Lp[g])
        else:
            assert abs(np.sum(Tg * L2[g].reshape(3, 3))) <= 1e-12 * np.abs(Tg).max() * np.abs(Lp[g]).max() * 9
            # closest point of the half-space {L : T : L >= 0}
            for _ in range(5):
                cand = L2[g] + rng.normal(size=9) * 0.1
                if np.sum(Tg * cand.reshape(3, 3)) >= 0:
                    assert np.linalg.norm(cand - Lp[g]) >= np.linalg.norm(L2[g] - Lp[g]) - 1e-12
        if beta >= 0:
            assert np.array_equal(V2[g], V[g])
        else:
            assert abs(V2[g] @ w) <= 1e-12 * np.linalg.norm(w) * np.linalg.norm(V[g]) * 3
            np.testing.assert_allclose(np.cross(V2[g] - V[g], w), 0, atol=1e-12 * np.linalg.norm(V[g]) * np.linalg.norm(w))


def test_dissipation_fix_zero_stress_changes_nothing():
    Lp = np.arange(9.0)[None]
    V = np.ones((1, 3))
    L2, V2 = OB.dissipation_fix(np.zeros((1, 9)), np.eye(3).reshape(1, 9), Lp, V)
    assert np.array_equal(L2, Lp) and np.array_equal(V2, V)
