"""GPU parity of the block coupling (dd_block_average, dd_block_to_gauss,
dd_dissipation_fix) against the FP64 oracle (oracle/blocks.py), which
assembles the block mesh's mass matrix and solves it densely where the GPU
uses separable tridiagonal solves.  Tolerance 1e-12 relative to the field's
largest value."""
import numpy as np
import pytest
import torch

from oracle import blocks as OB
import paper_2005_02498_amd as dd

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def _t(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device=DEV)


@pytest.mark.parametrize("n,m,c", [(1, 1, 1), (3, 4, 9), (5, 10, 3)])
def test_block_average(n, m, c):
    B, h = 2.0, 0.5
    rng = np.random.default_rng(n * 100 + m)
    f = rng.normal(size=((n * m) ** 2 * 8, c))
    got = dd.dd_block_average(_t(f), n, m, B, h).cpu().numpy()
    ref = OB.block_average(f, n, m, B, h)
    assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max()


@pytest.mark.parametrize("n,m,c", [(1, 1, 1), (2, 3, 3), (5, 10, 9), (7, 3, 16)])
def test_block_to_gauss(n, m, c):
    B, h = 1.7, 0.4
    rng = np.random.default_rng(n * 10 + m)
    fb = rng.normal(size=(n * n, c))
    got = dd.dd_block_to_gauss(_t(fb), n, m, B, h).cpu().numpy()
    ref = OB.block_to_gauss(fb, n, m, B, h)
    e = np.abs(got - ref).max() / np.abs(ref).max()
    print(f"n={n} m={m} c={c}: err {e:.2e}")
    assert e <= 1e-12


def test_block_to_gauss_large_sampled():
    """A 30 x 30 block mesh with 40 x 40 elements per block (1.44 million
    elements, 11.5 million Gauss points): constant blocks give the constant
    everywhere, and random blocks match the oracle on a sample of elements."""
    n, m, B, h = 30, 40, 1.0, 0.25
    ngp = (n * m) ** 2 * 8
    const = dd.dd_block_to_gauss(_t(np.full((n * n, 2), [3.5, -1.25])), n, m, B, h).cpu().numpy()
    np.testing.assert_allclose(const, np.tile([3.5, -1.25], (ngp, 1)), rtol=1e-12)
    rng = np.random.default_rng(9)
    fb = rng.normal(size=(n * n, 1))
    got = dd.dd_block_to_gauss(_t(fb), n, m, B, h).cpu().numpy()
    A = OB.l2_projection(fb, n, B, h)
    els = rng.integers(0, (n * m) ** 2, size=300)
    ref = OB.interpolate(A, n, m, B, h, elements=els)
    idx = (8 * els[:, None] + np.arange(8)[None]).ravel()
    e = np.abs(got[idx] - ref).max() / np.abs(ref).max()
    print(f"large sampled err {e:.2e}")
    assert e <= 1e-11


def test_dissipation_fix():
    rng = np.random.default_rng(4)
    ng = 20000
    T = rng.normal(size=(ng, 9))
    T[:50] = 0.0
    alpha = rng.normal(size=(ng, 9))
    Lp = rng.normal(size=(ng, 9))
    V = rng.normal(size=(ng, 3))
    L_ref, V_ref = OB.dissipation_fix(T, alpha, Lp, V)
    Lg, Vg = _t(Lp), _t(V)
    dd.dd_dissipation_fix(_t(T), _t(alpha), Lg, Vg)
    Lg, Vg = Lg.cpu().numpy(), Vg.cpu().numpy()
    assert np.abs(Lg - L_ref).max() <= 1e-13 * np.abs(L_ref).max()
    assert np.abs(Vg - V_ref).max() <= 1e-13 * np.abs(V_ref).max()
    unchanged = np.all(L_ref == Lp, axis=1)
    assert unchanged.sum() > 1000 and np.array_equal(Lg[unchanged], Lp[unchanged])
    # only Lp
    Lg2 = _t(Lp)
    dd.dd_dissipation_fix(_t(T), None, Lg2, None)
    assert np.abs(Lg2.cpu().numpy() - L_ref).max() <= 1e-13 * np.abs(L_ref).max()
