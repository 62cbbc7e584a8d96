"""The seeded generator (CPU only): reproducible, planar loops, in-plane
Burgers vectors, sizes of the five workloads."""
import math

import numpy as np
import pytest

from paper_2005_02498_amd import workloads as W


def test_fcc_tables():
    assert W.PLANE_NORMALS.shape == (4, 3) and W.SLIP_DIRS.shape == (4, 3, 3)
    for p in range(4):
        for d in range(3):
            assert abs(W.PLANE_NORMALS[p] @ W.SLIP_DIRS[p, d]) < 1e-15
            assert abs(np.linalg.norm(W.SLIP_DIRS[p, d]) - 1) < 1e-15


def test_config0_shape_and_geometry():
    c = W.config0()
    assert c.n_nodes == 256 and c.n_segs == 256
    assert c.x.dtype == np.float64 and c.seg_nodes.dtype == np.int32
    for l in range(8):
        sl = slice(32 * l, 32 * l + 32)
        n = c.normal[:, 32 * l]
        pts = c.x[:, sl]
        cen = pts.mean(1)
        assert np.abs(n @ (pts - cen[:, None])).max() < 1e-9          # planar
        assert np.abs(n @ c.burgers[:, sl]).max() < 1e-15            # b in plane
        np.testing.assert_allclose(np.linalg.norm(c.burgers[:, sl], axis=0), 1.0)
        r = np.linalg.norm(pts - cen[:, None], axis=0)
        assert 100 <= r[0] <= 500 and np.ptp(r) < 1e-9
        # counter-clockwise about n: (x_k - c) x t_k . n > 0
        t = c.x[:, c.seg_nodes[1, sl]] - c.x[:, c.seg_nodes[0, sl]]
        assert np.all(np.einsum("ij,ij->j", np.cross(pts - cen[:, None], t, axis=0), n[:, None] * np.ones(32)) > 0)
    assert np.all((c.x >= -500) & (c.x <= 2500))
    assert c.sigma_app[2] == 50e6 and np.count_nonzero(c.sigma_app) == 1


def test_reproducible():
    a, b = W.config0(), W.config0()
    np.testing.assert_array_equal(a.x, b.x)
    np.testing.assert_array_equal(a.burgers, b.burgers)
    c = W.burst_instance(1_000_007)
    d = W.burst_instance(1_000_007)
    np.testing.assert_array_equal(c.x, d.x)
    np.testing.assert_array_equal(c.sigma_app, d.sigma_app)


def test_burst_instance_ranges():
    for i in range(20):
        c = W.burst_instance(1_000_000 + i)
        k = c.meta["k"]
        assert 8 <= k <= 128 and c.n_segs == 32 * k
        assert 0.1 <= c.meta["f"] <= 0.9
        assert np.all(np.abs(c.sigma_app) <= 100e6)
        nm = c.meta["n_mobile_loops"]
        assert c.pinned[:32 * nm].sum() == 0 and np.all(c.pinned[32 * nm:] == 1)
        assert c.volume == 2000.0 ** 3


def test_pack_offsets():
    insts = [W.burst_instance(1_000_000 + i) for i in range(4)]
    b = W.pack(insts)
    assert b.node_off[0] == 0 and b.node_off[-1] == sum(i.n_nodes for i in insts)
    for i, inst in enumerate(insts):
        np.testing.assert_array_equal(b.x[:, b.node_off[i]:b.node_off[i + 1]], inst.x)
        np.testing.assert_array_equal(b.seg_nodes[:, b.seg_off[i]:b.seg_off[i + 1]], inst.seg_nodes)


def test_config1_config3_sizes():
    c1 = W.config1()
    assert c1.n_segs == 16384 and c1.volume == 1e12
    c3 = W.config3()
    assert c3.n_segs == 262144
    r = c3.meta["radii"]
    assert r.min() >= 50 and r.max() <= 2000
