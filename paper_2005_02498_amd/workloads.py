"""Seeded synthetic inputs: FCC glide-loop ensembles.

This module only *draws* inputs. It holds none of the force, mobility or
slip-rate arithmetic, so that the FP64 CPU oracle (``oracle/``) and the HIP
library can both be fed from it without sharing any of the method's code.

The paper's DD boxes were built by a third-party code from boundary-to-boundary
segments (Sec. "Construction of initial microstructure"); those files are not
available, so closed planar glide loops stand in for them:

* every loop is a regular 32-gon inscribed in a circle of radius R, lying in a
  {111} plane through its centre, first vertex at a random in-plane angle, nodes
  numbered counter-clockwise about the plane normal n (so the line sense t and
  the radial direction r satisfy r x t = +n);
* each loop draws one of the 4 {111} planes, one of the 3 in-plane 1/2<110>
  Burgers directions and a random sign;
* lengths are in units of the Burgers vector magnitude (|b| = 1), the core
  width is a = 1 b, stresses are in Pa, the drag B in Pa s and dt in s.

Material (FCC Cu): mu = 48 GPa, nu = 0.34, |b| = 0.2556 nm, a = 1 b,
B = 1e-4 Pa s.  The paper's table lists mu = 48 GPa and b = 2.55e-10 m.

Array layout (what the C ABI takes): positions ``x`` as SoA ``[3][n_nodes]``
float64, ``seg_nodes`` as ``[2][n_segs]`` int32 (node 1 -> node 2 gives the line
sense), ``burgers`` and ``normal`` as ``[3][n_segs]`` float64, ``pinned`` as
``[n_nodes]`` uint8, ``sigma_app`` as Voigt ``(xx, yy, zz, yz, xz, xy)``.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# ---------------------------------------------------------------------------
# material and run constants
# ---------------------------------------------------------------------------
MU = 48.0e9            # shear modulus, Pa
NU = 0.34              # Poisson ratio
B_SI = 0.2556e-9       # |b| in metres (length unit of every instance)
CORE_A = 1.0           # core width a, in b
DRAG_B = 1.0e-4        # drag coefficient, Pa s
DT = 2.0e-14           # forward-Euler step, s
SEGS_PER_LOOP = 32

# FCC {111} plane normals (crystal frame), and for each the three in-plane
# 1/2<110> directions.  Ordering convention of the 12 slip systems: system
# alpha = 3*p + d for plane p and direction d below.
_PLANES = np.array([[1, 1, 1], [-1, 1, 1], [1, -1, 1], [1, 1, -1]], float)
_DIRS = np.array([
    [[0, 1, -1], [1, 0, -1], [1, -1, 0]],
    [[0, 1, -1], [1, 0, 1], [1, 1, 0]],
    [[0, 1, 1], [1, 0, -1], [1, 1, 0]],
    [[0, 1, 1], [1, 0, 1], [1, -1, 0]],
], float)
PLANE_NORMALS = _PLANES / math.sqrt(3.0)
SLIP_DIRS = _DIRS / math.sqrt(2.0)


@dataclass
class Instance:
    """One DD volume: fixed topology, planar loops."""
    x: np.ndarray            # [3][n_nodes] float64, in b
    seg_nodes: np.ndarray    # [2][n_segs] int32
    burgers: np.ndarray      # [3][n_segs] float64, in b
    normal: np.ndarray       # [3][n_segs] float64, unit
    pinned: np.ndarray       # [n_nodes] uint8
    sigma_app: np.ndarray    # [6] float64 Voigt, Pa
    volume: float            # b^3
    meta: dict = field(default_factory=dict)

    @property
    def n_nodes(self) -> int:
        return int(self.x.shape[1])

    @property
    def n_segs(self) -> int:
        return int(self.seg_nodes.shape[1])


def material() -> dict:
    return {"mu": MU, "nu": NU, "a": CORE_A, "B": DRAG_B}


def _loops(rng, n_loops, box, rmin, rmax, log_radius=False, nseg=SEGS_PER_LOOP):
    """Draw n_loops regular nseg-gons; returns arrays for an Instance."""
    planes = rng.integers(0, 4, n_loops)
    dirs = rng.integers(0, 3, n_loops)
    signs = rng.integers(0, 2, n_loops) * 2 - 1
    if log_radius:
        radii = np.exp(rng.uniform(math.log(rmin), math.log(rmax), n_loops))
    else:
        radii = rng.uniform(rmin, rmax, n_loops)
    centres = rng.uniform(0.0, box, (n_loops, 3))
    phi0 = rng.uniform(0.0, 2.0 * math.pi, n_loops)
    return _loop_geometry(planes, dirs, signs, radii, centres, phi0, nseg)


def _loop_geometry(planes, dirs, signs, radii, centres, phi0, nseg=SEGS_PER_LOOP):
    """Nodes, connectivity, Burgers vectors and normals of the given loops."""
    n_loops = len(planes)
    n_nodes = n_loops * nseg
    k = np.arange(nseg)
    nrm = PLANE_NORMALS[planes]                      # [n_loops][3]
    e1 = SLIP_DIRS[planes, 0]                        # in-plane pair (e1, e2), e1 x e2 = n
    e2 = np.cross(nrm, e1)
    ang = phi0[:, None] + 2.0 * math.pi * k[None, :] / nseg          # [n_loops][nseg]
    pts = centres[:, :, None] + radii[:, None, None] * (np.cos(ang)[:, None, :] * e1[:, :, None]
                                                        + np.sin(ang)[:, None, :] * e2[:, :, None])
    x = np.ascontiguousarray(pts.transpose(1, 0, 2).reshape(3, n_nodes))
    base = (np.arange(n_loops) * nseg)[:, None]
    seg = np.ascontiguousarray(np.stack([(base + k[None, :]).ravel(),
                                         (base + (k[None, :] + 1) % nseg).ravel()]).astype(np.int32))
    bvec = signs[:, None] * SLIP_DIRS[planes, dirs]  # [n_loops][3]
    bur = np.ascontiguousarray(np.repeat(bvec.T, nseg, axis=1))
    nor = np.ascontiguousarray(np.repeat(nrm.T, nseg, axis=1))
    meta = {"planes": planes, "dirs": dirs, "signs": signs, "radii": radii,
            "centres": centres, "phi0": phi0}
    return x, seg, bur, nor, meta


def uniaxial_001(stress_pa: float) -> np.ndarray:
    return np.array([0.0, 0.0, stress_pa, 0.0, 0.0, 0.0])


def volume_instance(seed, n_loops, box, rmin=100.0, rmax=500.0, log_radius=False,
                    sigma_app=None) -> Instance:
    rng = np.random.default_rng(seed)
    x, seg, bur, nor, meta = _loops(rng, n_loops, box, rmin, rmax, log_radius)
    if sigma_app is None:
        sigma_app = uniaxial_001(50.0e6)
    return Instance(x, seg, bur, nor, np.zeros(x.shape[1], np.uint8),
                    np.asarray(sigma_app, float), float(box) ** 3,
                    dict(meta, seed=seed, box=box))


# --- the five workloads ------------------------------------------------------

def config0() -> Instance:
    """8 loops (256 segments) in a 2000 b cube, 50 MPa along [001]."""
    return volume_instance(0, 8, 2000.0)


def config1() -> Instance:
    """512 loops (16,384 segments) in a 10,000 b cube, 50 MPa along [001]."""
    return volume_instance(1, 512, 10000.0)


def config3() -> Instance:
    """8192 loops (262,144 segments), radii log-uniform 50-2000 b, 50,000 b cube."""
    return volume_instance(3, 8192, 50000.0, 50.0, 2000.0, log_radius=True)


def burst_instance(seed, box=2000.0, kmin=8, kmax=128) -> Instance:
    """A PTA-style burst volume: k ~ U{kmin..kmax} loops, a random applied
    stress (6 Voigt entries ~ U[-100, 100] MPa) and a mobile loop fraction
    f ~ U[0.1, 0.9]; the first round(f k) loops are mobile, the others have
    every node pinned (sessile)."""
    rng = np.random.default_rng(seed)
    k = int(rng.integers(kmin, kmax + 1))
    f = float(rng.uniform(0.1, 0.9))
    sig = rng.uniform(-100e6, 100e6, 6)
    x, seg, bur, nor, meta = _loops(rng, k, box, 100.0, 500.0)
    n_mob = int(round(f * k))
    pinned = np.zeros(x.shape[1], np.uint8)
    pinned[n_mob * SEGS_PER_LOOP:] = 1
    return Instance(x, seg, bur, nor, pinned, sig, float(box) ** 3,
                    dict(meta, seed=seed, box=box, k=k, f=f, n_mobile_loops=n_mob))


def config2(n_inst=512, seed0=1_000_000, **kw) -> list[Instance]:
    return [burst_instance(seed0 + i, **kw) for i in range(n_inst)]


@dataclass
class Batch:
    """Instances packed back to back; seg_nodes stay instance-local."""
    node_off: np.ndarray     # [n_inst+1] int64
    seg_off: np.ndarray      # [n_inst+1] int64
    x: np.ndarray            # [3][total nodes]
    seg_nodes: np.ndarray    # [2][total segs] int32, local to the instance
    burgers: np.ndarray
    normal: np.ndarray
    pinned: np.ndarray
    sigma_app: np.ndarray    # [n_inst][6]
    volume: np.ndarray       # [n_inst]

    @property
    def n_inst(self) -> int:
        return int(self.node_off.shape[0] - 1)


def pack(instances: list[Instance]) -> Batch:
    nn = np.array([0] + [i.n_nodes for i in instances], np.int64)
    ns = np.array([0] + [i.n_segs for i in instances], np.int64)
    return Batch(np.cumsum(nn), np.cumsum(ns),
                 np.ascontiguousarray(np.concatenate([i.x for i in instances], 1)),
                 np.ascontiguousarray(np.concatenate([i.seg_nodes for i in instances], 1)),
                 np.ascontiguousarray(np.concatenate([i.burgers for i in instances], 1)),
                 np.ascontiguousarray(np.concatenate([i.normal for i in instances], 1)),
                 np.ascontiguousarray(np.concatenate([i.pinned for i in instances])),
                 np.stack([i.sigma_app for i in instances]),
                 np.array([i.volume for i in instances]))


def subset(inst: Instance, n_loops: int) -> Instance:
    """The first n_loops loops of an instance (for small parity cases)."""
    n = n_loops * SEGS_PER_LOOP
    return Instance(inst.x[:, :n].copy(), inst.seg_nodes[:, :n].copy(),
                    inst.burgers[:, :n].copy(), inst.normal[:, :n].copy(),
                    inst.pinned[:n].copy(), inst.sigma_app.copy(),
                    inst.volume, dict(inst.meta, subset=n_loops))


def surrogate_state(seed) -> Instance:
    """One training/inference state for the slip-rate surrogate: a burst volume
    drawn like ``burst_instance`` from its own seed stream."""
    return burst_instance(seed)


def burst_instance_state(state_seed, micro_seed, box=2000.0, kmin=8, kmax=128) -> Instance:
    """A burst volume whose coarse state and fine microstructure come from two
    seeds.  ``state_seed`` fixes the applied stress, the loop count k, the
    mobile fraction and, per loop, its slip plane, Burgers direction and
    radius: hence the per-system resolved shear stresses and mobile/sessile
    line densities.  ``micro_seed`` draws what those leave free: loop centres,
    first-vertex angles and Burgers-vector signs."""
    rng = np.random.default_rng(state_seed)
    k = int(rng.integers(kmin, kmax + 1))
    f = float(rng.uniform(0.1, 0.9))
    sig = rng.uniform(-100e6, 100e6, 6)
    planes = rng.integers(0, 4, k)
    dirs = rng.integers(0, 3, k)
    radii = rng.uniform(100.0, 500.0, k)
    mrng = np.random.default_rng(micro_seed)
    signs = mrng.integers(0, 2, k) * 2 - 1
    centres = mrng.uniform(0.0, box, (k, 3))
    phi0 = mrng.uniform(0.0, 2.0 * math.pi, k)
    x, seg, bur, nor, meta = _loop_geometry(planes, dirs, signs, radii, centres, phi0)
    n_mob = int(round(f * k))
    pinned = np.zeros(x.shape[1], np.uint8)
    pinned[n_mob * SEGS_PER_LOOP:] = 1
    return Instance(x, seg, bur, nor, pinned, sig, float(box) ** 3,
                    dict(meta, seed=(state_seed, micro_seed), box=box, k=k, f=f, n_mobile_loops=n_mob))


# --- edge-case geometries ------------------------------------------------------

def _unit(v):
    v = np.asarray(v, float)
    return v / np.linalg.norm(v)


def collinear_chains(seed=5, n_targets=24, screw=True) -> Instance:
    """Nearly collinear far pairs: a straight open chain of 16 segments of
    50 b along a <110> line starting at an offset point (screw, b along the
    line, when ``screw``, else a random unit b), and ``n_targets`` short free
    segments (5-20 b, random unit Burgers vectors) placed on the line's
    extension at axial distances log-uniform in [100, 10,000] b beyond either
    end of the chain, 0-2 b off the line, tilted from it by at most 0.01 rad.
    No applied stress: every force comes from nearly collinear pairs."""
    rng = np.random.default_rng(seed)
    u = _unit([1.0, 1.0, 0.0])
    p = _unit(np.cross(u, [0.0, 0.0, 1.0]))         # two directions normal to the line
    q = np.cross(u, p)
    o = np.array([1234.5, -567.75, 910.125])
    n_chain = 16
    xs = [o + 50.0 * k * u for k in range(n_chain + 1)]
    seg = [(k, k + 1) for k in range(n_chain)]
    bc = u if screw else _unit(rng.normal(size=3))
    bur = [bc] * n_chain
    nor = [q] * n_chain
    length = 50.0 * n_chain
    for _ in range(n_targets):
        d = 10.0 ** rng.uniform(2.0, 4.0)
        s = length + d if rng.random() < 0.5 else -d
        off = rng.uniform(0.0, 2.0)
        ang = rng.uniform(0.0, 2.0 * math.pi)
        c = o + s * u + off * (math.cos(ang) * p + math.sin(ang) * q)
        tilt = rng.uniform(0.0, 0.01)
        ta = rng.uniform(0.0, 2.0 * math.pi)
        t = _unit(u + tilt * (math.cos(ta) * p + math.sin(ta) * q))
        L = rng.uniform(5.0, 20.0)
        n0 = len(xs)
        xs += [c - 0.5 * L * t, c + 0.5 * L * t]
        seg.append((n0, n0 + 1))
        bur.append(_unit(rng.normal(size=3)))
        nn = np.cross(t, p)
        nor.append(_unit(nn))
    x = np.ascontiguousarray(np.array(xs).T)
    return Instance(x, np.ascontiguousarray(np.array(seg, np.int32).T),
                    np.ascontiguousarray(np.array(bur).T), np.ascontiguousarray(np.array(nor).T),
                    np.zeros(x.shape[1], np.uint8), np.zeros(6), 1e12, dict(seed=seed, screw=screw))


def long_segment_volume(seed=6, n_small=24) -> Instance:
    """Very long segments: one glide loop of radius 1e5 b (32 segments of
    about 19,600 b) and ``n_small`` loops of radius 100-500 b whose centres lie
    50-500 b from a point of one of its segments (near its middle or near an
    end), same FCC planes and Burgers vectors as the loop workloads; 50 MPa
    along [001]."""
    rng = np.random.default_rng(seed)
    planes = np.concatenate([[0], rng.integers(0, 4, n_small)])
    dirs = np.concatenate([[0], rng.integers(0, 3, n_small)])
    signs = rng.integers(0, 2, n_small + 1) * 2 - 1
    radii = np.concatenate([[1e5], rng.uniform(100.0, 500.0, n_small)])
    phi0 = rng.uniform(0.0, 2.0 * math.pi, n_small + 1)
    big_c = np.array([3.0e4, -2.0e4, 1.0e4])
    n = PLANE_NORMALS[0]
    e1 = SLIP_DIRS[0, 0]
    e2 = np.cross(n, e1)
    centres = [big_c]
    for _ in range(n_small):
        k = int(rng.integers(0, SEGS_PER_LOOP))
        a0 = phi0[0] + 2.0 * math.pi * k / SEGS_PER_LOOP
        a1 = a0 + 2.0 * math.pi / SEGS_PER_LOOP
        pa = big_c + 1e5 * (math.cos(a0) * e1 + math.sin(a0) * e2)
        pb = big_c + 1e5 * (math.cos(a1) * e1 + math.sin(a1) * e2)
        s = rng.choice([rng.uniform(0.4, 0.6), rng.uniform(0.0, 0.05), rng.uniform(0.95, 1.0)])
        dirv = _unit(rng.normal(size=3))
        centres.append(pa + s * (pb - pa) + rng.uniform(50.0, 500.0) * dirv)
    x, seg, bur, nor, meta = _loop_geometry(planes, dirs, signs, radii, np.array(centres), phi0)
    return Instance(x, seg, bur, nor, np.zeros(x.shape[1], np.uint8), uniaxial_001(50.0e6),
                    1e15, dict(meta, seed=seed))


def relabel(inst: Instance, seed=7):
    """The same volume with its segments stored in a random order and its
    nodes renumbered by a random permutation (so that no run of segments is
    stored loop by loop).  Returns (instance, node_map) with node_map[n] the
    new index of old node n: forces on old node n appear at node_map[n]."""
    rng = np.random.default_rng(seed)
    nmap = rng.permutation(inst.n_nodes).astype(np.int64)
    sperm = rng.permutation(inst.n_segs)
    x = np.empty_like(inst.x)
    x[:, nmap] = inst.x
    pinned = np.empty_like(inst.pinned)
    pinned[nmap] = inst.pinned
    seg = np.ascontiguousarray(nmap[inst.seg_nodes[:, sperm]].astype(np.int32))
    return (Instance(x, seg, np.ascontiguousarray(inst.burgers[:, sperm]),
                     np.ascontiguousarray(inst.normal[:, sperm]), pinned, inst.sigma_app.copy(),
                     inst.volume, dict(inst.meta, relabel=seed)), nmap)


def with_junction_slots(inst: Instance, n_slots: int) -> Instance:
    """The instance with room for n_slots junction nodes: after its own nodes,
    n_slots node slots and two dummy nodes D1, D2, all pinned; after its own
    segments, n_slots free segment slots D1 -> D2 with Burgers vector 0 (they
    add no stress, feel no force and belong to no slip system).  D1 lies ten
    box widths off the volume on the x axis and D2 ten b beyond it; the free
    node slots sit at D1."""
    nn, ns = inst.n_nodes, inst.n_segs
    span = float(np.ptp(inst.x)) if nn else 1.0
    d1 = np.array([inst.x[0].min() - 10.0 * max(span, 1.0), 0.0, 0.0])
    d2 = d1 + np.array([10.0, 0.0, 0.0])
    x = np.concatenate([inst.x, np.tile(d1[:, None], (1, n_slots)), d1[:, None], d2[:, None]], axis=1)
    pinned = np.concatenate([np.asarray(inst.pinned, np.uint8), np.ones(n_slots + 2, np.uint8)])
    D1, D2 = nn + n_slots, nn + n_slots + 1
    sn = np.concatenate([inst.seg_nodes, np.tile(np.array([[D1], [D2]], np.int32), (1, n_slots))], axis=1)
    bur = np.concatenate([inst.burgers, np.zeros((3, n_slots))], axis=1)
    nrm = np.concatenate([inst.normal, np.tile(np.array([[0.0], [0.0], [1.0]]), (1, n_slots))], axis=1)
    meta = dict(inst.meta)
    meta["junction_slots"] = n_slots
    return Instance(x=x, seg_nodes=sn.astype(np.int32), burgers=bur, normal=nrm, pinned=pinned,
                    sigma_app=np.array(inst.sigma_app, float), volume=inst.volume, meta=meta)


def junction_forest(seed, n_loops=2, n_chains=4, near=10.0, chain_segs=4, chain_len=150.0, box=2000.0,
                    sigma_app=None) -> Instance:
    """Mobile loops and a forest of sessile lines (straight chains of pinned
    nodes) that pass close to them: chain c runs through a point at distance
    near * U[0.2, 0.8] from the midpoint of a random loop segment, along a
    random direction, so that mobile-sessile approaches closer than `near`
    exist from the start.  Sessile lines carry a random Burgers vector and
    plane of the FCC set.  Stress: uniaxial 200 MPa along [001] unless given."""
    rng = np.random.default_rng(seed)
    x, seg, bur, nor, meta = _loops(rng, n_loops, box, 100.0, 300.0)
    nn, ns = x.shape[1], seg.shape[1]
    xs, sns, bs, ns_ = [x], [seg], [bur], [nor]
    node = nn
    for c in range(n_chains):
        s = int(rng.integers(0, ns))
        a, b = x[:, seg[0, s]], x[:, seg[1, s]]
        m = 0.5 * (a + b)
        t = (b - a) / np.linalg.norm(b - a)
        # a direction not along the segment, and an offset perpendicular to both
        u = rng.normal(size=3)
        u -= u.dot(t) * t
        u /= np.linalg.norm(u)
        w = np.cross(t, u)
        p0 = m + near * rng.uniform(0.2, 0.8) * w
        k = np.arange(chain_segs + 1) - chain_segs / 2.0
        pts = p0[:, None] + (chain_len * k)[None, :] * u[:, None]
        xs.append(pts)
        sns.append(np.stack([np.arange(chain_segs) + node, np.arange(chain_segs) + node + 1]).astype(np.int32))
        pl, di = int(rng.integers(0, 4)), int(rng.integers(0, 3))
        bs.append(np.tile(SLIP_DIRS[pl, di][:, None], (1, chain_segs)))
        ns_.append(np.tile(PLANE_NORMALS[pl][:, None], (1, chain_segs)))
        node += chain_segs + 1
    x = np.concatenate(xs, axis=1)
    pinned = np.zeros(x.shape[1], np.uint8)
    pinned[nn:] = 1
    sig = uniaxial_001(200e6) if sigma_app is None else np.asarray(sigma_app, float)
    return Instance(x=np.ascontiguousarray(x), seg_nodes=np.ascontiguousarray(np.concatenate(sns, axis=1)),
                    burgers=np.ascontiguousarray(np.concatenate(bs, axis=1)),
                    normal=np.ascontiguousarray(np.concatenate(ns_, axis=1)), pinned=pinned, sigma_app=sig,
                    volume=box ** 3, meta=meta)
