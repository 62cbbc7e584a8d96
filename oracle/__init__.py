"""FP64 CPU oracle for the DD pair-force hot path -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product library (``include/dd.h``,
``paper_2005_02498_amd``) never imports, links or calls it, and shares no code
with it: the only common input is the seeded generator in
``paper_2005_02498_amd/workloads.py``, which holds none of the method's
arithmetic.

``ddo.c`` is plain single-threaded C (gcc -O2, no fast-math).  This module
compiles it on first use (or through ``build()``) and wraps it with NumPy.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ddo.c")
_LIB = os.path.join(_HERE, "libddoracle.so")
_LIB_OMP = os.path.join(_HERE, "libddoracle_omp.so")   # the same source with OpenMP over targets
_lib = None
_lib_omp = None
_use_omp = False


class Material(C.Structure):
    _fields_ = [("mu", C.c_double), ("nu", C.c_double), ("a", C.c_double), ("B", C.c_double)]


def _compile(out, extra):
    tmp = out + ".tmp%d" % os.getpid()
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-Wall", "-Wno-unknown-pragmas", "-fPIC", "-shared",
                           *extra, _SRC, "-o", tmp, "-lm"])
    os.replace(tmp, out)


def build(force: bool = True) -> str:
    """Compile ddo.c into libddoracle.so (single-threaded, the oracle) and
    libddoracle_omp.so (the same code with its target loop spread over
    OpenMP threads: identical sums, used only to time the oracle on all host
    cores)."""
    global _lib, _lib_omp
    if force or not os.path.exists(_LIB):
        _compile(_LIB, [])
        _lib = None
    if force or not os.path.exists(_LIB_OMP):
        _compile(_LIB_OMP, ["-fopenmp"])
        _lib_omp = None
    return _LIB


def lib():
    """The single-threaded oracle library (the OpenMP build inside `openmp()`)."""
    global _lib, _lib_omp
    if _use_omp:
        if _lib_omp is None:
            if not os.path.exists(_LIB_OMP) or os.path.getmtime(_LIB_OMP) < os.path.getmtime(_SRC):
                _compile(_LIB_OMP, ["-fopenmp"])
            _lib_omp = C.CDLL(_LIB_OMP)
            _setup(_lib_omp)
        return _lib_omp
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            _compile(_LIB, [])
        _lib = C.CDLL(_LIB)
        _setup(_lib)
    return _lib


class openmp:
    """Context manager: inside, the wrappers below call the OpenMP build of
    the same source (targets in parallel, sums in the same order, so the same
    numbers); used to time the oracle on every host core."""

    def __enter__(self):
        global _use_omp
        _use_omp = True
        return self

    def __exit__(self, *exc):
        global _use_omp
        _use_omp = False


def threads() -> int:
    """Threads the force routines of the current build use."""
    return int(lib().ddo_threads())


_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int32)
_lp = C.POINTER(C.c_int64)
_up = C.POINTER(C.c_uint8)


def _setup(L):
    L.ddo_gauss_legendre.argtypes = [C.c_int, _dp, _dp]
    L.ddo_kernel.argtypes = [_dp, _dp, _dp, C.c_double, C.c_double, C.c_double, _dp]
    L.ddo_kernel.restype = None
    L.ddo_segment_stress.argtypes = [_dp, _dp, _dp, _dp, C.c_double, C.c_double, C.c_double, _dp]
    L.ddo_segment_stress.restype = None
    L.ddo_segment_stress_quad.argtypes = [_dp, _dp, _dp, _dp, C.c_double, C.c_double,
                                          C.c_double, C.c_int, C.c_int, _dp]
    L.ddo_segment_stress_quad.restype = None
    L.ddo_nodal_forces.argtypes = [C.c_int64, _dp, C.c_int64, _ip, _dp, _dp, _dp,
                                   C.POINTER(Material), C.c_int, C.c_int, _dp]
    L.ddo_nodal_forces_sampled.argtypes = [C.c_int64, _dp, C.c_int64, _ip, _dp, _dp,
                                           C.POINTER(Material), C.c_int, C.c_int64,
                                           C.c_int64, _dp]
    L.ddo_segment_end_forces.argtypes = [C.c_int64, _dp, C.c_int64, _ip, _dp, _dp,
                                         C.POINTER(Material), C.c_int, C.c_int64,
                                         C.c_int64, _dp]
    L.ddo_pair_exact.argtypes = [_dp, _dp, _dp, _dp, _dp, _dp, C.c_double, C.c_double,
                                 C.c_double, _dp, _dp]
    L.ddo_set_exact_band.argtypes = [C.c_double]
    L.ddo_set_source_quadrature.argtypes = [C.c_int, C.c_int]
    L.ddo_threads.argtypes = []
    L.ddo_threads.restype = C.c_int
    L.ddo_glide_step.argtypes = [C.c_int64, _dp, _dp, C.c_int64, _ip, _dp, _up,
                                 C.POINTER(Material), C.c_double, _dp]
    L.ddo_fcc_system.argtypes = [C.c_int, _dp, _dp]
    L.ddo_fcc_system.restype = None
    L.ddo_resolved_shear.argtypes = [_dp, _dp]
    L.ddo_resolved_shear.restype = None
    L.ddo_burst.argtypes = [C.c_int64, _dp, C.c_int64, _ip, _dp, _dp, _up, _dp,
                            C.c_double, C.POINTER(Material), C.c_int, C.c_int,
                            C.c_double, _dp, _dp]
    L.ddo_burst_batch.argtypes = [C.c_int32, _lp, _lp, _dp, _ip, _dp, _dp, _up, _dp,
                                  _dp, C.POINTER(Material), C.c_int, C.c_int,
                                  C.c_double, _dp, _dp]


def _d(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(_dp)


def _i(a):
    a = np.ascontiguousarray(a, dtype=np.int32)
    return a, a.ctypes.data_as(_ip)


def _u(a):
    a = np.ascontiguousarray(a, dtype=np.uint8)
    return a, a.ctypes.data_as(_up)


def _l(a):
    a = np.ascontiguousarray(a, dtype=np.int64)
    return a, a.ctypes.data_as(_lp)


def _mat(mu, nu, a, B=1.0):
    return Material(float(mu), float(nu), float(a), float(B))


def _check(rc, what):
    if rc != 0:
        raise ValueError(f"oracle {what} rejected its arguments (rc={rc})")


# --- elementary pieces -------------------------------------------------------

def gauss_legendre(n: int):
    s = np.zeros(n)
    w = np.zeros(n)
    _check(lib().ddo_gauss_legendre(n, s.ctypes.data_as(_dp), w.ctypes.data_as(_dp)), "gauss_legendre")
    return s, w


def kernel(R, b, t, mu, nu, a):
    out = np.zeros(9)
    R, pR = _d(R); b, pb = _d(b); t, pt = _d(t)
    lib().ddo_kernel(pR, pb, pt, mu, nu, a, out.ctypes.data_as(_dp))
    return out.reshape(3, 3)


def segment_stress(x, x1, x2, b, mu, nu, a):
    out = np.zeros(9)
    x, px = _d(x); x1, p1 = _d(x1); x2, p2 = _d(x2); b, pb = _d(b)
    lib().ddo_segment_stress(px, p1, p2, pb, mu, nu, a, out.ctypes.data_as(_dp))
    return out.reshape(3, 3)


def segment_stress_quad(x, x1, x2, b, mu, nu, a, n=64, panels=64):
    out = np.zeros(9)
    x, px = _d(x); x1, p1 = _d(x1); x2, p2 = _d(x2); b, pb = _d(b)
    lib().ddo_segment_stress_quad(px, p1, p2, pb, mu, nu, a, n, panels, out.ctypes.data_as(_dp))
    return out.reshape(3, 3)


def pair_exact(xa, xb, bj, y1, y2, bi, mu, nu, a):
    """(F1, F2): what source y1 -> y2 sends to the two nodes of target xa -> xb,
    with the target integral taken exactly (adaptive quadrature)."""
    F1 = np.zeros(3); F2 = np.zeros(3)
    xa, p0 = _d(xa); xb, p1 = _d(xb); bj, p2 = _d(bj); y1, p3 = _d(y1); y2, p4 = _d(y2); bi, p5 = _d(bi)
    _check(lib().ddo_pair_exact(p0, p1, p2, p3, p4, p5, mu, nu, a, F1.ctypes.data_as(_dp),
                                F2.ctypes.data_as(_dp)), "pair_exact")
    return F1, F2


def set_exact_band(eta: float):
    """Process-wide exact band of every later force call (0 = Q-point rule only)."""
    _check(lib().ddo_set_exact_band(float(eta)), "set_exact_band")


class exact_band:
    """Context manager: the exact band eta inside, 0 again on exit."""

    def __init__(self, eta):
        self.eta = eta

    def __enter__(self):
        set_exact_band(self.eta)
        return self

    def __exit__(self, *exc):
        set_exact_band(0.0)


class source_quadrature:
    """Context manager: inside, the force routines take each source's field by
    n-point Gauss-Legendre quadrature on `panels` equal panels of the source
    instead of the closed form (the slow reference where the closed form's
    endpoint differences lose digits); the closed form again on exit."""

    def __init__(self, n=64, panels=64):
        self.n, self.panels = n, panels

    def __enter__(self):
        _check(lib().ddo_set_source_quadrature(self.n, self.panels), "set_source_quadrature")
        return self

    def __exit__(self, *exc):
        lib().ddo_set_source_quadrature(0, 0)


def fcc_system(alpha: int):
    n = np.zeros(3); m = np.zeros(3)
    lib().ddo_fcc_system(alpha, n.ctypes.data_as(_dp), m.ctypes.data_as(_dp))
    return n, m


def resolved_shear(sigma_voigt):
    s, ps = _d(sigma_voigt)
    out = np.zeros(12)
    lib().ddo_resolved_shear(ps, out.ctypes.data_as(_dp))
    return out


# --- whole-path calls --------------------------------------------------------

def nodal_forces(x, seg_nodes, burgers, sigma_app, mu, nu, a, n_gauss, include_self=False,
                 normal=None):
    x, px = _d(x); sn, psn = _i(seg_nodes); b, pb = _d(burgers); sg, psg = _d(sigma_app)
    nn, ns = x.shape[1], sn.shape[1]
    nrm, pn = _d(normal if normal is not None else np.zeros((3, ns)))
    out = np.zeros((3, nn))
    m = _mat(mu, nu, a)
    _check(lib().ddo_nodal_forces(nn, px, ns, psn, pb, pn, psg, C.byref(m), n_gauss,
                                  int(include_self), out.ctypes.data_as(_dp)), "nodal_forces")
    return out


def nodal_forces_sampled(x, seg_nodes, burgers, sigma_app, mu, nu, a, n_gauss, t0, t1):
    x, px = _d(x); sn, psn = _i(seg_nodes); b, pb = _d(burgers); sg, psg = _d(sigma_app)
    out = np.zeros((3, x.shape[1]))
    m = _mat(mu, nu, a)
    _check(lib().ddo_nodal_forces_sampled(x.shape[1], px, sn.shape[1], psn, pb, psg,
                                          C.byref(m), n_gauss, t0, t1,
                                          out.ctypes.data_as(_dp)), "nodal_forces_sampled")
    return out


def segment_end_forces(x, seg_nodes, burgers, sigma_app, mu, nu, a, n_gauss, t0, t1):
    """[t1-t0][2][3]: what each segment sends to its node 1 and node 2."""
    x, px = _d(x); sn, psn = _i(seg_nodes); b, pb = _d(burgers); sg, psg = _d(sigma_app)
    out = np.zeros((t1 - t0, 2, 3))
    m = _mat(mu, nu, a)
    _check(lib().ddo_segment_end_forces(x.shape[1], px, sn.shape[1], psn, pb, psg,
                                        C.byref(m), n_gauss, t0, t1,
                                        out.ctypes.data_as(_dp)), "segment_end_forces")
    return out


def glide_step(x, force, seg_nodes, normal, pinned, B, dt):
    """Returns (new x, velocities); x is not modified."""
    xn = np.array(x, dtype=np.float64, order="C", copy=True)
    f, pf = _d(force); sn, psn = _i(seg_nodes); nrm, pn = _d(normal)
    pin, pp = _u(pinned if pinned is not None else np.zeros(xn.shape[1], np.uint8))
    v = np.zeros_like(xn)
    m = _mat(1.0, 0.0, 1.0, B)
    _check(lib().ddo_glide_step(xn.shape[1], xn.ctypes.data_as(_dp), pf, sn.shape[1], psn,
                                pn, pp, C.byref(m), dt, v.ctypes.data_as(_dp)), "glide_step")
    return xn, v


def burst(inst, mat, n_gauss, n_steps, dt):
    """One burst of an Instance; returns (x_final, rate_avg[12], features[36])."""
    x = np.array(inst.x, dtype=np.float64, order="C", copy=True)
    sn, psn = _i(inst.seg_nodes); b, pb = _d(inst.burgers); nrm, pn = _d(inst.normal)
    pin, pp = _u(inst.pinned); sg, psg = _d(inst.sigma_app)
    rate = np.zeros(12); feat = np.zeros(36)
    m = _mat(mat["mu"], mat["nu"], mat["a"], mat["B"])
    _check(lib().ddo_burst(x.shape[1], x.ctypes.data_as(_dp), sn.shape[1], psn, pb, pn, pp,
                           psg, float(inst.volume), C.byref(m), n_gauss, n_steps, dt,
                           rate.ctypes.data_as(_dp), feat.ctypes.data_as(_dp)), "burst")
    return x, rate, feat


def burst_batch(batch, mat, n_gauss, n_steps, dt):
    """Packed batch (workloads.Batch); returns (x_final, rates [n][12], features [n][36])."""
    x = np.array(batch.x, dtype=np.float64, order="C", copy=True)
    no, pno = _l(batch.node_off); so, pso = _l(batch.seg_off)
    sn, psn = _i(batch.seg_nodes); b, pb = _d(batch.burgers); nrm, pn = _d(batch.normal)
    pin, pp = _u(batch.pinned); sg, psg = _d(batch.sigma_app); vol, pv = _d(batch.volume)
    n = batch.n_inst
    rate = np.zeros((n, 12)); feat = np.zeros((n, 36))
    m = _mat(mat["mu"], mat["nu"], mat["a"], mat["B"])
    _check(lib().ddo_burst_batch(n, pno, pso, x.ctypes.data_as(_dp), psn, pb, pn, pp, psg, pv,
                                 C.byref(m), n_gauss, n_steps, dt, rate.ctypes.data_as(_dp),
                                 feat.ctypes.data_as(_dp)), "burst_batch")
    return x, rate, feat
