"""Python binding of libdd.so: argument marshalling only.

Every function here has the name of the C entry point it wraps
(``include/dd.h``) and takes PyTorch-ROCm tensors that already live on the GPU;
it checks dtype, device, contiguity and shapes, passes raw device pointers and
the current HIP stream to the library, and raises ``DDError`` on a non-zero
return code.  No arithmetic of the method happens in Python and there is no
CPU fallback: if ``libdd.so`` is missing, importing the binding's functions
raises.
"""
from __future__ import annotations

import ctypes as C
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdd.so")

DD_FP64, DD_MIXED = 0, 1
DD_OK, DD_EINVAL, DD_EHIP, DD_ENOMEM, DD_ENONFINITE, DD_ECAPACITY, DD_EIO = 0, -1, -2, -3, -4, -5, -6
N_SYSTEMS, N_FEATURES = 12, 36
MLP_IN, MLP_HIDDEN, MLP_OUT, MLP_PARAMS = 36, 256, 12, 144140

EXPORTS = [
    "dd_last_error", "dd_version", "dd_set_validation", "dd_shutdown",
    "dd_timing_enable", "dd_timing_read", "dd_vector_peak", "dd_set_autotune", "dd_set_burst_mode", "dd_check", "dd_set_plan", "dd_last_plan",
    "dd_nodal_forces", "dd_nodal_forces_noalloc", "dd_glide_step", "dd_step", "dd_burst_batch", "dd_burst_batch_junctions", "dd_burst_batch_junction_nodes", "dd_pta_step", "dd_pta_step_junctions", "dd_pta_step_junction_nodes",
    "dd_block_average", "dd_block_to_gauss", "dd_dissipation_fix",
    "dd_mlp_create", "dd_mlp_destroy", "dd_mlp_set_params", "dd_mlp_get_params", "dd_mlp_save", "dd_mlp_load", "dd_mlp_info",
    "dd_mlp_set_scaling", "dd_mlp_set_log_densities", "dd_mlp_set_spread_floor", "dd_mlp_train_step", "dd_mlp_gradients",
    "dd_surrogate_rates",
]


class DDError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libdd error {code}: {msg}")
        self.code = code


class BlockMesh(C.Structure):
    """n x n blocks of side B and thickness h, each meshed by m x m x 1 elements (dd.h)."""
    _fields_ = [("n", C.c_int32), ("m", C.c_int32), ("B", C.c_double), ("h", C.c_double)]


class Junctions(C.Structure):
    """dd_junctions of dd.h (device pointers as integers)."""
    _fields_ = [("capture_radius", C.c_double), ("max_break_time", C.c_double), ("t0", C.c_double),
                ("n_fractions", C.c_int32), ("fractions", C.c_void_p), ("junction", C.c_void_p),
                ("release", C.c_void_p), ("ignore", C.c_void_p), ("count", C.c_void_p)]


class JunctionNodes(C.Structure):
    """dd_junction_nodes of dd.h (device pointers as integers)."""
    _fields_ = [("capture_radius", C.c_double), ("max_break_time", C.c_double), ("t0", C.c_double),
                ("min_length", C.c_double), ("n_slots", C.c_int32), ("n_fractions", C.c_int32),
                ("fractions", C.c_void_p), ("release", C.c_void_p), ("ses", C.c_void_p), ("ignore", C.c_void_p),
                ("point", C.c_void_p), ("count", C.c_void_p), ("missed", C.c_void_p)]


class Material(C.Structure):
    _fields_ = [("mu", C.c_double), ("nu", C.c_double), ("a", C.c_double), ("B", C.c_double)]


class PTAParams(C.Structure):
    """dd_pta_params (see dd.h); the paper's values are the defaults where it gives them."""
    _fields_ = [("dt", C.c_double), ("chunk_steps", C.c_int32), ("max_chunks", C.c_int32),
                ("tol_rho", C.c_double), ("tol_lp", C.c_double), ("lpdot_max", C.c_double),
                ("delta", C.c_double), ("strain_step", C.c_double), ("h_max", C.c_double),
                ("max_jumps", C.c_int32)]

    def __init__(self, dt, chunk_steps=10, max_chunks=20, tol_rho=1e-2, tol_lp=3e-2, lpdot_max=0.05,
                 delta=0.1, strain_step=0.002, h_max=1.0, max_jumps=2):
        super().__init__(dt, chunk_steps, max_chunks, tol_rho, tol_lp, lpdot_max, delta, strain_step,
                         h_max, max_jumps)


DD_PTA_OUT = 64


_lib = None


def lib():
    """The loaded libdd.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_2005_02498_amd.build` (no CPU fallback exists)")
        L = C.CDLL(LIB_PATH)
        _declare(L)
        _lib = L
    return _lib


def _declare(L):
    i64, i32, vp, dbl = C.c_int64, C.c_int32, C.c_void_p, C.c_double
    fp = C.POINTER(C.c_float)
    sig = {
        "dd_last_error": (C.c_char_p, []),
        "dd_version": (C.c_int, []),
        "dd_set_validation": (C.c_int, [C.c_int]),
        "dd_shutdown": (C.c_int, []),
        "dd_timing_enable": (C.c_int, [C.c_int]),
        "dd_set_autotune": (C.c_int, [C.c_int]),
        "dd_set_burst_mode": (C.c_int, [C.c_int]),
        "dd_last_plan": (C.c_int, [C.POINTER(C.c_int64), C.POINTER(C.c_int64), C.POINTER(C.c_int)]),
        "dd_timing_read": (C.c_int, [C.POINTER(C.c_double), C.POINTER(C.c_int64),
                                     C.POINTER(C.c_int64), C.POINTER(C.c_int64), C.c_int]),
        "dd_vector_peak": (C.c_int, [C.c_int, C.c_int, C.POINTER(C.c_double), vp]),
        "dd_pta_step": (C.c_int, [C.c_int32, C.POINTER(C.c_int64), C.POINTER(C.c_int64), vp, vp, vp, vp,
                                  vp, vp, C.POINTER(C.c_double), C.POINTER(C.c_double),
                                  C.POINTER(PTAParams), C.POINTER(Material), C.c_int, C.c_int, dbl, dbl,
                                  C.POINTER(C.c_double), vp]),
        "dd_pta_step_junctions": (C.c_int, [C.c_int32, C.POINTER(C.c_int64), C.POINTER(C.c_int64), vp, vp, vp,
                                            vp, vp, vp, C.POINTER(C.c_double), C.POINTER(C.c_double),
                                            C.POINTER(PTAParams), C.POINTER(Material), C.c_int, C.c_int, dbl,
                                            dbl, C.POINTER(Junctions), C.POINTER(C.c_int64),
                                            C.POINTER(C.c_double), vp]),
        "dd_pta_step_junction_nodes": (C.c_int, [C.c_int32, C.POINTER(C.c_int64), C.POINTER(C.c_int64), vp, vp,
                                                 vp, vp, vp, vp, C.POINTER(C.c_double), C.POINTER(C.c_double),
                                                 C.POINTER(PTAParams), C.POINTER(Material), C.c_int, C.c_int, dbl,
                                                 C.POINTER(JunctionNodes), C.POINTER(C.c_int64),
                                                 C.POINTER(C.c_double), vp]),
        "dd_set_plan": (C.c_int, [i64, C.c_int]),
        "dd_check": (C.c_int, [vp]),
        "dd_block_average": (C.c_int, [C.POINTER(BlockMesh), C.c_int, vp, vp, vp]),
        "dd_block_to_gauss": (C.c_int, [C.POINTER(BlockMesh), C.c_int, vp, vp, vp]),
        "dd_dissipation_fix": (C.c_int, [i64, vp, vp, vp, vp, vp]),
        "dd_nodal_forces": (C.c_int, [i64, vp, i64, vp, vp, vp, C.POINTER(C.c_double),
                                      C.POINTER(Material), C.c_int, C.c_int, dbl, dbl, vp, vp]),
        "dd_nodal_forces_noalloc": (C.c_int, [i64, vp, i64, vp, vp, vp, C.POINTER(C.c_double),
                                              C.POINTER(Material), C.c_int, C.c_int, dbl, vp, vp]),
        "dd_glide_step": (C.c_int, [i64, vp, vp, i64, vp, vp, vp, C.POINTER(Material), dbl,
                                    vp, vp]),
        "dd_step": (C.c_int, [i64, vp, i64, vp, vp, vp, vp, C.POINTER(C.c_double), C.POINTER(Material), C.c_int,
                              C.c_int, dbl, dbl, dbl, vp, vp, vp]),
        "dd_burst_batch": (C.c_int, [i32, C.POINTER(C.c_int64), C.POINTER(C.c_int64), vp, vp,
                                     vp, vp, vp, vp, vp, C.POINTER(Material), C.c_int, C.c_int,
                                     dbl, dbl, C.c_int, dbl, vp, vp, vp]),
        "dd_burst_batch_junctions": (C.c_int, [i32, C.POINTER(C.c_int64), C.POINTER(C.c_int64), vp, vp,
                                               vp, vp, vp, vp, vp, C.POINTER(Material), C.c_int, C.c_int,
                                               dbl, dbl, C.c_int, dbl, C.POINTER(Junctions), vp, vp, vp]),
        "dd_burst_batch_junction_nodes": (C.c_int, [i32, C.POINTER(C.c_int64), C.POINTER(C.c_int64), vp, vp,
                                                    vp, vp, vp, vp, vp, C.POINTER(Material), C.c_int, C.c_int,
                                                    dbl, C.c_int, dbl, C.POINTER(JunctionNodes), vp, vp, vp]),
        "dd_mlp_create": (C.c_int, [C.c_int, C.c_uint64, C.POINTER(vp)]),
        "dd_mlp_destroy": (C.c_int, [vp]),
        "dd_mlp_set_params": (C.c_int, [vp, C.c_int, fp]),
        "dd_mlp_get_params": (C.c_int, [vp, C.c_int, fp]),
        "dd_mlp_save": (C.c_int, [vp, C.c_char_p]),
        "dd_mlp_load": (C.c_int, [C.c_char_p, C.POINTER(vp)]),
        "dd_mlp_info": (C.c_int, [vp, C.POINTER(C.c_int), C.POINTER(i64)]),
        "dd_mlp_set_scaling": (C.c_int, [vp, fp, fp, fp, fp]),
        "dd_mlp_set_log_densities": (C.c_int, [vp, C.c_float, C.c_float]),
        "dd_mlp_set_spread_floor": (C.c_int, [vp, C.c_float]),
        "dd_mlp_train_step": (C.c_int, [vp, i64, vp, vp, C.c_float, vp, vp]),
        "dd_mlp_gradients": (C.c_int, [vp, i64, vp, vp, vp, vp, vp]),
        "dd_surrogate_rates": (C.c_int, [vp, i64, vp, vp, vp, vp, C.c_float, vp]),
    }
    for name, (res, args) in sig.items():
        if hasattr(L, name):
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args


def _check(rc):
    if rc != 0:
        raise DDError(rc, lib().dd_last_error().decode())


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _dev(t, dtype, shape=None, name="tensor", nullable=False):
    if t is None:
        if nullable:
            return None
        raise ValueError(f"{name} is required")
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    return C.c_void_p(t.data_ptr())


def material(mu, nu, a, B=1.0):
    return Material(float(mu), float(nu), float(a), float(B))


def _mat(m):
    if isinstance(m, Material):
        return m
    if isinstance(m, dict):
        return material(m["mu"], m["nu"], m["a"], m.get("B", 1.0))
    return material(*m)


def _prec(p):
    if p in (DD_FP64, "fp64", "f64"):
        return DD_FP64
    if p in (DD_MIXED, "mixed"):
        return DD_MIXED
    raise ValueError(f"unknown precision {p!r}")


# ----------------------------------------------------------------- general --
def dd_version() -> int:
    return lib().dd_version()


def dd_set_validation(on: bool) -> bool:
    return bool(lib().dd_set_validation(1 if on else 0))


def dd_shutdown():
    _check(lib().dd_shutdown())


def dd_last_error() -> str:
    return lib().dd_last_error().decode()


def dd_set_autotune(on: bool) -> bool:
    return bool(lib().dd_set_autotune(1 if on else 0))


BURST_AUTO, BURST_GRAPH, BURST_PERSISTENT_ONE = 0, 1, 2


def dd_set_burst_mode(mode: int) -> int:
    """How dd_burst_batch runs its steps (dd.h): 0 automatic, 1 step graph,
    2 persistent with one workgroup per instance.  Returns the previous mode."""
    rc = lib().dd_set_burst_mode(int(mode))
    if rc < 0:
        _check(rc)
    return rc


def dd_check(stream=None):
    """Synchronise the stream and raise DDError for conditions the device-side
    checks raised since the last report (calls made with validation off)."""
    _check(lib().dd_check(_stream(stream)))


def _block_args(n, m, B, h):
    return BlockMesh(int(n), int(m), float(B), float(h))


def dd_block_average(f_gp, n, m, B, h, out=None, stream=None):
    """Block averages [n*n][c] of a Gauss-point field [n_gp][c] (float64, device); see dd.h."""
    ngp = (n * m) ** 2 * 8
    c = f_gp.shape[1] if f_gp.dim() == 2 else -1
    pf = _dev(f_gp, torch.float64, (ngp, c), "f_gp")
    if out is None:
        out = torch.empty((n * n, c), dtype=torch.float64, device=f_gp.device)
    po = _dev(out, torch.float64, (n * n, c), "out")
    mesh = _block_args(n, m, B, h)
    _check(lib().dd_block_average(C.byref(mesh), c, pf, po, _stream(stream)))
    return out


def dd_block_to_gauss(f_block, n, m, B, h, out=None, stream=None):
    """Blockwise-constant field [n*n][c] -> L2 projection on the block mesh ->
    two-level interpolation to every Gauss point [n_gp][c]; see dd.h."""
    ngp = (n * m) ** 2 * 8
    c = f_block.shape[1] if f_block.dim() == 2 else -1
    pf = _dev(f_block, torch.float64, (n * n, c), "f_block")
    if out is None:
        out = torch.empty((ngp, c), dtype=torch.float64, device=f_block.device)
    po = _dev(out, torch.float64, (ngp, c), "out")
    mesh = _block_args(n, m, B, h)
    _check(lib().dd_block_to_gauss(C.byref(mesh), c, pf, po, _stream(stream)))
    return out


def dd_dissipation_fix(T, alpha=None, Lp=None, V=None, stream=None):
    """In place: Eq. Lp_gauss on Lp and Eq. V_gauss on V ([n][9], [n][9], [n][9], [n][3])."""
    n = T.shape[0]
    pt = _dev(T, torch.float64, (n, 9), "T")
    pa = _dev(alpha, torch.float64, (n, 9), "alpha", nullable=True)
    pl = _dev(Lp, torch.float64, (n, 9), "Lp", nullable=True)
    pv = _dev(V, torch.float64, (n, 3), "V", nullable=True)
    _check(lib().dd_dissipation_fix(int(n), pt, pa, pl, pv, _stream(stream)))
    return Lp, V


def dd_set_plan(chunk_len: int = -1, variant: int = 0):
    """Fix the work split (chunk_len 0 = heuristic, >= 256; mixed variant 0/1);
    chunk_len < 0 returns to the automatic choice."""
    _check(lib().dd_set_plan(int(chunk_len), int(variant)))


def dd_last_plan():
    """(source-range length, work items, mixed-kernel variant) of the last force evaluation."""
    c, n, v = C.c_int64(), C.c_int64(), C.c_int()
    _check(lib().dd_last_plan(C.byref(c), C.byref(n), C.byref(v)))
    return c.value, n.value, v.value


def dd_timing_enable(on: bool) -> bool:
    return bool(lib().dd_timing_enable(1 if on else 0))


def dd_timing_read(reset=True):
    """(summed pair-kernel milliseconds, launches, mixed-kernel FP64 near-field
    evaluations, mixed-kernel FP32 source-quadrature evaluations)."""
    ms, n, near, quad = C.c_double(), C.c_int64(), C.c_int64(), C.c_int64()
    _check(lib().dd_timing_read(C.byref(ms), C.byref(n), C.byref(near), C.byref(quad),
                                1 if reset else 0))
    return ms.value, n.value, near.value, quad.value


def dd_vector_peak(kind: str = "fp64", reps: int = 20, stream=None) -> float:
    """Measured FMA throughput in TFLOP/s.  kind: "fp64" / "fp32" (one operand
    from a scalar register), "fp64_vec" / "fp32_vec" (all operands per lane);
    FP32 is unpacked."""
    k = {"fp64": 0, "fp32": 1, "fp64_vec": 2, "fp32_vec": 3}[kind]
    t = C.c_double()
    _check(lib().dd_vector_peak(k, int(reps), C.byref(t), _stream(stream)))
    return t.value


# -------------------------------------------------------------- force path --
def dd_nodal_forces(x, seg_nodes, burgers, normal, sigma_app, mat, n_gauss=2,
                    precision=DD_FP64, near_cutoff_a=20.0, force_out=None, stream=None, exact_eta=0.0):
    """Nodal forces [3][n_nodes] (float64) of the volume; exact_eta > 0 turns
    the exact band on (see dd.h)."""
    nn = x.shape[1] if x.dim() == 2 else -1
    ns = seg_nodes.shape[1] if seg_nodes.dim() == 2 else -1
    px = _dev(x, torch.float64, (3, nn), "x")
    psn = _dev(seg_nodes, torch.int32, (2, ns), "seg_nodes")
    pb = _dev(burgers, torch.float64, (3, ns), "burgers")
    pn = _dev(normal, torch.float64, (3, ns), "normal")
    if force_out is None:
        force_out = torch.empty((3, nn), dtype=torch.float64, device=x.device)
    pf = _dev(force_out, torch.float64, (3, nn), "force_out")
    sig = (C.c_double * 6)(*[float(v) for v in sigma_app])
    m = _mat(mat)
    _check(lib().dd_nodal_forces(nn, px, ns, psn, pb, pn, sig, C.byref(m), int(n_gauss),
                                 _prec(precision), float(near_cutoff_a), float(exact_eta), pf, _stream(stream)))
    return force_out


def dd_nodal_forces_noalloc(x, seg_nodes, burgers, normal, sigma_app, mat, force_out, n_gauss=2,
                            precision=DD_FP64, near_cutoff_a=20.0, stream=None):
    """dd_nodal_forces from the library's fixed scratch array (no allocation,
    no synchronisation; see dd.h).  force_out [3][n_nodes] is required."""
    nn = x.shape[1] if x.dim() == 2 else -1
    ns = seg_nodes.shape[1] if seg_nodes.dim() == 2 else -1
    px = _dev(x, torch.float64, (3, nn), "x")
    psn = _dev(seg_nodes, torch.int32, (2, ns), "seg_nodes")
    pb = _dev(burgers, torch.float64, (3, ns), "burgers")
    pn = _dev(normal, torch.float64, (3, ns), "normal")
    pf = _dev(force_out, torch.float64, (3, nn), "force_out")
    sig = (C.c_double * 6)(*[float(v) for v in sigma_app])
    m = _mat(mat)
    _check(lib().dd_nodal_forces_noalloc(nn, px, ns, psn, pb, pn, sig, C.byref(m), int(n_gauss),
                                         _prec(precision), float(near_cutoff_a), pf, _stream(stream)))
    return force_out


def dd_glide_step(x, force, seg_nodes, normal, pinned, mat, dt, vel_out=None, stream=None):
    """Advance x in place by one glide step; returns the velocities."""
    nn = x.shape[1]
    ns = seg_nodes.shape[1]
    px = _dev(x, torch.float64, (3, nn), "x")
    pf = _dev(force, torch.float64, (3, nn), "force")
    psn = _dev(seg_nodes, torch.int32, (2, ns), "seg_nodes")
    pn = _dev(normal, torch.float64, (3, ns), "normal")
    pp = _dev(pinned, torch.uint8, (nn,), "pinned", nullable=True)
    if vel_out is None:
        vel_out = torch.empty((3, nn), dtype=torch.float64, device=x.device)
    pv = _dev(vel_out, torch.float64, (3, nn), "vel_out")
    m = _mat(mat)
    _check(lib().dd_glide_step(nn, px, pf, ns, psn, pn, pp, C.byref(m), float(dt), pv,
                               _stream(stream)))
    return vel_out


def dd_step(x, seg_nodes, burgers, normal, pinned, sigma_app, mat, dt, n_gauss=2, precision=DD_FP64,
            near_cutoff_a=20.0, force_out=None, vel_out=None, stream=None, exact_eta=0.0):
    """One DD step (nodal forces, then the glide step) in one call; x advances
    in place.  Returns (force, vel) [3][n_nodes] (None where the library used
    its workspace because the output was not requested: pass tensors to keep
    them)."""
    nn = x.shape[1] if x.dim() == 2 else -1
    ns = seg_nodes.shape[1] if seg_nodes.dim() == 2 else -1
    px = _dev(x, torch.float64, (3, nn), "x")
    psn = _dev(seg_nodes, torch.int32, (2, ns), "seg_nodes")
    pb = _dev(burgers, torch.float64, (3, ns), "burgers")
    pn = _dev(normal, torch.float64, (3, ns), "normal")
    pp = _dev(pinned, torch.uint8, (nn,), "pinned", nullable=True)
    pf = _dev(force_out, torch.float64, (3, nn), "force_out", nullable=True)
    pv = _dev(vel_out, torch.float64, (3, nn), "vel_out", nullable=True)
    sig = (C.c_double * 6)(*[float(v) for v in sigma_app])
    m = _mat(mat)
    _check(lib().dd_step(nn, px, ns, psn, pb, pn, pp, sig, C.byref(m), int(n_gauss), _prec(precision),
                         float(near_cutoff_a), float(exact_eta), float(dt), pf, pv, _stream(stream)))
    return force_out, vel_out


def dd_burst_batch(node_off, seg_off, x, seg_nodes, burgers, normal, pinned, sigma_app,
                   volume, mat, n_gauss=2, precision=DD_MIXED, near_cutoff_a=20.0,
                   n_steps=200, dt=2e-14, rate_avg_out=None, features_out=None,
                   want_features=False, stream=None, exact_eta=0.0):
    """Batched bursts; node_off/seg_off are host sequences (length n_inst+1).
    Returns (rate_avg [n_inst][12], features [n_inst][36] or None); x advances."""
    no = (C.c_int64 * len(node_off))(*[int(v) for v in node_off])
    so = (C.c_int64 * len(seg_off))(*[int(v) for v in seg_off])
    n_inst = len(node_off) - 1
    if len(seg_off) != n_inst + 1:
        raise ValueError("node_off and seg_off must have the same length")
    nn, ns = int(node_off[-1]), int(seg_off[-1])
    dev = x.device
    px = _dev(x, torch.float64, (3, nn), "x")
    psn = _dev(seg_nodes, torch.int32, (2, ns), "seg_nodes")
    pb = _dev(burgers, torch.float64, (3, ns), "burgers")
    pn = _dev(normal, torch.float64, (3, ns), "normal")
    pp = _dev(pinned, torch.uint8, (nn,), "pinned", nullable=True)
    ps = _dev(sigma_app, torch.float64, (n_inst, 6), "sigma_app")
    pv = _dev(volume, torch.float64, (n_inst,), "volume")
    if rate_avg_out is None:
        rate_avg_out = torch.empty((n_inst, 12), dtype=torch.float64, device=dev)
    pr = _dev(rate_avg_out, torch.float64, (n_inst, 12), "rate_avg_out")
    if features_out is None and want_features:
        features_out = torch.empty((n_inst, 36), dtype=torch.float64, device=dev)
    pfe = _dev(features_out, torch.float64, (n_inst, 36), "features_out", nullable=True)
    m = _mat(mat)
    _check(lib().dd_burst_batch(n_inst, no, so, px, psn, pb, pn, pp, ps, pv, C.byref(m),
                                int(n_gauss), _prec(precision), float(near_cutoff_a), float(exact_eta),
                                int(n_steps), float(dt), pr, pfe, _stream(stream)))
    return rate_avg_out, features_out


def dd_burst_batch_junctions(node_off, seg_off, x, seg_nodes, burgers, normal, pinned, sigma_app, volume,
                             mat, state, fractions, capture_radius, max_break_time, t0=0.0, n_gauss=2,
                             precision=DD_MIXED, near_cutoff_a=20.0, n_steps=200, dt=2e-14,
                             rate_avg_out=None, stream=None, exact_eta=0.0):
    """Batched bursts with junctions (dd.h, dd_junctions).  state: dict of device
    tensors junction (int32), release (float64), ignore (int32), count (int32),
    each [n_nodes], updated in place; fractions [n_nodes][K] float64 (device).
    Returns rate_avg [n_inst][12]; x advances."""
    no = (C.c_int64 * len(node_off))(*[int(v) for v in node_off])
    so = (C.c_int64 * len(seg_off))(*[int(v) for v in seg_off])
    n_inst = len(node_off) - 1
    if len(seg_off) != n_inst + 1:
        raise ValueError("node_off and seg_off must have the same length")
    nn, ns = int(node_off[-1]), int(seg_off[-1])
    dev = x.device
    px = _dev(x, torch.float64, (3, nn), "x")
    psn = _dev(seg_nodes, torch.int32, (2, ns), "seg_nodes")
    pb = _dev(burgers, torch.float64, (3, ns), "burgers")
    pn = _dev(normal, torch.float64, (3, ns), "normal")
    pp = _dev(pinned, torch.uint8, (nn,), "pinned", nullable=True)
    ps = _dev(sigma_app, torch.float64, (n_inst, 6), "sigma_app")
    pv = _dev(volume, torch.float64, (n_inst,), "volume")
    jn = _junction_args(state, fractions, capture_radius, max_break_time, nn, t0)
    if rate_avg_out is None:
        rate_avg_out = torch.empty((n_inst, 12), dtype=torch.float64, device=dev)
    pr = _dev(rate_avg_out, torch.float64, (n_inst, 12), "rate_avg_out")
    m = _mat(mat)
    _check(lib().dd_burst_batch_junctions(n_inst, no, so, px, psn, pb, pn, pp, ps, pv, C.byref(m),
                                          int(n_gauss), _prec(precision), float(near_cutoff_a), float(exact_eta),
                                          int(n_steps), float(dt), C.byref(jn), pr, None, _stream(stream)))
    return rate_avg_out


def junction_node_state(n_nodes, n_segs, n_inst, device):
    """Initial state of dd_burst_batch_junction_nodes (no junctions): release
    [n_nodes] float64, ses [n_nodes] int32 = -1, ignore [n_segs] int32 = 0,
    point [3][n_segs] float64, count and missed [n_inst] int32 = 0."""
    return {"release": torch.zeros(n_nodes, dtype=torch.float64, device=device),
            "ses": torch.full((n_nodes,), -1, dtype=torch.int32, device=device),
            "ignore": torch.zeros(n_segs, dtype=torch.int32, device=device),
            "point": torch.zeros((3, n_segs), dtype=torch.float64, device=device),
            "count": torch.zeros(n_inst, dtype=torch.int32, device=device),
            "missed": torch.zeros(n_inst, dtype=torch.int32, device=device)}


def dd_burst_batch_junction_nodes(node_off, seg_off, x, seg_nodes, burgers, normal, pinned, sigma_app, volume,
                                  mat, state, fractions, capture_radius, max_break_time, min_length, n_slots,
                                  t0=0.0, n_gauss=2, precision=DD_MIXED, near_cutoff_a=20.0, n_steps=200,
                                  dt=2e-14, rate_avg_out=None, features_out=None, want_features=False,
                                  stream=None):
    """Batched bursts with junction nodes (dd.h, dd_junction_nodes): every
    instance ends with n_slots node slots, two dummy nodes and n_slots segment
    slots (workloads.with_junction_slots).  x, seg_nodes, burgers, normal and
    the state (junction_node_state) change in place; fractions [n_inst][K]
    float64 (device).  Returns (rate_avg [n_inst][12], features or None)."""
    no = (C.c_int64 * len(node_off))(*[int(v) for v in node_off])
    so = (C.c_int64 * len(seg_off))(*[int(v) for v in seg_off])
    n_inst = len(node_off) - 1
    if len(seg_off) != n_inst + 1:
        raise ValueError("node_off and seg_off must have the same length")
    nn, ns = int(node_off[-1]), int(seg_off[-1])
    dev = x.device
    px = _dev(x, torch.float64, (3, nn), "x")
    psn = _dev(seg_nodes, torch.int32, (2, ns), "seg_nodes")
    pb = _dev(burgers, torch.float64, (3, ns), "burgers")
    pn = _dev(normal, torch.float64, (3, ns), "normal")
    pp = _dev(pinned, torch.uint8, (nn,), "pinned", nullable=True)
    ps = _dev(sigma_app, torch.float64, (n_inst, 6), "sigma_app")
    pv = _dev(volume, torch.float64, (n_inst,), "volume")
    jn = _jnode_args(state, fractions, capture_radius, max_break_time, min_length, n_slots, t0, nn, ns, n_inst)
    if rate_avg_out is None:
        rate_avg_out = torch.empty((n_inst, 12), dtype=torch.float64, device=dev)
    pr = _dev(rate_avg_out, torch.float64, (n_inst, 12), "rate_avg_out")
    if features_out is None and want_features:
        features_out = torch.empty((n_inst, 36), dtype=torch.float64, device=dev)
    pfe = _dev(features_out, torch.float64, (n_inst, 36), "features_out", nullable=True)
    m = _mat(mat)
    _check(lib().dd_burst_batch_junction_nodes(n_inst, no, so, px, psn, pb, pn, pp, ps, pv, C.byref(m),
                                               int(n_gauss), _prec(precision), float(near_cutoff_a), int(n_steps),
                                               float(dt), C.byref(jn), pr, pfe, _stream(stream)))
    return rate_avg_out, features_out


def _jnode_args(state, fractions, capture_radius, max_break_time, min_length, n_slots, t0, nn, ns, n_inst):
    K = fractions.shape[1] if fractions.dim() == 2 else -1
    pf = _dev(fractions, torch.float64, (n_inst, K), "fractions")
    return JunctionNodes(float(capture_radius), float(max_break_time), float(t0), float(min_length), int(n_slots),
                         int(K), pf.value,
                         _dev(state["release"], torch.float64, (nn,), "release").value,
                         _dev(state["ses"], torch.int32, (nn,), "ses").value,
                         _dev(state["ignore"], torch.int32, (ns,), "ignore").value,
                         _dev(state["point"], torch.float64, (3, ns), "point").value,
                         _dev(state["count"], torch.int32, (n_inst,), "count").value,
                         _dev(state["missed"], torch.int32, (n_inst,), "missed").value)


def _junction_args(state, fractions, capture_radius, max_break_time, nn, t0=0.0):
    K = fractions.shape[1] if fractions.dim() == 2 else -1
    pf = _dev(fractions, torch.float64, (nn, K), "fractions")
    pj = _dev(state["junction"], torch.int32, (nn,), "junction")
    prl = _dev(state["release"], torch.float64, (nn,), "release")
    pig = _dev(state["ignore"], torch.int32, (nn,), "ignore")
    pc = _dev(state["count"], torch.int32, (nn,), "count")
    return Junctions(float(capture_radius), float(max_break_time), float(t0), int(K), pf.value, pj.value,
                     prl.value, pig.value, pc.value)


def dd_pta_step(node_off, seg_off, x, seg_nodes, burgers, normal, pinned, volume, stress_rate, t,
                params, mat, n_gauss=2, precision=DD_FP64, near_cutoff_a=20.0, stream=None, junctions=None,
                exact_eta=0.0, junction_nodes=None):
    """One PTA slow-time step for every instance (see dd.h); x advances to the
    microstructure for the next step.  stress_rate [n_inst][6] (Pa/s) and t
    [n_inst] (s) are host sequences.  Returns a dict of NumPy arrays.

    junctions: None, or a dict with keys state (device tensors as
    dd_burst_batch_junctions, updated in place), fractions, capture_radius,
    max_break_time and fast_steps (host int64 array [n_inst], updated in
    place); then dd_pta_step_junctions runs.

    junction_nodes: None, or a dict with keys state (junction_node_state),
    fractions (device [n_inst][K]), capture_radius, max_break_time,
    min_length, n_slots and fast_steps (host int64 [n_inst], updated in
    place); then dd_pta_step_junction_nodes runs, and seg_nodes, burgers and
    normal change in place with the topology."""
    import numpy as np
    no = (C.c_int64 * len(node_off))(*[int(v) for v in node_off])
    so = (C.c_int64 * len(seg_off))(*[int(v) for v in seg_off])
    n_inst = len(node_off) - 1
    if len(seg_off) != n_inst + 1:
        raise ValueError("node_off and seg_off must have the same length")
    nn, ns = int(node_off[-1]), int(seg_off[-1])
    px = _dev(x, torch.float64, (3, nn), "x")
    psn = _dev(seg_nodes, torch.int32, (2, ns), "seg_nodes")
    pb = _dev(burgers, torch.float64, (3, ns), "burgers")
    pn = _dev(normal, torch.float64, (3, ns), "normal")
    pp = _dev(pinned, torch.uint8, (nn,), "pinned", nullable=True)
    pv = _dev(volume, torch.float64, (n_inst,), "volume")
    sr = np.ascontiguousarray(stress_rate, dtype=np.float64).reshape(n_inst, 6)
    tt = np.ascontiguousarray(t, dtype=np.float64).reshape(n_inst)
    out = np.zeros((n_inst, DD_PTA_OUT))
    m = _mat(mat)
    dp = C.POINTER(C.c_double)
    if junction_nodes is not None:
        J = junction_nodes
        jn = _jnode_args(J["state"], J["fractions"], J["capture_radius"], J["max_break_time"], J["min_length"],
                         J["n_slots"], 0.0, nn, ns, n_inst)
        fs = J["fast_steps"]
        if not (isinstance(fs, np.ndarray) and fs.dtype == np.int64 and fs.shape == (n_inst,)
                and fs.flags.c_contiguous):
            raise ValueError("junction_nodes['fast_steps'] must be a contiguous int64 array of length n_inst")
        _check(lib().dd_pta_step_junction_nodes(n_inst, no, so, px, psn, pb, pn, pp, pv, sr.ctypes.data_as(dp),
                                                tt.ctypes.data_as(dp), C.byref(params), C.byref(m), int(n_gauss),
                                                _prec(precision), float(near_cutoff_a), C.byref(jn),
                                                fs.ctypes.data_as(C.POINTER(C.c_int64)), out.ctypes.data_as(dp),
                                                _stream(stream)))
    elif junctions is None:
        _check(lib().dd_pta_step(n_inst, no, so, px, psn, pb, pn, pp, pv, sr.ctypes.data_as(dp),
                                 tt.ctypes.data_as(dp), C.byref(params), C.byref(m), int(n_gauss),
                                 _prec(precision), float(near_cutoff_a), float(exact_eta), out.ctypes.data_as(dp),
                                 _stream(stream)))
    else:
        jn = _junction_args(junctions["state"], junctions["fractions"], junctions["capture_radius"],
                            junctions["max_break_time"], nn)
        fs = junctions["fast_steps"]
        if not (isinstance(fs, np.ndarray) and fs.dtype == np.int64 and fs.shape == (n_inst,)
                and fs.flags.c_contiguous):
            raise ValueError("junctions['fast_steps'] must be a contiguous int64 array of length n_inst")
        _check(lib().dd_pta_step_junctions(n_inst, no, so, px, psn, pb, pn, pp, pv, sr.ctypes.data_as(dp),
                                           tt.ctypes.data_as(dp), C.byref(params), C.byref(m), int(n_gauss),
                                           _prec(precision), float(near_cutoff_a), float(exact_eta), C.byref(jn),
                                           fs.ctypes.data_as(C.POINTER(C.c_int64)), out.ctypes.data_as(dp),
                                           _stream(stream)))
    return {"rho_a": out[:, 0], "rho_b": out[:, 1], "g_a": out[:, 2:14], "g_b": out[:, 14:26],
            "lp_a": out[:, 26:35].reshape(n_inst, 3, 3), "lp_b": out[:, 35:44].reshape(n_inst, 3, 3),
            "lpdot": out[:, 44:53].reshape(n_inst, 3, 3), "rhodot": out[:, 53], "h": out[:, 54],
            "steps_a": out[:, 55].astype(int), "steps_b": out[:, 56].astype(int),
            "conv_a": out[:, 57] > 0, "conv_b": out[:, 58] > 0, "jumps": out[:, 59].astype(int),
            "rerun_chunks": out[:, 60].astype(int)}


def dd_pta_step_junctions(node_off, seg_off, x, seg_nodes, burgers, normal, pinned, volume, stress_rate, t,
                          params, mat, junctions, n_gauss=2, precision=DD_FP64, near_cutoff_a=20.0, stream=None,
                          exact_eta=0.0):
    """dd_pta_step with junctions (dd.h); `junctions` as in dd_pta_step."""
    if junctions is None:
        raise ValueError("junctions is required")
    return dd_pta_step(node_off, seg_off, x, seg_nodes, burgers, normal, pinned, volume, stress_rate, t, params,
                       mat, n_gauss, precision, near_cutoff_a, stream, junctions, exact_eta)


def dd_pta_step_junction_nodes(node_off, seg_off, x, seg_nodes, burgers, normal, pinned, volume, stress_rate, t,
                               params, mat, junction_nodes, n_gauss=2, precision=DD_FP64, near_cutoff_a=20.0,
                               stream=None):
    """dd_pta_step with junction nodes (dd.h); `junction_nodes` as in dd_pta_step."""
    if junction_nodes is None:
        raise ValueError("junction_nodes is required")
    return dd_pta_step(node_off, seg_off, x, seg_nodes, burgers, normal, pinned, volume, stress_rate, t, params,
                       mat, n_gauss, precision, near_cutoff_a, stream, junction_nodes=junction_nodes)


# --------------------------------------------------------------- surrogate --
def _host_f32(a, n, name):
    import numpy as np
    a = np.ascontiguousarray(a, dtype=np.float32).reshape(-1)
    if a.size != n:
        raise ValueError(f"{name} must have {n} entries")
    return a, a.ctypes.data_as(C.POINTER(C.c_float))


class SurrogateModel:
    """Owns a dd_mlp handle (ensemble of MLPs on the current device)."""

    def __init__(self, n_members=4, seed=0, _handle=None):
        if _handle is None:
            h = C.c_void_p()
            _check(lib().dd_mlp_create(int(n_members), C.c_uint64(int(seed)), C.byref(h)))
            _handle = h
        self.handle = _handle
        self.n_members = n_members

    def save(self, path):
        """Write the ensemble (parameters, Adam state, scaling) to `path`."""
        _check(lib().dd_mlp_save(self.handle, os.fsencode(path)))

    @classmethod
    def load(cls, path):
        """An ensemble read from a file written by save(), on the current device."""
        h = C.c_void_p()
        _check(lib().dd_mlp_load(os.fsencode(path), C.byref(h)))
        m = C.c_int()
        _check(lib().dd_mlp_info(h, C.byref(m), None))
        return cls(m.value, _handle=h)

    def adam_steps(self):
        t = C.c_int64()
        _check(lib().dd_mlp_info(self.handle, None, C.byref(t)))
        return t.value

    def close(self):
        if self.handle:
            _check(lib().dd_mlp_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, member, params):
        import numpy as np
        a, p = _host_f32(params, MLP_PARAMS, "params")
        _check(lib().dd_mlp_set_params(self.handle, int(member), p))

    def get_params(self, member):
        import numpy as np
        out = np.zeros(MLP_PARAMS, np.float32)
        _check(lib().dd_mlp_get_params(self.handle, int(member),
                                       out.ctypes.data_as(C.POINTER(C.c_float))))
        return out

    def set_scaling(self, in_shift, in_scale, out_shift, out_scale):
        a, p1 = _host_f32(in_shift, MLP_IN, "in_shift")
        b, p2 = _host_f32(in_scale, MLP_IN, "in_scale")
        c, p3 = _host_f32(out_shift, MLP_OUT, "out_shift")
        d, p4 = _host_f32(out_scale, MLP_OUT, "out_scale")
        _check(lib().dd_mlp_set_scaling(self.handle, p1, p2, p3, p4))

    def set_spread_floor(self, floor):
        _check(lib().dd_mlp_set_spread_floor(self.handle, C.c_float(floor)))

    def set_log_densities(self, dens_scale, dens_floor):
        _check(lib().dd_mlp_set_log_densities(self.handle, C.c_float(dens_scale), C.c_float(dens_floor)))


def dd_mlp_train_step(model: SurrogateModel, feat, target, lr=1e-3, loss_out=None, stream=None):
    n = feat.shape[0]
    pf = _dev(feat, torch.float32, (n, MLP_IN), "feat")
    pt = _dev(target, torch.float32, (n, MLP_OUT), "target")
    if loss_out is None:
        loss_out = torch.empty(model.n_members, dtype=torch.float32, device=feat.device)
    pl = _dev(loss_out, torch.float32, (model.n_members,), "loss_out")
    _check(lib().dd_mlp_train_step(model.handle, n, pf, pt, C.c_float(lr), pl, _stream(stream)))
    return loss_out


def dd_mlp_gradients(model: SurrogateModel, feat, target, grad_out=None, loss_out=None,
                     stream=None):
    """Per-member gradients [n_members][144140] and losses, without a step."""
    n = feat.shape[0]
    pf = _dev(feat, torch.float32, (n, MLP_IN), "feat")
    pt = _dev(target, torch.float32, (n, MLP_OUT), "target")
    if grad_out is None:
        grad_out = torch.empty((model.n_members, MLP_PARAMS), dtype=torch.float32, device=feat.device)
    pg = _dev(grad_out, torch.float32, (model.n_members, MLP_PARAMS), "grad_out")
    if loss_out is None:
        loss_out = torch.empty(model.n_members, dtype=torch.float32, device=feat.device)
    pl = _dev(loss_out, torch.float32, (model.n_members,), "loss_out")
    _check(lib().dd_mlp_gradients(model.handle, n, pf, pt, pg, pl, _stream(stream)))
    return grad_out, loss_out


def dd_surrogate_rates(model: SurrogateModel, feat, spread_tol=0.05, rates=None, spread=None,
                       needs_dd=None, stream=None):
    n = feat.shape[0]
    dev = feat.device
    pf = _dev(feat, torch.float32, (n, MLP_IN), "feat")
    if rates is None:
        rates = torch.empty((n, MLP_OUT), dtype=torch.float32, device=dev)
    if spread is None:
        spread = torch.empty((n,), dtype=torch.float32, device=dev)
    if needs_dd is None:
        needs_dd = torch.empty((n,), dtype=torch.uint8, device=dev)
    pr = _dev(rates, torch.float32, (n, MLP_OUT), "rates")
    ps = _dev(spread, torch.float32, (n,), "spread")
    pn = _dev(needs_dd, torch.uint8, (n,), "needs_dd")
    _check(lib().dd_surrogate_rates(model.handle, n, pf, pr, ps, pn, C.c_float(spread_tol),
                                    _stream(stream)))
    return rates, spread, needs_dd
