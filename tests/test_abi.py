"""The C ABI (CPU only, no GPU calls): libdd.so loads and exports every
function include/dd.h declares, and the Python binding wraps each of them."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dd.h")
LIB = os.path.join(ROOT, "paper_2005_02498_amd", "libdd.so")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(dd_\w+)\s*\(", src, flags=re.M)))


def test_header_declares_the_four_calls():
    names = declared()
    for f in ("dd_nodal_forces", "dd_glide_step", "dd_burst_batch", "dd_surrogate_rates"):
        assert f in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libdd.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="libdd.so not built")
def test_binding_covers_header():
    import paper_2005_02498_amd as dd
    assert sorted(dd.EXPORTS) == declared()
    for n in declared():
        if n in ("dd_mlp_create", "dd_mlp_destroy", "dd_mlp_set_params", "dd_mlp_get_params",
                 "dd_mlp_set_scaling", "dd_mlp_set_log_densities", "dd_mlp_set_spread_floor",
                 "dd_mlp_save", "dd_mlp_load", "dd_mlp_info"):
            continue   # wrapped as SurrogateModel methods
        assert hasattr(dd, n), n


@pytest.mark.skipif(not os.path.exists(LIB), reason="libdd.so not built")
def test_host_only_calls_without_gpu():
    import paper_2005_02498_amd as dd
    assert dd.dd_version() >= 10000
    prev = dd.dd_set_validation(False)
    assert dd.dd_set_validation(prev) is False
    assert isinstance(dd.dd_last_error(), str)
    for bad in ((8, 0), (0, 3), (256, -1)):
        with pytest.raises(dd.DDError):
            dd.dd_set_plan(*bad)
    dd.dd_set_plan(-1)
    assert dd.dd_set_burst_mode(1) == 0 and dd.dd_set_burst_mode(0) == 1
    with pytest.raises(dd.DDError):
        dd.dd_set_burst_mode(3)
    # block-coupling argument checks happen before any device work
    fake = ctypes.c_void_p(256)
    for bad in ((0, 1, 1.0, 1.0), (1, 0, 1.0, 1.0), (1, 1, 0.0, 1.0), (1, 1, 1.0, float("nan")),
                (70000, 1, 1.0, 1.0), (46341, 1, 1.0, 1.0)):
        mesh = dd.BlockMesh(*bad)
        assert dd.lib().dd_block_average(ctypes.byref(mesh), 1, fake, fake, None) == dd.DD_EINVAL
        assert dd.lib().dd_block_to_gauss(ctypes.byref(mesh), 1, fake, fake, None) == dd.DD_EINVAL
    ok = dd.BlockMesh(1, 1, 1.0, 1.0)
    for c in (0, 17):
        assert dd.lib().dd_block_average(ctypes.byref(ok), c, fake, fake, None) == dd.DD_EINVAL
    assert dd.lib().dd_dissipation_fix(-1, fake, fake, fake, fake, None) == dd.DD_EINVAL
    assert dd.lib().dd_dissipation_fix(4, None, fake, fake, fake, None) == dd.DD_EINVAL
    assert dd.lib().dd_dissipation_fix(4, fake, None, None, fake, None) == dd.DD_EINVAL
    off = (ctypes.c_int64 * 2)(0, 4)
    m = dd.Material(1.0, 0.3, 1.0, 1.0)
    assert dd.lib().dd_burst_batch_junctions(1, off, off, fake, fake, fake, fake, fake, fake, fake,
                                             ctypes.byref(m), 2, 0, 20.0, 0.0, 1, 1.0, None, fake, None,
                                             None) == dd.DD_EINVAL
    sig = (ctypes.c_double * 6)()
    # the mixed path's near-field cutoff is at least one core width
    for cut in (0.5, 0.0, float("nan")):
        assert dd.lib().dd_nodal_forces(4, fake, 4, fake, fake, fake, sig, ctypes.byref(m), 2, 1, cut, 0.0,
                                        fake, None) == dd.DD_EINVAL
    assert "near_cutoff_a" in dd.dd_last_error()
    # the exact band's eta is finite and >= 0, for every call that takes it
    for eta in (-1.0, float("nan"), float("inf")):
        assert dd.lib().dd_nodal_forces(4, fake, 4, fake, fake, fake, sig, ctypes.byref(m), 2, 0, 20.0, eta,
                                        fake, None) == dd.DD_EINVAL
        assert "exact_eta" in dd.dd_last_error()
        assert dd.lib().dd_step(4, fake, 4, fake, fake, fake, None, sig, ctypes.byref(m), 2, 0, 20.0, eta,
                                1.0, None, None, None) == dd.DD_EINVAL
        assert dd.lib().dd_burst_batch(1, off, off, fake, fake, fake, fake, fake, fake, fake,
                                       ctypes.byref(m), 2, 0, 20.0, eta, 1, 1.0, fake, None,
                                       None) == dd.DD_EINVAL
    for args in ((-1, 1.0), (4, 0.0), (4, float("nan"))):   # negative count, dt <= 0, NaN dt
        assert dd.lib().dd_step(args[0], fake, 4, fake, fake, fake, None, sig, ctypes.byref(m), 2, 0, 20.0, 0.0,
                                args[1], None, None, None) == dd.DD_EINVAL
    P = dd.PTAParams(dt=1e-14)
    d1 = (ctypes.c_double * 6)()
    assert dd.lib().dd_pta_step_junctions(1, off, off, fake, fake, fake, fake, fake, fake, d1, d1,
                                          ctypes.byref(P), ctypes.byref(m), 2, 0, 20.0, 0.0, None, None, d1,
                                          None) == dd.DD_EINVAL
    # junction nodes: parameters are checked before any device work
    assert dd.lib().dd_burst_batch_junction_nodes(1, off, off, fake, fake, fake, fake, fake, fake, fake,
                                                  ctypes.byref(m), 2, 0, 20.0, 1, 1.0, None, fake, None,
                                                  None) == dd.DD_EINVAL
    for bad in (dict(n_slots=0), dict(n_fractions=0), dict(capture_radius=-1.0), dict(min_length=float("nan")),
                dict(t0=float("inf")), dict(n_slots=4)):   # n_slots = 4: the instance has 4 nodes, needs 6
        kw = dict(capture_radius=5.0, max_break_time=1.0, t0=0.0, min_length=1.0, n_slots=1, n_fractions=1)
        kw.update(bad)
        jn = dd.JunctionNodes(kw["capture_radius"], kw["max_break_time"], kw["t0"], kw["min_length"],
                              kw["n_slots"], kw["n_fractions"], 256, 256, 256, 256, 256, 256, 256)
        assert dd.lib().dd_burst_batch_junction_nodes(1, off, off, fake, fake, fake, fake, fake, fake, fake,
                                                      ctypes.byref(m), 2, 0, 20.0, 1, 1.0, ctypes.byref(jn), fake,
                                                      None, None) == dd.DD_EINVAL, bad
        assert "junction nodes" in dd.dd_last_error()


@pytest.mark.skipif(not os.path.exists(LIB), reason="libdd.so not built")
def test_surrogate_file_checks_without_gpu(tmp_path):
    """dd_mlp_load checks the whole file before any device call: a missing
    file, a wrong magic, a foreign shape, a truncated file, a flipped byte
    and trailing bytes are each DD_EIO, and the handle stays NULL."""
    import struct
    import paper_2005_02498_amd as dd
    P, SCAL = dd.MLP_PARAMS, 2 * dd.MLP_IN + 2 * dd.MLP_OUT + 3

    def fnv(b):
        h = 0xcbf29ce484222325
        for c in b:
            h = ((h ^ c) * 0x100000001b3) & 0xFFFFFFFFFFFFFFFF
        return h

    def body(members=1, shape=(36, 256, 12)):
        b = b"DDMLP\0\0\x01" + struct.pack("<6i", members, *shape, P, SCAL) + struct.pack("<q", 3)
        return b + struct.pack(f"<{SCAL}f", *([0.5] * SCAL)) + bytes(4 * 3 * members * P)

    def load(path):
        h = ctypes.c_void_p(1234)
        rc = dd.lib().dd_mlp_load(os.fsencode(str(path)), ctypes.byref(h))
        return rc, h.value

    cases = {}
    good = body()
    cases["missing"] = None
    cases["magic"] = b"XXMLP\0\0\x01" + good[8:]
    cases["shape"] = body(shape=(36, 128, 12))
    cases["truncated"] = good[:-100]
    flipped = bytearray(good)
    flipped[5000] ^= 1
    cases["checksum"] = bytes(flipped) + struct.pack("<Q", fnv(good))
    cases["trailing"] = good + struct.pack("<Q", fnv(good)) + b"\0"
    for name, data in cases.items():
        path = tmp_path / f"{name}.ddmlp"
        if data is not None:
            path.write_bytes(data)
        rc, h = load(path)
        assert rc == dd.DD_EIO and h is None, (name, rc, dd.lib().dd_last_error())
    # a null output pointer or path is DD_EINVAL
    assert dd.lib().dd_mlp_load(b"x", None) == dd.DD_EINVAL
    h = ctypes.c_void_p()
    assert dd.lib().dd_mlp_load(None, ctypes.byref(h)) == dd.DD_EINVAL


@pytest.mark.skipif(not os.path.exists(LIB), reason="libdd.so not built")
def test_library_links_roctx():
    """The host runtime's roctx ranges come from the rocprofiler-sdk roctx
    library, which libdd.so records as a dependency."""
    import subprocess
    out = subprocess.run(["readelf", "-d", LIB], capture_output=True, text=True).stdout
    assert "librocprofiler-sdk-roctx" in out
