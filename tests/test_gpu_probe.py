"""dd_vector_peak: the measured FMA throughput used as a second roofline
reference.  Plausibility only: the published vector peaks of the device bound
what a correct measurement can return."""
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


def test_vector_peak_plausible():
    import paper_2005_02498_amd as dd
    # published vector peaks of MI355X: FP64 78.6, FP32 157.3 TFLOP/s
    for kind, peak in (("fp64", 78.6), ("fp32", 157.3), ("fp64_vec", 78.6), ("fp32_vec", 157.3)):
        r = dd.dd_vector_peak(kind, 5)
        assert 5.0 < r < peak * 1.05, (kind, r)


def test_vector_peak_invalid():
    import ctypes as C
    import paper_2005_02498_amd as dd
    EINVAL = -1
    t = C.c_double()
    assert dd.lib().dd_vector_peak(4, 5, C.byref(t), None) == EINVAL
    assert dd.lib().dd_vector_peak(0, 0, C.byref(t), None) == EINVAL
    assert dd.lib().dd_vector_peak(0, 5, None, None) == EINVAL
    with pytest.raises(dd.DDError):
        dd.dd_vector_peak("fp64", 1001)
