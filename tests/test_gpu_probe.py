"""The ceiling probes (qb_probe_fma, qb_probe_copy) return rates in the
range an MI355X can reach: nonzero, and below its datasheet peaks with
margin for clock variation (vector FMA 157.3 TFLOP/s packed float32,
78.6 TFLOP/s float64; HBM 8 TB/s, a copy counting read plus write)."""
import pytest

pytestmark = pytest.mark.gpu


def test_fma_probe_rates_are_plausible():
    from paper_1408_1782_amd import _lib
    f32 = _lib.probe_fma("f32", 1024)
    f64 = _lib.probe_fma("f64", 1024)
    assert 5.0 < f32 < 180.0 and 5.0 < f64 < 90.0, (f32, f64)


def test_copy_probe_rate_is_plausible():
    from paper_1408_1782_amd import _lib
    g = _lib.probe_copy(256, 3)
    assert 500.0 < g < 20000.0, g


def test_probes_reject_bad_arguments():
    import paper_1408_1782_amd as qb
    from paper_1408_1782_amd import _lib
    with pytest.raises(qb.QBError):
        _lib.probe_fma("f32", 0)
