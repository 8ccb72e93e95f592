"""The achievable-peak probes return rates in the range an MI355X can reach:
published dense FP16 2.5 PFLOP/s, FP64 matrix 78.6 TFLOP/s, HBM 8 TB/s
(bounds are generous: the probes measure, they do not assert a target)."""
import pytest

pytestmark = pytest.mark.gpu


def test_peak_probes(tai):
    ctx = tai.context(0)
    f16 = ctx.peak_probe(0)
    f64 = ctx.peak_probe(1)
    hbm = ctx.peak_probe(2)
    print(f"probe: FP16 MFMA {f16:.0f} TFLOP/s, FP64 MFMA {f64:.1f} TFLOP/s, HBM copy {hbm:.0f} GB/s")
    assert 500.0 < f16 < 5000.0
    assert 20.0 < f64 < 200.0
    assert 1000.0 < hbm < 12000.0


def test_peak_probe_rejects_bad_kind(tai):
    ctx = tai.context(0)
    with pytest.raises(tai.TaiError) as e:
        ctx.peak_probe(3)
    assert e.value.status == tai.TAI_ERR_INVALID_ARG
