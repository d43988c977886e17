"""ensf_measure_mfma_rate: the attainable matrix-core rate of the card for each form's MFMA,
a measurement (no reference value exists): it must be positive, below the published dense
peak with a small margin for clock boost, and above a quarter of it (a rate that low means
the probe did not keep the matrix cores busy)."""
import pytest

torch = pytest.importorskip("torch")

from paper_2407_12168_amd import ensf

pytestmark = pytest.mark.gpu

PEAK = {"fp32": 157.3, "bf16x3": 2500.0, "bf16": 2500.0}


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_measured_mfma_rate_is_plausible(dev, precision):
    rate = ensf.ensf_measure_mfma_rate(precision)
    print(f"{precision}: {rate:.1f} TFLOP/s = {rate / PEAK[precision]:.3f} of the published peak")
    assert 0.25 * PEAK[precision] < rate < 1.05 * PEAK[precision]


def test_measured_mfma_rate_rejects_bad_precision(dev):
    L = ensf._lib()
    import ctypes
    out = ctypes.c_double(0.0)
    assert L.ensf_measure_mfma_rate(7, ctypes.byref(out), None) == ensf.ENSF_EINVAL
    assert L.ensf_measure_mfma_rate(0, None, None) == ensf.ENSF_EINVAL
