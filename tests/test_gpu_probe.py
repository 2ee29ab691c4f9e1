"""tn_probe_mfma: the matrix-core rate with no memory traffic lies between a
tenth of MI355X's nominal dense peak and the peak itself (FP32 MFMA 157.3
TFLOP/s, bf16 2516.6); other precisions are refused."""
import pytest

from paper_2507_20667_amd import lib

pytestmark = pytest.mark.gpu


def test_probe_rates():
    with lib.Context(64 << 20) as c:
        f32 = lib.tn_probe_mfma(c.handle, lib.TN_PREC_FP32)
        bf16 = lib.tn_probe_mfma(c.handle, lib.TN_PREC_BF16X3)
        assert 15.7 < f32 <= 157.3 * 1.01, f32
        assert 251.7 < bf16 <= 2516.6 * 1.01, bf16
        assert bf16 > 4 * f32
        with pytest.raises(lib.TnError) as e:
            lib.tn_probe_mfma(c.handle, 7)
        assert e.value.status == lib.TN_E_INVALID_ARG
