"""tn_probe_mfma: the matrix-core rate with no memory traffic, on changing
or constant operands, lies between a tenth of MI355X's nominal dense peak
and the peak itself (FP32 MFMA 157.3 TFLOP/s, bf16 2516.6); other
precisions are refused."""
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
        # constant operands: within the same bounds, and not much slower than
        # changing ones (less switching: no lower clock)
        f32c = lib.tn_probe_mfma(c.handle, lib.TN_PREC_FP32 | lib.TN_PROBE_CONST_OPERANDS)
        bf16c = lib.tn_probe_mfma(c.handle, lib.TN_PREC_BF16X3 | lib.TN_PROBE_CONST_OPERANDS)
        assert 15.7 < f32c <= 157.3 * 1.01, f32c
        assert 251.7 < bf16c <= 2516.6 * 1.01, bf16c
        assert f32c > 0.9 * f32 and bf16c > 0.9 * bf16, (f32, f32c, bf16, bf16c)
        with pytest.raises(lib.TnError) as e:
            lib.tn_probe_mfma(c.handle, 7)
        assert e.value.status == lib.TN_E_INVALID_ARG
