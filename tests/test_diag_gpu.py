"""The MFMA stream diagnostic (hess_mfma_stream_rate): each instruction's register-only
rate stays below the device's published dense peak for it, and the BF16 streams come
within reach of it.  A stream kernel whose accumulators are copied between register
files every iteration measured about half the BF16 peak, which the floor catches."""
import pytest

pytestmark = pytest.mark.gpu

# published dense peaks of the device (TFLOP/s): FP32 and FP64 matrix, BF16 dense
PEAK = {"f32_16x16x4": 157.3, "bf16_16x16x32": 2500.0, "bf16_32x32x16": 2500.0, "f64_16x16x4": 78.6}


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_1905_05559_amd import api
    assert torch.cuda.is_available()
    return api.Context(0)


@pytest.mark.parametrize("kind", sorted(PEAK))
def test_stream_rate_below_peak(ctx, kind):
    rate = ctx.mfma_stream_rate(kind, 20000)
    print("case stream %s: %.1f TFLOP/s" % (kind, rate), flush=True)
    assert 0.0 < rate <= 1.1 * PEAK[kind]


@pytest.mark.parametrize("kind", ["bf16_16x16x32", "bf16_32x32x16"])
def test_bf16_stream_reaches_most_of_peak(ctx, kind):
    rate = ctx.mfma_stream_rate(kind, 200000)
    print("case stream %s: %.1f TFLOP/s" % (kind, rate), flush=True)
    assert rate >= 0.7 * PEAK[kind]
