"""The measured roofline denominators: each MFMA form reaches a plausible share of
its published dense peak and the copy a plausible share of the HBM bandwidth (the
bounds only catch a broken probe, e.g. a wrong FLOP count per instruction or a
copy that moves a fraction of the buffer)."""
import pytest
import torch

pytestmark = pytest.mark.gpu

SPEC = {"fp32": 157.3, "bf16": 2500.0, "fp8": 5000.0}


@pytest.mark.parametrize("precision,iters", [("fp32", 20000), ("bf16", 40000), ("fp8", 20000)])
def test_mfma_probe(precision, iters):
    from paper_2501_05520_amd import trk
    t = trk.trk_probe_mfma(precision, iters)
    print(f"{precision}: {t:.1f} TFLOP/s measured, {SPEC[precision]} published")
    assert 0.3 * SPEC[precision] <= t <= 1.05 * SPEC[precision]


@pytest.mark.parametrize("n", [64 << 20, (64 << 20) + 12, 4])
def test_copy_probe(n):
    # distinct words, so that a copy to the wrong place is seen; sizes with and
    # without a tail past the four-load steps, and a single 16-byte unit
    from paper_2501_05520_amd import trk
    a = torch.arange(n, dtype=torch.int32, device="cuda")
    b = torch.full_like(a, -1)
    g = trk.trk_probe_copy(a, b, reps=3)
    torch.cuda.synchronize()
    print(f"copy of {4 * n} bytes: {g:.0f} GB/s")
    assert torch.equal(a, b)
    if n >= 1 << 20:
        assert 1000.0 <= g <= 8000.0
