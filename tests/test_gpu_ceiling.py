"""The measured rate ceilings (nmf_ceiling): every rate is positive and
below the published MI355X peak of its kind (a rate above it would mean the
work is miscounted), and the read stream visits every item of its buffer
exactly once (its per-workgroup sums of a buffer of ones add up to the item
count)."""
import numpy as np
import pytest

from paper_1003_3272_amd import nmf

pytestmark = pytest.mark.gpu

# published peaks: HBM bytes/s; dense flop/s of each instruction's type
PEAK = {"hbm_read": 8.0e12, "mfma_f32": 157.3e12, "mfma_bf16": 2.5e15, "mfma_f64": 78.6e12,
        "fma_f64": 78.6e12, "mfma_f32_32": 157.3e12, "mfma_bf16_32": 2.5e15}


@pytest.fixture(scope="module")
def buf():
    import torch
    b = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
    yield b
    del b
    torch.cuda.empty_cache()


@pytest.mark.parametrize("kind", sorted(nmf.CEILING_KINDS))
def test_rate_is_below_the_published_peak(buf, kind):
    rate = nmf.ceiling(kind, buf, reps=3)
    print(f"{kind}: {rate:.4g}", flush=True)
    assert 0.2 * PEAK[kind] < rate <= 1.02 * PEAK[kind]


def test_read_stream_visits_every_item_once(buf):
    import torch
    sink_bytes = 4 << 20
    items = (buf.numel() - sink_bytes) // 4
    buf.view(torch.float32).fill_(1.0)
    nmf.ceiling("hbm_read", buf, reps=1)
    torch.cuda.synchronize()
    sums = buf[buf.numel() - sink_bytes:].view(torch.float32)[:4096].cpu().numpy()
    # each workgroup's sum is an integer below 2^24, exact in float32
    assert np.all(sums == np.round(sums))
    assert float(np.sum(sums.astype(np.float64))) == float(items)


def test_small_buffer_is_rejected():
    import torch
    b = torch.empty(32 << 20, dtype=torch.uint8, device="cuda")
    with pytest.raises(nmf.NmfError):
        nmf.ceiling("mfma_f32", b)
