"""The bandwidth diagnostics the benchmark uses: the copy kernel copies, the gather only reads its region
and rejects bad line sizes and misaligned regions."""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


def test_diag_copy_copies(hc):
    src = torch.randint(0, 255, (1 << 22,), dtype=torch.uint8, device="cuda")
    dst = torch.zeros_like(src)
    hc.hc_diag_copy(dst, src)
    torch.cuda.synchronize()
    assert torch.equal(src, dst)
    with pytest.raises(hc.HcError) as e:
        hc.hc_diag_copy(dst[:17], src[:17])
    assert e.value.code == hc.E_ARG
    sink = torch.zeros(1, dtype=torch.uint32, device="cuda")
    hc.hc_diag_read(src, sink)
    hc.hc_diag_copy(dst[: (1 << 22) - 48], src[48:])  # a size that leaves a tail for the second loop
    torch.cuda.synchronize()
    assert torch.equal(dst[: (1 << 22) - 48], src[48:])


@pytest.mark.parametrize("line_bytes", [32, 64, 128])
def test_diag_gather_runs_in_bounds(hc, line_bytes):
    region = torch.arange(1 << 20, dtype=torch.int32, device="cuda").view(torch.uint8)
    sink = torch.zeros(1, dtype=torch.uint32, device="cuda")
    before = region.clone()
    hc.hc_diag_gather(region.data_ptr(), region.numel(), line_bytes, 1 << 16, sink, 7)
    torch.cuda.synchronize()
    assert torch.equal(region, before)  # reads only
    with pytest.raises(hc.HcError) as e:
        hc.hc_diag_gather(region.data_ptr(), region.numel(), 48, 16, sink)
    assert e.value.code == hc.E_ARG
    with pytest.raises(hc.HcError) as e:
        hc.hc_diag_gather(region.data_ptr() + 4, region.numel() - 128, line_bytes, 16, sink)
    assert e.value.code == hc.E_ARG


def test_diag_atomics_stay_in_region(hc):
    region = torch.zeros(1 << 16, dtype=torch.int64, device="cuda")
    sink = torch.zeros(1, dtype=torch.uint32, device="cuda")
    hc.hc_diag_atomic(region, True, 1 << 15, sink, 3)  # CAS of 0 into zero words: every word changes at most once
    torch.cuda.synchronize()
    changed = int((region != 0).sum().item())
    assert 0 < changed <= 1 << 15
    region.zero_()
    hc.hc_diag_atomic(region, False, 1 << 15, sink, 5)  # ORs: at most one bit per op
    torch.cuda.synchronize()
    bits = int(np.unpackbits(region.cpu().numpy().view(np.uint8)).sum())
    assert 0 < bits <= 1 << 15
    with pytest.raises(hc.HcError) as e:
        hc.hc_diag_atomic(region[:0], True, 16, sink)
    assert e.value.code == hc.E_ARG
