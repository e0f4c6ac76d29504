"""The allocation-free scan entry point (``mag_scan_noalloc``) against
``mag_scan_async`` (GPU).

Both are called through the C ABI on the same plans and texts; the records and
counts must be identical (and equal to the oracle's), on two calls in a row,
the second with a smaller text, for filter, deferred-filter and both dense
plans, with outputs small enough for the in-LDS finishing sort and large
enough for the device-wide radix sort. Argument errors are checked before
anything is enqueued.
"""

import numpy as np
import pytest

from oracle import match as om
from synth import gen_patterns, gen_text

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    return torch


@pytest.fixture(scope="module")
def mag():
    import paper_1405_5483_amd as m
    return m


def _records(torch, mag, fn, text, plan, cap):
    out = torch.full((cap, 2), -1, dtype=torch.int64, device="cuda")
    cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
    st = torch.zeros(7, dtype=torch.int64, device="cuda")
    fn(text, plan, out, cnt, st)
    torch.cuda.synchronize()
    z = int(cnt.item())
    return z, out[:min(z, cap)].cpu().numpy(), st.cpu().numpy()


CASES = [
    # name, sigma, n, r, m, plan keywords, out_cap
    ("filter", 4, 400_003, 100, 16, {}, 4096),
    ("deferred", 20, 300_001, 200, 16, dict(q=3, k=1, sigma_prime=4, mode="filter",
                                            verify="deferred", verify_buffer=4096), 4096),
    ("dense-slices", 20, 500_000, 20_000, 16, dict(mode="dense", dense_probe="slices"), 1 << 20),
    ("dense-bloom", 4, 300_000, 3000, 8, dict(mode="dense", dense_probe="bloom"), 1 << 18),
]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_noalloc_equals_scan_async(torch_cuda, mag, case):
    name, sigma, n, r, m, kw, cap = case
    T = gen_text(n, sigma, rng=n + 5)
    P = gen_patterns(T, r, m, (3 * r) // 4, sigma, rng=r + 6)
    plan = mag.Plan(P, **kw)
    for size in (n, n // 3):          # two calls in a row, the second smaller
        t = T[:size]
        text = torch_cuda.from_numpy(t).cuda()
        za, ra, sa = _records(torch_cuda, mag, mag.scan_async, text, plan, cap)
        zb, rb, sb = _records(torch_cuda, mag, mag.scan_noalloc, text, plan, cap)
        pos, ids = om.occ_hashed(t, P)
        assert za == zb == pos.size, (name, size, za, zb, pos.size)
        assert zb <= cap
        assert np.array_equal(ra, rb), (name, size)
        assert np.array_equal(rb[:, 0].astype(np.uint64), pos)
        assert np.array_equal(rb[:, 1].astype(np.uint32), ids)
        assert np.array_equal(sa, sb)
    plan.close()


def test_noalloc_argument_errors(torch_cuda, mag):
    T = gen_text(10_000, 4, rng=1)
    P = gen_patterns(T, 10, 16, 5, 4, rng=2)
    text = torch_cuda.from_numpy(T).cuda()
    cnt = torch_cuda.zeros(1, dtype=torch_cuda.int64, device="cuda")
    fresh = mag.Plan(P)                 # never scanned: its tables are not on the device
    small = torch_cuda.empty((16, 2), dtype=torch_cuda.int64, device="cuda")
    with pytest.raises(mag.MagError):
        mag.scan_noalloc(text, fresh, small, cnt)
    mag.scan_async(text, fresh, small, cnt)          # uploads the plan
    torch_cuda.cuda.synchronize()
    big = torch_cuda.empty(((1 << 20) + 1, 2), dtype=torch_cuda.int64, device="cuda")
    with pytest.raises(mag.MagError):
        mag.scan_noalloc(text, fresh, big, cnt)
    mag.scan_noalloc(text, fresh, small, cnt)
    torch_cuda.cuda.synchronize()
    assert int(cnt.item()) == om.occ_hashed(T, P)[0].size
