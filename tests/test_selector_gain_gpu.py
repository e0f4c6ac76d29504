"""What the trained selector gains over the method's fixed heuristic (GPU).

Held-out pattern sets (drawn from a seed the training never saw) over 64 MiB
texts: each set is scanned with the heuristic's (q, k, sigma') and with the
network's pick, and the scan kernel's device time is compared. Both plans
are exact, so they must find the same number of occurrences; a few learned
plans are also checked against the oracle in full.
"""

import math

import numpy as np
import pytest

from oracle import match as om

pytestmark = pytest.mark.gpu

SETS = 120


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    return torch


def _kernel_ms(mag, text, plan, out, cnt):
    best = math.inf
    mag.profile_enable(True)
    for _ in range(2):
        mag.profile_read()
        mag.scan_async(text, plan, out, cnt)
        best = min(best, mag.profile_read()["scan_ms"])
    mag.profile_enable(False)
    return best


def test_learned_picks_beat_the_fixed_heuristic(torch_cuda):
    torch = torch_cuda
    import synth
    import paper_1405_5483_amd as mag
    from paper_1405_5483_amd import train_selector as ts

    texts = ts.make_texts(synth, 64 << 20, 6)
    dtexts = [torch.from_numpy(t).cuda() for t in texts]
    recipes = ts.set_recipes(SETS, 6)
    sets = [ts.make_set(synth, texts, rec) for rec in recipes]
    sel = mag.Selector.load()
    picks = sel.picks(sets)
    assert sum(p["select"] == "learned" for p in picks) == SETS
    out = torch.empty((8192, 2), dtype=torch.int64, device="cuda")
    cnt = torch.empty(1, dtype=torch.int64, device="cuda")
    ratios, th, tl = [], 0.0, 0.0
    for i, (rec, P, pk) in enumerate(zip(recipes, sets, picks)):
        hp, lp = mag.Plan(P), mag.Plan(P, **pk)
        h = _kernel_ms(mag, dtexts[rec[0]], hp, out, cnt)
        zh = int(cnt.item())
        lt = _kernel_ms(mag, dtexts[rec[0]], lp, out, cnt)
        assert int(cnt.item()) == zh, i
        if i < 3:       # full parity of a few learned plans
            occ = mag.scan(dtexts[rec[0]], lp).cpu().numpy()
            pos, ids = om.occ_hashed(texts[rec[0]], P)
            assert np.array_equal(occ[:, 0].astype(np.uint64), pos)
            assert np.array_equal(occ[:, 1].astype(np.uint32), ids)
        ratios.append(h / lt)
        th += h
        tl += lt
        hp.close()
        lp.close()
    geo = math.exp(sum(math.log(r) for r in ratios) / len(ratios))
    win = sum(r > 1 for r in ratios) / len(ratios)
    print(f"held-out sets {SETS}: geometric-mean speedup {geo:.3f}, win rate {win:.2f}, "
          f"total {th:.1f} ms -> {tl:.1f} ms")
    assert geo > 1.2 and win > 0.55
