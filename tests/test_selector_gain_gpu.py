"""What the trained selector gains over the method's fixed heuristic (GPU).

Held-out pattern sets (drawn from a seed the training never saw) over 64 MiB
texts: each set is scanned with the heuristic's plan and with the network's
pick, and the scan kernel's device time is compared. Both plans are exact,
so their sorted occurrence lists must be identical (compared in full for
every set with at most 2^20 occurrences); every 20th learned list is also
checked against the oracle.
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
    cap = 1 << 20
    out_h = torch.empty((cap, 2), dtype=torch.int64, device="cuda")
    out_l = torch.empty((cap, 2), dtype=torch.int64, device="cuda")
    cnt_h = torch.empty(1, dtype=torch.int64, device="cuda")
    cnt_l = torch.empty(1, dtype=torch.int64, device="cuda")
    ratios, th, tl, compared = [], 0.0, 0.0, 0
    for i, (rec, P, pk) in enumerate(zip(recipes, sets, picks)):
        hp, lp = mag.Plan(P), mag.Plan(P, **pk)
        h = _kernel_ms(mag, dtexts[rec[0]], hp, out_h, cnt_h)
        lt = _kernel_ms(mag, dtexts[rec[0]], lp, out_l, cnt_l)
        zh, zl = int(cnt_h.item()), int(cnt_l.item())
        assert zl == zh, i
        if zh <= cap:   # both sorted lists in full
            compared += 1
            assert torch.equal(out_h[:zh], out_l[:zl]), i
        if i % 20 == 0:  # and against the oracle
            occ = out_l[:zl].cpu().numpy()
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
    assert compared >= SETS * 3 // 4      # sets over 2^20 occurrences compare counts only
    assert geo > 1.2 and win > 0.55
