"""Parity of the selector network's HIP kernels (forward, gradient, Adam,
selection) with the float64 oracle, and a training run on the device (GPU).

Tolerances: the kernels compute in FP32 with fused multiply-adds over at most
64 terms per unit, so outputs and gradients are compared with a relative
error bound of 1e-4 of the largest magnitude in the compared array (float32
epsilon 1.2e-7 times a few hundred accumulated roundings), plus 1e-6.
"""

import numpy as np
import pytest

from oracle import mlp as omlp

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


def _close(a, b, rel=1e-4, abs_=1e-6):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    bound = rel * max(1.0, float(np.abs(b).max(initial=0.0))) + abs_
    err = float(np.abs(a - b).max(initial=0.0))
    assert err <= bound, (err, bound)


def _params(seed):
    rng = np.random.default_rng(seed)
    return (omlp.init_params(rng) + rng.normal(0, 0.05, omlp.param_count())).astype(np.float32)


@pytest.mark.parametrize("B", [1, 37, 300])
def test_forward_matches_oracle(torch_cuda, mag, B):
    torch = torch_cuda
    p = _params(B)
    X = np.random.default_rng(B + 1).random((B, 16)).astype(np.float32)
    sel = mag.Selector(p)
    y = sel.forward(torch.from_numpy(X).cuda()).cpu().numpy()
    ref, _ = omlp.forward(p.astype(np.float64), X.astype(np.float64))
    _close(y, ref)
    sel.close()


@pytest.mark.parametrize("B", [1, 50, 257])
def test_gradient_and_loss_match_oracle(torch_cuda, mag, B):
    torch = torch_cuda
    rng = np.random.default_rng(7 + B)
    p = _params(100 + B)
    X = rng.random((B, 16)).astype(np.float32)
    T = rng.normal(size=(B, 64)).astype(np.float32)
    M = (rng.random((B, 64)) < 0.25).astype(np.uint8)
    M[0, 0] = 1
    sel = mag.Selector(p)
    g, loss = sel.grad(torch.from_numpy(X).cuda(), torch.from_numpy(T).cuda(),
                       torch.from_numpy(M).cuda())
    L, gref = omlp.loss_and_grad(p.astype(np.float64), X.astype(np.float64), T.astype(np.float64), M)
    _close(g.cpu().numpy(), gref)
    assert abs(float(loss.item()) - L) <= 1e-4 * max(1.0, L)
    sel.close()


def test_gradient_of_unlabelled_batch_is_zero(torch_cuda, mag):
    torch = torch_cuda
    sel = mag.Selector(_params(3))
    X = torch.rand((9, 16), device="cuda")
    g, loss = sel.grad(X, torch.zeros((9, 64), device="cuda"),
                       torch.zeros((9, 64), dtype=torch.uint8, device="cuda"))
    assert float(g.abs().max().item()) == 0.0 and float(loss.item()) == 0.0
    sel.close()


def test_adam_steps_match_oracle(torch_cuda, mag):
    torch = torch_cuda
    rng = np.random.default_rng(21)
    p = _params(21)
    sel = mag.Selector(p)
    ref = p.astype(np.float64)
    m = np.zeros_like(ref)
    v = np.zeros_like(ref)
    for t in range(1, 4):
        g = rng.normal(0, 0.1, p.size).astype(np.float32)
        sel.adam(torch.from_numpy(g).cuda(), 1e-3)
        ref, m, v = omlp.adam_step(ref, g.astype(np.float64), m, v, t, 1e-3)
    torch.cuda.synchronize()
    _close(sel.get_params(), ref, rel=1e-5)
    sel.close()


def test_select_is_the_masked_argmin(torch_cuda, mag):
    torch = torch_cuda
    rng = np.random.default_rng(31)
    B = 200
    p = _params(31)
    X = rng.random((B, 16)).astype(np.float32)
    F = (rng.random((B, 64)) < 0.3).astype(np.uint8)
    F[:5] = 0                                   # nothing feasible
    sel = mag.Selector(p)
    xd = torch.from_numpy(X).cuda()
    pick = sel.select(xd, torch.from_numpy(F).cuda()).cpu().numpy()
    y = sel.forward(xd).cpu().numpy()
    ref, _ = omlp.forward(p.astype(np.float64), X.astype(np.float64))
    for b in range(B):
        if not F[b].any():
            assert pick[b] == -1
            continue
        feas = np.flatnonzero(F[b])
        assert F[b, pick[b]] == 1
        # the decision is taken in FP32 on the kernel's own outputs
        ymin = y[b, feas].min()
        assert y[b, pick[b]] == ymin and pick[b] == feas[np.argmax(y[b, feas] == ymin)]
        # and agrees with the float64 oracle wherever its margin is clear
        r = ref[b, feas]
        order = np.sort(r)
        if order.size > 1 and order[1] - order[0] > 1e-3:
            assert pick[b] == feas[np.argmin(r)]
    sel.close()


def test_learned_pick_and_fallback(torch_cuda, mag):
    from synth import make_job
    job = make_job(100_000, 20, "uniform", 300, 16, 0.5, 5)
    empty = mag.Selector()                      # no parameters set: heuristic fallback
    assert empty.pick(job.patterns) == {"select": "heuristic"}
    empty.close()
    sel = mag.Selector(_params(5))
    got = sel.pick(job.patterns)
    cand = mag.select_candidates(job.patterns)
    assert got["select"] == "learned"
    assert got in [mag.choice_kwargs(c) for c in cand if c is not None]
    many = sel.picks([job.patterns] * 3)
    assert all({k: v for k, v in d.items() if k != "candidate"} == got for d in many)
    assert all(cand[d["candidate"]] is not None for d in many)
    sel.close()


def test_training_on_device_fits_a_known_cost(torch_cuda, mag):
    """Train from scratch on targets the network can represent (a fixed
    random network's outputs); the device's own kernels must cut the loss by
    two orders of magnitude."""
    torch = torch_cuda
    rng = np.random.default_rng(41)
    teacher = _params(41)
    X = rng.random((2048, 16)).astype(np.float32)
    T, _ = omlp.forward(teacher.astype(np.float64), X.astype(np.float64))
    M = (rng.random((2048, 64)) < 0.2).astype(np.uint8)
    student = mag.Selector(omlp.init_params(np.random.default_rng(42)).astype(np.float32))
    xd = torch.from_numpy(X).cuda()
    td = torch.from_numpy(T.astype(np.float32)).cuda()
    md = torch.from_numpy(M).cuda()
    _, l0 = student.grad(xd, td, md)
    loss0 = float(l0.item())
    loss = torch.empty(1, device="cuda")
    for step in range(1500):
        i = (step * 256) % 2048
        student.train_step(xd[i:i + 256], td[i:i + 256], md[i:i + 256], 3e-3, loss)
    _, l1 = student.grad(xd, td, md)
    assert float(l1.item()) < loss0 / 100, (loss0, float(l1.item()))
    student.close()
