"""Pins of the oracle's training-step pieces (Sec. 3.3-3.4): softplus density,
cosine learning-rate schedules, Adam with held groups, the densification
score and its multinomial sampling, and the pruning rule.

Library routines serve as independent references where they exist (torch's
softplus, CosineAnnealingLR and Adam, all in float64); the rest is checked on
hand-built cases and invariants.
"""

import math

import numpy as np
import pytest
import torch

from oracle import training as tr


def test_softplus_matches_torch():
    x = np.concatenate([np.linspace(-5, 5, 2001), [-3.1, 0.0, 2.5]])   # |beta x| <= 50: torch's exp stays finite
    xt = torch.tensor(x, dtype=torch.float64, requires_grad=True)
    ref = torch.nn.functional.softplus(xt, beta=10.0, threshold=1e9)
    np.testing.assert_allclose(tr.softplus(x), ref.detach().numpy(), rtol=1e-14, atol=1e-300)
    ref.sum().backward()
    np.testing.assert_allclose(tr.softplus_grad(x), xt.grad.numpy(), rtol=1e-13, atol=1e-300)
    assert tr.softplus(0.0) == pytest.approx(math.log(2.0) / 10.0, rel=1e-15)
    assert tr.softplus(80.0) == pytest.approx(80.0, rel=1e-15)
    assert 0.0 < tr.softplus(-60.0) == pytest.approx(math.exp(-600.0) / 10.0, rel=1e-12)
    assert tr.softplus_grad(-60.0) == pytest.approx(math.exp(-600.0), rel=1e-12) and tr.softplus_grad(80.0) == 1.0


def test_cosine_schedule_matches_torch():
    total = 50
    for lr0, lr_end in ((2e-4, 2e-6), (1e-1, 1e-2)):
        p = torch.zeros(1, requires_grad=True)
        opt = torch.optim.SGD([p], lr=lr0)
        sch = torch.optim.lr_scheduler.CosineAnnealingLR(opt, T_max=total, eta_min=lr_end)
        for it in range(total):
            assert tr.cosine_lr(it, total, lr0, lr_end) == pytest.approx(opt.param_groups[0]["lr"], rel=1e-12)
            opt.step()
            sch.step()
    s0, s_end = tr.schedule(0, 20000), tr.schedule(19999, 20000)
    assert s0["lr"]["sites"] == pytest.approx(2e-4) and s0["lr"]["sh_high"] == 0.0
    assert s_end["lr"]["sites"] == 0.0 and s_end["lr"]["density"] == pytest.approx(1e-2, rel=1e-6)
    assert tr.schedule(4999, 20000)["lr"]["sh_high"] == 0.0 and tr.schedule(5000, 20000)["lr"]["sh_high"] > 0.0
    assert tr.schedule(17999, 20000)["lr"]["sites"] > 0.0 and tr.schedule(18000, 20000)["lr"]["sites"] == 0.0


def test_adam_steps_match_torch_with_held_groups():
    """A whole short run of the schedule against torch.optim.Adam (float64),
    holding a group by giving it no gradient (torch then advances neither its
    moments nor its step count)."""
    rng = np.random.default_rng(1)
    N, B, total = 7, 4, 20
    p = {"sites": rng.standard_normal((N, 3)), "density": rng.standard_normal(N) * 0.3,
         "sh": rng.standard_normal((N, B, 3))}
    m = {k: np.zeros_like(v) for k, v in p.items()}
    v = {k: np.zeros_like(x) for k, x in p.items()}
    tp = {"sites": torch.tensor(p["sites"], requires_grad=True),
          "density": torch.tensor(p["density"], requires_grad=True),
          "sh0": torch.tensor(p["sh"][:, :1].copy(), requires_grad=True),
          "sh_high": torch.tensor(p["sh"][:, 1:].copy(), requires_grad=True)}
    opt = torch.optim.Adam([{"params": [tp[g]], "name": g} for g in tr.GROUPS], lr=1.0, betas=(0.9, 0.999),
                           eps=1e-15)
    for it in range(total):
        g = {"sites": rng.standard_normal((N, 3)), "density": rng.standard_normal(N),
             "sh": rng.standard_normal((N, B, 3))}
        p, m, v = tr.adam_step(p, g, m, v, it, total, softplus_density=True)
        sc = tr.schedule(it, total)
        gd = torch.tensor(g["density"]) * torch.sigmoid(10.0 * tp["density"].detach())
        grads = {"sites": torch.tensor(g["sites"]), "density": gd, "sh0": torch.tensor(g["sh"][:, :1].copy()),
                 "sh_high": torch.tensor(g["sh"][:, 1:].copy())}
        for grp in opt.param_groups:
            name = grp["name"]
            grp["lr"] = sc["lr"][name]
            tp[name].grad = grads[name] if sc["lr"][name] > 0 else None
        opt.step()
        np.testing.assert_allclose(p["sites"], tp["sites"].detach().numpy(), rtol=1e-12, atol=1e-14)
        np.testing.assert_allclose(p["density"], tp["density"].detach().numpy(), rtol=1e-12, atol=1e-14)
        np.testing.assert_allclose(p["sh"][:, :1], tp["sh0"].detach().numpy(), rtol=1e-12, atol=1e-14)
        np.testing.assert_allclose(p["sh"][:, 1:], tp["sh_high"].detach().numpy(), rtol=1e-12, atol=1e-14)


def test_adam_first_step_is_a_signed_learning_rate():
    """With zero moments, the bias-corrected first step is lr * g / (|g| + eps)."""
    g = np.array([3.0, -0.2, 1e-3, 0.0])
    x, m, v = tr.adam_update(np.zeros(4), g, np.zeros(4), np.zeros(4), lr=0.01, t=1, eps=1e-15)
    np.testing.assert_allclose(x, -0.01 * g / (np.abs(g) + 1e-15), rtol=1e-12)


def _tetra():
    # a regular-ish tetrahedron plus one far site joined to vertex 0 only
    sites = np.array([[0, 0, 0], [2, 0, 0], [0, 2, 0], [0, 0, 2], [6, 0, 0]], dtype=np.float64)
    nbrs = [[1, 2, 3, 4], [0, 2, 3], [0, 1, 3], [0, 1, 2], [0]]
    off = np.concatenate([[0], np.cumsum([len(n) for n in nbrs])]).astype(np.int32)
    idx = np.concatenate(nbrs).astype(np.int32)
    return sites, off, idx


def test_densify_score_by_hand():
    sites, off, idx = _tetra()
    r = tr.cell_radius(sites, off, idx)
    s2 = 2 * math.sqrt(2.0)
    np.testing.assert_allclose(r, [0.5 * (2 + 2 + 2 + 6) / 4, 0.5 * (2 + s2 + s2) / 3, 0.5 * (2 + s2 + s2) / 3,
                                   0.5 * (2 + s2 + s2) / 3, 0.5 * 6], rtol=1e-15)
    g = np.array([[3, 4, 0], [0, 0, 1], [0, 0, 0], [1, 1, 1], [0, -2, 0]], dtype=np.float64)
    np.testing.assert_allclose(tr.densify_scores(sites, off, idx, g), r * [5, 1, 0, math.sqrt(3), 2], rtol=1e-15)
    # scaling positions by s scales radii (and scores at fixed gradients) by s
    np.testing.assert_allclose(tr.cell_radius(sites * 3.0, off, idx), 3.0 * r, rtol=1e-15)


def test_sampling_follows_the_distribution():
    rng = np.random.default_rng(2)
    scores = rng.uniform(0, 1, 50) * (rng.uniform(0, 1, 50) > 0.3)
    K = 100000
    u = (np.arange(K) + 0.5) / K                   # stratified: counts within one of K p
    counts = np.bincount(tr.sample_cells(scores, u), minlength=50)
    np.testing.assert_allclose(counts, K * scores / scores.sum(), atol=1.0 + 1e-9)
    assert np.all(counts[scores == 0] == 0)
    first, last = np.nonzero(scores)[0][[0, -1]]
    assert tr.sample_cells(scores, [0.0])[0] == first
    assert tr.sample_cells(scores, [1.0 - 1e-16])[0] == last
    # cell i owns [C_{i-1}, C_i) of the cumulative sum: exact boundaries go to
    # the next cell with a positive score, never to an empty one
    exact = np.array([0.0, 0.0, 1.0, 1.0, 0.0, 2.0])
    np.testing.assert_array_equal(tr.sample_cells(exact, [0.0, 0.25, 0.5, 0.75]), [2, 3, 5, 5])


def test_prune_mask_by_hand():
    # a path 0-1-2-3-4 and an isolated cell 5
    off = np.array([0, 1, 3, 5, 7, 8, 8], dtype=np.int32)
    idx = np.array([1, 0, 2, 1, 3, 2, 4, 3], dtype=np.int32)
    dens = np.array([0.0, 0.0, 0.5, 0.001, 0.0, 0.0])
    np.testing.assert_array_equal(tr.prune_mask(dens, off, idx, 0.01), [True, False, False, False, True, True])
    np.testing.assert_array_equal(tr.prune_mask(dens, off, idx, 0.6), [True] * 6)
    np.testing.assert_array_equal(tr.prune_mask(dens, off, idx, 0.0), [False] * 6)
