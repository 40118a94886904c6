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


# ---------------------------------------------------------------------------
# inserting and removing sites, growth and rebuild schedules
# ---------------------------------------------------------------------------

def _small_scene(n, seed, sh_deg=1):
    import synth

    return synth.small_scene("clustered", n, seed=seed, sh_deg=sh_deg)


def _unit_ball(rng, n):
    u = rng.standard_normal((n, 3))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    return u * rng.uniform(0, 1, (n, 1)) ** (1 / 3)


def test_inserted_sites_lie_inside_their_parents_cells():
    sc = _small_scene(600, 41)
    rng = np.random.default_rng(42)
    parents = rng.integers(0, sc.n_sites, 400)
    x = sc.sites.astype(np.float64)
    # the inscribed radius is half the distance to the nearest site at all (brute force)
    d = np.linalg.norm(x[:, None, :] - x[None, :, :], axis=-1)
    np.fill_diagonal(d, np.inf)
    np.testing.assert_allclose(tr.inscribed_radius(x, sc.off, sc.idx), 0.5 * d.min(axis=1), rtol=1e-15)
    for frac in (0.5, 0.999):
        new = tr.insert_sites(x, sc.off, sc.idx, parents, _unit_ball(rng, 400), frac=frac)
        nn = np.argmin(np.linalg.norm(new[:, None, :] - x[None, :, :], axis=-1), axis=1)
        np.testing.assert_array_equal(nn, parents)
    # towards the nearest neighbour the cell ends exactly at the inscribed radius
    p = parents[:50]
    j = np.argmin(d[p], axis=1)
    u = (x[j] - x[p]) / np.linalg.norm(x[j] - x[p], axis=1, keepdims=True)
    out = tr.insert_sites(x, sc.off, sc.idx, p, u, frac=1.001)
    closer = np.linalg.norm(out - x[j], axis=1) < np.linalg.norm(out - x[p], axis=1)
    assert closer.all()


def _render(sites, density, sh, sh_deg, o, d, t):
    import oracle
    import synth

    s32 = np.asarray(sites, dtype=np.float32)
    off, idx = synth.build_adjacency(s32)
    osc = oracle.OracleScene(s32, off, idx, density, sh, sh_deg)
    start = synth.nearest_site(s32, o).astype(np.int32)
    return oracle.forward(osc, o, d, t, start, eps=0.0)


def _rays(rng, n):
    o = rng.uniform(-0.8, 0.8, (n, 3))
    d = rng.standard_normal((n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    return o, d, np.full(n, 0.9)


def test_densify_and_prune_change_the_render_as_the_geometry_says():
    """The field is piecewise constant. A child with its parent's density and
    colour, placed at a distance f r_p from its parent, moves only bisectors
    near the parent by O(f r_p): the mean change of the renders is linear in f
    (with a wrong copy of the attributes the child's half of the parent's cell
    would change them at any f). Removing an empty cell whose neighbours are all empty
    hands its volume to those neighbours (a point's second-nearest site is a
    Delaunay neighbour of its nearest): no render changes (transmittance test
    off)."""
    sc = _small_scene(800, 43)
    rng = np.random.default_rng(44)
    o, d, t = _rays(rng, 300)
    x = sc.sites.astype(np.float32).astype(np.float64)
    dens = sc.density.astype(np.float64)
    sh = sc.sh.astype(np.float64)
    ref_rgb, ref_t, _ = _render(x, dens, sh, 1, o, d, t)
    parents = rng.integers(0, sc.n_sites, 200)
    u = _unit_ball(rng, 200)
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    moments = [{"sites": np.ones_like(x), "density": np.ones_like(dens), "sh": np.ones_like(sh)}]
    change = []
    for frac in (1e-3, 1e-4):
        new = tr.insert_sites(x, sc.off, sc.idx, parents, u, frac=frac)
        params, mom = tr.densify({"sites": x, "density": dens, "sh": sh}, moments, parents, new)
        assert params["sites"].shape == (1000, 3) and np.all(mom[0]["density"][800:] == 0)
        assert np.all(mom[0]["sh"][:800] == 1)
        np.testing.assert_array_equal(params["sh"][800:], sh[parents])
        np.testing.assert_array_equal(params["density"][800:], dens[parents])
        rgb, T, steps = _render(params["sites"], params["density"], params["sh"], 1, o, d, t)
        change.append(np.abs(rgb - ref_rgb).mean())
    # the mean change over the rays is linear in f
    assert 7.0 < change[0] / change[1] < 14.0, change
    assert change[1] < 1e-4 * np.abs(ref_rgb).mean()
    # empty cells with empty neighbours: removing them changes nothing
    dens2 = dens.copy()
    dens2[rng.uniform(0, 1, len(dens2)) < 0.95] = 0.0
    ref2 = _render(x, dens2, sh, 1, o, d, t)
    keep = ~tr.prune_mask(dens2, sc.off, sc.idx, 1e-30)
    assert 20 < (~keep).sum() < 790
    p2, m2 = tr.remove_sites({"sites": x, "density": dens2, "sh": sh}, moments, keep)
    got2 = _render(p2["sites"], p2["density"], p2["sh"], 1, o, d, t)
    np.testing.assert_allclose(got2[0], ref2[0], rtol=0, atol=1e-12)
    np.testing.assert_allclose(got2[1], ref2[1], rtol=1e-12)
    np.testing.assert_array_equal(p2["sites"], x[keep])
    # a cell with density is never removed
    assert np.all(keep[dens2 > 0])


def test_growth_and_rebuild_schedules_by_hand():
    assert [tr.grow_target(i, 100, 10, 110, 10) for i in (0, 10, 30, 50, 99)] == [10, 10, 60, 110, 110]
    # rebuilt after the step of a densification, then after 1, 2, 3, ... steps
    assert tr.rebuild_steps(30, [0]) == [0, 1, 3, 6, 10, 15, 21, 28]
    assert tr.rebuild_steps(30, [0, 12]) == [0, 1, 3, 6, 10, 12, 13, 15, 18, 22, 27]
    long = tr.rebuild_steps(20000, [0])
    gaps = np.diff(long)
    assert gaps.max() == 100 and gaps[0] == 1 and np.all(np.diff(gaps) >= 0)
