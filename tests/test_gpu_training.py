"""Training-step kernels on the GPU (Sec. 3.3-3.4) against the float64 oracle:
softplus density in the pack, Adam with the paper's schedule, densification
scores and candidate sampling, the pruning mask, and a short fit that uses
them all around the walk.

Tolerances: FP32 arithmetic against float64 on the same FP32 inputs; Adam
values after many steps within 2e-6 absolute + 1e-5 relative (each step moves
a value by at most ~lr, with FP32 rounding of ~1e-7 relative); indices and
masks bit-exact, except sampled cells whose draw lands within 1e-9 of a
cumulative-sum boundary (double sums in a different order), which only need
to be one of the two cells at that boundary.
"""

import numpy as np
import pytest

import oracle
import synth
from oracle import training as otr

pytestmark = pytest.mark.gpu


def _dv(a):
    import torch

    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.fixture(scope="module")
def scene():
    return synth.small_scene("clustered", 20000, seed=81, sh_deg=3)


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_softplus_density_in_the_pack(scene, dtype):
    import paper_2502_01157_amd as rf

    x = np.random.default_rng(82).normal(0.0, 1.5, scene.n_sites).astype(np.float32)
    x[:6] = [-30.0, -3.0, 0.0, 1.99, 2.01, 40.0]
    p = rf.PackedScene(*map(_dv, (scene.sites, scene.off, scene.idx, x, scene.sh)), 3, dtype,
                       density_activation="softplus")
    got = p.attributes()[0].cpu().numpy().astype(np.float64)
    ref = otr.softplus(x.astype(np.float64))
    if dtype == "f32":
        np.testing.assert_allclose(got, ref, rtol=1e-6, atol=1e-30)
    else:
        # bf16 of the FP32 value: within one bf16 step of the exact value
        np.testing.assert_allclose(got, ref, rtol=1.01 * 2 ** -8, atol=1e-30)
    with pytest.raises(KeyError):
        rf.PackedScene(*map(_dv, (scene.sites, scene.off, scene.idx, x, scene.sh)), 3, density_activation="relu")


def test_schedule_matches_oracle():
    import paper_2502_01157_amd as rf

    for total in (40, 20000):
        for it in sorted({0, 1, total // 4 - 1, total // 4, total // 2, total - total // 10 - 1,
                          total - total // 10, total - 1}):
            a = rf.train_schedule(it, total)
            ref = otr.schedule(it, total)
            for g, name in enumerate(otr.GROUPS):
                assert a.lr[g] == pytest.approx(ref["lr"][name], rel=1e-6, abs=0.0)
                assert a.t[g] == ref["t"][name]
            assert a.softplus_density == 1 and a.beta1 == pytest.approx(0.9) and a.eps == pytest.approx(1e-15)
    with pytest.raises(rf.RfError):
        rf.train_schedule(40, 40)


@pytest.mark.parametrize("aligned", [True, False])
def test_adam_run_matches_oracle(aligned):
    """A 36-step run of the schedule (total 40: SH warm-up for 10 steps,
    positions held from step 36), one step at a time against the oracle."""
    import torch

    import paper_2502_01157_amd as rf

    rng = np.random.default_rng(83)
    N, B, total = 1001, 16, 40
    p = {"sites": rng.standard_normal((N, 3)).astype(np.float32),
         "density": rng.normal(0, 0.5, N).astype(np.float32),
         "sh": rng.standard_normal((N, B, 3)).astype(np.float32)}
    m = {k: np.zeros(v.shape) for k, v in p.items()}
    v = {k: np.zeros(x.shape) for k, x in p.items()}

    def place(a):
        # unaligned: a view one float into a larger buffer, so the kernel takes its scalar path
        t = _dv(a.reshape(-1))
        if not aligned:
            buf = torch.empty(t.numel() + 1, dtype=torch.float32, device=t.device)
            buf[1:] = t
            t = buf[1:]
        return t.view(a.shape)

    gp = {k: place(x) for k, x in p.items()}
    st = rf.AdamState(N, 3, gp["sites"].device)
    if not aligned:
        for k in list(st.tensors):
            st.tensors[k] = place(np.zeros(tuple(st.tensors[k].shape), dtype=np.float32))
        st.desc = type(st.desc)(*[st.tensors[k].data_ptr() for k in ("m_sites", "v_sites", "m_density",
                                                                      "v_density", "m_sh", "v_sh")])
    ref = {k: x.astype(np.float64) for k, x in p.items()}
    for it in range(36):
        g = {"sites": rng.standard_normal((N, 3)).astype(np.float32),
             "density": rng.standard_normal(N).astype(np.float32),
             "sh": rng.standard_normal((N, B, 3)).astype(np.float32)}
        rf.adam_step(rf.train_schedule(it, total), st, gp["sites"], gp["density"], gp["sh"], place(g["sites"]),
                     place(g["density"]), place(g["sh"]))
        # the kernel's hyperparameters are FP32: the oracle takes the same values
        ref, m, v = otr.adam_step(ref, {k: x.astype(np.float64) for k, x in g.items()}, m, v, it, total,
                                  beta1=float(np.float32(0.9)), beta2=float(np.float32(0.999)),
                                  eps=float(np.float32(1e-15)))
        torch.cuda.synchronize()
        for k in ("sites", "density", "sh"):
            got = gp[k].cpu().numpy()
            np.testing.assert_allclose(got, ref[k], rtol=1e-5, atol=2e-6, err_msg=f"{k} at step {it}")
    # the moments too, at the end
    np.testing.assert_allclose(st.tensors["m_sh"].cpu().numpy(), m["sh"], rtol=1e-5, atol=1e-6)
    np.testing.assert_allclose(st.tensors["v_density"].cpu().numpy(), v["density"], rtol=1e-5, atol=1e-7)


def test_densify_scores_match_oracle(scene):
    import paper_2502_01157_amd as rf

    g = np.random.default_rng(84).standard_normal((scene.n_sites, 3)).astype(np.float32)
    got = rf.densify_scores(*map(_dv, (scene.sites, scene.off, scene.idx, g))).cpu().numpy()
    ref = otr.densify_scores(scene.sites, scene.off, scene.idx, g)
    np.testing.assert_allclose(got, ref, rtol=2e-6, atol=0)


@pytest.mark.parametrize("n", [1, 1000, 1024, 5000, 300001])
def test_sample_cells_match_oracle(n):
    import paper_2502_01157_amd as rf

    rng = np.random.default_rng(85 + n)
    scores = (rng.exponential(1.0, n) * (rng.uniform(0, 1, n) > 0.25)).astype(np.float32)
    scores[0] = max(scores[0], 0.5)
    draws = rng.uniform(0, 1, 200000).astype(np.float32)
    draws[:3] = [0.0, np.nextafter(np.float32(1.0), np.float32(0.0)), 0.5]
    got = rf.sample_cells(_dv(scores), _dv(draws)).cpu().numpy()
    ref = otr.sample_cells(scores, draws)
    c = np.cumsum(scores.astype(np.float64))
    target = draws.astype(np.float64) * c[-1]
    near = np.abs(c[np.minimum(ref, n - 1)] - target) < 1e-9 * c[-1]
    near |= np.abs(c[np.maximum(ref - 1, 0)] - target) < 1e-9 * c[-1]
    np.testing.assert_array_equal(got[~near], ref[~near])
    assert np.all(scores[got] > 0)
    # exact boundaries: a cell owns [C_{i-1}, C_i)
    exact = np.array([0.0, 0.0, 1.0, 1.0, 0.0, 2.0], dtype=np.float32)
    got = rf.sample_cells(_dv(exact), _dv(np.array([0.0, 0.25, 0.5, 0.75], dtype=np.float32))).cpu().numpy()
    np.testing.assert_array_equal(got, [2, 3, 5, 5])


def test_prune_mask_matches_oracle(scene):
    import paper_2502_01157_amd as rf

    dens = scene.density.astype(np.float32).copy()
    dens[np.random.default_rng(86).uniform(0, 1, len(dens)) < 0.6] = 0.0
    for q in (0.0, 0.3, 0.7):
        thr = np.float32(np.quantile(dens, q) + 1e-6)
        got = rf.prune_mask(*map(_dv, (dens, scene.off, scene.idx)), float(thr)).cpu().numpy()
        ref = otr.prune_mask(dens, scene.off, scene.idx, float(thr))
        np.testing.assert_array_equal(got, ref)
    assert got.any() and not got.all()


def test_fit_reduces_the_loss():
    """Fit densities and colours (softplus density, Adam with the schedule) to
    renders of a target scene with the same sites: 60 steps of raygen-free
    rays, logged forward, L2 loss gradient, backward, Adam."""
    import torch

    import paper_2502_01157_amd as rf

    sc = synth.small_scene("clustered", 5000, seed=87, sh_deg=3)
    rng = np.random.default_rng(88)
    from parity import inside_rays
    o, d, t, s = inside_rays(sc, rng, 8192, -0.9, 0.9)
    o, d, t, s = map(_dv, (o, d, t, s))
    sites, off, idx = map(_dv, (sc.sites, sc.off, sc.idx))
    target_scene = rf.PackedScene(sites, off, idx, _dv(sc.density), _dv(sc.sh), 3)
    target, _, _ = rf.render_forward(target_scene, o, d, t, s)
    # start: flat density x (sigma ~ 0.07) and zero colour
    x = torch.full((sc.n_sites,), 0.0, device="cuda")
    sh = torch.zeros((sc.n_sites, 16, 3), device="cuda")
    pos = sites.clone()
    state = rf.AdamState(sc.n_sites, 3, "cuda")
    packed = rf.PackedScene(pos, off, idx, x, sh, 3, density_activation="softplus")
    log = rf.WalkLog(len(t), 256, "cuda")
    losses = []
    total = 60
    for it in range(total):
        packed.pack(pos, x, sh)
        rgb, tf, _ = rf.render_forward(packed, o, d, t, s, log=log)
        diff = rgb - target
        losses.append(float((diff * diff).mean()))
        gs, gd, gsh = rf.render_backward(packed, o, d, t, s, rgb, tf, (2.0 / diff.numel()) * diff, log=log)
        rf.adam_step(rf.train_schedule(it, total), state, pos, x, sh, gs, gd, gsh)
    assert losses[-1] < 0.5 * losses[0], losses[::10]
    assert all(np.isfinite(losses))


# ---------------------------------------------------------------------------
# densification and pruning applied, and a run with a changing adjacency
# ---------------------------------------------------------------------------

def _unit_ball(rng, n):
    u = rng.standard_normal((n, 3))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    return (u * rng.uniform(0, 1, (n, 1)) ** (1 / 3)).astype(np.float32)


def test_insert_gather_keep_match_oracle(scene):
    import torch

    import paper_2502_01157_amd as rf

    rng = np.random.default_rng(90)
    n = scene.n_sites
    parents = rng.integers(0, n, 5001).astype(np.int32)
    parents[:2] = [-1, n]  # out of range: NaN coordinates
    u = _unit_ball(rng, len(parents))
    sites, off, idx = map(_dv, (scene.sites, scene.off, scene.idx))
    got = rf.insert_sites(sites, off, idx, _dv(parents), _dv(u), 0.5).cpu().numpy()
    assert np.isnan(got[:2]).all()
    ref = otr.insert_sites(scene.sites.astype(np.float64), scene.off, scene.idx, parents[2:], u[2:], frac=0.5)
    # formed in double and rounded once: within one FP32 rounding of the oracle's value
    np.testing.assert_allclose(got[2:], ref, rtol=2 ** -23, atol=0)
    # every new site lies in its parent's cell (nearest site by brute force)
    nn = synth.nearest_site(scene.sites, got[2:])
    np.testing.assert_array_equal(nn, parents[2:])
    # rows gathered bit for bit; indices out of range give NaN rows
    sh = _dv(scene.sh)
    rows = rng.integers(0, n, 777).astype(np.int32)
    np.testing.assert_array_equal(rf.gather_rows(sh, _dv(rows)).cpu().numpy(), scene.sh[rows])
    bad = rf.gather_rows(sites, _dv(np.array([3, -2, n], dtype=np.int32))).cpu().numpy()
    np.testing.assert_array_equal(bad[0], scene.sites[3])
    assert np.isnan(bad[1:]).all()
    # kept indices in order, for ragged sizes and edge cases
    for size, p in ((0, 0.5), (1, 1.0), (1023, 0.3), (1024, 0.0), (1025, 1.0), (100003, 0.7)):
        keep = rng.uniform(0, 1, size) < p
        got = rf.keep_index(_dv(keep)).cpu().numpy() if size else rf.keep_index(
            torch.zeros(0, dtype=torch.bool, device="cuda")).cpu().numpy()
        np.testing.assert_array_equal(got, np.nonzero(keep)[0])


def test_training_with_changing_adjacency():
    """A short run of the training loop on synthetic targets: renders of a
    3,000-site scene from 8,192 interior rays, fitted from 800 random sites
    with flat density and zero colour, densified at three steps (pruned,
    sites inserted by the score, graph rebuilt) up to 2,000 sites. The loss
    falls, the number of sites follows the growth schedule, the rebuilds
    follow the schedule, and every rebuilt graph is the Delaunay graph of the
    sites on the device at that moment (a fresh Qhull build)."""
    import torch

    import paper_2502_01157_amd as rf
    from paper_2502_01157_amd.training import TrainConfig, Trainer
    from parity import inside_rays

    tgt = synth.small_scene("clustered", 3000, seed=91, sh_deg=3)
    rng = np.random.default_rng(92)
    o, d, t, s = inside_rays(tgt, rng, 8192, -0.9, 0.9)
    od, dd, td, sd = map(_dv, (o, d, t, s))
    target_scene = rf.PackedScene(*map(_dv, (tgt.sites, tgt.off, tgt.idx, tgt.density, tgt.sh)), 3)
    target, _, _ = rf.render_forward(target_scene, od, dd, td, sd)

    checked = []

    class CheckedTrainer(Trainer):
        def rebuild(self):
            super().rebuild()
            cpu_sites = self.sites.cpu().numpy()
            off, idx = synth.build_adjacency(cpu_sites)
            np.testing.assert_array_equal(self.off.cpu().numpy(), off)
            np.testing.assert_array_equal(self.idx.cpu().numpy(), idx)
            checked.append(len(cpu_sites))

    init = rng.uniform(-0.95, 0.95, (800, 3)).astype(np.float32)
    cfg = TrainConfig(total=90, n_max=2000, densify_every=15, prune_threshold=1e-3, seed=93)
    tr = CheckedTrainer(_dv(init), torch.zeros(800, device="cuda"), torch.zeros((800, 16, 3), device="cuda"), 3,
                        cfg)
    hist = tr.run((od, dd, td), target)
    losses = [h.loss for h in hist]
    print(f"losses {losses[0]:.5f} -> {losses[-1]:.5f}; sites {[h.n_sites for h in hist if h.densified]}; "
          f"rebuilds {tr.rebuilds}; graphs checked {len(checked)}", flush=True)
    assert all(np.isfinite(losses))
    assert losses[-1] < 0.5 * losses[0]
    assert tr.densify_at == [15, 30, 45]
    sizes = {h.it: h.n_sites for h in hist}
    assert sizes[45] == 2000 and sizes[89] == 2000
    assert 800 < sizes[15] < sizes[30] < 2000
    assert tr.rebuilds == otr.rebuild_steps(90, [16, 31, 46])
    assert len(checked) >= len(tr.rebuilds)
    # positions are frozen for the last tenth of the run, so the start cells
    # located at the last rebuild are the nearest sites of the ray origins
    same = tr.starts.cpu().numpy() == synth.nearest_site(tr.sites.cpu().numpy(), o)
    assert tr.rebuilds[-1] >= 81 and same.mean() > 0.999
