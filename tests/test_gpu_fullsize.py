"""Parity at the workloads' full sizes, in the launch configuration the benchmark times.

The GPU walks every ray of the full frame (one launch over all rays, 8x8 tile
order, the same kernels as the benchmark). The oracle computes the same
frame's colours, transmittances and decision margins for every ray, the
visited cells of every ray (near-tie rays against the oracle's alternative
walks), and the full-frame gradients with upstream gradients N(0,1) on the
rays whose gradients are compared (zero on the others, identically on both
sides).
"""

import time

import numpy as np
import pytest

import oracle
import synth

from parity import (T_ATOL, camera_rays, check_gradients, colour_ratio, decidable, flip_table, gradient_decidable,
                    resolve_near_ties)

# surface decisions (a crossing inside a cell or past its exit, a grazing
# crossing, near-critical refraction) closer than this are not compared: both
# sides form the legs in double, so only the exit distances' FP32 plane error
# (~eps32 / cos) can move such a decision
KAPPA_SURF = 1e-6

pytestmark = pytest.mark.gpu


def _dv(a):
    import torch

    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def frame_check(rf, p, osc, rays, sel, rgb, tf, steps, eps=1e-4, chunk=131072, max_len=512, gpu_cells=None,
                label=""):
    """Parity of the rays ``sel`` of a batch already rendered on the GPU (rgb,
    tf, steps of the whole batch): the oracle's colour, transmittance and
    margins for every ray of ``sel``; the visited cells of every ray, in
    chunks (from the GPU's trace kernel, or ``gpu_cells(idx)`` for bent walks);
    near-tie rays matched with the oracle's alternative walks. Prints the
    decidable share, the unresolved share and the flip-versus-margin table."""
    o, d, t, s = rays
    t0 = time.time()
    ref = oracle.trace(osc, o[sel], d[sel], t[sel], s[sel], eps=eps, max_len=1)
    dec = decidable(ref, eps)
    print(f"{label}: oracle on {len(sel)} rays in {time.time() - t0:.1f}s; decidable {dec.mean():.5f}", flush=True)
    rgb, tf, steps = rgb[sel], tf[sel], steps[sel]
    mean_abs = float(np.abs(ref["rgb"]).mean())
    cr = colour_ratio(rgb[dec], ref["rgb"][dec], mean_abs)
    print(f"{label}: decidable rays: colour error / tolerance max {cr.max(initial=0):.3f}", flush=True)
    assert cr.max(initial=0) <= 1.0
    assert np.abs(tf[dec] - ref["t_final"][dec]).max(initial=0) <= T_ATOL
    np.testing.assert_array_equal(steps[dec], ref["steps"][dec])

    # visited cells of every ray, chunk by chunk
    t1 = time.time()
    und_idx, und_cells, und_len = [], [], []
    seq_bad = 0
    for a in range(0, len(sel), chunk):
        q = np.arange(a, min(a + chunk, len(sel)))
        rq = sel[q]
        if gpu_cells is None:
            tr = rf.render_trace(p, *map(_dv, (o[rq], d[rq], t[rq], s[rq])), eps=eps, max_len=max_len)
            gc = tr["cells"].cpu().numpy()
            gs = tr["steps"].cpu().numpy()
            glen = np.where(gs >= 0, gs, 0)
        else:
            gc, glen = gpu_cells(rq)
        oc = oracle.trace(osc, o[rq], d[rq], t[rq], s[rq], eps=eps, max_len=max_len)
        dq = dec[q]
        same = (oc["len"] == glen) & np.all(oc["cells"] == gc[:, :max_len], axis=1)
        within = oc["len"] <= max_len
        seq_bad += int((dq & within & ~same).sum())
        und_idx.append(q[~dq])
        und_cells.append(gc[~dq])
        und_len.append(glen[~dq])
    print(f"{label}: cell sequences of all {len(sel)} rays compared in {time.time() - t1:.1f}s, "
          f"{seq_bad} decidable rays differ", flush=True)
    assert seq_bad == 0

    # near-tie rays: the GPU's walk among the oracle's alternatives
    und = np.concatenate(und_idx)
    cells = np.concatenate(und_cells) if len(und) else np.zeros((0, max_len), np.int32)
    lens = np.concatenate(und_len) if len(und) else np.zeros(0, np.int64)
    t2 = time.time()
    res = resolve_near_ties(osc, (o, d, t, s), sel[und], cells, lens, eps, max_len=max_len)
    matched = np.array([m is not None for m in res["match"]], dtype=bool)
    bad = (~matched) & res["complete"]
    unresolved = int((~matched).sum())
    print(f"{label}: {len(und)} near-tie rays ({len(und) / len(sel):.4%}) resolved in {time.time() - t2:.1f}s: "
          f"{int(matched.sum())} matched ({int((res['flips'] > 0).sum())} took an alternative), "
          f"{unresolved} unresolved ({unresolved / len(sel):.5%}), {int(bad.sum())} unmatched with complete "
          f"alternatives", flush=True)
    flipped = res["flips"] > 0
    print(f"{label}: flips against the oracle's margin (lo, hi, near-tie rays, rays whose GPU walk took an "
          f"alternative): {flip_table(ref['margin'][und], flipped)}", flush=True)
    assert not bad.any()
    assert unresolved <= 1e-3 * len(sel)
    worst = 0.0
    for k, r in enumerate(und):
        m = res["match"][k]
        if m is None:
            continue
        worst = max(worst, float(colour_ratio(rgb[r], m["rgb"], mean_abs)[0]))
        assert abs(tf[r] - m["t_final"]) <= T_ATOL
        assert steps[r] == m["steps"]
    print(f"{label}: near-tie rays: colour error / tolerance max {worst:.3f}", flush=True)
    assert worst <= 1.0
    return ref, dec


@pytest.mark.parametrize("name,dtype", [("clustered_200k", "f32"), ("clustered_1m", "f32"), ("clustered_1m", "bf16")])
def test_full_frame_forward_backward(name, dtype):
    import torch

    import paper_2502_01157_amd as rf

    t0 = time.time()
    scene, rng = synth.make_scene(name, return_rng=True)
    cam = synth.make_cameras(name, rng)[0]
    R = cam.width * cam.height
    g = synth.make_upstream_grads(rng, R)
    o, d, t, s, _ = camera_rays(scene, cam)
    print(f"\n{name}/{dtype}: scene {scene.n_sites} sites built in {time.time() - t0:.1f}s", flush=True)

    dens, sh = scene.density, scene.sh
    if dtype == "bf16":
        dens = oracle.bf16_to_f32(oracle.bf16_round(dens))
        sh = oracle.bf16_to_f32(oracle.bf16_round(sh))
    osc = oracle.OracleScene.from_scene(scene, density=dens, sh=sh)

    p = rf.PackedScene(*map(_dv, (scene.sites, scene.off, scene.idx, scene.density, scene.sh)), scene.sh_deg,
                       dtype, validate=True)
    od, dd, td, sd = map(_dv, (o, d, t, s))
    rgb_d, tf_d, steps_d = rf.render_forward(p, od, dd, td, sd)
    torch.cuda.synchronize()
    rgb, tf, steps = rgb_d.cpu().numpy(), tf_d.cpu().numpy(), steps_d.cpu().numpy()
    full, dec = frame_check(rf, p, osc, (o, d, t, s), np.arange(R), rgb, tf, steps, label=f"{name}/{dtype}")
    if dtype == "bf16":
        # the total error of BF16 storage: against the oracle on the original FP32 attributes
        ref32 = oracle.forward(oracle.OracleScene.from_scene(scene), o, d, t, s, eps=1e-4)[0]
        err = np.abs(rgb - ref32)
        scale = np.abs(ref32).max()
        print(f"bf16 total colour error against the FP32-attribute oracle: max {err.max() / scale:.3e}, "
              f"p99 {np.quantile(err, 0.99) / scale:.3e}, mean {err.mean() / scale:.3e} of the largest colour",
              flush=True)

    # full-frame gradients (upstream gradients on the rays whose gradients are compared)
    keep = gradient_decidable(full, 1e-4)
    print(f"gradients compared on {keep.mean():.4%} of the rays", flush=True)
    gm = np.where(keep[:, None], g, 0.0).astype(np.float32)
    t2 = time.time()
    ref_g = oracle.backward(osc, o, d, t, s, gm, eps=1e-4)
    print(f"oracle backward in {time.time() - t2:.1f}s", flush=True)
    mism = torch.zeros(1, dtype=torch.int32, device=od.device)
    grads = rf.render_backward(p, od, dd, td, sd, rgb_d, tf_d, _dv(gm), steps=steps_d, mismatches=mism)
    torch.cuda.synchronize()
    # every recomputed walk ends with the forward's transmittance (bit for bit) and visit count
    assert int(mism.item()) == 0
    print(f"gradient error ratios, recomputing backward (inf-norm, per element): "
          f"{check_gradients(grads, ref_g)}", flush=True)
    # the training step with a walk log
    cap = 512  # reflected paths run longer than refracted ones
    log = rf.WalkLog(R, cap, od.device)
    rgb_l, tf_l, _ = rf.render_forward(p, od, dd, td, sd, log=log)
    assert torch.equal(rgb_l, rgb_d) and torch.equal(tf_l, tf_d)
    grads = rf.render_backward(p, od, dd, td, sd, rgb_l, tf_l, _dv(gm), log=log)
    torch.cuda.synchronize()
    print(f"gradient error ratios, logged backward: {check_gradients(grads, ref_g)}", flush=True)


def test_shell_3m_eight_cameras_sampled():
    """The 3M-site shell scene (BF16 attributes), all eight cameras' rays in one launch.

    The oracle checks a sample of 8x8 tiles per camera: colour, transmittance,
    steps and visited cells of every sampled ray (near ties against the
    oracle's alternatives), and the gradients of a backward launch over every
    ray whose upstream gradient is non-zero only on the sampled rays whose
    gradients are compared (so the accumulated sums are exactly those of the
    sample).
    """
    import torch

    import paper_2502_01157_amd as rf

    t0 = time.time()
    scene, rng = synth.make_scene("shell_3m", return_rng=True)
    cams = synth.make_cameras("shell_3m", rng)
    print(f"\nshell_3m: scene {scene.n_sites} sites built in {time.time() - t0:.1f}s", flush=True)
    per_cam = [camera_rays(scene, c) for c in cams]
    o, d, t, s = (np.concatenate([r[k] for r in per_cam]) for k in range(4))
    R = len(t)
    assert R == sum(c.width * c.height for c in cams)

    dens = oracle.bf16_to_f32(oracle.bf16_round(scene.density))
    sh = oracle.bf16_to_f32(oracle.bf16_round(scene.sh))
    osc = oracle.OracleScene.from_scene(scene, density=dens, sh=sh)

    # 256 wave-sized blocks of 64 consecutive rays (one 8x8 tile where the tile is
    # whole) per camera; a camera's last block may be short
    srng = np.random.default_rng(4)
    sel = []
    base = 0
    for c in cams:
        n = c.width * c.height
        for tile in np.sort(srng.choice((n + 63) // 64, size=256, replace=False)):
            sel.append(base + tile * 64 + np.arange(64)[: max(0, min(64, n - tile * 64))])
        base += n
    sel = np.concatenate(sel)

    p = rf.PackedScene(*map(_dv, (scene.sites, scene.off, scene.idx, scene.density, scene.sh)), scene.sh_deg,
                       "bf16", validate=True)
    od, dd, td, sd = map(_dv, (o, d, t, s))
    rgb_d, tf_d, steps_d = rf.render_forward(p, od, dd, td, sd)
    torch.cuda.synchronize()
    assert (steps_d.cpu().numpy() >= 0).all()
    ref, dec = frame_check(rf, p, osc, (o, d, t, s), sel, rgb_d.cpu().numpy(), tf_d.cpu().numpy(),
                           steps_d.cpu().numpy(), max_len=1024, label="shell_3m/bf16 sample")

    g = np.zeros((R, 3), dtype=np.float32)
    g_sel = synth.make_upstream_grads(rng, len(sel))
    gdec = gradient_decidable(ref, 1e-4)
    g[sel[gdec]] = g_sel[gdec]
    t2 = time.time()
    ref_g = oracle.backward(osc, o[sel], d[sel], t[sel], s[sel], g[sel], eps=1e-4)
    print(f"oracle backward on the sample in {time.time() - t2:.1f}s", flush=True)
    grads = rf.render_backward(p, od, dd, td, sd, rgb_d, tf_d, _dv(g))
    torch.cuda.synchronize()
    print(f"gradient error ratios (inf-norm, per element): {check_gradients(grads, ref_g)}", flush=True)


@pytest.mark.parametrize("kind", ["glass", "mirror"])
def test_bent_full_frame_sphere(kind):
    """The clustered_1m frame with the benchmark's sphere (radius 0.3 at the
    centre; glass of index 1.5, or a mirror), against the oracle's exact legs:
    every ray's colour, transmittance, visited cells and crossings (from the
    walk log), and the full-frame gradients of the logged backward."""
    import torch

    import paper_2502_01157_amd as rf

    scene, rng = synth.make_scene("clustered_1m", return_rng=True)
    cam = synth.make_cameras("clustered_1m", rng)[0]
    R = cam.width * cam.height
    g = synth.make_upstream_grads(rng, R)
    o, d, t, s, _ = camera_rays(scene, cam)
    bound = synth.CONFIGS["clustered_1m"]["bound"]
    # the sphere in FP32, as the library takes it; exact legs
    radius = float(np.float32(0.3))
    osf = oracle.Surface(kind, (0.0, 0.0, 0.0), radius, bound, ior=1.5, max_bounces=8)
    osc = oracle.OracleScene.from_scene(scene, surface=osf)
    p = rf.PackedScene(*map(_dv, (scene.sites, scene.off, scene.idx, scene.density, scene.sh)), 3, "f32")
    od, dd, td, sd = map(_dv, (o, d, t, s))
    sf = rf.Surface(kind, (0.0, 0.0, 0.0), radius, bound, ior=1.5, max_bounces=8)
    cap = 512  # reflected paths run longer than refracted ones
    log = rf.WalkLog(R, cap, od.device)
    rgb, tf, steps = rf.render_forward(p, od, dd, td, sd, log=log, surface=sf)
    torch.cuda.synchronize()
    tail = log.tail.cpu().numpy()
    code = log.code.cpu().numpy().view(np.uint32)
    bent = tail[:, 3] > 0
    assert bent.mean() > 0.5

    def gpu_cells(rq):
        c = (code[:, rq].T & 0x1FFFFFFF).astype(np.int32)
        n = tail[rq, 2]
        c = np.where(np.arange(cap)[None, :] < n[:, None], c, -1)
        return c, n

    t1 = time.time()
    full = oracle.trace(osc, o, d, t, s, eps=1e-4, max_len=1)
    surf_ok = full["surf_margin"] > KAPPA_SURF
    print(f"\n{kind}: oracle frame in {time.time() - t1:.1f}s; surface decisions clear for {surf_ok.mean():.5f}",
          flush=True)
    # rays whose surface decisions are near ties are not resolved by the alternatives
    sel = np.nonzero(surf_ok & (tail[:, 2] <= cap))[0]
    assert len(sel) >= 0.995 * R
    ref, dec = frame_check(rf, p, osc, (o, d, t, s), sel, rgb.cpu().numpy(), tf.cpu().numpy(),
                           steps.cpu().numpy(), max_len=cap, gpu_cells=gpu_cells, label=kind)
    keep = np.zeros(R, dtype=bool)
    keep[sel] = gradient_decidable(ref, 1e-4)
    gm = np.where(keep[:, None], g, 0.0).astype(np.float32)
    t2 = time.time()
    ref_g = oracle.backward(osc, o, d, t, s, gm, eps=1e-4)
    print(f"oracle {kind} backward in {time.time() - t2:.1f}s; gradients on {keep.mean():.4%} of the rays", flush=True)
    grads = rf.render_backward(p, od, dd, td, sd, rgb, tf, _dv(gm), log=log, surface=sf)
    torch.cuda.synchronize()
    print(f"bent gradient error ratios: {check_gradients(grads, ref_g)}", flush=True)


def test_full_frame_quantiles():
    """The quantile regulariser on the whole clustered_1m frame (the training
    step's walk log): every decidable ray's two quantiles and loss against the
    oracle. The quantile's depth L_j is reached inside segment k, so the depth
    before it, tau_<k, is at most L_j and the per-ray bound of the quantile
    tests, 5e-5 (1 + L_j + tau_<k) / sigma_k, is at most 5e-5 (1 + 2 L_j) / sigma_k."""
    import torch

    import paper_2502_01157_amd as rf

    scene, rng = synth.make_scene("clustered_1m", return_rng=True)
    cam = synth.make_cameras("clustered_1m", rng)[0]
    o, d, t, s, _ = camera_rays(scene, cam)
    R = len(t)
    u = np.random.default_rng(66).uniform(size=(R, 2)).astype(np.float32)
    osc = oracle.OracleScene.from_scene(scene)
    t1 = time.time()
    tq_ref, loss_ref = oracle.quantile(osc, o, d, t, s, u.astype(np.float64), eps=1e-4)
    full = oracle.trace(osc, o, d, t, s, eps=1e-4, max_len=1)
    dec = decidable(full, 1e-4)
    print(f"\noracle quantiles of {R} rays in {time.time() - t1:.1f}s", flush=True)
    p = rf.PackedScene(*map(_dv, (scene.sites, scene.off, scene.idx, scene.density, scene.sh)), 3, "f32")
    od, dd, td, sd = map(_dv, (o, d, t, s))
    cap = 512  # reflected paths run longer than refracted ones
    log = rf.WalkLog(R, cap, od.device)
    rgb, tf, _ = rf.render_forward(p, od, dd, td, sd, log=log)
    q, loss = rf.quantile_forward(p, od, dd, td, sd, tf, log, _dv(u))
    torch.cuda.synchronize()
    # a plain walk's log tail counts no surface crossings
    assert bool((log.tail[:, 3] == 0).all())
    tq, seg, sig, loss = (x.cpu().numpy() for x in (q.t, q.segment, q.sigma, loss))
    A = 1.0 - full["t_final"]
    has = dec & (A > 0)
    L = -np.log1p(-u.astype(np.float64) * A[:, None])
    ok = has[:, None] & (seg >= 0)
    tol = 5e-5 * (1.0 + 2.0 * L) / np.where(ok, sig, 1.0) + 1e-6 * np.abs(tq_ref)
    err = np.where(ok, np.abs(tq - tq_ref), 0.0)
    print(f"quantiles compared on {ok.mean():.4%} of the draws; error / bound max {(err / tol).max():.3f}",
          flush=True)
    assert ok.sum() > 0.95 * 2 * has.sum()
    assert np.all(err <= tol)
    lerr = np.abs(loss - loss_ref)[has]
    ltol = (tol[:, 0] + tol[:, 1])[has]
    assert np.all(lerr <= ltol)


def test_training_kernels_full_size():
    """The optimizer step, densification scores, candidate sampling and the
    pruning mask on the 1M-site scene's full arrays, as the benchmark runs
    them, against the oracle on every value."""
    import torch

    import paper_2502_01157_amd as rf
    from oracle import training as otr

    scene = synth.make_scene("clustered_1m")
    n = scene.n_sites
    rng = np.random.default_rng(91)
    x = {"sites": scene.sites.astype(np.float32), "density": rng.normal(0, 1, n).astype(np.float32),
         "sh": scene.sh.astype(np.float32)}
    gr = {"sites": rng.standard_normal((n, 3)).astype(np.float32),
          "density": rng.standard_normal(n).astype(np.float32),
          "sh": rng.standard_normal((n, 16, 3)).astype(np.float32)}
    gp = {k: _dv(v) for k, v in x.items()}
    st = rf.AdamState(n, 3, gp["sites"].device)
    it, total = 10000, 20000
    rf.adam_step(rf.train_schedule(it, total), st, gp["sites"], gp["density"], gp["sh"], _dv(gr["sites"]),
                 _dv(gr["density"]), _dv(gr["sh"]))
    zeros = {k: np.zeros(v.shape) for k, v in x.items()}
    ref, _, _ = otr.adam_step({k: v.astype(np.float64) for k, v in x.items()},
                              {k: v.astype(np.float64) for k, v in gr.items()}, zeros, dict(zeros), it, total,
                              beta1=float(np.float32(0.9)), beta2=float(np.float32(0.999)),
                              eps=float(np.float32(1e-15)))
    torch.cuda.synchronize()
    for k in ("sites", "density", "sh"):
        np.testing.assert_allclose(gp[k].cpu().numpy(), ref[k], rtol=1e-5, atol=2e-6, err_msg=k)
    g = rng.standard_normal((n, 3)).astype(np.float32)
    sites, off, idx = map(_dv, (scene.sites, scene.off, scene.idx))
    score = rf.densify_scores(sites, off, idx, _dv(g))
    ref_score = otr.densify_scores(scene.sites, scene.off, scene.idx, g)
    np.testing.assert_allclose(score.cpu().numpy(), ref_score, rtol=2e-6, atol=0)
    draws = rng.uniform(0, 1, n // 10).astype(np.float32)
    got = rf.sample_cells(score, _dv(draws)).cpu().numpy()
    sc = score.cpu().numpy()
    ref_s = otr.sample_cells(sc, draws)
    c = np.cumsum(sc.astype(np.float64))
    target = draws.astype(np.float64) * c[-1]
    near = (np.abs(c[ref_s] - target) < 1e-9 * c[-1]) | (np.abs(c[np.maximum(ref_s - 1, 0)] - target) < 1e-9 * c[-1])
    np.testing.assert_array_equal(got[~near], ref_s[~near])
    # most cells emptied, so that a good share is pruned (a cell and all its neighbours empty)
    dens = scene.density.astype(np.float32).copy()
    dens[rng.uniform(0, 1, n) < 0.9] = 0.0
    thr = 1e-3
    mask = rf.prune_mask(_dv(dens), off, idx, thr).cpu().numpy()
    np.testing.assert_array_equal(mask, otr.prune_mask(dens, scene.off, scene.idx, thr))
    assert 0.05 < mask.mean() < 0.5
