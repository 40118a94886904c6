"""Ray-based effects on the GPU (Fig. 3) against the FP64 oracle: secondary
rays at a mirror or glass sphere, and the equidistant fisheye camera.

The oracle's legs are exact (the reflection and refraction laws in double).
The library keeps each leg after a crossing in double for its exit
distances, clipping and next crossing, and takes only its face decisions in
FP32 on the leg's rounding, as for any ray: so the plain walk's tolerances
apply, with the face decisions' margin (KAPPA_T, whose error scale includes
the rounding of the leg's origin and direction) and the surface decisions
(a crossing next to an exit, a grazing crossing, near-critical refraction)
clearing KAPPA_SURF.
"""

import numpy as np
import pytest

import oracle
import synth

from parity import (COLOUR_RTOL, KAPPA_G, KAPPA_T, KAPPA_TERM, KAPPA_X, check_gradients, colour_err, colour_ratio,
                    grad_err)

pytestmark = pytest.mark.gpu

# the library takes the sphere in FP32: both sides get the same FP32 values
CENTRE = tuple(float(np.float32(c)) for c in (0.05, -0.1, 0.0))
RADIUS = float(np.float32(0.35))
BOX = ("box", -1.0, 1.0)
KAPPA_SURF = 1e-6
EPS = 1e-4


def _dv(a):
    import torch

    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def aimed_rays(scene, rng, n, spread=0.3):
    """FP32 rays from points outside the sphere towards its neighbourhood."""
    c = np.array(CENTRE)
    o = []
    while len(o) < n:
        p = rng.uniform(-0.9, 0.9, 3)
        if np.linalg.norm(p - c) > RADIUS + 0.05:
            o.append(p)
    o = np.array(o, dtype=np.float32)
    d = c + spread * rng.standard_normal((n, 3)) - o
    d = (d / np.linalg.norm(d, axis=1, keepdims=True)).astype(np.float32)
    od, dd = o.astype(np.float64), d.astype(np.float64)
    with np.errstate(divide="ignore"):
        t = np.minimum(np.where(dd > 0, (1.0 - od) / dd, np.inf), np.where(dd < 0, (-1.0 - od) / dd, np.inf))
    return o, d, t.min(1).astype(np.float32), synth.nearest_site(scene.sites, o).astype(np.int32)


@pytest.fixture(scope="module")
def setup():
    scene = synth.small_scene("clustered", 20000, seed=71, sh_deg=3)
    rays = aimed_rays(scene, np.random.default_rng(72), 2048)
    return scene, rays


def _surfaces(rf, kind, ior=1.5, max_bounces=8):
    ior = float(np.float32(ior))
    return (rf.Surface(kind, CENTRE, RADIUS, BOX, ior=ior, max_bounces=max_bounces),
            oracle.Surface(kind, CENTRE, RADIUS, BOX, ior=ior, max_bounces=max_bounces))


def _packed(rf, scene, dtype="f32", density=None):
    dens = scene.density if density is None else density
    return rf.PackedScene(*map(_dv, (scene.sites, scene.off, scene.idx, dens, scene.sh)), scene.sh_deg, dtype)


def _decidable_bent(tr):
    return ((tr["margin"] > KAPPA_T) & (tr["graze"] > KAPPA_G) & (tr["term"] > KAPPA_TERM)
            & (tr["surf_margin"] > KAPPA_SURF))


def _read_log(log, R):
    code = log.code.cpu().numpy().view(np.uint32)
    tail = log.tail.cpu().numpy()
    return code, tail


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
@pytest.mark.parametrize("kind", ["mirror", "glass"])
def test_bent_forward_matches_oracle(setup, kind, dtype):
    import torch

    import paper_2502_01157_amd as rf

    scene, rays = setup
    R = len(rays[2])
    sf, osf = _surfaces(rf, kind)
    dens, sh = scene.density, scene.sh
    if dtype == "bf16":
        dens = oracle.bf16_to_f32(oracle.bf16_round(dens))
        sh = oracle.bf16_to_f32(oracle.bf16_round(sh))
    osc = oracle.OracleScene.from_scene(scene, density=dens, sh=sh, surface=osf)
    tr = oracle.trace(osc, *rays, eps=EPS, max_len=1024)
    ok = _decidable_bent(tr)
    bent = np.array([tr["bounce"][r, :tr["len"][r]].any() for r in range(R)])
    assert (ok & bent).sum() > 0.3 * R, ((ok & bent).sum(), R)

    p = _packed(rf, scene, dtype)
    o, d, t, s = map(_dv, rays)
    log = rf.WalkLog(R, 256, o.device)
    rgb, tf, steps = rf.render_forward(p, o, d, t, s, eps=EPS, log=log, surface=sf)
    rgb2, tf2, steps2 = rf.render_forward(p, o, d, t, s, eps=EPS, surface=sf)
    torch.cuda.synchronize()
    # the logged and the plain forward give the same outputs bit for bit
    assert torch.equal(rgb, rgb2) and torch.equal(tf, tf2) and torch.equal(steps, steps2)
    rgb, tf, steps = rgb.cpu().numpy(), tf.cpu().numpy(), steps.cpu().numpy()
    assert colour_ratio(rgb[ok], tr["rgb"][ok], np.abs(tr["rgb"]).mean()).max() <= 1.0
    assert np.abs(tf[ok] - tr["t_final"][ok]).max() <= 1e-4
    np.testing.assert_array_equal(steps[ok], tr["steps"][ok])
    # visited cells and crossings, from the walk log
    code, tail = _read_log(log, R)
    bad = 0
    for r in np.nonzero(ok)[0]:
        L = tr["len"][r]
        assert tail[r, 2] == L
        assert tail[r, 3] == tr["bounce"][r, :L].sum()
        Lc = min(L, 256)
        cells = (code[:Lc, r] & 0x1FFFFFFF).astype(np.int64)
        cross = (code[:Lc, r] >> 29) & 1
        if not (np.array_equal(cells, tr["cells"][r, :Lc]) and np.array_equal(cross, tr["bounce"][r, :Lc])):
            bad += 1
    assert bad == 0


def test_zero_bounces_is_the_plain_walk(setup):
    import torch

    import paper_2502_01157_amd as rf

    scene, rays = setup
    p = _packed(rf, scene)
    o, d, t, s = map(_dv, rays)
    plain = rf.render_forward(p, o, d, t, s, eps=EPS)
    for kind in ("mirror", "glass"):
        sf, _ = _surfaces(rf, kind, max_bounces=0)
        bent = rf.render_forward(p, o, d, t, s, eps=EPS, surface=sf)
        for a, b in zip(plain, bent):
            assert torch.equal(a, b)


def test_index_one_glass_renders_as_no_surface(setup):
    import paper_2502_01157_amd as rf

    scene, rays = setup
    p = _packed(rf, scene)
    o, d, t, s = map(_dv, rays)
    sf, _ = _surfaces(rf, "glass", ior=1.0)
    plain = [x.cpu().numpy() for x in rf.render_forward(p, o, d, t, s, eps=EPS)]
    glass = [x.cpu().numpy() for x in rf.render_forward(p, o, d, t, s, eps=EPS, surface=sf)]
    # splitting a segment at the crossing only reorders FP32 rounding
    assert colour_err(glass[0], plain[0]) <= COLOUR_RTOL
    assert np.abs(glass[1] - plain[1]).max() <= 1e-4


@pytest.mark.parametrize("cap", [256, 16, None])
@pytest.mark.parametrize("kind", ["mirror", "glass"])
def test_bent_backward_matches_oracle(setup, kind, cap):
    import torch

    import paper_2502_01157_amd as rf

    scene, rays = setup
    sf, osf = _surfaces(rf, kind, ior=1.45)
    osc = oracle.OracleScene.from_scene(scene, surface=osf)
    tr = oracle.trace(osc, *rays, eps=EPS, max_len=1024)
    keep = _decidable_bent(tr) & (tr["exit_cos"] > KAPPA_X)
    rays_k = tuple(a[keep] for a in rays)
    n = len(rays_k[2])
    rng = np.random.default_rng(73)
    g = rng.standard_normal((n, 3)).astype(np.float32)
    gT = rng.standard_normal(n).astype(np.float32)
    ref = oracle.backward(osc, *rays_k, g, gT, eps=EPS)
    p = _packed(rf, scene)
    o, d, t, s = map(_dv, rays_k)
    log = rf.WalkLog(n, cap, o.device) if cap is not None else None
    rgb, tf, _ = rf.render_forward(p, o, d, t, s, eps=EPS, log=log, surface=sf)
    got = rf.render_backward(p, o, d, t, s, rgb, tf, _dv(g), _dv(gT), eps=EPS, log=log, surface=sf)
    torch.cuda.synchronize()
    check_gradients(got, ref)


def test_bent_autograd_and_errors(setup):
    import torch

    import paper_2502_01157_amd as rf

    scene, rays = setup
    rays = tuple(a[:256] for a in rays)
    R = 256
    sf, _ = _surfaces(rf, "glass")
    sites, off, idx, dens, sh = map(_dv, (scene.sites, scene.off, scene.idx, scene.density, scene.sh))
    for x in (sites, dens, sh):
        x.requires_grad_(True)
    o, d, t, s = map(_dv, rays)
    rgb, tf, steps = rf.render(sites, dens, sh, off, idx, o, d, t, s, 3, surface=sf)
    g = torch.randn_like(rgb)
    (rgb * g).sum().backward()
    p = _packed(rf, scene)
    log = rf.WalkLog(R, 256, o.device)
    rgb2, tf2, _ = rf.render_forward(p, o, d, t, s, log=log, surface=sf)
    assert torch.equal(rgb.detach(), rgb2)
    ref = rf.render_backward(p, o, d, t, s, rgb2, tf2, g, log=log, surface=sf)
    for x, y in zip((sites.grad, dens.grad, sh.grad), ref):
        assert grad_err(x.cpu().numpy(), y.cpu().numpy()) < 1e-5
    # the quantile regulariser leaves bent rays out
    q, loss = rf.quantile_forward(p, o, d, t, s, tf2, log, torch.rand((R, 2), device=o.device))
    bent = log.tail[:, 3].cpu().numpy() > 0
    assert bent.any()
    assert np.all(loss.cpu().numpy()[bent] == 0) and np.all(q.segment.cpu().numpy()[bent] == -1)
    with pytest.raises(ValueError):
        rf.render(sites, dens, sh, off, idx, o, d, t, s, 3, quantile_draws=torch.rand((R, 2), device=o.device),
                  surface=sf)
    with pytest.raises(ValueError):
        rf.render_backward(p, o, d, t, s, rgb2, tf2, g, mode=1, surface=sf)
    # invalid surfaces are rejected by the library
    for bad in (dict(radius=0.0), dict(ior=0.0), dict(max_bounces=-1), dict(max_bounces=5000)):
        args = dict(kind="glass", centre=CENTRE, radius=RADIUS, bound=BOX, ior=1.5, max_bounces=4)
        args.update(bad)
        with pytest.raises(rf.RfError):
            rf.render_forward(p, o, d, t, s, surface=rf.Surface(**args))
    with pytest.raises(ValueError):
        rf.Surface("lens", CENTRE, RADIUS, BOX)


# ---------------------------------------------------------------------------
# fisheye camera
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("W,H,fov", [(64, 48, 180.0), (33, 17, 360.0), (20, 20, 90.0)])
def test_fisheye_raygen_matches_oracle(W, H, fov):
    import paper_2502_01157_amd as rf

    cam = synth.make_cameras("clustered_200k", np.random.default_rng(W), n=1, res=(W, H))[0]
    pose = np.float32(cam.pose12()).astype(np.float64)
    o, d, t, px = oracle.raygen(pose, fov, W, H, BOX, model="fisheye")
    go, gd, gt, gs, gpx = rf.raygen(pose, fov, W, H, BOX, 5, model="fisheye")
    np.testing.assert_array_equal(gpx.cpu().numpy(), px)
    np.testing.assert_array_equal(go.cpu().numpy(), o.astype(np.float32))
    assert np.abs(gd.cpu().numpy() - d).max() < 2e-6
    tt = gt.cpu().numpy()
    np.testing.assert_allclose(tt, t, rtol=2e-5, atol=2e-6)
    assert np.all(gs.cpu().numpy() == 5)
    with pytest.raises(rf.RfError):
        rf.raygen(pose, 400.0, W, H, BOX, 0, model="fisheye")
