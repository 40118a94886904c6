"""Pins of the oracle's ray-based effects (Fig. 3): secondary rays at an
analytic mirror or glass sphere, and a non-linear (equidistant fisheye)
camera.

Each test checks the oracle against something other than its own code: the
laws of reflection and refraction written as vector identities, brute-force
nearest sites (eq. (5)) along every leg, the index-one glass that must leave
every render unchanged, the reversibility of light paths, the closed form of
a homogeneous medium over the whole bent path, central finite differences,
and the fisheye's defining angle-proportional-to-radius property.
"""

import numpy as np
import pytest

import oracle
import synth

from test_oracle_pins import brute_nn, hand_scene, unit

BOX = ("box", -1.0, 1.0)
CENTRE = np.array([0.08, -0.05, 0.02])
RADIUS = 0.42


def surface(kind, ior=1.5, max_bounces=8):
    return oracle.Surface(kind, CENTRE, RADIUS, BOX, ior=ior, max_bounces=max_bounces)


def box_exit(o, d, lo=-1.0, hi=1.0):
    t = np.full(len(d), np.inf)
    for a in range(3):
        with np.errstate(divide="ignore", invalid="ignore"):
            ta = np.where(d[:, a] > 0, (hi - o[:, a]) / d[:, a], np.where(d[:, a] < 0, (lo - o[:, a]) / d[:, a],
                                                                          np.inf))
        t = np.minimum(t, ta)
    return t


def aimed_rays(rng, n, sites, spread=0.35):
    """Origins in the box outside the sphere, aimed near the sphere's centre,
    so that most rays cross it."""
    o = []
    while len(o) < n:
        p = rng.uniform(-0.95, 0.95, 3)
        if np.linalg.norm(p - CENTRE) > RADIUS + 0.05:
            o.append(p)
    o = np.array(o)
    target = CENTRE + spread * rng.standard_normal((n, 3))
    d = unit(target - o)
    return o, d, box_exit(o, d), brute_nn(sites, o)[0].astype(np.int32)


@pytest.fixture(scope="module")
def scene():
    return synth.small_scene("uniform11", 300, seed=31, sh_deg=3)


def _legs(tr, r):
    """Per visit of ray r: cell, exit t, bounce flag, leg origin, leg direction."""
    L = tr["len"][r]
    return (tr["cells"][r, :L], tr["t_exit"][r, :L], tr["bounce"][r, :L].astype(bool), tr["legs"][r, :L, :3],
            tr["legs"][r, :L, 3:])


# ---------------------------------------------------------------------------
# secondary rays
# ---------------------------------------------------------------------------

def test_zero_bounces_and_no_surface_are_identical(scene):
    rng = np.random.default_rng(1)
    o, d, tmax, start = aimed_rays(rng, 80, scene.sites)
    base = oracle.forward(oracle.OracleScene.from_scene(scene), o, d, tmax, start)
    for kind in ("mirror", "glass"):
        off = oracle.forward(oracle.OracleScene.from_scene(scene, surface=surface(kind, max_bounces=0)), o, d, tmax,
                             start)
        for a, b in zip(base, off):
            np.testing.assert_array_equal(a, b)


def test_index_one_glass_changes_nothing(scene):
    """Glass with the index of its surroundings does not bend rays: the render
    equals the one without a surface (the crossing only splits a segment in
    two, and e^-a e^-b = e^-(a+b) within one cell)."""
    rng = np.random.default_rng(2)
    o, d, tmax, start = aimed_rays(rng, 150, scene.sites)
    base = oracle.OracleScene.from_scene(scene)
    glass = oracle.OracleScene.from_scene(scene, surface=surface("glass", ior=1.0))
    for eps in (0.0, 1e-2):
        a = oracle.forward(base, o, d, tmax, start, eps=eps)
        b = oracle.forward(glass, o, d, tmax, start, eps=eps)
        np.testing.assert_allclose(b[0], a[0], rtol=1e-11, atol=1e-12)
        np.testing.assert_allclose(b[1], a[1], rtol=1e-11, atol=1e-13)
    tr = oracle.trace(glass, o, d, tmax, start, eps=0.0, legs=True)
    ref = oracle.trace(base, o, d, tmax, start, eps=0.0)
    crossed = 0
    for r in range(len(d)):
        cells, te, bounce, lo_, ld_ = _legs(tr, r)
        crossed += bounce.any()
        np.testing.assert_allclose(ld_, np.broadcast_to(d[r], ld_.shape), atol=1e-15)
        # merging each split visit with the one after it gives the plain walk
        merged = [c for n, c in enumerate(cells) if n == 0 or not bounce[n - 1]]
        np.testing.assert_array_equal(merged, ref["cells"][r, :ref["len"][r]])
    assert crossed > 60


@pytest.mark.parametrize("kind", ["mirror", "glass"])
def test_crossings_obey_reflection_and_snell(scene, kind):
    rng = np.random.default_rng(3)
    o, d, tmax, start = aimed_rays(rng, 200, scene.sites)
    ior = 1.5
    osc = oracle.OracleScene.from_scene(scene, surface=surface(kind, ior=ior))
    tr = oracle.trace(osc, o, d, tmax, start, eps=0.0, legs=True)
    n_refl = n_refr = n_tir = 0
    for r in range(len(d)):
        cells, te, bounce, lo_, ld_ = _legs(tr, r)
        for n in np.nonzero(bounce)[0]:
            assert n + 1 < len(cells), "a crossing always continues the walk"
            p = lo_[n] + te[n] * ld_[n]
            np.testing.assert_allclose(lo_[n + 1], p, atol=1e-15)        # the new leg starts at the crossing
            assert cells[n + 1] == cells[n]                              # in the same cell
            assert abs(np.linalg.norm(p - CENTRE) - RADIUS) < 1e-12      # on the sphere
            N = unit(p - CENTRE)
            a, b = ld_[n], ld_[n + 1]
            assert abs(np.linalg.norm(b) - 1.0) < 1e-14
            assert abs(np.dot(np.cross(a, b), N)) < 1e-12                # a, b and N coplanar
            reflected = np.dot(a, N) * np.dot(b, N) < 0
            if reflected:
                # the tangential component is kept, the normal one flips
                np.testing.assert_allclose(b - np.dot(b, N) * N, a - np.dot(a, N) * N, atol=1e-12)
                assert abs(np.dot(a, N) + np.dot(b, N)) < 1e-12
                if kind == "glass":
                    # only total internal reflection, from inside at beyond the critical angle
                    assert np.dot(a, N) > 0 and ior * np.linalg.norm(np.cross(a, N)) > 1.0 - 1e-12
                    n_tir += 1
                else:
                    n_refl += 1
            else:
                assert kind == "glass"
                n1, n2 = (1.0, ior) if np.dot(a, N) < 0 else (ior, 1.0)
                assert abs(n1 * np.linalg.norm(np.cross(a, N)) - n2 * np.linalg.norm(np.cross(b, N))) < 1e-12
                n_refr += 1
    if kind == "mirror":
        assert n_refl > 100
    else:
        assert n_refr > 200 and n_tir >= 0


@pytest.mark.parametrize("kind", ["mirror", "glass"])
def test_every_segment_lies_in_its_cell(scene, kind):
    """eq. (5) by brute force along every leg, and with eps = 0 each leg's
    segments tile it from its origin to the crossing or the box."""
    rng = np.random.default_rng(4)
    o, d, tmax, start = aimed_rays(rng, 60, scene.sites)
    osc = oracle.OracleScene.from_scene(scene, surface=surface(kind))
    tr = oracle.trace(osc, o, d, tmax, start, eps=0.0, legs=True)
    x = scene.sites.astype(np.float64)
    checked = 0
    for r in range(len(d)):
        cells, te, bounce, lo_, ld_ = _legs(tr, r)
        t0 = 0.0
        for n in range(len(cells)):
            if te[n] - t0 > 1e-9:
                nn, _ = brute_nn(x, lo_[n] + 0.5 * (t0 + te[n]) * ld_[n])
                assert nn[0] == cells[n], (r, n)
                checked += 1
            if bounce[n]:
                t0 = 0.0
                continue
            if n + 1 == len(cells):
                end = box_exit(lo_[n][None], ld_[n][None])[0] if (n > 0 and bounce[:n].any()) else tmax[r]
                assert abs(te[n] - end) <= 1e-12 * max(1.0, end)
            t0 = te[n]
    assert checked > 500


@pytest.mark.parametrize("kind", ["mirror", "glass"])
def test_fp32_legs_are_rounded_exact_legs(scene, kind):
    """With fp32_legs every leg after a crossing starts from the exact leg's
    origin and direction rounded to FP32, and the walk along it still obeys
    eq. (5) (brute-force nearest sites at every segment midpoint)."""
    rng = np.random.default_rng(41)
    o, d, tmax, start = aimed_rays(rng, 60, scene.sites)
    o, d = o.astype(np.float32).astype(np.float64), d.astype(np.float32).astype(np.float64)
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    ex = oracle.trace(oracle.OracleScene.from_scene(scene, surface=surface(kind)), o, d, tmax, start, eps=0.0,
                      legs=True)
    sf32 = oracle.Surface(kind, CENTRE, RADIUS, BOX, ior=1.5, max_bounces=8, fp32_legs=True)
    f32 = oracle.trace(oracle.OracleScene.from_scene(scene, surface=sf32), o, d, tmax, start, eps=0.0, legs=True)
    x = scene.sites.astype(np.float64)
    checked = 0
    for r in range(len(d)):
        cells, te, bounce, lo_, ld_ = _legs(f32, r)
        e_cells, e_te, e_bounce, e_lo, e_ld = _legs(ex, r)
        n1 = np.nonzero(bounce)[0]
        if len(n1) == 0:
            continue
        b = n1[0]
        # the first crossing is the same; the leg after it is the exact one rounded
        assert e_bounce[b] and abs(te[b] - e_te[b]) <= 1e-12
        np.testing.assert_array_equal(lo_[b + 1], e_lo[b + 1].astype(np.float32).astype(np.float64))
        np.testing.assert_array_equal(ld_[b + 1], e_ld[b + 1].astype(np.float32).astype(np.float64))
        t0 = 0.0
        for n in range(len(cells)):
            if te[n] - t0 > 1e-9:
                assert brute_nn(x, lo_[n] + 0.5 * (t0 + te[n]) * ld_[n])[0][0] == cells[n]
                checked += 1
            t0 = 0.0 if bounce[n] else te[n]
    assert checked > 300


@pytest.mark.parametrize("kind", ["mirror", "glass"])
def test_reversed_path_retraces_the_cells(scene, kind):
    """Light paths are reversible: from the end of the last leg, walking back
    along its reversed direction crosses the sphere at the same points and
    visits the same cells in reverse order."""
    rng = np.random.default_rng(5)
    o, d, tmax, start = aimed_rays(rng, 80, scene.sites)
    osc = oracle.OracleScene.from_scene(scene, surface=surface(kind, ior=1.33))
    fw = oracle.trace(osc, o, d, tmax, start, eps=0.0, legs=True)
    ends, dirs, last = [], [], []
    for r in range(len(d)):
        cells, te, bounce, lo_, ld_ = _legs(fw, r)
        # start the reversed walk at the middle of the last segment (inside the last cell)
        t0 = te[-2] if len(te) > 1 and not bounce[-2] else 0.0
        ends.append(lo_[-1] + 0.5 * (t0 + te[-1]) * ld_[-1])
        dirs.append(-ld_[-1])
        last.append(cells[-1])
    ends, dirs = np.array(ends), np.array(dirs)
    back = oracle.trace(osc, ends, dirs, box_exit(ends, dirs), np.array(last, dtype=np.int32), eps=0.0, legs=True)
    ok = 0
    for r in range(len(d)):
        if min(fw["margin"][r], back["margin"][r], fw["surf_margin"][r], back["surf_margin"][r]) < 1e-7:
            continue
        if min(fw["graze"][r], back["graze"][r]) < 1e-7:
            continue
        a = fw["cells"][r, :fw["len"][r]]
        b = back["cells"][r, :back["len"][r]]
        ba = fw["bounce"][r, :fw["len"][r]]
        bb = back["bounce"][r, :back["len"][r]]
        # the reversed walk goes on past the original origin: compare up to it
        np.testing.assert_array_equal(b[:len(a)], a[::-1])
        assert ba.sum() == bb[:len(a)].sum()
        ok += 1
    assert ok > 50


@pytest.mark.parametrize("kind", ["mirror", "glass"])
def test_homogeneous_medium_over_the_bent_path(kind):
    """One density and one colour everywhere: C = c (1 - e^{-sigma L}) and
    T = e^{-sigma L}, with L the length of the whole path (the sum of the legs'
    lengths, each from its origin to the crossing or the box)."""
    rng = np.random.default_rng(6)
    sites = rng.uniform(-1, 1, size=(250, 3))
    col = np.array([0.3, 0.6, 0.9])
    sig = 1.3
    base = hand_scene(sites, density=sig, colour=col)
    osc = oracle.OracleScene(base.sites, base.off, base.idx, base.density, base.sh, 0,
                             surface(kind, ior=1.6))
    o, d, tmax, start = aimed_rays(rng, 100, base.sites)
    rgb, T, _ = oracle.forward(osc, o, d, tmax, start, eps=0.0)
    tr = oracle.trace(osc, o, d, tmax, start, eps=0.0, legs=True)
    for r in range(len(d)):
        cells, te, bounce, lo_, ld_ = _legs(tr, r)
        length = te[bounce].sum() + te[-1]
        # each leg ends on the sphere or on the box: check the geometry independently
        for n in np.nonzero(bounce)[0]:
            assert abs(np.linalg.norm(lo_[n] + te[n] * ld_[n] - CENTRE) - RADIUS) < 1e-12
        assert abs(np.abs(lo_[-1] + te[-1] * ld_[-1]).max() - 1.0) < 1e-12
        np.testing.assert_allclose(T[r], np.exp(-sig * length), rtol=1e-12)
        np.testing.assert_allclose(rgb[r], col * (1 - np.exp(-sig * length)), rtol=1e-11, atol=1e-14)


@pytest.mark.parametrize("kind", ["mirror", "glass"])
def test_bent_render_composes_its_legs(scene, kind):
    """With eps = 0 a bent ray's colour is its legs' colours composited in
    order, C = sum_k (prod_{j<k} T_j) C_k and T = prod_k T_k, where leg k is
    rendered as a plain ray (no surface) from its origin, in its own direction,
    over its own length, starting in the nearest cell of its origin. The leg
    directions are rebuilt here from the reflection law (mirror) or taken from
    the trace (glass, whose directions the Snell pin checks)."""
    rng = np.random.default_rng(10)
    o, d, tmax, start = aimed_rays(rng, 60, scene.sites)
    osc = oracle.OracleScene.from_scene(scene, surface=surface(kind, ior=1.4))
    plain = oracle.OracleScene.from_scene(scene)
    rgb, T, _ = oracle.forward(osc, o, d, tmax, start, eps=0.0)
    tr = oracle.trace(osc, o, d, tmax, start, eps=0.0, legs=True)
    x = scene.sites.astype(np.float64)
    bent = 0
    for r in range(len(d)):
        cells, te, bounce, lo_, ld_ = _legs(tr, r)
        if not bounce.any():
            continue
        bent += 1
        ends = list(np.nonzero(bounce)[0]) + [len(cells) - 1]
        lo, ld = o[r].copy(), d[r].copy()
        C, Tacc = np.zeros(3), 1.0
        for k, n in enumerate(ends):
            if kind == "glass":
                lo, ld = lo_[n], ld_[n]
            np.testing.assert_allclose(ld, ld_[n], atol=1e-13)
            s0 = brute_nn(x, lo)[0].astype(np.int32)
            ck, tk, _ = oracle.forward(plain, lo[None], ld[None], np.array([te[n]]), s0, eps=0.0)
            C += Tacc * ck[0]
            Tacc *= tk[0]
            if kind == "mirror" and k + 1 < len(ends):
                p = lo + te[n] * ld
                N = (p - CENTRE) / np.linalg.norm(p - CENTRE)
                lo, ld = p, ld - 2.0 * np.dot(ld, N) * N
        np.testing.assert_allclose(rgb[r], C, rtol=1e-9, atol=1e-12)
        np.testing.assert_allclose(T[r], Tacc, rtol=1e-9)
    assert bent > 30


def _loss(osc, o, d, tmax, start, g, gT, eps):
    rgb, T, _ = oracle.forward(osc, o, d, tmax, start, eps=eps, threads=1)
    return (rgb * g).sum() + (T * gT).sum()


@pytest.mark.parametrize("kind,eps", [("mirror", 0.0), ("glass", 0.0), ("glass", 1e-2)])
def test_gradients_with_a_surface_match_finite_differences(kind, eps):
    sc = synth.small_scene("uniform11", 120, seed=32, sh_deg=3)
    rng = np.random.default_rng(7)
    o, d, tmax, start = aimed_rays(rng, 50, sc.sites)
    dens = sc.density.astype(np.float64) * (4.0 if eps else 1.0)
    sf = surface(kind, ior=1.45)
    osc = oracle.OracleScene(sc.sites, sc.off, sc.idx, dens, sc.sh, 3, sf)
    tr = oracle.trace(osc, o, d, tmax, start, eps=eps)
    keep = ((tr["margin"] > 1e-4) & (tr["graze"] > 1e-4) & (tr["surf_margin"] > 1e-4)
            & ((tr["term"] > 1e-2) | (eps == 0)))
    crossed = np.array([tr["bounce"][r, :tr["len"][r]].any() for r in range(len(d))])
    keep &= crossed
    o, d, tmax, start = o[keep], d[keep], tmax[keep], start[keep]
    assert len(d) >= 20
    g = rng.standard_normal((len(d), 3))
    gT = rng.standard_normal(len(d))
    gs, gd, gsh = oracle.backward(osc, o, d, tmax, start, g, gT, eps=eps, threads=1)
    sites = sc.sites.astype(np.float64)
    sh = sc.sh.astype(np.float64)

    def L(sites_=sites, dens_=dens, sh_=sh):
        s = oracle.OracleScene(sites_, sc.off, sc.idx, dens_, sh_, 3, sf)
        return _loss(s, o, d, tmax, start, g, gT, eps)

    h = 1e-6
    touched = np.unique(np.concatenate([tr["cells"][keep][r, :tr["len"][keep][r]] for r in range(len(d))]))
    rng2 = np.random.default_rng(8)
    for i in rng2.choice(touched, size=min(20, len(touched)), replace=False):
        for a in range(3):
            sp, sm = sites.copy(), sites.copy()
            sp[i, a] += h
            sm[i, a] -= h
            fd = (L(sites_=sp) - L(sites_=sm)) / (2 * h)
            assert abs(fd - gs[i, a]) <= 1e-5 * max(1.0, abs(fd)), (i, a, fd, gs[i, a])
        dp, dm = dens.copy(), dens.copy()
        dp[i] += h
        dm[i] -= h
        fd = (L(dens_=dp) - L(dens_=dm)) / (2 * h)
        assert abs(fd - gd[i]) <= 1e-6 * max(1.0, abs(fd)), (i, fd, gd[i])
        b, ch = rng2.integers(16), rng2.integers(3)
        hp, hm = sh.copy(), sh.copy()
        hp[i, b, ch] += 1e-3
        hm[i, b, ch] -= 1e-3
        fd = (L(sh_=hp) - L(sh_=hm)) / 2e-3
        assert abs(fd - gsh[i, b, ch]) <= 1e-10 * max(1.0, abs(fd))


def test_quantiles_reject_a_surface(scene):
    osc = oracle.OracleScene.from_scene(scene, surface=surface("mirror"))
    o, d, tmax, start = aimed_rays(np.random.default_rng(9), 4, scene.sites)
    with pytest.raises(ValueError):
        oracle.quantile(osc, o, d, tmax, start, np.full((4, 2), 0.5))


# ---------------------------------------------------------------------------
# equidistant fisheye camera
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("W,H,fov", [(32, 24, 180.0), (17, 9, 120.0), (40, 40, 360.0)])
def test_fisheye_angle_is_proportional_to_radius(W, H, fov):
    rng = np.random.default_rng(W + H)
    cam = synth.make_cameras("shell_3m", rng, n=1, res=(W, H))[0]
    o, d, tmax, pix = oracle.raygen(cam.pose12(), fov, W, H, BOX, model="fisheye")
    assert sorted(pix.tolist()) == list(range(W * H))
    np.testing.assert_allclose(np.linalg.norm(d, axis=1), 1.0, atol=1e-15)
    cam_d = d @ cam.rotation                       # camera frame (right, down, forward)
    u = pix % W + 0.5 - 0.5 * W
    v = pix // W + 0.5 - 0.5 * H
    rho = np.hypot(u, v)
    theta = np.arctan2(np.hypot(cam_d[:, 0], cam_d[:, 1]), cam_d[:, 2])
    np.testing.assert_allclose(theta, np.minimum(rho * np.radians(fov) / W, np.pi) if fov < 360 else
                               np.where(rho * np.radians(fov) / W <= np.pi, rho * np.radians(fov) / W,
                                        2 * np.pi - rho * np.radians(fov) / W), atol=1e-12)
    # the direction's image-plane part points along (u, v), wherever it is not at a pole
    side = np.abs(np.sin(rho * np.radians(fov) / W)) > 1e-9
    sgn = np.sign(np.sin(rho * np.radians(fov) / W))
    cross = cam_d[:, 0] * v - cam_d[:, 1] * u
    dotp = (cam_d[:, 0] * u + cam_d[:, 1] * v) * sgn
    np.testing.assert_allclose(cross[side], 0.0, atol=1e-12)
    assert np.all(dotp[side] > 0)
    # exits on the box
    p = o + tmax[:, None] * d
    np.testing.assert_allclose(np.abs(p).max(1), 1.0, atol=1e-12)


def test_narrow_fisheye_approaches_the_pinhole():
    """theta = rho (fov/2)/(W/2) and tan(theta) = rho/f differ by O(theta^3)."""
    rng = np.random.default_rng(11)
    cam = synth.make_cameras("shell_3m", rng, n=1, res=(24, 16))[0]
    _, dp, _, _ = oracle.raygen(cam.pose12(), 0.5, 24, 16, BOX)
    _, df, _, _ = oracle.raygen(cam.pose12(), 0.5, 24, 16, BOX, model="fisheye")
    np.testing.assert_allclose(df, dp, atol=1e-7)
    assert np.abs(df - dp).max() > 0                # different models


def test_fisheye_rejects_bad_fov():
    cam = synth.make_cameras("shell_3m", np.random.default_rng(12), n=1, res=(4, 4))[0]
    for fov in (0.0, 361.0, -5.0):
        with pytest.raises(ValueError):
            oracle.raygen(cam.pose12(), fov, 4, 4, BOX, model="fisheye")
    oracle.raygen(cam.pose12(), 360.0, 4, 4, BOX, model="fisheye")
    with pytest.raises(ValueError):
        oracle.raygen(cam.pose12(), 180.0, 4, 4, BOX)       # pinhole needs fov < 180
