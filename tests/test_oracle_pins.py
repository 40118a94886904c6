"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

Each test checks the oracle against something other than itself: brute-force
nearest-site search (eq. (5)), closed forms of the compositing sum (eq. (3)-(4)
on special media), library routines (scipy's spherical harmonics, torch's
bfloat16 rounding), geometric invariants, quadrature of the continuous
integral (eq. (1)-(2)), and central finite differences for the gradients.
"""

import json
import os

import numpy as np
import pytest

import oracle
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------------------
# helpers (test-side brute force; independent of the oracle's walk)
# ---------------------------------------------------------------------------

def brute_nn(sites, pts):
    """Nearest site of each point by exhaustive search, fp64."""
    s = np.asarray(sites, dtype=np.float64)
    p = np.atleast_2d(pts)
    d2 = ((p[:, None, :] - s[None, :, :]) ** 2).sum(-1)
    return np.argmin(d2, axis=1), np.sort(d2, axis=1)


def unit(v):
    v = np.asarray(v, dtype=np.float64)
    return v / np.linalg.norm(v, axis=-1, keepdims=True)


def random_inside_rays(rng, n, lo, hi, sites, margin=0.0):
    o = rng.uniform(lo + margin, hi - margin, size=(n, 3))
    d = unit(rng.standard_normal((n, 3)))
    tmax = np.empty(n)
    for r in range(n):
        ts = []
        for a in range(3):
            if d[r, a] > 0:
                ts.append((hi - o[r, a]) / d[r, a])
            elif d[r, a] < 0:
                ts.append((lo - o[r, a]) / d[r, a])
        tmax[r] = min(ts)
    start = brute_nn(sites, o)[0].astype(np.int32)
    return o, d, tmax, start


def hand_scene(sites, sh_deg=0, density=None, colour=None):
    sites = np.asarray(sites, dtype=np.float64)
    off, idx = synth.build_adjacency(sites.astype(np.float32))
    n = len(sites)
    b = (sh_deg + 1) ** 2
    dens = np.ones(n) if density is None else np.broadcast_to(density, (n,)).astype(np.float64)
    sh = np.zeros((n, b, 3))
    if colour is not None:
        sh[:, 0, :] = np.asarray(colour) / (0.5 * np.sqrt(1.0 / np.pi))
    return oracle.OracleScene(sites.astype(np.float32), off, idx, dens, sh, sh_deg)


@pytest.fixture(scope="module")
def uniform_scene():
    return synth.small_scene("uniform01", 400, seed=11, sh_deg=3)


@pytest.fixture(scope="module")
def clustered_scene():
    return synth.small_scene("clustered", 500, seed=12, sh_deg=3)


# ---------------------------------------------------------------------------
# spherical harmonics (Sec. 3.4: view-dependent colour via SH of degree 3)
# ---------------------------------------------------------------------------

def scipy_real_sh(l, m, d):
    from scipy.special import sph_harm_y

    x, y, z = d[:, 0], d[:, 1], d[:, 2]
    theta = np.arccos(np.clip(z, -1, 1))
    phi = np.mod(np.arctan2(y, x), 2 * np.pi)
    if m == 0:
        return sph_harm_y(l, 0, theta, phi).real
    c = sph_harm_y(l, abs(m), theta, phi)
    if m > 0:
        return np.sqrt(2) * (-1) ** m * c.real
    return np.sqrt(2) * (-1) ** m * c.imag


def test_sh_matches_scipy_real_form():
    rng = np.random.default_rng(0)
    d = unit(rng.standard_normal((200, 3)))
    Y = oracle.sh_basis(3, d)
    k = 0
    for l in range(4):
        for m in range(-l, l + 1):
            np.testing.assert_allclose(Y[:, k], scipy_real_sh(l, m, d), rtol=0, atol=1e-13,
                                       err_msg=f"l={l} m={m}")
            k += 1


def test_sh_orthonormal_by_quadrature():
    # Gauss-Legendre in cos(theta) x uniform phi is exact for these degree<=6 products.
    xg, wg = np.polynomial.legendre.leggauss(12)
    phi = (np.arange(24) + 0.5) * 2 * np.pi / 24
    ct, ph = np.meshgrid(xg, phi, indexing="ij")
    st = np.sqrt(1 - ct ** 2)
    d = np.stack([st * np.cos(ph), st * np.sin(ph), ct], -1).reshape(-1, 3)
    w = (wg[:, None] * np.full(phi.shape, 2 * np.pi / 24)[None, :]).reshape(-1)
    Y = oracle.sh_basis(3, d)
    G = (Y * w[:, None]).T @ Y
    np.testing.assert_allclose(G, np.eye(16), atol=1e-12)


def test_sh_degree_prefix_and_y00():
    d = unit(np.array([[0.3, -0.4, 0.866]]))
    Y3 = oracle.sh_basis(3, d)
    for deg in range(3):
        np.testing.assert_array_equal(oracle.sh_basis(deg, d)[0], Y3[0, :(deg + 1) ** 2])
    assert abs(Y3[0, 0] - 0.28209479177387814) < 1e-16


# ---------------------------------------------------------------------------
# bfloat16 rounding (stored attribute precision)
# ---------------------------------------------------------------------------

def test_bf16_round_matches_torch():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(1)
    x = np.concatenate([
        rng.standard_normal(20000).astype(np.float32) * np.float32(10.0) ** rng.integers(-30, 30, 20000),
        np.array([0.0, -0.0, 1.0, -1.0, np.inf, -np.inf, 3.4e38, -3.4e38, 1e-40, -1e-40, 1e-45],
                 dtype=np.float32),
        # exact ties: low 16 bits == 0x8000 with even and odd upper halves
        np.array([0x3F808000, 0x3F818000, 0xBF808000, 0x7F7F8000, 0x00008000, 0x00018000],
                 dtype=np.uint32).view(np.float32),
    ]).astype(np.float32)
    ours = oracle.bf16_round(x)
    ref = torch.from_numpy(x).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    np.testing.assert_array_equal(ours, ref)
    nan = oracle.bf16_round(np.array([np.nan], dtype=np.float32))
    assert np.isnan(oracle.bf16_to_f32(nan))[0]


# ---------------------------------------------------------------------------
# face planes: the bisector of (x_i, x_j) is the set of points equidistant to both
# ---------------------------------------------------------------------------

def test_face_planes_are_bisectors(uniform_scene):
    sc = uniform_scene
    P = oracle.face_planes(sc.sites, sc.off, sc.idx)
    rng = np.random.default_rng(2)
    x = sc.sites.astype(np.float64)
    rows = np.repeat(np.arange(sc.n_sites), np.diff(sc.off))
    k = rng.integers(0, sc.n_edges, 300)
    xi, xj, n, c = x[rows[k]], x[sc.idx[k]], P[k, :3], P[k, 3]
    np.testing.assert_allclose(n, xj - xi, atol=0)
    # a point on the plane: foot of a random point, projected along n
    q = rng.uniform(-1, 2, size=(len(k), 3))
    p = q - ((q * n).sum(1) - c)[:, None] * n / (n * n).sum(1, keepdims=True)
    np.testing.assert_allclose(((p - xi) ** 2).sum(1), ((p - xj) ** 2).sum(1), atol=1e-12)
    # the directed pair (j, i) has exactly the negated plane
    for kk in k[:50]:
        i, j = rows[kk], sc.idx[kk]
        back = sc.off[j] + np.searchsorted(sc.idx[sc.off[j]:sc.off[j + 1]], i)
        np.testing.assert_array_equal(P[back], -P[kk])


def test_csr_check_rejects_bad_adjacency(uniform_scene):
    sc = uniform_scene
    assert oracle.check_csr(sc.off, sc.idx, sc.n_sites)
    bad = sc.idx.copy()
    bad[5] = sc.n_sites
    assert not oracle.check_csr(sc.off, bad, sc.n_sites)
    selfloop = sc.idx.copy()
    selfloop[sc.off[3]] = 3
    assert not oracle.check_csr(sc.off, selfloop, sc.n_sites)
    off = sc.off.copy()
    off[10], off[11] = off[11], off[10]
    assert not oracle.check_csr(off, sc.idx, sc.n_sites)


# ---------------------------------------------------------------------------
# camera rays (pinhole, 8x8 tile order)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("W,H", [(64, 64), (20, 13), (1, 1), (9, 17)])
def test_raygen_projects_back_to_pixel_centres(W, H):
    rng = np.random.default_rng(W * 100 + H)
    cam = synth.make_cameras("shell_3m", rng, n=1, res=(W, H))[0]
    o, d, tmax, pix = oracle.raygen(cam.pose12(), cam.fov_deg, W, H, ("box", -1.0, 1.0))
    assert sorted(pix.tolist()) == list(range(W * H))
    np.testing.assert_allclose(np.linalg.norm(d, axis=1), 1.0, atol=1e-15)
    cam_d = d @ cam.rotation                      # R^T d, rows
    f = 0.5 * W / np.tan(np.radians(cam.fov_deg) / 2)
    u = cam_d[:, 0] / cam_d[:, 2] * f + 0.5 * W
    v = cam_d[:, 1] / cam_d[:, 2] * f + 0.5 * H
    np.testing.assert_allclose(u, pix % W + 0.5, atol=1e-9)
    np.testing.assert_allclose(v, pix // W + 0.5, atol=1e-9)
    # tile order: every aligned run of rays inside one 8x8 tile, tiles row-major
    tile = (pix // W // 8) * ((W + 7) // 8) + (pix % W) // 8
    assert np.all(np.diff(tile) >= 0)
    within = (pix // W % 8) * 8 + pix % W % 8
    for t in np.unique(tile):
        assert np.all(np.diff(within[tile == t]) > 0)
    # exit point lies on the box surface
    p = o + tmax[:, None] * d
    np.testing.assert_allclose(np.abs(p).max(1), 1.0, atol=1e-12)
    assert np.all(np.abs(p) <= 1 + 1e-12)


def test_raygen_sphere_bound():
    rng = np.random.default_rng(3)
    cam = synth.make_cameras("shell_3m", rng, n=1, res=(16, 8))[0]
    o, d, tmax, _ = oracle.raygen(cam.pose12(), cam.fov_deg, 16, 8, ("sphere", 5.0))
    np.testing.assert_allclose(np.linalg.norm(o + tmax[:, None] * d, axis=1), 5.0, atol=1e-12)
    assert np.all(tmax > 0)


# ---------------------------------------------------------------------------
# the walk (Algorithm 1) against eq. (5) by brute force
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("which", ["uniform_scene", "clustered_scene"])
def test_segments_lie_in_their_voronoi_cell(which, request):
    sc = request.getfixturevalue(which)
    lo, hi = (0.0, 1.0) if which == "uniform_scene" else (-1.0, 1.0)
    rng = np.random.default_rng(4)
    o, d, tmax, start = random_inside_rays(rng, 120, lo, hi, sc.sites)
    osc = oracle.OracleScene.from_scene(sc)
    tr = oracle.trace(osc, o, d, tmax, start, eps=0.0)
    x = sc.sites.astype(np.float64)
    n_checked = 0
    for r in range(len(d)):
        L = tr["len"][r]
        assert tr["steps"][r] == L
        t0 = 0.0
        for n in range(L):
            te = tr["t_exit"][r, n]
            cell = tr["cells"][r, n]
            if te - t0 > 1e-9:
                nn, _ = brute_nn(x, o[r] + 0.5 * (t0 + te) * d[r])
                assert nn[0] == cell, (r, n)
                n_checked += 1
            if n + 1 < L:
                # the exit point is equidistant to the two cells' sites, and no site is closer
                p = o[r] + te * d[r]
                nxt = tr["cells"][r, n + 1]
                di = ((p - x[cell]) ** 2).sum()
                dj = ((p - x[nxt]) ** 2).sum()
                assert abs(di - dj) <= 1e-9 * max(1.0, di)
                _, d2 = brute_nn(x, p)
                assert d2[0, 0] >= di - 1e-9
            t0 = te
        # coverage: with eps = 0 the segments tile [0, t_max]
        assert abs(t0 - tmax[r]) <= 1e-12 * max(1.0, tmax[r])
    assert n_checked > 500


def test_dense_sampling_run_lengths_match_sequence(clustered_scene):
    sc = clustered_scene
    rng = np.random.default_rng(5)
    o, d, tmax, start = random_inside_rays(rng, 30, -1.0, 1.0, sc.sites)
    tr = oracle.trace(oracle.OracleScene.from_scene(sc), o, d, tmax, start, eps=0.0)
    x = sc.sites.astype(np.float64)
    h = 2e-4
    for r in range(len(d)):
        ts = np.arange(h / 2, tmax[r], h)
        nn, _ = brute_nn(x, o[r] + ts[:, None] * d[r])
        runs = nn[np.r_[True, nn[1:] != nn[:-1]]]
        seq = tr["cells"][r, :tr["len"][r]]
        # every sampled run appears in order in the oracle's sequence; segments
        # shorter than the step may be skipped by the sampling only
        deltas = np.diff(np.r_[0.0, tr["t_exit"][r, :tr["len"][r]]])
        pos = 0
        for c in runs:
            while seq[pos] != c:
                assert deltas[pos] < 2 * h, (r, pos)
                pos += 1
            pos += 1
        assert np.all(deltas[pos:] < 2 * h)


def test_start_cell_is_nearest_site(uniform_scene):
    rng = np.random.default_rng(6)
    pts = rng.uniform(0, 1, size=(200, 3))
    np.testing.assert_array_equal(synth.nearest_site(uniform_scene.sites, pts),
                                  brute_nn(uniform_scene.sites, pts)[0])


# ---------------------------------------------------------------------------
# compositing closed forms (eq. (3)-(4))
# ---------------------------------------------------------------------------

def test_homogeneous_medium_closed_form(uniform_scene):
    sc = uniform_scene
    rng = np.random.default_rng(7)
    o, d, tmax, start = random_inside_rays(rng, 200, 0.0, 1.0, sc.sites)
    sig = 1.7
    col = np.array([0.3, -0.2, 0.9])
    osc = hand_scene(sc.sites, 0, density=sig, colour=col)
    rgb, T, steps = oracle.forward(osc, o, d, tmax, start, eps=0.0)
    np.testing.assert_allclose(T, np.exp(-sig * tmax), rtol=1e-12)
    np.testing.assert_allclose(rgb, (1 - np.exp(-sig * tmax))[:, None] * col[None, :], rtol=1e-12, atol=1e-15)
    assert np.all(steps > 0)


def test_zero_density_is_transparent(uniform_scene):
    sc = uniform_scene
    rng = np.random.default_rng(8)
    o, d, tmax, start = random_inside_rays(rng, 50, 0.0, 1.0, sc.sites)
    osc = oracle.OracleScene.from_scene(sc, density=np.zeros(sc.n_sites))
    rgb, T, _ = oracle.forward(osc, o, d, tmax, start, eps=0.0)
    assert np.all(rgb == 0.0) and np.all(T == 1.0)


def test_two_sites_bisector_and_single_cell():
    # sites at x=0 and x=2: the bisector is the plane x = 1
    osc = hand_scene([[0, 0, 0], [2, 0, 0], [0, 5, 0], [0, 0, 5], [-5, -5, -5]], 0,
                     density=[0.5, 2.0, 0, 0, 0], colour=[1.0, 0.5, 0.25])
    o = np.array([[-0.5, 0.3, 0.2]])
    d = unit([[1.0, 0.1, -0.05]])
    tr = oracle.trace(osc, o, d, [4.0], [0], eps=0.0)
    assert tr["cells"][0, :2].tolist() == [0, 1]
    t_cross = (1.0 - o[0, 0]) / d[0, 0]
    assert abs(tr["t_exit"][0, 0] - t_cross) < 1e-14
    # single cell: a ray that never leaves cell 0 gives alpha = 1 - exp(-sigma t)
    rgb, T, steps = oracle.forward(osc, [[0.2, 0.1, 0.1]], unit([[-1.0, 0.05, 0.02]]), [0.9], [0], eps=0.0)
    assert steps[0] == 1
    np.testing.assert_allclose(T[0], np.exp(-0.5 * 0.9), rtol=1e-15)
    np.testing.assert_allclose(rgb[0], (1 - np.exp(-0.5 * 0.9)) * np.array([1.0, 0.5, 0.25]), rtol=1e-14)


def test_golden_lattice_walk():
    with open(os.path.join(GOLDEN, "lattice_walk.json")) as f:
        g = json.load(f)
    h = g["spacing"]
    n = g["n"]
    rng = np.random.default_rng(g["seed"])
    ii = np.stack(np.meshgrid(*[np.arange(n)] * 3, indexing="ij"), -1).reshape(-1, 3)
    sites = (ii + 0.5) * h + rng.uniform(-g["jitter"], g["jitter"], size=ii.shape) * h
    osc = hand_scene(sites, 0, density=1.0, colour=[1, 1, 1])
    for case in g["rays"]:
        o = np.array([case["origin"]])
        d = unit([case["dir"]])
        start = brute_nn(sites, o)[0]
        tr = oracle.trace(osc, o, d, [case["tmax"]], start, eps=0.0)
        L = tr["len"][0]
        cells = [tuple(ii[c]) for c in tr["cells"][0, :L]]
        assert cells == [tuple(c) for c in case["cells"]]
        np.testing.assert_allclose(tr["t_exit"][0, :L], case["t_exit"], atol=case["t_tol"])


def test_transmittance_threshold_rule(uniform_scene):
    sc = uniform_scene
    rng = np.random.default_rng(9)
    o, d, tmax, start = random_inside_rays(rng, 100, 0.0, 1.0, sc.sites)
    osc = oracle.OracleScene.from_scene(sc, density=np.full(sc.n_sites, 30.0))
    eps = 1e-3
    tr = oracle.trace(osc, o, d, tmax, start, eps=eps)
    for r in range(len(d)):
        L = tr["len"][r]
        te = tr["t_exit"][r, :L]
        T_before_last = np.exp(-30.0 * (te[-2] if L > 1 else 0.0))
        assert T_before_last > eps
        reached_end = abs(te[-1] - tmax[r]) < 1e-12
        assert reached_end or tr["t_final"][r] <= eps
        np.testing.assert_allclose(tr["t_final"][r], np.exp(-30.0 * te[-1]), rtol=1e-12)


def test_status_codes(uniform_scene):
    sc = uniform_scene
    osc = oracle.OracleScene.from_scene(sc)
    rng = np.random.default_rng(10)
    o, d, tmax, start = random_inside_rays(rng, 20, 0.0, 1.0, sc.sites)
    start_bad = start.copy()
    start_bad[:5] = [-1, sc.n_sites, sc.n_sites + 7, -100, 2 ** 31 - 1]
    rgb, T, steps = oracle.forward(osc, o, d, tmax, start_bad, eps=0.0)
    assert np.all(steps[:5] == oracle.BAD_START)
    assert np.all(rgb[:5] == 0) and np.all(T[:5] == 1)
    tr = oracle.trace(osc, o, d, tmax, start, eps=0.0, max_steps=3)
    long_rays = tr["len"] == 3
    assert np.any(long_rays)
    assert np.all(tr["steps"][long_rays & (tr["t_exit"][:, 2] < tmax - 1e-12)] == oracle.MAX_STEPS)
    with pytest.raises(ValueError):
        oracle.forward(osc, o, d * 1.01, tmax, start)


# ---------------------------------------------------------------------------
# invariants
# ---------------------------------------------------------------------------

def test_reversal_gives_reversed_sequence(clustered_scene):
    sc = clustered_scene
    rng = np.random.default_rng(13)
    o, d, tmax, start = random_inside_rays(rng, 60, -1.0, 1.0, sc.sites, margin=0.05)
    tmax = tmax * 0.97                       # end strictly inside the box
    osc = oracle.OracleScene.from_scene(sc)
    fw = oracle.trace(osc, o, d, tmax, start, eps=0.0)
    ends = o + tmax[:, None] * d
    last = fw["cells"][np.arange(len(d)), fw["len"] - 1]
    bw = oracle.trace(osc, ends, -d, tmax, last, eps=0.0)
    ok = 0
    for r in range(len(d)):
        if fw["margin"][r] < 1e-9 or bw["margin"][r] < 1e-9:
            continue
        a = fw["cells"][r, :fw["len"][r]]
        b = bw["cells"][r, :bw["len"][r]]
        np.testing.assert_array_equal(a, b[::-1])
        ok += 1
    assert ok > 50


def test_scale_invariance(clustered_scene):
    sc = clustered_scene
    rng = np.random.default_rng(14)
    o, d, tmax, start = random_inside_rays(rng, 80, -1.0, 1.0, sc.sites)
    s = 4.0                                   # power of two: the scaled sites are exact
    base = oracle.forward(oracle.OracleScene.from_scene(sc), o, d, tmax, start, eps=0.0)
    big = oracle.OracleScene(sc.sites * s, sc.off, sc.idx, sc.density / s, sc.sh, sc.sh_deg)
    scaled = oracle.forward(big, o * s, d, tmax * s, start, eps=0.0)
    np.testing.assert_allclose(scaled[0], base[0], rtol=1e-10, atol=1e-13)
    np.testing.assert_allclose(scaled[1], base[1], rtol=1e-10)
    np.testing.assert_array_equal(scaled[2], base[2])


def test_riemann_sums_converge_to_walk(clustered_scene):
    """Eq. (1)-(2) integrated numerically with brute-force nearest sites converges to eq. (3)."""
    sc = clustered_scene
    rng = np.random.default_rng(15)
    o, d, tmax, start = random_inside_rays(rng, 6, -1.0, 1.0, sc.sites)
    osc = oracle.OracleScene.from_scene(sc)
    rgb, T, _ = oracle.forward(osc, o, d, tmax, start, eps=0.0)
    x = sc.sites.astype(np.float64)
    Y = oracle.sh_basis(3, d)
    errs = []
    for h in (4e-3, 1e-3, 2.5e-4):
        e = 0.0
        for r in range(len(d)):
            ts = np.arange(h / 2, tmax[r], h)
            hh = np.full(ts.shape, h)
            hh[-1] = tmax[r] - (ts[-1] - h / 2)
            nn, _ = brute_nn(x, o[r] + ts[:, None] * d[r])
            sig = sc.density[nn].astype(np.float64)
            col = np.einsum("nbc,b->nc", sc.sh[nn].astype(np.float64), Y[r])
            tau = sig * hh
            Tb = np.exp(-np.concatenate([[0.0], np.cumsum(tau)[:-1]]))
            c_num = (Tb[:, None] * (1 - np.exp(-tau))[:, None] * col).sum(0)
            e = max(e, np.abs(c_num - rgb[r]).max())
        errs.append(e)
    assert errs[2] < errs[1] < errs[0]
    assert errs[2] < 0.05 * max(1.0, np.abs(rgb).max())


# ---------------------------------------------------------------------------
# statistics of a Poisson-Voronoi tessellation
# ---------------------------------------------------------------------------

@pytest.mark.slow
def test_crossings_per_unit_length_poisson_voronoi():
    """A line meets Poisson-Voronoi faces at rate S_V/2 = 1.4552 lambda^(1/3) (Meijering)."""
    sc = synth.small_scene("uniform01", 30000, seed=16, sh_deg=0)
    rng = np.random.default_rng(17)
    n = 1500
    o = rng.uniform(0.25, 0.75, size=(n, 3))
    d = unit(rng.standard_normal((n, 3)))
    L = 0.2
    start = synth.nearest_site(sc.sites, o)
    tr = oracle.trace(oracle.OracleScene.from_scene(sc, density=np.zeros(sc.n_sites)), o, d,
                      np.full(n, L), start, eps=0.0)
    rate = (tr["len"] - 1).sum() / (n * L)
    expect = 1.4552 * 30000 ** (1 / 3)
    assert abs(rate / expect - 1) < 0.03, (rate, expect)


# ---------------------------------------------------------------------------
# gradients: central finite differences on the FP64 oracle
# ---------------------------------------------------------------------------

def _loss(osc, o, d, tmax, start, g, gT, eps):
    rgb, T, _ = oracle.forward(osc, o, d, tmax, start, eps=eps, threads=1)
    return (rgb * g).sum() + (T * gT).sum()


@pytest.mark.parametrize("eps", [0.0, 1e-2])
def test_gradients_match_finite_differences(eps):
    sc = synth.small_scene("uniform11", 120, seed=18, sh_deg=3)
    rng = np.random.default_rng(19)
    o, d, tmax, start = random_inside_rays(rng, 60, -0.9, 0.9, sc.sites)
    dens = sc.density.astype(np.float64) * (4.0 if eps else 1.0)
    osc = oracle.OracleScene(sc.sites, sc.off, sc.idx, dens, sc.sh, 3)
    tr = oracle.trace(osc, o, d, tmax, start, eps=eps)
    keep = (tr["margin"] > 1e-4) & (tr["graze"] > 1e-4) & ((tr["term"] > 1e-2) | (eps == 0))
    o, d, tmax, start = o[keep], d[keep], tmax[keep], start[keep]
    assert len(d) >= 30
    g = rng.standard_normal((len(d), 3))
    gT = rng.standard_normal(len(d))
    gs, gd, gsh = oracle.backward(osc, o, d, tmax, start, g, gT, eps=eps, threads=1)

    sites = sc.sites.astype(np.float64)
    sh = sc.sh.astype(np.float64)

    def L(sites_=sites, dens_=dens, sh_=sh):
        s = oracle.OracleScene(sites_, sc.off, sc.idx, dens_, sh_, 3)
        return _loss(s, o, d, tmax, start, g, gT, eps)

    h = 1e-6
    touched = np.unique(np.concatenate([tr["cells"][keep][r, :tr["len"][keep][r]] for r in range(len(d))]))
    rng2 = np.random.default_rng(20)
    for i in rng2.choice(touched, size=min(25, len(touched)), replace=False):
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
        fd = (L(sh_=hp) - L(sh_=hm)) / 2e-3          # colour is linear in the coefficients
        assert abs(fd - gsh[i, b, ch]) <= 1e-10 * max(1.0, abs(fd))
    untouched = np.setdiff1d(np.arange(sc.n_sites), touched)
    assert np.all(gd[untouched] == 0) and np.all(gsh[untouched] == 0)


def test_site_gradient_sums_match_translation():
    """Moving every site and the ray origins together leaves the render unchanged, so
    the summed site gradient equals minus the origin gradient (checked by FD on origins)."""
    sc = synth.small_scene("uniform11", 150, seed=21, sh_deg=1)
    rng = np.random.default_rng(22)
    o, d, tmax, start = random_inside_rays(rng, 40, -0.8, 0.8, sc.sites)
    osc = oracle.OracleScene.from_scene(sc)
    tr = oracle.trace(osc, o, d, tmax, start, eps=0.0)
    keep = (tr["margin"] > 1e-4) & (tr["graze"] > 1e-4)
    o, d, tmax, start = o[keep], d[keep], tmax[keep], start[keep]
    g = rng.standard_normal((len(d), 3))
    gs, _, _ = oracle.backward(osc, o, d, tmax, start, g, eps=0.0, threads=1)
    h = 1e-6
    for a in range(3):
        e = np.zeros(3)
        e[a] = h
        Lp = _loss(osc, o - e, d, tmax, start, g, 0 * tmax, 0.0)
        Lm = _loss(osc, o + e, d, tmax, start, g, 0 * tmax, 0.0)
        fd = (Lp - Lm) / (2 * h)                 # = sum_i dL/dx_i (translation of all sites)
        assert abs(fd - gs[:, a].sum()) < 1e-6 * max(1.0, abs(fd))


# ---------------------------------------------------------------------------
# nearest site (the cell of a point, eq. (5)): start-cell location
# ---------------------------------------------------------------------------

def test_nearest_site_by_hand_on_a_line():
    # sites at x = 0, 1, 3; the bisectors are x = 0.5 and x = 2
    sites = np.array([[0.0, 0, 0], [1.0, 0, 0], [3.0, 0, 0]])
    q = np.array([[0.4, 0, 0], [0.5, 0, 0], [0.6, 0, 0], [2.0, 0, 0], [2.1, 0, 0], [3.0, 0, 0], [-5.0, 2, 0]])
    idx, gap = oracle.nearest_site(sites, q, return_gap=True)
    np.testing.assert_array_equal(idx, [0, 0, 1, 1, 2, 2, 0])  # exact ties keep the lower index
    # 0.6: d2 = 0.36 to site 0 and 0.16 to site 1; a point on a bisector has gap 0; a site has gap 1
    np.testing.assert_allclose(gap[[1, 2, 3, 5]], [0.0, (0.36 - 0.16) / 0.36, 0.0, 1.0])


def test_nearest_site_matches_kdtree():
    from scipy.spatial import cKDTree

    scene = synth.small_scene("clustered", 5000, seed=41, sh_deg=0)
    rng = np.random.default_rng(42)
    q = np.concatenate([rng.uniform(-1.2, 1.2, size=(3000, 3)), scene.sites[:50].astype(np.float64),
                        rng.standard_normal((200, 3)) * 10.0])
    idx, gap = oracle.nearest_site(scene.sites, q, return_gap=True)
    dist, ref = cKDTree(scene.sites.astype(np.float64)).query(q, k=1)
    clear = gap > 1e-9
    assert clear.mean() > 0.99
    np.testing.assert_array_equal(idx[clear], ref[clear])
    mine = np.linalg.norm(q - scene.sites[idx].astype(np.float64), axis=1)
    np.testing.assert_allclose(mine, dist, rtol=1e-12, atol=0)
    np.testing.assert_array_equal(idx[3000:3050], np.arange(50))


# ---------------------------------------------------------------------------
# quantile regulariser (Sec. 3.4, training objectives)
# ---------------------------------------------------------------------------

def test_quantile_homogeneous_medium_closed_form(uniform_scene):
    # constant sigma along the whole ray: tau(t) = sigma t, so the normalised
    # CDF is (1 - e^{-sigma t}) / (1 - e^{-sigma t_max}) and its inverse is
    # -ln(1 - u (1 - e^{-sigma t_max})) / sigma
    sc = uniform_scene
    rng = np.random.default_rng(31)
    o, d, tmax, start = random_inside_rays(rng, 150, 0.0, 1.0, sc.sites)
    sig = 2.3
    osc = hand_scene(sc.sites, 0, density=sig, colour=[0.5, 0.5, 0.5])
    u = rng.uniform(size=(150, 2))
    u[:5] = [[0.0, 1.0], [1.0, 0.0], [0.5, 0.5], [0.25, 0.75], [1e-9, 1 - 1e-9]]
    tq, loss = oracle.quantile(osc, o, d, tmax, start, u, eps=0.0)
    ref = -np.log1p(-u * (1.0 - np.exp(-sig * tmax))[:, None]) / sig
    np.testing.assert_allclose(tq, ref, rtol=1e-10, atol=1e-12)
    np.testing.assert_allclose(loss, np.abs(ref[:, 0] - ref[:, 1]), rtol=1e-10, atol=1e-12)
    np.testing.assert_allclose(tq[0], [0.0, tmax[0]], atol=1e-12)  # u = 0 and u = 1: the ends of the support
    assert loss[2] == 0.0


def test_quantile_inverts_the_weight_cdf_by_bisection(clustered_scene):
    # W(t) = 1 - exp(-tau(t)), tau(t) summed over the traced segments with the
    # scene's densities; bisection on W(t) = u W(end) must land on the oracle's quantile
    sc = clustered_scene
    rng = np.random.default_rng(32)
    o, d, tmax, start = random_inside_rays(rng, 40, -0.9, 0.9, sc.sites)
    osc = oracle.OracleScene.from_scene(sc)
    u = rng.uniform(size=(40, 2))
    tq, loss = oracle.quantile(osc, o, d, tmax, start, u, eps=1e-3)
    tr = oracle.trace(osc, o, d, tmax, start, eps=1e-3, max_len=512)
    dens = sc.density.astype(np.float64)
    for r in range(40):
        L = tr["len"][r]
        cells, te = tr["cells"][r, :L], tr["t_exit"][r, :L]
        t0 = np.concatenate([[0.0], te[:-1]])

        def W(t):
            return 1.0 - np.exp(-(dens[cells] * np.clip(np.minimum(te, t) - t0, 0, None)).sum())

        total = W(te[-1])
        for q in range(2):
            lo, hi = 0.0, te[-1]
            for _ in range(200):
                mid = 0.5 * (lo + hi)
                lo, hi = (mid, hi) if W(mid) < u[r, q] * total else (lo, mid)
            assert abs(tq[r, q] - hi) <= 1e-9 * max(1.0, te[-1]), (r, q, tq[r, q], hi)


def test_quantile_scale_invariance(clustered_scene):
    sc = clustered_scene
    rng = np.random.default_rng(33)
    o, d, tmax, start = random_inside_rays(rng, 60, -0.9, 0.9, sc.sites)
    u = rng.uniform(size=(60, 2))
    osc = oracle.OracleScene.from_scene(sc)
    tq, loss = oracle.quantile(osc, o, d, tmax, start, u, eps=1e-3)
    s = 4.0
    osc2 = oracle.OracleScene(sc.sites.astype(np.float64) * s, sc.off, sc.idx, sc.density.astype(np.float64) / s,
                              sc.sh, sc.sh_deg)
    tq2, loss2 = oracle.quantile(osc2, o * s, d, tmax * s, start, u, eps=1e-3)
    np.testing.assert_allclose(tq2, s * tq, rtol=1e-9, atol=1e-12)


@pytest.mark.parametrize("eps", [0.0, 1e-2])
def test_quantile_gradients_match_finite_differences(eps):
    sc = synth.small_scene("uniform11", 120, seed=34, sh_deg=0)
    rng = np.random.default_rng(35)
    o, d, tmax, start = random_inside_rays(rng, 60, -0.9, 0.9, sc.sites)
    dens = sc.density.astype(np.float64) * (4.0 if eps else 1.0)
    osc = oracle.OracleScene(sc.sites, sc.off, sc.idx, dens, sc.sh, 0)
    tr = oracle.trace(osc, o, d, tmax, start, eps=eps)
    keep = (tr["margin"] > 1e-4) & (tr["graze"] > 1e-4) & ((tr["term"] > 1e-2) | (eps == 0))
    o, d, tmax, start = o[keep], d[keep], tmax[keep], start[keep]
    u = rng.uniform(0.05, 0.95, size=(len(d), 2))
    g = rng.standard_normal(len(d))
    tq, loss, gs, gd = oracle.quantile(osc, o, d, tmax, start, u, g, eps=eps, threads=1)
    assert len(d) >= 30 and np.all(tq[:, 0] != tq[:, 1])
    sites = sc.sites.astype(np.float64)

    def L(sites_=sites, dens_=dens):
        s = oracle.OracleScene(sites_, sc.off, sc.idx, dens_, sc.sh, 0)
        return (oracle.quantile(s, o, d, tmax, start, u, eps=eps, threads=1)[1] * g).sum()

    h = 1e-6
    touched = np.unique(np.concatenate([tr["cells"][keep][r, :tr["len"][keep][r]] for r in range(len(d))]))
    rng2 = np.random.default_rng(36)
    for i in rng2.choice(touched, size=min(25, len(touched)), replace=False):
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
        assert abs(fd - gd[i]) <= 1e-5 * max(1.0, abs(fd)), (i, fd, gd[i])
    untouched = np.setdiff1d(np.arange(sc.n_sites), touched)
    assert np.all(gd[untouched] == 0)
    # a walk that ends on the transmittance test still has a moving last exit,
    # so the site of the cell behind it (never visited) gets a gradient too
    beyond = untouched[np.abs(gs[untouched]).max(axis=1) > 0]
    assert eps > 0 or len(beyond) == 0
    for i in beyond[:10]:
        for a in range(3):
            sp, sm = sites.copy(), sites.copy()
            sp[i, a] += h
            sm[i, a] -= h
            fd = (L(sites_=sp) - L(sites_=sm)) / (2 * h)
            assert abs(fd - gs[i, a]) <= 1e-5 * max(1.0, abs(fd)), (i, a, fd, gs[i, a])
