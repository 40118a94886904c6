"""Pins of the oracle's forced walks and near-tie alternatives.

A near tie is a decision of Algorithm 1 that a computation in FP32 may take
either way: two exit faces at almost the same distance (a ray through a
Voronoi edge), an exit face at almost t_max, or a transmittance almost at
eps. The oracle lists each such decision with its alternative choices and
walks a ray with given choices (``walk_forced``); ``alternatives`` enumerates
every walk over the near ties. The pins: an unforced walk is the plain walk;
at an exact tie each alternative is the limit of the plain walk of a ray
moved to one side of the Voronoi edge (sequence, colour and gradient);
forced stops composite exactly the first segments of the plain walk; and in
a homogeneous medium every combination of choices keeps the closed form.
"""

import numpy as np
import pytest

import oracle
import synth


def unit(v):
    v = np.asarray(v, dtype=np.float64)
    return v / np.linalg.norm(v, axis=-1, keepdims=True)


def edge_scene(density=None, sh_deg=1):
    """Sites 0 (origin), 1 = (1, 0.6, 0) and 2 = (1, -0.6, 0): the Voronoi edge
    of the three is the line x = 0.68, y = 0; a cloud of far sites bounds the cells."""
    rng = np.random.default_rng(3)
    far = unit(rng.standard_normal((60, 3))) * rng.uniform(3.0, 4.0, (60, 1))
    sites = np.concatenate([[[0, 0, 0], [1, 0.6, 0], [1, -0.6, 0]], far]).astype(np.float32)
    off, idx = synth.build_adjacency(sites)
    n = len(sites)
    b = (sh_deg + 1) ** 2
    dens = rng.uniform(0.5, 2.0, n) if density is None else np.full(n, density)
    sh = rng.normal(0, 0.5, (n, b, 3))
    return oracle.OracleScene(sites, off, idx, dens, sh, sh_deg)


def edge_ray(dy=0.0):
    """A ray in the plane z = 0.1 through the point (x_e, dy, 0.1), crossing the
    edge line at dy = 0; x_e = (1 + 0.6^2)/2 with the sites' FP32 value of 0.6."""
    y1 = float(np.float32(0.6))
    p = np.array([(1.0 + y1 * y1) / 2.0, dy, 0.1])
    o = np.array([0.05, 0.3, 0.1])
    d = unit(p - o)
    return o[None], d[None], np.array([2.5]), np.array([0], dtype=np.int32)


def test_unforced_walk_is_the_plain_walk():
    scene = synth.small_scene("clustered", 500, seed=12, sh_deg=3)
    osc = oracle.OracleScene.from_scene(scene)
    rng = np.random.default_rng(5)
    o = rng.uniform(-0.8, 0.8, (200, 3))
    d = unit(rng.standard_normal((200, 3)))
    t = np.full(200, 1.5)
    s = synth.nearest_site(scene.sites, o).astype(np.int32)
    tr = oracle.trace(osc, o, d, t, s, eps=1e-4, max_len=256)
    w = oracle.walk_forced(osc, o, d, t, s, np.arange(200), [[] for _ in range(200)], eps=1e-4, max_len=256)
    np.testing.assert_array_equal(w["rgb"], tr["rgb"])
    np.testing.assert_array_equal(w["t_final"], tr["t_final"])
    np.testing.assert_array_equal(w["len"], tr["len"])
    np.testing.assert_array_equal(w["cells"], tr["cells"])
    assert not w["bad"].any()


def test_exact_tie_alternatives_are_the_one_sided_limits():
    osc = edge_scene()
    o, d, t, s = edge_ray(0.0)
    alt = oracle.alternatives(osc, o, d, t, s, [0], kappa_t=1e-9, kappa_T=0.0, eps=0.0)
    leaves = alt["leaves"][0]
    assert alt["complete"][0]
    seqs = {tuple(lf["cells"][:3].tolist()) for lf in leaves}
    # through the edge: leave cell 0 into 1 (then a zero-length sliver of 1 into 2) or straight into 2
    assert (0, 1, 2) in seqs and any(q[:2] == (0, 2) for q in seqs), seqs
    # the slivers have zero length: every alternative has the same colour
    for lf in leaves[1:]:
        np.testing.assert_allclose(lf["rgb"], leaves[0]["rgb"], rtol=0, atol=1e-12)
    # moved to either side of the edge, the plain walk takes one of the alternatives, and its
    # colour and gradients tend to that alternative's
    g = np.array([[0.3, -1.2, 0.7]])
    for dy in (1e-7, -1e-7):
        od, dd, td, sd = edge_ray(dy)
        tr = oracle.trace(osc, od, dd, td, sd, eps=0.0, max_len=64)
        seq = tr["cells"][0, :tr["len"][0]]
        seq = seq[[0] + [k for k in range(1, len(seq)) if seq[k] != seq[k - 1]]]
        match = [lf for lf in leaves if np.array_equal(lf["cells"][:lf["len"]][:len(seq)], seq)
                 or np.array_equal(np.array([c for c in lf["cells"][:lf["len"]] if c != 1 or seq[1] == 1])[:len(seq)],
                                   seq)]
        assert match, (dy, seq, [lf["cells"][:lf["len"]] for lf in leaves])
        np.testing.assert_allclose(tr["rgb"][0], leaves[0]["rgb"], atol=1e-5)
        side = [lf for lf in leaves if lf["cells"][1] == seq[1]]
        assert side
        if seq[1] == 1:
            # this side crosses a sliver of cell 1 whose exit moves, while at the tie the
            # sliver has zero length and its exit is clamped (no gradient through it):
            # the gradient is one-sided there, several answers are correct
            continue
        # the side that enters cell 2 directly: the forced walk's gradient is the limit
        gf = oracle.backward(osc, o, d, t, s, g, eps=0.0, forced=[side[0]["forced"]])
        gp = oracle.backward(osc, od, dd, td, sd, g, eps=0.0)
        for a, b in zip(gf, gp):
            np.testing.assert_allclose(a, b, rtol=0, atol=2e-4 * max(np.abs(b).max(), 1e-12))


def test_forced_stop_composites_the_first_segments():
    scene = synth.small_scene("clustered", 500, seed=12, sh_deg=3)
    osc = oracle.OracleScene.from_scene(scene)
    rng = np.random.default_rng(8)
    o = rng.uniform(-0.5, 0.5, (20, 3))
    d = unit(rng.standard_normal((20, 3)))
    t = np.full(20, 1.5)
    s = synth.nearest_site(scene.sites, o).astype(np.int32)
    tr = oracle.trace(osc, o, d, t, s, eps=0.0, max_len=512)
    Y = oracle.sh_basis(3, d)
    for r in range(20):
        L = int(tr["len"][r])
        if L < 4:
            continue
        n = L // 2
        w = oracle.walk_forced(osc, o, d, t, s, [r], [[(n, oracle.CH_STOP)]], eps=0.0, max_len=512)
        assert w["len"][0] == n and w["steps"][0] == n
        # composite the first n traced segments by hand (eq. (3)-(4), exclusive transmittance)
        C, T, t0 = np.zeros(3), 1.0, 0.0
        for k in range(n):
            cell = tr["cells"][r, k]
            te = tr["t_exit"][r, k]
            tau = osc.density[cell] * (te - t0)
            c = (osc.sh[cell] * Y[r][:, None]).sum(0)
            C += T * (1 - np.exp(-tau)) * c
            T *= np.exp(-tau)
            t0 = te
        np.testing.assert_allclose(w["rgb"][0], C, rtol=1e-12, atol=1e-14)
        np.testing.assert_allclose(w["t_final"][0], T, rtol=1e-12)
        # and a forced pass of a failed test continues: with eps above T_n the walk
        # would stop at n, forcing GO there resumes the eps = 0 walk
        eps = T * 1.0000001
        w2 = oracle.walk_forced(osc, o, d, t, s, [r], [[(n, oracle.CH_GO)]], eps=eps, max_len=512)
        plain = oracle.trace(osc, o[r:r + 1], d[r:r + 1], t[r:r + 1], s[r:r + 1], eps=eps, max_len=512)
        assert plain["len"][0] == n
        assert w2["len"][0] > n
        np.testing.assert_array_equal(w2["cells"][0, :n + 1], tr["cells"][r, :n + 1])


def test_homogeneous_medium_keeps_the_closed_form_under_any_choices():
    scene = synth.small_scene("uniform01", 400, seed=11, sh_deg=0)
    n = scene.n_sites
    sig, col = 1.7, np.array([0.2, -0.4, 0.9])
    sh = np.broadcast_to(col / 0.28209479177387814, (n, 1, 3))
    osc = oracle.OracleScene(scene.sites, scene.off, scene.idx, np.full(n, sig), sh, 0)
    rng = np.random.default_rng(9)
    o = rng.uniform(0.2, 0.8, (60, 3))
    d = unit(rng.standard_normal((60, 3)))
    t = rng.uniform(0.2, 0.6, 60)
    s = synth.nearest_site(scene.sites, o).astype(np.int32)
    # a generous kappa turns many decisions into "near ties", so many choices are exercised
    alt = oracle.alternatives(osc, o, d, t, s, np.arange(60), kappa_t=3e-2, kappa_T=0.0, eps=0.0, max_leaves=8)
    n_alt = 0
    for r in range(60):
        ref = col * (1 - np.exp(-sig * t[r]))
        for lf in alt["leaves"][r]:
            np.testing.assert_allclose(lf["rgb"], ref, rtol=1e-11, atol=1e-13)
            np.testing.assert_allclose(lf["t_final"], np.exp(-sig * t[r]), rtol=1e-11)
            n_alt += bool(lf["forced"])
    assert n_alt > 30
