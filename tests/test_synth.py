"""Input generators: determinism, CSR structure and Poisson-Voronoi statistics."""

import numpy as np
import pytest

import synth


def test_scene_is_seeded_and_csr_sorted_symmetric():
    a = synth.small_scene("clustered", 3000, seed=3)
    b = synth.small_scene("clustered", 3000, seed=3)
    for k in ("sites", "off", "idx", "density", "sh"):
        np.testing.assert_array_equal(getattr(a, k), getattr(b, k))
    assert a.sites.dtype == np.float32 and a.idx.dtype == np.int32 and a.off.dtype == np.int32
    rows = np.repeat(np.arange(a.n_sites), np.diff(a.off))
    assert np.all(a.idx != rows)
    for i in range(0, a.n_sites, 97):
        r = a.idx[a.off[i]:a.off[i + 1]]
        assert np.all(np.diff(r) > 0)
    fwd = set(zip(rows.tolist(), a.idx.tolist()))
    assert all((j, i) in fwd for (i, j) in list(fwd)[:5000])
    assert np.all(a.density > 0)
    assert np.all(np.abs(a.sites) < 1)


def test_interior_mean_degree_matches_poisson_voronoi():
    """Mean number of faces of a Poisson-Voronoi cell: 2 + 48 pi^2 / 35 = 15.535."""
    sc = synth.small_scene("uniform01", 40000, seed=4, sh_deg=0)
    deg = np.diff(sc.off)
    inner = np.all((sc.sites > 0.2) & (sc.sites < 0.8), axis=1)
    assert abs(deg[inner].mean() - (2 + 48 * np.pi ** 2 / 35)) < 0.08


def test_cameras_and_requests():
    rng = np.random.default_rng(0)
    cams = synth.make_cameras("clustered_1m", rng)
    assert len(cams) == 1 and (cams[0].width, cams[0].height) == (1920, 1080)
    np.testing.assert_allclose(np.linalg.norm(cams[0].position), 0.8, rtol=1e-6)
    R = cams[0].rotation
    np.testing.assert_allclose(R.T @ R, np.eye(3), atol=1e-12)
    assert np.linalg.det(R) > 0
    fwd = R[:, 2]
    np.testing.assert_allclose(fwd, -cams[0].position / np.linalg.norm(cams[0].position), atol=1e-6)
    reqs = synth.make_serving_requests(np.random.default_rng(1), n=512)
    t = np.array([r["arrival"] for r in reqs])
    assert np.all(np.diff(t) > 0)
    assert abs(512 / t[-1] - 200) < 30
    sizes = {(r["camera"].width, r["camera"].height) for r in reqs}
    assert sizes == {(256, 256), (512, 512), (1024, 1024), (1920, 1080)}
    assert all(np.all(np.abs(r["camera"].position) <= 0.8) for r in reqs)
