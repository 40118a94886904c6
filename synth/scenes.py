"""Seeded synthetic scenes, cameras and request streams.

The workloads follow the shapes of the paper's experiments (Sec. 4): dense
site clouds concentrated on surface-like sheets with a sparse background,
per-cell density and degree-3 spherical-harmonic colour (Sec. 3.4), pinhole
cameras looking into the scene. The paper's datasets (Mip-NeRF 360, Deep
Blending) are not available; these seeded scenes stand in for them.

Conventions
-----------
* ``numpy.random.default_rng(seed)``; draws happen in the order sites,
  density, SH coefficients, cameras, upstream gradients.
* "N(0, s)" means standard deviation ``s``; density is lognormal(0, 1).
* Sites are generated in float64, rounded to float32 (the width the walk
  stores), and the Delaunay adjacency is built on the rounded coordinates so
  that the CSR describes exactly the tessellation of the stored sites.
* Each CSR row is sorted ascending (ties between equal exit distances are
  broken by CSR order, i.e. lowest neighbour id first).
* Cameras use the pinhole model with a 60 degree horizontal field of view and
  the rotation's columns are (right, down, forward).
"""

from __future__ import annotations

import dataclasses
import hashlib
import os
from typing import Dict, List, Optional, Tuple

import numpy as np

# ----------------------------------------------------------------------------
# Workload table
# ----------------------------------------------------------------------------

#: The five workloads. ``kind`` selects the site distribution; ``bound`` is
#: the region whose boundary ends each camera ray (``t_max``).
CONFIGS: Dict[str, dict] = {
    "uniform_4k": dict(n_sites=4096, kind="uniform01", sh_deg=0, sh_std=0.5,
                 res=[(64, 64)], n_cams=1, camera="cube_centre",
                 bound=("box", 0.0, 1.0), backward=False, seed=1),
    "clustered_200k": dict(n_sites=200_000, kind="clustered", sh_deg=3, sh_std=0.3,
                 res=[(800, 800)], n_cams=1, camera="orbit",
                 bound=("box", -1.0, 1.0), backward=True, seed=2),
    "clustered_1m": dict(n_sites=1_000_000, kind="clustered", sh_deg=3, sh_std=0.3,
                 res=[(1920, 1080)], n_cams=1, camera="orbit",
                 bound=("box", -1.0, 1.0), backward=True, seed=3),
    "shell_3m": dict(n_sites=3_000_000, kind="clustered_shell", sh_deg=3, sh_std=0.3,
                 res=[(1600, 1066)], n_cams=8, camera="inside",
                 bound=("sphere", 5.0), backward=True, seed=4),
    "serving_1m": dict(n_sites=1_000_000, kind="clustered", sh_deg=3, sh_std=0.3,
                 res=[(256, 256), (512, 512), (1024, 1024), (1920, 1080)],
                 n_cams=512, camera="inside", bound=("box", -1.0, 1.0),
                 backward=False, seed=5, rate_hz=200.0),
}

FOV_DEG = 60.0
ORBIT_RADIUS = 0.8
N_CLUSTERS = 64
CLUSTER_STD = (0.15, 0.15, 0.01)
MIN_SEPARATION = 1e-7


@dataclasses.dataclass
class Scene:
    """A Voronoi scene: sites, Delaunay neighbour CSR and per-cell attributes."""

    name: str
    sites: np.ndarray      # float32 [N, 3]
    off: np.ndarray        # int32 [N + 1]
    idx: np.ndarray        # int32 [E]
    density: np.ndarray    # float32 [N], >= 0
    sh: np.ndarray         # float32 [N, B, 3], B = (deg + 1) ** 2
    sh_deg: int
    bound: tuple           # ("box", lo, hi) or ("sphere", radius)

    @property
    def n_sites(self) -> int:
        return int(self.sites.shape[0])

    @property
    def n_edges(self) -> int:
        return int(self.idx.shape[0])


@dataclasses.dataclass
class Camera:
    """Pinhole camera: world position, rotation (columns right, down, forward)."""

    position: np.ndarray   # float64 [3]
    rotation: np.ndarray   # float64 [3, 3]
    width: int
    height: int
    fov_deg: float = FOV_DEG

    def pose12(self) -> np.ndarray:
        """Row-major 3x4 [R | p] as float64[12]."""
        return np.concatenate([np.hstack([self.rotation, self.position[:, None]]).ravel()])


# ----------------------------------------------------------------------------
# Sites
# ----------------------------------------------------------------------------

def _random_rotation(rng: np.random.Generator) -> np.ndarray:
    q, r = np.linalg.qr(rng.standard_normal((3, 3)))
    q = q * np.sign(np.diag(r))[None, :]
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    return q


def _clustered(rng: np.random.Generator, n: int, lo: float = -1.0, hi: float = 1.0) -> np.ndarray:
    """90 % from 64 thin anisotropic Gaussians, 10 % uniform, all inside [lo, hi]^3."""
    n_bg = n // 10
    n_cl = n - n_bg
    means = rng.uniform(-0.8, 0.8, size=(N_CLUSTERS, 3))
    rots = np.stack([_random_rotation(rng) for _ in range(N_CLUSTERS)])
    std = np.asarray(CLUSTER_STD)
    out = np.empty((n_cl, 3))
    filled = 0
    while filled < n_cl:
        m = n_cl - filled
        comp = rng.integers(0, N_CLUSTERS, size=m)
        z = rng.standard_normal((m, 3)) * std
        p = means[comp] + np.einsum("nij,nj->ni", rots[comp], z)
        keep = np.all((p > lo) & (p < hi), axis=1)
        p = p[keep]
        out[filled:filled + len(p)] = p
        filled += len(p)
    bg = rng.uniform(lo, hi, size=(n_bg, 3))
    pts = np.concatenate([out, bg])
    return pts[rng.permutation(len(pts))]


def _shell(rng: np.random.Generator, n: int) -> np.ndarray:
    """Uniform directions, radius uniform in [3.8, 4.2] (never exactly co-spherical)."""
    v = rng.standard_normal((n, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    r = rng.uniform(3.8, 4.2, size=(n, 1))
    return v * r


def _make_sites(kind: str, n: int, rng: np.random.Generator) -> np.ndarray:
    if kind == "uniform01":
        return rng.uniform(0.0, 1.0, size=(n, 3))
    if kind == "uniform11":
        return rng.uniform(-1.0, 1.0, size=(n, 3))
    if kind == "clustered":
        return _clustered(rng, n)
    if kind == "clustered_shell":
        n_shell = n // 20
        return np.concatenate([_clustered(rng, n - n_shell), _shell(rng, n_shell)])
    raise ValueError(f"unknown site distribution {kind!r}")


def _dedupe_f32(pts: np.ndarray, rng: np.random.Generator, kind: str) -> np.ndarray:
    """Round to float32 and redraw any site within MIN_SEPARATION of another."""
    from scipy.spatial import cKDTree

    pts = pts.astype(np.float32)
    for _ in range(10):
        pairs = cKDTree(pts.astype(np.float64)).query_pairs(MIN_SEPARATION, output_type="ndarray")
        if len(pairs) == 0:
            return pts
        bad = np.unique(pairs[:, 1])
        pts[bad] = _make_sites(kind, len(bad), rng).astype(np.float32)
    raise RuntimeError("could not separate near-duplicate sites")


# ----------------------------------------------------------------------------
# Delaunay adjacency (the CPU builder)
# ----------------------------------------------------------------------------

def build_adjacency(sites: np.ndarray) -> Tuple[np.ndarray, np.ndarray]:
    """Delaunay neighbour CSR of float32 sites via Qhull; rows sorted ascending.

    Raises if Qhull drops any input point (near-duplicates / degeneracy).
    """
    from scipy.spatial import Delaunay

    tri = Delaunay(sites.astype(np.float64))
    if len(tri.coplanar):
        raise RuntimeError(f"Qhull dropped {len(tri.coplanar)} points")
    indptr, indices = tri.vertex_neighbor_vertices
    n = sites.shape[0]
    rows = np.repeat(np.arange(n, dtype=np.int64), np.diff(indptr))
    # one sort of row * n + neighbour orders every row ascending
    idx = (np.sort(rows * n + indices) % n).astype(np.int32)
    off = indptr.astype(np.int32)
    return off, idx


# ----------------------------------------------------------------------------
# Scenes
# ----------------------------------------------------------------------------

def _cache_path(key: str) -> Optional[str]:
    d = os.environ.get("RF_SCENE_CACHE")
    if not d:
        return None
    os.makedirs(d, exist_ok=True)
    return os.path.join(d, key + ".npz")


def _assemble(name: str, sites: np.ndarray, rng: np.random.Generator, sh_deg: int,
              sh_std: float, bound: tuple) -> Scene:
    off, idx = build_adjacency(sites)
    n = sites.shape[0]
    density = rng.lognormal(mean=0.0, sigma=1.0, size=n).astype(np.float32)
    b = (sh_deg + 1) ** 2
    sh = (rng.standard_normal((n, b, 3)) * sh_std).astype(np.float32)
    return Scene(name, sites, off, idx, density, sh, sh_deg, bound)


def make_scene(name: str, seed: Optional[int] = None, n_sites: Optional[int] = None,
               return_rng: bool = False):
    """Scene for workload ``name`` ("uniform_4k" ... "serving_1m").

    ``n_sites`` overrides the site count (same distribution, for scaled-down
    tests). The generator is left positioned after the SH draw so that the
    caller can continue with cameras and gradients (``return_rng=True``).
    """
    cfg = CONFIGS[name]
    seed = cfg["seed"] if seed is None else seed
    n = cfg["n_sites"] if n_sites is None else int(n_sites)
    key = f"scene_v1_{name}_{seed}_{n}"
    path = _cache_path(key)
    rng = np.random.default_rng(seed)
    if path and os.path.exists(path):
        z = np.load(path)
        scene = Scene(name, z["sites"], z["off"], z["idx"], z["density"], z["sh"],
                      int(z["sh_deg"]), cfg["bound"])
        rng.bit_generator.state = _state_from_array(z["rng_state"])
    else:
        sites = _dedupe_f32(_make_sites(cfg["kind"], n, rng), rng, cfg["kind"])
        scene = _assemble(name, sites, rng, cfg["sh_deg"], cfg["sh_std"], cfg["bound"])
        if path:
            np.savez(path, sites=scene.sites, off=scene.off, idx=scene.idx,
                     density=scene.density, sh=scene.sh, sh_deg=scene.sh_deg,
                     rng_state=_state_to_array(rng.bit_generator.state))
    return (scene, rng) if return_rng else scene


def small_scene(kind: str, n: int, seed: int, sh_deg: int = 3, sh_std: float = 0.3,
                bound: Optional[tuple] = None, return_rng: bool = False):
    """Scaled-down scene of a given site distribution (for oracle and parity tests)."""
    rng = np.random.default_rng(seed)
    sites = _dedupe_f32(_make_sites(kind, n, rng), rng, kind)
    if bound is None:
        bound = ("box", 0.0, 1.0) if kind == "uniform01" else ("box", -1.0, 1.0)
    scene = _assemble(f"{kind}{n}", sites, rng, sh_deg, sh_std, bound)
    return (scene, rng) if return_rng else scene


def _state_to_array(state: dict) -> np.ndarray:
    s = state["state"]
    return np.array([s["state"], s["inc"], state["has_uint32"], state["uinteger"]], dtype=object).astype(str)


def _state_from_array(a: np.ndarray) -> dict:
    return {"bit_generator": "PCG64", "state": {"state": int(a[0]), "inc": int(a[1])},
            "has_uint32": int(a[2]), "uinteger": int(a[3])}


# ----------------------------------------------------------------------------
# Cameras, start cells, upstream gradients
# ----------------------------------------------------------------------------

def _look_rotation(forward: np.ndarray) -> np.ndarray:
    f = forward / np.linalg.norm(forward)
    up = np.array([0.0, 0.0, 1.0]) if abs(f[2]) < 0.99 else np.array([1.0, 0.0, 0.0])
    right = np.cross(f, up)
    right /= np.linalg.norm(right)
    down = np.cross(f, right)
    return np.stack([right, down, f], axis=1)


def _random_direction(rng: np.random.Generator) -> np.ndarray:
    v = rng.standard_normal(3)
    return v / np.linalg.norm(v)


def make_cameras(name: str, rng: np.random.Generator, n: Optional[int] = None,
                 res: Optional[Tuple[int, int]] = None) -> List[Camera]:
    """Cameras of workload ``name``; ``res`` overrides (W, H) for scaled tests."""
    cfg = CONFIGS[name]
    n = cfg["n_cams"] if n is None else n
    cams = []
    for _ in range(n):
        w, h = res if res is not None else cfg["res"][rng.integers(len(cfg["res"]))] \
            if len(cfg["res"]) > 1 else cfg["res"][0]
        if cfg["camera"] == "cube_centre":
            pos = np.array([0.5, 0.5, 0.5])
            rot = _look_rotation(np.array([1.0, 0.0, 0.0]))
        elif cfg["camera"] == "orbit":
            phi = rng.uniform(0.0, 2.0 * np.pi)
            pos = ORBIT_RADIUS * np.array([np.cos(phi), np.sin(phi), 0.0])
            rot = _look_rotation(-pos)
        elif cfg["camera"] == "inside":
            pos = rng.uniform(-0.8, 0.8, size=3)
            rot = _look_rotation(_random_direction(rng))
        else:
            raise ValueError(cfg["camera"])
        cams.append(Camera(pos.astype(np.float32).astype(np.float64), rot, int(w), int(h)))
    return cams


def nearest_site(sites: np.ndarray, points: np.ndarray) -> np.ndarray:
    """Index of the nearest site (KD-tree), lowest index on exact ties."""
    from scipy.spatial import cKDTree

    tree = cKDTree(sites.astype(np.float64))
    pts = np.atleast_2d(np.asarray(points, dtype=np.float64))
    _, i = tree.query(pts, k=1)
    return np.asarray(i, dtype=np.int32)


def make_upstream_grads(rng: np.random.Generator, n_rays: int) -> np.ndarray:
    """Per-ray, per-channel upstream colour gradients, N(0, 1), float32 [R, 3]."""
    return rng.standard_normal((n_rays, 3)).astype(np.float32)


def make_serving_requests(rng: np.random.Generator, n: int = 512, rate_hz: float = 200.0,
                          sizes=None) -> List[dict]:
    """Poisson arrival stream of render requests (arrival time in seconds, camera)."""
    sizes = sizes or CONFIGS["serving_1m"]["res"]
    t = np.cumsum(rng.exponential(1.0 / rate_hz, size=n))
    reqs = []
    for k in range(n):
        w, h = sizes[rng.integers(len(sizes))]
        pos = rng.uniform(-0.8, 0.8, size=3)
        rot = _look_rotation(_random_direction(rng))
        reqs.append(dict(arrival=float(t[k]),
                         camera=Camera(pos.astype(np.float32).astype(np.float64), rot, int(w), int(h))))
    return reqs


def scene_digest(scene: Scene) -> str:
    h = hashlib.sha1()
    for a in (scene.sites, scene.off, scene.idx, scene.density, scene.sh):
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()[:16]
