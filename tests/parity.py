"""Shared helpers of the GPU parity tests: seeded cases, decidability, near ties, tolerances.

The oracle runs in FP64 on exactly the FP32 inputs the GPU sees. The GPU takes
each face decision in FP32 (its exit distances are formed in double), so it
can take a decision differently from the oracle only where the exact winner's
margin lies within FP32 error. The tolerances:

* decidable rays: every decision of the oracle's walk clears KAPPA_T (the gap
  between the winning face and any other front face or t_max, in units of the
  exit distances' FP32 error scale (1 + |o| + |t|)(1/cos_1 + 1/cos_j)), KAPPA_G
  (|cos| of any non-front face) and KAPPA_TERM (|ln T - ln eps| at every
  transmittance test). An FP32 exit distance carries an absolute error of a
  few eps32 (|o| + t) / cos, so gaps below ~6 eps32 = 3.6e-7 in these units can
  legitimately flip; KAPPA_T sits at that scale. A decidable ray's visited
  cells must equal the oracle's exactly.
* near-tie rays (not decidable): the oracle lists every walk that takes, at
  each near tie, the exact winner or a near alternative (``oracle.alternatives``);
  the GPU's visited cells must equal one of them exactly, and its colour,
  transmittance and visit count are compared with that walk's. A ray with too
  many such walks (or a near-grazing face, KAPPA_G) is left unresolved and
  counted.
* colour, per element on every resolved ray:
  |c - c_ref| <= COLOUR_RTOL * max(|c_ref|, mean |C_ref|), the mean over the
  batch (a composited sum's error scales with the cells' colours, and a pixel's
  colour can cancel to ~0);
* final transmittance: |T - T_ref| <= T_ATOL (T lies in [0, 1]);
* exit distances of decidable rays: |t - t_ref| <= T_EXIT_ATOL + 1e-4 |t_ref|;
* gradients, per tensor max|g - g_ref| <= GRAD_RTOL * max|g_ref| and per
  element |g - g_ref| <= GRAD_RTOL |g_ref| + GRAD_ATOL_REL * max|g_ref|, from
  the rays that are decidable and whose moving exits are all at least KAPPA_X
  away from grazing (|cos| of the exit face, oracle's exit_cos); the others get
  zero upstream gradient on both sides. Near a tie several gradients are
  correct (a sliver's exit may be clamped or move). A site-gradient term is
  (dL/dt) (p - x) / (n.d); the FP32 packed normal puts a relative error of
  ~eps32 |p - m| / cos on the exit point, and that term is its ray's largest.
"""

from __future__ import annotations

import numpy as np

import oracle
import synth

KAPPA_T = 3e-7
KAPPA_G = 1e-6
KAPPA_TERM = 1e-4
COLOUR_RTOL = 1e-4
T_ATOL = 1e-4
T_EXIT_ATOL = 1e-4
GRAD_RTOL = 1e-4
GRAD_ATOL_REL = 1e-6
KAPPA_X = 1e-2


def camera_rays(scene, cam, threads=None):
    """Rays of a camera from the oracle's FP64 ray generation, rounded to FP32 inputs."""
    o, d, t, pix = oracle.raygen(cam.pose12(), cam.fov_deg, cam.width, cam.height, scene.bound)
    start = int(synth.nearest_site(scene.sites, o[:1])[0])
    return (o.astype(np.float32), d.astype(np.float32), t.astype(np.float32),
            np.full(len(t), start, dtype=np.int32), pix)


def inside_rays(scene, rng, n, lo, hi):
    """Rays from random points inside [lo, hi]^3 in random directions, to the box boundary."""
    o = rng.uniform(lo, hi, size=(n, 3)).astype(np.float32)
    d = rng.standard_normal((n, 3))
    d = (d / np.linalg.norm(d, axis=1, keepdims=True)).astype(np.float32)
    od, dd = o.astype(np.float64), d.astype(np.float64)
    with np.errstate(divide="ignore"):
        t_hi = np.where(dd > 0, (hi - od) / dd, np.inf)
        t_lo = np.where(dd < 0, (lo - od) / dd, np.inf)
    tmax = np.minimum(t_hi, t_lo).min(axis=1).astype(np.float32)
    start = synth.nearest_site(scene.sites, o).astype(np.int32)
    return o, d, tmax, start


def decidable(tr: dict, eps: float) -> np.ndarray:
    ok = (tr["margin"] > KAPPA_T) & (tr["graze"] > KAPPA_G)
    if eps > 0:
        ok &= tr["term"] > KAPPA_TERM
    return ok


def gradient_decidable(tr: dict, eps: float) -> np.ndarray:
    """Rays whose gradients are compared: decidable, and no moving exit within KAPPA_X of grazing."""
    return decidable(tr, eps) & (tr["exit_cos"] > KAPPA_X)


def colour_err(x, ref) -> float:
    """max |x - ref| / max |ref| over the batch."""
    x = np.asarray(x, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    if x.size == 0:
        return 0.0
    return float(np.abs(x - ref).max() / max(np.abs(ref).max(), 1e-30))


def colour_ratio(x, ref, mean_abs=None) -> np.ndarray:
    """Per ray, max over channels of |x - ref| / (COLOUR_RTOL max(|ref|, mean |C_ref|)); <= 1 passes.
    ``mean_abs``: the batch's mean |C_ref| (default: over ``ref``)."""
    x = np.asarray(x, dtype=np.float64).reshape(-1, 3)
    ref = np.asarray(ref, dtype=np.float64).reshape(-1, 3)
    if x.size == 0:
        return np.zeros(0)
    m = float(np.abs(ref).mean()) if mean_abs is None else float(mean_abs)
    return (np.abs(x - ref) / (COLOUR_RTOL * np.maximum(np.abs(ref), max(m, 1e-30)))).max(axis=1)


def grad_err(g, ref) -> float:
    g = np.asarray(g, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    scale = np.abs(ref).max()
    if scale == 0:
        return float(np.abs(g).max())
    return float(np.abs(g - ref).max() / scale)


def grad_element_ratio(g, ref) -> float:
    """max over elements of |g - g_ref| / (GRAD_RTOL |g_ref| + GRAD_ATOL_REL max|g_ref|); <= 1 passes."""
    g = np.asarray(g, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    scale = np.abs(ref).max()
    if g.size == 0:
        return 0.0
    tol = GRAD_RTOL * np.abs(ref) + GRAD_ATOL_REL * max(scale, 1e-300)
    return float((np.abs(g - ref) / tol).max())


def check_gradients(grads, ref_g, names=("sites", "density", "sh")) -> dict:
    """Both gradient bounds on each tensor; returns the ratios for printing."""
    out = {}
    for name, x, y in zip(names, grads, ref_g):
        x = np.asarray(x.cpu().numpy() if hasattr(x, "cpu") else x)
        inf_err, el = grad_err(x, y), grad_element_ratio(x, y)
        out[name] = (inf_err, el)
        assert inf_err <= GRAD_RTOL, (name, inf_err)
        assert el <= 1.0, (name, el)
    return out


def compare_sequences(gpu_cells, gpu_len, ref: dict, mask) -> int:
    """Number of rays in ``mask`` whose visited-cell sequence differs."""
    bad = 0
    for r in np.nonzero(mask)[0]:
        L = int(ref["len"][r])
        if int(gpu_len[r]) != L or not np.array_equal(gpu_cells[r, :L], ref["cells"][r, :L]):
            bad += 1
    return bad


def resolve_near_ties(osc, rays, ray_idx, gpu_cells, gpu_len, eps: float, max_steps: int = 8192,
                      max_len: int = 1024, max_leaves: int = 32) -> dict:
    """Matches each near-tie ray's GPU walk (cells [J, >=L], len [J]) with one of
    the oracle's alternative walks. Returns per ray the matched leaf (None if
    none matched), whether its alternatives were complete, and the number of
    forced choices of the match (0: the exact walk)."""
    o, d, t, s = rays
    alt = oracle.alternatives(osc, o, d, t, s, ray_idx, kappa_t=KAPPA_T, kappa_T=KAPPA_TERM if eps > 0 else 0.0,
                              eps=eps, max_steps=max_steps, max_len=max_len, max_leaves=max_leaves)
    match, flips = [], []
    for q in range(len(ray_idx)):
        L = int(gpu_len[q])
        m = None
        for lf in alt["leaves"][q]:
            if lf["len"] == L and L <= max_len and np.array_equal(lf["cells"][:L], gpu_cells[q, :L]):
                m = lf
                break
        match.append(m)
        flips.append(-1 if m is None else len(m["forced"]))
    return dict(match=match, complete=alt["complete"], flips=np.array(flips, dtype=np.int64),
                n_leaves=np.array([len(x) for x in alt["leaves"]]))


MARGIN_BINS = (0.0, 1e-12, 1e-11, 1e-10, 1e-9, 1e-8, 3e-8, 1e-7, KAPPA_T)


def flip_table(margins, flipped) -> list:
    """Rows (lo, hi, near-tie rays, rays whose GPU walk took an alternative) over MARGIN_BINS."""
    rows = []
    for lo, hi in zip(MARGIN_BINS[:-1], MARGIN_BINS[1:]):
        sel = (margins >= lo) & (margins < hi)
        rows.append((lo, hi, int(sel.sum()), int((sel & flipped).sum())))
    return rows
