"""Training-step pieces around the walk, in float64 numpy (Sec. 3.3 and the
implementation details of Sec. 3.4).

TEST INFRASTRUCTURE ONLY, like the rest of this package: the plain statement
of what the GPU library's training kernels compute.

* density activation: softplus with beta = 10, sigma = ln(1 + e^{beta x}) / beta,
  whose derivative is the logistic function of beta x;
* learning-rate schedules: cosine annealing from a start to an end rate over
  the run (positions 2e-4 -> 2e-6, density 1e-1 -> 1e-2, SH 5e-3 -> 5e-4);
  higher-order SH coefficients are held for the first quarter of the run,
  positions for its last tenth (the paper's last 2k of 20k iterations);
* Adam (Kingma and Ba) per parameter, with per-group step counts (a group that
  is held does not advance its moments or its count);
* densification score: the norm of a site's gradient times the cell's
  approximate radius (read as half the mean distance to its Delaunay
  neighbours), and candidates drawn from the multinomial distribution
  proportional to it by inverting its cumulative sum at given uniform draws;
* pruning: a cell goes when its density and every neighbour's density are
  below a threshold;
* insertion of the drawn candidates: each new site lies inside its parent's
  cell, at x_p + f r_p u with r_p the radius of the largest ball about x_p
  inside the cell (half the distance to the nearest Delaunay neighbour), u a
  caller-supplied point of the unit ball and f < 1; the new site starts with
  its parent's density and colour and zero optimizer moments, so that the
  piecewise-constant field, and every render, is unchanged by the insertion;
* removal of pruned sites: the kept sites in their order, attributes and
  moments with them;
* the growth schedule: the number of sites grows linearly from the initial
  count to the maximum up to half the run;
* the rebuild schedule: after a densification the Delaunay graph is rebuilt
  after every optimizer step, then the steps between rebuilds grow by one
  per rebuild up to 100 (the paper's ratio of 1:1 rising to 1:100).
"""

from __future__ import annotations

import math

import numpy as np

SOFTPLUS_BETA = 10.0


def softplus(x, beta: float = SOFTPLUS_BETA) -> np.ndarray:
    """ln(1 + e^{beta x}) / beta, evaluated without overflow."""
    return np.logaddexp(0.0, beta * np.asarray(x, dtype=np.float64)) / beta


def softplus_grad(x, beta: float = SOFTPLUS_BETA) -> np.ndarray:
    """d softplus / dx = 1 / (1 + e^{-beta x})."""
    z = beta * np.asarray(x, dtype=np.float64)
    return np.where(z >= 0, 1.0 / (1.0 + np.exp(-np.abs(z))), np.exp(-np.abs(z)) / (1.0 + np.exp(-np.abs(z))))


def cosine_lr(it: int, total: int, lr0: float, lr_end: float) -> float:
    """Cosine annealing from lr0 at iteration 0 towards lr_end at iteration total."""
    return lr_end + (lr0 - lr_end) * (1.0 + math.cos(math.pi * it / total)) / 2.0


GROUPS = ("sites", "density", "sh0", "sh_high")
LR_START = {"sites": 2e-4, "density": 1e-1, "sh0": 5e-3, "sh_high": 5e-3}
LR_END = {"sites": 2e-6, "density": 1e-2, "sh0": 5e-4, "sh_high": 5e-4}


def schedule(it: int, total: int) -> dict:
    """Learning rate and Adam step count (after this step) per group for 0-based iteration it."""
    warm = total // 4                  # higher SH orders held before this
    freeze = total - total // 10       # positions held from this on
    lr = {g: cosine_lr(it, total, LR_START[g], LR_END[g]) for g in GROUPS}
    t = {"sites": min(it + 1, freeze), "density": it + 1, "sh0": it + 1, "sh_high": max(0, it + 1 - warm)}
    if it >= freeze:
        lr["sites"] = 0.0
    if it < warm:
        lr["sh_high"] = 0.0
    return {"lr": lr, "t": t}


def adam_update(x, g, m, v, lr: float, t: int, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-15):
    """One Adam step (in place on float64 copies); returns (x, m, v). lr == 0 holds the group."""
    x, g, m, v = (np.array(a, dtype=np.float64) for a in (x, g, m, v))
    if lr == 0.0:
        return x, m, v
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1 ** t)
    vhat = v / (1.0 - beta2 ** t)
    x = x - lr * mhat / (np.sqrt(vhat) + eps)
    return x, m, v


def adam_step(params: dict, grads: dict, m: dict, v: dict, it: int, total: int, softplus_density: bool = True,
              beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-15):
    """The training step's optimizer update with the paper's schedule.

    params/grads/m/v hold "sites" [N,3], "density" [N] (the raw parameter when
    softplus_density; its gradient is taken w.r.t. the activated density) and
    "sh" [N,B,3]. Returns new (params, m, v) dicts."""
    sc = schedule(it, total)
    out_p, out_m, out_v = {}, {}, {}
    gd = np.asarray(grads["density"], dtype=np.float64)
    if softplus_density:
        gd = gd * softplus_grad(params["density"])
    for name, g in (("sites", grads["sites"]), ("density", gd)):
        out_p[name], out_m[name], out_v[name] = adam_update(params[name], g, m[name], v[name], sc["lr"][name],
                                                            sc["t"][name], beta1, beta2, eps)
    sh, gsh, msh, vsh = (np.array(a, dtype=np.float64) for a in (params["sh"], grads["sh"], m["sh"], v["sh"]))
    for grp, sl in (("sh0", np.s_[:, :1, :]), ("sh_high", np.s_[:, 1:, :])):
        sh[sl], msh[sl], vsh[sl] = adam_update(sh[sl], gsh[sl], msh[sl], vsh[sl], sc["lr"][grp], sc["t"][grp], beta1,
                                               beta2, eps)
    out_p["sh"], out_m["sh"], out_v["sh"] = sh, msh, vsh
    return out_p, out_m, out_v


def cell_radius(sites, off, idx) -> np.ndarray:
    """Half the mean distance from each site to its Delaunay neighbours (0 for an isolated site)."""
    x = np.asarray(sites, dtype=np.float64)
    n = len(x)
    r = np.zeros(n)
    for i in range(n):
        nb = idx[off[i]:off[i + 1]]
        if len(nb):
            r[i] = 0.5 * np.linalg.norm(x[nb] - x[i], axis=1).mean()
    return r


def densify_scores(sites, off, idx, grad_sites) -> np.ndarray:
    """|d L / d x_i| times the approximate radius of cell i."""
    return np.linalg.norm(np.asarray(grad_sites, dtype=np.float64), axis=1) * cell_radius(sites, off, idx)


def sample_cells(scores, draws) -> np.ndarray:
    """Multinomial draws proportional to scores: for each uniform u in [0, 1),
    the first cell whose cumulative score exceeds u times the total."""
    c = np.cumsum(np.asarray(scores, dtype=np.float64))
    target = np.asarray(draws, dtype=np.float64) * c[-1]
    return np.minimum(np.searchsorted(c, target, side="right"), len(c) - 1).astype(np.int32)


def prune_mask(density, off, idx, threshold: float) -> np.ndarray:
    """True where the cell's density and all its neighbours' are below threshold."""
    s = np.asarray(density, dtype=np.float64)
    n = len(s)
    out = np.zeros(n, dtype=bool)
    for i in range(n):
        nb = idx[off[i]:off[i + 1]]
        out[i] = s[i] < threshold and bool(np.all(s[nb] < threshold))
    return out


def inscribed_radius(sites, off, idx) -> np.ndarray:
    """Radius of the largest ball about each site inside its Voronoi cell: the
    cell is bounded by the bisector planes, the nearest at half the distance to
    the nearest Delaunay neighbour (inf for a site without neighbours)."""
    x = np.asarray(sites, dtype=np.float64)
    r = np.full(len(x), np.inf)
    for i in range(len(x)):
        nb = idx[off[i]:off[i + 1]]
        if len(nb):
            r[i] = 0.5 * np.linalg.norm(x[nb] - x[i], axis=1).min()
    return r


INSERT_FRACTION = 0.5


def insert_sites(sites, off, idx, parents, u, frac: float = INSERT_FRACTION) -> np.ndarray:
    """New sites x_p + frac r_p u for each parent p (r_p the inscribed radius)
    and offset u (|u| <= 1): strictly inside the parent's cell when frac < 1."""
    x = np.asarray(sites, dtype=np.float64)
    p = np.asarray(parents, dtype=np.int64)
    r = inscribed_radius(x, off, idx)[p]
    return x[p] + frac * r[:, None] * np.asarray(u, dtype=np.float64)


def densify(params: dict, moments: list, parents, new_sites):
    """Appends the new sites with their parents' density and SH; their optimizer
    moments start at zero. params: "sites" [N,3], "density" [N], "sh" [N,B,3];
    moments: dicts of the same shapes. Returns (params, moments)."""
    p = np.asarray(parents, dtype=np.int64)
    out = {"sites": np.concatenate([params["sites"], np.asarray(new_sites, dtype=np.float64)]),
           "density": np.concatenate([params["density"], np.asarray(params["density"])[p]]),
           "sh": np.concatenate([params["sh"], np.asarray(params["sh"])[p]])}
    mom = [{k: np.concatenate([mm[k], np.zeros((len(p),) + np.shape(mm[k])[1:])]) for k in mm} for mm in moments]
    return out, mom


def remove_sites(params: dict, moments: list, keep):
    """Keeps the sites where keep is True, in their order, with attributes and moments."""
    k = np.asarray(keep, dtype=bool)
    return ({name: np.asarray(a)[k] for name, a in params.items()},
            [{name: np.asarray(a)[k] for name, a in mm.items()} for mm in moments])


def grow_target(it: int, total: int, n0: int, n_max: int, start: int = 0) -> int:
    """Number of sites wanted after iteration it: n0 until start, then linear
    growth reaching n_max at half the run."""
    half = total // 2
    if it <= start or half <= start:
        return n0 if it <= start else n_max
    f = min(1.0, (it - start) / (half - start))
    return int(round(n0 + (n_max - n0) * f))


def rebuild_steps(total: int, densify_at, max_interval: int = 100) -> list:
    """Iterations (0-based, before the step) at which the Delaunay graph is
    rebuilt: right after each densification, then after 1, 2, 3, ... optimizer
    steps, the interval growing by one per rebuild up to max_interval."""
    d = sorted(set(int(i) for i in densify_at))
    out = []
    it, k = 0, 0
    nxt = 0
    while it < total:
        if d and it >= d[0]:
            while d and it >= d[0]:
                d.pop(0)
            k = 0
            nxt = it
        if it == nxt:
            out.append(it)
            k = min(k + 1, max_interval)
            nxt = it + k
        it += 1
    return out
