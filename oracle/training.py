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
  below a threshold.
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
