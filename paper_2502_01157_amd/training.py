"""The training loop around the walk with a changing set of sites (Sec. 3.3
"Densification" and "Pruning", Sec. 3.4 "Training" and "Voronoi
optimization"): render, photometric loss, backward, Adam with the paper's
schedule, and at a densification step the pruning of empty cells, the
insertion of sites drawn by the densification score, and a rebuild of the
Delaunay graph; between densifications the graph is rebuilt after 1, 2, 3,
... optimizer steps, up to every 100 steps.

Every step of the walk and of the training pieces runs in librf.so; this
module only sequences the calls. The Delaunay graph is built on the host
(Qhull) from the current sites, as the library takes the adjacency as an
input; the start cell of each ray is then located on the device.
"""

from __future__ import annotations

from dataclasses import dataclass
from typing import List, Optional

import numpy as np
import torch

from . import ops


def delaunay_csr(sites: np.ndarray):
    """Delaunay neighbour CSR (off int32 [n+1], idx int32 [E], rows ascending)
    of float32 sites, by Qhull on the host. Raises if Qhull drops a point."""
    from scipy.spatial import Delaunay

    tri = Delaunay(np.asarray(sites, dtype=np.float64))
    if len(tri.coplanar):
        raise RuntimeError(f"Qhull dropped {len(tri.coplanar)} points")
    indptr, indices = tri.vertex_neighbor_vertices
    n = len(sites)
    rows = np.repeat(np.arange(n, dtype=np.int64), np.diff(indptr))
    idx = (np.sort(rows * n + indices) % n).astype(np.int32)
    return indptr.astype(np.int32), idx


def grow_target(it: int, total: int, n0: int, n_max: int, start: int = 0) -> int:
    """Sites wanted after iteration ``it``: n0 until ``start``, then linear growth to n_max at half the run."""
    half = total // 2
    if it <= start or half <= start:
        return n0 if it <= start else n_max
    f = min(1.0, (it - start) / (half - start))
    return int(round(n0 + (n_max - n0) * f))


@dataclass
class TrainConfig:
    total: int                      # optimizer steps of the run
    n_max: int                      # sites wanted at half the run
    densify_every: int = 100        # steps between densifications (until half the run)
    densify_start: int = 0          # first densification after this step
    prune_threshold: float = 1e-3   # a cell and all its neighbours below this density are removed
    insert_frac: float = 0.5        # new site at x_p + frac r_p u (r_p: inscribed radius of the parent's cell)
    rebuild_max_interval: int = 100
    quantile_weight: float = 0.0    # lambda of the quantile regulariser (0: off)
    eps: float = ops.DEFAULT_EPS
    seed: int = 0


@dataclass
class StepStats:
    it: int
    loss: float
    n_sites: int
    rebuilt: bool
    densified: bool


class Trainer:
    """Optimizes sites, raw densities (softplus) and SH coefficients of a
    Voronoi scene so that renders of fixed rays match target colours.

    rays: (origin [R,3], dir [R,3], t_max [R]) on the device; the start cell of
    each ray is located on the device after every rebuild."""

    def __init__(self, sites: torch.Tensor, density_raw: torch.Tensor, sh: torch.Tensor, sh_degree: int,
                 cfg: TrainConfig):
        self.cfg = cfg
        self.sh_degree = int(sh_degree)
        self.dev = sites.device
        self.sites = sites.detach().contiguous().clone()
        self.x = density_raw.detach().contiguous().clone()
        self.sh = sh.detach().contiguous().clone()
        self.adam = ops.AdamState(self.n_sites, self.sh_degree, self.dev)
        self.gen = torch.Generator(device=self.dev)
        self.gen.manual_seed(cfg.seed)
        self.densify_at = [it for it in range(cfg.densify_start + cfg.densify_every, cfg.total // 2 + 1,
                                              cfg.densify_every)]
        self.history: List[StepStats] = []
        self.rebuilds: List[int] = []
        self._interval = 0
        self._next_rebuild = 0
        self.starts: Optional[torch.Tensor] = None
        self._n0 = self.n_sites
        self.rebuild()

    @property
    def n_sites(self) -> int:
        return int(self.sites.shape[0])

    # -- Delaunay graph -------------------------------------------------
    def rebuild(self) -> None:
        """Rebuilds the Delaunay CSR from the current sites (host Qhull) and packs the scene."""
        off, idx = delaunay_csr(self.sites.cpu().numpy())
        self.off = torch.from_numpy(off).to(self.dev)
        self.idx = torch.from_numpy(idx).to(self.dev)
        self.packed = ops.PackedScene(self.sites, self.off, self.idx, self.x, self.sh, self.sh_degree,
                                      density_activation="softplus")
        self._located = False

    def _locate(self, origin: torch.Tensor) -> torch.Tensor:
        if not self._located or self.starts is None or self.starts.shape[0] != origin.shape[0]:
            seed = None
            if self.starts is not None and self.starts.shape[0] == origin.shape[0]:
                seed = self.starts.clamp(0, self.n_sites - 1).contiguous()
            self.starts = ops.locate(self.packed, origin.contiguous(), seed)
            self._located = True
        return self.starts

    # -- densification and pruning -----------------------------------------
    def _resize_adam(self, rows: Optional[torch.Tensor], n_new: int) -> None:
        old = self.adam.tensors
        new = ops.AdamState(self.n_sites, self.sh_degree, self.dev)
        for k, t in old.items():
            kept = ops.gather_rows(t.contiguous(), rows) if rows is not None else t
            new.tensors[k][: kept.shape[0]].copy_(kept)  # appended sites start with zero moments
        self.adam = new

    def prune(self) -> Optional[torch.Tensor]:
        """Removes the sites whose density and all neighbours' densities are
        below the threshold; returns the kept sites' old indices (None if none
        is removed)."""
        sigma, _ = self.packed.attributes()
        mask = ops.prune_mask(sigma, self.off, self.idx, self.cfg.prune_threshold)
        if not bool(mask.any()):
            return None
        kept = ops.keep_index(~mask)
        if kept.shape[0] < 5:  # keep a triangulable scene
            return None
        n_old = self.n_sites
        self.sites = ops.gather_rows(self.sites, kept)
        self.x = ops.gather_rows(self.x, kept)
        self.sh = ops.gather_rows(self.sh, kept)
        self._resize_adam(kept, 0)
        if self.starts is not None:
            # start cells as seeds of the next location: a removed cell seeds from cell 0
            remap = torch.zeros(n_old, dtype=torch.int32, device=self.dev)
            remap[kept.long()] = torch.arange(kept.shape[0], dtype=torch.int32, device=self.dev)
            self.starts = remap[self.starts.long()]
        return kept

    def densify(self, grad_sites: torch.Tensor, n_new: int) -> int:
        """Inserts n_new sites inside cells drawn by the densification score."""
        if n_new <= 0:
            return 0
        scores = ops.densify_scores(self.sites, self.off, self.idx, grad_sites)
        if not bool((scores > 0).any()):
            return 0
        draws = torch.rand(n_new, device=self.dev, generator=self.gen)
        parents = ops.sample_cells(scores, draws)
        u = torch.randn((n_new, 3), device=self.dev, generator=self.gen)
        u = u / u.norm(dim=1, keepdim=True).clamp_min(1e-12) * torch.rand(
            (n_new, 1), device=self.dev, generator=self.gen) ** (1.0 / 3.0)
        new_sites = ops.insert_sites(self.sites, self.off, self.idx, parents, u.contiguous(), self.cfg.insert_frac)
        self.sites = torch.cat([self.sites, new_sites])
        self.x = torch.cat([self.x, ops.gather_rows(self.x, parents)])
        self.sh = torch.cat([self.sh, ops.gather_rows(self.sh, parents)])
        self._resize_adam(None, n_new)
        return n_new

    # -- one optimizer step ---------------------------------------------------
    def step(self, it: int, rays, target: torch.Tensor, quantile_draws: Optional[torch.Tensor] = None) -> StepStats:
        cfg = self.cfg
        o, d, t = rays
        if it == self._next_rebuild and it not in self.rebuilds:
            if it > 0:
                self.rebuild()
            self.rebuilds.append(it)
            self._interval = min(self._interval + 1, cfg.rebuild_max_interval)
            self._next_rebuild = it + self._interval
            rebuilt = True
        else:
            rebuilt = False
        self.packed.pack(self.sites, self.x, self.sh)
        s = self._locate(o)
        use_q = cfg.quantile_weight > 0 and quantile_draws is not None
        log = ops.WalkLog(int(d.shape[0]), 0, self.dev) if use_q else None
        rgb, tf, _ = ops.render_forward(self.packed, o, d, t, s, eps=cfg.eps, log=log)
        diff = rgb - target
        loss = float((diff * diff).mean())
        g_rgb = ((2.0 / diff.numel()) * diff).contiguous()
        kw = {}
        if use_q:
            q, qloss = ops.quantile_forward(self.packed, o, d, t, s, tf, log, quantile_draws, cfg.eps)
            loss += cfg.quantile_weight * float(qloss.mean())
            kw = dict(quantiles=q, grad_loss=torch.full_like(qloss, cfg.quantile_weight / qloss.numel()))
        gs, gd, gsh = ops.render_backward(self.packed, o, d, t, s, rgb, tf, g_rgb, eps=cfg.eps, log=log, **kw)
        ops.adam_step(ops.train_schedule(it, cfg.total), self.adam, self.sites, self.x, self.sh, gs, gd, gsh)
        densified = False
        if it in self.densify_at:
            kept = self.prune()
            # the score uses this step's site gradients, of the kept sites, and
            # the kept sites' Delaunay graph (cell radii, inscribed balls)
            g_kept = gs
            if kept is not None:
                g_kept = ops.gather_rows(gs, kept)
                self.rebuild()
            want = grow_target(it, cfg.total, self._n0, cfg.n_max, cfg.densify_start)
            self.densify(g_kept, want - self.n_sites)
            densified = True
            # after a densification the graph is rebuilt before the next step, then at growing intervals
            self.rebuild()
            self.rebuilds.append(it + 1)
            self._interval = 1
            self._next_rebuild = it + 1 + self._interval
            self._located = False
        st = StepStats(it, loss, self.n_sites, rebuilt, densified)
        self.history.append(st)
        return st

    def run(self, rays, target: torch.Tensor, quantile_draws=None) -> List[StepStats]:
        self._n0 = self.n_sites
        for it in range(self.cfg.total):
            self.step(it, rays, target, quantile_draws)
        return self.history
