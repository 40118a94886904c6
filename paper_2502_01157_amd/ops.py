"""Torch-facing wrappers of the C ABI: packed scenes, ray generation, the
forward/backward walk and the autograd Function.

PyTorch provides device memory and the current HIP stream; all arithmetic of
the walk runs in librf.so.
"""

from __future__ import annotations

import ctypes
from typing import Optional, Sequence, Tuple

import torch

from . import _lib as L

DEFAULT_EPS = 1e-4
DEFAULT_MAX_STEPS = 8192
# The differentiable forward keeps no walk log by default: its backward
# recomputes each walk from the saved colour and transmittance. A caller may
# ask for a log of up to `log_capacity` visits per ray (12 B each); it is cut
# to what fits in LOG_MEMORY_FRACTION of the free device memory, and walks
# longer than the log are recomputed by the backward.
DEFAULT_LOG_CAPACITY = 0
LOG_MEMORY_FRACTION = 0.5


def fitting_log_capacity(n_rays: int, requested: int, device=None) -> int:
    """The largest walk-log capacity <= ``requested`` whose buffers
    (n_rays * (12 * capacity + 16) bytes) fit in LOG_MEMORY_FRACTION of the
    device's free memory (0: no log)."""
    if requested <= 0 or n_rays <= 0:
        return 0
    free, _total = torch.cuda.mem_get_info(device)
    fit = int((free * LOG_MEMORY_FRACTION - 16 * n_rays) // (12 * n_rays))
    return max(0, min(int(requested), fit))


def _stream(device: Optional[torch.device] = None) -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _ptr(t: Optional[torch.Tensor]) -> Optional[int]:
    return None if t is None else t.data_ptr()


def _dev(t: torch.Tensor, dtype: torch.dtype, shape: Sequence[int], name: str) -> torch.Tensor:
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t


def sh_count(deg: int) -> int:
    return (deg + 1) ** 2


class PackedScene:
    """Device-resident packed scene (face planes, neighbour rows, cell records).

    The workspace is one uint8 CUDA tensor owned by this object. ``pack`` can be
    called again after the scene's sites or attributes change (same sizes).
    """

    def __init__(self, sites: torch.Tensor, off: torch.Tensor, idx: torch.Tensor, density: torch.Tensor,
                 sh: torch.Tensor, sh_degree: int, attr_dtype: str = "f32", validate: bool = True,
                 density_activation: str = "plain"):
        """``density_activation="softplus"``: ``density`` holds the raw parameter x and the
        walk sees sigma = ln(1 + e^{10 x}) / 10 (applied by the pack)."""
        self.density_activation = {"plain": L.RF_DENSITY_PLAIN, "softplus": L.RF_DENSITY_SOFTPLUS}[density_activation]
        self.n_sites = int(sites.shape[0])
        self.n_edges = int(idx.shape[0])
        self.sh_degree = int(sh_degree)
        self.attr_dtype = {"f32": L.RF_F32, "bf16": L.RF_BF16}[attr_dtype]
        nbytes = ctypes.c_size_t()
        L.check(L.lib().rf_packed_bytes(self.n_sites, self.n_edges, self.sh_degree, self.attr_dtype,
                                        ctypes.byref(nbytes)))
        self.workspace = torch.empty(int(nbytes.value), dtype=torch.uint8, device=sites.device)
        self.desc = L.PackedSceneDesc()
        self.off = off
        self.idx = idx
        self.pack(sites, density, sh, validate=validate)

    def pack(self, sites: torch.Tensor, density: torch.Tensor, sh: torch.Tensor, validate: bool = False) -> None:
        n, B = self.n_sites, sh_count(self.sh_degree)
        _dev(sites, torch.float32, (n, 3), "sites")
        _dev(self.off, torch.int32, (n + 1,), "off")
        _dev(self.idx, torch.int32, (self.n_edges,), "idx")
        _dev(density, torch.float32, (n,), "density")
        _dev(sh, torch.float32, (n, B, 3), "sh")
        sc = L.Scene(sites.data_ptr(), self.off.data_ptr(), self.idx.data_ptr(), density.data_ptr(),
                     sh.data_ptr(), n, self.n_edges, self.sh_degree, self.density_activation)
        L.check(L.lib().rf_pack_scene(ctypes.byref(sc), self.attr_dtype, self.workspace.data_ptr(),
                                      self.workspace.numel(), int(validate), ctypes.byref(self.desc),
                                      _stream(sites.device)))

    def errors(self) -> Tuple[int, int]:
        e = (ctypes.c_int32 * 2)()
        L.check(L.lib().rf_packed_errors(ctypes.byref(self.desc), ctypes.addressof(e),
                                         _stream(self.workspace.device)))
        return int(e[0]), int(e[1])

    def planes(self) -> torch.Tensor:
        out = torch.empty((self.n_edges, 4), dtype=torch.float32, device=self.workspace.device)
        L.check(L.lib().rf_packed_planes(ctypes.byref(self.desc), out.data_ptr(), _stream(out.device)))
        return out

    def attributes(self) -> Tuple[torch.Tensor, torch.Tensor]:
        dev = self.workspace.device
        dens = torch.empty(self.n_sites, dtype=torch.float32, device=dev)
        sh = torch.empty((self.n_sites, sh_count(self.sh_degree), 3), dtype=torch.float32, device=dev)
        L.check(L.lib().rf_packed_attributes(ctypes.byref(self.desc), dens.data_ptr(), sh.data_ptr(),
                                             _stream(dev)))
        return dens, sh


def _rays(origin, direction, t_max, start) -> L.Rays:
    R = int(direction.shape[0])
    _dev(origin, torch.float32, (R, 3), "origin")
    _dev(direction, torch.float32, (R, 3), "dir")
    _dev(t_max, torch.float32, (R,), "t_max")
    _dev(start, torch.int32, (R,), "start_cell")
    return L.Rays(origin.data_ptr(), direction.data_ptr(), t_max.data_ptr(), start.data_ptr(), R)


def _params(eps: float, max_steps: int) -> L.Params:
    return L.Params(float(eps), int(max_steps))


CAMERA_MODELS = {"pinhole": 0, "fisheye": 1}


def camera_desc(pose12, fov_deg: float, width: int, height: int, model: str = "pinhole") -> L.CameraDesc:
    c = L.CameraDesc()
    for k, v in enumerate(pose12):
        c.pose[k] = float(v)
    c.fov_deg = float(fov_deg)
    c.width = int(width)
    c.height = int(height)
    c.model = CAMERA_MODELS[model]
    return c


def bound_desc(bound: tuple) -> L.BoundDesc:
    b = L.BoundDesc()
    if bound[0] == "box":
        lo, hi = bound[1], bound[2]
        vals = [lo] * 3 + [hi] * 3 if isinstance(lo, (int, float)) else list(lo) + list(hi)
        b.kind = 0
    elif bound[0] == "sphere":
        vals = [bound[1], 0, 0, 0, 0, 0]
        b.kind = 1
    else:
        raise ValueError(bound)
    for k in range(6):
        b.p[k] = float(vals[k])
    return b


def raygen(pose12, fov_deg: float, width: int, height: int, bound: tuple, start: int,
           device="cuda", with_pixel: bool = True, model: str = "pinhole", out=None):
    """Camera rays (pinhole or equidistant fisheye) in 8x8 tile order: (origin, dir, t_max, start_cell, pixel).

    ``out`` = (origin [R,3], dir [R,3], t_max [R], start [R]) writes the rays into
    existing contiguous tensors (e.g. one camera's rows of a multi-camera batch)."""
    R = int(width) * int(height)
    dev = torch.device(device)
    if out is None:
        o = torch.empty((R, 3), dtype=torch.float32, device=dev)
        d = torch.empty((R, 3), dtype=torch.float32, device=dev)
        t = torch.empty(R, dtype=torch.float32, device=dev)
        s = torch.empty(R, dtype=torch.int32, device=dev)
    else:
        o, d, t, s = out
        _dev(o, torch.float32, (R, 3), "origin")
        _dev(d, torch.float32, (R, 3), "dir")
        _dev(t, torch.float32, (R,), "t_max")
        _dev(s, torch.int32, (R,), "start_cell")
        dev = o.device
    px = torch.empty(R, dtype=torch.int32, device=dev) if with_pixel else None
    cam = camera_desc(pose12, fov_deg, width, height, model)
    b = bound_desc(bound)
    L.check(L.lib().rf_raygen(ctypes.byref(cam), ctypes.byref(b), int(start), o.data_ptr(), d.data_ptr(),
                              t.data_ptr(), s.data_ptr(), _ptr(px), _stream(dev)))
    return o, d, t, s, px


SURFACE_KINDS = {"mirror": 1, "glass": 2}


class Surface:
    """An analytic sphere that bends rays (``rf_surface``): a ``"mirror"`` or
    ``"glass"`` of refractive index ``ior`` inside; legs after a crossing end
    at ``bound`` (as in ``raygen``); crossings after the first
    ``max_bounces`` are ignored."""

    def __init__(self, kind: str, centre, radius: float, bound: tuple, ior: float = 1.5, max_bounces: int = 8):
        if kind not in SURFACE_KINDS:
            raise ValueError(f"surface kind must be one of {sorted(SURFACE_KINDS)}")
        self.kind, self.centre, self.radius, self.ior = kind, tuple(float(c) for c in centre), radius, ior
        self.bound, self.max_bounces = bound, max_bounces
        d = L.SurfaceDesc()
        d.kind = SURFACE_KINDS[kind]
        d.max_bounces = int(max_bounces)
        for k in range(3):
            d.centre[k] = self.centre[k]
        d.radius = float(radius)
        d.ior = float(ior)
        d.bound = bound_desc(bound)
        self.desc = d


class Quantiles:
    """The quantile regulariser's per-ray state (``rf_quantiles``): the two
    draws [R,2] and, after ``quantile_forward``, the quantiles, the visit
    holding each and its density (what the backward needs)."""

    def __init__(self, draws: torch.Tensor):
        R = int(draws.shape[0])
        _dev(draws, torch.float32, (R, 2), "draws")
        self.draws = draws
        self.t = torch.zeros((R, 2), dtype=torch.float32, device=draws.device)
        self.segment = torch.full((R, 2), -1, dtype=torch.int32, device=draws.device)
        self.sigma = torch.zeros((R, 2), dtype=torch.float32, device=draws.device)
        self.desc = L.Quantiles(_ptr(draws) if R else None, _ptr(self.t) if R else None,
                                _ptr(self.segment) if R else None, _ptr(self.sigma) if R else None)


def quantile_forward(scene: PackedScene, origin, direction, t_max, start, t_final, log: WalkLog, draws,
                     eps: float = DEFAULT_EPS, max_steps: int = DEFAULT_MAX_STEPS):
    """Quantile regulariser of the walks in ``log``: (Quantiles, loss [R]) with
    loss = |W^-1(u1) - W^-1(u2)| per ray (Sec. 3.4)."""
    R = int(direction.shape[0])
    dev = direction.device
    log.check(R)
    _dev(t_final, torch.float32, (R,), "t_final")
    q = Quantiles(draws)
    loss = torch.empty(R, dtype=torch.float32, device=dev)
    rays = _rays(origin, direction, t_max, start)
    p = _params(eps, max_steps)
    L.check(L.lib().rf_quantile_forward(ctypes.byref(scene.desc), ctypes.byref(rays), ctypes.byref(p),
                                        _ptr(t_final) if R else None, ctypes.byref(log.desc), ctypes.byref(q.desc),
                                        _ptr(loss) if R else None, _stream(dev)))
    return q, loss


def locate(scene: PackedScene, points, seed=None, max_steps: int = 1 << 20):
    """Nearest site of each point [M,3] (the cell containing it): int32 [M];
    -1 for a seed out of range, -2 if ``max_steps`` greedy steps did not
    suffice. ``seed`` (int32 [M], optional) is where each walk starts."""
    M = int(points.shape[0])
    dev = points.device
    _dev(points, torch.float32, (M, 3), "points")
    if seed is not None:
        _dev(seed, torch.int32, (M,), "seed")
    cells = torch.empty(M, dtype=torch.int32, device=dev)
    L.check(L.lib().rf_locate(ctypes.byref(scene.desc), _ptr(points) if M else None, M, _ptr(seed),
                              int(max_steps), _ptr(cells) if M else None, _stream(dev)))
    return cells


class WalkLog:
    """Device buffers of a walk log (``rf_walk_log``): per ray, the first
    ``capacity`` visits of the forward walk (cell and flags, exit distance in
    double) and a tail record, so that the backward skips the face scans.
    Takes ``n_rays * (12 * capacity + 16)`` bytes."""

    def __init__(self, n_rays: int, capacity: int, device=None):
        if capacity < 0:
            raise ValueError("capacity must be >= 0")
        self.n_rays, self.capacity = int(n_rays), int(capacity)
        self.code = torch.empty((self.capacity, self.n_rays), dtype=torch.int32, device=device)
        self.t_exit = torch.empty((self.capacity, self.n_rays), dtype=torch.float64, device=device)
        self.tail = torch.empty((self.n_rays, 4), dtype=torch.int32, device=device)
        self.desc = L.WalkLog(_ptr(self.code) if self.code.numel() else None,
                              _ptr(self.t_exit) if self.t_exit.numel() else None,
                              _ptr(self.tail) if self.tail.numel() else None, self.capacity)

    def check(self, n_rays: int) -> None:
        if n_rays != self.n_rays:
            raise ValueError(f"walk log holds {self.n_rays} rays, the call has {n_rays}")


def render_forward(scene: PackedScene, origin, direction, t_max, start, eps: float = DEFAULT_EPS,
                   max_steps: int = DEFAULT_MAX_STEPS, out=None, log: Optional[WalkLog] = None,
                   surface: Optional[Surface] = None):
    """rgb [R,3], t_final [R], steps [R] (int32; < 0 flags RF_RAY_*); also fills ``log`` if given.
    With ``surface`` the rays bend at it (secondary rays)."""
    R = int(direction.shape[0])
    dev = direction.device
    if out is None:
        out = (torch.empty((R, 3), dtype=torch.float32, device=dev),
               torch.empty(R, dtype=torch.float32, device=dev),
               torch.empty(R, dtype=torch.int32, device=dev))
    rgb, tf, steps = out
    rays = _rays(origin, direction, t_max, start)
    p = _params(eps, max_steps)
    if surface is not None:
        if log is not None:
            log.check(R)
        L.check(L.lib().rf_render_forward_surface(ctypes.byref(scene.desc), ctypes.byref(rays), ctypes.byref(p),
                                                  ctypes.byref(surface.desc), rgb.data_ptr(), tf.data_ptr(),
                                                  steps.data_ptr(), ctypes.byref(log.desc) if log is not None else None,
                                                  _stream(dev)))
    elif log is None:
        L.check(L.lib().rf_render_forward(ctypes.byref(scene.desc), ctypes.byref(rays), ctypes.byref(p),
                                          rgb.data_ptr(), tf.data_ptr(), steps.data_ptr(), _stream(dev)))
    else:
        log.check(R)
        L.check(L.lib().rf_render_forward_logged(ctypes.byref(scene.desc), ctypes.byref(rays), ctypes.byref(p),
                                                 rgb.data_ptr(), tf.data_ptr(), steps.data_ptr(),
                                                 ctypes.byref(log.desc), _stream(dev)))
    return rgb, tf, steps


def render_trace(scene: PackedScene, origin, direction, t_max, start, eps: float = DEFAULT_EPS,
                 max_steps: int = DEFAULT_MAX_STEPS, max_len: int = 1024):
    R = int(direction.shape[0])
    dev = direction.device
    rgb = torch.empty((R, 3), dtype=torch.float32, device=dev)
    tf = torch.empty(R, dtype=torch.float32, device=dev)
    steps = torch.empty(R, dtype=torch.int32, device=dev)
    cells = torch.full((R, max_len), -1, dtype=torch.int32, device=dev)
    t_exit = torch.full((R, max_len), float("nan"), dtype=torch.float32, device=dev)
    rays = _rays(origin, direction, t_max, start)
    p = _params(eps, max_steps)
    L.check(L.lib().rf_render_trace(ctypes.byref(scene.desc), ctypes.byref(rays), ctypes.byref(p), int(max_len),
                                    rgb.data_ptr(), tf.data_ptr(), steps.data_ptr(), cells.data_ptr(),
                                    t_exit.data_ptr(), _stream(dev)))
    return dict(rgb=rgb, t_final=tf, steps=steps, cells=cells, t_exit=t_exit)


def render_backward(scene: PackedScene, origin, direction, t_max, start, rgb, t_final, grad_rgb,
                    grad_t_final=None, eps: float = DEFAULT_EPS, max_steps: int = DEFAULT_MAX_STEPS,
                    mode: int = 0, grads=None, log: Optional[WalkLog] = None,
                    quantiles: Optional["Quantiles"] = None, grad_loss=None, surface: Optional[Surface] = None,
                    steps=None, mismatches=None):
    """Gradients (sites [N,3], density [N], sh [N,B,3]); accumulated into ``grads`` if given.

    With ``log`` (filled by ``render_forward`` on the same scene, rays and
    parameters) the visits are read from the log instead of recomputed; with
    ``quantiles`` (from ``quantile_forward`` on that log) and ``grad_loss`` [R]
    the quantile regulariser's gradient is included. The recomputing form
    (no log, no surface, no quantiles) checks each recomputed walk against the
    forward's outputs when ``mismatches`` (int32 [1], zeroed by the caller) is
    given: it counts the rays whose final transmittance, or visit count in
    ``steps`` (the forward's, optional), differs."""
    R = int(direction.shape[0])
    dev = direction.device
    n, B = scene.n_sites, sh_count(scene.sh_degree)
    if grads is None:
        grads = (torch.zeros((n, 3), dtype=torch.float32, device=dev),
                 torch.zeros(n, dtype=torch.float32, device=dev),
                 torch.zeros((n, B, 3), dtype=torch.float32, device=dev))
    gs, gd, gsh = grads
    _dev(rgb, torch.float32, (R, 3), "rgb")
    _dev(t_final, torch.float32, (R,), "t_final")
    _dev(grad_rgb, torch.float32, (R, 3), "grad_rgb")
    if grad_t_final is not None:
        _dev(grad_t_final, torch.float32, (R,), "grad_t_final")
    _dev(gs, torch.float32, (n, 3), "grad_sites")
    _dev(gd, torch.float32, (n,), "grad_density")
    _dev(gsh, torch.float32, (n, B, 3), "grad_sh")
    rays = _rays(origin, direction, t_max, start)
    p = _params(eps, max_steps)
    if surface is not None:
        if quantiles is not None:
            raise ValueError("the quantile regulariser is defined for unbent rays only")
        if mode != 0:
            raise ValueError("with a surface the backward always reduces per wavefront (mode 0)")
        if log is not None:
            log.check(R)
        L.check(L.lib().rf_render_backward_surface(ctypes.byref(scene.desc), ctypes.byref(rays), ctypes.byref(p),
                                                   ctypes.byref(surface.desc), rgb.data_ptr(), t_final.data_ptr(),
                                                   grad_rgb.data_ptr(), _ptr(grad_t_final),
                                                   ctypes.byref(log.desc) if log is not None else None,
                                                   gs.data_ptr(), gd.data_ptr(), gsh.data_ptr(), _stream(dev)))
    elif quantiles is not None:
        if log is None or grad_loss is None:
            raise ValueError("the quantile term needs the walk log and grad_loss")
        log.check(R)
        _dev(grad_loss, torch.float32, (R,), "grad_loss")
        L.check(L.lib().rf_render_backward_quantile(ctypes.byref(scene.desc), ctypes.byref(rays), ctypes.byref(p),
                                                    rgb.data_ptr(), t_final.data_ptr(), grad_rgb.data_ptr(),
                                                    _ptr(grad_t_final), ctypes.byref(log.desc),
                                                    ctypes.byref(quantiles.desc), grad_loss.data_ptr(),
                                                    gs.data_ptr(), gd.data_ptr(), gsh.data_ptr(), int(mode),
                                                    _stream(dev)))
    elif log is None:
        if steps is not None:
            _dev(steps, torch.int32, (R,), "steps")
        if mismatches is not None:
            _dev(mismatches, torch.int32, (1,), "mismatches")
        L.check(L.lib().rf_render_backward(ctypes.byref(scene.desc), ctypes.byref(rays), ctypes.byref(p),
                                           rgb.data_ptr(), t_final.data_ptr(), _ptr(steps), grad_rgb.data_ptr(),
                                           _ptr(grad_t_final), gs.data_ptr(), gd.data_ptr(), gsh.data_ptr(),
                                           int(mode), _ptr(mismatches), _stream(dev)))
    else:
        log.check(R)
        L.check(L.lib().rf_render_backward_logged(ctypes.byref(scene.desc), ctypes.byref(rays), ctypes.byref(p),
                                                  rgb.data_ptr(), t_final.data_ptr(), grad_rgb.data_ptr(),
                                                  _ptr(grad_t_final), ctypes.byref(log.desc), gs.data_ptr(),
                                                  gd.data_ptr(), gsh.data_ptr(), int(mode), _stream(dev)))
    return gs, gd, gsh


class RadFoamRender(torch.autograd.Function):
    """Differentiable render of rays through a Voronoi scene.

    forward(sites, density, sh, off, idx, origin, dir, t_max, start, sh_degree,
            attr_dtype, eps, max_steps, log_capacity, quantile_draws, surface)
        -> (rgb [R,3], t_final [R], steps [R], quantile_loss [R])

    Packs the scene (face planes from the current sites, attributes in
    ``attr_dtype``) and walks every ray; the backward recomputes each walk
    from the saved colour and final transmittance. With ``log_capacity`` > 0
    the forward also saves a walk log of up to that many visits per ray (cut
    to what fits in free device memory) and the backward reads it instead. With ``quantile_draws`` [R,2] it also returns the quantile
    regulariser |W^-1(u1) - W^-1(u2)| per ray (Sec. 3.4; zeros otherwise).
    With ``surface`` (a ``Surface``) the rays bend at it; the quantile
    regulariser is then not available.
    Gradients flow to sites, density and sh; none to the rays or the adjacency.
    """

    @staticmethod
    def forward(ctx, sites, density, sh, off, idx, origin, direction, t_max, start, sh_degree: int = 3,
                attr_dtype: str = "f32", eps: float = DEFAULT_EPS, max_steps: int = DEFAULT_MAX_STEPS,
                log_capacity: int = DEFAULT_LOG_CAPACITY, quantile_draws=None, surface=None):
        if surface is not None and quantile_draws is not None:
            raise ValueError("the quantile regulariser is defined for unbent rays only")
        sites_c, dens_c, sh_c = sites.detach().contiguous(), density.detach().contiguous(), sh.detach().contiguous()
        scene = PackedScene(sites_c, off, idx, dens_c, sh_c, sh_degree, attr_dtype, validate=False)
        R = int(direction.shape[0])
        cap = fitting_log_capacity(R, log_capacity, direction.device)
        want_log = cap > 0 or quantile_draws is not None
        log = WalkLog(R, cap, direction.device) if want_log else None
        rgb, tf, steps = render_forward(scene, origin, direction, t_max, start, eps, max_steps, log=log,
                                        surface=surface)
        q = None
        if quantile_draws is not None:
            q, qloss = quantile_forward(scene, origin, direction, t_max, start, tf, log,
                                        quantile_draws.detach().contiguous().float(), eps, max_steps)
        else:
            qloss = torch.zeros(R, dtype=torch.float32, device=direction.device)
        ctx.scene = scene
        ctx.log = log
        ctx.q = q
        ctx.surface = surface
        ctx.hyper = (eps, max_steps)
        ctx.save_for_backward(origin, direction, t_max, start, rgb, tf)
        ctx.mark_non_differentiable(steps)
        if q is None:
            ctx.mark_non_differentiable(qloss)
        return rgb, tf, steps, qloss

    @staticmethod
    def backward(ctx, grad_rgb, grad_tf, _grad_steps, grad_q):
        origin, direction, t_max, start, rgb, tf = ctx.saved_tensors
        eps, max_steps = ctx.hyper
        if grad_rgb is None:
            grad_rgb = torch.zeros_like(rgb)
        q = ctx.q
        if q is not None and grad_q is None:
            q = None
        gs, gd, gsh = render_backward(ctx.scene, origin, direction, t_max, start, rgb, tf,
                                      grad_rgb.contiguous().float(),
                                      None if grad_tf is None else grad_tf.contiguous().float(), eps, max_steps,
                                      log=ctx.log, quantiles=q,
                                      grad_loss=None if q is None else grad_q.contiguous().float(),
                                      surface=ctx.surface)
        ctx.log = None
        ctx.q = None
        return gs, gd, gsh, None, None, None, None, None, None, None, None, None, None, None, None, None


def render(sites, density, sh, off, idx, origin, direction, t_max, start, sh_degree: int = 3,
           attr_dtype: str = "f32", eps: float = DEFAULT_EPS, max_steps: int = DEFAULT_MAX_STEPS,
           log_capacity: int = DEFAULT_LOG_CAPACITY, quantile_draws=None, surface=None):
    """Autograd entry point: (rgb, t_final, steps), plus the per-ray quantile
    loss when ``quantile_draws`` [R,2] is given; ``surface`` bends the rays."""
    out = RadFoamRender.apply(sites, density, sh, off, idx, origin, direction, t_max, start, sh_degree,
                              attr_dtype, eps, max_steps, log_capacity, quantile_draws, surface)
    return out if quantile_draws is not None else out[:3]


# ---------------------------------------------------------------------------
# Training-step pieces (Sec. 3.3-3.4): schedule, Adam, densification, pruning.
# ---------------------------------------------------------------------------

def train_schedule(iteration: int, total: int) -> L.AdamArgs:
    """Adam settings of 0-based ``iteration`` of a ``total``-iteration run (the paper's schedule)."""
    a = L.AdamArgs()
    L.check(L.lib().rf_train_schedule(int(iteration), int(total), ctypes.byref(a)))
    return a


class AdamState:
    """First and second moments of the positions, density and SH (zeros at the start)."""

    def __init__(self, n_sites: int, sh_degree: int, device=None):
        B = sh_count(sh_degree)
        self.tensors = {k: torch.zeros(shape, dtype=torch.float32, device=device) for k, shape in
                        (("m_sites", (n_sites, 3)), ("v_sites", (n_sites, 3)), ("m_density", (n_sites,)),
                         ("v_density", (n_sites,)), ("m_sh", (n_sites, B, 3)), ("v_sh", (n_sites, B, 3)))}
        self.desc = L.AdamState(*[_ptr(self.tensors[k]) for k in ("m_sites", "v_sites", "m_density", "v_density",
                                                                   "m_sh", "v_sh")])


def adam_step(args: L.AdamArgs, state: AdamState, sites, density, sh, grad_sites, grad_density, grad_sh) -> None:
    """One Adam step of the three parameter tensors, in place (see ``rf_adam_step``)."""
    n = int(sites.shape[0])
    B = int(sh.shape[1]) if sh.dim() == 3 else -1
    if B not in (1, 4, 9, 16):
        raise ValueError("sh must be [n, B, 3] with B = (degree + 1)^2, degree 0..3")
    for t, shape, name in ((sites, (n, 3), "sites"), (density, (n,), "density"), (sh, (n, B, 3), "sh"),
                           (grad_sites, (n, 3), "grad_sites"), (grad_density, (n,), "grad_density"),
                           (grad_sh, (n, B, 3), "grad_sh")):
        _dev(t, torch.float32, shape, name)
    deg = int(round(B ** 0.5)) - 1
    L.check(L.lib().rf_adam_step(n, deg, ctypes.byref(args), sites.data_ptr(), density.data_ptr(), sh.data_ptr(),
                                 grad_sites.data_ptr(), grad_density.data_ptr(), grad_sh.data_ptr(),
                                 ctypes.byref(state.desc), _stream(sites.device)))


def densify_scores(sites, off, idx, grad_sites) -> torch.Tensor:
    """|dL/dx_i| times the cell's approximate radius, per cell."""
    n = int(sites.shape[0])
    _dev(sites, torch.float32, (n, 3), "sites")
    _dev(off, torch.int32, (n + 1,), "off")
    _dev(idx, torch.int32, (int(idx.shape[0]),), "idx")
    _dev(grad_sites, torch.float32, (n, 3), "grad_sites")
    out = torch.empty(n, dtype=torch.float32, device=sites.device)
    L.check(L.lib().rf_densify_scores(sites.data_ptr(), off.data_ptr(), _ptr(idx) if idx.numel() else None, n,
                                      grad_sites.data_ptr(), out.data_ptr(), _stream(sites.device)))
    return out


def sample_cells(scores, draws) -> torch.Tensor:
    """Multinomial candidates proportional to ``scores`` at uniform ``draws`` in [0, 1) (int32)."""
    n, k = int(scores.shape[0]), int(draws.shape[0])
    _dev(scores, torch.float32, (n,), "scores")
    _dev(draws, torch.float32, (k,), "draws")
    nbytes = ctypes.c_size_t()
    L.check(L.lib().rf_sample_workspace(n, ctypes.byref(nbytes)))
    ws = torch.empty(max(int(nbytes.value) // 8, 1), dtype=torch.float64, device=scores.device)
    out = torch.empty(k, dtype=torch.int32, device=scores.device)
    L.check(L.lib().rf_sample_cells(scores.data_ptr(), n, draws.data_ptr(), k, out.data_ptr(), ws.data_ptr(),
                                    ws.numel() * 8, _stream(scores.device)))
    return out


def prune_mask(density, off, idx, threshold: float) -> torch.Tensor:
    """True where the cell's density (sigma) and all its neighbours' are below ``threshold``."""
    n = int(density.shape[0])
    _dev(density, torch.float32, (n,), "density")
    _dev(off, torch.int32, (n + 1,), "off")
    _dev(idx, torch.int32, (int(idx.shape[0]),), "idx")
    out = torch.empty(n, dtype=torch.uint8, device=density.device)
    L.check(L.lib().rf_prune_mask(density.data_ptr(), off.data_ptr(), _ptr(idx) if idx.numel() else None, n,
                                  float(threshold), out.data_ptr(), _stream(density.device)))
    return out.bool()


def insert_sites(sites, off, idx, parents, offsets, frac: float = 0.5) -> torch.Tensor:
    """New sites inside their parents' cells: x_p + frac r_p u (r_p half the
    distance to p's nearest Delaunay neighbour, u = offsets[k] in the unit ball)."""
    n, k = int(sites.shape[0]), int(parents.shape[0])
    _dev(sites, torch.float32, (n, 3), "sites")
    _dev(off, torch.int32, (n + 1,), "off")
    _dev(idx, torch.int32, (int(idx.shape[0]),), "idx")
    _dev(parents, torch.int32, (k,), "parents")
    _dev(offsets, torch.float32, (k, 3), "offsets")
    out = torch.empty((k, 3), dtype=torch.float32, device=sites.device)
    L.check(L.lib().rf_insert_sites(sites.data_ptr(), off.data_ptr(), _ptr(idx) if idx.numel() else None, n,
                                    _ptr(parents) if k else None, _ptr(offsets) if k else None, k, float(frac),
                                    _ptr(out) if k else None, _stream(sites.device)))
    return out


def gather_rows(x, rows) -> torch.Tensor:
    """x[rows] for a float32 tensor x [n, ...] and int32 rows [k] (``rf_gather_rows``)."""
    n, k = int(x.shape[0]), int(rows.shape[0])
    if x.dtype != torch.float32 or not x.is_cuda or not x.is_contiguous():
        raise TypeError("x must be a contiguous float32 CUDA tensor")
    _dev(rows, torch.int32, (k,), "rows")
    width = int(x[0].numel()) if n else int(torch.Size(x.shape[1:]).numel())
    out = torch.empty((k,) + tuple(x.shape[1:]), dtype=torch.float32, device=x.device)
    L.check(L.lib().rf_gather_rows(_ptr(x) if x.numel() else None, n, max(width, 1), _ptr(rows) if k else None, k,
                                   _ptr(out) if out.numel() else None, _stream(x.device)))
    return out


def keep_index(keep) -> torch.Tensor:
    """Indices where ``keep`` (bool or uint8 [n]) is set, in order (int32); synchronises for the count."""
    n = int(keep.shape[0])
    k8 = keep.to(torch.uint8) if keep.dtype == torch.bool else keep
    _dev(k8, torch.uint8, (n,), "keep")
    nbytes = ctypes.c_size_t()
    L.check(L.lib().rf_keep_workspace(n, ctypes.byref(nbytes)))
    ws = torch.empty(max(int(nbytes.value) // 8, 1), dtype=torch.int64, device=keep.device)
    kept = torch.empty(max(n, 1), dtype=torch.int32, device=keep.device)
    count = torch.empty(1, dtype=torch.int64, device=keep.device)
    L.check(L.lib().rf_keep_index(_ptr(k8) if n else None, n, kept.data_ptr(), count.data_ptr(), ws.data_ptr(),
                                  ws.numel() * 8, _stream(keep.device)))
    return kept[: int(count.item())]
