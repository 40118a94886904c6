"""FP64 CPU oracle of the differentiable Voronoi ray walk (ctypes binding).

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the
benchmark's CPU-baseline leg use this package; the GPU library never does.
The arithmetic lives in ``oracle.c`` (plain C, double precision, pthreads);
this module only marshals numpy arrays. Every float input is widened to
float64 exactly before the call.
"""

from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
# a sanitizer build of the same source (see build_sanitized); the tests run the
# pins against it in a child process that preloads the ASan runtime
_SAN_LIB_PATH = os.path.join(_HERE, "liboracle_san.so")
if os.environ.get("ORACLE_SANITIZED") == "1":
    _LIB_PATH = _SAN_LIB_PATH

BAD_START = -1
MAX_STEPS = -2
DEFAULT_EPS = 1e-4
DEFAULT_MAX_STEPS = 8192


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so with gcc (no fast-math)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-std=c11", "-O2", "-fPIC", "-shared", "-pthread",
                               "-D_GNU_SOURCE", "-Wall", "-Wextra", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def build_sanitized() -> str:
    """Compile oracle.c with AddressSanitizer and UndefinedBehaviorSanitizer
    (every UB report aborts) into liboracle_san.so, for the sanitizer test."""
    tmp = _SAN_LIB_PATH + f".tmp{os.getpid()}"
    subprocess.check_call(["gcc", "-std=c11", "-O1", "-g", "-fPIC", "-shared", "-pthread", "-D_GNU_SOURCE",
                           "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
                           "-fno-omit-frame-pointer", "-Wall", "-Wextra", "-o", tmp, _SRC, "-lm"])
    os.replace(tmp, _SAN_LIB_PATH)
    return _SAN_LIB_PATH


class _Surface(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("max_bounces", ctypes.c_int32), ("centre", ctypes.c_double * 3),
                ("radius", ctypes.c_double), ("ior", ctypes.c_double), ("bound_kind", ctypes.c_int32),
                ("bound", ctypes.c_double * 6), ("fp32_legs", ctypes.c_int32)]


class _Scene(ctypes.Structure):
    _fields_ = [("sites", ctypes.c_void_p), ("off", ctypes.c_void_p), ("idx", ctypes.c_void_p),
                ("density", ctypes.c_void_p), ("sh", ctypes.c_void_p),
                ("n_sites", ctypes.c_int64), ("sh_deg", ctypes.c_int32), ("surf", ctypes.POINTER(_Surface))]


SURFACE_KINDS = {"none": 0, "mirror": 1, "glass": 2}


class Surface:
    """An analytic sphere in the scene that bends rays (mirror, or glass of
    refractive index ``ior`` inside); legs after a crossing end at ``bound``
    (the raygen bound); crossings after the first ``max_bounces`` are ignored.
    ``fp32_legs`` rounds each new leg's origin and direction to FP32, as the
    GPU library's interface defines its legs (every leg is then a ray with FP32
    origin and direction, like the caller's); by default legs are exact."""

    def __init__(self, kind: str, centre, radius: float, bound: tuple, ior: float = 1.5, max_bounces: int = 8,
                 fp32_legs: bool = False):
        self.kind, self.centre, self.radius, self.ior = kind, tuple(float(c) for c in centre), float(radius), float(ior)
        self.bound, self.max_bounces = bound, int(max_bounces)
        bk, bp = encode_bound(bound)
        self._c = _Surface(SURFACE_KINDS[kind], self.max_bounces, (ctypes.c_double * 3)(*self.centre), self.radius,
                           self.ior, bk, (ctypes.c_double * 6)(*bp), int(bool(fp32_legs)))


_lib = None


def _load():
    global _lib
    if _lib is None:
        if _LIB_PATH == _SAN_LIB_PATH:
            if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
                build_sanitized()
        elif not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
            build()
        lib = ctypes.CDLL(_LIB_PATH)
        P = ctypes.c_void_p
        lib.orc_sh_basis.argtypes = [ctypes.c_int, P, ctypes.c_int64, P]
        lib.orc_raygen.argtypes = [P, ctypes.c_double, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, P, P,
                                   P, P, P]
        lib.orc_face_planes.argtypes = [P, P, P, ctypes.c_int64, P]
        lib.orc_bf16_round.argtypes = [P, P, ctypes.c_int64]
        lib.orc_nearest_site.argtypes = [P, ctypes.c_int64, P, ctypes.c_int64, P, P]
        lib.orc_quantile.argtypes = [ctypes.POINTER(_Scene), P, P, P, P, ctypes.c_int64, ctypes.c_double,
                                     ctypes.c_int32, P, P, ctypes.c_int, P, P, P, P]
        lib.orc_bf16_round.restype = None
        lib.orc_check_csr.argtypes = [P, P, ctypes.c_int64, ctypes.c_int64]
        lib.orc_forward.argtypes = [ctypes.POINTER(_Scene), P, P, P, P, ctypes.c_int64, ctypes.c_double,
                                    ctypes.c_int32, ctypes.c_int, P, P, P]
        lib.orc_trace.argtypes = [ctypes.POINTER(_Scene), P, P, P, P, ctypes.c_int64, ctypes.c_double,
                                  ctypes.c_int32, ctypes.c_int32, ctypes.c_int, P, P, P, P, P, P, P, P, P, P, P, P, P]
        lib.orc_backward.argtypes = [ctypes.POINTER(_Scene), P, P, P, P, ctypes.c_int64, ctypes.c_double,
                                     ctypes.c_int32, P, P, ctypes.c_int, P, P, P, P, P, P]
        lib.orc_walk_forced.argtypes = [ctypes.POINTER(_Scene), P, P, P, P, ctypes.c_int64, P, ctypes.c_int64, P, P,
                                        P, ctypes.c_double, ctypes.c_int32, ctypes.c_double, ctypes.c_double,
                                        ctypes.c_int32, ctypes.c_int32, ctypes.c_int, P, P, P, P, P, P, P, P, P]
        _lib = lib
    return _lib


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _i32(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.int32))


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data


def _check(rc: int, what: str) -> None:
    if rc != 0:
        raise ValueError(f"oracle {what} rejected its arguments (code {rc})")


def default_threads() -> int:
    return max(1, min(os.cpu_count() or 1, 64))


class OracleScene:
    """Scene arrays widened to float64 and held alive for the C calls."""

    def __init__(self, sites, off, idx, density, sh, sh_deg: int, surface: Optional[Surface] = None):
        self.sites = _f64(sites).reshape(-1, 3)
        self.off = _i32(off)
        self.idx = _i32(idx)
        self.density = _f64(density).reshape(-1)
        b = (sh_deg + 1) ** 2
        self.sh = _f64(sh).reshape(-1, b, 3)
        self.sh_deg = int(sh_deg)
        n = self.sites.shape[0]
        if self.off.shape[0] != n + 1 or self.density.shape[0] != n or self.sh.shape[0] != n:
            raise ValueError("scene arrays disagree on the number of sites")
        self.surface = surface
        self._c = _Scene(_ptr(self.sites), _ptr(self.off), _ptr(self.idx), _ptr(self.density), _ptr(self.sh),
                         n, self.sh_deg, ctypes.pointer(surface._c) if surface is not None else None)

    @classmethod
    def from_scene(cls, scene, density=None, sh=None, surface: Optional[Surface] = None) -> "OracleScene":
        return cls(scene.sites, scene.off, scene.idx, scene.density if density is None else density,
                   scene.sh if sh is None else sh, scene.sh_deg, surface)

    @property
    def n_sites(self) -> int:
        return self.sites.shape[0]

    @property
    def B(self) -> int:
        return (self.sh_deg + 1) ** 2


def sh_basis(deg: int, dirs) -> np.ndarray:
    """Real SH basis [n, (deg+1)^2] of unit directions [n, 3]."""
    d = _f64(dirs).reshape(-1, 3)
    out = np.empty((d.shape[0], (deg + 1) ** 2))
    _check(_load().orc_sh_basis(deg, _ptr(d), d.shape[0], _ptr(out)), "sh_basis")
    return out


CAMERA_MODELS = {"pinhole": 0, "fisheye": 1}


def raygen(pose12, fov_deg: float, width: int, height: int, bound: tuple, model: str = "pinhole"):
    """Camera rays (pinhole, or equidistant fisheye) in 8x8 tile order. Returns (origin, dir, tmax, pixel)."""
    pose = _f64(pose12).reshape(12)
    kind, params = encode_bound(bound)
    R = width * height
    o = np.empty((R, 3))
    d = np.empty((R, 3))
    t = np.empty(R)
    px = np.empty(R, dtype=np.int32)
    _check(_load().orc_raygen(_ptr(pose), float(fov_deg), int(width), int(height), CAMERA_MODELS[model], kind,
                              _ptr(params),
                              _ptr(o), _ptr(d), _ptr(t), _ptr(px)), "raygen")
    return o, d, t, px


def encode_bound(bound: tuple):
    if bound[0] == "box":
        lo, hi = bound[1], bound[2]
        lo = np.broadcast_to(np.asarray(lo, dtype=np.float64), (3,))
        hi = np.broadcast_to(np.asarray(hi, dtype=np.float64), (3,))
        return 0, _f64(np.concatenate([lo, hi]))
    if bound[0] == "sphere":
        return 1, _f64([bound[1], 0, 0, 0, 0, 0])
    raise ValueError(bound)


def face_planes(sites, off, idx) -> np.ndarray:
    """[E, 4] planes (n = x_j - x_i, c = n.(x_i + x_j)/2) in float64."""
    s = _f64(sites).reshape(-1, 3)
    o = _i32(off)
    i = _i32(idx)
    out = np.empty((i.shape[0], 4))
    _check(_load().orc_face_planes(_ptr(s), _ptr(o), _ptr(i), s.shape[0], _ptr(out)), "face_planes")
    return out


def nearest_site(sites, points, return_gap: bool = False):
    """Index of each point's nearest site (eq. (5)) by exhaustive FP64 search,
    lowest index on exact ties; with ``return_gap`` also the runner-up's
    relative squared-distance gap."""
    s = _f64(sites).reshape(-1, 3)
    p = _f64(points).reshape(-1, 3)
    out = np.empty(len(p), dtype=np.int32)
    gap = np.empty(len(p), dtype=np.float64)
    _check(_load().orc_nearest_site(_ptr(s), len(s), _ptr(p), len(p), _ptr(out), _ptr(gap)), "nearest_site")
    return (out, gap) if return_gap else out


def bf16_round(x) -> np.ndarray:
    """float32 -> bfloat16 bit patterns (uint16), round to nearest even."""
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    out = np.empty(a.shape, dtype=np.uint16)
    _load().orc_bf16_round(_ptr(a), _ptr(out), a.size)
    return out


def bf16_to_f32(bits) -> np.ndarray:
    """Exact widening of bfloat16 bit patterns to float32."""
    b = np.asarray(bits, dtype=np.uint16).astype(np.uint32) << 16
    return b.view(np.float32)


def check_csr(off, idx, n_sites: int) -> bool:
    o = _i32(off)
    i = _i32(idx)
    return _load().orc_check_csr(_ptr(o), _ptr(i), int(n_sites), i.shape[0]) == 0


def _rays(o, d, tmax, start):
    o = _f64(o).reshape(-1, 3)
    d = _f64(d).reshape(-1, 3)
    R = d.shape[0]
    o = np.ascontiguousarray(np.broadcast_to(o, (R, 3)))
    t = np.ascontiguousarray(np.broadcast_to(_f64(tmax).reshape(-1), (R,)))
    s = np.ascontiguousarray(np.broadcast_to(_i32(start).reshape(-1), (R,)))
    return o, d, t, s, R


def forward(scene: OracleScene, o, d, tmax, start, eps: float = DEFAULT_EPS,
            max_steps: int = DEFAULT_MAX_STEPS, threads: Optional[int] = None):
    """Composited colour [R,3], final transmittance [R], status/visit count [R]."""
    o, d, t, s, R = _rays(o, d, tmax, start)
    rgb = np.empty((R, 3))
    tf = np.empty(R)
    steps = np.empty(R, dtype=np.int32)
    _check(_load().orc_forward(ctypes.byref(scene._c), _ptr(o), _ptr(d), _ptr(t), _ptr(s), R, float(eps),
                               int(max_steps), threads or default_threads(), _ptr(rgb), _ptr(tf), _ptr(steps)),
           "forward")
    return rgb, tf, steps


def trace(scene: OracleScene, o, d, tmax, start, eps: float = DEFAULT_EPS,
          max_steps: int = DEFAULT_MAX_STEPS, max_len: int = 1024, threads: Optional[int] = None,
          legs: bool = False) -> dict:
    """Forward plus per-visit cells, exit distances (along each visit's leg), decision margins,
    per-visit surface crossings (``bounce``), the surface decisions' margin (``surf_margin``) and the
    smallest |cos| of an exit face whose exit moves (``exit_cos``);
    with ``legs`` also each visit's leg origin and direction [R, max_len, 6]."""
    o, d, t, s, R = _rays(o, d, tmax, start)
    out = dict(rgb=np.empty((R, 3)), t_final=np.empty(R), steps=np.empty(R, dtype=np.int32),
               cells=np.full((R, max_len), -1, dtype=np.int32), t_exit=np.full((R, max_len), np.nan),
               len=np.empty(R, dtype=np.int32), margin=np.empty(R), graze=np.empty(R), term=np.empty(R),
               bounce=np.zeros((R, max_len), dtype=np.int8), surf_margin=np.empty(R), exit_cos=np.empty(R))
    if legs:
        out["legs"] = np.full((R, max_len, 6), np.nan)
    _check(_load().orc_trace(ctypes.byref(scene._c), _ptr(o), _ptr(d), _ptr(t), _ptr(s), R, float(eps),
                             int(max_steps), int(max_len), threads or default_threads(),
                             *[_ptr(out.get(k)) for k in ("rgb", "t_final", "steps", "cells", "t_exit", "len",
                                                          "margin", "graze", "term", "bounce", "legs",
                                                          "surf_margin", "exit_cos")]), "trace")
    return out


def backward(scene: OracleScene, o, d, tmax, start, grad_rgb, grad_t=None, eps: float = DEFAULT_EPS,
             max_steps: int = DEFAULT_MAX_STEPS, threads: Optional[int] = None, forced=None):
    """Gradients (sites [N,3], density [N], sh [N,B,3]) of sum(grad_rgb*rgb) + sum(grad_t*T).

    ``forced`` (optional): per ray a list of (visit, choice) pairs in walk
    order (see ``walk_forced``); each ray then walks with those choices."""
    o, d, t, s, R = _rays(o, d, tmax, start)
    f_off = f_visit = f_choice = None
    if forced is not None:
        if len(forced) != R:
            raise ValueError("forced needs one list per ray")
        f_off, f_visit, f_choice = _pack_forced(forced)
    g = _f64(grad_rgb).reshape(R, 3)
    gt = None if grad_t is None else _f64(grad_t).reshape(R)
    n = scene.n_sites
    gs = np.zeros((n, 3))
    gd = np.zeros(n)
    gsh = np.zeros((n, scene.B, 3))
    _check(_load().orc_backward(ctypes.byref(scene._c), _ptr(o), _ptr(d), _ptr(t), _ptr(s), R, float(eps),
                                int(max_steps), _ptr(g), _ptr(gt), threads or default_threads(),
                                _ptr(gs), _ptr(gd), _ptr(gsh), _ptr(f_off), _ptr(f_visit), _ptr(f_choice)),
           "backward")
    return gs, gd, gsh


# Choice codes of a decision (besides a neighbour id: leave through the face to it).
CH_CLIP = -3  # the ray ends in this cell at t_max
CH_STOP = -4  # the transmittance test before the visit fails
CH_GO = -5    # the transmittance test before the visit passes


def _pack_forced(forced):
    f_off = np.zeros(len(forced) + 1, dtype=np.int64)
    f_off[1:] = np.cumsum([len(f) for f in forced])
    flat = [c for f in forced for c in f]
    f_visit = np.ascontiguousarray(np.array([v for v, _ in flat] or [0], dtype=np.int32))
    f_choice = np.ascontiguousarray(np.array([c for _, c in flat] or [0], dtype=np.int32))
    return f_off, f_visit, f_choice


def walk_forced(scene: OracleScene, o, d, tmax, start, ray_idx, forced, eps: float = DEFAULT_EPS,
                max_steps: int = DEFAULT_MAX_STEPS, kappa_t: float = 0.0, kappa_T: float = 0.0,
                max_len: int = 1024, nt_cap: int = 16, threads: Optional[int] = None) -> dict:
    """Walks of rays ``ray_idx`` (jobs) with the forced choices ``forced`` (per
    job a list of (visit, choice) in walk order; a decision is the
    transmittance test before visit n, choice CH_STOP or CH_GO, or the exit of
    visit n, a neighbour id or CH_CLIP). Returns per job the colour,
    transmittance, status, cells, visit count, and the near ties after its
    last forced decision: decisions whose exact winner is within kappa_t
    (faces and t_max, in the decision-margin units of ``trace``) or kappa_T
    (|ln T - ln eps|) of an alternative, as (visit, alternative choice) pairs
    (``nt_len`` -1: more than ``nt_cap``); ``bad`` flags a forced choice that
    was not available."""
    o, d, t, s, R = _rays(o, d, tmax, start)
    idx = np.ascontiguousarray(np.asarray(ray_idx, dtype=np.int32))
    J = len(idx)
    f_off, f_visit, f_choice = _pack_forced(forced)
    out = dict(rgb=np.empty((J, 3)), t_final=np.empty(J), steps=np.empty(J, dtype=np.int32),
               cells=np.full((J, max_len), -1, dtype=np.int32), len=np.empty(J, dtype=np.int32),
               nt_visit=np.zeros((J, max(nt_cap, 1)), dtype=np.int32),
               nt_choice=np.zeros((J, max(nt_cap, 1)), dtype=np.int32), nt_len=np.empty(J, dtype=np.int32),
               bad=np.empty(J, dtype=np.int32))
    _check(_load().orc_walk_forced(ctypes.byref(scene._c), _ptr(o), _ptr(d), _ptr(t), _ptr(s), R, _ptr(idx), J,
                                   _ptr(f_off), _ptr(f_visit), _ptr(f_choice), float(eps), int(max_steps),
                                   float(kappa_t), float(kappa_T), int(max_len), int(nt_cap),
                                   threads or default_threads(),
                                   *[_ptr(out[k]) for k in ("rgb", "t_final", "steps", "cells", "len", "nt_visit",
                                                            "nt_choice", "nt_len", "bad")]), "walk_forced")
    return out


def alternatives(scene: OracleScene, o, d, tmax, start, ray_idx, kappa_t: float, kappa_T: float,
                 eps: float = DEFAULT_EPS, max_steps: int = DEFAULT_MAX_STEPS, max_len: int = 1024,
                 max_leaves: int = 32, threads: Optional[int] = None) -> dict:
    """Every walk of rays ``ray_idx`` that takes, at each near tie (see
    ``walk_forced``), the exact winner or one of its near alternatives: the
    walks a computation whose face and transmittance decisions err only
    within kappa_t / kappa_T may produce. Searched level by level (walks with
    k forced choices, then k + 1); a ray with more than ``max_leaves`` such
    walks, or with more near ties on one walk than can be listed, is marked
    ``complete`` False. Returns per ray a list of leaves, each a dict (forced,
    cells, len, rgb, t_final, steps), the exact walk first."""
    idx = np.asarray(ray_idx, dtype=np.int64)
    leaves = [[] for _ in idx]
    complete = np.ones(len(idx), dtype=bool)
    pending = [(q, []) for q in range(len(idx))]
    while pending:
        jobs = [q for q, _ in pending]
        forced = [f for _, f in pending]
        w = walk_forced(scene, o, d, tmax, start, idx[jobs], forced, eps=eps, max_steps=max_steps, kappa_t=kappa_t,
                        kappa_T=kappa_T, max_len=max_len, nt_cap=16, threads=threads)
        nxt = []
        for k, (q, f) in enumerate(pending):
            if w["bad"][k]:
                complete[q] = False
                continue
            L = int(w["len"][k])
            leaves[q].append(dict(forced=f, cells=w["cells"][k, :min(L, max_len)].copy(), len=L,
                                  rgb=w["rgb"][k].copy(), t_final=float(w["t_final"][k]), steps=int(w["steps"][k])))
            n_nt = int(w["nt_len"][k])
            if n_nt < 0 or L > max_len:
                complete[q] = False
                continue
            for m in range(n_nt):
                nxt.append((q, f + [(int(w["nt_visit"][k, m]), int(w["nt_choice"][k, m]))]))
        pending = []
        queued = {}
        for q, f in nxt:
            if len(leaves[q]) + queued.get(q, 0) >= max_leaves:
                complete[q] = False
                continue
            queued[q] = queued.get(q, 0) + 1
            pending.append((q, f))
    return dict(leaves=leaves, complete=complete)


def quantile(scene: OracleScene, o, d, tmax, start, u, grad_loss=None, eps: float = DEFAULT_EPS,
             max_steps: int = DEFAULT_MAX_STEPS, threads: Optional[int] = None):
    """Quantile regulariser (Sec. 3.4): per ray, the quantiles W^-1(u1), W^-1(u2) [R,2] of the
    normalised weight distribution along the walk and the loss |W^-1(u1) - W^-1(u2)| [R]; with
    ``grad_loss`` [R] also the gradients (sites [N,3], density [N]) of sum(grad_loss * loss)."""
    o, d, t, s, R = _rays(o, d, tmax, start)
    uu = np.ascontiguousarray(_f64(u).reshape(R, 2))
    gl = None if grad_loss is None else np.ascontiguousarray(_f64(grad_loss).reshape(R))
    tq = np.empty((R, 2))
    loss = np.empty(R)
    n = scene.n_sites
    gs = np.zeros((n, 3)) if gl is not None else None
    gd = np.zeros(n) if gl is not None else None
    _check(_load().orc_quantile(ctypes.byref(scene._c), _ptr(o), _ptr(d), _ptr(t), _ptr(s), R, float(eps),
                                int(max_steps), _ptr(uu), _ptr(gl), threads or default_threads(), _ptr(tq),
                                _ptr(loss), _ptr(gs), _ptr(gd)), "quantile")
    return (tq, loss) if gl is None else (tq, loss, gs, gd)
