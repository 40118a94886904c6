"""Continuous-batching render server (binding of the rf_server_* C ABI) and a
request loop that replays a timed stream of render requests.

The server keeps a packed scene resident; its scheduler thread builds each
kernel launch from the pending 8x8 tiles of every admitted request, so
requests admitted while others are on the GPU share launches with them.
Requests are admitted whenever a slot and output-pool memory are free.
"""

from __future__ import annotations

import collections
import ctypes
import time
from typing import Dict, List, Optional, Sequence

import numpy as np

from . import _lib as L
from .ops import PackedScene, bound_desc, camera_desc


class Server:
    """A running server. Use as a context manager or call ``close()``."""

    MODES = {"launches": 0, "persistent": 1}

    def __init__(self, scene: PackedScene, bound: tuple, pool_bytes: int = 1 << 30, max_inflight: int = 32,
                 eps: float = 1e-4, max_steps: int = 8192, mode: str = "launches"):
        """``mode="persistent"``: one persistent kernel serves requests as they
        arrive (``RF_SERVE_PERSISTENT``); ``"launches"``: batched launches."""
        self.scene = scene  # keeps the packed workspace alive
        self._h = ctypes.c_void_p()
        p = L.Params(float(eps), int(max_steps))
        b = bound_desc(bound)
        L.check(L.lib().rf_server_create_mode(ctypes.byref(scene.desc), ctypes.byref(p), ctypes.byref(b),
                                              int(pool_bytes), int(max_inflight), self.MODES[mode],
                                              ctypes.byref(self._h)))
        self.mode = mode
        self.max_inflight = int(max_inflight)
        self._ids = (ctypes.c_uint64 * self.max_inflight)()
        self.sizes: Dict[int, tuple] = {}

    def submit(self, pose12, fov_deg: float, width: int, height: int, start_cell: int,
               model: str = "pinhole") -> Optional[int]:
        """Request id, or None if not admissible now (no free slot or pool space)."""
        cam = camera_desc(pose12, fov_deg, width, height, model)
        rid = ctypes.c_uint64()
        st = L.lib().rf_server_submit(self._h, ctypes.byref(cam), int(start_cell), ctypes.byref(rid))
        if st == L.RF_ERR_BUSY:
            return None
        L.check(st)
        self.sizes[int(rid.value)] = (int(height), int(width))
        return int(rid.value)

    def poll(self) -> List[int]:
        n = ctypes.c_int32()
        L.check(L.lib().rf_server_poll(self._h, self._ids, self.max_inflight, ctypes.byref(n)))
        return [int(self._ids[k]) for k in range(n.value)]

    def result(self, rid: int, copy: bool = True) -> Optional[np.ndarray]:
        """RGBA float32 image [H, W, 4] (RGB, final transmittance); frees the request's slot."""
        h, w = self.sizes.pop(rid)
        out = np.empty((h, w, 4), dtype=np.float32) if copy else None
        L.check(L.lib().rf_server_result(self._h, ctypes.c_uint64(rid),
                                         None if out is None else out.ctypes.data,
                                         0 if out is None else out.nbytes))
        return out

    def stats(self) -> dict:
        s = L.ServerStats()
        L.check(L.lib().rf_server_stats_get(self._h, ctypes.byref(s)))
        return {k: getattr(s, k) for k, _ in s._fields_}

    def close(self) -> None:
        if self._h:
            st = L.lib().rf_server_destroy(self._h)
            self._h = ctypes.c_void_p()
            L.check(st)

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def replay(server: Server, requests: Sequence[dict], keep: Sequence[int] = (), time_scale: float = 1.0,
           timeout_s: float = 120.0) -> dict:
    """Replays timed requests through ``server`` in arrival order (FIFO admission).

    Each request is a dict with ``arrival`` (seconds from the start), ``pose12``,
    ``fov_deg``, ``width``, ``height`` and ``start_cell``. A request enters the
    queue at its arrival time; the head of the queue is submitted as soon as the
    server admits it. Latency is arrival -> completion observed by the host
    (polling; requests that finish together are observed together, and new
    arrivals are submitted before their images are copied out); the copy-out
    of the image is timed separately. Returns latencies,
    throughput and the images of the requests whose indices are in ``keep``.
    """
    n = len(requests)
    keep = set(keep)
    order = np.argsort([r["arrival"] for r in requests], kind="stable")
    queue: collections.deque = collections.deque()
    rid_of: Dict[int, int] = {}
    latency = np.full(n, np.nan)
    copy_ms = np.full(n, np.nan)
    admitted_at = np.full(n, np.nan)
    images: Dict[int, np.ndarray] = {}
    nxt = 0
    done = 0
    rays = 0
    t0 = time.perf_counter()

    def admit() -> None:
        # arrivals join the queue; its head is submitted while the server admits it
        nonlocal nxt
        now = time.perf_counter() - t0
        while nxt < n and requests[order[nxt]]["arrival"] * time_scale <= now:
            queue.append(int(order[nxt]))
            nxt += 1
        while queue:
            i = queue[0]
            r = requests[i]
            rid = server.submit(r["pose12"], r["fov_deg"], r["width"], r["height"], r["start_cell"],
                                r.get("model", "pinhole"))
            if rid is None:
                break
            queue.popleft()
            rid_of[rid] = i
            admitted_at[i] = time.perf_counter() - t0

    while done < n:
        if time.perf_counter() - t0 > timeout_s:
            raise TimeoutError(f"replay: {done}/{n} requests finished after {timeout_s} s")
        admit()
        finished = server.poll()
        if finished:
            # completions are observed together; new arrivals are submitted
            # before the copies out, so that no copy holds the GPU's next work
            t_done = time.perf_counter() - t0
            for rid in finished:
                i = rid_of[rid]
                latency[i] = t_done - requests[i]["arrival"] * time_scale
            admit()
            for rid in finished:
                i = rid_of.pop(rid)
                a = time.perf_counter()
                img = server.result(rid, copy=True)
                copy_ms[i] = (time.perf_counter() - a) * 1e3
                if i in keep:
                    images[i] = img
                rays += requests[i]["width"] * requests[i]["height"]
                done += 1
                admit()
        elif queue:
            time.sleep(5e-5)  # the head waits for a slot or pool space
        if not queue and nxt < n:
            wait = requests[order[nxt]]["arrival"] * time_scale - (time.perf_counter() - t0)
            if wait > 2e-4:
                time.sleep(min(wait, 1e-3))
    span = time.perf_counter() - t0
    first = min(r["arrival"] for r in requests) * time_scale
    return {
        "latency_s": latency,
        "copy_ms": copy_ms,
        "queue_s": admitted_at - np.array([r["arrival"] * time_scale for r in requests]),
        "p50_ms": float(np.percentile(latency, 50) * 1e3),
        "p99_ms": float(np.percentile(latency, 99) * 1e3),
        "mean_ms": float(np.mean(latency) * 1e3),
        "rays": int(rays),
        "span_s": span - first,
        "mrays_per_s": rays / (span - first) / 1e6,
        "images": images,
    }
