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
import queue
import threading
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

    def result(self, rid: int, copy: bool = True, out: Optional[np.ndarray] = None) -> Optional[np.ndarray]:
        """RGBA float32 image [H, W, 4] (RGB, final transmittance), into ``out``
        if given (C-contiguous float32 of that shape); frees the request's slot.
        May run on another thread than submit and poll (the copy does not hold
        the server's lock)."""
        h, w = self.sizes[rid]
        if out is not None:
            if out.dtype != np.float32 or out.shape != (h, w, 4) or not out.flags.c_contiguous:
                raise ValueError(f"out must be a C-contiguous float32 array of shape {(h, w, 4)}")
        elif copy:
            out = np.empty((h, w, 4), dtype=np.float32)
        L.check(L.lib().rf_server_result(self._h, ctypes.c_uint64(rid),
                                         None if out is None else out.ctypes.data,
                                         0 if out is None else out.nbytes))
        self.sizes.pop(rid, None)
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
    server admits it. Latency is arrival -> completion observed by the polling
    thread (requests that finish together are observed together). A collector
    thread copies finished images out of the server's pool, which frees their
    slots and pool space for admission: into one reused buffer per image size
    (as a front end that hands images on would), or into a new array for the
    requests whose indices are in ``keep``; the copy-out is timed separately.
    Returns latencies, throughput and the kept images.
    """
    n = len(requests)
    keep = set(keep)
    order = np.argsort([r["arrival"] for r in requests], kind="stable")
    waiting: collections.deque = collections.deque()
    rid_of: Dict[int, int] = {}
    latency = np.full(n, np.nan)
    copy_ms = np.full(n, np.nan)
    admitted_at = np.full(n, np.nan)
    images: Dict[int, np.ndarray] = {}
    seen: set = set()
    nxt = 0
    t0 = time.perf_counter()
    to_collect: "queue.Queue" = queue.Queue()
    state = {"collected": 0, "rays": 0, "error": None}
    buffers: Dict[tuple, np.ndarray] = {}

    def collector() -> None:
        while True:
            item = to_collect.get()
            if item is None:
                return
            rid, i = item
            r = requests[i]
            shape = (r["height"], r["width"], 4)
            try:
                out = np.empty(shape, np.float32) if i in keep else buffers.setdefault(shape, np.empty(shape, np.float32))
                a = time.perf_counter()
                server.result(rid, out=out)
                copy_ms[i] = (time.perf_counter() - a) * 1e3
            except Exception as e:  # reported by the polling thread
                state["error"] = e
                return
            if i in keep:
                images[i] = out
            state["rays"] += r["width"] * r["height"]
            state["collected"] += 1

    def admit() -> None:
        # arrivals join the queue; its head is submitted while the server admits it
        nonlocal nxt
        now = time.perf_counter() - t0
        while nxt < n and requests[order[nxt]]["arrival"] * time_scale <= now:
            waiting.append(int(order[nxt]))
            nxt += 1
        while waiting:
            i = waiting[0]
            r = requests[i]
            rid = server.submit(r["pose12"], r["fov_deg"], r["width"], r["height"], r["start_cell"],
                                r.get("model", "pinhole"))
            if rid is None:
                break
            waiting.popleft()
            rid_of[rid] = i
            admitted_at[i] = time.perf_counter() - t0

    th = threading.Thread(target=collector, name="replay-collector", daemon=True)
    th.start()
    try:
        while state["collected"] < n:
            if state["error"] is not None:
                raise state["error"]
            if time.perf_counter() - t0 > timeout_s:
                raise TimeoutError(f"replay: {state['collected']}/{n} requests finished after {timeout_s} s")
            admit()
            # finished requests stay listed until the collector has taken them
            new = [rid for rid in server.poll() if rid not in seen]
            if new:
                t_done = time.perf_counter() - t0
                for rid in new:
                    seen.add(rid)
                    i = rid_of[rid]
                    latency[i] = t_done - requests[i]["arrival"] * time_scale
                    to_collect.put((rid, i))
                admit()
                continue
            if waiting or len(seen) == n or len(seen) > state["collected"]:
                time.sleep(5e-5)  # the head waits for a slot or pool space, or the collector is copying
            elif nxt < n:
                wait = requests[order[nxt]]["arrival"] * time_scale - (time.perf_counter() - t0)
                if wait > 2e-4:
                    time.sleep(min(wait, 1e-3))
    finally:
        to_collect.put(None)
        th.join(timeout=60.0)
    span = time.perf_counter() - t0
    first = min(r["arrival"] for r in requests) * time_scale
    return {
        "latency_s": latency,
        "copy_ms": copy_ms,
        "queue_s": admitted_at - np.array([r["arrival"] * time_scale for r in requests]),
        "p50_ms": float(np.percentile(latency, 50) * 1e3),
        "p99_ms": float(np.percentile(latency, 99) * 1e3),
        "mean_ms": float(np.mean(latency) * 1e3),
        "rays": int(state["rays"]),
        "span_s": span - first,
        "mrays_per_s": state["rays"] / (span - first) / 1e6,
        "images": images,
    }
