"""Benchmark of the Voronoi ray walk on one MI355X.

Workload (default): 1M sites from 64 thin anisotropic Gaussian clusters plus
10 % uniform background in [-1,1]^3, SH degree 3, one 1920x1080 camera on an
orbit of radius 0.8, forward + backward with per-pixel N(0,1) upstream
gradients. One step is the whole hot path on one batch:
camera rays (8x8 tiles) -> scene pack (face planes + cell records) ->
forward walk -> backward walk (gradients for sites, density, SH; the backward
recomputes each walk from the saved colour and transmittance). With
--config shell_3m a batch is the rays of all eight cameras, one pack per step.

Prints ONE JSON line. `value` is forward+backward Mrays/s with FP32 attributes;
forward-only and BF16-attribute rates, the training step whose backward reads
a walk log, per-kernel times, step-latency percentiles, the HBM roofline of
every walk kernel (rocprofv3 DRAM bytes over the HIP-event duration) with its
vector-ALU companion, and the FP64 CPU oracle's rate on a bounded sample of
the same workload are added fields.

Usage: python bench.py [--gpus 1] [--steps 20] [--warmup 5] [--config clustered_1m]
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X published FP32 vector peak (packed FP32), and the rate without packed
# math (256 CUs x 64 FMA lanes x 2 flops x 2.4 GHz), which is what this build
# can issue: packed FP32 instructions are disabled.
FP32_PEAK_TFLOPS = 157.3
VALU_PEAK_TFLOPS = 256 * 64 * 2 * 2.4e9 / 1e12
HBM_PEAK_GBS = 8000.0


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


WALK_SOURCES = ("walk.hip", "rf_walk.hpp", "rf_device.hpp", "rf_kernels.hpp")


def kernel_source_digest() -> str:
    """Digest of the sources the walk kernels are built from; HBM traffic figures
    are only valid for the digest they were taken on."""
    h = hashlib.sha1()
    for name in WALK_SOURCES:
        with open(os.path.join(ROOT, "paper_2502_01157_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:12]


def measured_traffic(workload: str, dtype: str, label: str):
    """HBM bytes per launch (read + written) of the launch `label` (e.g.
    "backward (recomputing)") with `dtype` attributes, from the committed
    rocprofv3 PMC summary of `workload`, or None if there is none for these
    kernel sources."""
    path = os.path.join(ROOT, "profiles", f"walk_kernels_{workload}_hbm_traffic.md")
    if not label or not os.path.exists(path):
        return None
    text = open(path).read()
    m = re.search(r"kernel source digest: ([0-9a-f]+)", text)
    if not m or m.group(1) != kernel_source_digest():
        return None
    kernel, _, rest = label.partition(" ")
    rest = rest.strip("()") or kernel
    m = re.search(rf"^\| k_{kernel} \| {re.escape(rest)} \| {dtype} \| \d+ \| [0-9.]+ \| [0-9.]+ \| ([0-9.]+) \| "
                  rf"([0-9.]+) \|", text, re.M)
    if not m:
        return None
    return int(round((float(m.group(1)) + float(m.group(2))) * 1e6))


def site_count(n: int) -> str:
    """1M, 3M, 200k or the count itself."""
    if n % 1_000_000 == 0:
        return f"{n // 1_000_000}M"
    if n % 1_000 == 0:
        return f"{n // 1_000}k"
    return f"{n:,}"


def visit_bytes(mean_deg: float, B: int, dt: str, kind: str = "forward") -> float:
    """Bytes the method touches per visited cell, with no reuse: its row offsets
    (4), neighbour ids (4 per face) and positions (12 per face), and its SH and
    density. A backward adds the cell's gradient package before any reduction
    ((3B + 1 + 3) floats, read-modify-write counted once); the backward that
    reads the walk log reads 12 B of log and the site (12 B) instead of the faces."""
    attr = (3 * B + 1) * (2 if dt == "bf16" else 4)
    scan = 4 + 16 * mean_deg
    grad = 4 * (3 * B + 4)
    return {"forward": scan + attr, "backward_recompute": scan + attr + grad,
            "backward": 12 + 12 + attr + grad}[kind]


def flops_per_visit(mean_deg: float, B: int, kernel: str) -> float:
    """Arithmetic the walk itself requires per visited cell (FMA = 2 flops).

    Forward: per face den = n.d (5), num = c - n.o (6) and the nearest-face
    compare (2); per cell the colour sum_b k_b Y_b (2 per coefficient, 3B
    coefficients) and the compositing update (12). The backward adds the
    transmittance derivative (14), the per-cell SH/density gradient
    (2 x 3B + 2) and the two site gradients of the exit face (20); a backward
    that reads the visits from the forward's log does no face tests, one that
    recomputes the walk does them again.
    """
    scan = 13.0 * mean_deg
    cell = 6.0 * B + 12.0
    grad = 14.0 + 6.0 * B + 2.0 + 20.0
    return {"forward": scan + cell, "backward": cell + grad, "backward_recompute": scan + cell + grad}[kernel]


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--config", default="clustered_1m", choices=["uniform_4k", "clustered_200k", "clustered_1m", "shell_3m"])
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="target CPU time of the oracle sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--mode", type=int, default=0, help="backward reduction mode (0 wave-reduced, 1 per-lane)")
    ap.add_argument("--log-capacity", type=int, default=256,
                    help="visits per ray kept in the walk log of the logged training step")
    ap.add_argument("--only", choices=["f32", "bf16"], default=None, help="time one attribute precision only")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving replay (512 Poisson requests)")
    ap.add_argument("--no-locate", action="store_true", help="skip the start-cell location timing")
    ap.add_argument("--no-quantile", action="store_true", help="skip the quantile regulariser timing")
    ap.add_argument("--no-effects", action="store_true", help="skip the secondary-ray and fisheye timing")
    ap.add_argument("--no-training", action="store_true", help="skip the optimizer / densification timing")
    ap.add_argument("--no-log-compare", action="store_true",
                    help="skip timing the training step whose backward reads a walk log")
    ap.add_argument("--extras-only", action="store_true",
                    help="time only the headline step once (no BF16, no forward-only or logged forms) before the "
                         "added measurements (serving, location, ...); for profiling those")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 1 GiB device copy (reference for HBM byte counters)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on exactly one GPU: the walk is measured on one GPU's share "
              "(multi-GPU sharding is described in the design notes, not run)", file=sys.stderr)
        return 2

    import torch

    import paper_2502_01157_amd as rf
    import synth
    from synth.scenes import CONFIGS

    cfg = CONFIGS[args.config]
    t0 = time.time()
    scene, rng = synth.make_scene(args.config, return_rng=True)
    cams = synth.make_cameras(args.config, rng)
    cam = cams[0]
    R = sum(c.width * c.height for c in cams)
    g_np = synth.make_upstream_grads(rng, R)
    starts = [int(x) for x in synth.nearest_site(scene.sites, np.stack([c.position for c in cams]))]
    start = starts[0]
    log(f"scene {args.config}: {scene.n_sites} sites, {scene.n_edges} directed edges, "
        f"{len(cams)} camera(s), {R} rays per step, built in {time.time() - t0:.1f}s")

    dev = torch.device("cuda:0")

    def dv(a):
        return torch.from_numpy(np.ascontiguousarray(a)).to(dev)

    sites, off, idx, dens, sh = map(dv, (scene.sites, scene.off, scene.idx, scene.density, scene.sh))
    grad_rgb = dv(g_np)
    B = (scene.sh_deg + 1) ** 2
    bound = cfg["bound"]

    scenes = {dt: rf.PackedScene(sites, off, idx, dens, sh, scene.sh_deg, dt, validate=True)
              for dt in ("f32", "bf16")}
    grads = (torch.zeros((scene.n_sites, 3), device=dev), torch.zeros(scene.n_sites, device=dev),
             torch.zeros((scene.n_sites, B, 3), device=dev))
    # one batch: the rays of every camera of the workload, camera after camera
    rays = (torch.empty((R, 3), device=dev), torch.empty((R, 3), device=dev), torch.empty(R, device=dev),
            torch.empty(R, dtype=torch.int32, device=dev))
    cam_rows = np.concatenate([[0], np.cumsum([c.width * c.height for c in cams])])

    def raygen_all():
        for c, st, a, b in zip(cams, starts, cam_rows[:-1], cam_rows[1:]):
            rf.raygen(c.pose12(), c.fov_deg, c.width, c.height, bound, st, device=dev, with_pixel=False,
                      out=tuple(x[a:b] for x in rays))
        return rays

    raygen_all()
    fwd_out = (torch.empty((R, 3), device=dev), torch.empty(R, device=dev),
               torch.empty(R, dtype=torch.int32, device=dev))
    walk_log = None if args.no_log_compare else rf.WalkLog(R, args.log_capacity, dev)
    ev = {k: (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for k in ("raygen", "pack", "forward", "backward")}

    def step(dt: str, backward: bool, timed: dict = None, use_log: bool = False):
        def mark(k, i):
            if timed is not None:
                ev[k][i].record()

        mark("raygen", 0)
        o, d, t, s = raygen_all()
        mark("raygen", 1)
        mark("pack", 0)
        scenes[dt].pack(sites, dens, sh)
        mark("pack", 1)
        mark("forward", 0)
        # the logged form's forward keeps the walk log for its backward
        log = walk_log if backward and use_log else None
        rgb, tf, steps = rf.render_forward(scenes[dt], o, d, t, s, out=fwd_out, log=log)
        mark("forward", 1)
        if backward:
            for gbuf in grads:
                gbuf.zero_()
            mark("backward", 0)
            rf.render_backward(scenes[dt], o, d, t, s, rgb, tf, grad_rgb, None, mode=args.mode, grads=grads,
                               log=log)
            mark("backward", 1)
        if timed is not None:
            torch.cuda.synchronize()
            for k in ev:
                if k == "backward" and not backward:
                    continue
                timed.setdefault(k, []).append(ev[k][0].elapsed_time(ev[k][1]))

    def run(dt: str, backward: bool, use_log: bool = False):
        for _ in range(args.warmup):
            step(dt, backward, use_log=use_log)
        torch.cuda.synchronize()
        # whole-job throughput: K steps bracketed by synchronisation
        t_start = time.perf_counter()
        for _ in range(args.steps):
            step(dt, backward, use_log=use_log)
        torch.cuda.synchronize()
        total = time.perf_counter() - t_start
        # per-kernel and per-step latency: the same steps again with events
        timed, lat = {}, []
        for _ in range(args.steps):
            a = time.perf_counter()
            step(dt, backward, timed, use_log=use_log)
            lat.append((time.perf_counter() - a) * 1e3)
        return total / args.steps * 1e3, {k: float(np.mean(v)) for k, v in timed.items()}, lat

    # visits per batch (the work unit of the walk)
    o, d, t, s = rays
    _, _, steps_fp32 = rf.render_forward(scenes["f32"], o, d, t, s)
    torch.cuda.synchronize()
    steps_np = steps_fp32.cpu().numpy()
    visits = int(np.clip(steps_np, 0, None).sum())
    # mean degree of visited cells, from a traced sample of tiles
    mid = min(R // 2, cam_rows[1] // 2)
    sample = slice(max(mid - 8192, 0), min(mid + 8192, R))
    tr = rf.render_trace(scenes["f32"], o[sample].contiguous(), d[sample].contiguous(), t[sample].contiguous(),
                         s[sample].contiguous(), max_len=1024)
    cells = tr["cells"].cpu().numpy()
    cells = cells[cells >= 0]
    deg = np.diff(scene.off)
    mean_deg = float(deg[cells].mean())
    log(f"visits/batch {visits} ({visits / R:.1f} per ray), mean visited degree {mean_deg:.2f}, "
        f"flagged rays {(steps_np < 0).sum()}")

    if args.copy_calibration:
        src = torch.empty(1 << 28, dtype=torch.float32, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log("copy calibration: 1 GiB read + 1 GiB written by one device copy kernel")
        del src, dst

    # forms of the step: the training step with the recomputing backward (the
    # headline), the forward alone, and the training step whose forward keeps
    # a walk log that its backward reads
    forms = [("fwd_bwd", True, False), ("fwd", False, False)]
    if walk_log is not None:
        forms.append(("fwd_bwd_logged", True, True))
    if args.extras_only:
        forms = [("fwd_bwd", True, False), ("fwd", False, False)]
        args.only = args.only or "f32"
    results = {}
    for dt in (("f32", "bf16") if args.only is None else (args.only,)):
        for form, bwd, use_log in forms:
            ms, kern, lat = run(dt, bwd, use_log)
            results[(dt, form)] = (ms, kern, lat)
            log(f"{dt} {form}: {ms:.3f} ms/step, {R / ms / 1e3:.1f} Mrays/s, "
                f"kernels(ms) {json.dumps({k: round(v, 4) for k, v in kern.items()})}")

    # the colour error BF16-stored attributes introduce, against the FP32-attribute frame
    bf16_err = None
    if args.only is None:
        o, d, t, s = rays
        c32 = rf.render_forward(scenes["f32"], o, d, t, s)[0]
        c16 = rf.render_forward(scenes["bf16"], o, d, t, s)[0]
        diff = (c16 - c32).abs()
        scale = float(c32.abs().max())
        bf16_err = {"max_rel": round(float(diff.max()) / scale, 6), "mean_rel": round(float(diff.mean()) / scale, 8),
                    "p99_rel": round(float(torch.quantile(diff.flatten()[:: 7][: 1 << 24].float(), 0.99)) / scale, 7)}
        log(f"bf16 colour error against the fp32-attribute frame: max {bf16_err['max_rel']:.2e}, "
            f"p99 {bf16_err['p99_rel']:.2e}, mean {bf16_err['mean_rel']:.2e} of the largest colour")

    # the attribute precision each workload is specified with (the 3M-site
    # multi-camera workload stores its attributes in BF16)
    main_dt = args.only or {"shell_3m": "bf16"}.get(args.config, "f32")
    dts = sorted({k[0] for k in results}, key=lambda x: x != "f32")
    ms, kern, lat = results[(main_dt, "fwd_bwd")]
    value = R / (ms * 1e-3) / 1e6

    def roofline(dt: str, form: str, kernel: str) -> dict:
        """HBM roofline of one kernel of a step form: measured DRAM bytes per launch
        (rocprofv3, when the committed summary matches these kernel sources) over
        the HIP-event duration; beside it the method's per-visit bytes and flops."""
        k_ms = results[(dt, form)][1][kernel]
        kind = {("forward", False): "forward", ("backward", False): "backward_recompute",
                ("forward", True): "forward", ("backward", True): "backward"}[(kernel, form == "fwd_bwd_logged")]
        label = {"fwd_bwd": {"forward": "forward", "backward": "backward (recomputing)"},
                 "fwd": {"forward": "forward", "backward": ""},
                 "fwd_bwd_logged": {"forward": "forward (logged)", "backward": "backward (log kernel)"}}[form][kernel]
        traffic = measured_traffic(args.config, dt, label)
        achieved = traffic / (k_ms * 1e-3) / 1e9 if traffic else None
        fl = flops_per_visit(mean_deg, B, kind) * visits
        tf = fl / (k_ms * 1e-3) / 1e12
        vb = visits * visit_bytes(mean_deg, B, dt, kind)
        return {"bound": "hbm", "kernel": f"k_{kernel}, {label} ({dt} attributes)", "ms": round(k_ms, 4),
                "achieved": None if achieved is None else round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": None if achieved is None else round(achieved / HBM_PEAK_GBS, 4),
                "traffic": traffic,
                "visit_bytes": int(vb), "visit_gbs": round(vb / (k_ms * 1e-3) / 1e9, 1),
                "alu": {"achieved": round(tf, 3), "unit": "TFLOP/s", "peak": FP32_PEAK_TFLOPS,
                        "frac": round(tf / FP32_PEAK_TFLOPS, 4), "peak_nonpacked": round(VALU_PEAK_TFLOPS, 2),
                        "frac_nonpacked": round(tf / VALU_PEAK_TFLOPS, 4)}}

    dominant = max(("forward", "backward"), key=lambda k: kern[k])
    rooflines = {f"{dt}_{form}_{k}": roofline(dt, form, k) for dt in dts for form, bwd, _ in forms
                 for k in (("forward", "backward") if bwd else ("forward",))}

    workload = (f"{args.config}: {scene.n_sites} sites {synth.CONFIGS[args.config]['kind']}, SH deg {scene.sh_deg}, "
                f"{len(cams)} x {cams[0].width}x{cams[0].height} camera{'s' if len(cams) > 1 else ''}, "
                f"raygen+pack+forward+backward (the backward recomputes each walk from the saved colour "
                f"and transmittance)")
    out = {
        "metric": f"Mrays/s fwd+bwd at {site_count(scene.n_sites)} sites ({main_dt.upper().replace('F32', 'FP32')} "
                  f"attributes, recomputing backward); fwd, walk-log and "
                  f"{'FP32' if main_dt == 'bf16' else 'BF16'} rates and p50/p99 step latency in added fields",
        "value": round(value, 3),
        "unit": "Mrays/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded clustered Voronoi scene, Delaunay CSR from Qhull)",
        "config": {"workload": workload, "rays_per_step": R, "cameras": len(cams), "visits_per_step": visits,
                   "mean_visited_degree": round(mean_deg, 3), "parallelism": "single GPU"},
        "fwd_mrays_s": {dt: round(R / results[(dt, "fwd")][0] / 1e3, 3) for dt in dts},
        "fwd_bwd_mrays_s": {dt: round(R / results[(dt, "fwd_bwd")][0] / 1e3, 3) for dt in dts},
        "fwd_bwd_logged": ({dt: {"mrays_s": round(R / results[(dt, "fwd_bwd_logged")][0] / 1e3, 3),
                                 "ms_per_step": round(results[(dt, "fwd_bwd_logged")][0], 4),
                                 "log_capacity": args.log_capacity,
                                 "log_bytes": int(R * (12 * args.log_capacity + 16))} for dt in dts}
                           if (main_dt, "fwd_bwd_logged") in results else None),
        "bf16_colour_error": bf16_err,
        "bf16_speedup_fwd_bwd": (round(results[("f32", "fwd_bwd")][0] / results[("bf16", "fwd_bwd")][0], 4)
                                 if len(dts) == 2 else None),
        "bf16_speedup_fwd": (round(results[("f32", "fwd")][0] / results[("bf16", "fwd")][0], 4)
                             if len(dts) == 2 else None),
        "step_latency_ms": {f"{dt}_{form}": {
            "p50": round(float(np.percentile(results[(dt, form)][2], 50)), 4),
            "p99": round(float(np.percentile(results[(dt, form)][2], 99)), 4)} for dt in dts
            for form, _, _ in forms},
        "kernel_ms": {f"{dt}_{form}": {k: round(v, 4) for k, v in results[(dt, form)][1].items()}
                      for dt in dts for form, _, _ in forms},
        "roofline": dict(rooflines[f"{main_dt}_fwd_bwd_{dominant}"]),
        "rooflines": rooflines,
        "kernel_source_digest": kernel_source_digest(),
    }
    if not args.no_serving and args.config == "clustered_1m":
        out["serving"] = serving(rf, scenes, scene, bound, dts)
    if not args.no_locate:
        out["locate"] = locate(rf, scenes["f32"], bound, dev)
    if not args.no_quantile and walk_log is not None:
        out["quantile"] = quantile_cost(rf, scenes["f32"], rays, grad_rgb, walk_log, dev, args.steps)
    if not args.no_training:
        out["training"] = training_cost(rf, scene, sites, off, idx, dens, sh, grads, dev, args.steps)
    if not args.no_effects and walk_log is not None and len(cams) == 1:
        out["effects"] = effects_cost(rf, scenes["f32"], rays, grad_rgb, walk_log, bound, cam.pose12(), cam.fov_deg,
                                      cam.width, cam.height, start, dev, args.steps)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(scene, cam, bound, start, g_np, visits / R, args.cpu_seconds)
    print(json.dumps(out), flush=True)
    return 0


def training_cost(rf, scene, sites, off, idx, dens, sh, grads, dev, reps: int):
    """The optimizer step (Adam over positions, density and SH with the
    paper's schedule, mid-run) against the HBM roofline (28 bytes per value:
    x, g, m, v read; x, m, v written), and the densification score, the
    sampling of 10% of the cells as candidates and the pruning mask."""
    import torch

    p = [sites.clone(), dens.clone(), sh.clone()]
    st = rf.AdamState(scene.n_sites, scene.sh_deg, dev)
    args = rf.train_schedule(10000, 20000)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        ms = []
        for _ in range(reps):
            ev[0].record()
            fn()
            ev[1].record()
            torch.cuda.synchronize()
            ms.append(ev[0].elapsed_time(ev[1]))
        return float(np.mean(ms))

    ms_adam = timed(lambda: rf.adam_step(args, st, p[0], p[1], p[2], grads[0], grads[1], grads[2]))
    values = p[0].numel() + p[1].numel() + p[2].numel()
    gbs = values * 28 / (ms_adam * 1e-3) / 1e9
    g = torch.Generator(device=dev)
    g.manual_seed(13)
    gsites = torch.randn((scene.n_sites, 3), device=dev, generator=g)
    draws = torch.rand(scene.n_sites // 10, device=dev, generator=g)
    ms_score = timed(lambda: rf.densify_scores(sites, off, idx, gsites))
    scores = rf.densify_scores(sites, off, idx, gsites)
    ms_sample = timed(lambda: rf.sample_cells(scores, draws))
    ms_prune = timed(lambda: rf.prune_mask(dens, off, idx, 0.01))
    log(f"adam step: {values} values in {ms_adam:.3f} ms ({gbs:.0f} GB/s of {HBM_PEAK_GBS:.0f}); densify score "
        f"{ms_score:.3f} ms, sampling {len(draws)} candidates {ms_sample:.3f} ms, prune mask {ms_prune:.3f} ms")
    return {"adam_ms": round(ms_adam, 4), "adam_values": values,
            "adam_roofline": {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                              "frac": round(gbs / HBM_PEAK_GBS, 4), "bytes_per_value": 28},
            "densify_score_ms": round(ms_score, 4), "sample_ms": round(ms_sample, 4),
            "sample_draws": len(draws), "prune_mask_ms": round(ms_prune, 4)}


def effects_cost(rf, packed, rays, grad_rgb, walk_log, bound, pose, fov, W, H, start, dev, reps: int):
    """Ray-based effects on the same frame (FP32 attributes): the logged
    training step (forward + backward) with a glass sphere (index 1.5,
    radius 0.3 at the scene's centre, filling the middle of the view) and
    with a mirror sphere, and a 180-degree fisheye camera's raygen + forward."""
    import torch

    o, d, t, s = rays
    R = int(d.shape[0])
    n, B = packed.n_sites, (packed.sh_degree + 1) ** 2
    grads = (torch.zeros((n, 3), device=dev), torch.zeros(n, device=dev), torch.zeros((n, B, 3), device=dev))
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    out = {}
    for kind in ("glass", "mirror"):
        sf = rf.Surface(kind, (0.0, 0.0, 0.0), 0.3, bound, ior=1.5, max_bounces=8)
        fw, bw = [], []
        for k in range(reps + 1):
            ev[0].record()
            rgb, tf, _ = rf.render_forward(packed, o, d, t, s, log=walk_log, surface=sf)
            ev[1].record()
            rf.render_backward(packed, o, d, t, s, rgb, tf, grad_rgb, grads=grads, log=walk_log, surface=sf)
            ev[2].record()
            torch.cuda.synchronize()
            if k:
                fw.append(ev[0].elapsed_time(ev[1]))
                bw.append(ev[1].elapsed_time(ev[2]))
        bent = float((walk_log.tail[:, 3] > 0).float().mean())
        ms = float(np.mean(fw) + np.mean(bw))
        out[kind] = {"forward_ms": round(float(np.mean(fw)), 4), "backward_ms": round(float(np.mean(bw)), 4),
                     "fwd_bwd_mrays_s": round(R / ms / 1e3, 2), "rays_bent": round(bent, 4)}
        log(f"{kind} sphere: forward {np.mean(fw):.3f} ms, backward {np.mean(bw):.3f} ms "
            f"({R / ms / 1e3:.1f} Mrays/s fwd+bwd), {bent:.1%} of rays bent")
    fe = []
    for k in range(reps + 1):
        ev[0].record()
        fo, fd, ft, fs, _ = rf.raygen(pose, 180.0, W, H, bound, start, device=dev, with_pixel=False, model="fisheye")
        rf.render_forward(packed, fo, fd, ft, fs)
        ev[1].record()
        torch.cuda.synchronize()
        if k:
            fe.append(ev[0].elapsed_time(ev[1]))
    out["fisheye_180"] = {"raygen_forward_ms": round(float(np.mean(fe)), 4),
                          "fwd_mrays_s": round(R / float(np.mean(fe)) / 1e3, 2)}
    log(f"fisheye 180 deg: raygen + forward {np.mean(fe):.3f} ms")
    return out


def quantile_cost(rf, packed, rays, grad_rgb, walk_log, dev, reps: int):
    """Cost of the quantile regulariser (Sec. 3.4) on top of a logged training
    step: the quantile kernel over the walk log, and the logged backward with
    and without the quantile term (FP32 attributes, uniform draws)."""
    import torch

    o, d, t, s = rays
    R = int(d.shape[0])
    g = torch.Generator(device=dev)
    g.manual_seed(11)
    draws = torch.rand((R, 2), device=dev, generator=g)
    grad_loss = torch.full((R,), 1.0 / R, device=dev)
    n, B = packed.n_sites, (packed.sh_degree + 1) ** 2
    grads = (torch.zeros((n, 3), device=dev), torch.zeros(n, device=dev), torch.zeros((n, B, 3), device=dev))
    rgb, tf, _ = rf.render_forward(packed, o, d, t, s, log=walk_log)
    q, loss = rf.quantile_forward(packed, o, d, t, s, tf, walk_log, draws)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        ms = []
        for _ in range(reps):
            ev[0].record()
            fn()
            ev[1].record()
            torch.cuda.synchronize()
            ms.append(ev[0].elapsed_time(ev[1]))
        return float(np.mean(ms))

    ms_q = timed(lambda: rf.quantile_forward(packed, o, d, t, s, tf, walk_log, draws))
    ms_b = timed(lambda: rf.render_backward(packed, o, d, t, s, rgb, tf, grad_rgb, grads=grads, log=walk_log))
    ms_bq = timed(lambda: rf.render_backward(packed, o, d, t, s, rgb, tf, grad_rgb, grads=grads, log=walk_log,
                                             quantiles=q, grad_loss=grad_loss))
    mean_loss = float(loss.mean())
    log(f"quantile: kernel {ms_q:.3f} ms, backward {ms_b:.3f} ms without / {ms_bq:.3f} ms with the quantile "
        f"term, mean loss {mean_loss:.5f}")
    return {"quantile_kernel_ms": round(ms_q, 4), "backward_ms": round(ms_b, 4),
            "backward_with_quantile_ms": round(ms_bq, 4), "mean_loss": round(mean_loss, 6)}


def locate(rf, packed, bound, dev, n_points: int = 1 << 20, grid: int = 32):
    """Start-cell location (nearest site) of random points in the bound's box:
    walks seeded from a grid^3 lattice of located cells, and walks from cell 0."""
    import torch

    lo = torch.tensor([bound[1]] * 3 if bound[0] == "box" else [-bound[1]] * 3, device=dev)
    hi = torch.tensor([bound[2]] * 3 if bound[0] == "box" else [bound[1]] * 3, device=dev)
    g = torch.Generator(device=dev)
    g.manual_seed(7)
    pts = lo + (hi - lo) * torch.rand((n_points, 3), device=dev, generator=g)
    ax = (torch.arange(grid, device=dev, dtype=torch.float32) + 0.5) / grid
    cz, cy, cx = torch.meshgrid(ax, ax, ax, indexing="ij")
    centres = (lo + (hi - lo) * torch.stack([cx, cy, cz], -1).reshape(-1, 3)).contiguous()
    lattice = rf.locate(packed, centres)
    ijk = ((pts - lo) / (hi - lo) * grid).long().clamp_(0, grid - 1)
    seeds = lattice[(ijk[:, 2] * grid + ijk[:, 1]) * grid + ijk[:, 0]].contiguous()

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    ms_seeded = timed(lambda: rf.locate(packed, pts, seeds), 10)
    cold = pts[: n_points // 16].contiguous()
    ms_cold = timed(lambda: rf.locate(packed, cold), 3)
    cells = rf.locate(packed, pts, seeds)
    log(f"locate: {n_points} points seeded from a {grid}^3 lattice {ms_seeded:.3f} ms, "
        f"{len(cold)} from cell 0 {ms_cold:.3f} ms, flagged {(cells < 0).sum().item()}")
    return {"points": n_points, "seed": f"{grid}^3 lattice of located cells", "ms": round(ms_seeded, 4),
            "mpoints_s": round(n_points / ms_seeded / 1e3, 2), "cold_points": len(cold),
            "cold_ms": round(ms_cold, 4), "cold_mpoints_s": round(len(cold) / ms_cold / 1e3, 3)}


def serving(rf, packed, scene, bound, dts):
    """Continuous-batching replay of 512 render requests (exponential inter-arrivals,
    mean 5 ms; sizes uniform over 256^2, 512^2, 1024^2, 1920x1080; poses inside
    [-0.8, 0.8]^3) against the resident 1M-site scene, forward only; then the same
    requests all arriving at once, whose throughput is the server's capacity. Both
    forms of the server (batched launches; one persistent kernel). The replay is
    timed on a fresh server, and again on a server warmed up with 16 of the
    requests; the capacity run follows a warm-up too."""
    import numpy as np

    import synth
    from paper_2502_01157_amd.serve import Server, replay

    rng = np.random.default_rng(5)
    reqs = synth.make_serving_requests(rng, n=512, rate_hz=200.0)
    starts = synth.nearest_site(scene.sites, np.stack([r["camera"].position for r in reqs]))
    stream = [dict(arrival=r["arrival"], pose12=r["camera"].pose12(), fov_deg=r["camera"].fov_deg,
                   width=r["camera"].width, height=r["camera"].height, start_cell=int(st))
              for r, st in zip(reqs, starts)]
    offered = sum(r["width"] * r["height"] for r in stream) / (stream[-1]["arrival"] - stream[0]["arrival"]) / 1e6
    res = {"requests": len(stream), "offered_mrays_s": round(offered, 2)}
    # the same requests all at once: the server's capacity
    burst = [dict(r, arrival=0.0) for r in stream]
    # a fresh server on a device that has been idle serves its first requests
    # slowly: 16 requests all at once warm it up before each timed replay
    warm = [dict(r, arrival=0.0) for r in stream[:16]]
    for dt in dts:
        res[dt] = {}
        for mode in ("launches", "persistent"):
            def server():
                return Server(packed[dt], bound, pool_bytes=1 << 30, max_inflight=64, mode=mode)

            # a fresh server, no warm-up: the first requests arrive on a just-created server
            with server() as srv:
                cold = replay(srv, stream, timeout_s=120)
            with server() as srv:
                replay(srv, warm, timeout_s=120)
                st0 = srv.stats()
                out = replay(srv, stream, timeout_s=120)
                st = srv.stats()
            with server() as srv:
                replay(srv, warm, timeout_s=120)
                cap = replay(srv, burst, timeout_s=120)
            res[dt][mode] = {"p50_ms": round(out["p50_ms"], 3), "p99_ms": round(out["p99_ms"], 3),
                             "mean_ms": round(out["mean_ms"], 3), "mrays_s": round(out["mrays_per_s"], 2),
                             "cold_p50_ms": round(cold["p50_ms"], 3), "cold_p99_ms": round(cold["p99_ms"], 3),
                             "cold_max_ms": round(float(np.nanmax(cold["latency_s"])) * 1e3, 3),
                             "launches": int(st["launches"] - st0["launches"]),
                             "busy_rejections": int(st["rejected_busy"] - st0["rejected_busy"]),
                             "copy_out_ms_mean": round(float(np.nanmean(out["copy_ms"])), 3),
                             "burst_mrays_s": round(cap["mrays_per_s"], 2)}
            log(f"serving {dt} {mode}: p50 {out['p50_ms']:.2f} ms, p99 {out['p99_ms']:.2f} ms "
                f"(fresh server: p50 {cold['p50_ms']:.2f}, p99 {cold['p99_ms']:.2f} ms), "
                f"{out['mrays_per_s']:.1f} Mrays/s sustained (offered {offered:.1f}), "
                f"{res[dt][mode]['launches']} launches; all {len(burst)} requests at once: "
                f"{cap['mrays_per_s']:.1f} Mrays/s")
    return res


def cpu_baseline(scene, cam, bound, start, g_np, visits_per_ray, target_s):
    """The FP64 oracle on a bounded contiguous band of screen tiles of the same frame."""
    import oracle

    threads = oracle.default_threads()
    osc = oracle.OracleScene.from_scene(scene)
    o, d, t, _ = oracle.raygen(cam.pose12(), cam.fov_deg, cam.width, cam.height, bound)
    R = len(t)
    # calibrate the forward on 16384 rays, then size the sample so that forward
    # plus backward (about three forward walks) take ~target_s
    mid = R // 4
    n0 = 16384
    sl = slice(mid, mid + n0)
    a = time.perf_counter()
    oracle.forward(osc, o[sl], d[sl], t[sl], start, threads=threads)
    per_ray = (time.perf_counter() - a) / n0
    n = int(min(R - mid, max(n0, target_s / 3.0 / max(per_ray, 1e-9))))
    n = n // 64 * 64
    sl = slice(mid, mid + n)
    a = time.perf_counter()
    oracle.forward(osc, o[sl].astype(np.float32), d[sl].astype(np.float32), t[sl].astype(np.float32), start,
                   threads=threads)
    tf = time.perf_counter() - a
    a = time.perf_counter()
    oracle.backward(osc, o[sl].astype(np.float32), d[sl].astype(np.float32), t[sl].astype(np.float32),
                    np.full(n, start, dtype=np.int32), g_np[sl], threads=threads)
    tb = time.perf_counter() - a
    log(f"oracle on {n} rays with {threads} threads: fwd {tf:.2f}s, bwd (recomputes the walk) {tb:.2f}s")
    # one core, on the first sixteenth of the same sample
    n1 = max(64, n // 16 // 64 * 64)
    s1 = slice(mid, mid + n1)
    a = time.perf_counter()
    oracle.forward(osc, o[s1].astype(np.float32), d[s1].astype(np.float32), t[s1].astype(np.float32), start,
                   threads=1)
    oracle.backward(osc, o[s1].astype(np.float32), d[s1].astype(np.float32), t[s1].astype(np.float32),
                    np.full(n1, start, dtype=np.int32), g_np[s1], threads=1)
    t1 = time.perf_counter() - a
    log(f"oracle on {n1} rays with 1 thread: forward + backward {t1:.2f}s")
    return {"value": round(n / (tf + tb) / 1e6, 5), "unit": "Mrays/s", "cores": threads, "kind": "oracle",
            "sample": f"{n} rays ({n // 64} consecutive 8x8 tiles starting a quarter into the same frame), "
                      f"forward then backward, FP64 C oracle",
            "fwd_mrays_s": round(n / tf / 1e6, 5),
            "one_core": {"value": round(n1 / t1 / 1e6, 5), "sample": f"the first {n1} rays of that sample"}}


if __name__ == "__main__":
    sys.exit(main())
