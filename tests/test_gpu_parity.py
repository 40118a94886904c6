"""GPU parity: the HIP walk (through the C ABI) against the FP64 oracle.

Inputs are seeded synthetic scenes shaped like the paper's workloads; rays come
from the oracle's FP64 ray generation (rounded to FP32) or from random interior
points. The oracle runs on exactly the FP32 inputs the GPU sees, widened to FP64.
"""

import numpy as np
import pytest

import oracle
import synth

from parity import (COLOUR_RTOL, GRAD_RTOL, T_ATOL, T_EXIT_ATOL, camera_rays, check_gradients, colour_err,
                    colour_ratio, compare_sequences, decidable, grad_err, gradient_decidable, inside_rays,
                    resolve_near_ties)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rf():
    import torch

    if not torch.cuda.is_available():
        pytest.fail("no GPU visible to torch")
    import paper_2502_01157_amd as rf_mod

    return rf_mod


def to_dev(*arrays):
    import torch

    return [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in arrays]


def packed(rf, scene, dtype="f32"):
    import torch

    sites, off, idx, dens, sh = to_dev(scene.sites, scene.off, scene.idx, scene.density, scene.sh)
    p = rf.PackedScene(sites, off, idx, dens, sh, scene.sh_deg, dtype, validate=True)
    torch.cuda.synchronize()
    return p, (sites, off, idx, dens, sh)


def gpu_trace(rf, p, rays, eps, max_steps=8192, max_len=1024):
    o, d, t, s = to_dev(*rays)
    tr = rf.render_trace(p, o, d, t, s, eps=eps, max_steps=max_steps, max_len=max_len)
    out = {k: v.cpu().numpy() for k, v in tr.items()}
    steps = out["steps"]
    out["len"] = np.where(steps >= 0, steps, np.where(steps == -2, max_steps, 0))
    return out


def check_forward(rf, scene, rays, eps, dtype="f32", max_unresolved=0.002, max_steps=8192):
    """Every ray: exact cells on decidable rays, the GPU's walk among the
    oracle's alternatives on near-tie rays, and colour, transmittance and
    visit count against the matching walk."""
    p, _ = packed(rf, scene, dtype)
    osc = oracle.OracleScene.from_scene(scene)
    if dtype == "bf16":
        dens = oracle.bf16_to_f32(oracle.bf16_round(scene.density))
        sh = oracle.bf16_to_f32(oracle.bf16_round(scene.sh))
        osc = oracle.OracleScene.from_scene(scene, density=dens, sh=sh)
    ref = oracle.trace(osc, *rays, eps=eps, max_len=1024, max_steps=max_steps)
    g = gpu_trace(rf, p, rays, eps, max_steps=max_steps)
    dec = decidable(ref, eps)
    assert compare_sequences(g["cells"], g["len"], ref, dec) == 0
    np.testing.assert_array_equal(g["steps"][dec], ref["steps"][dec])
    mean_abs = float(np.abs(ref["rgb"]).mean())
    assert colour_ratio(g["rgb"][dec], ref["rgb"][dec], mean_abs).max(initial=0) <= 1.0
    assert np.abs(g["t_final"][dec] - ref["t_final"][dec]).max(initial=0) <= T_ATOL
    und = np.nonzero(~dec)[0]
    if len(und):
        res = resolve_near_ties(osc, rays, und, g["cells"][und], g["len"][und], eps, max_steps=max_steps)
        unresolved = 0
        for q, r in enumerate(und):
            m = res["match"][q]
            if m is None:
                # no alternative matched: only allowed where the alternatives were not all listed
                assert not res["complete"][q], f"ray {r}: the GPU's walk is none of the oracle's alternatives"
                unresolved += 1
                continue
            assert colour_ratio(g["rgb"][r], m["rgb"], mean_abs)[0] <= 1.0, r
            assert abs(g["t_final"][r] - m["t_final"]) <= T_ATOL, r
            assert g["steps"][r] == m["steps"], r
        assert unresolved <= max_unresolved * len(dec), (unresolved, len(dec))
    # exit distances of decidable rays
    for r in np.nonzero(dec)[0][:2000]:
        L = ref["len"][r]
        np.testing.assert_allclose(g["t_exit"][r, :L], ref["t_exit"][r, :L], rtol=1e-4, atol=T_EXIT_ATOL)
    return p, ref, g, dec


# ---------------------------------------------------------------------------
# scenes
# ---------------------------------------------------------------------------

@pytest.fixture(scope="module")
def uniform_4k():
    scene, rng = synth.make_scene("uniform_4k", return_rng=True)
    cam = synth.make_cameras("uniform_4k", rng)[0]
    return scene, cam


@pytest.fixture(scope="module")
def clustered():
    scene, rng = synth.small_scene("clustered", 20000, seed=31, sh_deg=3, return_rng=True)
    cams = synth.make_cameras("clustered_200k", rng, n=1, res=(96, 72))
    return scene, cams[0], rng


class _Deg:
    def __init__(self, scene, deg):
        self.__dict__.update(scene.__dict__)
        b = (deg + 1) ** 2
        self.sh = np.ascontiguousarray(scene.sh[:, :b, :])
        self.sh_deg = deg


# ---------------------------------------------------------------------------
# a1: packing
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_pack_planes_and_records(rf, clustered, dtype):
    scene = clustered[0]
    p, _ = packed(rf, scene, dtype)
    planes = p.planes().cpu().numpy().astype(np.float64)
    ref = oracle.face_planes(scene.sites, scene.off, scene.idx)
    # n = x_j - x_i is one fp32 subtraction of fp32 values: within half an ulp
    np.testing.assert_allclose(planes[:, :3], ref[:, :3], rtol=2 ** -24, atol=0)
    scale = np.linalg.norm(ref[:, :3], axis=1) * np.linalg.norm(scene.sites, axis=1).max()
    assert np.all(np.abs(planes[:, 3] - ref[:, 3]) <= 4e-7 * scale + 1e-30)
    # each face's neighbour row (j | deg_j << 24, row start of j), exactly
    a0 = p.desc.off_adj
    adj = p.workspace[a0:a0 + 8 * scene.n_edges].cpu().numpy().view(np.uint32).reshape(-1, 2)
    j = scene.idx.astype(np.int64)
    deg = np.diff(scene.off).astype(np.int64)
    np.testing.assert_array_equal(adj[:, 0], (j | (deg[j] << 24)).astype(np.uint32))
    np.testing.assert_array_equal(adj[:, 1], scene.off[j].astype(np.uint32))
    dens, sh = (t.cpu().numpy() for t in p.attributes())
    if dtype == "f32":
        np.testing.assert_array_equal(dens, scene.density)
        np.testing.assert_array_equal(sh, scene.sh)
    else:
        np.testing.assert_array_equal(dens, oracle.bf16_to_f32(oracle.bf16_round(scene.density)))
        np.testing.assert_array_equal(sh, oracle.bf16_to_f32(oracle.bf16_round(scene.sh)))
    assert p.errors() == (0, 0)


def test_pack_rejects_bad_csr_without_faulting(rf, clustered):
    import torch

    scene = clustered[0]
    sites, off, idx, dens, sh = to_dev(scene.sites, scene.off, scene.idx, scene.density, scene.sh)
    bad_idx = idx.clone()
    bad_idx[7] = scene.n_sites + 5
    bad_idx[100] = -3
    with pytest.raises(rf.RfError, match="INVALID_ARG"):
        rf.PackedScene(sites, off, bad_idx, dens, sh, 3, validate=True)
    bad_off = off.clone()
    bad_off[50] = scene.n_edges + 1000
    p = rf.PackedScene(sites, bad_off, idx, dens, sh, 3, validate=False)
    assert p.errors()[0] > 0
    # the corrupt scene still renders without touching memory out of range
    o, d, t, s = to_dev(*inside_rays(scene, np.random.default_rng(0), 300, -0.9, 0.9))
    rgb, tf, steps = rf.render_forward(p, o, d, t, s)
    torch.cuda.synchronize()
    assert torch.isfinite(rgb).all()


# ---------------------------------------------------------------------------
# a2: camera rays
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("W,H,bound", [(64, 64, ("box", 0.0, 1.0)), (100, 37, ("box", -1.0, 1.0)),
                                       (33, 70, ("sphere", 5.0))])
def test_raygen_matches_oracle(rf, W, H, bound):
    rng = np.random.default_rng(W + H)
    cam = synth.make_cameras("shell_3m", rng, n=1, res=(W, H))[0]
    if bound[1] == 0.0:
        cam.position = np.array([0.5, 0.4, 0.6])
    o, d, t, s, px = rf.raygen(cam.pose12(), cam.fov_deg, W, H, bound, start=123)
    ro, rd, rt, rpx = oracle.raygen(np.float32(cam.pose12()).astype(np.float64), cam.fov_deg, W, H, bound)
    np.testing.assert_array_equal(px.cpu().numpy(), rpx)
    np.testing.assert_allclose(d.cpu().numpy(), rd, atol=2e-6)
    np.testing.assert_allclose(o.cpu().numpy(), ro, atol=1e-7)
    np.testing.assert_allclose(t.cpu().numpy(), rt, rtol=2e-5, atol=2e-6)
    assert np.all(s.cpu().numpy() == 123)


# ---------------------------------------------------------------------------
# a3: forward walk
# ---------------------------------------------------------------------------

def test_uniform_4k_full_frame_forward(rf, uniform_4k):
    scene, cam = uniform_4k
    rays = camera_rays(scene, cam)[:4]
    check_forward(rf, scene, rays, eps=1e-4)


@pytest.mark.parametrize("deg", [0, 1, 2, 3])
def test_clustered_camera_forward(rf, clustered, deg):
    scene, cam, _ = clustered
    rays = camera_rays(scene, cam)[:4]
    check_forward(rf, _Deg(scene, deg), rays, eps=1e-4)


@pytest.mark.parametrize("n_rays", [1, 63, 65, 257, 1000])
def test_ragged_interior_rays_eps0(rf, clustered, n_rays):
    scene = clustered[0]
    rays = inside_rays(scene, np.random.default_rng(n_rays), n_rays, -0.95, 0.95)
    check_forward(rf, scene, rays, eps=0.0)


def test_forward_bitwise_deterministic(rf, clustered):
    scene, cam, _ = clustered
    p, _ = packed(rf, scene)
    o, d, t, s = to_dev(*camera_rays(scene, cam)[:4])
    a = [x.cpu().numpy() for x in rf.render_forward(p, o, d, t, s)]
    b = [x.cpu().numpy() for x in rf.render_forward(p, o, d, t, s)]
    for x, y in zip(a, b):
        np.testing.assert_array_equal(x, y)


def test_edge_cases(rf, clustered):
    import torch

    scene = clustered[0]
    p, _ = packed(rf, scene)
    # empty batch
    z = torch.empty((0, 3), device="cuda")
    rgb, tf, steps = rf.render_forward(p, z, z.clone(), torch.empty(0, device="cuda"),
                                       torch.empty(0, dtype=torch.int32, device="cuda"))
    assert rgb.shape == (0, 3)
    # invalid start cells, zero-length rays, a max_steps cap
    o, d, t, s = inside_rays(scene, np.random.default_rng(5), 200, -0.9, 0.9)
    s[:4] = [-1, scene.n_sites, 2 ** 31 - 1, -(2 ** 31)]
    t[4:8] = 0.0
    ref = oracle.trace(oracle.OracleScene.from_scene(scene), o, d, t, s, eps=1e-4, max_steps=5)
    g = gpu_trace(rf, p, (o, d, t, s), eps=1e-4, max_steps=5)
    np.testing.assert_array_equal(g["steps"][:4], -1)
    np.testing.assert_array_equal(g["rgb"][:4], 0)
    np.testing.assert_array_equal(g["t_final"][:4], 1)
    np.testing.assert_array_equal(g["steps"][4:8], 1)
    np.testing.assert_array_equal(g["t_final"][4:8], 1)
    dec = decidable(ref, 1e-4)
    np.testing.assert_array_equal(g["steps"][dec], ref["steps"][dec])
    assert np.any(g["steps"] == -2)
    assert colour_ratio(g["rgb"][dec], ref["rgb"][dec], np.abs(ref["rgb"]).mean()).max() <= 1.0
    # zero density everywhere: fully transparent
    p0 = rf.PackedScene(*to_dev(scene.sites, scene.off, scene.idx, np.zeros_like(scene.density), scene.sh), 3)
    rgb, tf, _ = rf.render_forward(p0, *to_dev(o[8:], d[8:], t[8:], s[8:]))
    assert torch.all(rgb == 0) and torch.all(tf == 1)
    # bad arguments are rejected on the host
    with pytest.raises(rf.RfError, match="INVALID_ARG"):
        rf.render_forward(p, *to_dev(o, d, t, s), eps=-1.0)
    with pytest.raises(rf.RfError, match="INVALID_ARG"):
        rf.render_forward(p, *to_dev(o, d, t, s), max_steps=0)


# ---------------------------------------------------------------------------
# a4/a5: backward walk and its wavefront reduction
# ---------------------------------------------------------------------------

def check_backward(rf, scene, rays, eps, mode=0, dtype="f32", with_gt=True, seed=0, log_capacity=None):
    import torch

    osc = oracle.OracleScene.from_scene(scene)
    if dtype == "bf16":
        osc = oracle.OracleScene.from_scene(scene, density=oracle.bf16_to_f32(oracle.bf16_round(scene.density)),
                                            sh=oracle.bf16_to_f32(oracle.bf16_round(scene.sh)))
    ref = oracle.trace(osc, *rays, eps=eps, max_len=1024)
    dec = gradient_decidable(ref, eps)
    rays = tuple(a[dec] for a in rays)
    rng = np.random.default_rng(seed)
    g = rng.standard_normal((len(rays[1]), 3)).astype(np.float32)
    gT = rng.standard_normal(len(rays[1])).astype(np.float32) if with_gt else None
    ref_g = oracle.backward(osc, *rays, g, gT, eps=eps)
    p, _ = packed(rf, scene, dtype)
    o, d, t, s = to_dev(*rays)
    log = None if log_capacity is None else rf.WalkLog(len(rays[1]), log_capacity, o.device)
    rgb, tf, steps = rf.render_forward(p, o, d, t, s, eps=eps, log=log)
    gg, = to_dev(g)
    gt_dev = to_dev(gT)[0] if with_gt else None
    mism = torch.zeros(1, dtype=torch.int32, device=o.device) if log is None else None
    gs, gd, gsh = rf.render_backward(p, o, d, t, s, rgb, tf, gg, gt_dev, eps=eps, mode=mode, log=log,
                                     steps=steps if log is None else None, mismatches=mism)
    torch.cuda.synchronize()
    if mism is not None:
        assert int(mism.item()) == 0
    return check_gradients((gs, gd, gsh), ref_g)


@pytest.mark.parametrize("mode", [0, 1])
def test_backward_camera_rays(rf, clustered, mode):
    scene, cam, _ = clustered
    check_backward(rf, scene, camera_rays(scene, cam)[:4], eps=1e-4, mode=mode)


@pytest.mark.parametrize("deg", [0, 1, 2])
def test_backward_lower_sh_degrees(rf, clustered, deg):
    scene, cam, _ = clustered
    check_backward(rf, _Deg(scene, deg), camera_rays(scene, cam)[:4], eps=1e-4)


def test_backward_interior_rays_eps0_and_dense_termination(rf, clustered):
    scene = clustered[0]
    rays = inside_rays(scene, np.random.default_rng(7), 777, -0.95, 0.95)
    check_backward(rf, scene, rays, eps=0.0, seed=1)
    dense = _Deg(scene, 3)
    dense.density = scene.density * 40.0          # most rays end by the transmittance test
    check_backward(rf, dense, rays, eps=1e-2, seed=2)


def test_backward_consistency_check_counts_disagreeing_rays(rf, clustered):
    """The recomputing backward compares each recomputed walk with the
    forward's outputs: none differ for the forward's own outputs; a final
    transmittance or a visit count changed on the host is counted per ray."""
    import torch

    scene, cam, _ = clustered
    p, _ = packed(rf, scene)
    o, d, t, s = to_dev(*camera_rays(scene, cam)[:4])
    R = int(t.shape[0])
    rgb, tf, steps = rf.render_forward(p, o, d, t, s)
    g = torch.randn_like(rgb)
    mism = torch.zeros(1, dtype=torch.int32, device=o.device)
    rf.render_backward(p, o, d, t, s, rgb, tf, g, steps=steps, mismatches=mism)
    torch.cuda.synchronize()
    assert int(mism.item()) == 0
    tf_bad = tf.clone()
    tf_bad[:100] = torch.nextafter(tf_bad[:100], torch.full_like(tf_bad[:100], 2.0))
    steps_bad = steps.clone()
    steps_bad[R - 50:] += 1
    mism.zero_()
    rf.render_backward(p, o, d, t, s, rgb, tf_bad, g, steps=steps_bad, mismatches=mism)
    torch.cuda.synchronize()
    assert int(mism.item()) == 150


def test_backward_modes_agree(rf, clustered):
    import torch

    scene, cam, _ = clustered
    p, _ = packed(rf, scene)
    o, d, t, s = to_dev(*camera_rays(scene, cam)[:4])
    rgb, tf, _ = rf.render_forward(p, o, d, t, s)
    g = torch.randn_like(rgb)
    a = rf.render_backward(p, o, d, t, s, rgb, tf, g, mode=0)
    b = rf.render_backward(p, o, d, t, s, rgb, tf, g, mode=1)
    for x, y in zip(a, b):
        assert grad_err(x.cpu().numpy(), y.cpu().numpy()) < 1e-5


@pytest.mark.parametrize("cap", [256, "half", 1, 0])
@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_logged_walk(rf, clustered, dtype, cap):
    """The logged forward returns the plain forward's outputs bit for bit and
    logs exactly the traced visits; the logged backward gives the recomputing
    backward's gradients, for a log that holds every walk (256), about half of
    them (the rest resume from the tail), one visit, or none."""
    import torch

    scene, cam, _ = clustered
    rays = camera_rays(scene, cam)[:4]
    R = len(rays[2])
    p, _ = packed(rf, scene, dtype)
    o, d, t, s = to_dev(*rays)
    plain = rf.render_forward(p, o, d, t, s)
    steps_np = plain[2].cpu().numpy()
    if cap == "half":
        cap = int(np.median(steps_np))
    log = rf.WalkLog(R, cap, o.device)
    out = rf.render_forward(p, o, d, t, s, log=log)
    for x, y in zip(plain, out):
        assert torch.equal(x, y)
    if cap == int(np.median(steps_np)):
        assert (steps_np > cap).any() and (steps_np <= cap).any()

    tail = log.tail.cpu().numpy()
    np.testing.assert_array_equal(tail[:, 2], steps_np)  # every ray here starts in a cell and ends normally
    tr = rf.render_trace(p, o, d, t, s, max_len=1024)
    cells, t_exit = tr["cells"].cpu().numpy(), tr["t_exit"].cpu().numpy()
    code = log.code.cpu().numpy().view(np.uint32)
    te = log.t_exit.cpu().numpy()
    for r in range(R):
        n = min(int(steps_np[r]), cap)
        np.testing.assert_array_equal(code[:n, r] & ((1 << 30) - 1), cells[r, :n])
        np.testing.assert_array_equal(te[:n, r].astype(np.float32), t_exit[r, :n])
        clipped = (code[:n, r] >> 30) & 1
        assert not clipped[: max(n - 1, 0)].any()
        if n == steps_np[r] and n > 0:  # the last visit is in the log: clipped iff it ends at t_max
            assert bool(clipped[n - 1]) == (te[n - 1, r] == np.float64(rays[2][r]))

    g = torch.randn_like(out[0])
    gT = torch.randn_like(out[1])
    for mode in (0, 1):
        a = rf.render_backward(p, o, d, t, s, out[0], out[1], g, gT, mode=mode)
        b = rf.render_backward(p, o, d, t, s, out[0], out[1], g, gT, mode=mode, log=log)
        for x, y in zip(b, a):
            assert grad_err(x.cpu().numpy(), y.cpu().numpy()) < 1e-5


@pytest.mark.parametrize("cap", [256, 20])
def test_logged_backward_matches_oracle(rf, clustered, cap):
    scene, cam, _ = clustered
    check_backward(rf, scene, camera_rays(scene, cam)[:4], eps=1e-4, log_capacity=cap)
    rays = inside_rays(scene, np.random.default_rng(7), 777, -0.95, 0.95)
    dense = _Deg(scene, 3)
    dense.density = scene.density * 40.0
    check_backward(rf, dense, rays, eps=1e-2, seed=2, log_capacity=cap)


def test_logged_walk_argument_errors(rf, clustered):
    import ctypes

    import torch

    from paper_2502_01157_amd import _lib as L
    from paper_2502_01157_amd.ops import _params, _rays, _stream

    scene, cam, _ = clustered
    p, _ = packed(rf, scene)
    o, d, t, s = to_dev(*camera_rays(scene, cam)[:4])
    R = int(t.shape[0])
    with pytest.raises(ValueError):
        rf.WalkLog(R, -1, o.device)
    with pytest.raises(ValueError):
        rf.render_forward(p, o, d, t, s, log=rf.WalkLog(R + 1, 8, o.device))
    rgb, tf, steps = (torch.empty((R, 3), device=o.device), torch.empty(R, device=o.device),
                      torch.empty(R, dtype=torch.int32, device=o.device))
    rays, prm = _rays(o, d, t, s), _params(1e-4, 8192)
    lib = L.lib()
    args = (ctypes.byref(p.desc), ctypes.byref(rays), ctypes.byref(prm), rgb.data_ptr(), tf.data_ptr(),
            steps.data_ptr())
    assert lib.rf_render_forward_logged(*args, None, _stream(o.device)) == L.RF_ERR_INVALID_ARG
    bad = rf.WalkLog(R, 4, o.device)
    bad.desc.capacity = -1
    assert lib.rf_render_forward_logged(*args, ctypes.byref(bad.desc), _stream(o.device)) == L.RF_ERR_INVALID_ARG
    bad.desc.capacity = 4
    bad.desc.t_exit = bad.t_exit.data_ptr() + 4  # misaligned doubles
    assert lib.rf_render_forward_logged(*args, ctypes.byref(bad.desc), _stream(o.device)) == L.RF_ERR_INVALID_ARG
    bad.desc.t_exit = None
    assert lib.rf_render_forward_logged(*args, ctypes.byref(bad.desc), _stream(o.device)) == L.RF_ERR_INVALID_ARG
    torch.cuda.synchronize()


def test_autograd_function(rf, clustered):
    import torch

    scene, cam, _ = clustered
    sites, off, idx, dens, sh = to_dev(scene.sites, scene.off, scene.idx, scene.density, scene.sh)
    sites.requires_grad_(True)
    dens.requires_grad_(True)
    sh.requires_grad_(True)
    o, d, t, s = to_dev(*camera_rays(scene, cam)[:4])
    rgb, tf, steps = rf.render(sites, dens, sh, off, idx, o, d, t, s, 3)
    g = torch.randn_like(rgb)
    (rgb * g).sum().backward()
    p, _ = packed(rf, scene)
    ref = rf.render_backward(p, o, d, t, s, rgb.detach(), tf.detach(), g)
    for x, y in zip((sites.grad, dens.grad, sh.grad), ref):
        assert grad_err(x.cpu().numpy(), y.cpu().numpy()) < 1e-5


@pytest.mark.parametrize("log_capacity", [0, 256])
def test_autograd_matches_oracle(rf, clustered, log_capacity):
    """rf.render(...).backward() (the torch.autograd.Function, with the
    recomputing backward and with a walk log) against the oracle's gradient of
    the same loss sum(g . rgb) + sum(g_T T), for sites, density and SH."""
    import torch

    scene, cam, _ = clustered
    rays = camera_rays(scene, cam)[:4]
    osc = oracle.OracleScene.from_scene(scene)
    ref = oracle.trace(osc, *rays, eps=1e-4, max_len=1)
    keep = gradient_decidable(ref, 1e-4)
    rng = np.random.default_rng(17)
    g = np.where(keep[:, None], rng.standard_normal((len(keep), 3)), 0.0).astype(np.float32)
    gT = np.where(keep, rng.standard_normal(len(keep)), 0.0).astype(np.float32)
    sites, off, idx, dens, sh = to_dev(scene.sites, scene.off, scene.idx, scene.density, scene.sh)
    for x in (sites, dens, sh):
        x.requires_grad_(True)
    o, d, t, s = to_dev(*rays)
    rgb, tf, steps = rf.render(sites, dens, sh, off, idx, o, d, t, s, 3, log_capacity=log_capacity)
    gg, gtt = to_dev(g, gT)
    ((rgb * gg).sum() + (tf * gtt).sum()).backward()
    torch.cuda.synchronize()
    ref_g = oracle.backward(osc, *rays, g, gT, eps=1e-4)
    check_gradients((sites.grad, dens.grad, sh.grad), ref_g)
    dec = decidable(ref, 1e-4)
    c = rgb.detach().cpu().numpy()
    assert colour_ratio(c[dec], ref["rgb"][dec], np.abs(ref["rgb"]).mean()).max() <= 1.0


# ---------------------------------------------------------------------------
# a7: bf16-stored attributes
# ---------------------------------------------------------------------------

def test_bf16_forward_and_backward(rf, clustered):
    scene, cam, _ = clustered
    rays = camera_rays(scene, cam)[:4]
    p, ref, g, dec = check_forward(rf, scene, rays, eps=1e-4, dtype="bf16")
    check_backward(rf, scene, rays, eps=1e-4, dtype="bf16")
    # total error against the fp32-attribute oracle stays at bf16 rounding level
    full = oracle.forward(oracle.OracleScene.from_scene(scene), *rays, eps=1e-4)
    assert colour_err(g["rgb"], full[0]) < 1e-2


def test_gpu_finite_differences(rf, clustered):
    """Central finite differences of the GPU forward against the GPU backward
    (FP32 renders, the loss summed in double on the host): the largest density
    and SH gradients, and the largest site gradients (the loss restricted to
    the rays whose cells a small site step does not change)."""
    import torch

    scene, cam, _ = clustered
    rays = camera_rays(scene, cam)[:4]
    o, d, t, s = to_dev(*rays)
    g = np.random.default_rng(23).standard_normal((len(rays[2]), 3)).astype(np.float32)
    gg, = to_dev(g)
    sites0, dens0, sh0 = (a.astype(np.float32).copy() for a in (scene.sites, scene.density, scene.sh))
    off, idx = to_dev(scene.off, scene.idx)

    def loss(sites, dens, sh):
        p = rf.PackedScene(*to_dev(sites, scene.off, scene.idx, dens, sh), 3)
        rgb, _, _ = rf.render_forward(p, o, d, t, s)
        torch.cuda.synchronize()
        return float((rgb.cpu().numpy().astype(np.float64) * g).sum())

    p = rf.PackedScene(*to_dev(sites0, scene.off, scene.idx, dens0, sh0), 3)
    rgb, tf, steps = rf.render_forward(p, o, d, t, s)
    gs, gd, gsh = (x.cpu().numpy() for x in rf.render_backward(p, o, d, t, s, rgb, tf, gg))
    for i in np.argsort(-np.abs(gd))[:3]:
        h = 1e-2 * dens0[i]
        dp, dm = dens0.copy(), dens0.copy()
        dp[i] += h
        dm[i] -= h
        fd = (loss(sites0, dp, sh0) - loss(sites0, dm, sh0)) / (float(dp[i]) - float(dm[i]))
        assert abs(fd - gd[i]) <= 1e-2 * abs(gd[i]), (i, fd, gd[i])
    flat = np.argsort(-np.abs(gsh.ravel()))[:3]
    for f in flat:
        h = 1e-2
        sp, sm = sh0.copy(), sh0.copy()
        sp.ravel()[f] += h
        sm.ravel()[f] -= h
        fd = (loss(sites0, dens0, sp) - loss(sites0, dens0, sm)) / (float(sp.ravel()[f]) - float(sm.ravel()[f]))
        assert abs(fd - gsh.ravel()[f]) <= 1e-3 * abs(gsh.ravel()[f]), (f, fd, gsh.ravel()[f])
    ref = oracle.trace(oracle.OracleScene.from_scene(scene), *rays, eps=1e-4, max_len=1024)
    gpu_cells = rf.render_trace(p, o, d, t, s, max_len=1024)["cells"].cpu().numpy()
    checked = 0
    for f in np.argsort(-np.abs(gs.ravel()))[:40]:
        if checked >= 4:
            break
        i, c = divmod(int(f), 3)
        h = 4e-5
        steps_ = []
        for hh in (h, h / 2):
            sp, sm = sites0.copy(), sites0.copy()
            sp[i, c] += hh
            sm[i, c] -= hh
            steps_.append((sp, sm))
        # rays whose cells a step changes (a face decision flips: the loss is
        # not differentiable there) get no upstream gradient on either side
        keep = np.ones(len(rays[2]), dtype=bool)
        for sx in (x for pair in steps_ for x in pair):
            tr = oracle.trace(oracle.OracleScene(sx, scene.off, scene.idx, dens0, sh0, 3), *rays, eps=1e-4,
                              max_len=1024)
            keep &= np.all(tr["cells"] == ref["cells"], axis=1) & (tr["len"] == ref["len"])
            # the GPU's own FP32 decisions too: a flip there, at a tie the
            # oracle resolves the other way, is a jump of the GPU's loss
            pk = rf.PackedScene(*to_dev(sx, scene.off, scene.idx, dens0, sh0), 3)
            keep &= np.all(rf.render_trace(pk, o, d, t, s, max_len=1024)["cells"].cpu().numpy() == gpu_cells, axis=1)
        gk = np.where(keep[:, None], g, 0.0).astype(np.float32)
        gks, = to_dev(gk)
        gsk = rf.render_backward(p, o, d, t, s, rgb, tf, gks)[0].cpu().numpy()
        if abs(gsk[i, c]) < 1e-2 * abs(gs[i, c]):
            continue

        def lk(sites):
            pk = rf.PackedScene(*to_dev(sites, scene.off, scene.idx, dens0, sh0), 3)
            rk, _, _ = rf.render_forward(pk, o, d, t, s)
            torch.cuda.synchronize()
            return float((rk.cpu().numpy().astype(np.float64) * gk).sum())

        fds = [(lk(sp) - lk(sm)) / (float(sp[i, c]) - float(sm[i, c])) for sp, sm in steps_]
        # a site whose exits are nearly grazing is not smooth at this step: the
        # two differences disagree, and it is not a test of the gradient
        if abs(fds[0] - fds[1]) > 2e-2 * abs(fds[1]):
            continue
        fd = (4.0 * fds[1] - fds[0]) / 3.0  # Richardson: the h^2 term cancels
        assert abs(fd - gsk[i, c]) <= 2e-2 * abs(gsk[i, c]), (i, c, fds, gsk[i, c], int((~keep).sum()))
        checked += 1
    assert checked >= 3
