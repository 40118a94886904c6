"""Continuous-batching server: results alone and in the mix, admission by memory, errors."""

import numpy as np
import pytest

import oracle
import synth

from parity import T_ATOL, colour_ratio, decidable

pytestmark = pytest.mark.gpu

SIZES = [(64, 48), (33, 17), (128, 96), (8, 8), (100, 70), (1, 1), (56, 80), (130, 9)]


@pytest.fixture(scope="module")
def setup():
    import torch

    if not torch.cuda.is_available():
        pytest.fail("no GPU visible to torch")
    import paper_2502_01157_amd as rf

    scene, rng = synth.small_scene("clustered", 20000, seed=41, sh_deg=3, return_rng=True)
    reqs = []
    for k in range(24):
        w, h = SIZES[k % len(SIZES)]
        cam = synth.make_cameras("serving_1m", rng, n=1, res=(w, h))[0]
        start = int(synth.nearest_site(scene.sites, cam.position[None, :])[0])
        reqs.append(dict(arrival=0.002 * k, pose12=cam.pose12(), fov_deg=cam.fov_deg, width=w, height=h,
                         start_cell=start, camera=cam))
    dv = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()  # noqa: E731
    packed = rf.PackedScene(*map(dv, (scene.sites, scene.off, scene.idx, scene.density, scene.sh)), 3, "f32")
    # each request rendered alone by the batch path (ray generation + forward walk)
    alone = []
    for r in reqs:
        o, d, t, s, px = rf.raygen(r["pose12"], r["fov_deg"], r["width"], r["height"], scene.bound,
                                   r["start_cell"])
        rgb, tf, _ = rf.render_forward(packed, o, d, t, s)
        img = np.zeros((r["height"] * r["width"], 4), dtype=np.float32)
        img[px.cpu().numpy()] = np.concatenate([rgb.cpu().numpy(), tf.cpu().numpy()[:, None]], 1)
        alone.append(img.reshape(r["height"], r["width"], 4))
    torch.cuda.synchronize()
    return rf, scene, packed, reqs, alone


def test_mix_equals_alone_bitwise(setup):
    rf, scene, packed, reqs, alone = setup
    from paper_2502_01157_amd.serve import Server, replay

    # all requests arrive at once: 16 are admitted together and share launches,
    # the rest are admitted as slots free up
    burst = [dict(r, arrival=0.0) for r in reqs]
    with Server(packed, scene.bound, pool_bytes=8 << 20, max_inflight=16) as srv:
        out = replay(srv, burst, keep=range(len(reqs)), timeout_s=20)
        st = srv.stats()
    assert st["completed"] == len(reqs) and st["inflight"] == 0 and st["pool_used_bytes"] == 0
    assert st["launches"] < len(reqs)
    for i, r in enumerate(reqs):
        np.testing.assert_array_equal(out["images"][i], alone[i], err_msg=f"request {i}")
    # staggered arrivals (2 ms apart)
    with Server(packed, scene.bound, pool_bytes=8 << 20, max_inflight=16) as srv:
        out = replay(srv, reqs, keep=range(len(reqs)), timeout_s=20)
    for i, r in enumerate(reqs):
        np.testing.assert_array_equal(out["images"][i], alone[i], err_msg=f"request {i}")
    # and each request alone in the server
    with Server(packed, scene.bound, pool_bytes=8 << 20, max_inflight=4) as srv:
        for i in (0, 2, 5, 7):
            one = replay(srv, [dict(reqs[i], arrival=0.0)], keep=[0], timeout_s=20)
            np.testing.assert_array_equal(one["images"][0], alone[i])


def test_persistent_server_mix_equals_alone_bitwise(setup):
    """The persistent form (one kernel serving requests as they arrive):
    bitwise the batch path's images in a burst, with staggered arrivals, with
    requests whose camera cell the dispatcher locates itself, and after the
    kernel has idled out and been relaunched."""
    import time

    rf, scene, packed, reqs, alone = setup
    from paper_2502_01157_amd.serve import Server, replay

    burst = [dict(r, arrival=0.0) for r in reqs]
    with Server(packed, scene.bound, pool_bytes=8 << 20, max_inflight=16, mode="persistent") as srv:
        print("persistent server: burst", flush=True)
        out = replay(srv, burst, keep=range(len(reqs)), timeout_s=20)
        st = srv.stats()
        for i in range(len(reqs)):
            np.testing.assert_array_equal(out["images"][i], alone[i], err_msg=f"request {i}")
        assert st["completed"] == len(reqs) and st["inflight"] == 0 and st["pool_used_bytes"] == 0
        print("persistent server: staggered, located start cells", flush=True)
        located = [dict(r, start_cell=-1) for r in reqs]
        out = replay(srv, located, keep=range(len(reqs)), timeout_s=20)
        for i in range(len(reqs)):
            np.testing.assert_array_equal(out["images"][i], alone[i], err_msg=f"located request {i}")
        # idle long enough for the kernel to leave, then serve again (a relaunch)
        time.sleep(0.05)
        n0 = srv.stats()["launches"]
        print("persistent server: after idling", flush=True)
        out = replay(srv, burst[:6], keep=range(6), timeout_s=20)
        for i in range(6):
            np.testing.assert_array_equal(out["images"][i], alone[i])
        assert srv.stats()["launches"] > n0


def test_served_images_match_oracle(setup):
    """The served images (the batch path's, which the server reproduces bit
    for bit) against the oracle on the same FP32 rays: colour per element and
    transmittance on every decidable ray."""
    rf, scene, packed, reqs, alone = setup
    osc = oracle.OracleScene.from_scene(scene)
    for i in (0, 2, 4, 6):
        r = reqs[i]
        rays = rf.raygen(r["pose12"], r["fov_deg"], r["width"], r["height"], scene.bound, r["start_cell"])
        o, d, t, s, px = (x.cpu().numpy() for x in rays)
        ref = oracle.trace(osc, o, d, t, s, eps=1e-4, max_len=1)
        dec = decidable(ref, 1e-4)
        assert dec.mean() > 0.9, (i, dec.mean())
        img = alone[i].reshape(-1, 4)[px]
        mean_abs = float(np.abs(ref["rgb"]).mean())
        assert colour_ratio(img[dec, :3], ref["rgb"][dec], mean_abs).max(initial=0.0) <= 1.0, i
        assert np.abs(img[dec, 3] - ref["t_final"][dec]).max(initial=0.0) <= T_ATOL, i


@pytest.mark.parametrize("mode", ["launches", "persistent"])
def test_bf16_scene_served_equals_batch_path(setup, mode):
    """A BF16-attribute scene served in a burst and with staggered arrivals:
    every image bit for bit the BF16 batch path's."""
    import torch

    rf, scene, _, reqs, _ = setup
    from paper_2502_01157_amd.serve import Server, replay

    dv = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()  # noqa: E731
    packed = rf.PackedScene(*map(dv, (scene.sites, scene.off, scene.idx, scene.density, scene.sh)), 3, "bf16")
    alone = []
    for r in reqs:
        o, d, t, s, px = rf.raygen(r["pose12"], r["fov_deg"], r["width"], r["height"], scene.bound,
                                   r["start_cell"])
        rgb, tf, _ = rf.render_forward(packed, o, d, t, s)
        img = np.zeros((r["height"] * r["width"], 4), dtype=np.float32)
        img[px.cpu().numpy()] = np.concatenate([rgb.cpu().numpy(), tf.cpu().numpy()[:, None]], 1)
        alone.append(img.reshape(r["height"], r["width"], 4))
    burst = [dict(r, arrival=0.0) for r in reqs]
    with Server(packed, scene.bound, pool_bytes=8 << 20, max_inflight=16, mode=mode) as srv:
        for label, stream in (("burst", burst), ("staggered", reqs)):
            print(f"bf16 {mode} server: {label}", flush=True)
            out = replay(srv, stream, keep=range(len(reqs)), timeout_s=20)
            for i in range(len(reqs)):
                np.testing.assert_array_equal(out["images"][i], alone[i], err_msg=f"{label} request {i}")


@pytest.mark.parametrize("mode", ["launches", "persistent"])
def test_large_requests_stage_and_equal_batch_path(setup, mode):
    """Launches of 8,192 tiles (the most a launch takes) walk with the cells
    staged in LDS (the batch forward's walk), smaller ones without; the
    persistent workers stage the tiles of requests of 8,192 tiles or more.
    The images are the batch path's bit for bit either way. A 1021x519
    request is 128 x 65 = 8,320 tiles (edge tiles with lanes past the
    image): alone in the launches form, a staged launch of 8,192 tiles and a
    plain one of 128, so both walks render parts of one image; a burst of
    three such requests and a small one fills staged launches that mix
    requests (in the persistent form, workers move between staged and plain
    tiles)."""
    rf, scene, packed, reqs, alone = setup
    from paper_2502_01157_amd.serve import Server, replay

    W, H = 1021, 519
    big = [dict(r, width=W, height=H, arrival=0.0) for r in reqs[:3]] + [dict(reqs[0], arrival=0.0)]
    ref = []
    for r in big:
        o, d, t, s, px = rf.raygen(r["pose12"], r["fov_deg"], r["width"], r["height"], scene.bound,
                                   r["start_cell"])
        rgb, tf, _ = rf.render_forward(packed, o, d, t, s)
        img = np.zeros((r["height"] * r["width"], 4), dtype=np.float32)
        img[px.cpu().numpy()] = np.concatenate([rgb.cpu().numpy(), tf.cpu().numpy()[:, None]], 1)
        ref.append(img.reshape(r["height"], r["width"], 4))
    with Server(packed, scene.bound, pool_bytes=64 << 20, max_inflight=8, mode=mode) as srv:
        one = replay(srv, big[:1], keep=[0], timeout_s=30)
        np.testing.assert_array_equal(one["images"][0], ref[0])
        out = replay(srv, big, keep=range(len(big)), timeout_s=30)
    for i in range(len(big)):
        np.testing.assert_array_equal(out["images"][i], ref[i], err_msg=f"request {i}")


def test_admission_by_memory_and_fifo(setup):
    rf, scene, packed, reqs, alone = setup
    from paper_2502_01157_amd.serve import Server, replay

    big = [dict(r, width=128, height=96) for r in reqs[:6]]
    # room for two 128x96 outputs at a time
    with Server(packed, scene.bound, pool_bytes=2 * 128 * 96 * 16 + 1024, max_inflight=8) as srv:
        ids = [srv.submit(r["pose12"], r["fov_deg"], 128, 96, r["start_cell"]) for r in big[:3]]
        assert ids[0] is not None and ids[1] is not None and ids[2] is None
        with pytest.raises(rf.RfError, match="UNSUPPORTED"):
            srv.submit(big[0]["pose12"], 60.0, 512, 512, 0)
        import time

        t0 = time.time()
        done = set()  # a finished request stays listed until its result is collected
        while len(done) < 2 and time.time() - t0 < 20:
            done.update(srv.poll())
        assert sorted(done) == sorted(ids[:2])
        for rid in done:
            srv.result(rid)
        out = replay(srv, big, keep=range(6), timeout_s=20)
        assert srv.stats()["rejected_busy"] >= 1
    assert np.all(np.isfinite(out["latency_s"]))
    for i in range(6):
        assert out["images"][i].shape == (96, 128, 4)


def test_server_argument_errors(setup):
    rf, scene, packed, reqs, alone = setup
    from paper_2502_01157_amd.serve import Server

    with pytest.raises(rf.RfError, match="INVALID_ARG"):
        Server(packed, scene.bound, max_inflight=0)
    with pytest.raises(rf.RfError, match="INVALID_ARG"):
        Server(packed, scene.bound, max_inflight=65)
    with pytest.raises(rf.RfError, match="INVALID_ARG"):
        Server(packed, scene.bound, pool_bytes=16)
    with pytest.raises(rf.RfError, match="INVALID_ARG"):
        Server(packed, ("box", 0.0, 1.0), eps=-1.0)
    with Server(packed, scene.bound, pool_bytes=1 << 20, max_inflight=2) as srv:
        with pytest.raises(rf.RfError, match="INVALID_ARG"):
            srv.submit(reqs[0]["pose12"], 0.0, 8, 8, 0)
        assert srv.poll() == []


def test_device_located_start_cells(setup):
    """Requests submitted without a start cell (start_cell < 0) are located on
    the device; where the camera's nearest site is not an FP64 near-tie the
    cell is the host's, so the image is the same bit for bit."""
    rf, scene, packed, reqs, alone = setup
    from paper_2502_01157_amd.serve import Server, replay

    pos = np.stack([r["camera"].position for r in reqs]).astype(np.float32)
    ref, gap = oracle.nearest_site(scene.sites, pos, return_gap=True)
    assert (gap > 1e-12).all()
    np.testing.assert_array_equal(ref, [r["start_cell"] for r in reqs])
    located = [dict(r, start_cell=-1) for r in reqs]
    with Server(packed, scene.bound, pool_bytes=8 << 20, max_inflight=16) as srv:
        out = replay(srv, located, keep=range(len(reqs)), timeout_s=20)
    for i in range(len(reqs)):
        np.testing.assert_array_equal(out["images"][i], alone[i], err_msg=f"request {i}")


def test_fisheye_requests_in_the_mix(setup):
    """Fisheye requests (180 and 360 degrees) served among pinhole ones give the
    batch path's images (fisheye raygen + forward walk) bit for bit."""
    import torch

    rf, scene, packed, reqs, alone = setup
    from paper_2502_01157_amd.serve import Server, replay

    mixed, ref = [], []
    for k, r in enumerate(reqs[:12]):
        if k % 3 == 0:
            r = dict(r, model="fisheye", fov_deg=180.0 if k % 2 == 0 else 360.0)
            o, d, t, s, px = rf.raygen(r["pose12"], r["fov_deg"], r["width"], r["height"], scene.bound,
                                       r["start_cell"], model="fisheye")
            rgb, tf, _ = rf.render_forward(packed, o, d, t, s)
            img = np.zeros((r["height"] * r["width"], 4), dtype=np.float32)
            img[px.cpu().numpy()] = np.concatenate([rgb.cpu().numpy(), tf.cpu().numpy()[:, None]], 1)
            ref.append(img.reshape(r["height"], r["width"], 4))
        else:
            ref.append(alone[k])
        mixed.append(dict(r, arrival=0.0))
    torch.cuda.synchronize()
    with Server(packed, scene.bound, pool_bytes=8 << 20, max_inflight=16) as srv:
        out = replay(srv, mixed, keep=range(len(mixed)), timeout_s=20)
        with pytest.raises(rf.RfError):
            srv.submit(reqs[0]["pose12"], 400.0, 8, 8, 0, model="fisheye")
    for i in range(len(mixed)):
        np.testing.assert_array_equal(out["images"][i], ref[i], err_msg=f"request {i}")
