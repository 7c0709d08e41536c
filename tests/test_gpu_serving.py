"""Continuous-batching server (needs an MI355X): every request renders the same
alone and in the mix, served images match the CPU oracle on sampled pixels
(also on the resident 3M-Gaussian serving scene), admission by device memory,
completion records."""
import dataclasses

import numpy as np
import pytest
import torch

import oracle as O
from paper_2311_17089_amd import msgs as M
from paper_2311_17089_amd import scenegen as G

IMG_TOL = 1e-5

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)


def _scene(ctx, with_host=False):
    sc = G.make_scene([60000, 15000, 3750, 940], 41, 3, [-4.2 + 1.4 * l for l in range(4)],
                      blob_fraction0=0.5)
    dsc = M.DeviceScene(ctx, sc)
    M.calibrate(ctx, dsc, G.calibration_cameras(1041, 640, 360, 750.0))
    if with_host:
        return dsc, _host_scene(sc, dsc)
    return dsc


def _host_scene(sc, dsc):
    """The host copy of a device scene with the ranges its calibration wrote."""
    smax, smin = dsc.ranges()
    return dataclasses.replace(sc, s_max=smax, s_min=smin)


def _check_against_oracle(host, reqs, imgs, m, seed):
    """m sampled pixels of every served image against brute-force compositing."""
    rng = np.random.default_rng(seed)
    for i, ((cam, ds, sel), img) in enumerate(zip(reqs, imgs)):
        H, W = img.shape[:2]
        idx = rng.choice(W * H, size=min(m, W * H), replace=False)
        pix = np.stack([idx % W, idx // W], 1).astype(np.int32)
        ref, _, _ = O.render_pixels(host, cam, pix, downscale=ds, selective=sel)
        err = float(np.abs(img[pix[:, 1], pix[:, 0]] - ref).max())
        assert err <= IMG_TOL, (i, ds, sel, err)


def _requests(n, seed):
    rng = np.random.default_rng(seed)
    poses = G.sphere_poses(n, seed, 2.0, 6.0)
    out = []
    for i in range(n):
        ds = int(rng.choice([1, 2, 4, 8, 16, 32]))
        out.append((G.lookat_camera(poses[i], 640, 360, 750.0), ds, bool(rng.integers(2))))
    return out


def _alone(ctx, dsc, reqs):
    imgs = []
    for cam, ds, sel in reqs:
        imgs.append(M.render(ctx, dsc, cam, downscale=ds, selective=sel).clone())
    torch.cuda.synchronize()
    return [x.cpu().numpy() for x in imgs]


def _served(ctx, dsc, reqs, inflight):
    srv = M.Server(ctx, dsc, max_inflight=inflight)
    outs = [torch.full((c.height // ds, c.width // ds, 3), -1.0, device="cuda") for c, ds, _ in reqs]
    torch.cuda.synchronize()
    for i, ((cam, ds, sel), o) in enumerate(zip(reqs, outs)):
        srv.submit(cam, o, i, downscale=ds, selective=sel)
    done = []
    while len(done) < len(reqs):
        done += srv.poll(64, timeout_us=2_000_000)
    srv.close()
    torch.cuda.synchronize()
    return [o.cpu().numpy() for o in outs], done


def test_results_identical_alone_and_in_the_mix():
    ctx = M.Context(0)
    dsc, host = _scene(ctx, with_host=True)
    reqs = _requests(24, 7)
    ref = _alone(ctx, dsc, reqs)
    got, done = _served(ctx, dsc, reqs, inflight=4)
    _check_against_oracle(host, reqs, got, 200, 7)
    assert sorted(d["req_id"] for d in done) == list(range(len(reqs)))
    for d in done:
        assert d["status"] == 0
        assert d["t_submit_us"] <= d["t_start_us"] <= d["t_admit_us"] <= d["t_done_us"]
    for i, (a, b) in enumerate(zip(ref, got)):
        assert np.abs(a - b).max() <= 1e-5, i
        np.testing.assert_array_equal(a, b)
    dsc.close()


def test_admission_under_a_memory_budget():
    # measure the largest request (what its frame keeps; the peak while it
    # renders is about twice that), then allow about three of those at a time:
    # requests must wait for memory, not fail, and stay identical
    probe = M.Context(0)
    dsc = _scene(probe)
    reqs = _requests(16, 9)
    biggest = 0
    for cam, ds, sel in reqs:
        _, fr = M.render(probe, dsc, cam, downscale=ds, selective=sel, keep_frame=True)
        torch.cuda.synchronize()
        biggest = max(biggest, probe.bytes_in_use())
        fr.release()
    ref = _alone(probe, dsc, reqs)
    dsc.close()
    ctx = M.Context(0, pool_bytes=int(biggest * 3))
    dsc2 = _scene(ctx)
    got, done = _served(ctx, dsc2, reqs, inflight=6)
    _say(f"  budget {int(biggest * 3)} bytes, {len(done)} completions")
    assert all(d["status"] == 0 for d in done)
    for a, b in zip(ref, got):
        np.testing.assert_array_equal(a, b)
    # a request that cannot fit even alone completes with MSGS_E_NOMEM
    tiny = M.Context(0, pool_bytes=1 << 20)
    dsc3 = M.DeviceScene(tiny, G.make_scene([200000], 3, 0, [-3.0]))
    srv = M.Server(tiny, dsc3, max_inflight=2)
    cam = G.lookat_camera([0, 0, -3], 640, 360, 750.0)
    out = torch.empty((360, 640, 3), device="cuda")
    torch.cuda.synchronize()
    srv.submit(cam, out, 77)
    d = []
    while not d:
        d = srv.poll(4, timeout_us=2_000_000)
    assert d[0]["req_id"] == 77 and d[0]["status"] == M.E_NOMEM
    srv.close()
    dsc3.close()
    dsc2.close()


def test_invalid_submission_is_rejected():
    ctx = M.Context(0)
    dsc = M.DeviceScene(ctx, G.make_scene([100], 3, 0, [-3.0]))
    srv = M.Server(ctx, dsc, max_inflight=1)
    cam = G.lookat_camera([0, 0, -3], 64, 64, 64.0)
    with pytest.raises(M.MsgsError) as e:
        srv.submit(cam, torch.empty((1, 1, 3), device="cuda"), 1, downscale=0)
    assert e.value.code == M.E_INVALID
    srv.close()
    dsc.close()


def test_serving_scene_3m_matches_oracle():
    # the resident 3M-Gaussian, 4-level serving scene: a few requests of the
    # serving mix (poses on a sphere of radius 2-12, 1920x1080 downscaled by
    # 1..128, selective and single-scale) served concurrently, sampled pixels
    # of each against brute force, and identical to the same renders alone
    ctx = M.Context(0)
    sc = G.large_scene(3_000_000, 4, 3)
    dsc = M.DeviceScene(ctx, sc)
    M.calibrate(ctx, dsc, G.calibration_cameras(1003, 1920, 1080, 2250.0))
    host = _host_scene(sc, dsc)
    rng = np.random.default_rng(44)
    poses = G.sphere_poses(6, 44, 2.0, 12.0)
    reqs = [(G.lookat_camera(poses[i], 1920, 1080, 2250.0), int(d), bool(s))
            for i, (d, s) in enumerate(zip((1, 128, 8, 32, 2, 64), rng.integers(0, 2, 6)))]
    reqs[0] = (reqs[0][0], 1, True)
    _say("  3M scene: " + ", ".join(f"ds={d} sel={s}" for _, d, s in reqs))
    ref = _alone(ctx, dsc, reqs)
    got, done = _served(ctx, dsc, reqs, inflight=3)
    assert all(d["status"] == 0 for d in done)
    for a, b in zip(ref, got):
        np.testing.assert_array_equal(a, b)
    _check_against_oracle(host, reqs, got, 256, 45)
    dsc.close()
