"""Multi-view training step at full size (needs an MI355X): the 6M-Gaussian,
5-level scene, 8 views with seeded poses, one at each downscale 1, 2, ..., 128
of 1920x1080, rendered in order with the range update on (level l is updated
by the view at downscale 4^l, after that view's selection) and the gradients
of the per-view L2 losses accumulated into one set of planes.

Checks: S^max/S^min after the step bit-exact against the oracle applying the
same updates in the same order; the accumulated gradient of sampled Gaussians
against the sum over views of the fp64 oracle gradient (each view with the
ranges it saw), on the pixels of the Gaussian's tiles; accumulation into zeros
equals the written gradient bit for bit.
"""
import numpy as np
import pytest
import torch

import oracle as O
from oracle import grad64
from paper_2311_17089_amd import msgs as M
from paper_2311_17089_amd import scenegen as G

pytestmark = pytest.mark.gpu

W_FULL, H_FULL, F_FULL = 1920, 1080, 2250.0
NAMES = ("means", "scales", "quats", "opacity", "sh")


def _say(*a):
    print(*a, flush=True)


def _views():
    poses = G.sphere_poses(8, 5, 2.0, 12.0)
    return [(G.lookat_camera(poses[i], W_FULL, H_FULL, F_FULL), 2 ** i) for i in range(8)]


def _tiles_px(r, W, H):
    x0, x1 = int(r[0]) * 16, min(W, (int(r[1]) + 1) * 16)
    y0, y1 = int(r[2]) * 16, min(H, (int(r[3]) + 1) * 16)
    yy, xx = np.mgrid[y0:y1, x0:x1]
    return np.stack([xx.ravel(), yy.ravel()], 1).astype(np.int32)


def test_training_step_6m_eight_views():
    _say("  building the 6M-Gaussian 5-level scene and its oracle calibration")
    sc = G.large_scene(6_000_000, 5, 5)
    cal = O.calibrate(sc, G.calibration_cameras(1005, W_FULL, H_FULL, F_FULL))
    views = _views()
    ctx = M.Context(0)
    dsc = M.DeviceScene(ctx, cal)
    grads = {k: torch.zeros_like(dsc.t[k]) for k in NAMES}
    dls = []
    torch.cuda.synchronize()
    for i, (cam, d) in enumerate(views):
        _say(f"  view {i}: downscale {d}")
        rgb, fr = M.render(ctx, dsc, cam, downscale=d, update_range=True, keep_frame=True)
        img = rgb.cpu().numpy()
        target = G.random_target(100 + i, img.shape[0], img.shape[1])
        dl = (2.0 * (img.astype(np.float64) - target) / img.size).astype(np.float32)
        dls.append(dl)
        M.render_backward(ctx, fr, torch.from_numpy(dl).cuda(), grads=grads, accumulate=True)
        fr.release()
    torch.cuda.synchronize()
    got = {k: v.cpu().numpy() for k, v in grads.items()}
    smax_g, smin_g = dsc.ranges()

    # the oracle: the same updates in the same order, keeping each view's ranges
    state = cal.copy()
    ranges, projs = [], []
    for cam, d in views:
        ranges.append((state.s_max.copy(), state.s_min.copy()))
        p = O.project(state, cam, downscale=d)
        projs.append({"ntiles": p["ntiles"], "rect": p["rect"]})
        del p
        O.update_range(state, cam, d)
    np.testing.assert_array_equal(smax_g, state.s_max)
    np.testing.assert_array_equal(smin_g, state.s_min)
    _say("  ranges after the step match the oracle")

    # Gaussians drawn in some view with a small footprint in every view that draws them
    drawn = np.stack([p["ntiles"] > 0 for p in projs])            # [8, n]
    small = np.all(np.stack([p["ntiles"] for p in projs]) <= 4, axis=0)
    nviews = drawn.sum(0)
    cand2 = np.nonzero((nviews >= 2) & small & (got["opacity"] != 0))[0]
    cand1 = np.nonzero((nviews >= 1) & small & (got["opacity"] != 0))[0]
    rng = np.random.default_rng(505)
    ks = list(rng.choice(cand2, size=min(4, cand2.size), replace=False)) + \
        list(rng.choice(cand1, size=4, replace=False))
    rms = {k: float(np.sqrt(np.mean(got[k].astype(np.float64) ** 2))) for k in NAMES}
    for k in ks:
        ref = {name: 0.0 for name in NAMES}
        for i, (cam, d) in enumerate(views):
            p = projs[i]
            if p["ntiles"][k] == 0:
                continue
            W, H = W_FULL // d, H_FULL // d
            r = p["rect"][:, k]
            lo_x, hi_x, lo_y, hi_y = p["rect"]
            near = np.nonzero((p["ntiles"] > 0) & (lo_x <= r[1]) & (hi_x >= r[0]) &
                              (lo_y <= r[3]) & (hi_y >= r[2]))[0]
            sub = cal.subset(near)
            sub.s_max[:] = ranges[i][0][near]
            sub.s_min[:] = ranges[i][1][near]
            kk = int(np.searchsorted(near, k))
            pix = _tiles_px(r, W, H)
            Fz = grad64.Frozen(sub, cam, d, pix_xy=pix)
            g = Fz.grad(dls[i][pix[:, 1], pix[:, 0]].astype(np.float64))
            for name in NAMES:
                ref[name] = ref[name] + (g[name][kk] if name == "opacity" else g[name][:, kk])
        for name in NAMES:
            a = got[name][k] if name == "opacity" else got[name][:, k]
            b = np.asarray(ref[name])
            tol = 1e-3 * np.maximum(np.abs(b), 1e-2 * rms[name]) + 1e-12
            assert np.all(np.abs(a - b) <= tol), (name, int(k), int(nviews[k]), a, b)
    _say(f"  accumulated gradients of {len(ks)} Gaussians match the oracle "
         f"({min(4, cand2.size)} drawn in two or more views)")

    # accumulating into zeros == writing
    cam, d = views[2]
    rgb, fr = M.render(ctx, dsc, cam, downscale=d, keep_frame=True)
    dl = torch.from_numpy(dls[2]).cuda()
    w = M.render_backward(ctx, fr, dl)
    z = {k: torch.zeros_like(dsc.t[k]) for k in NAMES}
    M.render_backward(ctx, fr, dl, grads=z, accumulate=True)
    torch.cuda.synchronize()
    fr.release()
    for name in NAMES:
        np.testing.assert_array_equal(w[name].cpu().numpy(), z[name].cpu().numpy())
    dsc.close()
