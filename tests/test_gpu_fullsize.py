"""Full-size parity on the 3M-Gaussian, 4-level scene at 1920x1080 (needs an
MI355X): forward at 1x and 8x against the oracle (selection bit-exact over all
3M Gaussians, sampled pixels against brute force), and the backward of the L2
loss against a seeded random target, checked on 64 parameters stratified over
(means, scales, quats, opacity, SH) against frozen-branch central differences
of the fp64 oracle, plus the fp64 oracle gradient of every parameter of the
sampled Gaussians.

A Gaussian's parameters change only the pixels of its tiles, so each check
runs the fp64 oracle on those pixels over the Gaussians whose tile rectangle
meets them (a superset of the pixels' contributors, which leaves every
per-pixel decision as it is in the full scene).
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
IMG_TOL = 1e-5
GROUPS = (("means", 3), ("scales", 3), ("quats", 4), ("opacity", 1), ("sh", 48))


def _say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def setup():
    _say("  building the 3M-Gaussian 4-level scene and its oracle calibration")
    sc = G.large_scene(3_000_000, 4, 3)
    cal = O.calibrate(sc, G.calibration_cameras(1003, W_FULL, H_FULL, F_FULL))
    cam = G.Camera(R=np.eye(3, dtype=np.float32).reshape(9), t=np.array([0, 0, 3], np.float32),
                   fx=F_FULL, fy=F_FULL, cx=W_FULL / 2.0, cy=H_FULL / 2.0, width=W_FULL,
                   height=H_FULL)
    ctx = M.Context(0)
    dsc = M.DeviceScene(ctx, cal)
    yield ctx, cal, dsc, cam
    dsc.close()
    torch.cuda.synchronize()


def _tiles_px(r, W, H):
    """Pixels of the tile rectangle r = (x_lo, x_hi, y_lo, y_hi) (inclusive tiles)."""
    x0, x1 = int(r[0]) * 16, min(W, (int(r[1]) + 1) * 16)
    y0, y1 = int(r[2]) * 16, min(H, (int(r[3]) + 1) * 16)
    yy, xx = np.mgrid[y0:y1, x0:x1]
    return np.stack([xx.ravel(), yy.ravel()], 1).astype(np.int32)


@pytest.mark.parametrize("ds", [1, 8])
def test_full_size_forward_and_gradient(setup, ds):
    ctx, sc, dsc, cam = setup
    W, H = W_FULL // ds, H_FULL // ds
    _say(f"  3M scene {W}x{H} (downscale {ds}): forward")
    rgb, fr = M.render(ctx, dsc, cam, downscale=ds, keep_frame=True)
    torch.cuda.synchronize()
    st = fr.stats()
    p = O.project(sc, cam, downscale=ds)
    np.testing.assert_array_equal(fr.selection(), p["sel"])
    assert st["n_instances"] == int(p["ntiles"].sum())
    assert st["n_visible"] == int((p["ntiles"] > 0).sum())
    if ds == 8:
        kg, vg = fr.keys()
        ko, vo = O.keys(sc, cam, downscale=ds)
        np.testing.assert_array_equal(kg, ko)
        np.testing.assert_array_equal(vg, vo)
    rng = np.random.default_rng(ds)
    idx = rng.choice(W * H, size=1000, replace=False)
    pix = np.stack([idx % W, idx // W], 1).astype(np.int32)
    img = rgb.cpu().numpy()
    T_g, nc_g = fr.state()
    r_o, T_o, n_o = O.render_pixels(sc, cam, pix, downscale=ds)
    assert np.abs(img[pix[:, 1], pix[:, 0]] - r_o).max() <= IMG_TOL
    assert np.abs(T_g[pix[:, 1], pix[:, 0]] - T_o).max() <= IMG_TOL
    np.testing.assert_array_equal(nc_g[pix[:, 1], pix[:, 0]], n_o)

    _say("  backward of the L2 loss")
    target = G.random_target(103, H, W)
    dl = (2.0 * (img.astype(np.float64) - target) / img.size).astype(np.float32)
    g = M.render_backward(ctx, fr, torch.from_numpy(dl).cuda())
    torch.cuda.synchronize()
    got = {k: v.cpu().numpy() for k, v in g.items()}
    fr.release()
    rms = {k: float(np.sqrt(np.mean(got[k].astype(np.float64) ** 2))) for k, _ in GROUPS}

    # Gaussians with a small footprint that contribute; 64 parameters over them
    rect = p["rect"]
    cand = np.nonzero((p["ntiles"] > 0) & (p["ntiles"] <= 4) & (got["opacity"] != 0))[0]
    frng = np.random.default_rng(203)
    ks = frng.choice(cand, size=16, replace=False)
    lo_x, hi_x, lo_y, hi_y = rect
    checked = 0
    for k in ks:
        pix_k = _tiles_px(rect[:, k], W, H)
        r = rect[:, k]
        near = np.nonzero((p["ntiles"] > 0) & (lo_x <= r[1]) & (hi_x >= r[0]) &
                          (lo_y <= r[3]) & (hi_y >= r[2]))[0]
        sub = sc.subset(near)
        kk = int(np.searchsorted(near, k))
        assert near[kk] == k
        Fz = grad64.Frozen(sub, cam, ds, pix_xy=pix_k)
        Gw = dl[pix_k[:, 1], pix_k[:, 0]].astype(np.float64)
        # oracle gradient of every parameter of Gaussian k
        ref = Fz.grad(Gw)
        for name, ncomp in GROUPS:
            a = got[name][k] if name == "opacity" else got[name][:, k]
            b = ref[name][kk] if name == "opacity" else ref[name][:, kk]
            tol = 1e-3 * np.maximum(np.abs(b), 1e-2 * rms[name]) + 1e-12
            assert np.all(np.abs(a - b) <= tol), (name, int(k), a, b)
        # four parameters of this Gaussian against central differences
        for name, ncomp in [GROUPS[i] for i in frng.choice(5, size=4, replace=False)]:
            c = int(frng.integers(ncomp))
            fd = Fz.loss_fd(Gw, name, c, kk, h=1e-3)
            gv = got[name][k] if name == "opacity" else got[name][c, k]
            scale = max(abs(fd), 1e-2 * rms[name])
            assert abs(gv - fd) <= 1e-3 * scale + 1e-12, (name, c, int(k), gv, fd)
            checked += 1
    assert checked == 64
    _say(f"  checked {checked} parameters by central differences and "
         f"{len(ks)} Gaussians against the oracle gradient")
