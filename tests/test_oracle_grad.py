"""Pins of the oracle's fp64 frozen-decision gradient (CPU only).

Finite differences of the same fp64 forward do not use autograd, so they pin
the autograd gradient; the SH and opacity closed forms pin it independently of
the forward's implementation."""
import numpy as np
import pytest
import torch

import oracle as O
from oracle import grad64
from paper_2311_17089_amd import scenegen as G
from _helpers import axis_camera, tiny_scene


def _scene(seed, n=400, D=3):
    sc = G.make_scene([int(n * 0.75), n - int(n * 0.75)], seed, D, [-3.2, -2.2], sh_std=0.25)
    return G.open_ranges(sc)


@pytest.mark.parametrize("seed", [5, 6])
def test_autograd_matches_central_differences(seed):
    sc = _scene(seed)
    cam = G.lookat_camera(G.sphere_poses(1, seed, 2.8, 3.2)[0], 64, 48, 60.0)
    F = grad64.Frozen(sc, cam)
    rng = np.random.default_rng(seed)
    Gw = rng.standard_normal((F.pix.shape[0], 3))
    g = F.grad(Gw)
    used = np.unique(F.ks)
    for which, ncomp in (("means", 3), ("scales", 3), ("quats", 4), ("opacity", 1), ("sh", 48)):
        for _ in range(4):
            k = int(rng.choice(used))
            c = int(rng.integers(ncomp))
            an = g[which][k] if which == "opacity" else g[which][c, k]
            fd = F.loss_fd(Gw, which, c, k, h=1e-3)
            assert abs(an - fd) <= 1e-6 * max(abs(fd), 1e-4), (which, c, k, an, fd)


def test_sh_gradient_closed_form():
    # dL/df_{j,c} = Y_j(dir) * sum_p G_pc alpha_p T_p for an unclamped channel,
    # so grad_sh[j, c] / grad_sh[0, c] = Y_j(dir) / Y_0.
    sc = _scene(8, n=200)
    cam = G.lookat_camera([0.2, -0.4, -3.0], 48, 48, 50.0)
    F = grad64.Frozen(sc, cam)
    Gw = np.random.default_rng(1).standard_normal((F.pix.shape[0], 3))
    g = F.grad(Gw)["sh"].reshape(16, 3, sc.n)
    C = -(np.asarray(cam.R, np.float64).reshape(3, 3).T @ np.asarray(cam.t, np.float64))
    checked = 0
    for k in np.unique(F.ks)[:40]:
        d = sc.means[:, k].astype(np.float64) - C
        d /= np.linalg.norm(d)
        Y = O.sh_basis(3, d[:, None])[:, 0]
        for c in range(3):
            if F.proj["cclamp"][c, k] or abs(g[0, c, k]) < 1e-9:
                continue
            np.testing.assert_allclose(g[:, c, k] / g[0, c, k], Y / Y[0], rtol=1e-9, atol=1e-12)
            checked += 1
    assert checked > 20


def test_opacity_gradient_single_gaussian_closed_form():
    # one Gaussian, bg = 0: image = c alpha with alpha = sigma e^power, so
    # dL/dsigma = sum_p G_p . c alpha_p / sigma over unclamped contributing pixels.
    s = tiny_scene([[0.05, 0.0, 4.0]], [[0.06, 0.04, 0.05]], opacity=[0.6],
                   colors=[[0.8, 0.3, 0.5]])
    cam = axis_camera(W=32, H=32, f=64.0)
    F = grad64.Frozen(s, cam)
    Gw = np.random.default_rng(2).standard_normal((F.pix.shape[0], 3))
    g = F.grad(Gw)
    rgb, _ = F.forward(grad64.scene_params64(s, False))
    rgb = rgb.numpy()
    ref = float((Gw * rgb).sum() / float(np.float32(0.6)))
    assert abs(g["opacity"][0] - ref) <= 1e-10 * abs(ref)
