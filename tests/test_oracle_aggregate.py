"""Pins of the aggregation oracle (Alg. 1 and its supplementary details)
against closed forms and hand-worked cases."""
import dataclasses

import numpy as np
import pytest

import oracle as O
from oracle import aggregate as A
from paper_2311_17089_amd import scenegen as G

F32 = np.float32


def _one(means, scales, opacity=0.9, level=0, sh_degree=0, quats=None):
    """Scene of the given Gaussians (columns), identity rotations by default."""
    means = np.asarray(means, F32).reshape(3, -1)
    n = means.shape[1]
    scales = np.asarray(scales, F32).reshape(3, -1)
    q = np.zeros((4, n), F32)
    q[0] = 1.0
    if quats is not None:
        q = np.asarray(quats, F32).reshape(4, n)
    K3 = 3 * (sh_degree + 1) ** 2
    sh = np.linspace(-0.3, 0.4, K3 * n, dtype=F32).reshape(K3, n)
    return G.Scene(n=n, sh_degree=sh_degree, n_levels=4, means=means, scales=scales, quats=q,
                   opacity=np.full(n, opacity, F32) if np.isscalar(opacity) else np.asarray(opacity, F32),
                   sh=sh, level=np.full(n, level, np.uint8) if np.isscalar(level) else np.asarray(level, np.uint8),
                   s_max=np.zeros(n, F32), s_min=np.full(n, np.inf, F32))


def _front_cam(W=256, H=192, f=300.0):
    # at distance 3 on the -z side looking at the origin: axis-aligned, R = I
    return G.Camera(R=np.eye(3, dtype=F32).reshape(9), t=np.array([0, 0, 3], F32), fx=f, fy=f,
                    cx=W / 2.0, cy=H / 2.0, width=W, height=H)


def test_normalise_inside_is_linear_and_outside_contracts():
    B = F32(3.0)
    x = np.array([[0.5, -2.9, 3.0], [1.0, 0.0, -3.0], [-2.0, 1.5, 0.25]], F32)
    np.testing.assert_array_equal(A.normalise(x, B), (x / B).astype(F32))
    # continuity at the cube surface, contraction and the bound 2 outside
    d = np.array([0.3, -0.8, 1.0], F32)
    ms = np.array([3.0, 3.0001, 4.0, 30.0, 3e4], F32)
    pts = (d[:, None] * ms[None, :]).astype(F32)
    xn = A.normalise(pts, B)
    r = np.max(np.abs(xn), axis=0)
    assert abs(r[0] - 1.0) < 1e-6 and abs(r[1] - 1.0) < 1e-4
    assert np.all(np.diff(r) > 0) and np.all(r < 2.0)
    np.testing.assert_allclose(r[2:], 2.0 - 3.0 / ms[2:], rtol=1e-6)
    # direction is kept
    np.testing.assert_allclose(xn / r, pts / np.max(np.abs(pts), 0), rtol=1e-6)


def test_voxel_ids_by_hand():
    xn = np.array([[-2.0, 1.99, 2.0, 0.0], [-2.0, 0.0, 2.0, -0.01], [-2.0, -1.0, 2.0, 1.0]], F32)
    v = A.voxel_ids(xn, 4)
    # (-2,-2,-2) -> 0; (1.99, 0, -1) -> x 3, y 2, z 1; +2 clamps to 3; (0,-0.01,1) -> 2,1,3
    assert list(v) == [0, (1 * 4 + 2) * 4 + 3, (3 * 4 + 3) * 4 + 3, (3 * 4 + 1) * 4 + 2]
    assert A.grid_resolution(1) == 200 and A.grid_resolution(2) == 133 and A.grid_resolution(3) == 100


def test_choice_truth_table():
    cam_a = _front_cam()
    cam_b = G.Camera(R=np.eye(3, dtype=F32).reshape(9), t=np.array([0, 0, 0.5], F32), fx=300.0,
                     fy=300.0, cx=128.0, cy=96.0, width=256, height=192)
    sc = _one([[0.0, 0.3, 0.0, -0.3, 0.0], [0.0, 0.0, 0.0, 0.0, 0.3], [0.0, 0.0, -4.0, 0.0, 0.0]],
              [[0.004, 0.2, 0.004, 0.004, 0.004]] * 3, level=[0, 0, 0, 1, 0])
    smin, below = A.min_coverage(sc, [cam_a, cam_b], 1)
    pa = O.project(sc, cam_a, downscale=4, selective=False)
    pb = O.project(sc, cam_b, downscale=4, selective=False)
    # Gaussian 2 is behind both cameras (z = -4 < near of each)
    assert pa["ntiles"][2] == 0 and pb["ntiles"][2] == 0 and np.isinf(smin[2])
    # Gaussian 3 is of level 1: never a candidate for level 1
    assert not below[3] and np.isinf(smin[3])
    # the minimum over the cameras that draw the Gaussian
    for k in (0, 1, 4):
        s = [p["S"][k] for p in (pa, pb) if p["ntiles"][k] > 0]
        assert smin[k] == min(s)
    _, chosen, _ = A.aggregate_level(sc, [cam_a, cam_b], 1)
    assert chosen[0] and chosen[4] and not chosen[1] and not chosen[2] and not chosen[3]
    assert smin[1] >= 2.0 and smin[0] < 2.0


def test_single_gaussian_is_enlarged_to_the_threshold():
    cam = _front_cam()
    sc = _one([[0.05], [-0.02], [0.1]], [[0.003], [0.004], [0.0035]],
              quats=[[0.9], [0.1], [-0.2], [0.3]], sh_degree=1)
    part, chosen, _ = A.aggregate_level(sc, [cam], 1)
    assert chosen[0] and part.n == 1
    np.testing.assert_allclose(part.means[:, 0], sc.means[:, 0], rtol=1e-7)
    q = sc.quats[:, 0].astype(np.float64)
    np.testing.assert_allclose(part.quats[:, 0], q / np.linalg.norm(q), rtol=1e-6)
    np.testing.assert_allclose(part.sh[:, 0], sc.sh[:, 0], rtol=1e-7)
    assert part.opacity[0] == sc.opacity[0] and part.level[0] == 1
    S = O.project(sc, cam, downscale=4, selective=False)["S"][0]
    np.testing.assert_allclose(part.scales[:, 0], sc.scales[:, 0] * (2.0 / S), rtol=1e-6)
    # the enlarged Gaussian covers S_T = 2 px at that camera and scale
    S2 = O.project(part, cam, downscale=4, selective=False)["S"][0]
    assert abs(S2 - 2.0) < 2e-5


def test_enlarged_bandwidth_is_below_nyquist():
    # supplementary closed form: after enlargement the Gaussian's screen-space
    # exponent a' = 1 / (2 var) equals ln(N) (here ln(255 sigma)), so its 3 dB
    # bandwidth sqrt(a' ln sqrt 2) / pi is 0.441 px^-1 for sigma -> 1
    cam = _front_cam()
    sig = 0.999999
    sc = _one([[0.0], [0.0], [0.0]], [[0.003]] * 3, opacity=sig)
    part, _, _ = A.aggregate_level(sc, [cam], 1)
    p = O.project(part, cam, downscale=4, selective=False)
    var = float(p["V"][0, 0])
    assert abs(float(p["V"][1, 0]) / var) < 1e-6 and abs(float(p["V"][2, 0]) - var) < 1e-5 * var
    a2 = 1.0 / (2.0 * var)
    assert abs(a2 - np.log(255.0 * sig)) < 2e-4 * a2
    f3db = np.sqrt(a2 * np.log(np.sqrt(2.0))) / np.pi
    assert abs(f3db - 0.441) < 5e-4 and f3db < 0.5


def test_two_gaussians_share_a_voxel():
    cam = _front_cam()
    sc = _one([[0.001, 0.0012], [0.002, 0.0021], [0.0, 0.0001]],
              [[0.002, 0.004], [0.003, 0.002], [0.0025, 0.003]], opacity=[0.5, 0.9],
              quats=[[1.0, 0.8], [0.0, 0.2], [0.0, 0.0], [0.0, 0.6]], sh_degree=0)
    part, chosen, vox = A.aggregate_level(sc, [cam], 1)
    assert chosen.all() and part.n == 1 and vox.size == 1
    p = O.project(sc, cam, downscale=4, selective=False)
    q = sc.quats.astype(np.float64)
    q = q / np.linalg.norm(q, axis=0)
    np.testing.assert_allclose(part.means[:, 0], sc.means.astype(np.float64).mean(1), rtol=1e-6)
    np.testing.assert_allclose(part.quats[:, 0], q.mean(1), rtol=1e-6)
    assert abs(part.opacity[0] - 0.7) < 1e-7
    np.testing.assert_allclose(part.sh[:, 0], sc.sh.astype(np.float64).mean(1), rtol=1e-6)
    s_avg = (float(p["S"][0]) + float(p["S"][1])) / 2.0
    np.testing.assert_allclose(part.scales[:, 0],
                               sc.scales.astype(np.float64).mean(1) * 2.0 / s_avg, rtol=1e-6)


def test_levels_build_on_the_levels_below():
    sc = G.make_scene([6000], 3, 1, [-4.6])
    cams = G.calibration_cameras(1011, 192, 128, 180.0)
    full, added = A.build_levels(sc, cams, 3)
    assert full.n == sc.n + sum(added) and full.n_levels == 3
    assert np.bincount(full.level, minlength=3).tolist() == [sc.n] + added
    # level-2 aggregation draws on the level-1 Gaussians created before it
    lvl1 = np.nonzero(full.level == 1)[0]
    smin, below = A.min_coverage(full, cams, 2)
    assert below[lvl1].all() and np.any(smin[lvl1] < 2.0)
    assert added[0] > 0 and added[1] > 0
