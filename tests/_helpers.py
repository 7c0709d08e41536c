"""Hand-built tiny scenes and cameras for the tests."""
import numpy as np

from paper_2311_17089_amd.scenegen import Camera, Scene

Y00 = 0.5 / np.sqrt(np.pi)


def tiny_scene(means, scales, quats=None, opacity=None, colors=None, levels=None,
               n_levels=1, s_max=None, s_min=None, sh_degree=0, sh=None):
    means = np.asarray(means, np.float32).reshape(-1, 3).T.copy()
    n = means.shape[1]
    scales = np.asarray(scales, np.float32).reshape(-1, 3).T.copy()
    if quats is None:
        quats = np.tile(np.array([[1.0], [0.0], [0.0], [0.0]], np.float32), (1, n))
    else:
        quats = np.asarray(quats, np.float32).reshape(-1, 4).T.copy()
    opacity = (np.full(n, 0.8, np.float32) if opacity is None
               else np.asarray(opacity, np.float32).reshape(n))
    K = (sh_degree + 1) ** 2
    if sh is None:
        sh = np.zeros((K * 3, n), np.float32)
        if colors is not None:
            c = np.asarray(colors, np.float64).reshape(n, 3)
            sh[0:3] = ((c - 0.5) / Y00).T
    levels = np.zeros(n, np.uint8) if levels is None else np.asarray(levels, np.uint8)
    s_max = np.full(n, np.inf, np.float32) if s_max is None else np.asarray(s_max, np.float32)
    s_min = np.zeros(n, np.float32) if s_min is None else np.asarray(s_min, np.float32)
    return Scene(n=n, sh_degree=sh_degree, n_levels=n_levels, means=means, scales=scales,
                 quats=quats, opacity=opacity, sh=np.asarray(sh, np.float32), level=levels,
                 s_max=s_max, s_min=s_min)


def axis_camera(W=64, H=64, f=64.0, tz=0.0, cx=None, cy=None):
    """R = I camera at the origin shifted by t = (0, 0, tz)."""
    return Camera(R=np.eye(3, dtype=np.float32).reshape(9), t=np.array([0, 0, tz], np.float32),
                  fx=f, fy=f, cx=W / 2.0 if cx is None else cx, cy=H / 2.0 if cy is None else cy,
                  width=W, height=H)


def quat_to_matrix64(q):
    """Rotation matrix of a (w, x, y, z) quaternion via scipy (an independent route)."""
    from scipy.spatial.transform import Rotation
    w, x, y, z = [float(v) for v in q]
    return Rotation.from_quat([x, y, z, w]).as_matrix()


def pinhole64(cam, mu, downscale=1):
    R = np.asarray(cam.R, np.float64).reshape(3, 3)
    t = np.asarray(cam.t, np.float64)
    pc = R @ np.asarray(mu, np.float64) + t
    return np.array([cam.fx / downscale * pc[0] / pc[2] + cam.cx / downscale,
                     cam.fy / downscale * pc[1] / pc[2] + cam.cy / downscale])


def screen_cov64(cam, mu, scale, quat, downscale=1):
    """V = Jac Sigma Jac^T with Jac the central-difference Jacobian of the pinhole
    map at mu, Sigma = R diag(s^2) R^T from scipy's rotation."""
    Rq = quat_to_matrix64(quat)
    Sig = Rq @ np.diag(np.asarray(scale, np.float64) ** 2) @ Rq.T
    h = 1e-6
    Jac = np.zeros((2, 3))
    for i in range(3):
        e = np.zeros(3)
        e[i] = h
        Jac[:, i] = (pinhole64(cam, np.asarray(mu) + e, downscale)
                     - pinhole64(cam, np.asarray(mu) - e, downscale)) / (2 * h)
    return Jac @ Sig @ Jac.T


def expected_tile_counts(p, Tx, Ty):
    """Per-tile number of drawable Gaussians whose tile rectangle covers the
    tile, from the oracle's projection (2-D difference array over the
    rectangles, no sort)."""
    live = np.nonzero(p["ntiles"] > 0)[0]
    x0, x1, y0, y1 = (p["rect"][i, live].astype(np.int64) for i in range(4))
    diff = np.zeros((Ty + 1, Tx + 1), np.int64)
    np.add.at(diff, (y0, x0), 1)
    np.add.at(diff, (y0, x1 + 1), -1)
    np.add.at(diff, (y1 + 1, x0), -1)
    np.add.at(diff, (y1 + 1, x1 + 1), 1)
    return diff.cumsum(0).cumsum(1)[:Ty, :Tx].ravel()


def assert_keys_match_oracle_definition(kg, vg, p, Tx, chunk=1 << 24):
    """The sorted (tile, depth) list kg/vg against the oracle's definition
    without sorting it on the CPU: (1) every drawable Gaussian k appears
    exactly ntiles[k] times; (2) every instance's tile lies in its Gaussian's
    rectangle and its low 32 bits are the oracle's depth bits of k; (3) the
    list is strictly increasing in (key, k).  (3) rules out a repeated
    (tile, k) pair, so with (1) and (2) the instances of k are exactly the
    tiles of its rectangle; (3) then fixes their order as the stable sort of
    the emission order.  So the list equals the oracle's keys element by
    element."""
    n = p["ntiles"].size
    assert kg.size == vg.size == int(p["ntiles"].sum())
    np.testing.assert_array_equal(np.bincount(vg, minlength=n), p["ntiles"])
    depth_bits = p["depth"].view(np.uint32)
    for a in range(0, kg.size, chunk):
        b = min(kg.size, a + chunk)
        k, v = kg[a:b], vg[a:b]
        tile = (k >> np.uint64(32)).astype(np.int64)
        tx, ty = tile % Tx, tile // Tx
        r = p["rect"][:, v]
        assert np.all((tx >= r[0]) & (tx <= r[1]) & (ty >= r[2]) & (ty <= r[3]))
        np.testing.assert_array_equal((k & np.uint64(0xFFFFFFFF)).astype(np.uint32),
                                      depth_bits[v])
        e = min(kg.size, b + 1)
        k2, v2 = kg[a:e], vg[a:e]
        inc = (k2[1:] > k2[:-1]) | ((k2[1:] == k2[:-1]) & (v2[1:] > v2[:-1]))
        assert np.all(inc)
