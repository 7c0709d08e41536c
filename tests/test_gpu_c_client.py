"""The C ABI from a plain C99 program (tests/c_client/render_c.c, built by
__graft_entry__.build()): the same scene and camera rendered and
differentiated by the C client and by the Python binding give identical
images, counts and opacity gradients (needs an MI355X)."""
import os
import subprocess
import tempfile

import numpy as np
import pytest
import torch

from paper_2311_17089_amd import msgs as M
from paper_2311_17089_amd import scenegen as G

pytestmark = pytest.mark.gpu
CLIENT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c_client", "render_c")


def _write_input(path, sc, cam, ds, selective):
    with open(path, "wb") as f:
        f.write(np.int64(sc.n).tobytes())
        f.write(np.array([sc.sh_degree, sc.n_levels, ds, int(selective)], np.int32).tobytes())
        f.write(np.asarray(cam.R, np.float32).tobytes())
        f.write(np.asarray(cam.t, np.float32).tobytes())
        f.write(np.array([cam.fx, cam.fy, cam.cx, cam.cy], np.float32).tobytes())
        f.write(np.array([cam.width, cam.height], np.int32).tobytes())
        for a in (sc.means, sc.scales, sc.quats, sc.opacity, sc.sh):
            f.write(np.ascontiguousarray(a, np.float32).tobytes())
        f.write(np.ascontiguousarray(sc.level, np.uint8).tobytes())
        f.write(np.ascontiguousarray(sc.s_max, np.float32).tobytes())
        f.write(np.ascontiguousarray(sc.s_min, np.float32).tobytes())


def _read_output(path, n):
    b = open(path, "rb").read()
    W, H = np.frombuffer(b, np.int32, 2)
    o = 8
    rgb = np.frombuffer(b, np.float32, H * W * 3, o).reshape(H, W, 3)
    o += H * W * 3 * 4
    cnt = np.frombuffer(b, np.int64, 3, o)
    o += 24
    dop = np.frombuffer(b, np.float32, n, o)
    return rgb, cnt, dop


@pytest.mark.parametrize("ds,selective", [(1, True), (4, True), (2, False)])
def test_c_client_matches_python_binding(ds, selective):
    assert os.path.exists(CLIENT), "run __graft_entry__.build() first"
    sc = G.make_scene([6000, 1500, 375], 21, 3, [-4.2, -2.8, -1.4])
    cams = G.calibration_cameras(1021, 192, 128, 220.0)
    ctx = M.Context(0)
    dsc = M.DeviceScene(ctx, sc)
    M.calibrate(ctx, dsc, cams)
    s_max, s_min = dsc.ranges()
    sc.s_max[:] = s_max
    sc.s_min[:] = s_min
    cam = G.lookat_camera([0.3, -0.2, -2.6], 192, 128, 220.0)
    rgb, fr = M.render(ctx, dsc, cam, downscale=ds, selective=selective, keep_frame=True)
    st = fr.stats()
    g = M.render_backward(ctx, fr, torch.ones_like(rgb))
    torch.cuda.synchronize()
    ref_rgb, ref_dop = rgb.cpu().numpy(), g["opacity"].cpu().numpy()
    fr.release()
    dsc.close()
    with tempfile.TemporaryDirectory() as d:
        fin, fout = os.path.join(d, "in.bin"), os.path.join(d, "out.bin")
        _write_input(fin, sc, cam, ds, selective)
        r = subprocess.run([CLIENT, fin, fout], capture_output=True, text=True, timeout=120)
        assert r.returncode == 0, r.stderr
        got_rgb, cnt, got_dop = _read_output(fout, sc.n)
    np.testing.assert_array_equal(got_rgb, ref_rgb)
    assert list(cnt) == [st["n_selected"], st["n_instances"], st["n_blends"]]
    np.testing.assert_array_equal(got_dop, ref_dop)
