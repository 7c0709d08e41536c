"""The render entry point that allocates nothing (msgs_render_noalloc), through
the C ABI, against msgs_render on the same inputs: bit-identical images on two
calls in a row, the second with a smaller scene and frame; the counts it
reports; no device memory taken from the context; size limits rejected with
MSGS_E_CAPACITY."""
import numpy as np
import pytest
import torch

from paper_2311_17089_amd import msgs as M
from paper_2311_17089_amd import scenegen as G

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)


def _case(ctx, counts, n_per_level, seed, W, H, ds, selective):
    sc = G.make_scene(n_per_level, seed, 3, [-4.2 + 1.4 * l for l in range(len(n_per_level))],
                      blob_fraction0=0.5)
    dsc = M.DeviceScene(ctx, sc)
    M.calibrate(ctx, dsc, G.calibration_cameras(seed + 1000, W, H, 1.2 * W))
    cam = G.lookat_camera(G.sphere_poses(1, seed, 2.4, 3.4)[0], W, H, 1.2 * W)
    ref, fr = M.render(ctx, dsc, cam, downscale=ds, selective=selective, keep_frame=True)
    st = fr.stats()
    fr.release()
    torch.cuda.synchronize()
    used = ctx.bytes_in_use()
    out = torch.full_like(ref, -1.0)
    M.render_noalloc(ctx, dsc, cam, out, counts, downscale=ds, selective=selective)
    torch.cuda.synchronize()
    assert ctx.bytes_in_use() == used  # nothing taken from the context
    np.testing.assert_array_equal(out.cpu().numpy(), ref.cpu().numpy())
    c = counts.cpu().numpy()
    assert c[0] == st["n_visible"] and c[1] == st["n_instances"] and c[2] == c[1], (c, st)
    _say(f"  noalloc n={sc.n} {W}x{H} ds={ds}: {c[1]} instances, identical")
    return dsc, cam


def test_noalloc_matches_render_twice_then_smaller():
    ctx = M.Context(0)
    counts = torch.zeros(3, dtype=torch.int64, device="cuda")
    a, _ = _case(ctx, counts, [80000, 20000, 5000, 1250], 81, 640, 480, 1, True)
    b, _ = _case(ctx, counts, [6000, 1500, 380], 82, 200, 150, 2, False)
    a.close()
    b.close()
    ctx.close()


def test_noalloc_capacity_limits():
    ctx = M.Context(0)
    sc = G.make_scene([3000], 83, 0, [-3.0])
    dsc = M.DeviceScene(ctx, sc)
    cam = G.lookat_camera([0.1, 0.2, -3.0], 320, 240, 300.0)
    out = torch.empty((240, 320, 3), device="cuda")
    counts = torch.zeros(3, dtype=torch.int64, device="cuda")
    # a capacity that does not fit in the scratch
    with pytest.raises(M.MsgsError) as e:
        M.render_noalloc(ctx, dsc, cam, out, counts, capacity=(1 << 32) - 1)
    assert e.value.code == M.E_CAPACITY
    # a capacity smaller than the frame needs: the counts say so
    ref = M.render(ctx, dsc, cam)
    M.render_noalloc(ctx, dsc, cam, out, counts, capacity=10)
    torch.cuda.synchronize()
    c = counts.cpu().numpy()
    assert c[2] == 10 and c[1] > 10
    # an explicit capacity that fits gives the full image
    M.render_noalloc(ctx, dsc, cam, out, counts, capacity=int(c[1]))
    torch.cuda.synchronize()
    np.testing.assert_array_equal(out.cpu().numpy(), ref.cpu().numpy())
    # a frame whose per-pixel buffers alone exceed the scratch
    big = G.lookat_camera([0.1, 0.2, -3.0], 8192, 8192, 8000.0)
    with pytest.raises(M.MsgsError) as e:
        M.render_noalloc(ctx, dsc, big, torch.empty((1, 1, 3), device="cuda"))
    assert e.value.code == M.E_CAPACITY
    dsc.close()
    ctx.close()
