"""Multi-view backward (needs an MI355X): msgs_render_backward_views against
msgs_render_backward called per view, the first call writing (or adding) and
the rest adding.  Both add the same fp32 per-view contributions in the same
order, so the gradient planes must agree bit for bit.

Cases: SH degrees 3 and 1; ten views (more than one chain pass of eight); a
view that draws nothing (near plane beyond the scene); one view; accumulation
onto non-zero planes; frames of two scenes are rejected.
"""
import numpy as np
import pytest
import torch

from paper_2311_17089_amd import msgs as M
from paper_2311_17089_amd import scenegen as G

pytestmark = pytest.mark.gpu

NAMES = ("means", "scales", "quats", "opacity", "sh")


def _say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def ctx():
    c = M.Context(0)
    yield c
    torch.cuda.synchronize()


def _scene(ctx, sh_degree, seed):
    sc = G.make_scene(G.level_counts(120_000, 3), seed, sh_degree, [-4.5 + 1.4 * l for l in range(3)])
    dsc = M.DeviceScene(ctx, sc)
    M.calibrate(ctx, dsc, G.calibration_cameras(seed + 7, 640, 360, 750.0, k=4))
    return dsc


def _frames(ctx, dsc, nviews, seed, empty_view=None):
    poses = G.sphere_poses(nviews, seed, 2.0, 8.0)
    frames, dls = [], []
    for i in range(nviews):
        cam = G.lookat_camera(poses[i], 640, 360, 750.0)
        d = (1, 2, 4)[i % 3]
        near = 1e6 if i == empty_view else 0.2
        _, fr = M.render(ctx, dsc, cam, downscale=d, update_range=(i % 2 == 0), near=near,
                         keep_frame=True)
        gen = torch.Generator().manual_seed(seed * 100 + i)
        dls.append((torch.randn((360 // d, 640 // d, 3), generator=gen) * 1e-4).cuda())
        frames.append(fr)
    return frames, dls


def _sequential(ctx, dsc, frames, dls, init=None):
    g = ({k: torch.empty_like(dsc.t[k]) for k in NAMES} if init is None
         else {k: v.clone() for k, v in init.items()})
    for i, (fr, dl) in enumerate(zip(frames, dls)):
        M.render_backward(ctx, fr, dl, grads=g, accumulate=(init is not None or i > 0))
    return g


def _batched(ctx, dsc, frames, dls, init=None):
    g = ({k: torch.empty_like(dsc.t[k]).fill_(float("nan")) for k in NAMES} if init is None
         else {k: v.clone() for k, v in init.items()})
    M.render_backward_views(ctx, frames, dls, grads=g, accumulate=init is not None)
    return g


def _equal(a, b, what):
    torch.cuda.synchronize()
    for k in NAMES:
        x, y = a[k].cpu().numpy(), b[k].cpu().numpy()
        assert np.array_equal(x, y), (what, k, int(np.sum(x != y)))


@pytest.mark.parametrize("sh_degree,nviews,empty_view", [(3, 10, 4), (1, 3, None), (3, 1, None)])
def test_views_equal_sequential(ctx, sh_degree, nviews, empty_view):
    _say(f"  views: SH degree {sh_degree}, {nviews} views, empty view {empty_view}")
    dsc = _scene(ctx, sh_degree, 31 + sh_degree)
    frames, dls = _frames(ctx, dsc, nviews, 40 + nviews, empty_view)
    if empty_view is not None:
        assert frames[empty_view].stats()["n_instances"] == 0
    seq = _sequential(ctx, dsc, frames, dls)
    bat = _batched(ctx, dsc, frames, dls)
    _equal(seq, bat, "write")
    nz = sum(int(torch.count_nonzero(bat[k])) for k in NAMES)
    assert nz > 0
    _say(f"  written planes equal ({nz} non-zero values)")
    gen = torch.Generator().manual_seed(77)
    init = {k: torch.randn(dsc.t[k].shape, generator=gen).cuda() * 1e-3 for k in NAMES}
    _equal(_sequential(ctx, dsc, frames, dls, init), _batched(ctx, dsc, frames, dls, init),
           "accumulate")
    _say("  accumulated planes equal")
    for fr in frames:
        fr.release()
    dsc.close()


def test_views_reject_mixed_scenes(ctx):
    a = _scene(ctx, 1, 51)
    b = _scene(ctx, 1, 52)
    fa, da = _frames(ctx, a, 1, 60)
    fb, db = _frames(ctx, b, 1, 61)
    with pytest.raises(M.MsgsError):
        M.render_backward_views(ctx, fa + fb, da + db, grads=None)
    with pytest.raises(ValueError):
        M.render_backward_views(ctx, [], [])
    # the C entry point itself: no views, and a frame of another context
    g = {k: torch.empty_like(a.t[k]) for k in NAMES}
    gs = M.Grads(*[g[k].data_ptr() for k in NAMES], 0)
    L = M.lib()
    fr_arr = (M.C.c_void_p * 1)(fa[0].h)
    dl_arr = (M.C.c_void_p * 1)(da[0].data_ptr())
    assert L.msgs_render_backward_views(ctx.h, fr_arr, dl_arr, 0, M.C.byref(gs), None) == \
        M.E_INVALID
    other = M.Context(0)
    assert L.msgs_render_backward_views(other.h, fr_arr, dl_arr, 1, M.C.byref(gs), None) == \
        M.E_INVALID
    assert L.msgs_render_backward_views(ctx.h, fr_arr, dl_arr, 1, M.C.byref(gs), None) == M.OK
    torch.cuda.synchronize()
    for fr in fa + fb:
        fr.release()
    a.close()
    b.close()
