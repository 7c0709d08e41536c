"""Fixed-capacity renders and a training step captured in a HIP graph (needs
an MI355X).  A fixed tile-instance capacity removes the render's only host
synchronisation, so forward and backward can be captured; results must equal
the exact mode bit for bit, overflow must be reported, and every replay of the
captured step must reproduce the eager step, also with one graph per frame
captured on several streams and replayed concurrently."""
import numpy as np
import pytest
import torch

from paper_2311_17089_amd import msgs as M
from paper_2311_17089_amd import scenegen as G

pytestmark = pytest.mark.gpu

NAMES = ("means", "scales", "quats", "opacity", "sh")


def _say(*a):
    print(*a, flush=True)


def _scene(ctx):
    sc = G.make_scene([40000, 10000, 2500, 620], 71, 2, [-4.2 + 1.4 * l for l in range(4)],
                      blob_fraction0=0.5)
    dsc = M.DeviceScene(ctx, sc)
    M.calibrate(ctx, dsc, G.calibration_cameras(1071, 320, 240, 300.0))
    return dsc


def _views():
    poses = G.sphere_poses(4, 71, 2.4, 3.4)
    return [(G.lookat_camera(poses[i], 320, 240, 300.0), 2 ** i) for i in range(4)]


def test_fixed_capacity_matches_exact_and_reports_overflow():
    ctx = M.Context(0)
    dsc = _scene(ctx)
    cam, d = _views()[0]
    dl = torch.randn((240 // d, 320 // d, 3), generator=torch.Generator().manual_seed(3)).cuda()
    rgb0, f0 = M.render(ctx, dsc, cam, downscale=d, keep_frame=True)
    st0 = f0.stats()
    g0 = M.render_backward(ctx, f0, dl)
    I = st0["n_instances"]
    for cap in (I, 2 * I + 7):
        rgb1, f1 = M.render(ctx, dsc, cam, downscale=d, keep_frame=True, capacity=cap)
        st1 = f1.stats()
        g1 = M.render_backward(ctx, f1, dl)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(rgb0.cpu().numpy(), rgb1.cpu().numpy())
        for k in ("n_selected", "n_visible", "n_instances", "n_blends", "n_visits"):
            assert st0[k] == st1[k], k
        for a, b in zip(f0.keys(), f1.keys()):
            np.testing.assert_array_equal(a, b)
        for a, b in zip(f0.state(), f1.state()):
            np.testing.assert_array_equal(a, b)
        for k in NAMES:
            np.testing.assert_array_equal(g0[k].cpu().numpy(), g1[k].cpu().numpy())
        f1.release()
    # too small a capacity: the frame and its backward complete without fault
    # (every per-Gaussian slot range is clipped to the capacity) and the frame
    # says so
    _, f2 = M.render(ctx, dsc, cam, downscale=d, keep_frame=True, capacity=I // 2)
    M.render_backward(ctx, f2, dl)
    M.render_backward_views(ctx, [f2], [dl])
    torch.cuda.synchronize()
    with pytest.raises(M.MsgsError) as e:
        f2.stats()
    assert e.value.code == M.E_CAPACITY
    f2.release()
    f0.release()
    dsc.close()


@pytest.mark.parametrize("mode", ["per_view", "views_backward", "multi_view"])
def test_captured_training_step_replays_exactly(mode):
    # per_view: one render and one backward call per view; views_backward: one
    # render call per view, one multi-view backward; multi_view: one
    # multi-view render call (its views run on the library's fork streams
    # inside the capture) and one multi-view backward
    _say(f"  captured step, {mode}")
    views_backward = mode != "per_view"
    ctx = M.Context(0)
    dsc = _scene(ctx)
    views = _views()
    dls = [torch.randn((240 // d, 320 // d, 3), generator=torch.Generator().manual_seed(10 + i))
           .cuda() * 1e-3 for i, (_, d) in enumerate(views)]
    caps = []
    for cam, d in views:
        _, fr = M.render(ctx, dsc, cam, downscale=d, keep_frame=True)
        caps.append(int(fr.stats()["n_instances"] * 1.25) + 64)
        fr.release()
    grads = {k: torch.zeros_like(dsc.t[k]) for k in NAMES}
    zeros = {k: torch.zeros_like(dsc.t[k]) for k in NAMES}
    outs = [torch.empty((240 // d, 320 // d, 3), device="cuda") for _, d in views]
    frames = []

    def step():
        if not views_backward:
            for k in NAMES:
                grads[k].copy_(zeros[k])
        fs = []
        if mode == "multi_view":
            vl = [(cam, {"downscale": d, "capacity": cap}) for (cam, d), cap in zip(views, caps)]
            _, fs = M.render_views(ctx, dsc, vl, keep_frames=True, outs=outs)
        for (cam, d), dl, cap, o in zip(views, dls, caps, outs):
            if mode == "multi_view":
                break
            _, fr = M.render(ctx, dsc, cam, downscale=d, keep_frame=True, capacity=cap, out=o)
            if not views_backward:
                M.render_backward(ctx, fr, dl, grads=grads, accumulate=True)
            fs.append(fr)
        if views_backward:
            M.render_backward_views(ctx, fs, dls, grads=grads)
        return fs

    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        for _ in range(2):  # eager runs on the capture stream warm the allocator up
            for fr in step():
                fr.release()
        ref_frames = step()
    torch.cuda.synchronize()
    for fr in ref_frames:
        fr.stats()  # no overflow
    ref_g = {k: v.cpu().numpy() for k, v in grads.items()}
    ref_img = [o.cpu().numpy() for o in outs]
    for fr in ref_frames:
        fr.release()
    torch.cuda.synchronize()

    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=side):
        frames = step()
    torch.cuda.synchronize()
    for rep in range(3):
        for k in NAMES:
            grads[k].fill_(7.0)
        for o in outs:
            o.fill_(-1.0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for k in NAMES:
            np.testing.assert_array_equal(grads[k].cpu().numpy(), ref_g[k])
        for o, r in zip(outs, ref_img):
            np.testing.assert_array_equal(o.cpu().numpy(), r)
        # unrelated eager work between replays, on another context's memory
        other = M.Context(0)
        o2 = M.DeviceScene(other, G.make_scene([3000], 5 + rep, 0, [-3.0]))
        M.render(other, o2, views[0][0], downscale=2)
        torch.cuda.synchronize()
        o2.close()
    _say(f"  captured {len(views)} views, 3 replays identical to the eager step")
    del g
    torch.cuda.synchronize()
    for fr in frames:
        fr.release()
    dsc.close()


def test_frames_captured_on_several_streams():
    """One graph per frame, each captured on its own stream while the
    library's block cache also holds blocks freed on the other streams (the
    cache must then take only the capturing stream's blocks: an event query
    would invalidate the capture); the graphs replayed concurrently must
    reproduce the eager frames bit for bit."""
    _say("  frames captured on three streams")
    ctx = M.Context(0)
    dsc = _scene(ctx)
    views = _views()[:3]
    dls = [torch.randn((240 // d, 320 // d, 3), generator=torch.Generator().manual_seed(30 + i))
           .cuda() * 1e-3 for i, (_, d) in enumerate(views)]
    caps = []
    for cam, d in views:
        _, fr = M.render(ctx, dsc, cam, downscale=d, keep_frame=True)
        caps.append(int(fr.stats()["n_instances"] * 1.25) + 64)
        fr.release()
    outs = [torch.empty((240 // d, 320 // d, 3), device="cuda") for _, d in views]
    grads = [{k: torch.empty_like(dsc.t[k]) for k in NAMES} for _ in views]
    streams = [torch.cuda.Stream() for _ in views]
    for s in streams:
        s.wait_stream(torch.cuda.current_stream())

    def frame(i, keep=False):
        cam, d = views[i]
        _, fr = M.render(ctx, dsc, cam, downscale=d, keep_frame=True, capacity=caps[i],
                         out=outs[i], stream=streams[i])
        M.render_backward(ctx, fr, dls[i], stream=streams[i], grads=grads[i])
        if keep:
            return fr
        fr.release()
        return None

    # eager runs on every stream leave freed blocks of all three in the cache
    for _ in range(2):
        for i in range(len(views)):
            with torch.cuda.stream(streams[i]):
                frame(i)
    torch.cuda.synchronize()
    for i in range(len(views)):
        with torch.cuda.stream(streams[i]):
            frame(i)
    torch.cuda.synchronize()
    ref_img = [o.cpu().numpy() for o in outs]
    ref_g = [{k: v.cpu().numpy() for k, v in g.items()} for g in grads]

    graphs, frames = [], []
    for i in range(len(views)):
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=streams[i]):
            frames.append(frame(i, keep=True))
        graphs.append(g)
    torch.cuda.synchronize()
    for rep in range(2):
        for i in range(len(views)):
            outs[i].fill_(-1.0)
            for k in NAMES:
                grads[i][k].fill_(7.0)
        torch.cuda.synchronize()
        for i in range(len(views)):
            streams[i].wait_stream(torch.cuda.current_stream())
            with torch.cuda.stream(streams[i]):
                graphs[i].replay()
        torch.cuda.synchronize()
        for i in range(len(views)):
            np.testing.assert_array_equal(outs[i].cpu().numpy(), ref_img[i])
            for k in NAMES:
                np.testing.assert_array_equal(grads[i][k].cpu().numpy(), ref_g[i][k])
            frames[i].stats()  # no overflow
    _say("  2 concurrent replays identical to the eager frames")
    del graphs
    torch.cuda.synchronize()
    for fr in frames:
        fr.release()
    dsc.close()


def test_capture_with_a_cold_block_cache_and_eager_work_between_replays():
    """A frame captured with nothing cached for its stream (new blocks are
    made during the capture), replayed with eager renders and backward passes
    of another view on the same stream in between: replays and eager results
    must both match their references, and the eager frame kept across a replay
    must still give its own gradients (scratch freed inside the capture is not
    handed to eager work)."""
    _say("  capture with a cold block cache, eager work between replays")
    ctx = M.Context(0)
    dsc = _scene(ctx)
    (cam0, d0), (cam1, d1) = _views()[:2]
    dl0 = torch.randn((240 // d0, 320 // d0, 3), generator=torch.Generator().manual_seed(41)).cuda()
    dl1 = torch.randn((240 // d1, 320 // d1, 3), generator=torch.Generator().manual_seed(42)).cuda()
    ref = []
    for cam, d, dl in ((cam0, d0, dl0), (cam1, d1, dl1)):
        img, fr = M.render(ctx, dsc, cam, downscale=d, keep_frame=True)
        cap = int(fr.stats()["n_instances"] * 1.25) + 64
        g = M.render_backward(ctx, fr, dl)
        torch.cuda.synchronize()
        ref.append((cap, img.cpu().numpy(), {k: v.cpu().numpy() for k, v in g.items()}))
        fr.release()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    out0 = torch.empty((240 // d0, 320 // d0, 3), device="cuda")
    g0 = {k: torch.empty_like(dsc.t[k]) for k in NAMES}
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=s):
        _, f0 = M.render(ctx, dsc, cam0, downscale=d0, keep_frame=True, capacity=ref[0][0],
                         out=out0, stream=s)
        M.render_backward(ctx, f0, dl0, stream=s, grads=g0)
    torch.cuda.synchronize()
    for rep in range(2):
        with torch.cuda.stream(s):
            out0.fill_(-1.0)
            # an eager frame of the other view on the capture stream, kept
            # across the replay
            img1, f1 = M.render(ctx, dsc, cam1, downscale=d1, keep_frame=True, stream=s,
                                capacity=ref[1][0])
            graph.replay()
            g1 = M.render_backward(ctx, f1, dl1, stream=s)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(out0.cpu().numpy(), ref[0][1])
        np.testing.assert_array_equal(img1.cpu().numpy(), ref[1][1])
        for k in NAMES:
            np.testing.assert_array_equal(g0[k].cpu().numpy(), ref[0][2][k])
            np.testing.assert_array_equal(g1[k].cpu().numpy(), ref[1][2][k])
        f1.release()
    _say("  2 replays and the eager frames between them match their references")
    del graph
    torch.cuda.synchronize()
    f0.release()
    dsc.close()
