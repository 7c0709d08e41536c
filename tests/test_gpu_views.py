"""Several views of one scene in one call (msgs_render_views, needs an MI355X):
the shared projection pass gives results bit-identical to rendering the views
one after another (images, selection masks, sorted keys, ranges, per-pixel
state, statistics, range updates, gradients of the multi-view backward), and
sampled pixels match the CPU oracle."""
import dataclasses

import numpy as np
import pytest
import torch

import oracle as O
from paper_2311_17089_amd import msgs as M
from paper_2311_17089_amd import scenegen as G

pytestmark = pytest.mark.gpu

IMG_TOL = 1e-5


@pytest.fixture(scope="module")
def ctx():
    c = M.Context(0)
    yield c
    torch.cuda.synchronize()


def _say(*a):
    print(*a, flush=True)


def _scene(seed=91, counts=(30000, 7500, 1900, 470)):
    sc = G.make_scene(list(counts), seed, 3, [-4.2 + 1.4 * l for l in range(len(counts))],
                      blob_fraction0=0.5)
    return O.calibrate(sc, G.calibration_cameras(seed + 1000, 480, 320, 520.0))


def _views(seed, n, W=480, H=320):
    rng = np.random.default_rng(seed)
    poses = G.sphere_poses(n, seed, 2.2, 4.0)
    out = []
    for i in range(n):
        ds = int(rng.choice([1, 2, 4, 8, 16, 64]))
        kw = {"downscale": ds, "selective": bool(rng.integers(0, 4) > 0),
              "bg": tuple(float(x) for x in rng.uniform(0, 0.5, 3))}
        out.append((G.lookat_camera(poses[i], W, H, 1.1 * W), kw))
    return out


def _frame_data(fr, img):
    T, nc = fr.state()
    k, v = fr.keys()
    st = fr.stats()
    return {"img": img.cpu().numpy(), "sel": fr.selection(), "keys": k, "vals": v,
            "ranges": fr.ranges(), "T": T, "nc": nc,
            "stats": {q: st[q] for q in ("n_selected", "n_visible", "n_instances", "n_blends",
                                         "n_visits", "n_evals", "n_prefiltered")}}


def _same(a, b, tag):
    for key in ("img", "sel", "keys", "vals", "ranges", "T", "nc"):
        np.testing.assert_array_equal(a[key], b[key], err_msg=f"{tag} {key}")
    assert a["stats"] == b["stats"], (tag, a["stats"], b["stats"])


@pytest.mark.parametrize("nviews", [1, 3, 8, 11])
def test_views_match_sequential_renders(ctx, nviews):
    _say(f"  {nviews} views")
    sc = _scene()
    dsc = M.DeviceScene(ctx, sc)
    views = _views(100 + nviews, nviews)
    seq = []
    for cam, kw in views:
        img, fr = M.render(ctx, dsc, cam, keep_frame=True, **kw)
        seq.append(_frame_data(fr, img))
        fr.release()
    imgs, frames = M.render_views(ctx, dsc, views, keep_frames=True)
    for i, (img, fr) in enumerate(zip(imgs, frames)):
        _same(_frame_data(fr, img), seq[i], f"view {i}")
        fr.release()
    # sampled pixels of two views against brute force
    rng = np.random.default_rng(nviews)
    for i in range(min(2, nviews)):
        cam, kw = views[i]
        img = seq[i]["img"]
        H, W = img.shape[:2]
        idx = rng.choice(W * H, size=min(300, W * H), replace=False)
        pix = np.stack([idx % W, idx // W], 1).astype(np.int32)
        ref, _, _ = O.render_pixels(sc, cam, pix, downscale=kw["downscale"],
                                    selective=kw["selective"], bg=kw["bg"])
        assert np.abs(img[pix[:, 1], pix[:, 0]] - ref).max() <= IMG_TOL
    dsc.close()


def test_views_range_update_matches_sequential(ctx):
    # views at the levels' creation downscales with the range update on: the
    # ranges after one multi-view call equal those after the renders in order,
    # and so do the images (selection reads the ranges earlier views updated)
    sc = G.reset_ranges(_scene(92))
    cams = G.calibration_cameras(1092, 480, 320, 520.0)[:3]
    views = [(cam, {"downscale": 4 ** l, "update_range": True}) for cam in cams
             for l in range(sc.n_levels)]
    a = M.DeviceScene(ctx, sc)
    b = M.DeviceScene(ctx, sc)
    seq = [M.render(ctx, a, cam, **kw).cpu().numpy() for cam, kw in views]
    got = [x.cpu().numpy() for x in M.render_views(ctx, b, views)]
    for i, (x, y) in enumerate(zip(got, seq)):
        np.testing.assert_array_equal(x, y, err_msg=f"view {i}")
    for u, w in zip(a.ranges(), b.ranges()):
        np.testing.assert_array_equal(u, w)
    # and the oracle's range update agrees
    ref = sc.copy()
    for cam, kw in views:
        O.update_range(ref, cam, kw["downscale"])
    np.testing.assert_array_equal(b.ranges()[0], ref.s_max)
    np.testing.assert_array_equal(b.ranges()[1], ref.s_min)
    a.close()
    b.close()


def test_views_capacity_mode_and_multi_view_backward(ctx):
    # fixed-capacity views (no host synchronisation) and the multi-view
    # backward of their frames: identical to sequential exact-mode frames
    sc = _scene(93)
    dsc = M.DeviceScene(ctx, sc)
    views = _views(193, 5)
    dls, caps, seq_frames = [], [], []
    for i, (cam, kw) in enumerate(views):
        img, fr = M.render(ctx, dsc, cam, keep_frame=True, **kw)
        caps.append(fr.stats()["n_instances"] + 777)
        g = torch.Generator().manual_seed(300 + i)
        dls.append((torch.randn(img.shape, generator=g) * 1e-2).cuda())
        seq_frames.append(fr)
    ref = {k: v.cpu().numpy() for k, v in M.render_backward_views(ctx, seq_frames, dls).items()}
    seq_imgs = [M.render(ctx, dsc, cam, **kw).cpu().numpy() for cam, kw in views]
    for fr in seq_frames:
        fr.release()
    cviews = [(cam, dict(kw, capacity=c)) for (cam, kw), c in zip(views, caps)]
    imgs, frames = M.render_views(ctx, dsc, cviews, keep_frames=True)
    got = {k: v.cpu().numpy() for k, v in M.render_backward_views(ctx, frames, dls).items()}
    for i, img in enumerate(imgs):
        np.testing.assert_array_equal(img.cpu().numpy(), seq_imgs[i], err_msg=f"view {i}")
        assert frames[i].stats()["n_instances"] <= caps[i]
    for k in ref:
        np.testing.assert_array_equal(got[k], ref[k], err_msg=k)
    for fr in frames:
        fr.release()
    dsc.close()


def test_views_mixed_modes_and_backward_on_another_stream(ctx):
    # one call mixing exact and fixed-capacity views (the capacity views' second
    # phase waits for the exact views' count readback), rendered on one stream
    # and differentiated on another, frames released right after: the same
    # frames, images and gradients as sequential renders on the default stream
    sc = _scene(95)
    dsc = M.DeviceScene(ctx, sc)
    views = _views(195, 6)
    seq, caps, dls, seq_frames = [], [], [], []
    for i, (cam, kw) in enumerate(views):
        img, fr = M.render(ctx, dsc, cam, keep_frame=True, **kw)
        seq.append(_frame_data(fr, img))
        caps.append(fr.stats()["n_instances"] + 321 if i % 2 else 0)
        g = torch.Generator().manual_seed(500 + i)
        dls.append((torch.randn(img.shape, generator=g) * 1e-2).cuda())
        seq_frames.append(fr)
    ref = {k: v.cpu().numpy() for k, v in M.render_backward_views(ctx, seq_frames, dls).items()}
    for fr in seq_frames:
        fr.release()
    mviews = [(cam, dict(kw, capacity=c)) for (cam, kw), c in zip(views, caps)]
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    s1.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s1):
        imgs, frames = M.render_views(ctx, dsc, mviews, keep_frames=True)
    for i, (img, fr) in enumerate(zip(imgs, frames)):
        s1.synchronize()
        got = _frame_data(fr, img)
        if caps[i]:
            # a fixed-capacity frame counts the capacity as its instances
            for key in ("img", "sel", "T", "nc"):
                np.testing.assert_array_equal(got[key], seq[i][key], err_msg=f"view {i} {key}")
        else:
            _same(got, seq[i], f"view {i}")
    s2.wait_stream(s1)
    with torch.cuda.stream(s2):
        grads = M.render_backward_views(ctx, frames, dls)
    for fr in frames:
        fr.release()
    # unrelated work that may take the released blocks
    with torch.cuda.stream(s1):
        M.render(ctx, dsc, views[0][0], **views[0][1])
    torch.cuda.synchronize()
    for k in ref:
        np.testing.assert_array_equal(grads[k].cpu().numpy(), ref[k], err_msg=k)
    dsc.close()


def test_views_on_many_caller_streams():
    # a context keeps fork streams for up to 64 caller streams; multi-view
    # renders on further streams run their views on the caller's stream, with
    # the same results
    c = M.Context(0)
    sc = _scene(97, counts=(3000, 750, 190, 47))
    dsc = M.DeviceScene(c, sc)
    views = _views(197, 2, W=96, H=64)
    ref = [x.cpu().numpy() for x in M.render_views(c, dsc, views)]
    streams = [torch.cuda.Stream() for _ in range(70)]
    for i, st in enumerate(streams):
        st.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(st):
            got = M.render_views(c, dsc, views)
        st.synchronize()
        for v, (a, b) in enumerate(zip(got, ref)):
            np.testing.assert_array_equal(a.cpu().numpy(), b, err_msg=f"stream {i} view {v}")
    _say(f"  {len(streams)} caller streams")
    dsc.close()


def test_views_invalid_arguments(ctx):
    sc = G.make_scene([100], 1, 0, [-3.0])
    dsc = M.DeviceScene(ctx, sc)
    cam = G.lookat_camera([0, 0, -3], 40, 30, 40.0)
    with pytest.raises(M.MsgsError) as e:
        M.render_views(ctx, dsc, [(cam, {"downscale": 64})])
    assert e.value.code == M.E_INVALID
    with pytest.raises(M.MsgsError) as e:
        M.render_views(ctx, dsc, [(cam, {})] * 65)
    assert e.value.code == M.E_INVALID
    with pytest.raises(M.MsgsError) as e:
        M.render_views(ctx, dsc, [])
    assert e.value.code == M.E_INVALID
    dsc.close()
