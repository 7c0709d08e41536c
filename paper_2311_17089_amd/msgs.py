"""Python binding of libmsgs (ctypes; argument marshalling only).

Every step of the rasteriser runs in the HIP library.  PyTorch provides device
memory (tensors' data pointers) and the stream (the current torch stream is
passed to every call).  If the library is missing this module raises: there is
no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmsgs.so")

OK, E_INVALID, E_NOMEM, E_DEVICE, E_CAPACITY, E_BUSY = 0, -1, -2, -3, -4, -5


class MsgsError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"msgs error {code}: {msg}")
        self.code = code


class SceneDesc(C.Structure):
    _fields_ = [("n", C.c_int64), ("sh_degree", C.c_int), ("n_levels", C.c_int),
                ("means", C.c_void_p), ("scales", C.c_void_p), ("quats", C.c_void_p),
                ("opacity", C.c_void_p), ("sh", C.c_void_p), ("level", C.c_void_p),
                ("s_max", C.c_void_p), ("s_min", C.c_void_p), ("ptrs_on_device", C.c_int)]


class CameraC(C.Structure):
    _fields_ = [("R", C.c_float * 9), ("t", C.c_float * 3), ("fx", C.c_float), ("fy", C.c_float),
                ("cx", C.c_float), ("cy", C.c_float), ("width", C.c_int), ("height", C.c_int)]


class RenderOpts(C.Structure):
    _fields_ = [("downscale", C.c_int), ("selective", C.c_int), ("update_range", C.c_int),
                ("lowpass", C.c_float), ("near_z", C.c_float), ("bg", C.c_float * 3),
                ("profile", C.c_int), ("no_prefilter", C.c_int),
                ("instance_capacity", C.c_longlong)]


class Stats(C.Structure):
    _fields_ = [("n_gaussians", C.c_int64), ("n_selected", C.c_int64), ("n_visible", C.c_int64),
                ("n_instances", C.c_int64), ("n_blends", C.c_int64), ("n_visits", C.c_int64),
                ("n_evals", C.c_int64),
                ("width", C.c_int), ("height", C.c_int), ("tiles_x", C.c_int), ("tiles_y", C.c_int),
                ("stage_us", C.c_float * 12), ("n_prefiltered", C.c_int64)]


class Grads(C.Structure):
    _fields_ = [("means", C.c_void_p), ("scales", C.c_void_p), ("quats", C.c_void_p),
                ("opacity", C.c_void_p), ("sh", C.c_void_p), ("accumulate", C.c_int)]


class Gaussians(C.Structure):
    _fields_ = [("means", C.c_void_p), ("scales", C.c_void_p), ("quats", C.c_void_p),
                ("opacity", C.c_void_p), ("sh", C.c_void_p), ("cap", C.c_int64)]


class Completion(C.Structure):
    _fields_ = [("req_id", C.c_uint64), ("status", C.c_int), ("t_submit_us", C.c_double),
                ("t_admit_us", C.c_double), ("t_start_us", C.c_double), ("t_done_us", C.c_double),
                ("n_blends", C.c_int64)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


_lib = None

EXPORTS = {
    "msgs_version": ([], C.c_int),
    "msgs_last_error": ([], C.c_char_p),
    "msgs_default_opts": ([C.c_void_p], None),
    "msgs_context_create": ([C.c_int, C.c_size_t, C.c_void_p], C.c_int),
    "msgs_context_destroy": ([C.c_void_p], C.c_int),
    "msgs_context_bytes_in_use": ([C.c_void_p, C.c_void_p], C.c_int),
    "msgs_scene_create": ([C.c_void_p, C.c_void_p, C.c_int, C.c_void_p], C.c_int),
    "msgs_scene_destroy": ([C.c_void_p], C.c_int),
    "msgs_scene_get_ranges": ([C.c_void_p, C.c_void_p, C.c_void_p], C.c_int),
    "msgs_render": ([C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                     C.c_void_p], C.c_int),
    "msgs_render_backward": ([C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p], C.c_int),
    "msgs_render_views": ([C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                           C.c_int, C.c_void_p], C.c_int),
    "msgs_render_noalloc": ([C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                             C.c_void_p], C.c_int),
    "msgs_debug_sort_pairs": ([C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_int,
                               C.c_int, C.c_void_p], C.c_int),
    "msgs_render_backward_views": ([C.c_void_p, C.c_void_p, C.c_void_p, C.c_int, C.c_void_p,
                                    C.c_void_p], C.c_int),
    "msgs_frame_release": ([C.c_void_p], C.c_int),
    "msgs_frame_stats": ([C.c_void_p, C.c_void_p], C.c_int),
    "msgs_frame_get_selection": ([C.c_void_p, C.c_void_p], C.c_int),
    "msgs_frame_get_keys": ([C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p], C.c_int),
    "msgs_frame_get_state": ([C.c_void_p, C.c_void_p, C.c_void_p], C.c_int),
    "msgs_frame_get_ranges": ([C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p], C.c_int),
    "msgs_debug_exp": ([C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p], C.c_int),
    "msgs_debug_log": ([C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p], C.c_int),
    "msgs_server_create": ([C.c_void_p, C.c_void_p, C.c_int, C.c_void_p], C.c_int),
    "msgs_server_submit": ([C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_uint64], C.c_int),
    "msgs_server_poll": ([C.c_void_p, C.c_void_p, C.c_int, C.c_void_p, C.c_int], C.c_int),
    "msgs_server_pending": ([C.c_void_p, C.c_void_p, C.c_void_p], C.c_int),
    "msgs_server_destroy": ([C.c_void_p], C.c_int),
    "msgs_aggregate_level": ([C.c_void_p, C.c_void_p, C.c_void_p, C.c_int, C.c_int, C.c_float,
                              C.c_float, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p], C.c_int),
    "msgs_build_levels": ([C.c_void_p, C.c_void_p, C.c_void_p, C.c_int, C.c_int, C.c_float,
                           C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p], C.c_int),
}


def lib():
    """Load libmsgs.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"libmsgs.so not found at {LIB_PATH}; run "
                              f"python -m paper_2311_17089_amd.build (no fallback exists)")
        L = C.CDLL(LIB_PATH)
        for name, (args, res) in EXPORTS.items():
            f = getattr(L, name, None)
            if f is None:
                continue
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def check(rc: int) -> None:
    if rc != OK:
        raise MsgsError(rc, lib().msgs_last_error().decode(errors="replace"))


def _stream(stream=None) -> int:
    if stream is None:
        stream = torch.cuda.current_stream()
    return int(stream.cuda_stream)


def camera_c(cam) -> CameraC:
    c = CameraC()
    for i in range(9):
        c.R[i] = float(np.float32(cam.R[i]))
    for i in range(3):
        c.t[i] = float(np.float32(cam.t[i]))
    c.fx, c.fy, c.cx, c.cy = float(cam.fx), float(cam.fy), float(cam.cx), float(cam.cy)
    c.width, c.height = int(cam.width), int(cam.height)
    return c


def opts_c(downscale=1, selective=True, update_range=False, lowpass=0.3, near=0.2,
           bg: Sequence[float] = (0.0, 0.0, 0.0), profile=False, prefilter=True,
           capacity=0) -> RenderOpts:
    o = RenderOpts()
    o.instance_capacity = int(capacity)
    o.profile = 1 if profile else 0
    o.no_prefilter = 0 if prefilter else 1
    o.downscale = int(downscale)
    o.selective = 1 if selective else 0
    o.update_range = 1 if update_range else 0
    o.lowpass = float(lowpass)
    o.near_z = float(near)
    for i in range(3):
        o.bg[i] = float(bg[i])
    return o


class Context:
    def __init__(self, device: int = 0, pool_bytes: int = 0):
        self.device = device
        h = C.c_void_p()
        check(lib().msgs_context_create(device, pool_bytes, C.byref(h)))
        self.h = h

    def bytes_in_use(self) -> int:
        v = C.c_size_t()
        check(lib().msgs_context_bytes_in_use(self.h, C.byref(v)))
        return int(v.value)

    def close(self):
        if self.h:
            check(lib().msgs_context_destroy(self.h))
            self.h = None


class DeviceScene:
    """A scene resident in HBM.  From a numpy `scenegen.Scene` the arrays are
    uploaded as torch tensors and borrowed by the library (copy=0), so that the
    torch tensors double as the parameters of the autograd path."""

    FIELDS = ("means", "scales", "quats", "opacity", "sh", "level", "s_max", "s_min")

    def __init__(self, ctx: Context, scene, device: Optional[torch.device] = None):
        self.ctx = ctx
        dev = device or torch.device("cuda", ctx.device)
        self.n = int(scene.n)
        self.sh_degree = int(scene.sh_degree)
        self.n_levels = int(scene.n_levels)
        self.t = {}
        for k in self.FIELDS:
            a = getattr(scene, k)
            if isinstance(a, torch.Tensor):
                t = a.to(dev).contiguous()
            else:
                t = torch.from_numpy(np.ascontiguousarray(a)).to(dev)
            self.t[k] = t
        assert self.t["level"].dtype == torch.uint8
        for k in self.FIELDS:
            if k != "level":
                assert self.t[k].dtype == torch.float32, k
        d = SceneDesc(self.n, self.sh_degree, self.n_levels,
                      *[self.t[k].data_ptr() for k in self.FIELDS], 1)
        h = C.c_void_p()
        check(lib().msgs_scene_create(ctx.h, C.byref(d), 0, C.byref(h)))
        self.h = h

    def ranges(self):
        smax = np.empty(self.n, np.float32)
        smin = np.empty(self.n, np.float32)
        check(lib().msgs_scene_get_ranges(self.h, smax.ctypes.data, smin.ctypes.data))
        return smax, smin

    def close(self):
        if self.h:
            check(lib().msgs_scene_destroy(self.h))
            self.h = None


class Frame:
    """Saved state of one render (for the backward pass and the getters)."""

    def __init__(self, h, scene: DeviceScene, W: int, H: int):
        self.h, self.scene, self.W, self.H = h, scene, W, H

    def stats(self) -> dict:
        s = Stats()
        check(lib().msgs_frame_stats(self.h, C.byref(s)))
        d = {f: getattr(s, f) for f, _ in Stats._fields_}
        d["stage_us"] = list(s.stage_us)
        return d

    def selection(self) -> np.ndarray:
        m = np.empty(self.scene.n, np.uint8)
        check(lib().msgs_frame_get_selection(self.h, m.ctypes.data))
        return m

    def keys(self):
        n = C.c_size_t()
        check(lib().msgs_frame_get_keys(self.h, None, None, 0, C.byref(n)))
        k = np.empty(max(n.value, 1), np.uint64)
        v = np.empty(max(n.value, 1), np.uint32)
        check(lib().msgs_frame_get_keys(self.h, k.ctypes.data, v.ctypes.data, n.value, C.byref(n)))
        return k[:n.value], v[:n.value]

    def state(self):
        T = np.empty((self.H, self.W), np.float32)
        nc = np.empty((self.H, self.W), np.uint32)
        check(lib().msgs_frame_get_state(self.h, T.ctypes.data, nc.ctypes.data))
        return T, nc

    def ranges(self) -> np.ndarray:
        n = C.c_size_t()
        check(lib().msgs_frame_get_ranges(self.h, None, 0, C.byref(n)))
        r = np.empty((n.value, 2), np.uint32)
        check(lib().msgs_frame_get_ranges(self.h, r.ctypes.data, n.value, C.byref(n)))
        return r

    def release(self):
        if self.h:
            check(lib().msgs_frame_release(self.h))
            self.h = None

    def __del__(self):
        try:
            self.release()
        except Exception:
            pass


def render(ctx: Context, scene: DeviceScene, cam, downscale=1, selective=True,
           update_range=False, lowpass=0.3, near=0.2, bg=(0.0, 0.0, 0.0), keep_frame=False,
           out: Optional[torch.Tensor] = None, stream=None, profile=False, prefilter=True,
           capacity=0):
    """Render one view; returns the image tensor [H_d, W_d, 3] (and the Frame
    when keep_frame)."""
    W, H = (cam.width // downscale, cam.height // downscale) if downscale >= 1 else (0, 0)
    if out is None:
        out = torch.empty((H, W, 3), dtype=torch.float32, device=torch.device("cuda", ctx.device))
    assert out.is_contiguous() and out.dtype == torch.float32
    if W > 0 and H > 0:
        assert tuple(out.shape) == (H, W, 3), (tuple(out.shape), (H, W, 3))
    c = camera_c(cam)
    o = opts_c(downscale, selective, update_range, lowpass, near, bg, profile, prefilter, capacity)
    fh = C.c_void_p()
    check(lib().msgs_render(ctx.h, scene.h, C.byref(c), C.byref(o), C.c_void_p(out.data_ptr()),
                            C.byref(fh) if keep_frame else None, C.c_void_p(_stream(stream))))
    if keep_frame:
        return out, Frame(fh, scene, W, H)
    return out


def render_views(ctx: Context, scene: DeviceScene, views, keep_frames=False, outs=None,
                 stream=None):
    """Render several views of one scene in one call (see msgs_render_views).
    `views` is a list of (camera, options dict) with the keyword options of
    `render` (downscale, selective, update_range, lowpass, near, bg, prefilter,
    capacity).  Returns the images (and the Frames when keep_frames)."""
    nv = len(views)
    cams = (CameraC * nv)(*[camera_c(c) for c, _ in views])
    ops = []
    imgs = []
    for i, (cam, kw) in enumerate(views):
        d = int(kw.get("downscale", 1))
        ops.append(opts_c(d, kw.get("selective", True), kw.get("update_range", False),
                          kw.get("lowpass", 0.3), kw.get("near", 0.2), kw.get("bg", (0.0, 0.0, 0.0)),
                          False, kw.get("prefilter", True), kw.get("capacity", 0)))
        W, H = cam.width // d, cam.height // d
        out = outs[i] if outs is not None else torch.empty(
            (H, W, 3), dtype=torch.float32, device=torch.device("cuda", ctx.device))
        assert out.is_contiguous() and out.dtype == torch.float32
        imgs.append(out)
    oa = (RenderOpts * nv)(*ops)
    ra = (C.c_void_p * nv)(*[o.data_ptr() for o in imgs])
    fa = (C.c_void_p * nv)() if keep_frames else None
    check(lib().msgs_render_views(ctx.h, scene.h, cams, oa, ra, fa, nv,
                                  C.c_void_p(_stream(stream))))
    if keep_frames:
        frames = [Frame(C.c_void_p(fa[i]), scene, imgs[i].shape[1], imgs[i].shape[0])
                  for i in range(nv)]
        return imgs, frames
    return imgs


def render_noalloc(ctx: Context, scene: DeviceScene, cam, out: torch.Tensor,
                   counts: Optional[torch.Tensor] = None, downscale=1, selective=True,
                   lowpass=0.3, near=0.2, bg=(0.0, 0.0, 0.0), capacity=0, stream=None):
    """Render into `out` [H_d, W_d, 3] without any device allocation (see
    msgs_render_noalloc); `counts` (int64 device tensor of 3) receives the
    drawable Gaussians, the tile instances needed and those that fit."""
    assert out.is_contiguous() and out.dtype == torch.float32 and out.is_cuda
    if counts is not None:
        assert counts.dtype == torch.int64 and counts.numel() >= 3 and counts.is_cuda
    c = camera_c(cam)
    o = opts_c(downscale, selective, False, lowpass, near, bg, False, True, capacity)
    check(lib().msgs_render_noalloc(ctx.h, scene.h, C.byref(c), C.byref(o),
                                    C.c_void_p(out.data_ptr()),
                                    C.c_void_p(counts.data_ptr()) if counts is not None else None,
                                    C.c_void_p(_stream(stream))))
    return out


def _grad_planes(sc, grads, accumulate):
    names = ("means", "scales", "quats", "opacity", "sh")
    if grads is None:
        if accumulate:
            raise ValueError("accumulate needs caller-owned grads")
        g = {k: torch.empty_like(sc.t[k]) for k in names}
    else:
        g = grads
        for k in names:
            t = g[k]
            assert t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()
            assert t.shape == sc.t[k].shape, k
    return g, Grads(*[g[k].data_ptr() for k in names], 1 if accumulate else 0)


def render_backward(ctx: Context, frame: Frame, dL_drgb: torch.Tensor, stream=None,
                    grads: Optional[dict] = None, accumulate: bool = False) -> dict:
    """Adjoint of `render` for the frame's decisions; returns gradient tensors
    w.r.t. means, scales (linear), quats (raw), opacity and sh.  With `grads`
    (tensors shaped like the scene's) they receive the result; with
    accumulate=True it is added to them."""
    assert dL_drgb.is_contiguous() and dL_drgb.dtype == torch.float32
    g, gs = _grad_planes(frame.scene, grads, accumulate)
    check(lib().msgs_render_backward(ctx.h, frame.h, C.c_void_p(dL_drgb.data_ptr()), C.byref(gs),
                                     C.c_void_p(_stream(stream))))
    return g


def render_backward_views(ctx: Context, frames, dL_drgbs, stream=None,
                          grads: Optional[dict] = None, accumulate: bool = False) -> dict:
    """Backward of several renders of one scene at once: the sum over views of
    `render_backward`, bit-identical to calling it per view with the first
    call writing (or adding, with accumulate=True) and the rest adding."""
    frames, dL_drgbs = list(frames), list(dL_drgbs)
    if len(frames) != len(dL_drgbs):
        raise ValueError("one dL_drgb per frame")
    for d in dL_drgbs:
        assert d.is_contiguous() and d.dtype == torch.float32
    if not frames:
        raise ValueError("no frames")
    g, gs = _grad_planes(frames[0].scene, grads, accumulate)
    fa = (C.c_void_p * len(frames))(*[f.h for f in frames])
    da = (C.c_void_p * len(frames))(*[d.data_ptr() for d in dL_drgbs])
    check(lib().msgs_render_backward_views(ctx.h, fa, da, len(frames), C.byref(gs),
                                           C.c_void_p(_stream(stream))))
    return g


def debug_sort_pairs(ctx: Context, keys: torch.Tensor, vals: torch.Tensor, begin_bit=0, end_bit=32,
                     d_n: Optional[torch.Tensor] = None, stream=None):
    """Sort (keys, vals) (int32 device tensors holding u32 bit patterns) in place
    by key bits [begin_bit, end_bit) with the library's stable radix sort."""
    assert keys.is_cuda and vals.is_cuda and keys.numel() == vals.numel()
    assert keys.dtype == torch.int32 and vals.dtype == torch.int32
    assert keys.is_contiguous() and vals.is_contiguous()
    dn = C.c_void_p(d_n.data_ptr()) if d_n is not None else None
    check(lib().msgs_debug_sort_pairs(ctx.h, C.c_void_p(keys.data_ptr()),
                                      C.c_void_p(vals.data_ptr()), dn, keys.numel(), begin_bit,
                                      end_bit, C.c_void_p(_stream(stream))))


def debug_exp(x: torch.Tensor, stream=None) -> torch.Tensor:
    y = torch.empty_like(x)
    check(lib().msgs_debug_exp(C.c_void_p(x.data_ptr()), C.c_void_p(y.data_ptr()), x.numel(),
                               C.c_void_p(_stream(stream))))
    return y


def debug_log(x: torch.Tensor, stream=None) -> torch.Tensor:
    y = torch.empty_like(x)
    check(lib().msgs_debug_log(C.c_void_p(x.data_ptr()), C.c_void_p(y.data_ptr()), x.numel(),
                               C.c_void_p(_stream(stream))))
    return y


def calibrate(ctx: Context, scene: DeviceScene, cams, near=0.2):
    """Establish S^max/S^min on the device with the library's range update:
    starting from (0, +inf), render level l at downscale 4^l for every camera."""
    scene.t["s_max"].zero_()
    scene.t["s_min"].fill_(float("inf"))
    for l in range(scene.n_levels):
        for cam in cams:
            render(ctx, scene, cam, downscale=4 ** l, update_range=True, near=near)
    torch.cuda.synchronize()


# ---------------------------------------------------------------- autograd
class _RenderFn(torch.autograd.Function):
    """Differentiable render: forward and backward both run in libmsgs; the
    scene is borrowed from the input tensors for the duration of the call."""

    @staticmethod
    def forward(fctx, means, scales, quats, opacity, sh, state):
        ctx, level, s_max, s_min, n_levels, sh_degree, cam, kw = state
        t = {"means": means.contiguous(), "scales": scales.contiguous(),
             "quats": quats.contiguous(), "opacity": opacity.contiguous(),
             "sh": sh.contiguous(), "level": level, "s_max": s_max, "s_min": s_min}
        scene = _BorrowedScene(ctx, t, n_levels, sh_degree)
        rgb, frame = render(ctx, scene, cam, keep_frame=True, **kw)
        fctx.msgs = (ctx, scene, frame)
        fctx.mark_non_differentiable()
        return rgb

    @staticmethod
    def backward(fctx, grad_rgb):
        ctx, scene, frame = fctx.msgs
        g = render_backward(ctx, frame, grad_rgb.contiguous())
        frame.release()
        scene.close()
        fctx.msgs = None
        return g["means"], g["scales"], g["quats"], g["opacity"], g["sh"], None


class _BorrowedScene(DeviceScene):
    def __init__(self, ctx: Context, t: dict, n_levels: int, sh_degree: int):
        self.ctx = ctx
        self.t = t
        self.n = int(t["opacity"].numel())
        self.sh_degree = int(sh_degree)
        self.n_levels = int(n_levels)
        d = SceneDesc(self.n, self.sh_degree, self.n_levels,
                      *[t[k].data_ptr() for k in self.FIELDS], 1)
        h = C.c_void_p()
        check(lib().msgs_scene_create(ctx.h, C.byref(d), 0, C.byref(h)))
        self.h = h


def render_differentiable(ctx: Context, means, scales, quats, opacity, sh, level, s_max, s_min,
                          n_levels: int, sh_degree: int, cam, **kw) -> torch.Tensor:
    """Image [H_d, W_d, 3] differentiable w.r.t. means [3,n], scales [3,n]
    (linear), quats [4,n] (raw), opacity [n] (sigma) and sh [(D+1)^2*3, n]."""
    return _RenderFn.apply(means, scales, quats, opacity, sh,
                           (ctx, level, s_max, s_min, n_levels, sh_degree, cam, kw))


# ---------------------------------------------------------------- serving
class Server:
    """Continuous-batching render server over one resident scene (see
    msgs_server_* in msgs.h)."""

    def __init__(self, ctx: Context, scene: DeviceScene, max_inflight: int = 4):
        self.ctx, self.scene = ctx, scene
        h = C.c_void_p()
        check(lib().msgs_server_create(ctx.h, scene.h, int(max_inflight), C.byref(h)))
        self.h = h
        self._keep = {}

    def submit(self, cam, out: torch.Tensor, req_id: int, downscale=1, selective=True,
               lowpass=0.3, near=0.2, bg=(0.0, 0.0, 0.0)) -> None:
        assert out.is_contiguous() and out.dtype == torch.float32
        c = camera_c(cam)
        o = opts_c(downscale, selective, False, lowpass, near, bg)
        check(lib().msgs_server_submit(self.h, C.byref(c), C.byref(o), C.c_void_p(out.data_ptr()),
                                       C.c_uint64(req_id)))
        self._keep[req_id] = out

    def poll(self, max_n: int = 64, timeout_us: int = 0):
        arr = (Completion * max_n)()
        n = C.c_int()
        check(lib().msgs_server_poll(self.h, arr, max_n, C.byref(n), int(timeout_us)))
        res = [arr[i].as_dict() for i in range(n.value)]
        for r in res:
            self._keep.pop(r["req_id"], None)
        return res

    def pending(self):
        q, f = C.c_int(), C.c_int()
        check(lib().msgs_server_pending(self.h, C.byref(q), C.byref(f)))
        return q.value, f.value

    def close(self):
        if self.h:
            check(lib().msgs_server_destroy(self.h))
            self.h = None


class SceneOut(C.Structure):
    _fields_ = [("means", C.c_void_p), ("scales", C.c_void_p), ("quats", C.c_void_p),
                ("opacity", C.c_void_p), ("sh", C.c_void_p), ("level", C.c_void_p),
                ("s_max", C.c_void_p), ("s_min", C.c_void_p), ("cap", C.c_int64)]


def aggregate_level(ctx: Context, scene: DeviceScene, cams, level: int, s_thresh: float = 0.0,
                    extent: float = 0.0, grid: int = 0, stream=None) -> dict:
    """New Gaussians of `level` aggregated from the small Gaussians below it
    (see msgs_aggregate_level; 0 selects the library's default threshold,
    camera extent and voxel grid); returns device tensors in voxel order."""
    dev = scene.t["means"].device
    cap = max(1, scene.n)
    K3 = 3 * (scene.sh_degree + 1) ** 2
    out = {"means": torch.empty((3, cap), device=dev), "scales": torch.empty((3, cap), device=dev),
           "quats": torch.empty((4, cap), device=dev), "opacity": torch.empty(cap, device=dev),
           "sh": torch.empty((K3, cap), device=dev)}
    g = Gaussians(*[out[k].data_ptr() for k in ("means", "scales", "quats", "opacity", "sh")], cap)
    arr = (CameraC * len(cams))(*[camera_c(c) for c in cams])
    n_out = C.c_int64()
    check(lib().msgs_aggregate_level(ctx.h, scene.h, arr, len(cams), int(level), float(s_thresh),
                                     float(extent), int(grid), C.byref(g), C.byref(n_out),
                                     C.c_void_p(_stream(stream))))
    m = n_out.value
    return {k: v[..., :m].contiguous() for k, v in out.items()}


def build_levels(ctx: Context, scene0, cams, n_levels: int, s_thresh: float = 0.0):
    """Alg. 1 over every coarse level in the library (msgs_build_levels): from
    the level-0 Gaussians of `scene0` (numpy scenegen.Scene), aggregate for
    l = 1 .. n_levels - 1 and append each new level (uncalibrated range).
    Returns the numpy scene and the number of Gaussians added per level."""
    from .scenegen import Scene
    n0 = int(scene0.n)
    K3 = 3 * (scene0.sh_degree + 1) ** 2
    host = [np.ascontiguousarray(getattr(scene0, k)) for k in DeviceScene.FIELDS]
    base = SceneDesc(n0, int(scene0.sh_degree), int(n_levels), *[a.ctypes.data for a in host], 0)
    arr = (CameraC * len(cams))(*[camera_c(c) for c in cams])
    added = (C.c_int64 * max(1, n_levels - 1))()
    cap = 2 * n0 + 1024
    dev = torch.device("cuda", ctx.device)
    while True:
        out = {"means": torch.empty((3, cap), device=dev), "scales": torch.empty((3, cap), device=dev),
               "quats": torch.empty((4, cap), device=dev), "opacity": torch.empty(cap, device=dev),
               "sh": torch.empty((K3, cap), device=dev),
               "level": torch.empty(cap, dtype=torch.uint8, device=dev),
               "s_max": torch.empty(cap, device=dev), "s_min": torch.empty(cap, device=dev)}
        so = SceneOut(*[out[k].data_ptr() for k in DeviceScene.FIELDS], cap)
        n_out = C.c_int64()
        rc = lib().msgs_build_levels(ctx.h, C.byref(base), arr, len(cams), int(n_levels),
                                     float(s_thresh), C.byref(so), C.byref(n_out), added,
                                     C.c_void_p(_stream()))
        if rc == E_CAPACITY:
            cap = max(2 * cap, 2 * n_out.value)
            continue
        check(rc)
        break
    m = n_out.value
    h = {k: out[k][..., :m].cpu().numpy() for k in DeviceScene.FIELDS}
    scene = Scene(n=m, sh_degree=scene0.sh_degree, n_levels=n_levels,
                  **{k: np.ascontiguousarray(h[k]) for k in DeviceScene.FIELDS})
    return scene, [int(added[i]) for i in range(n_levels - 1)]
