"""fp64 image and gradient with the discrete decisions frozen (TEST INFRASTRUCTURE).

Plain PyTorch on the CPU.  The decisions -- which Gaussians each pixel
composites, in which order, which alphas are clamped at 0.99 and which colour
channels are clamped at 0 -- are those of the oracle's fp32 path (the GPU takes
them in fp32 too).  Every continuous quantity is recomputed here in fp64:

  * EWA projection (Sec. 3.1): rotation from the normalised quaternion,
    Sigma = (R_q S)(R_q S)^T, V = (J W) Sigma (J W)^T, dilated by h I
    (the merged kernel G_{V^k+V^h}, Sec. 3.2), conic A = (V + h I)^-1;
  * colour: real orthonormal spherical harmonics (no Condon-Shortley phase),
    built here from derivatives of the Legendre polynomials in Cartesian form,
    offset 0.5;
  * front-to-back compositing: C = sum_j c_j alpha_j T_j with
    T_j = prod_{m<j} (1 - alpha_m), image = C + T_final * bg.

The gradient comes from torch autograd over that forward; it is pinned by
central finite differences of the same forward (tests/test_oracle_grad.py),
which do not use autograd.
"""
from __future__ import annotations

import math
from typing import Dict, Optional, Sequence

import numpy as np
import torch

from . import project as _project, trace as _trace, frame_size

PARAMS = ("means", "scales", "quats", "opacity", "sh")


def sh_basis_t(degree: int, d: torch.Tensor) -> torch.Tensor:
    """Real SH basis [(D+1)^2, m] at unit directions d [3, m]:
    Y_l^0 = K P_l(z); Y_l^{+-m} = sqrt2 K (d^m P_l/dz^m)(z) * Re/Im (x + i y)^m,
    K = sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!)."""
    x, y, z = d[0], d[1], d[2]
    # (x + i y)^m for m = 0..D
    re = [torch.ones_like(x)]
    im = [torch.zeros_like(x)]
    for m in range(1, degree + 1):
        r0, i0 = re[-1], im[-1]
        re.append(r0 * x - i0 * y)
        im.append(r0 * y + i0 * x)
    out = []
    for l in range(degree + 1):
        Pl = np.polynomial.legendre.Legendre.basis(l).convert(kind=np.polynomial.Polynomial)
        for m in range(-l, l + 1):
            am = abs(m)
            K = math.sqrt((2 * l + 1) / (4 * math.pi) * math.factorial(l - am) / math.factorial(l + am))
            coef = (Pl.deriv(am) if am > 0 else Pl).coef
            pz = torch.zeros_like(z)
            for i in reversed(range(len(coef))):
                pz = pz * z + float(coef[i])
            if m == 0:
                out.append(K * pz)
            elif m > 0:
                out.append(math.sqrt(2.0) * K * pz * re[am])
            else:
                out.append(math.sqrt(2.0) * K * pz * im[am])
    return torch.stack(out)


def _cam64(cam, downscale):
    d = float(np.float32(downscale))
    f32 = np.float32
    fx = float(f32(f32(cam.fx) / f32(d)))
    fy = float(f32(f32(cam.fy) / f32(d)))
    cx = float(f32(f32(cam.cx) / f32(d)))
    cy = float(f32(f32(cam.cy) / f32(d)))
    R = torch.tensor(np.asarray(cam.R, np.float32).astype(np.float64).reshape(3, 3))
    t = torch.tensor(np.asarray(cam.t, np.float32).astype(np.float64))
    return R, t, fx, fy, cx, cy


def project64(p: Dict[str, torch.Tensor], idx: torch.Tensor, cam, downscale: int,
              lowpass: float, sh_degree: int, cclamp: np.ndarray):
    """fp64 projection of the Gaussians `idx`: centre u [2,m], conic A [3,m],
    opacity [m], colour [3,m] (clamped channels held at 0)."""
    R, t, fx, fy, cx, cy = _cam64(cam, downscale)
    mu = p["means"][:, idx]
    sc = p["scales"][:, idx]
    q = p["quats"][:, idx]
    q = q / torch.sqrt((q * q).sum(0))
    w, x, y, z = q[0], q[1], q[2], q[3]
    Q = torch.stack([
        torch.stack([1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)]),
        torch.stack([2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)]),
        torch.stack([2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]),
    ])  # [3,3,m]
    M = Q * sc.unsqueeze(0)                     # M_ij = Q_ij s_j
    Sig = torch.einsum("ikm,jkm->ijm", M, M)     # M M^T
    pc = torch.einsum("ij,jm->im", R, mu) + t[:, None]
    px, py, pz = pc[0], pc[1], pc[2]
    zero = torch.zeros_like(pz)
    J = torch.stack([torch.stack([fx / pz, zero, -fx * px / (pz * pz)]),
                     torch.stack([zero, fy / pz, -fy * py / (pz * pz)])])  # [2,3,m]
    Tm = torch.einsum("ikm,kj->ijm", J, R)
    V = torch.einsum("ikm,klm,jlm->ijm", Tm, Sig, Tm)
    W11 = V[0, 0] + lowpass
    W22 = V[1, 1] + lowpass
    W12 = V[0, 1]
    det = W11 * W22 - W12 * W12
    A = torch.stack([W22 / det, -W12 / det, W11 / det])
    u = torch.stack([fx * px / pz + cx, fy * py / pz + cy])
    # colour towards the camera centre
    Cc = -(R.T @ t)
    dv = mu - Cc[:, None]
    dv = dv / torch.sqrt((dv * dv).sum(0))
    Y = sh_basis_t(sh_degree, dv)  # [K, m]
    K = (sh_degree + 1) ** 2
    sh = p["sh"][:, idx].reshape(K, 3, -1)
    col = torch.einsum("jm,jcm->cm", Y, sh) + 0.5
    keep = torch.tensor(1 - cclamp[:, idx.numpy()], dtype=torch.float64)
    col = col * keep
    return u, A, p["opacity"][idx], col


def frozen_render64(p: Dict[str, torch.Tensor], cam, downscale: int, pix_xy: np.ndarray,
                    off: np.ndarray, ks: np.ndarray, flags: np.ndarray, cclamp: np.ndarray,
                    lowpass: float = 0.3, bg=(0.0, 0.0, 0.0), sh_degree: int = 0):
    """fp64 colour [m,3] and T_final [m] of the pixels pix_xy [m,2] with the
    contributor lists (off, ks, flags) and colour clamps frozen."""
    m = pix_xy.shape[0]
    counts = np.diff(off)
    Lmax = int(counts.max()) if m else 0
    if ks.size == 0:
        rgb = torch.zeros(m, 3, dtype=torch.float64) + torch.tensor(bg, dtype=torch.float64)
        return rgb, torch.ones(m, dtype=torch.float64)
    uk, inv = np.unique(ks, return_inverse=True)
    u, A, sig, col = project64(p, torch.from_numpy(uk), cam, downscale, lowpass, sh_degree, cclamp)
    pix_of = np.repeat(np.arange(m), counts)
    slot = np.arange(ks.size) - np.repeat(off[:-1], counts)
    inv_t = torch.from_numpy(inv)
    pcx = torch.tensor(pix_xy[pix_of, 0].astype(np.float64) + 0.5)
    pcy = torch.tensor(pix_xy[pix_of, 1].astype(np.float64) + 0.5)
    dx = pcx - u[0, inv_t]
    dy = pcy - u[1, inv_t]
    power = -0.5 * (A[0, inv_t] * dx * dx + A[2, inv_t] * dy * dy) - A[1, inv_t] * dx * dy
    alpha = sig[inv_t] * torch.exp(power)
    clamped = torch.from_numpy(flags.astype(bool))
    alpha = torch.where(clamped, torch.full_like(alpha, 0.99), alpha)
    # dense [m, Lmax] layout for the transmittance products
    lin = torch.from_numpy(pix_of * Lmax + slot)
    one_minus = torch.ones(m * Lmax, dtype=torch.float64).index_put((lin,), 1.0 - alpha).view(m, Lmax)
    Tincl = torch.cumprod(one_minus, dim=1)
    Texcl = torch.cat([torch.ones(m, 1, dtype=torch.float64), Tincl[:, :-1]], dim=1)
    Tj = Texcl.reshape(-1)[lin]
    w = alpha * Tj
    cj = col[:, inv_t]  # [3, E]
    rgb = torch.zeros(3, m, dtype=torch.float64).index_add(1, torch.from_numpy(pix_of), cj * w)
    Tf = Tincl[:, -1]
    rgb = rgb.T + Tf[:, None] * torch.tensor(bg, dtype=torch.float64)
    return rgb, Tf


def scene_params64(scene, requires_grad=True) -> Dict[str, torch.Tensor]:
    return {k: torch.tensor(np.asarray(getattr(scene, k), np.float64), requires_grad=requires_grad)
            for k in PARAMS}


def all_pixels(W: int, H: int) -> np.ndarray:
    yy, xx = np.mgrid[0:H, 0:W]
    return np.stack([xx.reshape(-1), yy.reshape(-1)], 1).astype(np.int32)


class Frozen:
    """Decisions of the fp32 path for one render, and the fp64 forward over them."""

    def __init__(self, scene, cam, downscale=1, selective=True, lowpass=0.3, near=0.2,
                 pix_xy: Optional[np.ndarray] = None, bg=(0.0, 0.0, 0.0)):
        self.scene, self.cam, self.ds = scene, cam, downscale
        self.lowpass, self.bg = lowpass, bg
        W, H = frame_size(cam, downscale)
        self.W, self.H = W, H
        self.pix = all_pixels(W, H) if pix_xy is None else np.ascontiguousarray(pix_xy, np.int32)
        self.proj = _project(scene, cam, downscale, selective, lowpass, near)
        self.off, self.ks, self.flags = _trace(scene, cam, self.pix, downscale, selective, lowpass, near)

    def forward(self, p: Dict[str, torch.Tensor]):
        return frozen_render64(p, self.cam, self.ds, self.pix, self.off, self.ks, self.flags,
                               self.proj["cclamp"], self.lowpass, self.bg, self.scene.sh_degree)

    def grad(self, G: np.ndarray) -> Dict[str, np.ndarray]:
        """Gradient of sum(G * image) (G [m,3] per listed pixel) w.r.t. means,
        scales (linear), quats (raw), opacity, sh."""
        p = scene_params64(self.scene)
        rgb, _ = self.forward(p)
        (rgb * torch.tensor(np.asarray(G, np.float64))).sum().backward()
        return {k: p[k].grad.numpy().copy() for k in PARAMS}

    def loss_fd(self, G: np.ndarray, which: str, comp: int, k: int, h: float = 1e-3,
                richardson: bool = True) -> float:
        """Central difference of sum(G * image) in the parameter (which, comp, k),
        stepping in the optimisation parameterisation: means and quats directly,
        log of the scale, logit of the opacity, SH directly.  Returned as a
        derivative w.r.t. the linear parameter (chain rule of exp / sigmoid)."""
        base = scene_params64(self.scene, requires_grad=False)
        Gt = torch.tensor(np.asarray(G, np.float64))

        def L(delta):
            p = {kk: v.clone() for kk, v in base.items()}
            if which == "scales":
                v = p["scales"][comp, k]
                p["scales"][comp, k] = torch.exp(torch.log(v) + delta)
            elif which == "opacity":
                v = p["opacity"][k]
                lg = torch.log(v / (1 - v))
                p["opacity"][k] = 1.0 / (1.0 + torch.exp(-(lg + delta)))
            elif which == "means" or which == "quats" or which == "sh":
                p[which][comp, k] = p[which][comp, k] + delta
            else:
                raise ValueError(which)
            rgb, _ = self.forward(p)
            return float((rgb * Gt).sum())

        def D(hh):
            return (L(hh) - L(-hh)) / (2 * hh)

        d = (4 * D(h / 2) - D(h)) / 3 if richardson else D(h)
        if which == "scales":
            d = d / float(base["scales"][comp, k])
        elif which == "opacity":
            v = float(base["opacity"][k])
            d = d / (v * (1 - v))
        return d
