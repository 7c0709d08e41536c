"""Pins of the oracle's hand-written fp32 exp / log and SH basis (CPU only)."""
import numpy as np
import pytest

import oracle as O


def _ulp_err(got, ref64):
    ref32 = ref64.astype(np.float32)
    return np.abs(got.astype(np.float64) - ref64) / np.spacing(np.abs(ref32))


def test_exp_spec_within_2ulp_exhaustive():
    # every fp32 value of [-5.6, -0] (about 1.09e9), in chunks
    lo = np.float32(-5.6).view(np.uint32)
    hi = np.uint32(0x80000000)  # -0.0
    worst = 0.0
    step = 1 << 24
    for start in range(int(hi), int(lo) + 1, step):
        bits = np.arange(start, min(int(lo) + 1, start + step), dtype=np.uint32)
        x = bits.view(np.float32)
        y = O.exp_spec(x)
        worst = max(worst, float(_ulp_err(y, np.exp(x.astype(np.float64))).max()))
    assert worst <= 2.0, worst


def test_exp_spec_exact_points():
    x = np.array([0.0, -0.0, -np.log(2) * 3], np.float32)
    y = O.exp_spec(x)
    assert y[0] == 1.0 and y[1] == 1.0
    assert abs(float(y[2]) - 0.125) <= 2 * np.spacing(np.float32(0.125))


def test_log_spec_within_2ulp_exhaustive():
    # all fp32 values in (1, 256)
    lo = np.float32(1.0).view(np.uint32) + 1
    hi = np.float32(256.0).view(np.uint32)
    worst = 0.0
    step = 1 << 24
    for start in range(int(lo), int(hi), step):
        bits = np.arange(start, min(int(hi), start + step), dtype=np.uint64)
        x = bits.astype(np.uint32).view(np.float32)
        y = O.log_spec(x)
        worst = max(worst, float(_ulp_err(y, np.log(x.astype(np.float64))).max()))
    assert worst <= 2.0, worst


def test_log_spec_powers_of_two():
    x = np.array([2.0, 4.0, 128.0], np.float32)
    y = O.log_spec(x)
    assert np.all(np.abs(y - np.log(x.astype(np.float64))) <= 2 * np.spacing(y))


def _sphere_quadrature(nz=8, nphi=16):
    # Gauss-Legendre in z times uniform phi: exact for polynomials of degree < 2 nz
    z, wz = np.polynomial.legendre.leggauss(nz)
    phi = (np.arange(nphi) + 0.5) * 2 * np.pi / nphi
    Z, P = np.meshgrid(z, phi, indexing="ij")
    W = np.repeat(wz[:, None], nphi, 1) * (2 * np.pi / nphi)
    s = np.sqrt(1 - Z ** 2)
    d = np.stack([s * np.cos(P), s * np.sin(P), Z]).reshape(3, -1)
    return d, W.reshape(-1)


def test_sh_basis_orthonormal():
    d, w = _sphere_quadrature()
    Y = O.sh_basis(3, d)
    gram = (Y * w) @ Y.T
    assert np.abs(gram - np.eye(16)).max() < 1e-12


def test_sh_basis_known_members_and_parity():
    rng = np.random.default_rng(3)
    d = rng.standard_normal((3, 50))
    d /= np.linalg.norm(d, axis=0)
    Y = O.sh_basis(3, d)
    # textbook members: Y_00 = 1/(2 sqrt(pi)); Y_1,{-1,0,1} = sqrt(3/(4 pi)) (y, z, x)
    assert np.allclose(Y[0], 0.5 / np.sqrt(np.pi))
    c1 = np.sqrt(3 / (4 * np.pi))
    assert np.allclose(Y[1], c1 * d[1]) and np.allclose(Y[2], c1 * d[2]) and np.allclose(Y[3], c1 * d[0])
    # Y_2,-2 = (1/2) sqrt(15/pi) x y
    assert np.allclose(Y[4], 0.5 * np.sqrt(15 / np.pi) * d[0] * d[1])
    # parity: Y_lm(-d) = (-1)^l Y_lm(d)
    Yn = O.sh_basis(3, -d)
    for l in range(4):
        for j in range(l * l, (l + 1) ** 2):
            assert np.allclose(Yn[j], (-1) ** l * Y[j])


def test_sh_basis_two_routes_agree():
    import torch
    from oracle import grad64
    rng = np.random.default_rng(5)
    d = rng.standard_normal((3, 400))
    d /= np.linalg.norm(d, axis=0)
    a = O.sh_basis(3, d)
    b = grad64.sh_basis_t(3, torch.tensor(d)).numpy()
    assert np.abs(a - b).max() < 1e-12
