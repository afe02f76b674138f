"""Pins of the oracle's FP64 SH evaluation (H): c(d) = H w(d) (Sec. II).

  * the 16 basis functions equal the real SH built from scipy's complex
    spherical harmonics (library routine) in the 3DGS renderer's convention
    Y_lm = sqrt2 Re Y_l^m (m > 0), Y_l0, sqrt2 Im Y_l^|m| (m < 0), k = l^2+l+m;
  * they are orthonormal under an exact product quadrature;
  * DC-only colour is H_0 / (2 sqrt(pi)) everywhere; Parseval holds;
  * decode_eval equals the decoded, dequantised texels times the basis.
"""
import numpy as np
import pytest
import scipy.special as sp

import oracle as O
from paper_2607_14513_amd import synth


def _quadrature():
    xg, wg = np.polynomial.legendre.leggauss(8)          # in cos(theta)
    phi = 2 * np.pi * np.arange(16) / 16
    z = np.repeat(xg, 16)
    w = np.repeat(wg, 16) * (2 * np.pi / 16)
    s = np.sqrt(1 - z * z)
    p = np.tile(phi, 8)
    return np.stack([s * np.cos(p), s * np.sin(p), z], 1), w


def test_matches_scipy_real_sh():
    rng = np.random.default_rng(0)
    d = rng.normal(size=(300, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    theta = np.arccos(np.clip(d[:, 2], -1, 1))
    phi = np.arctan2(d[:, 1], d[:, 0])
    for i in range(len(d)):
        Y = O.sh_basis(d[i])
        for l in range(4):
            for m in range(-l, l + 1):
                c = sp.sph_harm_y(l, abs(m), theta[i], phi[i])
                ref = c.real if m == 0 else np.sqrt(2) * (c.real if m > 0 else c.imag)
                assert abs(Y[l * l + l + m] - ref) < 1e-12


def test_orthonormal():
    pts, w = _quadrature()
    B = np.array([O.sh_basis(p) for p in pts])
    G = (B * w[:, None]).T @ B
    assert np.abs(G - np.eye(16)).max() < 1e-12


def test_dc_only_and_parseval():
    rng = np.random.default_rng(1)
    H = rng.normal(size=16)
    pts, w = _quadrature()
    c = np.array([O.sh_basis(p) @ H for p in pts])
    assert abs((w * c * c).sum() / (4 * np.pi) - (H * H).sum() / (4 * np.pi)) < 1e-12
    Hd = np.zeros(16)
    Hd[0] = 0.7
    for p in pts[::11]:
        assert abs(O.sh_basis(p) @ Hd - 0.7 / (2 * np.sqrt(np.pi))) < 1e-15


def test_decode_eval_is_dequantised_texels_times_basis():
    pos, sh = synth.make_scene(600, seed=5)
    perm, tex, vmin, vmax = O.reorder(pos, sh)
    nblk = tex.shape[1]
    fmt = np.array([7] + [1] * 15, np.uint8)
    payload, off, _ = O.encode(tex, fmt)
    dirs = synth.make_dirs(9, seed=5)
    slots = np.array([0, 1, 15, 16, 17, 300, 599], np.uint32)
    out, scale = O.decode_eval(payload, off, fmt, vmin, vmax, dirs, slots)
    dec = O.decode_stream(payload, off, fmt, nblk)
    z = [[0, 1, 4, 5], [2, 3, 6, 7], [8, 9, 12, 13], [10, 11, 14, 15]]
    where = {z[y][x]: 4 * y + x for y in range(4) for x in range(4)}
    for j, s in enumerate(slots):
        q = dec[:, s // 16, where[s % 16], :3].astype(np.float64)          # [16][3]
        delta = (vmax.astype(np.float64) - vmin.astype(np.float64)) / 255.0
        H = vmin.astype(np.float64)[:, None] + q * delta[:, None]
        for v in range(len(dirs)):
            Y = O.sh_basis(dirs[v].astype(np.float64))
            assert np.allclose(out[v, j], Y @ H, rtol=0, atol=1e-13)
            assert np.allclose(scale[v, j], np.abs(Y[:, None] * H).sum(0), rtol=0, atol=1e-13)
