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


def test_decode_eval_dropped_bands_are_zero():
    """Streams given 0 bits (format 3) contribute nothing: with every band but
    the DC dropped the colour is H_0 / (2 sqrt(pi)) in every direction, and
    dropping bands changes the colour by exactly their terms."""
    pos, sh = synth.make_scene(300, seed=6)
    perm, tex, vmin, vmax = O.reorder(pos, sh)
    nblk = tex.shape[1]
    dirs = synth.make_dirs(7, seed=6)
    slots = np.array([0, 5, 16, 150, 299], np.uint32)
    only_dc = np.array([7] + [3] * 15, np.uint8)
    payload, off, _ = O.encode(tex, only_dc)
    assert payload.size == nblk * 16
    out = O.decode_eval(payload, off, only_dc, vmin, vmax, dirs, slots, with_scale=False)
    dec = O.decode_stream(payload, off, only_dc, nblk)
    assert not dec[1:].any()
    z = [[0, 1, 4, 5], [2, 3, 6, 7], [8, 9, 12, 13], [10, 11, 14, 15]]
    where = {z[y][x]: 4 * y + x for y in range(4) for x in range(4)}
    d0 = (np.float64(vmax[0]) - np.float64(vmin[0])) / 255.0
    for j, s in enumerate(slots):
        h0 = np.float64(vmin[0]) + dec[0, s // 16, where[s % 16], :3].astype(np.float64) * d0
        assert np.abs(out[:, j] - h0 / (2 * np.sqrt(np.pi))).max() < 1e-14
    full = np.array([7] + [1] * 15, np.uint8)
    some = full.copy()
    some[[3, 8, 15]] = 3
    pf, of, _ = O.encode(tex, full)
    ps, os_, _ = O.encode(tex, some)
    a = O.decode_eval(pf, of, full, vmin, vmax, dirs, slots, with_scale=False)
    b = O.decode_eval(ps, os_, some, vmin, vmax, dirs, slots, with_scale=False)
    for j, s in enumerate(slots):
        H = _decoded_H(pf, of, full, vmin, vmax, nblk, s)
        for v in range(len(dirs)):
            Y = O.sh_basis(dirs[v].astype(np.float64))
            dropped = sum(H[k] * Y[k] for k in (3, 8, 15))
            assert np.allclose(a[v, j] - b[v, j], dropped, rtol=0, atol=1e-13)


def _decoded_H(payload, off, fmt, vmin, vmax, nblk, s):
    dec = O.decode_stream(payload, off, fmt, nblk)
    z = [[0, 1, 4, 5], [2, 3, 6, 7], [8, 9, 12, 13], [10, 11, 14, 15]]
    where = {z[y][x]: 4 * y + x for y in range(4) for x in range(4)}
    q = dec[:, s // 16, where[s % 16], :3].astype(np.float64)
    delta = (vmax.astype(np.float64) - vmin.astype(np.float64)) / 255.0
    return vmin.astype(np.float64)[:, None] + q * delta[:, None]


def test_view_colour_closed_forms():
    """decode_eval_view (Sec. II, c(f) = H w(f - p)): a view position straight
    above a primitive sees it along +z, where only Y_0, Y_2, Y_6 and Y_12 are
    non-zero: 1/(2 sqrt pi), sqrt(3/4pi), (1/2) sqrt(5/pi), (1/2) sqrt(7/pi);
    a view position at the primitive itself (d = 0) leaves the DC term."""
    pos, sh = synth.make_scene(700, seed=8)
    perm, tex, vmin, vmax = O.reorder(pos, sh)
    nblk = tex.shape[1]
    fmt = np.array([7, 1, 7, 1] + [1] * 12, np.uint8)
    payload, off, _ = O.encode(tex, fmt)
    up = np.zeros(16)
    up[0] = 0.5 / np.sqrt(np.pi)
    up[2] = np.sqrt(3 / (4 * np.pi))
    up[6] = 0.5 * np.sqrt(5 / np.pi)
    up[12] = 0.5 * np.sqrt(7 / np.pi)
    for s in (0, 5, 16, 333, 699):
        p = pos[perm[s]]
        H = _decoded_H(payload, off, fmt, vmin, vmax, nblk, s)
        above = np.array([p[0], p[1], p[2] + np.float32(3.0)], np.float32)
        assert above[2] > p[2]
        out = O.decode_eval_view(payload, off, fmt, vmin, vmax, pos, perm, above, np.array([s], np.uint32),
                                 with_scale=False)
        assert np.allclose(out[0], up @ H, rtol=0, atol=1e-13)
        at = O.decode_eval_view(payload, off, fmt, vmin, vmax, pos, perm, p, np.array([s], np.uint32),
                                with_scale=False)
        assert np.allclose(at[0], H[0] * 0.5 / np.sqrt(np.pi), rtol=0, atol=1e-15)


def test_view_colour_direction_is_towards_the_view_position():
    """Moving the view position along the ray from a primitive does not
    change its colour (only the direction counts), and mirroring it through
    the primitive flips the odd-degree terms: c(p + u) - c(p - u) =
    2 sum_{l odd} H_lm Y_lm(u)."""
    pos, sh = synth.make_scene(300, seed=9)
    perm, tex, vmin, vmax = O.reorder(pos, sh)
    nblk = tex.shape[1]
    fmt = np.array([7] + [1] * 15, np.uint8)
    payload, off, _ = O.encode(tex, fmt)
    rng = np.random.default_rng(3)
    odd = np.array([0, 1, 1, 1, 0, 0, 0, 0, 0, 1, 1, 1, 1, 1, 1, 1], np.float64)
    for s in (3, 77, 299):
        p = pos[perm[s]].astype(np.float64)
        u = rng.normal(size=3)
        u /= np.linalg.norm(u)
        H = _decoded_H(payload, off, fmt, vmin, vmax, nblk, s)
        sl = np.array([s], np.uint32)
        cols = []
        for lam in (0.5, 4.0, -0.5):
            f = (p + lam * u).astype(np.float32)
            cols.append(O.decode_eval_view(payload, off, fmt, vmin, vmax, pos, perm, f, sl, with_scale=False)[0])
        assert np.allclose(cols[0], cols[1], rtol=0, atol=1e-6)     # float32 view positions
        Yu = O.sh_basis(u)
        assert np.allclose(cols[0] - cols[2], 2 * (odd * Yu) @ H, rtol=0, atol=1e-5)
