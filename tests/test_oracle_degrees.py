"""Pins of the oracle's variable number of bands (Sec. IV-B): degree
classes, the class-major sort, the per-class textures, and decode_eval of a
scene whose higher bands were dropped."""
import numpy as np
import pytest

import oracle as O
from paper_2607_14513_amd import synth


def test_degree_of_single_coefficients():
    """One coefficient above tau in band k (any channel, either sign) puts the
    primitive in degree floor(sqrt(k)); a value equal to tau does not count."""
    tau = np.float32(0.01)
    rows = []
    want = []
    for k in range(16):
        for c in range(3):
            for v in (0.5, -0.5):
                x = np.zeros((16, 3), np.float32)
                x[k, c] = v
                x[0] = 0.3                                   # the DC band never matters
                rows.append(x)
                want.append(0 if k == 0 else int(np.sqrt(k)))
    x = np.zeros((16, 3), np.float32)
    x[9:, :] = tau                                            # at tau: not above
    rows.append(x)
    want.append(0)
    x = np.zeros((16, 3), np.float32)
    x[4, 2] = np.nextafter(tau, np.float32(1))               # just above
    x[2, 0] = 1.0
    rows.append(x)
    want.append(2)
    got = O.degrees(np.stack(rows), float(tau))
    assert got.tolist() == want


def test_degree_mix_scene_recovers_the_drawn_degrees():
    """Bands above each primitive's drawn degree hold |x| <= small: tau =
    small recovers the degree whenever some kept coefficient of the top
    degree exceeds small (Laplace draws: all but a handful)."""
    n = 4000
    mix = (0.3, 0.2, 0.2, 0.3)
    pos, sh = synth.make_scene(n, seed=17, degree_mix=mix, small=1e-4)
    deg = O.degrees(sh, 1e-4)
    frac = np.bincount(deg, minlength=4) / n
    assert np.all(np.abs(frac - np.array(mix)) < 0.04), frac
    assert np.all(O.degrees(sh, 0.0) == 3)                   # nothing is exactly zero


@pytest.mark.parametrize("tau", [0.0, 1e-4])
def test_reorder_degrees_structure(tau):
    n = 3001
    pos, sh = synth.make_scene(n, seed=18, degree_mix=(0.25, 0.25, 0.25, 0.25), small=1e-4 if tau else 0.0)
    perm, counts, tex, vmin, vmax = O.reorder_degrees(pos, sh, tau)
    deg = O.degrees(sh, tau)
    assert counts.sum() == n and np.array_equal(counts, np.bincount(deg, minlength=4))
    assert np.array_equal(np.sort(perm), np.arange(n))
    # classes in increasing degree; inside a class the order of the plain keys
    assert np.all(np.diff(deg[perm].astype(int)) >= 0)
    lo, hi = O.pos_aabb(pos)
    q = O.quantise(sh, vmin, vmax)
    plain = O.keys(pos, q, 3, lo, hi)
    start = np.concatenate([[0], np.cumsum(counts)])
    for L in range(4):
        part = perm[start[L]:start[L + 1]]
        assert np.all(deg[part] == L)
        kp = plain[part]
        assert np.all((kp[1:] > kp[:-1]) | ((kp[1:] == kp[:-1]) & (part[1:] > part[:-1])))
        t = tex[L]
        nb = (L + 1) ** 2
        assert t.shape == (nb, (counts[L] + 15) // 16, 16, 4)
        # slot j of the class at block j/16, zigzag texel: its kept bands' codes
        for j in (0, counts[L] // 2, counts[L] - 1):
            texel = O.zigzag_texel(j % 16)
            assert np.array_equal(t[:, j // 16, texel, :3], q[part[j], :nb])


def test_decode_eval_of_dropped_bands_is_zero():
    """A degree-1 class scene (4 streams): colours equal the decoded kept
    bands dotted with the first 4 basis functions, the others contributing
    nothing."""
    n = 500
    pos, sh = synth.make_scene(n, seed=19, degree_mix=(0.0, 1.0, 0.0, 0.0))
    perm, counts, tex, vmin, vmax = O.reorder_degrees(pos, sh, 0.0)
    assert counts.tolist() == [0, n, 0, 0]
    fmt = np.array([7, 1, 1, 1], np.uint8)
    payload, off, _ = O.encode(tex[1], fmt)
    dirs = synth.make_dirs(6, seed=19)
    slots = np.arange(n, dtype=np.uint32)
    out = O.decode_eval(payload, off, fmt, vmin, vmax, dirs, slots, with_scale=False)
    dec = O.decode_stream(payload, off, fmt, tex[1].shape[1])
    delta = (vmax.astype(np.float64) - vmin.astype(np.float64)) / 255.0
    H = np.zeros((n, 16, 3))
    for j in range(n):
        codes = dec[:, j // 16, O.zigzag_texel(j % 16), :3].astype(np.float64)
        H[j, :4] = vmin[:4, None] + codes * delta[:4, None]
    Y = np.stack([O.sh_basis(d) for d in dirs])
    assert np.allclose(out, np.einsum("vk,jkc->vjc", Y, H), rtol=0, atol=1e-12)


def test_setup_c_block_layout():
    """Fig. SetupC: block b of the degree-1 class holds class slots 4b..4b+3,
    slot i of the block on row i and band k (0..3) in column k -- its four
    texels are that primitive's four kept codes; the other classes keep the
    per-band streams.  Padded slots repeat the class's last primitive."""
    n = 1003
    pos, sh = synth.make_scene(n, seed=20, degree_mix=(0.25, 0.35, 0.15, 0.25))
    perm, counts, tex, vmin, vmax = O.reorder_degrees(pos, sh, 0.0, arrangement=O.ARR_QUAD)
    p2, c2, t2, _, _ = O.reorder_degrees(pos, sh, 0.0)
    assert np.array_equal(perm, p2) and np.array_equal(counts, c2)
    for L in (0, 2, 3):
        assert np.array_equal(tex[L], t2[L])
    q = O.quantise(sh, vmin, vmax)
    c1 = int(counts[1])
    part = perm[counts[0]:counts[0] + c1]
    t = tex[1]
    npad = (c1 + 15) // 16 * 16
    assert t.shape == (1, npad // 4, 16, 4)
    for j in range(npad):
        src = part[min(j, c1 - 1)]
        block = t[0, j // 4]
        assert np.array_equal(block[4 * (j % 4):4 * (j % 4) + 4, :3], q[src, :4]), j
        assert np.all(block[:, 3] == 255)
    # the same codes as the per-band class textures, moved
    for j in range(c1):
        for k in range(4):
            assert np.array_equal(t[0, j // 4, 4 * (j % 4) + k, :3], t2[1][k, j // 16, O.zigzag_texel(j % 16), :3])


def test_setup_c_decode_eval():
    """decode_eval of a Fig. SetupC scene: each slot's four texels of its
    block, dequantised, dotted with the first four basis functions; bands
    4..15 contribute nothing."""
    n = 500
    pos, sh = synth.make_scene(n, seed=21, degree_mix=(0.0, 1.0, 0.0, 0.0))
    perm, counts, tex, vmin, vmax = O.reorder_degrees(pos, sh, 0.0, arrangement=O.ARR_QUAD)
    assert counts.tolist() == [0, n, 0, 0] and tex[1].shape[0] == 1
    for f in (1, 7):
        fmt = np.array([f], np.uint8)
        payload, off, _ = O.encode(tex[1], fmt)
        dirs = synth.make_dirs(5, seed=21)
        slots = np.arange(n, dtype=np.uint32)
        out = O.decode_eval(payload, off, fmt, vmin, vmax, dirs, slots, with_scale=False, arrangement=O.ARR_QUAD)
        dec = O.decode_stream(payload, off, fmt, tex[1].shape[1])
        delta = (vmax.astype(np.float64) - vmin.astype(np.float64)) / 255.0
        H = np.zeros((n, 16, 3))
        for j in range(n):
            codes = dec[0, j // 4, 4 * (j % 4):4 * (j % 4) + 4, :3].astype(np.float64)
            H[j, :4] = vmin[:4, None] + codes * delta[:4, None]
        Y = np.stack([O.sh_basis(d) for d in dirs])
        assert np.allclose(out, np.einsum("vk,jkc->vjc", Y, H), rtol=0, atol=1e-12)
