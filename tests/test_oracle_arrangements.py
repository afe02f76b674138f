"""Pins of the oracle's block arrangements (Sec. IV-B): Fig. SetupA (one
primitive per block) and Fig. SetupB (four primitives per four blocks),
beside the band arrangement of Fig. SetupD.  The packers are checked against
array reshapes written independently of the C loops, for membership and
bijectivity on identity-coded inputs, and decode_eval against a route
through whole decoded textures."""
import numpy as np
import pytest

import oracle as O
from paper_2607_14513_amd import synth


def _slot_vectors(q, perm):
    """q[perm] padded to a multiple of 16 slots by repeating the last slot."""
    n = perm.shape[0]
    npad = (n + 15) // 16 * 16
    idx = np.concatenate([perm, np.full(npad - n, perm[-1], perm.dtype)])
    return q[idx]


@pytest.mark.parametrize("n", [1, 17, 1003])
def test_packers_equal_array_reshapes(n):
    pos, sh = synth.make_scene(n, seed=60 + n)
    perm, _, vmin, vmax = O.reorder(pos, sh)
    q = O.quantise(sh, vmin, vmax)
    qs = _slot_vectors(q, perm)                       # [npad][16][3]
    npad = qs.shape[0]
    a = O.pack(q, perm, O.ARR_PRIM)
    assert a.shape == (1, npad, 16, 4)
    assert np.array_equal(a[0, :, :, :3], qs)         # block s = slot s, texel k = band k
    assert np.all(a[..., 3] == 255)
    b = O.pack(q, perm, O.ARR_QUAD)
    assert b.shape == (4, npad // 4, 16, 4)
    # [block][slot in group][band group][band in group][rgb] -> [group][block][row slot][col band]
    want = qs.reshape(npad // 4, 4, 4, 4, 3).transpose(2, 0, 1, 3, 4).reshape(4, npad // 4, 16, 3)
    assert np.array_equal(b[..., :3], want)
    assert np.all(b[..., 3] == 255)
    d = O.pack(q, perm, O.ARR_BANDS)
    assert np.array_equal(d, O.pack(q, perm))


def test_membership_and_bijection():
    """q[i][k] = (i mod 256, i div 256, k) names every (primitive, band)
    vector: every one lands exactly once among the first n slots, a SetupA
    block holds one primitive, a SetupB block holds four consecutive slots
    and four bands of one group."""
    n = 3000
    q = np.empty((n, 16, 3), np.uint8)
    i = np.arange(n)
    q[:, :, 0] = (i % 256)[:, None]
    q[:, :, 1] = (i // 256)[:, None]
    q[:, :, 2] = np.arange(16)[None, :]
    perm = np.random.default_rng(5).permutation(n).astype(np.uint32)
    npad = (n + 15) // 16 * 16
    inv = np.empty(n, np.int64)
    inv[perm] = np.arange(n)
    for arr in (O.ARR_PRIM, O.ARR_QUAD, O.ARR_BANDS):
        tex = O.pack(q, perm, arr)
        S, nblk = tex.shape[:2]
        assert S * nblk == npad
        prim = tex[..., 0].astype(np.int64) + 256 * tex[..., 1].astype(np.int64)
        band = tex[..., 2].astype(np.int64)
        slot = inv[prim]
        real = slot < n - 1                            # padding repeats slot n-1
        pairs = slot[real] * 16 + band[real]
        assert np.array_equal(np.sort(pairs), np.arange((n - 1) * 16))
        if arr == O.ARR_PRIM:
            assert np.all(slot == np.minimum(np.arange(nblk), n - 1)[None, :, None])
            assert np.all(band == np.arange(16)[None, None, :])
        elif arr == O.ARR_QUAD:
            for g in range(4):
                assert np.all(band[g] // 4 == g)
            blk = np.arange(nblk)[None, :, None]
            assert np.all((slot // 4 == blk) | (slot == n - 1))


@pytest.mark.parametrize("arr,fmt", [(O.ARR_PRIM, [7]), (O.ARR_PRIM, [1]), (O.ARR_QUAD, [7, 1, 1, 1]),
                                     (O.ARR_QUAD, [1, 7, 1, 7])])
def test_decode_eval_follows_the_arrangement(arr, fmt):
    n, V = 203, 5
    pos, sh = synth.make_scene(n, seed=66)
    perm, tex, vmin, vmax = O.reorder(pos, sh, arrangement=arr)
    fmt = np.array(fmt, np.uint8)
    payload, off, _ = O.encode(tex, fmt)
    dirs = synth.make_dirs(V, seed=66)
    slots = np.arange(n, dtype=np.uint32)
    out = O.decode_eval(payload, off, fmt, vmin, vmax, dirs, slots, with_scale=False, arrangement=arr)
    # the same colours through whole decoded textures, unpacked by reshapes
    dec = O.decode_stream(payload, off, fmt, tex.shape[1])[..., :3]
    npad = tex.shape[0] * tex.shape[1]
    if arr == O.ARR_PRIM:
        codes = dec[0]
    else:
        codes = dec.reshape(4, npad // 4, 4, 4, 3).transpose(1, 2, 0, 3, 4).reshape(npad, 16, 3)
    delta = (vmax.astype(np.float64) - vmin.astype(np.float64)) / 255.0
    H = vmin.astype(np.float64)[None, :, None] + codes[:n].astype(np.float64) * delta[None, :, None]
    Y = np.stack([O.sh_basis(d) for d in dirs])               # [V][16]
    want = np.einsum("vk,jkc->vjc", Y, H)
    assert np.allclose(out, want, rtol=0, atol=1e-12)
    view = np.array([0.3, -2.0, 0.7], np.float32)
    ov = O.decode_eval_view(payload, off, fmt, vmin, vmax, pos, perm, view, slots, with_scale=False,
                            arrangement=arr)
    d = view.astype(np.float64)[None, :] - pos[perm].astype(np.float64)
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    Yv = np.stack([O.sh_basis(x) for x in d])
    assert np.allclose(ov, np.einsum("jk,jkc->jc", Yv, H), rtol=0, atol=1e-12)
