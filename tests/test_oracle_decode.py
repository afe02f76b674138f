"""Pins of the oracle's BC1 (D1) and BC7 (D2) decoders.

* hand-built blocks whose texels were derived by hand from the format
  definitions (tests/golden/bc_handbuilt.txt);
* Pillow's BCn decoder (an independent implementation, used by running it):
  BC7 bit-exact on random blocks of every mode; BC1 exact on endpoint and
  black texels and within 1 elsewhere (Pillow floors the 1/3, 2/3 and 1/2
  entries, this oracle rounds to nearest -- both are valid BC1 decoders).
"""
import numpy as np
import pytest

import oracle as O
from conftest import load_golden

PIL = pytest.importorskip("PIL.Image")


def _pillow(blocks, n):
    bsz = blocks.shape[1]
    im = PIL.frombytes("RGBA", (4 * blocks.shape[0], 4), blocks.tobytes(), "bcn", n)
    a = np.asarray(im)
    return a.reshape(4, blocks.shape[0], 4, 4).transpose(1, 0, 2, 3).reshape(blocks.shape[0], 16, 4)


def _mode(b0):
    for m in range(8):
        if (b0 >> m) & 1:
            return m
    return 8


def test_handbuilt_blocks():
    n = 0
    for fmt, blk, exp in load_golden("bc_handbuilt.txt"):
        arr = np.frombuffer(blk, np.uint8)
        dec = O.bc1_decode(arr)[0] if fmt == "bc1" else O.bc7_decode(arr)[0]
        for i, px in exp.items():
            assert tuple(int(x) for x in dec[i]) == px, (fmt, blk.hex(), i)
            n += 1
    assert n >= 25


def test_bc7_matches_pillow_on_random_blocks():
    rng = np.random.default_rng(0)
    blk = rng.integers(0, 256, (40000, 16), dtype=np.uint8)
    blk = blk[blk[:, 0] != 0]          # the reserved mode is checked separately
    modes = np.array([_mode(int(b)) for b in blk[:, 0]])
    assert set(modes.tolist()) == set(range(8))
    ours = O.bc7_decode(blk)
    pil = _pillow(blk, 7)
    assert np.array_equal(ours, pil)


def test_bc7_partition_maps_revealed():
    """Mode-1 blocks with a black subset 0 and a white subset 1 show each
    2-subset partition map; mode-2 blocks with black/grey/white subsets show
    each 3-subset map.  Pillow and the oracle must draw the same maps."""
    blocks = []
    for p in range(64):
        v, pos = 0, 0
        def put(x, n):
            nonlocal v, pos
            v |= x << pos
            pos += n
        put(2, 2); put(p, 6)
        for _ in range(3):
            put(0, 6); put(0, 6); put(63, 6); put(63, 6)
        put(0, 1); put(1, 1)
        put(0, 128 - pos)
        blocks.append(v.to_bytes(16, "little"))
    for p in range(64):
        v, pos = 0, 0
        def put(x, n):
            nonlocal v, pos
            v |= x << pos
            pos += n
        put(4, 3); put(p, 6)
        for _ in range(3):
            put(0, 5); put(0, 5); put(16, 5); put(16, 5); put(31, 5); put(31, 5)
        put(0, 128 - pos)
        blocks.append(v.to_bytes(16, "little"))
    arr = np.frombuffer(b"".join(blocks), np.uint8).reshape(-1, 16)
    ours = O.bc7_decode(arr)
    assert np.array_equal(ours, _pillow(arr, 7))
    # each map uses every subset and texel 0 is always in subset 0
    for b in range(128):
        vals = ours[b, :, 0]
        assert vals[0] == 0
        assert len(set(vals.tolist())) == (2 if b < 64 else 3)


def test_bc7_anchor_indices():
    """With every stored index field set to ones, a wrong anchor table would
    shift all later index bits; the decoders must still agree."""
    blocks = []
    for p in range(64):
        for mode in (1, 2):
            v, pos = 0, 0
            def put(x, n):
                nonlocal v, pos
                v |= x << pos
                pos += n
            if mode == 1:
                put(2, 2); put(p, 6)
                for _ in range(3):
                    put(5, 6); put(40, 6); put(20, 6); put(60, 6)
                put(1, 1); put(0, 1)
            else:
                put(4, 3); put(p, 6)
                for _ in range(3):
                    put(3, 5); put(29, 5); put(9, 5); put(17, 5); put(1, 5); put(25, 5)
            put((1 << (128 - pos)) - 1, 128 - pos)
            blocks.append(v.to_bytes(16, "little"))
    arr = np.frombuffer(b"".join(blocks), np.uint8).reshape(-1, 16)
    assert np.array_equal(O.bc7_decode(arr), _pillow(arr, 7))


def test_bc7_reserved_mode_is_zero():
    blk = np.zeros((3, 16), np.uint8)
    blk[1, 1:] = 0xFF
    blk[2, 5] = 0x5A
    assert not O.bc7_decode(blk).any()


def test_bc1_matches_pillow_within_rounding():
    rng = np.random.default_rng(1)
    blk = rng.integers(0, 256, (40000, 8), dtype=np.uint8)
    blk[:100, 2:4] = blk[:100, 0:2]                      # c0 == c1 cases
    ours = O.bc1_decode(blk).astype(int)
    pil = _pillow(blk, 1).astype(int)
    idx = np.stack([(blk[:, 4:8].copy().view("<u4")[:, 0] >> (2 * i)) & 3 for i in range(16)], 1)
    c0 = blk[:, 0].astype(int) | blk[:, 1].astype(int) << 8
    c1 = blk[:, 2].astype(int) | blk[:, 3].astype(int) << 8
    three = (c0 <= c1)[:, None]
    exact = (idx < 2) | (three & (idx == 3))
    d = np.abs(ours - pil)
    assert d[exact].max() == 0
    assert d[~exact].max() <= 1
    # the rounding reading: interpolated entries are the nearest integer to
    # the exact rational (2a+b)/3, (a+2b)/3, (a+b)/2
    assert (d[~exact] == 1).any()
