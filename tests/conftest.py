import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP C-ABI library)")
    config.addinivalue_line("markers", "slow: long-running CPU pin")


def rgba(tex_rgb):
    """uint8[..., 16, 3] -> uint8[..., 16, 4] with alpha 255."""
    a = np.full(tex_rgb.shape[:-1] + (1,), 255, np.uint8)
    return np.concatenate([tex_rgb.astype(np.uint8), a], axis=-1)


def smooth_blocks(n, seed, spread=12):
    """Blocks of 16 texels near one base colour (the statistics sorted bands have)."""
    rng = np.random.default_rng(seed)
    base = rng.integers(0, 256, (n, 1, 3))
    return rgba(np.clip(base + rng.integers(-spread, spread + 1, (n, 16, 3)), 0, 255))


def random_blocks(n, seed):
    rng = np.random.default_rng(seed)
    return rgba(rng.integers(0, 256, (n, 16, 3)))


def load_golden(name):
    """Parse tests/golden/bc_handbuilt.txt style lines."""
    out = []
    with open(os.path.join(ROOT, "tests", "golden", name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            fmt, hexb, *tex = line.split()
            exp = {}
            for t in tex:
                i, v = t.split(":")
                exp[int(i)] = tuple(int(x) for x in v.split(","))
            out.append((fmt, bytes.fromhex(hexb), exp))
    return out


def oracle_blend_tiles_subset(rtex, fmt, vmin, vmax, pos, rperm, view, mu, foot, tile_start, lst, pick,
                              tiles_x, tiles_y):
    """The oracle's FP64 colour stage on the tiles in ``pick`` only, with a
    payload encoded from just the blocks their lists reach (a scene too
    large for the oracle to encode whole).  ``lst`` holds primitive ids in
    input order, ``rperm`` is the oracle's slot -> primitive order; every
    other tile's list is left empty.  Returns what ``O.blend_tiles`` does
    (image, transmittance and their bounds); only the picked tiles carry the
    scene's values.  Also returns the number of blocks encoded per band."""
    import oracle as O
    ts = np.asarray(tile_start, np.int64)
    pick = np.unique(np.asarray(pick, np.int64))         # the lists in tile order
    L = np.diff(ts)
    rslot = np.argsort(rperm).astype(np.uint32)
    slots = rslot[np.concatenate([lst[ts[t]:ts[t + 1]] for t in pick])]
    need = np.unique(slots)
    blk = np.unique(need // 16)
    payload, off, _ = O.encode(rtex[:, blk], fmt)
    renum = (16 * np.searchsorted(blk, need // 16) + need % 16).astype(np.uint32)
    perm_o = np.zeros(16 * blk.size, np.uint32)
    perm_o[renum] = rperm[need]
    cnt = np.zeros(tiles_x * tiles_y, np.int64)
    cnt[pick] = L[pick]
    ts_o = np.concatenate([[0], np.cumsum(cnt)]).astype(np.uint32)
    lst_o = renum[np.searchsorted(need, slots)]
    return O.blend_tiles(payload, off, fmt, vmin, vmax, pos, perm_o, view, mu, foot, ts_o, lst_o, tiles_x,
                         tiles_y), blk.size
