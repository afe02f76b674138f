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
