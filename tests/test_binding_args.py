"""The Python binding rejects tensors whose shape or size disagrees with the
counts and the stream descriptor before any library call: the C ABI takes
bare pointers and cannot see a tensor's extent.  CPU only: a context object is
made without a device, so a check that were missing would reach the library
with a NULL context and fail with GsbcError instead of ValueError."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
from paper_2607_14513_amd import gsbc  # noqa: E402


@pytest.fixture
def ctx():
    c = object.__new__(gsbc.Context)
    c._h = None
    c.device = torch.device("cpu")
    return c


def _desc(n, fmt=1, streams=16):
    d = gsbc.StreamDesc()
    nblk = (n + 15) // 16
    d.n_prims, d.n_pad, d.blocks_per_stream = n, nblk * 16, nblk
    d.arrangement, d.n_streams = gsbc.ARR_BANDS, streams
    pos = 0
    for k in range(streams):
        d.format[k] = fmt
        d.offset[k] = pos
        pos = (pos + nblk * (8 if fmt == 1 else 16) + 15) // 16 * 16
    d.payload_bytes = pos
    return d


def test_reorder_shapes(ctx):
    n = 37
    pos = torch.zeros((n, 3), dtype=torch.float32)
    sh = torch.zeros((n, 16, 3), dtype=torch.float32)
    with pytest.raises(ValueError):
        ctx.reorder(pos.reshape(-1), sh)                       # flat positions
    with pytest.raises(ValueError):
        ctx.reorder(pos, torch.zeros((n, 9, 3), dtype=torch.float32))   # degree-2 SH
    with pytest.raises(ValueError):
        ctx.reorder(pos, sh[:-1].contiguous())
    with pytest.raises(ValueError):
        ctx.reorder(pos, sh, opacity=torch.zeros(n + 1, dtype=torch.float32))
    perm_short = torch.zeros(n - 1, dtype=torch.int32)
    tex = torch.zeros((16, 3, 16, 4), dtype=torch.uint8)
    with pytest.raises(ValueError):
        ctx.reorder(pos, sh, out=(perm_short, tex))
    with pytest.raises(ValueError):
        ctx.reorder(pos, sh, out=(torch.zeros(n, dtype=torch.int32), tex[:, :2].contiguous()))
    with pytest.raises(TypeError):
        ctx.reorder(pos.double(), sh)
    with pytest.raises(TypeError):                              # right shapes, host memory
        ctx.reorder(pos, sh)
    with pytest.raises(ValueError):
        ctx.reorder_degrees(pos, torch.zeros((n, 16, 4), dtype=torch.float32))


def test_encode_and_decode_sizes(ctx):
    n = 100
    d = _desc(n)
    nblk = d.blocks_per_stream
    with pytest.raises(ValueError):
        ctx.encode(torch.zeros(16 * nblk * 64 - 1, dtype=torch.uint8), d, fmt=gsbc.FMT_BC1,
                   blocks=torch.zeros(d.payload_bytes, dtype=torch.uint8))
    # a descriptor whose sizes disagree is not sized here: the library rejects
    # it before anything is enqueued (host tensors stop at the device check)
    bad = _desc(n)
    bad.n_streams = 0
    with pytest.raises(TypeError):
        ctx.encode(torch.zeros(16 * nblk * 64, dtype=torch.uint8), bad, fmt=gsbc.FMT_BC1,
                   blocks=torch.zeros(d.payload_bytes, dtype=torch.uint8))
    with pytest.raises(ValueError):
        ctx.decode(torch.zeros(d.payload_bytes - 16, dtype=torch.uint8), d)
    with pytest.raises(ValueError):
        ctx.decode(torch.zeros(d.payload_bytes, dtype=torch.uint8), d,
                   out=torch.zeros((16, nblk - 1, 16, 4), dtype=torch.uint8))
    with pytest.raises(ValueError):
        ctx.save("unused.gsbc", torch.zeros(d.payload_bytes - 1, dtype=torch.uint8), d)
    with pytest.raises(ValueError):
        ctx.encode_batch([torch.zeros(64, dtype=torch.uint8)], [d], [torch.zeros(d.payload_bytes, dtype=torch.uint8)])


def test_decode_eval_shapes(ctx):
    n, V = 50, 7
    d = _desc(n, fmt=7)
    blocks = torch.zeros(d.payload_bytes, dtype=torch.uint8)
    dirs = torch.zeros((V, 3), dtype=torch.float32)
    with pytest.raises(ValueError):
        ctx.decode_eval(blocks[:-1], d, dirs)
    with pytest.raises(ValueError):
        ctx.decode_eval(blocks, d, torch.zeros((V, 4), dtype=torch.float32))
    with pytest.raises(ValueError):
        ctx.decode_eval(blocks, d, dirs.reshape(-1))
    with pytest.raises(ValueError):
        ctx.decode_eval(blocks, d, dirs, out=torch.zeros((V, n - 1, 3), dtype=torch.float32))
    with pytest.raises(ValueError):
        ctx.decode_eval(blocks, d, dirs, prim_idx=torch.zeros((2, 3), dtype=torch.int32))
    with pytest.raises(TypeError):
        ctx.decode_eval(blocks, d, dirs)
    pos = torch.zeros((n, 3), dtype=torch.float32)
    perm = torch.zeros(n, dtype=torch.int32)
    with pytest.raises(ValueError):
        ctx.decode_eval_view(blocks, d, pos[:-1].contiguous(), perm, (0.0, 0.0, 1.0))
    with pytest.raises(ValueError):
        ctx.decode_eval_view(blocks, d, pos, perm[:-1].contiguous(), (0.0, 0.0, 1.0))
    with pytest.raises(ValueError):
        ctx.decode_eval_view(blocks, d, pos, perm, (0.0, 0.0, 1.0), out=torch.zeros((n, 4), dtype=torch.float32))
    with pytest.raises(TypeError):
        ctx.decode_eval_view(blocks, d, pos, perm, (0.0, 0.0, 1.0))
    assert np.all(d.formats() == 7)
