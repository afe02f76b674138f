"""GPU: gsbc_decode_eval_noalloc (the allocation-free decode_eval, whose
basis scratch is the library's static device array) gives the same colours
as gsbc_decode_eval, bit for bit, on two calls in a row -- the second with
fewer primitives and directions, so it reads only rows it rewrote -- and
rejects more directions than its array holds."""
import sys

import numpy as np
import pytest

from paper_2607_14513_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def _scene(ctx, gsbc, n, seed):
    pos, sh = synth.make_scene(n, seed=seed)
    _, tex, d = ctx.reorder(torch.from_numpy(pos).cuda(), torch.from_numpy(sh).cuda())
    blocks, d2, _ = ctx.encode(tex, d, fmt=gsbc.FMT_AUTO, rate=6.0)
    return blocks, d2


def test_noalloc_equals_decode_eval():
    from paper_2607_14513_amd import gsbc
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    with gsbc.Context(0) as ctx:
        for n, V, seed in ((20_011, 1024, 81), (4_101, 37, 82)):
            say("noalloc decode_eval", n, V)
            blocks, d = _scene(ctx, gsbc, n, seed)
            dirs = torch.from_numpy(synth.make_dirs(V, seed=seed)).cuda()
            ref = ctx.decode_eval(blocks, d, dirs)
            out = torch.full((V, n, 3), float("nan"), dtype=torch.float32, device="cuda")
            ctx.decode_eval(blocks, d, dirs, out=out, noalloc=True)
            torch.cuda.synchronize()
            assert torch.equal(out, ref), (n, V)
            # a slot subset through the same scratch
            idx = torch.tensor([n - 1, 0, 17, 5], dtype=torch.int32, device="cuda")
            few = dirs[:3].contiguous()
            sub = ctx.decode_eval(blocks, d, few, prim_idx=idx, noalloc=True)
            ref_sub = ctx.decode_eval(blocks, d, few, prim_idx=idx)
            torch.cuda.synchronize()
            assert torch.equal(sub, ref_sub)
        too_many = torch.from_numpy(synth.make_dirs(1025, seed=1)).cuda()
        with pytest.raises(gsbc.GsbcError) as e:
            ctx.decode_eval(blocks, d, too_many, noalloc=True)
        assert e.value.status == gsbc.E_ARG
