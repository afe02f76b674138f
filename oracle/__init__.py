"""CPU oracle for the 3DGS SH BC1/BC7 coding path -- TEST INFRASTRUCTURE ONLY.

Plain, slow, obviously-correct reference implementation (``gsbc_oracle.c``)
of every step of the path, wrapped for numpy.  Only the test suite, the smoke
check and the CPU-baseline leg of the benchmark may import it; the GPU library
never does, and this package imports nothing from the GPU library.

Steps (see the C file for the definitions and paper sections):
  band_range / pos_aabb / quantise   -- Q (Sec. V-A)
  keys                               -- K (Sec. III-C, Fig. Bit4Scan)
  sort                               -- S (Sec. III-C)
  pack                               -- B (Fig. SetupD, Fig. ZigZagScan;
                                        Figs. SetupA and SetupB)
  bc1_decode / bc7_decode            -- D1 / D2 (BC formats, Sec. III-B)
  bc1_encode / bc7_encode            -- E1 / E2 (BTC, Sec. III-A)
  rate_select / rate_select_zero /
  band_hist / encode_auto            -- R (Sec. IV-B)
  sh_basis / decode_eval             -- H (Sec. II colour equation), FP64
  blend_tiles                        -- C (Sec. II, eqs. blend, preblend,
                                        premult), FP64
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

FMT_BC1 = 1
FMT_BC7 = 7
FMT_NONE = 3   # a stream given 0 bits: not stored, its bands decode to zero

# Arrangements of the band coefficients into blocks (Sec. IV-B)
ARR_BANDS = 0   # Fig. SetupD: 16 primitives per block, one stream per band
ARR_PRIM = 1    # Fig. SetupA: one primitive per block, one stream
ARR_QUAD = 2    # Fig. SetupB: four primitives per four blocks, four streams
N_STREAMS = {ARR_BANDS: 16, ARR_PRIM: 1, ARR_QUAD: 4}


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build as _b
            _b.build()
        _lib = ctypes.CDLL(_LIB_PATH)
        u64, u32, i32 = ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int
        P = ctypes.c_void_p
        sig = {
            "ref_band_range": (None, [P, u64, P, P]),
            "ref_pos_aabb": (None, [P, u64, P, P]),
            "ref_quantise": (None, [P, u64, P, P, P]),
            "ref_premultiply": (None, [P, P, u64, P]),
            "ref_band_range_coverage": (None, [P, u64, u32, u32, P, P]),
            "ref_morton_rgb": (u32, [u32, u32, u32]),
            "ref_morton3": (u32, [u32, u32, u32, u32]),
            "ref_keys": (None, [P, P, u64, u32, P, P, P]),
            "ref_sort": (None, [P, u64, P]),
            "ref_zigzag_texel": (u32, [u32]),
            "ref_pack": (None, [P, P, u64, P]),
            "ref_pack_prim": (None, [P, P, u64, P]),
            "ref_pack_quad": (None, [P, P, u64, P]),
            "ref_principal_axis": (None, [i32, P, P]),
            "ref_bc7_ls_endpoints": (i32, [i32, P, P, i32, i32, P]),
            "ref_bc1_decode_block": (None, [P, P]),
            "ref_bc7_decode_block": (None, [P, P]),
            "ref_bc1_encode_block": (u32, [P, u32, P]),
            "ref_bc7_encode_block": (u32, [P, u32, P]),
            "ref_bc7_candidate": (i32, [i32, P, P, P, P]),
            "ref_init": (None, []),
            "ref_bc1_encode": (None, [P, u64, u32, P, P]),
            "ref_bc7_encode": (None, [P, u64, u32, P, P]),
            "ref_bc1_decode": (None, [P, u64, P]),
            "ref_bc7_decode": (None, [P, u64, P]),
            "ref_rate_select": (i32, [P, P, P, P, u32, ctypes.c_double, P]),
            "ref_rate_select_zero": (i32, [P, P, P, P, P, u32, ctypes.c_double, P]),
            "ref_sh_basis": (None, [ctypes.c_double] * 3 + [P]),
            "ref_decode_eval": (None, [P, P, P, u32, u32, P, P, P, u32, P, u64, P, P]),
            "ref_decode_eval_view": (None, [P, P, P, u32, u32, P, P, P, P, P, P, u64, P, P]),
            "ref_degrees": (None, [P, u64, ctypes.c_float, P]),
            "ref_blend_tiles": (None, [P, P, P, u32, u32, P, P, P, P, P, P, P, P, P, u32, u32, P, P, P, P]),
        }
        for name, (res, args) in sig.items():
            f = getattr(_lib, name)
            f.restype = res
            f.argtypes = args
    return _lib


def _p(a):
    return ctypes.c_void_p(a.ctypes.data) if a is not None else None


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def set_threads(n):
    """Threads used by the block-parallel loops (OpenMP)."""
    try:
        ctypes.CDLL("libgomp.so.1").omp_set_num_threads(int(n))
    except OSError:
        pass


# ---------------------------------------------------------------- Q, K, S, B
def band_range(sh):
    sh = _c(sh, np.float32)
    n = sh.shape[0]
    vmin = np.empty(16, np.float32)
    vmax = np.empty(16, np.float32)
    _load().ref_band_range(_p(sh), n, _p(vmin), _p(vmax))
    return vmin, vmax


def premultiply(sh, opacity):
    """H~ = mu H per primitive, FP32."""
    sh = _c(sh, np.float32)
    out = np.empty_like(sh)
    _load().ref_premultiply(_p(sh), _p(_c(opacity, np.float32)), sh.shape[0], _p(out))
    return out


def band_range_coverage(sh, num=995, den=1000):
    """Symmetric per-band range [-t, t] holding num/den of the coefficients."""
    sh = _c(sh, np.float32)
    vmin = np.empty(16, np.float32)
    vmax = np.empty(16, np.float32)
    _load().ref_band_range_coverage(_p(sh), sh.shape[0], int(num), int(den), _p(vmin), _p(vmax))
    return vmin, vmax


def pos_aabb(pos):
    pos = _c(pos, np.float32)
    lo = np.empty(3, np.float32)
    hi = np.empty(3, np.float32)
    _load().ref_pos_aabb(_p(pos), pos.shape[0], _p(lo), _p(hi))
    return lo, hi


def quantise(sh, vmin, vmax):
    sh = _c(sh, np.float32)
    q = np.empty((sh.shape[0], 16, 3), np.uint8)
    _load().ref_quantise(_p(sh), sh.shape[0], _p(_c(vmin, np.float32)), _p(_c(vmax, np.float32)), _p(q))
    return q


def morton_rgb(r, g, b):
    return int(_load().ref_morton_rgb(int(r), int(g), int(b)))


def zigzag_texel(j):
    return int(_load().ref_zigzag_texel(int(j)))


def keys(pos, q, grid_bits, lo, hi):
    pos = _c(pos, np.float32)
    q = _c(q, np.uint8)
    out = np.empty(pos.shape[0], np.uint64)
    _load().ref_keys(_p(pos), _p(q), pos.shape[0], int(grid_bits), _p(_c(lo, np.float32)),
                     _p(_c(hi, np.float32)), _p(out))
    return out


def sort(k):
    k = _c(k, np.uint64)
    perm = np.empty(k.shape[0], np.uint32)
    _load().ref_sort(_p(k), k.shape[0], _p(perm))
    return perm


def pack(q, perm, arrangement=ARR_BANDS):
    """textures uint8[S][npad/S][16][4] of the arrangement (S streams)."""
    q = _c(q, np.uint8)
    perm = _c(perm, np.uint32)
    n = perm.shape[0]
    npad = (n + 15) // 16 * 16
    S = N_STREAMS[arrangement]
    tex = np.empty((S, npad // S, 16, 4), np.uint8)
    fn = {ARR_BANDS: "ref_pack", ARR_PRIM: "ref_pack_prim", ARR_QUAD: "ref_pack_quad"}[arrangement]
    getattr(_load(), fn)(_p(q), _p(perm), n, _p(tex))
    return tex


def reorder(pos, sh, grid_bits=3, opacity=None, quantiser=0, arrangement=ARR_BANDS):
    """Q + K + S + B.  Returns (perm, textures[S][nblk][16][4], vmin, vmax).
    opacity: premultiply the coefficients first; quantiser 1: the symmetric
    99.5 % coverage range instead of min/max; arrangement: the block packing."""
    if opacity is not None:
        sh = premultiply(sh, opacity)
    vmin, vmax = band_range_coverage(sh) if quantiser == 1 else band_range(sh)
    lo, hi = pos_aabb(pos)
    q = quantise(sh, vmin, vmax)
    k = keys(pos, q, grid_bits, lo, hi)
    perm = sort(k)
    return perm, pack(q, perm, arrangement), vmin, vmax


def degrees(sh, tau=0.0):
    """uint8[n] degree class of every primitive (coefficients above tau)."""
    sh = _c(sh, np.float32)
    out = np.empty(sh.shape[0], np.uint8)
    _load().ref_degrees(_p(sh), sh.shape[0], float(tau), _p(out))
    return out


def reorder_degrees(pos, sh, tau=0.0, grid_bits=3, opacity=None, quantiser=0, arrangement=ARR_BANDS):
    """Variable number of bands (Sec. IV-B): every primitive goes to the
    bitstreams of its degree class, with (L+1)^2 bands.  Key = degree above
    the spatial cell and colour fields, so the sort groups the classes (in
    increasing degree) and orders each by cell and colour.  The quantiser
    range is taken over all coefficients, dropped ones included.  Returns
    (perm, counts[4], textures: list of 4 (uint8[(L+1)^2][nblk_L][16][4], or
    None for an empty class), vmin, vmax); class L owns slots
    sum(counts[:L]) .. sum(counts[:L+1]) - 1 of perm.  arrangement ARR_QUAD
    packs the degree-1 class as Fig. SetupC: its four bands of four
    primitives per block, which is the first stream of Fig. SetupB's
    packing (uint8[1][pad16(counts[1])/4][16][4])."""
    if opacity is not None:
        sh = premultiply(sh, opacity)
    vmin, vmax = band_range_coverage(sh) if quantiser == 1 else band_range(sh)
    lo, hi = pos_aabb(pos)
    q = quantise(sh, vmin, vmax)
    deg = degrees(sh, tau)
    k = keys(pos, q, grid_bits, lo, hi) | (deg.astype(np.uint64) << np.uint64(24 + 3 * grid_bits))
    perm = sort(k)
    counts = np.bincount(deg, minlength=4).astype(np.int64)
    start = np.concatenate([[0], np.cumsum(counts)])
    tex = []
    for L in range(4):
        if counts[L] == 0:
            tex.append(None)
            continue
        part = perm[start[L]:start[L + 1]]
        if L == 1 and arrangement == ARR_QUAD:
            tex.append(pack(q, part, ARR_QUAD)[:1])
        else:
            tex.append(pack(q, part)[:(L + 1) ** 2])
    return perm, counts, tex, vmin, vmax


# ---------------------------------------------------------------- D, E
def principal_axis(x):
    """Integer power-iteration axis (E1 step 2) of the triples x[n][3]."""
    x = _c(np.asarray(x), np.int32).reshape(-1, 3)
    v = np.zeros(3, np.int64)
    _load().ref_principal_axis(x.shape[0], _p(x), _p(v))
    return v


def bc7_ls_endpoints(x, idx, nb):
    """E2 step (d): least-squares endpoints of the members x[n][nch] for
    their nb-bit indices -> (lo[nch], hi[nch]) or None when singular."""
    x = np.asarray(x)
    nch = 1 if x.ndim == 1 else x.shape[1]
    xx = np.zeros((len(x), 3), np.int32)
    xx[:, :nch] = x.reshape(len(x), nch)
    ii = _c(np.asarray(idx), np.int32)
    out = np.zeros(6, np.int32)
    if not _load().ref_bc7_ls_endpoints(len(x), _p(xx), _p(ii), int(nb), nch, _p(out)):
        return None
    return out[:nch].copy(), out[3:3 + nch].copy()


def bc1_decode(blocks):
    blocks = _c(blocks, np.uint8).reshape(-1, 8)
    out = np.empty((blocks.shape[0], 16, 4), np.uint8)
    _load().ref_bc1_decode(_p(blocks), blocks.shape[0], _p(out))
    return out


def bc7_decode(blocks):
    blocks = _c(blocks, np.uint8).reshape(-1, 16)
    out = np.empty((blocks.shape[0], 16, 4), np.uint8)
    _load().ref_bc7_decode(_p(blocks), blocks.shape[0], _p(out))
    return out


def bc1_encode(tex, refine_steps=2):
    """tex uint8[nblk][16][4] -> (blocks uint8[nblk][8], sse uint32[nblk])."""
    tex = _c(tex, np.uint8).reshape(-1, 16, 4)
    nb = tex.shape[0]
    blocks = np.empty((nb, 8), np.uint8)
    sse = np.empty(nb, np.uint32)
    _load().ref_bc1_encode(_p(tex), nb, int(refine_steps), _p(blocks), _p(sse))
    return blocks, sse


def bc7_encode(tex, mode_mask=0xFF):
    """tex uint8[nblk][16][4] -> (blocks uint8[nblk][16], sse uint32[nblk])."""
    tex = _c(tex, np.uint8).reshape(-1, 16, 4)
    nb = tex.shape[0]
    blocks = np.empty((nb, 16), np.uint8)
    sse = np.empty(nb, np.uint32)
    _load().ref_bc7_encode(_p(tex), nb, int(mode_mask), _p(blocks), _p(sse))
    return blocks, sse


def bc7_candidate(ci):
    m, p, r, s = (ctypes.c_int() for _ in range(4))
    rc = _load().ref_bc7_candidate(int(ci), ctypes.byref(m), ctypes.byref(p), ctypes.byref(r), ctypes.byref(s))
    if rc != 0:
        raise IndexError(ci)
    return m.value, p.value, r.value, s.value


# ---------------------------------------------------------------- R
def rate_select(sse1, sse7, vmin, vmax, rate, S=16):
    """Per-band formats (uint8[S], 1 or 7) of an S-band scene, or None when
    the rate is infeasible: band 0 BC7, the k = rate*S/4 - S - 1 largest-gain
    bands of 1..S-1 BC7."""
    fmt = np.zeros(16, np.uint8)
    rc = _load().ref_rate_select(_p(_c(sse1, np.int64)), _p(_c(sse7, np.int64)),
                                 _p(_c(vmin, np.float32)), _p(_c(vmax, np.float32)),
                                 int(S), float(rate), _p(fmt))
    return None if rc != 0 else fmt[:S].copy()


def band_hist(tex):
    """Code histograms of each stream's R, G and B channels: uint64[S][256]
    (the input of the 0-bit option's distortion)."""
    tex = _c(tex, np.uint8)
    S = tex.shape[0]
    h = np.zeros((16, 256), np.uint64)
    for b in range(S):
        h[b] = np.bincount(tex[b][..., :3].reshape(-1), minlength=256).astype(np.uint64)
    return h[:S]


def rate_select_zero(sse1, sse7, hist, vmin, vmax, rate, S=16):
    """Per-band formats (uint8[S]: 7, 1 or FMT_NONE) with the 0-bit option,
    or None when infeasible (see ref_rate_select_zero)."""
    h = np.zeros((16, 256), np.uint64)
    h[:S] = np.asarray(hist, np.uint64)[:S]
    fmt = np.zeros(16, np.uint8)
    rc = _load().ref_rate_select_zero(_p(_c(sse1, np.int64)), _p(_c(sse7, np.int64)), _p(h),
                                      _p(_c(vmin, np.float32)), _p(_c(vmax, np.float32)),
                                      int(S), float(rate), _p(fmt))
    return None if rc != 0 else fmt[:S].copy()


def stream_layout(fmt, nblk):
    """Byte offset of each stream in the concatenated payload (streams in order,
    each 16-byte aligned; one per entry of fmt; a 0-bit stream takes no bytes)
    and the total payload size."""
    off = np.zeros(len(fmt), np.uint64)
    pos = 0
    for b in range(len(fmt)):
        off[b] = pos
        f = int(fmt[b])
        pos += 0 if f == FMT_NONE else nblk * (8 if f == FMT_BC1 else 16)
        pos = (pos + 15) // 16 * 16
    return off, pos


def encode(tex, fmt, refine_steps=2, mode_mask=0xFF):
    """Encode every stream of tex[S][nblk][16][4] in the given per-stream formats
    (the first S entries of fmt; FMT_NONE streams are not stored); returns
    (payload uint8[], offsets uint64[S], sse int64[S], 0 for FMT_NONE)."""
    tex = _c(tex, np.uint8)
    S, nblk = tex.shape[0], tex.shape[1]
    fmt = np.asarray(fmt)[:S]
    off, total = stream_layout(fmt, nblk)
    payload = np.zeros(total, np.uint8)
    sse = np.zeros(S, np.int64)
    for b in range(S):
        if int(fmt[b]) == FMT_NONE:
            continue
        if int(fmt[b]) == FMT_BC1:
            blk, s = bc1_encode(tex[b], refine_steps)
        else:
            blk, s = bc7_encode(tex[b], mode_mask)
        o = int(off[b])
        payload[o:o + blk.size] = blk.reshape(-1)
        sse[b] = int(s.astype(np.int64).sum())
    return payload, off, sse


def encode_auto(tex, vmin, vmax, rate, refine_steps=2, mode_mask=0xFF, zero=False):
    """Rate-controlled encode of an S-band scene tex[S][nblk][16][4]: band 0
    BC7; bands 1..S-1 encoded in both formats, then rate_select (or, with
    zero, rate_select_zero over the band code histograms).  Returns
    (payload, offsets, formats) or None when infeasible."""
    tex = _c(tex, np.uint8)
    S = tex.shape[0]
    sse1 = np.zeros(16, np.int64)
    sse7 = np.zeros(16, np.int64)
    for b in range(1, S):
        sse1[b] = int(bc1_encode(tex[b], refine_steps)[1].astype(np.int64).sum())
    for b in range(S):
        sse7[b] = int(bc7_encode(tex[b], mode_mask)[1].astype(np.int64).sum())
    if zero:
        fmt = rate_select_zero(sse1, sse7, band_hist(tex), vmin, vmax, rate, S)
    else:
        fmt = rate_select(sse1, sse7, vmin, vmax, rate, S)
    if fmt is None:
        return None
    payload, off, _ = encode(tex, fmt, refine_steps, mode_mask)
    return payload, off, fmt


def decode_stream(payload, off, fmt, nblk):
    """Decode every stream (one per entry of fmt) back to textures uint8[S][nblk][16][4]
    (a FMT_NONE stream to zero texels; its coefficients are zero, not vmin)."""
    out = np.empty((len(fmt), nblk, 16, 4), np.uint8)
    for b in range(len(fmt)):
        o = int(off[b])
        if int(fmt[b]) == FMT_NONE:   # no blocks: texels all zero
            out[b] = 0
        elif int(fmt[b]) == FMT_BC1:
            out[b] = bc1_decode(payload[o:o + nblk * 8])
        else:
            out[b] = bc7_decode(payload[o:o + nblk * 16])
    return out


# ---------------------------------------------------------------- H
def sh_basis(d):
    """FP64 real SH basis (16 values) at direction d (3-vector)."""
    Y = np.empty(16, np.float64)
    _load().ref_sh_basis(float(d[0]), float(d[1]), float(d[2]), _p(Y))
    return Y


def _streams16(fmt, off):
    """Pad per-stream formats and offsets to the 16 entries the C side reads."""
    f = np.zeros(16, np.uint8)
    o = np.zeros(16, np.uint64)
    f[:len(fmt)] = fmt
    o[:len(off)] = off
    return f, o


def decode_eval(payload, off, fmt, vmin, vmax, dirs, slots, with_scale=True, arrangement=ARR_BANDS):
    """FP64 decode_eval.  Returns out[V][M][3] (and scale[V][M][3]).  Fewer
    formats than the arrangement's streams mean a scene of lower-degree
    primitives (band arrangement: bands past the streams; quad arrangement
    with one stream: Fig. SetupC, bands 4..15): the missing bands are zero."""
    ns = len(fmt)
    fmt, off = _streams16(fmt, off)
    payload = _c(payload, np.uint8)
    dirs = _c(dirs, np.float32).reshape(-1, 3)
    slots = _c(slots, np.uint32)
    V, M = dirs.shape[0], slots.shape[0]
    out = np.empty((V, M, 3), np.float64)
    scale = np.empty((V, M, 3), np.float64) if with_scale else None
    _load().ref_decode_eval(_p(payload), _p(_c(fmt, np.uint8)), _p(_c(off, np.uint64)), int(arrangement), ns,
                            _p(_c(vmin, np.float32)), _p(_c(vmax, np.float32)), _p(dirs), V,
                            _p(slots), M, _p(out), _p(scale) if scale is not None else None)
    return (out, scale) if with_scale else out


def decode_eval_view(payload, off, fmt, vmin, vmax, pos, perm, view, slots, with_scale=True,
                     arrangement=ARR_BANDS):
    """FP64 colour of each slot seen from view position `view` (direction
    (view - p)/|view - p| per primitive).  Returns out[M][3] (and scale)."""
    ns = len(fmt)
    fmt, off = _streams16(fmt, off)
    payload = _c(payload, np.uint8)
    pos = _c(pos, np.float32).reshape(-1, 3)
    perm = _c(perm, np.uint32)
    slots = _c(slots, np.uint32)
    view = _c(np.asarray(view, np.float32).reshape(3), np.float32)
    M = slots.shape[0]
    out = np.empty((M, 3), np.float64)
    scale = np.empty((M, 3), np.float64) if with_scale else None
    _load().ref_decode_eval_view(_p(payload), _p(_c(fmt, np.uint8)), _p(_c(off, np.uint64)), int(arrangement), ns,
                                 _p(_c(vmin, np.float32)), _p(_c(vmax, np.float32)), _p(pos), _p(perm),
                                 _p(view), _p(slots), M, _p(out), _p(scale) if scale is not None else None)
    return (out, scale) if with_scale else out


# ---------------------------------------------------------------- C
def blend_tiles(payload, off, fmt, vmin, vmax, pos, perm, view, mu, foot, tile_start, lst, tiles_x, tiles_y,
                arrangement=ARR_BANDS):
    """FP64 colour stage (see ref_blend_tiles): returns (image[H][W][3],
    transmittance[H][W], bound[H][W][3], bound_t[H][W][3]) for an image of
    tiles_x by tiles_y 16x16-pixel tiles."""
    ns = len(fmt)
    fmt, off = _streams16(fmt, off)
    H, W = 16 * int(tiles_y), 16 * int(tiles_x)
    out = np.empty((H, W, 3), np.float64)
    trans = np.empty((H, W), np.float64)
    bound = np.empty((H, W, 3), np.float64)
    bound_t = np.empty((H, W, 3), np.float64)
    _load().ref_blend_tiles(_p(_c(payload, np.uint8)), _p(_c(fmt, np.uint8)), _p(_c(off, np.uint64)), int(arrangement),
                            ns, _p(_c(vmin, np.float32)), _p(_c(vmax, np.float32)),
                            _p(_c(pos, np.float32).reshape(-1, 3)), _p(_c(perm, np.uint32)),
                            _p(_c(view, np.float32).reshape(3)), _p(_c(mu, np.float32)),
                            _p(_c(foot, np.float32).reshape(-1, 5)), _p(_c(tile_start, np.uint32)),
                            _p(_c(lst, np.uint32)), int(tiles_x), int(tiles_y), _p(out), _p(trans), _p(bound),
                            _p(bound_t))
    return out, trans, bound, bound_t
