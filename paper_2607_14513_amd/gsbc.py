"""ctypes binding of libgsbc.so (include/gsbc.h) over torch device tensors.

Argument marshalling only: every step runs in the library's HIP kernels.
The library must be built (``__graft_entry__.build()`` or
``python paper_2607_14513_amd/csrc/build.py``); importing this module without
it, or calling it without a GPU, raises -- there is no CPU fallback.
"""
import ctypes
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgsbc.so")

OK, E_ARG, E_UNSUPPORTED, E_NOMEM, E_INFEASIBLE, E_DEVICE, E_BUFFER, E_IO = 0, -1, -2, -3, -4, -5, -6, -7
FMT_AUTO, FMT_BC1, FMT_BANDS, FMT_NONE, FMT_AUTO_ZERO, FMT_BC7 = 0, 1, 2, 3, 4, 7
ARR_BANDS, ARR_PRIM, ARR_QUAD = 0, 1, 2
N_STREAMS = {ARR_BANDS: 16, ARR_PRIM: 1, ARR_QUAD: 4}

EXPORTED = ("gsbc_create", "gsbc_destroy", "gsbc_last_error", "gsbc_sync", "gsbc_reserve", "gsbc_arena_info",
            "gsbc_default_params",
            "gsbc_query_sizes", "gsbc_reorder", "gsbc_reorder_desc", "gsbc_reorder_degrees", "gsbc_encode", "gsbc_default_batch_tuning",
            "gsbc_encode_batch", "gsbc_decode", "gsbc_decode_eval", "gsbc_decode_eval_noalloc", "gsbc_decode_eval_view", "gsbc_blend_tiles", "gsbc_blend_tiles_colours",
            "gsbc_save", "gsbc_load",
            "gsbc_profile_enable", "gsbc_profile_read")


class GsbcError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"gsbc status {status}: {msg}")
        self.status = status


class Params(ctypes.Structure):
    _fields_ = [("grid_bits", ctypes.c_uint32), ("refine_steps", ctypes.c_uint32),
                ("bc7_mode_mask", ctypes.c_uint32), ("order", ctypes.c_uint32),
                ("arrangement", ctypes.c_uint32), ("quantiser", ctypes.c_uint32)]


class BatchTuning(ctypes.Structure):
    _fields_ = [("item_rounds", ctypes.c_uint32), ("wgs_per_cu", ctypes.c_uint32),
                ("bc1_lanes", ctypes.c_uint32), ("bc7_split", ctypes.c_uint32),
                ("concurrent", ctypes.c_uint32)]

    def as_dict(self):
        return {f: int(getattr(self, f)) for f, _ in self._fields_}


class StreamDesc(ctypes.Structure):
    _fields_ = [("format", ctypes.c_uint8 * 16), ("offset", ctypes.c_uint64 * 16),
                ("vmin", ctypes.c_float * 16), ("vmax", ctypes.c_float * 16),
                ("n_prims", ctypes.c_uint64), ("n_pad", ctypes.c_uint64),
                ("blocks_per_stream", ctypes.c_uint64), ("payload_bytes", ctypes.c_uint64),
                ("arrangement", ctypes.c_uint32), ("n_streams", ctypes.c_uint32)]

    def formats(self):
        """Per-stream formats (n_streams entries)."""
        return np.array(list(self.format)[:self.n_streams], np.uint8)

    def offsets(self):
        """Per-stream payload offsets (n_streams entries)."""
        return np.array(list(self.offset)[:self.n_streams], np.uint64)

    def ranges(self):
        return np.array(list(self.vmin), np.float32), np.array(list(self.vmax), np.float32)

    def copy(self):
        d = StreamDesc()
        ctypes.memmove(ctypes.byref(d), ctypes.byref(self), ctypes.sizeof(StreamDesc))
        return d


_lib = None


def load():
    """Load libgsbc.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        lib = ctypes.CDLL(LIB_PATH)
        P, u64, u32, i32 = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int32
        lib.gsbc_create.argtypes = [ctypes.POINTER(P), ctypes.c_int, P]
        lib.gsbc_destroy.argtypes = [P]
        lib.gsbc_last_error.argtypes = [P]
        lib.gsbc_last_error.restype = ctypes.c_char_p
        lib.gsbc_sync.argtypes = [P]
        lib.gsbc_reserve.argtypes = [P, u64, u32]
        lib.gsbc_arena_info.argtypes = [P, ctypes.POINTER(u64), ctypes.POINTER(u64)]
        lib.gsbc_default_params.argtypes = [ctypes.POINTER(Params)]
        lib.gsbc_default_params.restype = None
        lib.gsbc_query_sizes.argtypes = [u64, u32, ctypes.POINTER(u64), ctypes.POINTER(u64), ctypes.POINTER(u64)]
        lib.gsbc_reorder.argtypes = [P, P, P, P, u64, ctypes.POINTER(Params), P, P, ctypes.POINTER(StreamDesc)]
        lib.gsbc_reorder_desc.argtypes = [P, ctypes.POINTER(StreamDesc)]
        lib.gsbc_reorder_degrees.argtypes = [P, P, P, P, u64, ctypes.c_float, ctypes.POINTER(Params), P, P, u64,
                                             ctypes.POINTER(u64), ctypes.POINTER(u64), ctypes.POINTER(StreamDesc)]
        lib.gsbc_encode.argtypes = [P, P, ctypes.POINTER(StreamDesc), ctypes.c_int, ctypes.c_double,
                                    ctypes.POINTER(Params), P, u64, P]
        lib.gsbc_default_batch_tuning.argtypes = [ctypes.POINTER(BatchTuning)]
        lib.gsbc_default_batch_tuning.restype = None
        lib.gsbc_encode_batch.argtypes = [P, u32, P, P, P, P, ctypes.POINTER(Params),
                                          ctypes.POINTER(BatchTuning), P]
        lib.gsbc_decode.argtypes = [P, P, ctypes.POINTER(StreamDesc), P]
        lib.gsbc_decode_eval.argtypes = [P, P, ctypes.POINTER(StreamDesc), P, u32, P, u64, P]
        lib.gsbc_decode_eval_noalloc.argtypes = [P, P, ctypes.POINTER(StreamDesc), P, u32, P, u64, P]
        lib.gsbc_decode_eval_view.argtypes = [P, P, ctypes.POINTER(StreamDesc), P, P, P, P, u64, P]
        lib.gsbc_blend_tiles.argtypes = [P, P, ctypes.POINTER(StreamDesc), P, P, P, P, P, P, P, u64, u32, u32, P, P]
        lib.gsbc_blend_tiles_colours.argtypes = [P, P, u64, P, P, P, P, P, u64, u32, u32, P, P]
        lib.gsbc_save.argtypes = [P, P, ctypes.POINTER(StreamDesc), ctypes.c_char_p]
        lib.gsbc_load.argtypes = [P, ctypes.c_char_p, ctypes.POINTER(StreamDesc), P, u64]
        lib.gsbc_profile_enable.argtypes = [P, ctypes.c_int]
        lib.gsbc_profile_read.argtypes = [P, u32, P, P, P, ctypes.POINTER(u32)]
        for name in EXPORTED:
            if name not in ("gsbc_default_params", "gsbc_last_error", "gsbc_default_batch_tuning"):
                getattr(lib, name).restype = i32
        _lib = lib
    return _lib


def default_params(**kw):
    p = Params()
    load().gsbc_default_params(ctypes.byref(p))
    for k, v in kw.items():
        if k not in dict(Params._fields_):
            raise TypeError(f"unknown parameter {k!r}")
        setattr(p, k, int(v))
    return p


def default_batch_tuning(**kw):
    t = BatchTuning()
    load().gsbc_default_batch_tuning(ctypes.byref(t))
    for k, v in kw.items():
        setattr(t, k, int(v))
    return t


def query_sizes(n, n_dirs=0):
    t, b, o = ctypes.c_uint64(), ctypes.c_uint64(), ctypes.c_uint64()
    st = load().gsbc_query_sizes(int(n), int(n_dirs), ctypes.byref(t), ctypes.byref(b), ctypes.byref(o))
    if st != OK:
        raise GsbcError(st, "query_sizes")
    return t.value, b.value, o.value


def load_header(path):
    """StreamDesc of a container file (host only, no device needed)."""
    d = StreamDesc()
    st = load().gsbc_load(None, os.fsencode(path), ctypes.byref(d), None, 0)
    if st != OK:
        raise GsbcError(st, f"cannot read container {path}")
    return d


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _check(t, dtype, name, shape=None, min_numel=None):
    """Type, layout and size of a tensor argument, checked on the host before
    anything reaches the library: the C ABI takes bare pointers, so a tensor
    too small for what the descriptor or the counts say would be read or
    written past its end by the kernels."""
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.dtype != dtype or not t.is_contiguous():
        raise TypeError(f"{name} must be a contiguous {dtype} tensor")
    if shape is not None and tuple(t.shape) != tuple(int(x) for x in shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(int(x) for x in shape)}")
    if min_numel is not None and t.numel() < int(min_numel):
        raise ValueError(f"{name} holds {t.numel()} elements, needs at least {int(min_numel)}")
    return t


def _on_device(*named):
    for name, t in named:
        if t is not None and not t.is_cuda:
            raise TypeError(f"{name} must be a device tensor")


def _dev_tensor(t, dtype, name, shape=None, min_numel=None):
    _check(t, dtype, name, shape, min_numel)
    _on_device((name, t))
    return t


def _desc_numbers(desc):
    """(n_streams, blocks_per_stream, payload_bytes, n_prims) of a descriptor
    whose sizes agree with each other, else None: the library rejects such a
    descriptor itself (GSBC_E_ARG) before anything is enqueued, so sizes
    derived from it are not checked here."""
    if not isinstance(desc, StreamDesc):
        raise TypeError("desc must be a StreamDesc")
    S, nblk, n, npad = int(desc.n_streams), int(desc.blocks_per_stream), int(desc.n_prims), int(desc.n_pad)
    arr = int(desc.arrangement)
    allowed = {ARR_BANDS: (1, 4, 9, 16), ARR_PRIM: (1,), ARR_QUAD: (1, 4)}.get(arr, ())
    per_block = {ARR_BANDS: 16, ARR_PRIM: 1, ARR_QUAD: 4}.get(arr, 0)
    if S not in allowed or n < 1 or npad != (n + 15) // 16 * 16 or nblk * N_STREAMS[arr] != npad or per_block == 0:
        return None
    return S, nblk, int(desc.payload_bytes), n


def _sizes(desc):
    """Expected sizes of a consistent descriptor, or a tuple of None."""
    r = _desc_numbers(desc)
    return r if r is not None else (None, None, None, None)


class Context:
    """One library context: device, stream (torch's current stream by default)
    and scratch arena."""

    def __init__(self, device=0, stream=None):
        lib = load()
        if not torch.cuda.is_available():
            raise RuntimeError("no HIP device: the library has no CPU path")
        self.device = torch.device("cuda", device)
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        self.stream = stream
        h = ctypes.c_void_p()
        st = lib.gsbc_create(ctypes.byref(h), int(device), ctypes.c_void_p(stream.cuda_stream))
        if st != OK:
            raise GsbcError(st, "gsbc_create failed")
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            load().gsbc_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def _check(self, st):
        if st != OK:
            raise GsbcError(st, load().gsbc_last_error(self._h).decode())

    def sync(self):
        self._check(load().gsbc_sync(self._h))

    def reserve(self, n_max, n_dirs_max=0):
        """Size the scratch arena once for scenes of up to n_max primitives and
        decode_evals of up to n_dirs_max directions."""
        self._check(load().gsbc_reserve(self._h, int(n_max), int(n_dirs_max)))

    def arena_info(self):
        """(arena bytes, times it has grown)."""
        b, g = ctypes.c_uint64(), ctypes.c_uint64()
        self._check(load().gsbc_arena_info(self._h, ctypes.byref(b), ctypes.byref(g)))
        return b.value, g.value

    def profile(self, on=True):
        """Bracket every kernel launch with HIP events on the context's stream."""
        self._check(load().gsbc_profile_enable(self._h, 1 if on else 0))

    def profile_read(self, max_entries=64):
        """{kernel name: (launches, total ms)} since the previous read."""
        names = ctypes.create_string_buffer(64 * max_entries)
        counts = (ctypes.c_uint32 * max_entries)()
        ms = (ctypes.c_double * max_entries)()
        n = ctypes.c_uint32()
        self._check(load().gsbc_profile_read(self._h, max_entries, names, counts, ms, ctypes.byref(n)))
        out = {}
        for q in range(n.value):
            name = names.raw[64 * q:64 * q + 64].split(b"\0")[0].decode()
            out[name] = (int(counts[q]), float(ms[q]))
        return out

    # ------------------------------------------------------------- calls
    def reorder(self, pos, sh, params=None, out=None, opacity=None, want_desc=True):
        """pos float32[n][3], sh float32[n][16][3], opacity float32[n] or None
        on the device -> (perm uint32-as-int32[n], textures uint8[16][nblk][16][4], desc).
        want_desc False: only enqueue (no wait; desc None, see reorder_desc)."""
        _check(pos, torch.float32, "pos")
        n = pos.shape[0] if pos.dim() == 2 else -1
        _check(pos, torch.float32, "pos", shape=(n, 3))
        _check(sh, torch.float32, "sh", shape=(n, 16, 3))
        if opacity is not None:
            _check(opacity, torch.float32, "opacity", shape=(n,))
        p = params if params is not None else default_params()
        S = N_STREAMS.get(int(p.arrangement), 16)
        npad = (n + 15) // 16 * 16
        if out is None:
            perm = torch.empty(n, dtype=torch.int32, device=self.device)
            tex = torch.empty((S, npad // S, 16, 4), dtype=torch.uint8, device=self.device)
        else:
            perm, tex = out
            _check(perm, torch.int32, "perm", shape=(n,))
            _check(tex, torch.uint8, "textures", min_numel=npad * 64)
        _on_device(("pos", pos), ("sh", sh), ("opacity", opacity), ("perm", perm), ("textures", tex))
        desc = StreamDesc() if want_desc else None
        self._check(load().gsbc_reorder(self._h, _ptr(pos), _ptr(sh),
                                        _ptr(opacity) if opacity is not None else None, n, ctypes.byref(p), _ptr(perm),
                                        _ptr(tex), ctypes.byref(desc) if want_desc else None))
        return perm, tex, desc

    def reorder_desc(self):
        """The desc of the last reorder (waits for the stream)."""
        desc = StreamDesc()
        self._check(load().gsbc_reorder_desc(self._h, ctypes.byref(desc)))
        return desc

    def reorder_degrees(self, pos, sh, tau=0.0, params=None, opacity=None):
        """Degree classes (variable number of bands).  Returns (perm int32[n],
        counts[4], textures: list of 4 device uint8 views [S][blocks][16][4]
        ([(L+1)^2][pad16/16] per band, or [1][pad16/4] for the degree-1 class
        in Fig. SetupC when params.arrangement is ARR_QUAD) or None for an
        empty class, descs: list of 4 StreamDesc)."""
        _check(pos, torch.float32, "pos")
        n = pos.shape[0] if pos.dim() == 2 else -1
        _check(pos, torch.float32, "pos", shape=(n, 3))
        _check(sh, torch.float32, "sh", shape=(n, 16, 3))
        if opacity is not None:
            _check(opacity, torch.float32, "opacity", shape=(n,))
        _on_device(("pos", pos), ("sh", sh), ("opacity", opacity))
        p = params if params is not None else default_params()
        cap = (n + 15) // 16 * 16 * 64 + 1800
        buf = torch.empty(cap, dtype=torch.uint8, device=self.device)
        perm = torch.empty(n, dtype=torch.int32, device=self.device)
        counts = (ctypes.c_uint64 * 4)()
        offs = (ctypes.c_uint64 * 4)()
        descs = (StreamDesc * 4)()
        self._check(load().gsbc_reorder_degrees(self._h, _ptr(pos), _ptr(sh),
                                                _ptr(opacity) if opacity is not None else None, n, float(tau),
                                                ctypes.byref(p), _ptr(perm), _ptr(buf), cap, counts, offs, descs))
        tex = []
        for L in range(4):
            c = int(counts[L])
            if c == 0:
                tex.append(None)
                continue
            d = descs[L]
            nb, nblk = int(d.n_streams), int(d.blocks_per_stream)
            o = int(offs[L])
            tex.append(buf[o:o + nb * nblk * 64].view(nb, nblk, 16, 4))
        return perm, [int(c) for c in counts], tex, [descs[L] for L in range(4)]

    def encode(self, textures, desc, fmt=FMT_AUTO, rate=6.0, params=None, blocks=None, want_sse=False):
        """Encode all streams -> (blocks uint8 device tensor, desc, band_sse int64[2][16] or None).
        fmt FMT_BANDS codes stream k in desc.format[k] (set by the caller:
        FMT_BC1, FMT_BC7 or, for band streams, FMT_NONE); FMT_AUTO and
        FMT_AUTO_ZERO choose per band at `rate` bits per texel."""
        S, nblk, _, _ = _sizes(desc)
        _check(textures, torch.uint8, "textures", min_numel=S * nblk * 64 if S else None)
        desc = desc.copy()
        if blocks is None:
            _, cap, _ = query_sizes(desc.n_prims)
            blocks = torch.empty(cap, dtype=torch.uint8, device=self.device)
        _check(blocks, torch.uint8, "blocks")
        _on_device(("textures", textures), ("blocks", blocks))
        sse = np.zeros(32, np.int64) if want_sse else None
        p = params if params is not None else default_params()
        self._check(load().gsbc_encode(self._h, _ptr(textures), ctypes.byref(desc), int(fmt), float(rate),
                                       ctypes.byref(p), _ptr(blocks), blocks.numel(),
                                       ctypes.c_void_p(sse.ctypes.data) if sse is not None else None))
        return blocks, desc, (sse.reshape(2, 16) if sse is not None else None)

    def encode_batch(self, textures, descs, blocks, params=None, tuning=None, want_sse=False):
        """textures: list of device uint8 tensors (reorder layout); descs: list
        of StreamDesc with format[16] set (each BC1, BC7 or NONE); blocks: list of
        device uint8 tensors.  Returns (descs filled, band_sse int64[n][16] or
        None).  Without want_sse the call returns once the graph is queued."""
        n = len(textures)
        if not (n == len(descs) == len(blocks)):
            raise ValueError("textures, descs and blocks differ in length")
        for i, t in enumerate(textures):
            S, nblk, _, _ = _sizes(descs[i])
            _dev_tensor(t, torch.uint8, f"textures[{i}]", min_numel=S * nblk * 64 if S else None)
            _dev_tensor(blocks[i], torch.uint8, f"blocks[{i}]")
        tp = (ctypes.c_void_p * n)(*[t.data_ptr() for t in textures])
        bp = (ctypes.c_void_p * n)(*[b.data_ptr() for b in blocks])
        cap = (ctypes.c_uint64 * n)(*[b.numel() for b in blocks])
        darr = (StreamDesc * n)()
        for i, d in enumerate(descs):
            ctypes.memmove(ctypes.byref(darr[i]), ctypes.byref(d), ctypes.sizeof(StreamDesc))
        sse = np.zeros(16 * n, np.int64) if want_sse else None
        p = params if params is not None else default_params()
        t = tuning if tuning is not None else default_batch_tuning()
        self._check(load().gsbc_encode_batch(self._h, n, tp, darr, bp, cap, ctypes.byref(p), ctypes.byref(t),
                                             ctypes.c_void_p(sse.ctypes.data) if sse is not None else None))
        out = [darr[i].copy() for i in range(n)]
        return out, (sse.reshape(n, 16) if sse is not None else None)

    def decode_eval_view(self, blocks, desc, pos, perm, view, prim_idx=None, out=None):
        """pos float32[N][3] (the scene in input order) and perm int32[n_prims]
        on the device (every perm value below N), view 3 floats (host) ->
        out float32[m][3]: each slot's colour seen from view."""
        _, _, payload, n = _sizes(desc)
        _check(blocks, torch.uint8, "blocks", min_numel=payload)
        # pos holds the whole scene in input order (a degree class reads
        # the rows its perm names), so it is at least as long as the slots
        _check(pos, torch.float32, "pos")
        if pos.dim() != 2 or pos.shape[1] != 3 or (n and pos.shape[0] < n):
            raise ValueError(f"pos has shape {tuple(pos.shape)}, expected (N, 3) with N >= {n}")
        _check(perm, torch.int32, "perm", shape=(n,) if n else None)
        m = int(desc.n_prims) if prim_idx is None else prim_idx.numel()
        if prim_idx is not None:
            _check(prim_idx, torch.int32, "prim_idx", shape=(m,))
        if out is None:
            out = torch.empty((m, 3), dtype=torch.float32, device=self.device)
        _check(out, torch.float32, "out", shape=(m, 3))
        _on_device(("blocks", blocks), ("pos", pos), ("perm", perm), ("prim_idx", prim_idx), ("out", out))
        f = (ctypes.c_float * 3)(*[float(x) for x in view])
        self._check(load().gsbc_decode_eval_view(self._h, _ptr(blocks), ctypes.byref(desc), _ptr(pos), _ptr(perm), f,
                                                 _ptr(prim_idx), m, _ptr(out)))
        return out

    def blend_tiles(self, blocks, desc, pos, perm, view, opacity, footprint, tile_start, lst, tiles_x, tiles_y,
                    image=None, transmittance=None, want_transmittance=True):
        """The colour stage over per-tile front-to-back lists (device tensors:
        pos float32[N][3], perm int32[n_prims], opacity float32[N],
        footprint float32[N][5], tile_start int32[tiles + 1], lst int32[L]
        of sorted-slot ids; view 3 host floats) -> (image float32[H][W][3],
        transmittance float32[H][W] or None)."""
        _, _, payload, n = _sizes(desc)
        _check(blocks, torch.uint8, "blocks", min_numel=payload)
        _check(pos, torch.float32, "pos")
        if pos.dim() != 2 or pos.shape[1] != 3 or (n and pos.shape[0] < n):
            raise ValueError(f"pos has shape {tuple(pos.shape)}, expected (N, 3) with N >= {n}")
        N = pos.shape[0]
        _check(perm, torch.int32, "perm", shape=(n,) if n else None)
        _check(opacity, torch.float32, "opacity", shape=(N,))
        _check(footprint, torch.float32, "footprint", shape=(N, 5))
        tiles = int(tiles_x) * int(tiles_y)
        _check(tile_start, torch.int32, "tile_start", shape=(tiles + 1,))
        _check(lst, torch.int32, "lst")
        H, W = 16 * int(tiles_y), 16 * int(tiles_x)
        if image is None:
            image = torch.empty((H, W, 3), dtype=torch.float32, device=self.device)
        _check(image, torch.float32, "image", shape=(H, W, 3))
        if transmittance is None and want_transmittance:
            transmittance = torch.empty((H, W), dtype=torch.float32, device=self.device)
        if transmittance is not None:
            _check(transmittance, torch.float32, "transmittance", shape=(H, W))
        _on_device(("blocks", blocks), ("pos", pos), ("perm", perm), ("opacity", opacity), ("footprint", footprint),
                   ("tile_start", tile_start), ("lst", lst), ("image", image), ("transmittance", transmittance))
        f = (ctypes.c_float * 3)(*[float(x) for x in view])
        self._check(load().gsbc_blend_tiles(self._h, _ptr(blocks), ctypes.byref(desc), _ptr(pos), _ptr(perm), f,
                                            _ptr(opacity), _ptr(footprint), _ptr(tile_start), _ptr(lst), lst.numel(),
                                            int(tiles_x), int(tiles_y), _ptr(image), _ptr(transmittance)))
        return image, transmittance

    def blend_tiles_colours(self, colours, perm, opacity, footprint, tile_start, lst, tiles_x, tiles_y,
                            image=None, transmittance=None, want_transmittance=True):
        """The colour stage with the colours computed beforehand (colours
        float32[n_prims][3] per slot, e.g. decode_eval_view over all slots);
        other arguments and the result as blend_tiles (perm from reorder:
        every value below N, the length of opacity and footprint)."""
        _check(colours, torch.float32, "colours")
        if colours.dim() != 2 or colours.shape[1] != 3:
            raise ValueError(f"colours has shape {tuple(colours.shape)}, expected (n_prims, 3)")
        n = colours.shape[0]
        _check(perm, torch.int32, "perm", shape=(n,))
        _check(opacity, torch.float32, "opacity")
        N = opacity.shape[0] if opacity.dim() == 1 else -1
        _check(opacity, torch.float32, "opacity", shape=(N,))
        _check(footprint, torch.float32, "footprint", shape=(N, 5))
        tiles = int(tiles_x) * int(tiles_y)
        _check(tile_start, torch.int32, "tile_start", shape=(tiles + 1,))
        _check(lst, torch.int32, "lst")
        H, W = 16 * int(tiles_y), 16 * int(tiles_x)
        if image is None:
            image = torch.empty((H, W, 3), dtype=torch.float32, device=self.device)
        _check(image, torch.float32, "image", shape=(H, W, 3))
        if transmittance is None and want_transmittance:
            transmittance = torch.empty((H, W), dtype=torch.float32, device=self.device)
        if transmittance is not None:
            _check(transmittance, torch.float32, "transmittance", shape=(H, W))
        _on_device(("colours", colours), ("perm", perm), ("opacity", opacity), ("footprint", footprint),
                   ("tile_start", tile_start), ("lst", lst), ("image", image), ("transmittance", transmittance))
        self._check(load().gsbc_blend_tiles_colours(self._h, _ptr(colours), n, _ptr(perm), _ptr(opacity),
                                                    _ptr(footprint), _ptr(tile_start), _ptr(lst), lst.numel(),
                                                    int(tiles_x), int(tiles_y), _ptr(image), _ptr(transmittance)))
        return image, transmittance

    def save(self, path, blocks, desc):
        """Write the coded scene (device blocks + desc) as a container file."""
        _dev_tensor(blocks, torch.uint8, "blocks", min_numel=_sizes(desc)[2])
        self._check(load().gsbc_save(self._h, _ptr(blocks), ctypes.byref(desc), os.fsencode(path)))

    def load(self, path):
        """Read a container file -> (device blocks tensor, desc)."""
        d = load_header(path)
        blocks = torch.empty(d.payload_bytes, dtype=torch.uint8, device=self.device)
        self._check(load().gsbc_load(self._h, os.fsencode(path), ctypes.byref(d), _ptr(blocks), blocks.numel()))
        return blocks, d

    def decode(self, blocks, desc, out=None):
        """blocks (device payload) -> textures uint8[n_streams][blocks_per_stream][16][4]."""
        S, nblk, payload, _ = _sizes(desc)
        _check(blocks, torch.uint8, "blocks", min_numel=payload)
        if out is None:
            out = torch.empty((int(desc.n_streams), int(desc.blocks_per_stream), 16, 4), dtype=torch.uint8,
                              device=self.device)
        _check(out, torch.uint8, "out", shape=(S, nblk, 16, 4) if S else None)
        _on_device(("blocks", blocks), ("out", out))
        self._check(load().gsbc_decode(self._h, _ptr(blocks), ctypes.byref(desc), _ptr(out)))
        return out

    def decode_eval(self, blocks, desc, dirs, prim_idx=None, out=None, noalloc=False):
        """dirs float32[V][3] device; prim_idx int32[m] sorted-slot ids or None
        -> out float32[V][m][3].  noalloc: through gsbc_decode_eval_noalloc
        (the library allocates nothing; V <= 1024; out must then be given by
        a caller that cannot allocate, though one is made here if not)."""
        _, _, payload, n = _sizes(desc)
        _check(blocks, torch.uint8, "blocks", min_numel=payload)
        _check(dirs, torch.float32, "dirs")
        V = dirs.shape[0] if dirs.dim() == 2 else -1
        _check(dirs, torch.float32, "dirs", shape=(V, 3))
        m = int(desc.n_prims) if prim_idx is None else prim_idx.numel()
        if prim_idx is not None:
            _check(prim_idx, torch.int32, "prim_idx", shape=(m,))
        if out is None:
            out = torch.empty((V, m, 3), dtype=torch.float32, device=self.device)
        _check(out, torch.float32, "out", shape=(V, m, 3))
        _on_device(("blocks", blocks), ("dirs", dirs), ("prim_idx", prim_idx), ("out", out))
        fn = load().gsbc_decode_eval_noalloc if noalloc else load().gsbc_decode_eval
        self._check(fn(self._h, _ptr(blocks), ctypes.byref(desc), _ptr(dirs), V, _ptr(prim_idx), m, _ptr(out)))
        return out
