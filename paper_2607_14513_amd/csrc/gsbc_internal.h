// gsbc_internal.h -- host-side declarations shared by the library's
// translation units: kernel launchers (one per kernel family) and the
// per-band launch arguments.  Nothing here is part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gsbc.h"

namespace gsbc {

// Kernel timing hooks around each launch; no-ops unless the calling context
// has profiling enabled (see gsbc_profile_enable).
void trace_begin(const char *kernel, hipStream_t st);
void trace_end(hipStream_t st);

// 24-bit multiplies (v_mul_i32_i24 / v_mul_u32_u24, full rate) whatever
// operand ranges the compiler can prove; the result is the low 32 bits of
// the product of the sign- (zero-) extended low 24 bits, so it is exact for
// operands in [-2^23, 2^23) (resp. [0, 2^24)) whose product fits 32 bits.
extern "C" __device__ int gsbc_llvm_mul_i24(int, int) __asm("llvm.amdgcn.mul.i24");
extern "C" __device__ unsigned gsbc_llvm_mul_u24(unsigned, unsigned) __asm("llvm.amdgcn.mul.u24");
__device__ __forceinline__ int mul_i24(int a, int b) { return gsbc_llvm_mul_i24(a, b); }
__device__ __forceinline__ uint32_t mul_u24(uint32_t a, uint32_t b) { return gsbc_llvm_mul_u24(a, b); }

// Add v (one value per lane; lanes with live == false add nothing) into
// sums[band].  Lanes of a wave usually share a band (consecutive blocks):
// then the wave sums in registers and one lane issues the atomic; otherwise
// each lane adds on its own.  Integer sums, so the result is independent of
// the order.
__device__ __forceinline__ void band_add(unsigned long long *sums, uint32_t band, uint32_t v, bool live)
{
    const uint32_t b0 = (uint32_t)__shfl((int)band, __ffsll((unsigned long long)__ballot(live)) - 1);
    const bool uniform = __ballot(live && band != b0) == 0;
    if (uniform) {
        unsigned long long x = live ? v : 0;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off);
        if (live && (__ballot(live) & __lanemask_lt()) == 0) atomicAdd(&sums[band], x);
    } else if (live) {
        atomicAdd(&sums[band], (unsigned long long)v);
    }
}

// Launch `kernel` bracketed by the timing hooks.
#define GSBC_LAUNCH(name, kernel, grid, block, shmem, st, ...)              \
    do {                                                                   \
        ::gsbc::trace_begin(name, st);                                     \
        hipLaunchKernelGGL(kernel, grid, block, shmem, st, __VA_ARGS__);   \
        ::gsbc::trace_end(st);                                             \
    } while (0)

// Workgroup b of a grid of G, as the hardware deals them to the 8 XCDs
// (b mod 8), mapped to a logical block so that each XCD takes one
// contiguous range of blocks in order: neighbouring blocks then share that
// XCD's L2 (rows gathered near each other, partial lines written by two
// neighbours).  A bijection on 0..G-1 for any G.
__device__ __forceinline__ uint32_t xcd_block(uint32_t b, uint32_t G)
{
    const uint32_t x = b & 7u, q = G >> 3, r = G & 7u;
    return x * q + (x < r ? x : r) + (b >> 3);
}

// Per-band stream description passed to kernels by value.
struct BandArgs {
    uint64_t offset[16];   // byte offset of each stream in the payload
    uint32_t format[16];   // per stream: 1 (BC1) or 7 (BC7)
    float vmin[16];        // per band, dequantisation: vmin + q * delta
    float delta[16];       // (vmax - vmin) / 255 in FP32 (the rate controller's gain weight)
    float dhi[16], dlo[16];  // the FP64 step split as dhi + dlo (FP32 each), for dequantising decoded codes
    uint32_t arrangement;  // 0 one stream per band, 1 one primitive per block, 2 four per four blocks
    uint32_t n_streams;    // 16, 1 or 4
};

// Range / scale record produced on the device by the reorder prologue.
struct RangeRec {
    float vmin[16], vmax[16];   // per-band range
    float scale[16];            // 255 / (vmax - vmin), 0 for a constant band
    float lo[3], hi[3];         // position bounding box
    float cell_scale[3];        // 2^g / (hi - lo), 0 for a flat axis
    // the range pass's running extremes (order-preserving integer encodings:
    // [0..15] band min, [16..31] band max, [32..34] position min, [35..37]
    // position max), left at their neutral values between calls
    uint32_t acc[38];
};

// ---- reorder (reorder.hip)
size_t reorder_scratch_bytes(uint64_t n, uint32_t grid_bits);
// identity: keep the input order (perm[s] = s) instead of sorting.
// opacity: null, or per-primitive weights multiplied into every coefficient
// first; quantiser: 0 = per-band min/max range, 1 = symmetric 99.5 % range.
// arrangement: the block packing of the textures (0 bands, 1 one primitive
// per block, 2 four primitives per four blocks).
hipError_t launch_reorder(const float *pos, const float *sh, const float *opacity, uint64_t n, uint32_t grid_bits,
                          uint32_t quantiser, bool identity, uint32_t arrangement, uint32_t *perm, uint8_t *textures,
                          void *scratch, RangeRec *range_dev, RangeRec *host_range, hipStream_t st);

// Variable number of bands: class L (SH degree L, (L+1)^2 bands) owns dense
// slots [slot_start[L], slot_start[L+1]) of perm and padded slots
// [pad_start[L], pad_start[L+1]) (each class padded to a multiple of 16);
// its textures start at word tex_word[L] of the textures buffer.
struct DegreeLayout {
    uint64_t slot_start[5];
    uint64_t pad_start[5];
    uint64_t tex_word[4];
    uint32_t quad1;   // 1: the degree-1 class in Fig. SetupC (one stream, four primitives per block)
};
// Range, keys with the degree class above the cell and colour fields, class
// counts (device uint32[4]) and the sort into perm.
hipError_t launch_degree_sort(const float *pos, const float *sh, const float *opacity, uint64_t n, uint32_t grid_bits,
                              uint32_t quantiser, float tau, uint32_t *perm, void *scratch, RangeRec *range_dev,
                              uint32_t *class_count, hipStream_t st);
hipError_t launch_pack_degrees(const float *sh, const float *opacity, const uint32_t *perm, const DegreeLayout &lay,
                               const RangeRec *range_dev, uint8_t *textures, hipStream_t st);

// ---- encoders (bc1_encode.hip, bc7_encode.hip)
// The encoders work on runs: a run is the consecutive blocks of one band of
// one scene, read from `src` (64-byte RGBA blocks) and written to `dst`
// (8- or 16-byte coded blocks), with their SSE added into *sse (int64
// atomics, order independent).  Runs sit in one global block index space at
// multiples of kRunAlign, so a 256-lane round never straddles two runs;
// indices past a run's end up to the next run are padding and code nothing.
constexpr uint32_t kRunAlign = 256;
struct BlockRun {
    const uint8_t *src;
    uint8_t *dst;
    unsigned long long *sse;        // may be null
    uint64_t gbase;                 // global index of the run's first block
    uint64_t nblk;
};
inline uint64_t run_span(uint64_t nblk) { return (nblk + kRunAlign - 1) / kRunAlign * kRunAlign; }

// Index of the run holding global block g (runs sorted by gbase, g >= run[0].gbase).
__device__ __forceinline__ uint32_t find_run(const BlockRun *run, uint32_t nrun, uint64_t g)
{
    uint32_t lo = 0, hi = nrun;
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (run[mid].gbase <= g) lo = mid;
        else hi = mid;
    }
    return lo;
}

// Work distribution of the encoder kernels: the global index space is cut
// into items of `item_rounds` x 256 blocks.  With queue == null each
// workgroup codes one item (grid = items); otherwise `grid` persistent
// workgroups pop items from *queue (zeroed beforehand) until none are left.
struct WorkSplit {
    uint32_t item_rounds;           // >= 1
    uint32_t grid;                  // persistent workgroups (queue != null)
    uint32_t *queue;                // one counter per kernel launch, or null
};

struct EncodeArgs {
    const BlockRun *run;            // device array
    uint32_t nrun;
    uint64_t total;                 // end of the global index space (multiple of 256)
    uint32_t refine_steps;
    uint32_t mode_mask;
    uint32_t *keys;                 // BC7 only: scratch of bc7_scratch_bytes(total)
};
// Scratch bytes the BC7 encoder needs for `blocks` global indices: a key and
// a bucket-list word per index, plus per-mode counters.
inline size_t bc7_scratch_bytes(uint64_t blocks) { return (size_t)blocks * 8 + 64 + ((blocks + 255) / 256) * 32; }
// How the BC7 candidate search is split over kernels: 0 -> three kernels
// (2-subset, 3-subset, 1-subset modes), 1 -> two (the 1-subset modes folded
// into the 3-subset kernel), 2 -> one kernel for all modes, 3 -> one kernel
// with (group, rounds) work items.  Every split gives the same bits (the
// winner is a minimum over a total order, combined with atomic minima).
hipError_t launch_bc1_encode(const EncodeArgs &a, const WorkSplit &w, uint32_t lanes, hipStream_t st);
// `searched`, when given, is recorded on st once the search kernels are
// enqueued (before the bucketing and emit kernels).
hipError_t launch_bc7_encode(const EncodeArgs &a, const WorkSplit *w3, uint32_t split, hipStream_t st,
                             hipEvent_t searched = nullptr);
hipError_t upload_bc1_tables(int device, hipStream_t st);
hipError_t upload_bc7_tables(int device, hipStream_t st);

// ---- rate control (rate.hip)
// sse1/sse7: [16] int64 band SSEs; writes format[16] and offsets[16] plus the
// payload size into sel (device), then copies the chosen streams from the
// two candidate payloads into `out`.
struct RateSel {
    uint32_t format[16];
    uint64_t offset[16];
    uint64_t payload_bytes;
};
hipError_t launch_rate_select(const unsigned long long *sse1, const unsigned long long *sse7,
                              const BandArgs &b, uint32_t S, uint32_t k, uint64_t nblk, RateSel *sel,
                              hipStream_t st);
// Code histograms of the R, G, B channels of each of the S band streams
// into hist[S][256] (which the caller clears).
hipError_t launch_band_hist(const uint8_t *tex, uint32_t S, uint64_t nblk, unsigned long long *hist, hipStream_t st);
hipError_t launch_rate_select_zero(const unsigned long long *sse1, const unsigned long long *sse7,
                                   const unsigned long long *hist, const BandArgs &b, uint32_t S, uint32_t U,
                                   uint64_t nblk, RateSel *sel, hipStream_t st);
hipError_t launch_copy_streams(const uint8_t *src1, const uint64_t *off1, const uint8_t *src7,
                               const uint64_t *off7, const RateSel *sel, uint32_t S, uint64_t nblk, uint8_t *out,
                               hipStream_t st);
hipError_t launch_fill_u64(unsigned long long *p, uint64_t n, unsigned long long v, hipStream_t st);

// ---- decoders (decode.hip)
hipError_t launch_decode(const uint8_t *blocks, const BandArgs &b, uint64_t nblk,
                         uint8_t *textures, hipStream_t st);
// Slots listed in prim_idx at or beyond n_prims give NaN outputs.
hipError_t launch_decode_eval(const uint8_t *blocks, const BandArgs &b, uint64_t n_prims,
                              const float *dirs, uint32_t n_dirs, const uint32_t *prim_idx,
                              uint64_t m, float *out, float *basis_scratch, hipStream_t st);

// The allocation-free decode_eval's basis scratch: a file-scope device
// array of kStaticScratchDirs x 16 floats in decode.hip.  init_static_scratch
// looks its address up on `device` (which must be current) once; after that
// static_scratch returns it (null before).
constexpr uint32_t kStaticScratchDirs = 1024;
constexpr int kMaxDevices = 64;
hipError_t init_static_scratch(int device);
float *static_scratch(int device);

// One view position: out[j] = colour of slot prim_idx[j] (or j) at the
// direction from its primitive (pos[perm[slot]]) towards `view`.
// Colour stage over per-tile front-to-back lists (Sec. II, eq. preblend);
// order: device scratch of tiles_x * tiles_y words (the tile schedule).
hipError_t launch_blend_tiles(const uint8_t *blocks, const BandArgs &b, uint64_t n_prims, const float *pos,
                              const uint32_t *perm, const float view[3], const float *mu, const float *foot,
                              const uint32_t *tile_start, const uint32_t *list, uint64_t list_len, uint32_t tiles_x,
                              uint32_t tiles_y, const float *colours, float *image, float *trans, uint32_t *order,
                              hipStream_t st);
hipError_t launch_decode_eval_view(const uint8_t *blocks, const BandArgs &b, uint64_t n_prims, const float *pos,
                                   const uint32_t *perm, const float view[3], const uint32_t *prim_idx, uint64_t m,
                                   float *out, hipStream_t st);

}  // namespace gsbc
