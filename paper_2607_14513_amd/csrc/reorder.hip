// reorder.hip -- colour/space reorder and block packing on gfx950.
//
//   range    per-band min/max of the SH coefficients and the position
//            bounding box (Sec. V-A quantiser range; Sec. III-C spatial
//            groups), one coalesced float4 pass with order-independent
//            integer atomics on an order-preserving encoding of the floats;
//   keys     (Morton cell of the position) << 24 | RGB bit interleave of the
//            quantised band-0 colour (Sec. III-C, Fig. Bit4Scan);
//   sort     stable LSD radix sort over digits of 8 or 9 bits, reduce then
//            scan: per pass, each 4,096-key tile's digit counts, their
//            exclusive scan over tiles per digit, then the scatter, where
//            each workgroup ranks its tile stably (per-wave LDS lane masks
//            of equal digits, waves in order), sorts it in LDS and writes
//            each digit's keys as one contiguous run; the digit totals of
//            every pass and the first pass's tile counts come from the
//            histogram taken while the keys are made;
//   pack     gather each slot's 48 coefficients, quantise, and write band k
//            of slot s to texel zigzag(s % 16) of block s / 16 (Fig. SetupD,
//            Fig. ZigZagScan).
#include "gsbc_internal.h"

#include <algorithm>

namespace gsbc {
namespace {

constexpr int kSortKPT = 16;                   // keys per thread of a sort tile
constexpr int kSortTile = 256 * kSortKPT;      // keys per tile (one workgroup)
constexpr int kMaxDigitBits = 9;
constexpr int kMaxBins = 1 << kMaxDigitBits;
constexpr int kMaxPasses = 7;                  // 56-bit keys (grid 10 bits, degree class) in 9-bit digits
constexpr int kRangeBlock = 384;               // coverage histogram block: a multiple of 12 and 3
constexpr int kMinMaxBlock = 768;              // min/max pass block (measured faster than 384 or 192)
static_assert(kRangeBlock % 12 == 0, "a block-size run of float4 chunks must hold whole primitives");

// Digits of each pass, low to high: ceil(bits / 9) passes of near-equal width.
struct SortPlan {
    int passes;
    int shift[kMaxPasses], bits[kMaxPasses];
};

SortPlan plan_sort(int key_bits)
{
    SortPlan P{};
    P.passes = (key_bits + kMaxDigitBits - 1) / kMaxDigitBits;
    int at = 0;
    for (int p = 0; p < P.passes; p++) {
        const int w = (key_bits - at) / (P.passes - p);   // remaining bits spread over the remaining passes
        P.shift[p] = at;
        P.bits[p] = w + ((key_bits - at) % (P.passes - p) ? 1 : 0);
        at += P.bits[p];
    }
    return P;
}

__device__ __forceinline__ uint32_t ord_of(float f)
{
    uint32_t u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float float_of(uint32_t u)
{
    return __uint_as_float((u & 0x80000000u) ? (u & 0x7FFFFFFFu) : ~u);
}

// Spread the low 10 bits of x to every third bit.
__device__ __forceinline__ uint32_t spread3(uint32_t x)
{
    x &= 0x3FF;
    x = (x | (x << 16)) & 0x030000FF;
    x = (x | (x << 8)) & 0x0300F00F;
    x = (x | (x << 4)) & 0x030C30C3;
    x = (x | (x << 2)) & 0x09249249;
    return x;
}

// 8-bit code of coefficient x in a band with range start vmin and scale s.
__device__ __forceinline__ uint32_t quant8(float x, float vmin, float s)
{
    float t = x - vmin;
    float u = t * s;
    int v = (int)rintf(u);
    v = v < 0 ? 0 : v;
    v = v > 255 ? 255 : v;
    return (uint32_t)v;
}

// acc (RangeRec::acc) layout: [0..15] band min, [16..31] band max, [32..34]
// pos min, [35..37] pos max.  It is neutral when a call starts (set so when
// the context is made, and put back by k_range_final once read).
constexpr int kAccWords = 38;
__device__ __forceinline__ bool acc_is_min(int i) { return i < 16 || (i >= 32 && i < 35); }

// dc: each primitive's band-0 colour (times its opacity), three floats,
// for the key pass.  Workgroup 0 also clears the sort's digit totals.
// Every wave streams one contiguous run of primitives (a multiple of
// kStepPrims = 32), a step at a time: the step's 384 float4
// chunks (six loads per lane) and 96 position floats (two), all in flight
// together, with no workgroup barrier.  Chunk u * 64 + lane of a step sits
// at place (lane + 4u) mod 12 of its primitive, one of three places per
// lane, whose extremes are kept apart and folded into bands at the end;
// position float x of a step is on axis x mod 3.  The step's band-0 colours
// go through the wave's own LDS and leave as two contiguous stores, issued
// before the next step's loads (so waiting on those never waits on a newer
// store).  DEG: also deg, each primitive's degree class: the
// largest SH degree l in 1..3 with a coefficient (after the opacity) above
// tau in magnitude in a band of degree l, else 0; per chunk a 3-bit mask of
// the degrees it shows, combined per primitive through the same LDS.
constexpr uint32_t kStepPrims = 32, kStepChunks = kStepPrims * 12, kStepLoads = kStepChunks / 64;
static_assert(kStepChunks % 64 == 0 && kMinMaxBlock % 64 == 0, "whole loads per lane and step");
typedef float f32x4 __attribute__((ext_vector_type(4)));
// SH rows above this many bytes are read by the range pass with
// non-temporal loads: MI355X's last-level (Infinity) cache holds 256 MiB.
// A scene that fits keeps its rows cached for the gather, which reads them
// again in key order; a larger one would only evict its own rows (3,145,728
// primitives: range pass 0.130 -> 0.104 ms; at 1,048,576 the cached rows
// save the gather 0.005 ms).
constexpr uint64_t kStreamRowBytes = 256ull << 20;
template <bool DEG>
__global__ __launch_bounds__(kMinMaxBlock) void k_range_partial(const float4 *sh4, const float *opacity,
                                                                const float *pos, uint64_t n, uint32_t *acc,
                                                                float *dc, uint32_t *meta, uint32_t meta_words,
                                                                float tau, uint8_t *deg, bool stream)
{
    __shared__ uint32_t s_acc[kAccWords];
    __shared__ float stage[kMinMaxBlock / 64][kStepPrims * 3];
    __shared__ uint8_t s_deg[DEG ? kMinMaxBlock / 64 : 1][kStepChunks];   // degree masks of the step's chunks
    const uint32_t tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    if (tid < kAccWords) s_acc[tid] = acc_is_min((int)tid) ? 0xFFFFFFFFu : 0u;
    if (blockIdx.x == 0)   // the sort's digit totals, for the key pass that follows
        for (uint32_t e = tid; e < meta_words; e += kMinMaxBlock) meta[e] = 0u;
    __syncthreads();
    const uint64_t waves = (uint64_t)gridDim.x * (kMinMaxBlock / 64), wg = (uint64_t)blockIdx.x * (kMinMaxBlock / 64) + wv;
    float mn[3][4], mx[3][4];
#pragma unroll
    for (int k = 0; k < 3; k++)
#pragma unroll
        for (int c = 0; c < 4; c++) { mn[k][c] = INFINITY; mx[k][c] = -INFINITY; }
    auto take = [&](float4 &v, int k, uint64_t q) {
        if (opacity) {   // H~ = mu H (FP32 products)
            const float mu = opacity[q / 12];
            v.x *= mu; v.y *= mu; v.z *= mu; v.w *= mu;
        }
        mn[k][0] = fminf(mn[k][0], v.x); mx[k][0] = fmaxf(mx[k][0], v.x);
        mn[k][1] = fminf(mn[k][1], v.y); mx[k][1] = fmaxf(mx[k][1], v.y);
        mn[k][2] = fminf(mn[k][2], v.z); mx[k][2] = fmaxf(mx[k][2], v.z);
        mn[k][3] = fminf(mn[k][3], v.w); mx[k][3] = fmaxf(mx[k][3], v.w);
    };
    float pmn[3], pmx[3];   // positions: extremes of axis (lane + k) mod 3
#pragma unroll
    for (int k = 0; k < 3; k++) { pmn[k] = INFINITY; pmx[k] = -INFINITY; }
    auto take_pos = [&](float a, int k) {
        pmn[k] = fminf(pmn[k], a);
        pmx[k] = fmaxf(pmx[k], a);
    };
    float *st = stage[wv];
    uint8_t *sd = s_deg[DEG ? wv : 0];
    // degrees (bits l - 1) shown by chunk place j's four floats 4j..4j+3
    auto degree_mask = [&](const float4 &v, int j) {
        const float f[4] = {v.x, v.y, v.z, v.w};
        uint32_t m = 0;
#pragma unroll
        for (int c = 0; c < 4; c++) {
            const int band = (4 * j + c) / 3, l = band >= 9 ? 3 : band >= 4 ? 2 : band >= 1 ? 1 : 0;
            if (l && fabsf(f[c]) > tau) m |= 1u << (l - 1);
        }
        return m;
    };
    // lanes m < count: the class of the step's primitive m from its 12 chunks' masks
    auto store_degrees = [&](uint64_t prim0, uint32_t count) {
        if (lane < count) {
            uint32_t m = 0;
#pragma unroll
            for (int i = 0; i < 12; i++) m |= sd[12 * lane + i];
            deg[prim0 + lane] = (uint8_t)(m ? 32 - __clz(m) : 0);
        }
    };
    {
        const uint64_t nq = n * 12;
        const uint64_t span = ((nq + waves - 1) / waves + kStepChunks - 1) / kStepChunks * kStepChunks;
        const uint64_t q0 = wg * span, q1 = min(nq, q0 + span);
        const uint64_t steps = q1 > q0 ? (q1 - q0) / kStepChunks : 0;
        uint64_t q = q0;   // first chunk of the step
        for (uint64_t k = 0; k < steps; k++, q += kStepChunks) {
            float4 v[kStepLoads];
            if (stream) {   // rows past the last-level cache: non-temporal loads
#pragma unroll
                for (int u = 0; u < (int)kStepLoads; u++) {
                    const f32x4 x = __builtin_nontemporal_load(reinterpret_cast<const f32x4 *>(sh4) + q + u * 64 + lane);
                    v[u] = make_float4(x.x, x.y, x.z, x.w);
                }
            } else {
#pragma unroll
                for (int u = 0; u < (int)kStepLoads; u++) v[u] = sh4[q + u * 64 + lane];
            }
            const float *ps = pos + q / 4;   // the step's positions: floats 3 (q / 12) ..
            const bool two = lane < kStepPrims * 3 - 64;   // lanes with a second position float
            const float a0 = ps[lane], a1 = ps[two ? 64 + lane : lane];
            take_pos(a0, 0);                             // axis lane mod 3
            take_pos(two ? a1 : __builtin_nanf(""), 1);  // axis (lane + 1) mod 3; NaN leaves fminf/fmaxf as they are
#pragma unroll
            for (int u = 0; u < (int)kStepLoads; u++) {
                take(v[u], u % 3, q + u * 64 + lane);
                const uint32_t c = u * 64 + lane;   // chunk within the step
                if (DEG) sd[c] = (uint8_t)degree_mask(v[u], (int)((lane + 4 * (u % 3)) % 12));
                if (c % 12 == 0) {
                    st[c / 12 * 3] = v[u].x;
                    st[c / 12 * 3 + 1] = v[u].y;
                    st[c / 12 * 3 + 2] = v[u].z;
                }
            }
            float *o = dc + q / 12 * 3;   // the step's 32 colours: 96 contiguous floats
            o[lane] = st[lane];
            if (lane < kStepPrims * 3 - 64) o[64 + lane] = st[64 + lane];
            if (DEG) store_degrees(q / 12, kStepPrims);
        }
        // the rest of the run, less than one step
        const uint32_t rest = (uint32_t)(q1 > q ? (q1 - q) / 12 : 0);   // primitives
#pragma unroll
        for (int u = 0; u < 2; u++)
            if (u * 64 + lane < rest * 3) take_pos(pos[q / 4 + u * 64 + lane], u);
#pragma unroll
        for (int u = 0; u < (int)kStepLoads; u++) {
            const uint64_t qq = q + u * 64 + lane;
            if (qq < q1) {
                float4 v = sh4[qq];
                take(v, u % 3, qq);
                if (DEG) sd[u * 64 + lane] = (uint8_t)degree_mask(v, (int)((lane + 4 * (u % 3)) % 12));
                if ((u * 64 + lane) % 12 == 0) {
                    float *o = dc + qq / 12 * 3;
                    o[0] = v.x;
                    o[1] = v.y;
                    o[2] = v.z;
                }
            }
        }
        if (DEG) store_degrees(q / 12, rest);
    }
    // fold: place j = (lane + 4k) mod 12 holds floats 4j..4j+3 (bands (4j+c)/3)
#pragma unroll
    for (int k = 0; k < 3; k++) {
        const int j = (int)((lane + 4 * k) % 12), bandA = (4 * j) / 3, bandB = (4 * j + 3) / 3;
        float minA = INFINITY, maxA = -INFINITY, minB = INFINITY, maxB = -INFINITY;
#pragma unroll
        for (int c = 0; c < 4; c++) {
            if ((4 * j + c) / 3 == bandA) { minA = fminf(minA, mn[k][c]); maxA = fmaxf(maxA, mx[k][c]); }
            else { minB = fminf(minB, mn[k][c]); maxB = fmaxf(maxB, mx[k][c]); }
        }
        atomicMin(&s_acc[bandA], ord_of(minA));
        atomicMax(&s_acc[16 + bandA], ord_of(maxA));
        if (bandB != bandA) {
            atomicMin(&s_acc[bandB], ord_of(minB));
            atomicMax(&s_acc[16 + bandB], ord_of(maxB));
        }
        const int axis = (int)((lane + k) % 3);
        atomicMin(&s_acc[32 + axis], ord_of(pmn[k]));
        atomicMax(&s_acc[35 + axis], ord_of(pmx[k]));
    }
    __syncthreads();
    if (tid < kAccWords) {
        if (acc_is_min((int)tid)) atomicMin(&acc[tid], s_acc[tid]);
        else atomicMax(&acc[tid], s_acc[tid]);
    }
}

// Signed zero: the range endpoints are values, stored as +0 when zero.
__device__ __forceinline__ float canon_zero(float x) { return x == 0.0f ? 0.0f : x; }

// The range record's fields from the extremes acc: lane k < 16 band k,
// lane k < 3 also axis k.  cov: null for the min/max range, else the
// coverage state (prefix[16] = bit pattern of t per band after the last
// selection pass) for [-t, t].
__device__ __forceinline__ void band_range(const uint32_t *acc, int k, float &lo, float &hi, float &scale)
{
    lo = canon_zero(float_of(acc[k]));
    hi = canon_zero(float_of(acc[16 + k]));
    const float range = hi - lo;
    scale = range > 0.0f ? 255.0f / range : 0.0f;
}
__device__ __forceinline__ void axis_range(const uint32_t *acc, int a, uint32_t grid_bits, float &lo, float &hi,
                                           float &cell_scale)
{
    lo = canon_zero(float_of(acc[32 + a]));
    hi = canon_zero(float_of(acc[35 + a]));
    const float ext = hi - lo;
    cell_scale = ext > 0.0f ? (float)(1u << grid_bits) / ext : 0.0f;
}
__device__ void finish_range(const uint32_t *acc, const uint32_t *cov, uint32_t grid_bits, RangeRec *r, int k)
{
    if (k < 16) {
        float lo, hi, scale;
        band_range(acc, k, lo, hi, scale);
        if (cov) {
            const float t = __uint_as_float(cov[k]);
            lo = canon_zero(-t);
            hi = t;
            const float range = hi - lo;
            scale = range > 0.0f ? 255.0f / range : 0.0f;
        }
        r->vmin[k] = lo;
        r->vmax[k] = hi;
        r->scale[k] = scale;
    }
    if (k < 3) axis_range(acc, k, grid_bits, r->lo[k], r->hi[k], r->cell_scale[k]);
}

// The range record from r->acc (and cov), then r->acc back to neutral; for
// calls whose key pass does not finish the range itself (an identity order,
// or the coverage range).
__global__ __launch_bounds__(64) void k_range_final(const uint32_t *cov, uint32_t grid_bits, RangeRec *r)
{
    __shared__ uint32_t acc[kAccWords];
    const int k = threadIdx.x;
    if (k < kAccWords) {
        acc[k] = r->acc[k];
        r->acc[k] = acc_is_min(k) ? 0xFFFFFFFFu : 0u;
    }
    __syncthreads();
    finish_range(acc, cov, grid_bits, r, k);
}

// Keys, 4,096 per workgroup: (Morton cell << 24) | colour interleave, and
// the digit counts of every sort pass.  DEG: also the degree class (from
// the range pass's deg bytes) above the cell and colour fields, and the
// class counts.  A workgroup's
// keys are the first sort pass's tile: its counts of that pass's digit go
// to tcount[digit][tile].  idx_bits > 0: each word is key << idx_bits | i
// (the sort then carries the index in the key word).
// 512 threads, 8 keys each: more waves per CU hide the loads behind the
// key arithmetic better than 256 x 16
constexpr int kKeysThreads = 512, kKeysKPT = kSortTile / kKeysThreads;
template <bool DEG>
__global__ __launch_bounds__(kKeysThreads) void k_keys(const float *pos, const float *dc, const uint8_t *deg,
                                              uint64_t n, uint32_t grid_bits,
                                              RangeRec *r, bool self_range, SortPlan plan, uint64_t *keys,
                                              uint32_t *gcount, uint32_t *tcount, uint32_t ntiles, uint32_t idx_bits,
                                              uint32_t *class_count)
{
    __shared__ uint32_t hist[kMaxPasses][kMaxBins];
    __shared__ uint32_t cls[4];
    for (int e = threadIdx.x; e < kMaxPasses * kMaxBins; e += kKeysThreads) (&hist[0][0])[e] = 0u;
    if (DEG && threadIdx.x < 4) cls[threadIdx.x] = 0u;
    // the ranges this pass needs (band 0, the three axes): self_range, from
    // the range pass's extremes (workgroup 0 also fills the whole record);
    // else from the record
    float vmin0, scale0, lo[3], cell_scale[3];
    if (self_range) {
        float hi;
        band_range(r->acc, 0, vmin0, hi, scale0);
#pragma unroll
        for (int a = 0; a < 3; a++) axis_range(r->acc, a, grid_bits, lo[a], hi, cell_scale[a]);
        if (blockIdx.x == 0 && threadIdx.x < 16) finish_range(r->acc, nullptr, grid_bits, r, (int)threadIdx.x);
    } else {
        vmin0 = r->vmin[0];
        scale0 = r->scale[0];
#pragma unroll
        for (int a = 0; a < 3; a++) { lo[a] = r->lo[a]; cell_scale[a] = r->cell_scale[a]; }
    }
    __syncthreads();
    const uint32_t cmax = (1u << grid_bits) - 1u;
    const uint32_t tile = xcd_block(blockIdx.x, gridDim.x);
    // every load of the tile first (the last element stands in past the end),
    // so the workgroup has them all in flight at once
    float px[kKeysKPT][3], pc[kKeysKPT][3];
    uint32_t pl[kKeysKPT];
#pragma unroll
    for (int it = 0; it < kKeysKPT; it++) {
        const uint64_t i = (uint64_t)tile * kSortTile + (uint64_t)it * kKeysThreads + threadIdx.x;
        const uint64_t ic = i < n ? i : n - 1;
#pragma unroll
        for (int a = 0; a < 3; a++) {
            px[it][a] = pos[ic * 3 + a];
            pc[it][a] = dc[ic * 3 + a];
        }
        pl[it] = DEG ? deg[ic] : 0u;
    }
#pragma unroll
    for (int it = 0; it < kKeysKPT; it++) {
        const uint64_t i = (uint64_t)tile * kSortTile + (uint64_t)it * kKeysThreads + threadIdx.x;
        if (i >= n) break;
        uint32_t cell[3];
#pragma unroll
        for (int a = 0; a < 3; a++) {
            float t = px[it][a] - lo[a];
            float u = t * cell_scale[a];
            uint32_t v = (uint32_t)floorf(u);
            cell[a] = v < cmax ? v : cmax;
        }
        // band-0 colour, as the range pass stored it (times the opacity)
        const float d0 = pc[it][0], d1 = pc[it][1], d2 = pc[it][2];
        const uint32_t q0 = quant8(d0, vmin0, scale0);
        const uint32_t q1 = quant8(d1, vmin0, scale0);
        const uint32_t q2 = quant8(d2, vmin0, scale0);
        const uint64_t chunk = spread3(cell[0]) | (spread3(cell[1]) << 1) | (spread3(cell[2]) << 2);
        const uint32_t colour = (spread3(q0) << 2) | (spread3(q1) << 1) | spread3(q2);
        uint64_t key = (chunk << 24) | colour;
        if (DEG) {   // the degree class the range pass found
            const uint32_t L = pl[it];
            key |= (uint64_t)L << (24 + 3 * grid_bits);
            atomicAdd(&cls[L], 1u);
        }
        keys[i] = idx_bits ? key << idx_bits | i : key;
#pragma unroll
        for (int p = 0; p < kMaxPasses; p++)
            if (p < plan.passes) atomicAdd(&hist[p][(uint32_t)(key >> plan.shift[p]) & ((1u << plan.bits[p]) - 1u)], 1u);
    }
    __syncthreads();
#pragma unroll
    for (int p = 0; p < kMaxPasses; p++)
        if (p < plan.passes)
            for (int d = threadIdx.x; d < (1 << plan.bits[p]); d += kKeysThreads)
                if (hist[p][d]) atomicAdd(&gcount[p * kMaxBins + d], hist[p][d]);
    for (int d = threadIdx.x; d < (1 << plan.bits[0]); d += kKeysThreads) tcount[(uint64_t)d * ntiles + tile] = hist[0][d];
    if (DEG && threadIdx.x < 4 && cls[threadIdx.x]) atomicAdd(&class_count[threadIdx.x], cls[threadIdx.x]);
}

// The sort is reduce-then-scan, three steps per pass: each tile's digit
// counts (for the first pass, from the key kernel), an exclusive scan of
// the counts over tiles for every digit, offset by the digit's start in the
// output, then the scatter.  No tile ever waits on another, so any number
// of tiles may run at once or in any order.  Counts and offsets are stored
// [digit][tile].

// Digit counts of one tile of 4,096 keys (passes after the first).
__global__ __launch_bounds__(256) void k_tile_hist(const uint64_t *kin, uint64_t n, int shift, int bits,
                                                   uint32_t ntiles, uint32_t *tcount)
{
    __shared__ uint32_t h[kMaxBins];
    const uint32_t tid = threadIdx.x, nbins = 1u << bits, mask = nbins - 1u;
    h[tid] = 0u;
    h[tid + 256] = 0u;
    const uint32_t tile = xcd_block(blockIdx.x, gridDim.x);
    const uint64_t t0 = (uint64_t)tile * kSortTile;
    uint64_t key[kSortKPT];
#pragma unroll
    for (int it = 0; it < kSortKPT; it++) {
        const uint64_t e = t0 + (uint64_t)it * 256 + tid;
        key[it] = e < n ? kin[e] : 0ull;
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < kSortKPT; it++)
        if (t0 + (uint64_t)it * 256 + tid < n) atomicAdd(&h[(uint32_t)(key[it] >> shift) & mask], 1u);
    __syncthreads();
    for (uint32_t d = tid; d < nbins; d += 256) tcount[(uint64_t)d * ntiles + tile] = h[d];
}

// Workgroup d: toff[d][t] = (keys of digits below d) + (keys of digit d in
// tiles before t), from the pass's digit totals and the tile counts.  Each
// thread scans kScanPer consecutive tiles per round.
constexpr int kScanPer = 4;
__global__ __launch_bounds__(256) void k_tile_scan(const uint32_t *tcount, const uint32_t *gcount, uint32_t ntiles,
                                                   uint32_t *toff)
{
    __shared__ uint32_t wsum[4];
    __shared__ uint32_t s_base;
    const uint32_t d = blockIdx.x, tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
    const uint32_t *c = tcount + (uint64_t)d * ntiles;
    uint32_t *out = toff + (uint64_t)d * ntiles;
    // the first round's counts are read together with the digit totals
    uint32_t v[kScanPer];
#pragma unroll
    for (int i = 0; i < kScanPer; i++) v[i] = tid * kScanPer + i < ntiles ? c[tid * kScanPer + i] : 0u;
    // keys of the lower digits: a block sum over gcount[0 .. d)
    uint32_t b = 0;
    for (uint32_t e = tid; e < d; e += 256) b += gcount[e];
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) b += __shfl_xor(b, o);
    if (lane == 0) wsum[w] = b;
    __syncthreads();
    if (tid == 0) s_base = wsum[0] + wsum[1] + wsum[2] + wsum[3];
    __syncthreads();
    uint32_t carry = s_base;
    for (uint32_t r0 = 0; r0 < ntiles; r0 += 256 * kScanPer) {
        const uint32_t t = r0 + tid * kScanPer;
        if (r0 > 0)
#pragma unroll
            for (int i = 0; i < kScanPer; i++) v[i] = t + i < ntiles ? c[t + i] : 0u;
        uint32_t sum = 0;
#pragma unroll
        for (int i = 0; i < kScanPer; i++) sum += v[i];
        uint32_t inc = sum;   // inclusive scan of the per-thread sums over the wave
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t x = __shfl_up(inc, o);
            if (lane >= (uint32_t)o) inc += x;
        }
        __syncthreads();   // wsum of the previous round has been read
        if (lane == 63) wsum[w] = inc;
        __syncthreads();
        uint32_t ex = carry + inc - sum;
        for (uint32_t q = 0; q < w; q++) ex += wsum[q];
#pragma unroll
        for (int i = 0; i < kScanPer; i++) {
            if (t + i < ntiles) out[t + i] = ex;
            ex += v[i];
        }
        carry += wsum[0] + wsum[1] + wsum[2] + wsum[3];
    }
}

// One pass of the stable LSD sort over digit (shift, bits): the scatter of
// tile blockIdx.x, given toff.  PACKED: the words hold the element index in
// their low idx_bits bits (vin unused); else vin holds the values (null: the
// element indices).  kout null: only the values (the indices) are written,
// to vout (the last pass, into perm).  reset (the first pass): the range
// extremes to put back to neutral, the key pass having read them.
template <bool PACKED>
__global__ __launch_bounds__(256) void k_sort_pass(const uint64_t *kin, const uint32_t *vin, uint64_t *kout,
                                                   uint32_t *vout, uint64_t n, int shift, int bits,
                                                   const uint32_t *toff, uint32_t ntiles, uint32_t idx_bits,
                                                   RangeRec *reset)
{
    // 52 KB of LDS, so three workgroups share a CU.  The ranking's lane
    // masks and the sorted keys use the same LDS at different times; the
    // values are not staged: the sorted position keeps the element's index
    // in the tile and the value is read back from the input (a cache hit).
    __shared__ uint64_t skey[kSortTile];
    __shared__ uint16_t sidx[PACKED ? 1 : kSortTile];
    __shared__ uint32_t ctr[4][kMaxBins];    // per wave: running digit counts, then the wave's offset in the tile
    uint64_t(*peer)[kMaxBins] = reinterpret_cast<uint64_t(*)[kMaxBins]>(skey);   // per wave: lanes of one step
                                                                                 // holding each digit
    __shared__ uint32_t lstart[kMaxBins];    // first tile-local sorted position of each digit
    __shared__ int32_t gadj[kMaxBins];       // output index of sorted position j of digit d: gadj[d] + j
    __shared__ uint32_t wsum[4];
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
    if (reset && blockIdx.x == 0 && tid < kAccWords)   // the key pass has read the extremes: back to neutral
        reset->acc[tid] = acc_is_min(tid) ? 0xFFFFFFFFu : 0u;
    for (int e = tid; e < 4 * kMaxBins; e += 256) {
        (&ctr[0][0])[e] = 0u;
        (&peer[0][0])[e] = 0ull;
    }
    __syncthreads();
    const uint32_t tile = xcd_block(blockIdx.x, gridDim.x);
    const uint32_t nbins = 1u << bits, mask = nbins - 1u;
    const uint64_t t0 = (uint64_t)tile * kSortTile;
    // this tile's output offsets, in flight during the ranking
    uint32_t off[2];
#pragma unroll
    for (int h = 0; h < 2; h++) {
        const uint32_t d = 2 * tid + h;
        off[h] = d < nbins ? toff[(uint64_t)d * ntiles + tile] : 0u;
    }
    // wave w holds tile elements [w T/4, (w + 1) T/4), 64 consecutive per step
    const uint64_t wbase = t0 + (uint64_t)w * (kSortTile / 4);
    const uint64_t below = lane ? (~0ull >> (64 - lane)) : 0ull;
    uint64_t key[kSortKPT];
    uint32_t rk[kSortKPT];
#pragma unroll
    for (int it = 0; it < kSortKPT; it++) {
        const uint64_t e = wbase + (uint64_t)it * 64 + lane;
        key[it] = e < n ? kin[e] : 0ull;
    }
    // rank of each key among the equal digits before it in its wave: per
    // step, each lane ORs its bit into its digit's LDS mask, reads the mask
    // back (the lanes of this step with the same digit) and the digit's
    // running count; the lowest such lane advances the count and clears the
    // mask (LDS operations of one wave complete in issue order)
#pragma unroll
    for (int it = 0; it < kSortKPT; it++) {
        const bool ok = wbase + (uint64_t)it * 64 + lane < n;
        const uint32_t d = (uint32_t)(key[it] >> shift) & mask;
        if (ok) atomicOr(&peer[w][d], 1ull << lane);
        __builtin_amdgcn_wave_barrier();
        const uint64_t peers = ok ? peer[w][d] : 0ull;
        const uint32_t before = ok ? ctr[w][d] : 0u;
        rk[it] = before + (uint32_t)__popcll(peers & below);
        __builtin_amdgcn_wave_barrier();
        if (ok && (peers & below) == 0) {
            ctr[w][d] = before + (uint32_t)__popcll(peers);
            peer[w][d] = 0ull;
        }
        __builtin_amdgcn_wave_barrier();
    }
    __syncthreads();
    // thread tid: digits 2 tid and 2 tid + 1.  Wave offsets within the tile,
    // the tile's counts, their prefix over the digits (the local start)
    uint32_t cnt[2];
#pragma unroll
    for (int h = 0; h < 2; h++) {
        const uint32_t d = 2 * tid + h;
        uint32_t c = 0;
        if (d < nbins) {
#pragma unroll
            for (int q = 0; q < 4; q++) {
                const uint32_t x = ctr[q][d];
                ctr[q][d] = c;
                c += x;
            }
        }
        cnt[h] = c;
    }
    uint32_t lc = cnt[0] + cnt[1];
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t a = __shfl_up(lc, o);
        if (lane >= o) lc += a;
    }
    if (lane == 63) wsum[w] = lc;
    __syncthreads();
    uint32_t lex = lc - (cnt[0] + cnt[1]);
    for (int q = 0; q < w; q++) lex += wsum[q];
#pragma unroll
    for (int h = 0; h < 2; h++) {
        const uint32_t d = 2 * tid + h;
        if (d < nbins) {
            lstart[d] = lex;
            gadj[d] = (int32_t)off[h] - (int32_t)lex;
        }
        lex += cnt[h];
    }
    __syncthreads();
    // the tile sorted by digit in LDS (stable: waves in order, then rank)
#pragma unroll
    for (int it = 0; it < kSortKPT; it++) {
        if (wbase + (uint64_t)it * 64 + lane < n) {
            const uint32_t d = (uint32_t)(key[it] >> shift) & mask;
            const uint32_t lp = lstart[d] + ctr[w][d] + rk[it];
            skey[lp] = key[it];
            if (!PACKED) sidx[lp] = (uint16_t)(w * (kSortTile / 4) + it * 64 + lane);
        }
    }
    __syncthreads();
    // each digit's keys leave as one contiguous run
    const uint32_t tn = (uint32_t)(n - t0 < (uint64_t)kSortTile ? n - t0 : (uint64_t)kSortTile);
    const uint64_t imask = (1ull << idx_bits) - 1ull;
    for (uint32_t j = tid; j < tn; j += 256) {
        const uint64_t k = skey[j];
        const uint32_t o = (uint32_t)(gadj[(uint32_t)(k >> shift) & mask] + (int32_t)j);
        if (PACKED) {
            if (kout) kout[o] = k;
            else vout[o] = (uint32_t)(k & imask);
        } else {
            const uint64_t e = t0 + sidx[j];
            if (kout) kout[o] = k;
            vout[o] = vin ? vin[e] : (uint32_t)e;
        }
    }
}

// One thread per slot s < npad: quantise its 16 band vectors and place them
// by the arrangement (0: stream k, block s/16, texel zigzag(s%16); 1: block
// s, texel k; 2: stream k/4, block s/4, texel 4 (s%4) + k%4).
// host_range (host memory the device can write, or null): workgroup 0 also
// copies the range record there, so a caller waiting for the stream needs
// no separate read-back.
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void k_gather_pack(const float *sh, const float *opacity, const uint32_t *perm,
                                                     uint64_t n, uint64_t npad, uint32_t arrangement,
                                                     const RangeRec *r, uint32_t *tex, RangeRec *host_range)
{
    static_assert(sizeof(RangeRec) % 4 == 0 && sizeof(RangeRec) / 4 <= 256, "one word per thread");
    if (host_range && blockIdx.x == 0 && threadIdx.x < sizeof(RangeRec) / 4)
        reinterpret_cast<uint32_t *>(host_range)[threadIdx.x] = reinterpret_cast<const uint32_t *>(r)[threadIdx.x];
    uint64_t s = (uint64_t)xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (s >= npad) return;
    uint32_t src = perm[s < n ? s : n - 1];
    const float4 *p = reinterpret_cast<const float4 *>(sh + (uint64_t)src * 48);
    float f[48];
#pragma unroll
    for (int c = 0; c < 12; c++) {
        float4 v = p[c];
        f[4 * c] = v.x; f[4 * c + 1] = v.y; f[4 * c + 2] = v.z; f[4 * c + 3] = v.w;
    }
    if (opacity) {
        const float mu = opacity[src];
#pragma unroll
        for (int e = 0; e < 48; e++) f[e] = mu * f[e];
    }
    uint32_t w[16];
#pragma unroll
    for (int k = 0; k < 16; k++) {
        float vm = r->vmin[k], sc = r->scale[k];
        w[k] = quant8(f[3 * k], vm, sc) | (quant8(f[3 * k + 1], vm, sc) << 8) |
               (quant8(f[3 * k + 2], vm, sc) << 16) | 0xFF000000u;
    }
    // The textures leave with non-temporal stores: they are read again only
    // by the encoders, and lines not kept dirty in the caches leave room for
    // the next call's reads (3,145,728 primitives: gather 0.190 -> 0.184 ms,
    // the following range pass 0.138 -> 0.131 ms).
    if (arrangement == 1) {            // one primitive per block: 64 contiguous bytes
        u32x4 *d = reinterpret_cast<u32x4 *>(tex + s * 16);
#pragma unroll
        for (int q = 0; q < 4; q++)
            __builtin_nontemporal_store(u32x4{w[4 * q], w[4 * q + 1], w[4 * q + 2], w[4 * q + 3]}, d + q);
    } else if (arrangement == 2) {     // four primitives per four blocks: one 16-byte row per stream
        const uint64_t bps = npad / 4;
#pragma unroll
        for (int g = 0; g < 4; g++)
            __builtin_nontemporal_store(u32x4{w[4 * g], w[4 * g + 1], w[4 * g + 2], w[4 * g + 3]},
                                        reinterpret_cast<u32x4 *>(tex + ((uint64_t)g * bps + (s >> 2)) * 16 + 4 * (s & 3)));
    } else {
        const uint64_t nblk = npad / 16;
        const uint32_t j = (uint32_t)(s & 15);
        const uint32_t x = (j & 1u) | (((j >> 2) & 1u) << 1);
        const uint32_t y = ((j >> 1) & 1u) | (((j >> 3) & 1u) << 1);
        const uint64_t texel = (s >> 4) * 16 + 4 * y + x;
#pragma unroll
        for (int k = 0; k < 16; k++) __builtin_nontemporal_store(w[k], &tex[(uint64_t)k * nblk * 16 + texel]);
    }
}

// ---- the coverage range: per band the r-th smallest |x| over its 3n
// coefficients, by radix selection on the bit patterns of |x| (non-negative
// floats order like their bits): four passes over bits 30..23, 22..15,
// 14..7 and 6..0, each a histogram of the next digit among the values that
// match the prefix chosen so far, then a scan that picks the digit holding
// the remaining rank.
constexpr int kCovWG = 256;
constexpr uint64_t kCoverNum = 995, kCoverDen = 1000;   // 99.5 % of each band inside [-t, t]                    // workgroups of the histogram pass
constexpr int kCovShift[4] = {23, 15, 7, 0};
constexpr int kCovWidth[4] = {8, 8, 8, 7};

// part[wg][band][256]: this workgroup's digit counts; state[band] = prefix,
// state[16 + band] = remaining rank.
__global__ __launch_bounds__(kRangeBlock) void k_cov_hist(const float4 *sh4, const float *opacity, uint64_t n,
                                                          int pass, const uint32_t *state, uint32_t *part)
{
    __shared__ uint32_t h[16][256];
    for (int e = threadIdx.x; e < 16 * 256; e += kRangeBlock) h[e >> 8][e & 255] = 0;
    __syncthreads();
    const int shift = kCovShift[pass], width = kCovWidth[pass];
    const uint64_t T = (uint64_t)gridDim.x * blockDim.x;
    const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int j = (int)(t % 12);
    const uint64_t nq = n * 12;
    for (uint64_t q = t; q < nq; q += T) {
        float4 v = sh4[q];
        float f[4] = {v.x, v.y, v.z, v.w};
        const float mu = opacity ? opacity[q / 12] : 1.0f;
#pragma unroll
        for (int c = 0; c < 4; c++) {
            const int band = (4 * j + c) / 3;
            const uint32_t u = __float_as_uint(opacity ? mu * f[c] : f[c]) & 0x7FFFFFFFu;
            if (pass > 0 && (u >> (shift + width)) != state[band]) continue;
            atomicAdd(&h[band][(u >> shift) & ((1u << width) - 1u)], 1u);
        }
    }
    __syncthreads();
    for (int e = threadIdx.x; e < 16 * 256; e += kRangeBlock)
        part[(uint64_t)blockIdx.x * 4096 + e] = h[e >> 8][e & 255];
}

// One workgroup per band, one thread per digit: total the partial counts,
// scan, and keep the digit whose cumulative count reaches the rank.
__global__ __launch_bounds__(256) void k_cov_select(const uint32_t *part, uint32_t nwg, int pass, uint32_t *state)
{
    __shared__ uint32_t scan[256];
    const int band = blockIdx.x, d = threadIdx.x;
    uint32_t c = 0;
    for (uint32_t w = 0; w < nwg; w++) c += part[(uint64_t)w * 4096 + band * 256 + d];
    scan[d] = c;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {   // inclusive scan
        const uint32_t x = d >= off ? scan[d - off] : 0u;
        __syncthreads();
        scan[d] += x;
        __syncthreads();
    }
    const uint32_t rank = state[16 + band], incl = scan[d], excl = incl - c;
    if (c > 0 && excl < rank && rank <= incl) {
        state[band] = (state[band] << kCovWidth[pass]) | (uint32_t)d;
        state[16 + band] = rank - excl;
    }
}

__global__ void k_cov_init(uint32_t *state, uint32_t rank)
{
    if (threadIdx.x < 16) {
        state[threadIdx.x] = 0;
        state[16 + threadIdx.x] = rank;
    }
}

__global__ void k_zero4(uint32_t *c)
{
    if (threadIdx.x < 4) c[threadIdx.x] = 0;
}

// One thread per padded slot of every class: thread t of class L (t in
// [pad_start[L], pad_start[L+1])) is class slot j = t - pad_start[L], the
// dense slot slot_start[L] + min(j, count[L] - 1); its (L+1)^2 kept bands go
// to stream k of the class, block j/16, zigzag texel of j%16 -- or, for the
// degree-1 class in Fig. SetupC, bands 0..3 to texels 4 (j%4) + k of block
// j/4 of the class's one stream.
__global__ __launch_bounds__(256) void k_pack_degrees(const float *sh, const float *opacity, const uint32_t *perm,
                                                      DegreeLayout lay, const RangeRec *r, uint32_t *tex)
{
    const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= lay.pad_start[4]) return;
    int L = 0;
    while (L < 3 && t >= lay.pad_start[L + 1]) L++;
    const uint64_t j = t - lay.pad_start[L];
    const uint64_t cnt = lay.slot_start[L + 1] - lay.slot_start[L];
    const uint32_t src = perm[lay.slot_start[L] + (j < cnt ? j : cnt - 1)];
    const float4 *p = reinterpret_cast<const float4 *>(sh + (uint64_t)src * 48);
    float f[48];
#pragma unroll
    for (int c = 0; c < 12; c++) {
        const float4 v = p[c];
        f[4 * c] = v.x; f[4 * c + 1] = v.y; f[4 * c + 2] = v.z; f[4 * c + 3] = v.w;
    }
    if (opacity) {
        const float mu = opacity[src];
#pragma unroll
        for (int e = 0; e < 48; e++) f[e] = mu * f[e];
    }
    const int nb = (L + 1) * (L + 1);
    if (L == 1 && lay.quad1) {
        uint32_t *blk = tex + lay.tex_word[1] + (j >> 2) * 16 + 4 * (j & 3);
#pragma unroll
        for (int k = 0; k < 4; k++) {
            const float vm = r->vmin[k], sc = r->scale[k];
            blk[k] = quant8(f[3 * k], vm, sc) | (quant8(f[3 * k + 1], vm, sc) << 8) |
                     (quant8(f[3 * k + 2], vm, sc) << 16) | 0xFF000000u;
        }
        return;
    }
    const uint64_t nblk = (lay.pad_start[L + 1] - lay.pad_start[L]) / 16;
    const uint32_t jj = (uint32_t)(j & 15);
    const uint32_t x = (jj & 1u) | (((jj >> 2) & 1u) << 1);
    const uint32_t y = ((jj >> 1) & 1u) | (((jj >> 3) & 1u) << 1);
    uint32_t *base = tex + lay.tex_word[L] + (j >> 4) * 16 + 4 * y + x;
#pragma unroll
    for (int k = 0; k < 16; k++) {
        if (k < nb) {
            const float vm = r->vmin[k], sc = r->scale[k];
            base[(uint64_t)k * nblk * 16] = quant8(f[3 * k], vm, sc) | (quant8(f[3 * k + 1], vm, sc) << 8) |
                                            (quant8(f[3 * k + 2], vm, sc) << 16) | 0xFF000000u;
        }
    }
}

struct Layout {
    size_t keys_a, keys_b, vals_a, vals_b, dc, deg, tcount, toff, meta, cov_state, cov_part, bytes;
    uint64_t ntiles;
};

// meta: digit totals [kMaxPasses][kMaxBins]
constexpr uint32_t kMetaWords = kMaxPasses * kMaxBins;

Layout layout(uint64_t n)
{
    auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
    Layout L;
    L.ntiles = (n + kSortTile - 1) / kSortTile;
    size_t o = 0;
    L.keys_a = o; o += al(n * 8);
    L.keys_b = o; o += al(n * 8);
    L.vals_a = o; o += al(n * 4);
    L.vals_b = o; o += al(n * 4);
    L.dc = o; o += al(n * 12);
    L.deg = o; o += al(n);   // degree classes (the degree-class reorder)
    L.tcount = o; o += al(L.ntiles * kMaxBins * 4);   // [digit][tile] counts of the current pass
    L.toff = o; o += al(L.ntiles * kMaxBins * 4);     // [digit][tile] output offsets
    L.meta = o; o += al(kMetaWords * 4);
    L.cov_state = o; o += al(32 * 4);
    L.cov_part = o; o += al((size_t)kCovWG * 4096 * 4);
    L.bytes = o;
    return L;
}

}  // namespace

size_t reorder_scratch_bytes(uint64_t n, uint32_t) { return layout(n).bytes; }

// perm[s] = s (the unsorted order).
__global__ void k_iota(uint32_t *perm, uint64_t n)
{
    const uint64_t s = (uint64_t)blockIdx.x * 256 + threadIdx.x;
    if (s < n) perm[s] = (uint32_t)s;
}

namespace {

// Range prologue: min/max (and the coverage range when asked) into range_dev.
// keys_finish: the key pass will fill the range record (and put the extremes
// back) itself, so no finishing launch is needed unless the coverage range
// replaces the band ranges.
// deg_tau >= 0: also each primitive's degree class (threshold deg_tau) into
// the arena's deg bytes, for the degree-class key pass.
void enqueue_range(const float *pos, const float *sh, const float *opacity, uint64_t n, uint32_t grid_bits,
                   uint32_t quantiser, bool keys_finish, float deg_tau, const Layout &L, char *s, RangeRec *range_dev,
                   hipStream_t st)
{
    uint64_t want = (n * 12 + kRangeBlock - 1) / kRangeBlock;
    // at most 512 workgroups of 768 (two per CU, each one contiguous span)
    const uint32_t nb = (uint32_t)std::min<uint64_t>(std::max<uint64_t>((n * 12 + kMinMaxBlock - 1) / kMinMaxBlock, 1), 512);
    const bool stream = n * 192 > kStreamRowBytes;
    if (deg_tau >= 0.0f)
        GSBC_LAUNCH("range_partial", k_range_partial<true>, dim3(nb), dim3(kMinMaxBlock), 0, st,
                    reinterpret_cast<const float4 *>(sh), opacity, pos, n, range_dev->acc,
                    reinterpret_cast<float *>(s + L.dc), reinterpret_cast<uint32_t *>(s + L.meta), kMetaWords, deg_tau,
                    reinterpret_cast<uint8_t *>(s + L.deg), stream);
    else
        GSBC_LAUNCH("range_partial", k_range_partial<false>, dim3(nb), dim3(kMinMaxBlock), 0, st,
                    reinterpret_cast<const float4 *>(sh), opacity, pos, n, range_dev->acc,
                    reinterpret_cast<float *>(s + L.dc), reinterpret_cast<uint32_t *>(s + L.meta), kMetaWords, 0.0f,
                    nullptr, stream);
    uint32_t *cov = nullptr;
    if (quantiser == 1) {
        cov = reinterpret_cast<uint32_t *>(s + L.cov_state);
        uint32_t *part = reinterpret_cast<uint32_t *>(s + L.cov_part);
        // 1-based rank of the covering magnitude among the 3n per band
        const uint32_t rank = (uint32_t)((3 * n * kCoverNum + kCoverDen - 1) / kCoverDen);
        GSBC_LAUNCH("cov_init", k_cov_init, dim3(1), dim3(64), 0, st, cov, rank);
        const uint32_t ncw = (uint32_t)std::min<uint64_t>(std::max<uint64_t>(want, 1), kCovWG);
        for (int pass = 0; pass < 4; pass++) {
            GSBC_LAUNCH("cov_hist", k_cov_hist, dim3(ncw), dim3(kRangeBlock), 0, st,
                        reinterpret_cast<const float4 *>(sh), opacity, n, pass, cov, part);
            GSBC_LAUNCH("cov_select", k_cov_select, dim3(16), dim3(256), 0, st, part, ncw, pass, cov);
        }
    }
    if (quantiser == 1 || !keys_finish)
        GSBC_LAUNCH("range_final", k_range_final, dim3(1), dim3(64), 0, st, cov, grid_bits, range_dev);
}

// The keys in keys_a with their digit totals and the first pass's tile
// counts (the key pass), then per pass: the tile counts (after the first),
// the offsets, the scatter; the last pass writes the values (the original
// indices) to perm.
template <bool DEG>
void enqueue_keys_and_sort(const float *pos, uint64_t n, uint32_t grid_bits, bool self_range, const Layout &L, char *s,
                           RangeRec *range_dev, uint32_t *class_count, uint32_t *perm, hipStream_t st)
{
    const int key_bits = (DEG ? 26 : 24) + 3 * (int)grid_bits;
    const SortPlan P = plan_sort(key_bits);
    // the index rides in the low bits of the key word when both fit in 64
    uint32_t idx_bits = 1;
    while (idx_bits < 32 && (1ull << idx_bits) < n) idx_bits++;
    const bool packed = key_bits + (int)idx_bits <= 64;
    const uint32_t ib = packed ? idx_bits : 0u;
    uint64_t *ka = reinterpret_cast<uint64_t *>(s + L.keys_a), *kb = reinterpret_cast<uint64_t *>(s + L.keys_b);
    uint32_t *va = reinterpret_cast<uint32_t *>(s + L.vals_a), *vb = reinterpret_cast<uint32_t *>(s + L.vals_b);
    uint32_t *tcount = reinterpret_cast<uint32_t *>(s + L.tcount), *toff = reinterpret_cast<uint32_t *>(s + L.toff);
    uint32_t *gcount = reinterpret_cast<uint32_t *>(s + L.meta);
    const uint32_t ntiles = (uint32_t)L.ntiles;
    const dim3 grid(ntiles);
    GSBC_LAUNCH(DEG ? "keys_degree" : "keys", k_keys<DEG>, grid, dim3(kKeysThreads), 0, st, pos,
                reinterpret_cast<const float *>(s + L.dc), reinterpret_cast<const uint8_t *>(s + L.deg), n, grid_bits,
                range_dev, self_range, P, ka, gcount, tcount, ntiles, ib, class_count);
    const uint64_t *kin = ka;
    uint64_t *kout = kb;
    const uint32_t *vin = nullptr;
    uint32_t *vout = va;
    for (int p = 0; p < P.passes; p++) {
        const bool last = p == P.passes - 1;
        const int shift = P.shift[p] + (int)ib;
        if (p > 0)
            GSBC_LAUNCH("tile_hist", k_tile_hist, grid, dim3(256), 0, st, kin, n, shift, P.bits[p], ntiles, tcount);
        GSBC_LAUNCH("tile_scan", k_tile_scan, dim3(1u << P.bits[p]), dim3(256), 0, st, tcount,
                    gcount + p * kMaxBins, ntiles, toff);
        if (packed)
            GSBC_LAUNCH("sort_pass", k_sort_pass<true>, grid, dim3(256), 0, st, kin, nullptr, last ? nullptr : kout,
                        last ? perm : nullptr, n, shift, P.bits[p], toff, ntiles, ib, p == 0 ? range_dev : nullptr);
        else
            GSBC_LAUNCH("sort_pass", k_sort_pass<false>, grid, dim3(256), 0, st, kin, vin, last ? nullptr : kout,
                        last ? perm : vout, n, shift, P.bits[p], toff, ntiles, 0u, p == 0 ? range_dev : nullptr);
        const uint64_t *kt = kin;
        kin = kout;
        kout = const_cast<uint64_t *>(kt);
        vin = vout;
        vout = vout == va ? vb : va;
    }
}

}  // namespace

hipError_t launch_reorder(const float *pos, const float *sh, const float *opacity, uint64_t n, uint32_t grid_bits,
                          uint32_t quantiser, bool identity, uint32_t arrangement, uint32_t *perm, uint8_t *textures,
                          void *scratch, RangeRec *range_dev, RangeRec *host_range, hipStream_t st)
{
    Layout L = layout(n);
    char *s = static_cast<char *>(scratch);
    enqueue_range(pos, sh, opacity, n, grid_bits, quantiser, !identity, -1.0f, L, s, range_dev, st);
    if (identity) {
        GSBC_LAUNCH("iota", k_iota, dim3((uint32_t)((n + 255) / 256)), dim3(256), 0, st, perm, n);
    } else {
        enqueue_keys_and_sort<false>(pos, n, grid_bits, quantiser != 1, L, s, range_dev, nullptr, perm, st);
    }
    const uint64_t npad = (n + 15) / 16 * 16;
    GSBC_LAUNCH("gather_pack", k_gather_pack, dim3((uint32_t)((npad + 255) / 256)), dim3(256), 0, st,
                       sh, opacity, perm, n, npad, arrangement, range_dev, reinterpret_cast<uint32_t *>(textures),
                       host_range);
    return hipGetLastError();
}

hipError_t launch_degree_sort(const float *pos, const float *sh, const float *opacity, uint64_t n, uint32_t grid_bits,
                              uint32_t quantiser, float tau, uint32_t *perm, void *scratch, RangeRec *range_dev,
                              uint32_t *class_count, hipStream_t st)
{
    Layout L = layout(n);
    char *s = static_cast<char *>(scratch);
    enqueue_range(pos, sh, opacity, n, grid_bits, quantiser, true, tau, L, s, range_dev, st);
    GSBC_LAUNCH("fill_count", k_zero4, dim3(1), dim3(64), 0, st, class_count);
    enqueue_keys_and_sort<true>(pos, n, grid_bits, quantiser != 1, L, s, range_dev, class_count, perm, st);
    return hipGetLastError();
}

hipError_t launch_pack_degrees(const float *sh, const float *opacity, const uint32_t *perm, const DegreeLayout &lay,
                               const RangeRec *range_dev, uint8_t *textures, hipStream_t st)
{
    const uint64_t threads = lay.pad_start[4];
    if (threads == 0) return hipSuccess;
    GSBC_LAUNCH("pack_degrees", k_pack_degrees, dim3((uint32_t)((threads + 255) / 256)), dim3(256), 0, st,
                       sh, opacity, perm, lay, range_dev, reinterpret_cast<uint32_t *>(textures));
    return hipGetLastError();
}

}  // namespace gsbc
