// reorder.hip -- colour/space reorder and block packing on gfx950.
//
//   range    per-band min/max of the SH coefficients and the position
//            bounding box (Sec. V-A quantiser range; Sec. III-C spatial
//            groups), one coalesced float4 pass with order-independent
//            integer atomics on an order-preserving encoding of the floats;
//   keys     (Morton cell of the position) << 24 | RGB bit interleave of the
//            quantised band-0 colour (Sec. III-C, Fig. Bit4Scan);
//   sort     stable LSD radix sort, 11-bit digits, per-wave tiles with
//            LDS-local counters and wave-ballot ranking (stable by
//            construction: a wave walks its tile in order);
//   pack     gather each slot's 48 coefficients, quantise, and write band k
//            of slot s to texel zigzag(s % 16) of block s / 16 (Fig. SetupD,
//            Fig. ZigZagScan).
#include "gsbc_internal.h"

#include <algorithm>

namespace gsbc {
namespace {

constexpr int kDigitBits = 11;
constexpr int kDigits = 1 << kDigitBits;
constexpr int kWaveItems = 16;                 // keys per lane per tile
constexpr int kTile = 64 * kWaveItems;         // keys per wave tile
constexpr int kChunkTiles = 16;                // tiles per chunk of the column scan
constexpr int kRangeBlock = 384;               // multiple of 12 and 3

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

// acc layout: [0..15] band min, [16..31] band max, [32..34] pos min, [35..37] pos max
__global__ void k_range_init(uint32_t *acc)
{
    int t = threadIdx.x;
    if (t < 38) acc[t] = (t < 16 || (t >= 32 && t < 35)) ? 0xFFFFFFFFu : 0u;
}

__global__ __launch_bounds__(kRangeBlock) void k_range_partial(const float4 *sh4, const float *opacity,
                                                               const float *pos, uint64_t n, uint32_t *acc)
{
    __shared__ uint32_t s_acc[38];
    if (threadIdx.x < 38) s_acc[threadIdx.x] = (threadIdx.x < 16 || (threadIdx.x >= 32 && threadIdx.x < 35)) ? 0xFFFFFFFFu : 0u;
    __syncthreads();
    const uint64_t T = (uint64_t)gridDim.x * blockDim.x;
    const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    // float4 chunk j of a primitive holds floats 4j..4j+3 -> bands (4j+c)/3
    const int j = (int)(t % 12);
    const int bandA = (4 * j) / 3, bandB = (4 * j + 3) / 3;
    float minA = INFINITY, maxA = -INFINITY, minB = INFINITY, maxB = -INFINITY;
    const uint64_t nq = n * 12;
    auto take = [&](float4 v, uint64_t q) {
        float f[4] = {v.x, v.y, v.z, v.w};
        if (opacity) {   // H~ = mu H (FP32 products)
            const float mu = opacity[q / 12];
#pragma unroll
            for (int c = 0; c < 4; c++) f[c] = mu * f[c];
        }
#pragma unroll
        for (int c = 0; c < 4; c++) {
            if ((4 * j + c) / 3 == bandA) { minA = fminf(minA, f[c]); maxA = fmaxf(maxA, f[c]); }
            else { minB = fminf(minB, f[c]); maxB = fmaxf(maxB, f[c]); }
        }
    };
    // four loads in flight per lane, then the remainder one at a time
    uint64_t q = t;
    for (; q + 3 * T < nq; q += 4 * T) {
        const float4 v0 = sh4[q], v1 = sh4[q + T], v2 = sh4[q + 2 * T], v3 = sh4[q + 3 * T];
        take(v0, q);
        take(v1, q + T);
        take(v2, q + 2 * T);
        take(v3, q + 3 * T);
    }
    for (; q < nq; q += T) take(sh4[q], q);
    const int axis = (int)(t % 3);
    float pmin = INFINITY, pmax = -INFINITY;
    for (uint64_t f = t; f < n * 3; f += T) {
        float v = pos[f];
        pmin = fminf(pmin, v);
        pmax = fmaxf(pmax, v);
    }
    atomicMin(&s_acc[bandA], ord_of(minA));
    atomicMax(&s_acc[16 + bandA], ord_of(maxA));
    if (bandB != bandA) {
        atomicMin(&s_acc[bandB], ord_of(minB));
        atomicMax(&s_acc[16 + bandB], ord_of(maxB));
    }
    atomicMin(&s_acc[32 + axis], ord_of(pmin));
    atomicMax(&s_acc[35 + axis], ord_of(pmax));
    __syncthreads();
    if (threadIdx.x < 38) {
        int i = threadIdx.x;
        if (i < 16 || (i >= 32 && i < 35)) atomicMin(&acc[i], s_acc[i]);
        else atomicMax(&acc[i], s_acc[i]);
    }
}

// Signed zero: the range endpoints are values, stored as +0 when zero.
__device__ __forceinline__ float canon_zero(float x) { return x == 0.0f ? 0.0f : x; }

// cov: null for the min/max range, else the coverage state (prefix[16] =
// bit pattern of t per band after the last selection pass) for [-t, t].
__global__ void k_range_final(const uint32_t *acc, const uint32_t *cov, uint32_t grid_bits, RangeRec *r)
{
    int k = threadIdx.x;
    if (k < 16) {
        float lo = canon_zero(float_of(acc[k])), hi = canon_zero(float_of(acc[16 + k]));
        if (cov) {
            const float t = __uint_as_float(cov[k]);
            lo = canon_zero(-t);
            hi = t;
        }
        r->vmin[k] = lo;
        r->vmax[k] = hi;
        float range = hi - lo;
        r->scale[k] = range > 0.0f ? 255.0f / range : 0.0f;
    }
    if (k < 3) {
        float lo = canon_zero(float_of(acc[32 + k])), hi = canon_zero(float_of(acc[35 + k]));
        r->lo[k] = lo;
        r->hi[k] = hi;
        float ext = hi - lo;
        r->cell_scale[k] = ext > 0.0f ? (float)(1u << grid_bits) / ext : 0.0f;
    }
}

// DEG: also the degree class (the largest SH degree with a coefficient above
// tau in magnitude, 0 if none) above the cell and colour fields, and the
// class counts.
template <bool DEG>
__global__ __launch_bounds__(256) void k_keys(const float *pos, const float *sh, const float *opacity, uint64_t n,
                                              uint32_t grid_bits, const RangeRec *r,
                                              uint64_t *keys, uint32_t *vals, float tau, uint32_t *class_count)
{
    __shared__ uint32_t cls[4];
    if (DEG) {
        if (threadIdx.x < 4) cls[threadIdx.x] = 0;
        __syncthreads();
    }
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (!DEG && i >= n) return;
    if (i < n) {
    const uint32_t cmax = (1u << grid_bits) - 1u;
    uint32_t cell[3];
#pragma unroll
    for (int a = 0; a < 3; a++) {
        float t = pos[i * 3 + a] - r->lo[a];
        float u = t * r->cell_scale[a];
        uint32_t v = (uint32_t)floorf(u);
        cell[a] = v < cmax ? v : cmax;
    }
    const float *dc = sh + i * 48;
    const float mu = opacity ? opacity[i] : 1.0f;
    float d0 = dc[0], d1 = dc[1], d2 = dc[2];
    if (opacity) { d0 = mu * d0; d1 = mu * d1; d2 = mu * d2; }
    uint32_t q0 = quant8(d0, r->vmin[0], r->scale[0]);
    uint32_t q1 = quant8(d1, r->vmin[0], r->scale[0]);
    uint32_t q2 = quant8(d2, r->vmin[0], r->scale[0]);
    uint64_t chunk = spread3(cell[0]) | (spread3(cell[1]) << 1) | (spread3(cell[2]) << 2);
    uint32_t colour = (spread3(q0) << 2) | (spread3(q1) << 1) | spread3(q2);
    uint64_t key = (chunk << 24) | colour;
    if (DEG) {
        const float4 *p4 = reinterpret_cast<const float4 *>(dc);
        float f[48];
#pragma unroll
        for (int c = 0; c < 12; c++) {
            const float4 v = p4[c];
            f[4 * c] = v.x; f[4 * c + 1] = v.y; f[4 * c + 2] = v.z; f[4 * c + 3] = v.w;
        }
        uint32_t L = 0;
#pragma unroll
        for (int e = 3; e < 48; e++) {       // bands 1..15; band k has degree floor(sqrt(k))
            const int k = e / 3, l = k >= 9 ? 3 : k >= 4 ? 2 : 1;
            const float x = opacity ? mu * f[e] : f[e];
            if (fabsf(x) > tau) L = L > (uint32_t)l ? L : (uint32_t)l;
        }
        key |= (uint64_t)L << (24 + 3 * grid_bits);
        atomicAdd(&cls[L], 1u);
    }
    keys[i] = key;
    vals[i] = (uint32_t)i;
    }
    if (DEG) {
        __syncthreads();
        if (threadIdx.x < 4 && cls[threadIdx.x]) atomicAdd(&class_count[threadIdx.x], cls[threadIdx.x]);
    }
}

// Digit counts of each wave tile; hist is tile-major: hist[tile][digit].
__global__ __launch_bounds__(256) void k_radix_hist(const uint64_t *keys, uint64_t n, int shift,
                                                    uint32_t ntiles, uint32_t *hist)
{
    __shared__ uint32_t cnt[4][kDigits];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int d = lane; d < kDigits; d += 64) cnt[w][d] = 0;
    __syncthreads();
    const uint32_t tile = blockIdx.x * 4 + w;
    if (tile < ntiles) {
        const uint64_t base = (uint64_t)tile * kTile;
        for (int it = 0; it < kWaveItems; it++) {
            uint64_t i = base + (uint64_t)it * 64 + lane;
            if (i < n) atomicAdd(&cnt[w][(keys[i] >> shift) & (kDigits - 1)], 1u);
        }
    }
    __syncthreads();
    if (tile < ntiles)
        for (int d = lane; d < kDigits; d += 64) hist[(uint64_t)tile * kDigits + d] = cnt[w][d];
}

// Column scan in two levels (grid: chunks x digit blocks).  Chunk level:
// thread (digit d, chunk c) turns its kChunkTiles counts into exclusive
// prefixes within the chunk (all loads issued before any store) and leaves
// the chunk total in ctot[c][d].
__global__ __launch_bounds__(256) void k_radix_chunkscan(uint32_t *hist, uint32_t ntiles, uint32_t *ctot)
{
    const int d = blockIdx.y * blockDim.x + threadIdx.x;
    const uint32_t t0 = blockIdx.x * kChunkTiles;
    uint32_t c[kChunkTiles];
#pragma unroll
    for (int j = 0; j < kChunkTiles; j++) c[j] = t0 + j < ntiles ? hist[(uint64_t)(t0 + j) * kDigits + d] : 0u;
    uint32_t run = 0;
#pragma unroll
    for (int j = 0; j < kChunkTiles; j++) {
        if (t0 + j < ntiles) hist[(uint64_t)(t0 + j) * kDigits + d] = run;
        run += c[j];
    }
    ctot[(uint64_t)blockIdx.x * kDigits + d] = run;
}

// Chunk totals level: per digit, exclusive prefixes over the chunks (in
// place, sixteen loads in flight) and the digit total.
__global__ __launch_bounds__(256) void k_radix_chunkprefix(uint32_t *ctot, uint32_t nchunks, uint32_t *total)
{
    const int d = blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t run = 0;
    for (uint32_t c0 = 0; c0 < nchunks; c0 += 16) {
        uint32_t c[16];
#pragma unroll
        for (int j = 0; j < 16; j++) c[j] = c0 + j < nchunks ? ctot[(uint64_t)(c0 + j) * kDigits + d] : 0u;
#pragma unroll
        for (int j = 0; j < 16; j++) {
            if (c0 + j < nchunks) ctot[(uint64_t)(c0 + j) * kDigits + d] = run;
            run += c[j];
        }
    }
    total[d] = run;
}

// Exclusive scan of the digit totals (one workgroup of 1024 threads, two
// digits each): pair sums, an inclusive scan over the 1024 pairs in LDS
// (ten doubling steps), then each pair's exclusive offsets.
__global__ __launch_bounds__(1024) void k_radix_digitscan(uint32_t *total)
{
    __shared__ uint32_t s[1024];
    const int t = threadIdx.x;
    const uint32_t a = total[2 * t], b = total[2 * t + 1];
    s[t] = a + b;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const uint32_t x = t >= off ? s[t - off] : 0u;
        __syncthreads();
        s[t] += x;
        __syncthreads();
    }
    const uint32_t before = s[t] - (a + b);
    total[2 * t] = before;
    total[2 * t + 1] = before + a;
}

// Stable scatter: each wave walks its tile in order; lanes with equal digits
// are ranked by lane id through ballots over the digit bits.
__global__ __launch_bounds__(256) void k_radix_scatter(const uint64_t *keys_in, const uint32_t *vals_in,
                                                       uint64_t n, int shift, uint32_t ntiles,
                                                       const uint32_t *hist, const uint32_t *chunk_base,
                                                       const uint32_t *digit_base,
                                                       uint64_t *keys_out, uint32_t *vals_out)
{
    __shared__ uint32_t ctr[4][kDigits];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const uint32_t tile = blockIdx.x * 4 + w;
    if (tile >= ntiles) return;   // whole wave leaves; no block barrier below
    const uint32_t *cb = chunk_base + (uint64_t)(tile / kChunkTiles) * kDigits;
    for (int d = lane; d < kDigits; d += 64)
        ctr[w][d] = hist[(uint64_t)tile * kDigits + d] + cb[d] + digit_base[d];
    __builtin_amdgcn_wave_barrier();
    const uint64_t base = (uint64_t)tile * kTile;
    const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    for (int it = 0; it < kWaveItems; it++) {
        uint64_t i = base + (uint64_t)it * 64 + lane;
        bool valid = i < n;
        uint64_t key = valid ? keys_in[i] : 0;
        uint32_t val = valid ? vals_in[i] : 0;
        uint32_t d = (uint32_t)(key >> shift) & (kDigits - 1);
        uint64_t peers = __ballot(valid);
        if (peers == 0) break;
#pragma unroll
        for (int b = 0; b < kDigitBits; b++) {
            uint64_t bal = __ballot((d >> b) & 1);
            peers &= ((d >> b) & 1) ? bal : ~bal;
        }
        if (valid) {
            uint32_t rank = (uint32_t)__popcll(peers & below);
            uint32_t off = ctr[w][d] + rank;
            keys_out[off] = key;
            vals_out[off] = val;
        }
        __builtin_amdgcn_wave_barrier();
        if (valid && (peers & below) == 0) ctr[w][d] += (uint32_t)__popcll(peers);
        __builtin_amdgcn_wave_barrier();
    }
}

// One thread per slot s < npad: quantise its 16 band vectors and place them
// by the arrangement (0: stream k, block s/16, texel zigzag(s%16); 1: block
// s, texel k; 2: stream k/4, block s/4, texel 4 (s%4) + k%4).
__global__ __launch_bounds__(256) void k_gather_pack(const float *sh, const float *opacity, const uint32_t *perm,
                                                     uint64_t n, uint64_t npad, uint32_t arrangement,
                                                     const RangeRec *r, uint32_t *tex)
{
    uint64_t s = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
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
    if (arrangement == 1) {            // one primitive per block: 64 contiguous bytes
        uint4 *d = reinterpret_cast<uint4 *>(tex + s * 16);
#pragma unroll
        for (int q = 0; q < 4; q++) d[q] = make_uint4(w[4 * q], w[4 * q + 1], w[4 * q + 2], w[4 * q + 3]);
    } else if (arrangement == 2) {     // four primitives per four blocks: one 16-byte row per stream
        const uint64_t bps = npad / 4;
#pragma unroll
        for (int g = 0; g < 4; g++)
            *reinterpret_cast<uint4 *>(tex + ((uint64_t)g * bps + (s >> 2)) * 16 + 4 * (s & 3)) =
                make_uint4(w[4 * g], w[4 * g + 1], w[4 * g + 2], w[4 * g + 3]);
    } else {
        const uint64_t nblk = npad / 16;
        const uint32_t j = (uint32_t)(s & 15);
        const uint32_t x = (j & 1u) | (((j >> 2) & 1u) << 1);
        const uint32_t y = ((j >> 1) & 1u) | (((j >> 3) & 1u) << 1);
        const uint64_t texel = (s >> 4) * 16 + 4 * y + x;
#pragma unroll
        for (int k = 0; k < 16; k++) tex[(uint64_t)k * nblk * 16 + texel] = w[k];
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
    size_t acc, keys_a, keys_b, vals_a, vals_b, hist, ctot, total, cov_state, cov_part, bytes;
};

Layout layout(uint64_t n)
{
    auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
    uint64_t ntiles = (n + kTile - 1) / kTile;
    Layout L;
    size_t o = 0;
    L.acc = o; o += al(64 * 4);
    L.keys_a = o; o += al(n * 8);
    L.keys_b = o; o += al(n * 8);
    L.vals_a = o; o += al(n * 4);
    L.vals_b = o; o += al(n * 4);
    L.hist = o; o += al(ntiles * kDigits * 4);
    L.ctot = o; o += al((ntiles + kChunkTiles - 1) / kChunkTiles * kDigits * 4);
    L.total = o; o += al(kDigits * 4);
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
void enqueue_range(const float *pos, const float *sh, const float *opacity, uint64_t n, uint32_t grid_bits,
                   uint32_t quantiser, const Layout &L, char *s, RangeRec *range_dev, hipStream_t st)
{
    uint32_t *acc = reinterpret_cast<uint32_t *>(s + L.acc);
    GSBC_LAUNCH("range_init", k_range_init, dim3(1), dim3(64), 0, st, acc);
    uint64_t want = (n * 12 + kRangeBlock - 1) / kRangeBlock;
    uint32_t nb = (uint32_t)std::min<uint64_t>(std::max<uint64_t>(want, 1), 2048);
    GSBC_LAUNCH("range_partial", k_range_partial, dim3(nb), dim3(kRangeBlock), 0, st,
                       reinterpret_cast<const float4 *>(sh), opacity, pos, n, acc);
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
    GSBC_LAUNCH("range_final", k_range_final, dim3(1), dim3(64), 0, st, acc, cov, grid_bits, range_dev);
}

// LSD radix sort of the keys in keys_a (values vals_a) over key_bits bits;
// the last pass writes the values to perm.
void enqueue_sort(uint64_t n, int key_bits, const Layout &L, char *s, uint32_t *perm, hipStream_t st)
{
    uint64_t *ka = reinterpret_cast<uint64_t *>(s + L.keys_a), *kb = reinterpret_cast<uint64_t *>(s + L.keys_b);
    uint32_t *va = reinterpret_cast<uint32_t *>(s + L.vals_a), *vb = reinterpret_cast<uint32_t *>(s + L.vals_b);
    uint32_t *hist = reinterpret_cast<uint32_t *>(s + L.hist), *total = reinterpret_cast<uint32_t *>(s + L.total);
    uint32_t *ctot = reinterpret_cast<uint32_t *>(s + L.ctot);
    const int passes = (key_bits + kDigitBits - 1) / kDigitBits;
    const uint32_t ntiles = (uint32_t)((n + kTile - 1) / kTile);
    const uint32_t nchunks = (ntiles + kChunkTiles - 1) / kChunkTiles;
    const uint32_t nblocks = (ntiles + 3) / 4;
    uint64_t *kin = ka, *kout = kb;
    uint32_t *vin = va, *vout = vb;
    for (int p = 0; p < passes; p++) {
        int shift = p * kDigitBits;
        uint32_t *vdst = (p == passes - 1) ? perm : vout;
        GSBC_LAUNCH("radix_hist", k_radix_hist, dim3(nblocks), dim3(256), 0, st, kin, n, shift, ntiles, hist);
        GSBC_LAUNCH("radix_colscan", k_radix_chunkscan, dim3(nchunks, kDigits / 256), dim3(256), 0, st, hist,
                           ntiles, ctot);
        GSBC_LAUNCH("radix_colscan", k_radix_chunkprefix, dim3(kDigits / 256), dim3(256), 0, st, ctot, nchunks, total);
        GSBC_LAUNCH("radix_digitscan", k_radix_digitscan, dim3(1), dim3(1024), 0, st, total);
        GSBC_LAUNCH("radix_scatter", k_radix_scatter, dim3(nblocks), dim3(256), 0, st, kin, vin, n, shift,
                           ntiles, hist, ctot, total, kout, vdst);
        std::swap(kin, kout);
        vin = vdst;
        vout = (vdst == va) ? vb : va;
    }
}

}  // namespace

hipError_t launch_reorder(const float *pos, const float *sh, const float *opacity, uint64_t n, uint32_t grid_bits,
                          uint32_t quantiser, bool identity, uint32_t arrangement, uint32_t *perm, uint8_t *textures,
                          void *scratch, RangeRec *range_dev, hipStream_t st)
{
    Layout L = layout(n);
    char *s = static_cast<char *>(scratch);
    enqueue_range(pos, sh, opacity, n, grid_bits, quantiser, L, s, range_dev, st);
    if (identity) {
        GSBC_LAUNCH("iota", k_iota, dim3((uint32_t)((n + 255) / 256)), dim3(256), 0, st, perm, n);
    } else {
        uint64_t *ka = reinterpret_cast<uint64_t *>(s + L.keys_a);
        uint32_t *va = reinterpret_cast<uint32_t *>(s + L.vals_a);
        GSBC_LAUNCH("keys", k_keys<false>, dim3((uint32_t)((n + 255) / 256)), dim3(256), 0, st, pos, sh, opacity, n,
                           grid_bits, range_dev, ka, va, 0.0f, (uint32_t *)nullptr);
        enqueue_sort(n, 24 + 3 * (int)grid_bits, L, s, perm, st);
    }
    const uint64_t npad = (n + 15) / 16 * 16;
    GSBC_LAUNCH("gather_pack", k_gather_pack, dim3((uint32_t)((npad + 255) / 256)), dim3(256), 0, st,
                       sh, opacity, perm, n, npad, arrangement, range_dev, reinterpret_cast<uint32_t *>(textures));
    return hipGetLastError();
}

hipError_t launch_degree_sort(const float *pos, const float *sh, const float *opacity, uint64_t n, uint32_t grid_bits,
                              uint32_t quantiser, float tau, uint32_t *perm, void *scratch, RangeRec *range_dev,
                              uint32_t *class_count, hipStream_t st)
{
    Layout L = layout(n);
    char *s = static_cast<char *>(scratch);
    enqueue_range(pos, sh, opacity, n, grid_bits, quantiser, L, s, range_dev, st);
    GSBC_LAUNCH("fill_count", k_zero4, dim3(1), dim3(64), 0, st, class_count);
    uint64_t *ka = reinterpret_cast<uint64_t *>(s + L.keys_a);
    uint32_t *va = reinterpret_cast<uint32_t *>(s + L.vals_a);
    GSBC_LAUNCH("keys_degree", k_keys<true>, dim3((uint32_t)((n + 255) / 256)), dim3(256), 0, st, pos, sh, opacity,
                       n, grid_bits, range_dev, ka, va, tau, class_count);
    enqueue_sort(n, 26 + 3 * (int)grid_bits, L, s, perm, st);
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
