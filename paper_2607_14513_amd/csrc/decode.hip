// decode.hip -- random-access decode and SH evaluation on gfx950.
//
//   decode       every block of every band back to 8-bit RGBA texels;
//   decode_eval  for each listed slot (one per lane): find its 16 band blocks
//                by index x block size (random access, Sec. I), decode its
//                texel from each, dequantise (vmin + q * delta); then
//                c = sum_k Hhat_k Y_k(d) (Sec. II colour equation) for every
//                direction, computed as a K = 16 matrix product on the
//                matrix cores.
#include "gsbc_internal.h"
#include "bc_format.h"

#include <atomic>
#include <mutex>

namespace gsbc {
namespace {

constexpr int kEvalBlock = 256;

__device__ __forceinline__ uint32_t zigzag_texel(uint32_t j)
{
    uint32_t x = (j & 1u) | (((j >> 2) & 1u) << 1);
    uint32_t y = ((j >> 1) & 1u) | (((j >> 3) & 1u) << 1);
    return 4 * y + x;
}

template <class Lut = Bc7ConstLut>
__device__ __forceinline__ uint32_t band_texel(const uint8_t *blocks, const BandArgs &b, int k,
                                               uint64_t blk, int texel, const Lut &lut = Lut{})
{
    if (b.format[k] == GSBC_FMT_NONE) return 0u;   // a stream given 0 bits stores no blocks
    const uint8_t *base = blocks + b.offset[k];
    if (b.format[k] == 1) {
        uint2 w = *reinterpret_cast<const uint2 *>(base + blk * 8);
        return bc1_texel(w.x, w.y, texel);
    }
    ulonglong2 w = *reinterpret_cast<const ulonglong2 *>(base + blk * 16);
    Blk128 q{w.x, w.y};
    return bc7_texel(q, texel, lut);
}

// The band texels of slot s, each found through the arrangement:
// 0: stream k, block s/16, zigzag texel of s%16 (only the n_streams kept
// bands of a lower-degree scene; px[k] = 0 past them); 1: stream 0, block s,
// texel k; 2: stream k/4, block s/4, texel 4 (s%4) + k%4 (only the bands of
// the n_streams streams: one stream is Fig. SetupC, bands 0..3).
// One load per block, each decoded as it arrives (the fewest memory
// instructions, for gathers that issue little else):
template <int ARR, class Lut>
__device__ __forceinline__ void slot_texels_arr(const uint8_t *blocks, const BandArgs &b, uint32_t s, uint32_t px[16],
                                                const Lut &lut)
{
#pragma unroll
    for (int k = 0; k < 16; k++) {
        if (ARR == 1) px[k] = band_texel(blocks, b, 0, s, k, lut);
        else if (ARR == 2) px[k] = (uint32_t)(k >> 2) < b.n_streams
                                       ? band_texel(blocks, b, k >> 2, s >> 2, 4 * (int)(s & 3u) + (k & 3), lut) : 0u;
        else px[k] = (uint32_t)k < b.n_streams ? band_texel(blocks, b, k, s >> 4, (int)zigzag_texel(s & 15u), lut)
                                               : 0u;
    }
}

// or every block loaded before any is decoded, as two 8-byte halves (an
// 8-byte BC1 block loads its one half twice), so that the loads share one
// wait, and the BC7 tables read through `lut`:
template <int ARR, class Lut>
__device__ __forceinline__ void slot_texels_arr_batched(const uint8_t *blocks, const BandArgs &b, uint32_t s,
                                                        uint32_t px[16], const Lut &lut)
{
    uint2 lo[16], hi[16];
#pragma unroll
    for (int k = 0; k < 16; k++) {
        // stream of band k (a dropped band reads stream 0's block and ignores it)
        const int sk = ARR == 1 ? 0
                     : ARR == 2 ? ((uint32_t)(k >> 2) < b.n_streams ? (k >> 2) : 0)
                                : ((uint32_t)k < b.n_streams ? k : 0);
        const uint64_t blk = ARR == 1 ? s : ARR == 2 ? (s >> 2) : (s >> 4);
        const bool wide = b.format[sk] != 1;
        const uint8_t *q = blocks + b.offset[sk] + blk * (wide ? 16 : 8);
        // a stream given 0 bits stores no blocks: nothing to load
        const bool stored = b.format[sk] != GSBC_FMT_NONE;
        lo[k] = stored ? *reinterpret_cast<const uint2 *>(q) : make_uint2(0u, 0u);
        hi[k] = stored ? *reinterpret_cast<const uint2 *>(q + (wide ? 8 : 0)) : make_uint2(0u, 0u);
    }
#pragma unroll
    for (int k = 0; k < 16; k++) {
        const int sk = ARR == 1 ? 0 : ARR == 2 ? (k >> 2) : k;
        const int texel = ARR == 1 ? k : ARR == 2 ? 4 * (int)(s & 3u) + (k & 3) : (int)zigzag_texel(s & 15u);
        if ((ARR == 0 && (uint32_t)k >= b.n_streams) || (ARR == 2 && (uint32_t)(k >> 2) >= b.n_streams) ||
            b.format[sk] == GSBC_FMT_NONE)
            px[k] = 0u;
        else if (b.format[sk] == 1) px[k] = bc1_texel(lo[k].x, lo[k].y, texel);
        else px[k] = bc7_texel(Blk128{lo[k].x | (uint64_t)lo[k].y << 32, hi[k].x | (uint64_t)hi[k].y << 32}, texel, lut);
    }
}

// Dequantised coefficient of code q (low byte) in band k: vmin + q delta with
// the FP64 step delta = dhi + dlo (to 2^-48).  Each fused step rounds once,
// relative to its own result: vmin + q dhi, then + q dlo, so the value
// carries about one FP32 rounding of itself.  With delta rounded to FP32
// the step's error (2^-24 of the whole band range) would dominate whenever
// vmin and q delta nearly cancel.
__device__ __forceinline__ float dequant(uint32_t q, const BandArgs &b, int k)
{
    const float qf = (float)(q & 255u);
    return fmaf(qf, b.dlo[k], fmaf(qf, b.dhi[k], b.vmin[k]));
}

// Bands present in the scene: all 16, or the lowest n_streams (band
// arrangement) or 4 n_streams (quad arrangement, Fig. SetupC with one
// stream) of a lower-degree scene; the rest are exactly zero.
__device__ __forceinline__ uint32_t kept_bands(const BandArgs &b)
{
    return b.arrangement == 0 ? b.n_streams : b.arrangement == 2 ? 4u * b.n_streams : 16u;
}

// Band k has coded values: it is one of the scene's bands and its stream
// was not given 0 bits (band arrangement only); otherwise it is zero.
__device__ __forceinline__ bool band_coded(const BandArgs &b, int k)
{
    return (uint32_t)k < kept_bands(b) && !(b.arrangement == 0 && b.format[k] == GSBC_FMT_NONE);
}

// The BC7 tables come through lut: Bc7ConstLut (constant memory) or
// Bc7PackedLut (the workgroup's LDS copy, whose lookups wait on LDS
// instead of on a second memory round trip after the block's).
template <class Lut>
__device__ __forceinline__ void slot_texels(const uint8_t *blocks, const BandArgs &b, uint32_t s, uint32_t px[16],
                                            const Lut &lut)
{
    if (b.arrangement == 1) slot_texels_arr<1>(blocks, b, s, px, lut);
    else if (b.arrangement == 2) slot_texels_arr<2>(blocks, b, s, px, lut);
    else slot_texels_arr<0>(blocks, b, s, px, lut);
}

template <class Lut>
__device__ __forceinline__ void slot_texels_batched(const uint8_t *blocks, const BandArgs &b, uint32_t s,
                                                    uint32_t px[16], const Lut &lut)
{
    if (b.arrangement == 1) slot_texels_arr_batched<1>(blocks, b, s, px, lut);
    else if (b.arrangement == 2) slot_texels_arr_batched<2>(blocks, b, s, px, lut);
    else slot_texels_arr_batched<0>(blocks, b, s, px, lut);
}

__global__ __launch_bounds__(256) void k_decode(const uint8_t *blocks, BandArgs b, uint64_t nblk,
                                                uint32_t *tex)
{
    const uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= (uint64_t)b.n_streams * nblk) return;
    const int k = (int)(g / nblk);
    const uint64_t blk = g % nblk;
    uint32_t out[16];
#pragma unroll
    for (int i = 0; i < 16; i++) out[i] = band_texel(blocks, b, k, blk, i);
    uint4 *dst = reinterpret_cast<uint4 *>(tex + g * 16);
#pragma unroll
    for (int q = 0; q < 4; q++) dst[q] = make_uint4(out[4 * q], out[4 * q + 1], out[4 * q + 2], out[4 * q + 3]);
}

// Real SH basis of degree <= 3 in FP32 (3DGS sign convention, k = l^2+l+m).
__global__ void k_sh_basis(const float *dirs, uint32_t n, float *basis)
{
    const uint32_t v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    const float x = dirs[3 * v], y = dirs[3 * v + 1], z = dirs[3 * v + 2];
    const float c0 = 0.28209479177387814f, c1 = 0.4886025119029199f;
    const float c2a = 1.0925484305920792f, c2b = 0.31539156525252005f, c2c = 0.5462742152960396f;
    const float c3a = 0.5900435899266435f, c3b = 2.890611442640554f, c3c = 0.4570457994644658f;
    const float c3d = 0.3731763325901154f, c3e = 1.445305721320277f;
    const float xx = x * x, yy = y * y, zz = z * z;
    float *Y = basis + 16 * (uint64_t)v;
    Y[0] = c0;
    Y[1] = -c1 * y;
    Y[2] = c1 * z;
    Y[3] = -c1 * x;
    Y[4] = c2a * x * y;
    Y[5] = -c2a * y * z;
    Y[6] = c2b * (2.0f * zz - xx - yy);
    Y[7] = -c2a * x * z;
    Y[8] = c2c * (xx - yy);
    Y[9] = -c3a * y * (3.0f * xx - yy);
    Y[10] = c3b * x * y * z;
    Y[11] = -c3c * y * (4.0f * zz - xx - yy);
    Y[12] = c3d * z * (2.0f * zz - 3.0f * xx - 3.0f * yy);
    Y[13] = -c3c * x * (4.0f * zz - xx - yy);
    Y[14] = c3e * z * (xx - yy);
    Y[15] = -c3a * x * (xx - 3.0f * yy);
}

// decode_eval as a contraction: out[v][3j+c] = sum_k Y[v][k] * H[j][k][c], a
// (directions x 16) by (16 x 3m) product with K = 16.  A workgroup decodes 256
// slots once (one lane each) into an LDS matrix Hm[k][3*slot + c], then its
// four waves compute 16 x 16 output tiles with v_mfma_f32_16x16x4f32 (four
// K-steps each), holding their B operands in registers across the direction
// tiles.  Lane layout of that instruction: lane l supplies A[l%16][l/16] and
// B[l/16][l%16] and receives D[4*(l/16) + r][l%16], r = 0..3.
typedef float floatx4 __attribute__((ext_vector_type(4)));
constexpr int kSlots = 256;                 // slots per workgroup
constexpr int kCols = 3 * kSlots;           // output floats per direction
constexpr int kDirChunk = 256;              // directions per workgroup (grid.y); their basis rows sit in LDS
constexpr int kBasStride = 17;              // padded basis row in LDS
constexpr int kStageStride = 196;           // padded staging row (192 columns per wave)
// SR staging rows per wave: 16 (all rows of a 16-direction tile at once;
// two workgroups per CU) or 8 (the tile in two halves; 49.7 KB of LDS and at
// most 168 VGPRs, so three workgroups per CU).  Three hide the decode
// prologue better and win when a workgroup has few directions to write; at
// hundreds of directions the two-workgroup form writes faster.
template <int SR>
constexpr int lds_floats()
{
    return kDirChunk * kBasStride + 4 * SR * kStageStride > 16 * kCols + kBc7LutWords
               ? kDirChunk * kBasStride + 4 * SR * kStageStride
               : 16 * kCols + kBc7LutWords;
}

template <int SR>
__device__ __forceinline__ void decode_eval_body(const uint8_t *blocks, const BandArgs &b, const uint32_t *prim_idx,
                                                 uint64_t m, uint64_t n_prims, const float *basis, uint32_t n_dirs,
                                                 float *out)
{
    __shared__ __align__(16) float lds[lds_floats<SR>()];
    float(*Hm)[kCols] = reinterpret_cast<float(*)[kCols]>(lds);
    const int t = threadIdx.x, lane = t & 63;
    const int wave = __builtin_amdgcn_readfirstlane(t >> 6);   // wave-uniform: row addresses stay scalar
    const uint64_t j0 = (uint64_t)blockIdx.x * kSlots;
    // ---- decode: lane t -> slot j0 + t
    {
        const uint64_t j = j0 + t;
        const uint32_t s = j < m ? (prim_idx ? prim_idx[j] : (uint32_t)j) : 0u;
        // BC7 partition tables for the decode, in the LDS past Hm (their
        // loads issued with the slot's index load)
        uint32_t *lutw = reinterpret_cast<uint32_t *>(lds + 16 * kCols);
        if (t < kBc7LutWords) lutw[t] = bc7_lut_word(t);
        __syncthreads();
        float h[16][3];
        if (j < m) {
            if (s < n_prims) {
                uint32_t px[16];
                slot_texels_batched(blocks, b, s, px, Bc7PackedLut{lutw});
#pragma unroll
                for (int k = 0; k < 16; k++) {
                    const bool kept = band_coded(b, k);
#pragma unroll
                    for (int c = 0; c < 3; c++) h[k][c] = kept ? dequant(px[k] >> (8 * c), b, k) : 0.0f;
                }
            } else {   // not a slot of this scene: NaN colours, no block access
#pragma unroll
                for (int k = 0; k < 16; k++) h[k][0] = h[k][1] = h[k][2] = __builtin_nanf("");
            }
        } else {
#pragma unroll
            for (int k = 0; k < 16; k++) h[k][0] = h[k][1] = h[k][2] = 0.0f;
        }
#pragma unroll
        for (int k = 0; k < 16; k++) {
            Hm[k][3 * t] = h[k][0];
            Hm[k][3 * t + 1] = h[k][1];
            Hm[k][3 * t + 2] = h[k][2];
        }
    }
    __syncthreads();
    // ---- B operands of this wave's 12 column tiles, held across directions
    const int row = lane >> 4, col = lane & 15;
    float bop[12][4];
#pragma unroll
    for (int q = 0; q < 12; q++) {
        const int c0 = 16 * (wave * 12 + q);
#pragma unroll
        for (int s = 0; s < 4; s++) bop[q][s] = Hm[4 * s + row][c0 + col];
    }
    const uint64_t cols_valid = (m - j0 < (uint64_t)kSlots ? m - j0 : (uint64_t)kSlots) * 3;
    const uint64_t row_stride = 3 * m;
    // rows start 16-byte aligned (output base aligned, row length a multiple of 4 floats)
    const bool rows16 = (row_stride & 3) == 0 && (reinterpret_cast<uintptr_t>(out) & 15) == 0;
    const uint32_t wcol0 = 16 * 12 * wave;                  // this wave's first column
    float *obase = out + 3 * j0 + wcol0;
    // Hm is dead once every wave holds its B operands.  It then holds this
    // workgroup's basis rows (the A operands) and each wave's staging tile,
    // so the direction loop issues no vector-memory loads: on this ISA one
    // counter tracks loads and stores together, and waiting for a load would
    // also wait for every store issued before it.
    float *bas = lds;                                                  // [kDirChunk][kBasStride]
    float(*stage)[kStageStride] = reinterpret_cast<float(*)[kStageStride]>(lds + kDirChunk * kBasStride) + SR * wave;
    const uint32_t vc0 = blockIdx.y * kDirChunk;
    const uint32_t v_end = min(n_dirs, vc0 + kDirChunk);
    __syncthreads();           // every wave holds its B operands
    for (uint32_t e = t; e < kDirChunk * 16; e += kEvalBlock) {
        const uint32_t v = vc0 + e / 16;
        bas[(e / 16) * kBasStride + e % 16] = v < v_end ? basis[16 * (uint64_t)v + e % 16] : 0.0f;
    }
    __syncthreads();
    if constexpr (SR == 16) {
        for (uint32_t v0 = vc0; v0 < v_end; v0 += 16) {
            // A operand: Y[v0 + col][4s + row]
            float aop[4];
    #pragma unroll
            for (int s = 0; s < 4; s++) aop[s] = bas[(v0 - vc0 + col) * kBasStride + 4 * s + row];
            // all 12 tiles staged (16 rows x 192 columns), then each row leaves as
            // three back-to-back stores of 64 floats: 768 contiguous bytes
    #pragma unroll
            for (int q = 0; q < 12; q++) {
                floatx4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
    #pragma unroll
                for (int s = 0; s < 4; s++) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(aop[s], bop[q][s], acc, 0, 0, 0);
    #pragma unroll
                for (int r = 0; r < 4; r++) stage[4 * row + r][16 * q + col] = acc[r];
            }
            bool cok[3];
    #pragma unroll
            for (int h = 0; h < 3; h++) cok[h] = wcol0 + 64 * h + lane < cols_valid;
            float *o = obase + v0 * row_stride + lane;
            if (v0 + 16 <= v_end && wcol0 + 192 <= cols_valid && rows16) {
                // whole rows, every column valid, 16-byte aligned: lanes 0..47
                // store 4 consecutive columns each, one instruction per row
                if (lane < 48) {
                    floatx4 *o4 = reinterpret_cast<floatx4 *>(obase + v0 * row_stride) + lane;
    #pragma unroll
                    for (int half = 0; half < 2; half++) {
                        floatx4 x[8];
    #pragma unroll
                        for (int rr = 0; rr < 8; rr++)
                            x[rr] = *reinterpret_cast<const floatx4 *>(&stage[8 * half + rr][4 * lane]);
    #pragma unroll
                        for (int rr = 0; rr < 8; rr++)
                            __builtin_nontemporal_store(x[rr], o4 + (8 * half + rr) * (row_stride / 4));
                    }
                }
            } else if (v0 + 16 <= v_end) {
    #pragma unroll
                for (int half = 0; half < 2; half++) {
                    float x[8][3];
    #pragma unroll
                    for (int rr = 0; rr < 8; rr++)
    #pragma unroll
                        for (int h = 0; h < 3; h++) x[rr][h] = stage[8 * half + rr][64 * h + lane];
    #pragma unroll
                    for (int rr = 0; rr < 8; rr++)
    #pragma unroll
                        for (int h = 0; h < 3; h++)
                            if (cok[h]) __builtin_nontemporal_store(x[rr][h], o + (8 * half + rr) * row_stride + 64 * h);
                }
            } else {
                for (uint32_t rr = 0; v0 + rr < v_end; rr++)
    #pragma unroll
                    for (int h = 0; h < 3; h++)
                        if (cok[h]) __builtin_nontemporal_store(stage[rr][64 * h + lane], o + rr * row_stride + 64 * h);
            }
            // The four waves start each direction tile together, so their
            // 768-byte pieces of a row leave close in time (one 3 KB stretch
            // of it): a bare s_barrier, which waits on no memory counter.
            // Every wave runs the same iterations (v0 and v_end are uniform
            // over the workgroup); 7.27 -> 7.14 ms at 3,145,728 x 1,024.
            __builtin_amdgcn_s_barrier();
        }
    } else {
        for (uint32_t v0 = vc0; v0 < v_end; v0 += 16) {
            float aop[4];
    #pragma unroll
            for (int s = 0; s < 4; s++) aop[s] = bas[(v0 - vc0 + col) * kBasStride + 4 * s + row];
            floatx4 acc[12];
    #pragma unroll
            for (int q = 0; q < 12; q++) {
                acc[q] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
    #pragma unroll
                for (int s = 0; s < 4; s++) acc[q] = __builtin_amdgcn_mfma_f32_16x16x4f32(aop[s], bop[q][s], acc[q], 0, 0, 0);
            }
            bool cok[3];
    #pragma unroll
            for (int h = 0; h < 3; h++) cok[h] = wcol0 + 64 * h + lane < cols_valid;
            const bool fast = v0 + 16 <= v_end && wcol0 + 192 <= cols_valid && rows16;
            // half hr stages rows 4 i + 2 hr + e (i = 0..3, e = 0, 1) at staging row 2 i + e
    #pragma unroll
            for (int hr = 0; hr < 2; hr++) {
    #pragma unroll
                for (int q = 0; q < 12; q++)
    #pragma unroll
                    for (int e = 0; e < 2; e++) stage[2 * row + e][16 * q + col] = acc[q][2 * hr + e];
                if (fast) {
                    if (lane < 48) {
                        floatx4 *o4 = reinterpret_cast<floatx4 *>(obase + (v0 + 2 * hr) * row_stride) + lane;
    #pragma unroll
                        for (int g = 0; g < 8; g += 4) {
                            floatx4 x[4];
    #pragma unroll
                            for (int e = 0; e < 4; e++) x[e] = *reinterpret_cast<const floatx4 *>(&stage[g + e][4 * lane]);
    #pragma unroll
                            for (int e = 0; e < 4; e++)
                                __builtin_nontemporal_store(x[e], o4 + (4 * ((g + e) >> 1) + ((g + e) & 1)) * (row_stride / 4));
                        }
                    }
                } else {
                    float *o = obase + v0 * row_stride + lane;
                    for (int sr = 0; sr < 8; sr++) {
                        const uint32_t dv = 4 * (sr >> 1) + 2 * hr + (sr & 1);
                        if (v0 + dv < v_end)
    #pragma unroll
                            for (int h = 0; h < 3; h++)
                                if (cok[h]) __builtin_nontemporal_store(stage[sr][64 * h + lane], o + dv * row_stride + 64 * h);
                    }
                }
            }
        }
    }
}

__global__ __launch_bounds__(kEvalBlock) void k_decode_eval(const uint8_t *blocks, BandArgs b,
                                                            const uint32_t *prim_idx, uint64_t m,
                                                            uint64_t n_prims, const float *basis,
                                                            uint32_t n_dirs, float *out)
{
    decode_eval_body<16>(blocks, b, prim_idx, m, n_prims, basis, n_dirs, out);
}

__global__ __launch_bounds__(kEvalBlock) __attribute__((amdgpu_waves_per_eu(3))) void k_decode_eval_small(
    const uint8_t *blocks, BandArgs b, const uint32_t *prim_idx, uint64_t m, uint64_t n_prims, const float *basis,
    uint32_t n_dirs, float *out)
{
    decode_eval_body<8>(blocks, b, prim_idx, m, n_prims, basis, n_dirs, out);
}

// Colour of slot s seen from view position f (Sec. II, c(f) = H w(f - p)):
// its primitive's position through perm, d = (f - p)/|f - p| (zero when
// f = p), the 16 basis functions dotted with the decoded, dequantised texels
// (FP32, k order).  s must be below the scene's n_prims.
template <class Lut>
__device__ __forceinline__ void view_colour(const uint8_t *blocks, const BandArgs &b, uint32_t s, const float *pos,
                                            const uint32_t *perm, float fx, float fy, float fz, float c[3],
                                            const Lut &lut)
{
    const uint64_t pi = perm[s];
    float x = fx - pos[3 * pi], y = fy - pos[3 * pi + 1], z = fz - pos[3 * pi + 2];
    const float r = sqrtf(x * x + y * y + z * z);
    const float inv = r > 0.0f ? 1.0f / r : 0.0f;
    x *= inv;
    y *= inv;
    z *= inv;
    const float c0 = 0.28209479177387814f, c1 = 0.4886025119029199f;
    const float c2a = 1.0925484305920792f, c2b = 0.31539156525252005f, c2c = 0.5462742152960396f;
    const float c3a = 0.5900435899266435f, c3b = 2.890611442640554f, c3c = 0.4570457994644658f;
    const float c3d = 0.3731763325901154f, c3e = 1.445305721320277f;
    const float xx = x * x, yy = y * y, zz = z * z;
    float Y[16];
    Y[0] = c0;
    Y[1] = -c1 * y;
    Y[2] = c1 * z;
    Y[3] = -c1 * x;
    Y[4] = c2a * x * y;
    Y[5] = -c2a * y * z;
    Y[6] = c2b * (2.0f * zz - xx - yy);
    Y[7] = -c2a * x * z;
    Y[8] = c2c * (xx - yy);
    Y[9] = -c3a * y * (3.0f * xx - yy);
    Y[10] = c3b * x * y * z;
    Y[11] = -c3c * y * (4.0f * zz - xx - yy);
    Y[12] = c3d * z * (2.0f * zz - 3.0f * xx - 3.0f * yy);
    Y[13] = -c3c * x * (4.0f * zz - xx - yy);
    Y[14] = c3e * z * (xx - yy);
    Y[15] = -c3a * x * (xx - 3.0f * yy);
    uint32_t px[16];
    slot_texels(blocks, b, s, px, lut);
    c[0] = c[1] = c[2] = 0.0f;
#pragma unroll
    for (int k = 0; k < 16; k++) {
        if (band_coded(b, k)) {
#pragma unroll
            for (int ch = 0; ch < 3; ch++) c[ch] = fmaf(dequant(px[k] >> (8 * ch), b, k), Y[k], c[ch]);
        }
    }
}

// One lane per listed slot; out-of-range slot ids give NaN.  The BC7
// tables are read from the workgroup's LDS copy (the colour stage keeps
// them in constant memory: there the LDS copy measured slower).
__global__ __launch_bounds__(256) void k_decode_eval_view(const uint8_t *blocks, BandArgs b, const uint32_t *prim_idx,
                                                          uint64_t m, uint64_t n_prims, const float *pos,
                                                          const uint32_t *perm, float fx, float fy, float fz,
                                                          float *out)
{
    __shared__ uint32_t s_lut[kBc7LutWords];
    if (threadIdx.x < kBc7LutWords) s_lut[threadIdx.x] = bc7_lut_word(threadIdx.x);
    __syncthreads();
    const uint64_t j = (uint64_t)blockIdx.x * 256 + threadIdx.x;
    if (j >= m) return;
    const uint32_t s = prim_idx ? prim_idx[j] : (uint32_t)j;
    float c[3] = {__builtin_nanf(""), __builtin_nanf(""), __builtin_nanf("")};
    if (s < n_prims) view_colour(blocks, b, s, pos, perm, fx, fy, fz, c, Bc7PackedLut{s_lut});
    out[3 * j] = c[0];
    out[3 * j + 1] = c[1];
    out[3 * j + 2] = c[2];
}

// Tiles by decreasing list length (bucketed by floor(log2 L), empty tiles
// last): one workgroup counts, scans and scatters.  The blend takes tiles
// in this order so that the longest lists start first instead of ending
// the launch alone; the order within a bucket does not matter (each tile is
// computed on its own).
__global__ __launch_bounds__(1024) void k_tile_order(const uint32_t *tile_start, uint64_t list_len, uint32_t tiles,
                                                    uint32_t *order)
{
    __shared__ uint32_t cnt[33];
    const uint32_t t = threadIdx.x;
    if (t < 33) cnt[t] = 0u;
    __syncthreads();
    auto key = [&](uint32_t i) {
        const uint64_t e = min((uint64_t)tile_start[i + 1], list_len), s0 = min((uint64_t)tile_start[i], e);
        const uint64_t L = e - s0;
        return L == 0 ? 32u : (uint32_t)__clzll(L) - 32u;   // 31 - floor(log2 L) for L below 2^32
    };
    for (uint32_t i = t; i < tiles; i += 1024) atomicAdd(&cnt[key(i)], 1u);
    __syncthreads();
    if (t == 0) {
        uint32_t run = 0;
        for (int k = 0; k < 33; k++) {
            const uint32_t c = cnt[k];
            cnt[k] = run;
            run += c;
        }
    }
    __syncthreads();
    for (uint32_t i = t; i < tiles; i += 1024) order[atomicAdd(&cnt[key(i)], 1u)] = i;
}

// Colour stage of a tile rasteriser (Sec. II, eq. preblend with the
// premultiplied coefficients of eq. premult), one workgroup per 16x16 tile,
// one lane per pixel.  The tile's list is taken 256 entries at a time: lane t
// decodes entry t's colour c~ = Htilde w(f - p) from the bitstreams (no
// colour buffer in HBM) and stages it in LDS with the primitive's footprint
// and opacity mu, the conic turned into base-2 exponent coefficients
// (A, B, C) = -log2(e) (a/2, b, c/2); then every pixel walks the staged
// entries front to back: g = 2^(A dx^2 + B dx dy + C dy^2) at its centre,
// a += (g T) c~, T -= (T mu) g.  A list entry past n_prims gives NaN colour.
// Once every pixel of a wave (or of the tile) has T exactly 0, the remaining
// entries change nothing (g T = 0 and T stays 0 for finite colours) and are
// skipped.
__global__ __launch_bounds__(256) void k_blend_tiles(const uint8_t *blocks, BandArgs b, uint64_t n_prims,
                                                     const float *pos, const uint32_t *perm, float fx, float fy,
                                                     float fz, const float *mu, const float *foot,
                                                     const uint32_t *tile_start, const uint32_t *list,
                                                     uint64_t list_len, const uint32_t *order, uint32_t tiles_x,
                                                     const float *colours, float *image, float *trans)
{
    // per staged entry: mean x, mean y, A, B | C, mu, colour r, g | colour b
    // (rows of 12 floats: three 16-byte LDS reads per entry, all lanes
    // reading the same row)
    __shared__ __align__(16) float s_par[256][12];
    const uint32_t t = threadIdx.x, tile = order[blockIdx.x];
    const uint32_t tx = tile % tiles_x, ty = tile / tiles_x;
    const float x = (float)(16 * tx + (t & 15u)) + 0.5f, y = (float)(16 * ty + (t >> 4)) + 0.5f;
    const uint64_t b1 = min((uint64_t)tile_start[tile + 1], list_len);
    const uint64_t b0 = min((uint64_t)tile_start[tile], b1);
    constexpr float kLog2e = 1.4426950408889634f;
    float a0 = 0.0f, a1 = 0.0f, a2 = 0.0f, T = 1.0f;
    for (uint64_t base = b0; base < b1; base += 256) {
        const uint64_t e = base + t;
        if (e < b1) {
            const uint32_t s = list[e];
            float c[3] = {__builtin_nanf(""), __builtin_nanf(""), __builtin_nanf("")};
            uint64_t i = 0;
            if (s < n_prims) {
                if (colours) {   // the colour computed beforehand, once per primitive
                    c[0] = colours[3 * (uint64_t)s];
                    c[1] = colours[3 * (uint64_t)s + 1];
                    c[2] = colours[3 * (uint64_t)s + 2];
                } else {
                    view_colour(blocks, b, s, pos, perm, fx, fy, fz, c, Bc7ConstLut{});
                }
                i = perm[s];
            }
            s_par[t][0] = foot[5 * i];
            s_par[t][1] = foot[5 * i + 1];
            s_par[t][2] = -0.5f * kLog2e * foot[5 * i + 2];
            s_par[t][3] = -kLog2e * foot[5 * i + 3];
            s_par[t][4] = -0.5f * kLog2e * foot[5 * i + 4];
            s_par[t][5] = mu[i];
            s_par[t][6] = c[0];
            s_par[t][7] = c[1];
            s_par[t][8] = c[2];
        }
        __syncthreads();
        const uint32_t cnt = (uint32_t)(b1 - base < 256 ? b1 - base : 256);
        for (uint32_t j0 = 0; j0 < cnt; j0 += 32) {
            if (__all(T == 0.0f)) break;   // this wave is done for the chunk
            const uint32_t j1 = j0 + 32 < cnt ? j0 + 32 : cnt;
            // four entries' reads in flight at once
#pragma unroll 4
            for (uint32_t j = j0; j < j1; j++) {
                const float4 pa = *reinterpret_cast<const float4 *>(&s_par[j][0]);
                const float4 pb = *reinterpret_cast<const float4 *>(&s_par[j][4]);
                const float4 pc = *reinterpret_cast<const float4 *>(&s_par[j][8]);
                const float dx = x - pa.x, dy = y - pa.y;
                const float ex = fmaf(dx, fmaf(pa.z, dx, pa.w * dy), pb.x * dy * dy);
                const float g = __builtin_amdgcn_exp2f(ex);
                const float w = g * T, m = T * pb.y;
                a0 = fmaf(w, pb.z, a0);
                a1 = fmaf(w, pb.w, a1);
                a2 = fmaf(w, pc.x, a2);
                T = fmaf(-m, g, T);
            }
        }
        if (__syncthreads_and(T == 0.0f)) break;   // every pixel of the tile is covered
    }
    const uint64_t W = 16 * (uint64_t)tiles_x;
    const uint64_t o = (16 * (uint64_t)ty + (t >> 4)) * W + 16 * tx + (t & 15u);
    image[3 * o] = a0;
    image[3 * o + 1] = a1;
    image[3 * o + 2] = a2;
    if (trans) trans[o] = T;
}

}  // namespace

hipError_t launch_blend_tiles(const uint8_t *blocks, const BandArgs &b, uint64_t n_prims, const float *pos,
                              const uint32_t *perm, const float view[3], const float *mu, const float *foot,
                              const uint32_t *tile_start, const uint32_t *list, uint64_t list_len, uint32_t tiles_x,
                              uint32_t tiles_y, const float *colours, float *image, float *trans, uint32_t *order,
                              hipStream_t st)
{
    const uint64_t tiles = (uint64_t)tiles_x * tiles_y;
    if (tiles == 0) return hipSuccess;
    GSBC_LAUNCH("tile_order", k_tile_order, dim3(1), dim3(1024), 0, st, tile_start, list_len, (uint32_t)tiles, order);
    GSBC_LAUNCH("blend_tiles", k_blend_tiles, dim3((uint32_t)tiles), dim3(256), 0, st, blocks, b, n_prims, pos, perm,
                view[0], view[1], view[2], mu, foot, tile_start, list, list_len, order, tiles_x, colours, image, trans);
    return hipGetLastError();
}

hipError_t launch_decode_eval_view(const uint8_t *blocks, const BandArgs &b, uint64_t n_prims, const float *pos,
                                   const uint32_t *perm, const float view[3], const uint32_t *prim_idx, uint64_t m,
                                   float *out, hipStream_t st)
{
    if (m == 0) return hipSuccess;
    GSBC_LAUNCH("decode_eval_view", k_decode_eval_view, dim3((uint32_t)((m + 255) / 256)), dim3(256), 0, st, blocks, b,
                prim_idx, m, n_prims, pos, perm, view[0], view[1], view[2], out);
    return hipGetLastError();
}

hipError_t launch_decode(const uint8_t *blocks, const BandArgs &b, uint64_t nblk, uint8_t *textures,
                         hipStream_t st)
{
    uint64_t total = (uint64_t)b.n_streams * nblk;
    GSBC_LAUNCH("decode", k_decode, dim3((uint32_t)((total + 255) / 256)), dim3(256), 0, st, blocks, b, nblk,
                       reinterpret_cast<uint32_t *>(textures));
    return hipGetLastError();
}

// ---- scratch of the allocation-free decode_eval
// The basis rows (16 floats per direction) of gsbc_decode_eval_noalloc live
// in this file-scope device array: the library holds one copy on each GPU it
// runs on until the process ends.  Host code never uses the array's name as
// an address (on the host it is only a stand-in for the symbol); each
// device's address is looked up once, with that device current, and kept.
static __device__ __align__(256) float scratch[kStaticScratchDirs * 16];
static std::atomic<float *> g_scratch_ptr[kMaxDevices];
static std::mutex g_scratch_lock;

hipError_t init_static_scratch(int device)
{
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> guard(g_scratch_lock);
    if (g_scratch_ptr[device].load()) return hipSuccess;
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[device].store(static_cast<float *>(ptr));
    return hipSuccess;
}

float *static_scratch(int device)
{
    return device >= 0 && device < kMaxDevices ? g_scratch_ptr[device].load() : nullptr;
}

hipError_t launch_decode_eval(const uint8_t *blocks, const BandArgs &b, uint64_t n_prims, const float *dirs,
                              uint32_t n_dirs, const uint32_t *prim_idx, uint64_t m, float *out,
                              float *basis, hipStream_t st)
{
    if (m == 0 || n_dirs == 0) return hipSuccess;
    GSBC_LAUNCH("sh_basis", k_sh_basis, dim3((n_dirs + 255) / 256), dim3(256), 0, st, dirs, n_dirs, basis);
    dim3 grid((uint32_t)((m + kSlots - 1) / kSlots), (n_dirs + kDirChunk - 1) / kDirChunk);
    if (n_dirs <= (uint32_t)kDirChunk)   // one direction chunk per workgroup: three workgroups per CU
        GSBC_LAUNCH("decode_eval", k_decode_eval_small, grid, dim3(kEvalBlock), 0, st, blocks, b, prim_idx, m,
                    n_prims, basis, n_dirs, out);
    else
        GSBC_LAUNCH("decode_eval", k_decode_eval, grid, dim3(kEvalBlock), 0, st, blocks, b, prim_idx, m, n_prims,
                    basis, n_dirs, out);
    return hipGetLastError();
}

}  // namespace gsbc
