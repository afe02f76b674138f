// decode.hip -- random-access decode and SH evaluation on gfx950.
//
//   decode       every block of every band back to 8-bit RGBA texels;
//   decode_eval  for each listed slot (one per lane): find its 16 band blocks
//                by index x block size (random access, Sec. I), decode its
//                texel from each, dequantise (vmin + q * delta), then for
//                every view direction in the workgroup's tile evaluate
//                c = sum_k Hhat_k Y_k(d) (Sec. II colour equation) with the
//                basis of the direction held in scalar registers.
#include "gsbc_internal.h"
#include "bc_format.h"

namespace gsbc {
namespace {

constexpr int kEvalBlock = 256;
constexpr int kDirTile = 128;

__device__ __forceinline__ uint32_t zigzag_texel(uint32_t j)
{
    uint32_t x = (j & 1u) | (((j >> 2) & 1u) << 1);
    uint32_t y = ((j >> 1) & 1u) | (((j >> 3) & 1u) << 1);
    return 4 * y + x;
}

__device__ __forceinline__ uint32_t band_texel(const uint8_t *blocks, const BandArgs &b, int k,
                                               uint64_t blk, int texel)
{
    const uint8_t *base = blocks + b.offset[k];
    if (b.format[k] == 1) {
        uint2 w = *reinterpret_cast<const uint2 *>(base + blk * 8);
        return bc1_texel(w.x, w.y, texel);
    }
    ulonglong2 w = *reinterpret_cast<const ulonglong2 *>(base + blk * 16);
    Blk128 q{w.x, w.y};
    return bc7_texel(q, texel);
}

__global__ __launch_bounds__(256) void k_decode(const uint8_t *blocks, BandArgs b, uint64_t nblk,
                                                uint32_t *tex)
{
    const uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= 16 * nblk) return;
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

__global__ __launch_bounds__(kEvalBlock) void k_decode_eval(const uint8_t *blocks, BandArgs b,
                                                            const uint32_t *prim_idx, uint64_t m,
                                                            uint64_t n_prims, const float *basis,
                                                            uint32_t n_dirs, float *out)
{
    const uint64_t j = (uint64_t)blockIdx.x * kEvalBlock + threadIdx.x;
    if (j >= m) return;
    const uint32_t s = prim_idx ? prim_idx[j] : (uint32_t)j;
    const uint32_t v0 = blockIdx.y * kDirTile;
    const uint32_t v1 = min(n_dirs, v0 + kDirTile);
    if (s >= n_prims) {   // not a slot of this scene: NaN, no block access
        for (uint32_t v = v0; v < v1; v++) {
            float *o = out + ((uint64_t)v * m + j) * 3;
            o[0] = o[1] = o[2] = __builtin_nanf("");
        }
        return;
    }
    const uint64_t blk = s >> 4;
    const int texel = (int)zigzag_texel(s & 15u);
    float H[16][3];
#pragma unroll
    for (int k = 0; k < 16; k++) {
        uint32_t px = band_texel(blocks, b, k, blk, texel);
        H[k][0] = fmaf((float)(px & 255), b.delta[k], b.vmin[k]);
        H[k][1] = fmaf((float)((px >> 8) & 255), b.delta[k], b.vmin[k]);
        H[k][2] = fmaf((float)((px >> 16) & 255), b.delta[k], b.vmin[k]);
    }
    for (uint32_t v = v0; v < v1; v++) {
        const float *Y = basis + 16 * (uint64_t)v;
        float r = H[0][0] * Y[0], g = H[0][1] * Y[0], bl = H[0][2] * Y[0];
#pragma unroll
        for (int k = 1; k < 16; k++) {
            r = fmaf(H[k][0], Y[k], r);
            g = fmaf(H[k][1], Y[k], g);
            bl = fmaf(H[k][2], Y[k], bl);
        }
        float *o = out + ((uint64_t)v * m + j) * 3;
        __builtin_nontemporal_store(r, o);
        __builtin_nontemporal_store(g, o + 1);
        __builtin_nontemporal_store(bl, o + 2);
    }
}

}  // namespace

hipError_t launch_decode(const uint8_t *blocks, const BandArgs &b, uint64_t nblk, uint8_t *textures,
                         hipStream_t st)
{
    uint64_t total = 16 * nblk;
    GSBC_LAUNCH("decode", k_decode, dim3((uint32_t)((total + 255) / 256)), dim3(256), 0, st, blocks, b, nblk,
                       reinterpret_cast<uint32_t *>(textures));
    return hipGetLastError();
}

hipError_t launch_decode_eval(const uint8_t *blocks, const BandArgs &b, uint64_t n_prims, const float *dirs,
                              uint32_t n_dirs, const uint32_t *prim_idx, uint64_t m, float *out,
                              float *basis, hipStream_t st)
{
    if (m == 0 || n_dirs == 0) return hipSuccess;
    GSBC_LAUNCH("sh_basis", k_sh_basis, dim3((n_dirs + 255) / 256), dim3(256), 0, st, dirs, n_dirs, basis);
    dim3 grid((uint32_t)((m + kEvalBlock - 1) / kEvalBlock), (n_dirs + kDirTile - 1) / kDirTile);
    GSBC_LAUNCH("decode_eval", k_decode_eval, grid, dim3(kEvalBlock), 0, st, blocks, b, prim_idx, m, n_prims, basis,
                       n_dirs, out);
    return hipGetLastError();
}

}  // namespace gsbc
