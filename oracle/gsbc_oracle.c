/*
 * gsbc_oracle.c -- plain CPU oracle for the 3DGS spherical-harmonic BC1/BC7
 * coding path ("Compression of 3D Gaussian Splatting Data Using GPU-friendly
 * Graphics Texture Coding", Said & Rauwendaal).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously-correct
 * reference that the GPU library is checked against.  Only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark may load it.  It
 * shares no code, header, table or generator with the GPU library: every
 * table below (BC7 partitions, anchors, weights, SH constants) is written out
 * here on its own, and every step is a direct loop over its definition.
 *
 * Precision: the quantiser, keys and all encoder decisions are integer or an
 * FP32 expression fixed operation by operation (compiled with
 * -ffp-contract=off); the SH evaluation is FP64.
 *
 * Sections follow the paper:
 *   Q  band range + 8-bit quantisation          (Sec. V-A, experimental setup)
 *   K  colour key by RGB bit interleaving        (Sec. III-C, Fig. Bit4Scan)
 *      and spatial chunk                         (Sec. III-C, last paragraph)
 *   S  stable ascending sort                     (Sec. III-C, step 2)
 *   B  16 primitives of one band -> 4x4 block    (Sec. IV-B, Fig. SetupD),
 *      zigzag texel order                        (Sec. III-C, Fig. ZigZagScan);
 *      one primitive -> one block                (Fig. SetupA);
 *      four primitives -> four blocks            (Fig. SetupB)
 *   D1 BC1 decode, D2 BC7 decode                 (Sec. III-B, BC formats)
 *   E1 BC1 encode, E2 BC7 encode                 (Sec. III-A BTC palette and
 *      index rule; endpoint search is this project's deterministic definition)
 *   R  per-band format choice at a fixed rate    (Sec. IV-B), with or
 *      without a 0-bit option that drops a band
 *   H  SH colour c = H w(d)                      (Sec. II, colour equation)
 *   C  front-to-back blend of premultiplied      (Sec. II, eqs. blend,
 *      colours over per-tile lists                preblend and premult)
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>

#define EXPORT __attribute__((visibility("default")))

/* ======================================================================
 * Q -- per-band range and 8-bit quantisation (Sec. V-A: SH are scaled per
 * coefficient and quantised to 0..255; the range here is each band's
 * min/max over all primitives and RGB channels).
 * sh layout: float[n][16][3].
 * ====================================================================== */
EXPORT void ref_band_range(const float *sh, uint64_t n, float *vmin, float *vmax)
{
    for (int k = 0; k < 16; k++) {
        float lo = INFINITY, hi = -INFINITY;
        for (uint64_t i = 0; i < n; i++)
            for (int c = 0; c < 3; c++) {
                float x = sh[(i * 16 + k) * 3 + c];
                if (x < lo) lo = x;
                if (x > hi) hi = x;
            }
        /* the endpoints are values: a zero is stored as +0 */
        vmin[k] = lo == 0.0f ? 0.0f : lo;
        vmax[k] = hi == 0.0f ? 0.0f : hi;
    }
}

EXPORT void ref_pos_aabb(const float *pos, uint64_t n, float *lo, float *hi)
{
    for (int c = 0; c < 3; c++) {
        float a = INFINITY, b = -INFINITY;
        for (uint64_t i = 0; i < n; i++) {
            float x = pos[i * 3 + c];
            if (x < a) a = x;
            if (x > b) b = x;
        }
        lo[c] = a == 0.0f ? 0.0f : a;
        hi[c] = b == 0.0f ? 0.0f : b;
    }
}

/* Opacity premultiplication before coding (Sec. II: the coded coefficients
 * are H~ = mu H, eq. premult; Sec. V-A): out = mu_i * x in FP32. */
EXPORT void ref_premultiply(const float *sh, const float *opacity, uint64_t n, float *out)
{
    for (uint64_t i = 0; i < n; i++)
        for (int e = 0; e < 48; e++) out[i * 48 + e] = opacity[i] * sh[i * 48 + e];
}

static int cmp_float(const void *a, const void *b)
{
    float x = *(const float *)a, y = *(const float *)b;
    return (x > y) - (x < y);
}

/* The paper's range (Sec. V-A): per band a scale such that after
 * normalisation the given share (num/den, 995/1000 there) of the band's
 * coefficients lies in [-0.5, 0.5].  Read as the symmetric interval
 * [-t, t] with t the r-th smallest |x| over the band's 3n coefficients,
 * r = ceil(3n num / den): the least t with at least that share inside.
 * Quantisation is then the same rint((x - vmin) 255/(vmax - vmin)), clamped,
 * with vmin = -t, vmax = t. */
EXPORT void ref_band_range_coverage(const float *sh, uint64_t n, uint32_t num, uint32_t den, float *vmin,
                                    float *vmax)
{
    const uint64_t M = 3 * n;
    const uint64_t r = (M * num + den - 1) / den;   /* 1-based rank */
    float *a = (float *)malloc(M * sizeof(float));
    for (int k = 0; k < 16; k++) {
        for (uint64_t i = 0; i < n; i++)
            for (int c = 0; c < 3; c++) a[i * 3 + c] = fabsf(sh[(i * 16 + k) * 3 + c]);
        qsort(a, M, sizeof(float), cmp_float);
        float t = a[r - 1];
        vmin[k] = t == 0.0f ? 0.0f : -t;
        vmax[k] = t;
    }
    free(a);
}

EXPORT void ref_quantise(const float *sh, uint64_t n, const float *vmin,
                         const float *vmax, uint8_t *q)
{
    for (int k = 0; k < 16; k++) {
        float range = vmax[k] - vmin[k];
        float s = (range > 0.0f) ? 255.0f / range : 0.0f;
        for (uint64_t i = 0; i < n; i++)
            for (int c = 0; c < 3; c++) {
                float t = sh[(i * 16 + k) * 3 + c] - vmin[k];
                float u = t * s;
                int v = (int)rintf(u);
                if (v < 0) v = 0;
                if (v > 255) v = 255;
                q[(i * 16 + k) * 3 + c] = (uint8_t)v;
            }
    }
}

/* ======================================================================
 * K -- keys.  Colour key: the bits of the band-0 R, G, B bytes interleaved
 * into 24 bits, R most significant within each bit triple (Fig. Bit4Scan).
 * Chunk: a 2^g per-axis grid over the position bounding box, Morton order
 * with x in the lowest bit, placed above the colour key so that colour is
 * sorted inside each spatial group.
 * ====================================================================== */
EXPORT uint32_t ref_morton_rgb(uint32_t r, uint32_t g, uint32_t b)
{
    uint32_t key = 0;
    for (int bit = 0; bit < 8; bit++) {
        key |= ((b >> bit) & 1u) << (3 * bit);
        key |= ((g >> bit) & 1u) << (3 * bit + 1);
        key |= ((r >> bit) & 1u) << (3 * bit + 2);
    }
    return key;
}

EXPORT uint32_t ref_morton3(uint32_t cx, uint32_t cy, uint32_t cz, uint32_t g)
{
    uint32_t m = 0;
    for (uint32_t bit = 0; bit < g; bit++) {
        m |= ((cx >> bit) & 1u) << (3 * bit);
        m |= ((cy >> bit) & 1u) << (3 * bit + 1);
        m |= ((cz >> bit) & 1u) << (3 * bit + 2);
    }
    return m;
}

EXPORT void ref_keys(const float *pos, const uint8_t *q, uint64_t n, uint32_t g,
                     const float *lo, const float *hi, uint64_t *keys)
{
    float sc[3];
    uint32_t cmax = (1u << g) - 1u;
    for (int c = 0; c < 3; c++) {
        float ext = hi[c] - lo[c];
        sc[c] = (ext > 0.0f) ? (float)(1u << g) / ext : 0.0f;
    }
    for (uint64_t i = 0; i < n; i++) {
        uint32_t cell[3];
        for (int c = 0; c < 3; c++) {
            float t = pos[i * 3 + c] - lo[c];
            float u = t * sc[c];
            uint32_t v = (uint32_t)floorf(u);
            cell[c] = v < cmax ? v : cmax;
        }
        uint64_t chunk = ref_morton3(cell[0], cell[1], cell[2], g);
        const uint8_t *dc = q + (i * 16 + 0) * 3;
        keys[i] = (chunk << 24) | ref_morton_rgb(dc[0], dc[1], dc[2]);
    }
}

/* Degree class of each primitive for the variable number of bands (Sec.
 * IV-B: primitives whose higher-order SH are zero, or small enough to be
 * treated as zero, go to bitstreams with fewer bands): the largest SH degree
 * l in 1..3 with some coefficient of a degree-l band (bands l^2..l^2+2l)
 * above tau in magnitude, else 0.  The primitive keeps its (l+1)^2 lowest
 * bands; the higher ones are dropped and decode as zero. */
EXPORT void ref_degrees(const float *sh, uint64_t n, float tau, uint8_t *deg)
{
    for (uint64_t i = 0; i < n; i++) {
        int L = 0;
        for (int l = 1; l <= 3; l++)
            for (int k = l * l; k <= l * l + 2 * l; k++)
                for (int c = 0; c < 3; c++)
                    if (fabsf(sh[(i * 16 + (uint64_t)k) * 3 + c]) > tau) L = l;
        deg[i] = (uint8_t)L;
    }
}

/* ======================================================================
 * S -- stable ascending sort of the keys (Sec. III-C, step 2, increasing
 * order).  perm[s] = original index at sorted slot s.  Comparing (key, index)
 * makes the order total, so this is exactly the stable order.
 * ====================================================================== */
static const uint64_t *g_sort_keys;
static int cmp_slot(const void *a, const void *b)
{
    uint32_t i = *(const uint32_t *)a, j = *(const uint32_t *)b;
    uint64_t ki = g_sort_keys[i], kj = g_sort_keys[j];
    if (ki != kj) return ki < kj ? -1 : 1;
    return i < j ? -1 : (i > j);
}

EXPORT void ref_sort(const uint64_t *keys, uint64_t n, uint32_t *perm)
{
    for (uint64_t i = 0; i < n; i++) perm[i] = (uint32_t)i;
    g_sort_keys = keys;
    qsort(perm, n, sizeof(uint32_t), cmp_slot);
    g_sort_keys = NULL;
}

/* ======================================================================
 * B -- block packer (Fig. SetupD: one 4x4 block per SH band holds that band
 * of 16 primitives).  Slot s -> block s/16, j = s%16 placed at the 2-D
 * zigzag position x = j0 | j2<<1, y = j1 | j3<<1 (Fig. ZigZagScan); texel
 * index 4y+x.  Alpha 255.  Slots past n repeat primitive perm[n-1].
 * tex layout: uint8[16 bands][npad/16 blocks][16 texels][4].
 * ====================================================================== */
EXPORT uint32_t ref_zigzag_texel(uint32_t j)
{
    uint32_t x = (j & 1u) | ((j >> 2) & 1u) << 1;
    uint32_t y = ((j >> 1) & 1u) | ((j >> 3) & 1u) << 1;
    return 4 * y + x;
}

EXPORT void ref_pack(const uint8_t *q, const uint32_t *perm, uint64_t n, uint8_t *tex)
{
    uint64_t npad = (n + 15) / 16 * 16;
    uint64_t nblk = npad / 16;
    for (uint64_t s = 0; s < npad; s++) {
        uint32_t src = perm[s < n ? s : n - 1];
        uint64_t b = s / 16;
        uint32_t i = ref_zigzag_texel((uint32_t)(s % 16));
        for (int k = 0; k < 16; k++) {
            uint8_t *t = tex + (((uint64_t)k * nblk + b) * 16 + i) * 4;
            t[0] = q[((uint64_t)src * 16 + k) * 3 + 0];
            t[1] = q[((uint64_t)src * 16 + k) * 3 + 1];
            t[2] = q[((uint64_t)src * 16 + k) * 3 + 2];
            t[3] = 255;
        }
    }
}

/* The other two arrangements of Sec. IV-B.  Slots past n repeat perm[n-1]
 * as above; slots are padded to a multiple of 16 in every arrangement.
 *   Fig. SetupA (one primitive -> one block): a single stream of npad
 *   blocks; block s holds slot s, band k at texel k (raster order).
 *   Fig. SetupB (four primitives -> four blocks): four streams of npad/4
 *   blocks; stream g holds bands 4g..4g+3, block s/4 holds slots 4(s/4)..+3,
 *   slot s%4 on row y and band k%4 in column x: texel 4 (s%4) + k%4. */
EXPORT void ref_pack_prim(const uint8_t *q, const uint32_t *perm, uint64_t n, uint8_t *tex)
{
    uint64_t npad = (n + 15) / 16 * 16;
    for (uint64_t s = 0; s < npad; s++) {
        uint32_t src = perm[s < n ? s : n - 1];
        for (int k = 0; k < 16; k++) {
            uint8_t *t = tex + (s * 16 + (uint64_t)k) * 4;
            for (int c = 0; c < 3; c++) t[c] = q[((uint64_t)src * 16 + k) * 3 + c];
            t[3] = 255;
        }
    }
}

EXPORT void ref_pack_quad(const uint8_t *q, const uint32_t *perm, uint64_t n, uint8_t *tex)
{
    uint64_t npad = (n + 15) / 16 * 16;
    uint64_t nblk = npad / 4;
    for (uint64_t s = 0; s < npad; s++) {
        uint32_t src = perm[s < n ? s : n - 1];
        for (int k = 0; k < 16; k++) {
            uint64_t g = (uint64_t)k / 4, b = s / 4;
            uint32_t i = 4 * (uint32_t)(s % 4) + (uint32_t)(k % 4);
            uint8_t *t = tex + ((g * nblk + b) * 16 + i) * 4;
            for (int c = 0; c < 3; c++) t[c] = q[((uint64_t)src * 16 + k) * 3 + c];
            t[3] = 255;
        }
    }
}

/* Where band k of slot s lives: stream, block within the stream, texel. */
static void locate(uint32_t arr, uint32_t s, int k, int *stream, uint64_t *block, int *texel)
{
    if (arr == 1) {
        *stream = 0; *block = s; *texel = k;
    } else if (arr == 2) {
        *stream = k / 4; *block = s / 4; *texel = 4 * (int)(s % 4) + k % 4;
    } else {
        *stream = k; *block = s / 16; *texel = (int)ref_zigzag_texel(s % 16);
    }
}

/* ======================================================================
 * D1 -- BC1 decode (D3D11 BC1 format, the BTC scheme of Sec. III-A with
 * P = 16 bits per reference colour (RGB565) and Q = 2 bits per texel).
 * Interpolated entries are the exact rational rounded to nearest.
 * ====================================================================== */
static void bc1_expand(uint32_t c, int e[3])
{
    int r5 = (c >> 11) & 31, g6 = (c >> 5) & 63, b5 = c & 31;
    e[0] = (r5 << 3) | (r5 >> 2);
    e[1] = (g6 << 2) | (g6 >> 4);
    e[2] = (b5 << 3) | (b5 >> 2);
}

static void bc1_palette(uint32_t c0, uint32_t c1, int pal[4][4])
{
    int e0[3], e1[3];
    bc1_expand(c0, e0);
    bc1_expand(c1, e1);
    for (int c = 0; c < 3; c++) {
        pal[0][c] = e0[c];
        pal[1][c] = e1[c];
        if (c0 > c1) {
            pal[2][c] = (2 * e0[c] + e1[c] + 1) / 3;
            pal[3][c] = (e0[c] + 2 * e1[c] + 1) / 3;
        } else {
            pal[2][c] = (e0[c] + e1[c] + 1) >> 1;
            pal[3][c] = 0;
        }
    }
    pal[0][3] = pal[1][3] = pal[2][3] = 255;
    pal[3][3] = (c0 > c1) ? 255 : 0;
}

EXPORT void ref_bc1_decode_block(const uint8_t *blk, uint8_t *out)
{
    uint32_t c0 = blk[0] | (blk[1] << 8);
    uint32_t c1 = blk[2] | (blk[3] << 8);
    uint32_t idx = blk[4] | (blk[5] << 8) | (blk[6] << 16) | ((uint32_t)blk[7] << 24);
    int pal[4][4];
    bc1_palette(c0, c1, pal);
    for (int i = 0; i < 16; i++) {
        int k = (idx >> (2 * i)) & 3;
        for (int c = 0; c < 4; c++) out[i * 4 + c] = (uint8_t)pal[k][c];
    }
}

/* ======================================================================
 * D2 -- BC7 decode (D3D11 BC7 / BPTC format).  Tables transcribed from the
 * public format specification: partition maps for 2 and 3 subsets (one
 * character per texel, texel 0 first), anchor texels of the 2nd and 3rd
 * subsets, and the interpolation weights.
 * ====================================================================== */
static const char *P2[64] = {
    "0011001100110011", "0001000100010001", "0111011101110111", "0001001100110111",
    "0000000100010011", "0011011101111111", "0001001101111111", "0000000100110111",
    "0000000000010011", "0011011111111111", "0000000101111111", "0000000000010111",
    "0001011111111111", "0000000011111111", "0000111111111111", "0000000000001111",
    "0000100011101111", "0111000100000000", "0000000010001110", "0111001100010000",
    "0011000100000000", "0000100011001110", "0000000010001100", "0111001100110001",
    "0011000100010000", "0000100010001100", "0110011001100110", "0011011001101100",
    "0001011111101000", "0000111111110000", "0111000110001110", "0011100110011100",
    "0101010101010101", "0000111100001111", "0101101001011010", "0011001111001100",
    "0011110000111100", "0101010110101010", "0110100101101001", "0101101010100101",
    "0111001111001110", "0001001111001000", "0011001001001100", "0011101111011100",
    "0110100110010110", "0011110011000011", "0110011010011001", "0000011001100000",
    "0100111001000000", "0010011100100000", "0000001001110010", "0000010011100100",
    "0110110010010011", "0011011011001001", "0110001110011100", "0011100111000110",
    "0110110011001001", "0110001100111001", "0111111010000001", "0001100011100111",
    "0000111100110011", "0011001111110000", "0010001011101110", "0100010001110111",
};

static const char *P3[64] = {
    "0011001102212222", "0001001122112221", "0000200122112211", "0222002200110111",
    "0000000011221122", "0011001100220022", "0022002211111111", "0011001122112211",
    "0000000011112222", "0000111111112222", "0000111122222222", "0012001200120012",
    "0112011201120112", "0122012201220122", "0011011211221222", "0011200122002220",
    "0001001101121122", "0111001120012200", "0000112211221122", "0022002200221111",
    "0111011102220222", "0001000122212221", "0000001101220122", "0000110022102210",
    "0122012200110000", "0012001211222222", "0110122112210110", "0000011012211221",
    "0022110211020022", "0110011020022222", "0011012201220011", "0000200022112221",
    "0000000211221222", "0222002200120011", "0011001200220222", "0120012001200120",
    "0000111122220000", "0120120120120120", "0120201212010120", "0011220011220011",
    "0011112222000011", "0101010122222222", "0000000021212121", "0022112200221122",
    "0022001100220011", "0220122102201221", "0101222222220101", "0000212121212121",
    "0101010101012222", "0222011102220111", "0002111200021112", "0000211221122112",
    "0222011101110222", "0002111211120002", "0110011001102222", "0000000021122112",
    "0110011022222222", "0022001100110022", "0022112211220022", "0000000000002112",
    "0002000100020001", "0222122202221222", "0101222222222222", "0111201122012220",
};

static const int A2[64] = {
    15, 15, 15, 15, 15, 15, 15, 15, 15, 15, 15, 15, 15, 15, 15, 15,
    15, 2,  8,  2,  2,  8,  8,  15, 2,  8,  2,  2,  8,  8,  2,  2,
    15, 15, 6,  8,  2,  8,  15, 15, 2,  8,  2,  2,  2,  15, 15, 6,
    6,  2,  6,  8,  15, 15, 2,  2,  15, 15, 15, 15, 15, 2,  2,  15,
};
static const int A3a[64] = {
    3,  3,  15, 15, 8,  3,  15, 15, 8,  8,  6,  6,  6,  5,  3,  3,
    3,  3,  8,  15, 3,  3,  6,  10, 5,  8,  8,  6,  8,  5,  15, 15,
    8,  15, 3,  5,  6,  10, 8,  15, 15, 3,  15, 5,  15, 15, 15, 15,
    3,  15, 5,  5,  5,  8,  5,  10, 5,  10, 8,  13, 15, 12, 3,  3,
};
static const int A3b[64] = {
    15, 8,  8,  3,  15, 15, 3,  8,  15, 15, 15, 15, 15, 15, 15, 8,
    15, 8,  15, 3,  15, 8,  15, 8,  3,  15, 6,  10, 15, 15, 10, 8,
    15, 3,  15, 10, 10, 8,  9,  10, 6,  15, 8,  15, 3,  6,  6,  8,
    15, 3,  15, 15, 15, 15, 15, 15, 15, 15, 15, 15, 3,  15, 15, 8,
};

static const int W2[4] = {0, 21, 43, 64};
static const int W3[8] = {0, 9, 18, 27, 37, 46, 55, 64};
static const int W4[16] = {0, 4, 9, 13, 17, 21, 26, 30, 34, 38, 43, 47, 51, 55, 60, 64};

static const int *weights(int nb) { return nb == 2 ? W2 : nb == 3 ? W3 : W4; }

/* Per-mode layout.  pb: 0 none, 1 one p-bit per subset, 2 one per endpoint. */
typedef struct {
    int ns, partbits, rotbits, selbits, cb, ab, pb, ib, ib2;
} mode_t7;
static const mode_t7 M7[8] = {
    /* ns pb rb sb cb ab pb ib ib2 */
    {3, 4, 0, 0, 4, 0, 2, 3, 0},
    {2, 6, 0, 0, 6, 0, 1, 3, 0},
    {3, 6, 0, 0, 5, 0, 0, 2, 0},
    {2, 6, 0, 0, 7, 0, 2, 2, 0},
    {1, 0, 2, 1, 5, 6, 0, 2, 3},
    {1, 0, 2, 0, 7, 8, 0, 2, 2},
    {1, 0, 0, 0, 7, 7, 2, 4, 0},
    {2, 6, 0, 0, 5, 5, 2, 2, 0},
};

static int subset_of(int ns, int part, int texel)
{
    if (ns == 1) return 0;
    if (ns == 2) return P2[part][texel] - '0';
    return P3[part][texel] - '0';
}

static int anchor_of(int ns, int part, int subset)
{
    if (subset == 0) return 0;
    if (ns == 2) return A2[part];
    return subset == 1 ? A3a[part] : A3b[part];
}

static int is_anchor(int ns, int part, int texel)
{
    for (int s = 0; s < ns; s++)
        if (anchor_of(ns, part, s) == texel) return 1;
    return 0;
}

/* Expand an n-bit value (5 <= n <= 8) to 8 bits by bit replication. */
static int expand_bits(int v, int n)
{
    if (n >= 8) return v;
    return (v << (8 - n)) | (v >> (2 * n - 8));
}

static int interp64(int e0, int e1, int w) { return ((64 - w) * e0 + w * e1 + 32) >> 6; }

static uint32_t get_bits(const uint8_t *blk, int *pos, int n)
{
    uint32_t v = 0;
    for (int b = 0; b < n; b++) {
        int p = *pos + b;
        v |= (uint32_t)((blk[p >> 3] >> (p & 7)) & 1) << b;
    }
    *pos += n;
    return v;
}

EXPORT void ref_bc7_decode_block(const uint8_t *blk, uint8_t *out)
{
    int m = 0;
    while (m < 8 && !((blk[0] >> m) & 1)) m++;
    if (m == 8) { /* reserved mode: transparent black */
        memset(out, 0, 64);
        return;
    }
    const mode_t7 *md = &M7[m];
    int pos = m + 1;
    int part = (int)get_bits(blk, &pos, md->partbits);
    int rot = (int)get_bits(blk, &pos, md->rotbits);
    int sel = (int)get_bits(blk, &pos, md->selbits);
    int ne = 2 * md->ns;
    int code[6][4];
    for (int c = 0; c < 3; c++)
        for (int e = 0; e < ne; e++) code[e][c] = (int)get_bits(blk, &pos, md->cb);
    for (int e = 0; e < ne; e++) code[e][3] = md->ab ? (int)get_bits(blk, &pos, md->ab) : 0;
    int pbit[6] = {0, 0, 0, 0, 0, 0};
    if (md->pb == 2)
        for (int e = 0; e < ne; e++) pbit[e] = (int)get_bits(blk, &pos, 1);
    else if (md->pb == 1)
        for (int s = 0; s < md->ns; s++) pbit[2 * s] = pbit[2 * s + 1] = (int)get_bits(blk, &pos, 1);
    int ep[6][4];
    for (int e = 0; e < ne; e++) {
        for (int c = 0; c < 3; c++) {
            int v = code[e][c], n = md->cb;
            if (md->pb) { v = (v << 1) | pbit[e]; n++; }
            ep[e][c] = expand_bits(v, n);
        }
        if (md->ab) {
            int v = code[e][3], n = md->ab;
            if (md->pb) { v = (v << 1) | pbit[e]; n++; }
            ep[e][3] = expand_bits(v, n);
        } else {
            ep[e][3] = 255;
        }
    }
    int idx1[16], idx2[16];
    for (int i = 0; i < 16; i++)
        idx1[i] = (int)get_bits(blk, &pos, md->ib - is_anchor(md->ns, part, i));
    for (int i = 0; i < 16; i++)
        idx2[i] = md->ib2 ? (int)get_bits(blk, &pos, md->ib2 - (i == 0)) : 0;
    for (int i = 0; i < 16; i++) {
        int s = subset_of(md->ns, part, i);
        const int *e0 = ep[2 * s], *e1 = ep[2 * s + 1];
        int ci, ai, cn, an;
        if (md->ib2 == 0) { ci = ai = idx1[i]; cn = an = md->ib; }
        else if (sel == 0) { ci = idx1[i]; cn = md->ib; ai = idx2[i]; an = md->ib2; }
        else { ci = idx2[i]; cn = md->ib2; ai = idx1[i]; an = md->ib; }
        int px[4];
        for (int c = 0; c < 3; c++) px[c] = interp64(e0[c], e1[c], weights(cn)[ci]);
        px[3] = interp64(e0[3], e1[3], weights(an)[ai]);
        if (rot) { int t = px[3]; px[3] = px[rot - 1]; px[rot - 1] = t; }
        for (int c = 0; c < 4; c++) out[i * 4 + c] = (uint8_t)px[c];
    }
}

/* ======================================================================
 * Shared encoder pieces: the principal axis of a set of RGB triples by
 * integer power iteration.
 *   C = n * sum(x x^T) - S S^T   (exact),
 *   C' = C >> t with t the least shift making (max diag >> t) < 2^14,
 *   v = row of C' with the largest diagonal (lowest index on ties),
 *   8 times: u = C' v; s = least shift making (max|u| >> s) < 2^15; v = u >> s,
 *   v == 0 at the end -> (1,1,1).
 * ====================================================================== */
static void principal_axis(int n, const int (*x)[3], int64_t v[3])
{
    int64_t S[3] = {0, 0, 0}, XX[3][3] = {{0}};
    for (int i = 0; i < n; i++)
        for (int a = 0; a < 3; a++) {
            S[a] += x[i][a];
            for (int b = 0; b < 3; b++) XX[a][b] += (int64_t)x[i][a] * x[i][b];
        }
    int64_t C[3][3];
    for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++) C[a][b] = (int64_t)n * XX[a][b] - S[a] * S[b];
    int j = 0;
    for (int a = 1; a < 3; a++)
        if (C[a][a] > C[j][j]) j = a;
    int64_t dmax = C[j][j];
    int t = 0;
    while ((dmax >> t) >= (1 << 14)) t++;
    int64_t Cs[3][3];
    for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++) Cs[a][b] = C[a][b] >> t;
    for (int a = 0; a < 3; a++) v[a] = Cs[j][a];
    for (int it = 0; it < 8; it++) {
        int64_t u[3];
        for (int a = 0; a < 3; a++) u[a] = Cs[a][0] * v[0] + Cs[a][1] * v[1] + Cs[a][2] * v[2];
        int64_t m = 0;
        for (int a = 0; a < 3; a++) {
            int64_t au = u[a] < 0 ? -u[a] : u[a];
            if (au > m) m = au;
        }
        int s = 0;
        while ((m >> s) >= (1 << 15)) s++;
        for (int a = 0; a < 3; a++) v[a] = u[a] >> s;
    }
    if (v[0] == 0 && v[1] == 0 && v[2] == 0) v[0] = v[1] = v[2] = 1;
}

/* The axis of n triples x[n][3] (for the pins of the step above). */
EXPORT void ref_principal_axis(int n, const int *x, int64_t *v)
{
    principal_axis(n, (const int (*)[3])x, v);
}

/* floor(num/den) for den > 0 */
static int64_t floor_div(int64_t num, int64_t den)
{
    int64_t q = num / den;
    if ((num % den) != 0 && num < 0) q--;
    return q;
}

/* ======================================================================
 * E1 -- BC1 encoder (BTC with Q = 2; Sec. III-A).  SSE over RGB, integer.
 * ====================================================================== */
static int bc1_e(int code, int w) { return w == 5 ? (code << 3) | (code >> 2) : (code << 2) | (code >> 4); }
static const int BC1_W[3] = {5, 6, 5};

static uint32_t pack565(const int c[3]) { return ((uint32_t)c[0] << 11) | ((uint32_t)c[1] << 5) | (uint32_t)c[2]; }
static void unpack565(uint32_t p, int c[3]) { c[0] = (p >> 11) & 31; c[1] = (p >> 5) & 63; c[2] = p & 31; }

/* Put the endpoint pair in the order the mode needs (4-colour: c0 > c1;
 * 3-colour: c0 <= c1) and give every texel the palette entry of least SSE
 * (lowest index on ties).  Returns the block SSE. */
static uint32_t bc1_canon_index(uint32_t *c0, uint32_t *c1, int four, const int (*x)[3],
                                uint32_t *indices)
{
    if ((four && *c0 < *c1) || (!four && *c0 > *c1)) {
        uint32_t t = *c0; *c0 = *c1; *c1 = t;
    }
    int pal[4][4];
    bc1_palette(*c0, *c1, pal);
    uint32_t sse = 0, idx = 0;
    for (int i = 0; i < 16; i++) {
        int best = 0;
        uint32_t bd = 0xffffffffu;
        for (int k = 0; k < 4; k++) {
            uint32_t d = 0;
            for (int c = 0; c < 3; c++) {
                int e = x[i][c] - pal[k][c];
                d += (uint32_t)(e * e);
            }
            if (d < bd) { bd = d; best = k; }
        }
        sse += bd;
        idx |= (uint32_t)best << (2 * i);
    }
    *indices = idx;
    return sse;
}

/* Nearest code to num/den (den > 0): argmin_c |E(c)*den - num|, lowest c on ties. */
static int bc1_quant(int64_t num, int64_t den, int w)
{
    int best = 0;
    int64_t bd = -1;
    for (int c = 0; c < (1 << w); c++) {
        int64_t d = (int64_t)bc1_e(c, w) * den - num;
        if (d < 0) d = -d;
        if (bd < 0 || d < bd) { bd = d; best = c; }
    }
    return best;
}

/* Constant-colour tables, built by brute force: for channel width w and
 * target v, the code pair whose index-2 entry ((2E(a)+E(b)+1)/3 in 4-colour
 * mode, (E(a)+E(b)+1)>>1 in 3-colour mode) is nearest v; ties by smallest
 * |a-b|, then a, then b. */
static int bc1_tab_ready = 0;
static uint8_t T4a[2][256], T4b[2][256], T3a[2][256], T3b[2][256];
static int T4e[2][256], T3e[2][256];

static void bc1_build_tables(void)
{
    for (int wi = 0; wi < 2; wi++) {
        int w = wi ? 6 : 5, nc = 1 << w;
        for (int v = 0; v < 256; v++) {
            for (int mode = 0; mode < 2; mode++) {
                int be = 1 << 30, ba = 0, bb = 0;
                for (int a = 0; a < nc; a++)
                    for (int b = 0; b < nc; b++) {
                        int ea = bc1_e(a, w), eb = bc1_e(b, w);
                        int u = mode == 0 ? (2 * ea + eb + 1) / 3 : (ea + eb + 1) >> 1;
                        int err = abs(u - v);
                        int better = 0;
                        if (err < be) better = 1;
                        else if (err == be) {
                            int dab = abs(a - b), dbest = abs(ba - bb);
                            if (dab < dbest) better = 1;
                            else if (dab == dbest && (a < ba || (a == ba && b < bb))) better = 1;
                        }
                        if (better) { be = err; ba = a; bb = b; }
                    }
                if (mode == 0) { T4a[wi][v] = (uint8_t)ba; T4b[wi][v] = (uint8_t)bb; T4e[wi][v] = be; }
                else { T3a[wi][v] = (uint8_t)ba; T3b[wi][v] = (uint8_t)bb; T3e[wi][v] = be; }
            }
        }
    }
    bc1_tab_ready = 1;
}

static void bc1_emit(uint32_t c0, uint32_t c1, uint32_t idx, uint8_t *out)
{
    out[0] = c0 & 255; out[1] = c0 >> 8;
    out[2] = c1 & 255; out[3] = c1 >> 8;
    out[4] = idx & 255; out[5] = (idx >> 8) & 255; out[6] = (idx >> 16) & 255; out[7] = idx >> 24;
}

/* tex: 16 texels x RGBA (alpha ignored).  Returns the block SSE. */
EXPORT uint32_t ref_bc1_encode_block(const uint8_t *tex, uint32_t refine_steps, uint8_t *out)
{
    if (!bc1_tab_ready) bc1_build_tables();
    int x[16][3];
    for (int i = 0; i < 16; i++)
        for (int c = 0; c < 3; c++) x[i][c] = tex[i * 4 + c];

    /* 1. constant block */
    int constant = 1;
    for (int i = 1; i < 16; i++)
        for (int c = 0; c < 3; c++)
            if (x[i][c] != x[0][c]) constant = 0;
    if (constant) {
        int e4 = 0, e3 = 0, a4[3], b4[3], a3[3], b3[3];
        for (int c = 0; c < 3; c++) {
            int wi = BC1_W[c] == 6, v = x[0][c];
            a4[c] = T4a[wi][v]; b4[c] = T4b[wi][v]; e4 += T4e[wi][v] * T4e[wi][v];
            a3[c] = T3a[wi][v]; b3[c] = T3b[wi][v]; e3 += T3e[wi][v] * T3e[wi][v];
        }
        int four = e4 <= e3;
        uint32_t c0 = pack565(four ? a4 : a3), c1 = pack565(four ? b4 : b3), idx;
        uint32_t sse = bc1_canon_index(&c0, &c1, four, (const int (*)[3])x, &idx);
        bc1_emit(c0, c1, idx, out);
        return sse;
    }

    /* 2. principal axis, 3. order by (projection, texel index) */
    int64_t v[3];
    principal_axis(16, (const int (*)[3])x, v);
    int64_t proj[16];
    for (int i = 0; i < 16; i++) proj[i] = v[0] * x[i][0] + v[1] * x[i][1] + v[2] * x[i][2];
    int order[16];
    for (int i = 0; i < 16; i++) order[i] = i;
    for (int a = 1; a < 16; a++) { /* insertion sort, stable */
        int t = order[a], b = a - 1;
        while (b >= 0 && proj[order[b]] > proj[t]) { order[b + 1] = order[b]; b--; }
        order[b + 1] = t;
    }
    int xs[16][3];
    for (int k = 0; k < 16; k++)
        for (int c = 0; c < 3; c++) xs[k][c] = x[order[k]][c];

    /* 4. cluster fit over every split of the ordered texels */
    uint32_t best_sse = 0xffffffffu;
    int bq0[3] = {0, 0, 0}, bq1[3] = {0, 0, 0}, bfour = 1;
    for (int list = 0; list < 2; list++) {
        int four = list == 0;
        int F = four ? 3 : 2;        /* weights (alpha, beta) sum to F */
        int ncl = four ? 4 : 3;
        for (int s1 = 0; s1 <= 16; s1++)
            for (int s2 = s1; s2 <= 16; s2++)
                for (int s3 = (four ? s2 : 16); s3 <= 16; s3++) {
                    int bound[5] = {0, s1, s2, four ? s3 : 16, 16};
                    int64_t A = 0, B = 0, AB = 0;
                    int64_t SA[3] = {0, 0, 0}, SB[3] = {0, 0, 0};
                    for (int j = 0; j < ncl; j++) {
                        int al = F - j, be = j;
                        for (int k = bound[j]; k < bound[j + 1]; k++) {
                            A += al * al; B += be * be; AB += al * be;
                            for (int c = 0; c < 3; c++) { SA[c] += al * xs[k][c]; SB[c] += be * xs[k][c]; }
                        }
                    }
                    int64_t det = A * B - AB * AB;
                    if (det == 0) continue;
                    int q0[3], q1[3], e0[3], e1[3];
                    for (int c = 0; c < 3; c++) {
                        int64_t n0 = F * (B * SA[c] - AB * SB[c]);
                        int64_t n1 = F * (A * SB[c] - AB * SA[c]);
                        q0[c] = bc1_quant(n0, det, BC1_W[c]);
                        q1[c] = bc1_quant(n1, det, BC1_W[c]);
                        e0[c] = bc1_e(q0[c], BC1_W[c]);
                        e1[c] = bc1_e(q1[c], BC1_W[c]);
                    }
                    uint32_t sse = 0;
                    for (int j = 0; j < ncl; j++) {
                        int al = F - j, be = j;
                        for (int k = bound[j]; k < bound[j + 1]; k++)
                            for (int c = 0; c < 3; c++) {
                                int p = (al * e0[c] + be * e1[c] + 1) / F;
                                int d = xs[k][c] - p;
                                sse += (uint32_t)(d * d);
                            }
                    }
                    if (sse < best_sse) {
                        best_sse = sse;
                        memcpy(bq0, q0, sizeof q0); memcpy(bq1, q1, sizeof q1);
                        bfour = four;
                    }
                }
    }

    /* 5. canonical order + re-index */
    uint32_t c0 = pack565(bq0), c1 = pack565(bq1), idx;
    uint32_t sse = bc1_canon_index(&c0, &c1, bfour, (const int (*)[3])x, &idx);

    /* 6. refinement: 12 neighbours of the six endpoint channels */
    for (uint32_t step = 0; step < refine_steps; step++) {
        int four = c0 > c1;
        int cur[6];
        unpack565(c0, cur); unpack565(c1, cur + 3);
        uint32_t nb_sse = 0xffffffffu, nb_c0 = 0, nb_c1 = 0, nb_idx = 0;
        for (int j = 0; j < 6; j++)
            for (int dlt = -1; dlt <= 1; dlt += 2) {
                int cand[6];
                memcpy(cand, cur, sizeof cand);
                int maxc = (1 << BC1_W[j % 3]) - 1;
                cand[j] += dlt;
                if (cand[j] < 0) cand[j] = 0;
                if (cand[j] > maxc) cand[j] = maxc;
                uint32_t a = pack565(cand), b = pack565(cand + 3), ii;
                uint32_t s = bc1_canon_index(&a, &b, four, (const int (*)[3])x, &ii);
                if (s < nb_sse) { nb_sse = s; nb_c0 = a; nb_c1 = b; nb_idx = ii; }
            }
        if (nb_sse < sse) { sse = nb_sse; c0 = nb_c0; c1 = nb_c1; idx = nb_idx; }
        else break;
    }
    bc1_emit(c0, c1, idx, out);
    return sse;
}

/* ======================================================================
 * E2 -- BC7 encoder.  285 candidates in a fixed order; each is fitted
 * subset by subset and scored by the exact integer RGB SSE; the winner
 * minimises (SSE << 9) | candidate.
 * ====================================================================== */

/* Value of an endpoint code with p-bit p under mode precision (cb, pb). */
static int ep_value(int code, int p, int cb, int pb)
{
    if (pb) return expand_bits((code << 1) | p, cb + 1);
    return expand_bits(code, cb);
}

/* Nearest code to t for p-bit p (lowest code on ties). */
static int ep_nearest(int t, int p, int cb, int pb)
{
    int best = 0, bd = 1 << 30;
    for (int c = 0; c < (1 << cb); c++) {
        int d = abs(ep_value(c, p, cb, pb) - t);
        if (d < bd) { bd = d; best = c; }
    }
    return best;
}

/* Single-value tables: for precision class (cb, pb), p-bits (p0, p1) and
 * weight w, the code pair whose interpolation at w is nearest v; ties by
 * smallest |c0-c1|, then c0, then c1.  Built lazily per (cb, pb, p0, p1, w). */
typedef struct { uint8_t c0[256], c1[256]; uint16_t err[256]; int ready; } sv_tab;
static sv_tab SV[9][3][2][2][65]; /* [cb][pb][p0][p1][w] */

static const sv_tab *sv_get(int cb, int pb, int p0, int p1, int w)
{
    sv_tab *t = &SV[cb][pb][p0][p1][w];
    if (t->ready) return t;
    int nc = 1 << cb;
    for (int v = 0; v < 256; v++) {
        int be = 1 << 30, b0 = 0, b1 = 0;
        for (int a = 0; a < nc; a++)
            for (int b = 0; b < nc; b++) {
                int u = interp64(ep_value(a, p0, cb, pb), ep_value(b, p1, cb, pb), w);
                int err = abs(u - v), better = 0;
                if (err < be) better = 1;
                else if (err == be) {
                    int dab = abs(a - b), dbest = abs(b0 - b1);
                    if (dab < dbest) better = 1;
                    else if (dab == dbest && (a < b0 || (a == b0 && b < b1))) better = 1;
                }
                if (better) { be = err; b0 = a; b1 = b; }
            }
        t->c0[v] = (uint8_t)b0; t->c1[v] = (uint8_t)b1; t->err[v] = (uint16_t)be;
    }
    t->ready = 1;
    return t;
}

/* p-bit combinations of a mode, in binary order. */
static int pcombos(int pb) { return pb == 2 ? 4 : pb == 1 ? 2 : 1; }
static void pcombo(int pb, int pc, int *p0, int *p1)
{
    if (pb == 2) { *p0 = pc & 1; *p1 = pc >> 1; }
    else if (pb == 1) { *p0 = *p1 = pc; }
    else { *p0 = *p1 = 0; }
}

/* Fit state of one endpoint pair over a texel set with `nch` channels. */
typedef struct {
    int c0[3], c1[3], p0, p1;
    int idx[16];
    uint32_t sse;
} fit_t;

/* (c): quantise the two endpoint colours for each p-bit combination, index
 * every texel by least SSE, keep the best combination (lowest on ties). */
static void fit_eval(int nch, int n, const int (*x)[3], const int e_lo[3], const int e_hi[3],
                     int cb, int pb, int nb, fit_t *out)
{
    const int *W = weights(nb);
    out->sse = 0xffffffffu;
    for (int pc = 0; pc < pcombos(pb); pc++) {
        int p0, p1;
        pcombo(pb, pc, &p0, &p1);
        fit_t f;
        f.p0 = p0; f.p1 = p1;
        int d0[3], d1[3];
        for (int c = 0; c < nch; c++) {
            f.c0[c] = ep_nearest(e_lo[c], p0, cb, pb);
            f.c1[c] = ep_nearest(e_hi[c], p1, cb, pb);
            d0[c] = ep_value(f.c0[c], p0, cb, pb);
            d1[c] = ep_value(f.c1[c], p1, cb, pb);
        }
        f.sse = 0;
        for (int i = 0; i < n; i++) {
            uint32_t bd = 0xffffffffu;
            int bk = 0;
            for (int k = 0; k < (1 << nb); k++) {
                uint32_t d = 0;
                for (int c = 0; c < nch; c++) {
                    int e = x[i][c] - interp64(d0[c], d1[c], W[k]);
                    d += (uint32_t)(e * e);
                }
                if (d < bd) { bd = d; bk = k; }
            }
            f.idx[i] = bk;
            f.sse += bd;
        }
        if (f.sse < out->sse) *out = f;
    }
}

/* Fit one subset: n texels x[] with nch channels (3 for colour, 1 for the
 * scalar channel of modes 4/5). */
/* E2 (d): least-squares endpoints of n members x[i][0..nch-1] for their
 * indices idx[i] with weights w = W[idx] on (64 - w) e0 + w e1 = 64 x:
 * with A = sum (64-w)^2, B = sum w^2, AB = sum (64-w) w, SA, SB the sums of
 * (64-w) x and w x, e0 = 64 (B SA - AB SB) / det and e1 = 64 (A SB - AB SA)
 * / det (det = A B - AB^2), each rounded half up and clamped to [0, 255].
 * Returns 0 (endpoints untouched) when det = 0. */
static int ls_endpoints(int n, const int (*x)[3], const int *idx, const int *W, int nch, int *r_lo, int *r_hi)
{
    int64_t A = 0, B = 0, AB = 0, SA[3] = {0, 0, 0}, SB[3] = {0, 0, 0};
    for (int i = 0; i < n; i++) {
        int b = W[idx[i]], a = 64 - b;
        A += a * a; B += b * b; AB += a * b;
        for (int c = 0; c < nch; c++) { SA[c] += a * x[i][c]; SB[c] += b * x[i][c]; }
    }
    int64_t det = A * B - AB * AB;
    if (det == 0) return 0;
    for (int c = 0; c < nch; c++) {
        int64_t n0 = 64 * (B * SA[c] - AB * SB[c]);
        int64_t n1 = 64 * (A * SB[c] - AB * SA[c]);
        int64_t v0 = floor_div(2 * n0 + det, 2 * det);
        int64_t v1 = floor_div(2 * n1 + det, 2 * det);
        r_lo[c] = (int)(v0 < 0 ? 0 : v0 > 255 ? 255 : v0);
        r_hi[c] = (int)(v1 < 0 ? 0 : v1 > 255 ? 255 : v1);
    }
    return 1;
}

/* The same for the pins: weights of nb-bit indices, nch channels;
 * out[0..2] = low endpoint, out[3..5] = high endpoint. */
EXPORT int ref_bc7_ls_endpoints(int n, const int *x, const int *idx, int nb, int nch, int *out)
{
    return ls_endpoints(n, (const int (*)[3])x, idx, weights(nb), nch, out, out + 3);
}

static void fit_subset(int nch, int n, const int (*x)[3], int cb, int pb, int nb, fit_t *out)
{
    const int *W = weights(nb);
    int same = 1;
    for (int i = 1; i < n; i++)
        for (int c = 0; c < nch; c++)
            if (x[i][c] != x[0][c]) same = 0;
    if (same) {
        /* (a) single value: best (p-bits, index) over per-channel tables */
        uint32_t be = 0xffffffffu;
        for (int pc = 0; pc < pcombos(pb); pc++) {
            int p0, p1;
            pcombo(pb, pc, &p0, &p1);
            for (int k = 0; k < (1 << nb); k++) {
                uint32_t e = 0;
                fit_t f;
                for (int c = 0; c < nch; c++) {
                    const sv_tab *t = sv_get(cb, pb, p0, p1, W[k]);
                    f.c0[c] = t->c0[x[0][c]];
                    f.c1[c] = t->c1[x[0][c]];
                    e += (uint32_t)t->err[x[0][c]] * t->err[x[0][c]];
                }
                if (e < be) {
                    be = e;
                    f.p0 = p0; f.p1 = p1;
                    for (int i = 0; i < n; i++) f.idx[i] = k;
                    f.sse = e * (uint32_t)n;
                    *out = f;
                }
            }
        }
        return;
    }
    /* (b) endpoints: texels of least and greatest projection on the axis */
    int e_lo[3] = {0, 0, 0}, e_hi[3] = {0, 0, 0};
    if (nch == 3) {
        int64_t v[3];
        principal_axis(n, x, v);
        int ilo = 0, ihi = 0;
        int64_t plo = 0, phi = 0;
        for (int i = 0; i < n; i++) {
            int64_t p = v[0] * x[i][0] + v[1] * x[i][1] + v[2] * x[i][2];
            if (i == 0 || p < plo) { plo = p; ilo = i; }
            if (i == 0 || p > phi) { phi = p; ihi = i; }
        }
        for (int c = 0; c < 3; c++) { e_lo[c] = x[ilo][c]; e_hi[c] = x[ihi][c]; }
    } else {
        e_lo[0] = e_hi[0] = x[0][0];
        for (int i = 1; i < n; i++) {
            if (x[i][0] < e_lo[0]) e_lo[0] = x[i][0];
            if (x[i][0] > e_hi[0]) e_hi[0] = x[i][0];
        }
    }
    /* (c) */
    fit_eval(nch, n, x, e_lo, e_hi, cb, pb, nb, out);
    /* (d) one least-squares refinement with the chosen indices */
    int r_lo[3] = {0, 0, 0}, r_hi[3] = {0, 0, 0};
    if (!ls_endpoints(n, x, out->idx, W, nch, r_lo, r_hi)) return;
    fit_t g;
    fit_eval(nch, n, x, r_lo, r_hi, cb, pb, nb, &g);
    if (g.sse < out->sse) *out = g;
}

/* (e) anchor rule: the anchor texel's index must have its top bit clear;
 * otherwise swap the endpoints (and p-bits) and mirror every index. */
static void anchor_fix(fit_t *f, int n, int anchor_pos, int nch, int nb)
{
    int top = 1 << (nb - 1);
    if (!(f->idx[anchor_pos] & top)) return;
    for (int c = 0; c < nch; c++) { int t = f->c0[c]; f->c0[c] = f->c1[c]; f->c1[c] = t; }
    int t = f->p0; f->p0 = f->p1; f->p1 = t;
    for (int i = 0; i < n; i++) f->idx[i] = (1 << nb) - 1 - f->idx[i];
}

typedef struct { int mode, part, rot, sel; } cand_t;

EXPORT int ref_bc7_candidate(int ci, int *mode, int *part, int *rot, int *sel)
{
    *part = *rot = *sel = 0;
    if (ci < 16) { *mode = 0; *part = ci; return 0; }
    ci -= 16;
    if (ci < 64) { *mode = 1; *part = ci; return 0; }
    ci -= 64;
    if (ci < 64) { *mode = 2; *part = ci; return 0; }
    ci -= 64;
    if (ci < 64) { *mode = 3; *part = ci; return 0; }
    ci -= 64;
    if (ci < 8) { *mode = 4; *rot = ci >> 1; *sel = ci & 1; return 0; }
    ci -= 8;
    if (ci < 4) { *mode = 5; *rot = ci; return 0; }
    ci -= 4;
    if (ci < 1) { *mode = 6; return 0; }
    ci -= 1;
    if (ci < 64) { *mode = 7; *part = ci; return 0; }
    return -1;
}

static void put_bits(uint8_t *blk, int *pos, uint32_t v, int n)
{
    for (int b = 0; b < n; b++) {
        int p = *pos + b;
        if ((v >> b) & 1) blk[p >> 3] |= (uint8_t)(1u << (p & 7));
    }
    *pos += n;
}

typedef struct {
    int mode, part, rot, sel;
    fit_t sub[3];      /* colour fits, subset texel order */
    int members[3][16], count[3];
    fit_t scal;        /* scalar fit (modes 4, 5) */
    uint32_t sse;
} bc7_sol;

static void bc7_eval_candidate(const int (*X)[3], int ci, bc7_sol *sol)
{
    int m, part, rot, sel;
    ref_bc7_candidate(ci, &m, &part, &rot, &sel);
    const mode_t7 *md = &M7[m];
    sol->mode = m; sol->part = part; sol->rot = rot; sol->sel = sel;
    /* colour triple (rotation moves one channel to the scalar slot and puts
     * the constant 255 in its place) and scalar values */
    int T[16][3], Sv[16][3];
    for (int i = 0; i < 16; i++) {
        for (int c = 0; c < 3; c++) T[i][c] = X[i][c];
        Sv[i][0] = 255; Sv[i][1] = Sv[i][2] = 0;
        if (rot) { Sv[i][0] = X[i][rot - 1]; T[i][rot - 1] = 255; }
    }
    int cnb = md->ib, snb = md->ib2;
    if (m == 4 && sel == 1) { cnb = md->ib2; snb = md->ib; }
    sol->sse = 0;
    for (int s = 0; s < md->ns; s++) {
        int xs[16][3], n = 0;
        for (int i = 0; i < 16; i++)
            if (subset_of(md->ns, part, i) == s) {
                sol->members[s][n] = i;
                for (int c = 0; c < 3; c++) xs[n][c] = T[i][c];
                n++;
            }
        sol->count[s] = n;
        fit_subset(3, n, (const int (*)[3])xs, md->cb, md->pb, cnb, &sol->sub[s]);
        int anc = anchor_of(md->ns, part, s), apos = 0;
        for (int k = 0; k < n; k++)
            if (sol->members[s][k] == anc) apos = k;
        anchor_fix(&sol->sub[s], n, apos, 3, cnb);
        sol->sse += sol->sub[s].sse;
    }
    if (md->ab && (m == 4 || m == 5)) {
        fit_subset(1, 16, (const int (*)[3])Sv, md->ab, 0, snb, &sol->scal);
        anchor_fix(&sol->scal, 16, 0, 1, snb);
        if (rot) sol->sse += sol->scal.sse;
    }
}

static void bc7_emit(const bc7_sol *sol, uint8_t *out)
{
    const mode_t7 *md = &M7[sol->mode];
    int m = sol->mode;
    memset(out, 0, 16);
    int pos = 0;
    put_bits(out, &pos, 1u << m, m + 1);
    put_bits(out, &pos, (uint32_t)sol->part, md->partbits);
    put_bits(out, &pos, (uint32_t)sol->rot, md->rotbits);
    put_bits(out, &pos, (uint32_t)sol->sel, md->selbits);
    for (int c = 0; c < 3; c++)
        for (int s = 0; s < md->ns; s++) {
            put_bits(out, &pos, (uint32_t)sol->sub[s].c0[c], md->cb);
            put_bits(out, &pos, (uint32_t)sol->sub[s].c1[c], md->cb);
        }
    if (md->ab) {
        for (int s = 0; s < md->ns; s++) {
            if (m == 4 || m == 5) {
                put_bits(out, &pos, (uint32_t)sol->scal.c0[0], md->ab);
                put_bits(out, &pos, (uint32_t)sol->scal.c1[0], md->ab);
            } else { /* alpha unused: all-ones codes */
                put_bits(out, &pos, (1u << md->ab) - 1, md->ab);
                put_bits(out, &pos, (1u << md->ab) - 1, md->ab);
            }
        }
    }
    if (md->pb == 2)
        for (int s = 0; s < md->ns; s++) {
            put_bits(out, &pos, (uint32_t)sol->sub[s].p0, 1);
            put_bits(out, &pos, (uint32_t)sol->sub[s].p1, 1);
        }
    else if (md->pb == 1)
        for (int s = 0; s < md->ns; s++) put_bits(out, &pos, (uint32_t)sol->sub[s].p0, 1);
    /* per-texel colour index */
    int cidx[16];
    for (int s = 0; s < md->ns; s++)
        for (int k = 0; k < sol->count[s]; k++) cidx[sol->members[s][k]] = sol->sub[s].idx[k];
    int cnb = md->ib, snb = md->ib2;
    if (m == 4 && sol->sel == 1) { cnb = md->ib2; snb = md->ib; }
    if (m == 4 || m == 5) {
        /* primary set is ib bits, secondary ib2 bits */
        const int *first = (m == 4 && sol->sel == 1) ? sol->scal.idx : cidx;
        const int *second = (m == 4 && sol->sel == 1) ? cidx : sol->scal.idx;
        for (int i = 0; i < 16; i++) put_bits(out, &pos, (uint32_t)first[i], md->ib - (i == 0));
        for (int i = 0; i < 16; i++) put_bits(out, &pos, (uint32_t)second[i], md->ib2 - (i == 0));
        (void)cnb; (void)snb;
    } else {
        for (int i = 0; i < 16; i++)
            put_bits(out, &pos, (uint32_t)cidx[i], md->ib - is_anchor(md->ns, sol->part, i));
    }
}

EXPORT uint32_t ref_bc7_encode_block(const uint8_t *tex, uint32_t mode_mask, uint8_t *out)
{
    int X[16][3];
    for (int i = 0; i < 16; i++)
        for (int c = 0; c < 3; c++) X[i][c] = tex[i * 4 + c];
    uint32_t best_key = 0xffffffffu;
    bc7_sol best, cur;
    memset(&best, 0, sizeof best);
    for (int ci = 0; ci < 285; ci++) {
        int m, p, r, s;
        ref_bc7_candidate(ci, &m, &p, &r, &s);
        if (!((mode_mask >> m) & 1)) continue;
        bc7_eval_candidate((const int (*)[3])X, ci, &cur);
        uint32_t key = (cur.sse << 9) | (uint32_t)ci;
        if (key < best_key) { best_key = key; best = cur; }
    }
    bc7_emit(&best, out);
    return best_key >> 9;
}

/* Build every single-value table used by the encoders (so that the
 * parallel loops below only read them). */
EXPORT void ref_init(void)
{
    if (!bc1_tab_ready) bc1_build_tables();
    for (int m = 0; m < 8; m++) {
        const mode_t7 *md = &M7[m];
        int nbs[2] = {md->ib, md->ib2};
        for (int q = 0; q < 2; q++) {
            if (!nbs[q]) continue;
            const int *W = weights(nbs[q]);
            for (int pc = 0; pc < pcombos(md->pb); pc++) {
                int p0, p1;
                pcombo(md->pb, pc, &p0, &p1);
                for (int k = 0; k < (1 << nbs[q]); k++) {
                    sv_get(md->cb, md->pb, p0, p1, W[k]);
                    if (md->ab && (m == 4 || m == 5)) sv_get(md->ab, 0, 0, 0, W[k]);
                }
            }
        }
    }
}

/* ======================================================================
 * Whole-texture encode/decode.  Blocks are independent, so the loops may
 * run on several host threads without changing any output.
 * tex: uint8[nblk][16][4]; blocks: nblk x (8 or 16) bytes; sse per block.
 * ====================================================================== */
EXPORT void ref_bc1_encode(const uint8_t *tex, uint64_t nblk, uint32_t refine_steps,
                           uint8_t *blocks, uint32_t *sse)
{
    ref_init();
    #pragma omp parallel for schedule(dynamic, 64)
    for (int64_t b = 0; b < (int64_t)nblk; b++) {
        uint32_t s = ref_bc1_encode_block(tex + b * 64, refine_steps, blocks + b * 8);
        if (sse) sse[b] = s;
    }
}

EXPORT void ref_bc7_encode(const uint8_t *tex, uint64_t nblk, uint32_t mode_mask,
                           uint8_t *blocks, uint32_t *sse)
{
    ref_init();
    #pragma omp parallel for schedule(dynamic, 16)
    for (int64_t b = 0; b < (int64_t)nblk; b++) {
        uint32_t s = ref_bc7_encode_block(tex + b * 64, mode_mask, blocks + b * 16);
        if (sse) sse[b] = s;
    }
}

EXPORT void ref_bc1_decode(const uint8_t *blocks, uint64_t nblk, uint8_t *tex)
{
    for (uint64_t b = 0; b < nblk; b++) ref_bc1_decode_block(blocks + b * 8, tex + b * 64);
}

EXPORT void ref_bc7_decode(const uint8_t *blocks, uint64_t nblk, uint8_t *tex)
{
    for (uint64_t b = 0; b < nblk; b++) ref_bc7_decode_block(blocks + b * 16, tex + b * 64);
}

/* ======================================================================
 * R -- rate control (Sec. IV-B: fixed-size blocks per bitstream, the number
 * of bits per primitive varied by the choice of stream per band).
 * Band 0 is BC7; k of the bands 1..15 are BC7 and the rest BC1, so a group
 * of 16 primitives costs 128 + 128k + 64(15-k) bits over 256 texels:
 * mean bits/texel R = (1088 + 64k)/256, i.e. k = 4R - 17.  The k bands with
 * the largest coefficient-domain gain (SSE_BC1 - SSE_BC7) * delta^2 are
 * upgraded; the lower band wins ties.
 * Returns 0, or -4 when k is not an integer in [0, 15].
 * ====================================================================== */
/* Four-bit units of a rate target over S bands: rate * S / 4 bits per
 * texel-position, accepted within 1e-9 of an integer (a class scene of 9
 * bands has rates such as 44/9).  -1 when not an integer. */
static long rate_units(double rate, uint32_t S)
{
    double u = rate * (double)S / 4.0;
    double r = floor(u + 0.5);
    if (!(fabs(u - r) <= 1e-9) || r < 0.0 || r > 1e6) return -1;
    return (long)r;
}

/* Band 0 BC7; of bands 1..S-1 the k = rate*S/4 - S - 1 with the largest
 * (SSE_BC1 - SSE_BC7) * delta^2 are BC7, the rest BC1 (lower band first on
 * ties); S = 16 gives k = 4 rate - 17. */
EXPORT int ref_rate_select(const int64_t *sse1, const int64_t *sse7, const float *vmin,
                           const float *vmax, uint32_t S, double rate, uint8_t *fmt)
{
    if (S < 1 || S > 16) return -1;
    long units = rate_units(rate, S);
    long k = units - (long)S - 1;
    if (units < 0 || k < 0 || k > (long)S - 1) return -4;
    double gain[16];
    for (uint32_t b = 1; b < S; b++) {
        double delta = (double)((vmax[b] - vmin[b]) / 255.0f);
        gain[b] = (double)(sse1[b] - sse7[b]) * (delta * delta);
    }
    fmt[0] = 7;
    for (uint32_t b = 1; b < S; b++) fmt[b] = 1;
    for (long pick = 0; pick < k; pick++) {
        int best = -1;
        for (uint32_t b = 1; b < S; b++) {
            if (fmt[b] == 7) continue;
            if (best < 0 || gain[b] > gain[best]) best = (int)b;
        }
        fmt[best] = 7;
    }
    return 0;
}

/* R0 -- the choice with a 0-bit option (Sec. IV-B: bitstreams for a varying
 * number of nonzero SH vectors per primitive; a band given 0 bits is not
 * stored and decodes to zero).  Band 0 is BC7; each band b = 1..S-1 is
 * dropped (0 bits per texel), BC1 (4) or BC7 (8), with exactly rate bits per
 * texel over the S bands: U = rate*S/4 - 2 four-bit units over bands 1..S-1,
 * an integer in 0..2(S-1), else -4.
 * Distortion of band b, in coefficient units with the rate controller's
 * step delta_b = (double)((vmax_b - vmin_b)/255 in FP32):
 *   BC1  SSE_BC1 delta_b^2,   BC7  SSE_BC7 delta_b^2,
 *   dropped  the squared dequantised values of its texel channels,
 *            sum over q = 0..255 (ascending) of hist_b[q] * v_q^2 with
 *            v_q = vmin_b + q delta_b (hist_b: the band's code histogram
 *            over the R, G and B channels of all its texels).
 * Objective: the distortions summed from band S-1 down to band 1 (each
 * added to the sum of the later bands).  Of the assignments with the least
 * objective, the first in band order with BC7 before BC1 before dropped.
 * Computed by dynamic programming over bands S-1..1 and units left; the
 * least objective of bands b..S-1 with u units distributes over the choice
 * at band b because rounded addition is monotone. */
static double zero_distortion(const uint64_t *hist, float vmin, double delta)
{
    double z = 0.0;
    for (int q = 0; q < 256; q++) {
        double v = (double)vmin + (double)q * delta;
        z += (double)hist[q] * (v * v);
    }
    return z;
}

EXPORT int ref_rate_select_zero(const int64_t *sse1, const int64_t *sse7, const uint64_t *hist,
                                const float *vmin, const float *vmax, uint32_t S, double rate, uint8_t *fmt)
{
    if (S < 1 || S > 16) return -1;
    long units = rate_units(rate, S);
    long U = units - 2;
    if (units < 0 || U < 0 || U > 2 * ((long)S - 1)) return -4;
    static const int cost[3] = {2, 1, 0};          /* units of BC7, BC1, dropped */
    static const uint8_t code[3] = {7, 1, 3};
    double D[16][3];
    for (uint32_t b = 1; b < S; b++) {
        double delta = (double)((vmax[b] - vmin[b]) / 255.0f);
        D[b][0] = (double)sse7[b] * (delta * delta);
        D[b][1] = (double)sse1[b] * (delta * delta);
        D[b][2] = zero_distortion(hist + 256 * (size_t)b, vmin[b], delta);
    }
    /* best[b][u]: least objective of bands b..S-1 using exactly u units */
    double best[17][31];
    int ok[17][31];
    for (int u = 0; u <= 30; u++) ok[S][u] = (u == 0), best[S][u] = 0.0;
    for (int b = (int)S - 1; b >= 1; b--)
        for (int u = 0; u <= 30; u++) {
            ok[b][u] = 0;
            for (int o = 0; o < 3; o++) {
                int r = u - cost[o];
                if (r < 0 || !ok[b + 1][r]) continue;
                double v = D[b][o] + best[b + 1][r];
                if (!ok[b][u] || v < best[b][u]) best[b][u] = v, ok[b][u] = 1;
            }
        }
    fmt[0] = 7;
    int u = (int)U;
    if (S > 1 && !ok[1][u]) return -4;
    for (uint32_t b = 1; b < S; b++)
        for (int o = 0; o < 3; o++) {
            int r = u - cost[o];
            if (r < 0 || !ok[b + 1][r] || D[b][o] + best[b + 1][r] != best[b][u]) continue;
            fmt[b] = code[o];
            u = r;
            break;
        }
    return 0;
}

/* ======================================================================
 * H -- view-dependent colour c(d) = H w(d) (Sec. II), FP64.  The basis is
 * the real SH of degree <= 3 in the sign convention of the 3DGS renderer,
 * k = l^2 + l + m, written here from the closed forms.
 * ====================================================================== */
EXPORT void ref_sh_basis(double x, double y, double z, double *Y)
{
    const double pi = 3.14159265358979323846;
    double c0 = 0.5 * sqrt(1.0 / pi);
    double c1 = sqrt(3.0 / (4.0 * pi));
    double c2a = 0.5 * sqrt(15.0 / pi), c2b = 0.25 * sqrt(5.0 / pi), c2c = 0.25 * sqrt(15.0 / pi);
    double c3a = 0.25 * sqrt(35.0 / (2.0 * pi)), c3b = 0.5 * sqrt(105.0 / pi);
    double c3c = 0.25 * sqrt(21.0 / (2.0 * pi)), c3d = 0.25 * sqrt(7.0 / pi);
    double c3e = 0.25 * sqrt(105.0 / pi);
    double xx = x * x, yy = y * y, zz = z * z;
    Y[0] = c0;
    Y[1] = -c1 * y;
    Y[2] = c1 * z;
    Y[3] = -c1 * x;
    Y[4] = c2a * x * y;
    Y[5] = -c2a * y * z;
    Y[6] = c2b * (2.0 * zz - xx - yy);
    Y[7] = -c2a * x * z;
    Y[8] = c2c * (xx - yy);
    Y[9] = -c3a * y * (3.0 * xx - yy);
    Y[10] = c3b * x * y * z;
    Y[11] = -c3c * y * (4.0 * zz - xx - yy);
    Y[12] = c3d * z * (2.0 * zz - 3.0 * xx - 3.0 * yy);
    Y[13] = -c3c * x * (4.0 * zz - xx - yy);
    Y[14] = c3e * z * (xx - yy);
    Y[15] = -c3a * x * (xx - 3.0 * yy);
}

/* decode_eval oracle.  blocks: the concatenated band streams, band b at
 * offset[b] with format fmt[b] (1 BC1, 7 BC7, 3 no bits: zero); nblk blocks per band.
 * dirs float[V][3]; slots uint32[m] (sorted-slot ids).
 * out[v][j][c] = sum_k Hhat[slot][k][c] * Y_k(dir_v) with
 * Hhat = vmin_k + q * delta_k, delta_k = (vmax_k - vmin_k)/255, in FP64;
 * scale[v][j][c] = sum_k |Hhat * Y_k| (the size of the terms). */
/* Dequantised decoded band vectors of slot s; fmt and offset are per stream.
 * With the band arrangement, bands at or past n_streams are dropped bands
 * (a scene of lower-degree primitives) and are exactly zero; so are the
 * bands of the quad arrangement past its streams (one stream holds bands
 * 0..3 of four primitives per block: Fig. SetupC). */
static void slot_coefficients(const uint8_t *blocks, const uint8_t *fmt, const uint64_t *offset, uint32_t arr,
                              uint32_t n_streams, const float *vmin, const float *vmax, uint32_t s, double H[16][3])
{
    const uint32_t kept = arr == 0 ? n_streams : arr == 2 ? 4 * n_streams : 16;
    for (int k = 0; k < 16; k++) {
        if ((uint32_t)k >= kept) {
            H[k][0] = H[k][1] = H[k][2] = 0.0;
            continue;
        }
        int st, texel;
        uint64_t b;
        locate(arr, s, k, &st, &b, &texel);
        if (fmt[st] == 3) {   /* a stream given 0 bits: its bands are zero */
            H[k][0] = H[k][1] = H[k][2] = 0.0;
            continue;
        }
        uint8_t px[64];
        if (fmt[st] == 1) ref_bc1_decode_block(blocks + offset[st] + b * 8, px);
        else ref_bc7_decode_block(blocks + offset[st] + b * 16, px);
        double delta = ((double)vmax[k] - (double)vmin[k]) / 255.0;
        for (int c = 0; c < 3; c++) H[k][c] = (double)vmin[k] + (double)px[texel * 4 + c] * delta;
    }
}

EXPORT void ref_decode_eval(const uint8_t *blocks, const uint8_t *fmt, const uint64_t *offset, uint32_t arr,
                            uint32_t n_streams, const float *vmin, const float *vmax, const float *dirs, uint32_t V,
                            const uint32_t *slots, uint64_t m, double *out, double *scale)
{
    #pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < (int64_t)m; j++) {
        double H[16][3];
        slot_coefficients(blocks, fmt, offset, arr, n_streams, vmin, vmax, slots[j], H);
        for (uint32_t v = 0; v < V; v++) {
            double Y[16];
            ref_sh_basis((double)dirs[v * 3 + 0], (double)dirs[v * 3 + 1], (double)dirs[v * 3 + 2], Y);
            for (int c = 0; c < 3; c++) {
                double acc = 0.0, mag = 0.0;
                for (int k = 0; k < 16; k++) {
                    acc += H[k][c] * Y[k];
                    mag += fabs(H[k][c] * Y[k]);
                }
                out[((uint64_t)v * m + j) * 3 + c] = acc;
                if (scale) scale[((uint64_t)v * m + j) * 3 + c] = mag;
            }
        }
    }
}

/* View-dependent colour of each listed slot from one view position f
 * (Sec. II colour equation c(f) = H w(f - p)): the SH basis is evaluated at
 * the unit vector d = (f - p) / |f - p| from the primitive towards the view
 * position (d = 0 when f = p), all in FP64 from the FP32 inputs.  pos is in
 * input order; perm maps a slot to its primitive. */
EXPORT void ref_decode_eval_view(const uint8_t *blocks, const uint8_t *fmt, const uint64_t *offset, uint32_t arr,
                                 uint32_t n_streams, const float *vmin, const float *vmax, const float *pos, const uint32_t *perm,
                                 const float *view, const uint32_t *slots, uint64_t m, double *out, double *scale)
{
    #pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < (int64_t)m; j++) {
        uint32_t s = slots[j];
        const float *p = pos + 3 * (uint64_t)perm[s];
        double d[3], r2 = 0.0;
        for (int c = 0; c < 3; c++) {
            d[c] = (double)view[c] - (double)p[c];
            r2 += d[c] * d[c];
        }
        double r = sqrt(r2);
        for (int c = 0; c < 3; c++) d[c] = r > 0.0 ? d[c] / r : 0.0;
        double Y[16];
        ref_sh_basis(d[0], d[1], d[2], Y);
        double H[16][3];
        slot_coefficients(blocks, fmt, offset, arr, n_streams, vmin, vmax, s, H);
        for (int c = 0; c < 3; c++) {
            double acc = 0.0, mag = 0.0;
            for (int k = 0; k < 16; k++) {
                acc += H[k][c] * Y[k];
                mag += fabs(H[k][c] * Y[k]);
            }
            out[(uint64_t)j * 3 + c] = acc;
            if (scale) scale[(uint64_t)j * 3 + c] = mag;
        }
    }
}

/* Colour stage of a tile rasteriser (Sec. II, eq. preblend with the
 * premultiplied coefficients of eq. premult): for each pixel of a tile the
 * primitives of the tile's list, front to back, add
 *     g_i(x) * ctilde_i * T_i,   T_1 = 1,  T_{i+1} = T_i (1 - mu_i g_i(x)),
 * where ctilde_i = Htilde_i w(f - p_i) is the primitive's decoded colour seen
 * from the view position f (the stored coefficients are Htilde = mu H), mu_i
 * its opacity and g_i(x) = exp(-q/2), q = a dx^2 + 2 b dx dy + c dy^2 its
 * projected footprint at the pixel centre: (dx, dy) = (px + 1/2, py + 1/2)
 * minus the footprint's mean.  Image of tiles_x by tiles_y tiles of 16 by 16
 * pixels; list[tile_start[t] .. tile_start[t+1]) holds the slot ids of tile t
 * (t = ty * tiles_x + tx) in depth order; pos, mu and foot (mean x, mean y,
 * a, b, c) are per primitive in input order, perm maps a slot to its
 * primitive.  All in FP64 from the FP32 inputs; out[y][x][3] the colour,
 * trans[y][x] the final transmittance, bound[y][x][3] = sum_i g_i T_i
 * sum_k |Htilde_ik Y_k| (the size of the terms) and bound_t[y][x][3] =
 * sum_i i g_i sum_k |Htilde_ik Y_k| (i from 1: the terms weighted by the
 * number of transmittance factors before them). */
static void view_colour(const uint8_t *blocks, const uint8_t *fmt, const uint64_t *offset, uint32_t arr, uint32_t ns,
                        const float *vmin, const float *vmax, const float *pos, const uint32_t *perm,
                        const float *view, uint32_t s, double col[3], double mag[3])
{
    const float *p = pos + 3 * (uint64_t)perm[s];
    double d[3], r2 = 0.0;
    for (int c = 0; c < 3; c++) {
        d[c] = (double)view[c] - (double)p[c];
        r2 += d[c] * d[c];
    }
    double r = sqrt(r2);
    for (int c = 0; c < 3; c++) d[c] = r > 0.0 ? d[c] / r : 0.0;
    double Y[16], H[16][3];
    ref_sh_basis(d[0], d[1], d[2], Y);
    slot_coefficients(blocks, fmt, offset, arr, ns, vmin, vmax, s, H);
    for (int c = 0; c < 3; c++) {
        col[c] = 0.0;
        mag[c] = 0.0;
        for (int k = 0; k < 16; k++) {
            col[c] += H[k][c] * Y[k];
            mag[c] += fabs(H[k][c] * Y[k]);
        }
    }
}

EXPORT void ref_blend_tiles(const uint8_t *blocks, const uint8_t *fmt, const uint64_t *offset, uint32_t arr,
                            uint32_t n_streams, const float *vmin, const float *vmax, const float *pos,
                            const uint32_t *perm, const float *view, const float *mu, const float *foot,
                            const uint32_t *tile_start, const uint32_t *list, uint32_t tiles_x, uint32_t tiles_y,
                            double *out, double *trans, double *bound, double *bound_t)
{
    const uint64_t W = 16 * (uint64_t)tiles_x;
    #pragma omp parallel for schedule(dynamic)
    for (int64_t t = 0; t < (int64_t)tiles_x * tiles_y; t++) {
        const uint32_t b0 = tile_start[t], b1 = tile_start[t + 1];
        const uint64_t tx = (uint64_t)t % tiles_x, ty = (uint64_t)t / tiles_x;
        /* the colour of each listed primitive does not depend on the pixel */
        double (*col)[3] = malloc(sizeof(double[3]) * (b1 > b0 ? b1 - b0 : 1));
        double (*mag)[3] = malloc(sizeof(double[3]) * (b1 > b0 ? b1 - b0 : 1));
        for (uint32_t e = b0; e < b1; e++)
            view_colour(blocks, fmt, offset, arr, n_streams, vmin, vmax, pos, perm, view, list[e], col[e - b0],
                        mag[e - b0]);
        for (int py = 0; py < 16; py++)
            for (int px = 0; px < 16; px++) {
                const double x = (double)(16 * tx + px) + 0.5, y = (double)(16 * ty + py) + 0.5;
                double a[3] = {0.0, 0.0, 0.0}, bd[3] = {0.0, 0.0, 0.0}, bt[3] = {0.0, 0.0, 0.0}, T = 1.0;
                for (uint32_t e = b0; e < b1; e++) {
                    const uint32_t i = perm[list[e]];
                    const float *F = foot + 5 * (uint64_t)i;
                    const double dx = x - (double)F[0], dy = y - (double)F[1];
                    const double q = (double)F[2] * dx * dx + 2.0 * (double)F[3] * dx * dy + (double)F[4] * dy * dy;
                    const double g = exp(-0.5 * q);
                    for (int c = 0; c < 3; c++) {
                        a[c] += g * col[e - b0][c] * T;
                        bd[c] += g * T * mag[e - b0][c];
                        bt[c] += (double)(e - b0 + 1) * g * mag[e - b0][c];
                    }
                    T *= 1.0 - (double)mu[i] * g;
                }
                const uint64_t o = (16 * ty + (uint64_t)py) * W + 16 * tx + (uint64_t)px;
                for (int c = 0; c < 3; c++) {
                    out[3 * o + c] = a[c];
                    if (bound) bound[3 * o + c] = bd[c];
                    if (bound_t) bound_t[3 * o + c] = bt[c];
                }
                if (trans) trans[o] = T;
            }
        free(col);
        free(mag);
    }
}

/* ======================================================================
 * Brute-force searchers used only to pin the encoders on tiny inputs.
 * ====================================================================== */

/* Least BC1 SSE over every endpoint pair (c0, c1) in [0, 65536)^2 for a
 * block holding colour cols[j] count[j] times (j < nc), each texel taking
 * its best palette entry. */
EXPORT uint64_t ref_bc1_bruteforce(const int *cols, const int *count, int nc)
{
    uint64_t best = UINT64_MAX;
    #pragma omp parallel
    {
        uint64_t local = UINT64_MAX;
        #pragma omp for schedule(dynamic, 256)
        for (int c0 = 0; c0 < 65536; c0++) {
            for (int c1 = 0; c1 < 65536; c1++) {
                int pal[4][4];
                bc1_palette((uint32_t)c0, (uint32_t)c1, pal);
                uint64_t s = 0;
                for (int j = 0; j < nc; j++) {
                    int bd = 1 << 30;
                    for (int k = 0; k < 4; k++) {
                        int d = 0;
                        for (int c = 0; c < 3; c++) {
                            int e = cols[j * 3 + c] - pal[k][c];
                            d += e * e;
                        }
                        if (d < bd) bd = d;
                    }
                    s += (uint64_t)bd * (uint64_t)count[j];
                }
                if (s < local) local = s;
            }
        }
        #pragma omp critical
        if (local < best) best = local;
    }
    return best;
}
