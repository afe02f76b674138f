// bc1_encode.hip -- BC1 encoder for gfx950 (BTC with two RGB565 reference
// colours and 2-bit indices, Sec. III-A; the paper codes each 4x4 band block
// this way, Sec. V).
//
// One lane codes one block, so the whole split enumeration of the cluster
// fit runs in wave-uniform order: the split bounds, cluster weights and
// normal-equation determinants are scalar, and each lane only evaluates its
// own numerators, quantised endpoints and SSE.  Per-lane prefix sums of the
// ordered texels live in LDS, one column per lane (conflict-free reads at a
// uniform row), and so does the nearest-code table.  Every decision is
// integer; ties take the first candidate in the fixed enumeration order.
//
// Steps: constant block -> per-channel endpoint tables; otherwise principal
// axis by integer power iteration, texels ordered by projection, every
// 4-cluster and 3-cluster split fitted by least squares and scored by its
// exact SSE, the best canonicalised and re-indexed, then `refine_steps`
// rounds of +-1 moves of the six endpoint channels.
#include "gsbc_internal.h"
#include "bc_format.h"

#include <cstdlib>
#include <mutex>
#include <vector>

namespace gsbc {
namespace {


// Constant-colour endpoint tables per channel width (0: 5 bits, 1: 6 bits),
// the nearest-code table of the cluster fit (code[w][h] is the number of
// codes c < max with E(c) + E(c+1) < h), and for every split of the 4- and
// 3-cluster lists, in enumeration order, the division multiplier
// ceil(2^36 / det) of its determinant (0 where det = 0).
constexpr int kSplits4 = 969, kSplits3 = 153;
struct Bc1Tables {
    uint8_t a4[2][256], b4[2][256], e4[2][256];
    uint8_t a3[2][256], b3[2][256], e3[2][256];
    uint8_t code[2][512];
    uint32_t magic4[kSplits4], magic3[kSplits3];
};
__constant__ Bc1Tables kTab;

// Per-workgroup LDS: -2 x the prefix sums of the ordered texels (16-bit:
// |-2 P| <= 8160), row 3 s + c holding channel c of the sum over the first s
// texels, one column per lane; and the nearest-code table with its expanded
// values.
template <int LANES>
struct Bc1Lds {
    short m2P[17 * 3][LANES];
    uint8_t code[2][512];
    uint8_t val[2][512];
};

__host__ __device__ inline int e5(int c) { return (c << 3) | (c >> 2); }
__host__ __device__ inline int e6(int c) { return (c << 2) | (c >> 4); }
__host__ __device__ inline int ew(int c, int wide) { return wide ? e6(c) : e5(c); }

__device__ inline int bitlen(int x) { return 32 - __clz(x); }

typedef short short2_t __attribute__((ext_vector_type(2)));

// Nearest code to t = y / (2 det), det > 0 (least |E(c) det - y/2|, lowest c
// on ties).  E is strictly increasing, so moving from c to c+1 helps exactly
// when the midpoint (E(c) + E(c+1)) / 2 lies below t; the answer is the
// number of such midpoints, a table lookup at h = ceil(y / det) clamped to
// [0, 511] (every midpoint sum is an integer in [4, 506]).
// ceil(y / det) is taken as ceil(y * inv - 2^-24) in FP64: y / det is a
// multiple of 1/det >= 1/5184 (determinants of the split lists lie in
// [60, 5184]), so any value within 2^-24 below it has the same ceiling, and
// with inv within 2^-44 of 1/det and |y| < 2^25 the FP64 error is below
// 2^-28.
__device__ __forceinline__ double recip(int det)
{
    const double d = (double)det;
    const double x = (double)__builtin_amdgcn_rcpf((float)det);   // within 2^-22
    return fma(fma(-d, x, 1.0), x, x);                           // one Newton step
}

__device__ __forceinline__ int quant_h(int y, double inv)
{
    const int h = (int)ceil(fma((double)y, inv, -0x1p-24));
    return min(max(h, 0), 511);
}

// The same h in integer arithmetic for a wave-uniform det with M =
// ceil(2^36 / det): y is clamped to [1 - det, 511 det] (which leaves the
// clamped ceiling unchanged), then ceil(y / det) = floor(n / det) with
// n = y + det - 1 in [0, 2^22), and floor(n / det) = floor(n M / 2^36) for
// every n < 2^23 because det <= 2^13 (the multiplier's error n e / 2^36,
// e < 1, stays below 2^-13 <= 1/det, the least distance of n/det below the
// next integer).
__device__ __forceinline__ int quant_h_int(int y, int det, uint32_t M)
{
    // the clamp as a median of three (one v_med3_i32): 1 - det <= 0 < 511 det
    const int lo = 1 - det, hi = 511 * det;
    const int yc = max(min(y, lo), min(max(y, lo), hi));
    return (int)(__umulhi((uint32_t)(yc + det - 1), M) >> 4);
}

__device__ inline uint32_t pack565(int r, int g, int b) { return ((uint32_t)r << 11) | ((uint32_t)g << 5) | (uint32_t)b; }

// Order the pair for the mode (4-colour: c0 > c1, 3-colour: c0 <= c1), then
// give each texel its least-SSE palette entry (lowest index on ties).  With
// entry k held as (-128 pR, -128 pG), -128 pB and 64 |p|^2 + k, the key
// 64 (|p|^2 - 2 x.p) + k is one 24-bit multiply-add and one 16-bit dot
// product on the texel's (R, G) pair and B, both taken from its RGBA word
// (one byte permute and one bit-field extract).  The least keys summed over
// the 16 texels plus 64 sum |x|^2 (= 64 Q, the same for every palette) are
// 64 SSE + sum k, and the k terms stay below 64.  Indices enter a shift
// register from the top, so texel 0 ends in bits 0-1.  The texels stay as
// their 16 RGBA words (not unpacked) so that they hold few registers across
// the split search.
__device__ inline uint32_t canon_index(uint32_t &c0, uint32_t &c1, bool four, const uint32_t (&t)[16], int Q,
                                       uint32_t &indices)
{
    if ((four && c0 < c1) || (!four && c0 > c1)) { uint32_t u = c0; c0 = c1; c1 = u; }
    int p[4][3];
    int e0[3], e1[3];
    bc1_expand(c0, e0);
    bc1_expand(c1, e1);
    const bool m4 = c0 > c1;
#pragma unroll
    for (int c = 0; c < 3; c++) {
        p[0][c] = e0[c];
        p[1][c] = e1[c];
        if (m4) {
            p[2][c] = (uint32_t)(2 * e0[c] + e1[c] + 1) / 3u;
            p[3][c] = (uint32_t)(e0[c] + 2 * e1[c] + 1) / 3u;
        } else {
            p[2][c] = (e0[c] + e1[c] + 1) >> 1;
            p[3][c] = 0;
        }
    }
    uint32_t prg[4];
    int pb[4], pk[4];
#pragma unroll
    for (int k = 0; k < 4; k++) {
        prg[k] = ((uint32_t)(-128 * p[k][0]) & 0xFFFFu) | ((uint32_t)(-128 * p[k][1]) << 16);
        pb[k] = -128 * p[k][2];
        pk[k] = 64 * (mul_i24(p[k][0], p[k][0]) + mul_i24(p[k][1], p[k][1]) + mul_i24(p[k][2], p[k][2])) + k;
    }
    uint32_t acc = 64u * (uint32_t)Q, idx = 0;
#pragma unroll
    for (int i = 0; i < 16; i++) {
        // R | G << 16 (bytes 0 and 1 of the RGBA word to bytes 0 and 2) and B
        const uint32_t rg = __builtin_amdgcn_perm(0u, t[i], 0x0C010C00u);
        const int b = (int)__builtin_amdgcn_ubfe(t[i], 16, 8);
        int kb = 0x7FFFFFFF;
#pragma unroll
        for (int k = 0; k < 4; k++)
            kb = min(kb, __builtin_amdgcn_sdot2(__builtin_bit_cast(short2_t, rg), __builtin_bit_cast(short2_t, prg[k]),
                                                mul_i24(b, pb[k]) + pk[k], false));
        acc += (uint32_t)kb;
        idx = __builtin_amdgcn_alignbit((uint32_t)kb, idx, 2);
    }
    indices = idx;
    return acc >> 6;
}

// Cluster fit over one split list in enumeration order (4-colour: s1 <= s2 <=
// s3; 3-colour: s1 <= s2, s3 = 16).  The split bounds, weights and
// determinant are wave-uniform; each lane forms its numerators from the
// prefix sums, quantises, and scores the exact SSE of the split
//   Q + sum_j p_j (n_j p_j - 2 X_j)
// per channel.  With SA + SB = F tot, the numerators are
//   2 num0 = -F (B + AB) (-2 SA) - 2 F AB F tot
//   2 num1 =  F (A + AB) (-2 SA) + 2 F A F tot.
// The best split (strictly less SSE, so the first on ties) is kept by its
// packed bounds.
template <bool FOUR, class Lds>
__device__ __forceinline__ void split_list(const Lds &L, int lane, const int (&tot)[3], const int (&m2tot)[3],
                                           int Q, uint32_t &best, uint32_t &best_split)
{
    constexpr int F = FOUR ? 3 : 2;
    const uint32_t *magic = FOUR ? kTab.magic4 : kTab.magic3;
    int si = 0;   // split number in enumeration order
    for (int s1 = 0; s1 <= 16; s1++) {
        int a[3];
#pragma unroll
        for (int c = 0; c < 3; c++) a[c] = L.m2P[s1 * 3 + c][lane];
        for (int s2 = s1; s2 <= 16; s2++) {
            // prefix values of the outer bounds, and their sum and difference,
            // once per (s1, s2) instead of once per split
            int bq[3], ab[3];
            // (a, bq - a) and (-bq, m2tot) in 16-bit halves (|values| <= 2 * 16 * 255)
            short2_t abm[3], bm[3];
#pragma unroll
            for (int c = 0; c < 3; c++) {
                bq[c] = L.m2P[s2 * 3 + c][lane];
                ab[c] = a[c] + bq[c];
                abm[c] = short2_t{(short)a[c], (short)(bq[c] - a[c])};
                bm[c] = short2_t{(short)(-bq[c]), (short)m2tot[c]};
            }
            for (int s3 = FOUR ? s2 : 16; s3 <= 16; s3++) {
                const uint32_t M = magic[si++];
                const int n0 = s1, n1 = s2 - s1, n2 = s3 - s2, n3 = 16 - s3;
                const int A = FOUR ? 9 * n0 + 4 * n1 + n2 : 4 * n0 + n1;
                const int B = FOUR ? n1 + 4 * n2 + 9 * n3 : n1 + 4 * n2;
                const int AB = FOUR ? 2 * (n1 + n2) : n1;
                const int det = A * B - AB * AB;
                if (det == 0) continue;
                const short2_t n01 = {(short)n0, (short)n1}, n23 = {(short)n2, (short)n3};
                int sse = Q;
#pragma unroll
                for (int c = 0; c < 3; c++) {
                    const int wide = c == 1;
                    const int cq = FOUR ? L.m2P[s3 * 3 + c][lane] : m2tot[c];
                    const int sam = FOUR ? ab[c] + cq : ab[c];   // -2 SA
                    const int y0 = mul_i24(sam, -F * (B + AB)) + mul_i24(tot[c], -2 * F * F * AB);
                    const int y1 = mul_i24(sam, F * (A + AB)) + mul_i24(tot[c], 2 * F * F * A);
                    const int e0 = L.val[wide][quant_h_int(y0, det, M)];
                    const int e1 = L.val[wide][quant_h_int(y1, det, M)];
                    if (FOUR) {
                        // (2 e0 + e1 + 1) / 3 and (e0 + 2 e1 + 1) / 3 as (v * 43691) >> 17, exact for v < 2^17
                        const int p1 = (int)((mul_u24((uint32_t)(2 * e0 + e1), 43691u) + 43691u) >> 17);
                        const int p2 = (int)((mul_u24((uint32_t)(e0 + 2 * e1), 43691u) + 43691u) >> 17);
                        // p (n p + d) for the four clusters as two 16-bit
                        // multiply-adds and two dot products (|n p + d| < 2^14)
                        // codes and interpolants are 0..255: packed without masking
                        const short2_t pe01 = __builtin_bit_cast(short2_t, (uint32_t)e0 | ((uint32_t)p1 << 16));
                        const short2_t pe23 = __builtin_bit_cast(short2_t, (uint32_t)p2 | ((uint32_t)e1 << 16));
                        // (cq - bq, m2tot - cq) = (cq, cq) * (1, -1) + (-bq, m2tot)
                        const short2_t d23 = short2_t{(short)cq, (short)cq} * short2_t{1, -1} + bm[c];
                        sse = __builtin_amdgcn_sdot2(pe01, n01 * pe01 + abm[c], sse, false);
                        sse = __builtin_amdgcn_sdot2(pe23, n23 * pe23 + d23, sse, false);
                    } else {
                        const int p1 = (e0 + e1 + 1) >> 1;
                        const short2_t pe01 = __builtin_bit_cast(short2_t, (uint32_t)e0 | ((uint32_t)p1 << 16));
                        sse = __builtin_amdgcn_sdot2(pe01, n01 * pe01 + abm[c], sse, false);
                        sse += mul_i24(e1, mul_i24(n2, e1) + (m2tot[c] - bq[c]));
                    }
                }
                if ((uint32_t)sse < best) {
                    best = (uint32_t)sse;
                    best_split = (uint32_t)s1 | ((uint32_t)s2 << 5) | ((uint32_t)s3 << 10) | (FOUR ? 1u << 15 : 0u);
                }
            }
        }
    }
}

// Endpoint codes of one split (the same arithmetic as split_list).
template <class Lds>
__device__ __forceinline__ void split_codes(const Lds &L, int lane, const int (&tot)[3], const int (&m2tot)[3], uint32_t split,
                            int (&q0)[3], int (&q1)[3])
{
    const bool four = (split >> 15) & 1;
    const int s1 = split & 31, s2 = (split >> 5) & 31, s3 = (split >> 10) & 31;
    const int F = four ? 3 : 2;
    const int n0 = s1, n1 = s2 - s1, n2 = s3 - s2, n3 = 16 - s3;
    const int A = four ? 9 * n0 + 4 * n1 + n2 : 4 * n0 + n1;
    const int B = four ? n1 + 4 * n2 + 9 * n3 : n1 + 4 * n2;
    const int AB = four ? 2 * (n1 + n2) : n1;
    const int det = A * B - AB * AB;
    const double inv = recip(det);
#pragma unroll
    for (int c = 0; c < 3; c++) {
        const int wide = c == 1;
        const int a = L.m2P[s1 * 3 + c][lane], bq = L.m2P[s2 * 3 + c][lane];
        const int cq = four ? L.m2P[s3 * 3 + c][lane] : m2tot[c];
        const int sam = four ? a + bq + cq : a + bq;
        const int y0 = sam * (-F * (B + AB)) + tot[c] * (-2 * F * F * AB);
        const int y1 = sam * (F * (A + AB)) + tot[c] * (2 * F * F * A);
        q0[c] = L.code[wide][quant_h(y0, inv)];
        q1[c] = L.code[wide][quant_h(y1, inv)];
    }
}

template <class Lds>
__device__ __forceinline__ void encode_block(const uint32_t (&t)[16], uint32_t refine_steps, Lds &L, int lane, uint32_t &w0,
                             uint32_t &w1, uint32_t &sse_out)
{
    // sum of |x|^2 over the texels (the palette-independent part of the SSE)
    int Q = 0;
#pragma unroll
    for (int i = 0; i < 16; i++) {
        const uint32_t rgb = t[i] & 0xFFFFFFu;
        Q += (int)__builtin_amdgcn_udot4(rgb, rgb, 0u, false);
    }
    bool constant = true;
#pragma unroll
    for (int i = 1; i < 16; i++) constant &= ((t[i] ^ t[0]) & 0xFFFFFFu) == 0;

    uint32_t c0, c1, idx, sse;
    if (constant) {
        int a4[3], b4[3], a3[3], b3[3], err4 = 0, err3 = 0;
#pragma unroll
        for (int c = 0; c < 3; c++) {
            int wide = c == 1, v = (int)((t[0] >> (8 * c)) & 255u);
            a4[c] = kTab.a4[wide][v]; b4[c] = kTab.b4[wide][v];
            a3[c] = kTab.a3[wide][v]; b3[c] = kTab.b3[wide][v];
            int e4 = kTab.e4[wide][v], e3 = kTab.e3[wide][v];
            err4 += e4 * e4;
            err3 += e3 * e3;
        }
        bool four = err4 <= err3;
        c0 = four ? pack565(a4[0], a4[1], a4[2]) : pack565(a3[0], a3[1], a3[2]);
        c1 = four ? pack565(b4[0], b4[1], b4[2]) : pack565(b3[0], b3[1], b3[2]);
        sse = canon_index(c0, c1, four, t, Q, idx);
        w0 = c0 | (c1 << 16);
        w1 = idx;
        sse_out = sse;
        return;
    }

    // ---- principal axis (integer power iteration, int32 exact)
    int S[3] = {0, 0, 0}, XX[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
#pragma unroll
    for (int i = 0; i < 16; i++) {
        const int x[3] = {(int)(t[i] & 255u), (int)((t[i] >> 8) & 255u), (int)((t[i] >> 16) & 255u)};
#pragma unroll
        for (int a = 0; a < 3; a++) {
            S[a] += x[a];
#pragma unroll
            for (int b = a; b < 3; b++) XX[a][b] += x[a] * x[b];
        }
    }
    int C[3][3];
#pragma unroll
    for (int a = 0; a < 3; a++)
#pragma unroll
        for (int b = a; b < 3; b++) { C[a][b] = 16 * XX[a][b] - __mul24(S[a], S[b]); C[b][a] = C[a][b]; }
    // row of the largest diagonal entry (lowest index on ties), by selects
    const int j = (C[1][1] > C[0][0]) ? ((C[2][2] > C[1][1]) ? 2 : 1) : ((C[2][2] > C[0][0]) ? 2 : 0);
    const int dmax = j == 0 ? C[0][0] : (j == 1 ? C[1][1] : C[2][2]);
    const int tsh = max(0, bitlen(dmax) - 14);
    int Cs[3][3];
#pragma unroll
    for (int a = 0; a < 3; a++)
#pragma unroll
        for (int b = 0; b < 3; b++) Cs[a][b] = C[a][b] >> tsh;
    int v[3];
#pragma unroll
    for (int b = 0; b < 3; b++) v[b] = j == 0 ? Cs[0][b] : (j == 1 ? Cs[1][b] : Cs[2][b]);
    // |Cs| <= 2^14 and |v| <= 2^15: 16-bit dot products, exact 32-bit sums
    short2_t c01[3], c2[3];
#pragma unroll
    for (int a = 0; a < 3; a++) {
        c01[a] = short2_t{(short)Cs[a][0], (short)Cs[a][1]};
        c2[a] = short2_t{(short)Cs[a][2], (short)0};
    }
#pragma unroll
    for (int it = 0; it < 8; it++) {
        const short2_t v01 = {(short)v[0], (short)v[1]}, v2 = {(short)v[2], (short)0};
        int u[3];
#pragma unroll
        for (int a = 0; a < 3; a++)
            u[a] = __builtin_amdgcn_sdot2(c01[a], v01, __builtin_amdgcn_sdot2(c2[a], v2, 0, false), false);
        int m = max(abs(u[0]), max(abs(u[1]), abs(u[2])));
        int s = max(0, bitlen(m) - 15);
#pragma unroll
        for (int a = 0; a < 3; a++) v[a] = u[a] >> s;
    }
    if (v[0] == 0 && v[1] == 0 && v[2] == 0) v[0] = v[1] = v[2] = 1;

    // ---- order texels by (projection, index): rank, scatter, prefix sums
    const short2_t v01 = {(short)v[0], (short)v[1]};
    int proj[16];
#pragma unroll
    for (int i = 0; i < 16; i++)
        proj[i] = __builtin_amdgcn_sdot2(__builtin_bit_cast(short2_t, __builtin_amdgcn_perm(0u, t[i], 0x0C010C00u)), v01,
                                         __mul24((int)__builtin_amdgcn_ubfe(t[i], 16, 8), v[2]), false);
#pragma unroll
    for (int i = 0; i < 16; i++) {
        int r = 0;
#pragma unroll
        for (int k = 0; k < 16; k++)
            if (k != i) r += (k < i ? proj[k] <= proj[i] : proj[k] < proj[i]) ? 1 : 0;
        // texel of rank r parked in rows 3 r (R, G) and 3 r + 1 (B)
        L.m2P[3 * r][lane] = (short)(t[i] & 0xFFFFu);
        L.m2P[3 * r + 1][lane] = (short)((t[i] >> 16) & 255u);
    }
    // rows 3 k and 3 k + 1 still hold the texel of rank k when the prefix rows of k are written
    int run[3] = {0, 0, 0};
#pragma unroll
    for (int k = 0; k <= 16; k++) {
        const uint32_t x = k < 16 ? ((uint32_t)(uint16_t)L.m2P[3 * k][lane] | ((uint32_t)L.m2P[3 * k + 1][lane] << 16)) : 0u;
#pragma unroll
        for (int c = 0; c < 3; c++) L.m2P[3 * k + c][lane] = (short)(-2 * run[c]);
        run[0] += (int)(x & 255u);
        run[1] += (int)((x >> 8) & 255u);
        run[2] += (int)((x >> 16) & 255u);
    }
    const int tot[3] = {run[0], run[1], run[2]};
    const int m2tot[3] = {-2 * run[0], -2 * run[1], -2 * run[2]};

    // ---- cluster fit over every split (4-colour list, then 3-colour list)
    uint32_t best = 0xFFFFFFFFu, best_split = 1u << 15;
    split_list<true>(L, lane, tot, m2tot, Q, best, best_split);
    split_list<false>(L, lane, tot, m2tot, Q, best, best_split);
    int bq0[3], bq1[3];
    split_codes(L, lane, tot, m2tot, best_split, bq0, bq1);

    c0 = pack565(bq0[0], bq0[1], bq0[2]);
    c1 = pack565(bq1[0], bq1[1], bq1[2]);
    sse = canon_index(c0, c1, (best_split >> 15) & 1, t, Q, idx);

    // ---- refinement: best of the 12 one-step moves, taken if strictly better
    for (uint32_t step = 0; step < refine_steps; step++) {
        const bool four = c0 > c1;
        uint32_t nb_sse = 0xFFFFFFFFu, nb0 = 0, nb1 = 0, nbi = 0;
        // neighbour q moves channel q/2 (R0, G0, B0, R1, G1, B1) by -1 (q
        // even) or +1, clamped; one neighbour at a time (a rolled loop, so
        // that only one palette is live)
#pragma unroll 1
        for (int q = 0; q < 12; q++) {
            const int ch = q >> 1, c = ch % 3;
            const int shift = c == 0 ? 11 : c == 1 ? 5 : 0, maxc = c == 1 ? 63 : 31;
            const uint32_t word = ch < 3 ? c0 : c1;
            const int f = (int)((word >> shift) & (uint32_t)maxc) + ((q & 1) ? 1 : -1);
            const uint32_t moved = (word & ~((uint32_t)maxc << shift)) | ((uint32_t)min(max(f, 0), maxc) << shift);
            uint32_t a = ch < 3 ? moved : c0, b = ch < 3 ? c1 : moved, ii;
            const uint32_t s = canon_index(a, b, four, t, Q, ii);
            if (s < nb_sse) { nb_sse = s; nb0 = a; nb1 = b; nbi = ii; }
        }
        if (nb_sse < sse) { sse = nb_sse; c0 = nb0; c1 = nb1; idx = nbi; }
        else break;
    }
    w0 = c0 | (c1 << 16);
    w1 = idx;
    sse_out = sse;
}

// One lane per block over the run map; rounds of LANES blocks (a run never
// straddles a round since runs start at multiples of 256).
template <int LANES>
__global__ __launch_bounds__(LANES) __attribute__((amdgpu_waves_per_eu(4))) void k_bc1_encode(EncodeArgs a, WorkSplit w)
{
    __shared__ Bc1Lds<LANES> L;
    __shared__ uint32_t s_item;
    for (int e = threadIdx.x; e < 2 * 512; e += LANES) {
        const int wide = e >> 9, c = kTab.code[wide][e & 511];
        L.code[wide][e & 511] = (uint8_t)c;
        L.val[wide][e & 511] = (uint8_t)ew(c, wide);
    }
    __syncthreads();
    const uint64_t n_items = (a.total + (uint64_t)w.item_rounds * LANES - 1) / ((uint64_t)w.item_rounds * LANES);
    uint32_t item = blockIdx.x;
    if (w.queue) {
        if (threadIdx.x == 0) s_item = atomicAdd(w.queue, 1u);
        __syncthreads();
        item = s_item;
    }
    while (item < n_items) {
        for (uint32_t r = 0; r < w.item_rounds; r++) {
            const uint64_t g0 = ((uint64_t)item * w.item_rounds + r) * LANES;
            if (g0 >= a.total) break;
            const BlockRun run = a.run[find_run(a.run, a.nrun, g0)];
            const uint64_t b = g0 - run.gbase + threadIdx.x;
            const bool live = b < run.nblk;
            if (__ballot(live) == 0) continue;   // padding (per wave; no barriers below)
            const uint64_t bl = live ? b : run.nblk - 1;   // dead lanes redo the last block, write nothing
            const uint4 *src = reinterpret_cast<const uint4 *>(run.src + bl * 64);
            uint32_t t[16];
#pragma unroll
            for (int q = 0; q < 4; q++) {
                uint4 v = src[q];
                t[4 * q] = v.x; t[4 * q + 1] = v.y; t[4 * q + 2] = v.z; t[4 * q + 3] = v.w;
            }
            uint32_t w0, w1, sse;
            encode_block(t, a.refine_steps, L, threadIdx.x, w0, w1, sse);
            if (live) {
                uint2 *dst = reinterpret_cast<uint2 *>(run.dst + b * 8);
                *dst = make_uint2(w0, w1);
                if (b == run.nblk - 1 && (run.nblk & 1)) dst[1] = make_uint2(0, 0);   // 16-byte stream alignment
            }
            if (run.sse) band_add(run.sse, 0, sse, live);
        }
        if (!w.queue) break;
        __syncthreads();   // every thread has read s_item
        if (threadIdx.x == 0) s_item = atomicAdd(w.queue, 1u);
        __syncthreads();
        item = s_item;
    }
}

// Host-side construction of the constant-colour tables: for each channel
// width and target value, the code pair whose 4-colour 2/3 point (resp.
// 3-colour midpoint) is nearest the target; ties by |a-b|, then a, then b.
void build_tables(Bc1Tables &T)
{
    for (int wide = 0; wide < 2; wide++) {
        const int nc = wide ? 64 : 32;
        for (int mode = 0; mode < 2; mode++) {
            // every pair's value, then the best pair per target
            std::vector<int> val(nc * nc);
            for (int a = 0; a < nc; a++)
                for (int b = 0; b < nc; b++) {
                    int ea = ew(a, wide), eb = ew(b, wide);
                    val[a * nc + b] = mode == 0 ? (2 * ea + eb + 1) / 3 : (ea + eb + 1) >> 1;
                }
            for (int v = 0; v < 256; v++) {
                int best = -1;
                int be = 0, bd = 0;
                for (int pr = 0; pr < nc * nc; pr++) {
                    int a = pr / nc, b = pr % nc;
                    int e = val[pr] > v ? val[pr] - v : v - val[pr];
                    int d = a > b ? a - b : b - a;
                    // pairs are visited in (a, b) order, so strict comparisons keep the lowest
                    if (best < 0 || e < be || (e == be && d < bd)) { best = pr; be = e; bd = d; }
                }
                uint8_t *A = mode == 0 ? T.a4[wide] : T.a3[wide];
                uint8_t *B = mode == 0 ? T.b4[wide] : T.b3[wide];
                uint8_t *E = mode == 0 ? T.e4[wide] : T.e3[wide];
                A[v] = (uint8_t)(best / nc);
                B[v] = (uint8_t)(best % nc);
                E[v] = (uint8_t)be;
            }
        }
        for (int h = 0; h < 512; h++) {
            int n = 0;
            for (int c = 0; c + 1 < nc; c++) n += ew(c, wide) + ew(c + 1, wide) < h;
            T.code[wide][h] = (uint8_t)n;
        }
    }
    // split multipliers, enumerated as the device's split lists are
    for (int four = 0; four < 2; four++) {
        uint32_t *M = four ? T.magic4 : T.magic3;
        int si = 0;
        for (int s1 = 0; s1 <= 16; s1++)
            for (int s2 = s1; s2 <= 16; s2++)
                for (int s3 = four ? s2 : 16; s3 <= 16; s3++) {
                    const int n0 = s1, n1 = s2 - s1, n2 = s3 - s2, n3 = 16 - s3;
                    const int A = four ? 9 * n0 + 4 * n1 + n2 : 4 * n0 + n1;
                    const int B = four ? n1 + 4 * n2 + 9 * n3 : n1 + 4 * n2;
                    const int AB = four ? 2 * (n1 + n2) : n1;
                    const long long det = (long long)A * B - (long long)AB * AB;
                    M[si++] = det > 0 ? (uint32_t)(((1ull << 36) + (unsigned long long)det - 1) / (unsigned long long)det)
                                      : 0u;
                }
        if (si != (four ? kSplits4 : kSplits3)) abort();
    }
}

}  // namespace

// The tables are built once per process and copied once per device, under a
// lock (contexts may be created from several threads; a context made later
// must not rewrite the constant tables while kernels of another read them).
hipError_t upload_bc1_tables(int device, hipStream_t st)
{
    static std::mutex lock;
    static Bc1Tables host;
    static bool built = false;
    static bool uploaded[kMaxDevices] = {};
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> guard(lock);
    if (!built) { build_tables(host); built = true; }
    if (uploaded[device]) return hipSuccess;
    hipError_t e = hipMemcpyToSymbolAsync(HIP_SYMBOL(kTab), &host, sizeof(host), 0, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e == hipSuccess) uploaded[device] = true;
    return e;
}

hipError_t launch_bc1_encode(const EncodeArgs &a, const WorkSplit &w, uint32_t lanes, hipStream_t st)
{
    if (a.total == 0) return hipSuccess;
    if (lanes != 64 && lanes != 128 && lanes != 256) return hipErrorInvalidValue;
    if (w.queue) {
        hipError_t f = launch_fill_u64(reinterpret_cast<unsigned long long *>(w.queue), 1, 0, st);
        if (f != hipSuccess) return f;
    }
    const uint64_t rounds = a.total / lanes;
    const dim3 grid(w.queue ? w.grid : (uint32_t)((rounds + w.item_rounds - 1) / w.item_rounds));
    if (lanes == 64) GSBC_LAUNCH("bc1_encode", k_bc1_encode<64>, grid, dim3(64), 0, st, a, w);
    else if (lanes == 128) GSBC_LAUNCH("bc1_encode", k_bc1_encode<128>, grid, dim3(128), 0, st, a, w);
    else GSBC_LAUNCH("bc1_encode", k_bc1_encode<256>, grid, dim3(256), 0, st, a, w);
    return hipGetLastError();
}

}  // namespace gsbc
