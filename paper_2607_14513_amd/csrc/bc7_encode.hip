// bc7_encode.hip -- BC7 encoder for gfx950 (BTC with 1-3 reference-colour
// pairs per block, Sec. III-B; the paper codes 4x4 band blocks this way,
// Sec. V).
//
// Search: 285 candidates in a fixed order (mode 0 partitions 0..15; modes
// 1, 2, 3 partitions 0..63; mode 4 rotation x index-selection; mode 5
// rotation; mode 6; mode 7 partitions 0..63).  Each subset is fitted on its
// own: identical texels use precomputed single-value endpoint tables;
// otherwise the endpoints are the texels of least and greatest projection on
// the principal axis (integer power iteration), quantised for every p-bit
// choice, texels take their least-SSE palette entry, and one least-squares
// refit is kept if it lowers the SSE.  The winner minimises
// (SSE << 9) | candidate, a total order, so the result is independent of how
// candidates are spread over lanes.
//
// Layout on the GPU: one lane per block, all lanes of a wave walk the
// candidates in the same order, so partition masks, anchors and mode
// parameters are wave-uniform (scalar registers) and only the texel
// arithmetic is per lane.  Pass 1 keeps only the best key; pass 2 re-fits
// each lane's winner (identical arithmetic) to emit its bits.
#include "gsbc_internal.h"
#include "bc_format.h"

#include <vector>

namespace gsbc {
namespace {

constexpr int kBlock = 64;

// ---- tables (device global memory, built on the host at first use)
// nearest[cls][p][t]: code c minimising |value(c, p) - t| (lowest on ties)
// in the low byte, value(c, p) in the high byte; cls = (cb - 4) * 2 + has_pbit.
// sv[cls][p0 + 2 p1][slot][v]: single-value pair (c0 | c1 << 8 | err << 16)
// whose interpolation at weight(nb, K) is nearest v; slot = nb offset + K.
struct Tables {
    const uint16_t *nearest;
    const uint32_t *sv;
};
constexpr int kSlots = 28;
__host__ __device__ constexpr int slot_of(int nb, int k) { return (nb == 2 ? 0 : nb == 3 ? 4 : 12) + k; }
__host__ __device__ constexpr int cls_of(int cb, int pb) { return (cb - 4) * 2 + (pb ? 1 : 0); }

__host__ __device__ constexpr int ep_value(int code, int p, int cb, int pb)
{
    return pb ? expand_bits((code << 1) | p, cb + 1) : expand_bits(code, cb);
}

__device__ __forceinline__ int bitlen(int x) { return 32 - __clz(x); }

// ---- one subset fit
struct Fit {
    int c0[3], c1[3];
    int p0, p1;
    uint32_t sse;
    uint64_t idx;   // 4 bits per texel (members only)
};

template <int CB, int PB, int NB, int NCH>
__device__ __forceinline__ void fit_eval(const int (&x)[16][3], uint32_t mask, const int (&elo)[3],
                                         const int (&ehi)[3], const Tables &T, Fit &out)
{
    constexpr int NPC = PB == 2 ? 4 : PB == 1 ? 2 : 1;
    constexpr int cls = cls_of(CB, PB);
    out.sse = 0xFFFFFFFFu;
#pragma unroll
    for (int pc = 0; pc < NPC; pc++) {
        const int p0 = PB == 2 ? (pc & 1) : PB == 1 ? pc : 0;
        const int p1 = PB == 2 ? (pc >> 1) : PB == 1 ? pc : 0;
        Fit f;
        f.p0 = p0;
        f.p1 = p1;
        int d0[3] = {0, 0, 0}, d1[3] = {0, 0, 0};
#pragma unroll
        for (int c = 0; c < NCH; c++) {
            f.c0[c] = T.nearest[(cls * 2 + p0) * 256 + elo[c]] & 255;
            f.c1[c] = T.nearest[(cls * 2 + p1) * 256 + ehi[c]] & 255;
            d0[c] = ep_value(f.c0[c], p0, CB, PB);
            d1[c] = ep_value(f.c1[c], p1, CB, PB);
        }
        int pal[1 << NB][3];
#pragma unroll
        for (int k = 0; k < (1 << NB); k++)
#pragma unroll
            for (int c = 0; c < NCH; c++) pal[k][c] = interp64(d0[c], d1[c], bc7_weight(NB, k));
        uint32_t sse = 0;
        uint64_t idx = 0;
#pragma unroll
        for (int i = 0; i < 16; i++) {
            if (!((mask >> i) & 1)) continue;
            uint32_t best = 0xFFFFFFFFu;
#pragma unroll
            for (int k = 0; k < (1 << NB); k++) {
                uint32_t d = 0;
#pragma unroll
                for (int c = 0; c < NCH; c++) {
                    int e = x[i][c] - pal[k][c];
                    d += (uint32_t)(e * e);
                }
                uint32_t key = (d << 4) | (uint32_t)k;   // d < 2^18; lowest index on ties
                best = key < best ? key : best;
            }
            sse += best >> 4;
            idx |= (uint64_t)(best & 15u) << (4 * i);
        }
        f.sse = sse;
        f.idx = idx;
        if (sse < out.sse) out = f;
    }
}

template <int CB, int PB, int NB, int NCH>
__device__ __forceinline__ void fit_subset(const int (&x)[16][3], uint32_t mask, const Tables &T, Fit &out)
{
    constexpr int NPC = PB == 2 ? 4 : PB == 1 ? 2 : 1;
    constexpr int cls = cls_of(CB, PB);
    const int first = __ffs(mask) - 1;
    const int n = __popc(mask);
    bool same = true;
#pragma unroll
    for (int i = 0; i < 16; i++)
        if ((mask >> i) & 1)
#pragma unroll
            for (int c = 0; c < NCH; c++) same &= x[i][c] == x[first][c];
    if (same) {
        // (a) single value: best (p-bits, index) over per-channel tables
        out.sse = 0xFFFFFFFFu;
        int v[3] = {0, 0, 0};
#pragma unroll
        for (int c = 0; c < NCH; c++) v[c] = x[first][c];
#pragma unroll
        for (int pc = 0; pc < NPC; pc++) {
            const int p0 = PB == 2 ? (pc & 1) : PB == 1 ? pc : 0;
            const int p1 = PB == 2 ? (pc >> 1) : PB == 1 ? pc : 0;
            for (int k = 0; k < (1 << NB); k++) {
                const uint32_t *row = T.sv + ((uint64_t)(cls * 4 + p0 + 2 * p1) * kSlots + slot_of(NB, k)) * 256;
                uint32_t e = 0;
                uint32_t ent[3] = {0, 0, 0};
#pragma unroll
                for (int c = 0; c < NCH; c++) {
                    ent[c] = row[v[c]];
                    uint32_t er = ent[c] >> 16;
                    e += er * er;
                }
                if (e < out.sse) {
                    out.sse = e;
                    out.p0 = p0;
                    out.p1 = p1;
#pragma unroll
                    for (int c = 0; c < NCH; c++) { out.c0[c] = ent[c] & 255; out.c1[c] = (ent[c] >> 8) & 255; }
                    uint64_t idx = 0;
#pragma unroll
                    for (int i = 0; i < 16; i++) idx |= (uint64_t)k << (4 * i);
                    out.idx = idx;
                }
            }
        }
        out.sse *= (uint32_t)n;
        return;
    }
    // (b) endpoints: least and greatest projection on the principal axis
    int elo[3] = {0, 0, 0}, ehi[3] = {0, 0, 0};
    if (NCH == 3) {
        int S[3] = {0, 0, 0}, XX[6] = {0, 0, 0, 0, 0, 0};
#pragma unroll
        for (int i = 0; i < 16; i++) {
            if (!((mask >> i) & 1)) continue;
            S[0] += x[i][0]; S[1] += x[i][1]; S[2] += x[i][2];
            XX[0] += x[i][0] * x[i][0]; XX[1] += x[i][0] * x[i][1]; XX[2] += x[i][0] * x[i][2];
            XX[3] += x[i][1] * x[i][1]; XX[4] += x[i][1] * x[i][2]; XX[5] += x[i][2] * x[i][2];
        }
        int C[3][3];
        C[0][0] = n * XX[0] - S[0] * S[0];
        C[0][1] = C[1][0] = n * XX[1] - S[0] * S[1];
        C[0][2] = C[2][0] = n * XX[2] - S[0] * S[2];
        C[1][1] = n * XX[3] - S[1] * S[1];
        C[1][2] = C[2][1] = n * XX[4] - S[1] * S[2];
        C[2][2] = n * XX[5] - S[2] * S[2];
        // row of the largest diagonal entry (lowest index on ties), by selects
        const int j = (C[1][1] > C[0][0]) ? ((C[2][2] > C[1][1]) ? 2 : 1) : ((C[2][2] > C[0][0]) ? 2 : 0);
        const int tsh = max(0, bitlen(j == 0 ? C[0][0] : (j == 1 ? C[1][1] : C[2][2])) - 14);
        int Cs[3][3];
#pragma unroll
        for (int a = 0; a < 3; a++)
#pragma unroll
            for (int b = 0; b < 3; b++) Cs[a][b] = C[a][b] >> tsh;
        int v[3];
#pragma unroll
        for (int b = 0; b < 3; b++) v[b] = j == 0 ? Cs[0][b] : (j == 1 ? Cs[1][b] : Cs[2][b]);
#pragma unroll
        for (int it = 0; it < 8; it++) {
            int u[3];
#pragma unroll
            for (int a = 0; a < 3; a++) u[a] = Cs[a][0] * v[0] + Cs[a][1] * v[1] + Cs[a][2] * v[2];
            int m = max(abs(u[0]), max(abs(u[1]), abs(u[2])));
            int s = max(0, bitlen(m) - 15);
#pragma unroll
            for (int a = 0; a < 3; a++) v[a] = u[a] >> s;
        }
        if (v[0] == 0 && v[1] == 0 && v[2] == 0) v[0] = v[1] = v[2] = 1;
        int plo = 0, phi = 0, ilo = first, ihi = first;
        bool any = false;
#pragma unroll
        for (int i = 0; i < 16; i++) {
            if (!((mask >> i) & 1)) continue;
            int p = v[0] * x[i][0] + v[1] * x[i][1] + v[2] * x[i][2];
            if (!any || p < plo) { plo = p; ilo = i; }
            if (!any || p > phi) { phi = p; ihi = i; }
            any = true;
        }
#pragma unroll
        for (int c = 0; c < 3; c++) { elo[c] = x[ilo][c]; ehi[c] = x[ihi][c]; }
    } else {
        int lo = 255, hi = 0;
#pragma unroll
        for (int i = 0; i < 16; i++) {
            if (!((mask >> i) & 1)) continue;
            lo = min(lo, x[i][0]);
            hi = max(hi, x[i][0]);
        }
        elo[0] = lo;
        ehi[0] = hi;
    }
    // (c)
    fit_eval<CB, PB, NB, NCH>(x, mask, elo, ehi, T, out);
    // (d) one least-squares refit with the chosen indices
    int A = 0, B = 0, AB = 0, SA[3] = {0, 0, 0}, SB[3] = {0, 0, 0};
#pragma unroll
    for (int i = 0; i < 16; i++) {
        if (!((mask >> i) & 1)) continue;
        int k = (int)((out.idx >> (4 * i)) & 15);
        int b = bc7_weight(NB, k & ((1 << NB) - 1)), a = 64 - b;
        A += a * a; B += b * b; AB += a * b;
#pragma unroll
        for (int c = 0; c < NCH; c++) { SA[c] += a * x[i][c]; SB[c] += b * x[i][c]; }
    }
    const int64_t det = (int64_t)A * B - (int64_t)AB * AB;
    if (det == 0) return;
    int rlo[3] = {0, 0, 0}, rhi[3] = {0, 0, 0};
    const double ddet = (double)det;
#pragma unroll
    for (int c = 0; c < NCH; c++) {
        int64_t n0 = 64 * ((int64_t)B * SA[c] - (int64_t)AB * SB[c]);
        int64_t n1 = 64 * ((int64_t)A * SB[c] - (int64_t)AB * SA[c]);
        // floor(n/det + 1/2): the double quotient is within 2^-45 of the exact
        // value for any value in range, and a half-integer tie is exact
        double q0 = floor((double)n0 / ddet + 0.5), q1 = floor((double)n1 / ddet + 0.5);
        rlo[c] = q0 < 0.0 ? 0 : (q0 > 255.0 ? 255 : (int)q0);
        rhi[c] = q1 < 0.0 ? 0 : (q1 > 255.0 ? 255 : (int)q1);
    }
    Fit g;
    fit_eval<CB, PB, NB, NCH>(x, mask, rlo, rhi, T, g);
    if (g.sse < out.sse) out = g;
}

// Anchor rule: the anchor texel's index must have its top bit clear.
template <int NB, int NCH>
__device__ __forceinline__ void anchor_fix(Fit &f, uint32_t mask, int anchor)
{
    int k = (int)((f.idx >> (4 * anchor)) & 15);
    if (!(k >> (NB - 1))) return;
#pragma unroll
    for (int c = 0; c < NCH; c++) { int t = f.c0[c]; f.c0[c] = f.c1[c]; f.c1[c] = t; }
    int t = f.p0; f.p0 = f.p1; f.p1 = t;
    uint64_t idx = f.idx;
#pragma unroll
    for (int i = 0; i < 16; i++)
        if ((mask >> i) & 1) {
            uint64_t m = (uint64_t)15 << (4 * i);
            uint64_t nk = (uint64_t)(((1 << NB) - 1) - (int)((idx >> (4 * i)) & 15));
            idx = (idx & ~m) | (nk << (4 * i));
        }
    f.idx = idx;
}

// ---- candidate geometry
__device__ __forceinline__ uint32_t mask3(int p, int s)
{
    uint32_t w = kPart3[p], m = 0;
#pragma unroll
    for (int i = 0; i < 16; i++) m |= (((w >> (2 * i)) & 3) == (uint32_t)s ? 1u : 0u) << i;
    return m;
}
__device__ __forceinline__ uint32_t mask2(int p, int s)
{
    uint32_t w = kPart2[p];
    return s ? w : (~w & 0xFFFFu);
}

// Colour triple and scalar values for rotation r (modes 4, 5): rotation
// moves channel r-1 to the scalar slot and leaves 255 in its place.
__device__ __forceinline__ void rotate(const int (&x)[16][3], int r, int (&t)[16][3], int (&s)[16][3])
{
#pragma unroll
    for (int i = 0; i < 16; i++) {
#pragma unroll
        for (int c = 0; c < 3; c++) t[i][c] = x[i][c];
        s[i][0] = 255; s[i][1] = 0; s[i][2] = 0;
        if (r) { s[i][0] = x[i][r - 1]; t[i][r - 1] = 255; }
    }
}

// Candidate index -> (mode, partition, rotation, index selection)
__device__ __forceinline__ void candidate(int ci, int &m, int &p, int &r, int &s)
{
    p = r = s = 0;
    if (ci < 16) { m = 0; p = ci; }
    else if (ci < 80) { m = 1; p = ci - 16; }
    else if (ci < 144) { m = 2; p = ci - 80; }
    else if (ci < 208) { m = 3; p = ci - 144; }
    else if (ci < 216) { m = 4; r = (ci - 208) >> 1; s = (ci - 208) & 1; }
    else if (ci < 220) { m = 5; r = ci - 216; }
    else if (ci < 221) { m = 6; }
    else { m = 7; p = ci - 221; }
}

// ---- pass 1: SSE of every candidate, best key
//
// Texels sit in LDS, one column per lane, as 4x-scaled packed values
// (rg = 4R | 4G << 16, b = 4B), so one texel x palette-entry distance with
// its index tie-break is five VALU ops:
//   d  = rg - prg            (v_pk_sub_i16)
//   db = b - pb              (v_sub_u32)
//   k' = db*db + k           (v_mad_i32_i24)       = 16*dB^2 + k
//   k' = d.x*d.x + d.y*d.y + k'  (v_dot2c_i32_i16)  = 16*SSE + k
//   best = min(best, k')     (v_min_u32)
// Subset masks are wave-uniform, so texel loops walk the set bits of the
// mask with scalar control.  The principal axis and the extreme texels of a
// subset depend only on the partition, so they are found once and shared by
// every mode with that partition (2-subset: modes 1, 3, 7; 3-subset: modes 0
// and 2; whole block: modes 4, 5 and 6).
constexpr int kSearchWG = 256;
constexpr int kQEntries = 10 * 2 * 256;

struct SearchLds {
    uint32_t rg[16][kSearchWG];
    uint32_t b[16][kSearchWG];
    uint16_t q[kQEntries];        // nearest-code table: code | value << 8
};

typedef short short2_t __attribute__((ext_vector_type(2)));

// Texel i of this lane; rotation r puts 4*255 in channel r-1.
__device__ __forceinline__ void texel(const SearchLds &S, int i, int rot, uint32_t &rg, int &b)
{
    rg = S.rg[i][threadIdx.x];
    b = (int)S.b[i][threadIdx.x];
    if (rot == 1) rg = (rg & 0xFFFF0000u) | 1020u;
    else if (rot == 2) rg = (rg & 0xFFFFu) | (1020u << 16);
    else if (rot == 3) b = 1020;
}

__device__ __forceinline__ void unpack(uint32_t rg, int b, int (&x)[3])
{
    x[0] = (int)((rg & 0xFFFFu) >> 2);
    x[1] = (int)(rg >> 18);
    x[2] = b >> 2;
}

// Per-subset data shared across modes: whether every member is the same
// colour, and the two endpoint colours (texels of least and greatest
// projection on the principal axis, or the common colour).
struct Prep {
    bool same;
    int lo[3], hi[3];
};

__device__ __forceinline__ Prep prep_subset(const SearchLds &S, uint32_t mask, int rot)
{
    Prep P;
    const int first = __ffs(mask) - 1;
    uint32_t rg0;
    int b0;
    texel(S, first, rot, rg0, b0);
    bool same = true;
    int Sx[3] = {0, 0, 0}, XX[6] = {0, 0, 0, 0, 0, 0};
    for (uint32_t m = mask; m; m &= m - 1) {
        uint32_t rg;
        int b;
        texel(S, __ffs(m) - 1, rot, rg, b);
        same &= (rg == rg0) && (b == b0);
        int x[3];
        unpack(rg, b, x);
        Sx[0] += x[0]; Sx[1] += x[1]; Sx[2] += x[2];
        XX[0] += x[0] * x[0]; XX[1] += x[0] * x[1]; XX[2] += x[0] * x[2];
        XX[3] += x[1] * x[1]; XX[4] += x[1] * x[2]; XX[5] += x[2] * x[2];
    }
    P.same = same;
    unpack(rg0, b0, P.lo);
    P.hi[0] = P.lo[0]; P.hi[1] = P.lo[1]; P.hi[2] = P.lo[2];
    if (same) return P;
    const int n = __popc(mask);
    int C[3][3];
    C[0][0] = n * XX[0] - Sx[0] * Sx[0];
    C[0][1] = C[1][0] = n * XX[1] - Sx[0] * Sx[1];
    C[0][2] = C[2][0] = n * XX[2] - Sx[0] * Sx[2];
    C[1][1] = n * XX[3] - Sx[1] * Sx[1];
    C[1][2] = C[2][1] = n * XX[4] - Sx[1] * Sx[2];
    C[2][2] = n * XX[5] - Sx[2] * Sx[2];
    // row of the largest diagonal entry (lowest index on ties), by selects
    const int j = (C[1][1] > C[0][0]) ? ((C[2][2] > C[1][1]) ? 2 : 1) : ((C[2][2] > C[0][0]) ? 2 : 0);
    const int tsh = max(0, bitlen(j == 0 ? C[0][0] : (j == 1 ? C[1][1] : C[2][2])) - 14);
    int Cs[3][3];
#pragma unroll
    for (int a = 0; a < 3; a++)
#pragma unroll
        for (int c = 0; c < 3; c++) Cs[a][c] = C[a][c] >> tsh;
    int v[3];
#pragma unroll
    for (int c = 0; c < 3; c++) v[c] = j == 0 ? Cs[0][c] : (j == 1 ? Cs[1][c] : Cs[2][c]);
#pragma unroll
    for (int it = 0; it < 8; it++) {
        int u[3];
#pragma unroll
        for (int a = 0; a < 3; a++) u[a] = Cs[a][0] * v[0] + Cs[a][1] * v[1] + Cs[a][2] * v[2];
        int mx = max(abs(u[0]), max(abs(u[1]), abs(u[2])));
        int sh = max(0, bitlen(mx) - 15);
#pragma unroll
        for (int a = 0; a < 3; a++) v[a] = u[a] >> sh;
    }
    if (v[0] == 0 && v[1] == 0 && v[2] == 0) v[0] = v[1] = v[2] = 1;
    int plo = 0, phi = 0;
    bool any = false;
    for (uint32_t m = mask; m; m &= m - 1) {
        uint32_t rg;
        int b;
        texel(S, __ffs(m) - 1, rot, rg, b);
        int x[3];
        unpack(rg, b, x);
        int p = v[0] * x[0] + v[1] * x[1] + v[2] * x[2];
        if (!any || p < plo) { plo = p; P.lo[0] = x[0]; P.lo[1] = x[1]; P.lo[2] = x[2]; }
        if (!any || p > phi) { phi = p; P.hi[0] = x[0]; P.hi[1] = x[1]; P.hi[2] = x[2]; }
        any = true;
    }
    return P;
}

// (c) for one endpoint pair: best p-bit combination's SSE and indices.
template <int CB, int PB, int NB>
__device__ __forceinline__ uint32_t eval_pair(const SearchLds &S, uint32_t mask, int rot, const int (&lo)[3],
                                              const int (&hi)[3], uint64_t &idx_out)
{
    constexpr int NPC = PB == 2 ? 4 : PB == 1 ? 2 : 1;
    constexpr int cls = cls_of(CB, PB);
    uint32_t best_sse = 0xFFFFFFFFu;
    uint64_t best_idx = 0;
    for (int pc = 0; pc < NPC; pc++) {
        const int p0 = PB == 2 ? (pc & 1) : PB == 1 ? pc : 0;
        const int p1 = PB == 2 ? (pc >> 1) : PB == 1 ? pc : 0;
        const uint16_t *q0 = S.q + (cls * 2 + p0) * 256, *q1 = S.q + (cls * 2 + p1) * 256;
        int d0[3], d1[3];
#pragma unroll
        for (int c = 0; c < 3; c++) { d0[c] = q0[lo[c]] >> 8; d1[c] = q1[hi[c]] >> 8; }
        uint32_t prg[1 << NB];
        int pb[1 << NB];
#pragma unroll
        for (int k = 0; k < (1 << NB); k++) {
            const int w = bc7_weight(NB, k);
            int r = interp64(d0[0], d1[0], w), g = interp64(d0[1], d1[1], w), bb = interp64(d0[2], d1[2], w);
            prg[k] = ((uint32_t)r << 2) | ((uint32_t)g << 18);
            pb[k] = bb << 2;
        }
        uint32_t sse = 0;
        uint64_t idx = 0;
        for (uint32_t m = mask; m; m &= m - 1) {
            const int i = __ffs(m) - 1;
            uint32_t rg;
            int b;
            texel(S, i, rot, rg, b);
            uint32_t best = 0xFFFFFFFFu;
#pragma unroll
            for (int k = 0; k < (1 << NB); k++) {
                short2_t d = __builtin_bit_cast(short2_t, rg) - __builtin_bit_cast(short2_t, prg[k]);
                int db = b - pb[k];
                int key = __builtin_amdgcn_sdot2(d, d, __mul24(db, db) + k, false);
                best = min(best, (uint32_t)key);
            }
            sse += best >> 4;
            idx |= (uint64_t)(best & 15u) << (4 * i);
        }
        if (sse < best_sse) { best_sse = sse; best_idx = idx; }
    }
    idx_out = best_idx;
    return best_sse;
}

// (d) least-squares endpoints for the chosen indices; false if singular.
template <int NB>
__device__ __forceinline__ bool ls_endpoints(const SearchLds &S, uint32_t mask, int rot, uint64_t idx,
                                             int (&lo)[3], int (&hi)[3])
{
    int A = 0, B = 0, AB = 0, SA[3] = {0, 0, 0}, SB[3] = {0, 0, 0};
    for (uint32_t m = mask; m; m &= m - 1) {
        const int i = __ffs(m) - 1;
        uint32_t rg;
        int b;
        texel(S, i, rot, rg, b);
        int x[3];
        unpack(rg, b, x);
        const int k = (int)((idx >> (4 * i)) & 15);
        const int w = bc7_weight(NB, k), a = 64 - w;
        A += a * a; B += w * w; AB += a * w;
#pragma unroll
        for (int c = 0; c < 3; c++) { SA[c] += a * x[c]; SB[c] += w * x[c]; }
    }
    const double det = (double)A * (double)B - (double)AB * (double)AB;
    if (det == 0.0) return false;
#pragma unroll
    for (int c = 0; c < 3; c++) {
        // exact numerators (< 2^42); a correctly rounded quotient keeps the
        // floor(x + 1/2) decision of the exact rational for |x| <= 256
        double n0 = 64.0 * ((double)B * (double)SA[c] - (double)AB * (double)SB[c]);
        double n1 = 64.0 * ((double)A * (double)SB[c] - (double)AB * (double)SA[c]);
        double q0 = floor(n0 / det + 0.5), q1 = floor(n1 / det + 0.5);
        lo[c] = q0 < 0.0 ? 0 : (q0 > 255.0 ? 255 : (int)q0);
        hi[c] = q1 < 0.0 ? 0 : (q1 > 255.0 ? 255 : (int)q1);
    }
    return true;
}

// SSE of one colour subset fitted with precision (CB, PB) and NB-bit indices.
template <int CB, int PB, int NB>
__device__ __forceinline__ uint32_t fit_colour(const SearchLds &S, uint32_t mask, int rot, const Prep &P,
                                               const uint32_t *sv)
{
    constexpr int NPC = PB == 2 ? 4 : PB == 1 ? 2 : 1;
    constexpr int cls = cls_of(CB, PB);
    if (P.same) {
        uint32_t be = 0xFFFFFFFFu;
        for (int pc = 0; pc < NPC; pc++) {
            const int p0 = PB == 2 ? (pc & 1) : PB == 1 ? pc : 0;
            const int p1 = PB == 2 ? (pc >> 1) : PB == 1 ? pc : 0;
            for (int k = 0; k < (1 << NB); k++) {
                const uint32_t *row = sv + ((uint64_t)(cls * 4 + p0 + 2 * p1) * kSlots + slot_of(NB, k)) * 256;
                uint32_t e = 0;
#pragma unroll
                for (int c = 0; c < 3; c++) {
                    uint32_t er = row[P.lo[c]] >> 16;
                    e += er * er;
                }
                be = min(be, e);
            }
        }
        return be * (uint32_t)__popc(mask);
    }
    uint64_t idx;
    uint32_t sse = eval_pair<CB, PB, NB>(S, mask, rot, P.lo, P.hi, idx);
    int rlo[3], rhi[3];
    if (ls_endpoints<NB>(S, mask, rot, idx, rlo, rhi)) {
        uint64_t idx2;
        sse = min(sse, eval_pair<CB, PB, NB>(S, mask, rot, rlo, rhi, idx2));
    }
    return sse;
}

// SSE of the scalar channel (modes 4, 5, rotation r > 0): 16 values of
// channel r-1, precision AB bits (no p-bit), NB-bit indices.
template <int AB, int NB>
__device__ __forceinline__ uint32_t fit_scalar(const SearchLds &S, int rot, const uint32_t *sv)
{
    constexpr int cls = cls_of(AB, 0);
    auto value = [&](int i) {
        const uint32_t rg = S.rg[i][threadIdx.x];
        const int b = (int)S.b[i][threadIdx.x];
        return rot == 1 ? (int)((rg & 0xFFFFu) >> 2) : rot == 2 ? (int)(rg >> 18) : (b >> 2);
    };
    const int v0 = value(0);
    int lo = v0, hi = v0;
    bool same = true;
    for (int i = 1; i < 16; i++) {
        int v = value(i);
        same &= v == v0;
        lo = min(lo, v);
        hi = max(hi, v);
    }
    if (same) {
        uint32_t be = 0xFFFFFFFFu;
        for (int k = 0; k < (1 << NB); k++) {
            uint32_t er = sv[((uint64_t)(cls * 4) * kSlots + slot_of(NB, k)) * 256 + v0] >> 16;
            be = min(be, er * er);
        }
        return be * 16u;
    }
    uint32_t best = 0xFFFFFFFFu;
    int elo = lo, ehi = hi;
    for (int pass = 0; pass < 2; pass++) {
        const int d0 = S.q[cls * 2 * 256 + elo] >> 8, d1 = S.q[cls * 2 * 256 + ehi] >> 8;
        int pal[1 << NB];
#pragma unroll
        for (int k = 0; k < (1 << NB); k++) pal[k] = interp64(d0, d1, bc7_weight(NB, k)) << 2;
        uint32_t sse = 0;
        int A = 0, B = 0, AB2 = 0, SA = 0, SB = 0;
        for (int i = 0; i < 16; i++) {
            const int x = value(i);
            uint32_t kbest = 0xFFFFFFFFu;
#pragma unroll
            for (int k = 0; k < (1 << NB); k++) {
                int d = (x << 2) - pal[k];
                kbest = min(kbest, (uint32_t)(__mul24(d, d) + k));
            }
            sse += kbest >> 4;
            const int w = bc7_weight(NB, (int)(kbest & 15u)), a = 64 - w;
            A += a * a; B += w * w; AB2 += a * w; SA += a * x; SB += w * x;
        }
        best = min(best, sse);
        if (pass == 1) break;
        const double det = (double)A * (double)B - (double)AB2 * (double)AB2;
        if (det == 0.0) break;
        double n0 = 64.0 * ((double)B * (double)SA - (double)AB2 * (double)SB);
        double n1 = 64.0 * ((double)A * (double)SB - (double)AB2 * (double)SA);
        double q0 = floor(n0 / det + 0.5), q1 = floor(n1 / det + 0.5);
        elo = q0 < 0.0 ? 0 : (q0 > 255.0 ? 255 : (int)q0);
        ehi = q1 < 0.0 ? 0 : (q1 > 255.0 ? 255 : (int)q1);
    }
    return best;
}

__device__ __forceinline__ void consider(uint32_t sse, int ci, uint32_t &best)
{
    best = min(best, (sse << 9) | (uint32_t)ci);
}

// The candidates fall into three groups by partition shape; each group is
// its own kernel (smaller register footprint), and the block's key is the
// minimum over the groups.
template <int GROUP>
__device__ uint32_t search_group(const SearchLds &S, uint32_t mode_mask, const uint32_t *sv)
{
    uint32_t best = 0xFFFFFFFFu;
    if (GROUP == 0) {
        // 2-subset partitions: modes 1, 3, 7
        if (mode_mask & 0x8A)
            for (int p = 0; p < 64; p++) {
                const uint32_t m0 = mask2(p, 0), m1 = mask2(p, 1);
                const Prep P0 = prep_subset(S, m0, 0), P1 = prep_subset(S, m1, 0);
                if (mode_mask & 0x02)
                    consider(fit_colour<6, 1, 3>(S, m0, 0, P0, sv) + fit_colour<6, 1, 3>(S, m1, 0, P1, sv), 16 + p, best);
                if (mode_mask & 0x08)
                    consider(fit_colour<7, 2, 2>(S, m0, 0, P0, sv) + fit_colour<7, 2, 2>(S, m1, 0, P1, sv), 144 + p, best);
                if (mode_mask & 0x80)
                    consider(fit_colour<5, 2, 2>(S, m0, 0, P0, sv) + fit_colour<5, 2, 2>(S, m1, 0, P1, sv), 221 + p, best);
            }
    } else if (GROUP == 1) {
        // 3-subset partitions: mode 0 (partitions 0..15), mode 2
        if (mode_mask & 0x05)
            for (int p = 0; p < ((mode_mask & 0x04) ? 64 : 16); p++) {
                const uint32_t m0 = mask3(p, 0), m1 = mask3(p, 1), m2 = mask3(p, 2);
                const Prep P0 = prep_subset(S, m0, 0), P1 = prep_subset(S, m1, 0), P2 = prep_subset(S, m2, 0);
                if ((mode_mask & 0x01) && p < 16)
                    consider(fit_colour<4, 2, 3>(S, m0, 0, P0, sv) + fit_colour<4, 2, 3>(S, m1, 0, P1, sv) +
                                 fit_colour<4, 2, 3>(S, m2, 0, P2, sv), p, best);
                if (mode_mask & 0x04)
                    consider(fit_colour<5, 0, 2>(S, m0, 0, P0, sv) + fit_colour<5, 0, 2>(S, m1, 0, P1, sv) +
                                 fit_colour<5, 0, 2>(S, m2, 0, P2, sv), 80 + p, best);
            }
    } else {
        // one subset: mode 6, and modes 4 / 5 for every rotation
        if (mode_mask & 0x70)
            for (int r = 0; r < 4; r++) {
                if (r > 0 && !(mode_mask & 0x30)) break;
                const Prep P = prep_subset(S, 0xFFFFu, r);
                if (r == 0 && (mode_mask & 0x40)) consider(fit_colour<7, 2, 4>(S, 0xFFFFu, 0, P, sv), 220, best);
                if (mode_mask & 0x10) {
                    uint32_t s0 = fit_colour<5, 0, 2>(S, 0xFFFFu, r, P, sv);
                    uint32_t s1 = fit_colour<5, 0, 3>(S, 0xFFFFu, r, P, sv);
                    if (r) { s0 += fit_scalar<6, 3>(S, r, sv); s1 += fit_scalar<6, 2>(S, r, sv); }
                    consider(s0, 208 + 2 * r, best);
                    consider(s1, 209 + 2 * r, best);
                }
                if (mode_mask & 0x20) {
                    uint32_t s5 = fit_colour<7, 0, 2>(S, 0xFFFFu, r, P, sv);
                    if (r) s5 += fit_scalar<8, 2>(S, r, sv);
                    consider(s5, 216 + r, best);
                }
            }
    }
    return best;
}

// ---- pass 2: re-fit the winner and lay out its bits
struct Writer {
    uint64_t lo = 0, hi = 0;
    int pos = 0;
    __device__ void put(uint32_t v, int n)
    {
        uint64_t x = (uint64_t)v & ((1ull << n) - 1);
        if (pos >= 64) hi |= x << (pos - 64);
        else {
            lo |= x << pos;
            if (pos + n > 64) hi |= x >> (64 - pos);
        }
        pos += n;
    }
};

template <int M, int CB, int PB, int NB>
__device__ void emit_partitioned(const int (&x)[16][3], int p, const Tables &T, Writer &w)
{
    constexpr Bc7Mode md = bc7_mode(M);
    constexpr int NS = md.ns;
    Fit f[NS];
    uint32_t msk[NS];
    int anc[NS];
#pragma unroll
    for (int s = 0; s < NS; s++) {
        msk[s] = NS == 3 ? mask3(p, s) : mask2(p, s);
        anc[s] = bc7_anchor(NS, p, s);
        fit_subset<CB, PB, NB, 3>(x, msk[s], T, f[s]);
        anchor_fix<NB, 3>(f[s], msk[s], anc[s]);
    }
    w.put(1u << M, M + 1);
    w.put((uint32_t)p, md.partbits);
#pragma unroll
    for (int c = 0; c < 3; c++)
#pragma unroll
        for (int s = 0; s < NS; s++) { w.put(f[s].c0[c], CB); w.put(f[s].c1[c], CB); }
    if (md.ab)
#pragma unroll
        for (int s = 0; s < NS; s++) { w.put((1u << md.ab) - 1, md.ab); w.put((1u << md.ab) - 1, md.ab); }
    if (PB == 2)
#pragma unroll
        for (int s = 0; s < NS; s++) { w.put(f[s].p0, 1); w.put(f[s].p1, 1); }
    else if (PB == 1)
#pragma unroll
        for (int s = 0; s < NS; s++) w.put(f[s].p0, 1);
#pragma unroll
    for (int i = 0; i < 16; i++) {
        int s = 0;
#pragma unroll
        for (int q = 1; q < NS; q++) if ((msk[q] >> i) & 1) s = q;
        bool anchored = false;
#pragma unroll
        for (int q = 0; q < NS; q++) anchored |= anc[q] == i;
        uint64_t idx = f[0].idx;
#pragma unroll
        for (int q = 1; q < NS; q++) if (s == q) idx = f[q].idx;
        w.put((uint32_t)((idx >> (4 * i)) & 15), NB - (anchored ? 1 : 0));
    }
}

// Modes 4 and 5: one colour pair plus a scalar pair, rotation r.
template <int M, int CB, int AB, int CNB, int SNB>
__device__ void emit_rotated(const int (&x)[16][3], int r, int sel, const Tables &T, Writer &w)
{
    int t[16][3], sc[16][3];
    rotate(x, r, t, sc);
    Fit fc, fs;
    fit_subset<CB, 0, CNB, 3>(t, 0xFFFF, T, fc);
    anchor_fix<CNB, 3>(fc, 0xFFFF, 0);
    fit_subset<AB, 0, SNB, 1>(sc, 0xFFFF, T, fs);
    anchor_fix<SNB, 1>(fs, 0xFFFF, 0);
    w.put(1u << M, M + 1);
    w.put((uint32_t)r, 2);
    if (M == 4) w.put((uint32_t)sel, 1);
#pragma unroll
    for (int c = 0; c < 3; c++) { w.put(fc.c0[c], CB); w.put(fc.c1[c], CB); }
    w.put(fs.c0[0], AB);
    w.put(fs.c1[0], AB);
    // primary index set first, then the secondary set; index selection 1
    // stores the scalar indices in the primary set
    const Fit &first = (M == 4 && sel) ? fs : fc;
    const Fit &second = (M == 4 && sel) ? fc : fs;
    constexpr int NB1 = (M == 4) ? 2 : 2, NB2 = (M == 4) ? 3 : 2;
#pragma unroll
    for (int i = 0; i < 16; i++) w.put((uint32_t)((first.idx >> (4 * i)) & 15), NB1 - (i == 0));
#pragma unroll
    for (int i = 0; i < 16; i++) w.put((uint32_t)((second.idx >> (4 * i)) & 15), NB2 - (i == 0));
}

__device__ void emit(const int (&x)[16][3], int ci, const Tables &T, uint64_t &lo, uint64_t &hi)
{
    int m, p, r, s;
    candidate(ci, m, p, r, s);
    Writer w;
    switch (m) {
    case 0: emit_partitioned<0, 4, 2, 3>(x, p, T, w); break;
    case 1: emit_partitioned<1, 6, 1, 3>(x, p, T, w); break;
    case 2: emit_partitioned<2, 5, 0, 2>(x, p, T, w); break;
    case 3: emit_partitioned<3, 7, 2, 2>(x, p, T, w); break;
    case 4:
        if (s == 0) emit_rotated<4, 5, 6, 2, 3>(x, r, 0, T, w);
        else emit_rotated<4, 5, 6, 3, 2>(x, r, 1, T, w);
        break;
    case 5: emit_rotated<5, 7, 8, 2, 2>(x, r, 0, T, w); break;
    case 6: {
        Fit f;
        fit_subset<7, 2, 4, 3>(x, 0xFFFF, T, f);
        anchor_fix<4, 3>(f, 0xFFFF, 0);
        w.put(1u << 6, 7);
#pragma unroll
        for (int c = 0; c < 3; c++) { w.put(f.c0[c], 7); w.put(f.c1[c], 7); }
        w.put(127, 7); w.put(127, 7);
        w.put(f.p0, 1); w.put(f.p1, 1);
#pragma unroll
        for (int i = 0; i < 16; i++) w.put((uint32_t)((f.idx >> (4 * i)) & 15), 4 - (i == 0));
        break;
    }
    default: emit_partitioned<7, 5, 2, 2>(x, p, T, w); break;
    }
    lo = w.lo;
    hi = w.hi;
}

struct Bc7Launch {
    EncodeArgs a;
    Tables T;
};

__device__ __forceinline__ void load_block(const EncodeArgs &a, uint64_t g, uint32_t (&t)[16], uint32_t &band,
                                           uint64_t &b)
{
    band = a.band0 + (uint32_t)(g / a.nblk);
    b = g % a.nblk;
    const uint4 *src = reinterpret_cast<const uint4 *>(a.textures + ((uint64_t)band * a.nblk + b) * 64);
#pragma unroll
    for (int q = 0; q < 4; q++) {
        uint4 v = src[q];
        t[4 * q] = v.x; t[4 * q + 1] = v.y; t[4 * q + 2] = v.z; t[4 * q + 3] = v.w;
    }
}

// Pass 1: the best key of every block over one candidate group, min-combined
// into the first word of its output slot (group 0 writes it first).
template <int GROUP>
__global__ __launch_bounds__(kSearchWG) void k_bc7_search(Bc7Launch L)
{
    __shared__ SearchLds S;
    const EncodeArgs &a = L.a;
    for (int q = threadIdx.x; q < kQEntries / 2; q += kSearchWG)
        reinterpret_cast<uint32_t *>(S.q)[q] = reinterpret_cast<const uint32_t *>(L.T.nearest)[q];
    const uint64_t g = (uint64_t)blockIdx.x * kSearchWG + threadIdx.x;
    const uint64_t total = (uint64_t)a.nbands * a.nblk;
    uint32_t t[16] = {0};
    uint32_t band = 0;
    uint64_t b = 0;
    if (g < total) load_block(a, g, t, band, b);
#pragma unroll
    for (int i = 0; i < 16; i++) {
        S.rg[i][threadIdx.x] = ((t[i] & 255u) << 2) | (((t[i] >> 8) & 255u) << 18);
        S.b[i][threadIdx.x] = ((t[i] >> 16) & 255u) << 2;
    }
    __syncthreads();
    if (g >= total) return;
    uint32_t key = search_group<GROUP>(S, a.mode_mask, L.T.sv);
    uint32_t *slot = reinterpret_cast<uint32_t *>(a.out + a.out_offset[band] + b * 16);
    *slot = GROUP == 0 ? key : min(key, *slot);
}

// Pass 2: re-fit each block's winning candidate and write its bits.
__global__ __launch_bounds__(kBlock) void k_bc7_emit(Bc7Launch L)
{
    const EncodeArgs &a = L.a;
    const uint64_t g = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    const uint64_t total = (uint64_t)a.nbands * a.nblk;
    if (g >= total) return;
    uint32_t t[16], band;
    uint64_t b;
    load_block(a, g, t, band, b);
    int x[16][3];
#pragma unroll
    for (int i = 0; i < 16; i++) {
        x[i][0] = t[i] & 255;
        x[i][1] = (t[i] >> 8) & 255;
        x[i][2] = (t[i] >> 16) & 255;
    }
    uint8_t *slot = a.out + a.out_offset[band] + b * 16;
    const uint32_t key = *reinterpret_cast<const uint32_t *>(slot);
    uint64_t lo, hi;
    emit(x, (int)(key & 511u), L.T, lo, hi);
    *reinterpret_cast<ulonglong2 *>(slot) = make_ulonglong2(lo, hi);
    if (a.band_sse) atomicAdd(&a.band_sse[band], (unsigned long long)(key >> 9));
}

// ---- host-side table construction
struct HostTables {
    std::vector<uint16_t> nearest;  // [10][2][256]
    std::vector<uint32_t> sv;       // [10][4][kSlots][256]
};

void build_nearest(HostTables &H)
{
    H.nearest.assign(10 * 2 * 256, 0);
    for (int cb = 4; cb <= 8; cb++)
        for (int pb = 0; pb < 2; pb++)
            for (int p = 0; p < 2; p++) {
                if (!pb && p) continue;
                const int nc = 1 << cb;
                uint16_t *row = &H.nearest[(cls_of(cb, pb) * 2 + p) * 256];
                for (int t = 0; t < 256; t++) {
                    int bc = 0, bd = 1 << 30;
                    for (int c = 0; c < nc; c++) {
                        int d = ep_value(c, p, cb, pb) - t;
                        d = d < 0 ? -d : d;
                        if (d < bd) { bd = d; bc = c; }
                    }
                    row[t] = (uint16_t)(bc | (ep_value(bc, p, cb, pb) << 8));
                }
            }
}

// Best pair per target value v for one (class, p-bits, weight): first the
// best pair (by |c0-c1|, c0, c1) reaching each interpolated value u, then for
// each v the nearest reachable u (both sides of v compared by the same key).
void build_sv_entry(uint32_t *row, int cb, int pb, int p0, int p1, int wgt)
{
    const int nc = 1 << cb;
    int bestpair[256];
    for (int u = 0; u < 256; u++) bestpair[u] = -1;
    auto better = [&](int a0, int a1, int b0, int b1) {   // is (a0,a1) ahead of (b0,b1)?
        int da = a0 > a1 ? a0 - a1 : a1 - a0, db = b0 > b1 ? b0 - b1 : b1 - b0;
        if (da != db) return da < db;
        if (a0 != b0) return a0 < b0;
        return a1 < b1;
    };
    for (int a = 0; a < nc; a++)
        for (int b = 0; b < nc; b++) {
            int u = interp64(ep_value(a, p0, cb, pb), ep_value(b, p1, cb, pb), wgt);
            int cur = bestpair[u];
            if (cur < 0 || better(a, b, cur >> 8, cur & 255)) bestpair[u] = (a << 8) | b;
        }
    for (int v = 0; v < 256; v++) {
        for (int d = 0; d < 256; d++) {
            int pick = -1;
            for (int side = 0; side < 2; side++) {
                int u = side ? v + d : v - d;
                if (u < 0 || u > 255 || bestpair[u] < 0) continue;
                int pr = bestpair[u];
                if (pick < 0 || better(pr >> 8, pr & 255, pick >> 8, pick & 255)) pick = pr;
            }
            if (pick >= 0) {
                row[v] = (uint32_t)(pick >> 8) | ((uint32_t)(pick & 255) << 8) | ((uint32_t)d << 16);
                break;
            }
        }
    }
}

void build_sv(HostTables &H)
{
    H.sv.assign((size_t)10 * 4 * kSlots * 256, 0);
    struct Use { int cb, pb, nb; };
    const Use uses[] = {{4, 2, 3}, {6, 1, 3}, {5, 0, 2}, {7, 2, 2}, {5, 0, 3}, {6, 0, 3}, {6, 0, 2},
                        {7, 0, 2}, {8, 0, 2}, {7, 2, 4}, {5, 2, 2}};
    for (const Use &u : uses) {
        const int npc = u.pb == 2 ? 4 : u.pb == 1 ? 2 : 1;
        for (int pc = 0; pc < npc; pc++) {
            int p0 = u.pb == 2 ? (pc & 1) : u.pb == 1 ? pc : 0;
            int p1 = u.pb == 2 ? (pc >> 1) : u.pb == 1 ? pc : 0;
            for (int k = 0; k < (1 << u.nb); k++) {
                uint32_t *row = &H.sv[(((size_t)cls_of(u.cb, u.pb) * 4 + p0 + 2 * p1) * kSlots + slot_of(u.nb, k)) * 256];
                build_sv_entry(row, u.cb, u.pb, p0, p1, bc7_weight(u.nb, k));
            }
        }
    }
}

}  // namespace

// Device copies of the tables, one set per device, made on first use.
static void *g_tab[64];

hipError_t upload_bc7_tables(int device, hipStream_t st)
{
    if (device < 0 || device >= 64) return hipErrorInvalidDevice;
    if (g_tab[device]) return hipSuccess;
    static HostTables H;
    static bool built = false;
    if (!built) { build_nearest(H); build_sv(H); built = true; }
    size_t nb = H.nearest.size() * 2, sb = H.sv.size() * 4;
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, nb + sb);
    if (e != hipSuccess) return e;
    e = hipMemcpyAsync(p, H.nearest.data(), nb, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync((char *)p + nb, H.sv.data(), sb, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) { (void)hipFree(p); return e; }
    g_tab[device] = p;
    return hipSuccess;
}

hipError_t launch_bc7_encode(const EncodeArgs &a, hipStream_t st)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (!g_tab[dev]) return hipErrorNotInitialized;
    uint64_t total = (uint64_t)a.nbands * a.nblk;
    if (total == 0) return hipSuccess;
    Bc7Launch L;
    L.a = a;
    L.T.nearest = static_cast<const uint16_t *>(g_tab[dev]);
    L.T.sv = reinterpret_cast<const uint32_t *>(static_cast<const uint8_t *>(g_tab[dev]) + 10 * 2 * 256 * 2);
    const dim3 sgrid((uint32_t)((total + kSearchWG - 1) / kSearchWG));
    hipLaunchKernelGGL(k_bc7_search<0>, sgrid, dim3(kSearchWG), 0, st, L);
    hipLaunchKernelGGL(k_bc7_search<1>, sgrid, dim3(kSearchWG), 0, st, L);
    hipLaunchKernelGGL(k_bc7_search<2>, sgrid, dim3(kSearchWG), 0, st, L);
    hipLaunchKernelGGL(k_bc7_emit, dim3((uint32_t)((total + kBlock - 1) / kBlock)), dim3(kBlock), 0, st, L);
    return hipGetLastError();
}

}  // namespace gsbc
