/*
 * gsbc.h -- C ABI of the MI355X (gfx950) library that codes the spherical-
 * harmonic (SH) colour of 3D Gaussian Splatting primitives into BC1/BC7
 * texture blocks, and decodes and evaluates it.
 *
 * Method: A. Said, R. Rauwendaal, "Compression of 3D Gaussian Splatting Data
 * Using GPU-friendly Graphics Texture Coding".
 *   - primitives may be reordered freely; reordering by colour inside spatial
 *     groups makes BTC blocks cheaper to code (Sec. I; Sec. III-C);
 *   - the SH coefficients of one band of 16 primitives form one 4x4 texel
 *     block (Sec. IV-B, Fig. SetupD), coded with a fixed number of bits per
 *     block (Sec. III-A/B), one bitstream per band, and the number of bits
 *     per primitive is varied by choosing a format per bitstream (Sec. IV-B);
 *   - a block is found by multiplying its index by the block size, which
 *     gives random access for parallel decoding (Sec. I);
 *   - the view-dependent colour is c(d) = H w(d) (Sec. II).
 *
 * Conventions shared by every call
 *   - Pointers named "device" are HIP device memory owned by the caller; the
 *     library never frees them.  Pointers named "host" are host memory owned
 *     by the caller.  Every size is an element count unless it says bytes.
 *   - Calls enqueue work on the context's stream.  gsbc_reorder and
 *     gsbc_encode also copy a few header values back and wait for the stream
 *     before they return; the other calls return without waiting (except
 *     gsbc_encode_batch when asked for band SSEs).  Device
 *     faults surface as GSBC_E_DEVICE from the next call or from gsbc_sync.
 *   - Every call returns a gsbc_status; on error the context keeps a message
 *     (gsbc_last_error).  Argument errors are detected before any work is
 *     enqueued and leave the outputs untouched.
 *   - Outputs are in sorted-slot order: slot s holds primitive perm[s].
 *   - One context per host thread.  Contexts share only read-only tables.
 *   - Results do not depend on launch shapes: every encoder decision is
 *     integer (or a fixed FP32 expression), ties break by a fixed order.
 */
#ifndef GSBC_H
#define GSBC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GSBC_API __attribute__((visibility("default")))

typedef int32_t gsbc_status;

enum {
    GSBC_OK = 0,
    GSBC_E_ARG = -1,         /* invalid argument (null pointer, bad size, bad enum) */
    GSBC_E_UNSUPPORTED = -2, /* valid request the library does not implement */
    GSBC_E_NOMEM = -3,       /* scratch allocation failed */
    GSBC_E_INFEASIBLE = -4,  /* the rate target cannot be met exactly */
    GSBC_E_DEVICE = -5,      /* a HIP call or kernel failed */
    GSBC_E_BUFFER = -6,      /* a caller buffer is too small (see gsbc_query_sizes) */
    GSBC_E_IO = -7           /* a container file cannot be read or written, or is malformed */
};

/* Stream formats: BC1 (8 bytes per block), BC7 (16), or NONE: a band
 * stream given 0 bits (Sec. IV-B, bitstreams for a varying number of
 * nonzero SH vectors), which stores no blocks and whose coefficients decode
 * to exactly zero (band arrangement only).  AUTO and AUTO_ZERO ask
 * gsbc_encode to choose per band at a rate; BANDS takes desc->format. */
enum {
    GSBC_FMT_AUTO = 0,
    GSBC_FMT_BC1 = 1,
    GSBC_FMT_BANDS = 2,
    GSBC_FMT_NONE = 3,
    GSBC_FMT_AUTO_ZERO = 4,
    GSBC_FMT_BC7 = 7
};

/* Arrangements of the 16 band vectors of the primitives into 4x4 blocks
 * (Sec. IV-B).  Slots are padded to n_pad (a multiple of 16) by repeating
 * slot n-1; an arrangement with S streams has n_pad/S blocks per stream.
 *   GSBC_ARR_BANDS (Fig. SetupD, default): S = 16; stream k holds band k,
 *       block s/16, slot s%16 at the zigzag texel 4y+x, x = j0|j2<<1,
 *       y = j1|j3<<1 (j = s%16).
 *   GSBC_ARR_PRIM (Fig. SetupA): S = 1; block s holds slot s, band k at
 *       texel k.
 *   GSBC_ARR_QUAD (Fig. SetupB): S = 4; stream g holds bands 4g..4g+3,
 *       block s/4, texel 4*(s%4) + k%4 (slot on the row, band on the
 *       column).  With S = 1 it is Fig. SetupC: bands 0..3 of four
 *       primitives in one block (the degree-1 class of
 *       gsbc_reorder_degrees), bands 4..15 dropped. */
enum { GSBC_ARR_BANDS = 0, GSBC_ARR_PRIM = 1, GSBC_ARR_QUAD = 2 };

typedef struct gsbc_ctx gsbc_ctx;

typedef struct {
    uint32_t grid_bits;      /* spatial chunk grid: 2^g cells per axis, 0..10 (default 3) */
    uint32_t refine_steps;   /* BC1 endpoint refinement steps, 0..8 (default 2) */
    uint32_t bc7_mode_mask;  /* BC7 modes searched, bit m = mode m, nonzero (default 0xFF) */
    uint32_t order;          /* gsbc_reorder: 0 = sort by (spatial cell, colour) (default);
                                1 = keep the input order (perm[s] = s), the unsorted
                                baseline the paper compares sorting against (Sec. III-C) */
    uint32_t arrangement;    /* gsbc_reorder: GSBC_ARR_BANDS (default), GSBC_ARR_PRIM or GSBC_ARR_QUAD */
    uint32_t quantiser;      /* gsbc_reorder: per-band range of the 8-bit quantiser (Sec. V-A):
                                0 = [min, max] of the band's coefficients (default);
                                1 = [-t, t] with t the ceil(0.995 * 3n)-th smallest |x| of
                                    the band, so that 99.5 % of its coefficients lie inside
                                    and the rest clamp (vmin = +0 when t = 0) */
} gsbc_params;

/* Header of a coded scene: one bitstream per stream of the arrangement
 * (Sec. IV-A: typed bitstreams; the stream index selects the decoder). */
typedef struct {
    uint8_t format[16];          /* per stream: GSBC_FMT_BC1, GSBC_FMT_BC7 or (band arrangement)
                                    GSBC_FMT_NONE (entries past n_streams unused) */
    uint64_t offset[16];         /* byte offset of stream s in the payload (16-byte aligned) */
    float vmin[16], vmax[16];    /* per-band quantiser range: q = rint((x - vmin) * 255/(vmax - vmin)) */
    uint64_t n_prims;            /* N */
    uint64_t n_pad;              /* N rounded up to a multiple of 16 */
    uint64_t blocks_per_stream;  /* n_pad / 16 (BANDS), n_pad (PRIM), n_pad / 4 (QUAD, either S) */
    uint64_t payload_bytes;      /* bytes of the concatenated streams */
    uint32_t arrangement;        /* GSBC_ARR_* of the textures */
    uint32_t n_streams;          /* 16, 1 or 4 (BANDS, PRIM, QUAD); 1, 4 or 9 (BANDS) or 1
                                    (QUAD) for a degree class of gsbc_reorder_degrees: the bands
                                    past the streams' (n_streams, or 4 n_streams) are zero */
} gsbc_stream_desc;

/* ---------------------------------------------------------------- context */

/* Create a context on HIP device `device`.  `hip_stream` is a hipStream_t to
 * enqueue on, or NULL for a stream the context creates (default priority,
 * blocking: ordered with work on the legacy null stream).  The context owns
 * its scratch arena and, if it made it, its stream. */
GSBC_API gsbc_status gsbc_create(gsbc_ctx **out, int device, void *hip_stream);

/* Wait for the stream, free the scratch arena, destroy the context. */
GSBC_API gsbc_status gsbc_destroy(gsbc_ctx *ctx);

/* Message of the last error on this context ("" if none).  The string is
 * owned by the context and valid until its next call. */
GSBC_API const char *gsbc_last_error(const gsbc_ctx *ctx);

/* Wait for all work enqueued by this context. */
GSBC_API gsbc_status gsbc_sync(gsbc_ctx *ctx);

/* Size the context's scratch arena once for scenes of up to n_max primitives
 * and decode_evals of up to n_dirs_max directions, so that calls within those
 * sizes allocate nothing (a serving slot reserves its largest admissible
 * request up front instead of growing mid-stream).  Outgrown arenas are kept
 * until gsbc_destroy, since queued kernels may still read them and freeing
 * device memory waits for the whole device.
 * GSBC_E_ARG for n_max outside 1..2^31-1, GSBC_E_NOMEM if it cannot grow. */
GSBC_API gsbc_status gsbc_reserve(gsbc_ctx *ctx, uint64_t n_max, uint32_t n_dirs_max);

/* The arena's current size in bytes and how many times it has grown (either
 * output may be NULL). */
GSBC_API gsbc_status gsbc_arena_info(const gsbc_ctx *ctx, uint64_t *bytes, uint64_t *growths);

/* Fill `p` (host) with the defaults: grid_bits 3, refine_steps 2, mode mask 0xFF, order 0,
 * arrangement GSBC_ARR_BANDS, quantiser 0. */
GSBC_API void gsbc_default_params(gsbc_params *p);

/* Sizes in bytes for N primitives and V directions (any output may be NULL):
 * textures: n_pad * 64 bytes (uint8[S][n_pad/S][16][4] in every arrangement);
 * max_blocks: the payload when every stream is BC7 (an upper bound for any
 * format choice and arrangement);  out: float[V][N][3]. */
GSBC_API gsbc_status gsbc_query_sizes(uint64_t n, uint32_t n_dirs, uint64_t *textures_bytes,
                             uint64_t *max_blocks_bytes, uint64_t *out_bytes);

/* ---------------------------------------------------------------- calls */

/* Reorder and pack (Sec. III-C and Sec. IV-B, Fig. SetupD; preprocessing
 * and 8-bit quantiser of Sec. V-A).
 *   pos     device float[n][3]      primitive centres
 *   sh      device float[n][16][3]  SH colour coefficients (band-major per primitive)
 *   opacity device float[n] or NULL: when given, every coefficient of
 *           primitive i is first multiplied by opacity[i] in FP32 (the
 *           opacity-premultiplied colours of Sec. V-A); the range, keys and
 *           textures all use the products
 *   n       1 .. 2^31-1 primitives (quantiser 1: 3n < 2^32)
 *   params  host, NULL for defaults (grid_bits, order, arrangement and
 *           quantiser are used)
 *   perm    device uint32[n]        out: perm[s] = original index at slot s
 *   textures device uint8[S][n_pad/S][16][4] out: the 8-bit RGB (alpha 255)
 *           of every (slot, band) at the stream, block and texel the
 *           arrangement assigns (GSBC_ARR_*; n_pad * 64 bytes in every
 *           arrangement); slots past n repeat slot n-1
 *   desc    host, out: vmin, vmax, n_prims, n_pad, blocks_per_stream,
 *           arrangement, n_streams filled; the call waits for the stream to
 *           read the ranges back.  NULL: the call only enqueues the work and
 *           returns (perm and textures are ready when the stream gets
 *           there); gsbc_reorder_desc fills the desc later.
 * Keys: (Morton cell of the position on a 2^g grid over the bounding box) << 24
 * | interleaved bits of the band-0 quantised R,G,B (R highest in each triple);
 * stable ascending sort.  Inputs must be finite. */
GSBC_API gsbc_status gsbc_reorder(gsbc_ctx *ctx, const float *pos, const float *sh, const float *opacity,
                         uint64_t n, const gsbc_params *params, uint32_t *perm, uint8_t *textures,
                         gsbc_stream_desc *desc);

/* The desc of the last gsbc_reorder on this context (as that call fills it
 * when given a desc): waits for the stream, then reads the ranges back.
 * For callers that enqueue the reorder without waiting (desc NULL) and need
 * the ranges later, e.g. after queueing other work.
 *   desc  host, out
 * GSBC_E_ARG when no gsbc_reorder has run on the context since it was made
 * or since a gsbc_reorder_degrees (which reuses the range record). */
GSBC_API gsbc_status gsbc_reorder_desc(gsbc_ctx *ctx, gsbc_stream_desc *desc);

/* Variable number of bands (Sec. IV-B: primitives whose higher-order SH are
 * zero, or small enough to count as zero, go to bitstreams with fewer
 * bands; Fig. SetupD in its variable form, and Fig. SetupC for degree 1).
 * Each primitive's degree class
 * L is the largest SH degree l in 1..3 with a coefficient of a degree-l band
 * (bands l^2..l^2+2l) above tau in magnitude, else 0; the primitive keeps
 * its (L+1)^2 lowest bands and the others decode as exactly zero.  The sort
 * key is (L, Morton cell, colour), so class L is a contiguous range of perm
 * in increasing L, each ordered as gsbc_reorder orders a scene.  Every
 * class is an independent scene with its (L+1)^2 bands in (L+1)^2 band
 * streams (or, for degree 1, the one stream of Fig. SetupC), to be coded with gsbc_encode or gsbc_encode_batch (per-band or
 * whole formats; the rate controller needs all 16 bands) and decoded with
 * class-local slot ids.  The quantiser range covers all coefficients,
 * dropped ones included.
 *   pos, sh, opacity, n   as gsbc_reorder
 *   tau        >= 0, FP32 magnitudes at or below it count as zero (after
 *              opacity premultiplication)
 *   params     host, NULL for defaults (grid_bits and quantiser are used;
 *              order must be 0); arrangement GSBC_ARR_BANDS puts every
 *              class in per-band streams (Fig. SetupD), GSBC_ARR_QUAD the
 *              degree-1 class in one stream of blocks holding bands 0..3 of
 *              four primitives each (Fig. SetupC: texel 4 (j%4) + k of
 *              block j/4 for class slot j) and the others per band
 *   perm       device uint32[n] out: slot -> primitive; class L owns slots
 *              counts[0] + .. + counts[L-1] .. + counts[L] - 1
 *   textures   device, textures_capacity bytes, at least n_pad*64 + 1800
 *              (GSBC_E_BUFFER otherwise); out: class L's textures
 *              uint8[(L+1)^2][pad16(counts[L])/16][16][4] (the layout of
 *              gsbc_reorder), or for Fig. SetupC
 *              uint8[1][pad16(counts[1])/4][16][4], at byte offset
 *              tex_offset[L]
 *   counts     host uint64[4] out: primitives per class
 *   tex_offset host uint64[4] out
 *   descs      host gsbc_stream_desc[4] out: class L's scene (n_prims =
 *              counts[L], arrangement and n_streams: GSBC_ARR_BANDS with
 *              (L+1)^2, or GSBC_ARR_QUAD with 1 for Fig. SetupC; ranges);
 *              an empty class has n_prims 0 and is not a scene to code */
GSBC_API gsbc_status gsbc_reorder_degrees(gsbc_ctx *ctx, const float *pos, const float *sh, const float *opacity,
                                          uint64_t n, float tau, const gsbc_params *params, uint32_t *perm,
                                          uint8_t *textures, uint64_t textures_capacity, uint64_t counts[4],
                                          uint64_t tex_offset[4], gsbc_stream_desc descs[4]);

/* Encode every stream (Sec. III-A BTC; Sec. IV-B per-bitstream formats).
 *   textures device, layout of gsbc_reorder; desc host, in: n_prims, n_pad,
 *            blocks_per_stream, arrangement, n_streams, vmin, vmax; out:
 *            format, offset, payload_bytes
 *   format   GSBC_FMT_BC1 or GSBC_FMT_BC7 for all streams; GSBC_FMT_BANDS
 *            for the per-stream formats the caller put in desc->format[s]
 *            (each BC1, BC7 or, for band streams, NONE: e.g. band 0 BC7 and
 *            the rest BC1 as in Sec. V, or the first SetupB stream BC7 and
 *            the other three BC1 as in Table I); or a rate-controlled choice
 *            over the S = n_streams bands of a GSBC_ARR_BANDS scene (16, or
 *            (L+1)^2 for a degree class; other arrangements
 *            GSBC_E_UNSUPPORTED), at exactly `rate` bits per texel over the
 *            S bands: every band is coded in both formats, band 0 is BC7,
 *            and with U = rate*S/4 four-bit units in all (an integer to
 *            within 1e-9, else GSBC_E_INFEASIBLE):
 *            GSBC_FMT_AUTO  of bands 1..S-1 the k = U - S - 1 (0..S-1) with
 *                the largest (SSE_BC1 - SSE_BC7) * delta_k^2 are BC7 (lower
 *                band first on ties), the rest BC1; S = 16 gives
 *                k = 4*rate - 17;
 *            GSBC_FMT_AUTO_ZERO  each band 1..S-1 is BC7, BC1 or NONE, with
 *                U - 2 units (0..2(S-1)) over them (2, 1, 0 each), choosing
 *                the least total distortion: SSE_BC7 delta_k^2,
 *                SSE_BC1 delta_k^2, or for NONE the sum of the band's
 *                squared dequantised texel values (vmin_k + q delta_k)^2
 *                over its R, G, B codes q, summed in code order from a
 *                histogram; the bands' distortions are added from band S-1
 *                down to band 1; on ties the lower band takes BC7 before
 *                BC1 before NONE;
 *            delta_k = (vmax_k - vmin_k)/255 in FP32; `rate` is ignored
 *            otherwise
 *   params   host, NULL for defaults (refine_steps, bc7_mode_mask are used)
 *   blocks   device uint8[blocks_capacity] out: stream s's blocks at
 *            offset[s], 8 bytes (BC1) or 16 bytes (BC7) each; GSBC_E_BUFFER
 *            if blocks_capacity < payload size
 *   band_sse host int64[2][16] or NULL, out: total RGB SSE of each stream
 *            coded in BC1 (row 0) and BC7 (row 1) over all its blocks, -1
 *            where that format was not coded or the stream does not exist */
GSBC_API gsbc_status gsbc_encode(gsbc_ctx *ctx, const uint8_t *textures, gsbc_stream_desc *desc,
                        int format, double rate, const gsbc_params *params, uint8_t *blocks,
                        uint64_t blocks_capacity, int64_t *band_sse);

/* Work distribution of gsbc_encode_batch.  Every setting gives the same
 * bits: each block is coded on its own and every decision is a fixed
 * integer computation (results do not depend on launch shapes).
 *   item_rounds  256-block rounds per work item, 1..64
 *   wgs_per_cu   0: one workgroup per item (a plain grid); 1..16: that many
 *                persistent workgroups per compute unit pop items from a
 *                device counter until none are left
 *   bc1_lanes    BC1 workgroup size: 64, 128 or 256
 *   bc7_split    BC7 candidate groups per search kernel: 0 = three kernels
 *                (2-subset, 3-subset, 1-subset modes), 1 = two (the 3- and
 *                1-subset modes together), 2 = one kernel running all
 *                groups per block, 3 = one kernel whose work items are
 *                (group, rounds) pairs, heavy groups first
 *   concurrent   1: the BC1 blocks run on a second stream beside the BC7
 *                blocks; 0: after them on the context's stream */
typedef struct {
    uint32_t item_rounds;
    uint32_t wgs_per_cu;
    uint32_t bc1_lanes;
    uint32_t bc7_split;
    uint32_t concurrent;
} gsbc_batch_tuning;

/* Defaults: item_rounds 1, wgs_per_cu 0, bc1_lanes 128, bc7_split 3,
 * concurrent 0 (the launch shapes of gsbc_encode). */
GSBC_API void gsbc_default_batch_tuning(gsbc_batch_tuning *t);

/* Encode many scenes in one launch sequence.  Blocks are independent and
 * fixed-size (Sec. I; Sec. III-A), so the blocks of every band of every
 * scene in one format form a single index space that one kernel per step
 * covers, however uneven the scenes.  Scene i is coded exactly as
 * gsbc_encode(ctx, textures[i], &descs[i], GSBC_FMT_BANDS, ...) would code
 * it, bit for bit.  The launch sequence is captured once into a HIP graph
 * (on the context's stream, which must not be the legacy null stream) and
 * replayed while later calls pass the same scene count, pointers, block
 * counts, formats, params and tuning; otherwise the plan is rebuilt, which
 * allocates device memory the context holds until the next rebuild or
 * gsbc_destroy.
 *   n_scenes         1..4096
 *   textures         host array of n_scenes device pointers (gsbc_reorder layout)
 *   descs            host array of n_scenes; in: n_prims, n_pad,
 *                    blocks_per_stream, arrangement, n_streams, vmin, vmax
 *                    and format[s] (each BC1 or BC7) of every stream; out:
 *                    offset, payload_bytes
 *   blocks           host array of n_scenes device pointers, 16-byte aligned
 *   blocks_capacity  host uint64[n_scenes]: bytes behind each blocks[i]
 *                    (GSBC_E_BUFFER if below the scene's payload)
 *   params, tuning   host, or NULL for the defaults
 *   band_sse         host int64[n_scenes][16] or NULL, out: each stream's
 *                    SSE in its format (0 past n_streams); when given the call waits for the
 *                    stream, otherwise it returns once the graph is queued */
GSBC_API gsbc_status gsbc_encode_batch(gsbc_ctx *ctx, uint32_t n_scenes, const uint8_t *const *textures,
                                       gsbc_stream_desc *descs, uint8_t *const *blocks,
                                       const uint64_t *blocks_capacity, const gsbc_params *params,
                                       const gsbc_batch_tuning *tuning, int64_t *band_sse);

/* Decode every stream back to textures (layout of gsbc_reorder) -- BC1 and BC7
 * decoders of the format definitions; BC1 interpolants rounded to nearest.
 *   blocks device, desc host (filled by gsbc_encode), textures_out device. */
GSBC_API gsbc_status gsbc_decode(gsbc_ctx *ctx, const uint8_t *blocks, const gsbc_stream_desc *desc,
                        uint8_t *textures_out);

/* Random-access decode + SH evaluation (Sec. II colour equation; Sec. I
 * random access).  For every direction v and listed slot j:
 *   out[v][j][c] = sum_k Hhat_k[c] * Y_k(dir_v),
 *   Hhat_k = vmin_k + qhat * (vmax_k - vmin_k)/255 with qhat the decoded
 *   texel of (slot, band k), found through the arrangement,
 *   Y_k the real SH basis of degree <= 3 (k = l^2 + l + m, 3DGS signs), FP32.
 *   blocks   device payload; desc host (filled by gsbc_encode)
 *   dirs     device float[n_dirs][3], used as given (no normalisation)
 *   prim_idx device uint32[m] sorted-slot ids (< n_prims), or NULL for all
 *            slots 0..n_prims-1 (then m must equal n_prims)
 *   out      device float[n_dirs][m][3] */
GSBC_API gsbc_status gsbc_decode_eval(gsbc_ctx *ctx, const uint8_t *blocks, const gsbc_stream_desc *desc,
                             const float *dirs, uint32_t n_dirs, const uint32_t *prim_idx,
                             uint64_t m, float *out);

/* gsbc_decode_eval for callers that cannot allocate (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * arguments, checks, kernels and results, but the per-call scratch (16 basis
 * floats per direction) is a file-scope device array of the library instead
 * of the context's arena, so the call allocates nothing (no device, host or
 * event allocation; kernel timing is not recorded for it).
 *   n_dirs   at most 1024 (GSBC_E_ARG above: the array's fixed size)
 * Every call on one GPU shares that GPU's array (the library keeps it until
 * the process ends; gsbc_create looks its address up): calls that overlap on
 * one GPU, e.g. from two contexts on different streams, race on it and must
 * be serialised by the caller.  Each call writes the rows it reads before
 * reading them, so nothing needs clearing between calls. */
GSBC_API gsbc_status gsbc_decode_eval_noalloc(gsbc_ctx *ctx, const uint8_t *blocks, const gsbc_stream_desc *desc,
                                     const float *dirs, uint32_t n_dirs, const uint32_t *prim_idx,
                                     uint64_t m, float *out);

/* Colour of each listed slot seen from one view position f: the colour
 * equation c(f) = H w(f - p) of Sec. II evaluated per primitive at the unit
 * direction d = (f - p)/|f - p| towards the view position (d = 0 when f = p),
 * the per-primitive colour a rasteriser's blending stage consumes (Sec. II,
 * eq. preblend).  FP32: d from the FP32 inputs, then as gsbc_decode_eval.
 *   blocks, desc   as gsbc_decode_eval
 *   pos       device float[n_prims][3], primitive positions in input order
 *   perm      device uint32[n_prims] from gsbc_reorder (slot -> primitive)
 *   view      host float[3], the view position f
 *   prim_idx  device uint32[m] sorted-slot ids, or NULL for all slots (then
 *             m must equal n_prims); ids >= n_prims give NaN colours
 *   out       device float[m][3] */
GSBC_API gsbc_status gsbc_decode_eval_view(gsbc_ctx *ctx, const uint8_t *blocks, const gsbc_stream_desc *desc,
                                           const float *pos, const uint32_t *perm, const float *view,
                                           const uint32_t *prim_idx, uint64_t m, float *out);

/* Colour stage of a tile rasteriser (Sec. II: eq. blend written as
 * eq. preblend with the premultiplied coefficients Htilde = mu H of
 * eq. premult, which is what the bitstreams hold when gsbc_reorder was given
 * the opacities).  The image has tiles_x by tiles_y tiles of 16 by 16
 * pixels; tile t = ty * tiles_x + tx.  For each pixel, with centre
 * (16 tx + px + 1/2, 16 ty + py + 1/2), the entries i of its tile's list
 * front to back add
 *     a += g_i ctilde_i T,   then T *= 1 - mu_i g_i,   T starting at 1,
 * with ctilde_i = Htilde_i w(f - p_i) the primitive's colour decoded from the
 * bitstreams and evaluated towards the view position (as
 * gsbc_decode_eval_view, never written to memory) and
 * g_i = exp(-(a dx^2 + 2 b dx dy + c dy^2)/2) its footprint at the pixel.
 * FP32 throughout; no early termination.
 *   blocks, desc     as gsbc_decode_eval (a coded scene)
 *   pos, perm        as gsbc_decode_eval_view
 *   view             host float[3], the view position f
 *   opacity          device float[n_prims], mu per primitive (input order)
 *   footprint        device float[n_prims][5]: projected mean x, mean y (pixels)
 *                    and conic a, b, c (the inverse 2D covariance) per primitive
 *   tile_start       device uint32[tiles_x * tiles_y + 1]: tile t's entries are
 *                    list[tile_start[t] .. tile_start[t+1]) (clamped to list_len)
 *   list, list_len   device uint32[list_len]: sorted-slot ids, each tile's front
 *                    to back; ids >= n_prims give NaN
 *   image            device float[16 tiles_y][16 tiles_x][3] out
 *   transmittance    device float[16 tiles_y][16 tiles_x] out (final T), or NULL
 * GSBC_E_ARG for NULL pointers, misaligned arrays, an empty image or more
 * than 2^31 tiles, or a non-finite view position. */
GSBC_API gsbc_status gsbc_blend_tiles(gsbc_ctx *ctx, const uint8_t *blocks, const gsbc_stream_desc *desc,
                                      const float *pos, const uint32_t *perm, const float *view, const float *opacity,
                                      const float *footprint, const uint32_t *tile_start, const uint32_t *list,
                                      uint64_t list_len, uint32_t tiles_x, uint32_t tiles_y, float *image,
                                      float *transmittance);

/* The same colour stage with each primitive's colour computed beforehand,
 * once per primitive, instead of decoded from the bitstreams for every list
 * entry (a primitive sits in several tiles' lists): the two-pass form of
 * Sec. II eq. preblend.  With colours from gsbc_decode_eval_view over all
 * slots (prim_idx NULL) for the same blocks, desc, pos, perm and view, the
 * image and transmittance equal gsbc_blend_tiles' bit for bit.
 *   colours          device float[n_prims][3], slot s's colour ctilde
 *   n_prims          1 .. 2^31-1, the slots of the scene (list ids >= n_prims
 *                    give NaN)
 *   perm, opacity, footprint, tile_start, list, list_len, tiles_x, tiles_y,
 *   image, transmittance   as gsbc_blend_tiles
 * GSBC_E_ARG for NULL pointers, misaligned arrays, n_prims out of range, an
 * empty image or more than 2^31 tiles. */
GSBC_API gsbc_status gsbc_blend_tiles_colours(gsbc_ctx *ctx, const float *colours, uint64_t n_prims,
                                              const uint32_t *perm, const float *opacity, const float *footprint,
                                              const uint32_t *tile_start, const uint32_t *list, uint64_t list_len,
                                              uint32_t tiles_x, uint32_t tiles_y, float *image, float *transmittance);

/* ---------------------------------------------------------------- container */

/* The durable form of a coded scene: fixed-size blocks in one bitstream per
 * stream, found by index times block size (Sec. I; Sec. IV-A typed streams).
 * Little-endian file layout:
 *   bytes 0..63     header: "GSBC" magic, u32 version (2), u64 n_prims,
 *                   u64 n_pad, u64 blocks_per_stream, u64 payload_bytes,
 *                   u32 record bytes (24), u32 arrangement, u32 n_streams,
 *                   zero padding to 64 (version 1 files, written before
 *                   arrangements existed, hold GSBC_ARR_BANDS)
 *   16 x 24 bytes   records k = 0..15: u32 format of stream k (0 past
 *                   n_streams), u32 0, u64 offset of stream k, f32 vmin of
 *                   band k, f32 vmax of band k
 *   payload         payload_bytes bytes, stream s at offset[s]
 * gsbc_save copies the payload from the device (waits for the stream) and
 * writes the file.  gsbc_load reads and checks it (GSBC_E_IO if the magic,
 * version, record size, sizes or stream layout are wrong, or the file is
 * short), fills *desc, and when `blocks` (device) is non-NULL copies the
 * payload there (GSBC_E_BUFFER if blocks_capacity < payload_bytes; waits
 * for the stream).  With blocks == NULL, ctx may be NULL: only the header
 * is read. */
GSBC_API gsbc_status gsbc_save(gsbc_ctx *ctx, const uint8_t *blocks, const gsbc_stream_desc *desc,
                               const char *path);
GSBC_API gsbc_status gsbc_load(gsbc_ctx *ctx, const char *path, gsbc_stream_desc *desc, uint8_t *blocks,
                               uint64_t blocks_capacity);

/* ---------------------------------------------------------------- tracing */

/* Kernel timing, a tracing aid.  While enabled, every kernel this context
 * launches is bracketed by HIP events on the context's stream (so the times
 * are device times of that stream), and gsbc_encode runs its kernels one
 * after another there (without timing, its BC1 kernel overlaps the BC7
 * bucketing and emit kernels on a second stream).  gsbc_profile_read waits for the stream,
 * then returns per kernel name (at most max_entries of them, in first-launch
 * order) the number of launches and their total milliseconds since the
 * previous read, and forgets them.
 *   names   host char[max_entries][64] out (NUL-terminated kernel names)
 *   counts  host uint32[max_entries] out;  ms  host double[max_entries] out
 *   n_out   host out: number of entries written */
GSBC_API gsbc_status gsbc_profile_enable(gsbc_ctx *ctx, int on);
GSBC_API gsbc_status gsbc_profile_read(gsbc_ctx *ctx, uint32_t max_entries, char *names, uint32_t *counts,
                                       double *ms, uint32_t *n_out);

#ifdef __cplusplus
}
#endif

#endif /* GSBC_H */
