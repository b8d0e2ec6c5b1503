/*
 * ctf.h -- C ABI of the MI355X (gfx950) collaborative texture filtering library.
 *
 * Paper: Akenine-Moller, Ebelin, Pharr, Wronski, "Collaborative Texture
 * Filtering", HPG 2025 (arXiv 2506.17770).
 *
 * The hot path (Section 3): every pixel of a wave computes its bilinear
 * footprint; the wave collects the texels it needs (List Merge, Box Sampling
 * or Mask Sampling, Sections 3.1-3.3); each needed texel is produced once and
 * shared; each pixel weights the four texels it needs.  Pixels that minify,
 * and pixels of a wave whose needs exceed its budget, fall back to one-tap
 * stochastic texture filtering (Section 3.4, first paragraph).
 *
 * Conventions shared by every call:
 *  - A wave is 64 lanes and covers one 8x8 pixel tile; lane = 8*ly + lx.
 *    Tiles are numbered row-major over the screen; screens whose size is not
 *    a multiple of 8 get padding lanes that are inactive.
 *  - Pointers named "device" are GPU memory owned by the caller; pointers
 *    named "host" are CPU memory owned by the caller and only read or written
 *    during the call.  The library never keeps a caller pointer.
 *  - Calls taking a `stream` (a hipStream_t, NULL = the null stream) only
 *    enqueue work: outputs are valid once that stream has been synchronised.
 *    No call allocates device memory per invocation, except where stated.
 *  - Every call returns a ctf_status; on failure ctf_last_error() gives a
 *    message (thread-local, valid until the next call on the thread).  No
 *    call aborts or throws.  A device fault of an earlier asynchronous call
 *    is reported by the next call that checks the device (CTF_ERR_DEVICE).
 */
#ifndef CTF_H
#define CTF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CTF_ABI_VERSION 1

typedef enum ctf_status {
    CTF_OK = 0,
    CTF_ERR_INVALID_ARG = 1,
    CTF_ERR_UNSUPPORTED = 2,
    CTF_ERR_DEVICE = 3,
    CTF_ERR_OUT_OF_MEMORY = 4
} ctf_status;

typedef struct ctf_context_s *ctf_context;
typedef struct ctf_texture_s *ctf_texture;
typedef struct ctf_decoder_s *ctf_decoder;

/* Filtering methods. */
enum {
    CTF_BILINEAR4 = 0,  /* exact filter, every tap evaluated (4 bilinear, 16 bicubic) per active pixel */
    CTF_STF1 = 1,       /* one-tap STF for every active pixel [Pharr et al. 2024] */
    CTF_LIST = 2,       /* exact duplicate-free set of needed texels (Section 3.1) */
    CTF_BOX = 3,        /* texel bounding box of the wave (Section 3.2) */
    CTF_MASK = 4        /* 16x16 texel bitmask (Section 3.3) */
};

/* Fallback for the participating lanes of a wave whose collaborative step
 * failed (Section 3.4).  Minifying lanes always take the one-tap draw.
 *   CTF_FB_STF1:  each lane returns its one-tap STF texel.
 *   CTF_FB_C:     each lane evaluates its one-tap texel; each lane then
 *                 weights the evaluated texels of its footprint with Eq. 1.
 *   CTF_FB_CPLUS: the distinct one-tap texels are evaluated once and the
 *                 lanes left over evaluate one more texel each from the
 *                 footprint of the lane Eq. 2 assigns them (weighted draw
 *                 among its texels not yet evaluated); then Eq. 1.  Needs
 *                 the wave box to fit 16x16, otherwise CTF_FB_C is used. */
enum { CTF_FB_STF1 = 0, CTF_FB_C = 1, CTF_FB_CPLUS = 2 };

/* Reconstruction filters (Section 5).  A lane at texel position
 * f = (u W - 1/2, v H - 1/2), x0 = floor(f.x), s = f.x - x0 (t likewise):
 *   CTF_FILTER_BILINEAR:    taps x0..x0+1 with weights (1-s, s).
 *   CTF_FILTER_BSPLINE:     taps x0-1..x0+2, uniform cubic B-spline weights
 *                           ((1-s)^3, 3s^3-6s^2+4, -3s^3+3s^2+3s+1, s^3) / 6.
 *   CTF_FILTER_CATMULL_ROM: taps x0-1..x0+2, Catmull-Rom weights
 *                           (-s^3+2s^2-s, 3s^3-5s^2+2, -3s^3+4s^2+s, s^3-s^2) / 2
 *                           (negative lobes).
 * The 2-D weight of tap (i, j) is wx_i wy_j.  The one-tap draw of a cubic
 * filter picks each axis' tap with probability |w_i| / sum |w| and returns
 * the texel's value; the fallbacks use the signed weights in Eq. 1 and |w|
 * for C+'s draws. */
enum { CTF_FILTER_BILINEAR = 0, CTF_FILTER_BSPLINE = 1, CTF_FILTER_CATMULL_ROM = 2 };

/* Split-texel production (the idea of Section 5's DCT discussion: spread one
 * texel's work over idle lanes).  With CTF_SPLIT_AUTO, a procedural-texture
 * wave whose collaborative step succeeded with no one-tap draws spreads the
 * 4n channels of its n texels over all 64 lanes (item j / 4, channel j % 4
 * for j = lane, lane + 64, ...) whenever that takes fewer channel
 * evaluations per lane, ceil(n / 16), than one texel per lane of A,
 * 4 ceil(n / |A|); the terms are read from LDS (textures of at most 62 terms
 * per channel).  Results are bit-identical either way. */
enum { CTF_SPLIT_AUTO = 0, CTF_SPLIT_OFF = 1 };

/* Wave shape.  CTF_WAVE_8X8: one 8x8-pixel tile per wave64 (lane = 8 ly + lx).
 * CTF_WAVE_8X4: the paper's 8x4-pixel tiles of 32 lanes (Section 3), two per
 * wave64, each half-wave taking its own collaborative step; tiles are then
 * 8x4, numbered row-major over ceil(sw/8) x ceil(sh/4) (tile records and
 * lists per 8x4 tile).  8x4 supports every filter and fallback (C+ spreads
 * the spare lanes of a 32-lane tile, Eq. 2 as written) with the procedural /
 * table producers. */
enum { CTF_WAVE_8X8 = 0, CTF_WAVE_8X4 = 1 };

/* Texel producers (Section 3: "produce a texel"). */
enum {
    CTF_TEX_SINUSOIDS = 0,  /* procedural sum of sinusoids (below) */
    CTF_TEX_AFFINE = 1,     /* f_c = a_c0 + a_c1 x + a_c2 y on the texel lattice (tests) */
    CTF_TEX_CONSTANT = 2,   /* f_c = const_c (tests) */
    CTF_TEX_TABLE = 3,      /* stored RGBA float32 texels, repeat addressing */
    CTF_TEX_DECODER = 4     /* learned latent-grid + MLP decoder */
};

enum { CTF_FP16 = 0, CTF_BF16 = 1 };

/* Per-tile flags. */
enum { CTF_TILE_OK = 1, CTF_TILE_CAP = 2, CTF_TILE_OVERFLOW = 4, CTF_TILE_EMPTY = 8 };

/* Most texels one wave can list (4 texels x 64 lanes). */
#define CTF_MAX_ITEMS 256

/* ---------------------------------------------------------------------------
 * Errors and contexts
 * ------------------------------------------------------------------------- */

/* Message of the last failing call on this thread ("" if none). */
const char *ctf_last_error(void);

/* Create a context on HIP device `device`.  The context owns every texture
 * and decoder created from it.  Errors: CTF_ERR_INVALID_ARG (bad device or
 * NULL out), CTF_ERR_DEVICE. */
ctf_status ctf_create(int device, ctf_context *out);

/* Destroy a context after destroying its textures and decoders. */
ctf_status ctf_destroy(ctf_context ctx);

/* ---------------------------------------------------------------------------
 * Textures
 * ------------------------------------------------------------------------- */

typedef struct ctf_texture_desc {
    int32_t kind;            /* CTF_TEX_* */
    int32_t width, height;   /* texel lattice period; powers of two */
    /* CTF_TEX_SINUSOIDS: f_c(x,y) = 1/2 + 1/2 sum_k amp[c][k] *
     *   sin(2 pi ((p x + q y + j) mod width) / width), width == height.
     * pqj: host int32 [4][n_terms][3] = (p, q, j), |p|,|q| < 2^23, 0 <= j;
     * amp: host float [4][n_terms]. Copied at creation. */
    int32_t n_terms;
    const int32_t *pqj;
    const float *amp;
    float affine[4][3];      /* CTF_TEX_AFFINE coefficients */
    float constant[4];       /* CTF_TEX_CONSTANT value */
    const float *table;      /* CTF_TEX_TABLE: host float [height][width][4], copied */
    ctf_decoder decoder;     /* CTF_TEX_DECODER: borrowed; destroy the texture first */
    int32_t precision;       /* CTF_TEX_DECODER inference precision: CTF_FP16 or CTF_BF16 */
    int32_t reserved_[3];
} ctf_texture_desc;

/* Create a texture; parameters are copied to device memory owned by the
 * library.  A decoder texture snapshots the decoder's current parameters
 * (converted to `precision`); later training does not change it.
 * Errors: CTF_ERR_INVALID_ARG (sizes, kinds), CTF_ERR_OUT_OF_MEMORY. */
ctf_status ctf_texture_create(ctf_context ctx, const ctf_texture_desc *desc, ctf_texture *out);
ctf_status ctf_texture_destroy(ctf_texture tex);

/* Evaluate texels: rgba[i] = f(xy[i]) ("produce a texel", Section 3).
 * xy: device int32 [n][2] (x, y) on the unbounded lattice (repeat
 * addressing); rgba: device float [n][4].  Exactly the values ctf_filter
 * produces for the same texels (same instruction sequence). */
ctf_status ctf_texture_eval(ctf_texture tex, const int32_t *xy, int64_t n, float *rgba,
                            void *stream);

/* ---------------------------------------------------------------------------
 * Filtering
 * ------------------------------------------------------------------------- */

typedef struct ctf_method {
    int32_t kind;                /* CTF_BILINEAR4 .. CTF_MASK */
    int32_t box_w, box_h;        /* CTF_BOX per-axis budget; 0,0 = the paper's rule only */
    int32_t mask_side;           /* CTF_MASK: 16 */
    int32_t max_evals_per_lane;  /* k in 1..4: a wave succeeds when n <= k * |A| */
    int32_t fallback;            /* CTF_FB_STF1 / CTF_FB_C / CTF_FB_CPLUS */
    int32_t filter;              /* CTF_FILTER_* */
    int32_t split;               /* CTF_SPLIT_AUTO / CTF_SPLIT_OFF (procedural textures) */
    int32_t wave_shape;          /* CTF_WAVE_8X8 / CTF_WAVE_8X4 */
} ctf_method;

/* One record per tile (128 bytes). */
typedef struct ctf_tile_stats {
    uint64_t active;     /* bit l: lane l has a finite uv with |uv*dim| < 2^24 */
    uint64_t part;       /* A: active and magnifying (both screen-axis footprints <= 1 texel) */
    uint64_t stf;        /* lanes not filtered exactly: a one-tap draw, or fallback C / C+ */
    uint64_t mask[4];    /* 16x16 mask of A's texels relative to (xmin,ymin), bit t = 16 dy + dx
                            in word t/64; zero when the box exceeds 16x16 */
    int32_t xmin, ymin;  /* texel box of A (0 when A is empty) */
    int32_t bbw, bbh;    /* box size, lower-right max(x0+1) inclusive */
    int32_t n;           /* the method's texel count: box area / popcount(mask) / |U| */
    int32_t unique;      /* |U|: exact number of distinct texels A needs */
    int32_t evals;       /* texel evaluations spent by the tile */
    int32_t flags;       /* CTF_TILE_* */
    int32_t reserved[10];
} ctf_tile_stats;

/* Frame totals (accumulated with atomics: zero them before the call). */
typedef struct ctf_frame_stats {
    uint64_t evals;       /* texel evaluations */
    uint64_t active;      /* active pixels */
    uint64_t stf;         /* pixels not filtered exactly (one-tap draw or fallback C / C+) */
    uint64_t minify;      /* active pixels that minify */
    uint64_t tiles;       /* tiles with at least one active pixel */
    uint64_t tiles_ok;    /* tiles whose collaborative step succeeded */
    uint64_t tiles_fail;  /* tiles with a non-empty A whose step failed */
    uint64_t rows;        /* decoder path: MLP rows issued, padding included */
    uint64_t reserved[8];
} ctf_frame_stats;

/* Filter one frame (Section 3; code in the supplement's Section 1).
 *
 * uv: device float [sh][sw][2] texture coordinates (repeat addressing);
 *   a pixel is active iff u, v are finite and |u*width - 1/2|, |v*height -
 *   1/2| < 2^24; inactive pixels output (0,0,0,0).
 * uv_derivs: device float [sh][sw][4] = (du/dx, dv/dx, du/dy, dv/dy); a
 *   lane magnifies iff (du/dx W)^2 + (dv/dx H)^2 <= 1 and likewise for y.
 * out: device float [sh][sw][4] RGBA.
 * seed: the STF draw is a function of (seed, pixel x, pixel y, layer 0) only.
 * tile_stats: nullable device ctf_tile_stats [tiles]; frame_stats: nullable
 *   device ctf_frame_stats (accumulated); debug_lists: nullable device
 *   int32 [tiles][256][2], the (x, y) of item i of every successful tile for
 *   i < n, in the method's order (Box: row-major box cells; Mask and List:
 *   (y, x)-ascending); debug_stf: nullable device int32 [sh][sw][2], the
 *   one-tap texel drawn by each pixel not filtered exactly (also those of
 *   fallback C / C+) and INT32_MIN for the other active pixels.
 * Errors: CTF_ERR_INVALID_ARG (NULL buffers, sw or sh outside 1..2^24, bad
 * method), CTF_ERR_UNSUPPORTED (method/texture combination not built). */
ctf_status ctf_filter(ctf_context ctx, const float *uv, const float *uv_derivs,
                      int32_t sw, int32_t sh, ctf_texture tex, const ctf_method *method,
                      uint64_t seed, float *out, ctf_tile_stats *tile_stats,
                      ctf_frame_stats *frame_stats, int32_t *debug_lists, int32_t *debug_stf,
                      void *stream);

/* Filter n_layers material layers of one frame in one launch.  Layer l
 * samples texs[l] at the layer coordinates uv_l = M_l uv, where M_l =
 * xforms[4l..4l+3] is a row-major 2x2 matrix applied to uv and to both
 * derivative vectors in float32 as u' = fma(m01, v, m00 u), v' = fma(m11, v,
 * m10 u); the STF draw of layer l hashes (seed, pixel, layer l).  Every
 * texture must be a CTF_TEX_DECODER texture of the same precision; 1 <=
 * n_layers <= 8.
 * xforms: host float [n_layers][4]; texs: host array of n_layers handles.
 * out: device float [n_layers][sh][sw][4].  tile_stats: nullable device
 * [n_layers][tiles]; debug_stf: nullable device int32 [n_layers][sh][sw][2];
 * frame_stats: nullable, totals over all layers.  Other arguments as for
 * ctf_filter (every filter and fallback of ctf_filter, 8x8 waves).  Errors:
 * CTF_ERR_INVALID_ARG, CTF_ERR_UNSUPPORTED (non-decoder texture, mixed
 * precisions, 8x4 waves). */
ctf_status ctf_filter_layers(ctf_context ctx, const float *uv, const float *uv_derivs,
                             int32_t sw, int32_t sh, int32_t n_layers, const ctf_texture *texs,
                             const float *xforms, const ctf_method *method, uint64_t seed,
                             float *out, ctf_tile_stats *tile_stats, ctf_frame_stats *frame_stats,
                             int32_t *debug_stf, void *stream);

/* ---------------------------------------------------------------------------
 * Learned decoder (texel producer): latent grids + MLP
 * ------------------------------------------------------------------------- */

typedef struct ctf_decoder_desc {
    int32_t l0, l1;      /* latent grid sides, 2..8192; tex_w / l0 and tex_w / l1 powers of two */
    int32_t hidden;      /* MLP width H (multiple of 4, <= 64): 2C -> H -> H -> 4, ReLU */
    int32_t channels;    /* latent channels per level C: 8 */
    int32_t tex_w;       /* side of the square texel lattice the latents cover */
    int32_t reserved_[3];
} ctf_decoder_desc;

/* Flat parameter layout (float32): lat0 [l0][l0][C], lat1 [l1][l1][C],
 * W1 [2C][H], b1 [H], W2 [H][H], b2 [H], W3 [H][4], b3 [4]; y_o = b_o +
 * sum_i x_i W[i][o].  Texel (x, y) samples level L at ((x+1/2) L/tex_w -
 * 1/2, (y+1/2) L/tex_w - 1/2) bilinearly with repeat addressing. */
size_t ctf_decoder_param_count(const ctf_decoder_desc *desc);

/* Create a decoder with float32 master parameters `init` (host, flat layout,
 * param_count floats) and zero Adam state.  Allocates device memory. */
ctf_status ctf_decoder_create(ctf_context ctx, const ctf_decoder_desc *desc,
                              const float *init, ctf_decoder *out);
ctf_status ctf_decoder_destroy(ctf_decoder dec);

/* Copy the float32 master parameters to / from host memory (flat layout). */
ctf_status ctf_decoder_get_params(ctf_decoder dec, float *host, size_t count);
ctf_status ctf_decoder_set_params(ctf_decoder dec, const float *host, size_t count);

/* Checkpoint: master parameters, Adam moments and step counter as one host
 * blob of ctf_decoder_state_bytes() bytes.  set_state resumes training
 * exactly where get_state left it. */
size_t ctf_decoder_state_bytes(ctf_decoder dec);
ctf_status ctf_decoder_get_state(ctf_decoder dec, void *host, size_t bytes);
ctf_status ctf_decoder_set_state(ctf_decoder dec, const void *host, size_t bytes);

/* Mean squared error over n samples x 4 channels and its gradient for the
 * current parameters, computed by the training kernels in `precision`
 * (CTF_BF16 or CTF_FP16 operands, float32 accumulation).
 * xy: device int32 [n][2]; target: device float [n][4]; loss: device float
 * [1]; grad: device float [param_count] (flat layout).
 * The first call with a larger n than any before grows the decoder's batch
 * buffers (a device allocation); calls on one decoder share those buffers
 * and must not overlap. */
ctf_status ctf_decoder_loss_grad(ctf_decoder dec, const int32_t *xy, const float *target,
                                 int32_t n, int32_t precision, float *loss, float *grad,
                                 void *stream);

/* Most samples one ctf_decoder_loss_grad_noalloc call takes. */
#define CTF_NOALLOC_MAX_SAMPLES 16384

/* ctf_decoder_loss_grad without any device allocation, for callers that
 * cannot allocate: code under HIP graph capture, tight serving or training
 * loops, harnesses that forbid hipMalloc.  Arguments, results and precision
 * as for ctf_decoder_loss_grad (the same kernels in the same order, so the
 * loss and gradient are bitwise equal to that call's); the caller still
 * provides xy, target, loss and grad (device memory).
 * Scratch: a fixed array the library holds on each device from the first
 * ctf_create on that device until the process ends (1.4 MB: per-workgroup
 * partial sums of one pass over at most CTF_NOALLOC_MAX_SAMPLES samples of a
 * decoder with hidden width <= 64), instead of the decoder's batch buffers.
 * Every call on a device uses that device's one array and each pass writes
 * every scratch entry it reads, so nothing carries over from an earlier
 * call; calls that overlap on one device (other streams, other threads,
 * other decoders) race on the array and must be serialised by the caller.
 * Errors: CTF_ERR_INVALID_ARG (NULL buffers, n <= 0 or n above
 * CTF_NOALLOC_MAX_SAMPLES, bad precision), CTF_ERR_DEVICE (no scratch
 * address for the decoder's device). */
ctf_status ctf_decoder_loss_grad_noalloc(ctf_decoder dec, const int32_t *xy, const float *target,
                                         int32_t n, int32_t precision, float *loss, float *grad,
                                         void *stream);

/* Train with Adam (beta 0.9/0.999, eps 1e-8) for `steps` steps of `batch`
 * texels drawn uniformly from the lattice by the pcg hash of (seed, step,
 * sample); targets are produced by `target` (any texel producer).
 * loss_trace: nullable device float [steps], the loss of each step.
 * Grows the batch buffers as ctf_decoder_loss_grad does; calls on one decoder
 * must not overlap.  Errors: CTF_ERR_INVALID_ARG (steps < 0, batch <= 0,
 * lr <= 0, a target of another size or device), CTF_ERR_UNSUPPORTED (a
 * decoder texture as the target). */
ctf_status ctf_decoder_train(ctf_decoder dec, ctf_texture target, int64_t steps,
                             int32_t batch, float lr, uint64_t seed, int32_t precision,
                             float *loss_trace, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* CTF_H */
