/*
 * ctf_oracle.h -- CPU oracle for collaborative texture filtering.
 *
 * TEST INFRASTRUCTURE ONLY.  The plain, slow, obviously correct reference
 * the HIP library is checked against.  Only the test-suite, the smoke check
 * and the benchmark's CPU-baseline leg may load it.  It shares no code,
 * header or table with the HIP library: every type below is declared here
 * again on purpose, with the same field order where a record is compared
 * field by field.
 *
 * Paper: Akenine-Moller, Ebelin, Pharr, Wronski, "Collaborative Texture
 * Filtering", HPG 2025 (arXiv 2506.17770).
 *
 * Floating point: decisions (footprint, minification test, STF draw) are
 * taken in float32 with the exact operation sequence the method fixes
 * (compiled with -ffp-contract=off, fused multiply-adds written as fmaf);
 * colours and decoder arithmetic are float64.
 */
#ifndef CTF_ORACLE_H
#define CTF_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { CTFO_TEX_SINUSOIDS = 0, CTFO_TEX_AFFINE = 1, CTFO_TEX_CONSTANT = 2,
       CTFO_TEX_TABLE = 3, CTFO_TEX_DECODER = 4 };
/* CTFO_BILINEAR4 evaluates every tap of the filter (4, or 16 for bicubic) */
enum { CTFO_BILINEAR4 = 0, CTFO_STF1 = 1, CTFO_LIST = 2, CTFO_BOX = 3, CTFO_MASK = 4 };
enum { CTFO_FB_STF1 = 0, CTFO_FB_C = 1, CTFO_FB_CPLUS = 2 };
enum { CTFO_FILTER_BILINEAR = 0, CTFO_FILTER_BSPLINE = 1, CTFO_FILTER_CATMULL_ROM = 2 };
enum { CTFO_TILE_OK = 1, CTFO_TILE_CAP = 2, CTFO_TILE_OVERFLOW = 4, CTFO_TILE_EMPTY = 8 };

typedef struct ctfo_decoder {
    int32_t l0, l1;        /* latent grid sides (level 0, level 1) */
    int32_t hidden;        /* MLP width H: 2C -> H -> H -> 4 */
    int32_t channels;      /* latent channels C per level */
    int32_t tex_w;         /* side of the texel lattice the latents cover */
    int32_t pad_;
    const double *params;  /* flat: lat0, lat1, W1[2C][H], b1, W2[H][H], b2, W3[H][4], b3 */
} ctfo_decoder;

typedef struct ctfo_texture {
    int32_t kind;
    int32_t width, height;
    int32_t n_terms;            /* K, sinusoids per channel */
    const int32_t *pqj;         /* [4][K][3]: p, q, j */
    const float *amp;           /* [4][K] */
    double affine[4][3];        /* f_c = a0 + a1*x + a2*y */
    double constant[4];
    const float *table;         /* [height][width][4], repeat addressing */
    const ctfo_decoder *dec;
} ctfo_texture;

typedef struct ctfo_method {
    int32_t kind;
    int32_t box_w, box_h;        /* Box budget per axis; 0 = no cap */
    int32_t mask_side;           /* Mask Sampling side (16) */
    int32_t max_evals_per_lane;  /* k >= 1 */
    int32_t fallback;            /* CTFO_FB_* */
    int32_t filter;              /* CTFO_FILTER_*: 2x2 bilinear or 4x4 bicubic taps */
} ctfo_method;

/* One record per tile; same field order as the library's tile record. */
typedef struct ctfo_tile_stats {
    uint64_t active;     /* lanes with a finite, in-range uv */
    uint64_t part;       /* A: active and magnifying */
    uint64_t stf;        /* lanes whose output is a fallback draw */
    uint64_t mask[4];    /* 16x16 wave mask over A's footprints, 0 if box > 16 */
    int32_t xmin, ymin;  /* wave box over A */
    int32_t bbw, bbh;
    int32_t n;           /* the method's texel count */
    int32_t unique;      /* exact number of distinct footprint texels of A */
    int32_t evals;       /* texel evaluations spent by the tile */
    int32_t flags;
    int32_t reserved[10];
} ctfo_tile_stats;

uint32_t ctfo_pcg_hash(uint32_t v);
int ctfo_bit_select(const uint64_t B[4], int32_t i);   /* h(i,B) */
int ctfo_bit_rank(const uint64_t B[4], int32_t t);     /* h^-1(t,B) */

int ctfo_texel_eval(const ctfo_texture *tex, const int32_t *xy, int64_t n, double *rgba);
int ctfo_cplus_target(int32_t nA, int32_t ns, int32_t c);   /* Eq. 2 */

/* xform: nullable 2x2 row-major matrix M applied to uv and to each
 * derivative pair before the footprint (a material layer's texture
 * coordinates), in float32: u' = fma(m01, v, m00 u), v' = fma(m11, v, m10 u).
 * fb_items: nullable [tiles][CTFO_MAX_FB_ITEMS][3]; for a tile that takes
 * fallback C or C+ it receives the texels the fallback produced, in the
 * order they are produced, as (x, y, rank in A of the producing lane);
 * unused entries (and tiles without such a fallback) are left untouched. */
#define CTFO_MAX_FB_ITEMS 128
int ctfo_filter(const float *uv, const float *duv, int32_t sw, int32_t sh,
                int32_t tile_w, int32_t tile_h,
                const ctfo_texture *tex, const ctfo_method *m,
                uint64_t seed, int32_t layer, const float *xform,
                double *out, ctfo_tile_stats *stats, int32_t *lists, int32_t *stf_xy,
                int32_t *fb_items, int64_t tile_begin, int64_t tile_end);

int ctfo_decoder_loss_grad(const ctfo_decoder *dec, const int32_t *xy, const float *target,
                           int64_t n, double *loss, double *grad);

#ifdef __cplusplus
}
#endif
#endif
