/*
 * ctf_oracle.c -- CPU oracle for collaborative texture filtering.
 *
 * TEST INFRASTRUCTURE ONLY (see ctf_oracle.h).  Plain loops, one pixel and
 * one tile at a time, no blocking or fusion.  Colours are float64 sums of
 * all four bilinear texels; the discrete decisions are taken per tile from
 * the float32 inputs with the operation sequence the method fixes.
 *
 * Build: gcc -O2 -ffp-contract=off -fPIC -shared ctf_oracle.c -lm
 */
#include "ctf_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define MAX_LANES 64
#define MAX_ITEMS 256

/* ------------------------------------------------------------------------
 * Hash for the stochastic draw: the "pcg" hash of Jarzynski and Olano,
 * "Hash Functions for GPU Rendering", JCGT 9(3), 2020: one step of the PCG
 * linear congruential generator followed by its RXS-M-XS output permutation.
 * ---------------------------------------------------------------------- */
uint32_t ctfo_pcg_hash(uint32_t v)
{
    uint32_t state = v * 747796405u + 2891336453u;
    uint32_t word = ((state >> ((state >> 28u) + 4u)) ^ state) * 277803737u;
    return (word >> 22u) ^ word;
}

/* ------------------------------------------------------------------------
 * The bijection of Mask Sampling (Section 3.3, Figure 3): h(i,B) is the
 * position of the i-th set bit of the 256-bit mask B, counting from 0;
 * h^-1(t,B) is the number of set bits of B below position t.
 * ---------------------------------------------------------------------- */
static int bit_of(const uint64_t B[4], int t)
{
    return (int)((B[t >> 6] >> (t & 63)) & 1u);
}

int ctfo_bit_select(const uint64_t B[4], int32_t i)
{
    int seen = 0;
    for (int t = 0; t < 256; ++t) {
        if (bit_of(B, t)) {
            if (seen == i) return t;
            ++seen;
        }
    }
    return -1;
}

int ctfo_bit_rank(const uint64_t B[4], int32_t t)
{
    int r = 0;
    for (int b = 0; b < t && b < 256; ++b) r += bit_of(B, b);
    return r;
}

/* ------------------------------------------------------------------------
 * Texel values (float64).  The texel lattice is unbounded; textures repeat
 * with period (width, height).
 * ---------------------------------------------------------------------- */
static int64_t pmod(int64_t a, int64_t m)
{
    int64_t r = a % m;
    return r < 0 ? r + m : r;
}

static void decoder_features(const ctfo_decoder *d, int32_t x, int32_t y, double *feat,
                             int64_t corner_idx[2][4], double corner_w[2][4]);
static void decoder_mlp(const ctfo_decoder *d, const double *feat, double *z1, double *z2,
                        double *out);

static void texel_value(const ctfo_texture *tex, int32_t x, int32_t y, double rgba[4])
{
    switch (tex->kind) {
    case CTFO_TEX_SINUSOIDS: {
        /* f_c(x,y) = 1/2 + 1/2 sum_k a_ck sin(2 pi ((p x + q y + j) mod W) / W) */
        const int64_t W = tex->width;
        for (int c = 0; c < 4; ++c) {
            double acc = 0.0;
            for (int k = 0; k < tex->n_terms; ++k) {
                const int32_t *t = tex->pqj + ((int64_t)c * tex->n_terms + k) * 3;
                int64_t r = pmod((int64_t)t[0] * x + (int64_t)t[1] * y + t[2], W);
                double a = (double)tex->amp[c * tex->n_terms + k];
                acc += a * sin(2.0 * M_PI * (double)r / (double)W);
            }
            rgba[c] = 0.5 + 0.5 * acc;
        }
        break;
    }
    case CTFO_TEX_AFFINE:
        for (int c = 0; c < 4; ++c)
            rgba[c] = tex->affine[c][0] + tex->affine[c][1] * x + tex->affine[c][2] * y;
        break;
    case CTFO_TEX_CONSTANT:
        for (int c = 0; c < 4; ++c) rgba[c] = tex->constant[c];
        break;
    case CTFO_TEX_TABLE: {
        int64_t xx = pmod(x, tex->width), yy = pmod(y, tex->height);
        const float *p = tex->table + (yy * tex->width + xx) * 4;
        for (int c = 0; c < 4; ++c) rgba[c] = (double)p[c];
        break;
    }
    case CTFO_TEX_DECODER: {
        const ctfo_decoder *d = tex->dec;
        double feat[128], z1[256], z2[256];
        int64_t ci[2][4];
        double cw[2][4];
        decoder_features(d, x, y, feat, ci, cw);
        decoder_mlp(d, feat, z1, z2, rgba);
        break;
    }
    default:
        for (int c = 0; c < 4; ++c) rgba[c] = NAN;
    }
}

int ctfo_texel_eval(const ctfo_texture *tex, const int32_t *xy, int64_t n, double *rgba)
{
    if (!tex || (n > 0 && (!xy || !rgba))) return 1;
    for (int64_t i = 0; i < n; ++i) texel_value(tex, xy[2 * i], xy[2 * i + 1], rgba + 4 * i);
    return 0;
}

/* ------------------------------------------------------------------------
 * Per-lane footprint (Section 3 and the supplement's code): the float texel
 * position f = uv * dim - 1/2, texel floor(f), fractional part (s,t).
 * Bilinear uses the 2x2 texels x0..x0+1, y0..y0+1; the bicubic filters of
 * Section 5 (B-spline, Catmull-Rom) the 4x4 texels x0-1..x0+2, y0-1..y0+2.
 * (ox, oy) is the footprint's upper-left texel, F its side; tap (i, j) is
 * texel (ox + i, oy + j) with weight wx[i] wy[j].
 * Minification: a lane is magnifying when both screen-axis footprints span
 * at most one texel (squared lengths <= 1).
 * ---------------------------------------------------------------------- */
typedef struct { int32_t x, y; } texel_t;

typedef struct {
    int in_screen, active, magnify;
    int px, py;
    int32_t x0, y0;
    float s, t;
    int F;                   /* footprint side: 2 or 4 */
    int32_t ox, oy;          /* upper-left texel of the footprint */
    float wx[4], wy[4];      /* float32 tap weights (decisions) */
    double wx64[4], wy64[4]; /* float64 tap weights (colours) */
} lane_t;

static const float RANGE = 16777216.0f; /* |f| must stay below 2^24 */

/* 1-D tap weights at fractional position x in [0, 1).  Bilinear: (1-x, x).
 * Uniform cubic B-spline: (1-x)^3/6, (3x^3-6x^2+4)/6, (-3x^3+3x^2+3x+1)/6,
 * x^3/6.  Catmull-Rom (the cardinal cubic with tangent (f(i+1)-f(i-1))/2):
 * (-x^3+2x^2-x)/2, (3x^3-5x^2+2)/2, (-3x^3+4x^2+x)/2, (x^3-x^2)/2.
 * Both cubic sets sum to one; Catmull-Rom has negative weights. */
static void taps64(int filter, float xs, double w[4])
{
    const double x = xs, x2 = x * x, x3 = x2 * x;
    switch (filter) {
    case CTFO_FILTER_BSPLINE:
        w[0] = (1.0 - x) * (1.0 - x) * (1.0 - x) / 6.0;
        w[1] = (3.0 * x3 - 6.0 * x2 + 4.0) / 6.0;
        w[2] = (-3.0 * x3 + 3.0 * x2 + 3.0 * x + 1.0) / 6.0;
        w[3] = x3 / 6.0;
        break;
    case CTFO_FILTER_CATMULL_ROM:
        w[0] = (-x3 + 2.0 * x2 - x) / 2.0;
        w[1] = (3.0 * x3 - 5.0 * x2 + 2.0) / 2.0;
        w[2] = (-3.0 * x3 + 4.0 * x2 + x) / 2.0;
        w[3] = (x3 - x2) / 2.0;
        break;
    default:
        w[0] = 1.0 - x;
        w[1] = x;
        w[2] = w[3] = 0.0;
    }
}

/* The same weights in float32 with one fixed operation order (products,
 * then sums left to right, then the constant factor); the stochastic draws
 * and the fallbacks' discrete choices use these. */
static void taps32(int filter, float x, float w[4])
{
    const float x2 = x * x, x3 = x2 * x, om = 1.0f - x;
    const float sixth = (float)(1.0 / 6.0);
    switch (filter) {
    case CTFO_FILTER_BSPLINE:
        w[0] = ((om * om) * om) * sixth;
        w[1] = ((3.0f * x3 - 6.0f * x2) + 4.0f) * sixth;
        w[2] = (((-3.0f * x3 + 3.0f * x2) + 3.0f * x) + 1.0f) * sixth;
        w[3] = x3 * sixth;
        break;
    case CTFO_FILTER_CATMULL_ROM:
        w[0] = ((2.0f * x2 - x3) - x) * 0.5f;
        w[1] = ((3.0f * x3 - 5.0f * x2) + 2.0f) * 0.5f;
        w[2] = ((-3.0f * x3 + 4.0f * x2) + x) * 0.5f;
        w[3] = (x3 - x2) * 0.5f;
        break;
    default:
        w[0] = om;
        w[1] = x;
        w[2] = w[3] = 0.0f;
    }
}

static void footprint(const float *uv, const float *duv, int32_t W, int32_t H, int filter, lane_t *L)
{
    float u = uv[0], v = uv[1];
    L->active = 0;
    L->magnify = 0;
    if (!isfinite(u) || !isfinite(v)) return;
    float fx = fmaf(u, (float)W, -0.5f);
    float fy = fmaf(v, (float)H, -0.5f);
    if (!(fabsf(fx) < RANGE) || !(fabsf(fy) < RANGE)) return;
    float flx = floorf(fx), fly = floorf(fy);
    L->x0 = (int32_t)flx;
    L->y0 = (int32_t)fly;
    L->s = fx - flx;
    L->t = fy - fly;
    L->F = filter == CTFO_FILTER_BILINEAR ? 2 : 4;
    L->ox = L->x0 - (L->F == 4);
    L->oy = L->y0 - (L->F == 4);
    taps32(filter, L->s, L->wx);
    taps32(filter, L->t, L->wy);
    taps64(filter, L->s, L->wx64);
    taps64(filter, L->t, L->wy64);
    L->active = 1;
    float a = duv[0] * (float)W, b = duv[1] * (float)H;
    float c = duv[2] * (float)W, d = duv[3] * (float)H;
    float rx2 = fmaf(a, a, b * b);
    float ry2 = fmaf(c, c, d * d);
    L->magnify = (rx2 <= 1.0f) && (ry2 <= 1.0f);
}

/* One-tap STF draw: texel (x0 + [u1 < s], y0 + [u2 < t]) with u1, u2 24-bit
 * uniforms from the hash of (seed, layer, pixel).  Picks texel k with
 * probability equal to its bilinear weight (to 2^-24). */
static void stf_hashes(const lane_t *L, uint64_t seed, int32_t layer, uint32_t h[3])
{
    uint32_t lo = (uint32_t)seed, hi = (uint32_t)(seed >> 32);
    uint32_t g = ctfo_pcg_hash((uint32_t)layer ^ hi);
    g = ctfo_pcg_hash((uint32_t)L->py ^ g);
    g = ctfo_pcg_hash((uint32_t)L->px ^ g);
    h[0] = ctfo_pcg_hash(lo ^ g);
    h[1] = ctfo_pcg_hash(h[0]);
    h[2] = ctfo_pcg_hash(h[1]);   /* third draw: the C+ spare-lane choice */
}

static float unit24(uint32_t h) { return (float)(h >> 8) * 0x1p-24f; }

/* Cubic one-tap draw along one axis: tap i with probability |w_i| / sum |w|
 * (the absolute weights, so negative lobes are drawn too).  Partial sums in
 * float32, left to right; the drawn tap is the number of partial sums at or
 * below u * sum (a zero-weight tap has an empty interval, never drawn). */
static int cubic_tap(const float w[4], float u)
{
    const float a0 = fabsf(w[0]), a1 = fabsf(w[1]), a2 = fabsf(w[2]), a3 = fabsf(w[3]);
    const float p1 = a0, p2 = p1 + a1, p3 = p2 + a2, sum = p3 + a3;
    const float thr = u * sum;
    return (thr >= p1) + (thr >= p2) + (thr >= p3);
}

/* One-tap STF draw.  Bilinear: texel (x0 + [u1 < s], y0 + [u2 < t]), i.e.
 * texel k with probability equal to its weight (to 2^-24).  Bicubic: the
 * axes are drawn independently by cubic_tap, which picks a tap with
 * probability |wx_i| |wy_j| / (sum |wx|)(sum |wy|). */
static void stf_pick(const lane_t *L, uint64_t seed, int32_t layer, int32_t out[2])
{
    uint32_t h[3];
    stf_hashes(L, seed, layer, h);
    if (L->F == 2) {
        out[0] = L->x0 + (unit24(h[0]) < L->s ? 1 : 0);
        out[1] = L->y0 + (unit24(h[1]) < L->t ? 1 : 0);
    } else {
        out[0] = L->ox + cubic_tap(L->wx, unit24(h[0]));
        out[1] = L->oy + cubic_tap(L->wy, unit24(h[1]));
    }
}

/* Eq. 2 for a wave of nA participating lanes of which ns produce the
 * distinct one-tap texels: spare lane of rank c in [ns, nA) adds a texel of
 * the footprint of the lane of rank round((nA-1)(c-ns)/(nA-1-ns)) (ties up);
 * a single spare lane maps to rank 0. */
int ctfo_cplus_target(int32_t nA, int32_t ns, int32_t c)
{
    const int span = nA - 1 - ns;
    if (span <= 0) return 0;
    return (2 * (nA - 1) * (c - ns) + span) / (2 * span);
}

static int texel_in(const texel_t *set, int n, int32_t x, int32_t y)
{
    for (int i = 0; i < n; ++i)
        if (set[i].x == x && set[i].y == y) return 1;
    return 0;
}

/* ------------------------------------------------------------------------
 * Exact unique set of the footprint texels of the lanes in A, as keys
 * sorted by (y, x): plain collect, sort, drop duplicates.
 * ---------------------------------------------------------------------- */
static int cmp_texel(const void *a, const void *b)
{
    const texel_t *p = (const texel_t *)a, *q = (const texel_t *)b;
    if (p->y != q->y) return p->y < q->y ? -1 : 1;
    if (p->x != q->x) return p->x < q->x ? -1 : 1;
    return 0;
}

static int unique_set(const lane_t *lanes, int nl, uint64_t A, texel_t *U)
{
    texel_t all[16 * MAX_LANES];
    int m = 0;
    for (int l = 0; l < nl; ++l) {
        if (!((A >> l) & 1u)) continue;
        const int F = lanes[l].F;
        for (int k = 0; k < F * F; ++k) {
            all[m].x = lanes[l].ox + k % F;
            all[m].y = lanes[l].oy + k / F;
            ++m;
        }
    }
    qsort(all, (size_t)m, sizeof(texel_t), cmp_texel);
    int n = 0;
    for (int i = 0; i < m; ++i)
        if (n == 0 || cmp_texel(&all[i], &U[n - 1]) != 0) U[n++] = all[i];
    return n;
}

static int popcount64(uint64_t v)
{
    int c = 0;
    while (v) { c += (int)(v & 1u); v >>= 1; }
    return c;
}

/* ------------------------------------------------------------------------
 * The filter.  Tiles are tile_w x tile_h pixels, one wave each, lane =
 * tile_w * ly + lx, tiles row-major over the screen.
 * ---------------------------------------------------------------------- */
/* A material layer's coordinates: uv' = M uv and the same for each of the
 * two derivative vectors, in float32 with one fixed operation order. */
static void layer_transform(const float *M, const float *uv, const float *duv, float uv_out[2],
                            float duv_out[4])
{
    uv_out[0] = fmaf(M[1], uv[1], M[0] * uv[0]);
    uv_out[1] = fmaf(M[3], uv[1], M[2] * uv[0]);
    duv_out[0] = fmaf(M[1], duv[1], M[0] * duv[0]);
    duv_out[1] = fmaf(M[3], duv[1], M[2] * duv[0]);
    duv_out[2] = fmaf(M[1], duv[3], M[0] * duv[2]);
    duv_out[3] = fmaf(M[3], duv[3], M[2] * duv[2]);
}

int ctfo_filter(const float *uv, const float *duv, int32_t sw, int32_t sh,
                int32_t tile_w, int32_t tile_h,
                const ctfo_texture *tex, const ctfo_method *m,
                uint64_t seed, int32_t layer, const float *xform,
                double *out, ctfo_tile_stats *stats, int32_t *lists, int32_t *stf_xy,
                int32_t *fb_items, int64_t tile_begin, int64_t tile_end)
{
    if (!uv || !duv || !tex || !m || !out) return 1;
    if (sw <= 0 || sh <= 0 || tile_w <= 0 || tile_h <= 0 || tile_w * tile_h > MAX_LANES) return 1;
    if (m->max_evals_per_lane < 1 || m->max_evals_per_lane > 4) return 1;
    if (m->filter < CTFO_FILTER_BILINEAR || m->filter > CTFO_FILTER_CATMULL_ROM) return 1;
    if (m->fallback < CTFO_FB_STF1 || m->fallback > CTFO_FB_CPLUS) return 1;
    const int32_t W = tex->width, H = tex->height;
    const int nl = tile_w * tile_h;
    const int64_t tiles_x = (sw + tile_w - 1) / tile_w;
    const int64_t tiles_y = (sh + tile_h - 1) / tile_h;
    if (tile_end < 0 || tile_end > tiles_x * tiles_y) tile_end = tiles_x * tiles_y;

    for (int64_t tile = tile_begin; tile < tile_end; ++tile) {
        const int64_t tx = tile % tiles_x, ty = tile / tiles_x;
        lane_t lanes[MAX_LANES];
        uint64_t active = 0, A = 0;

        /* step 1: per-lane footprint, participation */
        for (int l = 0; l < nl; ++l) {
            lane_t *L = &lanes[l];
            L->px = (int)(tx * tile_w + l % tile_w);
            L->py = (int)(ty * tile_h + l / tile_w);
            L->in_screen = L->px < sw && L->py < sh;
            L->active = L->magnify = 0;
            if (L->in_screen) {
                int64_t p = (int64_t)L->py * sw + L->px;
                if (xform) {
                    float luv[2], lduv[4];
                    layer_transform(xform, uv + 2 * p, duv + 4 * p, luv, lduv);
                    footprint(luv, lduv, W, H, m->filter, L);
                } else {
                    footprint(uv + 2 * p, duv + 4 * p, W, H, m->filter, L);
                }
                for (int c = 0; c < 4; ++c) out[4 * p + c] = 0.0;
                if (stf_xy) stf_xy[2 * p] = stf_xy[2 * p + 1] = INT32_MIN;
            }
            if (L->active) active |= 1ull << l;
            if (L->active && L->magnify) A |= 1ull << l;
        }
        const int nA = popcount64(A);

        /* step 2: wave box over A (min of upper-left, max of lower-right) */
        int64_t xmin = 0, ymin = 0, xmax = -1, ymax = -1;
        int first = 1;
        for (int l = 0; l < nl; ++l) {
            if (!((A >> l) & 1u)) continue;
            int64_t x0 = lanes[l].ox, y0 = lanes[l].oy, e = lanes[l].F - 1;
            if (first || x0 < xmin) xmin = x0;
            if (first || y0 < ymin) ymin = y0;
            if (first || x0 + e > xmax) xmax = x0 + e;
            if (first || y0 + e > ymax) ymax = y0 + e;
            first = 0;
        }
        const int64_t bbw = nA ? xmax - xmin + 1 : 0;
        const int64_t bbh = nA ? ymax - ymin + 1 : 0;

        /* exact unique set (brute force) and 16x16 mask when the box fits */
        texel_t U[16 * MAX_LANES];
        const int nU = unique_set(lanes, nl, A, U);
        uint64_t B[4] = {0, 0, 0, 0};
        const int fits16 = nA && bbw <= 16 && bbh <= 16;
        if (fits16)
            for (int i = 0; i < nU; ++i) {
                int t = 16 * (int)(U[i].y - ymin) + (int)(U[i].x - xmin);
                B[t >> 6] |= 1ull << (t & 63);
            }

        /* step 3: the method's decision */
        const int k = m->max_evals_per_lane;
        int64_t n = 0;
        int cap_ok = 1, count_ok = 1, success = 0;
        texel_t items[MAX_ITEMS];
        switch (m->kind) {
        case CTFO_BILINEAR4:
        case CTFO_STF1:
            break;
        case CTFO_BOX:
            n = bbw * bbh;
            cap_ok = (m->box_w == 0 || bbw <= m->box_w) && (m->box_h == 0 || bbh <= m->box_h);
            count_ok = n <= (int64_t)k * nA;
            success = nA > 0 && cap_ok && count_ok;
            if (success)
                for (int64_t i = 0; i < n; ++i) {
                    items[i].x = (int32_t)(xmin + i % bbw);
                    items[i].y = (int32_t)(ymin + i / bbw);
                }
            break;
        case CTFO_MASK: {
            const int side = m->mask_side;
            if (side != 16) return 1;
            cap_ok = nA > 0 && bbw <= side && bbh <= side;
            if (cap_ok) {
                /* each lane of A sets the bits of its FxF texels; B is their OR */
                uint64_t Bm[4] = {0, 0, 0, 0};
                for (int l = 0; l < nl; ++l) {
                    if (!((A >> l) & 1u)) continue;
                    const int F = lanes[l].F;
                    for (int q = 0; q < F * F; ++q) {
                        const int tq = 16 * (int)(lanes[l].oy + q / F - ymin) + (int)(lanes[l].ox + q % F - xmin);
                        Bm[tq >> 6] |= 1ull << (tq & 63);
                    }
                }
                n = popcount64(Bm[0]) + popcount64(Bm[1]) + popcount64(Bm[2]) + popcount64(Bm[3]);
                count_ok = n <= (int64_t)k * nA;
                success = count_ok;
                if (success)
                    for (int64_t i = 0; i < n; ++i) {
                        int t = ctfo_bit_select(Bm, (int32_t)i);
                        items[i].x = (int32_t)(xmin + (t & 15));
                        items[i].y = (int32_t)(ymin + (t >> 4));
                    }
            }
            break;
        }
        case CTFO_LIST:
            n = nU;
            count_ok = n <= (int64_t)k * nA;
            success = nA > 0 && count_ok;
            if (success)
                for (int i = 0; i < nU; ++i) items[i] = U[i];
            break;
        default:
            return 1;
        }

        /* Fallback of the lanes of A when the wave fails (Section 3.4):
         * C: every lane of A produces its one-tap texel; C+: the distinct
         * one-tap texels (mask S, one bit per lane) are produced once and the
         * remaining lanes of A produce extra texels (Eq. 2); both weight the
         * produced texels of each footprint with Eq. 1.  C+ needs the wave
         * box to fit the 16x16 mask, otherwise C is used. */
        int fb = CTFO_FB_STF1;
        if (!success && nA > 0 && (m->kind == CTFO_LIST || m->kind == CTFO_BOX || m->kind == CTFO_MASK))
            fb = m->fallback;
        if (fb == CTFO_FB_CPLUS && !fits16) fb = CTFO_FB_C;
        texel_t prod[2 * MAX_LANES];
        int prod_rank[2 * MAX_LANES];   /* rank in A of the lane producing prod[i] */
        int nprod = 0, fb_evals = 0;
        if (fb == CTFO_FB_C) {
            for (int l = 0; l < nl; ++l) {
                if (!((A >> l) & 1u)) continue;
                int32_t pk[2];
                stf_pick(&lanes[l], seed, layer, pk);
                prod[nprod].x = pk[0];
                prod[nprod].y = pk[1];
                prod_rank[nprod] = nprod;
                ++nprod;
            }
            fb_evals = nA;
        } else if (fb == CTFO_FB_CPLUS) {
            uint64_t Sm[4] = {0, 0, 0, 0};
            int rank_lane[MAX_LANES];
            int r = 0;
            for (int l = 0; l < nl; ++l) {
                if (!((A >> l) & 1u)) continue;
                rank_lane[r++] = l;
                int32_t pk[2];
                stf_pick(&lanes[l], seed, layer, pk);
                int t = 16 * (int)(pk[1] - ymin) + (int)(pk[0] - xmin);
                Sm[t >> 6] |= 1ull << (t & 63);
            }
            const int ns = popcount64(Sm[0]) + popcount64(Sm[1]) + popcount64(Sm[2]) + popcount64(Sm[3]);
            for (int i = 0; i < ns; ++i) {           /* item i made by the lane of rank i */
                int t = ctfo_bit_select(Sm, i);
                prod[nprod].x = (int32_t)(xmin + (t & 15));
                prod[nprod].y = (int32_t)(ymin + (t >> 4));
                prod_rank[nprod] = i;
                ++nprod;
            }
            fb_evals = ns;
            for (int c = ns; c < nA; ++c) {           /* spare lanes, Eq. 2 */
                const int tr = ctfo_cplus_target(nA, ns, c);
                const lane_t *T = &lanes[rank_lane[tr]];
                const int F = T->F;
                /* candidates: the target's taps (row-major) with a nonzero
                 * float32 weight that are not in S, drawn by |weight| */
                float aw[16];
                int cand[16], nc = 0;
                float wsum = 0.0f;
                for (int q = 0; q < F * F; ++q) {
                    const float wq = T->wx[q % F] * T->wy[q / F];
                    const int tq = 16 * (int)(T->oy + q / F - ymin) + (int)(T->ox + q % F - xmin);
                    if (wq != 0.0f && !bit_of(Sm, tq)) {
                        aw[nc] = fabsf(wq);
                        cand[nc++] = q;
                        wsum += fabsf(wq);
                    }
                }
                if (nc == 0) continue;
                uint32_t h[3];
                stf_hashes(&lanes[rank_lane[c]], seed, layer, h);
                const float thr = unit24(h[2]) * wsum;
                int pickq = cand[nc - 1];
                float run = 0.0f;
                for (int k = 0; k < nc; ++k) {
                    run += aw[k];
                    if (run > thr) { pickq = cand[k]; break; }
                }
                prod[nprod].x = T->ox + pickq % F;
                prod[nprod].y = T->oy + pickq / F;
                prod_rank[nprod] = c;
                ++nprod;
                ++fb_evals;
            }
        }

        /* steps 4-6: produce, gather and weight; other non-exact lanes draw one texel */
        uint64_t stfmask = 0;
        int64_t evals = fb_evals;
        for (int l = 0; l < nl; ++l) {
            const lane_t *L = &lanes[l];
            if (!L->active) continue;
            const int64_t p = (int64_t)L->py * sw + L->px;
            double *o = out + 4 * p;
            int exact;
            if (m->kind == CTFO_BILINEAR4) exact = 1;
            else if (m->kind == CTFO_STF1) exact = 0;
            else exact = ((A >> l) & 1u) && success;
            const int F = L->F;
            if (!exact && fb != CTFO_FB_STF1 && ((A >> l) & 1u)) {
                /* Eq. 1 over the produced texels of this footprint with a
                 * nonzero (float32) weight */
                double f[4], acc[4] = {0, 0, 0, 0}, sum[4] = {0, 0, 0, 0}, wsum = 0.0;
                int N = 0;
                for (int q = 0; q < F * F; ++q) {
                    const int32_t x = L->ox + q % F, y = L->oy + q / F;
                    const float w32 = L->wx[q % F] * L->wy[q / F];
                    const double w = L->wx64[q % F] * L->wy64[q / F];
                    if (w32 == 0.0f || !texel_in(prod, nprod, x, y)) continue;
                    texel_value(tex, x, y, f);
                    for (int c = 0; c < 4; ++c) {
                        acc[c] += w * f[c];
                        sum[c] += f[c];
                    }
                    wsum += w;
                    ++N;
                }
                int32_t pick[2];
                stf_pick(L, seed, layer, pick);
                if (N == 0) {   /* only if the drawn texel's float32 weight underflowed */
                    texel_value(tex, pick[0], pick[1], f);
                    for (int c = 0; c < 4; ++c) o[c] = f[c];
                } else {
                    for (int c = 0; c < 4; ++c) o[c] = acc[c] + (1.0 - wsum) * sum[c] / N;
                }
                if (stf_xy) { stf_xy[2 * p] = pick[0]; stf_xy[2 * p + 1] = pick[1]; }
                stfmask |= 1ull << l;
                continue;
            }
            if (exact) {
                /* the plain definition: every tap of the filter */
                double f[4];
                for (int q = 0; q < F * F; ++q) {
                    const double w = L->wx64[q % F] * L->wy64[q / F];
                    texel_value(tex, L->ox + q % F, L->oy + q / F, f);
                    for (int c = 0; c < 4; ++c) o[c] += w * f[c];
                }
                if (m->kind == CTFO_BILINEAR4) evals += F * F;
            } else {
                int32_t pick[2];
                double f[4];
                stf_pick(L, seed, layer, pick);
                texel_value(tex, pick[0], pick[1], f);
                for (int c = 0; c < 4; ++c) o[c] = f[c];
                if (stf_xy) { stf_xy[2 * p] = pick[0]; stf_xy[2 * p + 1] = pick[1]; }
                stfmask |= 1ull << l;
                evals += 1;
            }
        }
        if (success) evals += n;

        if (fb_items && fb != CTFO_FB_STF1)
            for (int i = 0; i < nprod; ++i) {
                int32_t *e = fb_items + (tile * CTFO_MAX_FB_ITEMS + i) * 3;
                e[0] = prod[i].x;
                e[1] = prod[i].y;
                e[2] = prod_rank[i];
            }
        if (lists && success)
            for (int64_t i = 0; i < n; ++i) {
                lists[(tile * MAX_ITEMS + i) * 2] = items[i].x;
                lists[(tile * MAX_ITEMS + i) * 2 + 1] = items[i].y;
            }
        if (stats) {
            ctfo_tile_stats *S = &stats[tile];
            memset(S, 0, sizeof(*S));
            S->active = active;
            S->part = A;
            S->stf = stfmask;
            for (int q = 0; q < 4; ++q) S->mask[q] = B[q];
            S->xmin = (int32_t)(nA ? xmin : 0);
            S->ymin = (int32_t)(nA ? ymin : 0);
            S->bbw = (int32_t)bbw;
            S->bbh = (int32_t)bbh;
            S->n = (int32_t)(n > INT32_MAX ? INT32_MAX : n);
            S->unique = nU;
            S->evals = (int32_t)evals;
            S->flags = (success ? CTFO_TILE_OK : 0) |
                       (nA && !cap_ok ? CTFO_TILE_CAP : 0) |
                       (nA && cap_ok && !count_ok ? CTFO_TILE_OVERFLOW : 0) |
                       (nA == 0 ? CTFO_TILE_EMPTY : 0);
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------
 * Learned decoder (float64): two latent grids sampled bilinearly with
 * repeat addressing at g = (x + 1/2) L / W - 1/2, concatenated (level 0
 * channels, then level 1), then an MLP 2C -> H -> H -> 4 with ReLU on the
 * hidden layers and a linear output.
 * ---------------------------------------------------------------------- */
static void decoder_features(const ctfo_decoder *d, int32_t x, int32_t y, double *feat,
                             int64_t corner_idx[2][4], double corner_w[2][4])
{
    const int C = d->channels;
    const double *lat[2] = {d->params, d->params + (int64_t)d->l0 * d->l0 * C};
    const int sides[2] = {d->l0, d->l1};
    for (int lev = 0; lev < 2; ++lev) {
        const int L = sides[lev];
        double gx = ((double)x + 0.5) * L / d->tex_w - 0.5;
        double gy = ((double)y + 0.5) * L / d->tex_w - 0.5;
        double cx = floor(gx), cy = floor(gy);
        double fx = gx - cx, fy = gy - cy;
        int64_t x0 = pmod((int64_t)cx, L), x1 = pmod((int64_t)cx + 1, L);
        int64_t y0 = pmod((int64_t)cy, L), y1 = pmod((int64_t)cy + 1, L);
        int64_t idx[4] = {y0 * L + x0, y0 * L + x1, y1 * L + x0, y1 * L + x1};
        double w[4] = {(1 - fx) * (1 - fy), fx * (1 - fy), (1 - fx) * fy, fx * fy};
        for (int c = 0; c < C; ++c) {
            double v = 0.0;
            for (int q = 0; q < 4; ++q) v += w[q] * lat[lev][idx[q] * C + c];
            feat[lev * C + c] = v;
        }
        for (int q = 0; q < 4; ++q) {
            corner_idx[lev][q] = idx[q];
            corner_w[lev][q] = w[q];
        }
    }
}

typedef struct { int64_t W1, b1, W2, b2, W3, b3, lat1, total; } dec_offsets;

static dec_offsets offsets(const ctfo_decoder *d)
{
    const int64_t C = d->channels, H = d->hidden;
    dec_offsets o;
    o.lat1 = (int64_t)d->l0 * d->l0 * C;
    o.W1 = o.lat1 + (int64_t)d->l1 * d->l1 * C;
    o.b1 = o.W1 + 2 * C * H;
    o.W2 = o.b1 + H;
    o.b2 = o.W2 + H * H;
    o.W3 = o.b2 + H;
    o.b3 = o.W3 + H * 4;
    o.total = o.b3 + 4;
    return o;
}

static void decoder_mlp(const ctfo_decoder *d, const double *feat, double *z1, double *z2,
                        double *out)
{
    const int F = 2 * d->channels, H = d->hidden;
    const dec_offsets o = offsets(d);
    const double *P = d->params;
    for (int h = 0; h < H; ++h) {
        double a = P[o.b1 + h];
        for (int i = 0; i < F; ++i) a += feat[i] * P[o.W1 + (int64_t)i * H + h];
        z1[h] = a;
    }
    for (int h = 0; h < H; ++h) {
        double a = P[o.b2 + h];
        for (int i = 0; i < H; ++i) a += (z1[i] > 0 ? z1[i] : 0.0) * P[o.W2 + (int64_t)i * H + h];
        z2[h] = a;
    }
    for (int c = 0; c < 4; ++c) {
        double a = P[o.b3 + c];
        for (int i = 0; i < H; ++i) a += (z2[i] > 0 ? z2[i] : 0.0) * P[o.W3 + (int64_t)i * 4 + c];
        out[c] = a;
    }
}

/* Mean squared error over n samples and 4 channels, and its exact gradient
 * with respect to every parameter (flat layout), by the chain rule. */
int ctfo_decoder_loss_grad(const ctfo_decoder *d, const int32_t *xy, const float *target,
                           int64_t n, double *loss, double *grad)
{
    if (!d || !xy || !target || !loss || n <= 0) return 1;
    if (d->hidden > 256 || 2 * d->channels > 128) return 1;
    const int C = d->channels, F = 2 * C, H = d->hidden;
    const dec_offsets o = offsets(d);
    const double *P = d->params;
    if (grad) memset(grad, 0, sizeof(double) * (size_t)o.total);
    double sum = 0.0;
    const double scale = 1.0 / (4.0 * (double)n);
    for (int64_t s = 0; s < n; ++s) {
        double feat[128], z1[256], z2[256], y[4];
        int64_t ci[2][4];
        double cw[2][4];
        decoder_features(d, xy[2 * s], xy[2 * s + 1], feat, ci, cw);
        decoder_mlp(d, feat, z1, z2, y);
        double dy[4];
        for (int c = 0; c < 4; ++c) {
            double e = y[c] - (double)target[4 * s + c];
            sum += e * e;
            dy[c] = 2.0 * e * scale;
        }
        if (!grad) continue;
        double dz2[256], dz1[256], dx[128];
        for (int c = 0; c < 4; ++c) grad[o.b3 + c] += dy[c];
        for (int i = 0; i < H; ++i) {
            double a2 = z2[i] > 0 ? z2[i] : 0.0;
            double g = 0.0;
            for (int c = 0; c < 4; ++c) {
                grad[o.W3 + (int64_t)i * 4 + c] += a2 * dy[c];
                g += P[o.W3 + (int64_t)i * 4 + c] * dy[c];
            }
            dz2[i] = z2[i] > 0 ? g : 0.0;
        }
        for (int h = 0; h < H; ++h) grad[o.b2 + h] += dz2[h];
        for (int i = 0; i < H; ++i) {
            double a1 = z1[i] > 0 ? z1[i] : 0.0;
            double g = 0.0;
            for (int h = 0; h < H; ++h) {
                grad[o.W2 + (int64_t)i * H + h] += a1 * dz2[h];
                g += P[o.W2 + (int64_t)i * H + h] * dz2[h];
            }
            dz1[i] = z1[i] > 0 ? g : 0.0;
        }
        for (int h = 0; h < H; ++h) grad[o.b1 + h] += dz1[h];
        for (int i = 0; i < F; ++i) {
            double g = 0.0;
            for (int h = 0; h < H; ++h) {
                grad[o.W1 + (int64_t)i * H + h] += feat[i] * dz1[h];
                g += P[o.W1 + (int64_t)i * H + h] * dz1[h];
            }
            dx[i] = g;
        }
        for (int lev = 0; lev < 2; ++lev) {
            int64_t base = lev == 0 ? 0 : o.lat1;
            for (int q = 0; q < 4; ++q)
                for (int c = 0; c < C; ++c)
                    grad[base + ci[lev][q] * C + c] += cw[lev][q] * dx[lev * C + c];
        }
    }
    *loss = sum * scale;
    return 0;
}
