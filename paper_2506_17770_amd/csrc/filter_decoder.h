// filter_decoder.h -- collaborative filtering with the learned texel producer.
//
// Same decisions as the per-lane path (Sections 3.1-3.3, remapping, the
// fallbacks of Section 3.4 and the bicubic filters of Section 5), but texel
// production is batched: the wave writes the (x, y) of every texel it must
// produce into an LDS row list (the unique texels first, then one row per
// one-tap draw; in a wave that takes fallback C or C+, the planned texels of
// A, then the minifying lanes' draws) and decodes the rows 16 at a time on
// MFMA (decoder_mlp.h).  Dedup therefore turns the per-tap decode into one
// dense MLP pass over the wave's distinct texels.
//
// Waves are persistent: each loads the MLP weights into registers once and
// walks its share of the tiles.  Workgroups are dispatched round-robin over
// the 8 XCDs; XCD x takes every eighth strip of two tile rows (Band), so
// that the latent-grid reads of neighbouring tiles share an L2 while every
// XCD gets a like share of the frame's work.
//
// Instantiated per reconstruction filter (FxF footprints, F = 2 or 4): the
// bilinear kernels in filter_decoder.hip, the bicubic ones in
// filter_decoder_cubic.hip.
#pragma once

#include <stddef.h>

#include "ctf_device.h"
#include "ctf_internal.h"
#include "decoder_mlp.h"
#include "fallback.h"

namespace ctf {

namespace dec {

constexpr int kDecWaves = 4;

// vals, rows and keys are contiguous: the bicubic List sort uses the three
// as one 1024-key buffer before any row or value exists.
struct DecLds {
    float4 vals[kMaxItems];     // decoded texels, by row
    int2 rows[kMaxItems];       // texel coordinates to decode
    uint64_t keys[kMaxItems];   // List past 16x16 (bilinear): sorted unique keys
    uint8_t rank[256];          // Mask/List: position t -> row (h^-1)
    uint8_t bytes[256];         // footprint-corner scatter before the ballots
};
static_assert(offsetof(DecLds, rows) == 16 * kMaxItems && offsetof(DecLds, keys) == 24 * kMaxItems,
              "sort buffer layout");

// Sort buffer of the List past 16x16: F^2 keys per lane.
template <int F>
__device__ __forceinline__ uint64_t* dec_keys(DecLds& L)
{
    if constexpr (F == 2) return L.keys;
    else return reinterpret_cast<uint64_t*>(&L);
}

// Exact set of the wave's texels as sorted unique keys (any box size): a
// bitonic sort of the F^2 |A| footprint keys, then compaction of the first
// key of every run.  Returns n = |U|; dec_keys<F>(L)[0..n) hold U in (y, x)
// order.
template <int F>
__device__ int dec_list_sorted(DecLds& L, bool inA, int ox, int oy, int xmin, int ymin)
{
    constexpr int N = kWave * F * F;
    uint64_t* keys = dec_keys<F>(L);
    const int lane = lane_id();
#pragma unroll
    for (int q = 0; q < F * F; ++q) {
        uint64_t key = ~0ull;
        if (inA)
            key = ((uint64_t)(uint32_t)(oy + q / F - ymin) << 32) | (uint32_t)(ox + q % F - xmin);
        keys[F * F * lane + q] = key;
    }
    for (int size = 2; size <= N; size <<= 1)
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            wave_lds_sync();
#pragma unroll
            for (int h = 0; h < N / (2 * kWave); ++h) {
                const int p = lane + kWave * h;
                const int i = (p / stride) * stride * 2 + (p % stride);
                const int j = i + stride;
                const bool up = (i & size) == 0;
                const uint64_t x = keys[i], y = keys[j];
                if ((x > y) == up) {
                    keys[i] = y;
                    keys[j] = x;
                }
            }
        }
    // compaction in rounds of 64 keys: a write index never passes the read
    // index, and round r writes below every key of the later rounds
    int base = 0;
    for (int c = 0; c < F * F; ++c) {
        wave_lds_sync();
        const int i = kWave * c + lane;
        const uint64_t k = keys[i];
        const bool first = k != ~0ull && (i == 0 || keys[i - 1] != k);
        const uint64_t b = ballot(first);
        wave_lds_sync();
        if (first) keys[base + mbcnt(b)] = k;
        base += popc64(b);
    }
    wave_lds_sync();
    return base;
}

__device__ __forceinline__ int dec_list_find(const uint64_t* keys, int n, uint64_t key)
{
    int lo = 0, hi = n;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (keys[mid] < key) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// Rows past R read whatever the row list holds there (the index is kept
// inside the list): the inference fetch maps any texel to cells inside the
// grid, and those rows' results are never stored.
template <int P>
__device__ __forceinline__ void fetch_row(const int2* rows, int row, const InferGrid& G, const InferLane<P>& K,
                                          InferFetch& F)
{
    const int2 p = rows[row & (kMaxItems - 1)];
    infer_fetch<P>(G, K, p.x, p.y, F);
}

template <int P>
__device__ __forceinline__ void finish_row(float4* vals, int R, int row, const FwdWeights<P>& W,
                                           const Biases& Bz, const InferFetch& F, int g)
{
    const f4 y = mlp_forward_b<P>(W, Bz, infer_combine<P>(F), nullptr, nullptr);
    if (g == 0 && row < R) vals[row] = make_float4(y[0], y[1], y[2], y[3]);
}

// rows[0..R) -> vals[0..R) in 16-row tiles, two fetch buffers in ping-pong.
// Every prefetch is issued unconditionally, so each path reaches the next
// tile's MLP with the same loads outstanding and the wait before it covers
// only the current tile's gathers.
template <int P>
__device__ __forceinline__ void decode_rows(DecLds& L, int R, const InferGrid& G, const FwdWeights<P>& W,
                                            const Biases& Bz, int j, int g)
{
    const int T = (R + 15) >> 4;
    if (T == 0) return;
    const InferLane<P> K(G, g);
    InferFetch fa, fb;
    fetch_row<P>(L.rows, j, G, K, fa);
    for (int t = 0; t < T; t += 2) {
        fetch_row<P>(L.rows, 16 * (t + 1) + j, G, K, fb);
        finish_row<P>(L.vals, R, 16 * t + j, W, Bz, fa, g);
        if (t + 1 >= T) break;
        fetch_row<P>(L.rows, 16 * (t + 2) + j, G, K, fa);
        finish_row<P>(L.vals, R, 16 * (t + 1) + j, W, Bz, fb, g);
    }
    // The last prefetch (issued during the last MLP) is never used: wait for
    // it here, while it is nearly done, rather than where its registers are
    // next written, which may be after the next tile's inputs were requested
    // (memory counters drain in order, so that wait would cover them too).
    asm volatile("" ::"v"(fa.v[0]), "v"(fa.v[1]), "v"(fa.v[2]), "v"(fa.v[3]), "v"(fb.v[0]), "v"(fb.v[1]),
                 "v"(fb.v[2]), "v"(fb.v[3]));
}

__device__ __forceinline__ void write_tile_stats(const FilterArgs& a, int64_t tile, uint64_t act, uint64_t A,
                                                 uint64_t stfmask, bool fits16, const uint64_t B[4], int xmin,
                                                 int ymin, int bbw, int bbh, int n, int unique, int evals,
                                                 bool success, bool cap_ok, bool count_ok, int nA)
{
    ctf_tile_stats S;
    S.active = act;
    S.part = A;
    S.stf = stfmask;
    for (int w = 0; w < 4; ++w) S.mask[w] = fits16 ? B[w] : 0ull;
    S.xmin = xmin;
    S.ymin = ymin;
    S.bbw = bbw;
    S.bbh = bbh;
    S.n = n;
    S.unique = unique;
    S.evals = evals;
    S.flags = (success ? CTF_TILE_OK : 0) | (nA && !cap_ok ? CTF_TILE_CAP : 0) |
              (nA && cap_ok && !count_ok ? CTF_TILE_OVERFLOW : 0) | (nA == 0 ? CTF_TILE_EMPTY : 0);
    for (int r = 0; r < 10; ++r) S.reserved[r] = 0;
    a.tile_stats[tile] = S;
}

// One tile of the decoder-path filter: decisions, row list, MFMA decode,
// gather and outputs.  `f` is the lanes' footprint (already in this
// layer's coordinates); a.out / a.tile_stats / a.stf_xy point at this
// layer's planes.  `after_decode` runs once, right after the tile's (first)
// decode pass: the caller requests the next tile's inputs there, so that no
// wait for the decode's latent loads covers them.
template <int METHOD, int P, bool STATS, bool FB, int FILTER, class AfterDecode>
__device__ __forceinline__ void dec_tile(const FilterArgs& a, const InferGrid& G, const FwdWeights<P>& W,
                                         const Biases& Bz, DecLds& L, int64_t tile, int tx, int ty,
                                         const Footprint& f, FrameCounters& fc, AfterDecode&& after_decode)
{
    constexpr int F = Taps<FILTER>::F, O = Taps<FILTER>::O;
    const int lane = lane_id();
    const int j = lane & 15, g = lane >> 4;
    const int px = tx * kTile + (lane & 7), py = ty * kTile + (lane >> 3);
    const bool in_screen = px < a.sw && py < a.sh;
    const int64_t pix = (int64_t)py * a.sw + px;
    const int ox = f.x0 - O, oy = f.y0 - O;   // upper-left tap of the FxF footprint
    const bool inA = f.active && f.magnify;
    const uint64_t act = ballot(f.active);
    const uint64_t A = ballot(inA);
    const int nA = popc64(A);

    int xmin = 0, ymin = 0, bbw = 0, bbh = 0;
    constexpr bool kCollab = METHOD == CTF_LIST || METHOD == CTF_BOX || METHOD == CTF_MASK;
    if ((kCollab || STATS) && nA > 0) {
        xmin = wave_min(inA ? ox : INT32_MAX);
        ymin = wave_min(inA ? oy : INT32_MAX);
        bbw = wave_max(inA ? ox + F - 1 : INT32_MIN) - xmin + 1;
        bbh = wave_max(inA ? oy + F - 1 : INT32_MIN) - ymin + 1;
    }
    const bool fits16 = nA > 0 && bbw <= 16 && bbh <= 16;

    // ---- 16x16 wave mask B (Mask Sampling; also the exact set when it
    // fits).  Each lane of A marks only its footprint's upper-left texel
    // (mask C, one LDS byte and four ballots); B is C spread over the FxF
    // footprint with 256-bit shifts (rows of 16 do not wrap when the box
    // fits).
    uint64_t B[4] = {0, 0, 0, 0};
    int nmask = 0;
    constexpr bool kNeedMask = METHOD == CTF_MASK || METHOD == CTF_LIST || STATS;
    if (kNeedMask && fits16) {
        reinterpret_cast<uint32_t*>(L.bytes)[lane] = 0u;
        wave_lds_sync();
        if (inA) L.bytes[16 * (oy - ymin) + (ox - xmin)] = 1;
        wave_lds_sync();
        uint64_t C[4];
#pragma unroll
        for (int w = 0; w < 4; ++w) C[w] = ballot(L.bytes[64 * w + lane] != 0);
        footprint_mask_f<F>(C, B);
        nmask = popc64(B[0]) + popc64(B[1]) + popc64(B[2]) + popc64(B[3]);
    }

    const int k = a.max_evals;
    int n = 0;
    bool cap_ok = true, count_ok = true, success = false, sorted = false;
    int unique = nmask;
    if constexpr (METHOD == CTF_BOX) {
        const int64_t area = (int64_t)bbw * bbh;
        n = area > INT32_MAX ? INT32_MAX : (int)area;
        cap_ok = (a.box_w == 0 || bbw <= a.box_w) && (a.box_h == 0 || bbh <= a.box_h);
        count_ok = area <= (int64_t)k * nA;
        success = nA > 0 && cap_ok && count_ok;
    } else if constexpr (METHOD == CTF_MASK) {
        cap_ok = fits16;
        n = fits16 ? nmask : 0;
        count_ok = n <= k * nA;
        success = fits16 && count_ok;
    } else if constexpr (METHOD == CTF_LIST) {
        if (nA > 0 && !fits16) {
            n = dec_list_sorted<F>(L, inA, ox, oy, xmin, ymin);
            sorted = true;
        } else {
            n = nmask;
        }
        unique = n;
        count_ok = n <= k * nA;
        success = nA > 0 && count_ok;
    }
    if constexpr (STATS && METHOD != CTF_LIST) {
        if (nA > 0 && !fits16) unique = dec_list_sorted<F>(L, inA, ox, oy, xmin, ymin);
    }
    if (nA == 0) unique = 0;

    bool exact, draws;
    if constexpr (METHOD == CTF_BILINEAR4) {
        exact = f.active;
        draws = false;
    } else if constexpr (METHOD == CTF_STF1) {
        exact = false;
        draws = f.active;
    } else {
        exact = inA && success;
        draws = f.active && !exact;
    }
    const uint64_t stfmask = ballot(draws);
    const int nstf = popc64(stfmask);
    int2 pick = make_int2(INT32_MIN, INT32_MIN);
    uint32_t h1 = 0, h2 = 0;
    if (draws) {
        stf_hashes(a.seed, a.layer, px, py, h1, h2);
        pick = stf_pick_filter<FILTER>(f, h1, h2);
    }
    const int rank_act = mbcnt(act);

    if constexpr (METHOD == CTF_BILINEAR4 && F == 4) {
        // ---- the full 4x4 filter: 16 taps per active lane do not fit one
        // row list, so the footprint rows are decoded one at a time (4 taps
        // per lane, up to 256 rows) and accumulated as in the gather below
        float4 res = make_float4(0.f, 0.f, 0.f, 0.f);
        const int R = 4 * popc64(act);
        for (int jr = 0; jr < 4; ++jr) {
            if (f.active) {
#pragma unroll
                for (int i = 0; i < 4; ++i) L.rows[4 * rank_act + i] = make_int2(ox + i, oy + jr);
            }
            wave_lds_sync();
            decode_rows<P>(L, R, G, W, Bz, j, g);
            if (jr == 0) after_decode();
            wave_lds_sync();
            if (exact) {
                float wx[4], wy[4];
                taps32<FILTER>(f.s, wx);
                taps32<FILTER>(f.t, wy);
                const int b = 4 * rank_act;
                const float4 r = row4(wx, L.vals[b], L.vals[b + 1], L.vals[b + 2], L.vals[b + 3]);
                res = col_acc(wy[jr], r, res, jr == 0);
            }
            wave_lds_sync();
        }
        if (in_screen) {
            reinterpret_cast<float4*>(a.out)[pix] = res;
            if (a.stf_xy) reinterpret_cast<int2*>(a.stf_xy)[pix] = make_int2(INT32_MIN, INT32_MIN);
        }
        if (STATS && lane == 0 && a.tile_stats)
            write_tile_stats(a, tile, act, A, stfmask, fits16, B, xmin, ymin, bbw, bbh, n, unique, 4 * R, success,
                             cap_ok, count_ok, nA);
        if (act) fc.add(4 * R, popc64(act), nstf, popc64(act & ~A), 4 * ((R + 15) & ~15), false, false);
        return;
    }

    // fallback C / C+ for the lanes of A of a failed wave (fallback.h)
    const bool fallback = FB && !success && nA > 0;
    const uint64_t mdraw = stfmask & ~A;   // minifying draws in a fallback wave
    FallbackPlan fp{};

    // ---- row list: the texels to produce (unique texels first, in the
    // method's order, then one row per fallback draw) and the inverse table
    // of Mask/List
    const int ns = success ? n : 0;
    // List past 16x16: per-lane item indices of the F^2 taps, found before
    // the decode (bilinear: the rank table; bicubic: the keys array, free
    // once the sorted keys sit at the front of the sort buffer)
    uint8_t* const sidx = F == 2 ? L.rank : reinterpret_cast<uint8_t*>(L.keys);
    int R;
    if constexpr (METHOD == CTF_BILINEAR4) {
        R = 4 * popc64(act);
        if (f.active) {
#pragma unroll
            for (int q = 0; q < 4; ++q) L.rows[4 * rank_act + q] = make_int2(f.x0 + (q & 1), f.y0 + (q >> 1));
        }
    } else if (fallback) {
        fp = plan_fallback<FILTER>(L, a.fallback, inA, nA, mbcnt(A), f, pick, pcg_hash(h2), fits16, xmin, ymin);
        R = fp.nprod + popc64(mdraw);
        if (fp.produces) L.rows[fp.slot] = fp.texel;
        if (draws && !inA) L.rows[fp.nprod + mbcnt(mdraw)] = pick;
    } else {
        R = ns + nstf;
        if (success) {
            if (METHOD == CTF_BOX || sorted) {
                const uint64_t* keys = dec_keys<F>(L);
                for (int i = lane; i < ns; i += kWave) {
                    int ex, ey;
                    if (METHOD == CTF_BOX) {
                        ex = xmin + i % bbw;
                        ey = ymin + i / bbw;
                    } else {
                        const uint64_t key = keys[i];
                        ex = xmin + (int)(uint32_t)key;
                        ey = ymin + (int)(key >> 32);
                    }
                    L.rows[i] = make_int2(ex, ey);
                    if (STATS && a.lists) reinterpret_cast<int2*>(a.lists)[(size_t)tile * kMaxItems + i] = make_int2(ex, ey);
                }
            } else {
                // set bit t of B with rank r: row r, and rank[t] = r (h^-1)
                int base = 0;
#pragma unroll
                for (int w = 0; w < 4; ++w) {
                    if ((B[w] >> lane) & 1u) {
                        const int r = base + mbcnt(B[w]);
                        const int t = 64 * w + lane;
                        const int2 c = make_int2(xmin + (t & 15), ymin + (t >> 4));
                        L.rank[t] = (uint8_t)r;
                        L.rows[r] = c;
                        if (STATS && a.lists) reinterpret_cast<int2*>(a.lists)[(size_t)tile * kMaxItems + r] = c;
                    }
                    base += popc64(B[w]);
                }
            }
            if (sorted && inA) {
                const uint64_t* keys = dec_keys<F>(L);
#pragma unroll
                for (int q = 0; q < F * F; ++q) {
                    const uint64_t key = ((uint64_t)(uint32_t)(oy + q / F - ymin) << 32) |
                                         (uint32_t)(ox + q % F - xmin);
                    sidx[F * F * lane + q] = (uint8_t)dec_list_find(keys, n, key);
                }
            }
        }
        if (draws) L.rows[ns + mbcnt(stfmask)] = pick;
    }
    // the debug draws are known now; write them before the decode so the
    // draw is not kept live across it
    if (in_screen && a.stf_xy)
        reinterpret_cast<int2*>(a.stf_xy)[pix] = draws ? pick : make_int2(INT32_MIN, INT32_MIN);
    // where this lane's taps sit: tap (i, j) has item index gi + i + gd j
    // (Box: directly; Mask and List: through the table at gi)
    int gi = 0, gd = 0;
    if constexpr (METHOD == CTF_BOX) {
        gi = (ox - xmin) + (oy - ymin) * bbw;
        gd = bbw;
    } else if constexpr (METHOD == CTF_LIST || METHOD == CTF_MASK) {
        gi = sorted ? F * F * lane : 16 * (oy - ymin) + (ox - xmin);
        gd = sorted ? F : 16;
    }
    const int draw_row = ns + mbcnt(stfmask);
    wave_lds_sync();

    // ---- decode the rows, 16 per MFMA tile; the latent gathers of the
    // next tile are in flight during the MLP of the current one
    decode_rows<P>(L, R, G, W, Bz, j, g);
    after_decode();
    wave_lds_sync();

    // ---- gather and weight
    float4 res = make_float4(0.f, 0.f, 0.f, 0.f);
    if constexpr (METHOD == CTF_BILINEAR4) {
        if (exact) {
            const int b = 4 * rank_act;
            res = bilerp(f.s, f.t, L.vals[b], L.vals[b + 1], L.vals[b + 2], L.vals[b + 3]);
        }
    } else if (fallback) {
        if (draws && !inA) res = L.vals[fp.nprod + mbcnt(mdraw)];
        if (inA) res = fallback_color<FILTER>(L, fp, f, pick, xmin, ymin);
    } else {
        if (draws) res = L.vals[draw_row];
        if (kCollab && exact) {
            const uint8_t* tab = sorted ? sidx : L.rank;
            auto item = [&](int i, int jj) -> int {
                const int t = gi + i + gd * jj;
                if constexpr (METHOD == CTF_BOX) return t;
                else return tab[t];
            };
            if constexpr (F == 2) {
                res = bilerp(f.s, f.t, L.vals[item(0, 0)], L.vals[item(1, 0)], L.vals[item(0, 1)],
                             L.vals[item(1, 1)]);
            } else {
                float wx[4], wy[4];
                taps32<FILTER>(f.s, wx);
                taps32<FILTER>(f.t, wy);
#pragma unroll
                for (int jj = 0; jj < 4; ++jj) {
                    const float4 r = row4(wx, L.vals[item(0, jj)], L.vals[item(1, jj)], L.vals[item(2, jj)],
                                          L.vals[item(3, jj)]);
                    res = col_acc(wy[jj], r, res, jj == 0);
                }
            }
        }
    }
    if (in_screen) reinterpret_cast<float4*>(a.out)[pix] = res;
    if (STATS && lane == 0 && a.tile_stats)
        write_tile_stats(a, tile, act, A, stfmask, fits16, B, xmin, ymin, bbw, bbh, n, unique, R, success, cap_ok,
                         count_ok, nA);
    if (act) fc.add(R, popc64(act), nstf, popc64(act & ~A), (R + 15) & ~15, kCollab && success,
                    kCollab && nA && !success);
    wave_lds_sync();  // the next tile reuses this wave's LDS slice
}

// Pixel offset of this lane inside its tile, (lane / 8) sw + lane % 8: a
// tile's pixel addresses are a scalar base plus this per-lane constant.
__device__ __forceinline__ uint32_t lane_pixel(const FilterArgs& a)
{
    const int lane = lane_id();
    uint32_t lp = (uint32_t)(lane >> 3) * (uint32_t)a.sw + (uint32_t)(lane & 7);
    // opaque to the optimizer, so that an access stays "scalar base + this
    // 32-bit offset" (an SGPR-based global access) rather than a hoisted
    // 64-bit per-lane pointer
    asm volatile("" : "+v"(lp));
    return lp;
}

// First pixel of tile (tx, ty) and whether all of its pixels are on screen
// (both wave-uniform).
__device__ __forceinline__ int64_t tile_pixel0(const FilterArgs& a, int tx, int ty)
{
    return (int64_t)ty * kTile * a.sw + (int64_t)tx * kTile;
}

__device__ __forceinline__ bool tile_interior(const FilterArgs& a, int tx, int ty)
{
    return tx * kTile + kTile <= a.sw && ty * kTile + kTile <= a.sh;
}

__device__ __forceinline__ bool lane_on_screen(const FilterArgs& a, int tx, int ty)
{
    if (tile_interior(a, tx, ty)) return true;
    const int lane = lane_id();
    return tx * kTile + (lane & 7) < a.sw && ty * kTile + (lane >> 3) < a.sh;
}

// XCD-aware share of the tiles for this wave.  Workgroups go round-robin
// over the 8 XCDs, and XCD x takes the strips of kStripRows tile rows whose
// index is x mod 8 (neighbouring tile rows, which share latent cells, stay
// in one XCD's L2).  Contiguous eighths of the screen balance badly: the
// texels a tile decodes vary down a frame (a minifying region decodes one
// per pixel), so on a 3840x2160 frame of four planes the costliest eighth
// decoded twice the rows of the cheapest and its XCD finished last.  The
// XCD's waves take its tiles in turn (the launch makes the grid a multiple
// of 8).
constexpr int kStripLog = 1;   // strips of 2 tile rows
constexpr int kStripRows = 1 << kStripLog;

struct Band {
    int64_t end;   // every tile index is below it
    int lw, nw, xcd;
    __device__ Band(int64_t ntiles, int wid)
    {
        xcd = blockIdx.x & 7;
        lw = (int)(blockIdx.x >> 3) * kDecWaves + wid;
        nw = (int)(gridDim.x >> 3) * kDecWaves;
        end = ntiles;
    }
};

// A wave's walk over its XCD's tiles: the XCD's tile rows in order (row r of
// the XCD is tile row ((r / kStripRows) * 8 + xcd) * kStripRows + r mod
// kStripRows), each left to right, every nw-th tile from lw.  Past the last
// one, tile reads INT64_MAX.
struct StripWalk {
    int64_t tile;
    int tx, ty;
    int row, xoff, dtx, drow, tiles_x, tiles_y;
    __device__ __forceinline__ StripWalk(const Band& b, int64_t ntiles, int tiles_x_)
    {
        tiles_x = tiles_x_;
        tiles_y = (int)(ntiles / tiles_x_);
        xoff = b.xcd << kStripLog;
        row = b.lw / tiles_x_;
        tx = b.lw - row * tiles_x_;
        drow = b.nw / tiles_x_;
        dtx = b.nw - drow * tiles_x_;
        place();
    }
    __device__ __forceinline__ void place()
    {
        ty = (((row >> kStripLog) << (3 + kStripLog)) + xoff) | (row & (kStripRows - 1));
        tile = ty < tiles_y ? (int64_t)ty * tiles_x + tx : INT64_MAX;
    }
    __device__ __forceinline__ void advance()
    {
        tx += dtx;
        row += drow;
        if (tx >= tiles_x) {
            tx -= tiles_x;
            ++row;
        }
        place();
    }
};

// Workgroups a launch needs so that no wave visits more than
// kMaxWaveTileVisits tiles over its `layers` walks: an XCD's share of a
// frame's tiles is at most an eighth plus one strip.
inline int64_t dec_min_blocks(int64_t ntiles, int tiles_x, int layers)
{
    return counter_min_blocks((ntiles + (int64_t)8 * kStripRows * tiles_x) * layers, kDecWaves);
}

// Inputs of a tile for this lane, NaN (inactive) outside the band or screen
// (per-lane 64-bit addresses: the per-tile kernels run faster with these
// than with load_tile_px_s, measured).
__device__ __forceinline__ void load_tile_px(const FilterArgs& a, const StripWalk& t, int64_t band_e, float2& uv,
                                             float4& d)
{
    const int lane = lane_id();
    uv = make_float2(__builtin_nanf(""), 0.f);
    d = make_float4(0.f, 0.f, 0.f, 0.f);
    if (t.tile >= band_e) return;
    const int px = t.tx * kTile + (lane & 7), py = t.ty * kTile + (lane >> 3);
    if (px < a.sw && py < a.sh) {
        const int64_t q = (int64_t)py * a.sw + px;
        uv = reinterpret_cast<const float2*>(a.uv)[q];
        d = reinterpret_cast<const float4*>(a.duv)[q];
    }
}

// The same with a scalar tile base plus the lane's offset (the batched
// kernel).
__device__ __forceinline__ void load_tile_px_s(const FilterArgs& a, const StripWalk& t, int64_t band_e, float2& uv,
                                               float4& d)
{
    uv = make_float2(__builtin_nanf(""), 0.f);
    d = make_float4(0.f, 0.f, 0.f, 0.f);
    if (t.tile >= band_e) return;
    if (lane_on_screen(a, t.tx, t.ty)) {
        const int64_t p0 = tile_pixel0(a, t.tx, t.ty);
        const uint32_t lp = lane_pixel(a);
        const char* const ub = reinterpret_cast<const char*>(reinterpret_cast<const float2*>(a.uv) + p0);
        const char* const db = reinterpret_cast<const char*>(reinterpret_cast<const float4*>(a.duv) + p0);
        uv = *reinterpret_cast<const float2*>(ub + lp * 8u);
        d = *reinterpret_cast<const float4*>(db + lp * 16u);
    }
}

// Wait for the first tile's inputs before entering a tile loop.  The loop
// loads each next tile's inputs one tile ahead and copies them at the top of
// the next iteration; without this, the loads issued before the loop are
// still pending into the registers the first iteration reads, and the
// memory-counter wait placed at the loop head (counters drain in order)
// would also wait for the prefetch issued in every later iteration.
__device__ __forceinline__ void settle(const float2& uv, const float4& d)
{
    asm volatile("" ::"v"(uv.x), "v"(uv.y), "v"(d.x), "v"(d.y), "v"(d.z), "v"(d.w));
}

// Waves per SIMD the register budget of the single-layer kernel is sized
// for: the collaborative methods and the 4x4 full filter need the bound of
// three to fit in 168 registers; the others fit three anyway and keep the
// compiler's schedule.
template <int METHOD, int FILTER>
constexpr int dec_waves_per_simd()
{
    return METHOD == CTF_LIST || METHOD == CTF_BOX || METHOD == CTF_MASK ||
                   (METHOD == CTF_BILINEAR4 && FILTER != CTF_FILTER_BILINEAR)
               ? 3
               : 2;
}

template <int METHOD, int P, bool STATS, bool FB, int FILTER>
__global__ __launch_bounds__(64 * kDecWaves, (dec_waves_per_simd<METHOD, FILTER>())) void k_filter_dec(
    FilterArgs a, DevDecoderWeights D)
{
    __shared__ DecLds lds_all[kDecWaves];
    const int wid = wave_in_block();
    const int lane = lane_id();
    DecLds& L = lds_all[wid];
    FwdWeights<P> W;
    W.load(D.w, lane);
    Biases Bz;
    Bz.load(D.bias, lane);
    const float tex_w = (float)D.grid.tex_w;
    const Band band(a.ntiles, wid);
    FrameCounters fc;

    // the inputs of the wave's next tile are loaded one tile ahead
    float2 uv_next;
    float4 d_next;
    StripWalk next(band, a.ntiles, a.tiles_x);
    load_tile_px(a, next, band.end, uv_next, d_next);
    settle(uv_next, d_next);
    while (next.tile < band.end) {
        const StripWalk cur = next;
        const float2 uv = uv_next;
        const float4 d = d_next;
        const Footprint f = footprint(uv.x, uv.y, d, tex_w, tex_w);
        dec_tile<METHOD, P, STATS, FB, FILTER>(a, D.grid, W, Bz, L, cur.tile, cur.tx, cur.ty, f, fc, [&] {
            next.advance();
            load_tile_px(a, next, band.end, uv_next, d_next);
        });
    }
    if (lane == 0 && a.frame_stats) fc.flush(a.frame_stats);
}

// ---------------------------------------------------------------------------
// Batched decode (bilinear filter, no C / C+ fallback).  A wave plans each
// tile into a staging row list, then appends the rows to the decode batch;
// the batch of up to two tiles (at most 256 rows) is decoded in one pass, so
// a tile's few rows share the pass's start-up and its partial last MFMA
// tile with its neighbour.  A planned tile's per-lane state waits in LDS
// until its gather, so no two tiles' state is live in registers.
// ---------------------------------------------------------------------------

struct LaneState {
    float s, t;       // footprint position
    uint32_t idx;     // gi | gd << 16: tap (i, j) at item gi + i + gd j (via the rank table for Mask/List)
    uint32_t misc;    // draw_row | exact << 8 | draws << 9 | in_screen << 10
};

struct BatchLds {
    DecLds L;                   // vals, rows (the batch), keys (sort keys, then the staging rows), rank (slot 0), bytes
    uint8_t rank1[256];         // rank table of slot 1
    LaneState st[2][kWave];     // per-lane state by slot
};

struct Pending {
    int tx, ty;
    int base;                   // first row of the tile in the batch
};

// Plan one tile: decisions, staging rows (L.keys as int2), the rank table
// and per-lane state of `slot`, debug outputs, tile record and counters.
// Returns the tile's row count.
// The rows go behind the batch's rows (from row `base`) when they fit there,
// else to the staging area (L.keys) for the caller to move after a flush.
template <int METHOD, bool STATS>
__device__ __forceinline__ int plan_tile(const FilterArgs& a, BatchLds& BL, int slot, int base, int64_t tile, int tx,
                                         int ty, const Footprint& f, FrameCounters& fc)
{
    DecLds& L = BL.L;
    int2* const stage = reinterpret_cast<int2*>(L.keys);
    uint8_t* const rank = slot ? BL.rank1 : L.rank;
    const int lane = lane_id();
    const int px = tx * kTile + (lane & 7), py = ty * kTile + (lane >> 3);
    const bool in_screen = lane_on_screen(a, tx, ty);
    const bool inA = f.active && f.magnify;
    const uint64_t act = ballot(f.active);
    const uint64_t A = ballot(inA);
    const int nA = popc64(A);

    int xmin = 0, ymin = 0, bbw = 0, bbh = 0;
    constexpr bool kCollab = METHOD == CTF_LIST || METHOD == CTF_BOX || METHOD == CTF_MASK;
    // Mask and List only need a 16x16 window that holds every footprint of
    // A: try the one centred on a lane of A (lane 36 when it is in A) before
    // reducing the exact box.  Bit positions are relative to the window's
    // corner; the texels, their order and every decision are the same.
    bool window = false;
    if constexpr ((METHOD == CTF_LIST || METHOD == CTF_MASK) && !STATS) {
        if (nA > 0) {
            const int rl = ((A >> 36) & 1ull) ? 36 : (int)__builtin_ctzll(A);
            const int ox = __builtin_amdgcn_readlane(f.x0, rl) - 7, oy = __builtin_amdgcn_readlane(f.y0, rl) - 7;
            const bool outside =
                inA && ((uint32_t)f.x0 - (uint32_t)ox > 14u || (uint32_t)f.y0 - (uint32_t)oy > 14u);
            if (ballot(outside) == 0) {
                window = true;
                xmin = ox;
                ymin = oy;
            }
        }
    }
    if ((kCollab || STATS) && nA > 0 && !window) {
        xmin = wave_min(inA ? f.x0 : INT32_MAX);
        ymin = wave_min(inA ? f.y0 : INT32_MAX);
        bbw = wave_max(inA ? f.x0 + 1 : INT32_MIN) - xmin + 1;
        bbh = wave_max(inA ? f.y0 + 1 : INT32_MIN) - ymin + 1;
    }
    const bool fits16 = window || (nA > 0 && bbw <= 16 && bbh <= 16);

    uint64_t B[4] = {0, 0, 0, 0};
    int nmask = 0;
    constexpr bool kNeedMask = METHOD == CTF_MASK || METHOD == CTF_LIST || STATS;
    if (kNeedMask && fits16) {
        reinterpret_cast<uint32_t*>(L.bytes)[lane] = 0u;
        wave_lds_sync();
        if (inA) L.bytes[16 * (f.y0 - ymin) + (f.x0 - xmin)] = 1;
        wave_lds_sync();
        uint64_t C[4];
#pragma unroll
        for (int w = 0; w < 4; ++w) C[w] = ballot(L.bytes[64 * w + lane] != 0);
        footprint_mask(C, B);
        nmask = popc64(B[0]) + popc64(B[1]) + popc64(B[2]) + popc64(B[3]);
    }

    const int k = a.max_evals;
    int n = 0;
    bool cap_ok = true, count_ok = true, success = false, sorted = false;
    int unique = nmask;
    if constexpr (METHOD == CTF_BOX) {
        const int64_t area = (int64_t)bbw * bbh;
        n = area > INT32_MAX ? INT32_MAX : (int)area;
        cap_ok = (a.box_w == 0 || bbw <= a.box_w) && (a.box_h == 0 || bbh <= a.box_h);
        count_ok = area <= (int64_t)k * nA;
        success = nA > 0 && cap_ok && count_ok;
    } else if constexpr (METHOD == CTF_MASK) {
        cap_ok = fits16;
        n = fits16 ? nmask : 0;
        count_ok = n <= k * nA;
        success = fits16 && count_ok;
    } else if constexpr (METHOD == CTF_LIST) {
        if (nA > 0 && !fits16) {
            n = dec_list_sorted<2>(L, inA, f.x0, f.y0, xmin, ymin);
            sorted = true;
        } else {
            n = nmask;
        }
        unique = n;
        count_ok = n <= k * nA;
        success = nA > 0 && count_ok;
    }
    if constexpr (STATS && METHOD != CTF_LIST) {
        if (nA > 0 && !fits16) unique = dec_list_sorted<2>(L, inA, f.x0, f.y0, xmin, ymin);
    }
    if (nA == 0) unique = 0;

    bool exact, draws;
    if constexpr (METHOD == CTF_BILINEAR4) {
        exact = f.active;
        draws = false;
    } else if constexpr (METHOD == CTF_STF1) {
        exact = false;
        draws = f.active;
    } else {
        exact = inA && success;
        draws = f.active && !exact;
    }
    const uint64_t stfmask = ballot(draws);
    const int nstf = popc64(stfmask);
    int2 pick = make_int2(INT32_MIN, INT32_MIN);
    if (draws) {
        uint32_t h1, h2;
        stf_hashes(a.seed, a.layer, px, py, h1, h2);
        pick = stf_pick_h(f, h1, h2);
    }

    // rows (behind the batch or in the staging area) and the inverse table
    // of Mask/List.  Only the first tap of each footprint row is looked up
    // at gather time: in a row-major list the texel right of a footprint
    // texel is the next item.
    const int rank_act = mbcnt(act);
    const int ns = success ? n : 0;
    int R;
    if constexpr (METHOD == CTF_BILINEAR4) {
        R = 4 * popc64(act);
        int2* const dst = base + R <= kMaxItems ? L.rows + base : stage;
        if (f.active) {
#pragma unroll
            for (int q = 0; q < 4; ++q) dst[4 * rank_act + q] = make_int2(f.x0 + (q & 1), f.y0 + (q >> 1));
        }
    } else {
        R = ns + nstf;
        int2* const dst = base + R <= kMaxItems ? L.rows + base : stage;
        if (success) {
            if (sorted) {
                // the lane's item indices first (they read the sorted keys);
                // in place when the rows go to the staging area
                if (inA) {
#pragma unroll
                    for (int q = 0; q < 4; q += 2) {
                        const uint64_t key = ((uint64_t)(uint32_t)(f.y0 + (q >> 1) - ymin) << 32) |
                                             (uint32_t)(f.x0 - xmin);
                        rank[4 * lane + q] = (uint8_t)dec_list_find(L.keys, n, key);
                    }
                }
                wave_lds_sync();
            }
            if (METHOD == CTF_BOX || sorted) {
                for (int i = lane; i < ns; i += kWave) {
                    int ex, ey;
                    if (METHOD == CTF_BOX) {
                        ex = xmin + i % bbw;
                        ey = ymin + i / bbw;
                    } else {
                        const uint64_t key = L.keys[i];
                        ex = xmin + (int)(uint32_t)key;
                        ey = ymin + (int)(key >> 32);
                    }
                    dst[i] = make_int2(ex, ey);
                    if (STATS && a.lists) reinterpret_cast<int2*>(a.lists)[(size_t)tile * kMaxItems + i] = make_int2(ex, ey);
                }
            } else {
                // bit `lane` of word w is position 64 w + lane of the window:
                // column lane % 16, row 4 w + lane / 16
                const int cx = xmin + (lane & 15);
                int cy = ymin + (lane >> 4), first = 0;
#pragma unroll
                for (int w = 0; w < 4; ++w) {
                    if ((B[w] >> lane) & 1u) {
                        const int r = first + mbcnt(B[w]);
                        rank[64 * w + lane] = (uint8_t)r;
                        dst[r] = make_int2(cx, cy);
                        if (STATS && a.lists) reinterpret_cast<int2*>(a.lists)[(size_t)tile * kMaxItems + r] = make_int2(cx, cy);
                    }
                    first += popc64(B[w]);
                    cy += 4;
                }
            }
        }
        if (draws) dst[ns + mbcnt(stfmask)] = pick;
    }
    if (in_screen && a.stf_xy)
        reinterpret_cast<int2*>(a.stf_xy)[tile_pixel0(a, tx, ty) + lane_pixel(a)] =
            draws ? pick : make_int2(INT32_MIN, INT32_MIN);
    int gi = 0, gd = 0;
    if constexpr (METHOD == CTF_BILINEAR4) {
        gi = 4 * rank_act;
        gd = 2;
    } else if constexpr (METHOD == CTF_BOX) {
        gi = (f.x0 - xmin) + (f.y0 - ymin) * bbw;
        gd = bbw;
    } else if constexpr (METHOD == CTF_LIST || METHOD == CTF_MASK) {
        gi = sorted ? 4 * lane : 16 * (f.y0 - ymin) + (f.x0 - xmin);
        gd = sorted ? 2 : 16;
    }
    LaneState ls;
    ls.s = f.s;
    ls.t = f.t;
    ls.idx = (uint32_t)(gi & 0xffff) | ((uint32_t)(gd & 0xffff) << 16);
    ls.misc = (uint32_t)((ns + mbcnt(stfmask)) & 0xff) | (exact ? 1u << 8 : 0u) | (draws ? 1u << 9 : 0u) |
              (in_screen ? 1u << 10 : 0u);
    BL.st[slot][lane] = ls;
    if (STATS && lane == 0 && a.tile_stats)
        write_tile_stats(a, tile, act, A, stfmask, fits16, B, xmin, ymin, bbw, bbh, n, unique, R, success, cap_ok,
                         count_ok, nA);
    if (act) fc.add(R, popc64(act), nstf, popc64(act & ~A), 0, kCollab && success, kCollab && nA && !success);
    return R;
}

// Gather and weight a decoded tile from its per-lane state.
template <int METHOD>
__device__ __forceinline__ void gather_tile(const FilterArgs& a, BatchLds& BL, int slot, const Pending& pd)
{
    const int lane = lane_id();
    const LaneState ls = BL.st[slot][lane];
    const uint8_t* const rank = slot ? BL.rank1 : BL.L.rank;
    const float4* const vals = BL.L.vals + pd.base;
    const int gi = (int)(ls.idx & 0xffff), gd = (int)(ls.idx >> 16);
    const bool exact = (ls.misc >> 8) & 1u, draws = (ls.misc >> 9) & 1u, in_screen = (ls.misc >> 10) & 1u;
    float4 res = make_float4(0.f, 0.f, 0.f, 0.f);
    if (draws) res = vals[ls.misc & 0xff];
    if (exact) {
        // each footprint row is two consecutive items
        int i0 = gi, i2 = gi + gd;
        if constexpr (METHOD == CTF_LIST || METHOD == CTF_MASK) {
            i0 = rank[i0];
            i2 = rank[i2];
        }
        res = bilerp(ls.s, ls.t, vals[i0], vals[i0 + 1], vals[i2], vals[i2 + 1]);
    }
    if (in_screen) {
        char* const ob = reinterpret_cast<char*>(reinterpret_cast<float4*>(a.out) + tile_pixel0(a, pd.tx, pd.ty));
        *reinterpret_cast<float4*>(ob + lane_pixel(a) * 16u) = res;
    }
}

// The batch of planned tiles of one wave (slots 0 and 1, named so that no
// private array is indexed at run time).
struct Batch {
    Pending p0{}, p1{};
    int npend = 0, rows = 0;
};

// Decode the batch and gather its tiles in slot order.
template <int METHOD, int P>
__device__ __forceinline__ void batch_flush(const FilterArgs& a, BatchLds& BL, Batch& bt, const InferGrid& G,
                                            const FwdWeights<P>& W, const Biases& Bz, FrameCounters& fc)
{
    const int lane = lane_id();
    wave_lds_sync();
    decode_rows<P>(BL.L, bt.rows, G, W, Bz, lane & 15, lane >> 4);
    wave_lds_sync();
    if (bt.npend >= 1) gather_tile<METHOD>(a, BL, 0, bt.p0);
    if (bt.npend == 2) gather_tile<METHOD>(a, BL, 1, bt.p1);
    fc.rows += (uint32_t)((bt.rows + 15) & ~15);
    bt.npend = 0;
    bt.rows = 0;
    wave_lds_sync();
}

// Plan a tile and append its rows to the batch (decoding the batch first
// when the rows do not fit behind it).  The caller decodes a full batch (two
// tiles) before calling.
template <int METHOD, int P, bool STATS>
__device__ __forceinline__ void batch_add(const FilterArgs& a, BatchLds& BL, Batch& bt, const InferGrid& G,
                                          const FwdWeights<P>& W, const Biases& Bz, FrameCounters& fc,
                                          const StripWalk& cur, const Footprint& f)
{
    const int lane = lane_id();
    const int R = plan_tile<METHOD, STATS>(a, BL, bt.npend, bt.rows, cur.tile, cur.tx, cur.ty, f, fc);
    if (bt.rows + R > kMaxItems) {
        // planned into slot 1 with its rows staged: decode slot 0, then move
        // the state, the table and the rows
        batch_flush<METHOD, P>(a, BL, bt, G, W, Bz, fc);
        BL.st[0][lane] = BL.st[1][lane];
        reinterpret_cast<uint32_t*>(BL.L.rank)[lane] = reinterpret_cast<const uint32_t*>(BL.rank1)[lane];
        const int2* stage = reinterpret_cast<const int2*>(BL.L.keys);
        for (int i = lane; i < R; i += kWave) BL.L.rows[i] = stage[i];
    }
    wave_lds_sync();   // the next plan rewrites the keys
    Pending& pd = bt.npend ? bt.p1 : bt.p0;
    pd.tx = cur.tx;
    pd.ty = cur.ty;
    pd.base = bt.rows;
    ++bt.npend;
    bt.rows += R;
}

template <int METHOD, int P, bool STATS>
__global__ __launch_bounds__(64 * kDecWaves, 3) void k_filter_dec_batch(FilterArgs a, DevDecoderWeights D)
{
    __shared__ BatchLds lds_all[kDecWaves];
    const int wid = wave_in_block();
    const int lane = lane_id();
    BatchLds& BL = lds_all[wid];
    FwdWeights<P> W;
    W.load(D.w, lane);
    Biases Bz;
    Bz.load(D.bias, lane);
    const float tex_w = (float)D.grid.tex_w;
    const Band band(a.ntiles, wid);
    FrameCounters fc;
    Batch bt;
    float2 uv_next;
    float4 d_next;
    StripWalk next(band, a.ntiles, a.tiles_x);
    load_tile_px_s(a, next, band.end, uv_next, d_next);
    settle(uv_next, d_next);
    while (next.tile < band.end) {
        const StripWalk cur = next;
        const float2 uv = uv_next;
        const float4 d = d_next;
        // decode a full batch first, then request the next tile's inputs:
        // their latency is hidden by this tile's planning and the next
        // iteration's decode, and no wait inside the decode covers them
        if (bt.npend == 2) batch_flush<METHOD, P>(a, BL, bt, D.grid, W, Bz, fc);
        next.advance();
        load_tile_px_s(a, next, band.end, uv_next, d_next);
        const Footprint f = footprint(uv.x, uv.y, d, tex_w, tex_w);
        batch_add<METHOD, P, STATS>(a, BL, bt, D.grid, W, Bz, fc, cur, f);
    }
    if (bt.npend) batch_flush<METHOD, P>(a, BL, bt, D.grid, W, Bz, fc);
    if (lane == 0 && a.frame_stats) fc.flush(a.frame_stats);
}

inline int device_cus()
{
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    return cus > 0 ? cus : 256;
}

// Persistent grid: as many workgroups as fit on the device at once (from the
// kernel's register and LDS use), a multiple of the 8 XCDs.
template <typename K>
int64_t resident_blocks(K kernel, int threads, int64_t work_blocks, int64_t min_blocks)
{
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, 0) != hipSuccess || per_cu < 1)
        per_cu = 1;
    int64_t blocks = (int64_t)device_cus() * per_cu;
    if (blocks < min_blocks) blocks = min_blocks;
    if (blocks > work_blocks) blocks = work_blocks;
    return (blocks + 7) / 8 * 8;
}

constexpr bool collaborative(int m) { return m == CTF_LIST || m == CTF_BOX || m == CTF_MASK; }

// Instantiation for the call's statistics and fallback flags; waves of a
// collaborative method carry the C / C+ code only when it is asked for, so
// the common path keeps its register budget.
template <int METHOD, int P, template <int, int, bool, bool> class Go, class... Args>
hipError_t dispatch_flags(const FilterArgs& a, Args&&... args)
{
    // the instantiation with statistics also writes the texel lists; the
    // plain one writes the per-pixel draws only
    const bool st = a.tile_stats != nullptr || a.lists != nullptr;
    if constexpr (collaborative(METHOD)) {
        if (a.fallback != CTF_FB_STF1)
            return st ? Go<METHOD, P, true, true>::run(a, args...) : Go<METHOD, P, false, true>::run(a, args...);
    }
    return st ? Go<METHOD, P, true, false>::run(a, args...) : Go<METHOD, P, false, false>::run(a, args...);
}

template <int FILTER>
struct GoFilter {
    template <int METHOD, int P, bool STATS, bool FB>
    struct Go {
        static hipError_t run(const FilterArgs& a, const DevDecoderWeights& d, hipStream_t s)
        {
            const int64_t work = (a.ntiles + kDecWaves - 1) / kDecWaves;
            const int64_t least = dec_min_blocks(a.ntiles, a.tiles_x, 1);
            if constexpr (FILTER == CTF_FILTER_BILINEAR && !FB && METHOD != CTF_BILINEAR4) {
                // (the 4-tap filter's full tiles of 256 rows never share a batch)
                auto k = k_filter_dec_batch<METHOD, P, STATS>;
                const int64_t blocks = resident_blocks(k, 64 * kDecWaves, work, least);
                hipLaunchKernelGGL(k, dim3((unsigned)blocks), dim3(64 * kDecWaves), 0, s, a, d);
            } else {
                auto k = k_filter_dec<METHOD, P, STATS, FB, FILTER>;
                const int64_t blocks = resident_blocks(k, 64 * kDecWaves, work, least);
                hipLaunchKernelGGL(k, dim3((unsigned)blocks), dim3(64 * kDecWaves), 0, s, a, d);
            }
            return hipGetLastError();
        }
    };
};

template <int P, int FILTER>
hipError_t launch_dec_p(const FilterArgs& a, const DevDecoderWeights& d, hipStream_t s)
{
    switch (a.method) {
    case CTF_BILINEAR4: return dispatch_flags<CTF_BILINEAR4, P, GoFilter<FILTER>::template Go>(a, d, s);
    case CTF_STF1: return dispatch_flags<CTF_STF1, P, GoFilter<FILTER>::template Go>(a, d, s);
    case CTF_LIST: return dispatch_flags<CTF_LIST, P, GoFilter<FILTER>::template Go>(a, d, s);
    case CTF_BOX: return dispatch_flags<CTF_BOX, P, GoFilter<FILTER>::template Go>(a, d, s);
    case CTF_MASK: return dispatch_flags<CTF_MASK, P, GoFilter<FILTER>::template Go>(a, d, s);
    default: return hipErrorInvalidValue;
    }
}

// Several material layers in one launch: layer l samples its own decoder at
// uv_l = M_l uv (derivatives alike).  Layers are the outer loop so that one
// layer's latent grids stay resident in the L2 while its tiles are walked;
// each wave reloads the MLP weights once per layer.
constexpr int kMaxLayers = 8;

struct LayerSet {
    DevDecoderWeights dec[kMaxLayers];
    float xf[kMaxLayers][4];   // row-major 2x2
    int n;
};

template <int METHOD, int P, bool STATS, bool FB, int FILTER>
__global__ __launch_bounds__(64 * kDecWaves, (dec_waves_per_simd<METHOD, FILTER>())) void
k_filter_layers(FilterArgs a, LayerSet LS)
{
    __shared__ DecLds lds_all[kDecWaves];
    const int wid = wave_in_block();
    const int lane = lane_id();
    DecLds& L = lds_all[wid];
    const Band band(a.ntiles, wid);
    const int64_t npix = (int64_t)a.sw * a.sh;
    FrameCounters fc;
    for (int l = 0; l < LS.n; ++l) {
        const DevDecoderWeights& D = LS.dec[l];
        FwdWeights<P> W;
        W.load(D.w, lane);
        Biases Bz;
        Bz.load(D.bias, lane);
        const float tex_w = (float)D.grid.tex_w;
        const float m00 = LS.xf[l][0], m01 = LS.xf[l][1], m10 = LS.xf[l][2], m11 = LS.xf[l][3];
        FilterArgs al = a;
        al.out = a.out + (size_t)l * npix * 4;
        al.tile_stats = a.tile_stats ? a.tile_stats + (size_t)l * a.ntiles : nullptr;
        al.stf_xy = a.stf_xy ? a.stf_xy + (size_t)l * npix * 2 : nullptr;
        al.lists = nullptr;
        al.layer = (uint32_t)l;
        float2 uv_next;
        float4 d_next;
        StripWalk next(band, a.ntiles, a.tiles_x);
        load_tile_px(a, next, band.end, uv_next, d_next);
        settle(uv_next, d_next);
        while (next.tile < band.end) {
            const StripWalk cur = next;
            const float2 uv = uv_next;
            const float4 d = d_next;
            // layer coordinates, float32: u' = fma(m01, v, m00 u), v' = fma(m11, v, m10 u)
            const float lu = __builtin_fmaf(m01, uv.y, m00 * uv.x), lv = __builtin_fmaf(m11, uv.y, m10 * uv.x);
            const float4 ld = make_float4(__builtin_fmaf(m01, d.y, m00 * d.x), __builtin_fmaf(m11, d.y, m10 * d.x),
                                          __builtin_fmaf(m01, d.w, m00 * d.z), __builtin_fmaf(m11, d.w, m10 * d.z));
            const Footprint f = footprint(lu, lv, ld, tex_w, tex_w);
            dec_tile<METHOD, P, STATS, FB, FILTER>(al, D.grid, W, Bz, L, cur.tile, cur.tx, cur.ty, f, fc, [&] {
                next.advance();
                load_tile_px(a, next, band.end, uv_next, d_next);
            });
        }
    }
    if (lane == 0 && a.frame_stats) fc.flush(a.frame_stats);
}


template <int FILTER>
struct GoLayers {
    template <int METHOD, int P, bool STATS, bool FB>
    struct Go {
        static hipError_t run(const FilterArgs& a, const LayerSet& LS, hipStream_t s)
        {
            const int64_t work = (a.ntiles + kDecWaves - 1) / kDecWaves;
            auto k = k_filter_layers<METHOD, P, STATS, FB, FILTER>;
            const int64_t blocks =
                resident_blocks(k, 64 * kDecWaves, work, dec_min_blocks(a.ntiles, a.tiles_x, LS.n));
            hipLaunchKernelGGL(k, dim3((unsigned)blocks), dim3(64 * kDecWaves), 0, s, a, LS);
            return hipGetLastError();
        }
    };
};

template <int P, int FILTER>
hipError_t launch_layers_p(const FilterArgs& a, const LayerSet& LS, hipStream_t s)
{
    switch (a.method) {
    case CTF_BILINEAR4: return dispatch_flags<CTF_BILINEAR4, P, GoLayers<FILTER>::template Go>(a, LS, s);
    case CTF_STF1: return dispatch_flags<CTF_STF1, P, GoLayers<FILTER>::template Go>(a, LS, s);
    case CTF_LIST: return dispatch_flags<CTF_LIST, P, GoLayers<FILTER>::template Go>(a, LS, s);
    case CTF_BOX: return dispatch_flags<CTF_BOX, P, GoLayers<FILTER>::template Go>(a, LS, s);
    case CTF_MASK: return dispatch_flags<CTF_MASK, P, GoLayers<FILTER>::template Go>(a, LS, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace dec

}  // namespace ctf
