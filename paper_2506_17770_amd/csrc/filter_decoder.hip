// filter_decoder.hip -- collaborative filtering with the learned texel producer.
//
// Same decisions as the per-lane path (Sections 3.1-3.3, remapping and the
// fallbacks of Section 3.4), but texel production is batched: the wave
// writes the (x, y) of every texel it must produce into an LDS row list
// (the unique texels first, then one row per one-tap draw; in a wave that
// takes fallback C or C+, the planned texels of A, then the minifying
// lanes' draws) and decodes the rows 16 at a time on MFMA (decoder_mlp.h).  Dedup therefore turns the 4-texel
// bilinear decode into one dense MLP pass over the wave's distinct texels.
//
// Waves are persistent: each loads the MLP weights into registers once and
// walks a band of tiles.  Workgroups are dispatched round-robin over the 8
// XCDs; band b of the screen goes to the workgroups of XCD b so that the
// latent-grid reads of neighbouring tiles share an L2.
#include "ctf_device.h"
#include "ctf_internal.h"
#include "decoder_mlp.h"
#include "fallback.h"

namespace ctf {

namespace {

constexpr int kDecWaves = 4;

struct DecLds {
    float4 vals[kMaxItems];     // decoded texels, by row
    int2 rows[kMaxItems];       // texel coordinates to decode
    uint64_t keys[kMaxItems];   // List past 16x16: sorted unique keys
    uint8_t rank[256];          // Mask/List: position t -> row (h^-1)
    uint8_t bytes[256];         // footprint-corner scatter before the ballots
};


__device__ int dec_list_sorted(DecLds& L, bool inA, const Footprint& f, int xmin, int ymin)
{
    const int lane = lane_id();
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        uint64_t key = ~0ull;
        if (inA)
            key = ((uint64_t)(uint32_t)(f.y0 + (q >> 1) - ymin) << 32) | (uint32_t)(f.x0 + (q & 1) - xmin);
        L.keys[4 * lane + q] = key;
    }
    for (int size = 2; size <= kMaxItems; size <<= 1)
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            wave_lds_sync();
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int p = lane + kWave * h;
                const int i = (p / stride) * stride * 2 + (p % stride);
                const int j = i + stride;
                const bool up = (i & size) == 0;
                const uint64_t x = L.keys[i], y = L.keys[j];
                if ((x > y) == up) {
                    L.keys[i] = y;
                    L.keys[j] = x;
                }
            }
        }
    wave_lds_sync();
    uint64_t k4[4];
    bool first[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const int i = kWave * c + lane;
        k4[c] = L.keys[i];
        first[c] = k4[c] != ~0ull && (i == 0 || L.keys[i - 1] != k4[c]);
    }
    wave_lds_sync();
    int base = 0;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const uint64_t b = ballot(first[c]);
        if (first[c]) L.keys[base + mbcnt(b)] = k4[c];
        base += popc64(b);
    }
    wave_lds_sync();
    return base;
}

__device__ __forceinline__ int dec_list_find(const DecLds& L, int n, uint64_t key)
{
    int lo = 0, hi = n;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (L.keys[mid] < key) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

template <int P>
__device__ __forceinline__ void fetch_row(const int2* rows, int R, int row, const LatentGrid& G, int g,
                                          LatentFetch& F)
{
    const int2 p = row < R ? rows[row] : make_int2(0, 0);
    latent_fetch(G, p.x, p.y, g, F);
}

template <int P>
__device__ __forceinline__ void finish_row(float4* vals, int R, int row, const FwdWeights<P>& W,
                                           const Biases& Bz, const LatentFetch& F, int g)
{
    const f4 y = mlp_forward<P>(W, Bz, latent_combine<P>(F), nullptr, nullptr);
    if (g == 0 && row < R) vals[row] = make_float4(y[0], y[1], y[2], y[3]);
}

// rows[0..R) -> vals[0..R) in 16-row tiles, two fetch buffers in ping-pong.
// Every prefetch is issued unconditionally (rows past R fetch cell 0), so
// each path reaches the next tile's MLP with the same loads outstanding and
// the wait before it covers only the current tile's gathers.
template <int P>
__device__ __forceinline__ void decode_rows(DecLds& L, int R, const LatentGrid& G, const FwdWeights<P>& W,
                                            const Biases& Bz, int j, int g)
{
    const int T = (R + 15) >> 4;
    if (T == 0) return;
    LatentFetch fa, fb;
    fetch_row<P>(L.rows, R, j, G, g, fa);
    for (int t = 0; t < T; t += 2) {
        fetch_row<P>(L.rows, R, 16 * (t + 1) + j, G, g, fb);
        finish_row<P>(L.vals, R, 16 * t + j, W, Bz, fa, g);
        if (t + 1 >= T) break;
        fetch_row<P>(L.rows, R, 16 * (t + 2) + j, G, g, fa);
        finish_row<P>(L.vals, R, 16 * (t + 1) + j, W, Bz, fb, g);
    }
}

// One tile of the decoder-path filter: decisions, row list, MFMA decode,
// gather and outputs.  `f` is the lanes' footprint (already in this
// layer's coordinates); a.out / a.tile_stats / a.stf_xy point at this
// layer's planes.
template <int METHOD, int P, bool STATS, bool FB>
__device__ __forceinline__ void dec_tile(const FilterArgs& a, const LatentGrid& G, const FwdWeights<P>& W,
                                         const Biases& Bz, DecLds& L, int64_t tile, int tx, int ty,
                                         const Footprint& f, FrameCounters& fc)
{
    const int lane = lane_id();
    const int j = lane & 15, g = lane >> 4;
    const int px = tx * kTile + (lane & 7), py = ty * kTile + (lane >> 3);
    const bool in_screen = px < a.sw && py < a.sh;
    const int64_t pix = (int64_t)py * a.sw + px;
    const bool inA = f.active && f.magnify;
    const uint64_t act = ballot(f.active);
    const uint64_t A = ballot(inA);
    const int nA = popc64(A);

    int xmin = 0, ymin = 0, bbw = 0, bbh = 0;
    constexpr bool kCollab = METHOD == CTF_LIST || METHOD == CTF_BOX || METHOD == CTF_MASK;
    if ((kCollab || STATS) && nA > 0) {
        xmin = wave_min(inA ? f.x0 : INT32_MAX);
        ymin = wave_min(inA ? f.y0 : INT32_MAX);
        bbw = wave_max(inA ? f.x0 + 1 : INT32_MIN) - xmin + 1;
        bbh = wave_max(inA ? f.y0 + 1 : INT32_MIN) - ymin + 1;
    }
    const bool fits16 = nA > 0 && bbw <= 16 && bbh <= 16;

    // ---- 16x16 wave mask B (Mask Sampling; also the exact set when it
    // fits).  Each lane of A marks only its footprint's upper-left texel
    // (mask C, one LDS byte and four ballots); every footprint adds the
    // texels at +1, +16 and +17, so B = C | C<<1 | C<<16 | C<<17 (rows of
    // 16 do not wrap: corners have dx, dy <= 14 when the box fits).
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
            n = dec_list_sorted(L, inA, f, xmin, ymin);
            sorted = true;
        } else {
            n = nmask;
        }
        unique = n;
        count_ok = n <= k * nA;
        success = nA > 0 && count_ok;
    }
    if constexpr (STATS && METHOD != CTF_LIST) {
        if (nA > 0 && !fits16) unique = dec_list_sorted(L, inA, f, xmin, ymin);
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
        pick = stf_pick_h(f, h1, h2);
    }
    // fallback C / C+ for the lanes of A of a failed wave (fallback.h)
    const bool fallback = FB && !success && nA > 0;
    const uint64_t mdraw = stfmask & ~A;   // minifying draws in a fallback wave
    FallbackPlan fp{};

    // ---- row list: the texels to produce (unique texels first, in the
    // method's order, then one row per fallback draw) and the inverse table
    // of Mask/List
    const int rank_act = mbcnt(act);
    const int ns = success ? n : 0;
    int R;
    if constexpr (METHOD == CTF_BILINEAR4) {
        R = 4 * popc64(act);
        if (f.active) {
#pragma unroll
            for (int q = 0; q < 4; ++q) L.rows[4 * rank_act + q] = make_int2(f.x0 + (q & 1), f.y0 + (q >> 1));
        }
    } else if (fallback) {
        fp = plan_fallback<CTF_FILTER_BILINEAR>(L, a.fallback, inA, nA, mbcnt(A), f, pick, pcg_hash(h2), fits16, xmin, ymin);
        R = fp.nprod + popc64(mdraw);
        if (fp.produces) L.rows[fp.slot] = fp.texel;
        if (draws && !inA) L.rows[fp.nprod + mbcnt(mdraw)] = pick;
    } else {
        R = ns + nstf;
        if (success) {
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
                    L.rows[i] = make_int2(ex, ey);
                    if (a.lists) reinterpret_cast<int2*>(a.lists)[(size_t)tile * kMaxItems + i] = make_int2(ex, ey);
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
                        if (a.lists) reinterpret_cast<int2*>(a.lists)[(size_t)tile * kMaxItems + r] = c;
                    }
                    base += popc64(B[w]);
                }
            }
            if (sorted && inA) {
                // List past 16x16: the lane's four item indices by binary
                // search, kept in the (otherwise unused) rank table
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const uint64_t key = ((uint64_t)(uint32_t)(f.y0 + (q >> 1) - ymin) << 32) |
                                         (uint32_t)(f.x0 + (q & 1) - xmin);
                    L.rank[4 * lane + q] = (uint8_t)dec_list_find(L, n, key);
                }
            }
        }
        if (draws) L.rows[ns + mbcnt(stfmask)] = pick;
    }
    // the debug draws are known now; write them before the decode so the
    // draw is not kept live across it
    if (in_screen && a.stf_xy)
        reinterpret_cast<int2*>(a.stf_xy)[pix] = draws ? pick : make_int2(INT32_MIN, INT32_MIN);
    // where this lane's four texels sit: item indices gi + {0, 1, gd, gd + 1}
    // (Box: directly; Mask and List: through the rank table)
    int gi = 0, gd = 0;
    if constexpr (METHOD == CTF_BOX) {
        gi = (f.x0 - xmin) + (f.y0 - ymin) * bbw;
        gd = bbw;
    } else if constexpr (METHOD == CTF_LIST || METHOD == CTF_MASK) {
        gi = sorted ? 4 * lane : 16 * (f.y0 - ymin) + (f.x0 - xmin);
        gd = sorted ? 2 : 16;
    }
    const int draw_row = ns + mbcnt(stfmask);
    wave_lds_sync();

    // ---- decode the rows, 16 per MFMA tile; the latent gathers of the
    // next tile are in flight during the MLP of the current one
    decode_rows<P>(L, R, G, W, Bz, j, g);
    wave_lds_sync();

    int idx[4] = {gi, gi + 1, gi + gd, gi + gd + 1};
    if constexpr (METHOD == CTF_LIST || METHOD == CTF_MASK) {
        if (exact) {
#pragma unroll
            for (int q = 0; q < 4; ++q) idx[q] = L.rank[idx[q]];
        }
    }

    // ---- gather and weight
    float4 res = make_float4(0.f, 0.f, 0.f, 0.f);
    if constexpr (METHOD == CTF_BILINEAR4) {
        if (exact) {
            const int b = 4 * rank_act;
            res = bilerp(f.s, f.t, L.vals[b], L.vals[b + 1], L.vals[b + 2], L.vals[b + 3]);
        }
    } else if (fallback) {
        if (draws && !inA) res = L.vals[fp.nprod + mbcnt(mdraw)];
        if (inA) res = fallback_color<CTF_FILTER_BILINEAR>(L, fp, f, pick, xmin, ymin);
    } else {
        if (draws) res = L.vals[draw_row];
        if (kCollab && exact)
            res = bilerp(f.s, f.t, L.vals[idx[0]], L.vals[idx[1]], L.vals[idx[2]], L.vals[idx[3]]);
    }
    if (in_screen) reinterpret_cast<float4*>(a.out)[pix] = res;
    if (lane == 0) {
        if (a.tile_stats) {
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
            S.evals = R;
            S.flags = (success ? CTF_TILE_OK : 0) | (nA && !cap_ok ? CTF_TILE_CAP : 0) |
                      (nA && cap_ok && !count_ok ? CTF_TILE_OVERFLOW : 0) | (nA == 0 ? CTF_TILE_EMPTY : 0);
            for (int r = 0; r < 10; ++r) S.reserved[r] = 0;
            a.tile_stats[tile] = S;
        }
    }
    if (act) fc.add(R, popc64(act), nstf, popc64(act & ~A), (R + 15) & ~15, kCollab && success,
                    kCollab && nA && !success);
    wave_lds_sync();  // the next tile reuses this wave's LDS slice
}

// Inputs of a tile for this lane, NaN (inactive) outside the band or screen.
__device__ __forceinline__ void load_tile_px(const FilterArgs& a, const TileWalk& t, int64_t band_e, float2& uv,
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

// XCD-aware band of tiles for this wave: workgroups go round-robin over the
// 8 XCDs, so band b of the screen is walked by the workgroups of XCD b.
struct Band {
    int64_t begin, end;
    int lw, nw;
    __device__ Band(int64_t ntiles, int wid)
    {
        const int xcd = blockIdx.x & 7;
        lw = (int)(blockIdx.x >> 3) * kDecWaves + wid;
        nw = (int)(gridDim.x >> 3) * kDecWaves;
        begin = ntiles * xcd / 8;
        end = ntiles * (xcd + 1) / 8;
    }
};

// Waves per SIMD the register budget of the single-layer kernel is sized
// for: the collaborative methods need the bound of three to fit in 168
// registers; the others fit three anyway and keep the compiler's schedule.
template <int METHOD>
constexpr int dec_waves_per_simd() { return METHOD == CTF_LIST || METHOD == CTF_BOX || METHOD == CTF_MASK ? 3 : 2; }

template <int METHOD, int P, bool STATS, bool FB>
__global__ __launch_bounds__(64 * kDecWaves, dec_waves_per_simd<METHOD>()) void k_filter_dec(FilterArgs a,
                                                                                             DevDecoderWeights D)
{
    __shared__ DecLds lds_all[kDecWaves];
    const int wid = threadIdx.x >> 6;
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
    TileWalk next(band.begin + band.lw, band.nw, a.tiles_x);
    load_tile_px(a, next, band.end, uv_next, d_next);
    while (next.tile < band.end) {
        const TileWalk cur = next;
        const float2 uv = uv_next;
        const float4 d = d_next;
        next.advance(band.nw);
        load_tile_px(a, next, band.end, uv_next, d_next);
        const Footprint f = footprint(uv.x, uv.y, d, tex_w, tex_w);
        dec_tile<METHOD, P, STATS, FB>(a, D.grid, W, Bz, L, cur.tile, cur.tx, cur.ty, f, fc);
    }
    if (lane == 0 && a.frame_stats) fc.flush(a.frame_stats);
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

template <int METHOD, int P, bool STATS, bool FB>
__global__ __launch_bounds__(64 * kDecWaves, 2) void k_filter_layers(FilterArgs a, LayerSet LS)
{
    __shared__ DecLds lds_all[kDecWaves];
    const int wid = threadIdx.x >> 6;
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
        TileWalk next(band.begin + band.lw, band.nw, a.tiles_x);
        load_tile_px(a, next, band.end, uv_next, d_next);
        while (next.tile < band.end) {
            const TileWalk cur = next;
            const float2 uv = uv_next;
            const float4 d = d_next;
            next.advance(band.nw);
            load_tile_px(a, next, band.end, uv_next, d_next);
            // layer coordinates, float32: u' = fma(m01, v, m00 u), v' = fma(m11, v, m10 u)
            const float lu = __builtin_fmaf(m01, uv.y, m00 * uv.x), lv = __builtin_fmaf(m11, uv.y, m10 * uv.x);
            const float4 ld = make_float4(__builtin_fmaf(m01, d.y, m00 * d.x), __builtin_fmaf(m11, d.y, m10 * d.x),
                                          __builtin_fmaf(m01, d.w, m00 * d.z), __builtin_fmaf(m11, d.w, m10 * d.z));
            const Footprint f = footprint(lu, lv, ld, tex_w, tex_w);
            dec_tile<METHOD, P, STATS, FB>(al, D.grid, W, Bz, L, cur.tile, cur.tx, cur.ty, f, fc);
        }
    }
    if (lane == 0 && a.frame_stats) fc.flush(a.frame_stats);
}


// rgba[i] = decoder(xy[i]): 16 texels per MFMA tile, persistent waves; the
// same per-row instruction sequence as the filter's decode.
template <int P>
__global__ __launch_bounds__(256, 2) void k_decoder_eval(DevDecoderWeights D, const int2* __restrict__ xy,
                                                         int64_t n, float4* __restrict__ out)
{
    const int lane = lane_id();
    const int j = lane & 15, g = lane >> 4;
    FwdWeights<P> W;
    W.load(D.w, lane);
    Biases Bz;
    Bz.load(D.bias, lane);
    const int64_t gw = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const int64_t nw = (int64_t)gridDim.x * (blockDim.x >> 6);
    const int64_t ntiles = (n + 15) / 16;
    for (int64_t t = gw; t < ntiles; t += nw) {
        const int64_t row = t * 16 + j;
        const bool valid = row < n;
        const int2 p = valid ? xy[row] : make_int2(0, 0);
        LatentFetch F;
        latent_fetch(D.grid, p.x, p.y, g, F);
        const f4 y = mlp_forward<P>(W, Bz, latent_combine<P>(F), nullptr, nullptr);
        if (g == 0 && valid) out[row] = make_float4(y[0], y[1], y[2], y[3]);
    }
}

int device_cus()
{
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    return cus > 0 ? cus : 256;
}

// Persistent grid: as many workgroups as fit on the device at once (from the
// kernel's register and LDS use), a multiple of the 8 XCDs.
template <typename K>
int64_t resident_blocks(K kernel, int threads, int64_t work_blocks)
{
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, 0) != hipSuccess || per_cu < 1)
        per_cu = 1;
    int64_t blocks = (int64_t)device_cus() * per_cu;
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
    const bool st = a.tile_stats != nullptr;
    if constexpr (collaborative(METHOD)) {
        if (a.fallback != CTF_FB_STF1)
            return st ? Go<METHOD, P, true, true>::run(a, args...) : Go<METHOD, P, false, true>::run(a, args...);
    }
    return st ? Go<METHOD, P, true, false>::run(a, args...) : Go<METHOD, P, false, false>::run(a, args...);
}

template <int METHOD, int P, bool STATS, bool FB>
struct GoFilter {
    static hipError_t run(const FilterArgs& a, const DevDecoderWeights& d, hipStream_t s)
    {
        const int64_t work = (a.ntiles + kDecWaves - 1) / kDecWaves;
        auto k = k_filter_dec<METHOD, P, STATS, FB>;
        const int64_t blocks = resident_blocks(k, 64 * kDecWaves, work);
        hipLaunchKernelGGL(k, dim3((unsigned)blocks), dim3(64 * kDecWaves), 0, s, a, d);
        return hipGetLastError();
    }
};

template <int METHOD, int P, bool STATS, bool FB>
struct GoLayers {
    static hipError_t run(const FilterArgs& a, const LayerSet& LS, hipStream_t s)
    {
        const int64_t work = (a.ntiles + kDecWaves - 1) / kDecWaves;
        auto k = k_filter_layers<METHOD, P, STATS, FB>;
        const int64_t blocks = resident_blocks(k, 64 * kDecWaves, work);
        hipLaunchKernelGGL(k, dim3((unsigned)blocks), dim3(64 * kDecWaves), 0, s, a, LS);
        return hipGetLastError();
    }
};

template <int METHOD, int P>
hipError_t launch_dec(const FilterArgs& a, const DevDecoderWeights& d, hipStream_t s)
{
    return dispatch_flags<METHOD, P, GoFilter>(a, d, s);
}

template <int METHOD, int P>
hipError_t launch_layers(const FilterArgs& a, const LayerSet& LS, hipStream_t s)
{
    return dispatch_flags<METHOD, P, GoLayers>(a, LS, s);
}

template <int P>
hipError_t launch_layers_p(const FilterArgs& a, const LayerSet& LS, hipStream_t s)
{
    switch (a.method) {
    case CTF_BILINEAR4: return launch_layers<CTF_BILINEAR4, P>(a, LS, s);
    case CTF_STF1: return launch_layers<CTF_STF1, P>(a, LS, s);
    case CTF_LIST: return launch_layers<CTF_LIST, P>(a, LS, s);
    case CTF_BOX: return launch_layers<CTF_BOX, P>(a, LS, s);
    case CTF_MASK: return launch_layers<CTF_MASK, P>(a, LS, s);
    default: return hipErrorInvalidValue;
    }
}

template <int P>
hipError_t launch_dec_p(const FilterArgs& a, const DevDecoderWeights& d, hipStream_t s)
{
    switch (a.method) {
    case CTF_BILINEAR4: return launch_dec<CTF_BILINEAR4, P>(a, d, s);
    case CTF_STF1: return launch_dec<CTF_STF1, P>(a, d, s);
    case CTF_LIST: return launch_dec<CTF_LIST, P>(a, d, s);
    case CTF_BOX: return launch_dec<CTF_BOX, P>(a, d, s);
    case CTF_MASK: return launch_dec<CTF_MASK, P>(a, d, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace

}  // namespace ctf

using namespace ctf;

hipError_t ctf_internal_decoder_filter(const ctf_texture_s* t, const FilterArgs& a, hipStream_t s)
{
    const DevDecoderWeights& d = t->dec;
    return t->dec.precision == CTF_BF16 ? launch_dec_p<CTF_BF16>(a, d, s) : launch_dec_p<CTF_FP16>(a, d, s);
}

hipError_t ctf_internal_filter_layers(const ctf_texture_s* const* texs, const float* xforms, int n,
                                      const FilterArgs& a, hipStream_t s)
{
    if (n < 1 || n > kMaxLayers) return hipErrorInvalidValue;
    LayerSet LS;
    LS.n = n;
    const int prec = texs[0]->dec.precision;
    for (int l = 0; l < n; ++l) {
        if (texs[l]->dev.kind != CTF_TEX_DECODER || texs[l]->dec.precision != prec) return hipErrorInvalidValue;
        LS.dec[l] = texs[l]->dec;
        for (int k = 0; k < 4; ++k) LS.xf[l][k] = xforms[4 * l + k];
    }
    return prec == CTF_BF16 ? launch_layers_p<CTF_BF16>(a, LS, s) : launch_layers_p<CTF_FP16>(a, LS, s);
}

hipError_t ctf_internal_decoder_eval(const ctf_texture_s* t, const int32_t* xy, int64_t n, float* out,
                                     hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    const DevDecoderWeights& d = t->dec;
    int64_t blocks = ((n + 15) / 16 + 3) / 4;
    const int64_t cap = (int64_t)device_cus() * 2;
    if (blocks > cap) blocks = cap;
    const int2* p = reinterpret_cast<const int2*>(xy);
    float4* o = reinterpret_cast<float4*>(out);
    if (t->dec.precision == CTF_BF16)
        hipLaunchKernelGGL(k_decoder_eval<CTF_BF16>, dim3((unsigned)blocks), dim3(256), 0, s, d, p, n, o);
    else
        hipLaunchKernelGGL(k_decoder_eval<CTF_FP16>, dim3((unsigned)blocks), dim3(256), 0, s, d, p, n, o);
    return hipGetLastError();
}
