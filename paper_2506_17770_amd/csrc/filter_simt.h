// filter_simt.h -- collaborative filtering with per-lane texel production.
//
// One 8x8 tile per wave64, four waves per workgroup.  Each lane produces at
// most k texels per wave (k = max_evals_per_lane); the produced values are
// staged in the wave's LDS slice and gathered by item index.  Used for the
// procedural, stored-table and test texel producers (the decoder producer
// batches its texels into MFMA tiles instead, see filter_decoder.hip).
// Instantiated per reconstruction filter: FxF footprints, F = 2 (bilinear)
// or 4 (bicubic B-spline, Catmull-Rom).
//
// Paper: Section 3 (three-step flow), 3.1 List Merge, 3.2 Box Sampling,
// 3.3 Mask Sampling (bijection h of Figure 3), supplement Section 2 (edge
// remapping: item i is produced by lane h(i, A)), Section 3.4 (fallbacks:
// one-tap STF, C of Eq. 1 and C+ of Eq. 2, fallback.h), Section 5 (bicubic
// filters).
#pragma once

#include "ctf_device.h"
#include "ctf_internal.h"
#include "fallback.h"

namespace ctf {

namespace simt {

constexpr int kWavesPerBlock = 4;

template <int F>
struct WaveLds {
    float4 vals[kMaxItems];         // produced texel values, by item index
    uint64_t keys[kWave * F * F];   // List: sorted unique texel keys (dy << 32 | dx)
    uint16_t items[kMaxItems];      // Mask: item i -> mask position t = h(i, B)
    uint8_t rank[256];              // Mask: position t -> item index h^-1(t, B)
    uint8_t bytes[256];             // Mask: footprint-corner scatter before the ballots
};
static_assert(kWavesPerBlock * sizeof(WaveLds<2>) + kLdsTermEntries * sizeof(int4) <= 32768,
              "a bilinear per-lane workgroup must fit five to a CU");

// Exact set of the wave's texels as sorted unique keys (any box size): a
// bitonic sort of the F^2 |A| footprint keys in LDS, then compaction of the
// first key of every run.  Returns n = |U|; keys[0..n) hold U in (y, x)
// order.
template <int F>
__device__ int list_unique_sorted(WaveLds<F>& L, bool inA, int ox, int oy, int xmin, int ymin)
{
    constexpr int N = kWave * F * F;
    const int lane = lane_id();
#pragma unroll
    for (int q = 0; q < F * F; ++q) {
        uint64_t key = ~0ull;
        if (inA) {
            const uint32_t dx = (uint32_t)(ox + q % F - xmin);
            const uint32_t dy = (uint32_t)(oy + q / F - ymin);
            key = ((uint64_t)dy << 32) | dx;
        }
        L.keys[F * F * lane + q] = key;
    }
    for (int size = 2; size <= N; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            wave_lds_sync();
#pragma unroll
            for (int h = 0; h < N / (2 * kWave); ++h) {
                const int p = lane + kWave * h;                 // pair index
                const int i = (p / stride) * stride * 2 + (p % stride);
                const int j = i + stride;
                const bool up = (i & size) == 0;
                const uint64_t a = L.keys[i], b = L.keys[j];
                if ((a > b) == up) {
                    L.keys[i] = b;
                    L.keys[j] = a;
                }
            }
        }
    }
    // compaction in rounds of 64 keys: a write index never passes the read
    // index, and round r writes below every key of the later rounds
    int base = 0;
    for (int c = 0; c < F * F; ++c) {
        wave_lds_sync();
        const int i = kWave * c + lane;
        const uint64_t k = L.keys[i];
        const bool first = k != ~0ull && (i == 0 || L.keys[i - 1] != k);
        const uint64_t b = ballot(first);
        wave_lds_sync();
        if (first) L.keys[base + mbcnt(b)] = k;
        base += popc64(b);
    }
    wave_lds_sync();
    return base;
}

template <int F>
__device__ __forceinline__ int list_find(const WaveLds<F>& L, int n, uint64_t key)
{
    int lo = 0, hi = n;  // first index with keys[idx] >= key
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (L.keys[mid] < key) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// FB: the instantiation that plans fallback C / C+ for failed waves (the
// others fall back to one-tap STF only and carry none of that code, which
// keeps their scalar registers for the common path).  Bilinear: five waves
// per SIMD (at most 96 vector registers; the workgroup's LDS fits five per
// CU).  Bicubic: the LDS of the 16-tap footprints holds the occupancy lower,
// the registers are left to the compiler.
template <int FILTER>
constexpr int simt_min_waves()
{
    return Taps<FILTER>::F == 2 ? 5 : 1;
}

template <int METHOD, int TEX, bool STATS, int FILTER, bool FB>
__global__ __launch_bounds__(kWave * kWavesPerBlock, (simt_min_waves<FILTER>())) void k_filter_simt(FilterArgs a,
                                                                                                  DevTexture T)
{
    constexpr int F = Taps<FILTER>::F, O = Taps<FILTER>::O;
    constexpr bool kCanSplit = (METHOD == CTF_LIST || METHOD == CTF_BOX || METHOD == CTF_MASK) &&
                               TEX == CTF_TEX_SINUSOIDS;
    constexpr bool kStage = TEX == CTF_TEX_SINUSOIDS;
    __shared__ WaveLds<F> lds_all[kWavesPerBlock];
    // the texture's terms (split rounds read them by channel; a lane's own
    // texels read them by broadcast)
    __shared__ int4 terms_lds[kStage ? kLdsTermEntries : 1];
    const int wid = wave_in_block();
    const int lane = lane_id();
    WaveLds<F>& L = lds_all[wid];
    bool staged = false, split_ok = false;
    if constexpr (kStage) {
        staged = stage_terms(T, terms_lds);
        split_ok = kCanSplit && staged && a.split == CTF_SPLIT_AUTO;
    }
    const bool lds_float = staged && T.fterms != nullptr;
    auto texel = [&](int x, int y) __attribute__((always_inline)) -> float4 {
        return texel_eval_staged<TEX>(T, terms_lds, lds_float, x, y);
    };
    FrameCounters fc;
    const int64_t nw = (int64_t)gridDim.x * kWavesPerBlock;
    // The inputs of the wave's next tile are loaded one tile ahead, the
    // tile's output is stored at its end.  Both are unconditional (a lane off
    // the screen loads pixel 0 and its coordinates are replaced by NaN when
    // used; it repeats the store of lane 0, which is on the screen in every
    // tile): the memory counters complete in order, and a load or store
    // skipped on some path would make the wait for the next tile's inputs
    // also wait for this tile's store.
    auto load_px = [&](const TileWalk& t, float2& uv, float4& d) __attribute__((always_inline)) -> bool {
        const int qx = t.tx * kTile + (lane & 7), qy = t.ty * kTile + (lane >> 3);
        const bool ok = t.tile < a.ntiles && qx < a.sw && qy < a.sh;
        const int64_t q = ok ? (int64_t)qy * a.sw + qx : 0;
        uv = reinterpret_cast<const float2*>(a.uv)[q];
        d = reinterpret_cast<const float4*>(a.duv)[q];
        return ok;
    };
    TileWalk next((int64_t)blockIdx.x * kWavesPerBlock + wid, nw, a.tiles_x);
    float2 uv_next;
    float4 d_next;
    bool ok_next = load_px(next, uv_next, d_next);
    // wait for the first tile's inputs here, so that the loop head waits
    // only for what the previous iteration requested
    asm volatile("" ::"v"(uv_next.x), "v"(uv_next.y), "v"(d_next.x), "v"(d_next.y), "v"(d_next.z), "v"(d_next.w));
    while (next.tile < a.ntiles) {
        const TileWalk tw = next;
        const float2 uv_cur = ok_next ? uv_next : make_float2(__builtin_nanf(""), 0.f);
        const float4 d_cur = ok_next ? d_next : make_float4(0.f, 0.f, 0.f, 0.f);
        next.advance(nw);
        ok_next = load_px(next, uv_next, d_next);
        const int64_t tile = tw.tile;
        const int tx = tw.tx, ty = tw.ty;
        const int px = tx * kTile + (lane & 7), py = ty * kTile + (lane >> 3);
        const bool in_screen = px < a.sw && py < a.sh;
        const int64_t pix = (int64_t)py * a.sw + px;

        // ---- step 1: footprint, participation (A = active and magnifying)
        const Footprint f = footprint(uv_cur.x, uv_cur.y, d_cur, (float)T.width, (float)T.height);
        const int ox = f.x0 - O, oy = f.y0 - O;   // upper-left tap of the FxF footprint
        const bool inA = f.active && f.magnify;
        const uint64_t act = ballot(f.active);
        const uint64_t A = ballot(inA);
        const int nA = popc64(A);
        const int rankA = mbcnt(A);  // edge remapping: lane of rank r produces items r, r+|A|, ...

        // ---- step 2: wave texel box over A
        int xmin = 0, ymin = 0, bbw = 0, bbh = 0;
        constexpr bool kCollab = METHOD == CTF_LIST || METHOD == CTF_BOX || METHOD == CTF_MASK;
        // Mask and List only need a 16x16 window that holds every footprint
        // of A: try the one centred on a lane of A (lane 36 when it is in A)
        // before reducing the exact box.  Bit positions are relative to the
        // window's corner; the texels, their row-major order and every
        // decision are the same as with the box's corner.
        bool window = false;
        if constexpr ((METHOD == CTF_LIST || METHOD == CTF_MASK) && !STATS) {
            if (nA > 0) {
                constexpr int H = (16 - F) / 2;
                const int rl = ((A >> 36) & 1ull) ? 36 : (int)__builtin_ctzll(A);
                const int wx = __builtin_amdgcn_readlane(ox, rl) - H, wy = __builtin_amdgcn_readlane(oy, rl) - H;
                const bool outside =
                    inA && ((uint32_t)(ox - wx) > (uint32_t)(16 - F) || (uint32_t)(oy - wy) > (uint32_t)(16 - F));
                if (ballot(outside) == 0) {
                    window = true;
                    xmin = wx;
                    ymin = wy;
                }
            }
        }
        if (kCollab || STATS) {
            if (nA > 0 && !window) {
                xmin = wave_min(inA ? ox : INT32_MAX);
                ymin = wave_min(inA ? oy : INT32_MAX);
                bbw = wave_max(inA ? ox + F - 1 : INT32_MIN) - xmin + 1;
                bbh = wave_max(inA ? oy + F - 1 : INT32_MIN) - ymin + 1;
            }
        }
        const bool fits16 = window || (nA > 0 && bbw <= 16 && bbh <= 16);

        // ---- 16x16 wave mask B (Mask Sampling; also the exact set when it fits)
        uint64_t B[4] = {0, 0, 0, 0};
        int nmask = 0;
        constexpr bool kNeedMask = METHOD == CTF_MASK || METHOD == CTF_LIST || STATS;
        if (kNeedMask && fits16) {
            // corners of the footprints (mask C) by one LDS byte per lane and
            // four ballots; B = OR of C shifted over the FxF footprint
            reinterpret_cast<uint32_t*>(L.bytes)[lane] = 0u;
            wave_lds_sync();
            if (inA) L.bytes[16 * (oy - ymin) + (ox - xmin)] = 1;
            wave_lds_sync();
            uint64_t C[4];
#pragma unroll
            for (int w = 0; w < 4; ++w) C[w] = ballot(L.bytes[64 * w + lane] != 0);
            footprint_mask_f<F>(C, B);
            // h and h^-1 as tables: set bit t of rank r gives items[r] = t, rank[t] = r
            int base = 0;
#pragma unroll
            for (int w = 0; w < 4; ++w) {
                if ((B[w] >> lane) & 1u) {
                    const int r = base + mbcnt(B[w]);
                    L.items[r] = (uint16_t)(64 * w + lane);
                    L.rank[64 * w + lane] = (uint8_t)r;
                }
                base += popc64(B[w]);
            }
            nmask = base;
            wave_lds_sync();
        }

        // ---- step 3: the method's decision
        const int k = a.max_evals;
        int n = 0;
        bool cap_ok = true, count_ok = true, success = false, sorted = false;
        int unique = nmask;
        if constexpr (METHOD == CTF_BOX) {
            // area in 64 bits: sides can be large when A spans several surfaces
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
                n = list_unique_sorted<F>(L, inA, ox, oy, xmin, ymin);
                sorted = true;
            } else {
                n = nmask;
            }
            unique = n;
            count_ok = n <= k * nA;
            success = nA > 0 && count_ok;
        }
        if constexpr (STATS && METHOD != CTF_LIST) {
            if (nA > 0 && !fits16) unique = list_unique_sorted<F>(L, inA, ox, oy, xmin, ymin);
        }
        if (nA == 0) unique = 0;

        // lanes whose output is exact filtering vs a one-tap draw
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

        // ---- texel production: each lane evaluates at most one texel per round
        float4 res = make_float4(0.f, 0.f, 0.f, 0.f);
        int2 pick = make_int2(INT32_MIN, INT32_MIN);
        uint32_t h1 = 0, h2 = 0;
        if (draws) {
            stf_hashes(a.seed, a.layer, px, py, h1, h2);
            pick = stf_pick_filter<FILTER>(f, h1, h2);
        }
        // fallback C / C+ for the lanes of A of a failed wave
        const bool fallback = FB && kCollab && !success && nA > 0 && a.fallback != CTF_FB_STF1;
        FallbackPlan P{};
        if (fallback)
            P = plan_fallback<FILTER>(L, a.fallback, inA, nA, rankA, f, pick, pcg_hash(h2), fits16, xmin, ymin);

        if constexpr (METHOD == CTF_BILINEAR4) {
            if (exact) {
                if constexpr (F == 2) {
                    const float4 v0 = texel(f.x0, f.y0);
                    const float4 v1 = texel(f.x0 + 1, f.y0);
                    const float4 v2 = texel(f.x0, f.y0 + 1);
                    const float4 v3 = texel(f.x0 + 1, f.y0 + 1);
                    res = bilerp(f.s, f.t, v0, v1, v2, v3);
                } else {
                    float wx[4], wy[4];
                    taps32<FILTER>(f.s, wx);
                    taps32<FILTER>(f.t, wy);
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        const float4 r = row4(wx, texel(ox, oy + j), texel(ox + 1, oy + j),
                                              texel(ox + 2, oy + j), texel(ox + 3, oy + j));
                        res = col_acc(wy[j], r, res, j == 0);
                    }
                }
            }
        } else if (fallback) {
            // lanes of A evaluate the planned texels; minifying lanes draw
            const bool pa = inA && P.produces, pd = draws && !inA;
            if (pa || pd) {
                const int2 e = pa ? P.texel : pick;
                const float4 v = texel(e.x, e.y);
                if (pa) L.vals[P.slot] = v;
                else res = v;
            }
            wave_lds_sync();
            if (inA) res = fallback_color<FILTER>(L, P, f, pick, xmin, ymin);
        } else {
            // texel of item i of the method's order
            auto item_xy = [&](int item) -> int2 {
                if constexpr (METHOD == CTF_BOX) {
                    return make_int2(xmin + item % bbw, ymin + item / bbw);
                } else {
                    if (sorted) {
                        const uint64_t key = L.keys[item];
                        return make_int2(xmin + (int)(uint32_t)key, ymin + (int)(key >> 32));
                    }
                    const int t = L.items[item];
                    return make_int2(xmin + (t & 15), ymin + (t >> 4));
                }
            };
            auto list_out = [&](int item, int2 e) {
                if (STATS && a.lists) reinterpret_cast<int2*>(a.lists)[(size_t)tile * kMaxItems + item] = e;
            };
            // split-texel production: a successful wave with no one-tap
            // draws evaluates its 4n texel channels over all 64 lanes (lane l
            // takes channels l, l + 64, ...: item j / 4, channel j % 4), when
            // that takes fewer channel evaluations per lane, ceil(n / 16), than
            // one texel per lane of A, 4 ceil(n / |A|)
            bool split = false;
            if constexpr (kCanSplit) {
                split = split_ok && success && stfmask == 0 && (n + 15) / 16 < 4 * ((n + nA - 1) / nA);
                if (split) {
                    const int K = T.n_terms;
                    for (int j = lane; j < 4 * n; j += kWave) {
                        const int item = j >> 2, c = j & 3;
                        const int2 e = item_xy(item);
                        if (c == 0) list_out(item, e);
                        float* v = reinterpret_cast<float*>(&L.vals[item]);
                        const int xm = e.x & (int)T.wmask, ym = e.y & (int)T.wmask;
                        v[c] = T.fterms ? sinusoid_channel_f(reinterpret_cast<const float4*>(terms_lds) + c * (K + 1),
                                                             K, (float)xm, (float)ym)
                                        : sinusoid_channel(terms_lds + c * (K + 1), K, T.wmask, T.inv_w, xm, ym);
                    }
                }
            }
            for (int round = 0; !split && round < (kCollab ? k : 1); ++round) {
                const int item = rankA + round * nA;
                const bool produce = kCollab && success && inA && item < n;
                const bool draw_now = draws && round == 0;
                if (ballot(produce || draw_now) == 0) break;
                int2 e = pick;
                if (produce) {
                    e = item_xy(item);
                    list_out(item, e);
                }
                if (produce || draw_now) {
                    const float4 v = texel(e.x, e.y);
                    if (produce) L.vals[item] = v;
                    if (draw_now) res = v;
                }
            }
            if constexpr (kCollab) {
                // ---- gather: item index of each footprint texel, then weight
                wave_lds_sync();
                if (exact) {
                    // item index of the first tap of footprint row j; the
                    // row's other taps are the next items (the set holds the
                    // whole row, in row-major order for Mask and List)
                    auto row_item = [&](int j) -> int {
                        if constexpr (METHOD == CTF_BOX) {
                            return (ox - xmin) + (oy + j - ymin) * bbw;
                        } else {
                            if (sorted) {
                                const uint64_t key = ((uint64_t)(uint32_t)(oy + j - ymin) << 32) |
                                                     (uint32_t)(ox - xmin);
                                return list_find<F>(L, n, key);
                            }
                            return L.rank[16 * (oy + j - ymin) + (ox - xmin)];
                        }
                    };
                    if constexpr (F == 2) {
                        const int i0 = row_item(0), i2 = row_item(1);
                        res = bilerp(f.s, f.t, L.vals[i0], L.vals[i0 + 1], L.vals[i2], L.vals[i2 + 1]);
                    } else {
                        float wx[4], wy[4];
                        taps32<FILTER>(f.s, wx);
                        taps32<FILTER>(f.t, wy);
#pragma unroll
                        for (int j = 0; j < 4; ++j) {
                            const int i0 = row_item(j);
                            const float4 r = row4(wx, L.vals[i0], L.vals[i0 + 1], L.vals[i0 + 2], L.vals[i0 + 3]);
                            res = col_acc(wy[j], r, res, j == 0);
                        }
                    }
                }
            }
        }

        // ---- outputs
        {
            // (selected per component: a select of two float4 lvalues
            // would put both in memory)
            auto lane0 = [&](float v) { return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 0)); };
            const float4 o = make_float4(in_screen ? res.x : lane0(res.x), in_screen ? res.y : lane0(res.y),
                                         in_screen ? res.z : lane0(res.z), in_screen ? res.w : lane0(res.w));
            const int64_t pix0 = (int64_t)(ty * kTile) * a.sw + tx * kTile;
            reinterpret_cast<float4*>(a.out)[in_screen ? pix : pix0] = o;
        }
        if (in_screen && a.stf_xy)
            reinterpret_cast<int2*>(a.stf_xy)[pix] = draws ? pick : make_int2(INT32_MIN, INT32_MIN);
        const int nstf = popc64(stfmask);
        int evals;
        if constexpr (METHOD == CTF_BILINEAR4) evals = F * F * popc64(act);
        else if (fallback) evals = P.nprod + popc64(stfmask & ~A);
        else evals = (success ? n : 0) + nstf;

        if (lane == 0) {
            if (STATS && a.tile_stats) {
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
                          (nA && cap_ok && !count_ok ? CTF_TILE_OVERFLOW : 0) |
                          (nA == 0 ? CTF_TILE_EMPTY : 0);
                for (int r = 0; r < 10; ++r) S.reserved[r] = 0;
                a.tile_stats[tile] = S;
            }
        }
        if (act) fc.add(evals, popc64(act), nstf, popc64(act & ~A), 0, kCollab && success, kCollab && nA && !success);
        wave_lds_sync();  // the next tile reuses this wave's LDS slice
    }
    if (lane == 0 && a.frame_stats) fc.flush(a.frame_stats);
}

template <int METHOD, int TEX, int FILTER>
hipError_t launch_m_t(const FilterArgs& a, const DevTexture& T, hipStream_t s)
{
    constexpr bool kCollab = METHOD == CTF_LIST || METHOD == CTF_BOX || METHOD == CTF_MASK;
    // the instantiation with statistics also writes the texel lists
    const bool st = a.tile_stats != nullptr || a.lists != nullptr;
    void (*k)(FilterArgs, DevTexture);
    if (kCollab && a.fallback != CTF_FB_STF1)
        k = st ? k_filter_simt<METHOD, TEX, true, FILTER, kCollab> : k_filter_simt<METHOD, TEX, false, FILTER, kCollab>;
    else
        k = st ? k_filter_simt<METHOD, TEX, true, FILTER, false> : k_filter_simt<METHOD, TEX, false, FILTER, false>;
    // grid-stride over tiles: two rounds of the workgroups that fit on the
    // chip at once (the second round evens out the tiles' uneven costs),
    // several tiles per wave
    int dev = 0, cus = 256, per_cu = 0;
    if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, kWave * kWavesPerBlock, 0) != hipSuccess || per_cu < 1)
        per_cu = 4;
    int64_t blocks = (a.ntiles + kWavesPerBlock - 1) / kWavesPerBlock;
    if (blocks > (int64_t)cus * per_cu * 2) blocks = (int64_t)cus * per_cu * 2;
    const int64_t least = counter_min_blocks(a.ntiles, kWavesPerBlock);   // 32-bit frame counters
    if (blocks < least) blocks = least;
    hipLaunchKernelGGL(k, dim3((unsigned)blocks), dim3(kWave * kWavesPerBlock), 0, s, a, T);
    return hipGetLastError();
}

template <int TEX, int FILTER>
hipError_t launch_t(const FilterArgs& a, const DevTexture& T, hipStream_t s)
{
    switch (a.method) {
    case CTF_BILINEAR4: return launch_m_t<CTF_BILINEAR4, TEX, FILTER>(a, T, s);
    case CTF_STF1: return launch_m_t<CTF_STF1, TEX, FILTER>(a, T, s);
    case CTF_LIST: return launch_m_t<CTF_LIST, TEX, FILTER>(a, T, s);
    case CTF_BOX: return launch_m_t<CTF_BOX, TEX, FILTER>(a, T, s);
    case CTF_MASK: return launch_m_t<CTF_MASK, TEX, FILTER>(a, T, s);
    default: return hipErrorInvalidValue;
    }
}

template <int FILTER>
hipError_t launch_filter(const FilterArgs& a, const DevTexture& T, hipStream_t s)
{
    switch (T.kind) {
    case CTF_TEX_SINUSOIDS: return launch_t<CTF_TEX_SINUSOIDS, FILTER>(a, T, s);
    case CTF_TEX_AFFINE: return launch_t<CTF_TEX_AFFINE, FILTER>(a, T, s);
    case CTF_TEX_CONSTANT: return launch_t<CTF_TEX_CONSTANT, FILTER>(a, T, s);
    case CTF_TEX_TABLE: return launch_t<CTF_TEX_TABLE, FILTER>(a, T, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace simt

}  // namespace ctf
