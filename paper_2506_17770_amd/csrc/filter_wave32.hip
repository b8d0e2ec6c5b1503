// filter_wave32.hip -- the paper's wave shape on gfx950: 8x4-pixel tiles of
// 32 lanes (Section 3: 8x4 pixels per wave32), two per wave64, one per
// half-wave.  Each half-wave takes its own collaborative step (Box, Mask,
// List, remapping and the one-tap fallback) exactly as a wave32 would, so
// the success regions of Figure 4 (bilinear) and of the bicubic maps of the
// supplement's additional bicubic results, and the evaluation counts, can
// be checked on hardware.  Per-lane texel production, bilinear or bicubic
// (FxF footprints, F = 2 or 4) filters, one-tap STF fallback.
//
// Half-wave quantities are computed for both halves as scalars (ballots
// split into their 32-bit halves, DPP reductions combined per pair of
// 16-lane rows) and each lane selects its own half's value.
#include "ctf_device.h"
#include "ctf_internal.h"
#include "fallback.h"

namespace ctf {

namespace {

constexpr int kW32Waves = 4;
constexpr int kHalfItems = kMaxItems / 2;  // n <= k |A| <= 4 * 32 per half

template <int F>
struct W32Lds {
    float4 vals[2][kHalfItems];   // produced texel values, by half and item
    uint64_t keys[kWave * F * F]; // List past 16x16: sorted unique keys, half in bit 62
    uint16_t items[2][256];       // Mask: item i -> position t = h(i, B)
    uint8_t rank[2][256];         // Mask: position t -> item index h^-1(t, B); fallback: slot + 1
    uint8_t bytes[2][256];        // footprint-corner scatter before the ballots
    StashEntry stash[2][32];      // fallback C+: each lane's footprint, by half
    int2 produced[2][32];         // fallback C past 16x16: the produced texels, by slot
};

// min/max over each half-wave (all 64 lanes active): DPP over the 16-lane
// rows, then rows 0,1 make half 0 and rows 2,3 half 1.
template <class Op>
__device__ __forceinline__ void halves_reduce(int v, Op op, int& r0, int& r1)
{
    v = op(v, __builtin_amdgcn_mov_dpp(v, 0xB1, 0xF, 0xF, false));
    v = op(v, __builtin_amdgcn_mov_dpp(v, 0x4E, 0xF, 0xF, false));
    v = op(v, __builtin_amdgcn_mov_dpp(v, 0x141, 0xF, 0xF, false));
    v = op(v, __builtin_amdgcn_mov_dpp(v, 0x140, 0xF, 0xF, false));
    r0 = op(__builtin_amdgcn_readlane(v, 0), __builtin_amdgcn_readlane(v, 16));
    r1 = op(__builtin_amdgcn_readlane(v, 32), __builtin_amdgcn_readlane(v, 48));
}

__device__ __forceinline__ uint32_t lo32(uint64_t m) { return (uint32_t)m; }
__device__ __forceinline__ uint32_t hi32(uint64_t m) { return (uint32_t)(m >> 32); }

// Sorted unique keys of both halves (half 0 first) over the FxF footprints
// with upper-left taps (ox, oy); returns the total and the number of half-0
// keys in n0.
template <int F>
__device__ int w32_list_sorted(W32Lds<F>& L, bool inA, int h, int ox, int oy, int xmin, int ymin, int& n0)
{
    constexpr int N = kWave * F * F;
    const int lane = lane_id();
#pragma unroll
    for (int q = 0; q < F * F; ++q) {
        uint64_t key = ~0ull;
        if (inA)
            key = ((uint64_t)h << 62) | ((uint64_t)(uint32_t)(oy + q / F - ymin) << 32) |
                  (uint32_t)(ox + q % F - xmin);
        L.keys[F * F * lane + q] = key;
    }
    for (int size = 2; size <= N; size <<= 1)
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            wave_lds_sync();
#pragma unroll
            for (int hh = 0; hh < N / (2 * kWave); ++hh) {
                const int p = lane + kWave * hh;
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
    int base = 0;
    n0 = 0;
    for (int c = 0; c < N / kWave; ++c) {
        wave_lds_sync();
        const int i = kWave * c + lane;
        const uint64_t k = L.keys[i];
        const bool first = k != ~0ull && (i == 0 || L.keys[i - 1] != k);
        const uint64_t b = ballot(first);
        n0 += popc64(ballot(first && (k >> 62) == 0));
        wave_lds_sync();
        if (first) L.keys[base + mbcnt(b)] = k;
        base += popc64(b);
    }
    wave_lds_sync();
    return base;
}

template <int F>
__device__ __forceinline__ int w32_find(const W32Lds<F>& L, int lo, int hi, uint64_t key)
{
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (L.keys[mid] < key) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// Fallbacks C and C+ (Section 3.4, Eq. 1 and Eq. 2) per half-wave: the
// wave64 planning of fallback.h with every ballot, rank and table taken over
// the lanes of one 8x4 tile, so Eq. 2 spreads the spare lanes of a 32-lane
// wave as the paper writes it.  `fbl`: this lane's half takes the fallback.
struct W32Fallback {
    bool produces;
    int2 texel;
    int slot;
    bool table;
};

template <int FILTER, int F>
__device__ W32Fallback plan_fallback_w32(W32Lds<F>& L, int fb, bool fbl, bool inA, int h, int nA, int rankA,
                                         const Footprint& f, int2 pick, uint32_t h3, bool fits16, int xmin, int ymin,
                                         uint64_t Hm, int& nprod0, int& nprod1)
{
    const int lane = lane_id(), ll = lane & 31;
    const bool mine = fbl && inA;
    W32Fallback P;
    P.produces = mine;
    P.texel = pick;
    P.table = fits16;
    if (fb == CTF_FB_CPLUS && ballot(fbl && fits16) != 0) {
        const bool cplus = fbl && fits16;
        reinterpret_cast<uint32_t*>(L.bytes)[lane] = 0u;
        reinterpret_cast<uint32_t*>(L.bytes)[kWave + lane] = 0u;
        L.stash[h][ll] = StashEntry{f.x0, f.y0, f.s, f.t};
        wave_lds_sync();
        if (mine && cplus) L.bytes[h][16 * (pick.y - ymin) + (pick.x - xmin)] = 1;
        wave_lds_sync();
        // S per half: the distinct drawn texels of its lanes of A
        uint64_t S0[4], S1[4];
#pragma unroll
        for (int w = 0; w < 4; ++w) {
            const uint64_t b0 = ballot(L.bytes[h][64 * w + ll] != 0);
            const uint64_t b1 = ballot(L.bytes[h][64 * w + 32 + ll] != 0);
            S0[w] = (uint64_t)lo32(b0) | ((uint64_t)lo32(b1) << 32);
            S1[w] = (uint64_t)hi32(b0) | ((uint64_t)hi32(b1) << 32);
        }
        int ns0 = 0, ns1 = 0;
#pragma unroll
        for (int hh = 0; hh < 2; ++hh) {
            const uint64_t* Sh = hh ? S1 : S0;
            int base = 0;
#pragma unroll
            for (int w = 0; w < 4; ++w) {
                if ((Sh[w] >> lane) & 1u) L.items[hh][base + mbcnt(Sh[w])] = (uint16_t)(64 * w + lane);
                base += popc64(Sh[w]);
            }
            if (hh) ns1 = base;
            else ns0 = base;
        }
        wave_lds_sync();
        // lane of each rank of A in its half (the bytes are free after the ballots)
        if (inA) L.bytes[h][rankA] = (uint8_t)ll;
        wave_lds_sync();
        if (mine && cplus) {
            const int ns = h ? ns1 : ns0;
            P.produces = false;
            if (rankA < ns) {
                const int t = L.items[h][rankA];
                P.produces = true;
                P.texel = make_int2(xmin + (t & 15), ymin + (t >> 4));
            } else {
                constexpr int O = Taps<FILTER>::O;
                const StashEntry T = L.stash[h][L.bytes[h][cplus_target(nA, ns, rankA)]];
                float wx[4], wy[4];
                taps32<FILTER>(T.s, wx);
                taps32<FILTER>(T.t, wy);
                const int ox = T.x0 - O, oy = T.y0 - O;
                // candidates: taps (row-major) with a nonzero weight, not in S
                uint32_t cand = 0u;
                float wsum = 0.f;
#pragma unroll
                for (int q = 0; q < F * F; ++q) {
                    const float wq = wx[q % F] * wy[q / F];
                    const int tq = 16 * (oy + q / F - ymin) + (ox + q % F - xmin);
                    const uint64_t Sw = h ? S1[tq >> 6] : S0[tq >> 6];
                    if (wq != 0.0f && !((Sw >> (tq & 63)) & 1u)) {
                        cand |= 1u << q;
                        wsum += __builtin_fabsf(wq);
                    }
                }
                if (cand) {
                    const float thr = (float)(h3 >> 8) * 0x1p-24f * wsum;
                    float run = 0.f;
                    int pq = -1;
                    bool done = false;
#pragma unroll
                    for (int q = 0; q < F * F; ++q) {
                        if (!((cand >> q) & 1u) || done) continue;
                        pq = q;
                        run += __builtin_fabsf(wx[q % F] * wy[q / F]);
                        done = run > thr;
                    }
                    P.produces = true;
                    P.texel = make_int2(ox + pq % F, oy + pq / F);
                }
            }
        }
    }
    const uint64_t prod = ballot(P.produces);
    nprod0 = __popc(lo32(prod));
    nprod1 = __popc(hi32(prod));
    P.slot = mbcnt(prod & Hm);
    // slot table of the fallback halves (the other half keeps its rank table)
    if (fbl && fits16) {
        reinterpret_cast<uint32_t*>(L.rank[h])[ll] = 0u;
        reinterpret_cast<uint32_t*>(L.rank[h])[32 + ll] = 0u;
    }
    wave_lds_sync();
    if (P.produces) {
        if (P.table) L.rank[h][16 * (P.texel.y - ymin) + (P.texel.x - xmin)] = (uint8_t)(P.slot + 1);
        else L.produced[h][P.slot] = P.texel;
    }
    wave_lds_sync();
    return P;
}

// Eq. 1 for a lane of A of a fallback half (fallback_color of fallback.h over
// this half's slots).
template <int FILTER, int F>
__device__ float4 fallback_color_w32(const W32Lds<F>& L, const W32Fallback& P, int h, int nprod, const Footprint& f,
                                     int2 pick, int xmin, int ymin)
{
    constexpr int O = Taps<FILTER>::O;
    float wx[4], wy[4];
    taps32<FILTER>(f.s, wx);
    taps32<FILTER>(f.t, wy);
    float4 acc = make_float4(0.f, 0.f, 0.f, 0.f), sum = acc;
    float wsum = 0.f;
    int N = 0, own = 0;
#pragma unroll
    for (int q = 0; q < F * F; ++q) {
        const int x = f.x0 - O + q % F, y = f.y0 - O + q / F;
        const float wq = wx[q % F] * wy[q / F];
        int slot = -1;
        if (P.table) {
            slot = (int)L.rank[h][16 * (y - ymin) + (x - xmin)] - 1;
        } else {
            for (int r = 0; r < nprod; ++r) {
                const int2 e = L.produced[h][r];
                if (e.x == x && e.y == y) {
                    slot = r;
                    break;
                }
            }
        }
        if (x == pick.x && y == pick.y) own = slot;
        if (slot < 0 || wq == 0.0f) continue;
        const float4 v = L.vals[h][slot];
        acc.x = __builtin_fmaf(wq, v.x, acc.x);
        acc.y = __builtin_fmaf(wq, v.y, acc.y);
        acc.z = __builtin_fmaf(wq, v.z, acc.z);
        acc.w = __builtin_fmaf(wq, v.w, acc.w);
        sum.x += v.x;
        sum.y += v.y;
        sum.z += v.z;
        sum.w += v.w;
        wsum += wq;
        ++N;
    }
    if (N == 0) return L.vals[h][own];
    const float inv = 1.0f / (float)N, rest = 1.0f - wsum;
    return make_float4(__builtin_fmaf(rest, sum.x * inv, acc.x), __builtin_fmaf(rest, sum.y * inv, acc.y),
                       __builtin_fmaf(rest, sum.z * inv, acc.z), __builtin_fmaf(rest, sum.w * inv, acc.w));
}

struct HalfDecision {
    int n, unique;
    bool cap_ok, count_ok, success;
};

template <int METHOD, int TEX, bool STATS, int FILTER, bool FB>
__global__ __launch_bounds__(kWave * kW32Waves) void k_filter_w32(FilterArgs a, DevTexture T)
{
    constexpr int F = Taps<FILTER>::F, O = Taps<FILTER>::O;
    __shared__ W32Lds<F> lds_all[kW32Waves];
    __shared__ int4 terms_lds[TEX == CTF_TEX_SINUSOIDS && (METHOD == CTF_BILINEAR4 || METHOD == CTF_STF1)
                                  ? kLdsTermEntries
                                  : 1];
    const int wid = wave_in_block();
    const int lane = lane_id();
    const int h = lane >> 5, ll = lane & 31;
    W32Lds<F>& L = lds_all[wid];
    // Terms from LDS for the 4-tap and one-tap kernels; the collaborative
    // ones keep them in scalar registers (the LDS copy and the extra vector
    // registers cost them occupancy: List 8x4 at 1080p 21.3 against 24.0
    // Gpixels/s)
    constexpr bool kStage = TEX == CTF_TEX_SINUSOIDS && (METHOD == CTF_BILINEAR4 || METHOD == CTF_STF1);
    bool lds_float = false;
    if constexpr (kStage) lds_float = stage_terms(T, terms_lds) && T.fterms != nullptr;
    auto texel = [&](int x, int y) __attribute__((always_inline)) -> float4 {
        if constexpr (kStage) return texel_eval_staged<TEX>(T, terms_lds, lds_float, x, y);
        else return texel_eval<TEX>(T, x, y);
    };
    FrameCounters fc;
    const int64_t npairs = (a.ntiles + 1) / 2;
    const int64_t nw = (int64_t)gridDim.x * kW32Waves;
    for (int64_t pair = (int64_t)blockIdx.x * kW32Waves + wid; pair < npairs; pair += nw) {
        const int64_t tile = 2 * pair + h;
        const bool tile_ok = tile < a.ntiles;
        const int tx = tile_ok ? (int)(tile % a.tiles_x) : 0, ty = tile_ok ? (int)(tile / a.tiles_x) : 0;
        const int px = tx * 8 + (ll & 7), py = ty * 4 + (ll >> 3);
        const bool in_screen = tile_ok && px < a.sw && py < a.sh;
        const int64_t pix = (int64_t)py * a.sw + px;

        Footprint f;
        {
            float2 uv = make_float2(__builtin_nanf(""), 0.f);
            float4 d = make_float4(0.f, 0.f, 0.f, 0.f);
            if (in_screen) {
                uv = reinterpret_cast<const float2*>(a.uv)[pix];
                d = reinterpret_cast<const float4*>(a.duv)[pix];
            }
            f = footprint(uv.x, uv.y, d, (float)T.width, (float)T.height);
        }
        const bool inA = f.active && f.magnify;
        const int ox = f.x0 - O, oy = f.y0 - O;   // upper-left tap of the FxF footprint
        const uint64_t act = ballot(f.active);
        const uint64_t Aw = ballot(inA);
        const uint64_t Hm = h ? 0xffffffff00000000ull : 0x00000000ffffffffull;
        const uint64_t A = Aw & Hm;
        const int nA0 = __popc(lo32(Aw)), nA1 = __popc(hi32(Aw));
        const int nA = h ? nA1 : nA0;
        const int rankA = mbcnt(A);

        // ---- box per half
        int xmin0 = 0, ymin0 = 0, xmax0 = -1, ymax0 = -1, xmin1 = 0, ymin1 = 0, xmax1 = -1, ymax1 = -1;
        constexpr bool kCollab = METHOD == CTF_LIST || METHOD == CTF_BOX || METHOD == CTF_MASK;
        if ((kCollab || STATS) && (nA0 | nA1)) {
            halves_reduce(inA ? ox : INT32_MAX, MinOp(), xmin0, xmin1);
            halves_reduce(inA ? oy : INT32_MAX, MinOp(), ymin0, ymin1);
            halves_reduce(inA ? ox + F - 1 : INT32_MIN, MaxOp(), xmax0, xmax1);
            halves_reduce(inA ? oy + F - 1 : INT32_MIN, MaxOp(), ymax0, ymax1);
        }
        const int bbw0 = nA0 ? xmax0 - xmin0 + 1 : 0, bbh0 = nA0 ? ymax0 - ymin0 + 1 : 0;
        const int bbw1 = nA1 ? xmax1 - xmin1 + 1 : 0, bbh1 = nA1 ? ymax1 - ymin1 + 1 : 0;
        if (!nA0) xmin0 = ymin0 = 0;
        if (!nA1) xmin1 = ymin1 = 0;
        const bool fits0 = nA0 > 0 && bbw0 <= 16 && bbh0 <= 16;
        const bool fits1 = nA1 > 0 && bbw1 <= 16 && bbh1 <= 16;
        const int xmin = h ? xmin1 : xmin0, ymin = h ? ymin1 : ymin0;
        const int bbw = h ? bbw1 : bbw0;
        const bool fits16 = h ? fits1 : fits0;

        // ---- 16x16 masks per half: corner bytes, 8 ballots, corner spread
        uint64_t B0[4] = {0, 0, 0, 0}, B1[4] = {0, 0, 0, 0};
        int nmask0 = 0, nmask1 = 0;
        constexpr bool kNeedMask = METHOD == CTF_MASK || METHOD == CTF_LIST || STATS;
        if (kNeedMask && (fits0 || fits1)) {
            reinterpret_cast<uint32_t*>(L.bytes)[lane] = 0u;
            reinterpret_cast<uint32_t*>(L.bytes)[kWave + lane] = 0u;
            wave_lds_sync();
            if (inA && fits16) L.bytes[h][16 * (oy - ymin) + (ox - xmin)] = 1;
            wave_lds_sync();
            uint64_t C0[4], C1[4];
#pragma unroll
            for (int w = 0; w < 4; ++w) {
                const uint64_t b0 = ballot(L.bytes[h][64 * w + ll] != 0);
                const uint64_t b1 = ballot(L.bytes[h][64 * w + 32 + ll] != 0);
                C0[w] = (uint64_t)lo32(b0) | ((uint64_t)lo32(b1) << 32);
                C1[w] = (uint64_t)hi32(b0) | ((uint64_t)hi32(b1) << 32);
            }
            if (fits0) footprint_mask_f<F>(C0, B0);
            if (fits1) footprint_mask_f<F>(C1, B1);
#pragma unroll
            for (int hh = 0; hh < 2; ++hh) {
                const uint64_t* Bh = hh ? B1 : B0;
                int base = 0;
#pragma unroll
                for (int w = 0; w < 4; ++w) {
                    if ((Bh[w] >> lane) & 1u) {
                        const int r = base + mbcnt(Bh[w]);
                        L.items[hh][r] = (uint16_t)(64 * w + lane);
                        L.rank[hh][64 * w + lane] = (uint8_t)r;
                    }
                    base += popc64(Bh[w]);
                }
                if (hh) nmask1 = base;
                else nmask0 = base;
            }
            wave_lds_sync();
        }

        // ---- the method's decision, per half
        const int k = a.max_evals;
        HalfDecision D[2];
        bool sorted = false;
        int n0s = 0, ntot = 0;
        if constexpr (METHOD == CTF_LIST) {
            if ((nA0 && !fits0) || (nA1 && !fits1)) {
                ntot = w32_list_sorted<F>(L, inA, h, ox, oy, xmin, ymin, n0s);
                sorted = true;
            }
        }
#pragma unroll
        for (int hh = 0; hh < 2; ++hh) {
            const int nAh = hh ? nA1 : nA0, bw = hh ? bbw1 : bbw0, bh = hh ? bbh1 : bbh0;
            const bool fh = hh ? fits1 : fits0;
            const int nm = hh ? nmask1 : nmask0;
            HalfDecision& d = D[hh];
            d.cap_ok = true;
            d.count_ok = true;
            d.success = false;
            d.n = 0;
            d.unique = fh ? nm : 0;
            if constexpr (METHOD == CTF_BOX) {
                const int64_t area = (int64_t)bw * bh;
                d.n = area > INT32_MAX ? INT32_MAX : (int)area;
                d.cap_ok = (a.box_w == 0 || bw <= a.box_w) && (a.box_h == 0 || bh <= a.box_h);
                d.count_ok = area <= (int64_t)k * nAh;
                d.success = nAh > 0 && d.cap_ok && d.count_ok;
            } else if constexpr (METHOD == CTF_MASK) {
                d.cap_ok = fh;
                d.n = fh ? nm : 0;
                d.count_ok = d.n <= k * nAh;
                d.success = fh && d.count_ok;
            } else if constexpr (METHOD == CTF_LIST) {
                d.n = (nAh && !fh) ? (hh ? ntot - n0s : n0s) : nm;
                d.unique = d.n;
                d.count_ok = d.n <= k * nAh;
                d.success = nAh > 0 && d.count_ok;
            }
        }
        if constexpr (STATS && METHOD != CTF_LIST) {
            if ((nA0 && !fits0) || (nA1 && !fits1)) {
                int n0u = 0;
                const int nu = w32_list_sorted<F>(L, inA, h, ox, oy, xmin, ymin, n0u);
                if (nA0 && !fits0) D[0].unique = n0u;
                if (nA1 && !fits1) D[1].unique = nu - n0u;
            }
        }
        if (!nA0) D[0].unique = 0;
        if (!nA1) D[1].unique = 0;
        const int n = h ? D[1].n : D[0].n;
        const bool success = h ? D[1].success : D[0].success;
        const bool half_sorted = sorted && nA > 0 && !fits16;
        const int key_off = h ? n0s : 0;

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
        const uint64_t stfw = ballot(draws);

        // ---- production: each lane evaluates at most one texel per round
        float4 res = make_float4(0.f, 0.f, 0.f, 0.f);
        int2 pick = make_int2(INT32_MIN, INT32_MIN);
        uint32_t h1 = 0, h2 = 0;
        if (draws) {
            stf_hashes(a.seed, a.layer, px, py, h1, h2);
            pick = stf_pick_filter<FILTER>(f, h1, h2);
        }
        // fallback C / C+ for the lanes of A of a failed half
        bool fbl = false;
        W32Fallback P{};
        int nprod0 = 0, nprod1 = 0;
        if constexpr (FB && kCollab) {
            fbl = !success && nA > 0;
            if (ballot(fbl) != 0)
                P = plan_fallback_w32<FILTER, F>(L, a.fallback, fbl, inA, h, nA, rankA, f, pick, pcg_hash(h2), fits16,
                                                  xmin, ymin, Hm, nprod0, nprod1);
        }
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
        } else {
            for (int round = 0; round < (kCollab ? k : 1); ++round) {
                const int item = rankA + round * nA;
                const bool produce = kCollab && success && inA && item < n;
                const bool draw_now = draws && round == 0 && !(fbl && inA);
                if (ballot(produce || draw_now) == 0) break;
                int ex = pick.x, ey = pick.y;
                if (produce) {
                    if constexpr (METHOD == CTF_BOX) {
                        ex = xmin + item % bbw;
                        ey = ymin + item / bbw;
                    } else {
                        if (half_sorted) {
                            const uint64_t key = L.keys[key_off + item];
                            ex = xmin + (int)(uint32_t)key;
                            ey = ymin + (int)((key >> 32) & 0x3fffffffu);
                        } else {
                            const int t = L.items[h][item];
                            ex = xmin + (t & 15);
                            ey = ymin + (t >> 4);
                        }
                    }
                    if (STATS && a.lists) reinterpret_cast<int2*>(a.lists)[(size_t)tile * kMaxItems + item] = make_int2(ex, ey);
                }
                if (produce || draw_now) {
                    const float4 v = texel(ex, ey);
                    if (produce) L.vals[h][item] = v;
                    if (draw_now) res = v;
                }
            }
            if constexpr (FB && kCollab) {
                // the fallback halves' planned texels, then Eq. 1
                if (fbl && inA && P.produces) L.vals[h][P.slot] = texel(P.texel.x, P.texel.y);
                wave_lds_sync();
                if (fbl && inA) res = fallback_color_w32<FILTER, F>(L, P, h, h ? nprod1 : nprod0, f, pick, xmin, ymin);
            }
            if constexpr (kCollab) {
                wave_lds_sync();
                if (exact) {
                    // item index of tap (i, j) of this half's list
                    auto item_of = [&](int i, int j) -> int {
                        if constexpr (METHOD == CTF_BOX) {
                            return (ox + i - xmin) + (oy + j - ymin) * bbw;
                        } else {
                            if (half_sorted) {
                                const uint64_t key = ((uint64_t)h << 62) |
                                                     ((uint64_t)(uint32_t)(oy + j - ymin) << 32) |
                                                     (uint32_t)(ox + i - xmin);
                                return w32_find<F>(L, key_off, key_off + n, key) - key_off;
                            }
                            return L.rank[h][16 * (oy + j - ymin) + (ox + i - xmin)];
                        }
                    };
                    if constexpr (F == 2) {
                        res = bilerp(f.s, f.t, L.vals[h][item_of(0, 0)], L.vals[h][item_of(1, 0)],
                                     L.vals[h][item_of(0, 1)], L.vals[h][item_of(1, 1)]);
                    } else {
                        float wx[4], wy[4];
                        taps32<FILTER>(f.s, wx);
                        taps32<FILTER>(f.t, wy);
#pragma unroll
                        for (int j = 0; j < 4; ++j) {
                            const float4 r = row4(wx, L.vals[h][item_of(0, j)], L.vals[h][item_of(1, j)],
                                                  L.vals[h][item_of(2, j)], L.vals[h][item_of(3, j)]);
                            res = col_acc(wy[j], r, res, j == 0);
                        }
                    }
                }
            }
        }

        // ---- outputs, per-tile records (lanes 0 and 32), frame counters
        if (in_screen) {
            reinterpret_cast<float4*>(a.out)[pix] = res;
            if (a.stf_xy)
                reinterpret_cast<int2*>(a.stf_xy)[pix] = draws ? pick : make_int2(INT32_MIN, INT32_MIN);
        }
        int evals[2];
        const uint32_t actm[2] = {lo32(act), hi32(act)}, stfm[2] = {lo32(stfw), hi32(stfw)};
        const uint32_t Am[2] = {lo32(Aw), hi32(Aw)};
#pragma unroll
        for (int hh = 0; hh < 2; ++hh) {
            if constexpr (METHOD == CTF_BILINEAR4) evals[hh] = F * F * __popc(actm[hh]);
            else if (FB && kCollab && !D[hh].success && __popc(Am[hh]) > 0)
                evals[hh] = (hh ? nprod1 : nprod0) + __popc(stfm[hh] & ~Am[hh]);
            else evals[hh] = (D[hh].success ? D[hh].n : 0) + __popc(stfm[hh]);
        }
        if (STATS && ll == 0 && tile_ok && a.tile_stats) {
            const HalfDecision& d = D[h];
            const uint64_t* Bh = h ? B1 : B0;
            ctf_tile_stats S;
            S.active = actm[h];
            S.part = Am[h];
            S.stf = stfm[h];
            for (int w = 0; w < 4; ++w) S.mask[w] = fits16 ? Bh[w] : 0ull;
            S.xmin = xmin;
            S.ymin = ymin;
            S.bbw = h ? bbw1 : bbw0;
            S.bbh = h ? bbh1 : bbh0;
            S.n = d.n;
            S.unique = d.unique;
            S.evals = evals[h];
            S.flags = (d.success ? CTF_TILE_OK : 0) | (nA && !d.cap_ok ? CTF_TILE_CAP : 0) |
                      (nA && d.cap_ok && !d.count_ok ? CTF_TILE_OVERFLOW : 0) | (nA == 0 ? CTF_TILE_EMPTY : 0);
            for (int r = 0; r < 10; ++r) S.reserved[r] = 0;
            a.tile_stats[tile] = S;
        }
#pragma unroll
        for (int hh = 0; hh < 2; ++hh)
            if (actm[hh])
                fc.add(evals[hh], __popc(actm[hh]), __popc(stfm[hh]), __popc(actm[hh] & ~Am[hh]), 0,
                       kCollab && D[hh].success, kCollab && Am[hh] && !D[hh].success);
        wave_lds_sync();  // the next pair reuses this wave's LDS slice
    }
    if (lane == 0 && a.frame_stats) fc.flush(a.frame_stats);
}

template <int METHOD, int TEX, int FILTER>
hipError_t launch_w32_m_t(const FilterArgs& a, const DevTexture& T, hipStream_t s)
{
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    const int64_t npairs = (a.ntiles + 1) / 2;
    int64_t blocks = (npairs + kW32Waves - 1) / kW32Waves;
    if (blocks > (int64_t)cus * 8) blocks = (int64_t)cus * 8;
    const int64_t least = counter_min_blocks(a.ntiles, kW32Waves);   // 32-bit frame counters
    if (blocks < least) blocks = least;
    const dim3 grid((unsigned)blocks), block(kWave * kW32Waves);
    constexpr bool kCollab = METHOD == CTF_LIST || METHOD == CTF_BOX || METHOD == CTF_MASK;
    // the instantiation with statistics also writes the texel lists
    const bool st = a.tile_stats != nullptr || a.lists != nullptr;
    if (kCollab && a.fallback != CTF_FB_STF1) {
        if (st) hipLaunchKernelGGL((k_filter_w32<METHOD, TEX, true, FILTER, kCollab>), grid, block, 0, s, a, T);
        else hipLaunchKernelGGL((k_filter_w32<METHOD, TEX, false, FILTER, kCollab>), grid, block, 0, s, a, T);
    } else {
        if (st) hipLaunchKernelGGL((k_filter_w32<METHOD, TEX, true, FILTER, false>), grid, block, 0, s, a, T);
        else hipLaunchKernelGGL((k_filter_w32<METHOD, TEX, false, FILTER, false>), grid, block, 0, s, a, T);
    }
    return hipGetLastError();
}

template <int TEX, int FILTER>
hipError_t launch_w32_tf(const FilterArgs& a, const DevTexture& T, hipStream_t s)
{
    switch (a.method) {
    case CTF_BILINEAR4: return launch_w32_m_t<CTF_BILINEAR4, TEX, FILTER>(a, T, s);
    case CTF_STF1: return launch_w32_m_t<CTF_STF1, TEX, FILTER>(a, T, s);
    case CTF_LIST: return launch_w32_m_t<CTF_LIST, TEX, FILTER>(a, T, s);
    case CTF_BOX: return launch_w32_m_t<CTF_BOX, TEX, FILTER>(a, T, s);
    case CTF_MASK: return launch_w32_m_t<CTF_MASK, TEX, FILTER>(a, T, s);
    default: return hipErrorInvalidValue;
    }
}

template <int TEX>
hipError_t launch_w32_t(const FilterArgs& a, const DevTexture& T, hipStream_t s)
{
    switch (a.filter) {
    case CTF_FILTER_BILINEAR: return launch_w32_tf<TEX, CTF_FILTER_BILINEAR>(a, T, s);
    case CTF_FILTER_BSPLINE: return launch_w32_tf<TEX, CTF_FILTER_BSPLINE>(a, T, s);
    case CTF_FILTER_CATMULL_ROM: return launch_w32_tf<TEX, CTF_FILTER_CATMULL_ROM>(a, T, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace

hipError_t launch_filter_w32(const FilterArgs& a, const DevTexture& T, hipStream_t s)
{
    switch (T.kind) {
    case CTF_TEX_SINUSOIDS: return launch_w32_t<CTF_TEX_SINUSOIDS>(a, T, s);
    case CTF_TEX_AFFINE: return launch_w32_t<CTF_TEX_AFFINE>(a, T, s);
    case CTF_TEX_CONSTANT: return launch_w32_t<CTF_TEX_CONSTANT>(a, T, s);
    case CTF_TEX_TABLE: return launch_w32_t<CTF_TEX_TABLE>(a, T, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace ctf
