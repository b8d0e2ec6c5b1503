// fallback.h -- fallbacks C and C+ for the lanes of a wave whose
// collaborative step failed (Section 3.4, Eq. 1 and Eq. 2).
//
// Only the participating lanes A of a failed wave use them; minifying lanes
// keep the one-tap draw.  Every lane of A draws its one-tap texel first.
//   C:  every lane of A produces its drawn texel.
//   C+: the distinct drawn texels (mask S, one bit per texel) are produced
//       once, by the lanes of rank 0..|S|-1 in A; each remaining lane of
//       rank c adds a texel of the footprint of the lane of rank
//       round((|A|-1)(c-|S|)/(|A|-1-|S|)) (Eq. 2), drawn with probability
//       proportional to the absolute value of its float32 weight among that
//       footprint's nonzero-weight texels not in S (the last such texel if
//       the running sum never passes the threshold); a lane whose target
//       has no such texel produces nothing.
//       C+ needs the wave box to fit the 16x16 mask; otherwise C is used.
// Each lane of A then weights the produced texels of its footprint that
// have a nonzero float32 weight with Eq. 1.
//
// The producing lanes are compacted: the lane of rank r among them writes
// slot r of the wave's value array.  With the box inside 16x16 a 256-entry
// byte table maps a mask position to (slot + 1) of a lane that produced that
// texel; past 16x16 (fallback C only) the drawn texels are kept by slot and
// searched linearly.
#pragma once

#include "ctf_device.h"

namespace ctf {

// rank of the lane whose footprint spare lane c adds a texel from (Eq. 2,
// rounding half up; a single spare lane maps to rank 0)
__device__ __forceinline__ int cplus_target(int nA, int ns, int c)
{
    const int span = nA - 1 - ns;
    return span <= 0 ? 0 : (2 * (nA - 1) * (c - ns) + span) / (2 * span);
}

struct FallbackPlan {
    bool produces;   // this lane evaluates a texel
    int2 texel;      // ... this one
    int slot;        // ... into this slot of the value array
    int nprod;       // number of producing lanes (the wave's fallback evaluations)
    bool table;      // slots found through the 16x16 position table
};

struct StashEntry {  // a lane's footprint, read by the spare lanes of C+
    int x0, y0;
    float s, t;
};

// Plans the productions of a failed wave.  fb is CTF_FB_C or CTF_FB_CPLUS;
// C+ falls back to C when the box exceeds 16x16.  LDS is the kernel's
// per-wave struct; its members keys (>= 2 KB), rank and bytes (256 bytes
// each) are overwritten.  h3 is this lane's third hash of the draw chain.
template <int FILTER, class LDS>
__device__ FallbackPlan plan_fallback(LDS& L, int fb, bool inA, int nA, int rankA, const Footprint& f, int2 pick,
                                      uint32_t h3, bool fits16, int xmin, int ymin)
{
    const int lane = lane_id();
    FallbackPlan P;
    P.produces = inA;
    P.texel = pick;
    P.table = fits16;
    if (fb == CTF_FB_CPLUS && fits16) {
        // mask S of the drawn texels
        StashEntry* stash = reinterpret_cast<StashEntry*>(L.keys);           // 64 x 16 B
        uint16_t* sitems = reinterpret_cast<uint16_t*>(L.keys + 128);       // 64 x 2 B
        reinterpret_cast<uint32_t*>(L.bytes)[lane] = 0u;
        stash[lane] = StashEntry{f.x0, f.y0, f.s, f.t};
        wave_lds_sync();
        if (inA) L.bytes[16 * (pick.y - ymin) + (pick.x - xmin)] = 1;
        wave_lds_sync();
        uint64_t S[4];
#pragma unroll
        for (int w = 0; w < 4; ++w) S[w] = ballot(L.bytes[64 * w + lane] != 0);
        int ns = 0;
#pragma unroll
        for (int w = 0; w < 4; ++w) {
            if ((S[w] >> lane) & 1u) sitems[ns + mbcnt(S[w])] = (uint16_t)(64 * w + lane);
            ns += popc64(S[w]);
        }
        wave_lds_sync();
        // lane of each rank of A (the bytes array is free after the ballots)
        if (inA) L.bytes[rankA] = (uint8_t)lane;
        wave_lds_sync();
        P.produces = false;
        if (inA && rankA < ns) {
            const int t = sitems[rankA];
            P.produces = true;
            P.texel = make_int2(xmin + (t & 15), ymin + (t >> 4));
        } else if (inA) {
            constexpr int F = Taps<FILTER>::F, O = Taps<FILTER>::O;
            const StashEntry T = stash[L.bytes[cplus_target(nA, ns, rankA)]];
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
                if (wq != 0.0f && !((S[tq >> 6] >> (tq & 63)) & 1u)) {
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
    const uint64_t prod = ballot(P.produces);
    P.nprod = popc64(prod);
    P.slot = mbcnt(prod);
    if (fits16) {
        reinterpret_cast<uint32_t*>(L.rank)[lane] = 0u;
        wave_lds_sync();
        if (P.produces) L.rank[16 * (P.texel.y - ymin) + (P.texel.x - xmin)] = (uint8_t)(P.slot + 1);
    } else if (P.produces) {
        reinterpret_cast<int2*>(L.keys)[P.slot] = P.texel;
    }
    wave_lds_sync();
    return P;
}

// Eq. 1 for a lane of A, once the produced values are in vals[0..nprod):
// among its footprint's FxF taps (signed float32 weights wx_i wy_j), the
// produced texels with a nonzero weight, weighted, plus their mean times the
// weight of the missing texels.  If no texel qualifies (the drawn texel's
// weight underflowed to zero) the drawn texel's value is returned.
template <int FILTER, class LDS>
__device__ float4 fallback_color(const LDS& L, const FallbackPlan& P, const Footprint& f, int2 pick, int xmin,
                                 int ymin)
{
    constexpr int F = Taps<FILTER>::F, O = Taps<FILTER>::O;
    const int2* produced = reinterpret_cast<const int2*>(L.keys);
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
            slot = (int)L.rank[16 * (y - ymin) + (x - xmin)] - 1;
        } else {
            for (int r = 0; r < P.nprod; ++r) {
                const int2 e = produced[r];
                if (e.x == x && e.y == y) {
                    slot = r;
                    break;
                }
            }
        }
        if (x == pick.x && y == pick.y) own = slot;
        if (slot < 0 || wq == 0.0f) continue;
        const float4 v = L.vals[slot];
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
    if (N == 0) return L.vals[own];
    const float inv = 1.0f / (float)N, rest = 1.0f - wsum;
    return make_float4(__builtin_fmaf(rest, sum.x * inv, acc.x), __builtin_fmaf(rest, sum.y * inv, acc.y),
                       __builtin_fmaf(rest, sum.z * inv, acc.z), __builtin_fmaf(rest, sum.w * inv, acc.w));
}

}  // namespace ctf
