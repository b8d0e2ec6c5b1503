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
//       proportional to its float32 weight among that footprint's texels
//       not in S (the last such texel if the running sum never passes the
//       threshold); a lane whose target has no such texel produces nothing.
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

__device__ __forceinline__ void weights32(float s, float t, float w[4])
{
    const float is = 1.0f - s, it = 1.0f - t;
    w[0] = is * it;
    w[1] = s * it;
    w[2] = is * t;
    w[3] = s * t;
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
template <class LDS>
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
            const StashEntry T = stash[L.bytes[cplus_target(nA, ns, rankA)]];
            float w[4];
            weights32(T.s, T.t, w);
            float wsum = 0.f;
            bool cand[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int tq = 16 * (T.y0 + (q >> 1) - ymin) + (T.x0 + (q & 1) - xmin);
                cand[q] = w[q] > 0.0f && !((S[tq >> 6] >> (tq & 63)) & 1u);
                if (cand[q]) wsum += w[q];
            }
            if (wsum > 0.0f) {
                const float thr = (float)(h3 >> 8) * 0x1p-24f * wsum;
                float run = 0.f;
                int pq = -1;
                bool done = false;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    if (!cand[q] || done) continue;
                    pq = q;
                    run += w[q];
                    done = run > thr;
                }
                P.produces = true;
                P.texel = make_int2(T.x0 + (pq & 1), T.y0 + (pq >> 1));
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
// the produced texels of its footprint with a nonzero float32 weight,
// weighted, plus their mean times the weight of the missing texels.  If no
// texel qualifies (the drawn texel's weight underflowed to zero) the drawn
// texel's value is returned.
template <class LDS>
__device__ float4 fallback_color(const LDS& L, const FallbackPlan& P, const Footprint& f, int2 pick, int xmin,
                                 int ymin)
{
    const int2* produced = reinterpret_cast<const int2*>(L.keys);
    float w[4];
    weights32(f.s, f.t, w);
    float4 acc = make_float4(0.f, 0.f, 0.f, 0.f), sum = acc;
    float wsum = 0.f;
    int N = 0, own = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int x = f.x0 + (q & 1), y = f.y0 + (q >> 1);
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
        if (slot < 0 || !(w[q] > 0.0f)) continue;
        const float4 v = L.vals[slot];
        acc.x = __builtin_fmaf(w[q], v.x, acc.x);
        acc.y = __builtin_fmaf(w[q], v.y, acc.y);
        acc.z = __builtin_fmaf(w[q], v.z, acc.z);
        acc.w = __builtin_fmaf(w[q], v.w, acc.w);
        sum.x += v.x;
        sum.y += v.y;
        sum.z += v.z;
        sum.w += v.w;
        wsum += w[q];
        ++N;
    }
    if (N == 0) return L.vals[own];
    const float inv = 1.0f / (float)N, rest = 1.0f - wsum;
    return make_float4(__builtin_fmaf(rest, sum.x * inv, acc.x), __builtin_fmaf(rest, sum.y * inv, acc.y),
                       __builtin_fmaf(rest, sum.z * inv, acc.z), __builtin_fmaf(rest, sum.w * inv, acc.w));
}

}  // namespace ctf
