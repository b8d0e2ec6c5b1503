// ctf_device.h -- device-side building blocks for gfx950 (wave64).
//
// Wave primitives, the per-lane bilinear footprint, the stochastic draw and
// the texel producers shared by every filter kernel.  Compiled with
// -ffp-contract=off: every fused multiply-add below is written explicitly so
// the float32 decisions are the ones the method fixes.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ctf.h"

namespace ctf {

constexpr int kWave = 64;
constexpr int kTile = 8;              // 8x8 pixels per wave
constexpr int kMaxItems = CTF_MAX_ITEMS;
constexpr float kRange = 16777216.0f; // |texel position| < 2^24

// ---------------------------------------------------------------------------
// wave primitives
// ---------------------------------------------------------------------------

__device__ __forceinline__ int lane_id() { return __lane_id(); }

// Index of this wave in its workgroup, as a wave-uniform (scalar) value so
// that everything derived from it (tile walks, layer loops) stays scalar.
__device__ __forceinline__ int wave_in_block() { return __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)); }

__device__ __forceinline__ uint64_t ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }

// number of set bits of m below this lane (rank of the lane in m)
__device__ __forceinline__ int mbcnt(uint64_t m)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

__device__ __forceinline__ int popc64(uint64_t m) { return __popcll(m); }

// Cross-lane LDS hand-off inside one wave: the wave's LDS instructions
// execute in order, so only compiler reordering has to be prevented.
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Wave-wide min / max (all 64 lanes must be active): DPP exchanges reduce
// each row of 16 lanes (quad_perm [1,0,3,2], quad_perm [2,3,0,1],
// row_half_mirror, row_mirror), then the four row results are read with
// v_readlane and combined as scalars.  The result is wave-uniform.
template <class Op>
__device__ __forceinline__ int wave_reduce(int v, Op op)
{
    v = op(v, __builtin_amdgcn_mov_dpp(v, 0xB1, 0xF, 0xF, false));
    v = op(v, __builtin_amdgcn_mov_dpp(v, 0x4E, 0xF, 0xF, false));
    v = op(v, __builtin_amdgcn_mov_dpp(v, 0x141, 0xF, 0xF, false));
    v = op(v, __builtin_amdgcn_mov_dpp(v, 0x140, 0xF, 0xF, false));
    const int r0 = __builtin_amdgcn_readlane(v, 0), r1 = __builtin_amdgcn_readlane(v, 16);
    const int r2 = __builtin_amdgcn_readlane(v, 32), r3 = __builtin_amdgcn_readlane(v, 48);
    return op(op(r0, r1), op(r2, r3));
}

struct MinOp {
    __device__ __forceinline__ int operator()(int a, int b) const { return a < b ? a : b; }
};
struct MaxOp {
    __device__ __forceinline__ int operator()(int a, int b) const { return a > b ? a : b; }
};

__device__ __forceinline__ int wave_min(int v) { return wave_reduce(v, MinOp()); }
__device__ __forceinline__ int wave_max(int v) { return wave_reduce(v, MaxOp()); }

// ---------------------------------------------------------------------------
// per-lane footprint (Section 3 and the supplement's code listings)
// ---------------------------------------------------------------------------

struct Footprint {
    bool active;   // finite, in-range texel position
    bool magnify;  // both screen-axis footprints span at most one texel
    int x0, y0;    // upper-left texel of the 2x2 footprint
    float s, t;    // position inside the footprint, in [0,1)
};

__device__ __forceinline__ Footprint footprint(float u, float v, float4 d, float W, float H)
{
    Footprint f;
    f.active = false;
    f.magnify = false;
    f.x0 = f.y0 = 0;
    f.s = f.t = 0.f;
    if (!__builtin_isfinite(u) || !__builtin_isfinite(v)) return f;
    const float fx = __builtin_fmaf(u, W, -0.5f);
    const float fy = __builtin_fmaf(v, H, -0.5f);
    if (!(__builtin_fabsf(fx) < kRange) || !(__builtin_fabsf(fy) < kRange)) return f;
    const float flx = __builtin_floorf(fx), fly = __builtin_floorf(fy);
    f.x0 = (int)flx;
    f.y0 = (int)fly;
    f.s = fx - flx;
    f.t = fy - fly;
    f.active = true;
    const float a = d.x * W, b = d.y * H, c = d.z * W, e = d.w * H;
    const float rx2 = __builtin_fmaf(a, a, b * b);
    const float ry2 = __builtin_fmaf(c, c, e * e);
    f.magnify = (rx2 <= 1.0f) && (ry2 <= 1.0f);
    return f;
}

// Bilinear filtering of texels v0 = (x0,y0), v1 = (x0+1,y0), v2 = (x0,y0+1),
// v3 = (x0+1,y0+1) as two lerps in x and one in y, lerp(a, b, s) =
// fma(s, b - a, a): weights (1-s)(1-t), s(1-t), (1-s)t, st, with constants
// reproduced exactly.  One fixed op sequence used by every method, so exact
// filtering gives the same bits whichever lane produced the texels.
__device__ __forceinline__ float lerp1(float a, float b, float s)
{
    return __builtin_fmaf(s, b - a, a);
}

__device__ __forceinline__ float4 bilerp(float s, float t, float4 v0, float4 v1, float4 v2,
                                         float4 v3)
{
    float4 r;
    r.x = lerp1(lerp1(v0.x, v1.x, s), lerp1(v2.x, v3.x, s), t);
    r.y = lerp1(lerp1(v0.y, v1.y, s), lerp1(v2.y, v3.y, s), t);
    r.z = lerp1(lerp1(v0.z, v1.z, s), lerp1(v2.z, v3.z, s), t);
    r.w = lerp1(lerp1(v0.w, v1.w, s), lerp1(v2.w, v3.w, s), t);
    return r;
}

// ---------------------------------------------------------------------------
// one-tap STF draw [Pharr et al. 2024]: texel (x0 + [u1 < s], y0 + [u2 < t])
// ---------------------------------------------------------------------------

// The "pcg" hash of Jarzynski & Olano, "Hash Functions for GPU Rendering"
// (JCGT 2020): an LCG step followed by PCG's RXS-M-XS output permutation.
__device__ __forceinline__ uint32_t pcg_hash(uint32_t v)
{
    const uint32_t state = v * 747796405u + 2891336453u;
    const uint32_t word = ((state >> ((state >> 28u) + 4u)) ^ state) * 277803737u;
    return (word >> 22u) ^ word;
}

// The per-pixel hash chain of the one-tap draws: h1 and h2 choose the texel
// of the footprint (stf_pick); h3 = pcg(h2) is the spare-lane choice of
// fallback C+.
__device__ __forceinline__ void stf_hashes(uint64_t seed, uint32_t layer, int px, int py, uint32_t& h1,
                                           uint32_t& h2)
{
    uint32_t h = pcg_hash(layer ^ (uint32_t)(seed >> 32));
    h = pcg_hash((uint32_t)py ^ h);
    h = pcg_hash((uint32_t)px ^ h);
    h1 = pcg_hash((uint32_t)seed ^ h);
    h2 = pcg_hash(h1);
}

__device__ __forceinline__ int2 stf_pick_h(const Footprint& f, uint32_t h1, uint32_t h2)
{
    const float u1 = (float)(h1 >> 8) * 0x1p-24f;
    const float u2 = (float)(h2 >> 8) * 0x1p-24f;
    return make_int2(f.x0 + (u1 < f.s ? 1 : 0), f.y0 + (u2 < f.t ? 1 : 0));
}

__device__ __forceinline__ int2 stf_pick(const Footprint& f, uint64_t seed, uint32_t layer,
                                         int px, int py)
{
    uint32_t h1, h2;
    stf_hashes(seed, layer, px, py, h1, h2);
    return stf_pick_h(f, h1, h2);
}

// ---------------------------------------------------------------------------
// reconstruction filters (Section 5): 2x2 bilinear or 4x4 bicubic taps
// ---------------------------------------------------------------------------

template <int FILTER>
struct Taps {
    static constexpr int F = FILTER == CTF_FILTER_BILINEAR ? 2 : 4;  // footprint side
    static constexpr int O = F == 4 ? 1 : 0;                         // origin = x0 - O
};

// 1-D tap weights at position x in [0,1), float32, one fixed op order
// (products, then sums left to right, then the constant factor).
template <int FILTER>
__device__ __forceinline__ void taps32(float x, float w[4])
{
    const float x2 = x * x, x3 = x2 * x, om = 1.0f - x;
    if constexpr (FILTER == CTF_FILTER_BSPLINE) {
        const float sixth = (float)(1.0 / 6.0);
        w[0] = ((om * om) * om) * sixth;
        w[1] = ((3.0f * x3 - 6.0f * x2) + 4.0f) * sixth;
        w[2] = (((-3.0f * x3 + 3.0f * x2) + 3.0f * x) + 1.0f) * sixth;
        w[3] = x3 * sixth;
    } else if constexpr (FILTER == CTF_FILTER_CATMULL_ROM) {
        w[0] = ((2.0f * x2 - x3) - x) * 0.5f;
        w[1] = ((3.0f * x3 - 5.0f * x2) + 2.0f) * 0.5f;
        w[2] = ((-3.0f * x3 + 4.0f * x2) + x) * 0.5f;
        w[3] = (x3 - x2) * 0.5f;
    } else {
        w[0] = om;
        w[1] = x;
        w[2] = w[3] = 0.0f;
    }
}

// Cubic one-tap draw along one axis: tap i with probability |w_i| / sum |w|.
// The drawn tap is the number of float32 partial sums (left to right) at or
// below u * sum, so a zero-weight tap is never drawn.
__device__ __forceinline__ int cubic_tap(const float w[4], float u)
{
    const float a0 = __builtin_fabsf(w[0]), a1 = __builtin_fabsf(w[1]);
    const float a2 = __builtin_fabsf(w[2]), a3 = __builtin_fabsf(w[3]);
    const float p1 = a0, p2 = p1 + a1, p3 = p2 + a2, sum = p3 + a3;
    const float thr = u * sum;
    return (thr >= p1) + (thr >= p2) + (thr >= p3);
}

// One-tap draw for any filter (bilinear: stf_pick_h).
template <int FILTER>
__device__ __forceinline__ int2 stf_pick_filter(const Footprint& f, uint32_t h1, uint32_t h2)
{
    if constexpr (FILTER == CTF_FILTER_BILINEAR) {
        return stf_pick_h(f, h1, h2);
    } else {
        float wx[4], wy[4];
        taps32<FILTER>(f.s, wx);
        taps32<FILTER>(f.t, wy);
        return make_int2(f.x0 - 1 + cubic_tap(wx, (float)(h1 >> 8) * 0x1p-24f),
                         f.y0 - 1 + cubic_tap(wy, (float)(h2 >> 8) * 0x1p-24f));
    }
}

// Exact cubic filtering of 16 texels v[4j + i] (tap (i, j)): each row as a
// fused chain in x, then the rows in y.  One fixed op sequence for every
// method, like bilerp for the 2x2 case.
__device__ __forceinline__ float4 row4(const float wx[4], float4 a, float4 b, float4 c, float4 d)
{
    float4 r;
    r.x = __builtin_fmaf(wx[3], d.x, __builtin_fmaf(wx[2], c.x, __builtin_fmaf(wx[1], b.x, wx[0] * a.x)));
    r.y = __builtin_fmaf(wx[3], d.y, __builtin_fmaf(wx[2], c.y, __builtin_fmaf(wx[1], b.y, wx[0] * a.y)));
    r.z = __builtin_fmaf(wx[3], d.z, __builtin_fmaf(wx[2], c.z, __builtin_fmaf(wx[1], b.z, wx[0] * a.z)));
    r.w = __builtin_fmaf(wx[3], d.w, __builtin_fmaf(wx[2], c.w, __builtin_fmaf(wx[1], b.w, wx[0] * a.w)));
    return r;
}

// accumulate row j (weight wyj) into acc: j == 0 starts the chain
__device__ __forceinline__ float4 col_acc(float wyj, float4 r, float4 acc, bool first)
{
    if (first) return make_float4(wyj * r.x, wyj * r.y, wyj * r.z, wyj * r.w);
    return make_float4(__builtin_fmaf(wyj, r.x, acc.x), __builtin_fmaf(wyj, r.y, acc.y),
                       __builtin_fmaf(wyj, r.z, acc.z), __builtin_fmaf(wyj, r.w, acc.w));
}

// 256-bit footprint mask from the mask of footprint corners:
// B = C | C<<1 | C<<16 | C<<17 (words low first; wave-uniform, scalar ops).
__device__ __forceinline__ void footprint_mask(const uint64_t C[4], uint64_t B[4])
{
#pragma unroll
    for (int w = 0; w < 4; ++w) {
        const uint64_t lo = w > 0 ? C[w - 1] : 0ull;
        B[w] = C[w] | (C[w] << 1) | (lo >> 63) | (C[w] << 16) | (lo >> 48) | (C[w] << 17) | (lo >> 47);
    }
}

// The same for FxF footprints: B = OR over 0 <= dx, dy < F of C << (16 dy + dx)
// (corners of a box inside 16x16 have dx <= 16 - F, so no row wraps).
template <int F>
__device__ __forceinline__ void footprint_mask_f(const uint64_t C[4], uint64_t B[4])
{
    if constexpr (F == 2) {
        footprint_mask(C, B);
    } else {
        uint64_t Hm[4];   // the row spread: C | C<<1 | C<<2 | C<<3
#pragma unroll
        for (int w = 0; w < 4; ++w) {
            const uint64_t lo = w > 0 ? C[w - 1] : 0ull;
            Hm[w] = C[w] | (C[w] << 1) | (lo >> 63) | (C[w] << 2) | (lo >> 62) | (C[w] << 3) | (lo >> 61);
        }
#pragma unroll
        for (int w = 0; w < 4; ++w) {
            const uint64_t lo = w > 0 ? Hm[w - 1] : 0ull;
            B[w] = Hm[w] | (Hm[w] << 16) | (lo >> 48) | (Hm[w] << 32) | (lo >> 32) | (Hm[w] << 48) | (lo >> 16);
        }
    }
}

// A wave's walk over tiles t0, t0 + step, ... of a row-major tile grid,
// keeping (tx, ty) up to date with scalar adds: one division per wave
// instead of a 64-bit division per tile.
struct TileWalk {
    int64_t tile;
    int tx, ty;
    int dtx, dty, tiles_x;
    __device__ __forceinline__ TileWalk(int64_t t0, int64_t step, int tiles_x_) : tile(t0), tiles_x(tiles_x_)
    {
        tx = (int)(t0 % tiles_x_);
        ty = (int)(t0 / tiles_x_);
        dtx = (int)(step % tiles_x_);
        dty = (int)(step / tiles_x_);
    }
    __device__ __forceinline__ void advance(int64_t step)
    {
        tile += step;
        tx += dtx;
        ty += dty;
        if (tx >= tiles_x) {
            tx -= tiles_x;
            ++ty;
        }
    }
};

// Frame totals of one wave over all its tiles, added to the frame record
// once at the end (one set of atomics per wave).
// Per-wave sums of the frame counters, added to the frame's 64-bit counters
// at the end of the kernel.  32-bit (half the scalar registers): a tile adds
// at most 2^13 to any of them, and every launch gives each wave at most
// kMaxWaveTileVisits tile visits (layers counted once each), so none can
// overflow.
constexpr int64_t kMaxWaveTileVisits = int64_t(1) << 18;

// Workgroups of `waves_per_block` waves a launch needs so that no wave visits
// more than kMaxWaveTileVisits tiles.
inline int64_t counter_min_blocks(int64_t tile_visits, int waves_per_block)
{
    const int64_t waves = (tile_visits + kMaxWaveTileVisits - 1) / kMaxWaveTileVisits;
    return (waves + waves_per_block - 1) / waves_per_block;
}

struct FrameCounters {
    uint32_t evals = 0, active = 0, stf = 0, minify = 0, tiles = 0, rows = 0, ok = 0, fail = 0;
    __device__ __forceinline__ void add(int e, int act, int nstf, int mini, int rws, bool okk, bool fl)
    {
        evals += e;
        active += act;
        stf += nstf;
        minify += mini;
        rows += rws;
        tiles += 1;
        ok += okk;
        fail += fl;
    }
    __device__ __forceinline__ void flush(ctf_frame_stats* F) const
    {
        if (!tiles) return;
        atomicAdd((unsigned long long*)&F->evals, (unsigned long long)evals);
        atomicAdd((unsigned long long*)&F->active, (unsigned long long)active);
        atomicAdd((unsigned long long*)&F->stf, (unsigned long long)stf);
        atomicAdd((unsigned long long*)&F->minify, (unsigned long long)minify);
        atomicAdd((unsigned long long*)&F->tiles, (unsigned long long)tiles);
        atomicAdd((unsigned long long*)&F->rows, (unsigned long long)rows);
        atomicAdd((unsigned long long*)&F->tiles_ok, (unsigned long long)ok);
        atomicAdd((unsigned long long*)&F->tiles_fail, (unsigned long long)fail);
    }
};

// ---------------------------------------------------------------------------
// texel producers
// ---------------------------------------------------------------------------

struct DevTexture {
    int kind;
    int width, height;
    uint32_t wmask, hmask;
    float inv_w;
    int n_terms;
    const int4* __restrict__ terms;   // [4][K] = (p, q, j, bits of amp)
    // [4][K] = (p'/W, q'/W, j'/W, amp) with p', q' the residues of p, q mod W
    // in [-W/2, W/2) and j' = j mod W; null when W > 4096
    const float4* __restrict__ fterms;
    float affine[4][3];
    float constant[4];
    const float4* __restrict__ table; // [height][width]
};

// 1/2 + 1/2 sum_k a_k sin(2 pi r_k / W), r_k = (p x + q y + j) mod W.  The
// phase is an exact integer, r/W is exact in float32, and v_sin_f32 takes
// its argument in revolutions, so each term is one hardware sine.
// The term arrays in device memory are read through the constant address
// space: with a wave-uniform address each term is one scalar load
// (s_load_dwordx4 through the scalar cache) instead of a 64-lane broadcast
// vector load and its wait.  Only for global memory that the kernel never
// writes -- LDS-staged terms keep their generic pointer.
typedef int TermVec __attribute__((ext_vector_type(4)));
typedef const __attribute__((address_space(4))) TermVec* ConstTerms;

__device__ __forceinline__ ConstTerms const_terms(const int4* global_terms)
{
    return (ConstTerms)global_terms;
}

typedef float FTermVec __attribute__((ext_vector_type(4)));
typedef const __attribute__((address_space(4))) FTermVec* ConstFTerms;

__device__ __forceinline__ ConstFTerms const_fterms(const float4* global_terms)
{
    return (ConstFTerms)global_terms;
}

// The same channel from the float terms: v = p' x + q' y + j' is an integer
// with |v| < W^2 <= 2^24, so both fused products and sums below are exact
// and fract(v / W) is exactly (v mod W) / W, the argument the integer form
// passes to the sine: the results are bit-identical to sinusoid_channel, in
// five instructions per term instead of eight.
template <class TermPtr>
__device__ __forceinline__ float sinusoid_channel_f(TermPtr tc, int K, float xf, float yf)
{
    float acc = 0.0f;
    // eight terms per iteration: their loads are issued together (one wait)
    int k = 0;
    for (; k + 8 <= K; k += 8) {
        decltype(tc[0] + 0) t8[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) t8[u] = tc[k + u];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const float ph = __builtin_fmaf(t8[u].x, xf, __builtin_fmaf(t8[u].y, yf, t8[u].z));
            const float sn = __builtin_amdgcn_sinf(__builtin_amdgcn_fractf(ph));
            acc = __builtin_fmaf(t8[u].w, sn, acc);
        }
    }
    for (; k < K; ++k) {
        const auto tk = tc[k];
        const float ph = __builtin_fmaf(tk.x, xf, __builtin_fmaf(tk.y, yf, tk.z));
        const float sn = __builtin_amdgcn_sinf(__builtin_amdgcn_fractf(ph));
        acc = __builtin_fmaf(tk.w, sn, acc);
    }
    return __builtin_fmaf(0.5f, acc, 0.5f);
}

template <class TermPtr>
__device__ __forceinline__ float sinusoid_channel(TermPtr tc, int K, uint32_t wmask, float inv_w, int xm, int ym)
{
    float acc = 0.0f;
    for (int k = 0; k < K; ++k) {
        const auto tk = tc[k];
        const uint32_t r = (uint32_t)(__mul24(tk.x, xm) + __mul24(tk.y, ym) + tk.z) & wmask;
        const float sn = __builtin_amdgcn_sinf((float)r * inv_w);
        acc = __builtin_fmaf(__int_as_float(tk.w), sn, acc);
    }
    return __builtin_fmaf(0.5f, acc, 0.5f);
}

template <int KIND>
__device__ __forceinline__ float4 texel_eval(const DevTexture& T, int x, int y)
{
    float4 r;
    if constexpr (KIND == CTF_TEX_SINUSOIDS) {
        const int xm = x & (int)T.wmask, ym = y & (int)T.wmask;
        const int K = T.n_terms;
        if (T.fterms) {
            const ConstFTerms tc = const_fterms(T.fterms);
            const float xf = (float)xm, yf = (float)ym;
            r.x = sinusoid_channel_f(tc + 0 * K, K, xf, yf);
            r.y = sinusoid_channel_f(tc + 1 * K, K, xf, yf);
            r.z = sinusoid_channel_f(tc + 2 * K, K, xf, yf);
            r.w = sinusoid_channel_f(tc + 3 * K, K, xf, yf);
        } else {
            const ConstTerms tc = const_terms(T.terms);
            r.x = sinusoid_channel(tc + 0 * K, K, T.wmask, T.inv_w, xm, ym);
            r.y = sinusoid_channel(tc + 1 * K, K, T.wmask, T.inv_w, xm, ym);
            r.z = sinusoid_channel(tc + 2 * K, K, T.wmask, T.inv_w, xm, ym);
            r.w = sinusoid_channel(tc + 3 * K, K, T.wmask, T.inv_w, xm, ym);
        }
    } else if constexpr (KIND == CTF_TEX_AFFINE) {
        const float fx = (float)x, fy = (float)y;
        r.x = __builtin_fmaf(T.affine[0][2], fy, __builtin_fmaf(T.affine[0][1], fx, T.affine[0][0]));
        r.y = __builtin_fmaf(T.affine[1][2], fy, __builtin_fmaf(T.affine[1][1], fx, T.affine[1][0]));
        r.z = __builtin_fmaf(T.affine[2][2], fy, __builtin_fmaf(T.affine[2][1], fx, T.affine[2][0]));
        r.w = __builtin_fmaf(T.affine[3][2], fy, __builtin_fmaf(T.affine[3][1], fx, T.affine[3][0]));
    } else if constexpr (KIND == CTF_TEX_CONSTANT) {
        r = make_float4(T.constant[0], T.constant[1], T.constant[2], T.constant[3]);
    } else {  // CTF_TEX_TABLE
        r = T.table[(size_t)(y & (int)T.hmask) * T.width + (x & (int)T.wmask)];
    }
    return r;
}

// Terms of a sinusoid texture staged in a workgroup's LDS: [4][K + 1] entries
// (each channel's row padded by one entry, so that lanes reading the same
// term of different channels hit different banks), the float terms when the
// texture has them.  Textures with more terms are not staged.  62 terms:
// 4032 bytes, so that a per-lane workgroup (four 7 KiB wave slices and the
// terms) stays within 32 KiB and five of them fit in a CU's 160 KiB.
constexpr int kLdsTerms = 62;
constexpr int kLdsTermEntries = 4 * (kLdsTerms + 1);

// Every thread of the workgroup calls this (it synchronises the workgroup).
__device__ inline bool stage_terms(const DevTexture& T, int4* terms_lds)
{
    if (T.kind != CTF_TEX_SINUSOIDS || T.n_terms > kLdsTerms) return false;
    const int4* src = T.fterms ? reinterpret_cast<const int4*>(T.fterms) : T.terms;
    for (int i = threadIdx.x; i < 4 * T.n_terms; i += blockDim.x) terms_lds[i + i / T.n_terms] = src[i];
    __syncthreads();
    return true;
}

// A texel from staged float terms (every lane reads the same entry, a
// broadcast; the operands are then all vector registers, one instruction
// fewer per term than with terms in scalar registers).  Textures whose
// terms are not staged read them with vector loads: the scalar form would
// hold 32 scalar registers for its eight terms in flight across the whole
// kernel, and the per-lane kernels are short of scalar registers.  The same
// values either way.
template <int KIND>
__device__ __forceinline__ float4 texel_eval_staged(const DevTexture& T, const int4* terms_lds, bool lds_float, int x,
                                                    int y)
{
    if constexpr (KIND == CTF_TEX_SINUSOIDS) {
        const int K = T.n_terms;
        const int xm = x & (int)T.wmask, ym = y & (int)T.wmask;
        const float xf = (float)xm, yf = (float)ym;
        if (lds_float) {
            const float4* tl = reinterpret_cast<const float4*>(terms_lds);
            return make_float4(sinusoid_channel_f(tl + 0 * (K + 1), K, xf, yf),
                               sinusoid_channel_f(tl + 1 * (K + 1), K, xf, yf),
                               sinusoid_channel_f(tl + 2 * (K + 1), K, xf, yf),
                               sinusoid_channel_f(tl + 3 * (K + 1), K, xf, yf));
        }
        // (an offset the compiler cannot prove uniform keeps these loads in
        // vector registers)
        int zero = 0;
        asm volatile("" : "+v"(zero));
        if (T.fterms) {
            const float4* tf = T.fterms + zero;
            return make_float4(sinusoid_channel_f(tf + 0 * K, K, xf, yf), sinusoid_channel_f(tf + 1 * K, K, xf, yf),
                               sinusoid_channel_f(tf + 2 * K, K, xf, yf), sinusoid_channel_f(tf + 3 * K, K, xf, yf));
        }
        const int4* ti = T.terms + zero;
        return make_float4(sinusoid_channel(ti + 0 * K, K, T.wmask, T.inv_w, xm, ym),
                           sinusoid_channel(ti + 1 * K, K, T.wmask, T.inv_w, xm, ym),
                           sinusoid_channel(ti + 2 * K, K, T.wmask, T.inv_w, xm, ym),
                           sinusoid_channel(ti + 3 * K, K, T.wmask, T.inv_w, xm, ym));
    }
    return texel_eval<KIND>(T, x, y);
}

}  // namespace ctf
