// decoder_mlp.h -- the learned texel producer on MFMA (gfx950, wave64).
//
// A texel (x, y) is decoded from two latent grids (8 channels each) sampled
// bilinearly with repeat addressing, concatenated to 16 features, and fed to
// an MLP 16 -> 64 -> 64 -> 4 (ReLU on the hidden layers, linear output).
//
// Tiling.  One wave decodes 16 texels at a time in the transposed
// orientation: activations are (units x texels), weights are the A operand
// and texels the columns, so every layer is out^T = W^T in^T.  With the
// 16x16x{16,32} MFMA layouts (A: lane l holds row l%16 and k = K/4*(l/16)..;
// B: column l%16, same k; C: column l%16, rows 4*(l/16)..+3) the C result of
// one layer is already the B operand of the next once two 16-row blocks are
// interleaved: K slot s of lane group g in K-step kc is unit
//     pi(kc, g, s) = 32 kc + 16 (s / 4) + 4 g + s % 4,
// and the weights are stored with their K index permuted the same way.  No
// LDS round trip between layers.
//
// Weight blocks are stored in lane order (one 8- or 16-byte load per lane):
//   forward  W1T[4 hb][64][4]     row = hidden 16 hb + l%16, k = feature 4 g + i
//            W2T[4 ob][2 kc][64][8] row = out 16 ob + l%16,  k = in pi(kc, g, s)
//            W3T[2 kc][64][8]      row = channel l%16 (< 4), k = hidden pi(kc, g, s)
//   backward W3A[4 ob][64][4]     row = hidden 16 ob + l%16, k = channel 4 g + i
//            W2A[4 ib][2 kc][64][8] row = in 16 ib + l%16,   k = out pi(kc, g, s)
//            W1A[2 kc][64][8]      row = feature l%16,       k = hidden pi(kc, g, s)
//   biases   b1c[4][64][4], b2c[4][64][4], b3c[64][4] (float, C-operand order)
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ctf.h"

namespace ctf {

constexpr int kFeat = 16;     // 2 levels x 8 channels
constexpr int kHid = 64;      // MFMA hidden width (smaller H is zero padded)

// element offsets (16-bit elements) of the packed weight blocks
constexpr int kW1T = 0;
constexpr int kW2T = kW1T + 4 * 64 * 4;
constexpr int kW3T = kW2T + 4 * 2 * 64 * 8;
constexpr int kFwdElems = kW3T + 2 * 64 * 8;      // 6144
constexpr int kW3A = kFwdElems;
constexpr int kW2A = kW3A + 4 * 64 * 4;
constexpr int kW1A = kW2A + 4 * 2 * 64 * 8;
constexpr int kAllElems = kW1A + 2 * 64 * 8;      // 12288
// float offsets of the packed biases
constexpr int kB1C = 0;
constexpr int kB2C = 4 * 64 * 4;
constexpr int kB3C = 8 * 64 * 4;
constexpr int kBiasFloats = 9 * 64 * 4;           // 2304

typedef float f4 __attribute__((ext_vector_type(4)));
typedef unsigned short u16x4 __attribute__((ext_vector_type(4)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 h4 __attribute__((ext_vector_type(4)));
typedef _Float16 h8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef short s4 __attribute__((ext_vector_type(4)));

// pi(kc, g, s) and its inverse (for packing)
__host__ __device__ inline int unit_of(int kc, int g, int s) { return 32 * kc + 16 * (s >> 2) + 4 * g + (s & 3); }
__host__ __device__ inline int kc_of(int h) { return h >> 5; }
__host__ __device__ inline int g_of(int h) { return (h >> 2) & 3; }
__host__ __device__ inline int s_of(int h) { return (((h >> 4) & 1) << 2) | (h & 3); }

template <int P> struct Mfma;

template <> struct Mfma<CTF_FP16> {
    static __device__ __forceinline__ f4 k16(u16x4 a, u16x4 b, f4 c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x16f16(__builtin_bit_cast(h4, a), __builtin_bit_cast(h4, b), c, 0, 0, 0);
    }
    static __device__ __forceinline__ f4 k32(u16x8 a, u16x8 b, f4 c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(h8, a), __builtin_bit_cast(h8, b), c, 0, 0, 0);
    }
    static __device__ __forceinline__ unsigned short cvt(float x)
    {
        return __builtin_bit_cast(unsigned short, (_Float16)x);
    }
    static __device__ __forceinline__ float load(unsigned short u)
    {
        return (float)__builtin_bit_cast(_Float16, u);
    }
};

template <> struct Mfma<CTF_BF16> {
    static __device__ __forceinline__ f4 k16(u16x4 a, u16x4 b, f4 c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(__builtin_bit_cast(s4, a), __builtin_bit_cast(s4, b), c, 0, 0, 0);
    }
    static __device__ __forceinline__ f4 k32(u16x8 a, u16x8 b, f4 c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8, a), __builtin_bit_cast(bf8, b), c, 0, 0, 0);
    }
    static __device__ __forceinline__ unsigned short cvt(float x)
    {
        return __builtin_bit_cast(unsigned short, (__bf16)x);
    }
    static __device__ __forceinline__ float load(unsigned short u)
    {
        return __uint_as_float((uint32_t)u << 16);
    }
};

// Resident forward weights of one wave.
template <int P>
struct FwdWeights {
    u16x4 w1[4];
    u16x8 w2[4][2];
    u16x8 w3[2];

    __device__ __forceinline__ void load(const uint16_t* __restrict__ w, int lane)
    {
#pragma unroll
        for (int hb = 0; hb < 4; ++hb)
            w1[hb] = *reinterpret_cast<const u16x4*>(w + kW1T + (hb * 64 + lane) * 4);
#pragma unroll
        for (int ob = 0; ob < 4; ++ob)
#pragma unroll
            for (int kc = 0; kc < 2; ++kc)
                w2[ob][kc] = *reinterpret_cast<const u16x8*>(w + kW2T + ((ob * 2 + kc) * 64 + lane) * 8);
#pragma unroll
        for (int kc = 0; kc < 2; ++kc)
            w3[kc] = *reinterpret_cast<const u16x8*>(w + kW3T + (kc * 64 + lane) * 8);
    }
};

struct Biases {
    f4 b1[4], b2[4], b3;
    __device__ __forceinline__ void load(const float* __restrict__ b, int lane)
    {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            b1[i] = *reinterpret_cast<const f4*>(b + kB1C + (i * 64 + lane) * 4);
            b2[i] = *reinterpret_cast<const f4*>(b + kB2C + (i * 64 + lane) * 4);
        }
        b3 = *reinterpret_cast<const f4*>(b + kB3C + lane * 4);
    }
};

// Two floats -> one 32-bit word of two 16-bit values, round to nearest even
// (one v_cvt_pk_f16_f32 / v_cvt_pk_bf16_f32: written as a vector conversion
// so the backend keeps the packed form).
template <int P>
__device__ __forceinline__ uint32_t cvt2(float a, float b);

template <>
__device__ __forceinline__ uint32_t cvt2<CTF_FP16>(float a, float b)
{
    typedef _Float16 h2 __attribute__((ext_vector_type(2)));
    typedef float f2 __attribute__((ext_vector_type(2)));
    const f2 v = {a, b};
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, h2));
}

template <>
__device__ __forceinline__ uint32_t cvt2<CTF_BF16>(float a, float b)
{
    typedef __bf16 b2 __attribute__((ext_vector_type(2)));
    typedef float f2 __attribute__((ext_vector_type(2)));
    const f2 v = {a, b};
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, b2));
}

// ReLU on two packed 16-bit floats: both formats keep the sign in the top
// bit, so a signed 16-bit max against 0 clears negative values (one
// v_pk_max_i16, no NaN canonicalisation of the MFMA results).
__device__ __forceinline__ uint32_t relu2(uint32_t w)
{
    typedef short s2 __attribute__((ext_vector_type(2)));
    const s2 z = {0, 0};
    return __builtin_bit_cast(uint32_t, __builtin_elementwise_max(__builtin_bit_cast(s2, w), z));
}

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// ReLU and conversion of two C blocks into one K=32 B operand (pi order).
template <int P>
__device__ __forceinline__ u16x8 relu_pack(f4 lo, f4 hi)
{
    u32x4 r;
    r[0] = relu2(cvt2<P>(lo[0], lo[1]));
    r[1] = relu2(cvt2<P>(lo[2], lo[3]));
    r[2] = relu2(cvt2<P>(hi[0], hi[1]));
    r[3] = relu2(cvt2<P>(hi[2], hi[3]));
    return __builtin_bit_cast(u16x8, r);
}

template <int P>
__device__ __forceinline__ u16x8 pack8(f4 lo, f4 hi)
{
    u32x4 r;
    r[0] = cvt2<P>(lo[0], lo[1]);
    r[1] = cvt2<P>(lo[2], lo[3]);
    r[2] = cvt2<P>(hi[0], hi[1]);
    r[3] = cvt2<P>(hi[2], hi[3]);
    return __builtin_bit_cast(u16x8, r);
}

template <int P>
__device__ __forceinline__ u16x4 pack4(f4 x)
{
    typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
    u32x2 r;
    r[0] = cvt2<P>(x[0], x[1]);
    r[1] = cvt2<P>(x[2], x[3]);
    return __builtin_bit_cast(u16x4, r);
}

// Latent grids of one decoder: both levels in one allocation (level 1 at
// byte offset lvl1), cells of 8 16-bit channels (16 bytes), side 2^log_l.
struct LatentGrid {
    const uint16_t* __restrict__ base;
    uint32_t lvl1;          // byte offset of level 1
    int log_l0, log_l1;     // log2 of the sides
    int shift0, shift1;     // log2(tex_w / side)
    int tex_w;
};

// Latent taps of texel (x, y) for this lane (level g/2, channels 4 (g%2)..+3):
// sample point (x + 1/2) L / W - 1/2 for the wrapped coordinate (exact in
// float32), four corners with repeat addressing and their bilinear weights.
// latent_fetch issues the four 8-byte loads; latent_combine interpolates.
struct LatentFetch {
    u16x4 v[4];
    float w[4];
    uint32_t cell[4];
};

__device__ __forceinline__ void latent_fetch(const LatentGrid& G, int x, int y, int g, LatentFetch& F)
{
    const int level = g >> 1;
    const int logL = level ? G.log_l1 : G.log_l0;
    const int shift = level ? G.shift1 : G.shift0;
    const int m = (1 << logL) - 1;
    const int xw = x & (G.tex_w - 1), yw = y & (G.tex_w - 1);
    const float inv = __builtin_ldexpf(1.0f, -shift);
    const float off = __builtin_fmaf(0.5f, inv, -0.5f);
    const float gx = __builtin_fmaf((float)xw, inv, off);
    const float gy = __builtin_fmaf((float)yw, inv, off);
    const float cx = __builtin_floorf(gx), cy = __builtin_floorf(gy);
    const float fx = gx - cx, fy = gy - cy;
    const int icx = (int)cx, icy = (int)cy;
    const uint32_t x0 = (uint32_t)(icx & m), x1 = (uint32_t)((icx + 1) & m);
    const uint32_t y0 = (uint32_t)(icy & m) << logL, y1 = (uint32_t)((icy + 1) & m) << logL;
    F.cell[0] = y0 | x0;
    F.cell[1] = y0 | x1;
    F.cell[2] = y1 | x0;
    F.cell[3] = y1 | x1;
    const float ifx = 1.0f - fx, ify = 1.0f - fy;
    F.w[0] = ifx * ify;
    F.w[1] = fx * ify;
    F.w[2] = ifx * fy;
    F.w[3] = fx * fy;
    const uint32_t byte0 = (level ? G.lvl1 : 0u) + 8u * (uint32_t)(g & 1);
    const char* __restrict__ b = reinterpret_cast<const char*>(G.base);
#pragma unroll
    for (int q = 0; q < 4; ++q)
        F.v[q] = *reinterpret_cast<const u16x4*>(b + (byte0 + (F.cell[q] << 4)));
}

template <int P>
__device__ __forceinline__ f4 latent_combine(const LatentFetch& F)
{
    f4 r = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int i = 0; i < 4; ++i) r[i] = __builtin_fmaf(F.w[q], Mfma<P>::load(F.v[q][i]), r[i]);
    return r;
}

// Inference copy of the latents.  Each level is stored as (L+1) x (L+1)
// cells, cell (i, j) holding cell (i mod L, j mod L), so that the four
// corners of a sample are c, c + 1, c + (L+1), c + (L+2) with no wrapping.
// For texel x, the sample point (x + 1/2) L / W - 1/2 equals
// (2x + 1 - 2^s) / 2^(s+1) with W = 2^s L: the integer 2x + 1 - 2^s (taken
// modulo 2^32, which keeps its low bits) holds the cell index mod L in bits
// [s+1, s+1+log2 L) and the fraction in its low s+1 bits, for any x.
struct InferGrid {
    const uint16_t* __restrict__ base;
    uint32_t lvl1;          // byte offset of level 1
    int log_l0, log_l1;     // log2 of the sides
    int shift0, shift1;     // log2(tex_w / side)
    int tex_w;
};

// Per-lane constants of the inference fetch (level g/2, channels 4 (g%2)..+3).
template <int P>
struct InferLane {
    uint32_t off;      // byte offset of the level plus 8 (g % 2)
    uint32_t pitch;    // L + 1 cells
    uint32_t c;        // 1 - 2^s
    uint32_t sh;       // s + 1
    uint32_t logl;     // log2 L
    float scale;       // 2^-(s+1)

    __device__ __forceinline__ InferLane(const InferGrid& G, int g)
    {
        const bool l1 = g >= 2;
        const int s = l1 ? G.shift1 : G.shift0;
        logl = (uint32_t)(l1 ? G.log_l1 : G.log_l0);
        pitch = (1u << logl) + 1u;
        off = (l1 ? G.lvl1 : 0u) + 8u * (uint32_t)(g & 1);
        c = 1u - (1u << s);
        sh = (uint32_t)s + 1u;
        scale = __builtin_bit_cast(float, (uint32_t)(127 - s - 1) << 23);
    }
};

// The four corner vectors and the bilinear weights of one sample; fp16:
// weights packed as (w0, w1), (w2, w3) -- each a multiple of 2^-2(s+1) below
// 1, so exact in fp16 for s <= 4 (rounded to fp16 beyond); bf16: float.
struct InferFetch {
    u16x4 v[4];
    uint32_t w01, w23;
    float w[4];
};

typedef _Float16 h2 __attribute__((ext_vector_type(2)));

template <int P>
__device__ __forceinline__ void infer_fetch(const InferGrid& G, const InferLane<P>& K, int x, int y, InferFetch& F)
{
    const uint32_t gx = 2u * (uint32_t)x + K.c, gy = 2u * (uint32_t)y + K.c;
    const uint32_t cx = __builtin_amdgcn_ubfe(gx, K.sh, K.logl);
    const uint32_t cy = __builtin_amdgcn_ubfe(gy, K.sh, K.logl);
    const float fx = (float)__builtin_amdgcn_ubfe(gx, 0u, K.sh) * K.scale;
    const float fy = (float)__builtin_amdgcn_ubfe(gy, 0u, K.sh) * K.scale;
    const uint32_t o0 = (__umul24(cy, K.pitch) + cx) * 16u + K.off;
    const uint32_t o1 = o0 + K.pitch * 16u;
    const char* __restrict__ b = reinterpret_cast<const char*>(G.base);
    F.v[0] = *reinterpret_cast<const u16x4*>(b + o0);
    F.v[1] = *reinterpret_cast<const u16x4*>(b + o0 + 16u);
    F.v[2] = *reinterpret_cast<const u16x4*>(b + o1);
    F.v[3] = *reinterpret_cast<const u16x4*>(b + o1 + 16u);
    if (P == CTF_FP16) {
        const h2 f = __builtin_bit_cast(h2, cvt2<CTF_FP16>(fx, fy));
        const h2 one = {(_Float16)1.0f, (_Float16)1.0f};
        const h2 i = one - f;                                       // (1 - fx, 1 - fy)
        const h2 r = __builtin_shufflevector(i, f, 0, 2);           // (1 - fx, fx)
        F.w01 = __builtin_bit_cast(uint32_t, r * __builtin_shufflevector(i, i, 1, 1));
        F.w23 = __builtin_bit_cast(uint32_t, r * __builtin_shufflevector(f, f, 1, 1));
    } else {
        const float ifx = 1.0f - fx, ify = 1.0f - fy;
        F.w[0] = ifx * ify;
        F.w[1] = fx * ify;
        F.w[2] = ifx * fy;
        F.w[3] = fx * fy;
    }
}

// The interpolated features of the sample as the layer-1 B operand.  fp16:
// packed fp16 products and sums (v_pk_mul / v_pk_fma, each rounding to
// fp16); bf16: float32 sums rounded once.
template <int P>
__device__ __forceinline__ u16x4 infer_combine(const InferFetch& F)
{
    if (P == CTF_FP16) {
        const h2 w01 = __builtin_bit_cast(h2, F.w01), w23 = __builtin_bit_cast(h2, F.w23);
        const h2 ws[4] = {__builtin_shufflevector(w01, w01, 0, 0), __builtin_shufflevector(w01, w01, 1, 1),
                          __builtin_shufflevector(w23, w23, 0, 0), __builtin_shufflevector(w23, w23, 1, 1)};
        // (a subscript applied directly to a __builtin_bit_cast result is
        // miscompiled by this clang -- it reads element 0 -- so every
        // reinterpreted vector is named before it is indexed)
        typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
        u32x2 d[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) d[q] = __builtin_bit_cast(u32x2, F.v[q]);
        u32x2 r;
#pragma unroll
        for (int half = 0; half < 2; ++half) {
            const uint32_t d0 = d[0][half];
            h2 acc = __builtin_bit_cast(h2, d0) * ws[0];
#pragma unroll
            for (int q = 1; q < 4; ++q) {
                const uint32_t dq = d[q][half];
                acc = __builtin_elementwise_fma(__builtin_bit_cast(h2, dq), ws[q], acc);
            }
            r[half] = __builtin_bit_cast(uint32_t, acc);
        }
        return __builtin_bit_cast(u16x4, r);
    } else {
        f4 x = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int i = 0; i < 4; ++i) x[i] = __builtin_fmaf(F.w[q], Mfma<P>::load(F.v[q][i]), x[i]);
        return pack4<P>(x);
    }
}

// Forward pass of 16 texels whose features this lane holds (xb = features
// 4g..4g+3 of texel l%16 in the operand format; mlp_forward takes them as
// float).  Returns the output block (rows = channels; lanes 0..15 hold RGBA
// of their texel) and, if wanted, the pre-activations.
template <int P>
__device__ __forceinline__ f4 mlp_forward_b(const FwdWeights<P>& W, const Biases& B, u16x4 xb, f4* z1, f4* z2)
{
    f4 d1[4];
#pragma unroll
    for (int hb = 0; hb < 4; ++hb) d1[hb] = Mfma<P>::k16(W.w1[hb], xb, B.b1[hb]);
    u16x8 h1[2];
#pragma unroll
    for (int kc = 0; kc < 2; ++kc) h1[kc] = relu_pack<P>(d1[2 * kc], d1[2 * kc + 1]);
    f4 d2[4];
#pragma unroll
    for (int ob = 0; ob < 4; ++ob) {
        d2[ob] = Mfma<P>::k32(W.w2[ob][0], h1[0], B.b2[ob]);
        d2[ob] = Mfma<P>::k32(W.w2[ob][1], h1[1], d2[ob]);
    }
    u16x8 h2[2];
#pragma unroll
    for (int kc = 0; kc < 2; ++kc) h2[kc] = relu_pack<P>(d2[2 * kc], d2[2 * kc + 1]);
    f4 y = Mfma<P>::k32(W.w3[0], h2[0], B.b3);
    y = Mfma<P>::k32(W.w3[1], h2[1], y);
    if (z1) {
#pragma unroll
        for (int i = 0; i < 4; ++i) z1[i] = d1[i];
    }
    if (z2) {
#pragma unroll
        for (int i = 0; i < 4; ++i) z2[i] = d2[i];
    }
    return y;
}

template <int P>
__device__ __forceinline__ f4 mlp_forward(const FwdWeights<P>& W, const Biases& B, f4 X, f4* z1, f4* z2)
{
    return mlp_forward_b<P>(W, B, pack4<P>(X), z1, z2);
}

}  // namespace ctf
