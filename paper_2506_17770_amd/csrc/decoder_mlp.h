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

// Forward pass of 16 texels whose features this lane holds (X = features
// 4g..4g+3 of texel l%16).  Returns the output block (rows = channels; lanes
// 0..15 hold RGBA of their texel) and, if wanted, the pre-activations.
template <int P>
__device__ __forceinline__ f4 mlp_forward(const FwdWeights<P>& W, const Biases& B, f4 X, f4* z1,
                                          f4* z2)
{
    const u16x4 xb = pack4<P>(X);
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

}  // namespace ctf
