// decoder.hip -- learned texel producer: parameters, training kernels, C ABI.
//
// Float32 master parameters live on the device in the flat layout of
// include/ctf.h.  Training steps run four kernels on one stream:
//   k_sample   texel coordinates from the pcg hash of (seed, step, sample)
//              and their targets from a texel producer;
//   k_train    forward + backward on MFMA for 16-sample tiles (operands in
//              bf16 or fp16, float32 accumulation), latent gradients
//              scattered as 64-bit fixed-point atomics (order independent,
//              so training is bitwise reproducible), per-workgroup partial
//              sums of the MLP weight gradients (batch reductions on MFMA
//              after an LDS transpose of each 16x16 block, the waves' sums
//              added in LDS in a fixed order);
//   k_reduce   fixed-order sum of the partials (deterministic) and the loss;
//   k_adam     Adam on the master copy, rewriting the low-precision latent
//              copy and the packed MFMA weight blocks.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "ctf_internal.h"
#include "decoder_mlp.h"

using namespace ctf;

namespace {

struct Layout {
    int64_t lat0, lat1, W1, b1, W2, b2, W3, b3, total;
    int64_t mlp0, mlp_count;
};

Layout layout_of(const ctf_decoder_desc& d)
{
    Layout o;
    const int64_t C = d.channels, H = d.hidden;
    o.lat0 = 0;
    o.lat1 = (int64_t)d.l0 * d.l0 * C;
    o.W1 = o.lat1 + (int64_t)d.l1 * d.l1 * C;
    o.b1 = o.W1 + 2 * C * H;
    o.W2 = o.b1 + H;
    o.b2 = o.W2 + H * H;
    o.W3 = o.b2 + H;
    o.b3 = o.W3 + H * 4;
    o.total = o.b3 + 4;
    o.mlp0 = o.W1;
    o.mlp_count = o.total - o.W1;
    return o;
}

int ilog2(int v)
{
    int r = 0;
    while ((1 << r) < v) ++r;
    return r;
}

bool pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

}  // namespace

struct ctf_decoder_s {
    ctf_context ctx;
    ctf_decoder_desc desc;
    Layout lay;
    float* master = nullptr;   // [total]
    float* m = nullptr;        // Adam first moment [total]
    float* v = nullptr;        // Adam second moment [total]
    float* grad = nullptr;     // [total]; the latent part is filled from glat_fx
    int64_t* glat_fx = nullptr;  // latent gradient, fixed point (2^-44 units) [mlp0]
    int64_t step = 0;
    // low-precision training copies
    int lp_precision = -1;
    uint16_t* lat_lp = nullptr;    // [lat0 | lat1] in the flat order
    uint16_t* w_lp = nullptr;      // packed MFMA weights [kAllElems]
    float* bias_c = nullptr;       // packed C-operand biases [kBiasFloats]
    // batch buffers
    int32_t cap_batch = 0;
    int32_t* xy = nullptr;
    float* target = nullptr;
    float* partials = nullptr;     // [max waves][mlp_count]
    float* loss_part = nullptr;    // [max waves]
    float* loss_tmp = nullptr;     // [1]
};

namespace ctf {

// Packed positions of flat MLP parameter `rel` (relative to W1): a weight
// entry has one forward and one backward element of w_lp (weight(pos) is
// called for each); a bias has 16 float slots of bias_c (bias(pos) for
// each).  Positions are produced one at a time (no indexed local array, so
// the kernels using this need no private memory).
template <class OnWeight, class OnBias>
__host__ __device__ inline void packed_visit(int rel, int H, OnWeight&& weight, OnBias&& bias)
{
    const int nW1 = 16 * H, nW2 = H * H, nW3 = H * 4;
    if (rel < nW1) {
        const int f = rel / H, h = rel % H;
        weight(kW1T + ((h >> 4) * 64 + (f >> 2) * 16 + (h & 15)) * 4 + (f & 3));
        weight(kW1A + (kc_of(h) * 64 + g_of(h) * 16 + f) * 8 + s_of(h));
        return;
    }
    rel -= nW1;
    if (rel < H) {
        const int h = rel;
        for (int j = 0; j < 16; ++j) bias(kB1C + ((h >> 4) * 64 + ((h & 15) >> 2) * 16 + j) * 4 + (h & 3));
        return;
    }
    rel -= H;
    if (rel < nW2) {
        const int i = rel / H, o = rel % H;
        weight(kW2T + (((o >> 4) * 2 + kc_of(i)) * 64 + g_of(i) * 16 + (o & 15)) * 8 + s_of(i));
        weight(kW2A + (((i >> 4) * 2 + kc_of(o)) * 64 + g_of(o) * 16 + (i & 15)) * 8 + s_of(o));
        return;
    }
    rel -= nW2;
    if (rel < H) {
        const int o = rel;
        for (int j = 0; j < 16; ++j) bias(kB2C + ((o >> 4) * 64 + ((o & 15) >> 2) * 16 + j) * 4 + (o & 3));
        return;
    }
    rel -= H;
    if (rel < nW3) {
        const int h = rel / 4, c = rel % 4;
        weight(kW3T + (kc_of(h) * 64 + g_of(h) * 16 + c) * 8 + s_of(h));
        weight(kW3A + ((h >> 4) * 64 + (h & 15)) * 4 + c);
        return;
    }
    rel -= nW3;
    for (int j = 0; j < 16; ++j) bias(kB3C + j * 4 + rel);
}

// Host packing (inference textures and the first training copy).
static unsigned short to_half_bits(float x)
{
    _Float16 h = (_Float16)x;
    unsigned short u;
    std::memcpy(&u, &h, 2);
    return u;
}

static unsigned short to_bf16_bits(float x)
{
    uint32_t u;
    std::memcpy(&u, &x, 4);
    if ((u & 0x7f800000u) == 0x7f800000u) return (unsigned short)((u >> 16) | ((u & 0xffff) ? 0x40 : 0));
    u += 0x7fffu + ((u >> 16) & 1u);   // round to nearest even
    return (unsigned short)(u >> 16);
}

void pack_host(const float* P, const ctf_decoder_desc& d, int precision, std::vector<uint16_t>& lat,
               std::vector<uint16_t>& w, std::vector<float>& bias)
{
    const Layout lay = layout_of(d);
    auto cvt = [&](float x) { return precision == CTF_BF16 ? to_bf16_bits(x) : to_half_bits(x); };
    lat.resize((size_t)lay.mlp0);
    for (int64_t i = 0; i < lay.mlp0; ++i) lat[i] = cvt(P[i]);
    w.assign(kAllElems, 0);
    bias.assign(kBiasFloats, 0.f);
    for (int64_t r = 0; r < lay.mlp_count; ++r) {
        const float val = P[lay.mlp0 + r];
        packed_visit((int)r, d.hidden, [&](int q) { w[q] = cvt(val); }, [&](int q) { bias[q] = val; });
    }
}

}  // namespace ctf

namespace {

// ---------------------------------------------------------------------------
// kernels
// ---------------------------------------------------------------------------

__global__ void k_fill(float* __restrict__ p, int64_t n, float v)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// Latent gradients are summed as 64-bit fixed-point integers (units of
// 2^-44): integer addition is associative, so the scattered sums -- and the
// whole training run -- do not depend on the order of the atomics.
constexpr float kFxScale = 17592186044416.0f;        // 2^44
constexpr float kFxInv = 1.0f / 17592186044416.0f;   // 2^-44

__global__ void k_zero64(int64_t* __restrict__ p, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

__global__ void k_fx_to_float(const int64_t* __restrict__ fx, int64_t n, float* __restrict__ out)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        out[i] = (float)fx[i] * kFxInv;
}

__device__ __forceinline__ int2 sample_xy(uint64_t seed, uint32_t step, int i, int tex_w)
{
    const uint32_t base = pcg_hash((uint32_t)step ^
                                   pcg_hash((uint32_t)(seed >> 32) ^ pcg_hash((uint32_t)seed)));
    const uint32_t h = pcg_hash((uint32_t)i ^ base);
    return make_int2((int)(h & (uint32_t)(tex_w - 1)), (int)(pcg_hash(h) & (uint32_t)(tex_w - 1)));
}

template <int TEX>
__global__ void k_sample(DevTexture T, uint64_t seed, uint32_t step, int batch, int tex_w,
                         int2* __restrict__ xy, float4* __restrict__ target)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= batch) return;
    const int2 p = sample_xy(seed, step, i, tex_w);
    xy[i] = p;
    target[i] = texel_eval<TEX>(T, p.x, p.y);
}

// Procedural targets one channel per thread (channel = blockIdx.y, so the
// terms come through the scalar cache): four times the threads of k_sample
// for the same values.
__global__ void k_sample_sinusoid(DevTexture T, uint64_t seed, uint32_t step, int batch, int tex_w,
                                  int2* __restrict__ xy, float* __restrict__ target)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= batch) return;
    const int c = blockIdx.y;
    const int2 p = sample_xy(seed, step, i, tex_w);
    if (c == 0) xy[i] = p;
    const int xm = p.x & (int)T.wmask, ym = p.y & (int)T.wmask;
    target[4 * (int64_t)i + c] =
        T.fterms ? sinusoid_channel_f(const_fterms(T.fterms) + c * T.n_terms, T.n_terms, (float)xm, (float)ym)
                 : sinusoid_channel(const_terms(T.terms) + c * T.n_terms, T.n_terms, T.wmask, T.inv_w, xm, ym);
}

struct TrainArgs {
    LatentGrid grid;          // low-precision latent copy
    const uint16_t* w;        // packed weights (forward and backward blocks)
    const float* bias;        // packed biases
    int l0, hidden;
    const int2* xy;
    const float4* target;
    int n;                    // samples
    float gscale;             // 2 / (4 n)
    int64_t* glat;            // latent gradient, fixed point (flat, atomics)
    float* partials;          // [workgroups][mlp_count]
    float* loss_part;         // [workgroups]
    int mlp_count;
};

constexpr int kTrainWaves = 4;
// MLP parameters of a decoder with hidden width <= 64 (16H + H + H^2 + H + 4H + 4)
constexpr int kMlpMax = 16 * kHid + kHid + kHid * kHid + kHid + kHid * 4 + 4;

// 16x16 block in C layout (lane: column l%16, rows 4g..4g+3) -> the
// transposed operand (lane: row/column l%16 of the units, k = columns
// 4g..4g+3), through a 512-byte LDS slot.
template <int P>
__device__ __forceinline__ void stage_T(uint16_t* slot, f4 z, int lane)
{
    const int j = lane & 15, g = lane >> 4;
#pragma unroll
    for (int i = 0; i < 4; ++i) slot[(4 * g + i) * 16 + j] = Mfma<P>::cvt(z[i]);
}

__device__ __forceinline__ u16x4 read_T(const uint16_t* slot, int lane)
{
    const int h = lane & 15, g = lane >> 4;
    return *reinterpret_cast<const u16x4*>(slot + h * 16 + 4 * g);
}

// Latent-gradient scatter of one 16-sample tile, staged through LDS so that
// the 8 lanes of each group cover the 8 channels of one latent cell: one
// atomic instruction then touches 8 cache lines instead of 32 (the memory
// system's atomic rate is per line).  Staging per wave: dx [16][2][8] floats,
// corner weights [16][2][4] floats and cells [16][2][4].
struct GradStage {
    float dx[16][2][8];
    float w[16][2][4];
    uint32_t cell[16][2][4];
};

template <int P>
__global__ __launch_bounds__(64 * kTrainWaves, 1) void k_train(TrainArgs a)
{
    __shared__ uint16_t lds[kTrainWaves][18][256];
    __shared__ GradStage gst[kTrainWaves];
    __shared__ float red[kTrainWaves][kMlpMax];   // per-wave MLP gradient partials
    __shared__ float red_loss[kTrainWaves];
    const int wid = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    const int j = lane & 15, g = lane >> 4;
    uint16_t(*S)[256] = lds[wid];
    GradStage& GS = gst[wid];
    const int gw = blockIdx.x * kTrainWaves + wid;
    const int nw = gridDim.x * kTrainWaves;

    FwdWeights<P> W;
    W.load(a.w, lane);
    u16x4 w3a[4];
    u16x8 w2a[4][2], w1a[2];
#pragma unroll
    for (int ob = 0; ob < 4; ++ob) w3a[ob] = *reinterpret_cast<const u16x4*>(a.w + kW3A + (ob * 64 + lane) * 4);
#pragma unroll
    for (int ib = 0; ib < 4; ++ib)
#pragma unroll
        for (int kc = 0; kc < 2; ++kc)
            w2a[ib][kc] = *reinterpret_cast<const u16x8*>(a.w + kW2A + ((ib * 2 + kc) * 64 + lane) * 8);
#pragma unroll
    for (int kc = 0; kc < 2; ++kc) w1a[kc] = *reinterpret_cast<const u16x8*>(a.w + kW1A + (kc * 64 + lane) * 8);
    Biases B;
    B.load(a.bias, lane);

    const f4 zero = {0.f, 0.f, 0.f, 0.f};
    f4 acc1[4], acc2[4][4], acc3[4], ab1[4], ab2[4], ab3 = zero;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        acc1[i] = acc3[i] = ab1[i] = ab2[i] = zero;
#pragma unroll
        for (int k = 0; k < 4; ++k) acc2[i][k] = zero;
    }
    float loss = 0.f;

    // Inputs of a tile: sample coordinates one tile ahead, latent corners and
    // targets requested during the previous tile, before its atomics (the
    // memory counters complete in order, so a wait for loads issued after the
    // atomics would wait for the atomics too).  Every load is unconditional
    // (an index past the batch reads the last sample, n >= 1): a load skipped
    // on some path would make the loop head's wait count for the worst path.
    // A padded sample's features are zeroed, so its gradients are exact
    // zeros and its atomics add nothing.
    const int ntiles = (a.n + 15) / 16;
    const int last = a.n - 1;
    int tile = gw;
    int b = tile * 16 + j;
    int2 p = a.xy[min(b, last)];
    LatentFetch tap;
    latent_fetch(a.grid, p.x, p.y, g, tap);
    float4 t = a.target[min(b, last)];
    int bn = b + 16 * nw;
    int2 pn = a.xy[min(bn, last)];
    // Wait for every load of the prologue (weights, biases, the first tile's
    // inputs) here: the loop head then waits only for what the previous
    // iteration requested, not for its atomics.
    __builtin_amdgcn_s_waitcnt(0);
    for (; tile < ntiles; tile += nw, b = bn, bn += 16 * nw) {
        const bool valid = b < a.n;
        f4 X = latent_combine<P>(tap);
        if (!valid) X = zero;
        f4 z1[4], z2[4];
        const f4 y = mlp_forward<P>(W, B, X, z1, z2);

        // loss and dY (lanes 0..15 hold the 4 channels of their sample)
        f4 dy = zero;
        if (g == 0 && valid) {
            const float e0 = y[0] - t.x, e1 = y[1] - t.y, e2 = y[2] - t.z, e3 = y[3] - t.w;
            loss = __builtin_fmaf(e0, e0, __builtin_fmaf(e1, e1, __builtin_fmaf(e2, e2, __builtin_fmaf(e3, e3, loss))));
            dy[0] = e0 * a.gscale;
            dy[1] = e1 * a.gscale;
            dy[2] = e2 * a.gscale;
            dy[3] = e3 * a.gscale;
        }
        u16x4 dyb;
#pragma unroll
        for (int i = 0; i < 4; ++i) dyb[i] = Mfma<P>::cvt(dy[i]);

        // dZ2 = (W3 dY) * relu'(Z2)
        f4 dz2[4];
#pragma unroll
        for (int ob = 0; ob < 4; ++ob) {
            dz2[ob] = Mfma<P>::k16(w3a[ob], dyb, zero);
#pragma unroll
            for (int i = 0; i < 4; ++i) dz2[ob][i] = z2[ob][i] > 0.f ? dz2[ob][i] : 0.f;
        }
        u16x8 dz2b[2];
#pragma unroll
        for (int kc = 0; kc < 2; ++kc) dz2b[kc] = pack8<P>(dz2[2 * kc], dz2[2 * kc + 1]);
        // dZ1 = (W2 dZ2) * relu'(Z1)
        f4 dz1[4];
#pragma unroll
        for (int ib = 0; ib < 4; ++ib) {
            dz1[ib] = Mfma<P>::k32(w2a[ib][0], dz2b[0], zero);
            dz1[ib] = Mfma<P>::k32(w2a[ib][1], dz2b[1], dz1[ib]);
#pragma unroll
            for (int i = 0; i < 4; ++i) dz1[ib][i] = z1[ib][i] > 0.f ? dz1[ib][i] : 0.f;
        }
        u16x8 dz1b[2];
#pragma unroll
        for (int kc = 0; kc < 2; ++kc) dz1b[kc] = pack8<P>(dz1[2 * kc], dz1[2 * kc + 1]);
        // dX = W1 dZ1: this lane's features of its sample (level g/2,
        // channels 4(g%2)..+3), staged with the corner weights and cells
        f4 dx = Mfma<P>::k32(w1a[0], dz1b[0], zero);
        dx = Mfma<P>::k32(w1a[1], dz1b[1], dx);
        const int lv = g >> 1;
        *reinterpret_cast<f4*>(&GS.dx[j][lv][4 * (g & 1)]) = dx;
        if ((g & 1) == 0) {
            *reinterpret_cast<f4*>(&GS.w[j][lv][0]) = f4{tap.w[0], tap.w[1], tap.w[2], tap.w[3]};
            *reinterpret_cast<uint4*>(&GS.cell[j][lv][0]) = make_uint4(tap.cell[0], tap.cell[1], tap.cell[2], tap.cell[3]);
        }
        wave_lds_sync();

        // next tile's inputs
        latent_fetch(a.grid, pn.x, pn.y, g, tap);
        t = a.target[min(bn, last)];
        pn = a.xy[min(bn + 16 * nw, last)];

        // this tile's latent gradients: instruction k, lane group s8 = lane/8
        // adds channel lane%8 of (sample, level, corner) = combination 8k + s8
        {
            const int c = lane & 7, s8 = lane >> 3;
            const int64_t lvl1 = (int64_t)a.l0 * a.l0 * 8;
#pragma unroll
            for (int k = 0; k < 16; ++k) {
                const int combo = 8 * k + s8;
                const int sm = combo >> 3, l = (combo >> 2) & 1, q = combo & 3;
                const long long v = __float2ll_rn(GS.w[sm][l][q] * GS.dx[sm][l][c] * kFxScale);
                atomicAdd(reinterpret_cast<unsigned long long*>(a.glat + (l ? lvl1 : 0) +
                                                                (int64_t)GS.cell[sm][l][q] * 8 + c),
                          (unsigned long long)v);
            }
            wave_lds_sync();
        }

        // weight gradients: batch contractions on MFMA over the 16 samples
        f4 h1f[4], h2f[4];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                h1f[i][k] = z1[i][k] > 0.f ? z1[i][k] : 0.f;
                h2f[i][k] = z2[i][k] > 0.f ? z2[i][k] : 0.f;
            }
        stage_T<P>(S[0], X, lane);
        stage_T<P>(S[1], dy, lane);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            stage_T<P>(S[2 + i], h1f[i], lane);
            stage_T<P>(S[6 + i], h2f[i], lane);
            stage_T<P>(S[10 + i], dz1[i], lane);
            stage_T<P>(S[14 + i], dz2[i], lane);
        }
        wave_lds_sync();
        const u16x4 tX = read_T(S[0], lane), tdY = read_T(S[1], lane);
        u16x4 tH1[4], tH2[4], tdZ1[4], tdZ2[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            tH1[i] = read_T(S[2 + i], lane);
            tH2[i] = read_T(S[6 + i], lane);
            tdZ1[i] = read_T(S[10 + i], lane);
            tdZ2[i] = read_T(S[14 + i], lane);
        }
        wave_lds_sync();
#pragma unroll
        for (int hb = 0; hb < 4; ++hb) acc1[hb] = Mfma<P>::k16(tdZ1[hb], tX, acc1[hb]);
#pragma unroll
        for (int ob = 0; ob < 4; ++ob)
#pragma unroll
            for (int ib = 0; ib < 4; ++ib) acc2[ob][ib] = Mfma<P>::k16(tdZ2[ob], tH1[ib], acc2[ob][ib]);
#pragma unroll
        for (int ib = 0; ib < 4; ++ib) acc3[ib] = Mfma<P>::k16(tdY, tH2[ib], acc3[ib]);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            ab1[i] += dz1[i];
            ab2[i] += dz2[i];
        }
        ab3 += dy;
    }

    // bias gradients: sum the 16 sample columns of each lane group
#pragma unroll
    for (int o = 1; o < 16; o <<= 1) {
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                ab1[i][k] += __shfl_xor(ab1[i][k], o, 64);
                ab2[i][k] += __shfl_xor(ab2[i][k], o, 64);
            }
#pragma unroll
        for (int k = 0; k < 4; ++k) ab3[k] += __shfl_xor(ab3[k], o, 64);
    }
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) loss += __shfl_xor(loss, o, 64);

    // this wave's partial sums in the flat order (relative to W1), into the
    // workgroup's LDS rows; the workgroup then writes their fixed-order sum
    const int H = a.hidden;
    float* out = red[wid];
    const int oW1 = 0, ob1 = 16 * H, oW2 = ob1 + H, ob2 = oW2 + H * H, oW3 = ob2 + H, ob3 = oW3 + 4 * H;
#pragma unroll
    for (int hb = 0; hb < 4; ++hb)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int h = 16 * hb + 4 * g + r, f = j;
            if (h < H) out[oW1 + f * H + h] = acc1[hb][r];
        }
#pragma unroll
    for (int ob = 0; ob < 4; ++ob)
#pragma unroll
        for (int ib = 0; ib < 4; ++ib)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int o = 16 * ob + 4 * g + r, i = 16 * ib + j;
                if (o < H && i < H) out[oW2 + i * H + o] = acc2[ob][ib][r];
            }
    if (g == 0) {
#pragma unroll
        for (int ib = 0; ib < 4; ++ib)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int h = 16 * ib + j;
                if (h < H) out[oW3 + h * 4 + r] = acc3[ib][r];
            }
    }
    if (j == 0) {
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int h = 16 * i + 4 * g + r;
                if (h < H) {
                    out[ob1 + h] = ab1[i][r];
                    out[ob2 + h] = ab2[i][r];
                }
            }
        if (g == 0)
#pragma unroll
            for (int r = 0; r < 4; ++r) out[ob3 + r] = ab3[r];
    }
    if (lane == 0) red_loss[wid] = loss;
    __syncthreads();
    float* bout = a.partials + (int64_t)blockIdx.x * a.mlp_count;
    for (int i = threadIdx.x; i < a.mlp_count; i += blockDim.x) {
        float v = red[0][i];
#pragma unroll
        for (int w = 1; w < kTrainWaves; ++w) v += red[w][i];
        bout[i] = v;
    }
    if (threadIdx.x == 0) {
        float v = red_loss[0];
#pragma unroll
        for (int w = 1; w < kTrainWaves; ++w) v += red_loss[w];
        a.loss_part[blockIdx.x] = v;
    }
}

// Fixed-order sum of the per-workgroup partials (deterministic), one pass: block
// x sums columns [32x, 32x + 32) of the [rows][mlp_count] matrix (column
// mlp_count: the per-workgroup losses).  Thread (c, r) adds rows r, r + 32, ...
// of column c in order; the 32 row sums are then added as a fixed tree.
constexpr int kRedCols = 32, kRedRows = 32;

__global__ __launch_bounds__(kRedCols * kRedRows) void k_reduce(const float* __restrict__ partials,
                                                                 const float* __restrict__ loss_part, int waves,
                                                                 int mlp_count, float* __restrict__ grad_mlp,
                                                                 float inv_count, float* __restrict__ loss_out)
{
    __shared__ float part[kRedRows][kRedCols + 1];
    const int c = threadIdx.x % kRedCols, r = threadIdx.x / kRedCols;
    const int p = blockIdx.x * kRedCols + c;
    // column p of the partials, or the losses for p == mlp_count
    const float* col = p < mlp_count ? partials + p : loss_part;
    const int64_t stride = p < mlp_count ? (int64_t)mlp_count : 1;
    float s = 0.f;
    if (p <= mlp_count) {
        // eight rows requested at a time, added in row order
        int w = r;
        for (; w + 7 * kRedRows < waves; w += 8 * kRedRows) {
            float x[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) x[u] = col[(int64_t)(w + u * kRedRows) * stride];
#pragma unroll
            for (int u = 0; u < 8; ++u) s += x[u];
        }
        for (; w < waves; w += kRedRows) s += col[(int64_t)w * stride];
    }
    part[r][c] = s;
    __syncthreads();
#pragma unroll
    for (int h = kRedRows / 2; h > 0; h >>= 1) {
        if (r < h) part[r][c] += part[r + h][c];
        __syncthreads();
    }
    if (r == 0) {
        if (p < mlp_count) grad_mlp[p] = part[0][c];
        else if (p == mlp_count && loss_out) loss_out[0] = part[0][c] * inv_count;
    }
}

struct AdamArgs {
    float* master;
    float* m;
    float* v;
    const float* grad;        // MLP part (p >= mlp0)
    int64_t* glat_fx;   // latent part, fixed point
    int64_t total, mlp0;
    int hidden;
    float lr, b1, b2, eps, bc1, bc2;  // bias corrections 1 - beta^t
    uint16_t* lat_lp;
    uint16_t* w_lp;
    float* bias_c;
};

template <int P, bool UPDATE>
__global__ void k_adam(AdamArgs a)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= a.total) return;
    float th = a.master[p];
    if (UPDATE) {
        float gr;
        if (p < a.mlp0) {
            gr = (float)a.glat_fx[p] * kFxInv;
            a.glat_fx[p] = 0;   // ready for the next step's sums
        } else {
            gr = a.grad[p];
        }
        const float m = __builtin_fmaf(a.b1, a.m[p], (1.f - a.b1) * gr);
        const float v = __builtin_fmaf(a.b2, a.v[p], (1.f - a.b2) * gr * gr);
        a.m[p] = m;
        a.v[p] = v;
        const float mh = m / a.bc1, vh = v / a.bc2;
        th -= a.lr * mh / (__builtin_sqrtf(vh) + a.eps);
        a.master[p] = th;
    }
    if (p < a.mlp0) {
        a.lat_lp[p] = Mfma<P>::cvt(th);
    } else {
        const uint16_t lp = Mfma<P>::cvt(th);
        packed_visit((int)(p - a.mlp0), a.hidden, [&](int q) { a.w_lp[q] = lp; }, [&](int q) { a.bias_c[q] = th; });
    }
}

// ---------------------------------------------------------------------------
// host helpers
// ---------------------------------------------------------------------------

ctf_status fail(ctf_status st, const char* msg)
{
    set_error(msg);
    return st;
}

ctf_status hip_fail(hipError_t e, const char* where)
{
    set_error(std::string(where) + ": " + hipGetErrorString(e));
    return e == hipErrorOutOfMemory ? CTF_ERR_OUT_OF_MEMORY : CTF_ERR_DEVICE;
}

struct DeviceScope {
    int prev = -1;
    hipError_t err = hipSuccess;
    explicit DeviceScope(int dev)
    {
        err = hipGetDevice(&prev);
        if (err == hipSuccess && prev != dev) err = hipSetDevice(dev);
    }
    ~DeviceScope()
    {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

LatentGrid latent_grid(const ctf_decoder_desc& d, const uint16_t* base)
{
    LatentGrid G;
    G.base = base;
    G.lvl1 = (uint32_t)((size_t)d.l0 * d.l0 * 16);
    G.log_l0 = ilog2(d.l0);
    G.log_l1 = ilog2(d.l1);
    G.shift0 = ilog2(d.tex_w / d.l0);
    G.shift1 = ilog2(d.tex_w / d.l1);
    G.tex_w = d.tex_w;
    return G;
}

// The inference copy of the latents (see InferGrid): each level padded to
// (L+1) x (L+1) cells by repeating its first row and column.
InferGrid infer_grid(const ctf_decoder_desc& d, const uint16_t* base)
{
    InferGrid G;
    G.base = base;
    G.lvl1 = (uint32_t)((size_t)(d.l0 + 1) * (d.l0 + 1) * 16);
    G.log_l0 = ilog2(d.l0);
    G.log_l1 = ilog2(d.l1);
    G.shift0 = ilog2(d.tex_w / d.l0);
    G.shift1 = ilog2(d.tex_w / d.l1);
    G.tex_w = d.tex_w;
    return G;
}

std::vector<uint16_t> pad_latents(const std::vector<uint16_t>& lat, const ctf_decoder_desc& d)
{
    constexpr int C = 8;
    std::vector<uint16_t> out((size_t)((d.l0 + 1) * (d.l0 + 1) + (d.l1 + 1) * (d.l1 + 1)) * C);
    size_t src = 0, dst = 0;
    for (int L : {d.l0, d.l1}) {
        for (int i = 0; i <= L; ++i)
            for (int j = 0; j <= L; ++j, dst += C)
                for (int c = 0; c < C; ++c) out[dst + c] = lat[src + ((size_t)(i % L) * L + (j % L)) * C + c];
        src += (size_t)L * L * C;
    }
    return out;
}

int train_waves(int n)
{
    const int tiles = (n + 15) / 16;
    int waves = (tiles + 3) / 4;          // about 4 tiles per wave
    if (waves > 1024) waves = 1024;       // one wave per SIMD
    waves = (waves + kTrainWaves - 1) / kTrainWaves * kTrainWaves;
    return waves < kTrainWaves ? kTrainWaves : waves;
}

// Scratch of one loss/gradient pass: per-workgroup partial sums
// [waves / kTrainWaves][mlp_count] and per-workgroup losses.  Every entry a
// pass reads is written by the
// same pass first.
struct PassScratch {
    float* partials;
    float* loss_part;
};

hipError_t ensure_batch(ctf_decoder d, int32_t n)
{
    if (n <= d->cap_batch) return hipSuccess;
    for (void* p : {(void*)d->xy, (void*)d->target, (void*)d->partials, (void*)d->loss_part})
        if (p) (void)hipFree(p);
    d->xy = nullptr;
    d->target = nullptr;
    d->partials = nullptr;
    d->loss_part = nullptr;
    d->cap_batch = 0;
    const int waves = train_waves(n);
    hipError_t e = hipMalloc(&d->xy, (size_t)n * 8);
    if (e == hipSuccess) e = hipMalloc(&d->target, (size_t)n * 16);
    if (e == hipSuccess) e = hipMalloc(&d->partials, (size_t)(waves / kTrainWaves) * d->lay.mlp_count * 4);
    if (e == hipSuccess) e = hipMalloc(&d->loss_part, (size_t)(waves / kTrainWaves) * 4);
    if (e == hipSuccess) d->cap_batch = n;
    return e;
}

PassScratch batch_scratch(ctf_decoder d) { return PassScratch{d->partials, d->loss_part}; }

template <int P, bool UPDATE>
hipError_t launch_adam(ctf_decoder d, float lr, hipStream_t s)
{
    AdamArgs a;
    a.master = d->master;
    a.m = d->m;
    a.v = d->v;
    a.grad = d->grad;
    a.glat_fx = d->glat_fx;
    a.total = d->lay.total;
    a.mlp0 = d->lay.mlp0;
    a.hidden = d->desc.hidden;
    a.lr = lr;
    a.b1 = 0.9f;
    a.b2 = 0.999f;
    a.eps = 1e-8f;
    a.bc1 = (float)(1.0 - std::pow(0.9, (double)d->step));
    a.bc2 = (float)(1.0 - std::pow(0.999, (double)d->step));
    a.lat_lp = d->lat_lp;
    a.w_lp = d->w_lp;
    a.bias_c = d->bias_c;
    const int bs = 256;
    hipLaunchKernelGGL((k_adam<P, UPDATE>), dim3((unsigned)((a.total + bs - 1) / bs)), dim3(bs), 0, s, a);
    return hipGetLastError();
}

// Make the low-precision copies hold `precision` (repacked from the master).
hipError_t ensure_lp(ctf_decoder d, int precision, hipStream_t s)
{
    if (d->lp_precision == precision) return hipSuccess;
    // a fill kernel rather than a memset node, so the call can be captured
    hipLaunchKernelGGL(k_fill, dim3(8), dim3(256), 0, s, reinterpret_cast<float*>(d->w_lp), (int64_t)(kAllElems / 2), 0.f);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = precision == CTF_BF16 ? launch_adam<CTF_BF16, false>(d, 0.f, s) : launch_adam<CTF_FP16, false>(d, 0.f, s);
    if (e == hipSuccess) d->lp_precision = precision;
    return e;
}

// Loss and gradient of a batch: the MLP part lands in grad[mlp0..]; the
// latent part in d->glat_fx (fixed point), copied to grad[0..mlp0) as float
// when latent_to_grad is set (training reads the fixed-point sums directly).
// zero_latent clears the fixed-point sums first; the training loop clears
// them once and then relies on the Adam step, which zeroes what it reads.
template <int P>
hipError_t loss_grad_impl(ctf_decoder d, const int32_t* xy, const float* target, int32_t n,
                          float* loss, float* grad, bool latent_to_grad, bool zero_latent,
                          const PassScratch& sc, hipStream_t s)
{
    const Layout& L = d->lay;
    const int fb = 1024;
    if (zero_latent) hipLaunchKernelGGL(k_zero64, dim3(fb), dim3(256), 0, s, d->glat_fx, L.mlp0);
    TrainArgs a;
    a.grid = latent_grid(d->desc, d->lat_lp);
    a.w = d->w_lp;
    a.bias = d->bias_c;
    a.l0 = d->desc.l0;
    a.hidden = d->desc.hidden;
    a.xy = reinterpret_cast<const int2*>(xy);
    a.target = reinterpret_cast<const float4*>(target);
    a.n = n;
    a.gscale = 2.0f / (4.0f * (float)n);
    a.glat = d->glat_fx;
    a.partials = sc.partials;
    a.loss_part = sc.loss_part;
    a.mlp_count = (int)L.mlp_count;
    const int waves = train_waves(n);
    hipLaunchKernelGGL((k_train<P>), dim3(waves / kTrainWaves), dim3(64 * kTrainWaves), 0, s, a);
    const unsigned gx = (unsigned)((L.mlp_count + 1 + kRedCols - 1) / kRedCols);
    // one partial row per workgroup (the sum of its waves' rows)
    hipLaunchKernelGGL(k_reduce, dim3(gx), dim3(kRedCols * kRedRows), 0, s, sc.partials, sc.loss_part,
                       waves / kTrainWaves, (int)L.mlp_count, grad + L.mlp0, 1.0f / (4.0f * (float)n), loss);
    if (latent_to_grad) hipLaunchKernelGGL(k_fx_to_float, dim3(fb), dim3(256), 0, s, d->glat_fx, L.mlp0, grad);
    return hipGetLastError();
}

}  // namespace

// ---------------------------------------------------------------------------
// Scratch of the allocation-free loss/gradient call.  One fixed array per
// device (the code object's own copy), sized for CTF_NOALLOC_MAX_SAMPLES
// samples of a decoder with hidden width <= 64: the per-workgroup partial
// sums and losses of one pass (PassScratch).  Host code
// never passes `scratch` itself to a kernel: its device address is looked up
// once per device at context creation (ctf_create) and kept in
// g_scratch_dev.  Calls on one device share the array.
// ---------------------------------------------------------------------------

constexpr int kNoAllocWaves = 256;   // train_waves(CTF_NOALLOC_MAX_SAMPLES)
constexpr int kNoAllocMlp = 16 * kHid + kHid + kHid * kHid + kHid + kHid * 4 + 4;
constexpr int kNoAllocGroups = kNoAllocWaves / kTrainWaves;
constexpr size_t kNoAllocPartials = (size_t)kNoAllocGroups * kNoAllocMlp;
constexpr size_t kNoAllocFloats = kNoAllocPartials + kNoAllocGroups;
constexpr int kMaxScratchDevices = 64;

static __device__ __align__(256) float scratch[kNoAllocFloats];

namespace {
std::mutex g_scratch_mu;
float* g_scratch_dev[kMaxScratchDevices] = {};

float* scratch_address(int device)
{
    if (device < 0 || device >= kMaxScratchDevices) return nullptr;
    std::lock_guard<std::mutex> g(g_scratch_mu);
    return g_scratch_dev[device];
}
}  // namespace

// Called by ctf_create with `device` current.
hipError_t ctf::noalloc_scratch_init(int device)
{
    if (device < 0 || device >= kMaxScratchDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (g_scratch_dev[device]) return hipSuccess;
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch_dev[device] = static_cast<float*>(p);
    return hipSuccess;
}

extern "C" {

size_t ctf_decoder_param_count(const ctf_decoder_desc* d)
{
    if (!d) return 0;
    return (size_t)layout_of(*d).total;
}

ctf_status ctf_decoder_destroy(ctf_decoder d)
{
    if (!d) return fail(CTF_ERR_INVALID_ARG, "ctf_decoder_destroy: NULL decoder");
    DeviceScope ds(d->ctx->device);
    for (void* p : {(void*)d->master, (void*)d->m, (void*)d->v, (void*)d->grad, (void*)d->glat_fx, (void*)d->lat_lp,
                    (void*)d->w_lp, (void*)d->bias_c, (void*)d->xy, (void*)d->target,
                    (void*)d->partials, (void*)d->loss_part, (void*)d->loss_tmp})
        if (p) (void)hipFree(p);
    delete d;
    set_error("");
    return CTF_OK;
}

ctf_status ctf_decoder_create(ctf_context ctx, const ctf_decoder_desc* desc, const float* init,
                              ctf_decoder* out)
{
    set_error("");
    if (!ctx || !desc || !init || !out) return fail(CTF_ERR_INVALID_ARG, "ctf_decoder_create: NULL argument");
    *out = nullptr;
    const ctf_decoder_desc& d = *desc;
    if (d.channels != 8) return fail(CTF_ERR_UNSUPPORTED, "ctf_decoder_create: channels must be 8");
    if (d.hidden < 4 || d.hidden > kHid || d.hidden % 4)
        return fail(CTF_ERR_UNSUPPORTED, "ctf_decoder_create: hidden must be a multiple of 4 in 4..64");
    if (!pow2(d.tex_w) || !pow2(d.l0) || !pow2(d.l1) || d.l0 > d.tex_w || d.l1 > d.tex_w || d.l0 < 2 || d.l1 < 2 ||
        d.tex_w > (1 << 22))
        return fail(CTF_ERR_INVALID_ARG, "ctf_decoder_create: tex_w, l0, l1 powers of two, 2 <= l <= tex_w");
    // latent byte offsets are 32-bit (the inference copy pads each level to (l+1)^2 cells)
    if (d.l0 > 8192 || d.l1 > 8192) return fail(CTF_ERR_UNSUPPORTED, "ctf_decoder_create: l0, l1 above 8192");
    DeviceScope ds(ctx->device);
    if (ds.err != hipSuccess) return hip_fail(ds.err, "ctf_decoder_create: set device");
    ctf_decoder dec = new (std::nothrow) ctf_decoder_s;
    if (!dec) return fail(CTF_ERR_OUT_OF_MEMORY, "ctf_decoder_create: host allocation");
    dec->ctx = ctx;
    dec->desc = d;
    dec->lay = layout_of(d);
    const size_t bytes = (size_t)dec->lay.total * 4;
    hipError_t e = hipMalloc(&dec->master, bytes);
    if (e == hipSuccess) e = hipMalloc(&dec->m, bytes);
    if (e == hipSuccess) e = hipMalloc(&dec->v, bytes);
    if (e == hipSuccess) e = hipMalloc(&dec->grad, bytes);
    if (e == hipSuccess) e = hipMalloc(&dec->glat_fx, (size_t)dec->lay.mlp0 * 8);
    if (e == hipSuccess) e = hipMalloc(&dec->lat_lp, (size_t)dec->lay.mlp0 * 2);
    if (e == hipSuccess) e = hipMalloc(&dec->w_lp, kAllElems * 2);
    if (e == hipSuccess) e = hipMalloc(&dec->bias_c, kBiasFloats * 4);
    if (e == hipSuccess) e = hipMalloc(&dec->loss_tmp, 4);
    if (e == hipSuccess) e = hipMemcpy(dec->master, init, bytes, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemset(dec->m, 0, bytes);
    if (e == hipSuccess) e = hipMemset(dec->v, 0, bytes);
    if (e == hipSuccess) e = hipMemset(dec->bias_c, 0, kBiasFloats * 4);
    if (e != hipSuccess) {
        ctf_decoder_destroy(dec);
        return hip_fail(e, "ctf_decoder_create");
    }
    *out = dec;
    return CTF_OK;
}

ctf_status ctf_decoder_get_params(ctf_decoder d, float* host, size_t count)
{
    set_error("");
    if (!d || !host || count != (size_t)d->lay.total)
        return fail(CTF_ERR_INVALID_ARG, "ctf_decoder_get_params: bad arguments or count");
    DeviceScope ds(d->ctx->device);
    if (ds.err != hipSuccess) return hip_fail(ds.err, "ctf_decoder_get_params: set device");
    hipError_t e = hipDeviceSynchronize();
    if (e == hipSuccess) e = hipMemcpy(host, d->master, count * 4, hipMemcpyDeviceToHost);
    return e == hipSuccess ? CTF_OK : hip_fail(e, "ctf_decoder_get_params");
}

ctf_status ctf_decoder_set_params(ctf_decoder d, const float* host, size_t count)
{
    set_error("");
    if (!d || !host || count != (size_t)d->lay.total)
        return fail(CTF_ERR_INVALID_ARG, "ctf_decoder_set_params: bad arguments or count");
    DeviceScope ds(d->ctx->device);
    if (ds.err != hipSuccess) return hip_fail(ds.err, "ctf_decoder_set_params: set device");
    hipError_t e = hipDeviceSynchronize();
    if (e == hipSuccess) e = hipMemcpy(d->master, host, count * 4, hipMemcpyHostToDevice);
    d->lp_precision = -1;
    return e == hipSuccess ? CTF_OK : hip_fail(e, "ctf_decoder_set_params");
}

size_t ctf_decoder_state_bytes(ctf_decoder d)
{
    if (!d) return 0;
    return 16 + (size_t)d->lay.total * 12;
}

ctf_status ctf_decoder_get_state(ctf_decoder d, void* host, size_t bytes)
{
    set_error("");
    if (!d || !host || bytes != ctf_decoder_state_bytes(d))
        return fail(CTF_ERR_INVALID_ARG, "ctf_decoder_get_state: bad arguments or size");
    DeviceScope ds(d->ctx->device);
    if (ds.err != hipSuccess) return hip_fail(ds.err, "ctf_decoder_get_state: set device");
    char* p = static_cast<char*>(host);
    const int64_t hdr[2] = {d->step, d->lay.total};
    std::memcpy(p, hdr, 16);
    const size_t n = (size_t)d->lay.total * 4;
    hipError_t e = hipDeviceSynchronize();
    if (e == hipSuccess) e = hipMemcpy(p + 16, d->master, n, hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(p + 16 + n, d->m, n, hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(p + 16 + 2 * n, d->v, n, hipMemcpyDeviceToHost);
    return e == hipSuccess ? CTF_OK : hip_fail(e, "ctf_decoder_get_state");
}

ctf_status ctf_decoder_set_state(ctf_decoder d, const void* host, size_t bytes)
{
    set_error("");
    if (!d || !host || bytes != ctf_decoder_state_bytes(d))
        return fail(CTF_ERR_INVALID_ARG, "ctf_decoder_set_state: bad arguments or size");
    const char* p = static_cast<const char*>(host);
    int64_t hdr[2];
    std::memcpy(hdr, p, 16);
    if (hdr[1] != d->lay.total || hdr[0] < 0) return fail(CTF_ERR_INVALID_ARG, "ctf_decoder_set_state: blob mismatch");
    DeviceScope ds(d->ctx->device);
    if (ds.err != hipSuccess) return hip_fail(ds.err, "ctf_decoder_set_state: set device");
    const size_t n = (size_t)d->lay.total * 4;
    hipError_t e = hipDeviceSynchronize();
    if (e == hipSuccess) e = hipMemcpy(d->master, p + 16, n, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(d->m, p + 16 + n, n, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(d->v, p + 16 + 2 * n, n, hipMemcpyHostToDevice);
    d->step = hdr[0];
    d->lp_precision = -1;
    return e == hipSuccess ? CTF_OK : hip_fail(e, "ctf_decoder_set_state");
}

ctf_status ctf_decoder_loss_grad(ctf_decoder d, const int32_t* xy, const float* target, int32_t n,
                                 int32_t precision, float* loss, float* grad, void* stream)
{
    set_error("");
    if (!d || !xy || !target || !loss || !grad || n <= 0)
        return fail(CTF_ERR_INVALID_ARG, "ctf_decoder_loss_grad: bad arguments");
    if (precision != CTF_BF16 && precision != CTF_FP16)
        return fail(CTF_ERR_INVALID_ARG, "ctf_decoder_loss_grad: precision");
    DeviceScope ds(d->ctx->device);
    if (ds.err != hipSuccess) return hip_fail(ds.err, "ctf_decoder_loss_grad: set device");
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = ensure_batch(d, n);
    if (e == hipSuccess) e = ensure_lp(d, precision, s);
    if (e == hipSuccess)
        e = precision == CTF_BF16 ? loss_grad_impl<CTF_BF16>(d, xy, target, n, loss, grad, true, true, batch_scratch(d), s)
                                  : loss_grad_impl<CTF_FP16>(d, xy, target, n, loss, grad, true, true, batch_scratch(d), s);
    return e == hipSuccess ? CTF_OK : hip_fail(e, "ctf_decoder_loss_grad");
}

ctf_status ctf_decoder_loss_grad_noalloc(ctf_decoder d, const int32_t* xy, const float* target, int32_t n,
                                         int32_t precision, float* loss, float* grad, void* stream)
{
    set_error("");
    if (!d || !xy || !target || !loss || !grad || n <= 0)
        return fail(CTF_ERR_INVALID_ARG, "ctf_decoder_loss_grad_noalloc: bad arguments");
    if (n > CTF_NOALLOC_MAX_SAMPLES)
        return fail(CTF_ERR_INVALID_ARG, "ctf_decoder_loss_grad_noalloc: n above CTF_NOALLOC_MAX_SAMPLES");
    if (precision != CTF_BF16 && precision != CTF_FP16)
        return fail(CTF_ERR_INVALID_ARG, "ctf_decoder_loss_grad_noalloc: precision");
    if (train_waves(n) > kNoAllocWaves || d->lay.mlp_count > kNoAllocMlp)
        return fail(CTF_ERR_INVALID_ARG, "ctf_decoder_loss_grad_noalloc: pass does not fit the scratch array");
    float* base = scratch_address(d->ctx->device);
    if (!base) return fail(CTF_ERR_DEVICE, "ctf_decoder_loss_grad_noalloc: scratch address of the device not set up");
    DeviceScope ds(d->ctx->device);
    if (ds.err != hipSuccess) return hip_fail(ds.err, "ctf_decoder_loss_grad_noalloc: set device");
    hipStream_t s = (hipStream_t)stream;
    const PassScratch sc{base, base + kNoAllocPartials};
    hipError_t e = ensure_lp(d, precision, s);
    if (e == hipSuccess)
        e = precision == CTF_BF16 ? loss_grad_impl<CTF_BF16>(d, xy, target, n, loss, grad, true, true, sc, s)
                                  : loss_grad_impl<CTF_FP16>(d, xy, target, n, loss, grad, true, true, sc, s);
    return e == hipSuccess ? CTF_OK : hip_fail(e, "ctf_decoder_loss_grad_noalloc");
}

ctf_status ctf_decoder_train(ctf_decoder d, ctf_texture target, int64_t steps, int32_t batch, float lr,
                             uint64_t seed, int32_t precision, float* loss_trace, void* stream)
{
    set_error("");
    if (!d || !target || steps < 0 || batch <= 0 || !(lr > 0.f))
        return fail(CTF_ERR_INVALID_ARG, "ctf_decoder_train: bad arguments");
    if (precision != CTF_BF16 && precision != CTF_FP16)
        return fail(CTF_ERR_INVALID_ARG, "ctf_decoder_train: precision");
    const DevTexture& T = target->dev;
    if (target->ctx->device != d->ctx->device)
        return fail(CTF_ERR_INVALID_ARG, "ctf_decoder_train: target texture on another device");
    if (T.kind == CTF_TEX_DECODER) return fail(CTF_ERR_UNSUPPORTED, "ctf_decoder_train: decoder targets not built");
    if (T.width != d->desc.tex_w || T.height != d->desc.tex_w)
        return fail(CTF_ERR_INVALID_ARG, "ctf_decoder_train: target size differs from the decoder's tex_w");
    DeviceScope ds(d->ctx->device);
    if (ds.err != hipSuccess) return hip_fail(ds.err, "ctf_decoder_train: set device");
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = ensure_batch(d, batch);
    if (e == hipSuccess) e = ensure_lp(d, precision, s);
    if (e != hipSuccess) return hip_fail(e, "ctf_decoder_train: setup");
    const int sb = 256;
    if (steps > 0) hipLaunchKernelGGL(k_zero64, dim3(1024), dim3(256), 0, s, d->glat_fx, d->lay.mlp0);
    for (int64_t it = 0; it < steps && e == hipSuccess; ++it) {
        const dim3 sg((unsigned)((batch + sb - 1) / sb));
        int2* xy = reinterpret_cast<int2*>(d->xy);
        float4* tg = reinterpret_cast<float4*>(d->target);
        const uint32_t st = (uint32_t)d->step;
        switch (T.kind) {
        case CTF_TEX_SINUSOIDS:
            hipLaunchKernelGGL(k_sample_sinusoid, dim3(sg.x, 4), dim3(sb), 0, s, T, seed, st, batch, d->desc.tex_w, xy,
                               reinterpret_cast<float*>(tg));
            break;
        case CTF_TEX_AFFINE:
            hipLaunchKernelGGL(k_sample<CTF_TEX_AFFINE>, sg, dim3(sb), 0, s, T, seed, st, batch, d->desc.tex_w, xy, tg);
            break;
        case CTF_TEX_CONSTANT:
            hipLaunchKernelGGL(k_sample<CTF_TEX_CONSTANT>, sg, dim3(sb), 0, s, T, seed, st, batch, d->desc.tex_w, xy, tg);
            break;
        default:
            hipLaunchKernelGGL(k_sample<CTF_TEX_TABLE>, sg, dim3(sb), 0, s, T, seed, st, batch, d->desc.tex_w, xy, tg);
        }
        float* lt = loss_trace ? loss_trace + it : d->loss_tmp;
        e = precision == CTF_BF16
                ? loss_grad_impl<CTF_BF16>(d, d->xy, d->target, batch, lt, d->grad, false, false, batch_scratch(d), s)
                : loss_grad_impl<CTF_FP16>(d, d->xy, d->target, batch, lt, d->grad, false, false, batch_scratch(d), s);
        if (e != hipSuccess) break;
        d->step += 1;
        e = precision == CTF_BF16 ? launch_adam<CTF_BF16, true>(d, lr, s) : launch_adam<CTF_FP16, true>(d, lr, s);
    }
    return e == hipSuccess ? CTF_OK : hip_fail(e, "ctf_decoder_train");
}

}  // extern "C"

// ---------------------------------------------------------------------------
// inference snapshot for decoder textures
// ---------------------------------------------------------------------------

ctf_status ctf_internal_decoder_texture(ctf_texture t)
{
    ctf_decoder d = t->desc.decoder;
    const int prec = t->desc.precision;
    if (d->ctx->device != t->ctx->device)
        return fail(CTF_ERR_INVALID_ARG, "decoder texture: the decoder lives on another device");
    if (t->desc.width != d->desc.tex_w || t->desc.height != d->desc.tex_w)
        return fail(CTF_ERR_INVALID_ARG, "decoder texture: width/height must equal the decoder's tex_w");
    std::vector<float> P((size_t)d->lay.total);
    hipError_t e = hipDeviceSynchronize();
    if (e == hipSuccess) e = hipMemcpy(P.data(), d->master, P.size() * 4, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "decoder texture: read parameters");
    std::vector<uint16_t> lat, w;
    std::vector<float> bias;
    pack_host(P.data(), d->desc, prec, lat, w, bias);
    lat = pad_latents(lat, d->desc);
    const size_t lat_b = lat.size() * 2, w_b = w.size() * 2, b_b = bias.size() * 4;
    const size_t o_w = (lat_b + 255) / 256 * 256, o_b = o_w + (w_b + 255) / 256 * 256;
    char* buf = nullptr;
    e = hipMalloc(&buf, o_b + b_b);
    if (e == hipSuccess) e = hipMemcpy(buf, lat.data(), lat_b, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(buf + o_w, w.data(), w_b, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(buf + o_b, bias.data(), b_b, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        if (buf) (void)hipFree(buf);
        return hip_fail(e, "decoder texture: upload");
    }
    t->dec_buf = buf;
    DevDecoderWeights& W = t->dec;
    W.grid = infer_grid(d->desc, reinterpret_cast<const uint16_t*>(buf));
    W.precision = prec;
    W.w = reinterpret_cast<const uint16_t*>(buf + o_w);
    W.bias = reinterpret_cast<const float*>(buf + o_b);
    return CTF_OK;
}
