// filter_decoder.hip -- decoder-path filter for the bilinear filter, the
// multi-layer launch and raw decoder evaluation (tile logic in
// filter_decoder.h; the bicubic instantiations are compiled in
// filter_decoder_cubic.hip).
#include "filter_decoder.h"

hipError_t ctf_internal_decoder_filter_cubic(const ctf_texture_s* t, const ctf::FilterArgs& a, hipStream_t s);

namespace ctf {

namespace {

using namespace dec;

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
__global__ __launch_bounds__(64 * kDecWaves, (dec_waves_per_simd<METHOD, CTF_FILTER_BILINEAR>())) void
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
            dec_tile<METHOD, P, STATS, FB, CTF_FILTER_BILINEAR>(al, D.grid, W, Bz, L, cur.tile, cur.tx, cur.ty, f, fc);
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
    const InferLane<P> K(D.grid, g);
    const int64_t ntiles = (n + 15) / 16;
    for (int64_t t = gw; t < ntiles; t += nw) {
        const int64_t row = t * 16 + j;
        const bool valid = row < n;
        const int2 p = valid ? xy[row] : make_int2(0, 0);
        InferFetch F;
        infer_fetch<P>(D.grid, K, p.x, p.y, F);
        const f4 y = mlp_forward_b<P>(W, Bz, infer_combine<P>(F), nullptr, nullptr);
        if (g == 0 && valid) out[row] = make_float4(y[0], y[1], y[2], y[3]);
    }
}

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

}  // namespace

}  // namespace ctf

using namespace ctf;
using namespace ctf::dec;

hipError_t ctf_internal_decoder_filter(const ctf_texture_s* t, const FilterArgs& a, hipStream_t s)
{
    if (a.filter != CTF_FILTER_BILINEAR) return ctf_internal_decoder_filter_cubic(t, a, s);
    const DevDecoderWeights& d = t->dec;
    return t->dec.precision == CTF_BF16 ? launch_dec_p<CTF_BF16, CTF_FILTER_BILINEAR>(a, d, s)
                                        : launch_dec_p<CTF_FP16, CTF_FILTER_BILINEAR>(a, d, s);
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
