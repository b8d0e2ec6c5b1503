// filter_decoder.hip -- decoder-path filter for the bilinear filter, the
// multi-layer launch and raw decoder evaluation (tile logic in
// filter_decoder.h; the bicubic instantiations are compiled in
// filter_decoder_cubic.hip).
#include "filter_decoder.h"

hipError_t ctf_internal_decoder_filter_cubic(const ctf_texture_s* t, const ctf::FilterArgs& a, hipStream_t s);
hipError_t ctf_internal_filter_layers_cubic(const ctf::dec::LayerSet& LS, int precision, const ctf::FilterArgs& a,
                                            hipStream_t s);

namespace ctf {

namespace {

using namespace dec;

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
    if (a.filter != CTF_FILTER_BILINEAR) return ctf_internal_filter_layers_cubic(LS, prec, a, s);
    return prec == CTF_BF16 ? launch_layers_p<CTF_BF16, CTF_FILTER_BILINEAR>(a, LS, s)
                            : launch_layers_p<CTF_FP16, CTF_FILTER_BILINEAR>(a, LS, s);
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
