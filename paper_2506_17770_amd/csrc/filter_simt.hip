// filter_simt.hip -- per-lane filter kernels for the bilinear filter, the
// filter dispatcher and raw texel evaluation (kernels in filter_simt.h; the
// bicubic instantiations are compiled in filter_simt_cubic.hip).
#include "filter_simt.h"

namespace ctf {

namespace {

template <int TEX>
__global__ void k_texel_eval(DevTexture T, const int2* __restrict__ xy, int64_t n,
                             float4* __restrict__ out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        const int2 p = xy[i];
        out[i] = texel_eval<TEX>(T, p.x, p.y);
    }
}

}  // namespace

hipError_t launch_filter_simt(const FilterArgs& a, const DevTexture& T, hipStream_t s)
{
    switch (a.filter) {
    case CTF_FILTER_BILINEAR: return simt::launch_filter<CTF_FILTER_BILINEAR>(a, T, s);
    case CTF_FILTER_BSPLINE:
    case CTF_FILTER_CATMULL_ROM: return launch_filter_simt_cubic(a, T, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_texel_eval_simt(const DevTexture& T, const int32_t* xy, int64_t n, float* out,
                                  hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    const int bs = 256;
    // one launch per 2^30 points keeps the grid's work-item count within 32 bits
    constexpr int64_t kChunk = int64_t(1) << 30;
    for (int64_t off = 0; off < n; off += kChunk) {
        const int64_t m = n - off < kChunk ? n - off : kChunk;
        const dim3 grid((unsigned)((m + bs - 1) / bs));
        const int2* p = reinterpret_cast<const int2*>(xy) + off;
        float4* o = reinterpret_cast<float4*>(out) + off;
        switch (T.kind) {
        case CTF_TEX_SINUSOIDS:
            hipLaunchKernelGGL(k_texel_eval<CTF_TEX_SINUSOIDS>, grid, dim3(bs), 0, s, T, p, m, o);
            break;
        case CTF_TEX_AFFINE:
            hipLaunchKernelGGL(k_texel_eval<CTF_TEX_AFFINE>, grid, dim3(bs), 0, s, T, p, m, o);
            break;
        case CTF_TEX_CONSTANT:
            hipLaunchKernelGGL(k_texel_eval<CTF_TEX_CONSTANT>, grid, dim3(bs), 0, s, T, p, m, o);
            break;
        case CTF_TEX_TABLE:
            hipLaunchKernelGGL(k_texel_eval<CTF_TEX_TABLE>, grid, dim3(bs), 0, s, T, p, m, o);
            break;
        default: return hipErrorInvalidValue;
        }
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace ctf
