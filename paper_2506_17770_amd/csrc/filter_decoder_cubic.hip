// filter_decoder_cubic.hip -- decoder-path filter kernels for the bicubic
// filters of Section 5 (uniform cubic B-spline, Catmull-Rom; 4x4 footprints),
// single-layer and layered.
#include "filter_decoder.h"

using namespace ctf;
using namespace ctf::dec;

hipError_t ctf_internal_decoder_filter_cubic(const ctf_texture_s* t, const FilterArgs& a, hipStream_t s)
{
    const DevDecoderWeights& d = t->dec;
    const bool bf = t->dec.precision == CTF_BF16;
    if (a.filter == CTF_FILTER_BSPLINE)
        return bf ? launch_dec_p<CTF_BF16, CTF_FILTER_BSPLINE>(a, d, s) : launch_dec_p<CTF_FP16, CTF_FILTER_BSPLINE>(a, d, s);
    if (a.filter == CTF_FILTER_CATMULL_ROM)
        return bf ? launch_dec_p<CTF_BF16, CTF_FILTER_CATMULL_ROM>(a, d, s)
                  : launch_dec_p<CTF_FP16, CTF_FILTER_CATMULL_ROM>(a, d, s);
    return hipErrorInvalidValue;
}

hipError_t ctf_internal_filter_layers_cubic(const LayerSet& LS, int precision, const FilterArgs& a, hipStream_t s)
{
    const bool bf = precision == CTF_BF16;
    if (a.filter == CTF_FILTER_BSPLINE)
        return bf ? launch_layers_p<CTF_BF16, CTF_FILTER_BSPLINE>(a, LS, s)
                  : launch_layers_p<CTF_FP16, CTF_FILTER_BSPLINE>(a, LS, s);
    if (a.filter == CTF_FILTER_CATMULL_ROM)
        return bf ? launch_layers_p<CTF_BF16, CTF_FILTER_CATMULL_ROM>(a, LS, s)
                  : launch_layers_p<CTF_FP16, CTF_FILTER_CATMULL_ROM>(a, LS, s);
    return hipErrorInvalidValue;
}
