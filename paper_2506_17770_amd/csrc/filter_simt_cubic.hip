// filter_simt_cubic.hip -- per-lane filter kernels for the bicubic filters
// of Section 5 (uniform cubic B-spline, Catmull-Rom; 4x4 footprints).
#include "filter_simt.h"

namespace ctf {

hipError_t launch_filter_simt_cubic(const FilterArgs& a, const DevTexture& T, hipStream_t s)
{
    if (a.filter == CTF_FILTER_BSPLINE) return simt::launch_filter<CTF_FILTER_BSPLINE>(a, T, s);
    if (a.filter == CTF_FILTER_CATMULL_ROM) return simt::launch_filter<CTF_FILTER_CATMULL_ROM>(a, T, s);
    return hipErrorInvalidValue;
}

}  // namespace ctf
