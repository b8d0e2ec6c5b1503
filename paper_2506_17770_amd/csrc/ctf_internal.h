// ctf_internal.h -- host-side structures shared by the library's sources.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "ctf.h"
#include "ctf_device.h"
#include "decoder_mlp.h"

namespace ctf {

struct FilterArgs {
    const float* uv;
    const float* duv;
    float* out;
    int sw, sh;
    int tiles_x;
    int64_t ntiles;
    int method;
    int box_w, box_h;
    int max_evals;
    int fallback;               // CTF_FB_* for the lanes of a failed wave
    int filter;                 // CTF_FILTER_*
    int split;                  // CTF_SPLIT_*
    int wave_shape;             // CTF_WAVE_*
    uint64_t seed;
    uint32_t layer;
    ctf_tile_stats* tile_stats;
    ctf_frame_stats* frame_stats;
    int32_t* lists;
    int32_t* stf_xy;
};

// Decoder parameters in the layouts the MFMA kernels read (built once per
// texture from the float32 master copy; see decoder_mlp.h).
struct DevDecoderWeights {
    InferGrid grid;              // latents, 16-bit, both levels, padded inference layout
    int precision;               // CTF_FP16 / CTF_BF16
    const uint16_t* w;           // packed A-operand weight blocks
    const float* bias;           // packed C-operand biases
};

hipError_t launch_filter_simt(const FilterArgs& a, const DevTexture& T, hipStream_t s);
hipError_t launch_filter_simt_cubic(const FilterArgs& a, const DevTexture& T, hipStream_t s);
hipError_t launch_filter_w32(const FilterArgs& a, const DevTexture& T, hipStream_t s);
hipError_t launch_texel_eval_simt(const DevTexture& T, const int32_t* xy, int64_t n, float* out,
                                  hipStream_t s);

void set_error(const std::string& msg);

// Looks up the device address of the allocation-free call's scratch array
// for `device` (which must be current); done once per device.
hipError_t noalloc_scratch_init(int device);

}  // namespace ctf

struct ctf_context_s {
    int device;
};

struct ctf_decoder_s;

struct ctf_texture_s {
    ctf_context ctx;
    ctf_texture_desc desc;
    ctf::DevTexture dev;
    void* terms = nullptr;      // device int4 [4][K], then float4 [4][K] (DevTexture::fterms)
    void* table = nullptr;      // device float4 [H][W]
    void* dec_buf = nullptr;    // device decoder weights (one allocation)
    ctf::DevDecoderWeights dec{};
};
