// api.hip -- the C ABI (include/ctf.h): contexts, textures, filtering.
#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdio>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "ctf.h"
#include "ctf_internal.h"

namespace ctf {

static thread_local std::string g_error;

void set_error(const std::string& msg) { g_error = msg; }

}  // namespace ctf

using namespace ctf;

namespace {

ctf_status fail(ctf_status st, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    set_error(buf);
    return st;
}

ctf_status hip_fail(hipError_t e, const char* where)
{
    if (e == hipErrorOutOfMemory)
        return fail(CTF_ERR_OUT_OF_MEMORY, "%s: %s", where, hipGetErrorString(e));
    return fail(CTF_ERR_DEVICE, "%s: %s", where, hipGetErrorString(e));
}

// Makes the context's device current for the scope of a call.
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

bool pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

// Screen sides up to 2^24: a lane's pixel offset inside its tile (up to
// 7 rows of the screen, 16 bytes a pixel) then fits the kernels' 32-bit
// offsets, and pixel coordinates stay far from int32 overflow.
constexpr int32_t kMaxScreenSide = 1 << 24;

}  // namespace

// decoder.hip / filter_decoder.hip
ctf_status ctf_internal_decoder_texture(ctf_texture t);
hipError_t ctf_internal_decoder_eval(const ctf_texture_s* t, const int32_t* xy, int64_t n, float* out,
                                     hipStream_t s);
hipError_t ctf_internal_decoder_filter(const ctf_texture_s* t, const FilterArgs& a, hipStream_t s);
hipError_t ctf_internal_filter_layers(const ctf_texture_s* const* texs, const float* xforms, int n,
                                      const FilterArgs& a, hipStream_t s);

extern "C" {

const char* ctf_last_error(void) { return g_error.c_str(); }

ctf_status ctf_create(int device, ctf_context* out)
{
    set_error("");
    if (!out) return fail(CTF_ERR_INVALID_ARG, "ctf_create: out is NULL");
    *out = nullptr;
    int n = 0;
    hipError_t e = hipGetDeviceCount(&n);
    if (e != hipSuccess) return hip_fail(e, "ctf_create: hipGetDeviceCount");
    if (device < 0 || device >= n)
        return fail(CTF_ERR_INVALID_ARG, "ctf_create: device %d not in [0, %d)", device, n);
    hipDeviceProp_t prop;
    e = hipGetDeviceProperties(&prop, device);
    if (e != hipSuccess) return hip_fail(e, "ctf_create: hipGetDeviceProperties");
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(CTF_ERR_UNSUPPORTED, "ctf_create: device %d is %s, this library is built for gfx950",
                    device, prop.gcnArchName);
    {
        DeviceScope ds(device);
        if (ds.err != hipSuccess) return hip_fail(ds.err, "ctf_create: set device");
        e = noalloc_scratch_init(device);
        if (e != hipSuccess) return hip_fail(e, "ctf_create: scratch address");
    }
    ctf_context c = new (std::nothrow) ctf_context_s;
    if (!c) return fail(CTF_ERR_OUT_OF_MEMORY, "ctf_create: host allocation");
    c->device = device;
    *out = c;
    return CTF_OK;
}

ctf_status ctf_destroy(ctf_context ctx)
{
    set_error("");
    if (!ctx) return fail(CTF_ERR_INVALID_ARG, "ctf_destroy: NULL context");
    delete ctx;
    return CTF_OK;
}

ctf_status ctf_texture_create(ctf_context ctx, const ctf_texture_desc* d, ctf_texture* out)
{
    set_error("");
    if (!ctx || !d || !out) return fail(CTF_ERR_INVALID_ARG, "ctf_texture_create: NULL argument");
    *out = nullptr;
    if (!pow2(d->width) || !pow2(d->height) || d->width > (1 << 23) || d->height > (1 << 23))
        return fail(CTF_ERR_INVALID_ARG, "ctf_texture_create: width/height %d x %d must be powers of two <= 2^23",
                    d->width, d->height);
    DeviceScope ds(ctx->device);
    if (ds.err != hipSuccess) return hip_fail(ds.err, "ctf_texture_create: set device");

    ctf_texture t = new (std::nothrow) ctf_texture_s;
    if (!t) return fail(CTF_ERR_OUT_OF_MEMORY, "ctf_texture_create: host allocation");
    t->ctx = ctx;
    t->desc = *d;
    DevTexture& T = t->dev;
    std::memset(&T, 0, sizeof T);
    T.kind = d->kind;
    T.width = d->width;
    T.height = d->height;
    T.wmask = (uint32_t)d->width - 1u;
    T.hmask = (uint32_t)d->height - 1u;
    T.inv_w = 1.0f / (float)d->width;

    ctf_status st = CTF_OK;
    switch (d->kind) {
    case CTF_TEX_SINUSOIDS: {
        if (d->width != d->height) { st = fail(CTF_ERR_INVALID_ARG, "sinusoid texture must be square"); break; }
        if (d->n_terms <= 0 || d->n_terms > 4096 || !d->pqj || !d->amp) {
            st = fail(CTF_ERR_INVALID_ARG, "sinusoid texture: n_terms in 1..4096 and pqj/amp required");
            break;
        }
        const int K = d->n_terms;
        // the integer terms, then (W <= 4096) the float terms of the
        // five-instruction form: residues p', q' in [-W/2, W/2), j' in [0, W),
        // each divided by W (exact: W is a power of two)
        const bool float_phase = d->width <= 4096;
        std::vector<int32_t> host((size_t)4 * K * 4 * (float_phase ? 2 : 1));
        const int64_t W = d->width;
        auto centred = [&](int64_t v) {
            int64_t r = ((v % W) + W) % W;
            return r >= W / 2 ? r - W : r;
        };
        for (int i = 0; i < 4 * K; ++i) {
            const int32_t p = d->pqj[3 * i], q = d->pqj[3 * i + 1], j = d->pqj[3 * i + 2];
            if (p <= -(1 << 23) || p >= (1 << 23) || q <= -(1 << 23) || q >= (1 << 23) || j < 0) {
                st = fail(CTF_ERR_INVALID_ARG, "sinusoid term %d: |p|,|q| must be < 2^23 and j >= 0", i);
                break;
            }
            float amp = d->amp[i];
            int32_t bits;
            std::memcpy(&bits, &amp, 4);
            host[4 * i + 0] = p;
            host[4 * i + 1] = q;
            host[4 * i + 2] = j;
            host[4 * i + 3] = bits;
            if (float_phase) {
                const float f[4] = {(float)centred(p) / (float)W, (float)centred(q) / (float)W,
                                    (float)(((int64_t)j) % W) / (float)W, amp};
                std::memcpy(&host[(size_t)4 * 4 * K + 4 * i], f, 16);
            }
        }
        if (st != CTF_OK) break;
        hipError_t e = hipMalloc(&t->terms, host.size() * 4);
        if (e == hipSuccess) e = hipMemcpy(t->terms, host.data(), host.size() * 4, hipMemcpyHostToDevice);
        if (e != hipSuccess) { st = hip_fail(e, "ctf_texture_create: terms"); break; }
        T.n_terms = K;
        T.terms = reinterpret_cast<const int4*>(t->terms);
        T.fterms = float_phase ? reinterpret_cast<const float4*>(t->terms) + (size_t)4 * K : nullptr;
        break;
    }
    case CTF_TEX_AFFINE:
        std::memcpy(T.affine, d->affine, sizeof T.affine);
        break;
    case CTF_TEX_CONSTANT:
        std::memcpy(T.constant, d->constant, sizeof T.constant);
        break;
    case CTF_TEX_TABLE: {
        if (!d->table) { st = fail(CTF_ERR_INVALID_ARG, "table texture: table is NULL"); break; }
        const size_t bytes = (size_t)d->width * d->height * 16;
        hipError_t e = hipMalloc(&t->table, bytes);
        if (e == hipSuccess) e = hipMemcpy(t->table, d->table, bytes, hipMemcpyHostToDevice);
        if (e != hipSuccess) { st = hip_fail(e, "ctf_texture_create: table"); break; }
        T.table = reinterpret_cast<const float4*>(t->table);
        break;
    }
    case CTF_TEX_DECODER:
        if (!d->decoder) { st = fail(CTF_ERR_INVALID_ARG, "decoder texture: decoder is NULL"); break; }
        if (d->precision != CTF_FP16 && d->precision != CTF_BF16) {
            st = fail(CTF_ERR_INVALID_ARG, "decoder texture: precision must be CTF_FP16 or CTF_BF16");
            break;
        }
        st = ctf_internal_decoder_texture(t);
        break;
    default:
        st = fail(CTF_ERR_INVALID_ARG, "ctf_texture_create: unknown kind %d", d->kind);
    }
    if (st != CTF_OK) {
        std::string keep = g_error;
        ctf_texture_destroy(t);
        set_error(keep);
        return st;
    }
    *out = t;
    return CTF_OK;
}

ctf_status ctf_texture_destroy(ctf_texture t)
{
    if (!t) return fail(CTF_ERR_INVALID_ARG, "ctf_texture_destroy: NULL texture");
    DeviceScope ds(t->ctx->device);
    if (t->terms) (void)hipFree(t->terms);
    if (t->table) (void)hipFree(t->table);
    if (t->dec_buf) (void)hipFree(t->dec_buf);
    delete t;
    set_error("");
    return CTF_OK;
}

ctf_status ctf_texture_eval(ctf_texture t, const int32_t* xy, int64_t n, float* rgba, void* stream)
{
    set_error("");
    if (!t || n < 0 || (n > 0 && (!xy || !rgba)))
        return fail(CTF_ERR_INVALID_ARG, "ctf_texture_eval: bad arguments");
    DeviceScope ds(t->ctx->device);
    if (ds.err != hipSuccess) return hip_fail(ds.err, "ctf_texture_eval: set device");
    hipError_t e;
    if (t->dev.kind == CTF_TEX_DECODER)
        e = ctf_internal_decoder_eval(t, xy, n, rgba, (hipStream_t)stream);
    else
        e = launch_texel_eval_simt(t->dev, xy, n, rgba, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "ctf_texture_eval: launch");
    return CTF_OK;
}

static ctf_status check_method(const ctf_method* m, const char* who)
{
    if (m->kind < CTF_BILINEAR4 || m->kind > CTF_MASK)
        return fail(CTF_ERR_INVALID_ARG, "%s: unknown method %d", who, m->kind);
    if (m->max_evals_per_lane < 1 || m->max_evals_per_lane > 4)
        return fail(CTF_ERR_INVALID_ARG, "%s: max_evals_per_lane %d not in 1..4", who, m->max_evals_per_lane);
    if (m->kind == CTF_MASK && m->mask_side != 16)
        return fail(CTF_ERR_UNSUPPORTED, "%s: mask_side %d (16 is built)", who, m->mask_side);
    if (m->box_w < 0 || m->box_h < 0) return fail(CTF_ERR_INVALID_ARG, "%s: negative box budget", who);
    if (m->fallback < CTF_FB_STF1 || m->fallback > CTF_FB_CPLUS)
        return fail(CTF_ERR_INVALID_ARG, "%s: unknown fallback %d", who, m->fallback);
    if (m->filter < CTF_FILTER_BILINEAR || m->filter > CTF_FILTER_CATMULL_ROM)
        return fail(CTF_ERR_INVALID_ARG, "%s: unknown filter %d", who, m->filter);
    if (m->split != CTF_SPLIT_AUTO && m->split != CTF_SPLIT_OFF)
        return fail(CTF_ERR_INVALID_ARG, "%s: unknown split mode %d", who, m->split);
    if (m->wave_shape != CTF_WAVE_8X8 && m->wave_shape != CTF_WAVE_8X4)
        return fail(CTF_ERR_INVALID_ARG, "%s: unknown wave shape %d", who, m->wave_shape);
    return CTF_OK;
}

static FilterArgs filter_args(const float* uv, const float* duv, int32_t sw, int32_t sh, const ctf_method* m,
                              uint64_t seed, float* out, ctf_tile_stats* ts, ctf_frame_stats* fs, int32_t* lists,
                              int32_t* stf)
{
    FilterArgs a;
    a.uv = uv;
    a.duv = duv;
    a.out = out;
    a.sw = sw;
    a.sh = sh;
    const int tile_h = m->wave_shape == CTF_WAVE_8X4 ? 4 : kTile;
    a.tiles_x = (sw + kTile - 1) / kTile;
    a.ntiles = (int64_t)a.tiles_x * ((sh + tile_h - 1) / tile_h);
    a.method = m->kind;
    a.box_w = m->box_w;
    a.box_h = m->box_h;
    a.max_evals = m->max_evals_per_lane;
    a.fallback = m->fallback;
    a.filter = m->filter;
    a.split = m->split;
    a.wave_shape = m->wave_shape;
    a.seed = seed;
    a.layer = 0;
    a.tile_stats = ts;
    a.frame_stats = fs;
    a.lists = lists;
    a.stf_xy = stf;
    return a;
}

ctf_status ctf_filter_layers(ctf_context ctx, const float* uv, const float* uv_derivs, int32_t sw, int32_t sh,
                             int32_t n_layers, const ctf_texture* texs, const float* xforms,
                             const ctf_method* m, uint64_t seed, float* out, ctf_tile_stats* tile_stats,
                             ctf_frame_stats* frame_stats, int32_t* debug_stf, void* stream)
{
    set_error("");
    if (!ctx || !uv || !uv_derivs || !texs || !xforms || !m || !out)
        return fail(CTF_ERR_INVALID_ARG, "ctf_filter_layers: NULL argument");
    if (sw <= 0 || sh <= 0 || sw > kMaxScreenSide || sh > kMaxScreenSide)
        return fail(CTF_ERR_INVALID_ARG, "ctf_filter_layers: screen %d x %d (sides 1..2^24)", sw, sh);
    if (n_layers < 1 || n_layers > 8) return fail(CTF_ERR_INVALID_ARG, "ctf_filter_layers: n_layers %d", n_layers);
    ctf_status st = check_method(m, "ctf_filter_layers");
    if (st != CTF_OK) return st;
    if (m->wave_shape != CTF_WAVE_8X8)
        return fail(CTF_ERR_UNSUPPORTED, "ctf_filter_layers: the layered launch takes 8x8 waves only");
    for (int l = 0; l < n_layers; ++l) {
        if (!texs[l] || texs[l]->ctx != ctx) return fail(CTF_ERR_INVALID_ARG, "ctf_filter_layers: texture %d", l);
        if (texs[l]->dev.kind != CTF_TEX_DECODER || texs[l]->dec.precision != texs[0]->dec.precision)
            return fail(CTF_ERR_UNSUPPORTED, "ctf_filter_layers: layer %d is not a decoder texture of the common precision", l);
        for (int k = 0; k < 4; ++k)
            if (!std::isfinite(xforms[4 * l + k])) return fail(CTF_ERR_INVALID_ARG, "ctf_filter_layers: xform %d", l);
    }
    DeviceScope ds(ctx->device);
    if (ds.err != hipSuccess) return hip_fail(ds.err, "ctf_filter_layers: set device");
    const FilterArgs a = filter_args(uv, uv_derivs, sw, sh, m, seed, out, tile_stats, frame_stats, nullptr, debug_stf);
    const hipError_t e = ctf_internal_filter_layers(texs, xforms, n_layers, a, (hipStream_t)stream);
    if (e == hipErrorInvalidValue) return fail(CTF_ERR_UNSUPPORTED, "ctf_filter_layers: combination not built");
    if (e != hipSuccess) return hip_fail(e, "ctf_filter_layers: launch");
    return CTF_OK;
}

ctf_status ctf_filter(ctf_context ctx, const float* uv, const float* uv_derivs, int32_t sw,
                      int32_t sh, ctf_texture tex, const ctf_method* m, uint64_t seed, float* out,
                      ctf_tile_stats* tile_stats, ctf_frame_stats* frame_stats,
                      int32_t* debug_lists, int32_t* debug_stf, void* stream)
{
    set_error("");
    if (!ctx || !uv || !uv_derivs || !tex || !m || !out)
        return fail(CTF_ERR_INVALID_ARG, "ctf_filter: NULL argument");
    if (sw <= 0 || sh <= 0 || sw > kMaxScreenSide || sh > kMaxScreenSide)
        return fail(CTF_ERR_INVALID_ARG, "ctf_filter: screen %d x %d (sides 1..2^24)", sw, sh);
    ctf_status st = check_method(m, "ctf_filter");
    if (st != CTF_OK) return st;
    if (tex->ctx != ctx) return fail(CTF_ERR_INVALID_ARG, "ctf_filter: texture from another context");
    DeviceScope ds(ctx->device);
    if (ds.err != hipSuccess) return hip_fail(ds.err, "ctf_filter: set device");

    const FilterArgs a = filter_args(uv, uv_derivs, sw, sh, m, seed, out, tile_stats, frame_stats, debug_lists,
                                     debug_stf);
    hipError_t e;
    if (m->wave_shape == CTF_WAVE_8X4 && tex->dev.kind == CTF_TEX_DECODER)
        return fail(CTF_ERR_UNSUPPORTED, "ctf_filter: 8x4 waves take the procedural and table producers");
    if (tex->dev.kind == CTF_TEX_DECODER)
        e = ctf_internal_decoder_filter(tex, a, (hipStream_t)stream);
    else if (m->wave_shape == CTF_WAVE_8X4)
        e = launch_filter_w32(a, tex->dev, (hipStream_t)stream);
    else
        e = launch_filter_simt(a, tex->dev, (hipStream_t)stream);
    if (e == hipErrorInvalidValue) return fail(CTF_ERR_UNSUPPORTED, "ctf_filter: combination not built");
    if (e != hipSuccess) return hip_fail(e, "ctf_filter: launch");
    return CTF_OK;
}

}  // extern "C"
