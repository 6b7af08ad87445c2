// C ABI of libcgh: argument validation, workspace layout and stream-ordered
// dispatch of the kernels.  Every check happens on the host before the first
// HIP call, so an invalid request never enqueues work or touches an output.
#include <cmath>
#include <cstring>
#include <exception>
#include <mutex>
#include <vector>

#include "host.h"

namespace cgh {
namespace host {
Profiler& profiler() {
    static Profiler p;
    return p;
}
thread_local int g_last_hip_error = 0;
int hip_status(hipError_t e) {
    if (e == hipSuccess) return CGH_SUCCESS;
    g_last_hip_error = (int)e;
    return CGH_ERROR_HIP;
}
}  // namespace host
}  // namespace cgh

namespace {

using namespace cgh::host;

// The forward pass fits its layout: the operand panels fit the shared region and
// the second contraction's split-K partials fit the reserved partial holograms.
bool forward_fits(const cgh::Layout& lo, int ny, int nx, int levels, int layers, int precision) {
    return shared_fits(lo, lo.fwd_bytes) &&
           partials_fit(lo, second_split(lo, ny, nx, levels, layers, precision), (size_t)ny * nx);
}

// One forward pass of the hot path into `out` (validated arguments).  parts
// selects the approximation / detail levels (progressive stages); with_luts
// false reuses the fringe tables already in the workspace.
hipError_t forward(const float* object, const uint8_t* layer_index, int n_layers,
                   const float* saliency, const float* thr, const Optics& op, int ny, int nx,
                   int levels, int precision, const cgh::Layout& lo, char* ws, unsigned parts,
                   bool with_luts, int acc, float2* out, hipStream_t s, bool timers = true) {
    // stage timing (event pairs from the profiler's pool) unless the caller
    // must not create anything
    auto timed = [&](hipStream_t st, int stage, auto&& f) -> hipError_t {
        return timers ? cgh::host::timed(st, stage, f) : f();
    };
    uint8_t* fl = reinterpret_cast<uint8_t*>(ws + lo.flags);
    const cgh::NtBuffers nb = nt_buffers(ws, lo);
    const float* coef = reinterpret_cast<const float*>(ws + lo.coef);
    const float* lut_x = reinterpret_cast<const float*>(ws + lo.lut_x);
    const float* lut_y = reinterpret_cast<const float*>(ws + lo.lut_y);
    float2* partial = reinterpret_cast<float2*>(ws + lo.partial);
    const int tn2 = cgh::nt_second_tile_n(precision);
    const int tn1 = cgh::nt_first_tile_n(ny, nx, n_layers, levels, precision);
    const int split = second_split(lo, ny, nx, levels, n_layers, precision);

    FringeScale fs;
    fringe_scale(op, n_layers, precision, fs);
    // The fringe tables do not depend on the object: their launch comes first and also
    // clears the flags and counters that the coefficient stage sets (one launch fewer).
    // Without it a fill clears them.
    hipError_t e = hipSuccess;
    if (with_luts)
        e = timed(s, CGH_STAGE_LUT, [&] {
            return cgh::launch_luts_xy(nx, ny, n_layers, levels, op.c, op.one_re, op.one_im,
                                       reinterpret_cast<float*>(ws + lo.lut_x), fs.re, fs.im,
                                       reinterpret_cast<float*>(ws + lo.lut_y), ws + lo.gen_x,
                                       ws + lo.gen_y, precision, fl, lo.flags_fill, s);
        });
    if (e == hipSuccess)
        e = timed(s, CGH_STAGE_COEF, [&] {
            if (!with_luts) {
                const hipError_t r = cgh::launch_fill_u8(fl, lo.flags_fill, s);
                if (r != hipSuccess) return r;
            }
            // sparse coefficient planes: the panel gather consults the occupancy bytes
            return cgh::launch_dwt_mask(object, layer_index, saliency, ny, nx, n_layers, levels,
                                        thr, parts, reinterpret_cast<float*>(ws + lo.coef), fl,
                                        lo.flags_layer, reinterpret_cast<uint8_t*>(ws + lo.occ),
                                        reinterpret_cast<unsigned long long*>(ws + lo.ops), s);
        });
    if (e == hipSuccess)
        e = timed(s, CGH_STAGE_PLAN, [&] {
            const int tiles[4] = {cgh::nt_first_tile_m(precision), tn1,
                                  cgh::nt_second_tile_m(precision), tn2};
            const cgh::NtOutput o{out, split > 1 ? partial : nullptr, acc};
            hipError_t r = cgh::launch_nt_plan(
                fl, ny, nx, n_layers, levels, lo.flags_layer, precision, tiles, nb, o,
                reinterpret_cast<const unsigned long long*>(ws + lo.ops) + kAbsmaxWord, fs.e, s);
            if (r != hipSuccess) return r;
            return cgh::launch_nt_materialize(coef, lut_x, lut_y, ny, nx, n_layers, levels,
                                              precision, nb, !cgh::nt_first_generates(tn1), s);
        });
    if (e == hipSuccess)
        e = timed(s, CGH_STAGE_FIRST, [&] {
            // workgroups past the planned tile count exit at once: launch the bound for
            // this tile shape, not the layout's bound over every shape
            const long long bound = cgh::nt_first_tiles_bound(
                ny, nx, n_layers, levels, cgh::nt_first_tile_m(precision), tn1);
            const int grid = (int)std::min<long long>(lo.first_tiles_max, bound);
            return cgh::launch_nt_first(n_layers, levels, precision, nb, grid, tn1, s);
        });
    if (e == hipSuccess)
        e = timed(s, CGH_STAGE_SECOND,
                  [&] { return cgh::launch_nt_second(ny, nx, precision, split, nb, s); });
    if (e == hipSuccess && split > 1)
        e = timed(s, CGH_STAGE_REDUCE,
                  [&] { return cgh::launch_reduce_partial(ny, nx, split, partial, out, acc, s); });
    return e;
}

}  // namespace

namespace cgh {
hipError_t noalloc_scratch(void** ptr);  // noalloc.hip
}

extern "C" {

const char* cgh_status_string(int status) {
    switch (status) {
        case CGH_SUCCESS: return "CGH_SUCCESS";
        case CGH_ERROR_INVALID_VALUE: return "CGH_ERROR_INVALID_VALUE: invalid argument value";
        case CGH_ERROR_SHAPE: return "CGH_ERROR_SHAPE: sides must be divisible by 2^levels and within limits";
        case CGH_ERROR_UNSUPPORTED: return "CGH_ERROR_UNSUPPORTED: valid request not implemented by this build";
        case CGH_ERROR_OUT_OF_MEMORY: return "CGH_ERROR_OUT_OF_MEMORY";
        case CGH_ERROR_WORKSPACE: return "CGH_ERROR_WORKSPACE: workspace missing or too small";
        case CGH_ERROR_HIP: return "CGH_ERROR_HIP: HIP runtime or launch failure";
        case CGH_ERROR_INTERNAL: return "CGH_ERROR_INTERNAL: a launch does not fit the library's own workspace layout";
        case CGH_ERROR_SCRATCH_LIMIT: return "CGH_ERROR_SCRATCH_LIMIT: the problem needs more than the allocation-free entry point's static scratch (CGH_NOALLOC_SCRATCH_BYTES)";
        default: return "CGH_ERROR_UNKNOWN";
    }
}

int cgh_last_hip_error(void) { return cgh::host::g_last_hip_error; }

int cgh_version(void) { return 100; }

int cgh_haar_dwt(const float* x, int ny, int nx, int levels, float* coeffs, void* stream) {
    try {
        int st = check_shape(ny, nx, levels);
        if (st) return st;
        if (ny == 0 || nx == 0) return CGH_SUCCESS;
        if (!x || !coeffs || (const void*)x == (const void*)coeffs) return CGH_ERROR_INVALID_VALUE;
        const float thr[3] = {0.f, 0.f, 0.f};
        return hip_status(cgh::launch_dwt_mask(x, nullptr, nullptr, ny, nx, 1, levels, thr,
                                               cgh::kAllParts, coeffs, nullptr, 0, nullptr, nullptr,
                                               (hipStream_t)stream));
    } catch (...) {
        return CGH_ERROR_HIP;
    }
}

int cgh_haar_idwt(const float* coeffs, int ny, int nx, int levels, float* x, void* stream) {
    try {
        int st = check_shape(ny, nx, levels);
        if (st) return st;
        if (ny == 0 || nx == 0) return CGH_SUCCESS;
        if (!x || !coeffs || (const void*)x == (const void*)coeffs) return CGH_ERROR_INVALID_VALUE;
        return hip_status(cgh::launch_idwt(coeffs, ny, nx, levels, x, (hipStream_t)stream));
    } catch (...) {
        return CGH_ERROR_HIP;
    }
}

int cgh_workspace_size(int ny, int nx, int n_layers, int levels, int precision, size_t* bytes) {
    if (!bytes) return CGH_ERROR_INVALID_VALUE;
    int st = check_shape(ny, nx, levels);
    if (st) return st;
    if (n_layers < 1 || n_layers > CGH_MAX_LAYERS) return CGH_ERROR_INVALID_VALUE;
    if (precision < CGH_FP32 || precision > CGH_FP16_SPLIT) return CGH_ERROR_INVALID_VALUE;
    *bytes = (ny == 0 || nx == 0) ? 0 : make_layout(ny, nx, n_layers, levels).total;
    return CGH_SUCCESS;
}

int cgh_workspace_layout(int ny, int nx, int n_layers, int levels, int precision,
                         cgh_layout_info* info) {
    try {
        if (!info) return CGH_ERROR_INVALID_VALUE;
        size_t total = 0;
        int st = cgh_workspace_size(ny, nx, n_layers, levels, precision, &total);
        if (st) return st;
        std::memset(info, 0, sizeof(*info));
        if (ny == 0 || nx == 0) return CGH_SUCCESS;
        const cgh::Layout lo = make_layout(ny, nx, n_layers, levels);
        info->total = lo.total;
        info->shared_bytes = lo.big_bytes;
        info->partial_bytes = lo.partial_bytes;
        info->split_reserved = lo.split_k;
        info->split_second = second_split(lo, ny, nx, levels, n_layers, precision);
        info->forward_bytes = lo.fwd_bytes;
        info->backward_bytes = cgh::backward_bytes(ny, nx, n_layers, levels);
        info->backprop_bytes = cgh::dense_bytes(ny, nx, lo.split_k);
        info->literal_bytes = cgh::literal_bytes(ny, nx, n_layers, levels);
        info->fused_bytes = cgh::fused_bytes(ny, nx);
        info->lut_x_offset = lo.lut_x;
        info->lut_y_offset = lo.lut_y;
        info->gen_x_offset = lo.gen_x;
        info->gen_y_offset = lo.gen_y;
        info->koff_row_offset = lo.koff_row;
        info->koff_col_offset = lo.koff_col;
        return CGH_SUCCESS;
    } catch (...) {
        return CGH_ERROR_HIP;
    }
}

int cgh_progressive_hologram(const float* object, const uint8_t* layer_index, int n_layers,
                             const double* z, const float* saliency, const float* thresholds,
                             double lambda, double pitch, int ny, int nx, int levels,
                             int precision, unsigned flags, void* workspace,
                             size_t workspace_bytes, float* hologram, void* stream) {
    try {
        float thr[CGH_MAX_LEVELS];
        int st = check_common(n_layers, layer_index, z, thresholds, lambda, pitch, ny, nx, levels,
                              precision, flags, thr);
        if (st) return st;
        if (ny == 0 || nx == 0) return CGH_SUCCESS;
        if (!object || !hologram) return CGH_ERROR_INVALID_VALUE;
        const cgh::Layout lo = make_layout(ny, nx, n_layers, levels);
        if (!workspace || workspace_bytes < lo.total) return CGH_ERROR_WORKSPACE;
        if (!forward_fits(lo, ny, nx, levels, n_layers, precision)) return CGH_ERROR_INTERNAL;
        Optics op;
        make_optics(op, n_layers, z, lambda, pitch, (flags & CGH_FLAG_EQ1_PREFACTOR) != 0);
        return hip_status(forward(object, layer_index, n_layers, saliency, thr, op, ny, nx, levels,
                                  precision, lo, static_cast<char*>(workspace), cgh::kAllParts,
                                  true, (flags & CGH_FLAG_ACCUMULATE) ? 1 : 0,
                                  reinterpret_cast<float2*>(hologram), (hipStream_t)stream));
    } catch (...) {
        return CGH_ERROR_HIP;
    }
}

int cgh_progressive_hologram_noalloc(const float* object, const uint8_t* layer_index,
                                     int n_layers, const double* z, const float* saliency,
                                     const float* thresholds, double lambda, double pitch,
                                     int ny, int nx, int levels, int precision, unsigned flags,
                                     float* hologram, void* stream) {
    try {
        float thr[CGH_MAX_LEVELS];
        int st = check_common(n_layers, layer_index, z, thresholds, lambda, pitch, ny, nx, levels,
                              precision, flags, thr);
        if (st) return st;
        if (ny == 0 || nx == 0) return CGH_SUCCESS;
        if (!object || !hologram) return CGH_ERROR_INVALID_VALUE;
        const cgh::Layout lo = make_layout(ny, nx, n_layers, levels, LayoutUse::kForward);
        if (lo.total > CGH_NOALLOC_SCRATCH_BYTES) return CGH_ERROR_SCRATCH_LIMIT;
        if (!forward_fits(lo, ny, nx, levels, n_layers, precision)) return CGH_ERROR_INTERNAL;
        void* ws = nullptr;
        hipError_t e = cgh::noalloc_scratch(&ws);
        if (e != hipSuccess) return hip_status(e);
        Optics op;
        make_optics(op, n_layers, z, lambda, pitch, (flags & CGH_FLAG_EQ1_PREFACTOR) != 0);
        return hip_status(forward(object, layer_index, n_layers, saliency, thr, op, ny, nx, levels,
                                  precision, lo, static_cast<char*>(ws), cgh::kAllParts, true,
                                  (flags & CGH_FLAG_ACCUMULATE) ? 1 : 0,
                                  reinterpret_cast<float2*>(hologram), (hipStream_t)stream,
                                  false));
    } catch (...) {
        return CGH_ERROR_HIP;
    }
}

int cgh_progressive_stages(const float* object, const uint8_t* layer_index, int n_layers,
                           const double* z, const float* saliency, const float* thresholds,
                           double lambda, double pitch, int ny, int nx, int levels, int precision,
                           unsigned flags, void* workspace, size_t workspace_bytes, float* stages,
                           void* stream) {
    try {
        float thr[CGH_MAX_LEVELS];
        int st = check_common(n_layers, layer_index, z, thresholds, lambda, pitch, ny, nx, levels,
                              precision, flags, thr);
        if (st) return st;
        if (flags & CGH_FLAG_ACCUMULATE) return CGH_ERROR_INVALID_VALUE;
        if (ny == 0 || nx == 0) return CGH_SUCCESS;
        if (!object || !stages) return CGH_ERROR_INVALID_VALUE;
        const cgh::Layout lo = make_layout(ny, nx, n_layers, levels);
        if (!workspace || workspace_bytes < lo.total) return CGH_ERROR_WORKSPACE;
        if (!forward_fits(lo, ny, nx, levels, n_layers, precision)) return CGH_ERROR_INTERNAL;
        Optics op;
        make_optics(op, n_layers, z, lambda, pitch, (flags & CGH_FLAG_EQ1_PREFACTOR) != 0);
        hipStream_t s = (hipStream_t)stream;
        char* ws = static_cast<char*>(workspace);
        float2* out = reinterpret_cast<float2*>(stages);
        const size_t plane = (size_t)ny * nx;
        // stage 0: the approximation alone
        hipError_t e = forward(object, layer_index, n_layers, saliency, thr, op, ny, nx, levels,
                               precision, lo, ws, 1u << levels, true, 0, out, s);
        // stage j = stage j-1 + the salient details of level levels-j+1
        for (int j = 1; j <= levels && e == hipSuccess; ++j) {
            e = hipMemcpyAsync(out + j * plane, out + (j - 1) * plane, plane * sizeof(float2),
                               hipMemcpyDeviceToDevice, s);
            if (e == hipSuccess)
                e = forward(object, layer_index, n_layers, saliency, thr, op, ny, nx, levels,
                            precision, lo, ws, 1u << (levels - j), false, 1, out + j * plane, s);
        }
        return hip_status(e);
    } catch (...) {
        return CGH_ERROR_HIP;
    }
}

int cgh_literal_hologram(const float* object, const uint8_t* layer_index, int n_layers,
                         const double* z, const float* saliency, const float* thresholds,
                         double lambda, double pitch, int ny, int nx, int levels, int precision,
                         unsigned flags, void* workspace, size_t workspace_bytes, float* hologram,
                         void* stream) {
    try {
        float thr[CGH_MAX_LEVELS];
        int st = check_common(n_layers, layer_index, z, thresholds, lambda, pitch, ny, nx, levels,
                              precision, flags, thr);
        if (st) return st;
        if (ny == 0 || nx == 0) return CGH_SUCCESS;
        if (!object || !hologram) return CGH_ERROR_INVALID_VALUE;
        const cgh::Layout lo = make_layout(ny, nx, n_layers, levels);
        if (!workspace || workspace_bytes < lo.total) return CGH_ERROR_WORKSPACE;
        if (!partials_fit(lo, lo.split_k, (size_t)ny * nx) ||
            !shared_fits(lo, cgh::literal_bytes(ny, nx, n_layers, levels)))
            return CGH_ERROR_INTERNAL;
        hipStream_t s = (hipStream_t)stream;
        char* ws = static_cast<char*>(workspace);
        Optics op;
        make_optics(op, n_layers, z, lambda, pitch, (flags & CGH_FLAG_EQ1_PREFACTOR) != 0);
        FringeScale fs;
        fringe_scale(op, n_layers, precision, fs);
        uint8_t* fl = reinterpret_cast<uint8_t*>(ws + lo.flags);
        hipError_t e = cgh::launch_fill_u8(fl, lo.flags_fill, s);
        if (e == hipSuccess)
            e = cgh::launch_dwt_mask(object, layer_index, saliency, ny, nx, n_layers, levels, thr,
                                     cgh::kAllParts, reinterpret_cast<float*>(ws + lo.coef), fl,
                                     lo.flags_layer, nullptr,
                                     reinterpret_cast<unsigned long long*>(ws + lo.ops), s);
        if (e == hipSuccess)
            e = cgh::launch_luts_xy(nx, ny, n_layers, levels, op.c, op.one_re, op.one_im,
                                    reinterpret_cast<float*>(ws + lo.lut_x), fs.re, fs.im,
                                    reinterpret_cast<float*>(ws + lo.lut_y), nullptr, nullptr,
                                    0, nullptr, 0, s);
        if (e == hipSuccess) {
            const cgh::LitTables tb{op.c, op.one_re, op.one_im, fs.re, fs.im};
            e = cgh::launch_literal(reinterpret_cast<const float*>(ws + lo.coef),
                                    reinterpret_cast<const float*>(ws + lo.lut_x),
                                    reinterpret_cast<const float*>(ws + lo.lut_y), tb, ny, nx,
                                    n_layers, levels, precision, lo.split_k,
                                    reinterpret_cast<float2*>(ws + lo.partial),
                                    reinterpret_cast<float2*>(hologram),
                                    (flags & CGH_FLAG_ACCUMULATE) ? 1 : 0,
                                    reinterpret_cast<const unsigned long long*>(ws + lo.ops) +
                                        kAbsmaxWord,
                                    fs.e, ws + lo.big, s);
        }
        return hip_status(e);
    } catch (...) {
        return CGH_ERROR_HIP;
    }
}

int cgh_fused_hologram(const float* object, const uint8_t* layer_index, int n_layers,
                       const double* z, const float* saliency, const float* thresholds,
                       double lambda, double pitch, int ny, int nx, int levels, int precision,
                       unsigned flags, void* workspace, size_t workspace_bytes, float* hologram,
                       void* stream) {
    try {
        float thr[CGH_MAX_LEVELS];
        int st = check_common(n_layers, layer_index, z, thresholds, lambda, pitch, ny, nx, levels,
                              precision, flags, thr);
        if (st) return st;
        if (ny == 0 || nx == 0) return CGH_SUCCESS;
        if (!object || !hologram) return CGH_ERROR_INVALID_VALUE;
        const cgh::Layout lo = make_layout(ny, nx, n_layers, levels);
        if (!workspace || workspace_bytes < lo.total) return CGH_ERROR_WORKSPACE;
        if (!shared_fits(lo, cgh::fused_bytes(ny, nx))) return CGH_ERROR_INTERNAL;
        hipStream_t s = (hipStream_t)stream;
        char* ws = static_cast<char*>(workspace);
        Optics op;
        make_optics(op, n_layers, z, lambda, pitch, (flags & CGH_FLAG_EQ1_PREFACTOR) != 0);
        float* coef = reinterpret_cast<float*>(ws + lo.coef);
        // the coefficient stage also records max |object| (FP16 range scaling)
        uint8_t* fl = reinterpret_cast<uint8_t*>(ws + lo.flags);
        auto* ops = reinterpret_cast<unsigned long long*>(ws + lo.ops);
        FringeScale fs;
        fringe_scale(op, n_layers, precision, fs);
        hipError_t e = cgh::launch_fill_u8(fl, lo.flags_fill, s);
        if (e == hipSuccess)
            e = cgh::launch_dwt_mask(object, layer_index, saliency, ny, nx, n_layers, levels, thr,
                                     cgh::kAllParts, coef, fl, lo.flags_layer, nullptr, ops, s);
        char* scratch = ws + lo.big;
        float* recon = reinterpret_cast<float*>(scratch + cgh::fused_recon_offset(ny, nx));
        float* lut0_x = reinterpret_cast<float*>(ws + lo.lut0);
        float* lut0_y = lut0_x + 2 * cgh::lut_len(nx);
        const int acc = (flags & CGH_FLAG_ACCUMULATE) ? 1 : 0;
        // layer by layer: masked reconstruction, level-0 fringe tables, two dense products
        for (int d = 0; d < n_layers && e == hipSuccess; ++d) {
            e = cgh::launch_idwt(coef + (size_t)d * ny * nx, ny, nx, levels, recon, s);
            if (e == hipSuccess)
                e = cgh::launch_luts(nx, 1, 1, 0, &op.c[d], &op.one_re[d], &op.one_im[d], lut0_x,
                                     s);
            if (e == hipSuccess)
                e = cgh::launch_luts(ny, 1, 1, 0, &op.c[d], &fs.re[d], &fs.im[d], lut0_y, s);
            if (e == hipSuccess)
                e = cgh::launch_fused_layer(recon, lut0_x, lut0_y, ny, nx, precision,
                                            (d > 0 || acc) ? 1 : 0,
                                            reinterpret_cast<float2*>(hologram), scratch,
                                            reinterpret_cast<cgh::NtEntry*>(ws + lo.entries),
                                            reinterpret_cast<int*>(ws + lo.hdr),
                                            ops + kAbsmaxWord, fs.e, s);
        }
        return hip_status(e);
    } catch (...) {
        return CGH_ERROR_HIP;
    }
}

int cgh_exact_hologram(const float* object, const uint8_t* layer_index, int n_layers,
                       const double* z, const float* saliency, const float* thresholds,
                       double lambda, double pitch, int ny, int nx, int levels, unsigned flags,
                       void* workspace, size_t workspace_bytes, float* hologram, void* stream) {
    try {
        float thr[CGH_MAX_LEVELS];
        int st = check_common(n_layers, layer_index, z, thresholds, lambda, pitch, ny, nx, levels,
                              CGH_FP32, flags, thr);
        if (st) return st;
        if (flags & CGH_FLAG_EQ1_PREFACTOR) return CGH_ERROR_INVALID_VALUE;  // inherent here
        if (ny == 0 || nx == 0) return CGH_SUCCESS;
        if (!object || !hologram) return CGH_ERROR_INVALID_VALUE;
        const cgh::Layout lo = make_layout(ny, nx, n_layers, levels);
        if (!workspace || workspace_bytes < lo.total) return CGH_ERROR_WORKSPACE;
        if (!shared_fits(lo, (size_t)ny * nx * 4)) return CGH_ERROR_INTERNAL;
        hipStream_t s = (hipStream_t)stream;
        char* ws = static_cast<char*>(workspace);
        uint8_t* fl = reinterpret_cast<uint8_t*>(ws + lo.flags);
        float* coef = reinterpret_cast<float*>(ws + lo.coef);
        float* amp = reinterpret_cast<float*>(ws + lo.big);
        const size_t plane = (size_t)ny * nx;
        hipError_t e = cgh::launch_fill_u8(fl, lo.flags_fill, s);
        if (e == hipSuccess)
            e = cgh::launch_dwt_mask(object, layer_index, saliency, ny, nx, n_layers, levels, thr,
                                     cgh::kAllParts, coef, fl, lo.flags_layer, nullptr,
                                     reinterpret_cast<unsigned long long*>(ws + lo.ops), s);
        const int acc = (flags & CGH_FLAG_ACCUMULATE) ? 1 : 0;
        for (int d = 0; d < n_layers && e == hipSuccess; ++d) {
            e = cgh::launch_idwt(coef + d * plane, ny, nx, levels, amp, s);
            if (e == hipSuccess)
                e = cgh::launch_exact(amp, ny, nx, lambda, pitch, z[d], (d > 0 || acc) ? 1 : 0,
                                      reinterpret_cast<float2*>(hologram), s);
        }
        return hip_status(e);
    } catch (...) {
        return CGH_ERROR_HIP;
    }
}

int cgh_hologram_backward(const float* grad_hologram, const uint8_t* layer_index, int n_layers,
                          const double* z, const float* saliency, const float* thresholds,
                          double lambda, double pitch, int ny, int nx, int levels, int precision,
                          unsigned flags, void* workspace, size_t workspace_bytes,
                          float* grad_object, void* stream) {
    try {
        float thr[CGH_MAX_LEVELS];
        int st = check_common(n_layers, layer_index, z, thresholds, lambda, pitch, ny, nx, levels,
                              precision, flags, thr);
        if (st) return st;
        if (flags & CGH_FLAG_ACCUMULATE) return CGH_ERROR_INVALID_VALUE;
        if (ny == 0 || nx == 0) return CGH_SUCCESS;
        if (!grad_hologram || !grad_object) return CGH_ERROR_INVALID_VALUE;
        const cgh::Layout lo = make_layout(ny, nx, n_layers, levels);
        if (!workspace || workspace_bytes < lo.total) return CGH_ERROR_WORKSPACE;
        if (!shared_fits(lo, cgh::backward_bytes(ny, nx, n_layers, levels)))
            return CGH_ERROR_INTERNAL;

        hipStream_t s = (hipStream_t)stream;
        char* ws = static_cast<char*>(workspace);
        Optics op;
        make_optics(op, n_layers, z, lambda, pitch, (flags & CGH_FLAG_EQ1_PREFACTOR) != 0);
        FringeScale fs;
        fringe_scale(op, n_layers, precision, fs);
        // max-abs word of the cotangent (FP16 range scaling), cleared first
        auto* absmax = reinterpret_cast<unsigned long long*>(ws + lo.ops) + kAbsmaxWord;
        hipError_t e = hipSuccess;
        if (precision == CGH_FP16_SPLIT)
            e = cgh::launch_fill_u8(reinterpret_cast<uint8_t*>(absmax), 8, s);
        if (e == hipSuccess)
            e = cgh::launch_luts_xy(nx, ny, n_layers, levels, op.c, op.one_re, op.one_im,
                                    reinterpret_cast<float*>(ws + lo.lut_x), fs.re, fs.im,
                                    reinterpret_cast<float*>(ws + lo.lut_y), nullptr, nullptr,
                                    0, nullptr, 0, s);
        if (e == hipSuccess)
            e = cgh::launch_backward_nt(reinterpret_cast<const float2*>(grad_hologram),
                                        reinterpret_cast<const float*>(ws + lo.lut_x),
                                        reinterpret_cast<const float*>(ws + lo.lut_y), ny, nx,
                                        n_layers, levels, precision,
                                        reinterpret_cast<float*>(ws + lo.coef), ws + lo.big,
                                        absmax, fs.e, s);
        if (e == hipSuccess)
            e = cgh::launch_grad_synthesis(reinterpret_cast<const float*>(ws + lo.coef), layer_index,
                                           saliency, ny, nx, n_layers, levels, thr, grad_object, s);
        return hip_status(e);
    } catch (...) {
        return CGH_ERROR_HIP;
    }
}

int cgh_fresnel_backpropagate(const float* field_in, int ny, int nx, double lambda, double pitch,
                              double z, int precision, int adjoint, void* workspace,
                              size_t workspace_bytes, float* field_out, void* stream) {
    try {
        int st = check_shape(ny, nx, 1);
        if (st) return st;
        if (!finite_pos(lambda) || !finite_pos(pitch) || !finite_pos(z)) return CGH_ERROR_INVALID_VALUE;
        if ((st = check_precision(precision))) return st;
        if (ny == 0 || nx == 0) return CGH_SUCCESS;
        if (!field_in || !field_out || field_in == field_out) return CGH_ERROR_INVALID_VALUE;
        const cgh::Layout lo = make_layout(ny, nx, 1, 1);
        if (!workspace || workspace_bytes < lo.total) return CGH_ERROR_WORKSPACE;
        if (!partials_fit(lo, lo.split_k, (size_t)ny * nx) ||
            !shared_fits(lo, cgh::dense_bytes(ny, nx, lo.split_k)))
            return CGH_ERROR_INTERNAL;
        hipStream_t s = (hipStream_t)stream;
        char* ws = static_cast<char*>(workspace);
        const double c = pitch * pitch / (2.0 * lambda * z), one = 1.0, zero = 0.0;
        float* lut0_x = reinterpret_cast<float*>(ws + lo.lut0);
        float* lut0_y = lut0_x + 2 * cgh::lut_len(nx);
        // max-abs word of the input field (FP16 range scaling), cleared first
        auto* absmax = reinterpret_cast<unsigned long long*>(ws + lo.ops) + kAbsmaxWord;
        hipError_t e = hipSuccess;
        if (precision == CGH_FP16_SPLIT)
            e = cgh::launch_fill_u8(reinterpret_cast<uint8_t*>(absmax), 8, s);
        if (e == hipSuccess) e = cgh::launch_luts(nx, 1, 1, 0, &c, &one, &zero, lut0_x, s);
        if (e == hipSuccess)
            e = cgh::launch_luts(ny, 1, 1, 0, &c, &one, &zero, lut0_y, s);
        if (e == hipSuccess) {
            const cgh::DenseBuffers b = cgh::dense_buffers(
                ws + lo.big, ny, nx, lo.split_k, reinterpret_cast<float2*>(ws + lo.partial),
                reinterpret_cast<cgh::NtEntry*>(ws + lo.entries), reinterpret_cast<int*>(ws + lo.hdr),
                absmax);
            e = cgh::launch_dense_backprop(b, lut0_x, lut0_y,
                                           reinterpret_cast<const float2*>(field_in),
                                           reinterpret_cast<float2*>(field_out), ny, nx,
                                           adjoint ? 1 : 0,
                                           (float)(1.0 / ((double)ny * (double)nx)), precision,
                                           lo.split_k, s);
        }
        return hip_status(e);
    } catch (...) {
        return CGH_ERROR_HIP;
    }
}

size_t cgh_angular_spectrum_workspace_size(int ny, int nx) {
    if (!cgh::angular_length_ok(ny) || !cgh::angular_length_ok(nx)) return 0;
    return cgh::angular_bytes(ny, nx);
}

int cgh_angular_spectrum(const float* field, int ny, int nx, double lambda, double pitch, double z,
                         void* workspace, size_t workspace_bytes, float* out, void* stream) {
    try {
        if (ny < 0 || nx < 0) return CGH_ERROR_SHAPE;
        if (!finite_pos(lambda) || !finite_pos(pitch) || !std::isfinite(z))
            return CGH_ERROR_INVALID_VALUE;
        if (ny == 0 || nx == 0) return CGH_SUCCESS;
        if (!cgh::angular_length_ok(ny) || !cgh::angular_length_ok(nx)) return CGH_ERROR_SHAPE;
        if (!field || !out) return CGH_ERROR_INVALID_VALUE;
        if (!workspace || workspace_bytes < cgh::angular_bytes(ny, nx)) return CGH_ERROR_WORKSPACE;
        return hip_status(cgh::launch_angular(reinterpret_cast<const float2*>(field), ny, nx,
                                              lambda, pitch, z, reinterpret_cast<float2*>(out),
                                              static_cast<char*>(workspace), (hipStream_t)stream));
    } catch (...) {
        return CGH_ERROR_HIP;
    }
}

int cgh_mfma_peak(int kind, int zero_operands, int blocks, int iters, float* sink, double* flops,
                  void* stream) {
    try {
        if (kind < CGH_PEAK_FP32 || kind > CGH_PEAK_FP16) return CGH_ERROR_INVALID_VALUE;
        if (blocks < 1 || blocks > (1 << 20) || iters < 1 || iters > (1 << 24))
            return CGH_ERROR_INVALID_VALUE;
        if (!sink || !flops) return CGH_ERROR_INVALID_VALUE;
        *flops = cgh::mfma_peak_flops(kind, blocks, iters);
        return hip_status(cgh::launch_mfma_peak(kind, zero_operands ? 1 : 0, blocks, iters, sink,
                                                (hipStream_t)stream));
    } catch (...) {
        return CGH_ERROR_HIP;
    }
}

int cgh_profile_enable(int on) {
    Profiler& p = profiler();
    std::lock_guard<std::mutex> g(p.mu);
    p.on = on != 0;
    return CGH_SUCCESS;
}

int cgh_profile_stages(unsigned mask) {
    Profiler& p = profiler();
    std::lock_guard<std::mutex> g(p.mu);
    p.mask = mask;
    return CGH_SUCCESS;
}

int cgh_profile_read(double* ms, long long* launches, int reset) {
    try {
        Profiler& p = profiler();
        std::lock_guard<std::mutex> g(p.mu);
        int status = CGH_SUCCESS;
        for (auto& pr : p.pending) {
            float t = 0.f;
            hipError_t e = hipEventSynchronize(pr.b);
            if (e == hipSuccess) e = hipEventElapsedTime(&t, pr.a, pr.b);
            if (e != hipSuccess) {
                status = hip_status(e);
            } else {
                p.ms[pr.stage] += t;
                p.launches[pr.stage] += 1;
            }
            p.pool.push_back(pr.a);
            p.pool.push_back(pr.b);
        }
        p.pending.clear();
        for (int k = 0; k < CGH_STAGE_COUNT; ++k) {
            if (ms) ms[k] = p.ms[k];
            if (launches) launches[k] = p.launches[k];
            if (reset) { p.ms[k] = 0.0; p.launches[k] = 0; }
        }
        return status;
    } catch (...) {
        return CGH_ERROR_HIP;
    }
}

int cgh_workspace_stats(const void* workspace, int ny, int nx, int n_layers, int levels,
                        int precision, cgh_stats* stats, void* stream) {
    try {
        int st = check_shape(ny, nx, levels);
        if (st) return st;
        if (!stats || !workspace || n_layers < 1 || n_layers > CGH_MAX_LAYERS) return CGH_ERROR_INVALID_VALUE;
        if ((st = check_precision(precision))) return st;
        std::memset(stats, 0, sizeof(*stats));
        if (ny == 0 || nx == 0) return CGH_SUCCESS;
        const cgh::Layout lo = make_layout(ny, nx, n_layers, levels);
        hipStream_t s = (hipStream_t)stream;
        const char* ws = static_cast<const char*>(workspace);
        const int n_dl = n_layers * levels;
        std::vector<int> cr(n_dl), cc(n_dl), orient(n_dl);
        cgh::PlanHeader hdr{};
        unsigned long long ops[4] = {0, 0, 0, 0};
        hipError_t e = hipMemcpyAsync(cr.data(), ws + lo.cnt_row, n_dl * sizeof(int), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipMemcpyAsync(ops, ws + lo.ops, sizeof(ops), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipMemcpyAsync(cc.data(), ws + lo.cnt_col, n_dl * sizeof(int), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipMemcpyAsync(orient.data(), ws + lo.orient, n_dl * sizeof(int), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipMemcpyAsync(&hdr, ws + lo.hdr, sizeof(hdr), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return hip_status(e);
        double rc = 0.0;
        for (int k = 0; k < n_dl; ++k) rc += (double)cr[k] * (double)cc[k] * (orient[k] ? ny : nx);
        long long total = 0;
        for (int l = 1; l <= levels; ++l) total += cgh::band_side(ny, l);
        total *= n_layers;
        stats->k_active = hdr.k_active;
        stats->k_padded = hdr.kpad;
        stats->k_total = total;
        stats->k_tile = cgh::kKT;
        stats->split_k = second_split(lo, ny, nx, levels, n_layers, precision);
        stats->flops_first = 4.0 * rc;
        stats->flops_second = 8.0 * (double)ny * (double)nx * (double)hdr.k_active;
        stats->flops_second_issued = 8.0 * (double)ny * (double)nx * (double)hdr.kpad;
        stats->operators[0] = (long long)(ny >> levels) * (nx >> levels);
        for (int j = 1; j <= levels; ++j) stats->operators[j] = (long long)ops[levels - j];
        stats->operators_pointwise = (long long)ny * nx;
        return CGH_SUCCESS;
    } catch (...) {
        return CGH_ERROR_HIP;
    }
}

}  // extern "C"
