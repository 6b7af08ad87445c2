// Host-side helpers shared by the C ABI translation units (internal):
// argument checks, workspace layout, optics constants.
#pragma once

#include <cmath>
#include <cstring>
#include <mutex>
#include <vector>

#include "../../include/cgh.h"
#include "common.h"
#include "nt.h"

namespace cgh {
namespace host {

constexpr size_t kAlign = 256;  // workspace region alignment (bytes)
constexpr int kOpsWords = 5;    // operator counters [0..3], max-abs word [4]
constexpr int kAbsmaxWord = 4;
inline size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

inline bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

// Maps a HIP error to a status code, remembering it for cgh_last_hip_error().
int hip_status(hipError_t e);

inline int check_shape(int ny, int nx, int levels) {
    if (levels < 1) return CGH_ERROR_SHAPE;
    if (levels > CGH_MAX_LEVELS) return CGH_ERROR_UNSUPPORTED;
    if (ny < 0 || nx < 0 || ny > CGH_MAX_SIDE || nx > CGH_MAX_SIDE) return CGH_ERROR_SHAPE;
    const int b = 1 << levels;
    if (ny % b || nx % b) return CGH_ERROR_SHAPE;
    return CGH_SUCCESS;
}

inline int check_precision(int precision) {
    if (precision < CGH_FP32 || precision > CGH_FP16_SPLIT) return CGH_ERROR_INVALID_VALUE;
    return CGH_SUCCESS;
}

// target: resident workgroups of the launch (two on each of 256 CUs by default)
inline int choose_split(int ny, int nx, int levels, int layers, int tm = cgh::kNtTile,
                        int tn = cgh::kNtTile, int target = 512) {
    const int tiles = ((ny + tm - 1) / tm) * ((nx + tn - 1) / tn);
    int split = (target + tiles - 1) / tiles;
    // keep at least four K tiles per split of the dense K range
    const int kt = (int)(cgh::nt_sizes(ny, nx, layers, levels).kmax / cgh::kKT);
    if (split > kt / 4) split = kt / 4;
    if (split > 16) split = 16;
    if (split < 1) split = 1;
    return split;
}

// What a workspace layout serves:
//   kAll      single-scene calls: split-K partials, and a shared region large
//             enough for every path (forward panels, adjoint, back-propagation,
//             paper-literal and fused forms);
//   kForward  the forward pass only (partials as kAll, forward panels);
//   kBatch    one scene of a batched plan (forward panels, no split-K).
enum class LayoutUse { kAll, kForward, kBatch };

inline cgh::Layout make_layout(int ny, int nx, int layers, int levels,
                               LayoutUse use = LayoutUse::kAll) {
    cgh::Layout lo{};
    const size_t plane = (size_t)ny * nx;
    const int n_dl = layers * levels;
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t at = off; off = align_up(off + bytes); return at; };
    lo.coef = take((size_t)layers * plane * 4);
    lo.lut_x = take((size_t)layers * levels * 4 * cgh::lut_len(nx) * 4);
    lo.lut_y = take((size_t)layers * levels * 4 * cgh::lut_len(ny) * 4);
    lo.lut0 = take((size_t)(2 * cgh::lut_len(nx) + 2 * cgh::lut_len(ny)) * 4);
    // the level tables again in the operand format (8 bytes per entry, both parts, and a
    // zero band)
    lo.gen_x = take((size_t)layers * levels * 3 * cgh::lut_len(nx) * 8);
    lo.gen_y = take((size_t)layers * levels * 3 * cgh::lut_len(ny) * 8);
    lo.t_layer = 0;
    lo.flags_layer = 0;
    for (int l = 1; l <= levels; ++l) {
        lo.t_layer += (size_t)cgh::band_side(ny, l) * nx;
        lo.flags_layer += (size_t)cgh::band_side(ny, l) + cgh::band_side(nx, l);
    }
    const size_t flag_bytes = (size_t)layers * lo.flags_layer;
    // after the flags: four 64-bit operator counters, then the max-abs word of the
    // FP16 range scaling (kOpsWords words, cleared with the flags)
    lo.occ = take((size_t)layers * (size_t)(ny >> levels) * (size_t)(nx >> levels));
    lo.flags = take((flag_bytes + 7) / 8 * 8 + 8 * kOpsWords);
    lo.ops = lo.flags + (flag_bytes + 7) / 8 * 8;
    lo.flags_fill = lo.ops + 8 * kOpsWords - lo.flags;
    const cgh::NtSizes z = cgh::nt_sizes(ny, nx, layers, levels);
    lo.rowlist = take(z.rowlist * 4);
    lo.collist = take(z.collist * 4);
    lo.koff_row = take(cgh::dl_koff_off(ny, levels, layers, 1) * 4);
    lo.koff_col = take(cgh::dl_koff_off(nx, levels, layers, 1) * 4);
    lo.cnt_row = take((size_t)n_dl * 4);
    lo.cnt_col = take((size_t)n_dl * 4);
    lo.seg_row = take((size_t)n_dl * 4);
    lo.orient = take((size_t)n_dl * 4);
    lo.units = take((size_t)(3 * n_dl + 1) * 4);
    lo.tbeg = take((size_t)n_dl * 4);
    lo.hdr = take(sizeof(cgh::PlanHeader));
    lo.entries = take((size_t)(n_dl + 1) * sizeof(cgh::NtEntry));
    lo.entries_n = n_dl + 1;
    lo.first_tiles_max = z.first_tiles_max;
    // forward: the operand panels, 8 bytes per complex element in every precision (a
    // batched plan has no first-contraction fringe panel: its first contraction generates
    // that operand from the tables)
    const size_t fx_b = use == LayoutUse::kBatch ? 0 : align_up(z.fx_plane * 8);
    const size_t cb_b = align_up(z.cb_plane * 4);
    const size_t fy_b = align_up(z.fy_plane * 8), tc_b = align_up(z.tc_plane * 8);
    lo.fwd_bytes = fx_b + cb_b + fy_b + tc_b;
    size_t shared = lo.fwd_bytes;
    lo.split_k = use == LayoutUse::kBatch ? 1 : choose_split(ny, nx, levels, layers);
    if (use == LayoutUse::kAll) {
        // backward / back-propagation intermediate T (complex, >= one plane) and the
        // other paths' scratch share the region
        size_t t_bytes = (size_t)layers * lo.t_layer * 8;
        if (t_bytes < plane * 8) t_bytes = plane * 8;
        const size_t other[5] = {t_bytes, cgh::dense_bytes(ny, nx, lo.split_k),
                                 cgh::backward_bytes(ny, nx, layers, levels),
                                 cgh::literal_bytes(ny, nx, layers, levels),
                                 cgh::fused_bytes(ny, nx)};
        for (size_t v : other)
            if (v > shared) shared = v;
    }
    lo.big = take(shared);
    lo.big_bytes = shared;
    lo.t = lo.big;
    lo.fx = lo.big;
    lo.cb = lo.fx + fx_b;
    lo.fy = lo.cb + cb_b;
    lo.tc = lo.fy + fy_b;
    lo.fx_ps = z.fx_plane;
    lo.cb_ps = z.cb_plane;
    lo.fy_ps = z.fy_plane;
    lo.tc_ps = z.tc_plane;
    lo.partial_bytes = lo.split_k > 1 ? (size_t)lo.split_k * plane * 8 : 0;
    lo.partial = take(lo.partial_bytes);
    lo.total = off;
    return lo;
}

// Launch-time consistency with the layout (a failed check is a library bug and
// is reported as CGH_ERROR_INTERNAL before anything is enqueued): `split`
// partial planes of `plane` complex elements fit the reserved partials, and a
// path's scratch of `bytes` fits the shared region.
inline bool partials_fit(const cgh::Layout& lo, int split, size_t plane) {
    if (split < 1) return false;
    if (split == 1) return true;
    return split <= lo.split_k && (size_t)split * plane * 8 <= lo.partial_bytes;
}
inline bool shared_fits(const cgh::Layout& lo, size_t bytes) { return bytes <= lo.big_bytes; }

// Split of the single-scene second contraction: as many workgroups as can be
// resident with the precision's kernel and tile shape (FP32: two per CU; the split
// forms' kernel: one per CU, 144 KB of LDS), at most the layout's split (128 x 128
// tiles, 512 workgroups), which sized the partial buffer.
inline int second_split(const cgh::Layout& lo, int ny, int nx, int levels, int layers,
                        int precision) {
    const int tm = cgh::nt_second_tile_m(precision), tn = cgh::nt_second_tile_n(precision);
    const int target = precision == CGH_FP32 ? 512 : 256;
    const int split = choose_split(ny, nx, levels, layers, tm, tn, target);
    return split < lo.split_k ? split : lo.split_k;
}

inline cgh::NtBuffers nt_buffers(char* ws, const cgh::Layout& lo) {
    cgh::NtBuffers b{};
    b.rowlist = reinterpret_cast<int*>(ws + lo.rowlist);
    b.collist = reinterpret_cast<int*>(ws + lo.collist);
    b.cnt_row = reinterpret_cast<int*>(ws + lo.cnt_row);
    b.cnt_col = reinterpret_cast<int*>(ws + lo.cnt_col);
    b.seg_row = reinterpret_cast<int*>(ws + lo.seg_row);
    b.orient = reinterpret_cast<int*>(ws + lo.orient);
    b.units = reinterpret_cast<int*>(ws + lo.units);
    b.tbeg = reinterpret_cast<int*>(ws + lo.tbeg);
    b.occ = reinterpret_cast<const uint8_t*>(ws + lo.occ);
    b.hdr = reinterpret_cast<cgh::PlanHeader*>(ws + lo.hdr);
    b.first = reinterpret_cast<cgh::NtEntry*>(ws + lo.entries);
    b.second = b.first + (lo.entries_n - 1);
    b.fx = ws + lo.fx;
    b.cb = ws + lo.cb;
    b.fy = ws + lo.fy;
    b.tc = ws + lo.tc;
    b.fx_ps = lo.fx_ps;
    b.cb_ps = lo.cb_ps;
    b.fy_ps = lo.fy_ps;
    b.tc_ps = lo.tc_ps;
    b.gen_x = ws + lo.gen_x;
    b.gen_y = ws + lo.gen_y;
    b.koff_row = reinterpret_cast<int*>(ws + lo.koff_row);
    b.koff_col = reinterpret_cast<int*>(ws + lo.koff_col);
    return b;
}

struct Optics {
    double c[CGH_MAX_LAYERS];
    double pre_re[CGH_MAX_LAYERS], pre_im[CGH_MAX_LAYERS];
    double one_re[CGH_MAX_LAYERS], one_im[CGH_MAX_LAYERS];
};

inline void make_optics(Optics& o, int layers, const double* z, double lambda, double pitch, bool eq1) {
    for (int d = 0; d < layers; ++d) {
        o.c[d] = pitch * pitch / (2.0 * lambda * z[d]);
        o.one_re[d] = 1.0;
        o.one_im[d] = 0.0;
        if (eq1) {
            // exp(i k z) / z with k z = 2 pi z / lambda, reduced to a fraction of a cycle
            const double cyc = z[d] / lambda;
            const double fr = cyc - std::floor(cyc);
            o.pre_re[d] = std::cos(2.0 * M_PI * fr) / z[d];
            o.pre_im[d] = std::sin(2.0 * M_PI * fr) / z[d];
        } else {
            o.pre_re[d] = 1.0;
            o.pre_im[d] = 0.0;
        }
    }
}

// FP16 split operands: the y fringe tables carry the layer prefactors (magnitude
// 1, or 1/z_d with the Eq. 1 constant).  They are built from prefactors scaled by
// 2^-e, e the exponent of the largest magnitude, so that every table entry stays
// below 2^(levels+1); the last contraction's epilogue multiplies by 2^e.  Other
// precisions: e = 0 and the prefactors unchanged.
struct FringeScale {
    int e = 0;
    double re[CGH_MAX_LAYERS], im[CGH_MAX_LAYERS];
};

inline void fringe_scale(const Optics& op, int layers, int precision, FringeScale& f) {
    double m = 0.0;
    for (int d = 0; d < layers; ++d) m = std::fmax(m, std::hypot(op.pre_re[d], op.pre_im[d]));
    f.e = precision == CGH_FP16_SPLIT ? cgh::range_exp((float)m) : 0;
    for (int d = 0; d < layers; ++d) {
        f.re[d] = std::ldexp(op.pre_re[d], -f.e);
        f.im[d] = std::ldexp(op.pre_im[d], -f.e);
    }
}

inline int check_common(int n_layers, const uint8_t* layer_index, const double* z, const float* thresholds,
                 double lambda, double pitch, int ny, int nx, int levels, int precision,
                 unsigned flags, float* thr_out) {
    int st = check_shape(ny, nx, levels);
    if (st) return st;
    if (n_layers < 1 || n_layers > CGH_MAX_LAYERS) return CGH_ERROR_INVALID_VALUE;
    if (!layer_index && n_layers != 1) return CGH_ERROR_INVALID_VALUE;
    if (!z) return CGH_ERROR_INVALID_VALUE;
    for (int d = 0; d < n_layers; ++d)
        if (!finite_pos(z[d])) return CGH_ERROR_INVALID_VALUE;
    if (!finite_pos(lambda) || !finite_pos(pitch)) return CGH_ERROR_INVALID_VALUE;
    if (flags & ~(unsigned)(CGH_FLAG_ACCUMULATE | CGH_FLAG_EQ1_PREFACTOR)) return CGH_ERROR_INVALID_VALUE;
    for (int l = 0; l < CGH_MAX_LEVELS; ++l) thr_out[l] = 0.5f;
    if (thresholds) {
        for (int l = 0; l < levels; ++l) {
            const float t = thresholds[l];
            if (!(t >= 0.0f && t <= 1.0f)) return CGH_ERROR_INVALID_VALUE;
            thr_out[l] = t;
        }
    } else if (levels == 3) {
        thr_out[0] = 0.9f;
        thr_out[1] = 0.7f;
        thr_out[2] = 0.5f;
    }
    return check_precision(precision);
}

// Per-stage HIP event timing of the forward call (diagnostics).
struct Profiler {
    std::mutex mu;
    bool on = false;
    unsigned mask = ~0u;  // stages that record while on (bit 1 << stage)
    std::vector<hipEvent_t> pool;
    struct Pair { int stage; hipEvent_t a, b; };
    std::vector<Pair> pending;
    double ms[CGH_STAGE_COUNT] = {};
    long long launches[CGH_STAGE_COUNT] = {};

    hipEvent_t take() {
        if (!pool.empty()) { hipEvent_t e = pool.back(); pool.pop_back(); return e; }
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        return e;
    }
};

// The process-wide profiler (defined once, in the ABI translation unit).
Profiler& profiler();

// Records an event pair around one stage when profiling is on.
struct StageTimer {
    hipStream_t s;
    int stage;
    hipEvent_t a = nullptr, b = nullptr;
    StageTimer(hipStream_t st, int stg) : s(st), stage(stg) {
        Profiler& p = profiler();
        std::lock_guard<std::mutex> g(p.mu);
        if (!p.on || !((p.mask >> stage) & 1u)) return;
        a = p.take();
        b = p.take();
        if (a && b && hipEventRecord(a, s) == hipSuccess) return;
        if (a) p.pool.push_back(a);
        if (b) p.pool.push_back(b);
        a = b = nullptr;
    }
    void done() {
        if (!a || !b) return;
        if (hipEventRecord(b, s) != hipSuccess) return;  // destructor returns both to the pool
        Profiler& p = profiler();
        std::lock_guard<std::mutex> g(p.mu);
        p.pending.push_back({stage, a, b});
        a = b = nullptr;
    }
    ~StageTimer() {
        if (a || b) {  // stage failed before done(): give the events back unrecorded
            Profiler& p = profiler();
            std::lock_guard<std::mutex> g(p.mu);
            if (a) p.pool.push_back(a);
            if (b) p.pool.push_back(b);
        }
    }
};

template <class F>
inline hipError_t timed(hipStream_t s, int stage, F&& f) {
    StageTimer t(s, stage);
    hipError_t e = f();
    if (e == hipSuccess) t.done();
    return e;
}


}  // namespace host
}  // namespace cgh
