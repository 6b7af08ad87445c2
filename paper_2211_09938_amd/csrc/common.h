// Internal declarations shared by the libcgh HIP sources (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace cgh {

constexpr int kMaxLevels = 3;

// Operand representation of the contractions (values of cgh_precision).
enum Prec { P_FP32 = 0, P_BF16 = 1, P_FP16 = 2 };
constexpr int kLayerChunk = 64;  // layers per fringe-table launch (kernel-argument budget)

// Side length of the level-l square of Mallat coefficients along one axis
// (l >= 1): both subband halves, 2 * (n >> l).
__host__ __device__ inline int band_side(int n, int l) { return n >> (l - 1); }

// Fringe table of one axis: entry i holds g[m] for m = i - n_pix, i in [0, 2 n_pix).
__host__ __device__ inline int lut_len(int n_pix) { return 2 * n_pix; }

// Table index of (layer d, level l >= 1, band b, part) for `levels` levels.
__host__ __device__ inline size_t lut_table(int d, int l, int band, int part, int levels) {
    return ((size_t)(d * levels + (l - 1)) * 2 + band) * 2 + part;
}

// Operand-format fringe tables (the first contraction generates its fringe operand from
// them): per (layer d, level l >= 1) three bands of lut_len entries of 8 bytes -- band 0,
// band 1 (as the FP32 tables), then zeros; an entry holds both parts, FP32 (re, im) or
// for the split forms the words hi | lo << 16 of re and of im.  Returns the index of
// (d, l)'s band 0 in units of lut_len entries.
__host__ __device__ inline size_t gen_table(int d, int l, int levels) {
    return (size_t)(d * levels + (l - 1)) * 3;
}

// Offsets (in rows of s(l) for T, in bytes for flags) of level l inside one layer.
__host__ __device__ inline size_t t_level_rows(int ny, int l) {
    size_t rows = 0;
    for (int k = 1; k < l; ++k) rows += band_side(ny, k);
    return rows;
}
__host__ __device__ inline size_t flag_level_off(int ny, int nx, int l) {
    size_t off = 0;
    for (int k = 1; k < l; ++k) off += band_side(ny, k) + band_side(nx, k);
    return off;
}

// Range of the FP16 split operands.  FP16 keeps values below 65504 and normal
// above 2^-14, so its panels hold power-of-two scaled values (exact in FP32):
// data panels (coefficients, images, fields, cotangents) are scaled by 2^-e
// with e the exponent of the source's largest magnitude, panels written by a
// first contraction by 2^-t with t from a static bound of their magnitude, and
// the FP32 epilogue of the last contraction multiplies by the inverse of the
// product (a linear map commutes with the scaling, Eq. 3).  BF16 and FP32 keep
// the FP32 exponent range and use scale 1.
constexpr float kF16Ceiling = 32768.f;  // panel magnitudes are kept below 2^15

// e with m in [2^e, 2^(e+1)), clamped to [-100, 100]; 0 for 0, inf and NaN.
__host__ __device__ inline int range_exp(float m) {
    if (!(m > 0.f) || !(m <= 3.402823466e38f)) return 0;
    int e = 0;
    frexpf(m, &e);
    e -= 1;
    return e < -100 ? -100 : (e > 100 ? 100 : e);
}
// Smallest t >= 0 with bound * 2^-t <= kF16Ceiling.
__host__ __device__ inline int headroom_shift(float bound) {
    int t = 0;
    while (bound > kF16Ceiling) {
        bound *= 0.5f;
        ++t;
    }
    return t;
}
__host__ __device__ inline float pow2f(int e) { return ldexpf(1.0f, e); }
// Largest magnitude recorded by a max-abs word (float bits of a nonnegative
// value in the low half of a 64-bit word, raised with atomicMax).
__device__ inline float absmax_value(const unsigned long long* w) {
    return w ? __uint_as_float((unsigned)*w) : 0.f;
}

struct LayerConsts {
    double c[kLayerChunk];       // pitch^2 / (2 lambda z_d): kernel phase in cycles per px^2
    double pre_re[kLayerChunk];  // per-layer complex constant (1, or exp(i k z)/z)
    double pre_im[kLayerChunk];
};

// Byte offsets of every region inside the caller's workspace.
struct Layout {
    size_t coef;                 // masked Mallat coefficients, D * ny * nx floats
    size_t lut_x, lut_y;         // FP32 fringe tables
    size_t lut0;                 // level-0 table pair (x then y) for back-propagation
    size_t gen_x, gen_y;         // level tables in the operand format of the precision
    size_t koff_row, koff_col;   // beside the lists: offsets into the operand-format tables
    size_t flags;                // per layer: rows then cols of every level, bytes
    size_t occ;                  // per layer: one byte per 2^levels block (coefficients written)
    size_t rowlist, collist;     // active row / column indices per (layer, level)
    size_t cnt_row, cnt_col, seg_row, orient, tbeg;  // per (layer, level) counts, k' offsets,
                                                      // contraction order, tile offsets
    size_t units;                                    // panel work-unit table (3 D L + 1 ints)
    size_t hdr, entries;         // device plan header and GEMM problem table
    size_t big;                  // shared region: backward T, or the forward panels
    size_t big_bytes;            // its size
    size_t fwd_bytes;            // forward operand panels at the start of `big`
    size_t partial_bytes;        // size of the split-K partial region
    size_t t;                    // backward / back-propagation intermediate (complex)
    size_t fx, cb, fy, tc;       // forward operand panels (inside `big`)
    size_t fx_ps, cb_ps, fy_ps, tc_ps;  // their plane strides, elements
    size_t partial;              // split-K partial holograms
    size_t total;
    size_t t_layer;              // complex elements of T per layer
    size_t flags_layer;          // flag bytes per layer
    size_t ops;                  // 4 x u64 operator counters and the max-abs word, after the flags
    size_t flags_fill;           // bytes to clear from `flags` (flags and counters)
    int entries_n;               // problems in the table: one per (layer, level), then one
    int first_tiles_max;
    int split_k;
};

struct Launch;  // forward declaration for the host dispatcher

// ------------------------------------------------------------ launchers (host)
hipError_t launch_fill_u8(uint8_t* p, size_t n, hipStream_t s);
// *word = max(*word, bits of max |x[i]|) over n floats (word cleared by the caller).
hipError_t launch_absmax(const float* x, size_t n, unsigned long long* word, hipStream_t s);
// parts: bit l-1 keeps the level-l details, bit `levels` the approximation.
constexpr unsigned kAllParts = 0xFu;
// occ: null (every coefficient plane written in full) or one byte per (layer, block of
// 2^levels x 2^levels pixels), 1 where the layer has a pixel in the block; then only
// those blocks' coefficients are written (the rest are zero and left unwritten).
hipError_t launch_dwt_mask(const float* obj, const uint8_t* layer, const float* sal, int ny, int nx,
                           int layers, int levels, const float* thr, unsigned parts, float* coef,
                           uint8_t* flags, size_t flags_layer, uint8_t* occ,
                           unsigned long long* ops, hipStream_t s);
// One scene of a batched preparation (device-resident tables, batched plans).
struct DwtScene {
    const float* obj;
    const uint8_t* layer;
    const float* sal;
    int ny, nx, layers;
    float* coef;
    uint8_t* flags;
    size_t flags_layer;
    size_t flags_fill;  // bytes of flags and operator counters to clear
    unsigned long long* ops;
    uint8_t* occ;       // (layer, block) occupancy: only occupied blocks' coefficients written
};
// One fringe table set (one axis of one layer of one scene), FP32.
struct LutJob {
    int n_pix, d, levels;
    double c, pre_re, pre_im;
    float* table;  // the scene's table region of that axis
    void* gen;     // its operand-format tables (gen_table), or null
    int gen_prec;  // their precision
};
hipError_t launch_prep_fill(const DwtScene* scenes, int n, size_t max_fill, hipStream_t s);
hipError_t launch_dwt_mask_batch(const DwtScene* scenes, int n, int levels, const float* thr,
                                 int max_nbx, int max_nby, hipStream_t s);
hipError_t launch_luts_batch(const LutJob* jobs, int n_jobs, int max_len, int levels,
                             hipStream_t s);

// out (+)= sum of `split` partial holograms of ny x nx (split <= 1: nothing).
hipError_t launch_reduce_partial(int ny, int nx, int split, const float2* partial, float2* out,
                                 int accumulate, hipStream_t s);
// Angular-spectrum propagation (angular.hip): sides 2^a or 3 * 2^a in [2, 4096];
// workspace angular_bytes(ny, nx); field and out may be the same array.
bool angular_length_ok(int n);
size_t angular_bytes(int ny, int nx);
hipError_t launch_angular(const float2* field, int ny, int nx, double lambda, double pitch,
                          double z, float2* out, char* ws, hipStream_t s);
// Exact-distance Eq. 1 sum of one layer's points `amp` into `out` (exact.hip).
hipError_t launch_exact(const float* amp, int ny, int nx, double lambda, double pitch, double z,
                        int accumulate, float2* out, hipStream_t s);
hipError_t launch_idwt(const float* coef, int ny, int nx, int levels, float* out, hipStream_t s);
hipError_t launch_grad_synthesis(const float* gcoef, const uint8_t* layer, const float* sal, int ny,
                                 int nx, int layers, int levels, const float* thr, float* grad,
                                 hipStream_t s);
hipError_t launch_luts(int n_pix, int layers, int levels, int lmin, const double* c,
                       const double* pre_re, const double* pre_im, float* table, hipStream_t s);
// The level tables of both axes (as two launch_luts calls with lmin 1) in one launch;
// gen_x, gen_y (optional): the same tables in the operand format of precision gen_prec
// (gen_table), zero band included; clear
// (optional, 8-byte aligned, clear_bytes a multiple of 8) is zeroed by the same grid.
hipError_t launch_luts_xy(int nx, int ny, int layers, int levels, const double* c,
                          const double* x_re, const double* x_im, float* table_x,
                          const double* y_re, const double* y_im, float* table_y,
                          void* gen_x, void* gen_y, int gen_prec, uint8_t* clear,
                          size_t clear_bytes, hipStream_t s);
// Matrix-core throughput probe (peak.hip): real flops of a launch, and the launch.
double mfma_peak_flops(int kind, int blocks, int iters);
hipError_t launch_mfma_peak(int kind, int zero, int blocks, int iters, float* sink, hipStream_t s);

}  // namespace cgh
