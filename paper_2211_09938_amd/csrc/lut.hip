// Fringe tables of the block basis functions, one 1D table per axis.
//
// Under the Fresnel form of Eq. 1 the kernel of an integer pixel offset (dy, dx)
// factors as k(dy) k(dx) with k(m) = exp(i pi pitch^2 m^2 / (lambda z)).  The
// hologram of a Haar basis block (Sec. 2: a level-l coefficient spreads over a
// 2^l x 2^l block of points, each with its own fringe) therefore factors into
// 1D sums over the block's columns and rows:
//     lo band:  g_lo[m] = sum_{u <  2^l}     k(m - u)
//     hi band:  g_hi[m] = sum_{u <  2^(l-1)} k(m - u) - sum_{2^(l-1) <= u < 2^l} k(m - u)
// which are the separable rows of the paper's 2^l x 2^l look-up-table blocks.
//
// Phase evaluation: m^2 is formed exactly as a 64-bit integer, the phase in
// cycles is m^2 * c with c = pitch^2 / (2 lambda z) in FP64, its fractional
// part is taken in FP64 and sin/cos come from the HIP device library's FP64
// sincospi.  The sum is rounded once, to FP32 (the panel kernels round to the
// operand precision).
#include "common.h"
#include "split.h"

namespace cgh {

namespace {

// Writes entry idx of table (level lev, band) of layer d (lev 0: the point tables, pair d)
// from its FP64 value.  gen (optional, level tables): the same entry in the operand format
// of precision gen_prec, both parts in one 8-byte word pair -- FP32 (re, im), split forms
// (hi | lo << 16) of re, then of im -- with the zero band after band 1.
__device__ __forceinline__ void lut_store(int len, int d, int levels, int lev, int band, int idx,
                                          double re, double im, float* __restrict__ table,
                                          uint2* __restrict__ gen, int gen_prec) {
    const size_t t_re = (lev == 0) ? (size_t)(d * 2 + 0) : lut_table(d, lev, band, 0, levels);
    const size_t t_im = (lev == 0) ? (size_t)(d * 2 + 1) : lut_table(d, lev, band, 1, levels);
    const float fre = (float)re, fim = (float)im;
    table[t_re * len + idx] = fre;
    table[t_im * len + idx] = fim;
    if (gen && lev != 0) {
        uint2 w;
        if (gen_prec == P_FP32) {
            w = make_uint2(__float_as_uint(fre), __float_as_uint(fim));
        } else {
            uint16_t rh, rl, ih, il;
            if (gen_prec == P_BF16) {
                split16<P_BF16>(fre, rh, rl);
                split16<P_BF16>(fim, ih, il);
            } else {
                split16<P_FP16>(fre, rh, rl);
                split16<P_FP16>(fim, ih, il);
            }
            w = make_uint2(rh | ((unsigned)rl << 16), ih | ((unsigned)il << 16));
        }
        const size_t g = gen_table(d, lev, levels) * len + idx;
        gen[g + (size_t)band * len] = w;
        if (band == 1) gen[g + 2 * (size_t)len] = make_uint2(0u, 0u);  // the zero band
    }
}

// FP64 block sums of entry idx (m = idx - n_pix) at level lev: lo (and, with BOTH, hi)
// from one evaluation of the 2^lev kernel terms, times the layer constant (pre_re, pre_im).
// Zero where the block reaches past the image.
template <bool BOTH>
__device__ __forceinline__ void block_sums(int n_pix, int lev, double c, double pre_re,
                                           double pre_im, int idx, bool hi_only, double (&re)[2],
                                           double (&im)[2]) {
    const int m = idx - n_pix;
    const int bsz = 1 << lev;
    re[0] = re[1] = im[0] = im[1] = 0.0;
    if (m >= -(n_pix - bsz) && m <= n_pix - 1) {
        for (int u = 0; u < bsz; ++u) {
            const long long mm = (long long)(m - u);
            const double cyc_full = (double)(mm * mm) * c;
            const double cyc = cyc_full - floor(cyc_full);
            double s, co;
            sincospi(2.0 * cyc, &s, &co);
            const double sign = u < (bsz >> 1) ? 1.0 : -1.0;
            if (BOTH || !hi_only) {
                re[0] += co;
                im[0] += s;
            }
            if (BOTH || hi_only) {
                re[1] += sign * co;
                im[1] += sign * s;
            }
        }
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            const double r2 = re[b] * pre_re - im[b] * pre_im;
            const double i2 = re[b] * pre_im + im[b] * pre_re;
            re[b] = r2;
            im[b] = i2;
        }
    }
}

// Entry idx of table (level lev(combo), band(combo)) of layer d.
__device__ __forceinline__ void lut_entry(int n_pix, int d, int levels, int lmin, double c,
                                          double pre_re, double pre_im, int idx, int combo,
                                          float* __restrict__ table) {
    const int lev = (lmin == 0) ? 0 : 1 + combo / 2;
    const int band = (lmin == 0) ? 0 : combo % 2;
    double re[2], im[2];
    block_sums<false>(n_pix, lev, c, pre_re, pre_im, idx, band == 1, re, im);
    lut_store(lut_len(n_pix), d, levels, lev, band, idx, re[band], im[band], table, nullptr,
              P_FP32);
}

// Both bands of entry idx of level lev's tables of layer d from one evaluation of the
// kernel terms (the same sums, in the same order, as two lut_entry calls).
__device__ __forceinline__ void lut_entry_bands(int n_pix, int d, int levels, int lev, double c,
                                                double pre_re, double pre_im, int idx,
                                                float* __restrict__ table,
                                                uint2* __restrict__ gen, int gen_prec) {
    double re[2], im[2];
    block_sums<true>(n_pix, lev, c, pre_re, pre_im, idx, false, re, im);
    const int len = lut_len(n_pix);
    lut_store(len, d, levels, lev, 0, idx, re[0], im[0], table, gen, gen_prec);
    lut_store(len, d, levels, lev, 1, idx, re[1], im[1], table, gen, gen_prec);
}

__global__ __launch_bounds__(256) void lut_kernel(int n_pix, int d0, int levels, int lmin,
                                                  LayerConsts lc, float* __restrict__ table) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= lut_len(n_pix)) return;
    const int dl = blockIdx.z;
    lut_entry(n_pix, d0 + dl, levels, lmin, lc.c[dl], lc.pre_re[dl], lc.pre_im[dl], idx,
              blockIdx.y, table);
}

// Both axes' level tables of up to kLayerChunk layers in one launch: grid.z =
// 2 x layer + axis (0: x, 1: y), grid.y = level - 1 (a thread writes both bands); the
// axes share the phase constant and differ in their layer constants and lengths.
struct AxisConsts {
    double c[kLayerChunk];
    double pre_re[2][kLayerChunk];
    double pre_im[2][kLayerChunk];
};

// clear (optional): n8 eight-byte words zeroed by the grid beside the tables (the
// coefficient stage's flags, which it only sets, and which it runs after).
__global__ __launch_bounds__(256) void lut_xy_kernel(int nx, int ny, int d0, int levels,
                                                     AxisConsts ac, float* __restrict__ table_x,
                                                     float* __restrict__ table_y,
                                                     uint2* __restrict__ gen_x,
                                                     uint2* __restrict__ gen_y, int gen_prec,
                                                     uint2* __restrict__ clear, size_t n8) {
    if (clear) {
        const size_t wg = ((size_t)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
        const size_t stride = (size_t)gridDim.x * gridDim.y * gridDim.z * blockDim.x;
        for (size_t i = wg * blockDim.x + threadIdx.x; i < n8; i += stride)
            clear[i] = make_uint2(0u, 0u);
    }
    const int axis = blockIdx.z & 1, dl = blockIdx.z >> 1;
    const int n_pix = axis ? ny : nx;
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= lut_len(n_pix)) return;
    lut_entry_bands(n_pix, d0 + dl, levels, 1 + blockIdx.y, ac.c[dl], ac.pre_re[axis][dl],
                    ac.pre_im[axis][dl], idx, axis ? table_y : table_x, axis ? gen_y : gen_x,
                    gen_prec);
}

// Every (scene, layer, axis) table set of a batch: grid.z = job, grid.y = level - 1.
__global__ __launch_bounds__(256) void lut_batch_kernel(const LutJob* __restrict__ jobs,
                                                        int job0) {
    const LutJob j = jobs[job0 + blockIdx.z];
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= lut_len(j.n_pix)) return;
    lut_entry_bands(j.n_pix, j.d, j.levels, 1 + blockIdx.y, j.c, j.pre_re, j.pre_im, idx, j.table,
                    static_cast<uint2*>(j.gen), j.gen_prec);
}

}  // namespace

hipError_t launch_luts_batch(const LutJob* jobs, int n_jobs, int max_len, int levels,
                             hipStream_t s) {
    for (int j0 = 0; j0 < n_jobs; j0 += 65535) {
        const int nj = n_jobs - j0 < 65535 ? n_jobs - j0 : 65535;
        hipLaunchKernelGGL(lut_batch_kernel, dim3((max_len + 255) / 256, levels, nj),
                           dim3(256), 0, s, jobs, j0);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_luts(int n_pix, int layers, int levels, int lmin, const double* c,
                       const double* pre_re, const double* pre_im, float* table, hipStream_t s) {
    const int len = lut_len(n_pix);
    const int combos = (lmin == 0) ? 1 : 2 * levels;
    for (int d0 = 0; d0 < layers; d0 += kLayerChunk) {
        const int nd = (layers - d0 < kLayerChunk) ? layers - d0 : kLayerChunk;
        LayerConsts lc;
        for (int k = 0; k < kLayerChunk; ++k) {
            const int d = d0 + (k < nd ? k : 0);
            lc.c[k] = c[d];
            lc.pre_re[k] = pre_re[d];
            lc.pre_im[k] = pre_im[d];
        }
        dim3 grid((len + 255) / 256, combos, nd);
        hipLaunchKernelGGL(lut_kernel, grid, dim3(256), 0, s, n_pix, d0, levels, lmin, lc, table);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_luts_xy(int nx, int ny, int layers, int levels, const double* c,
                          const double* x_re, const double* x_im, float* table_x,
                          const double* y_re, const double* y_im, float* table_y,
                          void* gen_x, void* gen_y, int gen_prec, uint8_t* clear,
                          size_t clear_bytes, hipStream_t s) {
    if (clear && ((reinterpret_cast<uintptr_t>(clear) & 7) || (clear_bytes & 7)))
        return hipErrorInvalidValue;
    const int len = lut_len(nx > ny ? nx : ny);
    for (int d0 = 0; d0 < layers; d0 += kLayerChunk) {
        const int nd = (layers - d0 < kLayerChunk) ? layers - d0 : kLayerChunk;
        AxisConsts ac;
        for (int k = 0; k < kLayerChunk; ++k) {
            const int d = d0 + (k < nd ? k : 0);
            ac.c[k] = c[d];
            ac.pre_re[0][k] = x_re[d];
            ac.pre_im[0][k] = x_im[d];
            ac.pre_re[1][k] = y_re[d];
            ac.pre_im[1][k] = y_im[d];
        }
        dim3 grid((len + 255) / 256, levels, 2 * nd);
        uint2* c8 = d0 == 0 ? reinterpret_cast<uint2*>(clear) : nullptr;
        hipLaunchKernelGGL(lut_xy_kernel, grid, dim3(256), 0, s, nx, ny, d0, levels, ac, table_x,
                           table_y, static_cast<uint2*>(gen_x), static_cast<uint2*>(gen_y),
                           gen_prec, c8, c8 ? clear_bytes / 8 : (size_t)0);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace cgh
