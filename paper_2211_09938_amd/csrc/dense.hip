// Dense complex products with Toeplitz fringe panels on the MFMA kernel of the
// forward pass: the Fresnel back-propagation used by the differentiable form
// (numerical reconstruction, Sec. 2 last paragraph, with the Fresnel kernel)
// and its adjoint.
//
// With K[m][q] = k(m - q) (symmetric, k from the level-0 fringe table) and
// K' = conj(K) for the back-propagation, K' = K for its adjoint:
//     U = s * K'_y . H . K'_x
// as two NT products (operands K-contiguous, padded with zeros to 16):
//     step 1:  T[p][y] = sum_x K'_x[p][x] * H[y][x]       A = K'_x panel, B = H panel
//     step 2:  U[q][p] = sum_y s K'_y[q][y] * T[p][y]     A = s K'_y panel, B = T panel
// Both run split-K into FP32 partials; step 1's partials are summed straight
// into the operand planes of T.
#include "nt.h"
#include "split.h"

namespace cgh {

namespace {

inline int grid_1d(size_t n) {
    const size_t b = (n + 255) / 256;
    return (int)(b < 4096 ? (b > 0 ? b : 1) : 4096);
}

// out[r][c] = scale * k'(r - c) for c < cols, zero for cols <= c < ld (K-blocked panel).
// table: re part then im part, each lut_len(n_tab) floats, entry m + n_tab.
template <int P>
__global__ __launch_bounds__(256) void toeplitz_panel_kernel(const float* __restrict__ table,
                                                             int n_tab, int rows, int cols, int ld,
                                                             float scale, float im_sign,
                                                             void* __restrict__ out, size_t ps) {
    const size_t total = (size_t)rows * ld;
    const int len = lut_len(n_tab);
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (size_t)gridDim.x * blockDim.x) {
        int r, c;
        kblk_pos(e, rows, r, c);
        float re = 0.f, im = 0.f;
        if (c < cols) {
            const int idx = r - c + n_tab;
            re = scale * table[idx];
            im = im_sign * scale * table[len + idx];
        }
        put_c<P>(out, ps, e, re, im);
    }
}

// Interleaved complex64 [rows][cols] -> K-blocked operand planes [rows][ld], zero pad.
// absmax (FP16 range scaling, else null): values scaled by 2^-e, e the exponent of
// the input's largest component magnitude.
template <int P>
__global__ __launch_bounds__(256) void complex_panel_kernel(const float2* __restrict__ in,
                                                            int rows, int cols, int ld,
                                                            const unsigned long long* absmax,
                                                            void* __restrict__ out, size_t ps) {
    const size_t total = (size_t)rows * ld;
    const float sc = absmax ? pow2f(-range_exp(absmax_value(absmax))) : 1.f;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (size_t)gridDim.x * blockDim.x) {
        int r, c;
        kblk_pos(e, rows, r, c);
        const float2 v = c < cols ? in[(size_t)r * cols + c] : make_float2(0.f, 0.f);
        put_c<P>(out, ps, e, v.x * sc, v.y * sc);
    }
}

// Real image [rows][cols] -> K-blocked operand planes [rows][ld] (zeros for
// cols <= k < ld).
// absmax as for complex_panel_kernel.
template <int P>
__global__ __launch_bounds__(256) void real_panel_kernel(const float* __restrict__ in, int rows,
                                                         int cols, int ld,
                                                         const unsigned long long* absmax,
                                                         void* __restrict__ out, size_t ps) {
    const size_t total = (size_t)rows * ld;
    const float sc = absmax ? pow2f(-range_exp(absmax_value(absmax))) : 1.f;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (size_t)gridDim.x * blockDim.x) {
        int r, c;
        kblk_pos(e, rows, r, c);
        put_r<P>(out, ps, e, c < cols ? in[(size_t)r * cols + c] * sc : 0.f);
    }
}

// Sum of `split` FP32 partials [split][rows][cols] -> K-blocked operand planes [rows][ld].
// scale: multiplies the sums (a power of two: FP16 range scaling, else 1).
template <int P>
__global__ __launch_bounds__(256) void reduce_panel_kernel(const float2* __restrict__ partial,
                                                           int split, int rows, int cols, int ld,
                                                           float scale, void* __restrict__ out,
                                                           size_t ps) {
    const size_t total = (size_t)rows * ld, plane = (size_t)rows * cols;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (size_t)gridDim.x * blockDim.x) {
        int r, c;
        kblk_pos(e, rows, r, c);
        float re = 0.f, im = 0.f;
        if (c < cols) {
            const size_t i = (size_t)r * cols + c;
            for (int s = 0; s < split; ++s) {
                const float2 v = partial[(size_t)s * plane + i];
                re += v.x;
                im += v.y;
            }
        }
        put_c<P>(out, ps, e, re * scale, im * scale);
    }
}

// Writes one problem and its tile count where the contraction kernel reads them.
// With a max-abs word the problem's output scale becomes
// base * 2^(exponent of the word's value + shift) (FP16 range scaling).
__global__ void dense_entry_kernel(NtEntry e, int tiles, NtEntry* __restrict__ dst,
                                   int* __restrict__ count, const unsigned long long* absmax,
                                   int shift, float base) {
    if (threadIdx.x == 0) {
        if (absmax) e.out_scale = base * pow2f(range_exp(absmax_value(absmax)) + shift);
        *dst = e;
        *count = tiles;
    }
}

// FP16 range scaling: the field panel is scaled to [1, 2) times its largest
// component (|H'| < 2 sqrt 2), the step-1 product T = K'_x H' (|T| < 2 sqrt 2 nx)
// by 2^-t into its panel, and the 1 / (ny nx) factor moves from the K'_y panel
// (where it would fall below FP16's normal range) into step 2's epilogue, which
// multiplies by 2^(e + t) / (ny nx).
template <int P>
hipError_t dense_backprop(const DenseBuffers& b, const float* lut0_x, const float* lut0_y,
                          const float2* in, float2* out, int ny, int nx, int adjoint, float scale,
                          int split, hipStream_t s) {
    constexpr bool F16 = P == P_FP16;
    const int ldx = pad_kt(nx), ldy = pad_kt(ny);
    const float im_sign = adjoint ? 1.f : -1.f;
    const size_t kx_ps = (size_t)nx * ldx, ky_ps = (size_t)ny * ldy;
    const size_t h_ps = (size_t)ny * ldx, t_ps = (size_t)nx * ldy;
    const int t = F16 ? headroom_shift(3.f * (float)nx) : 0;
    hipError_t e = hipSuccess;
    if (F16) e = launch_absmax(reinterpret_cast<const float*>(in), 2 * (size_t)ny * nx, b.absmax, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(toeplitz_panel_kernel<P>, dim3(grid_1d(kx_ps)), dim3(256), 0, s, lut0_x,
                       nx, nx, nx, ldx, 1.f, im_sign, b.kx, kx_ps);
    hipLaunchKernelGGL(toeplitz_panel_kernel<P>, dim3(grid_1d(ky_ps)), dim3(256), 0, s, lut0_y,
                       ny, ny, ny, ldy, F16 ? 1.f : scale, im_sign, b.ky, ky_ps);
    hipLaunchKernelGGL(complex_panel_kernel<P>, dim3(grid_1d(h_ps)), dim3(256), 0, s, in, ny, nx,
                       ldx, F16 ? b.absmax : nullptr, b.h, h_ps);
    e = hipGetLastError();
    if (e != hipSuccess) return e;

    const int tn = nt_table_tile_n(kEpiComplex, P);
    const int tiles1 = nt_tiles(nx, ny, kNtTile, tn), tiles2 = nt_tiles(ny, nx, kNtTile, tn);
    NtEntry e1{};
    e1.a = b.kx;
    e1.b = b.h;
    e1.out = split > 1 ? b.partial : b.c1;
    e1.partial = b.partial;
    e1.a_ps = (long long)kx_ps;
    e1.b_ps = (long long)h_ps;
    e1.M = nx;
    e1.N = ny;
    e1.K = ldx;
    e1.lda = nx * 16;  // K'_x panel: nx rows
    e1.ldb = ny * 16;  // H panel: ny rows
    e1.out_ld = ny;
    e1.tiles_n = (ny + tn - 1) / tn;
    e1.tile_m = kNtTile;
    e1.tile_n = tn;
    e1.out_scale = 1.f;
    hipLaunchKernelGGL(dense_entry_kernel, dim3(1), dim3(64), 0, s, e1, tiles1, b.entries,
                       b.counts, nullptr, 0, 1.f);
    if ((e = launch_nt_table(kEpiComplex, P, b.entries, 1, b.counts, tiles1, split, s)) != hipSuccess) return e;
    hipLaunchKernelGGL(reduce_panel_kernel<P>, dim3(grid_1d(t_ps)), dim3(256), 0, s,
                       split > 1 ? b.partial : b.c1, split, nx, ny, ldy, pow2f(-t), b.t, t_ps);

    NtEntry e2{};
    e2.a = b.ky;
    e2.b = b.t;
    e2.out = out;
    e2.partial = b.partial;
    e2.a_ps = (long long)ky_ps;
    e2.b_ps = (long long)t_ps;
    e2.M = ny;
    e2.N = nx;
    e2.K = ldy;
    e2.lda = ny * 16;  // s K'_y panel: ny rows
    e2.ldb = nx * 16;  // T panel: nx rows
    e2.out_ld = nx;
    e2.tiles_n = (nx + tn - 1) / tn;
    e2.tile_m = kNtTile;
    e2.tile_n = tn;
    e2.out_scale = 1.f;
    hipLaunchKernelGGL(dense_entry_kernel, dim3(1), dim3(64), 0, s, e2, tiles2, b.entries + 1,
                       b.counts + 1, F16 ? b.absmax : nullptr, t, scale);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = launch_nt_table(kEpiComplex, P, b.entries + 1, 1, b.counts + 1, tiles2, split, s)) != hipSuccess)
        return e;
    return launch_reduce_partial(ny, nx, split, b.partial, out, 0, s);
}

// One layer of the dense form: H (+)= K_y A K_x^T for the real image A, with
// K_x[x][p] = g_x(x - p) and K_y[y][q] = g_y(y - q) from the level-0 tables
// (the layer's prefactor is in g_y).  Step 1 T[x][q] = sum_p A[q][p] K_x[x][p]
// (real x complex, written transposed as a K-blocked panel); step 2
// H[y][x] = sum_q K_y[y][q] T[x][q].
// FP16 range scaling: the reconstruction (|recon| <= (1 + 3L) max |object| <= 10 max
// |object| for the averaging Haar pair with details masked) is scaled by 2^-e, e the
// exponent of max |object| (absmax), so |A'| < 20; T = A' K_x^T (|T| < 20 nx) by
// 2^-t; step 2's epilogue multiplies by 2^(e + t + e_fringe).
template <int P>
hipError_t fused_layer(const float* recon, const float* lut0_x, const float* lut0_y, int ny,
                       int nx, int accumulate, float2* out, char* scratch, NtEntry* entries,
                       int* counts, const unsigned long long* absmax, int e_fringe,
                       hipStream_t s) {
    constexpr bool F16 = P == P_FP16;
    const int ts = F16 ? headroom_shift(20.f * (float)nx) : 0;
    auto al = [](size_t v) { return (v + 255) / 256 * 256; };
    const int ldx = pad_kt(nx), ldy = pad_kt(ny);
    const size_t kx_ps = (size_t)nx * ldx, ky_ps = (size_t)ny * ldy;
    const size_t a_ps = (size_t)ny * ldx, t_ps = (size_t)nx * ldy;
    char* kx = scratch;
    char* ky = kx + al(8 * kx_ps);
    char* a = ky + al(8 * ky_ps);
    char* t = a + al(4 * a_ps);
    hipLaunchKernelGGL(toeplitz_panel_kernel<P>, dim3(grid_1d(kx_ps)), dim3(256), 0, s, lut0_x,
                       nx, nx, nx, ldx, 1.f, 1.f, kx, kx_ps);
    hipLaunchKernelGGL(toeplitz_panel_kernel<P>, dim3(grid_1d(ky_ps)), dim3(256), 0, s, lut0_y,
                       ny, ny, ny, ldy, 1.f, 1.f, ky, ky_ps);
    hipLaunchKernelGGL(real_panel_kernel<P>, dim3(grid_1d(a_ps)), dim3(256), 0, s, recon, ny, nx,
                       ldx, F16 ? absmax : nullptr, a, a_ps);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;

    const int tiles1 = nt_tiles(ny, nx, kNtTile, kNtTile);
    NtEntry e1{};
    e1.a = a;
    e1.b = kx;
    e1.out = t;
    e1.a_ps = (long long)a_ps;
    e1.b_ps = (long long)kx_ps;
    e1.out_ps = (long long)t_ps;
    e1.M = ny;
    e1.N = nx;
    e1.K = ldx;
    e1.lda = ny * 16;     // A panel: ny rows
    e1.ldb = nx * 16;     // K_x panel: nx rows
    e1.out_ld = nx * 16;  // T panel: nx rows
    e1.tiles_n = (nx + kNtTile - 1) / kNtTile;
    e1.tile_m = e1.tile_n = kNtTile;
    e1.out_scale = pow2f(-ts);
    hipLaunchKernelGGL(dense_entry_kernel, dim3(1), dim3(64), 0, s, e1, tiles1, entries, counts,
                       nullptr, 0, 1.f);
    if ((e = launch_nt_first_table(P, entries, 1, counts, tiles1, s)) != hipSuccess) return e;

    const int tn = nt_table_tile_n(kEpiComplex, P);
    const int tiles2 = nt_tiles(ny, nx, kNtTile, tn);
    NtEntry e2{};
    e2.a = ky;
    e2.b = t;
    e2.out = out;
    e2.a_ps = (long long)ky_ps;
    e2.b_ps = (long long)t_ps;
    e2.M = ny;
    e2.N = nx;
    e2.K = ldy;
    e2.lda = ny * 16;  // K_y panel: ny rows
    e2.ldb = nx * 16;  // T panel: nx rows
    e2.out_ld = nx;
    e2.tiles_n = (nx + tn - 1) / tn;
    e2.tile_m = kNtTile;
    e2.tile_n = tn;
    e2.accumulate = accumulate;
    e2.out_scale = 1.f;
    hipLaunchKernelGGL(dense_entry_kernel, dim3(1), dim3(64), 0, s, e2, tiles2, entries + 1,
                       counts + 1, F16 ? absmax : nullptr, ts + e_fringe, 1.f);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    return launch_nt_table(kEpiComplex, P, entries + 1, 1, counts + 1, tiles2, 1, s);
}

}  // namespace

size_t dense_bytes(int ny, int nx, int split) {
    const size_t ldx = pad_kt(nx), ldy = pad_kt(ny);
    const size_t panels = 8 * ((size_t)nx * ldx + (size_t)ny * ldy + (size_t)ny * ldx +
                               (size_t)nx * ldy);
    return panels + 4 * 256 + (split > 1 ? 0 : 8 * (size_t)ny * nx);
}

DenseBuffers dense_buffers(char* base, int ny, int nx, int split, float2* partial,
                           NtEntry* entries, int* counts, unsigned long long* absmax) {
    auto al = [](size_t v) { return (v + 255) / 256 * 256; };
    const size_t ldx = pad_kt(nx), ldy = pad_kt(ny);
    DenseBuffers b{};
    size_t off = 0;
    b.kx = base + off;
    off += al(8 * (size_t)nx * ldx);
    b.ky = base + off;
    off += al(8 * (size_t)ny * ldy);
    b.h = base + off;
    off += al(8 * (size_t)ny * ldx);
    b.t = base + off;
    off += al(8 * (size_t)nx * ldy);
    b.c1 = split > 1 ? nullptr : reinterpret_cast<float2*>(base + off);
    b.partial = partial;
    b.entries = entries;
    b.counts = counts;
    b.absmax = absmax;
    return b;
}

hipError_t launch_dense_backprop(const DenseBuffers& b, const float* lut0_x, const float* lut0_y,
                                 const float2* in, float2* out, int ny, int nx, int adjoint,
                                 float scale, int precision, int split, hipStream_t s) {
    if (precision == P_BF16)
        return dense_backprop<P_BF16>(b, lut0_x, lut0_y, in, out, ny, nx, adjoint, scale, split, s);
    if (precision == P_FP16)
        return dense_backprop<P_FP16>(b, lut0_x, lut0_y, in, out, ny, nx, adjoint, scale, split, s);
    return dense_backprop<P_FP32>(b, lut0_x, lut0_y, in, out, ny, nx, adjoint, scale, split, s);
}

size_t fused_recon_offset(int ny, int nx) {
    auto al = [](size_t v) { return (v + 255) / 256 * 256; };
    const size_t ldx = pad_kt(nx), ldy = pad_kt(ny);
    return al(8 * (size_t)nx * ldx) + al(8 * (size_t)ny * ldy) + al(4 * (size_t)ny * ldx) +
           al(8 * (size_t)nx * ldy);
}

size_t fused_bytes(int ny, int nx) {
    return fused_recon_offset(ny, nx) + (4 * (size_t)ny * nx + 255) / 256 * 256;
}

hipError_t launch_fused_layer(const float* recon, const float* lut0_x, const float* lut0_y,
                              int ny, int nx, int precision, int accumulate, float2* out,
                              char* scratch, NtEntry* entries, int* counts,
                              const unsigned long long* absmax, int e_fringe, hipStream_t s) {
    if (precision == P_BF16)
        return fused_layer<P_BF16>(recon, lut0_x, lut0_y, ny, nx, accumulate, out, scratch,
                                   entries, counts, absmax, e_fringe, s);
    if (precision == P_FP16)
        return fused_layer<P_FP16>(recon, lut0_x, lut0_y, ny, nx, accumulate, out, scratch,
                                   entries, counts, absmax, e_fringe, s);
    return fused_layer<P_FP32>(recon, lut0_x, lut0_y, ny, nx, accumulate, out, scratch, entries,
                               counts, absmax, e_fringe, s);
}

}  // namespace cgh
