// Angular-spectrum propagation of a complex field; with z -> -z it is the
// inverse method the paper reconstructs its holograms with (Sec. 2):
//
//   out = IDFT2( DFT2(field) * T ),  T = exp(i 2 pi z sqrt(1/lambda^2 - fx^2 - fy^2)),
//
// fx = kx / (nx pitch), kx in [-nx/2, nx/2) in DFT order (likewise fy), T = 0
// for the evanescent components.  Five passes, each FFT one whole row held in
// LDS by one workgroup:
//   1. DFT along x of every row                   field -> out
//   2. transpose, 64 x 64 tiles through LDS      out [ny][nx] -> tmp [nx][ny]
//   3. per frequency column kx (a row of tmp): DFT along y, times T, inverse DFT
//   4. transpose                                 tmp -> out
//   5. inverse DFT along x of every row, scaled by 1 / (ny nx)
// FFT: Stockham autosort (results in natural order, no bit reversal): a
// radix-3 stage for lengths 3 * 2^a, radix-8 stages, then one radix-4 or
// radix-2 stage for the rest of the power of two (2048 = 8^3 * 4: four
// stages).  A stage reads the R inputs of each of its butterflies into
// registers, synchronises, and writes the R outputs back in place.
// Twiddles exp(-2 pi i m / n) come from a table computed with FP64 sincospi of
// the exact rational 2m/n and rounded to FP32.
// The transfer phase reaches 2 pi z / lambda (about 2.4e6 rad at 0.2 m), so in
// half-cycles it is split exactly as
//   2 (z/lambda) sqrt(1 - s) = 2 z/lambda - 2 (z/lambda) s / (1 + sqrt(1 - s)),
//   s = lambda^2 (fx^2 + fy^2),
// the constant reduced modulo 2 on the host in FP64, the rest evaluated and
// reduced in FP64 per frequency, FP64 sincospi of the reduced value.
#include <cmath>

#include "common.h"

namespace cgh {

namespace {

constexpr int kFftThreads = 256;
constexpr int kFftMax = 4096;

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// DFT of R points in registers (forward: exp(-2 pi i q q' / R); INV: conjugate).
template <int R, bool INV>
__device__ __forceinline__ void butterfly(float2* x) {
    if constexpr (R == 8) {
        // two 4-point DFTs (even and odd inputs), odd outputs times w8^k
        float2 e[4] = {x[0], x[2], x[4], x[6]}, o[4] = {x[1], x[3], x[5], x[7]};
        butterfly<4, INV>(e);
        butterfly<4, INV>(o);
        const float c = 0.70710678118654752440f;  // 1 / sqrt(2)
        const float2 o1 = o[1], o2 = o[2], o3 = o[3];
        // forward w8 = (1 - i) / sqrt(2); inverse its conjugate
        o[1] = INV ? make_float2(c * (o1.x - o1.y), c * (o1.x + o1.y))
                   : make_float2(c * (o1.x + o1.y), c * (o1.y - o1.x));
        o[2] = INV ? make_float2(-o2.y, o2.x) : make_float2(o2.y, -o2.x);
        o[3] = INV ? make_float2(-c * (o3.x + o3.y), c * (o3.x - o3.y))
                   : make_float2(c * (o3.y - o3.x), -c * (o3.x + o3.y));
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            x[k] = make_float2(e[k].x + o[k].x, e[k].y + o[k].y);
            x[k + 4] = make_float2(e[k].x - o[k].x, e[k].y - o[k].y);
        }
    } else if constexpr (R == 2) {
        const float2 a = x[0], b = x[1];
        x[0] = make_float2(a.x + b.x, a.y + b.y);
        x[1] = make_float2(a.x - b.x, a.y - b.y);
    } else if constexpr (R == 4) {
        const float2 t0 = make_float2(x[0].x + x[2].x, x[0].y + x[2].y);
        const float2 t1 = make_float2(x[0].x - x[2].x, x[0].y - x[2].y);
        const float2 t2 = make_float2(x[1].x + x[3].x, x[1].y + x[3].y);
        const float2 t3 = make_float2(x[1].x - x[3].x, x[1].y - x[3].y);
        // -i t3 (forward) or +i t3 (inverse)
        const float2 r3 = INV ? make_float2(-t3.y, t3.x) : make_float2(t3.y, -t3.x);
        x[0] = make_float2(t0.x + t2.x, t0.y + t2.y);
        x[2] = make_float2(t0.x - t2.x, t0.y - t2.y);
        x[1] = make_float2(t1.x + r3.x, t1.y + r3.y);
        x[3] = make_float2(t1.x - r3.x, t1.y - r3.y);
    } else {
        static_assert(R == 3, "radix 2, 3, 4 or 8");
        const float h = 0.86602540378443864676f;  // sqrt(3) / 2
        const float2 t = make_float2(x[1].x + x[2].x, x[1].y + x[2].y);
        const float2 u = make_float2(x[1].x - x[2].x, x[1].y - x[2].y);
        const float2 m = make_float2(x[0].x - 0.5f * t.x, x[0].y - 0.5f * t.y);
        // -i h u (forward) or +i h u (inverse)
        const float2 r = INV ? make_float2(-h * u.y, h * u.x) : make_float2(h * u.y, -h * u.x);
        x[0] = make_float2(x[0].x + t.x, x[0].y + t.y);
        x[1] = make_float2(m.x + r.x, m.y + r.y);
        x[2] = make_float2(m.x - r.x, m.y - r.y);
    }
}

// One Stockham stage of radix R on the n points in buf, after sub-transforms
// of length p: butterfly i (k = i mod p) takes buf[i + q n/R], q < R, scaled
// by w^(q k n/(p R)), and writes output q to buf[(i - k) R + k + q p].
template <int R, bool INV>
__device__ __forceinline__ void fft_stage(float2* buf, int n, int p, const float2* __restrict__ tw) {
    // butterflies per thread: n / R for the longest n of the radix (3 * 2^a <= 3072)
    constexpr int MB = (R == 3 ? 1024 : kFftMax / R) / kFftThreads;
    const int nb = n / R;
    const int step = n / (p * R);
    float2 v[MB][R];
#pragma unroll
    for (int b = 0; b < MB; ++b) {
        const int i = threadIdx.x + b * kFftThreads;
        if (i < nb) {
#pragma unroll
            for (int q = 0; q < R; ++q) v[b][q] = buf[i + q * nb];
        }
    }
    __syncthreads();
#pragma unroll
    for (int b = 0; b < MB; ++b) {
        const int i = threadIdx.x + b * kFftThreads;
        if (i < nb) {
            const int k = i % p;
#pragma unroll
            for (int q = 1; q < R; ++q) {
                float2 w = tw[q * k * step];
                if (INV) w.y = -w.y;
                v[b][q] = cmul(v[b][q], w);
            }
            butterfly<R, INV>(v[b]);
            const int j = (i - k) * R + k;
#pragma unroll
            for (int q = 0; q < R; ++q) buf[j + q * p] = v[b][q];
        }
    }
    __syncthreads();
}

// In-place DFT of the n points in LDS (n = 2^a or 3 * 2^a, 2 <= n <= 4096).
template <bool INV>
__device__ void fft_lds(float2* buf, int n, const float2* __restrict__ tw) {
    int p = 1;
    if (n % 3 == 0) {
        fft_stage<3, INV>(buf, n, p, tw);
        p *= 3;
    }
    while ((n / p) % 8 == 0) {
        fft_stage<8, INV>(buf, n, p, tw);
        p *= 8;
    }
    if (n / p == 4) fft_stage<4, INV>(buf, n, p, tw);
    else if (n / p == 2) fft_stage<2, INV>(buf, n, p, tw);
}

__global__ __launch_bounds__(256) void twiddle_kernel(float2* __restrict__ tw_x, int nx,
                                                      float2* __restrict__ tw_y, int ny) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    double sn, cs;
    if (i < nx) {
        sincospi(-2.0 * (double)i / (double)nx, &sn, &cs);
        tw_x[i] = make_float2((float)cs, (float)sn);
    }
    if (i < ny) {
        sincospi(-2.0 * (double)i / (double)ny, &sn, &cs);
        tw_y[i] = make_float2((float)cs, (float)sn);
    }
}

// Row r of in [rows][n] -> its DFT (INV: inverse, unnormalised) times scale,
// into row r of out (in and out may be the same array).
template <bool INV>
__global__ __launch_bounds__(kFftThreads) void fft_rows_kernel(const float2* in, float2* out, int n,
                                                               const float2* __restrict__ tw,
                                                               float scale) {
    __shared__ float2 buf[kFftMax];
    const size_t base = (size_t)blockIdx.x * n;
    for (int i = threadIdx.x; i < n; i += kFftThreads) buf[i] = in[base + i];
    __syncthreads();
    fft_lds<INV>(buf, n, tw);
    for (int i = threadIdx.x; i < n; i += kFftThreads) {
        const float2 v = buf[i];
        out[base + i] = make_float2(v.x * scale, v.y * scale);
    }
}

// Frequency column kx = row of data [nx][ny] (already transformed along x):
// DFT along y, multiply by the transfer T(kx, ky), inverse DFT along y.
__global__ __launch_bounds__(kFftThreads) void transfer_columns_kernel(
    float2* __restrict__ data, int nx, int ny, const float2* __restrict__ tw_y, double lam2,
    double fx_unit, double fy_unit, double zl, double c0) {
    __shared__ float2 buf[kFftMax];
    const int kx = blockIdx.x;
    float2* row = data + (size_t)kx * ny;
    for (int i = threadIdx.x; i < ny; i += kFftThreads) buf[i] = row[i];
    __syncthreads();
    fft_lds<false>(buf, ny, tw_y);
    const double fx = (double)(kx < (nx + 1) / 2 ? kx : kx - nx) * fx_unit;
    for (int ky = threadIdx.x; ky < ny; ky += kFftThreads) {
        const double fy = (double)(ky < (ny + 1) / 2 ? ky : ky - ny) * fy_unit;
        const double s = lam2 * (fx * fx + fy * fy);
        float2 t = make_float2(0.f, 0.f);
        if (s <= 1.0) {  // propagating
            double hc = c0 - 2.0 * zl * s / (1.0 + sqrt(1.0 - s));  // phase / pi
            hc -= 2.0 * floor(0.5 * hc);
            double sn, cs;
            sincospi(hc, &sn, &cs);
            t = make_float2((float)cs, (float)sn);
        }
        buf[ky] = cmul(buf[ky], t);
    }
    __syncthreads();
    fft_lds<true>(buf, ny, tw_y);
    for (int i = threadIdx.x; i < ny; i += kFftThreads) row[i] = buf[i];
}

// out[c][r] = in[r][c] for in [rows][cols]; 64 x 64 tiles, 256 threads.
__global__ __launch_bounds__(256) void transpose_kernel(const float2* __restrict__ in,
                                                        float2* __restrict__ out, int rows,
                                                        int cols) {
    __shared__ float2 t[64][65];
    const int c0 = blockIdx.x * 64, r0 = blockIdx.y * 64;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    for (int r = ty; r < 64; r += 4) {
        const int rr = r0 + r, cc = c0 + tx;
        if (rr < rows && cc < cols) t[r][tx] = in[(size_t)rr * cols + cc];
    }
    __syncthreads();
    for (int c = ty; c < 64; c += 4) {
        const int cc = c0 + c, rr = r0 + tx;
        if (cc < cols && rr < rows) out[(size_t)cc * rows + rr] = t[tx][c];
    }
}

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

}  // namespace

bool angular_length_ok(int n) {
    if (n < 2 || n > kFftMax) return false;
    if (n % 3 == 0) n /= 3;
    return (n & (n - 1)) == 0;
}

size_t angular_bytes(int ny, int nx) {
    return align256((size_t)ny * nx * sizeof(float2)) + align256((size_t)nx * sizeof(float2)) +
           align256((size_t)ny * sizeof(float2));
}

hipError_t launch_angular(const float2* field, int ny, int nx, double lambda, double pitch,
                          double z, float2* out, char* ws, hipStream_t s) {
    if (!angular_length_ok(ny) || !angular_length_ok(nx)) return hipErrorInvalidValue;
    float2* tmp = reinterpret_cast<float2*>(ws);
    float2* tw_x = reinterpret_cast<float2*>(ws + align256((size_t)ny * nx * sizeof(float2)));
    float2* tw_y = reinterpret_cast<float2*>(reinterpret_cast<char*>(tw_x) +
                                             align256((size_t)nx * sizeof(float2)));
    const int nmax = nx > ny ? nx : ny;
    hipLaunchKernelGGL(twiddle_kernel, dim3((nmax + 255) / 256), dim3(256), 0, s, tw_x, nx, tw_y,
                       ny);
    hipLaunchKernelGGL(fft_rows_kernel<false>, dim3(ny), dim3(kFftThreads), 0, s, field, out, nx,
                       tw_x, 1.0f);
    hipLaunchKernelGGL(transpose_kernel, dim3((nx + 63) / 64, (ny + 63) / 64), dim3(256), 0, s,
                       out, tmp, ny, nx);
    const double zl = z / lambda;
    const double c0 = std::fmod(2.0 * zl, 2.0);
    hipLaunchKernelGGL(transfer_columns_kernel, dim3(nx), dim3(kFftThreads), 0, s, tmp, nx, ny,
                       tw_y, lambda * lambda, 1.0 / ((double)nx * pitch),
                       1.0 / ((double)ny * pitch), zl, c0);
    hipLaunchKernelGGL(transpose_kernel, dim3((ny + 63) / 64, (nx + 63) / 64), dim3(256), 0, s,
                       tmp, out, nx, ny);
    hipLaunchKernelGGL(fft_rows_kernel<true>, dim3(ny), dim3(kFftThreads), 0, s, out, out, nx,
                       tw_x, (float)(1.0 / ((double)ny * (double)nx)));
    return hipGetLastError();
}

}  // namespace cgh
