// Eq. 1 with the exact distance: the evaluation kernel that measures the
// error of the Fresnel form used by the hot path.
//
//   H[y][x] += exp(i 2 pi frac(z / lambda)) *
//              sum_{q,p} A[q][p] / r * exp(i 2 pi (r - z) / lambda),
//   r = sqrt(pitch^2 ((x - p)^2 + (y - q)^2) + z^2)
//
// for one layer at distance z, A its masked reconstruction.  The phase in
// cycles is split as
//   (r - z) / lambda = m^2 c - rho^4 / (2 z lambda (r + z)^2),
//   m^2 = (x - p)^2 + (y - q)^2 (exact integer), c = pitch^2 / (2 lambda z),
// an identity (r - z = rho^2 / (r + z)).  The first term, up to thousands of
// cycles, is reduced exactly: m^2 c in FP64, fractional part in FP64.  The
// second is small (below 70 cycles for 2048^2 at 8 um and z = 0.1 m) and is
// taken in FP32 with the FP32 distance.  sin/cos of the reduced phase and the
// 1/r amplitude are FP32; each thread sums one point tile (kExactTile points)
// in FP32 and the tiles in FP64.  One thread per hologram pixel, one wave per
// workgroup (many resident workgroups per CU even for small holograms), the
// object points streamed through LDS; VALU-bound.
#include "common.h"

namespace cgh {

namespace {

constexpr int kExactTile = 64;

__global__ __launch_bounds__(kExactTile) void exact_kernel(const float* __restrict__ amp, int ny, int nx,
                                                    double c, float z, float p2, float k4,
                                                    float pre_re, float pre_im, int accumulate,
                                                    float2* __restrict__ out) {
    __shared__ float s_a[kExactTile];
    __shared__ int s_q[kExactTile], s_p[kExactTile];
    const int tid = threadIdx.x;
    const long long n = (long long)ny * nx;
    const long long pix = (long long)blockIdx.x * kExactTile + tid;
    const int y = pix < n ? (int)(pix / nx) : 0;
    const int x = pix < n ? (int)(pix - (long long)y * nx) : 0;
    const float z2 = z * z;
    double acc_re = 0.0, acc_im = 0.0;
    for (long long base = 0; base < n; base += kExactTile) {
        const long long i = base + tid;
        const int qi = i < n ? (int)(i / nx) : 0;
        s_a[tid] = i < n ? amp[i] : 0.f;
        s_q[tid] = qi;
        s_p[tid] = i < n ? (int)(i - (long long)qi * nx) : 0;
        __syncthreads();
        float tre = 0.f, tim = 0.f;
        for (int j = 0; j < kExactTile; ++j) {
            const float a = s_a[j];
            if (a == 0.f) continue;  // the same point for every lane
            const int dy = y - s_q[j], dx = x - s_p[j];
            const int m2 = dx * dx + dy * dy;
            const double cyc = (double)m2 * c;
            const float main = (float)(cyc - floor(cyc));
            const float rho2 = (float)m2 * p2;
            const float r2 = z2 + rho2;
            const float ir = rsqrtf(r2);  // 1/r
            const float rz = r2 * ir + z;
            const float ph = main - __fdividef(k4 * rho2 * rho2, rz * rz);
            float sn, cs;
            sincospif(2.f * ph, &sn, &cs);
            const float w = a * ir;
            tre += w * cs;
            tim += w * sn;
        }
        acc_re += tre;
        acc_im += tim;
        __syncthreads();
    }
    if (pix >= n) return;
    float2 v = make_float2((float)(acc_re * pre_re - acc_im * pre_im),
                           (float)(acc_re * pre_im + acc_im * pre_re));
    if (accumulate) {
        const float2 o = out[pix];
        v.x += o.x;
        v.y += o.y;
    }
    out[pix] = v;
}

}  // namespace

hipError_t launch_exact(const float* amp, int ny, int nx, double lambda, double pitch, double z,
                        int accumulate, float2* out, hipStream_t s) {
    const long long n = (long long)ny * nx;
    const double c = pitch * pitch / (2.0 * lambda * z);
    const double fz = z / lambda - floor(z / lambda);
    const double pr = cos(2.0 * M_PI * fz), pi = sin(2.0 * M_PI * fz);
    const float k4 = (float)(1.0 / (2.0 * z * lambda));
    hipLaunchKernelGGL(exact_kernel, dim3((unsigned)((n + kExactTile - 1) / kExactTile)),
                       dim3(kExactTile), 0, s, amp, ny,
                       nx, c, (float)z, (float)(pitch * pitch), k4, (float)pr, (float)pi,
                       accumulate, out);
    return hipGetLastError();
}

}  // namespace cgh
