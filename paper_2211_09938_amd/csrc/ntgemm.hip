// Batched NT complex GEMM on CDNA4 matrix cores for the compacted forward pass.
//
// C[m][n] = sum_k A[m][k] * B[n][k], A real or complex, B complex, both panels
// K-contiguous in the operand precision.  One workgroup computes a 128 x 128
// complex tile with 4 waves (2 x 2, 64 x 64 complex each, 2 x 2 blocks of
// 32 x 32 MFMA).  A device-resident problem table (NtEntry) describes every GEMM
// of a launch; blockIdx.x picks (problem, tile) by binary search over the
// tiles' prefix, and a K split.  Per K tile of 16 each thread moves four
// 16-byte chunks of A and four of B global -> registers -> LDS, the next tile's
// loads in flight during the current tile's MFMAs.
//
//  FP32:  v_mfma_f32_32x32x2f32; a lane's 16-byte LDS read gives it the
//         operands of 4 consecutive MFMAs (lane half g supplies k = 4g + t).
//  split: v_mfma_f32_32x32x16_{bf16,f16}; operands stored as hi and lo planes,
//         each real product as hi*hi + hi*lo + lo*hi, FP32 accumulation.
#include "gemm.h"
#include "nt.h"
#include "split.h"

namespace cgh {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 halfx8 __attribute__((ext_vector_type(8)));

namespace {

constexpr int T = kNtTile;  // 128

template <int P>
struct Fmt {
    static constexpr int ES = (P == P_FP32) ? 4 : 2;        // bytes per element
    static constexpr int PC = (P == P_FP32) ? 2 : 4;        // planes of a complex operand
    static constexpr int PR = (P == P_FP32) ? 1 : 2;        // planes of a real operand
    static constexpr int CPR = kKT * ES / 16;               // 16-byte chunks per row and plane
    static constexpr int PITCH = kKT * ES + 16;             // LDS bytes per row (with padding)
};

__device__ __forceinline__ floatx16 mfma32(float a, float b, floatx16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
}

template <int P>
__device__ __forceinline__ floatx16 mfma16(u32x4 a, u32x4 b, floatx16 c) {
    if constexpr (P == P_BF16)
        return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a),
                                                        __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
    else
        return __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(halfx8, a),
                                                       __builtin_bit_cast(halfx8, b), c, 0, 0, 0);
}

template <int P>
__device__ __forceinline__ floatx16 prod3(floatx16 acc, u32x4 xh, u32x4 xl, u32x4 yh, u32x4 yl) {
    acc = mfma16<P>(xh, yh, acc);
    acc = mfma16<P>(xh, yl, acc);
    acc = mfma16<P>(xl, yh, acc);
    return acc;
}

// Last entry whose tile range starts at or before t (entries with no tiles
// share tile_begin with the next one, so the last such entry owns t).
__device__ __forceinline__ int find_entry(const NtEntry* __restrict__ en, int n, int t) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (en[mid].tile_begin <= t) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Block id -> (K split s, tile t): split-major, block id = s * count + t.
// (Handing each XCD a contiguous range of tiles was measured to be no faster:
// the operand panels stay resident in the 256 MB Infinity Cache.)
__device__ __forceinline__ bool logical_tile(int bid, int count, int split, int& s, int& t) {
    if (bid >= count * split) return false;
    s = bid / count;
    t = bid - s * count;
    return true;
}

// Tile `local` of a problem -> its output origin (row-major over tiles).
__device__ __forceinline__ void tile_origin(const NtEntry& e, int local, int& m0, int& n0) {
    m0 = (local / e.tiles_n) * T;
    n0 = (local % e.tiles_n) * T;
}

// Stage-1 output: T_c[x][seg + r'] in the operand precision (transposed store).
template <int P>
struct FirstEpi {
    void* tc;
    size_t ps;
    const PlanHeader* hdr;
    __device__ void store4(const NtEntry& e, int s, int m, int n, const float* re,
                           const float* im) const {
        (void)s;
        if (m >= pad_kt(e.M) || n >= e.N) return;
        const size_t off = (size_t)n * hdr->kpad + e.out_off + m;
        if constexpr (P == P_FP32) {
            float* b = static_cast<float*>(tc);
            *reinterpret_cast<floatx4*>(b + off) = floatx4{re[0], re[1], re[2], re[3]};
            *reinterpret_cast<floatx4*>(b + ps + off) = floatx4{im[0], im[1], im[2], im[3]};
        } else {
            uint16_t* b = static_cast<uint16_t*>(tc);
            unsigned rh[4], rl[4], ih[4], il[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                uint16_t h, l;
                split16<P>(re[q], h, l);
                rh[q] = h;
                rl[q] = l;
                split16<P>(im[q], h, l);
                ih[q] = h;
                il[q] = l;
            }
            *reinterpret_cast<u32x2*>(b + off) = u32x2{rh[0] | (rh[1] << 16), rh[2] | (rh[3] << 16)};
            *reinterpret_cast<u32x2*>(b + ps + off) = u32x2{rl[0] | (rl[1] << 16), rl[2] | (rl[3] << 16)};
            *reinterpret_cast<u32x2*>(b + 2 * ps + off) = u32x2{ih[0] | (ih[1] << 16), ih[2] | (ih[3] << 16)};
            *reinterpret_cast<u32x2*>(b + 3 * ps + off) = u32x2{il[0] | (il[1] << 16), il[2] | (il[3] << 16)};
        }
    }
};

// Stage-2 output: complex64 hologram (or a split-K partial).
struct SecondEpi {
    float2* out;
    float2* partial;
    int ny, nx, split, accumulate;
    __device__ void store4(const NtEntry&, int s, int m, int n, const float* re,
                           const float* im) const {
        if (n >= nx) return;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int y = m + q;
            if (y >= ny) continue;
            const size_t i = (size_t)y * nx + n;
            float2 v = make_float2(re[q], im[q]);
            if (split == 1) {
                if (accumulate) {
                    const float2 o = out[i];
                    v.x += o.x;
                    v.y += o.y;
                }
                out[i] = v;
            } else {
                partial[(size_t)s * ny * nx + i] = v;
            }
        }
    }
};

template <int P, bool A_CPLX, class Epi>
__global__ __launch_bounds__(256, 2) void nt_kernel(const NtEntry* __restrict__ entries,
                                                    int n_entries,
                                                    const int* __restrict__ tile_count,
                                                    int split, const void* __restrict__ A,
                                                    size_t a_ps, const void* __restrict__ B,
                                                    size_t b_ps, Epi epi) {
    using F = Fmt<P>;
    constexpr int NPA = A_CPLX ? F::PC : F::PR;
    constexpr int NPB = F::PC;
    constexpr int PLANE = T * F::PITCH;
    __shared__ __attribute__((aligned(16))) unsigned char As[NPA * PLANE];
    __shared__ __attribute__((aligned(16))) unsigned char Bs[NPB * PLANE];

    int s, t;
    if (!logical_tile(blockIdx.x, *tile_count, split, s, t)) return;
    const int ei = find_entry(entries, n_entries, t);
    const NtEntry e = entries[ei];
    int m0, n0;
    tile_origin(e, t - e.tile_begin, m0, n0);
    const int chunk = pad_kt((e.K + split - 1) / split);
    const int kb = s * chunk;
    const int ke = min(e.K, kb + chunk);
    const int nk = ke > kb ? (ke - kb) / kKT : 0;

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int wm = (wave >> 1) * 64, wn = (wave & 1) * 64;
    const int l32 = lane & 31, g = lane >> 5;

    floatx16 cr[2][2], ci[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r) { cr[i][j][r] = 0.f; ci[i][j][r] = 0.f; }

    // chunk q -> (plane, row, c); A has NPA * T * CPR chunks, B has NPB * T * CPR.
    constexpr int QA = NPA * T * F::CPR / 256;
    constexpr int QB = NPB * T * F::CPR / 256;
    u32x4 ra[QA], rb[QB];
    const unsigned char* Ab = static_cast<const unsigned char*>(A);
    const unsigned char* Bb = static_cast<const unsigned char*>(B);

    // chunk q of an operand tile -> (plane, row, 16-byte chunk c of the row);
    // neighbouring threads read neighbouring chunks of a row (a row-fastest
    // assignment avoids LDS store conflicts but was measured 20% slower)
    auto decomp = [](int q, int& plane, int& row, int& c) {
        c = q % F::CPR;
        row = (q / F::CPR) % T;
        plane = q / (F::CPR * T);
    };
    auto load = [&](int kt) {
        const int k0 = kb + kt * kKT;
#pragma unroll
        for (int u = 0; u < QA; ++u) {
            int plane, row, c;
            decomp(tid + 256 * u, plane, row, c);
            const int m = m0 + row;
            if (m < e.M) {
                const size_t el = (size_t)plane * a_ps + (size_t)e.a_off + (size_t)m * e.lda + k0;
                ra[u] = *reinterpret_cast<const u32x4*>(Ab + el * F::ES + c * 16);
            } else {
                ra[u] = u32x4{0u, 0u, 0u, 0u};
            }
        }
#pragma unroll
        for (int u = 0; u < QB; ++u) {
            int plane, row, c;
            decomp(tid + 256 * u, plane, row, c);
            const int n = n0 + row;
            if (n < e.N) {
                const size_t el = (size_t)plane * b_ps + (size_t)e.b_off + (size_t)n * e.ldb + k0;
                rb[u] = *reinterpret_cast<const u32x4*>(Bb + el * F::ES + c * 16);
            } else {
                rb[u] = u32x4{0u, 0u, 0u, 0u};
            }
        }
    };
    auto stash = [&]() {
#pragma unroll
        for (int u = 0; u < QA; ++u) {
            int plane, row, c;
            decomp(tid + 256 * u, plane, row, c);
            *reinterpret_cast<u32x4*>(As + plane * PLANE + row * F::PITCH + c * 16) = ra[u];
        }
#pragma unroll
        for (int u = 0; u < QB; ++u) {
            int plane, row, c;
            decomp(tid + 256 * u, plane, row, c);
            *reinterpret_cast<u32x4*>(Bs + plane * PLANE + row * F::PITCH + c * 16) = rb[u];
        }
    };

    if (nk > 0) {
        load(0);
        stash();
    }
    __syncthreads();
    for (int kt = 0; kt < nk; ++kt) {
        if (kt + 1 < nk) load(kt + 1);
        if constexpr (P == P_FP32) {
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                floatx4 fa[2][NPA], fb[2][NPB];
#pragma unroll
                for (int i = 0; i < 2; ++i)
#pragma unroll
                    for (int c = 0; c < NPA; ++c)
                        fa[i][c] = *reinterpret_cast<const floatx4*>(
                            As + c * PLANE + (wm + 32 * i + l32) * F::PITCH + (8 * h + 4 * g) * 4);
#pragma unroll
                for (int j = 0; j < 2; ++j)
#pragma unroll
                    for (int c = 0; c < NPB; ++c)
                        fb[j][c] = *reinterpret_cast<const floatx4*>(
                            Bs + c * PLANE + (wn + 32 * j + l32) * F::PITCH + (8 * h + 4 * g) * 4);
#pragma unroll
                for (int tt = 0; tt < 4; ++tt) {
                    if constexpr (A_CPLX) {
#pragma unroll
                        for (int i = 0; i < 2; ++i)
#pragma unroll
                            for (int j = 0; j < 2; ++j) {
                                cr[i][j] = mfma32(fa[i][0][tt], fb[j][0][tt], cr[i][j]);
                                ci[i][j] = mfma32(fa[i][0][tt], fb[j][1][tt], ci[i][j]);
                            }
#pragma unroll
                        for (int i = 0; i < 2; ++i)
#pragma unroll
                            for (int j = 0; j < 2; ++j) {
                                cr[i][j] = mfma32(-fa[i][1][tt], fb[j][1][tt], cr[i][j]);
                                ci[i][j] = mfma32(fa[i][1][tt], fb[j][0][tt], ci[i][j]);
                            }
                    } else {
#pragma unroll
                        for (int i = 0; i < 2; ++i)
#pragma unroll
                            for (int j = 0; j < 2; ++j) {
                                cr[i][j] = mfma32(fa[i][0][tt], fb[j][0][tt], cr[i][j]);
                                ci[i][j] = mfma32(fa[i][0][tt], fb[j][1][tt], ci[i][j]);
                            }
                    }
                }
            }
        } else {
            u32x4 a[2][NPA], b[2][NPB];
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int c = 0; c < NPA; ++c)
                    a[i][c] = *reinterpret_cast<const u32x4*>(
                        As + c * PLANE + (wm + 32 * i + l32) * F::PITCH + g * 16);
#pragma unroll
            for (int j = 0; j < 2; ++j)
#pragma unroll
                for (int c = 0; c < NPB; ++c)
                    b[j][c] = *reinterpret_cast<const u32x4*>(
                        Bs + c * PLANE + (wn + 32 * j + l32) * F::PITCH + g * 16);
            if constexpr (A_CPLX) {
                u32x4 nah[2], nal[2];  // -A_im: flip the sign bit of every 16-bit half
#pragma unroll
                for (int i = 0; i < 2; ++i) {
                    nah[i] = a[i][2] ^ 0x80008000u;
                    nal[i] = a[i][3] ^ 0x80008000u;
                }
#pragma unroll
                for (int i = 0; i < 2; ++i)
#pragma unroll
                    for (int j = 0; j < 2; ++j) {
                        cr[i][j] = prod3<P>(cr[i][j], a[i][0], a[i][1], b[j][0], b[j][1]);
                        ci[i][j] = prod3<P>(ci[i][j], a[i][0], a[i][1], b[j][2], b[j][3]);
                    }
#pragma unroll
                for (int i = 0; i < 2; ++i)
#pragma unroll
                    for (int j = 0; j < 2; ++j) {
                        cr[i][j] = prod3<P>(cr[i][j], nah[i], nal[i], b[j][2], b[j][3]);
                        ci[i][j] = prod3<P>(ci[i][j], a[i][2], a[i][3], b[j][0], b[j][1]);
                    }
            } else {
#pragma unroll
                for (int i = 0; i < 2; ++i)
#pragma unroll
                    for (int j = 0; j < 2; ++j) {
                        cr[i][j] = prod3<P>(cr[i][j], a[i][0], a[i][1], b[j][0], b[j][1]);
                        ci[i][j] = prod3<P>(ci[i][j], a[i][0], a[i][1], b[j][2], b[j][3]);
                    }
            }
        }
        __syncthreads();
        if (kt + 1 < nk) stash();
        __syncthreads();
    }

#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int qd = 0; qd < 4; ++qd) {
                float re[4], im[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    re[q] = cr[i][j][4 * qd + q];
                    im[q] = ci[i][j][4 * qd + q];
                }
                epi.store4(e, s, m0 + wm + 32 * i + 8 * qd + 4 * g, n0 + wn + 32 * j + l32, re, im);
            }
}

template <int P>
hipError_t first(int ny, int nx, int layers, int levels, const NtBuffers& b, int max_tiles,
                 hipStream_t s) {
    if (max_tiles <= 0) return hipSuccess;
    FirstEpi<P> epi{b.tc, b.tc_ps, b.hdr};
    const int* count = &b.hdr->first_tiles;
    hipLaunchKernelGGL((nt_kernel<P, false, FirstEpi<P>>), dim3(max_tiles), dim3(256), 0, s,
                       b.entries, layers * levels, count, 1, b.cb, b.cb_ps, b.fx, b.fx_ps, epi);
    return hipGetLastError();
}

template <int P>
hipError_t second(int ny, int nx, int layers, int levels, int split, const NtBuffers& b,
                  float2* partial, float2* out, int accumulate, hipStream_t s) {
    SecondEpi epi{out, partial, ny, nx, split, accumulate};
    const int* count = &b.hdr->second_tiles;
    const int tiles = ((ny + T - 1) / T) * ((nx + T - 1) / T);
    hipLaunchKernelGGL((nt_kernel<P, true, SecondEpi>), dim3(tiles * split), dim3(256), 0, s,
                       b.entries + layers * levels, 1, count, split, b.fy, b.fy_ps, b.tc, b.tc_ps,
                       epi);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_nt_first(int ny, int nx, int layers, int levels, int precision,
                           const NtBuffers& b, int max_tiles, hipStream_t s) {
    if (precision == P_BF16) return first<P_BF16>(ny, nx, layers, levels, b, max_tiles, s);
    if (precision == P_FP16) return first<P_FP16>(ny, nx, layers, levels, b, max_tiles, s);
    return first<P_FP32>(ny, nx, layers, levels, b, max_tiles, s);
}

hipError_t launch_nt_second(int ny, int nx, int layers, int levels, int precision, int split,
                            const NtBuffers& b, float2* partial, float2* out, int accumulate,
                            hipStream_t s) {
    if (precision == P_BF16)
        return second<P_BF16>(ny, nx, layers, levels, split, b, partial, out, accumulate, s);
    if (precision == P_FP16)
        return second<P_FP16>(ny, nx, layers, levels, split, b, partial, out, accumulate, s);
    return second<P_FP32>(ny, nx, layers, levels, split, b, partial, out, accumulate, s);
}

}  // namespace cgh
