// Complex contractions of the adjoint on CDNA4 matrix cores (the forward pass
// uses the compacted kernels of ntgemm.hip, the back-propagation dense.hip).
//
// Per depth layer d and Haar level l the hologram contribution factors as
//     H_{d,l} = Fy_{d,l} * Cb_{d,l} * Fx_{d,l}^T                        (Eq. 3, separable Eq. 1)
// where Cb is the level-l square of Mallat coefficients (its LL quadrant empty
// for l < L) and F[pix, j] = g_band(j)[pix - (j mod n_l) * 2^l] is the
// strided-Toeplitz matrix of the 1D block fringes (lut.hip).  The adjoint is
//     Q_{d,l}  = Fy_{d,l}^H * G,   gC_{d,l} = Re(Q_{d,l} * conj(Fx_{d,l})).
// Fringe operands are never materialised: each K tile gathers its elements of
// the 1D table (a few KB, cache resident) straight into LDS.
//
// Kernel: 256 threads = 4 waves in a 2x2 grid, output tile 128 x 128 complex,
// each wave 64 x 64 complex as 2 x 2 blocks of v_mfma_f32_32x32x2f32, 4M complex
// products (re*re - im*im, re*im + im*re) reusing every operand fragment twice.
// K tiles of 16 are staged global -> registers -> LDS, the next tile's global
// loads in flight while the current one is multiplied.
#include "common.h"
#include "gemm.h"

namespace cgh {

typedef float floatx16 __attribute__((ext_vector_type(16)));

namespace {

constexpr int BM = kTileM, BN = kTileN, BK = kTileK, NT = 256, PAD = 4;
constexpr int LDA = BM + PAD, LDB = BN + PAD;

__device__ __forceinline__ float2 cz() { return make_float2(0.f, 0.f); }

__device__ __forceinline__ floatx16 mfma(float a, float b, floatx16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
}

// Flat grid over (layer, level, row tile, col tile), level 1 (largest) first.
struct FlatGrid {
    int levels;
    int cum[kMaxLevels + 1];   // cumulative tiles per layer up to level l
    int ctl[kMaxLevels + 1];   // column tiles of level l
    __device__ __forceinline__ void decode(int bid, int& d, int& l, int& m0, int& n0) const {
        const int per = cum[levels];
        d = bid / per;
        int r = bid - d * per;
        l = 1;
        while (l < levels && r >= cum[l]) ++l;
        r -= cum[l - 1];
        m0 = (r / ctl[l]) * BM;
        n0 = (r % ctl[l]) * BN;
    }
};

// ------------------------------------------------------------------ kernel
template <class Pb>
__global__ __launch_bounds__(NT, 2) void cgemm_f32_kernel(Pb pb) {
    __shared__ float As[2][BK][LDA];
    __shared__ float Bs[2][BK][LDB];
    typename Pb::Ctx cx;
    if (!pb.setup(cx)) return;
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int wm = (wave >> 1) * 64, wn = (wave & 1) * 64;
    const int l32 = lane & 31;

    floatx16 cr[2][2], ci[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r) { cr[i][j][r] = 0.f; ci[i][j][r] = 0.f; }

    float2 ra[8], rb[8];
    const int nk = pb.nk(cx);

    auto load = [&](int kt) {
        const typename Pb::KT kd = pb.kt(cx, kt);
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            int m, k;
            if (Pb::A_KFAST) { k = tid & 15; m = (tid >> 4) + 16 * e; }
            else { m = tid & 127; k = (tid >> 7) + 2 * e; }
            ra[e] = pb.a(cx, kd, m, k);
        }
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            int n, k;
            if (Pb::B_KFAST) { k = tid & 15; n = (tid >> 4) + 16 * e; }
            else { n = tid & 127; k = (tid >> 7) + 2 * e; }
            rb[e] = pb.b(cx, kd, k, n);
        }
    };
    auto stash = [&]() {
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            int m, k;
            if (Pb::A_KFAST) { k = tid & 15; m = (tid >> 4) + 16 * e; }
            else { m = tid & 127; k = (tid >> 7) + 2 * e; }
            As[0][k][m] = ra[e].x;
            if (Pb::A_CPLX) As[1][k][m] = ra[e].y;
        }
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            int n, k;
            if (Pb::B_KFAST) { k = tid & 15; n = (tid >> 4) + 16 * e; }
            else { n = tid & 127; k = (tid >> 7) + 2 * e; }
            Bs[0][k][n] = rb[e].x;
            if (Pb::B_CPLX) Bs[1][k][n] = rb[e].y;
        }
    };

    if (nk > 0) {
        load(0);
        stash();
    }
    __syncthreads();
    for (int kt = 0; kt < nk; ++kt) {
        if (kt + 1 < nk) load(kt + 1);
#pragma unroll
        for (int ks = 0; ks < BK / 2; ++ks) {
            const int kk = 2 * ks + (lane >> 5);
            float ar[2], ai[2], br[2], bi[2];
#pragma unroll
            for (int b = 0; b < 2; ++b) {
                ar[b] = As[0][kk][wm + 32 * b + l32];
                ai[b] = Pb::A_CPLX ? As[1][kk][wm + 32 * b + l32] : 0.f;
                br[b] = Bs[0][kk][wn + 32 * b + l32];
                bi[b] = Pb::B_CPLX ? Bs[1][kk][wn + 32 * b + l32] : 0.f;
            }
            if constexpr (Pb::A_CPLX && Pb::B_CPLX) {
                float nai[2] = {-ai[0], -ai[1]};
#pragma unroll
                for (int i = 0; i < 2; ++i)
#pragma unroll
                    for (int j = 0; j < 2; ++j) cr[i][j] = mfma(ar[i], br[j], cr[i][j]);
                if constexpr (!Pb::OUT_REAL) {
#pragma unroll
                    for (int i = 0; i < 2; ++i)
#pragma unroll
                        for (int j = 0; j < 2; ++j) ci[i][j] = mfma(ar[i], bi[j], ci[i][j]);
                }
#pragma unroll
                for (int i = 0; i < 2; ++i)
#pragma unroll
                    for (int j = 0; j < 2; ++j) cr[i][j] = mfma(nai[i], bi[j], cr[i][j]);
                if constexpr (!Pb::OUT_REAL) {
#pragma unroll
                    for (int i = 0; i < 2; ++i)
#pragma unroll
                        for (int j = 0; j < 2; ++j) ci[i][j] = mfma(ai[i], br[j], ci[i][j]);
                }
            } else if constexpr (Pb::A_CPLX) {
#pragma unroll
                for (int i = 0; i < 2; ++i)
#pragma unroll
                    for (int j = 0; j < 2; ++j) {
                        cr[i][j] = mfma(ar[i], br[j], cr[i][j]);
                        ci[i][j] = mfma(ai[i], br[j], ci[i][j]);
                    }
            } else {
#pragma unroll
                for (int i = 0; i < 2; ++i)
#pragma unroll
                    for (int j = 0; j < 2; ++j) {
                        cr[i][j] = mfma(ar[i], br[j], cr[i][j]);
                        ci[i][j] = mfma(ar[i], bi[j], ci[i][j]);
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
            for (int r = 0; r < 16; ++r) {
                const int m = wm + 32 * i + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
                const int n = wn + 32 * j + l32;
                pb.store(cx, m, n, cr[i][j][r], ci[i][j][r]);
            }
}

// ------------------------------------------------------ split-precision kernel
// Same tiles, loaders and epilogue as the FP32 kernel; every staged FP32 operand
// value v is split into hi = round16(v) and lo = round16(v - hi) (bf16 or fp16,
// round to nearest even) and each real product a*b is formed as
// a_hi*b_hi + a_hi*b_lo + a_lo*b_hi on v_mfma_f32_32x32x16_{bf16,f16} with FP32
// accumulation.  LDS holds, per component (re_hi, re_lo, im_hi, im_lo), a
// [row][k] tile with k contiguous so that each MFMA fragment (8 consecutive k
// of one row) is one 16-byte LDS read.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 halfx8 __attribute__((ext_vector_type(8)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

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
__device__ __forceinline__ void split_pair(float v, unsigned& hi, unsigned& lo) {
    if constexpr (P == P_BF16) {
        const __bf16 h = (__bf16)v;
        const __bf16 l = (__bf16)(v - (float)h);
        hi = __builtin_bit_cast(unsigned short, h);
        lo = __builtin_bit_cast(unsigned short, l);
    } else {
        const _Float16 h = (_Float16)v;
        const _Float16 l = (_Float16)(v - (float)h);
        hi = __builtin_bit_cast(unsigned short, h);
        lo = __builtin_bit_cast(unsigned short, l);
    }
}

// 8 values -> packed hi and lo halves (4 x 32-bit each).
template <int P>
__device__ __forceinline__ void split8(const float* v, u32x4& hi, u32x4& lo) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        unsigned h0, l0, h1, l1;
        split_pair<P>(v[2 * q], h0, l0);
        split_pair<P>(v[2 * q + 1], h1, l1);
        hi[q] = h0 | (h1 << 16);
        lo[q] = l0 | (l1 << 16);
    }
}

constexpr int SRS = 24;  // LDS row stride in 16-bit elements (16 k + 8 pad = 48 bytes)

template <class Pb, int P>
__global__ __launch_bounds__(NT) void cgemm_split_kernel(Pb pb) {
    constexpr int NCA = Pb::A_CPLX ? 4 : 2;
    constexpr int NCB = Pb::B_CPLX ? 4 : 2;
    __shared__ __attribute__((aligned(16))) uint16_t As[NCA][BM][SRS];
    __shared__ __attribute__((aligned(16))) uint16_t Bs[NCB][BN][SRS];
    typename Pb::Ctx cx;
    if (!pb.setup(cx)) return;
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int wm = (wave >> 1) * 64, wn = (wave & 1) * 64;
    const int l32 = lane & 31, kq = 8 * (lane >> 5);

    floatx16 cr[2][2], ci[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r) { cr[i][j][r] = 0.f; ci[i][j][r] = 0.f; }

    // staging: each thread owns 8 consecutive k of one row of A and of B
    const int ra_row = Pb::A_KFAST ? (tid >> 1) : (tid & 127);
    const int ra_k = Pb::A_KFAST ? 8 * (tid & 1) : 8 * (tid >> 7);
    const int rb_row = Pb::B_KFAST ? (tid >> 1) : (tid & 127);
    const int rb_k = Pb::B_KFAST ? 8 * (tid & 1) : 8 * (tid >> 7);
    float2 ra[8], rb[8];
    const int nk = pb.nk(cx);

    auto load = [&](int kt) {
        const typename Pb::KT kd = pb.kt(cx, kt);
#pragma unroll
        for (int e = 0; e < 8; ++e) ra[e] = pb.a(cx, kd, ra_row, ra_k + e);
#pragma unroll
        for (int e = 0; e < 8; ++e) rb[e] = pb.b(cx, kd, rb_k + e, rb_row);
    };
    auto stash = [&]() {
        float v[8];
        u32x4 hi, lo;
#pragma unroll
        for (int e = 0; e < 8; ++e) v[e] = ra[e].x;
        split8<P>(v, hi, lo);
        *reinterpret_cast<u32x4*>(&As[0][ra_row][ra_k]) = hi;
        *reinterpret_cast<u32x4*>(&As[1][ra_row][ra_k]) = lo;
        if constexpr (Pb::A_CPLX) {
#pragma unroll
            for (int e = 0; e < 8; ++e) v[e] = ra[e].y;
            split8<P>(v, hi, lo);
            *reinterpret_cast<u32x4*>(&As[2][ra_row][ra_k]) = hi;
            *reinterpret_cast<u32x4*>(&As[3][ra_row][ra_k]) = lo;
        }
#pragma unroll
        for (int e = 0; e < 8; ++e) v[e] = rb[e].x;
        split8<P>(v, hi, lo);
        *reinterpret_cast<u32x4*>(&Bs[0][rb_row][rb_k]) = hi;
        *reinterpret_cast<u32x4*>(&Bs[1][rb_row][rb_k]) = lo;
        if constexpr (Pb::B_CPLX) {
#pragma unroll
            for (int e = 0; e < 8; ++e) v[e] = rb[e].y;
            split8<P>(v, hi, lo);
            *reinterpret_cast<u32x4*>(&Bs[2][rb_row][rb_k]) = hi;
            *reinterpret_cast<u32x4*>(&Bs[3][rb_row][rb_k]) = lo;
        }
    };

    if (nk > 0) {
        load(0);
        stash();
    }
    __syncthreads();
    for (int kt = 0; kt < nk; ++kt) {
        if (kt + 1 < nk) load(kt + 1);
        u32x4 a[2][NCA], b[2][NCB];
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int c = 0; c < NCA; ++c)
                a[i][c] = *reinterpret_cast<const u32x4*>(&As[c][wm + 32 * i + l32][kq]);
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int c = 0; c < NCB; ++c)
                b[j][c] = *reinterpret_cast<const u32x4*>(&Bs[c][wn + 32 * j + l32][kq]);
        // three-term product of split operands: x_hi*y_hi + x_hi*y_lo + x_lo*y_hi
        auto prod3 = [&](floatx16 acc, const u32x4& xh, const u32x4& xl, const u32x4& yh,
                         const u32x4& yl) {
            acc = mfma16<P>(xh, yh, acc);
            acc = mfma16<P>(xh, yl, acc);
            acc = mfma16<P>(xl, yh, acc);
            return acc;
        };
        if constexpr (Pb::A_CPLX && Pb::B_CPLX) {
            u32x4 nah[2], nal[2];  // -A_im: flip the sign bit of every half
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                nah[i] = a[i][2] ^ 0x80008000u;
                nal[i] = a[i][3] ^ 0x80008000u;
            }
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j) {
                    cr[i][j] = prod3(cr[i][j], a[i][0], a[i][1], b[j][0], b[j][1]);
                    cr[i][j] = prod3(cr[i][j], nah[i], nal[i], b[j][2], b[j][3]);
                    if constexpr (!Pb::OUT_REAL) {
                        ci[i][j] = prod3(ci[i][j], a[i][0], a[i][1], b[j][2], b[j][3]);
                        ci[i][j] = prod3(ci[i][j], a[i][2], a[i][3], b[j][0], b[j][1]);
                    }
                }
        } else if constexpr (Pb::A_CPLX) {
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j) {
                    cr[i][j] = prod3(cr[i][j], a[i][0], a[i][1], b[j][0], b[j][1]);
                    ci[i][j] = prod3(ci[i][j], a[i][2], a[i][3], b[j][0], b[j][1]);
                }
        } else {
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j) {
                    cr[i][j] = prod3(cr[i][j], a[i][0], a[i][1], b[j][0], b[j][1]);
                    ci[i][j] = prod3(ci[i][j], a[i][0], a[i][1], b[j][2], b[j][3]);
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
            for (int r = 0; r < 16; ++r) {
                const int m = wm + 32 * i + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
                const int n = wn + 32 * j + l32;
                pb.store(cx, m, n, cr[i][j][r], ci[i][j][r]);
            }
}

// ------------------------------------------------------------ operand helpers
// Fringe table entry for pixel `pix` of coefficient column/row `coef` of a level
// with n_l coefficients per band: band = coef >= n_l, offset pix - (coef mod n_l) 2^l.
__device__ __forceinline__ float2 fringe(const float* __restrict__ lut_level, int len, int n_pix,
                                         int nl, int l, int pix, int coef, bool conj) {
    const int band = coef >= nl;
    const int c = coef - band * nl;
    const float* tb = lut_level + (size_t)band * 2 * len;
    const int idx = pix - (c << l) + n_pix;
    const float re = tb[idx], im = tb[len + idx];
    return make_float2(re, conj ? -im : im);
}

// --------------------------------------------------------- backward, stage 1
// Q_{d,l}[r, x] = sum_y conj(Fy_{d,l}[y, r]) * G[y, x]
struct BwdS1 {
    static constexpr bool A_CPLX = true, B_CPLX = true, OUT_REAL = false;
    static constexpr bool A_KFAST = true, B_KFAST = false;
    const float* lut;
    const float2* g_in;
    float2* q;
    int ny, nx, L;
    size_t t_layer;
    FlatGrid g;
    struct Ctx { int d, l, m0, n0, sy, nyl; const float* lut; float2* q; };
    struct KT { int y0; };
    __device__ bool setup(Ctx& cx) const {
        g.decode(blockIdx.x, cx.d, cx.l, cx.m0, cx.n0);
        cx.sy = band_side(ny, cx.l);
        cx.nyl = ny >> cx.l;
        cx.lut = lut + lut_table(cx.d, cx.l, 0, 0, L) * lut_len(ny);
        cx.q = q + (size_t)cx.d * t_layer + t_level_rows(ny, cx.l) * nx;
        return true;
    }
    __device__ int nk(const Ctx&) const { return (ny + BK - 1) / BK; }
    __device__ KT kt(const Ctx&, int i) const { return KT{i * BK}; }
    __device__ float2 a(const Ctx& cx, const KT& kd, int m, int k) const {
        const int r = cx.m0 + m, y = kd.y0 + k;
        if (r < cx.sy && y < ny) return fringe(cx.lut, lut_len(ny), ny, cx.nyl, cx.l, y, r, true);
        return cz();
    }
    __device__ float2 b(const Ctx& cx, const KT& kd, int k, int n) const {
        const int y = kd.y0 + k, x = cx.n0 + n;
        if (y < ny && x < nx) return g_in[(size_t)y * nx + x];
        return cz();
    }
    __device__ void store(const Ctx& cx, int m, int n, float re, float im) const {
        const int r = cx.m0 + m, x = cx.n0 + n;
        if (r < cx.sy && x < nx) cx.q[(size_t)r * nx + x] = make_float2(re, im);
    }
};

// --------------------------------------------------------- backward, stage 2
// gC_{d,l}[r, j] = Re( sum_x Q_{d,l}[r, x] * conj(Fx_{d,l}[x, j]) ), at level-l positions only
struct BwdS2 {
    static constexpr bool A_CPLX = true, B_CPLX = true, OUT_REAL = true;
    static constexpr bool A_KFAST = true, B_KFAST = true;
    const float* lut;
    const float2* q;
    float* gcoef;
    int ny, nx, L;
    size_t t_layer;
    FlatGrid g;
    struct Ctx { int d, l, m0, n0, sy, sx, nyl, nxl; const float* lut; const float2* q; float* gc; };
    struct KT { int x0; };
    __device__ bool setup(Ctx& cx) const {
        g.decode(blockIdx.x, cx.d, cx.l, cx.m0, cx.n0);
        const int l = cx.l;
        cx.sy = band_side(ny, l);
        cx.sx = band_side(nx, l);
        cx.nyl = ny >> l;
        cx.nxl = nx >> l;
        if (l < L && cx.m0 + BM <= cx.nyl && cx.n0 + BN <= cx.nxl) return false;  // coarser level's square
        cx.lut = lut + lut_table(cx.d, l, 0, 0, L) * lut_len(nx);
        cx.q = q + (size_t)cx.d * t_layer + t_level_rows(ny, l) * nx;
        cx.gc = gcoef + (size_t)cx.d * ny * nx;
        return true;
    }
    __device__ int nk(const Ctx&) const { return (nx + BK - 1) / BK; }
    __device__ KT kt(const Ctx&, int i) const { return KT{i * BK}; }
    __device__ float2 a(const Ctx& cx, const KT& kd, int m, int k) const {
        const int r = cx.m0 + m, x = kd.x0 + k;
        if (r < cx.sy && x < nx) return cx.q[(size_t)r * nx + x];
        return cz();
    }
    __device__ float2 b(const Ctx& cx, const KT& kd, int k, int n) const {
        const int x = kd.x0 + k, j = cx.n0 + n;
        if (j < cx.sx && x < nx) return fringe(cx.lut, lut_len(nx), nx, cx.nxl, cx.l, x, j, true);
        return cz();
    }
    __device__ void store(const Ctx& cx, int m, int n, float re, float) const {
        const int r = cx.m0 + m, j = cx.n0 + n;
        if (r < cx.sy && j < cx.sx && !(cx.l < L && r < cx.nyl && j < cx.nxl))
            cx.gc[(size_t)r * nx + j] = re;
    }
};

__global__ __launch_bounds__(256) void reduce_partial_kernel(const float2* __restrict__ partial,
                                                             int split, size_t n, int accumulate,
                                                             float2* __restrict__ out) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) {
        float2 v = accumulate ? out[i] : make_float2(0.f, 0.f);
        for (int s = 0; s < split; ++s) {
            const float2 p = partial[(size_t)s * n + i];
            v.x += p.x;
            v.y += p.y;
        }
        out[i] = v;
    }
}

template <class Pb>
hipError_t run(const Pb& pb, dim3 grid, hipStream_t s, int precision = P_FP32) {
    if (grid.x == 0 || grid.y == 0 || grid.z == 0) return hipSuccess;
    if (precision == P_BF16)
        hipLaunchKernelGGL((cgemm_split_kernel<Pb, P_BF16>), grid, dim3(NT), 0, s, pb);
    else if (precision == P_FP16)
        hipLaunchKernelGGL((cgemm_split_kernel<Pb, P_FP16>), grid, dim3(NT), 0, s, pb);
    else
        hipLaunchKernelGGL(cgemm_f32_kernel<Pb>, grid, dim3(NT), 0, s, pb);
    return hipGetLastError();
}

FlatGrid make_grid(int ny, int levels, const int* cols_per_level) {
    FlatGrid g{};
    g.levels = levels;
    g.cum[0] = 0;
    for (int l = 1; l <= levels; ++l) {
        const int rows = (band_side(ny, l) + BM - 1) / BM;
        g.ctl[l] = (cols_per_level[l] + BN - 1) / BN;
        g.cum[l] = g.cum[l - 1] + rows * g.ctl[l];
    }
    return g;
}

}  // namespace

// --------------------------------------------------------------- launchers
hipError_t launch_reduce_partial(const GemmShape& sh, const float2* partial, float2* out,
                                 int accumulate, hipStream_t s) {
    if (sh.split_k <= 1) return hipSuccess;
    const size_t n = (size_t)sh.ny * sh.nx;
    size_t blocks = (n + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(reduce_partial_kernel, dim3((unsigned)blocks), dim3(256), 0, s, partial,
                       sh.split_k, n, accumulate, out);
    return hipGetLastError();
}

hipError_t launch_backward(const GemmShape& sh, const float2* grad_h, const float* lut_x,
                               const float* lut_y, float2* q, float* gcoef, hipStream_t s) {
    int cols[kMaxLevels + 1];
    for (int l = 1; l <= sh.levels; ++l) cols[l] = sh.nx;
    BwdS1 p1{};
    p1.lut = lut_y;
    p1.g_in = grad_h;
    p1.q = q;
    p1.ny = sh.ny;
    p1.nx = sh.nx;
    p1.L = sh.levels;
    p1.t_layer = sh.t_layer;
    p1.g = make_grid(sh.ny, sh.levels, cols);
    hipError_t e = run(p1, dim3(p1.g.cum[sh.levels] * sh.layers), s, sh.precision);
    if (e != hipSuccess) return e;
    for (int l = 1; l <= sh.levels; ++l) cols[l] = band_side(sh.nx, l);
    BwdS2 p2{};
    p2.lut = lut_x;
    p2.q = q;
    p2.gcoef = gcoef;
    p2.ny = sh.ny;
    p2.nx = sh.nx;
    p2.L = sh.levels;
    p2.t_layer = sh.t_layer;
    p2.g = make_grid(sh.ny, sh.levels, cols);
    return run(p2, dim3(p2.g.cum[sh.levels] * sh.layers), s, sh.precision);
}

}  // namespace cgh
