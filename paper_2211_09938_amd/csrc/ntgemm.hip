// Batched NT complex GEMM on CDNA4 matrix cores for the compacted forward pass.
//
// C[m][n] = sum_k A[m][k] * B[n][k], A real or complex, B complex, both panels
// K-contiguous in the operand precision.  A workgroup of 4 waves (2 x 2)
// computes a TM x TN complex tile (TM, TN in {64, 128}); each wave owns
// (TM/64) x (TN/64) blocks of 32 x 32 MFMA output.  A device-resident table of
// self-contained problems (NtEntry) describes every GEMM of a launch; a tile
// index selects (problem, tile) by binary search over the tiles' prefix.
// Direct schedule: one workgroup per (tile, K split).  Persistent schedule:
// a grid sized to the machine pulls tiles from an atomic counter until the
// table is exhausted, so problems of very different sizes balance themselves.
// Per K tile of 16 each thread moves 16-byte chunks of A and B
// global -> registers -> LDS; a wave takes the tile's operands from LDS into
// registers, and after one barrier the next tile is stashed and the one after
// it loaded while the MFMAs run.
//
//  FP32:  v_mfma_f32_32x32x2f32; a lane's 16-byte LDS read gives it the
//         operands of 4 consecutive MFMAs (lane half g supplies k = 4g + t).
//         Complex x complex tiles of 128 x 64 and smaller use three real
//         products per complex product (Gauss), four otherwise.
//  split: v_mfma_f32_32x32x16_{bf16,f16}; operands stored as hi and lo planes,
//         each real product as hi*hi + hi*lo + lo*hi, FP32 accumulation.
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

// Operand format of precision P with KS rows of K per staged tile.  Measured
// on MI355X with K-blocked panels: both schedules run best at K 16 per staged
// tile with two workgroups per CU (K 32 at one workgroup per CU was 15% slower
// in the persistent split kernels).
template <int P, int KS = kKT>
struct Fmt {
    static constexpr int ES = (P == P_FP32) ? 4 : 2;        // bytes per element
    static constexpr int PC = (P == P_FP32) ? 2 : 4;        // planes of a complex operand
    static constexpr int PR = (P == P_FP32) ? 1 : 2;        // planes of a real operand
    static constexpr int KB = KS;                           // K per staged tile
    static constexpr int CPR = KB * ES / 16;                // 16-byte chunks per row and plane
    static constexpr int PITCH = KB * ES + 16;              // LDS bytes per row (with padding)
};

constexpr int kDirectKS = 16, kPersistKS = 16;
template <int P> constexpr int direct_occ() { return 2; }
template <int P> constexpr int persist_occ() { return 2; }

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

// First contraction output: T_c[x][k'] (transposed, operand precision);
// m is the first of 4 consecutive rows k', n the column x.
template <int P>
struct FirstEpi {
    static constexpr bool kImag = true;
    __device__ static void store4(const NtEntry& e, int, int, int m, int n, const float* re,
                                  const float* im) {
        if (m >= pad_kt(e.M) || n >= e.N) return;
        const size_t off = kblk_off(n, m, (size_t)e.out_ld);  // 4 consecutive k' of row n
        const size_t ps = (size_t)e.out_ps;
        if constexpr (P == P_FP32) {
            float* b = static_cast<float*>(e.out);
            *reinterpret_cast<floatx4*>(b + off) = floatx4{re[0], re[1], re[2], re[3]};
            *reinterpret_cast<floatx4*>(b + ps + off) = floatx4{im[0], im[1], im[2], im[3]};
        } else {
            uint16_t* b = static_cast<uint16_t*>(e.out);
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

// Second contraction output: complex64 hologram rows m..m+3, column n (or a
// split-K partial).
struct SecondEpi {
    static constexpr bool kImag = true;
    __device__ static void store4(const NtEntry& e, int s, int split, int m, int n,
                                  const float* re, const float* im) {
        if (n >= e.N) return;
        float2* out = static_cast<float2*>(e.out);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int y = m + q;
            if (y >= e.M) continue;
            const size_t i = (size_t)y * e.out_ld + n;
            float2 v = make_float2(re[q], im[q]);
            if (split == 1) {
                if (e.accumulate) {
                    const float2 o = out[i];
                    v.x += o.x;
                    v.y += o.y;
                }
                out[i] = v;
            } else {
                e.partial[(size_t)s * e.M * e.N + i] = v;
            }
        }
    }
};

// Complex product stored row-major into operand planes (the B panel of a
// following contraction): rows m..m+3, column n < pad16(N) (columns past N
// hold the zeros the K padding needs); split-K partials [s][M][N] otherwise.
template <int P>
struct PanelEpi {
    static constexpr bool kImag = true;
    __device__ static void store4(const NtEntry& e, int s, int split, int m, int n,
                                  const float* re, const float* im) {
        if (split > 1) {
            if (n >= e.N) return;
#pragma unroll
            for (int q = 0; q < 4; ++q)
                if (m + q < e.M)
                    e.partial[((size_t)s * e.M + m + q) * e.N + n] = make_float2(re[q], im[q]);
            return;
        }
        if (n >= pad_kt(e.N)) return;
#pragma unroll
        for (int q = 0; q < 4; ++q)
            if (m + q < e.M)
                put_c<P>(e.out, (size_t)e.out_ps, kblk_off(m + q, n, (size_t)e.out_ld), re[q],
                         im[q]);
    }
};

// Real part only (the imaginary products are skipped): out[m][n] floats with
// row stride out_ld, or split-K partials [s][M][N] floats.
struct RealEpi {
    static constexpr bool kImag = false;
    __device__ static void store4(const NtEntry& e, int s, int split, int m, int n,
                                  const float* re, const float*) {
        if (n >= e.N) return;
        float* part = reinterpret_cast<float*>(e.partial);
        float* out = static_cast<float*>(e.out);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            if (m + q >= e.M) continue;
            if (split > 1) part[((size_t)s * e.M + m + q) * e.N + n] = re[q];
            else out[(size_t)(m + q) * e.out_ld + n] = re[q];
        }
    }
};

// One output tile (m0, n0) of problem e over K tiles [kb, ke).
template <int P, bool A_CPLX, class Epi, int TM, int TN, int KS>
__device__ __forceinline__ void nt_tile(const NtEntry& e, int m0, int n0, int kb, int ke, int s,
                                        int split, unsigned char* As, unsigned char* Bs) {
    using F = Fmt<P, KS>;
    constexpr int NPA = A_CPLX ? F::PC : F::PR;
    constexpr int NPB = F::PC;
    constexpr int BI = TM / 64, BJ = TN / 64;  // 32 x 32 blocks per wave
    constexpr int APLANE = TM * F::PITCH, BPLANE = TN * F::PITCH;
    constexpr int QA = NPA * TM * F::CPR / 256;
    constexpr int QB = NPB * TN * F::CPR / 256;
    static_assert(QA >= 1 && QB >= 1, "tile too small for the staging layout");

    const int nk = ke > kb ? (ke - kb + F::KB - 1) / F::KB : 0;
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int wm = (wave >> 1) * (TM / 2), wn = (wave & 1) * (TN / 2);
    const int l32 = lane & 31, g = lane >> 5;

    // FP32 complex x complex: three real products per complex product (Gauss):
    // X = Ar Br, Y = Ai Bi, Z = (Ar + Ai)(Br + Bi); re = X - Y, im = Z - X - Y.
    // cr, ci, cz hold X, Y, Z there; cr, ci hold re, im otherwise.
    // (64 x 32 wave tiles and smaller: the third accumulator set of a 64 x 64
    // wave tile does not fit in the registers of two workgroups per CU)
    constexpr bool G3 = P == P_FP32 && A_CPLX && Epi::kImag && BI * BJ <= 2;
    constexpr int BZ = G3 ? BJ : 1;
    floatx16 cr[BI][BJ], ci[BI][BJ], cz[BI][BZ];
#pragma unroll
    for (int i = 0; i < BI; ++i)
#pragma unroll
        for (int j = 0; j < BJ; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                cr[i][j][r] = 0.f;
                ci[i][j][r] = 0.f;
                if constexpr (G3) cz[i][j][r] = 0.f;
            }

    // chunk q of an operand tile -> (plane, row, 16-byte chunk c of the row):
    // 8 consecutive threads take 8 consecutive rows at one chunk (with the
    // padded row pitch those 8 stores hit 8 different LDS bank groups), the
    // next 8 the next chunk of the same rows; with K-blocked panels the 64
    // threads of a wave still read one contiguous run of global memory
    u32x4 ra[QA], rb[QB];
    const unsigned char* Ab = static_cast<const unsigned char*>(e.a);
    const unsigned char* Bb = static_cast<const unsigned char*>(e.b);
    // a staged tile may run past the K range (ke is a multiple of 16 only):
    // chunks starting at or beyond ke read as zero
    constexpr int KPC = 16 / F::ES;  // k per 16-byte chunk
    auto load = [&](int kt) {
        const int k0 = kb + kt * F::KB;
#pragma unroll
        for (int u = 0; u < QA; ++u) {
            const int q = tid + 256 * u;
            const int c = (q >> 3) % F::CPR, rl = (q & 7) + 8 * (q / (8 * F::CPR));
            const int row = rl % TM, plane = rl / TM;
            const int m = m0 + row;
            if (m < e.M && (F::KB == kKT || k0 + c * KPC < ke)) {
                const size_t el = (size_t)plane * e.a_ps + kblk_off(m, k0 + c * KPC, e.lda);
                ra[u] = *reinterpret_cast<const u32x4*>(Ab + el * F::ES);
            } else {
                ra[u] = u32x4{0u, 0u, 0u, 0u};
            }
        }
#pragma unroll
        for (int u = 0; u < QB; ++u) {
            const int q = tid + 256 * u;
            const int c = (q >> 3) % F::CPR, rl = (q & 7) + 8 * (q / (8 * F::CPR));
            const int row = rl % TN, plane = rl / TN;
            const int n = n0 + row;
            if (n < e.N && (F::KB == kKT || k0 + c * KPC < ke)) {
                const size_t el = (size_t)plane * e.b_ps + kblk_off(n, k0 + c * KPC, e.ldb);
                rb[u] = *reinterpret_cast<const u32x4*>(Bb + el * F::ES);
            } else {
                rb[u] = u32x4{0u, 0u, 0u, 0u};
            }
        }
    };
    auto stash = [&]() {
#pragma unroll
        for (int u = 0; u < QA; ++u) {
            const int q = tid + 256 * u;
            const int c = (q >> 3) % F::CPR, rl = (q & 7) + 8 * (q / (8 * F::CPR));
            const int row = rl % TM, plane = rl / TM;
            *reinterpret_cast<u32x4*>(As + plane * APLANE + row * F::PITCH + c * 16) = ra[u];
        }
#pragma unroll
        for (int u = 0; u < QB; ++u) {
            const int q = tid + 256 * u;
            const int c = (q >> 3) % F::CPR, rl = (q & 7) + 8 * (q / (8 * F::CPR));
            const int row = rl % TN, plane = rl / TN;
            *reinterpret_cast<u32x4*>(Bs + plane * BPLANE + row * F::PITCH + c * 16) = rb[u];
        }
    };

    // Per K tile: this tile's operands LDS -> registers; barrier (the LDS tile
    // is free); stash the next tile and start loading the one after it; the
    // MFMAs on the registers (they cover the LDS writes and the global loads);
    // barrier (the next tile is visible).
    if (nk > 0) {
        load(0);
        stash();
    }
    __syncthreads();
    if (nk > 1) load(1);
    auto advance = [&](int kt) {
        __syncthreads();
        if (kt + 1 < nk) {
            stash();
            if (kt + 2 < nk) load(kt + 2);
        }
    };
    for (int kt = 0; kt < nk; ++kt) {
        if constexpr (P == P_FP32) {
            constexpr int NH = F::KB / 8;
            floatx4 fa[NH][BI][NPA], fb[NH][BJ][NPB];
#pragma unroll
            for (int h = 0; h < NH; ++h) {
#pragma unroll
                for (int i = 0; i < BI; ++i)
#pragma unroll
                    for (int c = 0; c < NPA; ++c)
                        fa[h][i][c] = *reinterpret_cast<const floatx4*>(
                            As + c * APLANE + (wm + 32 * i + l32) * F::PITCH + (8 * h + 4 * g) * 4);
#pragma unroll
                for (int j = 0; j < BJ; ++j)
#pragma unroll
                    for (int c = 0; c < NPB; ++c)
                        fb[h][j][c] = *reinterpret_cast<const floatx4*>(
                            Bs + c * BPLANE + (wn + 32 * j + l32) * F::PITCH + (8 * h + 4 * g) * 4);
            }
            advance(kt);
#pragma unroll
            for (int h = 0; h < NH; ++h) {
                if constexpr (G3) {
                    floatx4 sa[BI], sb[BJ];
#pragma unroll
                    for (int i = 0; i < BI; ++i) sa[i] = fa[h][i][0] + fa[h][i][1];
#pragma unroll
                    for (int j = 0; j < BJ; ++j) sb[j] = fb[h][j][0] + fb[h][j][1];
#pragma unroll
                    for (int tt = 0; tt < 4; ++tt)
#pragma unroll
                        for (int i = 0; i < BI; ++i)
#pragma unroll
                            for (int j = 0; j < BJ; ++j) {
                                cr[i][j] = mfma32(fa[h][i][0][tt], fb[h][j][0][tt], cr[i][j]);
                                ci[i][j] = mfma32(fa[h][i][1][tt], fb[h][j][1][tt], ci[i][j]);
                                cz[i][j] = mfma32(sa[i][tt], sb[j][tt], cz[i][j]);
                            }
                    continue;
                }
#pragma unroll
                for (int tt = 0; tt < 4; ++tt) {
#pragma unroll
                    for (int i = 0; i < BI; ++i)
#pragma unroll
                        for (int j = 0; j < BJ; ++j) {
                            cr[i][j] = mfma32(fa[h][i][0][tt], fb[h][j][0][tt], cr[i][j]);
                            if constexpr (Epi::kImag)
                                ci[i][j] = mfma32(fa[h][i][0][tt], fb[h][j][1][tt], ci[i][j]);
                        }
                    if constexpr (A_CPLX) {
#pragma unroll
                        for (int i = 0; i < BI; ++i)
#pragma unroll
                            for (int j = 0; j < BJ; ++j) {
                                cr[i][j] = mfma32(-fa[h][i][1][tt], fb[h][j][1][tt], cr[i][j]);
                                if constexpr (Epi::kImag)
                                    ci[i][j] = mfma32(fa[h][i][1][tt], fb[h][j][0][tt], ci[i][j]);
                            }
                    }
                }
            }
        } else {
            constexpr int NC = F::KB / 16;
            u32x4 a[NC][BI][NPA], b[NC][BJ][NPB];
#pragma unroll
            for (int kc = 0; kc < NC; ++kc) {
#pragma unroll
                for (int i = 0; i < BI; ++i)
#pragma unroll
                    for (int c = 0; c < NPA; ++c)
                        a[kc][i][c] = *reinterpret_cast<const u32x4*>(
                            As + c * APLANE + (wm + 32 * i + l32) * F::PITCH + kc * 32 + g * 16);
#pragma unroll
                for (int j = 0; j < BJ; ++j)
#pragma unroll
                    for (int c = 0; c < NPB; ++c)
                        b[kc][j][c] = *reinterpret_cast<const u32x4*>(
                            Bs + c * BPLANE + (wn + 32 * j + l32) * F::PITCH + kc * 32 + g * 16);
            }
            advance(kt);
#pragma unroll
            for (int kc = 0; kc < NC; ++kc) {
#pragma unroll
                for (int i = 0; i < BI; ++i)
#pragma unroll
                    for (int j = 0; j < BJ; ++j) {
                        cr[i][j] = prod3<P>(cr[i][j], a[kc][i][0], a[kc][i][1], b[kc][j][0], b[kc][j][1]);
                        if constexpr (Epi::kImag)
                            ci[i][j] = prod3<P>(ci[i][j], a[kc][i][0], a[kc][i][1], b[kc][j][2], b[kc][j][3]);
                    }
                if constexpr (A_CPLX) {
#pragma unroll
                    for (int i = 0; i < BI; ++i) {
                        // -A_im: flip the sign bit of every 16-bit half
                        const u32x4 nah = a[kc][i][2] ^ 0x80008000u, nal = a[kc][i][3] ^ 0x80008000u;
#pragma unroll
                        for (int j = 0; j < BJ; ++j) {
                            cr[i][j] = prod3<P>(cr[i][j], nah, nal, b[kc][j][2], b[kc][j][3]);
                            if constexpr (Epi::kImag)
                                ci[i][j] = prod3<P>(ci[i][j], a[kc][i][2], a[kc][i][3], b[kc][j][0], b[kc][j][1]);
                        }
                    }
                }
            }
        }
        __syncthreads();
    }

#pragma unroll
    for (int i = 0; i < BI; ++i)
#pragma unroll
        for (int j = 0; j < BJ; ++j)
#pragma unroll
            for (int qd = 0; qd < 4; ++qd) {
                float re[4], im[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    if constexpr (G3) {
                        const float x = cr[i][j][4 * qd + q], y = ci[i][j][4 * qd + q];
                        re[q] = x - y;
                        im[q] = cz[i][j][4 * qd + q] - x - y;
                    } else {
                        re[q] = cr[i][j][4 * qd + q];
                        im[q] = ci[i][j][4 * qd + q];
                    }
                }
                Epi::store4(e, s, split, m0 + wm + 32 * i + 8 * qd + 4 * g,
                            n0 + wn + 32 * j + l32, re, im);
            }
}

template <int P, bool A_CPLX, int TM, int TN, int KS>
struct Smem {
    using F = Fmt<P, KS>;
    static constexpr int NPA = A_CPLX ? F::PC : F::PR;
    static constexpr int A = NPA * TM * F::PITCH;
    static constexpr int B = F::PC * TN * F::PITCH;
};

// Resolves tile t of the table and runs it (K range of split s).
template <int P, bool A_CPLX, class Epi, int TM, int TN, int KS>
__device__ __forceinline__ void run_tile(const NtEntry* __restrict__ entries, int n_entries,
                                         int t, int s, int split, unsigned char* As,
                                         unsigned char* Bs) {
    const NtEntry e = entries[find_entry(entries, n_entries, t)];
    const int local = t - e.tile_begin;
    const int m0 = (local / e.tiles_n) * TM;
    const int n0 = (local % e.tiles_n) * TN;
    const int chunk = pad_kt((e.K + split - 1) / split);
    const int kb = s * chunk;
    const int ke = min(e.K, kb + chunk);
    nt_tile<P, A_CPLX, Epi, TM, TN, KS>(e, m0, n0, kb, ke, s, split, As, Bs);
}

// Direct schedule: block id = s * count + t.
template <int P, bool A_CPLX, class Epi, int TM, int TN>
__global__ __launch_bounds__(256, direct_occ<P>()) void nt_direct_kernel(
    const NtEntry* __restrict__ entries, int n_entries, const int* __restrict__ tile_count,
    int split) {
    using S = Smem<P, A_CPLX, TM, TN, kDirectKS>;
    __shared__ __attribute__((aligned(16))) unsigned char As[S::A];
    __shared__ __attribute__((aligned(16))) unsigned char Bs[S::B];
    const int count = *tile_count;
    const int bid = blockIdx.x;
    if (bid >= count * split) return;
    const int s = bid / count;
    run_tile<P, A_CPLX, Epi, TM, TN, kDirectKS>(entries, n_entries, bid - s * count, s, split, As, Bs);
}

// Persistent schedule: pull tiles from *queue until *tile_count is reached;
// every workgroup exits once the counter passes the end of the table.
template <int P, bool A_CPLX, class Epi, int TM, int TN>
__global__ __launch_bounds__(256, persist_occ<P>()) void nt_persistent_kernel(
    const NtEntry* __restrict__ entries, int n_entries, const int* __restrict__ tile_count,
    int* __restrict__ queue) {
    using S = Smem<P, A_CPLX, TM, TN, kPersistKS>;
    __shared__ __attribute__((aligned(16))) unsigned char As[S::A];
    __shared__ __attribute__((aligned(16))) unsigned char Bs[S::B];
    __shared__ int s_next;
    const int count = *tile_count;
    for (;;) {
        if (threadIdx.x == 0) s_next = atomicAdd(queue, 1);
        __syncthreads();
        const int t = s_next;
        __syncthreads();
        if (t >= count) break;
        run_tile<P, A_CPLX, Epi, TM, TN, kPersistKS>(entries, n_entries, t, 0, 1, As, Bs);
    }
}

template <int P, bool SECOND, int TM, int TN>
hipError_t persistent(const NtEntry* entries, int n_entries, const int* count, int* queue,
                      int grid, hipStream_t s) {
    if (SECOND)
        hipLaunchKernelGGL((nt_persistent_kernel<P, true, SecondEpi, TM, TN>), dim3(grid),
                           dim3(256), 0, s, entries, n_entries, count, queue);
    else
        hipLaunchKernelGGL((nt_persistent_kernel<P, false, FirstEpi<P>, TM, TN>), dim3(grid),
                           dim3(256), 0, s, entries, n_entries, count, queue);
    return hipGetLastError();
}

template <int P, bool SECOND>
hipError_t persistent_shape(int tm, int tn, const NtEntry* entries, int n_entries,
                            const int* count, int* queue, int grid, hipStream_t s) {
    if (tm == 128 && tn == 128) return persistent<P, SECOND, 128, 128>(entries, n_entries, count, queue, grid, s);
    if (tm == 64 && tn == 128) return persistent<P, SECOND, 64, 128>(entries, n_entries, count, queue, grid, s);
    if (tm == 128 && tn == 64) return persistent<P, SECOND, 128, 64>(entries, n_entries, count, queue, grid, s);
    if (tm == 64 && tn == 64) return persistent<P, SECOND, 64, 64>(entries, n_entries, count, queue, grid, s);
    return hipErrorInvalidValue;
}

template <int P>
hipError_t first_direct(int layers, int levels, const NtBuffers& b, int max_tiles, int tile_m,
                        hipStream_t s) {
    if (max_tiles <= 0) return hipSuccess;
    if (tile_m == 64)
        hipLaunchKernelGGL((nt_direct_kernel<P, false, FirstEpi<P>, 64, 128>), dim3(max_tiles),
                           dim3(256), 0, s, b.first, layers * levels, &b.hdr->first_tiles, 1);
    else
        hipLaunchKernelGGL((nt_direct_kernel<P, false, FirstEpi<P>, 128, 128>), dim3(max_tiles),
                           dim3(256), 0, s, b.first, layers * levels, &b.hdr->first_tiles, 1);
    return hipGetLastError();
}

template <int P, int TN>
hipError_t second_direct(int ny, int nx, int split, const NtBuffers& b, hipStream_t s) {
    const int tiles = nt_tiles(ny, nx, 128, TN);
    hipLaunchKernelGGL((nt_direct_kernel<P, true, SecondEpi, 128, TN>), dim3(tiles * split),
                       dim3(256), 0, s, b.second, 1, &b.hdr->second_tiles, split);
    return hipGetLastError();
}

}  // namespace

int nt_first_tile_m(int precision) { return precision == P_FP32 ? 64 : 128; }
int nt_second_tile_n(int precision) { return precision == P_FP32 ? 64 : 128; }

hipError_t launch_nt_first(int layers, int levels, int precision, const NtBuffers& b,
                           int max_tiles, hipStream_t s) {
    const int tm = nt_first_tile_m(precision);
    if (precision == P_BF16) return first_direct<P_BF16>(layers, levels, b, max_tiles, tm, s);
    if (precision == P_FP16) return first_direct<P_FP16>(layers, levels, b, max_tiles, tm, s);
    return first_direct<P_FP32>(layers, levels, b, max_tiles, tm, s);
}

hipError_t launch_nt_second(int ny, int nx, int precision, int split, const NtBuffers& b,
                            hipStream_t s) {
    if (precision == P_BF16) return second_direct<P_BF16, 128>(ny, nx, split, b, s);
    if (precision == P_FP16) return second_direct<P_FP16, 128>(ny, nx, split, b, s);
    return second_direct<P_FP32, 64>(ny, nx, split, b, s);
}

namespace {
template <int P, class Epi, int TN>
void table_launch(const NtEntry* entries, int n_entries, const int* tile_count, int tiles,
                  int split, hipStream_t s) {
    hipLaunchKernelGGL((nt_direct_kernel<P, true, Epi, 128, TN>), dim3(tiles * split),
                       dim3(256), 0, s, entries, n_entries, tile_count, split);
}
template <int P>
void table_epi(int epi, const NtEntry* entries, int n_entries, const int* tile_count, int tiles,
               int split, hipStream_t s) {
    constexpr int TN = P == P_FP32 ? 64 : 128;  // nt_table_tile_n for the complex epilogues
    if (epi == kEpiPanel) table_launch<P, PanelEpi<P>, TN>(entries, n_entries, tile_count, tiles, split, s);
    else if (epi == kEpiReal) table_launch<P, RealEpi, 128>(entries, n_entries, tile_count, tiles, split, s);
    else table_launch<P, SecondEpi, TN>(entries, n_entries, tile_count, tiles, split, s);
}
}  // namespace

hipError_t launch_nt_first_table(int precision, const NtEntry* entries, int n_entries,
                                 const int* tile_count, int tiles, hipStream_t s) {
    if (tiles <= 0 || n_entries <= 0) return hipSuccess;
    if (precision == P_BF16)
        hipLaunchKernelGGL((nt_direct_kernel<P_BF16, false, FirstEpi<P_BF16>, 128, 128>),
                           dim3(tiles), dim3(256), 0, s, entries, n_entries, tile_count, 1);
    else if (precision == P_FP16)
        hipLaunchKernelGGL((nt_direct_kernel<P_FP16, false, FirstEpi<P_FP16>, 128, 128>),
                           dim3(tiles), dim3(256), 0, s, entries, n_entries, tile_count, 1);
    else
        hipLaunchKernelGGL((nt_direct_kernel<P_FP32, false, FirstEpi<P_FP32>, 128, 128>),
                           dim3(tiles), dim3(256), 0, s, entries, n_entries, tile_count, 1);
    return hipGetLastError();
}

hipError_t launch_nt_table(int epi, int precision, const NtEntry* entries, int n_entries,
                           const int* tile_count, int tiles, int split, hipStream_t s) {
    if (tiles <= 0 || n_entries <= 0) return hipSuccess;
    if (precision == P_BF16) table_epi<P_BF16>(epi, entries, n_entries, tile_count, tiles, split, s);
    else if (precision == P_FP16) table_epi<P_FP16>(epi, entries, n_entries, tile_count, tiles, split, s);
    else table_epi<P_FP32>(epi, entries, n_entries, tile_count, tiles, split, s);
    return hipGetLastError();
}

hipError_t launch_nt_persistent(bool second, int precision, int tile_m, int tile_n,
                                const NtEntry* entries, int n_entries, const int* tile_count,
                                int* queue, int grid, hipStream_t s) {
    if (grid <= 0 || n_entries <= 0) return hipSuccess;
#define CGH_PERSIST(PR)                                                                          \
    return second ? persistent_shape<PR, true>(tile_m, tile_n, entries, n_entries, tile_count,  \
                                               queue, grid, s)                                   \
                  : persistent_shape<PR, false>(tile_m, tile_n, entries, n_entries, tile_count, \
                                                queue, grid, s);
    if (precision == P_BF16) { CGH_PERSIST(P_BF16) }
    if (precision == P_FP16) { CGH_PERSIST(P_FP16) }
    CGH_PERSIST(P_FP32)
#undef CGH_PERSIST
}

}  // namespace cgh
