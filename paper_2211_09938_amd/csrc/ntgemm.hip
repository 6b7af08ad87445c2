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
// The single-scene second contraction of the split forms has a kernel of its
// own (nt_pp_kernel, one workgroup per CU, operands global -> LDS by direct
// loads into a three-stage ring); see its comment.
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

// Operand panels are read through global-address-space pointers: generic
// (flat) loads also count against the LDS wait counter, so the wait before each
// barrier would stall on the global loads issued for the K tile after next.
typedef const u32x4 __attribute__((address_space(1)))* gptr_u32x4;
__device__ __forceinline__ u32x4 gload16(const unsigned char* base, size_t byte_off) {
    return *(gptr_u32x4)(base + byte_off);
}

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

// One output tile (m0, n0) of problem e over K tiles [kb, ke).  GEN: the B operand is
// generated from the fringe tables (NtEntry::g_lut) instead of read from its panel.
template <int P, bool A_CPLX, class Epi, int TM, int TN, int KS, bool GEN = false>
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

    // GEN: thread = (row pair gp, rows n = n0 + 2 gp and n + 1 of the B tile; 4
    // consecutive k' from gk).  Entries (n, k') and (n + 1, k') of the operand-format
    // tables are adjacent and the first is even (n, N and every offset even), so each k'
    // is one aligned 16-byte read, and the lanes of a wave read one contiguous run.  The
    // offsets of a K tile are read one tile ahead of the table reads that need them, so
    // that waiting for them never waits for the loads in flight behind them.
    // Lanes: tid = 16 a + 4 b + c takes row pair 4 a + c and k' group b (4 k' each), so
    // that the LDS stores of 8 (16) consecutive lanes spread over the banks (row pairs
    // 2 rows apart share banks every 4 pairs; the groups shift them by 16 (8) bytes).
    static_assert(!GEN || TN == 128, "generated B: 128-column tiles");
    constexpr int KPT = 4;
    const int gp = 4 * (tid >> 4) + (tid & 3), gk = 4 * ((tid >> 2) & 3);
    u32x4 gv[KPT];
    int gkoff[KPT];
    // the offset segment of a (layer, level) is padded to 16: a K tile's offsets are in
    // bounds (past g_count they are not used) and the 4 of a group are one aligned read
    auto gen_list = [&](int kt) {
        const int k = max(min(kb + kt * F::KB, ke - F::KB), 0) + gk;
        const u32x4 v = gload16(reinterpret_cast<const unsigned char*>(e.g_koff), (size_t)k * 4);
#pragma unroll
        for (int q = 0; q < 4; ++q) gkoff[q] = (int)v[q];
    };
    // rows past N (the last column tile of a ragged N) read row N - 2 and store zero
    const int gn_tab = min(n0 + 2 * gp, e.N - 2) + e.N;
    const bool grow_zero = n0 + TN > e.N && n0 + 2 * gp >= e.N;
    auto gen_load = [&](int kt) {
        const unsigned char* tb = static_cast<const unsigned char*>(e.g_lut);
#pragma unroll
        for (int q = 0; q < KPT; ++q) {
            // offsets in [2^l - N, 2N] and 3N (k' past the list: the zero band), so every
            // index is even and in [2, 6N - 2]
            const int idx = gn_tab + gkoff[q];
            gv[q] = gload16(tb, (unsigned)idx * 8u);
        }
        gen_list(kt + 1);
    };
    auto gen_stash = [&]() {
        if (grow_zero) {
#pragma unroll
            for (int q = 0; q < KPT; ++q) gv[q] = u32x4{0u, 0u, 0u, 0u};
        }
        // word w of entry pair q: 0 row n re, 1 row n im, 2 row n+1 re, 3 row n+1 im
        auto word = [&](int q, int w) -> unsigned { return gv[q][w]; };
        unsigned char* row = Bs + (2 * gp) * F::PITCH + gk * F::ES;
#pragma unroll
        for (int rr = 0; rr < 2; ++rr) {
            unsigned char* pr = row + rr * F::PITCH;
            if constexpr (P == P_FP32) {
                // planes re, im: 4 floats each
#pragma unroll
                for (int part = 0; part < 2; ++part)
                    *reinterpret_cast<u32x4*>(pr + part * BPLANE) =
                        u32x4{word(0, 2 * rr + part), word(1, 2 * rr + part),
                              word(2, 2 * rr + part), word(3, 2 * rr + part)};
            } else {
                // an entry word is hi | lo << 16; planes re hi, re lo, im hi, im lo hold
                // 4 halves each
#pragma unroll
                for (int part = 0; part < 2; ++part) {
                    unsigned hi[2], lo[2];
#pragma unroll
                    for (int q = 0; q < 4; q += 2) {
                        // v_perm_b32 bytes 0-3 from a, 4-7 from b: hi = a.lo16 | b.lo16 << 16,
                        // lo = a.hi16 | b.hi16 << 16
                        const unsigned a = word(q, 2 * rr + part), b = word(q + 1, 2 * rr + part);
                        hi[q / 2] = __builtin_amdgcn_perm(b, a, 0x05040100u);
                        lo[q / 2] = __builtin_amdgcn_perm(b, a, 0x07060302u);
                    }
                    unsigned char* ph = pr + (2 * part) * BPLANE;
                    *reinterpret_cast<u32x2*>(ph) = u32x2{hi[0], hi[1]};
                    *reinterpret_cast<u32x2*>(ph + BPLANE) = u32x2{lo[0], lo[1]};
                }
            }
        }
    };
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
                ra[u] = gload16(Ab, el * F::ES);
            } else {
                ra[u] = u32x4{0u, 0u, 0u, 0u};
            }
        }
        if constexpr (GEN) {
            gen_load(kt);
        } else {
#pragma unroll
            for (int u = 0; u < QB; ++u) {
                const int q = tid + 256 * u;
                const int c = (q >> 3) % F::CPR, rl = (q & 7) + 8 * (q / (8 * F::CPR));
                const int row = rl % TN, plane = rl / TN;
                const int n = n0 + row;
                if (n < e.N && (F::KB == kKT || k0 + c * KPC < ke)) {
                    const size_t el = (size_t)plane * e.b_ps + kblk_off(n, k0 + c * KPC, e.ldb);
                    rb[u] = gload16(Bb, el * F::ES);
                } else {
                    rb[u] = u32x4{0u, 0u, 0u, 0u};
                }
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
        if constexpr (GEN) {
            gen_stash();
        } else {
#pragma unroll
            for (int u = 0; u < QB; ++u) {
                const int q = tid + 256 * u;
                const int c = (q >> 3) % F::CPR, rl = (q & 7) + 8 * (q / (8 * F::CPR));
                const int row = rl % TN, plane = rl / TN;
                *reinterpret_cast<u32x4*>(Bs + plane * BPLANE + row * F::PITCH + c * 16) = rb[u];
            }
        }
    };

    // Per K tile: this tile's operands LDS -> registers; barrier (the LDS tile
    // is free); stash the next tile and start loading the one after it; the
    // MFMAs on the registers (they cover the LDS writes and the global loads);
    // barrier (the next tile is visible).
    if constexpr (GEN) gen_list(0);
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
                    if constexpr (P == P_FP16) {  // power-of-two range scale: exact
                        re[q] *= e.out_scale;
                        im[q] *= e.out_scale;
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
template <int P, bool A_CPLX, class Epi, int TM, int TN, int KS, bool GEN = false>
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
    nt_tile<P, A_CPLX, Epi, TM, TN, KS, GEN>(e, m0, n0, kb, ke, s, split, As, Bs);
}

// Workgroups reach the 8 XCDs round-robin (block b on XCD b % 8).  Renumbered
// so that each XCD takes one contiguous run of (split, tile) indices -- whole
// rows of tiles of one K split -- and its L2 holds the operand rows they share
// (the split kernel's single problem has the same K in every tile, so runs stay
// balanced): block b is the idx-th of XCD x, which owns the run starting at
// x * (total / 8) + min(x, total % 8).
__device__ __forceinline__ int xcd_run_index(int total) {
    const int x = blockIdx.x % 8, idx = blockIdx.x / 8;
    return x * (total / 8) + min(x, total % 8) + idx;
}

// Second contraction of the split forms at one workgroup per CU: 256 x 128
// tiles, each wave 128 x 64 (4 x 2 blocks of 32 x 32, 256 accumulators, which
// only the AGPR file of a lone wave per SIMD can hold).  With one wave per SIMD
// nothing hides a stall, so the K loop keeps every wait off the matrix cores:
//  * operands go global -> LDS by direct loads (global_load_lds_dwordx4: no
//    staging registers, no LDS stores) into a ring of three LDS stages, issued
//    two K tiles ahead of their use;
//  * the next K tile's operands are read LDS -> registers block row by block
//    row as the current tile's MFMAs release them (B through a second set);
//  * one barrier per K tile, preceded by the wait for the wave's own direct
//    loads of the next tile (the compiler schedules the two ahead of the first
//    block row's MFMAs; fenced after them they measured the same).
// LDS layout of a stage: per plane, blocks of 32 rows x 32 bytes (1 KB, one
// direct load of a wave); in a block, row r's 16-byte half h sits in slot
// 2r + (h ^ ((r >> 3) & 1)), so the 16 lanes of each phase of a 16-byte read
// (16 rows, one half) hit 16 different bank groups.
// Tile indices past the K range are clamped to its last tile (a harmless
// reload), and rows past M or N to the last row: the output rows and columns
// they feed are never stored, so the loop body has no branches.
struct PpShape {
    static constexpr int TM = 256, TN = 128;
    static constexpr int APLANE = TM * 32, BPLANE = TN * 32;      // bytes per K tile
    static constexpr int STAGE = 4 * APLANE + 4 * BPLANE;        // four 16-bit planes each
    static constexpr int NSTAGE = 3;
    static constexpr int LDS = NSTAGE * STAGE;
    static constexpr int ABLK = 4 * TM / 32, BBLK = 4 * TN / 32;  // 1 KB blocks per K tile
    static constexpr int DA = ABLK / 4, DB = BBLK / 4;            // direct loads per wave
};

typedef void __attribute__((address_space(3)))* lptr_t;
typedef const void __attribute__((address_space(1)))* gvptr_t;

// s_waitcnt with only the vector-memory counter constrained (gfx9 encoding:
// vmcnt bits 3:0 and 15:14, expcnt 6:4 and lgkmcnt 11:8 at their maxima).
template <int N>
__device__ __forceinline__ void wait_vmcnt() {
    static_assert(N >= 0 && N < 64, "vmcnt range");
    __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | 0x70 | 0xF00);
}

template <int P, class Epi>
__device__ __forceinline__ void pp_tile(const NtEntry& e, int m0, int n0, int kb, int ke, int s,
                                        int split, unsigned char* smem) {
    using C = PpShape;
    const int nk = ke > kb ? (ke - kb) / kKT : 0;
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int wm = (wave >> 1) * 128, wn = (wave & 1) * 64;
    const int l32 = lane & 31, g = lane >> 5;

    floatx16 cr[4][2], ci[4][2];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                cr[i][j][r] = 0.f;
                ci[i][j][r] = 0.f;
            }

    if (nk > 0) {
        const unsigned char* Ab = static_cast<const unsigned char*>(e.a);
        const unsigned char* Bb = static_cast<const unsigned char*>(e.b);
        // direct loads of this wave: A blocks wave + 4u, B blocks wave + 4u
        // (block = plane * rows / 32 + row block); lane -> (row, 16-byte half).
        // Address = wave-uniform base (plane, K tile, tile origin) + a 32-bit
        // lane offset below 8 KB (the row clamp keeps m - m0 in [0, 256)).
        const int lr = lane >> 1, lh = (lane & 1) ^ ((lr >> 3) & 1);
        unsigned aoff[C::DA], boff[C::DB];
#pragma unroll
        for (int u = 0; u < C::DA; ++u) {
            const int rb = (wave + 4 * u) % (C::TM / 32);
            const int m = min(m0 + 32 * rb + lr, e.M - 1);
            aoff[u] = (unsigned)(((m - m0) * 16 + 8 * lh) * 2);
        }
#pragma unroll
        for (int u = 0; u < C::DB; ++u) {
            const int rb = (wave + 4 * u) % (C::TN / 32);
            const int n = min(n0 + 32 * rb + lr, e.N - 1);
            boff[u] = (unsigned)(((n - n0) * 16 + 8 * lh) * 2);
        }
        const unsigned char* abase = Ab + ((size_t)(kb >> 4) * e.lda + (size_t)m0 * 16) * 2;
        const unsigned char* bbase = Bb + ((size_t)(kb >> 4) * e.ldb + (size_t)n0 * 16) * 2;
        // one K tile = one K block: lda / ldb elements (rows x 16) of 2 bytes
        const size_t astep = (size_t)e.lda * 2, bstep = (size_t)e.ldb * 2;
        const size_t aps = (size_t)e.a_ps * 2, bps = (size_t)e.b_ps * 2;     // bytes per plane
        auto issue = [&](int kt, int stage_off) {
            const int t = kt < nk ? kt : nk - 1;
            unsigned char* st = smem + stage_off;
#pragma unroll
            for (int u = 0; u < C::DA; ++u) {
                const int plane = (wave + 4 * u) / (C::TM / 32);
                const unsigned char* src = abase + (size_t)t * astep + plane * aps;
                __builtin_amdgcn_global_load_lds((gvptr_t)(src + aoff[u]),
                                                 (lptr_t)(st + (wave + 4 * u) * 1024), 16, 0, 0);
            }
#pragma unroll
            for (int u = 0; u < C::DB; ++u) {
                const int plane = (wave + 4 * u) / (C::TN / 32);
                const unsigned char* src = bbase + (size_t)t * bstep + plane * bps;
                __builtin_amdgcn_global_load_lds((gvptr_t)(src + boff[u]),
                                                 (lptr_t)(st + 4 * C::APLANE + (wave + 4 * u) * 1024),
                                                 16, 0, 0);
            }
        };
        // a lane's operands: row l32 of a 32-row block, K half g
        const int slot = (2 * l32 + (g ^ ((l32 >> 3) & 1))) * 16;
        // stage_off: byte offset of a stage (wave-uniform); the rest folds into
        // the read's immediate offset
        const int abyte = (wm >> 5) * 1024 + slot, bbyte = 4 * C::APLANE + (wn >> 5) * 1024 + slot;
        auto read_a = [&](int stage_off, int i, int c) {
            return *reinterpret_cast<const u32x4*>(smem + (stage_off + abyte) + c * C::APLANE + i * 1024);
        };
        auto read_b = [&](int stage_off, int j, int c) {
            return *reinterpret_cast<const u32x4*>(smem + (stage_off + bbyte) + c * C::BPLANE + j * 1024);
        };

        constexpr int NL = C::DA + C::DB;  // direct loads per wave and K tile
        issue(0, 0);
        issue(1, C::STAGE);
        issue(2, 2 * C::STAGE);
        wait_vmcnt<2 * NL>();
        __syncthreads();
        u32x4 a[4][4], b0[2][4], b1[2][4];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int c = 0; c < 4; ++c) a[i][c] = read_a(0, i, c);
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int c = 0; c < 4; ++c) b0[j][c] = read_b(0, j, c);

        // One K tile: (a, b) hold tile kt.  After the MFMAs of A block row i,
        // block row i of tile kt + 1 is read into its registers; B of tile
        // kt + 1 goes to bn.  The wait and the barrier belong to block row 0's
        // step (the compiler places them ahead of that row's MFMAs).
        // so_cur: stage of tile kt (takes tile kt + 3), so_nxt: stage of tile kt + 1;
        // rotated through the three stages by the loop
        int so_cur = 0, so_nxt = C::STAGE, so_far = 2 * C::STAGE;
        auto step = [&](int kt, u32x4 (&b)[2][4], u32x4 (&bn)[2][4]) {
            // -B_im: flip the sign bit of every 16-bit half
            u32x4 nb[2][2];
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                nb[j][0] = b[j][2] ^ 0x80008000u;
                nb[j][1] = b[j][3] ^ 0x80008000u;
            }
            const int sn = __builtin_amdgcn_readfirstlane(so_nxt);
#pragma unroll
            for (int i = 0; i < 4; ++i) {
#pragma unroll
                for (int j = 0; j < 2; ++j) {
                    cr[i][j] = prod3<P>(cr[i][j], a[i][0], a[i][1], b[j][0], b[j][1]);
                    ci[i][j] = prod3<P>(ci[i][j], a[i][0], a[i][1], b[j][2], b[j][3]);
                    cr[i][j] = prod3<P>(cr[i][j], a[i][2], a[i][3], nb[j][0], nb[j][1]);
                    ci[i][j] = prod3<P>(ci[i][j], a[i][2], a[i][3], b[j][0], b[j][1]);
                }
                if (i == 0) {
                    // own direct loads of tile kt + 1 done (tile kt + 2's may be in
                    // flight), then everyone's: tile kt + 1 visible, and stage
                    // kt % 3 (tile kt) read by every wave, so it takes tile kt + 3
                    wait_vmcnt<NL>();
                    __syncthreads();
                    issue(kt + 3, __builtin_amdgcn_readfirstlane(so_cur));
#pragma unroll
                    for (int j = 0; j < 2; ++j)
#pragma unroll
                        for (int c = 0; c < 4; ++c) bn[j][c] = read_b(sn, j, c);
                }
#pragma unroll
                for (int c = 0; c < 4; ++c) a[i][c] = read_a(sn, i, c);
                __builtin_amdgcn_sched_barrier(0);
            }
            const int t = so_cur;
            so_cur = so_nxt;
            so_nxt = so_far;
            so_far = t;
        };
        for (int kt = 0; kt < nk; ++kt) {
            step(kt, b0, b1);
#pragma unroll
            for (int j = 0; j < 2; ++j)
#pragma unroll
                for (int c = 0; c < 4; ++c) b0[j][c] = b1[j][c];
        }
        // no direct load may still write the LDS when the workgroup ends
        wait_vmcnt<0>();
    }

#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int qd = 0; qd < 4; ++qd) {
                float re[4], im[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    // power-of-two range scale of the FP16 form (exact; 1 for BF16,
                    // where the multiply also keeps the accumulators' move out of
                    // the AGPRs from spilling 21 of them to scratch)
                    re[q] = cr[i][j][4 * qd + q] * e.out_scale;
                    im[q] = ci[i][j][4 * qd + q] * e.out_scale;
                }
                Epi::store4(e, s, split, m0 + wm + 32 * i + 8 * qd + 4 * g,
                            n0 + wn + 32 * j + l32, re, im);
            }
}

// Direct schedule of the one-workgroup-per-CU split kernel (block id = s * count + t).
template <int P, class Epi>
__global__ __launch_bounds__(256, 1) void nt_pp_kernel(const NtEntry* __restrict__ entries,
                                                       int n_entries,
                                                       const int* __restrict__ tile_count,
                                                       int split) {
    __shared__ __attribute__((aligned(16))) unsigned char smem[PpShape::LDS];
    const int count = *tile_count;
    const int total = count * split;
    if ((int)blockIdx.x >= total) return;
    // one problem: XCD-contiguous runs; a table of scenes (different K): round-robin
    const int bid = n_entries == 1 ? xcd_run_index(total) : (int)blockIdx.x;
    const int s = bid / count;
    const int t = bid - s * count;
    const NtEntry e = entries[find_entry(entries, n_entries, t)];
    const int local = t - e.tile_begin;
    const int m0 = (local / e.tiles_n) * PpShape::TM;
    const int n0 = (local % e.tiles_n) * PpShape::TN;
    const int chunk = pad_kt((e.K + split - 1) / split);
    const int kb = s * chunk;
    const int ke = min(e.K, kb + chunk);
    pp_tile<P, Epi>(e, m0, n0, kb, ke, s, split, smem);
}

// Tile (mt, nt) of the `local`-th tile in band order: bands of kBandRows row
// tiles, column-major inside a band, so that a run of consecutive indices
// covers a near-square block of the output (the last band may be shorter).
constexpr int kBandRows = 8;
__device__ __forceinline__ void band_tile(int local, int tiles_m, int tiles_n, int& mt, int& nt) {
    const int band = local / (kBandRows * tiles_n);
    const int h = min(kBandRows, tiles_m - band * kBandRows);
    const int r = local - band * kBandRows * tiles_n;
    mt = band * kBandRows + r % h;
    nt = r / h;
}

// Direct schedule: block id = s * count + t.  A table of several problems runs
// round-robin over the XCDs (the first contraction's tables mix problems of very
// different K, which contiguous runs per XCD would leave unbalanced -- measured
// 1.8x slower).  A single problem (same K in every tile) gives each XCD one
// contiguous run of (split, tile) indices in band order: an XCD's workgroups
// then cover a block of about 8 x 8 output tiles and its L2 holds the A and B
// rows they share, instead of every XCD fetching the whole B panel for two rows
// of tiles.
template <int P, bool A_CPLX, class Epi, int TM, int TN, bool GEN = false>
__global__ __launch_bounds__(256, direct_occ<P>()) void nt_direct_kernel(
    const NtEntry* __restrict__ entries, int n_entries, const int* __restrict__ tile_count,
    int split) {
    using S = Smem<P, A_CPLX, TM, TN, kDirectKS>;
    __shared__ __attribute__((aligned(16))) unsigned char As[S::A];
    __shared__ __attribute__((aligned(16))) unsigned char Bs[S::B];
    const int count = *tile_count;
    const int total = count * split;
    if ((int)blockIdx.x >= total) return;
    if (n_entries == 1) {
        const int bid = xcd_run_index(total);
        const int s = bid / count;
        const NtEntry e = entries[0];
        int mt, nt;
        band_tile(bid - s * count - e.tile_begin, (e.M + TM - 1) / TM, e.tiles_n, mt, nt);
        const int chunk = pad_kt((e.K + split - 1) / split);
        const int kb = s * chunk;
        const int ke = min(e.K, kb + chunk);
        nt_tile<P, A_CPLX, Epi, TM, TN, kDirectKS, GEN>(e, mt * TM, nt * TN, kb, ke, s, split, As,
                                                        Bs);
        return;
    }
    const int bid = blockIdx.x;
    const int s = bid / count;
    run_tile<P, A_CPLX, Epi, TM, TN, kDirectKS, GEN>(entries, n_entries, bid - s * count, s, split,
                                                     As, Bs);
}

// Persistent schedule: pull tiles from *queue until *tile_count is reached;
// every workgroup exits once the counter passes the end of the table.
template <int P, bool A_CPLX, class Epi, int TM, int TN, bool GEN = false>
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
        run_tile<P, A_CPLX, Epi, TM, TN, kPersistKS, GEN>(entries, n_entries, t, 0, 1, As, Bs);
    }
}

template <int P, bool SECOND, int TM, int TN>
hipError_t persistent(const NtEntry* entries, int n_entries, const int* count, int* queue,
                      int grid, hipStream_t s) {
    if (SECOND)
        hipLaunchKernelGGL((nt_persistent_kernel<P, true, SecondEpi, TM, TN>), dim3(grid),
                           dim3(256), 0, s, entries, n_entries, count, queue);
    else
        // as the single-scene launch: 128-column tiles generate the fringe operand
        hipLaunchKernelGGL((nt_persistent_kernel<P, false, FirstEpi<P>, TM, TN,
                                                 nt_first_generates(TN)>),
                           dim3(grid), dim3(256), 0, s, entries, n_entries, count, queue);
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

template <int P, int TM, int TN>
void first_direct_shape(int layers, int levels, const NtBuffers& b, int max_tiles, hipStream_t s) {
    // 128-column tiles generate the fringe operand from the tables (its panel is not
    // gathered); the 64-column tiles of small scenes read the gathered panel
    hipLaunchKernelGGL((nt_direct_kernel<P, false, FirstEpi<P>, TM, TN, nt_first_generates(TN)>),
                       dim3(max_tiles), dim3(256), 0, s, b.first, layers * levels,
                       &b.hdr->first_tiles, 1);
}

template <int P>
hipError_t first_direct(int layers, int levels, const NtBuffers& b, int max_tiles, int tile_m,
                        int tile_n, hipStream_t s) {
    if (max_tiles <= 0) return hipSuccess;
    if (tile_m == 64 && tile_n == 64) first_direct_shape<P, 64, 64>(layers, levels, b, max_tiles, s);
    else if (tile_m == 64) first_direct_shape<P, 64, 128>(layers, levels, b, max_tiles, s);
    else if (tile_n == 64) first_direct_shape<P, 128, 64>(layers, levels, b, max_tiles, s);
    else first_direct_shape<P, 128, 128>(layers, levels, b, max_tiles, s);
    return hipGetLastError();
}

template <int P, int TN>
hipError_t second_direct(int ny, int nx, int split, const NtBuffers& b, hipStream_t s) {
    const int tiles = nt_tiles(ny, nx, 128, TN);
    hipLaunchKernelGGL((nt_direct_kernel<P, true, SecondEpi, 128, TN>), dim3(tiles * split),
                       dim3(256), 0, s, b.second, 1, &b.hdr->second_tiles, split);
    return hipGetLastError();
}

template <int P>
hipError_t second_pp(int ny, int nx, int split, const NtBuffers& b, hipStream_t s) {
    const int tiles = nt_tiles(ny, nx, PpShape::TM, PpShape::TN);
    hipLaunchKernelGGL((nt_pp_kernel<P, SecondEpi>), dim3(tiles * split), dim3(256), 0, s,
                       b.second, 1, &b.hdr->second_tiles, split);
    return hipGetLastError();
}

}  // namespace

int nt_first_tile_m(int precision) { return precision == P_FP32 ? 64 : 128; }

// 128-column tiles unless the scene is small: at most 512 tiles (two workgroups per
// CU) even with every row and column active, in either contraction order; 64-column
// tiles then give the launch twice the workgroups.
long long nt_first_tiles_bound(int ny, int nx, int layers, int levels, int tm, int tn) {
    long long tiles = 0;
    for (int l = 1; l <= levels; ++l) {
        const long long syl = band_side(ny, l), sxl = band_side(nx, l);
        const long long r = (syl + tm - 1) / tm * ((nx + tn - 1) / tn);
        const long long c = (sxl + tm - 1) / tm * ((ny + tn - 1) / tn);
        tiles += r > c ? r : c;
    }
    return tiles * layers;
}

int nt_first_tile_n(int ny, int nx, int layers, int levels, int precision) {
    return nt_first_tiles_bound(ny, nx, layers, levels, nt_first_tile_m(precision), 128) < 512
               ? 64
               : 128;
}
int nt_ring_tile_m() { return PpShape::TM; }
int nt_ring_tile_n() { return PpShape::TN; }

hipError_t launch_nt_ring_table(int precision, const NtEntry* entries, int n_entries,
                                const int* tile_count, int max_tiles, hipStream_t s) {
    if (max_tiles <= 0 || n_entries <= 0) return hipSuccess;
    if (precision == P_BF16)
        hipLaunchKernelGGL((nt_pp_kernel<P_BF16, SecondEpi>), dim3(max_tiles), dim3(256), 0, s,
                           entries, n_entries, tile_count, 1);
    else if (precision == P_FP16)
        hipLaunchKernelGGL((nt_pp_kernel<P_FP16, SecondEpi>), dim3(max_tiles), dim3(256), 0, s,
                           entries, n_entries, tile_count, 1);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

int nt_second_tile_m(int precision) { return precision == P_FP32 ? 128 : PpShape::TM; }
int nt_second_tile_n(int precision) { return precision == P_FP32 ? 64 : 128; }

hipError_t launch_nt_first(int layers, int levels, int precision, const NtBuffers& b,
                           int max_tiles, int tile_n, hipStream_t s) {
    const int tm = nt_first_tile_m(precision);
    if (precision == P_BF16) return first_direct<P_BF16>(layers, levels, b, max_tiles, tm, tile_n, s);
    if (precision == P_FP16) return first_direct<P_FP16>(layers, levels, b, max_tiles, tm, tile_n, s);
    return first_direct<P_FP32>(layers, levels, b, max_tiles, tm, tile_n, s);
}

hipError_t launch_nt_second(int ny, int nx, int precision, int split, const NtBuffers& b,
                            hipStream_t s) {
    if (precision == P_BF16) return second_pp<P_BF16>(ny, nx, split, b, s);
    if (precision == P_FP16) return second_pp<P_FP16>(ny, nx, split, b, s);
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
