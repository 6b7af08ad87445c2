// Block-local kernels of the coefficient stage:
//  * fused layer split + multi-level averaging Haar analysis + saliency
//    block-max quantisation + detail masking (Sec. 2 Eq. 2, algorithm step 1,
//    detail selection of steps 3-5), one thread per 2^L x 2^L block;
//  * plain Haar synthesis;
//  * gradient synthesis (transpose of the masked analysis, with the layer gather).
//
// The averaging Haar transform of 2^L levels never mixes pixels of different
// aligned 2^L blocks, so every block is independent: no halo, one pass over HBM.
#include "common.h"

namespace cgh {

namespace {

template <int B>
struct Pool {
    float s1[B / 2][B / 2];
    float s2[(B >= 4) ? B / 4 : 1][(B >= 4) ? B / 4 : 1];
    float s3[(B >= 8) ? B / 8 : 1][(B >= 8) ? B / 8 : 1];
};

template <int L>
__device__ __forceinline__ void pool_saliency(const float* __restrict__ sal, int nx, int by, int bx,
                                              Pool<(1 << L)>& p) {
    constexpr int B = 1 << L;
    float s[B][B];
#pragma unroll
    for (int r = 0; r < B; ++r)
#pragma unroll
        for (int c = 0; c < B; ++c) s[r][c] = sal[(size_t)(by * B + r) * nx + bx * B + c];
#pragma unroll
    for (int j = 0; j < B / 2; ++j)
#pragma unroll
        for (int i = 0; i < B / 2; ++i)
            p.s1[j][i] = fmaxf(fmaxf(s[2 * j][2 * i], s[2 * j][2 * i + 1]),
                               fmaxf(s[2 * j + 1][2 * i], s[2 * j + 1][2 * i + 1]));
    if constexpr (L >= 2) {
#pragma unroll
        for (int j = 0; j < B / 4; ++j)
#pragma unroll
            for (int i = 0; i < B / 4; ++i)
                p.s2[j][i] = fmaxf(fmaxf(p.s1[2 * j][2 * i], p.s1[2 * j][2 * i + 1]),
                                   fmaxf(p.s1[2 * j + 1][2 * i], p.s1[2 * j + 1][2 * i + 1]));
    }
    if constexpr (L >= 3) {
        p.s3[0][0] = fmaxf(fmaxf(p.s2[0][0], p.s2[0][1]), fmaxf(p.s2[1][0], p.s2[1][1]));
    }
}

template <int B>
__device__ __forceinline__ float pooled(const Pool<B>& p, int lev, int j, int i) {
    if (lev == 1) return p.s1[j][i];
    if (lev == 2) return p.s2[(B >= 4) ? j : 0][(B >= 4) ? i : 0];
    return p.s3[0][0];
}

// One thread per 2^L x 2^L block; threads along x are adjacent blocks.
//
// parts: bit l-1 enables the level-l details (l = 1..L), bit L the level-L
// approximation; a disabled part is written as zero (progressive stages).
// ops (optional, zeroed by the caller): ops[l-1] += 4 x the level-l detail
// positions whose block is salient, the operator count of Sec. 3 (one
// operator per point of the level's residual map that is processed).  The
// masks are the same for every layer, so they are counted once.
// Returns the largest |object| value of the block; with count_ops, wave_ops[l-1]
// receives the wave's level-l count (the same value in every lane that has a block).
// occ (optional): one byte per (layer, block), 1 where a pixel of the block belongs to
// the layer.  With occ the coefficients of the other (layer, block) pairs, all zero,
// are not written: readers of the coefficient planes consult occ.  Without occ
// every plane is written in full.
template <int L, bool MASK>
__device__ __forceinline__ float dwt_mask_body(
    const float* __restrict__ obj, const uint8_t* __restrict__ layer, const float* __restrict__ sal,
    int ny, int nx, int layers, float t1, float t2, float t3, unsigned parts,
    float* __restrict__ coef, uint8_t* __restrict__ flags, size_t flags_layer,
    uint8_t* __restrict__ occ, bool count_ops, unsigned long long (&wave_ops)[3], int bx,
    int by) {
    constexpr int B = 1 << L;
    const int nbx = nx >> L;
    if (bx >= nbx) return 0.f;

    float a[B][B];
    uint8_t li[B][B];
    // rows of B >= 4 floats start on 16-byte boundaries (nx is a multiple of B):
    // vector loads when the base pointers allow them
    const bool vec = B >= 4 && ((reinterpret_cast<uintptr_t>(obj) & 15) == 0) &&
                     (!layer || (reinterpret_cast<uintptr_t>(layer) & (B - 1)) == 0);
#pragma unroll
    for (int r = 0; r < B; ++r) {
        const size_t g = (size_t)(by * B + r) * nx + (size_t)bx * B;
        if (vec) {
            if constexpr (B >= 4) {
#pragma unroll
                for (int c = 0; c < B; c += 4) {
                    const float4 v = *reinterpret_cast<const float4*>(obj + g + c);
                    a[r][c] = v.x;
                    a[r][c + 1] = v.y;
                    a[r][c + 2] = v.z;
                    a[r][c + 3] = v.w;
                }
                if (layer) {
                    if constexpr (B == 8) {
                        const uint2 u = *reinterpret_cast<const uint2*>(layer + g);
#pragma unroll
                        for (int c = 0; c < 4; ++c) {
                            li[r][c] = (u.x >> (8 * c)) & 0xffu;
                            li[r][c + 4] = (u.y >> (8 * c)) & 0xffu;
                        }
                    } else {
                        const unsigned u = *reinterpret_cast<const unsigned*>(layer + g);
#pragma unroll
                        for (int c = 0; c < B; ++c) li[r][c] = (u >> (8 * c)) & 0xffu;
                    }
                } else {
#pragma unroll
                    for (int c = 0; c < B; ++c) li[r][c] = 0;
                }
            }
        } else {
#pragma unroll
            for (int c = 0; c < B; ++c) {
                a[r][c] = obj[g + c];
                li[r][c] = layer ? layer[g + c] : 0;
            }
        }
    }
    float amax = 0.f;
#pragma unroll
    for (int r = 0; r < B; ++r)
#pragma unroll
        for (int c = 0; c < B; ++c) amax = fmaxf(amax, fabsf(a[r][c]));
    Pool<B> pool;
    if (sal) pool_saliency<L>(sal, nx, by, bx, pool);
    const bool vst = (reinterpret_cast<uintptr_t>(coef) & 15) == 0;  // vector stores
    const float thr[3] = {t1, t2, t3};
    const size_t plane = (size_t)ny * nx;

    if (count_ops) {
        // the masks are shared by the layers: counted once, from the saliency alone
#pragma unroll
        for (int lev = 1; lev <= L; ++lev) {
            const int h = B >> lev;
#pragma unroll
            for (int j = 0; j < h; ++j)
#pragma unroll
                for (int i = 0; i < h; ++i) {
                    const bool salient = !sal || pooled<B>(pool, lev, j, i) > thr[lev - 1];
                    wave_ops[lev - 1] += __popcll(__ballot(salient));
                }
        }
    }

    const size_t blocks = (size_t)(ny >> L) * nbx;
    // MASK (at most 32 layers): bit (index mod 32) of every pixel's layer, a superset of the
    // layers the block holds; a layer no lane of the wave has costs only its occupancy byte.
    unsigned pres = 0u;
    if constexpr (MASK) {
#pragma unroll
        for (int r = 0; r < B; ++r)
#pragma unroll
            for (int c = 0; c < B; ++c) pres |= 1u << (li[r][c] & 31u);
    }
    for (int d = 0; d < layers; ++d) {
        if constexpr (MASK) {
            if (__ballot((pres >> d) & 1u) == 0ull) {
                if (occ) occ[(size_t)d * blocks + (size_t)by * nbx + bx] = 0;
                continue;
            }
        }
        float cur[B][B];
        bool present = false;
#pragma unroll
        for (int r = 0; r < B; ++r)
#pragma unroll
            for (int c = 0; c < B; ++c) {
                present |= li[r][c] == d;
                cur[r][c] = (li[r][c] == d) ? a[r][c] : 0.0f;
            }
        // with occ, a layer without a pixel in the block has only zero coefficients
        // and no flags: nothing to compute or store
        if (occ) {
            occ[(size_t)d * blocks + (size_t)by * nbx + bx] = present ? 1 : 0;
            if (!present) continue;
        }
        // lowest lane working on this layer: writes the row flags once per wave (all
        // lanes share by)
        const bool leader = (int)__lane_id() == __ffsll((long long)__ballot(1)) - 1;
        const size_t base = (size_t)d * plane;
        uint8_t* fl = flags ? flags + (size_t)d * flags_layer : nullptr;
#pragma unroll
        for (int lev = 1; lev <= L; ++lev) {
            const int h = B >> lev;
            const int nyl = ny >> lev, nxl = nx >> lev;
            uint8_t* frow = fl ? fl + flag_level_off(ny, nx, lev) : nullptr;
            uint8_t* fcol = frow ? frow + band_side(ny, lev) : nullptr;
            float lo[B][B / 2], hi[B][B / 2];
#pragma unroll
            for (int r = 0; r < 2 * h; ++r)
#pragma unroll
                for (int i = 0; i < h; ++i) {
                    lo[r][i] = (cur[r][2 * i] + cur[r][2 * i + 1]) * 0.5f;
                    hi[r][i] = (cur[r][2 * i] - cur[r][2 * i + 1]) * 0.5f;
                }
            bool col_lo[B / 2], col_hi[B / 2];  // column flags of this thread's h columns
#pragma unroll
            for (int i = 0; i < h; ++i) col_lo[i] = col_hi[i] = false;
#pragma unroll
            for (int j = 0; j < h; ++j) {
                float v[B / 2], hv[B / 2], dv[B / 2];
                bool row_top = false, row_bot = false;
#pragma unroll
                for (int i = 0; i < h; ++i) {
                    const float ll = (lo[2 * j][i] + lo[2 * j + 1][i]) * 0.5f;
                    const float hh = (lo[2 * j][i] - lo[2 * j + 1][i]) * 0.5f;
                    const float vv = (hi[2 * j][i] + hi[2 * j + 1][i]) * 0.5f;
                    const float dd = (hi[2 * j][i] - hi[2 * j + 1][i]) * 0.5f;
                    const bool salient = !sal || pooled<B>(pool, lev, j, i) > thr[lev - 1];
                    const bool keep = ((parts >> (lev - 1)) & 1u) && salient;
                    v[i] = keep ? vv : 0.0f;
                    hv[i] = keep ? hh : 0.0f;
                    dv[i] = keep ? dd : 0.0f;
                    row_top |= v[i] != 0.0f;
                    row_bot |= (hv[i] != 0.0f) || (dv[i] != 0.0f);
                    col_hi[i] |= (v[i] != 0.0f) || (dv[i] != 0.0f);
                    col_lo[i] |= hv[i] != 0.0f;
                    cur[j][i] = ll;
                }
                const int gy = by * h + j, gx0 = bx * h;
                float* pv = coef + base + (size_t)gy * nx + nxl + gx0;
                float* ph = coef + base + (size_t)(nyl + gy) * nx + gx0;
                float* pd = coef + base + (size_t)(nyl + gy) * nx + nxl + gx0;
                // h consecutive floats on an h*4-byte boundary (nx is a multiple of 2^L)
                if constexpr (B / 2 >= 4) {
                    if (h == 4 && vst) {
                        *reinterpret_cast<float4*>(pv) = make_float4(v[0], v[1], v[2], v[3]);
                        *reinterpret_cast<float4*>(ph) = make_float4(hv[0], hv[1], hv[2], hv[3]);
                        *reinterpret_cast<float4*>(pd) = make_float4(dv[0], dv[1], dv[2], dv[3]);
                    }
                }
                if constexpr (B / 2 >= 2) {
                    if (h == 2 && vst) {
                        *reinterpret_cast<float2*>(pv) = make_float2(v[0], v[1]);
                        *reinterpret_cast<float2*>(ph) = make_float2(hv[0], hv[1]);
                        *reinterpret_cast<float2*>(pd) = make_float2(dv[0], dv[1]);
                    }
                }
                if (h == 1 || !vst) {
#pragma unroll
                    for (int i = 0; i < h; ++i) {
                        pv[i] = v[i];
                        ph[i] = hv[i];
                        pd[i] = dv[i];
                    }
                }
                if (frow) {
                    const bool any_top = __ballot(row_top) != 0ull;
                    const bool any_bot = __ballot(row_bot) != 0ull;
                    if (leader && any_top) frow[gy] = 1;
                    if (leader && any_bot) frow[nyl + gy] = 1;
                }
            }
            if (fcol) {
#pragma unroll
                for (int i = 0; i < h; ++i) {
                    if (col_lo[i]) fcol[bx * h + i] = 1;
                    if (col_hi[i]) fcol[nxl + bx * h + i] = 1;
                }
            }
        }
        const float av = ((parts >> L) & 1u) ? cur[0][0] : 0.0f;
        coef[base + (size_t)by * nx + bx] = av;
        if (fl) {
            uint8_t* frow = fl + flag_level_off(ny, nx, L);
            const bool any_av = __ballot(av != 0.0f) != 0ull;  // every lane on this layer
            if (leader && any_av) frow[by] = 1;
            if (av != 0.0f) frow[band_side(ny, L) + bx] = 1;
        }
    }
    return amax;
}

// ops (optional): ops[0..2] operator counts, ops[4] max |object| as float bits (the
// range of the FP16 split operands), both zeroed by the caller.
template <int L, bool MASK>
__device__ __forceinline__ void dwt_mask_block(
    const float* __restrict__ obj, const uint8_t* __restrict__ layer, const float* __restrict__ sal,
    int ny, int nx, int layers, float t1, float t2, float t3, unsigned parts,
    float* __restrict__ coef, uint8_t* __restrict__ flags, size_t flags_layer,
    uint8_t* __restrict__ occ, unsigned long long* __restrict__ ops, int bx, int by) {
    unsigned long long wave_ops[3] = {0ull, 0ull, 0ull};
    float amax = dwt_mask_body<L, MASK>(obj, layer, sal, ny, nx, layers, t1, t2, t3, parts, coef, flags,
                                  flags_layer, occ, ops != nullptr, wave_ops, bx, by);
    if (ops) {
        // Counts and max |object| gathered over the workgroup first: one atomic per
        // counter and workgroup (atomics on one address from every wave of every XCD
        // serialise).  Every lane is active here: lanes past the row hold 0, and lane 0
        // of a wave that has any block holds the wave's counts.
        __shared__ unsigned long long s_ops[4][3];
        __shared__ float s_max[4];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) amax = fmaxf(amax, __shfl_xor(amax, off));
        const int w = threadIdx.x >> 6;
        if (__lane_id() == 0) {
            s_max[w] = amax;
            for (int l = 0; l < 3; ++l) s_ops[w][l] = wave_ops[l];
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            const int nw = blockDim.x >> 6;  // 4: the launches use 256 threads
            float m = 0.f;
            for (int k = 0; k < nw; ++k) m = fmaxf(m, s_max[k]);
            for (int l = 0; l < L; ++l) {
                unsigned long long c = 0ull;
                for (int k = 0; k < nw; ++k) c += s_ops[k][l];
                if (c) atomicAdd(&ops[l], 4ull * c);
            }
            if (m > 0.f) atomicMax(&ops[4], (unsigned long long)__float_as_uint(m));
        }
    }
}

template <int L, bool MASK>
__global__ __launch_bounds__(256) void dwt_mask_kernel(
    const float* __restrict__ obj, const uint8_t* __restrict__ layer, const float* __restrict__ sal,
    int ny, int nx, int layers, float t1, float t2, float t3, unsigned parts,
    float* __restrict__ coef, uint8_t* __restrict__ flags, size_t flags_layer,
    uint8_t* __restrict__ occ, unsigned long long* __restrict__ ops) {
    dwt_mask_block<L, MASK>(obj, layer, sal, ny, nx, layers, t1, t2, t3, parts, coef, flags,
                      flags_layer, occ, ops, blockIdx.x * blockDim.x + threadIdx.x, blockIdx.y);
}

// Every scene of a batch in one launch: grid.z = scene, x / y sized for the largest.
template <int L>
__global__ __launch_bounds__(256) void dwt_mask_batch_kernel(const DwtScene* __restrict__ scenes,
                                                             float t1, float t2, float t3) {
    const DwtScene sc = scenes[blockIdx.z];
    if ((int)blockIdx.y >= (sc.ny >> L)) return;
    dwt_mask_block<L, false>(sc.obj, sc.layer, sc.sal, sc.ny, sc.nx, sc.layers, t1, t2, t3, kAllParts,
                      sc.coef, sc.flags, sc.flags_layer, sc.occ, sc.ops,
                      blockIdx.x * blockDim.x + threadIdx.x, blockIdx.y);
}

// Synthesis of one block from Mallat coefficients (inverse of the analysis above).
template <int L>
__device__ __forceinline__ void synth_block(const float* __restrict__ c, int ny, int nx, int by,
                                            int bx, const float (*scale)[2], float out[1 << L][1 << L]) {
    constexpr int B = 1 << L;
    float cur[B][B];
    cur[0][0] = c[(size_t)by * nx + bx] * scale[L][0];
#pragma unroll
    for (int lev = L; lev >= 1; --lev) {
        const int h = B >> lev;
        const int nyl = ny >> lev, nxl = nx >> lev;
        float nxt[B][B];
#pragma unroll
        for (int j = 0; j < h; ++j)
#pragma unroll
            for (int i = 0; i < h; ++i) {
                const int gy = by * h + j, gx = bx * h + i;
                const float s = scale[lev][1];
                const float vv = c[(size_t)gy * nx + nxl + gx] * s;
                const float hh = c[(size_t)(nyl + gy) * nx + gx] * s;
                const float dd = c[(size_t)(nyl + gy) * nx + nxl + gx] * s;
                const float lo0 = cur[j][i] + hh, lo1 = cur[j][i] - hh;
                const float hi0 = vv + dd, hi1 = vv - dd;
                nxt[2 * j][2 * i] = lo0 + hi0;
                nxt[2 * j][2 * i + 1] = lo0 - hi0;
                nxt[2 * j + 1][2 * i] = lo1 + hi1;
                nxt[2 * j + 1][2 * i + 1] = lo1 - hi1;
            }
#pragma unroll
        for (int r = 0; r < 2 * h; ++r)
#pragma unroll
            for (int q = 0; q < 2 * h; ++q) cur[r][q] = nxt[r][q];
    }
#pragma unroll
    for (int r = 0; r < B; ++r)
#pragma unroll
        for (int q = 0; q < B; ++q) out[r][q] = cur[r][q];
}

template <int L>
__global__ __launch_bounds__(256) void idwt_kernel(const float* __restrict__ coef, int ny, int nx,
                                                   float* __restrict__ out) {
    constexpr int B = 1 << L;
    const int bx = blockIdx.x * blockDim.x + threadIdx.x;
    const int by = blockIdx.y;
    if (bx >= (nx >> L)) return;
    const float one[4][2] = {{1.f, 1.f}, {1.f, 1.f}, {1.f, 1.f}, {1.f, 1.f}};
    float px[B][B];
    synth_block<L>(coef, ny, nx, by, bx, one, px);
#pragma unroll
    for (int r = 0; r < B; ++r)
#pragma unroll
        for (int q = 0; q < B; ++q) out[(size_t)(by * B + r) * nx + bx * B + q] = px[r][q];
}

// grad[p] = sum_d [layer[p] == d] * S( Lambda M gcoef_d )[p], Lambda = 4^-level per coefficient.
template <int L>
__global__ __launch_bounds__(256) void grad_synthesis_kernel(
    const float* __restrict__ gcoef, const uint8_t* __restrict__ layer, const float* __restrict__ sal,
    int ny, int nx, int layers, float t1, float t2, float t3, float* __restrict__ grad) {
    constexpr int B = 1 << L;
    const int bx = blockIdx.x * blockDim.x + threadIdx.x;
    const int by = blockIdx.y;
    if (bx >= (nx >> L)) return;
    Pool<B> pool;
    if (sal) pool_saliency<L>(sal, nx, by, bx, pool);
    const float thr[3] = {t1, t2, t3};
    uint8_t li[B][B];
    float acc[B][B];
#pragma unroll
    for (int r = 0; r < B; ++r)
#pragma unroll
        for (int q = 0; q < B; ++q) {
            li[r][q] = layer ? layer[(size_t)(by * B + r) * nx + bx * B + q] : 0;
            acc[r][q] = 0.0f;
        }
    const size_t plane = (size_t)ny * nx;
    // Masked, scaled copy of this block's coefficients, then plain synthesis.
    for (int d = 0; d < layers; ++d) {
        bool present = false;
#pragma unroll
        for (int r = 0; r < B; ++r)
#pragma unroll
            for (int q = 0; q < B; ++q) present |= (li[r][q] == d);
        if (!present) continue;
        const float* c = gcoef + (size_t)d * plane;
        float cur[B][B];
        cur[0][0] = c[(size_t)by * nx + bx] * (1.0f / (float)(1 << (2 * L)));
#pragma unroll
        for (int lev = L; lev >= 1; --lev) {
            const int h = B >> lev;
            const int nyl = ny >> lev, nxl = nx >> lev;
            const float s = 1.0f / (float)(1 << (2 * lev));
            float nxt[B][B];
#pragma unroll
            for (int j = 0; j < h; ++j)
#pragma unroll
                for (int i = 0; i < h; ++i) {
                    const int gy = by * h + j, gx = bx * h + i;
                    const bool keep = !sal || pooled<B>(pool, lev, j, i) > thr[lev - 1];
                    const float k = keep ? s : 0.0f;
                    const float vv = c[(size_t)gy * nx + nxl + gx] * k;
                    const float hh = c[(size_t)(nyl + gy) * nx + gx] * k;
                    const float dd = c[(size_t)(nyl + gy) * nx + nxl + gx] * k;
                    const float lo0 = cur[j][i] + hh, lo1 = cur[j][i] - hh;
                    const float hi0 = vv + dd, hi1 = vv - dd;
                    nxt[2 * j][2 * i] = lo0 + hi0;
                    nxt[2 * j][2 * i + 1] = lo0 - hi0;
                    nxt[2 * j + 1][2 * i] = lo1 + hi1;
                    nxt[2 * j + 1][2 * i + 1] = lo1 - hi1;
                }
#pragma unroll
            for (int r = 0; r < 2 * h; ++r)
#pragma unroll
                for (int q = 0; q < 2 * h; ++q) cur[r][q] = nxt[r][q];
        }
#pragma unroll
        for (int r = 0; r < B; ++r)
#pragma unroll
            for (int q = 0; q < B; ++q) acc[r][q] += (li[r][q] == d) ? cur[r][q] : 0.0f;
    }
#pragma unroll
    for (int r = 0; r < B; ++r)
#pragma unroll
        for (int q = 0; q < B; ++q) grad[(size_t)(by * B + r) * nx + bx * B + q] = acc[r][q];
}

__global__ void fill_u8_kernel(uint8_t* p, size_t n) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) p[i] = 0;
}

__global__ void prep_fill_kernel(const DwtScene* __restrict__ scenes) {
    const DwtScene sc = scenes[blockIdx.y];
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < sc.flags_fill;
         i += (size_t)gridDim.x * blockDim.x)
        sc.flags[i] = 0;
}

}  // namespace

hipError_t launch_prep_fill(const DwtScene* scenes, int n, size_t max_fill, hipStream_t s) {
    size_t blocks = (max_fill + 255) / 256;
    if (blocks > 256) blocks = 256;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(prep_fill_kernel, dim3((unsigned)blocks, n), dim3(256), 0, s, scenes);
    return hipGetLastError();
}

hipError_t launch_dwt_mask_batch(const DwtScene* scenes, int n, int levels, const float* thr,
                                 int max_nbx, int max_nby, hipStream_t s) {
    const dim3 grid((max_nbx + 255) / 256, max_nby, n);
    const float t1 = thr[0], t2 = levels >= 2 ? thr[1] : 0.f, t3 = levels >= 3 ? thr[2] : 0.f;
    if (levels == 1) hipLaunchKernelGGL(dwt_mask_batch_kernel<1>, grid, dim3(256), 0, s, scenes, t1, t2, t3);
    else if (levels == 2) hipLaunchKernelGGL(dwt_mask_batch_kernel<2>, grid, dim3(256), 0, s, scenes, t1, t2, t3);
    else if (levels == 3) hipLaunchKernelGGL(dwt_mask_batch_kernel<3>, grid, dim3(256), 0, s, scenes, t1, t2, t3);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_fill_u8(uint8_t* p, size_t n, hipStream_t s) {
    if (n == 0) return hipSuccess;
    const int threads = 256;
    size_t blocks = (n + threads - 1) / threads;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(fill_u8_kernel, dim3((unsigned)blocks), dim3(threads), 0, s, p, n);
    return hipGetLastError();
}

template <int L>
static void dwt_launch(const float* obj, const uint8_t* layer, const float* sal, int ny, int nx,
                       int layers, const float* thr, unsigned parts, float* coef, uint8_t* flags,
                       size_t flags_layer, uint8_t* occ, unsigned long long* ops, hipStream_t s) {
    const int nbx = nx >> L;
    dim3 grid((nbx + 255) / 256, ny >> L);
    // the layer mask needs at most 32 layers, and occupancy bytes to record absent layers
    // (without them every plane is written in full)
    if (layers <= 32 && occ)
        hipLaunchKernelGGL((dwt_mask_kernel<L, true>), grid, dim3(256), 0, s, obj, layer, sal, ny,
                           nx, layers, thr[0], L >= 2 ? thr[1] : 0.f, L >= 3 ? thr[2] : 0.f, parts,
                           coef, flags, flags_layer, occ, ops);
    else
        hipLaunchKernelGGL((dwt_mask_kernel<L, false>), grid, dim3(256), 0, s, obj, layer, sal, ny,
                           nx, layers, thr[0], L >= 2 ? thr[1] : 0.f, L >= 3 ? thr[2] : 0.f, parts,
                           coef, flags, flags_layer, occ, ops);
}

hipError_t launch_dwt_mask(const float* obj, const uint8_t* layer, const float* sal, int ny, int nx,
                           int layers, int levels, const float* thr, unsigned parts, float* coef,
                           uint8_t* flags, size_t flags_layer, uint8_t* occ,
                           unsigned long long* ops, hipStream_t s) {
    if (levels == 1)
        dwt_launch<1>(obj, layer, sal, ny, nx, layers, thr, parts, coef, flags, flags_layer, occ,
                      ops, s);
    else if (levels == 2)
        dwt_launch<2>(obj, layer, sal, ny, nx, layers, thr, parts, coef, flags, flags_layer, occ,
                      ops, s);
    else if (levels == 3)
        dwt_launch<3>(obj, layer, sal, ny, nx, layers, thr, parts, coef, flags, flags_layer, occ,
                      ops, s);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_idwt(const float* coef, int ny, int nx, int levels, float* out, hipStream_t s) {
    const int nbx = nx >> levels;
    dim3 grid((nbx + 255) / 256, ny >> levels);
    if (levels == 1) hipLaunchKernelGGL(idwt_kernel<1>, grid, dim3(256), 0, s, coef, ny, nx, out);
    else if (levels == 2) hipLaunchKernelGGL(idwt_kernel<2>, grid, dim3(256), 0, s, coef, ny, nx, out);
    else if (levels == 3) hipLaunchKernelGGL(idwt_kernel<3>, grid, dim3(256), 0, s, coef, ny, nx, out);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_grad_synthesis(const float* gcoef, const uint8_t* layer, const float* sal, int ny,
                                 int nx, int layers, int levels, const float* thr, float* grad,
                                 hipStream_t s) {
    const int nbx = nx >> levels;
    dim3 grid((nbx + 255) / 256, ny >> levels);
    const float t1 = thr[0], t2 = levels >= 2 ? thr[1] : 0.f, t3 = levels >= 3 ? thr[2] : 0.f;
    if (levels == 1)
        hipLaunchKernelGGL(grad_synthesis_kernel<1>, grid, dim3(256), 0, s, gcoef, layer, sal, ny,
                           nx, layers, t1, t2, t3, grad);
    else if (levels == 2)
        hipLaunchKernelGGL(grad_synthesis_kernel<2>, grid, dim3(256), 0, s, gcoef, layer, sal, ny,
                           nx, layers, t1, t2, t3, grad);
    else if (levels == 3)
        hipLaunchKernelGGL(grad_synthesis_kernel<3>, grid, dim3(256), 0, s, gcoef, layer, sal, ny,
                           nx, layers, t1, t2, t3, grad);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

}  // namespace cgh
