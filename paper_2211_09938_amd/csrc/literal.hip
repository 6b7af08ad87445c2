// Paper-literal form of the progressive hologram on the contraction kernels.
//
// Sec. 2, steps 2-5, in the image domain: the coarsest approximation image
// (block means of 2^L x 2^L blocks) and then, level by level, the residual map
// between two consecutive approximation images, masked where the level's
// quantised saliency is below its threshold, each point of an image of block
// size 2^b multiplied onto the fringe of a uniform 2^b x 2^b block (the paper's
// look-up table) and added at the block's position.
//
// With averaging Haar the residual map of level l is the one-level synthesis
// of that level's (masked) detail coefficients alone:
//     R[2i+ay][2j+ax] = sx V[i][j] + sy H[i][j] + sx sy D[i][j],
//     sx = +1 (ax = 0) or -1 (ax = 1), sy likewise,
// and the uniform-block fringe factors per axis into the lo-band table of block
// size 2^b, so one term is Fy_b R_b Fx_b^T with F_b[m][j] = g_lo,b[m - j 2^b].
// Per layer d there are L + 1 terms (b = L for the approximation image, then
// b = L-1 .. 0 for the residuals of levels L .. 1), all dense (no compaction):
//     first:   T[x][k'] = sum_c R_{d,b}[r][c] Fx_{d,b}[x][c]      (per (d, b))
//     second:  H[y][x]  = sum_k' Fy[y][k'] T[x][k']               (k' over every (d, b))
// on the same NT kernels as the coefficient form, which it cross-checks.
#include "nt.h"
#include "split.h"

namespace cgh {

namespace {

inline int grid_1d(size_t n) {
    const size_t b = (n + 255) / 256;
    return (int)(b < 4096 ? (b > 0 ? b : 1) : 4096);
}

// Residual map (b < L) or approximation image (b == L) of layer d as a
// K-blocked real panel: rows ny >> b, K = nx >> b padded to 16.
// absmax (FP16 range scaling, else null): values scaled by 2^-e, e the exponent of
// max |object| (|residual| <= 3 max |object|).
template <int P>
__global__ __launch_bounds__(256) void residual_panel_kernel(const float* __restrict__ coef,
                                                             int ny, int nx, int L, int b,
                                                             const unsigned long long* absmax,
                                                             void* __restrict__ out, size_t ps) {
    const int rows = ny >> b, cols = nx >> b, ld = pad_kt(cols);
    const size_t total = (size_t)rows * ld;
    const float sc = absmax ? pow2f(-range_exp(absmax_value(absmax))) : 1.f;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (size_t)gridDim.x * blockDim.x) {
        int r, c;
        kblk_pos(e, rows, r, c);
        float v = 0.f;
        if (c < cols) {
            if (b == L) {
                v = coef[(size_t)r * nx + c];
            } else {
                const int l = b + 1, nyl = ny >> l, nxl = nx >> l;
                const int i = r >> 1, j = c >> 1;
                const float sy = (r & 1) ? -1.f : 1.f, sx = (c & 1) ? -1.f : 1.f;
                const float vv = coef[(size_t)i * nx + nxl + j];
                const float hh = coef[(size_t)(nyl + i) * nx + j];
                const float dd = coef[(size_t)(nyl + i) * nx + nxl + j];
                v = sx * vv + sy * hh + sx * sy * dd;
            }
        }
        put_r<P>(out, ps, e, v * sc);
    }
}

// Uniform-block fringe panel F_b[m][j] = g_lo,b[m - j 2^b] (rows n_pix, K = n_pix >> b)
// from a table (re part then im part, lut_len(n_pix) each), written K-blocked at
// element offset `off` of a panel whose K-block stride is rows x 16.
template <int P>
__global__ __launch_bounds__(256) void block_fringe_panel_kernel(const float* __restrict__ table,
                                                                 int n_pix, int b, size_t off,
                                                                 void* __restrict__ out,
                                                                 size_t ps) {
    const int cols = n_pix >> b, ld = pad_kt(cols), len = lut_len(n_pix);
    const size_t total = (size_t)n_pix * ld;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (size_t)gridDim.x * blockDim.x) {
        int m, j;
        kblk_pos(e, n_pix, m, j);
        float re = 0.f, im = 0.f;
        if (j < cols) {
            const int idx = m - (j << b) + n_pix;
            re = table[idx];
            im = table[len + idx];
        }
        put_c<P>(out, ps, off + e, re, im);
    }
}

struct LitArgs {
    int ny, nx, layers, L, es, split, tn2;
    const char* rb;       // residual panels, [d][b] in order b = L .. 0
    const char* fxb;      // x fringe panels, same order
    char* t;              // first-contraction products (K-blocked, rows nx)
    const char* fy;       // y fringe panel (K-blocked, rows ny)
    float2* hologram;
    float2* partial;
    long long rb_ps, fxb_ps, t_ps, fy_ps;
    int accumulate;
    NtEntry* first;       // [layers * (L + 1)]
    NtEntry* second;      // [1]
    int* counts;          // tile totals of the two contractions
    // FP16 range scaling: images scaled by 2^-e (|image'| < 6), the first products
    // (|T| < 6 x 8 nx) by 2^-t, the second epilogue by 2^(e + t + e_fringe)
    const unsigned long long* absmax;  // null unless FP16
    int t_shift, e_fringe;
};

// Problem tables; one thread (at most 256 x 4 problems with closed-form shapes).
__global__ void literal_entries_kernel(LitArgs a) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const float first_scale = a.absmax ? pow2f(-a.t_shift) : 1.f;
    const float second_scale =
        a.absmax ? pow2f(range_exp(absmax_value(a.absmax)) + a.t_shift + a.e_fringe) : 1.f;
    size_t rb_off = 0, fx_off = 0;
    int seg = 0, tiles = 0, t = 0;
    for (int d = 0; d < a.layers; ++d) {
        for (int b = a.L; b >= 0; --b) {
            const int rows = a.ny >> b, cols = a.nx >> b, kc = pad_kt(cols);
            NtEntry e{};
            e.a = a.rb + rb_off * a.es;
            e.b = a.fxb + fx_off * a.es;
            e.out = a.t + (size_t)seg * a.nx * a.es;  // K block seg / 16 of T
            e.a_ps = a.rb_ps;
            e.b_ps = a.fxb_ps;
            e.out_ps = a.t_ps;
            e.M = rows;
            e.N = a.nx;
            e.K = kc;
            e.lda = rows * 16;
            e.ldb = a.nx * 16;
            e.out_ld = a.nx * 16;
            e.tiles_n = (a.nx + kNtTile - 1) / kNtTile;
            e.tile_begin = tiles;
            e.tile_m = e.tile_n = kNtTile;
            e.out_scale = first_scale;
            a.first[t++] = e;
            tiles += nt_tiles(rows, a.nx, kNtTile, kNtTile);
            rb_off += (size_t)rows * kc;
            fx_off += (size_t)a.nx * kc;
            seg += pad_kt(rows);
        }
    }
    NtEntry e{};
    e.a = a.fy;
    e.b = a.t;
    e.out = a.hologram;
    e.partial = a.partial;
    e.a_ps = a.fy_ps;
    e.b_ps = a.t_ps;
    e.M = a.ny;
    e.N = a.nx;
    e.K = seg;
    e.lda = a.ny * 16;
    e.ldb = a.nx * 16;
    e.out_ld = a.nx;
    e.tiles_n = (a.nx + a.tn2 - 1) / a.tn2;
    e.accumulate = a.accumulate;
    e.tile_m = kNtTile;
    e.tile_n = a.tn2;
    e.out_scale = second_scale;
    a.second[0] = e;
    a.counts[0] = tiles;
    a.counts[1] = nt_tiles(a.ny, a.nx, kNtTile, a.tn2);
}

struct LitShape {
    size_t rb_ps, fxb_ps, kt;  // panel elements; concatenated K
    int first_tiles;
};

LitShape lit_shape(int ny, int nx, int layers, int L) {
    LitShape z{};
    for (int b = L; b >= 0; --b) {
        const int rows = ny >> b, kc = pad_kt(nx >> b);
        z.rb_ps += (size_t)rows * kc;
        z.fxb_ps += (size_t)nx * kc;
        z.kt += pad_kt(rows);
        z.first_tiles += nt_tiles(rows, nx, kNtTile, kNtTile);
    }
    z.rb_ps *= layers;
    z.fxb_ps *= layers;
    z.kt *= layers;
    z.first_tiles *= layers;
    return z;
}

struct LitRegions {
    char *rb, *fxb, *t, *fy, *lut0;
    NtEntry* entries;
    int* counts;
    size_t total;
};

LitRegions lit_regions(char* base, int ny, int nx, int layers, int L) {
    auto al = [](size_t v) { return (v + 255) / 256 * 256; };
    const LitShape z = lit_shape(ny, nx, layers, L);
    LitRegions r{};
    size_t off = 0;
    r.rb = base + off;
    off += al(4 * z.rb_ps);  // real: 4 B per element in every precision
    r.fxb = base + off;
    off += al(8 * z.fxb_ps);
    r.t = base + off;
    off += al(8 * (size_t)nx * z.kt);
    r.fy = base + off;
    off += al(8 * (size_t)ny * z.kt);
    r.lut0 = base + off;  // level-0 tables of every layer, x then y
    off += al(4 * (size_t)layers * 2 * (lut_len(nx) + lut_len(ny)));
    r.entries = reinterpret_cast<NtEntry*>(base + off);
    off += al(sizeof(NtEntry) * ((size_t)layers * (L + 1) + 1));
    r.counts = reinterpret_cast<int*>(base + off);
    off += al(2 * sizeof(int));
    r.total = off;
    return r;
}

template <int P>
hipError_t literal(const float* coef, const float* lut_x, const float* lut_y,
                   const LitTables& tb, int ny, int nx, int layers, int L, int split,
                   float2* partial, float2* hologram, int accumulate,
                   const unsigned long long* absmax, int e_fringe, char* base, hipStream_t s) {
    const unsigned long long* am = P == P_FP16 ? absmax : nullptr;
    const LitShape z = lit_shape(ny, nx, layers, L);
    const LitRegions r = lit_regions(base, ny, nx, layers, L);
    // level-0 (point) tables of every layer; y tables carry the per-layer prefactor
    float* l0x = reinterpret_cast<float*>(r.lut0);
    float* l0y = l0x + (size_t)layers * 2 * lut_len(nx);
    hipError_t e = launch_luts(nx, layers, 1, 0, tb.c, tb.one_re, tb.one_im, l0x, s);
    if (e == hipSuccess)
        e = launch_luts(ny, layers, 1, 0, tb.c, tb.pre_re, tb.pre_im, l0y, s);
    if (e != hipSuccess) return e;
    const int es = P == P_FP32 ? 4 : 2;
    size_t rb_off = 0, fx_off = 0, seg = 0;
    const int lenx = lut_len(nx), leny = lut_len(ny);
    for (int d = 0; d < layers; ++d) {
        for (int b = L; b >= 0; --b) {
            const int rows = ny >> b, kc = pad_kt(nx >> b);
            hipLaunchKernelGGL(residual_panel_kernel<P>, dim3(grid_1d((size_t)rows * kc)),
                               dim3(256), 0, s, coef + (size_t)d * ny * nx, ny, nx, L, b, am,
                               r.rb + rb_off * es, (size_t)z.rb_ps);
            const float* tx = b == 0 ? l0x + (size_t)d * 2 * lenx
                                     : lut_x + lut_table(d, b, 0, 0, L) * lenx;
            const float* ty = b == 0 ? l0y + (size_t)d * 2 * leny
                                     : lut_y + lut_table(d, b, 0, 0, L) * leny;
            hipLaunchKernelGGL(block_fringe_panel_kernel<P>, dim3(grid_1d((size_t)nx * kc)),
                               dim3(256), 0, s, tx, nx, b, fx_off, r.fxb, (size_t)z.fxb_ps);
            // the y panel's K segment of this term starts on a K-block boundary
            hipLaunchKernelGGL(block_fringe_panel_kernel<P>,
                               dim3(grid_1d((size_t)ny * pad_kt(rows))), dim3(256), 0, s, ty, ny,
                               b, seg * ny, r.fy, (size_t)ny * z.kt);
            rb_off += (size_t)rows * kc;
            fx_off += (size_t)nx * kc;
            seg += pad_kt(rows);
        }
    }
    LitArgs a{};
    a.ny = ny;
    a.nx = nx;
    a.layers = layers;
    a.L = L;
    a.es = es;
    a.split = split;
    a.tn2 = nt_table_tile_n(kEpiComplex, P);
    a.rb = r.rb;
    a.fxb = r.fxb;
    a.t = r.t;
    a.fy = r.fy;
    a.hologram = hologram;
    a.partial = split > 1 ? partial : nullptr;
    a.rb_ps = (long long)z.rb_ps;
    a.fxb_ps = (long long)z.fxb_ps;
    a.t_ps = (long long)nx * z.kt;
    a.fy_ps = (long long)ny * z.kt;
    a.accumulate = accumulate;
    a.first = r.entries;
    a.second = r.entries + (size_t)layers * (L + 1);
    a.counts = r.counts;
    a.absmax = am;
    a.t_shift = am ? headroom_shift(48.f * (float)nx) : 0;
    a.e_fringe = e_fringe;
    hipLaunchKernelGGL(literal_entries_kernel, dim3(1), dim3(64), 0, s, a);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    e = launch_nt_first_table(P, a.first, layers * (L + 1), a.counts, z.first_tiles, s);
    if (e != hipSuccess) return e;
    e = launch_nt_table(kEpiComplex, P, a.second, 1, a.counts + 1,
                        nt_tiles(ny, nx, kNtTile, a.tn2), split, s);
    if (e != hipSuccess) return e;
    return launch_reduce_partial(ny, nx, split, partial, hologram, accumulate, s);
}

}  // namespace

size_t literal_bytes(int ny, int nx, int layers, int levels) {
    return lit_regions(nullptr, ny, nx, layers, levels).total;
}

hipError_t launch_literal(const float* coef, const float* lut_x, const float* lut_y,
                          const LitTables& tb, int ny, int nx, int layers, int levels,
                          int precision, int split, float2* partial, float2* hologram,
                          int accumulate, const unsigned long long* absmax, int e_fringe,
                          void* region, hipStream_t s) {
    char* base = static_cast<char*>(region);
    if (precision == P_BF16)
        return literal<P_BF16>(coef, lut_x, lut_y, tb, ny, nx, layers, levels, split, partial,
                               hologram, accumulate, absmax, e_fringe, base, s);
    if (precision == P_FP16)
        return literal<P_FP16>(coef, lut_x, lut_y, tb, ny, nx, layers, levels, split, partial,
                               hologram, accumulate, absmax, e_fringe, base, s);
    return literal<P_FP32>(coef, lut_x, lut_y, tb, ny, nx, layers, levels, split, partial,
                           hologram, accumulate, absmax, e_fringe, base, s);
}

}  // namespace cgh
