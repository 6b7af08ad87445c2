// Adjoint of the progressive hologram with respect to the masked coefficients,
// as two batched NT contractions on the MFMA kernel of the forward pass.
//
// The forward pass adds H_{d,l} = Fy_{d,l} Cb_{d,l} Fx_{d,l}^T per layer d and
// level l (Eq. 3 with the separable Fresnel kernel).  For a real loss with
// cotangent G = dL/dRe H + i dL/dIm H the coefficient gradient is
//     gC_{d,l} = Re( Fy_{d,l}^H  G  conj(Fx_{d,l}) ),
// computed as
//     step A:  P_{d,l}[c][y]  = sum_x conj(Fx_{d,l}[x][c]) * G[y][x]
//              (A = FxH panel [c][x], B = G panel [y][x]; stored as operand planes)
//     step B:  gC_{d,l}[r][c] = Re sum_y conj(Fy_{d,l}[y][r]) * P_{d,l}[c][y]
//              (A = FyH panel [r][y], B = P panel [c][y]; real part only)
// Step B covers the level's Mallat square except its LL quadrant below the
// coarsest level (that quadrant belongs to the next level): two sub-blocks
// per level there, the whole square at the coarsest level.  The masks, the
// 4^-l weights, the synthesis and the gather by layer follow in
// grad_synthesis_kernel (dwt.hip).
#include "nt.h"
#include "split.h"

namespace cgh {

namespace {

inline int grid_1d(size_t n) {
    const size_t b = (n + 255) / 256;
    return (int)(b < 4096 ? (b > 0 ? b : 1) : 4096);
}

// Conjugated block-fringe panel of every (layer, level) of one axis:
//   out_{d,l}[j][pix] = conj(F_{d,l}[pix][j]) = conj(g_{band(j)}[pix - (j mod n_l) 2^l])
// rows j of the level square (s_l = n >> (l-1)), K = pix < ld (zero past n), K-blocked.
template <int P>
__global__ __launch_bounds__(256) void fringe_h_kernel(const float* __restrict__ lut, int n,
                                                       int levels, int ld, void* __restrict__ out,
                                                       size_t ps) {
    const int dl = blockIdx.y;
    const int d = dl / levels, l = dl % levels + 1;
    const int s = band_side(n, l), nl = n >> l, len = lut_len(n);
    size_t per = 0, off = 0;
    for (int k = 1; k <= levels; ++k) {
        if (k < l) off += (size_t)band_side(n, k) * ld;
        per += (size_t)band_side(n, k) * ld;
    }
    const size_t base = (size_t)d * per + off;
    const size_t total = (size_t)s * ld;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (size_t)gridDim.x * blockDim.x) {
        int j, pix;
        kblk_pos(e, s, j, pix);
        float re = 0.f, im = 0.f;
        if (pix < n) {
            const int band = j >= nl, jj = j - band * nl;
            const float* tb = lut + lut_table(d, l, band, 0, levels) * len;
            const int idx = pix - (jj << l) + n;
            re = tb[idx];
            im = -tb[len + idx];
        }
        put_c<P>(out, ps, base + e, re, im);
    }
}

// Interleaved complex64 [rows][cols] -> operand planes [rows][ld], zero pad.
// absmax (FP16 range scaling, else null): values scaled by 2^-e, e the exponent of
// the cotangent's largest component magnitude.
template <int P>
__global__ __launch_bounds__(256) void cotangent_panel_kernel(const float2* __restrict__ in,
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

struct BwArgs {
    int ny, nx, layers, levels, ldx, ldy, es, split_a, split_b, tn_a;
    int tiles_a_layer, tiles_b_layer;
    const char* g;            // G panel
    const char* fxh;          // FxH panels
    const char* fyh;          // FyH panels
    char* pt;                 // P panels
    float* gcoef;             // per-layer coefficient gradient planes
    char* partial;            // split-K partials (shared by both steps)
    long long g_ps, fxh_ps, fyh_ps, pt_ps;
    NtEntry* ea;              // step A problems [layers * levels]
    NtEntry* eb;              // step B problems [layers * (2 * levels - 1)]
    int* counts;              // tile totals of step A and step B
    // FP16 range scaling: G scaled by 2^-e (e from the cotangent's max-abs word),
    // P = conj(Fx) G (|P| < 2 sqrt 2 x 8 nx) stored times 2^-t, and step B's epilogue
    // multiplies by 2^(e + t + e_fringe); scale 1 otherwise
    const unsigned long long* absmax;  // null unless FP16
    int t_shift, e_fringe;
};

// One thread per layer writes that layer's problems; every layer has the same
// shapes, so tile offsets are closed-form.
__global__ void bw_entries_kernel(BwArgs a) {
    const int d = blockIdx.x * blockDim.x + threadIdx.x;
    const float a_scale = a.absmax ? pow2f(-a.t_shift) : 1.f;
    const float b_scale =
        a.absmax ? pow2f(range_exp(absmax_value(a.absmax)) + a.t_shift + a.e_fringe) : 1.f;
    if (d == 0) {
        a.counts[0] = a.layers * a.tiles_a_layer;
        a.counts[1] = a.layers * a.tiles_b_layer;
    }
    if (d >= a.layers) return;
    const int L = a.levels;
    size_t rows_x = 0, rows_y = 0;  // level-square rows per layer (x and y axes)
    for (int k = 1; k <= L; ++k) {
        rows_x += band_side(a.nx, k);
        rows_y += band_side(a.ny, k);
    }
    // partial offsets (elements of float2 for step A, floats for step B) per layer
    size_t pa_layer = 0, pb_layer = 0;
    for (int k = 1; k <= L; ++k) {
        const size_t sy = band_side(a.ny, k), sx = band_side(a.nx, k);
        pa_layer += sx * a.ny;
        pb_layer += (k < L) ? (sy * sx - (sy / 2) * (sx / 2)) : sy * sx;
    }
    size_t ox = 0, oy = 0, pa = 0, pb = 0;
    int ta = 0, tb = 0, nb = 0;
    for (int l = 1; l <= L; ++l) {
        const int sy = band_side(a.ny, l), sx = band_side(a.nx, l);
        const size_t fx_off = (size_t)d * rows_x * a.ldx + ox * a.ldx;
        const size_t pt_off = (size_t)d * rows_x * a.ldy + ox * a.ldy;
        const size_t fy_off = (size_t)d * rows_y * a.ldy + oy * a.ldy;
        NtEntry e{};
        e.a = a.fxh + fx_off * a.es;
        e.b = a.g;
        e.out = a.pt + pt_off * a.es;
        e.partial = reinterpret_cast<float2*>(a.partial) +
                    (size_t)a.split_a * ((size_t)d * pa_layer + pa);
        e.a_ps = a.fxh_ps;
        e.b_ps = a.g_ps;
        e.out_ps = a.pt_ps;
        e.M = sx;
        e.N = a.ny;
        e.K = a.ldx;
        e.lda = sx * 16;     // FxH_{d,l}: sx rows
        e.ldb = a.ny * 16;   // G: ny rows
        e.out_ld = sx * 16;  // P_{d,l}: sx rows
        e.tiles_n = (a.ny + a.tn_a - 1) / a.tn_a;
        e.tile_begin = d * a.tiles_a_layer + ta;
        e.tile_m = kNtTile;
        e.tile_n = a.tn_a;
        e.out_scale = a_scale;
        a.ea[d * L + l - 1] = e;
        ta += nt_tiles(sx, a.ny, kNtTile, a.tn_a);
        pa += (size_t)sx * a.ny;

        // step B sub-blocks: (r0, M, c0, N)
        int blk[2][4];
        int nblk = 0;
        if (l < L) {
            blk[0][0] = 0; blk[0][1] = sy / 2; blk[0][2] = sx / 2; blk[0][3] = sx / 2;
            blk[1][0] = sy / 2; blk[1][1] = sy / 2; blk[1][2] = 0; blk[1][3] = sx;
            nblk = 2;
        } else {
            blk[0][0] = 0; blk[0][1] = sy; blk[0][2] = 0; blk[0][3] = sx;
            nblk = 1;
        }
        for (int b = 0; b < nblk; ++b) {
            const int r0 = blk[b][0], M = blk[b][1], c0 = blk[b][2], N = blk[b][3];
            NtEntry f{};
            f.a = a.fyh + (fy_off + (size_t)r0 * 16) * a.es;  // row r0 of FyH_{d,l}
            f.b = a.pt + (pt_off + (size_t)c0 * 16) * a.es;   // row c0 of P_{d,l}
            f.out = a.gcoef + (size_t)d * a.ny * a.nx + (size_t)r0 * a.nx + c0;
            f.partial = reinterpret_cast<float2*>(
                reinterpret_cast<float*>(a.partial) +
                (size_t)a.split_b * ((size_t)d * pb_layer + pb));
            f.a_ps = a.fyh_ps;
            f.b_ps = a.pt_ps;
            f.M = M;
            f.N = N;
            f.K = a.ldy;
            f.lda = sy * 16;
            f.ldb = sx * 16;
            f.out_ld = a.nx;
            f.tiles_n = (N + kNtTile - 1) / kNtTile;
            f.tile_begin = d * a.tiles_b_layer + tb;
            f.tile_m = f.tile_n = kNtTile;
            f.out_scale = b_scale;
            a.eb[(size_t)d * (2 * L - 1) + nb] = f;
            ++nb;
            tb += nt_tiles(M, N, kNtTile, kNtTile);
            pb += (size_t)M * N;
        }
        ox += sx;
        oy += sy;
    }
}

// Split-K sums of step A into the operand planes of the P panels.
template <int P>
__global__ __launch_bounds__(256) void reduce_panel_entries_kernel(const NtEntry* __restrict__ en,
                                                                   int split) {
    const NtEntry e = en[blockIdx.y];
    const int ldp = pad_kt(e.N);
    const size_t total = (size_t)e.M * ldp, mn = (size_t)e.M * e.N;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (size_t)gridDim.x * blockDim.x) {
        int r, c;
        kblk_pos(i, e.M, r, c);
        float re = 0.f, im = 0.f;
        if (c < e.N) {
            for (int s = 0; s < split; ++s) {
                const float2 v = e.partial[(size_t)s * mn + (size_t)r * e.N + c];
                re += v.x;
                im += v.y;
            }
        }
        put_c<P>(e.out, (size_t)e.out_ps, i, re, im);  // e.out_ld == M * 16
    }
}

// Split-K sums of step B into the coefficient gradient.
__global__ __launch_bounds__(256) void reduce_real_entries_kernel(const NtEntry* __restrict__ en,
                                                                  int split) {
    const NtEntry e = en[blockIdx.y];
    const size_t mn = (size_t)e.M * e.N;
    const float* part = reinterpret_cast<const float*>(e.partial);
    float* out = static_cast<float*>(e.out);
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < mn;
         i += (size_t)gridDim.x * blockDim.x) {
        const int r = (int)(i / e.N), c = (int)(i - (size_t)r * e.N);
        float v = 0.f;
        for (int s = 0; s < split; ++s) v += part[(size_t)s * mn + i];
        out[(size_t)r * e.out_ld + c] = v;
    }
}

int pick_split(int tiles, int k) {
    int split = (512 + tiles - 1) / tiles;
    if (split > (k / kKT) / 4) split = (k / kKT) / 4;
    if (split > 16) split = 16;
    return split < 1 ? 1 : split;
}

struct BwShape {
    int ldx, ldy, split_a, split_b, tiles_a_layer, tiles_b_layer;
    size_t rows_x, rows_y, pa_layer, pb_layer;
    size_t g_b, fxh_b, fyh_b, pt_b, part_b, ent_b;  // bytes
};

// tn_a: column tile of step A (the workspace is sized with 128, whose split is
// the largest).
BwShape bw_shape(int ny, int nx, int layers, int levels, int tn_a = kNtTile) {
    BwShape z{};
    z.ldx = pad_kt(nx);
    z.ldy = pad_kt(ny);
    for (int l = 1; l <= levels; ++l) {
        const int sy = band_side(ny, l), sx = band_side(nx, l);
        z.rows_x += sx;
        z.rows_y += sy;
        z.tiles_a_layer += nt_tiles(sx, ny, kNtTile, tn_a);
        z.pa_layer += (size_t)sx * ny;
        if (l < levels) {
            z.tiles_b_layer += nt_tiles(sy / 2, sx / 2, kNtTile, kNtTile) +
                               nt_tiles(sy / 2, sx, kNtTile, kNtTile);
            z.pb_layer += (size_t)sy * sx - (size_t)(sy / 2) * (sx / 2);
        } else {
            z.tiles_b_layer += nt_tiles(sy, sx, kNtTile, kNtTile);
            z.pb_layer += (size_t)sy * sx;
        }
    }
    z.split_a = pick_split(layers * z.tiles_a_layer, z.ldx);
    z.split_b = pick_split(layers * z.tiles_b_layer, z.ldy);
    auto al = [](size_t v) { return (v + 255) / 256 * 256; };
    z.g_b = al(8 * (size_t)ny * z.ldx);
    z.fxh_b = al(8 * (size_t)layers * z.rows_x * z.ldx);
    z.fyh_b = al(8 * (size_t)layers * z.rows_y * z.ldy);
    z.pt_b = al(8 * (size_t)layers * z.rows_x * z.ldy);
    const size_t pa = z.split_a > 1 ? 8 * (size_t)z.split_a * layers * z.pa_layer : 0;
    const size_t pb = z.split_b > 1 ? 4 * (size_t)z.split_b * layers * z.pb_layer : 0;
    z.part_b = al(pa > pb ? pa : pb);
    z.ent_b = al(sizeof(NtEntry) * (size_t)layers * (3 * levels - 1) + 2 * sizeof(int));
    return z;
}

template <int P>
hipError_t backward_nt(const float2* grad_h, const float* lut_x, const float* lut_y, int ny,
                       int nx, int layers, int levels, float* gcoef, char* base,
                       unsigned long long* absmax, int e_fringe, hipStream_t s) {
    constexpr bool F16 = P == P_FP16;
    const int tn_a = nt_table_tile_n(kEpiPanel, P);
    const BwShape z = bw_shape(ny, nx, layers, levels, tn_a);
    BwArgs a{};
    a.tn_a = tn_a;
    a.ny = ny;
    a.nx = nx;
    a.layers = layers;
    a.levels = levels;
    a.ldx = z.ldx;
    a.ldy = z.ldy;
    a.es = P == P_FP32 ? 4 : 2;
    a.split_a = z.split_a;
    a.split_b = z.split_b;
    a.tiles_a_layer = z.tiles_a_layer;
    a.tiles_b_layer = z.tiles_b_layer;
    size_t off = 0;
    char* g = base + off;
    off += z.g_b;
    char* fxh = base + off;
    off += z.fxh_b;
    char* fyh = base + off;
    off += z.fyh_b;
    a.pt = base + off;
    off += z.pt_b;
    a.partial = base + off;
    off += z.part_b;
    a.ea = reinterpret_cast<NtEntry*>(base + off);
    a.eb = a.ea + (size_t)layers * levels;
    a.counts = reinterpret_cast<int*>(a.eb + (size_t)layers * (2 * levels - 1));
    a.g = g;
    a.fxh = fxh;
    a.fyh = fyh;
    a.gcoef = gcoef;
    a.g_ps = (long long)ny * z.ldx;
    a.fxh_ps = (long long)layers * z.rows_x * z.ldx;
    a.fyh_ps = (long long)layers * z.rows_y * z.ldy;
    a.pt_ps = (long long)layers * z.rows_x * z.ldy;
    a.absmax = F16 ? absmax : nullptr;
    a.t_shift = F16 ? headroom_shift(32.f * (float)nx) : 0;
    a.e_fringe = e_fringe;
    const int n_dl = layers * levels;

    if (F16) {
        hipError_t r = launch_absmax(reinterpret_cast<const float*>(grad_h), 2 * (size_t)ny * nx,
                                     absmax, s);
        if (r != hipSuccess) return r;
    }
    hipLaunchKernelGGL(cotangent_panel_kernel<P>, dim3(grid_1d((size_t)a.g_ps)), dim3(256), 0, s,
                       grad_h, ny, nx, z.ldx, a.absmax, g, (size_t)a.g_ps);
    hipLaunchKernelGGL(fringe_h_kernel<P>, dim3(grid_1d((size_t)nx * z.ldx), n_dl), dim3(256), 0,
                       s, lut_x, nx, levels, z.ldx, fxh, (size_t)a.fxh_ps);
    hipLaunchKernelGGL(fringe_h_kernel<P>, dim3(grid_1d((size_t)ny * z.ldy), n_dl), dim3(256), 0,
                       s, lut_y, ny, levels, z.ldy, fyh, (size_t)a.fyh_ps);
    hipLaunchKernelGGL(bw_entries_kernel, dim3((layers + 63) / 64), dim3(64), 0, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;

    e = launch_nt_table(kEpiPanel, P, a.ea, n_dl, a.counts, layers * z.tiles_a_layer, z.split_a, s);
    if (e != hipSuccess) return e;
    if (z.split_a > 1) {
        hipLaunchKernelGGL(reduce_panel_entries_kernel<P>,
                           dim3(grid_1d((size_t)band_side(nx, 1) * pad_kt(ny)), n_dl), dim3(256),
                           0, s, a.ea, z.split_a);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    const int n_b = layers * (2 * levels - 1);
    e = launch_nt_table(kEpiReal, P, a.eb, n_b, a.counts + 1, layers * z.tiles_b_layer, z.split_b,
                        s);
    if (e != hipSuccess) return e;
    if (z.split_b > 1) {
        hipLaunchKernelGGL(reduce_real_entries_kernel,
                           dim3(grid_1d((size_t)band_side(ny, 1) * band_side(nx, 1) / 2), n_b),
                           dim3(256), 0, s, a.eb, z.split_b);
        e = hipGetLastError();
    }
    return e;
}

}  // namespace

size_t backward_bytes(int ny, int nx, int layers, int levels) {
    const BwShape z = bw_shape(ny, nx, layers, levels);
    return z.g_b + z.fxh_b + z.fyh_b + z.pt_b + z.part_b + z.ent_b;
}

hipError_t launch_backward_nt(const float2* grad_h, const float* lut_x, const float* lut_y, int ny,
                              int nx, int layers, int levels, int precision, float* gcoef,
                              void* region, unsigned long long* absmax, int e_fringe,
                              hipStream_t s) {
    char* base = static_cast<char*>(region);
    if (precision == P_BF16)
        return backward_nt<P_BF16>(grad_h, lut_x, lut_y, ny, nx, layers, levels, gcoef, base,
                                   absmax, e_fringe, s);
    if (precision == P_FP16)
        return backward_nt<P_FP16>(grad_h, lut_x, lut_y, ny, nx, layers, levels, gcoef, base,
                                   absmax, e_fringe, s);
    return backward_nt<P_FP32>(grad_h, lut_x, lut_y, ny, nx, layers, levels, gcoef, base, absmax,
                               e_fringe, s);
}

}  // namespace cgh
