// Compacted "NT" formulation of the forward contractions (internal).
//
// Only coefficient rows / columns that hold a nonzero masked coefficient take
// part (the layer split and the saliency masks leave most of them empty):
//   first:   T_c[x][k'] = sum_c' Cb_c[r'][c'] * Fx_c[x][c']     per (layer, level)
//   second:  H[y][x]    = sum_k' Fy_c[y][k'] * T_c[x][k']
// r' / c' index the active rows / columns of a level's coefficient square; k'
// runs over the active rows of every (layer, level) in order, each segment
// padded with zero rows to a multiple of kKT.  Every operand panel is stored
// K-blocked: element (row r, k) of a panel of R rows sits at
//     (k / 16) * (R * 16) + r * 16 + k % 16
// so the 16-wide K slice of a tile of rows is one contiguous run (whole cache
// lines per load), in the operand precision: FP32 planes (re[, im]) or 16-bit
// split planes (re_hi, re_lo[, im_hi, im_lo]).
#pragma once

#include "common.h"

namespace cgh {

constexpr int kKT = 16;       // K tile; every K extent is a multiple of it
constexpr int kNtTile = 128;  // output tile rows and columns

__host__ __device__ inline int pad_kt(int v) { return (v + kKT - 1) / kKT * kKT; }

// Element (row r, k) of a K-blocked panel whose K-block stride is blk (rows x 16).
__host__ __device__ inline size_t kblk_off(int r, int k, size_t blk) {
    return (size_t)(k >> 4) * blk + (size_t)r * 16 + (k & 15);
}
// Inverse for writers that walk a panel of `rows` rows in storage order.  One
// panel holds at most 16384 x 16384 elements, so 32-bit arithmetic is exact.
__host__ __device__ inline void kblk_pos(size_t e, int rows, int& r, int& k) {
    const unsigned u = (unsigned)e, blk = (unsigned)rows * 16u;
    const unsigned b = u / blk, rem = u - b * blk;
    r = (int)(rem >> 4);
    k = (int)(b * 16u + (rem & 15u));
}

// One GEMM problem of the batched NT kernel (self-contained, so problems of
// different scenes can share one launch).
struct NtEntry {
    const void* a;          // A panel: plane 0, row 0, k 0
    const void* b;          // B panel: plane 0, row 0, k 0
    void* out;              // first: T_c plane 0 at this problem's k' segment; second: hologram
    float2* partial;        // second: split-K partial holograms (single-scene calls), else null
    long long a_ps, b_ps;   // plane strides of A and B (elements)
    long long out_ps;       // panel outputs: plane stride (elements)
    int M, N, K;            // output rows, output columns (complex), reduction length
    int lda, ldb;           // K-block strides of the A and B panels (rows x 16 elements)
    int out_ld;             // complex / real outputs: row stride; panel outputs
                            // (T_c, P): K-block stride (rows x 16 elements)
    int tiles_n;            // column tiles
    int tile_begin;         // exclusive prefix of tiles over the table
    int accumulate;         // second: hologram += result
    int tile_m, tile_n;     // tile shape the table was planned for
    float out_scale;        // the epilogue multiplies the FP32 products by it (a power of
                            // two undoing FP16 range scaling, else 1)
    // First contraction: where its B operand (the fringes of the active rows or columns
    // it sums over) comes from for kernels that generate it instead of reading the
    // panel at b.  g_lut: the (layer, level)'s operand-format tables (gen_table), and
    // element (n, k') is their entry n + N + g_koff[k'] (g_koff holds 3N, the zero band,
    // from g_count to the next multiple of 16); rows n >= N are zero.
    const void* g_lut;
    const int* g_koff;
    int g_count;
};

// Device-side plan written by the planning kernels (lives in the workspace).
struct PlanHeader {
    int kpad;          // K of the second contraction (sum of padded segment lengths)
    int first_tiles;   // tiles of the first contraction
    int k_active;      // active K of the second contraction: per (layer, level) its
                       // active rows, or its active columns where those go first
    int second_tiles;  // output tiles of the second contraction
    float cb_scale;    // scale of the coefficient panel (FP16 range scaling, else 1)
    int panel_units;   // work units of the operand-panel gather
};

// Element counts (dense upper bounds) of the compacted regions.
struct NtSizes {
    size_t rowlist, collist;  // ints
    size_t fx_plane;          // elements per plane of Fx_c
    size_t cb_plane;          // elements per plane of Cb_c
    size_t kmax;              // upper bound of kpad
    size_t fy_plane, tc_plane;
    int first_tiles_max;  // upper bound over every tile shape
};

// Each (layer, level) square is contracted rows-first (T = Cb Fx^T: K' = its padded
// active rows) or columns-first (T' = Cb^T Fy^T: K' = its padded active columns),
// whichever gives the second contraction the shorter K' segment.  The per-(layer,
// level) regions of the first contraction's operands are sized for either order:
// its fringe operand holds nx x pad(columns) or ny x pad(rows) elements, its
// coefficient operand rows x pad(columns) or columns x pad(rows).
__host__ __device__ inline size_t dl_first_fringe_elems(int ny, int nx, int l) {
    const size_t r = (size_t)nx * pad_kt(band_side(nx, l)), c = (size_t)ny * pad_kt(band_side(ny, l));
    return r > c ? r : c;
}
__host__ __device__ inline size_t dl_coef_elems(int ny, int nx, int l) {
    const int syl = band_side(ny, l), sxl = band_side(nx, l);
    const size_t r = (size_t)syl * pad_kt(sxl), c = (size_t)sxl * pad_kt(syl);
    return r > c ? r : c;
}
// The order of one (layer, level): columns-first iff its padded column count is
// the smaller (K' never exceeds the rows-first bound kmax).
__host__ __device__ inline bool columns_first(int rows, int cols) {
    return pad_kt(cols) < pad_kt(rows);
}

// Work units of the operand-panel gather of one (layer, level) with `rows` active
// rows and `cols` active columns: [0] tasks of the second contraction's fringe
// operand, [1] of the first contraction's (a task is kFringeRows rows x one
// 16-wide K block), [2] units of kCbUnit coefficient-operand elements.
constexpr int kFringeRows = 256;
constexpr int kCbUnit = 1024;  // 256 threads x 4 elements
__host__ __device__ inline void dl_panel_units(int ny, int nx, int rows, int cols, int u[3]) {
    u[0] = u[1] = u[2] = 0;
    if (rows == 0 || cols == 0) return;
    const bool cf = columns_first(rows, cols);
    const int n2 = cf ? nx : ny, k2 = cf ? cols : rows;  // the K' side
    const int n1 = cf ? ny : nx, k1 = cf ? rows : cols;  // the first contraction's K side
    u[0] = (n2 + kFringeRows - 1) / kFringeRows * (pad_kt(k2) / kKT);
    u[1] = (n1 + kFringeRows - 1) / kFringeRows * (pad_kt(k1) / kKT);
    u[2] = (int)(((long long)k2 * pad_kt(k1) + kCbUnit - 1) / kCbUnit);
}

// Upper bound of a scene's panel work units (every row and column active).
inline long long panel_units_bound(int ny, int nx, int layers, int levels) {
    long long t = 0;
    for (int l = 1; l <= levels; ++l) {
        int u[3];
        dl_panel_units(ny, nx, band_side(ny, l), band_side(nx, l), u);
        t += (long long)u[0] + u[1] + u[2];
    }
    return t * layers;
}

inline NtSizes nt_sizes(int ny, int nx, int layers, int levels) {
    NtSizes z{};
    size_t sy = 0, sx = 0, fx = 0, cb = 0, kmax = 0;
    int tiles = 0;
    for (int l = 1; l <= levels; ++l) {
        const int syl = band_side(ny, l), sxl = band_side(nx, l);
        sy += syl;
        sx += sxl;
        fx += dl_first_fringe_elems(ny, nx, l);
        cb += dl_coef_elems(ny, nx, l);
        kmax += pad_kt(syl);
        // bound for the smallest tile shape, in either order
        const int tr = ((syl + 63) / 64) * ((nx + 63) / 64);
        const int tc = ((sxl + 63) / 64) * ((ny + 63) / 64);
        tiles += tr > tc ? tr : tc;
    }
    z.rowlist = sy * layers;
    z.collist = sx * layers;
    z.fx_plane = fx * layers;
    z.cb_plane = cb * layers;
    z.kmax = kmax * layers;
    z.fy_plane = (size_t)ny * z.kmax;
    z.tc_plane = (size_t)nx * z.kmax;
    z.first_tiles_max = tiles * layers;
    return z;
}

// Dense offsets of (layer d, level l) inside the per-(d, l) regions.
// Offsets of (layer d, level l) in the per-axis table-offset arrays (koff_row over ny,
// koff_col over nx): one segment per (layer, level), the level's side padded to 16, so
// that a K tile's 16 offsets are one aligned run.
__host__ __device__ inline size_t dl_koff_off(int n, int levels, int d, int l) {
    size_t per = 0, at = 0;
    for (int k = 1; k <= levels; ++k) {
        if (k == l) at = per;
        per += (size_t)pad_kt(band_side(n, k));
    }
    return (size_t)d * per + at;
}
__host__ __device__ inline size_t dl_rows_off(int ny, int levels, int d, int l) {
    size_t per = 0;
    for (int k = 1; k <= levels; ++k) per += band_side(ny, k);
    return (size_t)d * per + t_level_rows(ny, l);
}
__host__ __device__ inline size_t dl_cols_off(int nx, int levels, int d, int l) {
    size_t per = 0, off = 0;
    for (int k = 1; k <= levels; ++k) {
        if (k < l) off += band_side(nx, k);
        per += band_side(nx, k);
    }
    return (size_t)d * per + off;
}
__host__ __device__ inline size_t dl_fx_off(int ny, int nx, int levels, int d, int l) {
    size_t per = 0, off = 0;
    for (int k = 1; k <= levels; ++k) {
        const size_t v = dl_first_fringe_elems(ny, nx, k);
        if (k < l) off += v;
        per += v;
    }
    return (size_t)d * per + off;
}
__host__ __device__ inline size_t dl_cb_off(int ny, int nx, int levels, int d, int l) {
    size_t per = 0, off = 0;
    for (int k = 1; k <= levels; ++k) {
        const size_t v = dl_coef_elems(ny, nx, k);
        if (k < l) off += v;
        per += v;
    }
    return (size_t)d * per + off;
}

struct NtBuffers {
    // lists and plan
    int* rowlist;
    int* collist;
    int* cnt_row;   // [D*L]
    int* cnt_col;   // [D*L]
    int* seg_row;   // [D*L] k' offset of the (layer, level) segment
    int* orient;    // [D*L] 1: contracted columns-first (set by the planning kernel)
    int* units;     // [3*D*L+1] start of the panel work units of kind k of (layer,
                    // level) t at entry k D L + t, then the total (planning kernel;
                    // the batched panel gather numbers its work by it)
    int* tbeg;      // [D*L] tile prefix (first contraction, local to the scene)
    const uint8_t* occ;  // (layer, block) occupancy of the coefficient planes
    PlanHeader* hdr;
    NtEntry* first;   // [D*L] first-contraction problems of this scene
    NtEntry* second;  // [1] second-contraction problem of this scene
    // panels (element type by precision), plane strides in elements
    void* fx; void* cb; void* fy; void* tc;
    size_t fx_ps, cb_ps, fy_ps, tc_ps;
    // the scene's level fringe tables (x, y) in the operand format (gen_table), and
    // beside the lists each active row's / column's offset into them (gen_koff)
    const void* gen_x;
    const void* gen_y;
    int* koff_row;
    int* koff_col;
};

// Output of the second contraction of one scene.
struct NtOutput {
    float2* hologram;
    float2* partial;   // split-K partials or null
    int accumulate;
};

// Arguments of the planning kernel of one scene (device-side tables).
struct PlanArgs {
    int ny, nx, layers, levels, esize;
    int fp16;                            // FP16 split operands: range scaling
    int e_fringe;                        // exponent the y fringe tables were scaled by (2^-e)
    const unsigned long long* absmax;    // max |object| of the scene (max-abs word)
    int tm1, tn1, tm2, tn2;  // tile shapes of the first and second contraction
    const int* cnt_row;
    const int* cnt_col;
    int* seg_row;
    int* orient;
    int* units;
    int* tbeg;
    PlanHeader* hdr;
    NtEntry* first;
    NtEntry* second;
    const void* cb;
    const void* fx;
    void* fy;
    void* tc;
    long long cb_ps, fx_ps, fy_ps, tc_ps;
    const int* koff_row;
    const int* koff_col;
    const void* gen_x;
    const void* gen_y;
    float2* hologram;
    float2* partial;
    int accumulate;
};

// tiles: {rows, cols} of the first contraction's tile, then of the second's.
PlanArgs make_plan_args(int ny, int nx, int layers, int levels, int precision, const int* tiles,
                        const NtBuffers& b, const NtOutput& o,
                        const unsigned long long* absmax = nullptr, int e_fringe = 0);

// One scene of a batched preparation: its flags, coefficients, tables and buffers.
struct PrepScene {
    const uint8_t* flags;
    const float* coef;
    const float* lut_x;
    const float* lut_y;
    int ny, nx, layers;
    size_t flags_layer;
    NtBuffers b;
};
// Batched launches over device tables of n scenes (grid sized for the largest).
hipError_t launch_lists_batch(const PrepScene* scenes, int n, int levels, int max_ndl,
                              hipStream_t s);
// max_ndl: the largest (layer, level) count of the scenes (sizes the workgroup).
hipError_t launch_plan_batch(const PlanArgs* args, int n, int max_ndl, hipStream_t s);
// scene_units: as written by launch_batch_prefix; units_bound: an estimate of the
// batch's panel work units (sizes the grid).
hipError_t launch_materialize_batch(const PrepScene* scenes, int n, int levels, int precision,
                                    const int* scene_units, long long units_bound,
                                    hipStream_t s);

// tiles: {rows, cols} of the first contraction's tile, then of the second's.
hipError_t launch_nt_plan(const uint8_t* flags, int ny, int nx, int layers, int levels,
                          size_t flags_layer, int precision, const int* tiles,
                          const NtBuffers& b, const NtOutput& o,
                          const unsigned long long* absmax, int e_fringe, hipStream_t s);
// first_panel: also gather the first contraction's fringe operand (when the first
// contraction does not generate it, see nt_first_generates).
hipError_t launch_nt_materialize(const float* coef, const float* lut_x, const float* lut_y, int ny,
                                 int nx, int layers, int levels, int precision,
                                 const NtBuffers& b, bool first_panel, hipStream_t s);
// Direct launches over one scene's table (split-K for the second).
// Row tile of the single-scene first contraction: 64 for FP32 (measured 10%
// faster there: the active row counts of a level are often far below 128), 128
// for the split forms.  Tile of the second: 128 x 64 for FP32 (the
// three-product complex form, two workgroups per CU), 256 x 128 for the split
// forms (one workgroup per CU, two LDS stages).
int nt_first_tile_m(int precision);
// Columns of the first contraction's tile for a single scene: 64 on scenes small enough
// that 128-column tiles would leave most compute units idle, else 128.
int nt_first_tile_n(int ny, int nx, int layers, int levels, int precision);
// Tiles of the first contraction at tm x tn tiles with every row and column active, in
// the order with more of them per (layer, level): a bound of the planned tile count.
long long nt_first_tiles_bound(int ny, int nx, int layers, int levels, int tm, int tn);
// Whether the first contraction (single-scene or batched) with tile_n-column tiles
// generates its fringe operand from the operand-format tables (else the panel gather
// writes it).
constexpr bool nt_first_generates(int tile_n) { return tile_n == 128; }
int nt_second_tile_m(int precision);
int nt_second_tile_n(int precision);
// The split forms' ring kernel over a table of second contractions (a batch of
// scenes, no split-K): tile shape, and a direct launch of max_tiles workgroups
// (at least the table's tile count, read from *tile_count on the device).
int nt_ring_tile_m();
int nt_ring_tile_n();
hipError_t launch_nt_ring_table(int precision, const NtEntry* entries, int n_entries,
                                const int* tile_count, int max_tiles, hipStream_t s);
hipError_t launch_nt_first(int layers, int levels, int precision, const NtBuffers& b,
                           int max_tiles, int tile_n, hipStream_t s);
hipError_t launch_nt_second(int ny, int nx, int precision, int split, const NtBuffers& b,
                            hipStream_t s);
// Persistent launch over a batched table: `grid` workgroups pull tiles from
// *queue (zeroed by the caller) until *tile_count is reached.
hipError_t launch_nt_persistent(bool second, int precision, int tile_m, int tile_n,
                                const NtEntry* entries, int n_entries, const int* tile_count,
                                int* queue, int grid, hipStream_t s);
// Adds each scene's tile offset to its problems in the batched tables, writes
// the two tile totals to counts[0..1] and zeroes queues[0..1].
// Also writes scene_units[0..n]: the exclusive prefix of the scenes' panel work
// units (the batched panel gather splits that range over its workgroups).
hipError_t launch_batch_prefix(const PlanHeader* hdrs, int n_scenes, const int* first_off,
                               NtEntry* first, NtEntry* second, int* counts, int* queues,
                               int* scene_units, hipStream_t s);
// Direct launch over a table of complex x complex problems (A and B complex,
// tile 128 x nt_table_tile_n(epi, precision); `tiles` bounds the device tile
// count, split-K when split > 1 into each problem's partial buffer).  Epilogues:
//   kEpiComplex  complex64 rows of `out` (row stride out_ld), partials [s][M][out_ld]
//   kEpiPanel    operand planes of `out` (row stride out_ld, plane stride out_ps),
//                columns up to pad16(N); partials [s][M][N]
//   kEpiReal     real part only into floats of `out`; partials [s][M][N] floats
enum { kEpiComplex = 0, kEpiPanel = 1, kEpiReal = 2 };
// Column tile of a table launch: 64 where FP32 products keep both parts (128 x 64
// tiles take the three-product complex form), 128 otherwise; tables built for
// launch_nt_table must use it for tiles_n and their tile counts.
__host__ __device__ inline int nt_table_tile_n(int epi, int precision) {
    return (precision == P_FP32 && epi != kEpiReal) ? 64 : kNtTile;
}
hipError_t launch_nt_table(int epi, int precision, const NtEntry* entries, int n_entries,
                           const int* tile_count, int tiles, int split, hipStream_t s);

// Dense products with Toeplitz fringe panels (Fresnel back-propagation).
struct DenseBuffers {
    void* kx;           // K'_x panel [p][x], nx x pad16(nx)
    void* ky;           // s K'_y panel [q][y], ny x pad16(ny)
    void* h;            // input field panel [y][x], ny x pad16(nx)
    void* t;            // step-1 product panel [p][y], nx x pad16(ny)
    float2* c1;         // step-1 FP32 product when the K range is not split
    float2* partial;    // split-K partials (split x ny x nx)
    NtEntry* entries;   // 2 problem slots
    int* counts;        // 2 tile counts
    unsigned long long* absmax;  // max-abs word of the input field (FP16 range scaling;
                                 // cleared by the caller)
};
// Bytes of the panel region (plus the unsplit step-1 product) for a split.
size_t dense_bytes(int ny, int nx, int split);
// Dense form of one layer (reconstruct the masked object first, then one
// contraction pair): out (+)= K_y recon K_x^T, K from the level-0 tables
// lut0_x / lut0_y (float re / im halves of lut_len(n) entries; the layer's
// prefactor in lut0_y).  scratch: fused_bytes(ny, nx); the ny * nx floats at
// fused_recon_offset(ny, nx) are not touched (room for the caller's recon);
// entries / counts: 2 slots.
size_t fused_bytes(int ny, int nx);
size_t fused_recon_offset(int ny, int nx);
// absmax: max |object| word of the coefficient stage, e_fringe: the exponent the y
// table's prefactor was scaled by (FP16 range scaling; ignored otherwise).
hipError_t launch_fused_layer(const float* recon, const float* lut0_x, const float* lut0_y,
                              int ny, int nx, int precision, int accumulate, float2* out,
                              char* scratch, NtEntry* entries, int* counts,
                              const unsigned long long* absmax, int e_fringe, hipStream_t s);
DenseBuffers dense_buffers(char* base, int ny, int nx, int split, float2* partial,
                           NtEntry* entries, int* counts, unsigned long long* absmax);
// out = scale * K'_y in K'_x, K' = conj(K) (adjoint == 0) or K (adjoint != 0).
hipError_t launch_dense_backprop(const DenseBuffers& b, const float* lut0_x, const float* lut0_y,
                                 const float2* in, float2* out, int ny, int nx, int adjoint,
                                 float scale, int precision, int split, hipStream_t s);

// Coefficient gradient of every layer and level (adjoint of the forward
// contractions) into gcoef (per layer an ny x nx plane at Mallat positions);
// `region` holds backward_bytes() of panels, partials and problem tables.
size_t backward_bytes(int ny, int nx, int layers, int levels);
// absmax: a cleared max-abs word for the cotangent and e_fringe the exponent the y
// tables' prefactors were scaled by (FP16 range scaling; ignored otherwise).
hipError_t launch_backward_nt(const float2* grad_h, const float* lut_x, const float* lut_y, int ny,
                              int nx, int layers, int levels, int precision, float* gcoef,
                              void* region, unsigned long long* absmax, int e_fringe,
                              hipStream_t s);

// Direct launch of first-contraction problems (A real, B complex, transposed
// K-blocked panel output) over a table; `tiles` bounds the device tile count.
hipError_t launch_nt_first_table(int precision, const NtEntry* entries, int n_entries,
                                 const int* tile_count, int tiles, hipStream_t s);

// Paper-literal form (image-domain residual maps times uniform-block fringes).
// Per-layer optical constants ([host] arrays of the layer count): c = p^2 / (2 lambda z)
// and the prefactors of the x (unit) and y (optional Eq. 1 constant) tables.
struct LitTables {
    const double *c, *one_re, *one_im, *pre_re, *pre_im;
};
size_t literal_bytes(int ny, int nx, int layers, int levels);
// absmax: max |object| word of the coefficient stage; e_fringe as for the backward
// (FP16 range scaling; ignored otherwise).
hipError_t launch_literal(const float* coef, const float* lut_x, const float* lut_y,
                          const LitTables& tb, int ny, int nx, int layers, int levels,
                          int precision, int split, float2* partial, float2* hologram,
                          int accumulate, const unsigned long long* absmax, int e_fringe,
                          void* region, hipStream_t s);

// Tiles of a problem with M rows and N columns under a tile shape.
__host__ __device__ inline int nt_tiles(int M, int N, int tm, int tn) {
    return ((M + tm - 1) / tm) * ((N + tn - 1) / tn);
}

}  // namespace cgh
