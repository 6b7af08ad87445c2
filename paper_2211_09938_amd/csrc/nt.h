// Compacted "NT" formulation of the forward contractions (internal).
//
// Only coefficient rows / columns that hold a nonzero masked coefficient take
// part (the layer split and the saliency masks leave most of them empty):
//   first:   T_c[x][k'] = sum_c' Cb_c[r'][c'] * Fx_c[x][c']     per (layer, level)
//   second:  H[y][x]    = sum_k' Fy_c[y][k'] * T_c[x][k']
// r' / c' index the active rows / columns of a level's coefficient square; k'
// runs over the active rows of every (layer, level) in order, each segment
// padded with zero rows to a multiple of kKT.  Every operand panel is stored
// K-contiguous ("row-major M x K" and "row-major N x K"), in the operand
// precision: FP32 planes (re[, im]) or 16-bit split planes
// (re_hi, re_lo[, im_hi, im_lo]).
#pragma once

#include "common.h"

namespace cgh {

constexpr int kKT = 16;       // K tile; every K extent is a multiple of it
constexpr int kNtTile = 128;  // output tile rows and columns

__host__ __device__ inline int pad_kt(int v) { return (v + kKT - 1) / kKT * kKT; }

// One GEMM problem of the batched NT kernel.
struct NtEntry {
    int M, N, K;           // output rows, output columns (complex), reduction length
    int lda, ldb;          // row strides of the A and B panels (elements)
    long long a_off;       // element offset of A's row 0 inside its planes
    long long b_off;       // element offset of B's row 0 inside its planes
    long long out_off;     // first contraction: k' segment offset of this problem
    int tiles_n;           // ceil(N / kNtTile)
    int tile_begin;        // exclusive prefix of tiles over the entries
};

// Device-side plan written by the planning kernels (lives in the workspace).
struct PlanHeader {
    int kpad;          // K of the second contraction (sum of padded row counts)
    int first_tiles;   // tiles of the first contraction
    int rows_active;   // sum of active row counts
    int second_tiles;  // output tiles of the second contraction
};

// Element counts (dense upper bounds) of the compacted regions.
struct NtSizes {
    size_t rowlist, collist;  // ints
    size_t fx_plane;          // elements per plane of Fx_c
    size_t cb_plane;          // elements per plane of Cb_c
    size_t kmax;              // upper bound of kpad
    size_t fy_plane, tc_plane;
    int first_tiles_max;
};

inline NtSizes nt_sizes(int ny, int nx, int layers, int levels) {
    NtSizes z{};
    size_t sy = 0, sx = 0, fx = 0, cb = 0, kmax = 0;
    int tiles = 0;
    for (int l = 1; l <= levels; ++l) {
        const int syl = band_side(ny, l), sxl = band_side(nx, l);
        sy += syl;
        sx += sxl;
        fx += (size_t)nx * pad_kt(sxl);
        cb += (size_t)syl * pad_kt(sxl);
        kmax += pad_kt(syl);
        tiles += ((syl + kNtTile - 1) / kNtTile) * ((nx + kNtTile - 1) / kNtTile);
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
__host__ __device__ inline size_t dl_fx_off(int nx, int levels, int d, int l) {
    size_t per = 0, off = 0;
    for (int k = 1; k <= levels; ++k) {
        const size_t v = (size_t)nx * pad_kt(band_side(nx, k));
        if (k < l) off += v;
        per += v;
    }
    return (size_t)d * per + off;
}
__host__ __device__ inline size_t dl_cb_off(int ny, int nx, int levels, int d, int l) {
    size_t per = 0, off = 0;
    for (int k = 1; k <= levels; ++k) {
        const size_t v = (size_t)band_side(ny, k) * pad_kt(band_side(nx, k));
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
    int* seg_row;   // [D*L]
    PlanHeader* hdr;
    NtEntry* entries;  // [D*L] first contraction, then 1 for the second
    // panels (element type by precision), plane strides in elements
    void* fx; void* cb; void* fy; void* tc;
    size_t fx_ps, cb_ps, fy_ps, tc_ps;
};

hipError_t launch_nt_plan(const uint8_t* flags, int ny, int nx, int layers, int levels,
                          size_t flags_layer, const NtBuffers& b, hipStream_t s);
hipError_t launch_nt_materialize(const float* coef, const float* lut_x, const float* lut_y, int ny,
                                 int nx, int layers, int levels, int precision,
                                 const NtBuffers& b, hipStream_t s);
hipError_t launch_nt_first(int ny, int nx, int layers, int levels, int precision,
                           const NtBuffers& b, int max_tiles, hipStream_t s);
hipError_t launch_nt_second(int ny, int nx, int layers, int levels, int precision, int split,
                            const NtBuffers& b, float2* partial, float2* out, int accumulate,
                            hipStream_t s);

}  // namespace cgh
