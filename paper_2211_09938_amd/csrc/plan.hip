// Planning and operand-panel kernels of the compacted forward contractions.
//
//  * lists:  per (layer, level), the active rows and columns of the level's
//            coefficient square (deterministic wave-ballot compaction);
//  * plan:   padded counts, k' segment offsets and the GEMM problem table;
//  * panels: K-contiguous operand panels in the operand precision --
//            the fringe operands (Fy_c[y][k'], Fx_c[x][c'], or their roles swapped
//            where a (layer, level) is contracted columns-first) gathered from the
//            1D fringe tables, Cb_c[r'][c'] (or its transpose) gathered from the
//            masked Mallat coefficients.
#include "nt.h"
#include "split.h"

namespace cgh {

namespace {

// Appends, in index order, every i in [0, n) with f[i] != 0 to out; returns the count.
__device__ int block_compact(const uint8_t* __restrict__ f, int n, int* __restrict__ out,
                             int* s_wave) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    int running = 0;
    for (int base = 0; base < n; base += blockDim.x) {
        const int i = base + (int)threadIdx.x;
        const bool pred = i < n && f[i] != 0;
        const unsigned long long m = __ballot(pred);
        const int pre = __popcll(m & ((1ull << lane) - 1ull));
        if (lane == 0) s_wave[w] = __popcll(m);
        __syncthreads();
        int off = 0, tot = 0;
        for (int k = 0; k < nw; ++k) {
            if (k < w) off += s_wave[k];
            tot += s_wave[k];
        }
        if (pred) out[running + off + pre] = i;
        running += tot;
        __syncthreads();
    }
    return running;
}

__device__ __forceinline__ void lists_block(const uint8_t* __restrict__ flags, int ny, int nx,
                                            int levels, size_t flags_layer,
                                            int* __restrict__ rowlist, int* __restrict__ collist,
                                            int* __restrict__ cnt_row, int* __restrict__ cnt_col,
                                            int dl, int* s_wave) {
    const int d = dl / levels, l = dl % levels + 1;
    const uint8_t* fr = flags + (size_t)d * flags_layer + flag_level_off(ny, nx, l);
    const int sy = band_side(ny, l), sx = band_side(nx, l);
    const int nr = block_compact(fr, sy, rowlist + dl_rows_off(ny, levels, d, l), s_wave);
    const int nc = block_compact(fr + sy, sx, collist + dl_cols_off(nx, levels, d, l), s_wave);
    if (threadIdx.x == 0) {
        cnt_row[dl] = nr;
        cnt_col[dl] = nc;
    }
}

__global__ __launch_bounds__(1024) void lists_kernel(const uint8_t* __restrict__ flags, int ny,
                                                     int nx, int levels, size_t flags_layer,
                                                     int* __restrict__ rowlist,
                                                     int* __restrict__ collist,
                                                     int* __restrict__ cnt_row,
                                                     int* __restrict__ cnt_col) {
    __shared__ int s_wave[16];
    lists_block(flags, ny, nx, levels, flags_layer, rowlist, collist, cnt_row, cnt_col,
                blockIdx.x, s_wave);
}

// Batched: grid.y = scene, grid.x sized for the scene with the most (layer, level) pairs.
__global__ __launch_bounds__(1024) void lists_batch_kernel(const PrepScene* __restrict__ scenes,
                                                           int levels) {
    __shared__ int s_wave[16];
    const PrepScene& sc = scenes[blockIdx.y];
    if ((int)blockIdx.x >= sc.layers * levels) return;
    lists_block(sc.flags, sc.ny, sc.nx, levels, sc.flags_layer, sc.b.rowlist, sc.b.collist,
                sc.b.cnt_row, sc.b.cnt_col, blockIdx.x, s_wave);
}

// Inclusive Hillis-Steele scan over the workgroup (blockDim.x <= 1024 threads).
__device__ int block_scan_incl(int v, int* sh) {
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int off = 1; off < (int)blockDim.x; off <<= 1) {
        const int add = (threadIdx.x >= (unsigned)off) ? sh[threadIdx.x - off] : 0;
        __syncthreads();
        sh[threadIdx.x] += add;
        __syncthreads();
    }
    const int r = sh[threadIdx.x];
    __syncthreads();
    return r;
}


__device__ __forceinline__ void plan_block(const PlanArgs& a, int* sh, int* last) {
    const int n_dl = a.layers * a.levels;
    int total_k = 0, total_t = 0, total_a = 0;
    // pass 1: the order of each (layer, level) (rows-first, or columns-first where
    // that gives the shorter padded K' segment: Eq. 3's sum is the same in either
    // order), its K' segment -> k' offsets, its first-contraction tiles -> tile prefix
    for (int base = 0; base < n_dl; base += blockDim.x) {
        const int t = base + (int)threadIdx.x;
        int seg = 0, tiles = 0, act = 0;
        if (t < n_dl) {
            const int cr = a.cnt_row[t], cc = a.cnt_col[t];
            const bool cf = columns_first(cr, cc);
            act = cf ? cc : cr;
            seg = pad_kt(act);
            // rows-first: cr x nx outputs; columns-first: cc x ny
            const int outer = cf ? a.ny : a.nx;
            tiles = act > 0 ? ((act + a.tm1 - 1) / a.tm1) * ((outer + a.tn1 - 1) / a.tn1) : 0;
            a.orient[t] = cf ? 1 : 0;
        }
        const int ik = block_scan_incl(seg, sh);
        const int it = block_scan_incl(tiles, sh);
        const int ia = block_scan_incl(act, sh);
        if (t < n_dl) {
            a.seg_row[t] = total_k + ik - seg;
            a.tbeg[t] = total_t + it - tiles;
        }
        if (threadIdx.x == blockDim.x - 1) {
            last[0] = ik;
            last[1] = it;
            last[2] = ia;
        }
        __syncthreads();
        total_k += last[0];
        total_t += last[1];
        total_a += last[2];
        __syncthreads();
    }
    const int kpad = total_k;
    // FP16 range scaling: coefficients to [1, 2) times their largest magnitude
    // (|coefficient| <= max |object| for the averaging Haar pair), the first
    // contraction's outputs below 2^15: a level-l fringe entry is a sum of 2^l unit
    // phasors (times the y tables' layer constant, scaled into [1, 2)), and a row
    // or column of a level's square has at most 2 n / 2^l active entries, so
    // |T| < 2 x 2 nx and |T'| < 2 x 2 x 2 ny, both below 16 max(ny, nx); the second
    // contraction's epilogue undoes the three scales
    float cb_scale = 1.f, first_scale = 1.f, second_scale = 1.f;
    if (a.fp16) {
        const int ea = range_exp(absmax_value(a.absmax));
        const int t = headroom_shift(16.f * (float)(a.ny > a.nx ? a.ny : a.nx));
        cb_scale = pow2f(-ea);
        first_scale = pow2f(-t);
        second_scale = pow2f(ea + t + a.e_fringe);
    }
    // pass 2: the problem table.  Rows-first: T = Cb_c Fx_c^T (cr x nx, K = padded
    // columns) into the B operand of the second contraction; columns-first:
    // T' = Cb_c^T Fy_c^T (cc x ny, K = padded rows) into its A operand.
    const char* cb = static_cast<const char*>(a.cb);
    const char* fx = static_cast<const char*>(a.fx);
    char* fy = static_cast<char*>(a.fy);
    char* tc = static_cast<char*>(a.tc);
    for (int t = threadIdx.x; t < n_dl; t += blockDim.x) {
        const int d = t / a.levels, l = t % a.levels + 1;
        const int cr = a.cnt_row[t], cc = a.cnt_col[t];
        const bool cf = columns_first(cr, cc);
        const int outer = cf ? a.ny : a.nx;
        NtEntry e;
        e.a = cb + dl_cb_off(a.ny, a.nx, a.levels, d, l) * a.esize;
        e.b = fx + dl_fx_off(a.ny, a.nx, a.levels, d, l) * a.esize;
        // K block seg/16 of the operand panel the result feeds
        e.out = (cf ? fy : tc) + (size_t)a.seg_row[t] * outer * a.esize;
        e.partial = nullptr;
        e.a_ps = a.cb_ps;
        e.b_ps = a.fx_ps;
        e.out_ps = cf ? a.fy_ps : a.tc_ps;
        e.M = cf ? cc : cr;
        e.N = outer;
        e.K = pad_kt(cf ? cr : cc);
        e.lda = e.M * 16;
        e.ldb = outer * 16;
        e.out_ld = outer * 16;
        e.tiles_n = (outer + a.tn1 - 1) / a.tn1;
        e.tile_begin = a.tbeg[t];
        e.accumulate = 0;
        e.tile_m = a.tm1;
        e.tile_n = a.tn1;
        e.out_scale = first_scale;
        a.first[t] = e;
    }
    if (threadIdx.x == 0) {
        a.hdr->kpad = kpad;
        a.hdr->first_tiles = total_t;
        a.hdr->k_active = total_a;
        a.hdr->second_tiles = nt_tiles(a.ny, a.nx, a.tm2, a.tn2);
        a.hdr->cb_scale = cb_scale;
        NtEntry e;
        e.a = a.fy;
        e.b = a.tc;
        e.out = a.hologram;
        e.partial = a.partial;
        e.a_ps = a.fy_ps;
        e.b_ps = a.tc_ps;
        e.out_ps = 0;
        e.M = a.ny;
        e.N = a.nx;
        e.K = kpad;
        e.lda = a.ny * 16;
        e.ldb = a.nx * 16;
        e.out_ld = a.nx;
        e.tiles_n = (a.nx + a.tn2 - 1) / a.tn2;
        e.tile_begin = 0;
        e.accumulate = a.accumulate;
        e.tile_m = a.tm2;
        e.tile_n = a.tn2;
        e.out_scale = second_scale;
        a.second[0] = e;
    }
}

__global__ __launch_bounds__(1024) void plan_kernel(PlanArgs a) {
    __shared__ int sh[1024];
    __shared__ int last[3];
    plan_block(a, sh, last);
}

// Batched: one workgroup per scene.
__global__ __launch_bounds__(1024) void plan_batch_kernel(const PlanArgs* __restrict__ args) {
    __shared__ int sh[1024];
    __shared__ int last[3];
    const PlanArgs a = args[blockIdx.x];
    plan_block(a, sh, last);
}

// Merges the per-scene problem tables of a batch: scene i's first-contraction
// entries (first_off[i] .. first_off[i+1]) and its second-contraction entry get
// the tile offset of every scene before it; writes the batch tile totals and
// clears the two work-queue counters.
__global__ __launch_bounds__(1024) void batch_prefix_kernel(const PlanHeader* __restrict__ hdrs,
                                                            int n_scenes,
                                                            const int* __restrict__ first_off,
                                                            NtEntry* __restrict__ first,
                                                            NtEntry* __restrict__ second,
                                                            int* __restrict__ counts,
                                                            int* __restrict__ queues) {
    __shared__ int sh[1024];
    __shared__ int last[2];
    int run1 = 0, run2 = 0;
    for (int base = 0; base < n_scenes; base += 1024) {
        const int i = base + (int)threadIdx.x;
        const int v1 = i < n_scenes ? hdrs[i].first_tiles : 0;
        const int v2 = i < n_scenes ? hdrs[i].second_tiles : 0;
        const int c1 = block_scan_incl(v1, sh);
        const int c2 = block_scan_incl(v2, sh);
        if (i < n_scenes) {
            const int o1 = run1 + c1 - v1;
            for (int e = first_off[i]; e < first_off[i + 1]; ++e) first[e].tile_begin += o1;
            second[i].tile_begin = run2 + c2 - v2;
        }
        if (threadIdx.x == blockDim.x - 1) {
            last[0] = c1;
            last[1] = c2;
        }
        __syncthreads();
        run1 += last[0];
        run2 += last[1];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        counts[0] = run1;
        counts[1] = run2;
        queues[0] = 0;
        queues[1] = 0;
    }
}

// Fringe panels through LDS.  Column k' of a panel is a contiguous slice of a 1D
// fringe table (row y reads entry y - j 2^l + n for the k'-th active row j).  A
// workgroup takes 256 rows x one 16-wide K block: it reads the table with the
// lanes along the rows (one contiguous run per k'), keeps the tile in LDS (row
// pitch 17 floats: the LDS stores of each table read hit 64 different banks; the
// chunk reads that follow can pair up on a bank), and writes the tile's K-blocked
// storage -- 256 rows x 16 elements, contiguous -- with consecutive lanes on
// consecutive 4-element chunks.
constexpr int kFringeRows = 256, kFringePitch = 17;

template <int P>
__device__ __forceinline__ void fringe_tiles(const float* __restrict__ lutl, int len,
                                             const int* __restrict__ list, int count, int half,
                                             int l, int n, int padded, void* panel, size_t ps,
                                             size_t base) {
    __shared__ float lre[kFringeRows * kFringePitch], lim[kFringeRows * kFringePitch];
    const int tid = threadIdx.x;
    const int ytiles = (n + kFringeRows - 1) / kFringeRows;
    const int tasks = ytiles * (padded / 16);
    for (int task = blockIdx.x; task < tasks; task += gridDim.x) {
        const int kb = task / ytiles, y0 = (task - kb * ytiles) * kFringeRows;
        const int y = y0 + tid;
#pragma unroll 4
        for (int q = 0; q < 16; ++q) {
            const int i = 16 * kb + q;
            float re = 0.f, im = 0.f;
            if (i < count && y < n) {
                const int r = list[i];
                const int band = r >= half, j = r - band * half;
                const float* tb = lutl + (size_t)band * 2 * len;
                const int idx = y - (j << l) + n;
                re = tb[idx];
                im = tb[len + idx];
            }
            lre[tid * kFringePitch + q] = re;
            lim[tid * kFringePitch + q] = im;
        }
        __syncthreads();
        // chunk c = 4 elements: row c / 4 of the tile, k' 4 (c % 4) .. + 3
        const size_t tile = base + ((size_t)kb * n + y0) * 16;
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4) {
            const int c = s4 * kFringeRows + tid, row = c >> 2, k4 = (c & 3) * 4;
            if (y0 + row < n) {
                float re[4], im[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    re[q] = lre[row * kFringePitch + k4 + q];
                    im[q] = lim[row * kFringePitch + k4 + q];
                }
                put_c4<P>(panel, ps, tile + 4 * (size_t)c, re, im);
            }
        }
        __syncthreads();
    }
}

// Fringe operand of the second contraction for one (layer, level): rows-first, the
// y fringes of its active rows (Fy_c, ny rows) at its k' segment of the A panel;
// columns-first, the x fringes of its active columns (nx rows) at its segment of
// the B panel (the first contraction fills the other operand's segment).
template <int P>
__device__ __forceinline__ void second_fringe_block(const float* __restrict__ lut_x,
                                                    const float* __restrict__ lut_y,
                                                    const NtBuffers& b, int ny, int nx,
                                                    int levels, int dl) {
    const int d = dl / levels, l = dl % levels + 1;
    const int cr = b.cnt_row[dl], cc = b.cnt_col[dl];
    if (cr == 0 || cc == 0) return;
    const size_t seg = (size_t)b.seg_row[dl];
    if (b.orient[dl]) {
        const int len = lut_len(nx);
        fringe_tiles<P>(lut_x + lut_table(d, l, 0, 0, levels) * len, len,
                        b.collist + dl_cols_off(nx, levels, d, l), cc, nx >> l, l, nx,
                        pad_kt(cc), b.tc, b.tc_ps, seg * nx);
    } else {
        const int len = lut_len(ny);
        fringe_tiles<P>(lut_y + lut_table(d, l, 0, 0, levels) * len, len,
                        b.rowlist + dl_rows_off(ny, levels, d, l), cr, ny >> l, l, ny,
                        pad_kt(cr), b.fy, b.fy_ps, seg * ny);
    }
}

// Fringe operand of the first contraction: rows-first, the x fringes of the active
// columns (Fx_c, nx rows); columns-first, the y fringes of the active rows (ny rows).
template <int P>
__device__ __forceinline__ void first_fringe_block(const float* __restrict__ lut_x,
                                                   const float* __restrict__ lut_y,
                                                   const NtBuffers& b, int ny, int nx,
                                                   int levels, int dl) {
    const int d = dl / levels, l = dl % levels + 1;
    const int cr = b.cnt_row[dl], cc = b.cnt_col[dl];
    if (cr == 0 || cc == 0) return;
    const size_t base = dl_fx_off(ny, nx, levels, d, l);
    if (b.orient[dl]) {
        const int len = lut_len(ny);
        fringe_tiles<P>(lut_y + lut_table(d, l, 0, 0, levels) * len, len,
                        b.rowlist + dl_rows_off(ny, levels, d, l), cr, ny >> l, l, ny,
                        pad_kt(cr), b.fx, b.fx_ps, base);
    } else {
        const int len = lut_len(nx);
        fringe_tiles<P>(lut_x + lut_table(d, l, 0, 0, levels) * len, len,
                        b.collist + dl_cols_off(nx, levels, d, l), cc, nx >> l, l, nx,
                        pad_kt(cc), b.fx, b.fx_ps, base);
    }
}

// Coefficient operand of the first contraction: Cb_c (active rows x padded active
// columns) rows-first, its transpose (active columns x padded active rows)
// columns-first; K-blocked, four consecutive k' per thread.
template <int P>
__device__ __forceinline__ void cb_block(const float* __restrict__ coef, const NtBuffers& b,
                                         int ny, int nx, int levels, int dl) {
    const int d = dl / levels, l = dl % levels + 1;
    const int cr = b.cnt_row[dl], cc = b.cnt_col[dl];
    if (cr == 0 || cc == 0) return;
    const bool cf = b.orient[dl] != 0;
    const int rows = cf ? cc : cr, kn = cf ? cr : cc, kp = pad_kt(kn);
    const float scale = b.hdr->cb_scale;  // written by the planning kernel
    const int nyl = ny >> l, nxl = nx >> l;
    // the coefficient stage wrote only the blocks that hold a pixel of the layer:
    // a level-l coefficient at quadrant position (i, j) covers block
    // (i >> (levels - l), j >> (levels - l)) of 2^levels pixels
    const int nbx = nx >> levels, sh = levels - l;
    const uint8_t* oc = b.occ + (size_t)d * (size_t)(ny >> levels) * nbx;
    const int* rl = b.rowlist + dl_rows_off(ny, levels, d, l);
    const int* cl = b.collist + dl_cols_off(nx, levels, d, l);
    const float* cd = coef + (size_t)d * ny * nx;
    const size_t base = dl_cb_off(ny, nx, levels, d, l);
    const long long total4 = (long long)rows * kp / 4;
    for (long long e4 = (long long)blockIdx.x * blockDim.x + threadIdx.x; e4 < total4;
         e4 += (long long)gridDim.x * blockDim.x) {
        const size_t e = (size_t)e4 * 4;
        int pr, k0;
        kblk_pos(e, rows, pr, k0);
        float v[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int k = k0 + q;
            v[q] = 0.f;
            if (k < kn) {
                const int r = rl[cf ? k : pr], j = cl[cf ? pr : k];
                const int brow = (r < nyl ? r : r - nyl) >> sh;
                const int bcol = (j < nxl ? j : j - nxl) >> sh;
                // the LL quadrant of a level below the top belongs to the coarser levels
                if (!(l < levels && r < nyl && j < nxl) && oc[(size_t)brow * nbx + bcol])
                    v[q] = cd[(size_t)r * nx + j] * scale;
            }
        }
        put_r4<P>(b.cb, b.cb_ps, base + e, v);
    }
}

// The three panels of one scene in one launch: grid.z selects the panel (0 the
// second contraction's fringe operand, 1 the first contraction's, 2 the coefficient
// operand), grid.y the (layer, level), grid.x strides over its chunks; the three
// gathers share the machine instead of each ending on a partial wave.
template <int P>
__global__ __launch_bounds__(256) void panels_kernel(const float* __restrict__ coef,
                                                     const float* __restrict__ lut_x,
                                                     const float* __restrict__ lut_y, int ny,
                                                     int nx, int levels, NtBuffers b) {
    const int dl = blockIdx.y;
    if (blockIdx.z == 0) second_fringe_block<P>(lut_x, lut_y, b, ny, nx, levels, dl);
    else if (blockIdx.z == 1) first_fringe_block<P>(lut_x, lut_y, b, ny, nx, levels, dl);
    else cb_block<P>(coef, b, ny, nx, levels, dl);
}

// Batched panels: grid.z = 3 x scene + panel (as panels_kernel), grid.y = (layer, level),
// grid.x = chunks.
template <int P>
__global__ __launch_bounds__(256) void panels_batch_kernel(const PrepScene* __restrict__ scenes,
                                                           int levels) {
    const PrepScene& sc = scenes[blockIdx.z / 3];
    if ((int)blockIdx.y >= sc.layers * levels) return;
    const int panel = blockIdx.z % 3, dl = blockIdx.y;
    if (panel == 0) second_fringe_block<P>(sc.lut_x, sc.lut_y, sc.b, sc.ny, sc.nx, levels, dl);
    else if (panel == 1) first_fringe_block<P>(sc.lut_x, sc.lut_y, sc.b, sc.ny, sc.nx, levels, dl);
    else cb_block<P>(sc.coef, sc.b, sc.ny, sc.nx, levels, dl);
}

int grid_for(long long elems) {
    long long g = (elems + 256 * 8 - 1) / (256 * 8);
    if (g < 1) g = 1;
    if (g > 512) g = 512;
    return (int)g;
}

}  // namespace

PlanArgs make_plan_args(int ny, int nx, int layers, int levels, int precision, const int* tiles,
                        const NtBuffers& b, const NtOutput& o, const unsigned long long* absmax,
                        int e_fringe) {
    PlanArgs a{};
    a.ny = ny;
    a.nx = nx;
    a.layers = layers;
    a.levels = levels;
    a.esize = precision == P_FP32 ? 4 : 2;
    a.fp16 = precision == P_FP16;
    a.e_fringe = e_fringe;
    a.absmax = absmax;
    a.tm1 = tiles[0];
    a.tn1 = tiles[1];
    a.tm2 = tiles[2];
    a.tn2 = tiles[3];
    a.cnt_row = b.cnt_row;
    a.cnt_col = b.cnt_col;
    a.seg_row = b.seg_row;
    a.orient = b.orient;
    a.tbeg = b.tbeg;
    a.hdr = b.hdr;
    a.first = b.first;
    a.second = b.second;
    a.cb = b.cb;
    a.fx = b.fx;
    a.fy = b.fy;
    a.tc = b.tc;
    a.cb_ps = (long long)b.cb_ps;
    a.fx_ps = (long long)b.fx_ps;
    a.fy_ps = (long long)b.fy_ps;
    a.tc_ps = (long long)b.tc_ps;
    a.hologram = o.hologram;
    a.partial = o.partial;
    a.accumulate = o.accumulate;
    return a;
}

hipError_t launch_nt_plan(const uint8_t* flags, int ny, int nx, int layers, int levels,
                          size_t flags_layer, int precision, const int* tiles,
                          const NtBuffers& b, const NtOutput& o,
                          const unsigned long long* absmax, int e_fringe, hipStream_t s) {
    const int n_dl = layers * levels;
    hipLaunchKernelGGL(lists_kernel, dim3(n_dl), dim3(1024), 0, s, flags, ny, nx, levels,
                       flags_layer, b.rowlist, b.collist, b.cnt_row, b.cnt_col);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const PlanArgs a = make_plan_args(ny, nx, layers, levels, precision, tiles, b, o, absmax,
                                      e_fringe);
    // one wave scans up to 64 (layer, level) pairs without a workgroup barrier's cost
    hipLaunchKernelGGL(plan_kernel, dim3(1), dim3(n_dl <= 64 ? 64 : 1024), 0, s, a);
    return hipGetLastError();
}

template <int P>
static hipError_t materialize(const float* coef, const float* lut_x, const float* lut_y, int ny,
                              int nx, int layers, int levels, const NtBuffers& b, hipStream_t s) {
    const int n_dl = layers * levels;
    const long long big_y = (long long)ny * pad_kt(band_side(ny, 1));
    const long long big_x = (long long)nx * pad_kt(band_side(nx, 1));
    const long long big_c = (long long)dl_coef_elems(ny, nx, 1);
    // fringe panels: one workgroup per 256 rows x 16 K = 4096 elements (grid_for sizes for
    // 2048); the coefficient panel four elements per thread; all three in one launch
    int gx = grid_for(big_y / 2);
    if (grid_for(big_x / 2) > gx) gx = grid_for(big_x / 2);
    if (grid_for(big_c) > gx) gx = grid_for(big_c);
    hipLaunchKernelGGL(panels_kernel<P>, dim3(gx, n_dl, 3), dim3(256), 0, s, coef, lut_x, lut_y,
                       ny, nx, levels, b);
    return hipGetLastError();
}

// Workgroups per (scene, layer, level) of the batched panel kernels: the scenes
// already give the launch its parallelism (a grid sized for the largest scene
// left most workgroups idle: measured 30% slower preparation on the 64-scene batch).
constexpr int kBatchPanelBlocks = 64;

template <int P>
static void materialize_batch(const PrepScene* scenes, int n, int levels, int max_ndl,
                              hipStream_t s) {
    hipLaunchKernelGGL(panels_batch_kernel<P>, dim3(kBatchPanelBlocks, max_ndl, 3 * n),
                       dim3(256), 0, s, scenes, levels);
}

hipError_t launch_lists_batch(const PrepScene* scenes, int n, int levels, int max_ndl,
                              hipStream_t s) {
    hipLaunchKernelGGL(lists_batch_kernel, dim3(max_ndl, n), dim3(1024), 0, s, scenes, levels);
    return hipGetLastError();
}

hipError_t launch_plan_batch(const PlanArgs* args, int n, int max_ndl, hipStream_t s) {
    hipLaunchKernelGGL(plan_batch_kernel, dim3(n), dim3(max_ndl <= 64 ? 64 : 1024), 0, s, args);
    return hipGetLastError();
}

hipError_t launch_materialize_batch(const PrepScene* scenes, int n, int levels, int precision,
                                    int max_ndl, hipStream_t s) {
    if (precision == P_BF16) materialize_batch<P_BF16>(scenes, n, levels, max_ndl, s);
    else if (precision == P_FP16) materialize_batch<P_FP16>(scenes, n, levels, max_ndl, s);
    else materialize_batch<P_FP32>(scenes, n, levels, max_ndl, s);
    return hipGetLastError();
}

hipError_t launch_batch_prefix(const PlanHeader* hdrs, int n_scenes, const int* first_off,
                               NtEntry* first, NtEntry* second, int* counts, int* queues,
                               hipStream_t s) {
    hipLaunchKernelGGL(batch_prefix_kernel, dim3(1), dim3(1024), 0, s, hdrs, n_scenes, first_off,
                       first, second, counts, queues);
    return hipGetLastError();
}

hipError_t launch_nt_materialize(const float* coef, const float* lut_x, const float* lut_y, int ny,
                                 int nx, int layers, int levels, int precision,
                                 const NtBuffers& b, hipStream_t s) {
    if (precision == P_BF16) return materialize<P_BF16>(coef, lut_x, lut_y, ny, nx, layers, levels, b, s);
    if (precision == P_FP16) return materialize<P_FP16>(coef, lut_x, lut_y, ny, nx, layers, levels, b, s);
    return materialize<P_FP32>(coef, lut_x, lut_y, ny, nx, layers, levels, b, s);
}

}  // namespace cgh
