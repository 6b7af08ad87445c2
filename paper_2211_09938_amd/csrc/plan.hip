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

// Offset of active row / column i's fringe in its (layer, level)'s operand-format tables
// (an axis of N points at level l): entry n + N + offset is the fringe at point n, in
// band 1 (table offset 2N) for i in the second half of the level's square.
__device__ __forceinline__ int gen_koff(int i, int N, int l) {
    const int half = N >> l;
    return i >= half ? 2 * N - ((i - half) << l) : -(i << l);
}

// Appends, in index order, every i in [0, n) with f[i] != 0 to out; returns the count.
// koff (optional): beside each i its gen_koff, and 3N (the zero band) from the count up
// to the next multiple of 16.
__device__ int block_compact(const uint8_t* __restrict__ f, int n, int* __restrict__ out,
                             int* s_wave, int* __restrict__ koff = nullptr, int N = 0,
                             int l = 0) {
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
        if (pred) {
            out[running + off + pre] = i;
            if (koff) koff[running + off + pre] = gen_koff(i, N, l);
        }
        running += tot;
        __syncthreads();
    }
    // the offsets up to the next multiple of 16 point at the zero band (the K padding)
    if (koff)
        for (int i = running + (int)threadIdx.x; i < pad_kt(running); i += blockDim.x)
            koff[i] = 3 * N;
    return running;
}

__device__ __forceinline__ void lists_block(const uint8_t* __restrict__ flags, int ny, int nx,
                                            int levels, size_t flags_layer,
                                            int* __restrict__ rowlist, int* __restrict__ collist,
                                            int* __restrict__ cnt_row, int* __restrict__ cnt_col,
                                            int dl, int* s_wave, int* __restrict__ koff_row = nullptr,
                                            int* __restrict__ koff_col = nullptr) {
    const int d = dl / levels, l = dl % levels + 1;
    const uint8_t* fr = flags + (size_t)d * flags_layer + flag_level_off(ny, nx, l);
    const int sy = band_side(ny, l), sx = band_side(nx, l);
    const int nr = block_compact(fr, sy, rowlist + dl_rows_off(ny, levels, d, l), s_wave,
                                 koff_row ? koff_row + dl_koff_off(ny, levels, d, l) : nullptr,
                                 ny, l);
    const int nc = block_compact(fr + sy, sx, collist + dl_cols_off(nx, levels, d, l), s_wave,
                                 koff_col ? koff_col + dl_koff_off(nx, levels, d, l) : nullptr,
                                 nx, l);
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
                                                     int* __restrict__ cnt_col,
                                                     int* __restrict__ koff_row,
                                                     int* __restrict__ koff_col) {
    __shared__ int s_wave[16];
    lists_block(flags, ny, nx, levels, flags_layer, rowlist, collist, cnt_row, cnt_col,
                blockIdx.x, s_wave, koff_row, koff_col);
}

// Batched: grid.y = scene, grid.x sized for the scene with the most (layer, level) pairs.
__global__ __launch_bounds__(1024) void lists_batch_kernel(const PrepScene* __restrict__ scenes,
                                                           int levels) {
    __shared__ int s_wave[16];
    const PrepScene& sc = scenes[blockIdx.y];
    if ((int)blockIdx.x >= sc.layers * levels) return;
    lists_block(sc.flags, sc.ny, sc.nx, levels, sc.flags_layer, sc.b.rowlist, sc.b.collist,
                sc.b.cnt_row, sc.b.cnt_col, blockIdx.x, s_wave, sc.b.koff_row, sc.b.koff_col);
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
    int total_k = 0, total_t = 0, total_a = 0, total_u0 = 0, total_u1 = 0, total_u2 = 0;
    // pass 1: the order of each (layer, level) (rows-first, or columns-first where
    // that gives the shorter padded K' segment: Eq. 3's sum is the same in either
    // order), its K' segment -> k' offsets, its first-contraction tiles -> tile prefix
    for (int base = 0; base < n_dl; base += blockDim.x) {
        const int t = base + (int)threadIdx.x;
        int seg = 0, tiles = 0, act = 0, pu[3] = {0, 0, 0};
        if (t < n_dl) {
            const int cr = a.cnt_row[t], cc = a.cnt_col[t];
            const bool cf = columns_first(cr, cc);
            act = cf ? cc : cr;
            seg = pad_kt(act);
            // rows-first: cr x nx outputs; columns-first: cc x ny
            const int outer = cf ? a.ny : a.nx;
            tiles = act > 0 ? ((act + a.tm1 - 1) / a.tm1) * ((outer + a.tn1 - 1) / a.tn1) : 0;
            a.orient[t] = cf ? 1 : 0;
            dl_panel_units(a.ny, a.nx, cr, cc, pu);
            if (nt_first_generates(a.tn1)) pu[1] = 0;  // generated by the first contraction
        }
        const int ik = block_scan_incl(seg, sh);
        const int it = block_scan_incl(tiles, sh);
        const int ia = block_scan_incl(act, sh);
        // the unit table only where a batched gather reads it (a.units is uniform)
        const int iu0 = a.units ? block_scan_incl(pu[0], sh) : 0;
        const int iu1 = a.units ? block_scan_incl(pu[1], sh) : 0;
        const int iu2 = a.units ? block_scan_incl(pu[2], sh) : 0;
        if (t < n_dl) {
            a.seg_row[t] = total_k + ik - seg;
            a.tbeg[t] = total_t + it - tiles;
            if (a.units) {
                // kind-local starts; the kinds' bases are added once their totals are known
                a.units[t] = total_u0 + iu0 - pu[0];
                a.units[n_dl + t] = total_u1 + iu1 - pu[1];
                a.units[2 * n_dl + t] = total_u2 + iu2 - pu[2];
            }
        }
        if (threadIdx.x == blockDim.x - 1) {
            last[0] = ik;
            last[1] = it;
            last[2] = ia;
            last[3] = iu0;
            last[4] = iu1;
            last[5] = iu2;
        }
        __syncthreads();
        total_k += last[0];
        total_t += last[1];
        total_a += last[2];
        total_u0 += last[3];
        total_u1 += last[4];
        total_u2 += last[5];
        __syncthreads();
    }
    // the unit table in kind-major order (every (layer, level)'s second-contraction
    // fringe tasks, then the first contraction's, then the coefficient units): the
    // workgroups resident at one time then write one panel (each thread adds the
    // bases to the entries it wrote above)
    for (int t = threadIdx.x; a.units && t < n_dl; t += blockDim.x) {
        a.units[n_dl + t] += total_u0;
        a.units[2 * n_dl + t] += total_u0 + total_u1;
    }
    const int total_u = total_u0 + total_u1 + total_u2;
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
        // the same operand from its table: rows-first the x fringes of the active columns,
        // columns-first the y fringes of the active rows
        e.g_lut = static_cast<const char*>(cf ? a.gen_y : a.gen_x) +
                  gen_table(d, l, a.levels) * lut_len(outer) * 8;
        e.g_koff = cf ? a.koff_row + dl_koff_off(a.ny, a.levels, d, l)
                      : a.koff_col + dl_koff_off(a.nx, a.levels, d, l);
        e.g_count = cf ? cr : cc;
        a.first[t] = e;
    }
    if (threadIdx.x == 0) {
        a.hdr->kpad = kpad;
        a.hdr->first_tiles = total_t;
        a.hdr->k_active = total_a;
        a.hdr->second_tiles = nt_tiles(a.ny, a.nx, a.tm2, a.tn2);
        a.hdr->cb_scale = cb_scale;
        a.hdr->panel_units = total_u;
        if (a.units) a.units[3 * n_dl] = total_u;
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
        e.g_lut = nullptr;
        e.g_koff = nullptr;
        e.g_count = 0;
        a.second[0] = e;
    }
}

__global__ __launch_bounds__(1024) void plan_kernel(PlanArgs a) {
    __shared__ int sh[1024];
    __shared__ int last[6];
    plan_block(a, sh, last);
}

// Batched: one workgroup per scene.
__global__ __launch_bounds__(1024) void plan_batch_kernel(const PlanArgs* __restrict__ args) {
    __shared__ int sh[1024];
    __shared__ int last[6];
    const PlanArgs a = args[blockIdx.x];
    plan_block(a, sh, last);
}

// Merges the per-scene problem tables of a batch: scene i's first-contraction
// entries (first_off[i] .. first_off[i+1]) and its second-contraction entry get
// the tile offset of every scene before it; writes the batch tile totals, clears
// the two work-queue counters, and writes the prefix of the scenes' panel work
// units (scene_units[n_scenes] = their total).
__global__ __launch_bounds__(1024) void batch_prefix_kernel(const PlanHeader* __restrict__ hdrs,
                                                            int n_scenes,
                                                            const int* __restrict__ first_off,
                                                            NtEntry* __restrict__ first,
                                                            NtEntry* __restrict__ second,
                                                            int* __restrict__ counts,
                                                            int* __restrict__ queues,
                                                            int* __restrict__ scene_units) {
    __shared__ int sh[1024];
    __shared__ int last[3];
    int run1 = 0, run2 = 0, run3 = 0;
    for (int base = 0; base < n_scenes; base += 1024) {
        const int i = base + (int)threadIdx.x;
        const int v1 = i < n_scenes ? hdrs[i].first_tiles : 0;
        const int v2 = i < n_scenes ? hdrs[i].second_tiles : 0;
        const int v3 = i < n_scenes ? hdrs[i].panel_units : 0;
        const int c1 = block_scan_incl(v1, sh);
        const int c2 = block_scan_incl(v2, sh);
        const int c3 = block_scan_incl(v3, sh);
        if (i < n_scenes) {
            const int o1 = run1 + c1 - v1;
            for (int e = first_off[i]; e < first_off[i + 1]; ++e) first[e].tile_begin += o1;
            second[i].tile_begin = run2 + c2 - v2;
            scene_units[i] = run3 + c3 - v3;
        }
        if (threadIdx.x == blockDim.x - 1) {
            last[0] = c1;
            last[1] = c2;
            last[2] = c3;
        }
        __syncthreads();
        run1 += last[0];
        run2 += last[1];
        run3 += last[2];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        counts[0] = run1;
        counts[1] = run2;
        queues[0] = 0;
        queues[1] = 0;
        scene_units[n_scenes] = run3;
    }
}

// Fringe operands through LDS.  Column k' of a fringe operand is a contiguous slice
// of a 1D fringe table (row y reads entry y - j 2^l + n for the k'-th active row or
// column j).  A task is kFringeRows rows x one 16-wide K block: the workgroup reads
// the table with the lanes along the rows (one contiguous run per k'), keeps the
// tile in LDS (row pitch 17 floats: the LDS stores of each table read hit 64
// different banks; the chunk reads that follow can pair up on a bank), and writes
// the tile's K-blocked storage -- 256 rows x 16 elements, contiguous -- with
// consecutive lanes on consecutive 4-element chunks.
constexpr int kFringePitch = 17;

template <int P>
__device__ __forceinline__ void fringe_task(const float* __restrict__ lutl, int len,
                                            const int* __restrict__ list, int count, int half,
                                            int l, int n, void* panel, size_t ps, size_t base,
                                            int task, float* lre, float* lim) {
    const int tid = threadIdx.x;
    const int ytiles = (n + kFringeRows - 1) / kFringeRows;
    const int kb = task / ytiles, y0 = (task - kb * ytiles) * kFringeRows;
    // every read is issued before the first is used: clamped, in-bounds addresses
    // (rows past n are never stored; k' past count store zero) instead of a branch
    // around each read, which serialised a thread's 32 reads into 16 round trips
    const int y = min(y0 + tid, n - 1);
    // the K block's 16 list entries: one load across the wave, then each is
    // broadcast from its lane (a read per entry waited for its value first)
    const int mine = list[min(16 * kb + (tid & 15), count - 1)];
    float re[16], im[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        const int r = __builtin_amdgcn_readlane(mine, q);
        const int band = r >= half, j = r - band * half;
        const float* tb = lutl + (size_t)band * 2 * len;
        const int idx = y - (j << l) + n;
        re[q] = tb[idx];
        im[q] = tb[len + idx];
    }
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        const bool live = 16 * kb + q < count;
        lre[tid * kFringePitch + q] = live ? re[q] : 0.f;
        lim[tid * kFringePitch + q] = live ? im[q] : 0.f;
    }
    __syncthreads();
    // chunk c = 4 elements: row c / 4 of the tile, k' 4 (c % 4) .. + 3
    const size_t tile = base + ((size_t)kb * n + y0) * 16;
#pragma unroll
    for (int s4 = 0; s4 < 4; ++s4) {
        const int c = s4 * kFringeRows + tid, row = c >> 2, k4 = (c & 3) * 4;
        if (y0 + row < n) {
            float vr[4], vi[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                vr[q] = lre[row * kFringePitch + k4 + q];
                vi[q] = lim[row * kFringePitch + k4 + q];
            }
            put_c4<P>(panel, ps, tile + 4 * (size_t)c, vr, vi);
        }
    }
    __syncthreads();
}

// One (layer, level) as the planning kernel left it.
struct DlPlan {
    int d, l, cr, cc, cf, seg;
};

__device__ __forceinline__ DlPlan load_dl(const NtBuffers& b, int levels, int dl) {
    DlPlan g;
    g.d = dl / levels;
    g.l = dl - g.d * levels + 1;
    g.cr = b.cnt_row[dl];
    g.cc = b.cnt_col[dl];
    g.cf = b.orient[dl];
    g.seg = b.seg_row[dl];
    return g;
}

// A fringe operand of one (layer, level): its table, list and destination.
struct FringeOp {
    const float* lut;
    const int* list;
    void* panel;
    size_t ps, base;
    int len, count, half, n;
};

// The x fringes of the active columns (nx rows) or the y fringes of the active rows.
__device__ __forceinline__ FringeOp fringe_op(const PrepScene& sc, int levels, const DlPlan& g,
                                              bool x_axis, void* panel, size_t ps, size_t base) {
    FringeOp f;
    f.n = x_axis ? sc.nx : sc.ny;
    f.len = lut_len(f.n);
    f.lut = (x_axis ? sc.lut_x : sc.lut_y) + lut_table(g.d, g.l, 0, 0, levels) * f.len;
    f.list = x_axis ? sc.b.collist + dl_cols_off(sc.nx, levels, g.d, g.l)
                    : sc.b.rowlist + dl_rows_off(sc.ny, levels, g.d, g.l);
    f.count = x_axis ? g.cc : g.cr;
    f.half = f.n >> g.l;
    f.panel = panel;
    f.ps = ps;
    f.base = base;
    return f;
}

// The second contraction's fringe operand: rows-first, the y fringes of the active
// rows (Fy_c, ny rows) at the level's k' segment of the A panel; columns-first,
// the x fringes of the active columns (nx rows) at its segment of the B panel (the
// first contraction fills the other operand's segment).
__device__ __forceinline__ FringeOp second_fringe(const PrepScene& sc, int levels,
                                                  const DlPlan& g) {
    const size_t seg = (size_t)g.seg;
    return g.cf ? fringe_op(sc, levels, g, true, sc.b.tc, sc.b.tc_ps, seg * sc.nx)
                : fringe_op(sc, levels, g, false, sc.b.fy, sc.b.fy_ps, seg * sc.ny);
}
// The first contraction's fringe operand: rows-first, the x fringes of the active
// columns (Fx_c, nx rows); columns-first, the y fringes of the active rows.
__device__ __forceinline__ FringeOp first_fringe(const PrepScene& sc, int levels,
                                                 const DlPlan& g) {
    const size_t base = dl_fx_off(sc.ny, sc.nx, levels, g.d, g.l);
    return fringe_op(sc, levels, g, !g.cf, sc.b.fx, sc.b.fx_ps, base);
}

template <int P>
__device__ __forceinline__ void run_fringe_task(const FringeOp& f, int l, int task, float* lre,
                                                float* lim) {
    fringe_task<P>(f.lut, f.len, f.list, f.count, f.half, l, f.n, f.panel, f.ps, f.base, task,
                   lre, lim);
}

// Chunk e4 (four consecutive k' of one row, in storage order) of the coefficient
// operand of the first contraction: Cb_c (active rows x padded active columns)
// rows-first, its transpose (active columns x padded active rows) columns-first.
template <int P>
__device__ __forceinline__ void cb_chunk(const PrepScene& sc, int levels, const DlPlan& g,
                                         float scale, long long e4) {
    const NtBuffers& b = sc.b;
    const int ny = sc.ny, nx = sc.nx, l = g.l;
    const bool cf = g.cf != 0;
    const int rows = cf ? g.cc : g.cr, kn = cf ? g.cr : g.cc;
    const int nyl = ny >> l, nxl = nx >> l;
    // the coefficient stage wrote only the blocks that hold a pixel of the layer:
    // a level-l coefficient at quadrant position (i, j) covers block
    // (i >> (levels - l), j >> (levels - l)) of 2^levels pixels
    const int nbx = nx >> levels, sh = levels - l;
    const uint8_t* oc = b.occ + (size_t)g.d * (size_t)(ny >> levels) * nbx;
    const int* rl = b.rowlist + dl_rows_off(ny, levels, g.d, l);
    const int* cl = b.collist + dl_cols_off(nx, levels, g.d, l);
    const float* cd = sc.coef + (size_t)g.d * ny * nx;
    const size_t e = (size_t)e4 * 4;
    int pr, k0;
    kblk_pos(e, rows, pr, k0);
    // reads issued together on clamped, in-bounds indices; the selects below zero
    // the padding k', the low-low quadrant of a level below the top (it belongs to
    // the coarser levels) and blocks without the layer
    int r[4], j[4];
    float c[4];
    uint8_t o[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int k = min(k0 + q, kn - 1);
        r[q] = rl[cf ? k : pr];
        j[q] = cl[cf ? pr : k];
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int brow = (r[q] < nyl ? r[q] : r[q] - nyl) >> sh;
        const int bcol = (j[q] < nxl ? j[q] : j[q] - nxl) >> sh;
        o[q] = oc[(size_t)brow * nbx + bcol];
        c[q] = cd[(size_t)r[q] * nx + j[q]];
    }
    float v[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const bool keep = k0 + q < kn && !(l < levels && r[q] < nyl && j[q] < nxl) && o[q];
        v[q] = keep ? c[q] * scale : 0.f;
    }
    put_r4<P>(b.cb, b.cb_ps, dl_cb_off(ny, nx, levels, g.d, l) + e, v);
}

__device__ __forceinline__ long long cb_chunks(const DlPlan& g) {
    return g.cf ? (long long)g.cc * pad_kt(g.cr) / 4 : (long long)g.cr * pad_kt(g.cc) / 4;
}

// The operand panels of one scene in one launch: grid.z selects the panel (0 the
// second contraction's fringe operand, 1 the coefficient operand, 2 the first
// contraction's fringe operand where that contraction does not generate it from the
// tables itself), grid.y the (layer, level), grid.x strides over its tasks or chunks.
// The dispatcher hands out the workgroups in that order, so those resident at one
// time write neighbouring parts of one panel.  The grid is sized for dense upper
// bounds, and a workgroup with nothing to do still holds its LDS until its counts
// arrive, so grid.x shares about kPanelGridTotal workgroups among the (layer, level)
// and panel pairs (at 2048^2 x 8 layers with all three panels, 72 pairs: 512 per pair
// measured 85 us, 128 measured 63 us, 32 measured 82 us).
template <int P>
__global__ __launch_bounds__(256) void panels_kernel(PrepScene sc, int levels) {
    __shared__ float lre[kFringeRows * kFringePitch], lim[kFringeRows * kFringePitch];
    const DlPlan g = load_dl(sc.b, levels, blockIdx.y);
    if (g.cr == 0 || g.cc == 0) return;
    if (blockIdx.z != 1) {
        const FringeOp f = blockIdx.z == 0 ? second_fringe(sc, levels, g)
                                           : first_fringe(sc, levels, g);
        const int tasks = (f.n + kFringeRows - 1) / kFringeRows * (pad_kt(f.count) / kKT);
        for (int t = blockIdx.x; t < tasks; t += gridDim.x)
            run_fringe_task<P>(f, g.l, t, lre, lim);
    } else {
        const float scale = sc.b.hdr->cb_scale;  // written by the planning kernel
        const long long total4 = cb_chunks(g);
        for (long long e4 = (long long)blockIdx.x * blockDim.x + threadIdx.x; e4 < total4;
             e4 += (long long)gridDim.x * blockDim.x)
            cb_chunk<P>(sc, levels, g, scale, e4);
    }
}

// Number of entries of the non-decreasing a[0..n) that are <= v (a prefix of it),
// counted by the whole workgroup.
__device__ __forceinline__ int count_le(const int* __restrict__ a, int n, int v) {
    int count = 0;
    for (int base = 0; base < n; base += blockDim.x) {
        const int i = base + (int)threadIdx.x;
        const int c = __syncthreads_count(i < n && a[i] <= v);
        count += c;
        if (c < (int)blockDim.x) break;
    }
    return count;
}

// Batched panels.  Every scene's planning kernel numbers its panel work in a unit
// table, kind-major (entry k D L + t starts kind k of (layer, level) t: every
// (layer, level)'s second-contraction fringe tasks, then the first contraction's,
// then the coefficient units of kCbUnit elements), and scene_units numbers the
// scenes' units one after the other.  Workgroup w takes units w, w + grid,
// w + 2 grid, ...: no workgroup is launched for an empty scene, (layer, level) or
// panel (a dense grid of upper bounds over 64 scenes of uneven size launched
// about 150 thousand mostly idle workgroups), and the ones resident at one time
// take neighbouring units.
template <int P>
__global__ __launch_bounds__(256) void panels_batch_kernel(const PrepScene* __restrict__ scenes,
                                                           int n_scenes, int levels,
                                                           const int* __restrict__ scene_units) {
    __shared__ float lre[kFringeRows * kFringePitch], lim[kFringeRows * kFringePitch];
    const int total = scene_units[n_scenes];
    for (int u = blockIdx.x; u < total; u += gridDim.x) {
        const int i = count_le(scene_units, n_scenes, u) - 1;
        const PrepScene& sc = scenes[i];
        const int v = u - scene_units[i], n_dl = sc.layers * levels;
        const int p = count_le(sc.b.units, 3 * n_dl, v) - 1;
        const int kind = p / n_dl, dl = p - kind * n_dl, local = v - sc.b.units[p];
        const DlPlan g = load_dl(sc.b, levels, dl);
        if (kind < 2) {
            const FringeOp f = kind == 0 ? second_fringe(sc, levels, g)
                                         : first_fringe(sc, levels, g);
            run_fringe_task<P>(f, g.l, local, lre, lim);
        } else {
            const long long e4 = (long long)local * (kCbUnit / 4) + threadIdx.x;
            if (e4 < cb_chunks(g)) cb_chunk<P>(sc, levels, g, sc.b.hdr->cb_scale, e4);
        }
    }
}

// Workgroups of the single-scene launch, shared among its (layer, level) and panel
// pairs (each pair between 32 and 512).
constexpr int kPanelGridTotal = 9216;
// Workgroups of the batched launch: four per CU (the LDS tile bounds residency).
constexpr int kPanelGrid = 1024;

int panel_grid(long long units_bound) {
    return (int)(units_bound < 1 ? 1 : (units_bound < kPanelGrid ? units_bound : kPanelGrid));
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
    a.units = b.units;
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
    a.koff_row = b.koff_row;
    a.koff_col = b.koff_col;
    a.gen_x = b.gen_x;
    a.gen_y = b.gen_y;
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
                       flags_layer, b.rowlist, b.collist, b.cnt_row, b.cnt_col, b.koff_row,
                       b.koff_col);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    PlanArgs a = make_plan_args(ny, nx, layers, levels, precision, tiles, b, o, absmax,
                                e_fringe);
    a.units = nullptr;  // the single-scene gather does not number its work
    // one wave scans up to 64 (layer, level) pairs without a workgroup barrier's cost
    hipLaunchKernelGGL(plan_kernel, dim3(1), dim3(n_dl <= 64 ? 64 : 1024), 0, s, a);
    return hipGetLastError();
}

template <int P>
static hipError_t materialize(const float* coef, const float* lut_x, const float* lut_y, int ny,
                              int nx, int layers, int levels, const NtBuffers& b, bool first_panel,
                              hipStream_t s) {
    PrepScene sc{};
    sc.coef = coef;
    sc.lut_x = lut_x;
    sc.lut_y = lut_y;
    sc.ny = ny;
    sc.nx = nx;
    sc.layers = layers;
    sc.b = b;
    // workgroups per (layer, level) and panel: the share of kPanelGridTotal, at most
    // the largest dense task or chunk count of one (layer, level)
    long long most = 1;
    for (int l = 1; l <= levels; ++l) {
        int u[3];
        dl_panel_units(ny, nx, band_side(ny, l), band_side(nx, l), u);
        const long long fringe = u[0] > u[1] ? u[0] : u[1];
        const long long chunks = ((long long)u[2] * kCbUnit / 4 + 255) / 256;
        if (fringe > most) most = fringe;
        if (chunks > most) most = chunks;
    }
    const int kinds = first_panel ? 3 : 2;
    int share = kPanelGridTotal / (kinds * layers * levels);
    share = share < 32 ? 32 : (share > 512 ? 512 : share);
    const int gx = (int)(most < share ? most : share);
    hipLaunchKernelGGL(panels_kernel<P>, dim3(gx, layers * levels, kinds), dim3(256), 0, s, sc,
                       levels);
    return hipGetLastError();
}

template <int P>
static void materialize_batch(const PrepScene* scenes, int n, int levels, const int* scene_units,
                              long long units_bound, hipStream_t s) {
    hipLaunchKernelGGL(panels_batch_kernel<P>, dim3(panel_grid(units_bound)), dim3(256), 0, s,
                       scenes, n, levels, scene_units);
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
                                    const int* scene_units, long long units_bound,
                                    hipStream_t s) {
    if (precision == P_BF16) materialize_batch<P_BF16>(scenes, n, levels, scene_units, units_bound, s);
    else if (precision == P_FP16) materialize_batch<P_FP16>(scenes, n, levels, scene_units, units_bound, s);
    else materialize_batch<P_FP32>(scenes, n, levels, scene_units, units_bound, s);
    return hipGetLastError();
}

hipError_t launch_batch_prefix(const PlanHeader* hdrs, int n_scenes, const int* first_off,
                               NtEntry* first, NtEntry* second, int* counts, int* queues,
                               int* scene_units, hipStream_t s) {
    hipLaunchKernelGGL(batch_prefix_kernel, dim3(1), dim3(1024), 0, s, hdrs, n_scenes, first_off,
                       first, second, counts, queues, scene_units);
    return hipGetLastError();
}

hipError_t launch_nt_materialize(const float* coef, const float* lut_x, const float* lut_y, int ny,
                                 int nx, int layers, int levels, int precision,
                                 const NtBuffers& b, bool first_panel, hipStream_t s) {
    if (precision == P_BF16)
        return materialize<P_BF16>(coef, lut_x, lut_y, ny, nx, layers, levels, b, first_panel, s);
    if (precision == P_FP16)
        return materialize<P_FP16>(coef, lut_x, lut_y, ny, nx, layers, levels, b, first_panel, s);
    return materialize<P_FP32>(coef, lut_x, lut_y, ny, nx, layers, levels, b, first_panel, s);
}

}  // namespace cgh
