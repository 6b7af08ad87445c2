// Batched plans: many scenes of uneven size planned, tuned and captured as one
// unit.  Every stage of cgh_progressive_hologram (coefficients, fringe tables,
// active lists, plans, panels) runs as one launch over every scene, driven by
// device-resident per-scene tables written at plan creation; the contraction
// problems of all scenes are merged into one table per contraction and each
// contraction runs as a single persistent launch over that table.  Tile shapes
// come from an autotuner (timed on this batch, cached as JSON lines).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <string>
#include <vector>

#include "host.h"

using namespace cgh::host;

struct cgh_plan {
    struct Scene {
        cgh_scene s;
        std::vector<double> z;
        size_t ws_off;
        cgh::Layout lo;
        int first_off;
        int e_fringe = 0;  // FP16 range scaling of the scene's y fringe tables (2^-e)
    };
    int levels = 3, precision = 0;
    unsigned flags = 0;
    double lambda = 0, pitch = 0;
    float thr[CGH_MAX_LEVELS] = {};
    std::vector<Scene> scenes;  // execution order: largest first
    char* mem = nullptr;
    size_t bytes = 0;
    cgh::NtEntry* first = nullptr;
    cgh::NtEntry* second = nullptr;
    int n_first = 0;
    cgh::PlanHeader* hdrs = nullptr;
    int* first_off = nullptr;
    int* scene_units = nullptr;  // [n + 1] prefix of the scenes' panel work units
    long long units_bound = 0;   // upper bound of their total (sizes the panel grid)
    int* counts = nullptr;
    int* queues = nullptr;
    int tiles[4] = {cgh::kNtTile, cgh::kNtTile, cgh::kNtTile, cgh::kNtTile};
    int grid = 512;
    int from_cache = 0;
    double ms_first = 0, ms_second = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    // batched preparation: device tables and the extents of the largest scene
    cgh::DwtScene* d_dwt = nullptr;
    cgh::PrepScene* d_prep = nullptr;
    cgh::LutJob* d_luts = nullptr;
    cgh::PlanArgs* d_args = nullptr;
    std::vector<cgh::PrepScene> h_prep;
    std::vector<cgh::PlanArgs> h_args;
    int n_luts = 0, max_nbx = 0, max_nby = 0, max_ndl = 0, max_len = 0;
    size_t max_fill = 0;
};

namespace {

constexpr int kMaxScenes = 4096;
constexpr int kCandidates[4][2] = {{128, 128}, {64, 128}, {128, 64}, {64, 64}};

struct Events {
    hipEvent_t a = nullptr, b = nullptr, c = nullptr;
};
// (a: before the operand-panel gather, whose work depends on the first contraction's
// tile shape; b: between the contractions; c: after the second)

// Every per-scene stage of the batch as one launch over all scenes, then the
// merge of the problem tables.  The planning arguments (tile shapes included)
// are the ones last uploaded by upload_args.
hipError_t enqueue_prep(const cgh_plan& p, hipStream_t s, const Events* ev = nullptr) {
    const int n = (int)p.scenes.size();
    hipError_t e = cgh::launch_prep_fill(p.d_dwt, n, p.max_fill, s);
    if (e == hipSuccess)
        e = cgh::launch_dwt_mask_batch(p.d_dwt, n, p.levels, p.thr, p.max_nbx, p.max_nby, s);
    if (e == hipSuccess) e = cgh::launch_luts_batch(p.d_luts, p.n_luts, p.max_len, p.levels, s);
    if (e == hipSuccess) e = cgh::launch_lists_batch(p.d_prep, n, p.levels, p.max_ndl, s);
    if (e == hipSuccess) e = cgh::launch_plan_batch(p.d_args, n, p.max_ndl, s);
    if (e == hipSuccess)
        e = cgh::launch_batch_prefix(p.hdrs, n, p.first_off, p.first, p.second, p.counts,
                                     p.queues, p.scene_units, s);
    if (e == hipSuccess && ev) e = hipEventRecord(ev->a, s);
    if (e != hipSuccess) return e;
    return cgh::launch_materialize_batch(p.d_prep, n, p.levels, p.precision, p.scene_units,
                                         p.units_bound, s);
}

// Planning arguments of every scene for the given tile shapes (synchronous).
hipError_t upload_args(cgh_plan& p, const int* tiles, hipStream_t s) {
    p.h_args.resize(p.scenes.size());
    for (size_t i = 0; i < p.scenes.size(); ++i) {
        const cgh_plan::Scene& sc = p.scenes[i];
        const cgh::NtOutput o{reinterpret_cast<float2*>(sc.s.hologram), nullptr, 0};
        const auto* absmax = reinterpret_cast<const unsigned long long*>(p.mem + sc.ws_off +
                                                                         sc.lo.ops) + kAbsmaxWord;
        p.h_args[i] = cgh::make_plan_args(sc.s.ny, sc.s.nx, sc.s.n_layers, p.levels, p.precision,
                                          tiles, p.h_prep[i].b, o, absmax, sc.e_fringe);
    }
    hipError_t e = hipMemcpyAsync(p.d_args, p.h_args.data(), p.h_args.size() * sizeof(cgh::PlanArgs),
                                  hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    return e;
}

hipError_t enqueue_first(const cgh_plan& p, hipStream_t s, const int* tiles) {
    // only the generating shapes: the plan's layout has no fringe panel for this operand
    if (!cgh::nt_first_generates(tiles[1])) return hipErrorInvalidValue;
    return cgh::launch_nt_persistent(false, p.precision, tiles[0], tiles[1], p.first, p.n_first,
                                     p.counts, p.queues, p.grid, s);
}

// The split forms' second contraction may also take the one-workgroup-per-CU
// ring kernel (a direct launch over every scene's tiles); the autotuner decides.
bool ring_second(const cgh_plan& p, const int* tiles) {
    return p.precision != CGH_FP32 && tiles[2] == cgh::nt_ring_tile_m() &&
           tiles[3] == cgh::nt_ring_tile_n();
}

hipError_t enqueue_second(const cgh_plan& p, hipStream_t s, const int* tiles) {
    if (ring_second(p, tiles)) {
        int max_tiles = 0;
        for (const auto& sc : p.scenes)
            max_tiles += cgh::nt_tiles(sc.s.ny, sc.s.nx, tiles[2], tiles[3]);
        return cgh::launch_nt_ring_table(p.precision, p.second, (int)p.scenes.size(), p.counts + 1,
                                         max_tiles, s);
    }
    return cgh::launch_nt_persistent(true, p.precision, tiles[2], tiles[3], p.second,
                                     (int)p.scenes.size(), p.counts + 1, p.queues + 1, p.grid, s);
}

// Enqueues the whole batch on `s` with the given tile shapes (the planning
// arguments must have been uploaded for them); records ev (if given) before the
// operand-panel gather (with 128-column first tiles the first contraction generates its
// fringe operand and the gather does less), between the contractions, and after the
// second.
hipError_t enqueue(const cgh_plan& p, hipStream_t s, const int* tiles, const Events* ev) {
    hipError_t e = enqueue_prep(p, s, ev);
    if (e == hipSuccess) e = enqueue_first(p, s, tiles);
    if (e == hipSuccess && ev) e = hipEventRecord(ev->b, s);
    if (e == hipSuccess) e = enqueue_second(p, s, tiles);
    if (e == hipSuccess && ev) e = hipEventRecord(ev->c, s);
    return e;
}

std::string arch_name() {
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess)
        return "unknown";
    std::string a = prop.gcnArchName;
    const size_t colon = a.find(':');
    return colon == std::string::npos ? a : a.substr(0, colon);
}

// Batch signature: architecture, precision, levels and the sorted scene shapes.
std::string tune_key(const cgh_plan& p) {
    std::vector<std::string> shapes;
    for (const auto& sc : p.scenes)
        shapes.push_back(std::to_string(sc.s.ny) + "x" + std::to_string(sc.s.nx) + "x" +
                         std::to_string(sc.s.n_layers));
    std::sort(shapes.begin(), shapes.end());
    std::string k = arch_name() + "/p" + std::to_string(p.precision) + "/L" + std::to_string(p.levels) + "/";
    for (size_t i = 0; i < shapes.size(); ++i) k += (i ? "," : "") + shapes[i];
    return k;
}

// Cache file: one JSON object per line,
// {"key": "...", "first": [tm, tn], "second": [tm, tn], "ms_first": x, "ms_second": y}
bool cache_lookup(const char* path, const std::string& key, bool split_form, int* tiles) {
    if (!path) return false;
    std::ifstream f(path);
    std::string line;
    const std::string want = "\"key\": \"" + key + "\"";
    while (std::getline(f, line)) {
        if (line.find(want) == std::string::npos) continue;
        const size_t a = line.find("\"first\": [");
        const size_t b = line.find("\"second\": [");
        if (a == std::string::npos || b == std::string::npos) continue;
        int t[4];
        if (std::sscanf(line.c_str() + a, "\"first\": [%d, %d]", &t[0], &t[1]) != 2) continue;
        if (std::sscanf(line.c_str() + b, "\"second\": [%d, %d]", &t[2], &t[3]) != 2) continue;
        bool ok = true;
        for (int q = 0; q < 2; ++q) {
            bool found = false;
            for (const auto& c : kCandidates) found |= (c[0] == t[2 * q] && c[1] == t[2 * q + 1]);
            // the ring shape, second contraction of the split forms only
            found |= q == 1 && split_form && t[2] == cgh::nt_ring_tile_m() && t[3] == cgh::nt_ring_tile_n();
            ok &= found;
        }
        // the batch's first contraction generates its fringe operand: 128-column tiles
        // only (a plan holds no room for that operand's panel)
        if (!ok || !cgh::nt_first_generates(t[1])) continue;
        for (int q = 0; q < 4; ++q) tiles[q] = t[q];
        return true;
    }
    return false;
}

void cache_store(const char* path, const std::string& key, const int* tiles, double ms1, double ms2) {
    if (!path) return;
    std::ofstream f(path, std::ios::app);
    char buf[160];
    std::snprintf(buf, sizeof(buf),
                  "\", \"first\": [%d, %d], \"second\": [%d, %d], \"ms_first\": %.4f, \"ms_second\": %.4f}\n",
                  tiles[0], tiles[1], tiles[2], tiles[3], ms1, ms2);
    f << "{\"key\": \"" << key << buf;
}

// Times every candidate shape on this batch and keeps the fastest per contraction;
// the split forms also time the ring kernel for the second contraction.  The first
// contraction takes the candidates' row counts with 128-column tiles only: with them it
// generates its fringe operand, and a plan holds no room for that operand's panel.
hipError_t autotune(cgh_plan& p, hipStream_t s) {
    Events ev;
    hipError_t e = hipEventCreate(&ev.a);
    if (e == hipSuccess) e = hipEventCreate(&ev.b);
    if (e == hipSuccess) e = hipEventCreate(&ev.c);
    double best1 = 1e30, best2 = 1e30;
    for (const auto& c : kCandidates) {
        if (e != hipSuccess) break;
        const int tiles[4] = {c[0], 128, c[0], c[1]};
        e = upload_args(p, tiles, s);
        double t1 = 1e30, t2 = 1e30;
        for (int rep = 0; rep < 3 && e == hipSuccess; ++rep) {  // first run warms up
            e = enqueue(p, s, tiles, &ev);
            if (e == hipSuccess) e = hipEventSynchronize(ev.c);
            float m1 = 0.f, m2 = 0.f;
            if (e == hipSuccess) e = hipEventElapsedTime(&m1, ev.a, ev.b);
            if (e == hipSuccess) e = hipEventElapsedTime(&m2, ev.b, ev.c);
            if (rep > 0) {
                t1 = std::min(t1, (double)m1);
                t2 = std::min(t2, (double)m2);
            }
        }
        if (t1 < best1) { best1 = t1; p.tiles[0] = tiles[0]; p.tiles[1] = tiles[1]; }
        if (t2 < best2) { best2 = t2; p.tiles[2] = c[0]; p.tiles[3] = c[1]; }
    }
    if (e == hipSuccess && p.precision != CGH_FP32) {
        // the ring kernel for the second contraction, with the first's best shape
        const int tiles[4] = {p.tiles[0], p.tiles[1], cgh::nt_ring_tile_m(), cgh::nt_ring_tile_n()};
        e = upload_args(p, tiles, s);
        double t2 = 1e30;
        for (int rep = 0; rep < 3 && e == hipSuccess; ++rep) {
            e = enqueue(p, s, tiles, &ev);
            if (e == hipSuccess) e = hipEventSynchronize(ev.c);
            float m2 = 0.f;
            if (e == hipSuccess) e = hipEventElapsedTime(&m2, ev.b, ev.c);
            if (rep > 0) t2 = std::min(t2, (double)m2);
        }
        if (t2 < best2) { best2 = t2; p.tiles[2] = tiles[2]; p.tiles[3] = tiles[3]; }
    }
    if (ev.a) (void)hipEventDestroy(ev.a);
    if (ev.b) (void)hipEventDestroy(ev.b);
    if (ev.c) (void)hipEventDestroy(ev.c);
    p.ms_first = best1;
    p.ms_second = best2;
    return e;
}

void release(cgh_plan* p) {
    if (!p) return;
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    if (p->mem) (void)hipFree(p->mem);
    delete p;
}

}  // namespace

extern "C" {

int cgh_plan_create(const cgh_scene* scenes, int n_scenes, int levels, double lambda, double pitch,
                    const float* thresholds, int precision, unsigned flags,
                    const char* tune_cache_path, void* stream, cgh_plan** plan) {
    if (!plan) return CGH_ERROR_INVALID_VALUE;
    *plan = nullptr;
    try {
        if (!scenes || n_scenes < 1 || n_scenes > kMaxScenes) return CGH_ERROR_INVALID_VALUE;
        if (flags & CGH_FLAG_ACCUMULATE) return CGH_ERROR_INVALID_VALUE;
        cgh_plan* p = new cgh_plan();
        p->levels = levels;
        p->precision = precision;
        p->flags = flags;
        p->lambda = lambda;
        p->pitch = pitch;
        // validate every scene on the host before touching the device
        for (int i = 0; i < n_scenes; ++i) {
            const cgh_scene& sc = scenes[i];
            int st = check_common(sc.n_layers, sc.layer_index, sc.z, thresholds, lambda, pitch,
                                  sc.ny, sc.nx, levels, precision, flags, p->thr);
            if (!st && (sc.ny == 0 || sc.nx == 0)) continue;  // empty scene: nothing to do
            if (!st && (!sc.object || !sc.hologram)) st = CGH_ERROR_INVALID_VALUE;
            if (st) {
                delete p;
                return st;
            }
            cgh_plan::Scene rec{};
            rec.s = sc;
            rec.z.assign(sc.z, sc.z + sc.n_layers);
            rec.lo = make_layout(sc.ny, sc.nx, sc.n_layers, levels, LayoutUse::kBatch);
            p->scenes.push_back(rec);
        }
        if (p->scenes.empty()) {
            delete p;
            return CGH_ERROR_INVALID_VALUE;
        }
        // largest scenes first: their tiles enter the work queues early
        std::stable_sort(p->scenes.begin(), p->scenes.end(), [](const auto& a, const auto& b) {
            const double ca = (double)a.s.ny * a.s.nx * (a.s.ny + a.s.nx) * a.s.n_layers;
            const double cb = (double)b.s.ny * b.s.nx * (b.s.ny + b.s.nx) * b.s.n_layers;
            return ca > cb;
        });
        size_t off = 0;
        int n_first = 0;
        for (auto& sc : p->scenes) {
            sc.ws_off = off;
            off = align_up(off + sc.lo.total);
            sc.first_off = n_first;
            n_first += sc.s.n_layers * levels;
        }
        const int n = (int)p->scenes.size();
        p->n_first = n_first;
        const size_t first_b = align_up((size_t)n_first * sizeof(cgh::NtEntry));
        const size_t second_b = align_up((size_t)n * sizeof(cgh::NtEntry));
        const size_t hdr_b = align_up((size_t)n * sizeof(cgh::PlanHeader));
        const size_t off_b = align_up((size_t)(n + 1) * sizeof(int));
        int n_luts = 0;
        for (const auto& sc : p->scenes) n_luts += 2 * sc.s.n_layers;
        p->n_luts = n_luts;
        const size_t dwt_b = align_up((size_t)n * sizeof(cgh::DwtScene));
        const size_t prep_b = align_up((size_t)n * sizeof(cgh::PrepScene));
        const size_t luts_b = align_up((size_t)n_luts * sizeof(cgh::LutJob));
        const size_t args_b = align_up((size_t)n * sizeof(cgh::PlanArgs));
        p->bytes = off + first_b + second_b + hdr_b + 2 * off_b + align_up(4 * sizeof(int)) +
                   dwt_b + prep_b + luts_b + args_b;

        const char* fail = std::getenv("CGH_TEST_FAIL_ALLOC");  // host-forced failure for tests
        if (fail && fail[0] == '1') {
            delete p;
            return CGH_ERROR_OUT_OF_MEMORY;
        }
        if (hipMalloc(reinterpret_cast<void**>(&p->mem), p->bytes) != hipSuccess) {
            (void)hipGetLastError();
            p->mem = nullptr;
            release(p);
            return CGH_ERROR_OUT_OF_MEMORY;
        }
        char* m = p->mem + off;
        p->first = reinterpret_cast<cgh::NtEntry*>(m);
        m += first_b;
        p->second = reinterpret_cast<cgh::NtEntry*>(m);
        m += second_b;
        p->hdrs = reinterpret_cast<cgh::PlanHeader*>(m);
        m += hdr_b;
        p->first_off = reinterpret_cast<int*>(m);
        m += off_b;
        p->scene_units = reinterpret_cast<int*>(m);
        m += off_b;
        p->counts = reinterpret_cast<int*>(m);
        p->queues = p->counts + 2;
        m += align_up(4 * sizeof(int));
        p->d_dwt = reinterpret_cast<cgh::DwtScene*>(m);
        m += dwt_b;
        p->d_prep = reinterpret_cast<cgh::PrepScene*>(m);
        m += prep_b;
        p->d_luts = reinterpret_cast<cgh::LutJob*>(m);
        m += luts_b;
        p->d_args = reinterpret_cast<cgh::PlanArgs*>(m);

        // per-scene tables of the batched preparation
        std::vector<cgh::DwtScene> h_dwt(n);
        std::vector<cgh::LutJob> h_luts;
        h_luts.reserve(n_luts);
        p->h_prep.resize(n);
        Optics op;
        FringeScale fs;
        for (int i = 0; i < n; ++i) {
            const cgh_plan::Scene& sc = p->scenes[i];
            const cgh::Layout& lo = sc.lo;
            char* ws = p->mem + sc.ws_off;
            const int ny = sc.s.ny, nx = sc.s.nx, nl = sc.s.n_layers;
            cgh::NtBuffers nb = nt_buffers(ws, lo);
            nb.first = p->first + sc.first_off;
            nb.second = p->second + i;
            nb.hdr = p->hdrs + i;
            h_dwt[i] = cgh::DwtScene{sc.s.object, sc.s.layer_index, sc.s.saliency, ny, nx, nl,
                                     reinterpret_cast<float*>(ws + lo.coef),
                                     reinterpret_cast<uint8_t*>(ws + lo.flags), lo.flags_layer,
                                     lo.flags_fill,
                                     reinterpret_cast<unsigned long long*>(ws + lo.ops),
                                     reinterpret_cast<uint8_t*>(ws + lo.occ)};
            p->h_prep[i] = cgh::PrepScene{reinterpret_cast<const uint8_t*>(ws + lo.flags),
                                          reinterpret_cast<const float*>(ws + lo.coef),
                                          reinterpret_cast<const float*>(ws + lo.lut_x),
                                          reinterpret_cast<const float*>(ws + lo.lut_y), ny, nx,
                                          nl, lo.flags_layer, nb};
            make_optics(op, nl, sc.z.data(), lambda, pitch, (flags & CGH_FLAG_EQ1_PREFACTOR) != 0);
            fringe_scale(op, nl, p->precision, fs);
            p->scenes[i].e_fringe = fs.e;
            for (int d = 0; d < nl; ++d) {
                h_luts.push_back(cgh::LutJob{nx, d, levels, op.c[d], op.one_re[d], op.one_im[d],
                                             reinterpret_cast<float*>(ws + lo.lut_x),
                                             ws + lo.gen_x, p->precision});
                h_luts.push_back(cgh::LutJob{ny, d, levels, op.c[d], fs.re[d], fs.im[d],
                                             reinterpret_cast<float*>(ws + lo.lut_y),
                                             ws + lo.gen_y, p->precision});
            }
            p->max_nbx = std::max(p->max_nbx, nx >> levels);
            p->max_nby = std::max(p->max_nby, ny >> levels);
            p->max_ndl = std::max(p->max_ndl, nl * levels);
            p->max_len = std::max(p->max_len, cgh::lut_len(std::max(nx, ny)));
            p->max_fill = std::max(p->max_fill, lo.flags_fill);
            p->units_bound += cgh::panel_units_bound(ny, nx, nl, levels);
        }

        hipStream_t s = (hipStream_t)stream;
        std::vector<int> fo(n + 1);
        for (int i = 0; i < n; ++i) fo[i] = p->scenes[i].first_off;
        fo[n] = n_first;
        hipError_t e = hipMemcpyAsync(p->first_off, fo.data(), (n + 1) * sizeof(int),
                                      hipMemcpyHostToDevice, s);
        if (e == hipSuccess)
            e = hipMemcpyAsync(p->d_dwt, h_dwt.data(), n * sizeof(cgh::DwtScene),
                               hipMemcpyHostToDevice, s);
        if (e == hipSuccess)
            e = hipMemcpyAsync(p->d_prep, p->h_prep.data(), n * sizeof(cgh::PrepScene),
                               hipMemcpyHostToDevice, s);
        if (e == hipSuccess)
            e = hipMemcpyAsync(p->d_luts, h_luts.data(), h_luts.size() * sizeof(cgh::LutJob),
                               hipMemcpyHostToDevice, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        int dev = 0;
        hipDeviceProp_t prop;
        if (e == hipSuccess) e = hipGetDevice(&dev);
        if (e == hipSuccess) e = hipGetDeviceProperties(&prop, dev);
        if (e == hipSuccess) p->grid = 2 * prop.multiProcessorCount;  // two resident per CU

        const std::string key = tune_key(*p);
        if (e == hipSuccess) {
            if (cache_lookup(tune_cache_path, key, p->precision != CGH_FP32, p->tiles)) {
                p->from_cache = 1;
            } else {
                e = autotune(*p, s);
                if (e == hipSuccess) cache_store(tune_cache_path, key, p->tiles, p->ms_first, p->ms_second);
            }
        }
        // the final tile shapes, then capture the batch on a private stream
        if (e == hipSuccess) e = upload_args(*p, p->tiles, s);
        hipStream_t cs = nullptr;
        if (e == hipSuccess) e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed);
        if (e == hipSuccess) {
            hipError_t ee = enqueue_prep(*p, cs);
            if (ee == hipSuccess) ee = enqueue_first(*p, cs, p->tiles);
            if (ee == hipSuccess) ee = enqueue_second(*p, cs, p->tiles);
            e = hipStreamEndCapture(cs, &p->graph);
            if (ee != hipSuccess) e = ee;
        }
        if (e == hipSuccess) e = hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0);
        if (cs) (void)hipStreamDestroy(cs);
        if (e != hipSuccess) {
            const int st = hip_status(e);
            release(p);
            return st;
        }
        *plan = p;
        return CGH_SUCCESS;
    } catch (...) {
        return CGH_ERROR_HIP;
    }
}

int cgh_plan_execute(cgh_plan* plan, void* stream) {
    if (!plan || !plan->exec) return CGH_ERROR_INVALID_VALUE;
    hipStream_t s = (hipStream_t)stream;
    bool profiling;
    {
        Profiler& pr = profiler();
        std::lock_guard<std::mutex> g(pr.mu);
        profiling = pr.on;
    }
    if (!profiling) return hip_status(hipGraphLaunch(plan->exec, s));
    // diagnostics: the same kernels launched eagerly, each stage timed on `s`
    const cgh_plan& p = *plan;
    hipError_t e = timed(s, CGH_STAGE_PLAN, [&] { return enqueue_prep(p, s); });
    if (e == hipSuccess) e = timed(s, CGH_STAGE_FIRST, [&] { return enqueue_first(p, s, p.tiles); });
    if (e == hipSuccess) e = timed(s, CGH_STAGE_SECOND, [&] { return enqueue_second(p, s, p.tiles); });
    return hip_status(e);
}

int cgh_plan_get_stats(const cgh_plan* plan, cgh_stats* stats, void* stream) {
    if (!plan || !stats) return CGH_ERROR_INVALID_VALUE;
    try {
        std::memset(stats, 0, sizeof(*stats));
        hipStream_t s = (hipStream_t)stream;
        const int n = (int)plan->scenes.size();
        std::vector<cgh::PlanHeader> hdrs(n);
        hipError_t e = hipMemcpyAsync(hdrs.data(), plan->hdrs, n * sizeof(cgh::PlanHeader),
                                      hipMemcpyDeviceToHost, s);
        std::vector<std::vector<int>> cr(n), cc(n), orient(n);
        std::vector<unsigned long long> ops(4 * (size_t)n, 0ull);
        for (int i = 0; i < n && e == hipSuccess; ++i) {
            const auto& sc = plan->scenes[i];
            const int n_dl = sc.s.n_layers * plan->levels;
            cr[i].resize(n_dl);
            cc[i].resize(n_dl);
            orient[i].resize(n_dl);
            const char* ws = plan->mem + sc.ws_off;
            e = hipMemcpyAsync(cr[i].data(), ws + sc.lo.cnt_row, n_dl * sizeof(int), hipMemcpyDeviceToHost, s);
            if (e == hipSuccess)
                e = hipMemcpyAsync(cc[i].data(), ws + sc.lo.cnt_col, n_dl * sizeof(int), hipMemcpyDeviceToHost, s);
            if (e == hipSuccess)
                e = hipMemcpyAsync(orient[i].data(), ws + sc.lo.orient, n_dl * sizeof(int), hipMemcpyDeviceToHost, s);
            if (e == hipSuccess)
                e = hipMemcpyAsync(ops.data() + 4 * i, ws + sc.lo.ops, 4 * sizeof(unsigned long long),
                                   hipMemcpyDeviceToHost, s);
        }
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return hip_status(e);
        for (int i = 0; i < n; ++i) {
            const auto& sc = plan->scenes[i];
            const double ny = sc.s.ny, nx = sc.s.nx;
            double rc = 0.0;
            for (size_t k = 0; k < cr[i].size(); ++k)
                rc += (double)cr[i][k] * cc[i][k] * (orient[i][k] ? ny : nx);
            long long total = 0;
            for (int l = 1; l <= plan->levels; ++l) total += cgh::band_side(sc.s.ny, l);
            total *= sc.s.n_layers;
            stats->k_active += hdrs[i].k_active;
            stats->k_padded += hdrs[i].kpad;
            stats->k_total += total;
            stats->flops_first += 4.0 * rc;
            stats->flops_second += 8.0 * ny * nx * hdrs[i].k_active;
            stats->flops_second_issued += 8.0 * ny * nx * hdrs[i].kpad;
            const int L = plan->levels;
            stats->operators[0] += (long long)(sc.s.ny >> L) * (sc.s.nx >> L);
            for (int j = 1; j <= L; ++j) stats->operators[j] += (long long)ops[4 * i + L - j];
            stats->operators_pointwise += (long long)sc.s.ny * sc.s.nx;
        }
        stats->k_tile = cgh::kKT;
        stats->split_k = 1;
        return CGH_SUCCESS;
    } catch (...) {
        return CGH_ERROR_HIP;
    }
}

int cgh_plan_destroy(cgh_plan* plan) {
    if (!plan) return CGH_ERROR_INVALID_VALUE;
    release(plan);
    return CGH_SUCCESS;
}

int cgh_plan_get_info(const cgh_plan* plan, cgh_plan_info* info) {
    if (!plan || !info) return CGH_ERROR_INVALID_VALUE;
    info->n_scenes = (int)plan->scenes.size();
    info->first_tile[0] = plan->tiles[0];
    info->first_tile[1] = plan->tiles[1];
    info->second_tile[0] = plan->tiles[2];
    info->second_tile[1] = plan->tiles[3];
    info->from_cache = plan->from_cache;
    info->persistent_grid = plan->grid;
    info->tune_ms_first = plan->from_cache ? 0.0 : plan->ms_first;
    info->tune_ms_second = plan->from_cache ? 0.0 : plan->ms_second;
    info->device_bytes = plan->bytes;
    return CGH_SUCCESS;
}

}  // extern "C"
