// Batched lattice sums, host side: the plan (schedule and device problem table),
// the launch entry point, the autotuner and native HIP-graph capture.
//
// Schedule: problems sorted by cost n * (6 d + 10) descending (longest first), so
// that the persistent workgroups finish the large problems early and the small
// ones fill the tail; tiles are numbered consecutively in that order.
//
// Autotuner: for a plan it times every candidate (points per thread 4/8/16 x
// workgroups per CU 1/2/4/8) on the actual batch with HIP events and keeps the
// fastest.  Results are cached per batch signature in the process and, if the
// environment variable QMC_AUTOTUNE_CACHE names a file, in that file (one line
// per signature), so a later process reuses them without re-timing.
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <numeric>
#include <string>
#include <vector>

#include "batched.hpp"
#include "common.hpp"
#include "kernels.hpp"
#include "qmc.h"
#include "status.hpp"

using qmc::fail;
using qmc::from_hip;
using qmc::ok;

struct qmc_batch_plan {
    int count = 0;
    int precision = 0;
    qmc_batch_config cfg{};
    std::vector<qmc_problem> probs;
    qmc::DevProblem* d_probs = nullptr;
    uint32_t total_tiles = 0;
    int grid = 0;
    size_t ws_bytes = 0;
};

struct qmc_graph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace {

constexpr int kMaxBatch = 200000;
constexpr int kDefaultPoints = 8;
constexpr int kDefaultWpc = 4;

int param_count(int family, int d) {
    switch (family) {
        case QMC_EXP_SUM: return d;
        case QMC_PRODUCT_PEAK:
        case QMC_GAUSSIAN: return 2 * d;
        case QMC_OSCILLATORY: return d + 1;
        case QMC_EXP_QUADRATIC: return 2 * d;
        default: return -1;
    }
}

qmc_status check_config(const qmc_batch_config& c) {
    if (c.points_per_thread != 4 && c.points_per_thread != 8 && c.points_per_thread != 16)
        return fail(QMC_ERR_INVALID_ARG, "points_per_thread = %d is not 4, 8 or 16", c.points_per_thread);
    if (c.workgroups_per_cu < 1 || c.workgroups_per_cu > 8)
        return fail(QMC_ERR_INVALID_ARG, "workgroups_per_cu = %d outside [1, 8]", c.workgroups_per_cu);
    if (c.order != 0 && c.order != 1) return fail(QMC_ERR_INVALID_ARG, "order = %d is not 0 or 1", c.order);
    return QMC_OK;
}

uint64_t tiles_of(int64_t n, int M) { return ((uint64_t)n + 256ull * M - 1) / (256ull * M); }

// Build the schedule and upload the problem table for the plan's configuration.
qmc_status build_tables(qmc_batch_plan* p) {
    const int M = p->cfg.points_per_thread;
    std::vector<int> ord(p->count);
    std::iota(ord.begin(), ord.end(), 0);
    if (p->cfg.order == 0) {
        std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) {
            const double cx = (double)p->probs[x].n * (6.0 * p->probs[x].d + 10.0);
            const double cy = (double)p->probs[y].n * (6.0 * p->probs[y].d + 10.0);
            return cx > cy;
        });
    }
    std::vector<qmc::DevProblem> h(p->count);
    uint64_t t = 0;
    for (int i = 0; i < p->count; ++i) {
        const qmc_problem& q = p->probs[ord[i]];
        qmc::DevProblem& e = h[i];
        e.z = q.z;
        e.params = q.params;
        e.shift = q.shift;
        e.n = (uint32_t)q.n;
        e.d = q.d;
        e.family = q.family;
        e.out_index = ord[i];
        e.inv_n = 1.0 / (double)q.n;
        e.tile_begin = (uint32_t)t;
        e.tiles = (uint32_t)tiles_of(q.n, M);
        t += e.tiles;
    }
    // The queue counter overshoots the tile count by at most the grid size; keeping
    // the count below 2^31 rules out any wrap-around of the 32-bit counter.
    if (t >= (1ull << 31)) return fail(QMC_ERR_UNSUPPORTED, "batch has %llu tiles (limit 2^31)", (unsigned long long)t);
    p->total_tiles = (uint32_t)t;
    if (!p->d_probs) {
        hipError_t e = hipMalloc(&p->d_probs, sizeof(qmc::DevProblem) * (size_t)p->count);
        if (e != hipSuccess) {
            p->d_probs = nullptr;
            return fail(QMC_ERR_OUT_OF_MEMORY, "hipMalloc of the problem table failed (%s)", hipGetErrorString(e));
        }
    }
    hipError_t e = hipMemcpy(p->d_probs, h.data(), sizeof(qmc::DevProblem) * (size_t)p->count,
                             hipMemcpyHostToDevice);
    if (e != hipSuccess) return from_hip(e, "qmc_batch_plan (problem table upload)");
    const uint64_t want = (uint64_t)qmc::device_cu_count() * (uint64_t)p->cfg.workgroups_per_cu;
    p->grid = (int)std::min<uint64_t>(want, std::max<uint64_t>(1, p->total_tiles));
    return QMC_OK;
}

std::string signature(const qmc_batch_plan* p) {
    double sn = 0, snd = 0;
    int fam[5] = {0, 0, 0, 0, 0}, maxd = 0;
    int64_t maxn = 0;
    for (const auto& q : p->probs) {
        sn += (double)q.n;
        snd += (double)q.n * q.d;
        fam[q.family]++;
        maxd = std::max(maxd, (int)q.d);
        maxn = std::max(maxn, (int64_t)q.n);
    }
    char buf[256];
    snprintf(buf, sizeof(buf), "batch:c%d:p%d:sn%.6e:snd%.6e:f%d-%d-%d-%d-%d:d%d:n%lld:cu%d", p->count,
             p->precision, sn, snd, fam[0], fam[1], fam[2], fam[3], fam[4], maxd, (long long)maxn,
             qmc::device_cu_count());
    return buf;
}

std::mutex g_cache_mu;
std::map<std::string, qmc_batch_config> g_cache;
bool g_cache_loaded = false;

void load_cache_file() {
    if (g_cache_loaded) return;
    g_cache_loaded = true;
    const char* path = getenv("QMC_AUTOTUNE_CACHE");
    if (!path || !*path) return;
    FILE* f = fopen(path, "r");
    if (!f) return;
    char key[256];
    int m, w, o;
    while (fscanf(f, "%255s %d %d %d", key, &m, &w, &o) == 4) g_cache[key] = qmc_batch_config{m, w, o};
    fclose(f);
}

void store_cache_file(const std::string& key, const qmc_batch_config& c) {
    const char* path = getenv("QMC_AUTOTUNE_CACHE");
    if (!path || !*path) return;
    FILE* f = fopen(path, "a");
    if (!f) return;
    fprintf(f, "%s %d %d %d\n", key.c_str(), c.points_per_thread, c.workgroups_per_cu, c.order);
    fclose(f);
}

qmc_status launch(const qmc_batch_plan* p, double* q_out, void* ws, hipStream_t stream) {
    qmc::BatchLaunch L;
    bool fi = true;  // the exact-float index step when every problem's n allows it
    for (const auto& q : p->probs) fi = fi && q.n <= (int64_t)qmc::kFloatIndexMaxN;
    L.float_index = fi;
    L.probs = p->d_probs;
    L.count = p->count;
    L.total_tiles = p->total_tiles;
    L.points_per_thread = p->cfg.points_per_thread;
    L.grid = p->grid;
    L.fp32 = p->precision == QMC_FP32_COMPENSATED;
    L.q_out = q_out;
    L.ws = ws;
    return from_hip(qmc::launch_batched(L, stream), "qmc_lattice_sum_batched");
}

qmc_status check_ws(const qmc_batch_plan* p, const void* ws, size_t ws_bytes) {
    if (!ws) return fail(QMC_ERR_WORKSPACE, "workspace pointer is NULL");
    if (((uintptr_t)ws) % 256 != 0) return fail(QMC_ERR_WORKSPACE, "workspace not 256-byte aligned");
    if (ws_bytes < p->ws_bytes)
        return fail(QMC_ERR_WORKSPACE, "workspace has %zu bytes, %zu needed", ws_bytes, p->ws_bytes);
    return QMC_OK;
}

}  // namespace

extern "C" {

qmc_status qmc_batch_plan_create(int32_t count, const qmc_problem* problems, int32_t precision,
                                 const qmc_batch_config* cfg, qmc_batch_plan** plan) {
    if (!plan) return fail(QMC_ERR_INVALID_ARG, "plan is NULL");
    *plan = nullptr;
    if (count < 1 || count > kMaxBatch) return fail(QMC_ERR_INVALID_ARG, "count = %d outside [1, %d]", count, kMaxBatch);
    if (!problems) return fail(QMC_ERR_INVALID_ARG, "problems is NULL");
    if (precision != QMC_FP64 && precision != QMC_FP32_COMPENSATED)
        return fail(QMC_ERR_INVALID_ARG, "unknown precision %d", precision);
    for (int i = 0; i < count; ++i) {
        const qmc_problem& q = problems[i];
        if (param_count(q.family, 1) < 0) return fail(QMC_ERR_INVALID_ARG, "problem %d: unknown family %d", i, q.family);
        if (q.d < 1 || q.d > 1024) return fail(QMC_ERR_INVALID_ARG, "problem %d: d = %d outside [1, 1024]", i, q.d);
        if (q.n < 1 || q.n >= ((int64_t)1 << 31))
            return fail(QMC_ERR_INVALID_ARG, "problem %d: n = %lld outside [1, 2^31)", i, (long long)q.n);
        if (!q.z || !q.params) return fail(QMC_ERR_INVALID_ARG, "problem %d: z and params must be non-NULL", i);
    }
    // QMC_VALIDATE=1: every problem's z and shift against their ranges (no-op otherwise)
    for (int i = 0; i < count; ++i) {
        const qmc_problem& q = problems[i];
        qmc_status s = qmc::validate_z(q.z, (size_t)q.d, q.n, nullptr, "qmc_batch_plan_create");
        if (s == QMC_OK) s = qmc::validate_shift(q.shift, (size_t)q.d, nullptr, "qmc_batch_plan_create");
        if (s != QMC_OK) return s;
    }
    qmc_batch_config c{kDefaultPoints, kDefaultWpc, 0};
    if (cfg) {
        c = *cfg;
        if (c.points_per_thread == 0) c.points_per_thread = kDefaultPoints;
        if (c.workgroups_per_cu == 0) c.workgroups_per_cu = kDefaultWpc;
    }
    qmc_status s = check_config(c);
    if (s != QMC_OK) return s;
    auto* p = new qmc_batch_plan();
    p->count = count;
    p->precision = precision;
    p->cfg = c;
    p->probs.assign(problems, problems + count);
    uint64_t max_tiles = 0;
    for (const auto& q : p->probs) max_tiles += tiles_of(q.n, 4);  // the smallest tile
    if (qmc::batched_counter_words(count) * sizeof(uint32_t) > qmc::kTicketBytes) {
        delete p;
        return fail(QMC_ERR_UNSUPPORTED, "too many problems for the workspace counter region");
    }
    p->ws_bytes = qmc::kZeroBytes + ((max_tiles * sizeof(double) + 255) / 256) * 256;
    s = build_tables(p);
    if (s != QMC_OK) {
        if (p->d_probs) (void)hipFree(p->d_probs);
        delete p;
        return s;
    }
    *plan = p;
    return ok();
}

qmc_status qmc_batch_plan_destroy(qmc_batch_plan* plan) {
    if (!plan) return ok();
    if (plan->d_probs) (void)hipFree(plan->d_probs);
    delete plan;
    return ok();
}

qmc_status qmc_batch_plan_config(const qmc_batch_plan* plan, qmc_batch_config* cfg) {
    if (!plan || !cfg) return fail(QMC_ERR_INVALID_ARG, "plan and cfg must be non-NULL");
    *cfg = plan->cfg;
    return ok();
}

qmc_status qmc_batch_plan_set_config(qmc_batch_plan* plan, const qmc_batch_config* cfg) {
    if (!plan || !cfg) return fail(QMC_ERR_INVALID_ARG, "plan and cfg must be non-NULL");
    qmc_status s = check_config(*cfg);
    if (s != QMC_OK) return s;
    plan->cfg = *cfg;
    s = build_tables(plan);
    return s == QMC_OK ? ok() : s;
}

qmc_status qmc_batch_workspace_size(const qmc_batch_plan* plan, size_t* bytes) {
    if (!plan || !bytes) return fail(QMC_ERR_INVALID_ARG, "plan and bytes must be non-NULL");
    *bytes = plan->ws_bytes;
    return ok();
}

qmc_status qmc_lattice_sum_batched(const qmc_batch_plan* plan, double* q_out, void* ws,
                                   size_t ws_bytes, void* stream) {
    if (!plan || !q_out) return fail(QMC_ERR_INVALID_ARG, "plan and q_out must be non-NULL");
    qmc_status s = check_ws(plan, ws, ws_bytes);
    if (s != QMC_OK) return s;
    return launch(plan, q_out, ws, (hipStream_t)stream);
}

qmc_status qmc_batch_autotune(qmc_batch_plan* plan, double* q_out, void* ws, size_t ws_bytes,
                              void* stream, int32_t reps, qmc_batch_config* best) {
    if (!plan || !q_out) return fail(QMC_ERR_INVALID_ARG, "plan and q_out must be non-NULL");
    qmc_status s = check_ws(plan, ws, ws_bytes);
    if (s != QMC_OK) return s;
    if (reps < 1) reps = 1;
    const std::string key = signature(plan);
    {
        std::lock_guard<std::mutex> lk(g_cache_mu);
        load_cache_file();
        auto it = g_cache.find(key);
        if (it != g_cache.end() && check_config(it->second) == QMC_OK) {
            plan->cfg = it->second;
            s = build_tables(plan);
            if (s != QMC_OK) return s;
            if (best) *best = plan->cfg;
            return ok();
        }
    }
    hipStream_t st = (hipStream_t)stream;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return fail(QMC_ERR_DEVICE, "hipEventCreate failed");
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(QMC_ERR_DEVICE, "hipEventCreate failed");
    }
    qmc_batch_config best_cfg = plan->cfg;
    float best_ms = 1e30f;
    const int Ms[3] = {4, 8, 16};
    const int Ws[4] = {1, 2, 4, 8};
    for (int mi = 0; mi < 3 && s == QMC_OK; ++mi) {
        for (int wi = 0; wi < 4 && s == QMC_OK; ++wi) {
            plan->cfg = qmc_batch_config{Ms[mi], Ws[wi], 0};
            s = build_tables(plan);
            if (s != QMC_OK) break;
            s = launch(plan, q_out, ws, st);  // warm-up
            if (s != QMC_OK) break;
            hipError_t he = hipEventRecord(e0, st);
            for (int r = 0; r < reps && he == hipSuccess && s == QMC_OK; ++r) s = launch(plan, q_out, ws, st);
            if (he == hipSuccess) he = hipEventRecord(e1, st);
            if (he == hipSuccess) he = hipEventSynchronize(e1);
            float ms = 0.0f;
            if (he == hipSuccess) he = hipEventElapsedTime(&ms, e0, e1);
            if (he != hipSuccess) s = from_hip(he, "qmc_batch_autotune");
            if (s == QMC_OK && ms < best_ms) {
                best_ms = ms;
                best_cfg = plan->cfg;
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (s != QMC_OK) return s;
    plan->cfg = best_cfg;
    s = build_tables(plan);
    if (s != QMC_OK) return s;
    {
        std::lock_guard<std::mutex> lk(g_cache_mu);
        g_cache[key] = best_cfg;
        store_cache_file(key, best_cfg);
    }
    if (best) *best = best_cfg;
    return ok();
}

qmc_status qmc_batch_graph_create(const qmc_batch_plan* plan, double* q_out, void* ws,
                                  size_t ws_bytes, qmc_graph** graph) {
    if (!plan || !q_out || !graph) return fail(QMC_ERR_INVALID_ARG, "plan, q_out and graph must be non-NULL");
    *graph = nullptr;
    qmc_status s = check_ws(plan, ws, ws_bytes);
    if (s != QMC_OK) return s;
    hipStream_t cs;
    hipError_t e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    if (e != hipSuccess) return from_hip(e, "qmc_batch_graph_create (stream)");
    auto* g = new qmc_graph();
    e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        s = launch(plan, q_out, ws, cs);
        hipGraph_t gr = nullptr;
        const hipError_t e2 = hipStreamEndCapture(cs, &gr);
        g->graph = gr;
        if (s == QMC_OK && e2 != hipSuccess) s = from_hip(e2, "qmc_batch_graph_create (end capture)");
    } else {
        s = from_hip(e, "qmc_batch_graph_create (begin capture)");
    }
    if (s == QMC_OK) {
        e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
        if (e != hipSuccess) s = from_hip(e, "qmc_batch_graph_create (instantiate)");
    }
    (void)hipStreamDestroy(cs);
    if (s != QMC_OK) {
        if (g->exec) (void)hipGraphExecDestroy(g->exec);
        if (g->graph) (void)hipGraphDestroy(g->graph);
        delete g;
        return s;
    }
    *graph = g;
    return ok();
}

qmc_status qmc_graph_launch(qmc_graph* graph, void* stream) {
    if (!graph || !graph->exec) return fail(QMC_ERR_INVALID_ARG, "graph is NULL");
    return from_hip(hipGraphLaunch(graph->exec, (hipStream_t)stream), "qmc_graph_launch");
}

qmc_status qmc_graph_destroy(qmc_graph* graph) {
    if (!graph) return ok();
    if (graph->exec) (void)hipGraphExecDestroy(graph->exec);
    if (graph->graph) (void)hipGraphDestroy(graph->graph);
    delete graph;
    return ok();
}

}  // extern "C"
