// C ABI of the batched engine (declared in include/aco.h): many independent
// instances of uneven size advance together, one persistent construct launch
// and one row-update launch per iteration, optionally replayed from a
// captured hipGraph.  Each instance evolves exactly as it would alone.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <numeric>
#include <vector>

#include "aco.h"
#include "construct.hpp"

namespace {

using aco::fail;
using aco::finite_positive;

constexpr int32_t kMaxRunIters = 65535;  // capacity of the device gamma table
constexpr int32_t kDefaultWaves = 256 * 16;

size_t align256(size_t x) { return aco::align_up(x, 256); }

int32_t batch_ld(int32_t n) { return (n + 31) / 32 * 32; }  // 128-byte rows

struct BatchLayout {
    size_t insts, tasks, queue_start, rows, sort_rows, queue, state, gammas, dist, tau, P, tours, lengths, succ, pred,
        weight, best_tour, best, row_min, lower, flags, sorted_p, sorted_j, walk_stats, total;
    int64_t mat_elems, tour_elems, succ_elems, ant_elems, city_elems, sorted_elems;
    int32_t max_task_count, nrows;
};

// Upper bound on the task count: one ant per task (64 lanes per ant).
BatchLayout make_batch_layout(const int32_t* n, const int32_t* m, int32_t count) {
    BatchLayout L{};
    for (int32_t i = 0; i < count; ++i) {
        L.mat_elems += static_cast<int64_t>(n[i]) * batch_ld(n[i]);
        L.tour_elems += static_cast<int64_t>(m[i]) * n[i];
        L.succ_elems += static_cast<int64_t>(n[i]) * m[i];
        L.ant_elems += m[i];
        L.city_elems += n[i];
        L.max_task_count += m[i];
        L.nrows += n[i];
        // room for whole sorted rows, for members the sorted walk may serve
        if (n[i] <= ACO_BATCH_SORTED_MAX_N) L.sorted_elems += static_cast<int64_t>(n[i]) * n[i];
    }
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t at = off;
        off = align256(off + bytes);
        return at;
    };
    L.insts = take(sizeof(aco::BatchInstance) * count);
    L.tasks = take(sizeof(aco::BatchTask) * L.max_task_count);
    L.queue_start = take(sizeof(int32_t) * (aco::kQueues + 1));
    L.rows = take(sizeof(aco::RowTask) * L.nrows);
    L.sort_rows = take(sizeof(aco::RowTask) * L.nrows);
    L.queue = take(sizeof(uint32_t) * aco::kQueues);
    L.state = take(sizeof(aco::IterState));
    L.gammas = take(sizeof(float) * (kMaxRunIters + 1));
    L.dist = take(sizeof(float) * L.mat_elems);
    L.tau = take(sizeof(float) * L.mat_elems);
    L.P = take(sizeof(float) * L.mat_elems);
    L.tours = take(sizeof(int32_t) * L.tour_elems);
    L.lengths = take(sizeof(float) * L.ant_elems);
    L.succ = take(sizeof(int32_t) * L.succ_elems);
    L.pred = take(sizeof(int32_t) * L.succ_elems);
    L.weight = take(sizeof(int64_t) * L.ant_elems);
    L.best_tour = take(sizeof(int32_t) * L.city_elems);
    L.best = take(sizeof(aco::BestRecord) * count);
    L.row_min = take(sizeof(float) * ACO_MAX_CITIES);
    L.lower = take(sizeof(double) * count);
    L.flags = take(sizeof(uint32_t) * 4);
    L.sorted_p = take(sizeof(float) * L.sorted_elems);
    L.sorted_j = take(sizeof(uint16_t) * L.sorted_elems);
    L.walk_stats = take(sizeof(unsigned long long) * 3);
    L.total = off;
    return L;
}

}  // namespace

struct aco_batch {
    int32_t count = 0;
    float alpha = 1.f, beta = 2.f, rho = 0.5f, Q = 1.f;
    aco_params params{1.0f, 0, 1.5f, 1.0f};
    hipStream_t stream = nullptr;
    int device = 0;
    char* ws = nullptr;
    BatchLayout layout{};
    aco::BatchDevice dev{};
    std::vector<aco::BatchInstance> insts;
    std::vector<int32_t> order;  // instances, largest first
    std::vector<aco_schedule_entry> table;
    int32_t waves = kDefaultWaves;
    int32_t ntasks = 0;
    size_t task_lds = 0;
    int32_t sort_rows = 0;    // rows of the members on the sorted walk, sorted each iteration
    int32_t max_ld = 0;
    uint32_t iter = 0;
    std::vector<float> gammas;  // host copy of the last run's schedule (kept alive for the copy)
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    bool graph_stale = true;
    std::vector<hipEvent_t> events;  // construct timing: a start/stop pair per iteration
    int32_t timed_launches = 0;

    ~aco_batch() {
        if (graph_exec) (void)hipGraphExecDestroy(graph_exec);
        if (graph) (void)hipGraphDestroy(graph);
        for (hipEvent_t e : events) (void)hipEventDestroy(e);
    }
};

namespace {

int32_t pick_schedule(const aco_batch* b, int32_t n) {
    for (const aco_schedule_entry& e : b->table)
        if (n <= e.n_max && e.schedule != ACO_SCHED_AUTO) return e.schedule;
    return aco::default_schedule(n);
}

bool schedule_ok(const aco_schedule_entry& e) {
    if (e.schedule == ACO_SCHED_AUTO) return true;
    const int32_t base = e.schedule & ~ACO_SCHED_SORTED;
    if (!aco::schedule_valid(base)) return false;
    if (e.schedule & ACO_SCHED_SORTED)
        return !aco::schedule_live(base) && e.n_max <= ACO_BATCH_SORTED_MAX_N;
    return true;
}

// Rebuild the construct task queues for the current schedule table and
// upload them.  Instances go, largest first, to the queue with the least work
// so far (work = ant-steps times row length, m (n - 1) n); within a queue the
// tasks keep that order.
aco_status upload_tasks(aco_batch* b) {
    std::vector<std::vector<aco::BatchTask>> per(aco::kQueues);
    std::vector<double> load(aco::kQueues, 0.0);
    size_t lds = 0;
    std::vector<aco::RowTask> sort_rows;
    for (int32_t i : b->order) {
        aco::BatchInstance& in = b->insts[i];
        const int32_t sched = pick_schedule(b, in.n);
        const int32_t base = sched & ~ACO_SCHED_SORTED;
        in.sorted = (sched & ACO_SCHED_SORTED) ? 1 : 0;
        if (in.sorted)
            for (int32_t r = 0; r < in.n; ++r) sort_rows.push_back(aco::RowTask{i, r});
        const int32_t per_wave = 64 / aco::schedule_lanes(base);
        const int32_t q = static_cast<int32_t>(
            std::min_element(load.begin(), load.end()) - load.begin());
        for (int32_t a = 0; a < in.m; a += per_wave)
            per[q].push_back(aco::BatchTask{i, a, std::min(per_wave, in.m - a), sched});
        load[q] += static_cast<double>(in.m) * (in.n - 1) * in.n;
        lds = std::max(lds, aco::wave_lds_bytes(in.n, sched));
    }
    std::vector<aco::BatchTask> tasks;
    std::vector<int32_t> start(aco::kQueues + 1, 0);
    for (int32_t q = 0; q < aco::kQueues; ++q) {
        start[q] = static_cast<int32_t>(tasks.size());
        tasks.insert(tasks.end(), per[q].begin(), per[q].end());
    }
    start[aco::kQueues] = static_cast<int32_t>(tasks.size());
    if (static_cast<int32_t>(tasks.size()) > b->layout.max_task_count)
        return fail(ACO_EINVAL, "batch: task table overflow");
    ACO_HIP(hipMemcpyAsync(b->dev.tasks, tasks.data(), sizeof(aco::BatchTask) * tasks.size(),
                           hipMemcpyHostToDevice, b->stream),
            "upload tasks");
    ACO_HIP(hipMemcpyAsync(b->dev.queue_start, start.data(), sizeof(int32_t) * start.size(),
                           hipMemcpyHostToDevice, b->stream),
            "upload queue starts");
    ACO_HIP(hipMemcpyAsync(b->dev.insts, b->insts.data(), sizeof(aco::BatchInstance) * b->count,
                           hipMemcpyHostToDevice, b->stream),
            "upload descriptors");
    if (!sort_rows.empty())
        ACO_HIP(hipMemcpyAsync(b->dev.sort_rows, sort_rows.data(),
                               sizeof(aco::RowTask) * sort_rows.size(), hipMemcpyHostToDevice,
                               b->stream),
                "upload sort rows");
    ACO_HIP(hipStreamSynchronize(b->stream), "upload tasks (sync)");
    b->ntasks = static_cast<int32_t>(tasks.size());
    b->sort_rows = static_cast<int32_t>(sort_rows.size());
    b->task_lds = lds;
    b->graph_stale = true;
    return ACO_OK;
}

aco_status enqueue_iteration(aco_batch* b, hipEvent_t before = nullptr,
                             hipEvent_t after = nullptr) {
    if (before) ACO_HIP(hipEventRecord(before, b->stream), "event record");
    ACO_HIP(aco::launch_batch_construct(b->dev, b->ntasks, b->task_lds, b->waves, b->stream),
            "batch construct");
    if (after) ACO_HIP(hipEventRecord(after, b->stream), "event record");
    ACO_HIP(aco::launch_batch_ants(b->dev, b->count, b->Q, b->stream), "batch ants");
    ACO_HIP(aco::launch_batch_rows(b->dev, b->layout.nrows, b->max_ld, &b->dev.state->gamma_next,
                                   true, b->alpha, b->beta, b->rho, b->stream),
            "batch rows");
    if (b->sort_rows > 0)
        ACO_HIP(aco::launch_batch_sort_rows(b->dev, b->sort_rows, b->stream), "batch sort rows");
    ACO_HIP(aco::launch_batch_advance(b->dev, b->stream), "batch advance");
    return ACO_OK;
}

aco_status build_graph(aco_batch* b) {
    if (b->graph_exec) {
        (void)hipGraphExecDestroy(b->graph_exec);
        b->graph_exec = nullptr;
    }
    if (b->graph) {
        (void)hipGraphDestroy(b->graph);
        b->graph = nullptr;
    }
    ACO_HIP(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal), "begin capture");
    const aco_status st = enqueue_iteration(b);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(b->stream, &g);
    if (st != ACO_OK) {
        if (g) (void)hipGraphDestroy(g);
        return st;
    }
    if (e != hipSuccess) return aco::hip_fail(e, "end capture");
    b->graph = g;
    ACO_HIP(hipGraphInstantiate(&b->graph_exec, g, nullptr, nullptr, 0), "instantiate graph");
    b->graph_stale = false;
    return ACO_OK;
}

}  // namespace

extern "C" {

size_t aco_batch_workspace_bytes(const int32_t* n_host, const int32_t* m_host, int32_t count) {
    if (!n_host || !m_host || count < 1) return 0;
    for (int32_t i = 0; i < count; ++i)
        if (n_host[i] < 3 || n_host[i] > ACO_MAX_CITIES || m_host[i] < 1) return 0;
    return make_batch_layout(n_host, m_host, count).total;
}

aco_status aco_batch_create(const float* dists_dev, const int64_t* dist_offsets_host,
                            const int32_t* n_host, const int32_t* m_host,
                            const uint64_t* seeds_host, int32_t count, float alpha, float beta,
                            float rho, float Q, const aco_params* params, void* workspace_dev,
                            size_t workspace_bytes, void* hip_stream, aco_batch** out) {
    aco::clear_error();
    if (!out) return fail(ACO_EINVAL, "aco_batch_create: out is NULL");
    *out = nullptr;
    if (!dists_dev || !dist_offsets_host || !n_host || !m_host || !seeds_host || count < 1)
        return fail(ACO_EINVAL, "aco_batch_create: missing input");
    for (int32_t i = 0; i < count; ++i) {
        if (n_host[i] < 3 || n_host[i] > ACO_MAX_CITIES)
            return fail(ACO_EINVAL, "aco_batch_create: n[%d] = %d outside [3, %d]", i, n_host[i],
                        ACO_MAX_CITIES);
        if (m_host[i] < 1) return fail(ACO_EINVAL, "aco_batch_create: m[%d] < 1", i);
        if (dist_offsets_host[i] < 0) return fail(ACO_EINVAL, "aco_batch_create: bad offset");
    }
    if (!(isfinite(alpha) && alpha >= 0.0f) || !(isfinite(beta) && beta >= 0.0f))
        return fail(ACO_EINVAL, "aco_batch_create: alpha, beta must be >= 0");
    if (!(isfinite(rho) && rho > 0.0f && rho <= 1.0f))
        return fail(ACO_EINVAL, "aco_batch_create: rho outside (0, 1]");
    if (!finite_positive(Q)) return fail(ACO_EINVAL, "aco_batch_create: Q <= 0");
    aco_params p{1.0f, 0, 1.5f, 1.0f};
    if (params) p = *params;
    if (!finite_positive(p.tau0) || p.elite_k < 0 || !finite_positive(p.gamma_max) ||
        !finite_positive(p.gamma_min))
        return fail(ACO_EINVAL, "aco_batch_create: bad params");
    if (!workspace_dev || reinterpret_cast<uintptr_t>(workspace_dev) % 256 != 0)
        return fail(ACO_EINVAL, "aco_batch_create: workspace NULL or not 256-byte aligned");
    const BatchLayout L = make_batch_layout(n_host, m_host, count);
    if (workspace_bytes < L.total)
        return fail(ACO_ENOMEM, "aco_batch_create: workspace %zu bytes < %zu needed",
                    workspace_bytes, L.total);

    aco_batch* b = new (std::nothrow) aco_batch();
    if (!b) return fail(ACO_ENOMEM, "aco_batch_create: host allocation failed");
    auto bail = [&](aco_status st) {
        delete b;
        return st;
    };
    b->count = count;
    b->alpha = alpha;
    b->beta = beta;
    b->rho = rho;
    b->Q = Q;
    b->params = p;
    b->stream = static_cast<hipStream_t>(hip_stream);
    b->ws = static_cast<char*>(workspace_dev);
    b->layout = L;
    char* w = b->ws;
    b->dev.insts = reinterpret_cast<aco::BatchInstance*>(w + L.insts);
    b->dev.tasks = reinterpret_cast<aco::BatchTask*>(w + L.tasks);
    b->dev.queue_start = reinterpret_cast<int32_t*>(w + L.queue_start);
    b->dev.rows = reinterpret_cast<aco::RowTask*>(w + L.rows);
    b->dev.sort_rows = reinterpret_cast<aco::RowTask*>(w + L.sort_rows);
    b->dev.queue = reinterpret_cast<uint32_t*>(w + L.queue);
    b->dev.state = reinterpret_cast<aco::IterState*>(w + L.state);
    b->dev.gammas = reinterpret_cast<float*>(w + L.gammas);
    b->dev.pools.dist = reinterpret_cast<float*>(w + L.dist);
    b->dev.pools.tau = reinterpret_cast<float*>(w + L.tau);
    b->dev.pools.P = reinterpret_cast<float*>(w + L.P);
    b->dev.pools.tours = reinterpret_cast<int32_t*>(w + L.tours);
    b->dev.pools.lengths = reinterpret_cast<float*>(w + L.lengths);
    b->dev.pools.succ = reinterpret_cast<int32_t*>(w + L.succ);
    b->dev.pools.pred = reinterpret_cast<int32_t*>(w + L.pred);
    b->dev.pools.weight = reinterpret_cast<int64_t*>(w + L.weight);
    b->dev.pools.best_tour = reinterpret_cast<int32_t*>(w + L.best_tour);
    b->dev.pools.best = reinterpret_cast<aco::BestRecord*>(w + L.best);
    b->dev.pools.sorted_p = reinterpret_cast<float*>(w + L.sorted_p);
    b->dev.pools.sorted_j = reinterpret_cast<uint16_t*>(w + L.sorted_j);
    b->dev.pools.walk_stats = reinterpret_cast<unsigned long long*>(w + L.walk_stats);
    float* row_min = reinterpret_cast<float*>(w + L.row_min);
    double* lower = reinterpret_cast<double*>(w + L.lower);
    uint32_t* flags = reinterpret_cast<uint32_t*>(w + L.flags);

    hipError_t e = hipGetDevice(&b->device);
    if (e == hipSuccess) e = aco::prepare_kernels();
    if (e != hipSuccess) return bail(aco::hip_fail(e, "batch set-up"));

    // validate every instance and get its nearest-neighbour bound
    std::vector<uint32_t> bad(count, 0u);
    for (int32_t i = 0; i < count; ++i) {
        e = aco::launch_validate(dists_dev + dist_offsets_host[i], n_host[i], true, row_min,
                                 lower + i, flags, b->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(&bad[i], flags, sizeof(uint32_t), hipMemcpyDeviceToHost, b->stream);
        if (e != hipSuccess) return bail(aco::hip_fail(e, "batch validate"));
    }
    std::vector<double> lb(count);
    e = hipMemcpyAsync(lb.data(), lower, sizeof(double) * count, hipMemcpyDeviceToHost, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) return bail(aco::hip_fail(e, "batch validate (read back)"));
    for (int32_t i = 0; i < count; ++i)
        if (bad[i]) return bail(fail(ACO_EINVAL, "aco_batch_create: bad distance matrix %d", i));

    // descriptors, largest instance first for the queues
    b->insts.resize(count);
    int64_t om = 0, ot = 0, os = 0, oa = 0, oc = 0, osr = 0;
    for (int32_t i = 0; i < count; ++i) {
        aco::BatchInstance& in = b->insts[i];
        in.n = n_host[i];
        in.ld = batch_ld(n_host[i]);
        in.m = m_host[i];
        in.elite_k = (p.elite_k > 0 && p.elite_k < m_host[i]) ? p.elite_k : 0;
        in.off_mat = om;
        in.off_tours = ot;
        in.off_succ = os;
        in.off_ants = oa;
        in.off_cities = oc;
        in.off_sorted = osr;
        in.key0 = static_cast<uint32_t>(seeds_host[i]);
        in.key1 = static_cast<uint32_t>(seeds_host[i] >> 32);
        in.S = aco::quantisation_exponent(lb[i], m_host[i], Q);
        in.sorted = 0;
        if (in.n <= ACO_BATCH_SORTED_MAX_N) osr += static_cast<int64_t>(in.n) * in.n;
        om += static_cast<int64_t>(in.n) * in.ld;
        ot += static_cast<int64_t>(in.m) * in.n;
        os += static_cast<int64_t>(in.n) * in.m;
        oa += in.m;
        oc += in.n;
        b->max_ld = std::max(b->max_ld, in.ld);
    }
    b->order.resize(count);
    std::iota(b->order.begin(), b->order.end(), 0);
    std::stable_sort(b->order.begin(), b->order.end(),
                     [&](int32_t x, int32_t y) { return n_host[x] > n_host[y]; });
    std::vector<aco::RowTask> rows;
    rows.reserve(L.nrows);
    for (int32_t i : b->order)
        for (int32_t r = 0; r < n_host[i]; ++r) rows.push_back(aco::RowTask{i, r});
    e = hipMemcpyAsync(b->dev.insts, b->insts.data(), sizeof(aco::BatchInstance) * count,
                       hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(b->dev.rows, rows.data(), sizeof(aco::RowTask) * rows.size(),
                           hipMemcpyHostToDevice, b->stream);
    for (int32_t i = 0; e == hipSuccess && i < count; ++i) {
        const aco::BatchInstance& in = b->insts[i];
        e = aco::launch_copy_padded(dists_dev + dist_offsets_host[i],
                                    b->dev.pools.dist + in.off_mat, in.n, in.ld, b->stream);
        if (e == hipSuccess)
            e = aco::launch_reset_tau(in.n, in.ld, p.tau0, b->dev.pools.tau + in.off_mat,
                                      b->dev.pools.P + in.off_mat, b->stream);
    }
    if (e == hipSuccess) e = aco::launch_clear_best(b->dev.pools.best, count, b->stream);
    if (e == hipSuccess) e = aco::launch_clear_counters(b->dev.pools.walk_stats, 3, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) return bail(aco::hip_fail(e, "batch init"));
    if (aco_status st = upload_tasks(b)) return bail(st);
    *out = b;
    return ACO_OK;
}

aco_status aco_batch_set_schedules(aco_batch* b, const aco_schedule_entry* table,
                                   int32_t entries, int32_t persistent_waves) {
    if (!b) return fail(ACO_EINVAL, "null batch");
    if (entries < 0 || (entries > 0 && !table))
        return fail(ACO_EINVAL, "aco_batch_set_schedules: bad table");
    for (int32_t k = 0; k < entries; ++k)
        if (!schedule_ok(table[k]))
            return fail(ACO_EINVAL, "aco_batch_set_schedules: schedule %d not allowed for n_max %d",
                        table[k].schedule, table[k].n_max);
    if (persistent_waves < 0) return fail(ACO_EINVAL, "aco_batch_set_schedules: waves < 0");
    b->table.assign(table, table + entries);
    std::stable_sort(b->table.begin(), b->table.end(),
                     [](const aco_schedule_entry& x, const aco_schedule_entry& y) {
                         return x.n_max < y.n_max;
                     });
    b->waves = persistent_waves > 0 ? persistent_waves : kDefaultWaves;
    return upload_tasks(b);
}

aco_status aco_batch_run(aco_batch* b, int32_t iters, int32_t flags) {
    const aco::TraceRange trace("aco_batch_run");
    if (!b) return fail(ACO_EINVAL, "null batch");
    if (iters < 0 || iters > kMaxRunIters)
        return fail(ACO_EINVAL, "aco_batch_run: iters outside [0, %d]", kMaxRunIters);
    int cur = -1;
    ACO_HIP(hipGetDevice(&cur), "hipGetDevice");
    if (cur != b->device) ACO_HIP(hipSetDevice(b->device), "hipSetDevice");
    // the schedule of Sec. 2.4's annealed gamma, computed on the host exactly as
    // a single-instance run computes it
    b->gammas.resize(static_cast<size_t>(iters) + 1);
    for (int32_t t = 0; t <= iters; ++t)
        b->gammas[t] = aco_gamma_schedule(t, iters, b->params.gamma_max, b->params.gamma_min);
    ACO_HIP(hipMemcpyAsync(b->dev.gammas, b->gammas.data(), sizeof(float) * b->gammas.size(),
                           hipMemcpyHostToDevice, b->stream),
            "upload gammas");
    ACO_HIP(hipStreamSynchronize(b->stream), "upload gammas (sync)");
    ACO_HIP(aco::launch_batch_arm(b->dev, b->iter, iters, b->stream), "arm");
    ACO_HIP(aco::launch_clear_best(b->dev.pools.best, b->count, b->stream), "clear best");
    ACO_HIP(aco::launch_batch_rows(b->dev, b->layout.nrows, b->max_ld, b->dev.gammas, false,
                                   b->alpha, b->beta, b->rho, b->stream),
            "batch transition");
    if (b->sort_rows > 0)
        ACO_HIP(aco::launch_batch_sort_rows(b->dev, b->sort_rows, b->stream), "batch sort rows");
    const bool timed = (flags & ACO_BATCH_TIME_CONSTRUCT) != 0;
    const bool graph = !timed && (flags & ACO_BATCH_GRAPH) && b->stream != nullptr;
    if (graph && (b->graph_stale || !b->graph_exec)) {
        if (aco_status st = build_graph(b)) return st;
    }
    b->timed_launches = 0;
    if (timed) {
        while (b->events.size() < 2 * static_cast<size_t>(iters)) {
            hipEvent_t ev = nullptr;
            ACO_HIP(hipEventCreate(&ev), "event create");
            b->events.push_back(ev);
        }
    }
    for (int32_t it = 0; it < iters; ++it) {
        if (graph) {
            ACO_HIP(hipGraphLaunch(b->graph_exec, b->stream), "graph launch");
        } else if (aco_status st = enqueue_iteration(b, timed ? b->events[2 * it] : nullptr,
                                                     timed ? b->events[2 * it + 1] : nullptr)) {
            return st;
        }
    }
    if (timed) b->timed_launches = iters;
    b->iter += static_cast<uint32_t>(iters);
    return ACO_OK;
}

aco_status aco_batch_best(aco_batch* b, float* lens_host, int32_t* iters_host,
                          int32_t* tours_host) {
    if (!b) return fail(ACO_EINVAL, "null batch");
    std::vector<aco::BestRecord> rec(b->count);
    ACO_HIP(hipMemcpyAsync(rec.data(), b->dev.pools.best, sizeof(aco::BestRecord) * b->count,
                           hipMemcpyDeviceToHost, b->stream),
            "read best");
    if (tours_host)
        ACO_HIP(hipMemcpyAsync(tours_host, b->dev.pools.best_tour,
                               sizeof(int32_t) * static_cast<size_t>(b->layout.city_elems),
                               hipMemcpyDeviceToHost, b->stream),
                "read best tours");
    ACO_HIP(hipStreamSynchronize(b->stream), "best (sync)");
    for (int32_t i = 0; i < b->count; ++i) {
        if (lens_host) lens_host[i] = rec[i].len;
        if (iters_host) iters_host[i] = rec[i].iter;
    }
    return ACO_OK;
}

aco_status aco_batch_instance(const aco_batch* b, int32_t i, aco_batch_view* view) {
    if (!b || !view) return fail(ACO_EINVAL, "null batch or view");
    if (i < 0 || i >= b->count) return fail(ACO_EINVAL, "aco_batch_instance: index out of range");
    const aco::BatchInstance& in = b->insts[i];
    view->n = in.n;
    view->ld = in.ld;
    view->m = in.m;
    view->deposit_scale = in.S;
    view->schedule = pick_schedule(b, in.n);
    view->tau = b->dev.pools.tau + in.off_mat;
    view->P = b->dev.pools.P + in.off_mat;
    view->tours = b->dev.pools.tours + in.off_tours;
    view->lengths = b->dev.pools.lengths + in.off_ants;
    view->best_tour = b->dev.pools.best_tour + in.off_cities;
    return ACO_OK;
}

aco_status aco_batch_construct_time(aco_batch* b, double* ms_total, int32_t* launches) {
    if (!b) return fail(ACO_EINVAL, "null batch");
    ACO_HIP(hipStreamSynchronize(b->stream), "construct time (sync)");
    double total = 0.0;
    for (int32_t it = 0; it < b->timed_launches; ++it) {
        float ms = 0.0f;
        ACO_HIP(hipEventElapsedTime(&ms, b->events[2 * it], b->events[2 * it + 1]), "elapsed");
        total += ms;
    }
    if (ms_total) *ms_total = total;
    if (launches) *launches = b->timed_launches;
    return ACO_OK;
}

aco_status aco_batch_sorted_walk_stats(aco_batch* b, uint64_t* out3) {
    if (!b) return fail(ACO_EINVAL, "null batch");
    if (!out3) return fail(ACO_EINVAL, "aco_batch_sorted_walk_stats: out is NULL");
    unsigned long long v[3] = {0, 0, 0};
    ACO_HIP(hipMemcpyAsync(v, b->dev.pools.walk_stats, sizeof(v), hipMemcpyDeviceToHost, b->stream),
            "batch walk stats");
    ACO_HIP(hipStreamSynchronize(b->stream), "batch walk stats (sync)");
    for (int k = 0; k < 3; ++k) out3[k] = static_cast<uint64_t>(v[k]);
    ACO_HIP(aco::launch_clear_counters(b->dev.pools.walk_stats, 3, b->stream), "walk stats reset");
    return ACO_OK;
}

aco_status aco_batch_sync(aco_batch* b) {
    if (!b) return fail(ACO_EINVAL, "null batch");
    ACO_HIP(hipStreamSynchronize(b->stream), "batch sync");
    return ACO_OK;
}

void aco_batch_destroy(aco_batch* b) { delete b; }

}  // extern "C"
