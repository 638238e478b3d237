// C ABI of the library (declared in include/aco.h): argument checks, workspace
// carving, the call-order state machine and the host loop of a run.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <new>

#include "aco.h"
#include "construct.hpp"

struct aco_ctx {
    int32_t n = 0, ld = 0, m_max = 0;
    float alpha = 1.f, beta = 2.f, rho = 0.5f, Q = 1.f;
    aco_params params{1.0f, 0, 1.5f, 1.0f};
    int32_t S = 0;
    double length_lower_bound = 0.0;
    hipStream_t stream = nullptr;
    int device = 0;
    char* workspace = nullptr;
    aco::Layout layout{};
    aco::Buffers buf{};
    bool eta_active = false;
    bool have_P = false;       // P is current (transition or update ran)
    bool have_tours = false;   // a construct ran since the last update
    int32_t last_m = 0;
    uint32_t last_iter = 0;
    uint32_t iter = 0;         // running iteration counter used by aco_run
    int32_t schedule = -1;     // construct schedule (ACO_SCHED_*), -1: by size
    int32_t selection = ACO_SELECT_ADAIR;  // per-step selection rule (ACO_SELECT_*)
    int32_t walk = 8;          // sorted batches a step reads before the scan
    bool rows_sorted = false;  // Ps / Js hold the sorted rows of the current P
    float tau_min = 0.0f;      // MAX-MIN bounds on tau after each update
    float tau_max = INFINITY;
};

namespace {

thread_local char g_error[512] = "";

using aco::fail;
using aco::hip_fail;
using aco::align_up;
using aco::finite_positive;

aco_status check_ctx(const aco_ctx* ctx) {
    if (!ctx) return fail(ACO_EINVAL, "null context");
    return ACO_OK;
}

aco_status bind_device(const aco_ctx* ctx) {
    int cur = -1;
    ACO_HIP(hipGetDevice(&cur), "hipGetDevice");
    if (cur != ctx->device) ACO_HIP(hipSetDevice(ctx->device), "hipSetDevice");
    return ACO_OK;
}

// Sort the rows of the current P for the sorted walk, unless that is done.
// Entries each sorted row keeps at a walk: none at 0 (the walk then reads no
// sorted entry and no row is sorted), else the prefix the walk may read.
int32_t kept_prefix(int32_t n, int32_t walk) {
    return walk > 0 ? aco::sorted_prefix(n, walk) : 0;
}

aco_status sort_rows_if_needed(aco_ctx* ctx) {
    if (ctx->selection != ACO_SELECT_ADAIR_SORTED || ctx->rows_sorted) return ACO_OK;
    if (ctx->walk > 0)
        ACO_HIP(aco::launch_sort_rows(ctx->buf.P, ctx->n, ctx->ld, ctx->walk, ctx->buf.Ps,
                                      ctx->buf.Js, ctx->stream),
                "sort rows");
    ctx->rows_sorted = true;
    return ACO_OK;
}

}  // namespace

namespace aco {

aco_status fail(aco_status st, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_error, sizeof(g_error), fmt, ap);
    va_end(ap);
    return st;
}

aco_status hip_fail(hipError_t e, const char* where) {
    return fail(ACO_EDEVICE, "%s: %s", where, hipGetErrorString(e));
}

void clear_error() { g_error[0] = '\0'; }

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

bool finite_positive(float x) { return isfinite(x) && x > 0.0f; }

int32_t quantisation_exponent(double lower_bound, int32_t m_max, float Q) {
    const double x = static_cast<double>(m_max) * static_cast<double>(Q) / lower_bound;
    int32_t S = static_cast<int32_t>(floor(62.0 - log2(x)));
    while (ldexp(x, S) >= 0x1p62) --S;
    while (ldexp(x, S + 1) < 0x1p62) ++S;
    return S;
}

hipError_t launch_init_state(const float* dist_dense, int32_t n, int32_t ld, float tau0,
                             const Buffers& B, hipStream_t stream) {
    hipError_t e = launch_copy_padded(dist_dense, B.dist, n, ld, stream);
    if (e != hipSuccess) return e;
    e = launch_reset_tau(n, ld, tau0, B.tau, B.P, stream);
    if (e != hipSuccess) return e;
    return launch_clear_best(B.best, 1, stream);
}

Layout make_layout(int32_t n, int32_t ld, int32_t m_max) {
    Layout L{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t at = off;
        off = align_up(off + bytes, 256);
        return at;
    };
    const size_t mat = sizeof(float) * static_cast<size_t>(n) * ld;
    L.off_dist = take(mat);
    L.off_tau = take(mat);
    L.off_P = take(mat);
    L.off_eta = take(mat);
    L.off_tours = take(sizeof(int32_t) * static_cast<size_t>(m_max) * n);
    L.off_lengths = take(sizeof(float) * static_cast<size_t>(m_max));
    L.off_succ = take(sizeof(int32_t) * static_cast<size_t>(n) * m_max);
    L.off_pred = take(sizeof(int32_t) * static_cast<size_t>(n) * m_max);
    L.off_weight = take(sizeof(int64_t) * static_cast<size_t>(m_max));
    L.off_best_tour = take(sizeof(int32_t) * static_cast<size_t>(n));
    L.off_best = take(sizeof(BestRecord));
    L.off_row_min = take(sizeof(float) * static_cast<size_t>(n));
    L.off_lower_bound = take(sizeof(double));
    L.off_flags = take(sizeof(uint32_t) * 4);
    L.off_Ps = take(mat);
    L.off_Js = take(sizeof(uint16_t) * static_cast<size_t>(n) * ld);
    L.off_walk_stats = take(sizeof(unsigned long long) * 3);
    L.total = off;
    return L;
}

Buffers carve(char* base, const Layout& L) {
    Buffers B{};
    B.dist = reinterpret_cast<float*>(base + L.off_dist);
    B.tau = reinterpret_cast<float*>(base + L.off_tau);
    B.P = reinterpret_cast<float*>(base + L.off_P);
    B.eta = reinterpret_cast<float*>(base + L.off_eta);
    B.tours = reinterpret_cast<int32_t*>(base + L.off_tours);
    B.lengths = reinterpret_cast<float*>(base + L.off_lengths);
    B.succ = reinterpret_cast<int32_t*>(base + L.off_succ);
    B.pred = reinterpret_cast<int32_t*>(base + L.off_pred);
    B.weight = reinterpret_cast<int64_t*>(base + L.off_weight);
    B.best_tour = reinterpret_cast<int32_t*>(base + L.off_best_tour);
    B.best = reinterpret_cast<BestRecord*>(base + L.off_best);
    B.row_min = reinterpret_cast<float*>(base + L.off_row_min);
    B.lower_bound = reinterpret_cast<double*>(base + L.off_lower_bound);
    B.flags = reinterpret_cast<uint32_t*>(base + L.off_flags);
    B.Ps = reinterpret_cast<float*>(base + L.off_Ps);
    B.Js = reinterpret_cast<uint16_t*>(base + L.off_Js);
    B.walk_stats = reinterpret_cast<unsigned long long*>(base + L.off_walk_stats);
    return B;
}

}  // namespace aco

extern "C" {

int32_t aco_leading_dim(int32_t n) {
    if (n <= 0) return 0;
    return (n + 63) / 64 * 64;
}

size_t aco_workspace_bytes(int32_t n, int32_t m_max) {
    if (n < 3 || n > ACO_MAX_CITIES || m_max < 1) return 0;
    return aco::make_layout(n, aco_leading_dim(n), m_max).total;
}

const char* aco_last_error(void) { return g_error; }

float aco_gamma_schedule(int32_t t, int32_t T, float gamma_max, float gamma_min) {
    if (T <= 1) return gamma_max;
    if (t > T - 1) t = T - 1;
    if (t < 0) t = 0;
    const double frac = static_cast<double>(t) / static_cast<double>(T - 1);
    const double half_span = 0.5 * (static_cast<double>(gamma_max) - static_cast<double>(gamma_min));
    return static_cast<float>(static_cast<double>(gamma_min) +
                              half_span * (1.0 + cos(M_PI * frac)));
}

aco_status aco_create(const float* dist_dev, int32_t n, float alpha, float beta, float rho,
                      float Q, int32_t m_max, void* workspace_dev, size_t workspace_bytes,
                      void* hip_stream, aco_ctx** out) {
    aco::clear_error();
    if (!out) return fail(ACO_EINVAL, "aco_create: out is NULL");
    *out = nullptr;
    if (!dist_dev) return fail(ACO_EINVAL, "aco_create: dist is NULL");
    if (n < 3 || n > ACO_MAX_CITIES)
        return fail(ACO_EINVAL, "aco_create: n = %d outside [3, %d]", n, ACO_MAX_CITIES);
    if (m_max < 1) return fail(ACO_EINVAL, "aco_create: m_max = %d < 1", m_max);
    if (!(isfinite(alpha) && alpha >= 0.0f)) return fail(ACO_EINVAL, "aco_create: alpha < 0");
    if (!(isfinite(beta) && beta >= 0.0f)) return fail(ACO_EINVAL, "aco_create: beta < 0");
    if (!(isfinite(rho) && rho > 0.0f && rho <= 1.0f))
        return fail(ACO_EINVAL, "aco_create: rho outside (0, 1]");
    if (!finite_positive(Q)) return fail(ACO_EINVAL, "aco_create: Q <= 0");
    if (!workspace_dev) return fail(ACO_EINVAL, "aco_create: workspace is NULL");
    if (reinterpret_cast<uintptr_t>(workspace_dev) % 256 != 0)
        return fail(ACO_EINVAL, "aco_create: workspace not 256-byte aligned");
    const int32_t ld = aco_leading_dim(n);
    const aco::Layout layout = aco::make_layout(n, ld, m_max);
    if (workspace_bytes < layout.total)
        return fail(ACO_ENOMEM, "aco_create: workspace %zu bytes < %zu needed", workspace_bytes,
                    layout.total);

    aco_ctx* ctx = new (std::nothrow) aco_ctx();
    if (!ctx) return fail(ACO_ENOMEM, "aco_create: host allocation failed");
    ctx->n = n;
    ctx->ld = ld;
    ctx->m_max = m_max;
    ctx->alpha = alpha;
    ctx->beta = beta;
    ctx->rho = rho;
    ctx->Q = Q;
    ctx->stream = static_cast<hipStream_t>(hip_stream);
    ctx->workspace = static_cast<char*>(workspace_dev);
    ctx->layout = layout;
    ctx->buf = aco::carve(ctx->workspace, layout);

    auto bail = [&](aco_status st) {
        delete ctx;
        return st;
    };
    hipError_t e = hipGetDevice(&ctx->device);
    if (e != hipSuccess) return bail(hip_fail(e, "hipGetDevice"));
    e = aco::prepare_kernels();
    if (e != hipSuccess) return bail(hip_fail(e, "prepare kernels"));
    e = aco::launch_validate(dist_dev, n, true, ctx->buf.row_min, ctx->buf.lower_bound,
                             ctx->buf.flags, ctx->stream);
    if (e != hipSuccess) return bail(hip_fail(e, "validate dist"));
    uint32_t flags = 0;
    double lower = 0.0;
    e = hipMemcpyAsync(&flags, ctx->buf.flags, sizeof(flags), hipMemcpyDeviceToHost, ctx->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(&lower, ctx->buf.lower_bound, sizeof(lower), hipMemcpyDeviceToHost,
                           ctx->stream);
    if (e == hipSuccess) e = aco::launch_clear_counters(ctx->buf.walk_stats, 3, ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) return bail(hip_fail(e, "validate dist (read back)"));
    if (flags) {
        return bail(fail(ACO_EINVAL,
                         "aco_create: bad distance matrix (%s%s%s%s)",
                         (flags & aco::kFlagNotFinite) ? "non-finite entry; " : "",
                         (flags & aco::kFlagNotPositive) ? "non-positive off-diagonal entry; " : "",
                         (flags & aco::kFlagAsymmetric) ? "not symmetric; " : "",
                         (flags & aco::kFlagDiagonal) ? "non-zero diagonal; " : ""));
    }
    ctx->length_lower_bound = lower;
    ctx->S = aco::quantisation_exponent(lower, m_max, Q);
    e = aco::launch_init_state(dist_dev, n, ld, ctx->params.tau0, ctx->buf, ctx->stream);
    if (e != hipSuccess) return bail(hip_fail(e, "init state"));
    *out = ctx;
    return ACO_OK;
}

aco_status aco_set_stream(aco_ctx* ctx, void* hip_stream) {
    if (aco_status st = check_ctx(ctx)) return st;
    ctx->stream = static_cast<hipStream_t>(hip_stream);
    return ACO_OK;
}

aco_status aco_set_params(aco_ctx* ctx, const aco_params* p) {
    if (aco_status st = check_ctx(ctx)) return st;
    if (!p) return fail(ACO_EINVAL, "aco_set_params: params is NULL");
    if (!finite_positive(p->tau0)) return fail(ACO_EINVAL, "aco_set_params: tau0 <= 0");
    if (p->elite_k < 0 || p->elite_k > ctx->m_max)
        return fail(ACO_EINVAL, "aco_set_params: elite_k = %d outside [0, m_max]", p->elite_k);
    if (!finite_positive(p->gamma_max) || !finite_positive(p->gamma_min))
        return fail(ACO_EINVAL, "aco_set_params: gamma <= 0");
    if (aco_status st = bind_device(ctx)) return st;
    ctx->params = *p;
    ACO_HIP(aco::launch_reset_tau(ctx->n, ctx->ld, p->tau0, ctx->buf.tau, ctx->buf.P, ctx->stream),
            "reset tau");
    ACO_HIP(aco::launch_clear_best(ctx->buf.best, 1, ctx->stream), "clear best");
    ctx->have_P = false;
    ctx->rows_sorted = false;
    ctx->have_tours = false;
    return ACO_OK;
}

aco_status aco_set_eta(aco_ctx* ctx, const float* eta_dev) {
    if (aco_status st = check_ctx(ctx)) return st;
    if (aco_status st = bind_device(ctx)) return st;
    ctx->have_P = false;
    ctx->rows_sorted = false;
    if (!eta_dev) {
        ctx->eta_active = false;
        return ACO_OK;
    }
    ACO_HIP(aco::launch_validate(eta_dev, ctx->n, false, nullptr, nullptr, ctx->buf.flags,
                                 ctx->stream),
            "validate eta");
    uint32_t flags = 0;
    ACO_HIP(hipMemcpyAsync(&flags, ctx->buf.flags, sizeof(flags), hipMemcpyDeviceToHost,
                           ctx->stream),
            "validate eta (read back)");
    ACO_HIP(hipStreamSynchronize(ctx->stream), "validate eta (sync)");
    if (flags) {
        ctx->eta_active = false;  // fall back to the plain heuristic 1/d
        return ACO_OK;
    }
    ACO_HIP(aco::launch_copy_padded(eta_dev, ctx->buf.eta, ctx->n, ctx->ld, ctx->stream),
            "copy eta");
    ctx->eta_active = true;
    return ACO_OK;
}

int32_t aco_eta_active(const aco_ctx* ctx) { return (ctx && ctx->eta_active) ? 1 : 0; }

aco_status aco_set_schedule(aco_ctx* ctx, int32_t schedule) {
    if (aco_status st = check_ctx(ctx)) return st;
    if (schedule != ACO_SCHED_AUTO && !aco::schedule_valid(schedule))
        return fail(ACO_EINVAL, "aco_set_schedule: unknown schedule %d", schedule);
    ctx->schedule = schedule;
    return ACO_OK;
}

aco_status aco_set_selection(aco_ctx* ctx, int32_t selection) {
    if (aco_status st = check_ctx(ctx)) return st;
    if (selection != ACO_SELECT_ADAIR && selection != ACO_SELECT_ROULETTE &&
        selection != ACO_SELECT_ADAIR_SORTED)
        return fail(ACO_EINVAL, "aco_set_selection: unknown selection %d", selection);
    ctx->selection = selection;
    return ACO_OK;
}

aco_status aco_set_tau_bounds(aco_ctx* ctx, float tau_min, float tau_max) {
    if (aco_status st = check_ctx(ctx)) return st;
    if (!(tau_min >= 0.0f) || !isfinite(tau_min) || !(tau_max > 0.0f) || isnan(tau_max) ||
        tau_min > tau_max)
        return fail(ACO_EINVAL, "aco_set_tau_bounds: need 0 <= tau_min <= tau_max, tau_max > 0");
    ctx->tau_min = tau_min;
    ctx->tau_max = tau_max;
    return ACO_OK;
}

aco_status aco_set_sorted_walk(aco_ctx* ctx, int32_t batches) {
    if (aco_status st = check_ctx(ctx)) return st;
    if (batches < 0 || batches > ACO_SORTED_WALK_MAX)
        return fail(ACO_EINVAL, "aco_set_sorted_walk: %d outside [0, %d]", batches,
                    ACO_SORTED_WALK_MAX);
    // another prefix length is another layout (rows are K entries apart)
    if (kept_prefix(ctx->n, batches) != kept_prefix(ctx->n, ctx->walk)) ctx->rows_sorted = false;
    ctx->walk = batches;
    return ACO_OK;
}

aco_status aco_transition(aco_ctx* ctx, float gamma) {
    const aco::TraceRange trace("aco_transition");
    if (aco_status st = check_ctx(ctx)) return st;
    if (!finite_positive(gamma)) return fail(ACO_EINVAL, "aco_transition: gamma <= 0");
    if (aco_status st = bind_device(ctx)) return st;
    ACO_HIP(aco::launch_rows(ctx->buf, ctx->n, ctx->ld, 0, ctx->m_max, false, ctx->eta_active,
                             ctx->alpha, ctx->beta, ctx->rho, ctx->S, gamma, ctx->tau_min,
                             ctx->tau_max, ctx->stream),
            "transition");
    ctx->have_P = true;
    ctx->rows_sorted = false;
    return sort_rows_if_needed(ctx);
}

aco_status aco_construct(aco_ctx* ctx, int32_t m, uint64_t seed, uint32_t iter) {
    const aco::TraceRange trace("aco_construct");
    if (aco_status st = check_ctx(ctx)) return st;
    if (m < 1 || m > ctx->m_max)
        return fail(ACO_EINVAL, "aco_construct: m = %d outside [1, %d]", m, ctx->m_max);
    if (!ctx->have_P) return fail(ACO_ESTATE, "aco_construct: no transition matrix yet");
    if (aco_status st = bind_device(ctx)) return st;
    const bool sorted = ctx->selection == ACO_SELECT_ADAIR_SORTED;
    int32_t sched = ctx->schedule >= 0 ? ctx->schedule : aco::default_schedule(ctx->n);
    if (sorted && ctx->schedule < 0) sched = aco::sorted_default_schedule(m);
    if (ctx->selection == ACO_SELECT_ROULETTE && !aco::roulette_fits(ctx->n, sched))
        return fail(ACO_EINVAL,
                    "aco_construct: schedule %d cannot run the roulette wheel at n = %d", sched,
                    ctx->n);
    if (aco_status st = sort_rows_if_needed(ctx)) return st;
    ACO_HIP(aco::launch_construct(ctx->buf, ctx->n, ctx->ld, m, ctx->m_max, seed, iter, sched,
                                  ctx->selection, ctx->walk, ctx->stream),
            "construct");
    ctx->have_tours = true;
    ctx->last_m = m;
    ctx->last_iter = iter;
    return ACO_OK;
}

aco_status aco_update(aco_ctx* ctx, float gamma_next) {
    const aco::TraceRange trace("aco_update");
    if (aco_status st = check_ctx(ctx)) return st;
    if (!finite_positive(gamma_next)) return fail(ACO_EINVAL, "aco_update: gamma <= 0");
    if (!ctx->have_tours) return fail(ACO_ESTATE, "aco_update: no construct since last update");
    if (aco_status st = bind_device(ctx)) return st;
    const int32_t m = ctx->last_m;
    ACO_HIP(aco::launch_ants(ctx->buf, ctx->n, m, ctx->last_iter, ctx->params.elite_k, ctx->Q,
                             ctx->S, ctx->stream),
            "best and deposit weights");
    ACO_HIP(aco::launch_rows(ctx->buf, ctx->n, ctx->ld, m, ctx->m_max, true, ctx->eta_active,
                             ctx->alpha, ctx->beta, ctx->rho, ctx->S, gamma_next, ctx->tau_min,
                             ctx->tau_max, ctx->stream),
            "update rows");
    ctx->have_tours = false;
    ctx->have_P = true;
    ctx->rows_sorted = false;
    return sort_rows_if_needed(ctx);
}

aco_status aco_run(aco_ctx* ctx, int32_t m, uint64_t seed, int32_t iters,
                   int32_t* best_tour_host, float* best_len_host) {
    const aco::TraceRange trace("aco_run");
    if (aco_status st = check_ctx(ctx)) return st;
    if (iters < 0) return fail(ACO_EINVAL, "aco_run: iters < 0");
    if (m < 1 || m > ctx->m_max)
        return fail(ACO_EINVAL, "aco_run: m = %d outside [1, %d]", m, ctx->m_max);
    if (aco_status st = bind_device(ctx)) return st;
    const float gmax = ctx->params.gamma_max, gmin = ctx->params.gamma_min;
    ACO_HIP(aco::launch_clear_best(ctx->buf.best, 1, ctx->stream), "clear best");
    if (aco_status st = aco_transition(ctx, aco_gamma_schedule(0, iters, gmax, gmin))) return st;
    for (int32_t it = 0; it < iters; ++it) {
        if (aco_status st = aco_construct(ctx, m, seed, ctx->iter)) return st;
        ++ctx->iter;
        if (aco_status st = aco_update(ctx, aco_gamma_schedule(it + 1, iters, gmax, gmin)))
            return st;
    }
    return aco_best(ctx, best_tour_host, best_len_host, nullptr);
}

const float* aco_pheromone(const aco_ctx* ctx) { return ctx ? ctx->buf.tau : nullptr; }
const float* aco_transition_matrix(const aco_ctx* ctx) { return ctx ? ctx->buf.P : nullptr; }
aco_status aco_sorted_walk_stats(aco_ctx* ctx, uint64_t* out3) {
    if (aco_status st = check_ctx(ctx)) return st;
    if (!out3) return fail(ACO_EINVAL, "aco_sorted_walk_stats: out is NULL");
    if (aco_status st = bind_device(ctx)) return st;
    unsigned long long v[3] = {0, 0, 0};
    ACO_HIP(hipMemcpyAsync(v, ctx->buf.walk_stats, sizeof(v), hipMemcpyDeviceToHost, ctx->stream),
            "walk stats");
    ACO_HIP(hipStreamSynchronize(ctx->stream), "walk stats (sync)");
    for (int k = 0; k < 3; ++k) out3[k] = static_cast<uint64_t>(v[k]);
    ACO_HIP(aco::launch_clear_counters(ctx->buf.walk_stats, 3, ctx->stream), "walk stats reset");
    return ACO_OK;
}

const float* aco_sorted_rows(const aco_ctx* ctx) { return ctx ? ctx->buf.Ps : nullptr; }
const uint16_t* aco_sorted_cities(const aco_ctx* ctx) { return ctx ? ctx->buf.Js : nullptr; }
int32_t aco_sorted_prefix(const aco_ctx* ctx) { return ctx ? kept_prefix(ctx->n, ctx->walk) : 0; }
const int32_t* aco_tours(const aco_ctx* ctx) { return ctx ? ctx->buf.tours : nullptr; }
const float* aco_lengths(const aco_ctx* ctx) { return ctx ? ctx->buf.lengths : nullptr; }
int32_t aco_deposit_scale(const aco_ctx* ctx) { return ctx ? ctx->S : -1; }

aco_status aco_best(aco_ctx* ctx, int32_t* tour_host, float* len_host, int32_t* iter_host) {
    if (aco_status st = check_ctx(ctx)) return st;
    if (aco_status st = bind_device(ctx)) return st;
    aco::BestRecord rec{};
    ACO_HIP(hipMemcpyAsync(&rec, ctx->buf.best, sizeof(rec), hipMemcpyDeviceToHost, ctx->stream),
            "read best");
    if (tour_host)
        ACO_HIP(hipMemcpyAsync(tour_host, ctx->buf.best_tour, sizeof(int32_t) * ctx->n,
                               hipMemcpyDeviceToHost, ctx->stream),
                "read best tour");
    ACO_HIP(hipStreamSynchronize(ctx->stream), "best (sync)");
    if (len_host) *len_host = rec.len;
    if (iter_host) *iter_host = rec.iter;
    return ACO_OK;
}

aco_status aco_get_state(const aco_ctx* ctx, float* tau_dev_out, uint32_t* iter_out) {
    if (aco_status st = check_ctx(ctx)) return st;
    if (aco_status st = bind_device(ctx)) return st;
    if (tau_dev_out)
        ACO_HIP(hipMemcpyAsync(tau_dev_out, ctx->buf.tau,
                               sizeof(float) * static_cast<size_t>(ctx->n) * ctx->ld,
                               hipMemcpyDeviceToDevice, ctx->stream),
                "copy tau out");
    if (iter_out) *iter_out = ctx->iter;
    return ACO_OK;
}

aco_status aco_set_state(aco_ctx* ctx, const float* tau_dev, uint32_t iter) {
    if (aco_status st = check_ctx(ctx)) return st;
    if (aco_status st = bind_device(ctx)) return st;
    if (tau_dev)
        ACO_HIP(hipMemcpyAsync(ctx->buf.tau, tau_dev,
                               sizeof(float) * static_cast<size_t>(ctx->n) * ctx->ld,
                               hipMemcpyDeviceToDevice, ctx->stream),
                "copy tau in");
    ctx->iter = iter;
    ctx->have_P = false;
    ctx->rows_sorted = false;
    ctx->have_tours = false;
    return ACO_OK;
}

aco_status aco_uniforms(uint64_t seed, uint32_t iter, uint32_t ant, uint32_t step, int32_t count,
                        float* out_dev, void* hip_stream) {
    if (count < 0) return fail(ACO_EINVAL, "aco_uniforms: count < 0");
    if (count > 0 && !out_dev) return fail(ACO_EINVAL, "aco_uniforms: out is NULL");
    ACO_HIP(aco::launch_uniforms(seed, iter, ant, step, count, out_dev,
                                 static_cast<hipStream_t>(hip_stream)),
            "uniforms");
    return ACO_OK;
}

aco_status aco_sync(aco_ctx* ctx) {
    if (aco_status st = check_ctx(ctx)) return st;
    if (aco_status st = bind_device(ctx)) return st;
    ACO_HIP(hipStreamSynchronize(ctx->stream), "sync");
    return ACO_OK;
}

void aco_destroy(aco_ctx* ctx) { delete ctx; }

}  // extern "C"
