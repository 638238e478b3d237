// C ABI of the learned edge heuristic (declared in include/aco.h).
#include <math.h>

#include <mutex>
#include <new>

#include "aco.h"
#include "learned.hpp"

namespace {

using aco::fail;

constexpr float kAdamB1 = 0.9f, kAdamB2 = 0.999f, kAdamEps = 1e-8f;

int32_t padded_batch(int32_t batch) { return (batch + 63) / 64 * 64; }

struct TrainerLayout {
    size_t master, m, v, eff, grad, bf, by, z, h1, a2, partial, partial_loss, loss, total;
};

TrainerLayout trainer_layout(int32_t batch) {
    const size_t B = static_cast<size_t>(padded_batch(batch));
    const size_t chunks = static_cast<size_t>(aco::mlp_chunks(static_cast<int32_t>(B)));
    TrainerLayout L{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t at = off;
        off = aco::align_up(off + bytes, 256);
        return at;
    };
    const size_t P = sizeof(float) * aco::kMlpParams;
    L.master = take(P);
    L.m = take(P);
    L.v = take(P);
    L.eff = take(P);
    L.grad = take(P);
    L.bf = take(sizeof(float) * 3 * B);
    L.by = take(sizeof(float) * B);
    L.z = take(sizeof(float) * B);
    L.h1 = take(sizeof(float) * 64 * B);
    L.a2 = take(sizeof(float) * 64 * B);
    L.partial = take(P * chunks);
    L.partial_loss = take(sizeof(double) * chunks);
    L.loss = take(sizeof(double));
    L.total = off;
    return L;
}

// ---- aco_mlp_gradient_noalloc: scratch in a fixed per-GPU array ----------------
// The gradient's scratch (per-edge activations z, h1, a2; per-chunk partial
// gradients and losses; the mean loss when the caller passes no loss buffer)
// for up to ACO_MLP_NOALLOC_MAX_EDGES edges.  Every GPU the library runs on
// holds its own copy for the life of the process.
constexpr size_t up256(size_t x) { return (x + 255) / 256 * 256; }

struct NoAllocLayout {
    size_t z, h1, a2, partial, partial_loss, loss, total;
};

constexpr NoAllocLayout noalloc_layout() {
    constexpr size_t E = ACO_MLP_NOALLOC_MAX_EDGES;
    constexpr size_t chunks = (E + aco::kMlpChunk - 1) / aco::kMlpChunk;
    NoAllocLayout L{};
    L.z = 0;
    L.h1 = up256(L.z + sizeof(float) * E);
    L.a2 = up256(L.h1 + sizeof(float) * 64 * E);
    L.partial = up256(L.a2 + sizeof(float) * 64 * E);
    L.partial_loss = up256(L.partial + sizeof(float) * aco::kMlpParams * chunks);
    L.loss = up256(L.partial_loss + sizeof(double) * chunks);
    L.total = up256(L.loss + sizeof(double));
    return L;
}

constexpr NoAllocLayout kNoAlloc = noalloc_layout();
// whole 32-edge forward tiles of the largest input stay inside z, h1 and a2
static_assert(ACO_MLP_NOALLOC_MAX_EDGES % 64 == 0, "maximum must be whole tiles and chunks");

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
char* g_scratch_dev[kMaxDevices] = {};  // device address of `scratch` on each GPU

}  // namespace

// Device memory of aco_mlp_gradient_noalloc.  In host code this name is only
// a handle for hipGetSymbolAddress, never a device address.
static __device__ __align__(256) char scratch[kNoAlloc.total];

namespace {

// Device address of `scratch` on the current device, looked up once per device.
aco_status noalloc_scratch(hipStream_t stream, char** out) {
    int dev = 0;
    ACO_HIP(hipGetDevice(&dev), "aco_mlp_gradient_noalloc: current device");
    if (stream) {
        hipDevice_t sdev = 0;
        ACO_HIP(hipStreamGetDevice(stream, &sdev), "aco_mlp_gradient_noalloc: stream device");
        if (sdev != dev)
            return fail(ACO_EINVAL,
                        "aco_mlp_gradient_noalloc: the stream is on device %d but device %d is "
                        "current; make the stream's device current", static_cast<int>(sdev), dev);
    }
    if (dev < 0 || dev >= kMaxDevices)
        return fail(ACO_EINVAL, "aco_mlp_gradient_noalloc: device %d beyond %d", dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_dev[dev]) {
        void* p = nullptr;
        ACO_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)),
                "aco_mlp_gradient_noalloc: scratch address");
        if (!p) return fail(ACO_EDEVICE, "aco_mlp_gradient_noalloc: scratch address is NULL");
        g_scratch_dev[dev] = static_cast<char*>(p);
    }
    *out = g_scratch_dev[dev];
    return ACO_OK;
}

}  // namespace

struct aco_mlp_trainer {
    int32_t batch = 0;
    int32_t last_count = 0;  // edges of the last gradient (for apply)
    int32_t step = 0;        // Adam steps taken
    hipStream_t stream = nullptr;
    char* ws = nullptr;
    TrainerLayout L{};
    float* ptr(size_t off) const { return reinterpret_cast<float*>(ws + off); }
    double* dptr(size_t off) const { return reinterpret_cast<double*>(ws + off); }
};

extern "C" {

aco_status aco_edge_ranks(const float* dist_dev, int32_t n, int32_t* rank_dev, float* nn_dist_dev,
                          double* mean_nn_dev, void* hip_stream) {
    if (!dist_dev || !rank_dev || !nn_dist_dev || !mean_nn_dev)
        return fail(ACO_EINVAL, "aco_edge_ranks: NULL pointer");
    if (n < 3 || n > ACO_MAX_CITIES)
        return fail(ACO_EINVAL, "aco_edge_ranks: n = %d outside [3, %d]", n, ACO_MAX_CITIES);
    ACO_HIP(aco::prepare_learned_kernels(), "prepare");
    ACO_HIP(aco::launch_ranks(dist_dev, n, rank_dev, nn_dist_dev, mean_nn_dev,
                              static_cast<hipStream_t>(hip_stream)),
            "ranks");
    return ACO_OK;
}

aco_status aco_mlp_eta(const float* params_dev, const float* dist_dev, const int32_t* rank_dev,
                       const double* mean_nn_dev, int32_t n, float kappa, float lambda,
                       float* eta_dev, uint32_t* nonfinite_dev, void* hip_stream) {
    if (!params_dev || !dist_dev || !rank_dev || !mean_nn_dev || !eta_dev || !nonfinite_dev)
        return fail(ACO_EINVAL, "aco_mlp_eta: NULL pointer");
    if (n < 3 || n > ACO_MAX_CITIES)
        return fail(ACO_EINVAL, "aco_mlp_eta: n = %d outside [3, %d]", n, ACO_MAX_CITIES);
    if (!(isfinite(kappa) && kappa >= 0.0f && isfinite(lambda) && lambda >= 0.0f))
        return fail(ACO_EINVAL, "aco_mlp_eta: kappa and lambda must be finite and >= 0");
    ACO_HIP(aco::launch_eta(params_dev, dist_dev, rank_dev, mean_nn_dev, n,
                            static_cast<double>(kappa), static_cast<double>(lambda), eta_dev,
                            nonfinite_dev, static_cast<hipStream_t>(hip_stream)),
            "eta");
    return ACO_OK;
}

aco_status aco_mlp_features(const float* dist_dev, const int32_t* rank_dev,
                            const double* mean_nn_dev, int32_t n, float* feats_dev,
                            void* hip_stream) {
    if (!dist_dev || !rank_dev || !mean_nn_dev || !feats_dev)
        return fail(ACO_EINVAL, "aco_mlp_features: NULL pointer");
    if (n < 3 || n > ACO_MAX_CITIES) return fail(ACO_EINVAL, "aco_mlp_features: bad n");
    ACO_HIP(aco::launch_features(dist_dev, rank_dev, mean_nn_dev, n, feats_dev,
                                 static_cast<hipStream_t>(hip_stream)),
            "features");
    return ACO_OK;
}

aco_status aco_mlp_targets(const float* tau_dev, int32_t n, int32_t ld, float* y_dev,
                           void* hip_stream) {
    if (!tau_dev || !y_dev) return fail(ACO_EINVAL, "aco_mlp_targets: NULL pointer");
    if (n < 3 || n > ACO_MAX_CITIES || ld < n) return fail(ACO_EINVAL, "aco_mlp_targets: bad size");
    ACO_HIP(aco::launch_targets(tau_dev, n, ld, y_dev, static_cast<hipStream_t>(hip_stream)),
            "targets");
    return ACO_OK;
}

aco_status aco_mlp_round(const float* params_dev, float* bf16_params_dev, void* hip_stream) {
    if (!params_dev || !bf16_params_dev) return fail(ACO_EINVAL, "aco_mlp_round: NULL pointer");
    ACO_HIP(aco::launch_round_params(params_dev, bf16_params_dev,
                                     static_cast<hipStream_t>(hip_stream)),
            "round");
    return ACO_OK;
}

size_t aco_mlp_trainer_workspace_bytes(int32_t batch) {
    if (batch < 1) return 0;
    return trainer_layout(batch).total;
}

aco_status aco_mlp_trainer_create(const float* init_params_dev, int32_t batch, void* workspace_dev,
                                  size_t workspace_bytes, void* hip_stream,
                                  aco_mlp_trainer** out) {
    aco::clear_error();
    if (!out) return fail(ACO_EINVAL, "aco_mlp_trainer_create: out is NULL");
    *out = nullptr;
    if (!init_params_dev || batch < 1)
        return fail(ACO_EINVAL, "aco_mlp_trainer_create: bad parameters or batch");
    if (!workspace_dev || reinterpret_cast<uintptr_t>(workspace_dev) % 256 != 0)
        return fail(ACO_EINVAL, "aco_mlp_trainer_create: workspace NULL or misaligned");
    const TrainerLayout L = trainer_layout(batch);
    if (workspace_bytes < L.total)
        return fail(ACO_ENOMEM, "aco_mlp_trainer_create: workspace %zu < %zu", workspace_bytes,
                    L.total);
    aco_mlp_trainer* t = new (std::nothrow) aco_mlp_trainer();
    if (!t) return fail(ACO_ENOMEM, "aco_mlp_trainer_create: host allocation failed");
    t->batch = batch;
    t->stream = static_cast<hipStream_t>(hip_stream);
    t->ws = static_cast<char*>(workspace_dev);
    t->L = L;
    const size_t P = sizeof(float) * aco::kMlpParams;
    hipError_t e = hipMemcpyAsync(t->ptr(L.master), init_params_dev, P, hipMemcpyDeviceToDevice,
                                  t->stream);
    if (e == hipSuccess) e = hipMemsetAsync(t->ptr(L.m), 0, P, t->stream);
    if (e == hipSuccess) e = hipMemsetAsync(t->ptr(L.v), 0, P, t->stream);
    if (e == hipSuccess) e = aco::launch_round_params(t->ptr(L.master), t->ptr(L.eff), t->stream);
    if (e != hipSuccess) {
        delete t;
        return aco::hip_fail(e, "aco_mlp_trainer_create");
    }
    *out = t;
    return ACO_OK;
}

aco_status aco_mlp_trainer_gradient(aco_mlp_trainer* t, const float* feats_dev,
                                    const float* y_dev, int32_t count, float* grad_dev) {
    if (!t || !feats_dev || !y_dev) return fail(ACO_EINVAL, "aco_mlp_trainer_gradient: NULL");
    if (count < 1 || count > t->batch)
        return fail(ACO_EINVAL, "aco_mlp_trainer_gradient: count outside [1, batch]");
    const TrainerLayout& L = t->L;
    ACO_HIP(aco::launch_forward_train(t->ptr(L.eff), feats_dev, count, t->ptr(L.z),
                                      t->ptr(L.h1), t->ptr(L.a2), t->stream),
            "forward");
    ACO_HIP(aco::launch_backward(t->ptr(L.eff), feats_dev, y_dev, t->ptr(L.z), t->ptr(L.h1),
                                 t->ptr(L.a2), count, t->ptr(L.partial), t->dptr(L.partial_loss),
                                 t->stream),
            "backward");
    ACO_HIP(aco::launch_reduce_adam(t->ptr(L.partial), t->dptr(L.partial_loss), count,
                                    t->ptr(L.grad), t->dptr(L.loss), nullptr, nullptr, nullptr,
                                    nullptr, false, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, t->stream),
            "reduce");
    if (grad_dev)
        ACO_HIP(hipMemcpyAsync(grad_dev, t->ptr(L.grad), sizeof(float) * aco::kMlpParams,
                               hipMemcpyDeviceToDevice, t->stream),
                "copy gradient");
    t->last_count = count;
    return ACO_OK;
}

aco_status aco_mlp_trainer_apply(aco_mlp_trainer* t, float lr) {
    if (!t) return fail(ACO_EINVAL, "aco_mlp_trainer_apply: NULL");
    if (t->last_count < 1) return fail(ACO_ESTATE, "aco_mlp_trainer_apply: no gradient yet");
    if (!(isfinite(lr) && lr > 0.0f)) return fail(ACO_EINVAL, "aco_mlp_trainer_apply: lr <= 0");
    const TrainerLayout& L = t->L;
    const int32_t step = t->step + 1;
    const double c1 = 1.0 - pow(static_cast<double>(kAdamB1), step);
    const double c2 = 1.0 - pow(static_cast<double>(kAdamB2), step);
    // the reduction re-runs over the last gradient's partials, then updates
    ACO_HIP(aco::launch_reduce_adam(t->ptr(L.partial), t->dptr(L.partial_loss), t->last_count,
                                    t->ptr(L.grad), t->dptr(L.loss), t->ptr(L.master), t->ptr(L.m),
                                    t->ptr(L.v), t->ptr(L.eff), true,
                                    static_cast<float>(lr / c1), static_cast<float>(1.0 / c2),
                                    kAdamB1, kAdamB2, kAdamEps, t->stream),
            "adam");
    t->step = step;
    return ACO_OK;
}

aco_status aco_mlp_trainer_step(aco_mlp_trainer* t, const float* feats_dev, const float* y_dev,
                                int64_t count, uint64_t seed, float lr) {
    if (!t || !feats_dev || !y_dev) return fail(ACO_EINVAL, "aco_mlp_trainer_step: NULL");
    if (count < 1 || count > 0xFFFFFFFFll)
        return fail(ACO_EINVAL, "aco_mlp_trainer_step: count outside [1, 2^32)");
    const TrainerLayout& L = t->L;
    ACO_HIP(aco::launch_sample(feats_dev, y_dev, count, t->batch, seed,
                               static_cast<uint32_t>(t->step), t->ptr(L.bf), t->ptr(L.by),
                               t->stream),
            "sample");
    if (aco_status st = aco_mlp_trainer_gradient(t, t->ptr(L.bf), t->ptr(L.by), t->batch, nullptr))
        return st;
    return aco_mlp_trainer_apply(t, lr);
}

aco_status aco_mlp_trainer_params(const aco_mlp_trainer* t, float* master_dev,
                                  float* bf16_params_dev) {
    if (!t) return fail(ACO_EINVAL, "aco_mlp_trainer_params: NULL");
    const size_t P = sizeof(float) * aco::kMlpParams;
    if (master_dev)
        ACO_HIP(hipMemcpyAsync(master_dev, t->ptr(t->L.master), P, hipMemcpyDeviceToDevice,
                               t->stream),
                "copy master");
    if (bf16_params_dev)
        ACO_HIP(hipMemcpyAsync(bf16_params_dev, t->ptr(t->L.eff), P, hipMemcpyDeviceToDevice,
                               t->stream),
                "copy effective");
    return ACO_OK;
}

aco_status aco_mlp_trainer_loss(aco_mlp_trainer* t, double* loss_host) {
    if (!t || !loss_host) return fail(ACO_EINVAL, "aco_mlp_trainer_loss: NULL");
    ACO_HIP(hipMemcpyAsync(loss_host, t->dptr(t->L.loss), sizeof(double), hipMemcpyDeviceToHost,
                           t->stream),
            "read loss");
    ACO_HIP(hipStreamSynchronize(t->stream), "loss (sync)");
    return ACO_OK;
}

void aco_mlp_trainer_destroy(aco_mlp_trainer* t) { delete t; }

aco_status aco_mlp_gradient_noalloc(const float* bf16_params_dev, const float* feats_dev,
                                    const float* y_dev, int32_t count, float* grad_dev,
                                    double* loss_dev, void* hip_stream) {
    if (!bf16_params_dev || !feats_dev || !y_dev || !grad_dev)
        return fail(ACO_EINVAL, "aco_mlp_gradient_noalloc: NULL pointer");
    if (count < 1 || count > ACO_MLP_NOALLOC_MAX_EDGES)
        return fail(ACO_EINVAL, "aco_mlp_gradient_noalloc: count = %d outside [1, %d]", count,
                    ACO_MLP_NOALLOC_MAX_EDGES);
    const hipStream_t stream = static_cast<hipStream_t>(hip_stream);
    char* ws = nullptr;
    if (aco_status st = noalloc_scratch(stream, &ws)) return st;
    float* z = reinterpret_cast<float*>(ws + kNoAlloc.z);
    float* h1 = reinterpret_cast<float*>(ws + kNoAlloc.h1);
    float* a2 = reinterpret_cast<float*>(ws + kNoAlloc.a2);
    float* partial = reinterpret_cast<float*>(ws + kNoAlloc.partial);
    double* partial_loss = reinterpret_cast<double*>(ws + kNoAlloc.partial_loss);
    double* loss = loss_dev ? loss_dev : reinterpret_cast<double*>(ws + kNoAlloc.loss);
    // every value the kernels read from the scratch is written earlier in the
    // same call, so nothing needs clearing
    ACO_HIP(aco::launch_forward_train(bf16_params_dev, feats_dev, count, z, h1, a2, stream),
            "aco_mlp_gradient_noalloc: forward");
    ACO_HIP(aco::launch_backward(bf16_params_dev, feats_dev, y_dev, z, h1, a2, count, partial,
                                 partial_loss, stream),
            "aco_mlp_gradient_noalloc: backward");
    ACO_HIP(aco::launch_reduce_adam(partial, partial_loss, count, grad_dev, loss, nullptr, nullptr,
                                    nullptr, nullptr, false, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, stream),
            "aco_mlp_gradient_noalloc: reduce");
    return ACO_OK;
}

}  // extern "C"
