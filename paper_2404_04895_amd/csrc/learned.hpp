// Declarations for the learned edge heuristic (kernels in learned.hip).
#pragma once

#include "internal.hpp"
#include "philox.hpp"

namespace aco {

constexpr int kMlpParams = 4481;  // W1[64][3], b1[64], W2[64][64], b2[64], W3[64], b3
constexpr int kMlpChunk = 64;     // edges per workgroup of the backward pass (one partial each)

int32_t mlp_rank_pow2(int32_t n);
int32_t mlp_chunks(int32_t count);
hipError_t prepare_learned_kernels();
hipError_t launch_ranks(const float* dist, int32_t n, int32_t* rank, float* nn_dist,
                        double* mean_nn, hipStream_t stream);
hipError_t launch_eta(const float* params, const float* dist, const int32_t* rank,
                      const double* mean_nn, int32_t n, double kappa, double lambda, float* eta,
                      uint32_t* nonfinite, hipStream_t stream);
hipError_t launch_features(const float* dist, const int32_t* rank, const double* mean_nn,
                           int32_t n, float* feats, hipStream_t stream);
hipError_t launch_targets(const float* tau, int32_t n, int32_t ld, float* y, hipStream_t stream);
hipError_t launch_sample(const float* feats, const float* y, int64_t count, int32_t batch,
                         uint64_t seed, uint32_t step, float* bf, float* by, hipStream_t stream);
hipError_t launch_forward_train(const float* params, const float* feats, int32_t count, float* z,
                                float* h1, float* a2, hipStream_t stream);
hipError_t launch_backward(const float* params, const float* feats, const float* y,
                           const float* z, const float* h1, const float* a2, int32_t count,
                           float* partial, double* partial_loss, hipStream_t stream);
hipError_t launch_reduce_adam(const float* partial, const double* partial_loss, int32_t count,
                              float* grad, double* loss, float* master, float* m, float* v,
                              float* effective, bool apply, float lr_t, float inv_c2, float b1,
                              float b2, float eps, hipStream_t stream);
hipError_t launch_round_params(const float* master, float* effective, hipStream_t stream);

}  // namespace aco
