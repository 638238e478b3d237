// Learned edge heuristic: an MLP over edge features whose output replaces
// eta = 1/d in the transition matrix of Eq. (1) (Sec. 2.1).  Not part of the
// paper: it is the learned extension of the method.
//
//   features  f1 = d_ij / dNN (dNN: mean nearest-neighbour distance),
//             f2 = log2(1 + rank_i(j)), f3 = log2(1 + rank_j(i)), rank_i(j) the
//             1-based position of j among i's neighbours by distance (ties to
//             the smaller index); each computed in FP64, rounded once to FP32
//   network   a1 = W1 f + b1 (FP64, rounded to FP32), h1 = relu(a1) rounded to
//             BF16; a2 = W2 h1 + b2 on MFMA (BF16 x BF16, FP32 accumulation);
//             h2 = relu(a2); z = W3 h2 + b3 (FP32)
//   heuristic eta = sigmoid(z)^kappa / f1^lambda in FP64 (the network's edge
//             probability times a power of the plain heuristic 1/d; the
//             constant dNN cancels in the row normalisation of Eq. (1))
//   params    4481 values: W1[64][3], b1[64], W2[64][64] (out x in), b2[64],
//             W3[64], b3; the network uses their BF16 roundings
//   training  mean BCE-with-logits against targets y, gradient with the
//             rounding points passed through as the identity, Adam on FP32
//             master parameters re-rounded to BF16 after every step.
//
// One wave computes 32 edges: layer 2 is a 32x64 by 64x64 product, i.e. two
// 32x32 output blocks of four v_mfma_f32_32x32x16_bf16 each.  Lane l holds
// edge l % 32; for the A operand of K-step s it supplies layer-1 units
// 16 s + 8 (l / 32) + 0..7 of its edge, for the B operand the same eight
// inputs of output unit 32 nb + l % 32 (contiguous in W2's row).  Accumulator
// element r of lane l is edge 8 (r / 4) + 4 (l / 32) + r % 4, unit
// 32 nb + l % 32.
#include <math.h>

#include <algorithm>

#include "learned.hpp"

namespace aco {

namespace {

constexpr int kH = 64;
constexpr int OFF_W1 = 0, OFF_B1 = 192, OFF_W2 = 256, OFF_B2 = 4352, OFF_W3 = 4416,
              OFF_B3 = 4480;
constexpr int kChunk = kMlpChunk;  // edges per workgroup in the backward pass

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

// Round to the nearest BF16 value, ties to even, by adding half a BF16 ulp
// (plus the tie bit) to the FP32 pattern and truncating.  NaN stays NaN.
__device__ __forceinline__ uint32_t bf16_pattern(float x) {
    uint32_t u = __float_as_uint(x);
    if ((u & 0x7F800000u) == 0x7F800000u && (u & 0x007FFFFFu)) return (u | 0x00400000u) >> 16;
    u += 0x7FFFu + ((u >> 16) & 1u);
    return u >> 16;
}

__device__ __forceinline__ float bf16_round(float x) { return __uint_as_float(bf16_pattern(x) << 16); }

__device__ __forceinline__ __bf16 as_bf16(float bf16_valued) {
    return __builtin_bit_cast(__bf16, static_cast<uint16_t>(__float_as_uint(bf16_valued) >> 16));
}

__device__ __forceinline__ float relu(float x) { return x > 0.0f ? x : 0.0f; }

// Sum over the 32 lanes of this lane's half of the wave (rows of 16 by DPP
// rotations, then the pair of rows by a permlane16 swap).
__device__ __forceinline__ float half_sum(float v) {
    v += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v),
                                                               0xB1, 0xF, 0xF, false));
    v += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v),
                                                               0x4E, 0xF, 0xF, false));
    v += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v),
                                                               0x124, 0xF, 0xF, false));
    v += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v),
                                                               0x128, 0xF, 0xF, false));
    const auto sw = __builtin_amdgcn_permlane16_swap(__float_as_uint(v), __float_as_uint(v),
                                                     false, false);
    return __uint_as_float(sw[0]) + __uint_as_float(sw[1]);
}

// Layer-1 pre-activation in FP64 with the reference order of operations,
// rounded to FP32 only after the ReLU.
__device__ __forceinline__ float layer1(const float* w, int u, float f0, float f1, float f2) {
    double s = static_cast<double>(w[OFF_B1 + u]);
    s = s + static_cast<double>(w[OFF_W1 + 3 * u + 0]) * static_cast<double>(f0);
    s = s + static_cast<double>(w[OFF_W1 + 3 * u + 1]) * static_cast<double>(f1);
    s = s + static_cast<double>(w[OFF_W1 + 3 * u + 2]) * static_cast<double>(f2);
    return static_cast<float>(s > 0.0 ? s : 0.0);
}

struct W2Fragments {
    bf16x8 b[4][2];
};

__device__ __forceinline__ W2Fragments load_w2(const float* w, int lane) {
    W2Fragments F;
    const int hf = lane >> 5, col = lane & 31;
#pragma unroll
    for (int ks = 0; ks < 4; ++ks)
#pragma unroll
        for (int nb = 0; nb < 2; ++nb)
#pragma unroll
            for (int t = 0; t < 8; ++t)
                F.b[ks][nb][t] = as_bf16(w[OFF_W2 + kH * (32 * nb + col) + 16 * ks + 8 * hf + t]);
    return F;
}

// Forward of the 32 edges of this wave.  Every lane passes its edge's
// features (lanes l and l + 32 carry the same edge).  Returns z for edge
// (lane & 31) in the lanes of the half that owns it (see edge_of_half); the
// optional outputs receive relu(a1) (FP32, before the BF16 rounding) for the
// 32 layer-1 units this lane computes, and a2 for this lane's accumulator
// elements.
struct TileOut {
    float z[16];  // z of edge 8 (r / 4) + 4 hf + r % 4, r = 0..15
};

__device__ __forceinline__ TileOut tile_forward(const float* w, const W2Fragments& F, int lane,
                                                float f0, float f1, float f2, int edge0,
                                                float* h1_out, float* a2_out) {
    const int hf = lane >> 5, col = lane & 31;
    f32x16 acc0 = {}, acc1 = {};
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
        bf16x8 a;
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            const int u = 16 * ks + 8 * hf + t;
            const float h = layer1(w, u, f0, f1, f2);
            if (h1_out) h1_out[static_cast<size_t>(edge0 + col) * kH + u] = h;
            a[t] = as_bf16(bf16_round(h));
        }
        acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, F.b[ks][0], acc0, 0, 0, 0);
        acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, F.b[ks][1], acc1, 0, 0, 0);
    }
    const float b2a = w[OFF_B2 + col], b2b = w[OFF_B2 + 32 + col];
    const float w3a = w[OFF_W3 + col], w3b = w[OFF_W3 + 32 + col];
    TileOut out;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int edge = 8 * (r >> 2) + 4 * hf + (r & 3);
        const float a2a = acc0[r] + b2a;
        const float a2b = acc1[r] + b2b;
        if (a2_out) {
            a2_out[static_cast<size_t>(edge0 + edge) * kH + col] = a2a;
            a2_out[static_cast<size_t>(edge0 + edge) * kH + 32 + col] = a2b;
        }
        out.z[r] = half_sum(w3a * relu(a2a) + w3b * relu(a2b)) + w[OFF_B3];
    }
    return out;
}

// In the half of lane l, lanes with (l & 31) < 16 hand out z of edge
// 8 (c / 4) + 4 hf + c % 4 with c = l & 31.
__device__ __forceinline__ float pick_z(const TileOut& t, int c) {
    float z = 0.0f;
#pragma unroll
    for (int r = 0; r < 16; ++r) z = (c == r) ? t.z[r] : z;
    return z;
}

__device__ __forceinline__ int edge_of_half(int c, int hf) { return 8 * (c >> 2) + 4 * hf + (c & 3); }

__device__ __forceinline__ void edge_features(const float* dist, const int32_t* rank, int32_t n,
                                              double mean_nn, int32_t i, int32_t j, float& f0,
                                              float& f1, float& f2) {
    const size_t ij = static_cast<size_t>(i) * n + j;
    f0 = static_cast<float>(static_cast<double>(dist[ij]) / mean_nn);
    f1 = static_cast<float>(log2(1.0 + static_cast<double>(rank[ij])));
    f2 = static_cast<float>(log2(1.0 + static_cast<double>(rank[static_cast<size_t>(j) * n + i])));
}

__device__ __forceinline__ float eta_of(float z, float f1, double kappa, double lambda) {
    const double nz = -static_cast<double>(z);
    const double log_sig = -((nz > 0.0 ? nz : 0.0) + log1p(exp(-fabs(nz))));  // -softplus(-z)
    return static_cast<float>(exp(kappa * log_sig - lambda * log(static_cast<double>(f1))));
}

// ---- ranks ---------------------------------------------------------------------
// One workgroup per row: (distance bits, index) keys sorted ascending by a
// bitonic network in LDS; rank = position + 1; the first key is the nearest
// neighbour.
__global__ __launch_bounds__(256) void rank_kernel(const float* __restrict__ dist, int32_t n,
                                                   int32_t pow2, int32_t* __restrict__ rank,
                                                   float* __restrict__ nn_dist) {
    extern __shared__ unsigned long long keys[];
    const int32_t i = blockIdx.x;
    const int32_t tid = threadIdx.x;
    for (int32_t j = tid; j < pow2; j += 256) {
        unsigned long long k = ~0ull;
        if (j < n && j != i)
            k = (static_cast<unsigned long long>(__float_as_uint(dist[static_cast<size_t>(i) * n + j]))
                 << 32) | static_cast<uint32_t>(j);
        keys[j] = k;
    }
    __syncthreads();
    for (int32_t size = 2; size <= pow2; size <<= 1) {
        for (int32_t stride = size >> 1; stride > 0; stride >>= 1) {
            for (int32_t t = tid; t < pow2; t += 256) {
                const int32_t p = t ^ stride;
                if (p > t) {
                    const unsigned long long a = keys[t], b = keys[p];
                    const bool ascending = (t & size) == 0;
                    if ((a > b) == ascending) {
                        keys[t] = b;
                        keys[p] = a;
                    }
                }
            }
            __syncthreads();
        }
    }
    for (int32_t p = tid; p < n - 1; p += 256)
        rank[static_cast<size_t>(i) * n + static_cast<uint32_t>(keys[p])] = p + 1;
    if (tid == 0) {
        rank[static_cast<size_t>(i) * n + i] = 0;
        nn_dist[i] = __uint_as_float(static_cast<uint32_t>(keys[0] >> 32));
    }
}

// Mean nearest-neighbour distance: the FP64 sum in city order, over n.
__global__ __launch_bounds__(256) void mean_kernel(const float* __restrict__ nn_dist, int32_t n,
                                                   double* __restrict__ out) {
    __shared__ double stage[kOrderedSumChunk];
    const double total = ordered_sum_f64(nn_dist, n, stage);
    if (threadIdx.x == 0) *out = total / static_cast<double>(n);
}

// ---- inference over every edge of an instance -------------------------------------
__global__ __launch_bounds__(256) void eta_kernel(const float* __restrict__ params,
                                                  const float* __restrict__ dist,
                                                  const int32_t* __restrict__ rank,
                                                  const double* __restrict__ mean_nn_ptr,
                                                  int32_t n, double kappa, double lambda,
                                                  float* __restrict__ eta,
                                                  uint32_t* __restrict__ nonfinite) {
    __shared__ float w[kMlpParams];
    for (int p = threadIdx.x; p < kMlpParams; p += 256) w[p] = params[p];
    __syncthreads();
    const double mean_nn = *mean_nn_ptr;
    const int lane = threadIdx.x & 63, hf = lane >> 5, col = lane & 31;
    const W2Fragments F = load_w2(w, lane);
    const int64_t edges = static_cast<int64_t>(n) * n;
    const int64_t tiles = (edges + 31) / 32;
    uint32_t bad = 0;
    for (int64_t tile = static_cast<int64_t>(blockIdx.x) * 4 + (threadIdx.x >> 6); tile < tiles;
         tile += static_cast<int64_t>(gridDim.x) * 4) {
        const int64_t e = tile * 32 + col;
        float f0 = 0.0f, f1 = 0.0f, f2 = 0.0f;
        int32_t i = 0, j = 0;
        if (e < edges) {
            i = static_cast<int32_t>(e / n);
            j = static_cast<int32_t>(e % n);
            if (i != j) edge_features(dist, rank, n, mean_nn, i, j, f0, f1, f2);
        }
        const TileOut t = tile_forward(w, F, lane, f0, f1, f2, 0, nullptr, nullptr);
        if (col < 16) {
            const int64_t e_out = tile * 32 + edge_of_half(col, hf);
            if (e_out < edges) {
                const int32_t io = static_cast<int32_t>(e_out / n), jo = static_cast<int32_t>(e_out % n);
                float v = 0.0f;
                if (io != jo) {
                    const float f1o = static_cast<float>(static_cast<double>(dist[e_out]) / mean_nn);
                    v = eta_of(pick_z(t, col), f1o, kappa, lambda);
                    if (!isfinite(v) || !(v > 0.0f)) ++bad;
                }
                eta[e_out] = v;
            }
        }
    }
    if (bad) atomicAdd(nonfinite, bad);
}

// Features of every off-diagonal edge, row-major with the diagonal skipped.
__global__ void features_kernel(const float* __restrict__ dist, const int32_t* __restrict__ rank,
                                const double* __restrict__ mean_nn_ptr, int32_t n,
                                float* __restrict__ feats) {
    const int64_t k = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    const int64_t total = static_cast<int64_t>(n) * (n - 1);
    if (k >= total) return;
    const int32_t i = static_cast<int32_t>(k / (n - 1));
    int32_t j = static_cast<int32_t>(k % (n - 1));
    if (j >= i) ++j;
    float f0, f1, f2;
    edge_features(dist, rank, n, *mean_nn_ptr, i, j, f0, f1, f2);
    feats[3 * k + 0] = f0;
    feats[3 * k + 1] = f1;
    feats[3 * k + 2] = f2;
}

// Targets y_ij = tau_ij / max_{k != i} tau_ik, same edge order as the features.
__global__ __launch_bounds__(256) void targets_kernel(const float* __restrict__ tau, int32_t n,
                                                      int32_t ld, float* __restrict__ y) {
    __shared__ float red[4];
    const int32_t i = blockIdx.x;
    float mx = 0.0f;
    for (int32_t j = threadIdx.x; j < n; j += 256)
        if (j != i) mx = fmaxf(mx, tau[static_cast<size_t>(i) * ld + j]);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) mx = fmaxf(mx, __shfl_xor(mx, off));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mx;
    __syncthreads();
    mx = fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
    for (int32_t j = threadIdx.x; j < n; j += 256) {
        if (j == i) continue;
        const int64_t k = static_cast<int64_t>(i) * (n - 1) + (j < i ? j : j - 1);
        y[k] = tau[static_cast<size_t>(i) * ld + j] / mx;
    }
}

// ---- training --------------------------------------------------------------------
// Minibatch: `batch` edges drawn uniformly with replacement from `count` by
// the counter-based generator (key = seed, counter = (b / 4, step, ~1, 0)).
__global__ void sample_kernel(const float* __restrict__ feats, const float* __restrict__ y,
                              int64_t count, int32_t batch, uint32_t key0, uint32_t key1,
                              uint32_t step, float* __restrict__ bf, float* __restrict__ by) {
    const int32_t b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= batch) return;
    const PhiloxOut r = philox10(static_cast<uint32_t>(b >> 2), step, 0xFFFFFFFEu, 0u, key0, key1);
    const uint32_t words[4] = {r.w0, r.w1, r.w2, r.w3};
    const int64_t k = static_cast<int64_t>(
        (static_cast<uint64_t>(words[b & 3]) * static_cast<uint64_t>(count)) >> 32);
    bf[3 * b + 0] = feats[3 * k + 0];
    bf[3 * b + 1] = feats[3 * k + 1];
    bf[3 * b + 2] = feats[3 * k + 2];
    by[b] = y[k];
}

// Forward over `count` edges of explicit features, keeping what the
// backward pass needs (count is padded to whole tiles with zero features).
__global__ __launch_bounds__(256) void forward_train_kernel(const float* __restrict__ params,
                                                            const float* __restrict__ feats,
                                                            int32_t count, float* __restrict__ z,
                                                            float* __restrict__ h1,
                                                            float* __restrict__ a2) {
    __shared__ float w[kMlpParams];
    for (int p = threadIdx.x; p < kMlpParams; p += 256) w[p] = params[p];
    __syncthreads();
    const int lane = threadIdx.x & 63, hf = lane >> 5, col = lane & 31;
    const W2Fragments F = load_w2(w, lane);
    const int32_t tiles = (count + 31) / 32;
    for (int32_t tile = blockIdx.x * 4 + (threadIdx.x >> 6); tile < tiles; tile += gridDim.x * 4) {
        const int32_t e = tile * 32 + col;
        float f0 = 0.0f, f1 = 0.0f, f2 = 0.0f;
        if (e < count) {
            f0 = feats[3 * e + 0];
            f1 = feats[3 * e + 1];
            f2 = feats[3 * e + 2];
        }
        const TileOut t = tile_forward(w, F, lane, f0, f1, f2, tile * 32, h1, a2);
        if (col < 16) z[tile * 32 + edge_of_half(col, hf)] = pick_z(t, col);
    }
}

// Backward over chunks of 64 edges: per-chunk partial gradients (and loss),
// summed afterwards in chunk order.
__global__ __launch_bounds__(256) void backward_kernel(
    const float* __restrict__ params, const float* __restrict__ feats,
    const float* __restrict__ y, const float* __restrict__ z, const float* __restrict__ h1,
    const float* __restrict__ a2, int32_t count, double inv_count,
    float* __restrict__ partial, double* __restrict__ partial_loss) {
    __shared__ float w2[kH * kH];
    __shared__ float g2[kChunk][kH + 1];
    __shared__ float h1r[kChunk][kH + 1];
    __shared__ float g1[kChunk][kH + 1];
    __shared__ float h2[kChunk][kH + 1];
    __shared__ float dz[kChunk];
    __shared__ float f[kChunk][3];
    __shared__ double lsum[kChunk];
    const int tid = threadIdx.x;
    const int32_t e0 = blockIdx.x * kChunk;
    for (int p = tid; p < kH * kH; p += 256) w2[p] = params[OFF_W2 + p];
    if (tid < kChunk) {
        const int32_t e = e0 + tid;
        float d = 0.0f;
        double l = 0.0;
        if (e < count) {
            const double zz = static_cast<double>(z[e]);
            const double yy = static_cast<double>(y[e]);
            d = static_cast<float>((1.0 / (1.0 + exp(-zz)) - yy) * inv_count);
            l = (zz > 0.0 ? zz : 0.0) + log1p(exp(-fabs(zz))) - yy * zz;
        }
        dz[tid] = d;
        lsum[tid] = l;
        for (int c = 0; c < 3; ++c) f[tid][c] = (e < count) ? feats[3 * e + c] : 0.0f;
    }
    __syncthreads();
    for (int idx = tid; idx < kChunk * kH; idx += 256) {
        const int e = idx / kH, u = idx % kH;
        const bool in = e0 + e < count;
        const size_t g = static_cast<size_t>(e0 + e) * kH + u;
        const float a = in ? a2[g] : 0.0f;
        const float h = in ? h1[g] : 0.0f;
        g2[e][u] = a > 0.0f ? dz[e] * params[OFF_W3 + u] : 0.0f;
        h2[e][u] = relu(a);
        h1r[e][u] = bf16_round(h);
        g1[e][u] = h;  // kept for the layer-1 mask
    }
    __syncthreads();
    for (int idx = tid; idx < kChunk * kH; idx += 256) {
        const int e = idx / kH, k = idx % kH;
        float s = 0.0f;
        if (g1[e][k] > 0.0f) {  // each thread reads and overwrites only its own entry
            for (int u = 0; u < kH; ++u) s += g2[e][u] * w2[u * kH + k];
        }
        g1[e][k] = s;
    }
    __syncthreads();
    float* out = partial + static_cast<size_t>(blockIdx.x) * kMlpParams;
    for (int p = tid; p < kH * kH; p += 256) {
        const int u = p / kH, k = p % kH;
        float s = 0.0f;
        for (int e = 0; e < kChunk; ++e) s += g2[e][u] * h1r[e][k];
        out[OFF_W2 + p] = s;
    }
    if (tid < kH) {
        const int u = tid;
        float sb2 = 0.0f, sw3 = 0.0f, sb1 = 0.0f, sw1a = 0.0f, sw1b = 0.0f, sw1c = 0.0f;
        for (int e = 0; e < kChunk; ++e) {
            sb2 += g2[e][u];
            sw3 += dz[e] * h2[e][u];
            sb1 += g1[e][u];
            sw1a += g1[e][u] * f[e][0];
            sw1b += g1[e][u] * f[e][1];
            sw1c += g1[e][u] * f[e][2];
        }
        out[OFF_B2 + u] = sb2;
        out[OFF_W3 + u] = sw3;
        out[OFF_B1 + u] = sb1;
        out[OFF_W1 + 3 * u + 0] = sw1a;
        out[OFF_W1 + 3 * u + 1] = sw1b;
        out[OFF_W1 + 3 * u + 2] = sw1c;
    }
    if (tid == 0) {
        float sb3 = 0.0f;
        double l = 0.0;
        for (int e = 0; e < kChunk; ++e) {
            sb3 += dz[e];
            l += lsum[e];
        }
        out[OFF_B3] = sb3;
        partial_loss[blockIdx.x] = l;
    }
}

// Sum the chunk partials in chunk order (FP64), then optionally one Adam step
// on the FP32 master parameters and their BF16 re-rounding.
__global__ void reduce_adam_kernel(const float* __restrict__ partial,
                                   const double* __restrict__ partial_loss, int32_t chunks,
                                   double inv_count, float* __restrict__ grad,
                                   double* __restrict__ loss, float* __restrict__ master,
                                   float* __restrict__ m, float* __restrict__ v,
                                   float* __restrict__ effective, int32_t apply, float lr_t,
                                   float inv_c2, float b1, float b2, float eps) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p == 0) {
        double l = 0.0;
        for (int c = 0; c < chunks; ++c) l += partial_loss[c];
        *loss = l * inv_count;
    }
    if (p >= kMlpParams) return;
    double s = 0.0;
    for (int c = 0; c < chunks; ++c) s += static_cast<double>(partial[static_cast<size_t>(c) * kMlpParams + p]);
    const float g = static_cast<float>(s);
    grad[p] = g;
    if (!apply) return;
    const float mm = b1 * m[p] + (1.0f - b1) * g;
    const float vv = b2 * v[p] + (1.0f - b2) * g * g;
    m[p] = mm;
    v[p] = vv;
    const float wnew = master[p] - lr_t * mm / (sqrtf(vv * inv_c2) + eps);
    master[p] = wnew;
    effective[p] = bf16_round(wnew);
}

__global__ void round_params_kernel(const float* __restrict__ master, float* __restrict__ eff) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < kMlpParams) eff[p] = bf16_round(master[p]);
}

}  // namespace

int32_t mlp_rank_pow2(int32_t n) {
    int32_t p = 1;
    while (p < n) p <<= 1;
    return p;
}

hipError_t prepare_learned_kernels() {
    return hipFuncSetAttribute(reinterpret_cast<const void*>(rank_kernel),
                               hipFuncAttributeMaxDynamicSharedMemorySize,
                               static_cast<int>(sizeof(unsigned long long) * ACO_MAX_CITIES));
}

hipError_t launch_ranks(const float* dist, int32_t n, int32_t* rank, float* nn_dist,
                        double* mean_nn, hipStream_t stream) {
    const int32_t pow2 = mlp_rank_pow2(n);
    hipLaunchKernelGGL(rank_kernel, dim3(n), dim3(256), sizeof(unsigned long long) * pow2, stream,
                       dist, n, pow2, rank, nn_dist);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(mean_kernel, dim3(1), dim3(256), 0, stream, nn_dist, n, mean_nn);
    return hipGetLastError();
}

hipError_t launch_eta(const float* params, const float* dist, const int32_t* rank,
                      const double* mean_nn, int32_t n, double kappa, double lambda, float* eta,
                      uint32_t* nonfinite, hipStream_t stream) {
    const int64_t tiles = (static_cast<int64_t>(n) * n + 31) / 32;
    const int64_t grid = std::min<int64_t>((tiles + 3) / 4, 8192);
    hipLaunchKernelGGL(eta_kernel, dim3(static_cast<uint32_t>(grid)), dim3(256), 0, stream, params,
                       dist, rank, mean_nn, n, kappa, lambda, eta, nonfinite);
    return hipGetLastError();
}

hipError_t launch_features(const float* dist, const int32_t* rank, const double* mean_nn,
                           int32_t n, float* feats, hipStream_t stream) {
    const int64_t total = static_cast<int64_t>(n) * (n - 1);
    hipLaunchKernelGGL(features_kernel, dim3(static_cast<uint32_t>((total + 255) / 256)),
                       dim3(256), 0, stream, dist, rank, mean_nn, n, feats);
    return hipGetLastError();
}

hipError_t launch_targets(const float* tau, int32_t n, int32_t ld, float* y, hipStream_t stream) {
    hipLaunchKernelGGL(targets_kernel, dim3(n), dim3(256), 0, stream, tau, n, ld, y);
    return hipGetLastError();
}

hipError_t launch_sample(const float* feats, const float* y, int64_t count, int32_t batch,
                         uint64_t seed, uint32_t step, float* bf, float* by, hipStream_t stream) {
    hipLaunchKernelGGL(sample_kernel, dim3((batch + 255) / 256), dim3(256), 0, stream, feats, y,
                       count, batch, static_cast<uint32_t>(seed),
                       static_cast<uint32_t>(seed >> 32), step, bf, by);
    return hipGetLastError();
}

hipError_t launch_forward_train(const float* params, const float* feats, int32_t count, float* z,
                                float* h1, float* a2, hipStream_t stream) {
    const int32_t tiles = (count + 31) / 32;
    hipLaunchKernelGGL(forward_train_kernel, dim3((tiles + 3) / 4), dim3(256), 0, stream, params,
                       feats, count, z, h1, a2);
    return hipGetLastError();
}

hipError_t launch_backward(const float* params, const float* feats, const float* y,
                           const float* z, const float* h1, const float* a2, int32_t count,
                           float* partial, double* partial_loss, hipStream_t stream) {
    const int32_t chunks = (count + kChunk - 1) / kChunk;
    hipLaunchKernelGGL(backward_kernel, dim3(chunks), dim3(256), 0, stream, params, feats, y, z,
                       h1, a2, count, 1.0 / static_cast<double>(count), partial, partial_loss);
    return hipGetLastError();
}

hipError_t launch_reduce_adam(const float* partial, const double* partial_loss, int32_t count,
                              float* grad, double* loss, float* master, float* m, float* v,
                              float* effective, bool apply, float lr_t, float inv_c2, float b1,
                              float b2, float eps, hipStream_t stream) {
    const int32_t chunks = (count + kChunk - 1) / kChunk;
    hipLaunchKernelGGL(reduce_adam_kernel, dim3((kMlpParams + 255) / 256), dim3(256), 0, stream,
                       partial, partial_loss, chunks, 1.0 / static_cast<double>(count), grad, loss,
                       master, m, v, effective, apply ? 1 : 0, lr_t, inv_c2, b1, b2, eps);
    return hipGetLastError();
}

hipError_t launch_round_params(const float* master, float* effective, hipStream_t stream) {
    hipLaunchKernelGGL(round_params_kernel, dim3((kMlpParams + 255) / 256), dim3(256), 0, stream,
                       master, effective);
    return hipGetLastError();
}

int32_t mlp_chunks(int32_t count) { return (count + kChunk - 1) / kChunk; }

}  // namespace aco
