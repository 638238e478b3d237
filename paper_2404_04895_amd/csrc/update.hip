// Pheromone update and transition matrix (Sec. 2.1 Eq. (1), Sec. 2.3 Eq. (2)-(3)),
// plus the small per-iteration and set-up kernels around them.
//
// The row kernel is the only O(n^2) pass per iteration.  One workgroup owns
// one row i of tau and P:
//   1. index-mapped deposit: for every ant, add its quantised weight at
//      columns succ_a(i) and pred_a(i) of an int64 row accumulator in LDS
//      (both orientations of every tour edge through i, i.e. row i of Eq. (3)'s
//      A summed over the elite set); integer adds, so the order is free;
//   2. evaporation + deposit, tau_ij <- fl32(fma(1-rho, tau_ij, dTau_ij)) in FP64;
//   3. ln W_ij = alpha ln tau_ij + beta ln eta_ij in FP64, kept in the same
//      LDS row (each thread overwrites only its own columns);
//   4. P_ij = exp((ln W_ij - ln sum_k W_ik) / gamma), the row sum taken after
//      shifting by the row maximum.
// HBM traffic per element: tau read+write, dist (or eta) read, P write.
#include <math.h>

#include "internal.hpp"

namespace aco {

namespace {

constexpr int kRowThreads = 256;
constexpr int kRowWaves = kRowThreads / 64;

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off));
    return v;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

__device__ __forceinline__ float wave_minf(float v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fminf(v, __shfl_xor(v, off));
    return v;
}

__global__ __launch_bounds__(kRowThreads) void row_kernel(
    float* __restrict__ tau, float* __restrict__ P, const float* __restrict__ dist,
    const float* __restrict__ eta, int32_t n, int32_t ld, int32_t m, int32_t m_max,
    const int32_t* __restrict__ succ, const int32_t* __restrict__ pred,
    const int64_t* __restrict__ weight, int32_t apply_deposit, double keep, double unit,
    double alpha, double beta, double gamma) {
    extern __shared__ double lnw[];  // ld entries; first holds the int64 deposit row
    __shared__ double red[kRowWaves];
    const int32_t i = blockIdx.x;
    const int32_t tid = threadIdx.x;
    const int32_t lane = tid & 63;
    const int32_t wave = tid >> 6;
    const size_t row_off = static_cast<size_t>(i) * ld;
    unsigned long long* acc = reinterpret_cast<unsigned long long*>(lnw);

    if (apply_deposit) {
        for (int32_t j = tid; j < n; j += kRowThreads) acc[j] = 0ull;
        __syncthreads();
        const int32_t* srow = succ + static_cast<size_t>(i) * m_max;
        const int32_t* prow = pred + static_cast<size_t>(i) * m_max;
        for (int32_t a = tid; a < m; a += kRowThreads) {
            const int64_t q = weight[a];
            if (q != 0) {
                atomicAdd(&acc[srow[a]], static_cast<unsigned long long>(q));
                atomicAdd(&acc[prow[a]], static_cast<unsigned long long>(q));
            }
        }
        __syncthreads();
    }

    double local_max = -INFINITY;
    for (int32_t j = tid; j < n; j += kRowThreads) {
        if (j == i) continue;
        float t = tau[row_off + j];
        if (apply_deposit) {
            const double add = static_cast<double>(static_cast<int64_t>(acc[j])) * unit;
            t = static_cast<float>(__fma_rn(keep, static_cast<double>(t), add));
            tau[row_off + j] = t;
        }
        const double ln_eta = eta ? log(static_cast<double>(eta[row_off + j]))
                                  : -log(static_cast<double>(dist[row_off + j]));
        const double w = alpha * log(static_cast<double>(t)) + beta * ln_eta;
        lnw[j] = w;
        local_max = fmax(local_max, w);
    }
    local_max = wave_max(local_max);
    if (lane == 0) red[wave] = local_max;
    __syncthreads();
    double row_max = red[0];
#pragma unroll
    for (int w = 1; w < kRowWaves; ++w) row_max = fmax(row_max, red[w]);
    __syncthreads();

    double local_sum = 0.0;
    for (int32_t j = tid; j < n; j += kRowThreads) {
        if (j != i) local_sum += exp(lnw[j] - row_max);
    }
    local_sum = wave_sum(local_sum);
    if (lane == 0) red[wave] = local_sum;
    __syncthreads();
    double total = red[0];
#pragma unroll
    for (int w = 1; w < kRowWaves; ++w) total += red[w];
    const double ln_total = row_max + log(total);

    for (int32_t j = tid; j < ld; j += kRowThreads) {
        float p = 0.0f;
        if (j < n && j != i) p = static_cast<float>(exp((lnw[j] - ln_total) / gamma));
        P[row_off + j] = p;
    }
}

// Quantised deposit weight of each ant: round(Q / L_a * 2^S) if the ant is in
// the elite set (the elite_k shortest by (length, index)), else 0.
__global__ void weights_kernel(const float* __restrict__ lengths, int32_t m, int32_t elite_k,
                               double Q, double scale, int64_t* __restrict__ weight) {
    const int32_t a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= m) return;
    const float La = lengths[a];
    bool elite = true;
    if (elite_k > 0 && elite_k < m) {
        int32_t rank = 0;
        for (int32_t b = 0; b < m; ++b) {
            const float Lb = lengths[b];
            rank += (Lb < La) || (Lb == La && b < a);
        }
        elite = rank < elite_k;
    }
    weight[a] = elite ? __double2ll_rn((Q / static_cast<double>(La)) * scale) : 0;
}

// Best-so-far: shortest tour of this iteration (ties to the smaller ant)
// replaces the record only if strictly shorter.
__global__ __launch_bounds__(1024) void best_kernel(const float* __restrict__ lengths,
                                                    const int32_t* __restrict__ tours, int32_t n,
                                                    int32_t m, uint32_t iter,
                                                    BestRecord* __restrict__ best,
                                                    int32_t* __restrict__ best_tour) {
    __shared__ float red_len[16];
    __shared__ int32_t red_ant[16];
    __shared__ int32_t winner;
    const int32_t tid = threadIdx.x;
    float bl = INFINITY;
    int32_t ba = 0x7FFFFFFF;
    for (int32_t a = tid; a < m; a += blockDim.x) {
        const float L = lengths[a];
        if (L < bl || (L == bl && a < ba)) {
            bl = L;
            ba = a;
        }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const float ol = __shfl_xor(bl, off);
        const int32_t oa = __shfl_xor(ba, off);
        if (ol < bl || (ol == bl && oa < ba)) {
            bl = ol;
            ba = oa;
        }
    }
    if ((tid & 63) == 0) {
        red_len[tid >> 6] = bl;
        red_ant[tid >> 6] = ba;
    }
    __syncthreads();
    if (tid == 0) {
        const int waves = (blockDim.x + 63) >> 6;
        for (int w = 1; w < waves; ++w) {
            if (red_len[w] < bl || (red_len[w] == bl && red_ant[w] < ba)) {
                bl = red_len[w];
                ba = red_ant[w];
            }
        }
        winner = (bl < best->len) ? ba : -1;
        if (winner >= 0) {
            best->len = bl;
            best->iter = static_cast<int32_t>(iter);
            best->ant = ba;
        }
    }
    __syncthreads();
    const int32_t w = winner;
    if (w >= 0) {
        const int32_t* src = tours + static_cast<size_t>(w) * n;
        for (int32_t s = tid; s < n; s += blockDim.x) best_tour[s] = src[s];
    }
}

__global__ void clear_best_kernel(BestRecord* best) {
    best->len = INFINITY;
    best->iter = -1;
    best->ant = -1;
    best->pad = 0;
}

// Copy a dense n x n matrix into the padded n x ld layout (zero padding).
__global__ void copy_padded_kernel(const float* __restrict__ src, float* __restrict__ dst,
                                   int32_t n, int32_t ld) {
    const int32_t i = blockIdx.y;
    for (int32_t j = blockIdx.x * blockDim.x + threadIdx.x; j < ld; j += gridDim.x * blockDim.x)
        dst[static_cast<size_t>(i) * ld + j] = (j < n) ? src[static_cast<size_t>(i) * n + j] : 0.0f;
}

__global__ void reset_tau_kernel(float* __restrict__ tau, float* __restrict__ P, int32_t n,
                                 int32_t ld, float tau0) {
    const int32_t i = blockIdx.y;
    for (int32_t j = blockIdx.x * blockDim.x + threadIdx.x; j < ld; j += gridDim.x * blockDim.x) {
        const size_t ij = static_cast<size_t>(i) * ld + j;
        tau[ij] = (j < n && j != i) ? tau0 : 0.0f;
        P[ij] = 0.0f;
    }
}

// Input check, one workgroup per row: finite, > 0 off the diagonal, zero on
// it (when checked), bitwise symmetric (when checked); row minimum off the
// diagonal.
__global__ __launch_bounds__(256) void validate_kernel(const float* __restrict__ mat, int32_t n,
                                                       int32_t check_symmetry,
                                                       int32_t check_diagonal,
                                                       float* __restrict__ row_min,
                                                       uint32_t* __restrict__ flags) {
    __shared__ float red[4];
    const int32_t i = blockIdx.x;
    uint32_t f = 0u;
    float mn = INFINITY;
    for (int32_t j = threadIdx.x; j < n; j += blockDim.x) {
        const float v = mat[static_cast<size_t>(i) * n + j];
        if (j == i) {
            if (check_diagonal && v != 0.0f) f |= kFlagDiagonal;
            continue;
        }
        if (!isfinite(v)) f |= kFlagNotFinite;
        if (!(v > 0.0f)) f |= kFlagNotPositive;
        if (check_symmetry &&
            __float_as_uint(v) != __float_as_uint(mat[static_cast<size_t>(j) * n + i]))
            f |= kFlagAsymmetric;
        mn = fminf(mn, v);
    }
    if (f) atomicOr(flags, f);
    if (row_min) {
        mn = wave_minf(mn);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mn;
        __syncthreads();
        if (threadIdx.x == 0) {
            float r = red[0];
            for (int w = 1; w < static_cast<int>(blockDim.x >> 6); ++w) r = fminf(r, red[w]);
            row_min[i] = r;
        }
    }
}

// Sum of the row minima in ascending city order (one thread: the order is the
// definition of the bound the quantisation exponent is derived from).
__global__ void lower_bound_kernel(const float* __restrict__ row_min, int32_t n,
                                   double* __restrict__ out) {
    double total = 0.0;
    for (int32_t i = 0; i < n; ++i) total += static_cast<double>(row_min[i]);
    *out = total;
}

}  // namespace

hipError_t prepare_kernels() {
    return hipFuncSetAttribute(reinterpret_cast<const void*>(row_kernel),
                               hipFuncAttributeMaxDynamicSharedMemorySize,
                               static_cast<int>(sizeof(double) * ACO_LDS_ROW_MAX));
}

hipError_t launch_copy_padded(const float* src_dense, float* dst, int32_t n, int32_t ld,
                              hipStream_t stream) {
    hipLaunchKernelGGL(copy_padded_kernel, dim3((ld + 255) / 256, n), dim3(256), 0, stream,
                       src_dense, dst, n, ld);
    return hipGetLastError();
}

hipError_t launch_reset_tau(int32_t n, int32_t ld, float tau0, const Buffers& B,
                            hipStream_t stream) {
    hipLaunchKernelGGL(reset_tau_kernel, dim3((ld + 255) / 256, n), dim3(256), 0, stream, B.tau,
                       B.P, n, ld, tau0);
    return hipGetLastError();
}

hipError_t launch_clear_best(const Buffers& B, hipStream_t stream) {
    hipLaunchKernelGGL(clear_best_kernel, dim3(1), dim3(1), 0, stream, B.best);
    return hipGetLastError();
}

hipError_t launch_init_state(const float* dist_dense, int32_t n, int32_t ld, float tau0,
                             const Buffers& B, hipStream_t stream) {
    hipError_t e = launch_copy_padded(dist_dense, B.dist, n, ld, stream);
    if (e != hipSuccess) return e;
    e = launch_reset_tau(n, ld, tau0, B, stream);
    if (e != hipSuccess) return e;
    return launch_clear_best(B, stream);
}

hipError_t launch_validate(const float* mat_dense, int32_t n, bool is_distance,
                           bool want_row_min, const Buffers& B, hipStream_t stream) {
    hipError_t e = hipMemsetAsync(B.flags, 0, sizeof(uint32_t) * 4, stream);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(validate_kernel, dim3(n), dim3(256), 0, stream, mat_dense, n,
                       is_distance ? 1 : 0, is_distance ? 1 : 0,
                       want_row_min ? B.row_min : nullptr, B.flags);
    e = hipGetLastError();
    if (e != hipSuccess || !want_row_min) return e;
    hipLaunchKernelGGL(lower_bound_kernel, dim3(1), dim3(1), 0, stream, B.row_min, n,
                       B.lower_bound);
    return hipGetLastError();
}

hipError_t launch_deposit_weights(const Buffers& B, int32_t m, int32_t elite_k, float Q,
                                  int32_t S, hipStream_t stream) {
    hipLaunchKernelGGL(weights_kernel, dim3((m + 255) / 256), dim3(256), 0, stream, B.lengths, m,
                       elite_k, static_cast<double>(Q), ldexp(1.0, S), B.weight);
    return hipGetLastError();
}

hipError_t launch_best(const Buffers& B, int32_t n, int32_t m, uint32_t iter,
                       hipStream_t stream) {
    hipLaunchKernelGGL(best_kernel, dim3(1), dim3(1024), 0, stream, B.lengths, B.tours, n, m,
                       iter, B.best, B.best_tour);
    return hipGetLastError();
}

hipError_t launch_rows(const Buffers& B, int32_t n, int32_t ld, int32_t m, int32_t m_max,
                       bool apply_deposit, bool use_eta, float alpha, float beta, float rho,
                       int32_t S, float gamma, hipStream_t stream) {
    const size_t lds = sizeof(double) * static_cast<size_t>(ld);
    hipLaunchKernelGGL(row_kernel, dim3(n), dim3(kRowThreads), lds, stream, B.tau, B.P, B.dist,
                       use_eta ? B.eta : nullptr, n, ld, m, m_max, B.succ, B.pred, B.weight,
                       apply_deposit ? 1 : 0, 1.0 - static_cast<double>(rho), ldexp(1.0, -S),
                       static_cast<double>(alpha), static_cast<double>(beta),
                       static_cast<double>(gamma));
    return hipGetLastError();
}

}  // namespace aco
