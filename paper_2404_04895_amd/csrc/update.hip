// Pheromone update and transition matrix (Sec. 2.1 Eq. (1), Sec. 2.3 Eq. (2)-(3)),
// plus the small per-iteration and set-up kernels around them.
//
// The row update is the only O(n^2) pass per iteration.  T threads own one
// row i of tau and P (T = 256 for one instance, one wave per row in a batch):
//   1. index-mapped deposit: for every ant, add its quantised weight at
//      columns succ_a(i) and pred_a(i) of an int64 row accumulator in LDS
//      (both orientations of every tour edge through i, i.e. row i of Eq. (3)'s
//      A summed over the elite set); integer adds, so the order is free;
//   2. evaporation + deposit, tau_ij <- fl32(fma(1-rho, tau_ij, dTau_ij)) in FP64;
//   3. ln W_ij = alpha ln tau_ij + beta ln eta_ij in FP64, kept in the same
//      LDS row (each thread overwrites only its own columns);
//   4. P_ij = exp((ln W_ij - ln sum_k W_ik) / gamma), the row sum taken after
//      shifting by the row maximum.
// When alpha and beta are small non-negative integers (alpha + beta <= 6, the
// common settings) steps 3-4 take the power form instead: W_ij itself by
// multiplication (and one division by d^beta), no shift, and P_ij = W_ij / S_i
// at gamma = 1 or exp((ln W_ij - ln S_i) / gamma) otherwise, the last with a
// short logarithm and exponential of our own (accurate to about 1e-13, far
// below the FP32 rounding of P).  No FP32 input can leave the FP64 normal
// range there (|log10 W| <= 6 * 44.9 < 307).
// HBM traffic per element: tau read+write, dist (or eta) read, P write.
#include <math.h>

#include "construct.hpp"
#include "fp64_math.hpp"

namespace aco {

namespace {

constexpr int kRowThreads = 512;

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

template <int T>
__device__ __forceinline__ void sync_row() {
    if constexpr (T > 64) {
        __syncthreads();
    } else {
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
    }
}

// Row maximum across the T threads; every thread gets the result (exact in
// any order).
template <int T>
__device__ __forceinline__ double row_max_all(double v, double* red) {
    v = wave_max(v);
    if constexpr (T > 64) {
        const int wave = threadIdx.x >> 6;
        if ((threadIdx.x & 63) == 0) red[wave] = v;
        __syncthreads();
        double r = red[0];
#pragma unroll
        for (int w = 1; w < T / 64; ++w) r = fmax(r, red[w]);
        __syncthreads();
        return r;
    }
    return v;
}

// Sum over j < n of f(j) in one fixed association for T = 64 and T = 512, so
// that one instance and a batch build bit-identical rows.  Column chunk
// c = j / 64 feeds partial (c mod 8, j mod 64), which adds its terms in
// ascending c from +0; each lane then adds its 8 partials in order, and the
// 64 lane totals meet in a butterfly (every lane gets the same bits: IEEE
// addition is commutative).  One LDS read and one add per term.
constexpr int32_t kSumGroups = 8;

template <int T, typename F>
__device__ __forceinline__ double row_sum_fixed(int32_t n, F f, double* partial) {
    static_assert(T == 64 || T == 64 * kSumGroups, "one wavefront, or one per partial group");
    const int32_t lane = threadIdx.x & 63;
    const int32_t nchunks = (n + 63) >> 6;
    if constexpr (T == 64) {
        double s[kSumGroups];
#pragma unroll
        for (int32_t w = 0; w < kSumGroups; ++w) s[w] = 0.0;
        for (int32_t c0 = 0; c0 < nchunks; c0 += kSumGroups) {
#pragma unroll
            for (int32_t w = 0; w < kSumGroups; ++w) {
                const int32_t j = ((c0 + w) << 6) + lane;
                if (j < n) s[w] += f(j);
            }
        }
        double t = s[0];
#pragma unroll
        for (int32_t w = 1; w < kSumGroups; ++w) t += s[w];
        return wave_sum(t);
    } else {
        const int32_t wave = threadIdx.x >> 6;
        double s = 0.0;
        for (int32_t c = wave; c < nchunks; c += kSumGroups) {
            const int32_t j = (c << 6) + lane;
            if (j < n) s += f(j);
        }
        partial[wave * 64 + lane] = s;
        __syncthreads();
        double t = partial[lane];
#pragma unroll
        for (int32_t w = 1; w < kSumGroups; ++w) t += partial[w * 64 + lane];
        const double total = wave_sum(t);
        __syncthreads();
        return total;
    }
}

struct RowArgs {
    float* tau;             // row i of tau
    float* P;               // row i of P
    const float* dist;      // row i of dist
    const float* eta;       // row i of eta, or null for 1/d
    const int32_t* succ;    // row i of succ (m entries)
    const int32_t* pred;    // row i of pred
    const int64_t* weight;  // m quantised ant weights
    int32_t n, ld, i, m;
    int32_t apply_deposit;
    double keep, unit, alpha, beta, gamma;
    float tau_min, tau_max;  // MAX-MIN bounds applied after the update (0, +inf: none)
};

// Loads are issued kUnroll iterations at a time, before any of them is used,
// so that a thread waits for memory once per kUnroll iterations.
constexpr int32_t kUnroll = 4;

// x^k for a small non-negative integer k (wave-uniform), by multiplication.
__device__ __forceinline__ double int_power(double x, int32_t k) {
    double r = 1.0;
    for (int32_t e = 0; e < k; ++e) r *= x;
    return r;
}

// 1/d seed for ln_positive: the hardware FP64 reciprocal.
struct HardwareRcp {
    __device__ double operator()(double d) const { return __builtin_amdgcn_rcp(d); }
};

template <int T>
__device__ void update_row(const RowArgs& a, double* lnw, double* red) {
    const int32_t tid = threadIdx.x & (T - 1);
    unsigned long long* acc = reinterpret_cast<unsigned long long*>(lnw);
    if (a.apply_deposit) {
        for (int32_t j = tid; j < a.n; j += T) acc[j] = 0ull;
        sync_row<T>();
        // every ant below m has a successor and a predecessor of row i, so
        // they are read whatever the ant's weight
        for (int32_t k0 = tid; k0 < a.m; k0 += T * kUnroll) {
            int64_t q[kUnroll];
            int32_t s[kUnroll], p[kUnroll];
#pragma unroll
            for (int32_t u = 0; u < kUnroll; ++u) {
                const int32_t k = k0 + u * T;
                q[u] = 0;
                s[u] = 0;
                p[u] = 0;
                if (k < a.m) {
                    q[u] = a.weight[k];
                    s[u] = a.succ[k];
                    p[u] = a.pred[k];
                }
            }
#pragma unroll
            for (int32_t u = 0; u < kUnroll; ++u) {
                if (q[u] != 0) {
                    atomicAdd(&acc[s[u]], static_cast<unsigned long long>(q[u]));
                    atomicAdd(&acc[p[u]], static_cast<unsigned long long>(q[u]));
                }
            }
        }
        sync_row<T>();
    }
    // power form: integer exponents with alpha + beta <= 6 (see the header)
    const bool power = a.alpha >= 0.0 && a.beta >= 0.0 && a.alpha + a.beta <= 6.0 &&
                       a.alpha == floor(a.alpha) && a.beta == floor(a.beta);
    const int32_t ia = static_cast<int32_t>(a.alpha), ib = static_cast<int32_t>(a.beta);
    double local_max = -INFINITY;
    for (int32_t j0 = tid; j0 < a.n; j0 += T * kUnroll) {
        float tv[kUnroll], ev[kUnroll];
#pragma unroll
        for (int32_t u = 0; u < kUnroll; ++u) {
            const int32_t j = j0 + u * T;
            tv[u] = 0.0f;
            ev[u] = 1.0f;
            if (j < a.n) {
                tv[u] = a.tau[j];
                ev[u] = a.eta ? a.eta[j] : a.dist[j];
            }
        }
#pragma unroll
        for (int32_t u = 0; u < kUnroll; ++u) {
            const int32_t j = j0 + u * T;
            const bool live = j < a.n && j != a.i;
            if (a.apply_deposit && live) {
                const double add = static_cast<double>(static_cast<int64_t>(acc[j])) * a.unit;
                const float t = static_cast<float>(__fma_rn(a.keep, static_cast<double>(tv[u]), add));
                tv[u] = fminf(fmaxf(t, a.tau_min), a.tau_max);
            }
            if (live) {
                if (power) {
                    // W = tau^alpha * eta^beta, eta = 1/d unless given
                    const double t = int_power(static_cast<double>(tv[u]), ia);
                    const double e = int_power(static_cast<double>(ev[u]), ib);
                    lnw[j] = a.eta ? t * e : t / e;
                } else {
                    const double ln_eta = a.eta ? log(static_cast<double>(ev[u]))
                                                : -log(static_cast<double>(ev[u]));
                    const double w = a.alpha * log(static_cast<double>(tv[u])) + a.beta * ln_eta;
                    lnw[j] = w;
                    local_max = fmax(local_max, w);
                }
            }
        }
        // The stores go last and are not branched per element: a store counts
        // in the same counter as the loads, and a wait for a load placed after
        // a conditional store would wait for the store too.  The diagonal
        // entry is written back unchanged.
        if (a.apply_deposit) {
#pragma unroll
            for (int32_t u = 0; u < kUnroll; ++u) {
                const int32_t j = j0 + u * T;
                if (j < a.n) a.tau[j] = tv[u];
            }
        }
    }
    if (power) {
        sync_row<T>();
        // lnw holds W itself here
        const double total =
            row_sum_fixed<T>(a.n, [&](int32_t j) { return j == a.i ? 0.0 : lnw[j]; }, red);
        if (a.gamma == 1.0) {
            // 0 * inf = NaN for an all-zero row, as the log form gives
            const double inv = 1.0 / total;
            for (int32_t j = tid; j < a.ld; j += T) {
                float p = 0.0f;
                if (j < a.n && j != a.i) p = static_cast<float>(lnw[j] * inv);
                a.P[j] = p;
            }
        } else if (total > 0.0 && total < INFINITY) {
            // every W is finite and at most the sum; W = 0 gives P = 0
            const double ln_total = ln_positive(total, HardwareRcp{});
            const double inv_gamma = 1.0 / a.gamma;
            for (int32_t j = tid; j < a.ld; j += T) {
                float p = 0.0f;
                if (j < a.n && j != a.i && lnw[j] > 0.0)
                    p = static_cast<float>(
                        exp_for_f32((ln_positive(lnw[j], HardwareRcp{}) - ln_total) * inv_gamma));
                a.P[j] = p;
            }
        } else {
            // an all-zero or overflowing row: NaN, as the log form gives
            const double ln_total = log(total);
            const double inv_gamma = 1.0 / a.gamma;
            for (int32_t j = tid; j < a.ld; j += T) {
                float p = 0.0f;
                if (j < a.n && j != a.i)
                    p = static_cast<float>(exp((log(lnw[j]) - ln_total) * inv_gamma));
                a.P[j] = p;
            }
        }
        return;
    }
    const double row_max = row_max_all<T>(local_max, red);
    sync_row<T>();
    const double total = row_sum_fixed<T>(
        a.n, [&](int32_t j) { return j == a.i ? 0.0 : exp(lnw[j] - row_max); }, red);
    const double ln_total = row_max + log(total);
    for (int32_t j = tid; j < a.ld; j += T) {
        float p = 0.0f;
        if (j < a.n && j != a.i) p = static_cast<float>(exp((lnw[j] - ln_total) / a.gamma));
        a.P[j] = p;
    }
}

__global__ __launch_bounds__(kRowThreads) void row_kernel(
    float* __restrict__ tau, float* __restrict__ P, const float* __restrict__ dist,
    const float* __restrict__ eta, int32_t n, int32_t ld, int32_t m, int32_t m_max,
    const int32_t* __restrict__ succ, const int32_t* __restrict__ pred,
    const int64_t* __restrict__ weight, int32_t apply_deposit, double keep, double unit,
    double alpha, double beta, double gamma, float tau_min, float tau_max) {
    extern __shared__ double lnw[];
    __shared__ double red[64 * kSumGroups];  // wave maxima, then the sum's partials
    const int32_t i = blockIdx.x;
    const size_t off = static_cast<size_t>(i) * ld;
    RowArgs a;
    a.tau = tau + off;
    a.P = P + off;
    a.dist = dist + off;
    a.eta = eta ? eta + off : nullptr;
    a.succ = succ + static_cast<size_t>(i) * m_max;
    a.pred = pred + static_cast<size_t>(i) * m_max;
    a.weight = weight;
    a.n = n;
    a.ld = ld;
    a.i = i;
    a.m = m;
    a.apply_deposit = apply_deposit;
    a.keep = keep;
    a.unit = unit;
    a.alpha = alpha;
    a.beta = beta;
    a.gamma = gamma;
    a.tau_min = tau_min;
    a.tau_max = tau_max;
    update_row<kRowThreads>(a, lnw, red);
}

// Quantised deposit weight of each ant: round(Q / L_a * 2^S) if the ant is in
// the elite set (the elite_k shortest by (length, index)), else 0.
__device__ __forceinline__ int64_t ant_weight(const float* lengths, int32_t a, int32_t m,
                                              int32_t elite_k, double Q, double scale) {
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
    return elite ? __double2ll_rn((Q / static_cast<double>(La)) * scale) : 0;
}


// Best-so-far: the shortest tour of this iteration (ties to the smaller ant)
// replaces the record only if strictly shorter.  T threads, one record.
template <int T>
__device__ void best_update(const float* __restrict__ lengths, const int32_t* __restrict__ tours,
                            int32_t n, int32_t m, uint32_t iter, BestRecord* __restrict__ best,
                            int32_t* __restrict__ best_tour) {
    __shared__ float red_len[T / 64];
    __shared__ int32_t red_ant[T / 64];
    __shared__ int32_t winner;
    const int32_t tid = threadIdx.x;
    float bl = INFINITY;
    int32_t ba = 0x7FFFFFFF;
    for (int32_t a = tid; a < m; a += T) {
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
        for (int w = 1; w < T / 64; ++w) {
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
        for (int32_t s = tid; s < n; s += T) best_tour[s] = src[s];
    }
}

// The iteration's per-ant work before the row update, in one launch: every
// ant's quantised deposit weight (all blocks, one thread per ant) and the
// best-so-far record (block 0).  Both only read the lengths and tours, and
// they write disjoint outputs.
__global__ __launch_bounds__(1024) void ants_kernel(const float* __restrict__ lengths,
                                                    const int32_t* __restrict__ tours, int32_t n,
                                                    int32_t m, uint32_t iter,
                                                    BestRecord* __restrict__ best,
                                                    int32_t* __restrict__ best_tour,
                                                    int32_t elite_k, double Q, double scale,
                                                    int64_t* __restrict__ weight) {
    const int32_t a = static_cast<int32_t>(blockIdx.x * blockDim.x + threadIdx.x);
    if (a < m) weight[a] = ant_weight(lengths, a, m, elite_k, Q, scale);
    if (blockIdx.x == 0) best_update<1024>(lengths, tours, n, m, iter, best, best_tour);
}

__global__ void clear_best_kernel(BestRecord* best, int32_t count) {
    const int32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= count) return;
    best[k].len = INFINITY;
    best[k].iter = -1;
    best[k].ant = -1;
    best[k].pad = 0;
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

__global__ void clear_flags_kernel(uint32_t* flags) {
    if (threadIdx.x < 4) flags[threadIdx.x] = 0u;
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

// Sum of the row minima in ascending city order (the order is the definition
// of the bound the quantisation exponent is derived from).
__global__ __launch_bounds__(256) void lower_bound_kernel(const float* __restrict__ row_min,
                                                          int32_t n, double* __restrict__ out) {
    __shared__ double stage[kOrderedSumChunk];
    const double total = ordered_sum_f64(row_min, n, stage);
    if (threadIdx.x == 0) *out = total;
}

// ---- batched engine kernels -------------------------------------------------

// One wave per (instance, row).
__global__ __launch_bounds__(64) void batch_rows_kernel(const BatchInstance* __restrict__ insts,
                                                        const RowTask* __restrict__ rows,
                                                        int32_t nrows, BatchPools pools,
                                                        const float* __restrict__ gamma_ptr,
                                                        int32_t apply_deposit, double keep,
                                                        double alpha, double beta) {
    extern __shared__ double lnw[];
    const int32_t r = blockIdx.x;
    if (r >= nrows) return;
    const RowTask rt = rows[r];
    const BatchInstance in = insts[rt.instance];
    const size_t off = static_cast<size_t>(in.off_mat) + static_cast<size_t>(rt.row) * in.ld;
    RowArgs a;
    a.tau = pools.tau + off;
    a.P = pools.P + off;
    a.dist = pools.dist + off;
    a.eta = nullptr;
    a.succ = pools.succ + in.off_succ + static_cast<size_t>(rt.row) * in.m;
    a.pred = pools.pred + in.off_succ + static_cast<size_t>(rt.row) * in.m;
    a.weight = pools.weight + in.off_ants;
    a.n = in.n;
    a.ld = in.ld;
    a.i = rt.row;
    a.m = in.m;
    a.apply_deposit = apply_deposit;
    a.keep = keep;
    a.unit = ldexp(1.0, -in.S);
    a.alpha = alpha;
    a.beta = beta;
    a.gamma = static_cast<double>(*gamma_ptr);
    a.tau_min = 0.0f;
    a.tau_max = INFINITY;
    update_row<64>(a, lnw, nullptr);
}

// One workgroup per instance: best-so-far record, then the ants' weights.
__global__ __launch_bounds__(256) void batch_ants_kernel(const BatchInstance* __restrict__ insts,
                                                         BatchPools pools,
                                                         const IterState* __restrict__ state,
                                                         double Q) {
    const BatchInstance in = insts[blockIdx.x];
    const float* lengths = pools.lengths + in.off_ants;
    best_update<256>(lengths, pools.tours + in.off_tours, in.n, in.m, state->iter,
                     pools.best + blockIdx.x, pools.best_tour + in.off_cities);
    const double scale = ldexp(1.0, in.S);
    for (int32_t a = threadIdx.x; a < in.m; a += 256)
        pools.weight[in.off_ants + a] = ant_weight(lengths, a, in.m, in.elite_k, Q, scale);
}

// Last kernel of an iteration: advance the counters and re-arm the queue.
__global__ void batch_advance_kernel(IterState* __restrict__ state,
                                     const float* __restrict__ gammas,
                                     uint32_t* __restrict__ queue) {
    IterState s = *state;
    s.iter += 1u;
    s.t += 1;
    s.gamma_next = gammas[min(s.t + 1, s.T)];
    *state = s;
    for (int32_t q = 0; q < kQueues; ++q) queue[q] = 0u;
}

__global__ void batch_arm_kernel(IterState* __restrict__ state, const float* __restrict__ gammas,
                                 uint32_t* __restrict__ queue, uint32_t iter0, int32_t T) {
    IterState s;
    s.iter = iter0;
    s.t = 0;
    s.T = T;
    s.gamma_next = gammas[min(1, T)];
    *state = s;
    for (int32_t q = 0; q < kQueues; ++q) queue[q] = 0u;
}

}  // namespace

hipError_t prepare_kernels() {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(row_kernel),
                                       hipFuncAttributeMaxDynamicSharedMemorySize,
                                       static_cast<int>(sizeof(double) * ACO_LDS_ROW_MAX));
    if (e != hipSuccess) return e;
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(batch_rows_kernel),
                            hipFuncAttributeMaxDynamicSharedMemorySize,
                            static_cast<int>(sizeof(double) * ACO_LDS_ROW_MAX));
    if (e != hipSuccess) return e;
    return prepare_sort_kernel();
}

hipError_t launch_copy_padded(const float* src_dense, float* dst, int32_t n, int32_t ld,
                              hipStream_t stream) {
    hipLaunchKernelGGL(copy_padded_kernel, dim3((ld + 255) / 256, n), dim3(256), 0, stream,
                       src_dense, dst, n, ld);
    return hipGetLastError();
}

hipError_t launch_reset_tau(int32_t n, int32_t ld, float tau0, float* tau, float* P,
                            hipStream_t stream) {
    hipLaunchKernelGGL(reset_tau_kernel, dim3((ld + 255) / 256, n), dim3(256), 0, stream, tau, P,
                       n, ld, tau0);
    return hipGetLastError();
}

hipError_t launch_clear_best(BestRecord* best, int32_t count, hipStream_t stream) {
    hipLaunchKernelGGL(clear_best_kernel, dim3((count + 255) / 256), dim3(256), 0, stream, best,
                       count);
    return hipGetLastError();
}

hipError_t launch_validate(const float* mat_dense, int32_t n, bool is_distance, float* row_min,
                           double* lower_bound, uint32_t* flags, hipStream_t stream) {
    hipLaunchKernelGGL(clear_flags_kernel, dim3(1), dim3(64), 0, stream, flags);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(validate_kernel, dim3(n), dim3(256), 0, stream, mat_dense, n,
                       is_distance ? 1 : 0, is_distance ? 1 : 0, row_min, flags);
    e = hipGetLastError();
    if (e != hipSuccess || !lower_bound) return e;
    hipLaunchKernelGGL(lower_bound_kernel, dim3(1), dim3(256), 0, stream, row_min, n, lower_bound);
    return hipGetLastError();
}

hipError_t launch_ants(const Buffers& B, int32_t n, int32_t m, uint32_t iter, int32_t elite_k,
                       float Q, int32_t S, hipStream_t stream) {
    hipLaunchKernelGGL(ants_kernel, dim3((m + 1023) / 1024), dim3(1024), 0, stream, B.lengths,
                       B.tours, n, m, iter, B.best, B.best_tour, elite_k, static_cast<double>(Q),
                       ldexp(1.0, S), B.weight);
    return hipGetLastError();
}

hipError_t launch_rows(const Buffers& B, int32_t n, int32_t ld, int32_t m, int32_t m_max,
                       bool apply_deposit, bool use_eta, float alpha, float beta, float rho,
                       int32_t S, float gamma, float tau_min, float tau_max,
                       hipStream_t stream) {
    const size_t lds = sizeof(double) * static_cast<size_t>(ld);
    hipLaunchKernelGGL(row_kernel, dim3(n), dim3(kRowThreads), lds, stream, B.tau, B.P, B.dist,
                       use_eta ? B.eta : nullptr, n, ld, m, m_max, B.succ, B.pred, B.weight,
                       apply_deposit ? 1 : 0, 1.0 - static_cast<double>(rho), ldexp(1.0, -S),
                       static_cast<double>(alpha), static_cast<double>(beta),
                       static_cast<double>(gamma), tau_min, tau_max);
    return hipGetLastError();
}

hipError_t launch_batch_rows(const BatchDevice& BD, int32_t nrows, int32_t max_ld,
                             const float* gamma_ptr, bool apply_deposit, float alpha, float beta,
                             float rho, hipStream_t stream) {
    const size_t lds = sizeof(double) * static_cast<size_t>(max_ld);
    hipLaunchKernelGGL(batch_rows_kernel, dim3(nrows), dim3(64), lds, stream, BD.insts, BD.rows,
                       nrows, BD.pools, gamma_ptr, apply_deposit ? 1 : 0,
                       1.0 - static_cast<double>(rho), static_cast<double>(alpha),
                       static_cast<double>(beta));
    return hipGetLastError();
}

hipError_t launch_batch_ants(const BatchDevice& BD, int32_t count, float Q, hipStream_t stream) {
    hipLaunchKernelGGL(batch_ants_kernel, dim3(count), dim3(256), 0, stream, BD.insts, BD.pools,
                       BD.state, static_cast<double>(Q));
    return hipGetLastError();
}

hipError_t launch_batch_advance(const BatchDevice& BD, hipStream_t stream) {
    hipLaunchKernelGGL(batch_advance_kernel, dim3(1), dim3(1), 0, stream, BD.state, BD.gammas,
                       BD.queue);
    return hipGetLastError();
}

hipError_t launch_batch_arm(const BatchDevice& BD, uint32_t iter0, int32_t T,
                            hipStream_t stream) {
    hipLaunchKernelGGL(batch_arm_kernel, dim3(1), dim3(1), 0, stream, BD.state, BD.gammas,
                       BD.queue, iter0, T);
    return hipGetLastError();
}

}  // namespace aco
