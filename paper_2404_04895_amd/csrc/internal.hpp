// Internal declarations shared by the kernels' launchers and the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <rocprofiler-sdk-roctx/roctx.h>
#include <stddef.h>
#include <stdint.h>

#include "aco.h"

// Largest row the update kernel keeps in LDS (FP64 entries).
#define ACO_LDS_ROW_MAX ACO_MAX_CITIES

namespace aco {

// A named roctx range over the host side of one C-ABI call (it encloses the
// enqueueing of that call's kernels), so that a kernel trace taken with
// rocprofv3 --marker-trace shows which call launched what.  Without a
// profiler attached a push and a pop are two cheap library calls.
struct TraceRange {
    explicit TraceRange(const char* name) { roctxRangePushA(name); }
    ~TraceRange() { roctxRangePop(); }
    TraceRange(const TraceRange&) = delete;
    TraceRange& operator=(const TraceRange&) = delete;
};

// Sum of x[0], ..., x[n-1] widened to FP64, added in ascending index order
// (the sequential sum, bit for bit), by one workgroup: its threads stage
// kOrderedSumChunk values at a time in `stage` (LDS), and thread 0 adds them
// in order.  The result is valid in thread 0.
constexpr int32_t kOrderedSumChunk = 1024;

__device__ __forceinline__ double ordered_sum_f64(const float* __restrict__ x, int32_t n,
                                                  double* stage) {
    double total = 0.0;
    for (int32_t base = 0; base < n; base += kOrderedSumChunk) {
        const int32_t cnt = min(kOrderedSumChunk, n - base);
        for (int32_t k = static_cast<int32_t>(threadIdx.x); k < cnt;
             k += static_cast<int32_t>(blockDim.x))
            stage[k] = static_cast<double>(x[base + k]);
        __syncthreads();
        if (threadIdx.x == 0)
            for (int32_t k = 0; k < cnt; ++k) total += stage[k];
        __syncthreads();
    }
    return total;
}

// Best-so-far record kept on the device (written by the best-tour kernel).
struct BestRecord {
    float len;     // +inf before the first update
    int32_t iter;  // iteration that produced it, -1 before
    int32_t ant;   // ant index within that iteration
    int32_t pad;
};

// Device buffers carved from the caller's workspace.
struct Buffers {
    float* dist;        // n x ld
    float* tau;         // n x ld
    float* P;           // n x ld
    float* eta;         // n x ld (caller heuristic, when active)
    int32_t* tours;     // m_max x n
    float* lengths;     // m_max
    int32_t* succ;      // n x m_max: succ[c*m_max + a] = city after c in ant a's tour
    int32_t* pred;      // n x m_max: pred[c*m_max + a] = city before c
    int64_t* weight;    // m_max: quantised deposit of each ant (0 if not elite)
    int32_t* best_tour; // n
    BestRecord* best;   // 1
    float* row_min;     // n: nearest-neighbour distance of each city
    double* lower_bound;// 1: sum of row_min
    uint32_t* flags;    // 4 validation flags
    float* Ps;          // n x ld: each row of P sorted by value, descending
    uint16_t* Js;       // n x ld: the city of each entry of Ps
    unsigned long long* walk_stats;  // 3: sorted entries read, steps scanned, blocks scanned
};

struct Layout {
    size_t off_dist, off_tau, off_P, off_eta, off_tours, off_lengths, off_succ, off_pred,
        off_weight, off_best_tour, off_best, off_row_min, off_lower_bound, off_flags, off_Ps,
        off_Js, off_walk_stats, total;
};

Layout make_layout(int32_t n, int32_t ld, int32_t m_max);
Buffers carve(char* base, const Layout& L);

// Validation flag bits (for the input check kernels).
enum : uint32_t {
    kFlagNotFinite = 1u,
    kFlagNotPositive = 2u,
    kFlagAsymmetric = 4u,
    kFlagDiagonal = 8u,
};

// ---- launchers (each enqueues on `stream`, returns the launch status) ----
hipError_t launch_init_state(const float* dist_dense, int32_t n, int32_t ld, float tau0,
                             const Buffers& B, hipStream_t stream);
hipError_t launch_reset_tau(int32_t n, int32_t ld, float tau0, float* tau, float* P,
                            hipStream_t stream);
hipError_t launch_validate(const float* mat_dense, int32_t n, bool is_distance, float* row_min,
                           double* lower_bound, uint32_t* flags, hipStream_t stream);
hipError_t launch_copy_padded(const float* src_dense, float* dst, int32_t n, int32_t ld,
                              hipStream_t stream);
// selection: ACO_SELECT_* (the roulette wheel needs roulette_fits; the sorted
// walk needs the sorted rows in B.Ps / B.Js).
// walk: a step reads at most 64 * walk sorted entries before it falls back
// to the scan (ACO_SELECT_ADAIR_SORTED only).
hipError_t launch_construct(const Buffers& B, int32_t n, int32_t ld, int32_t m, int32_t m_max,
                            uint64_t seed, uint32_t iter, int32_t sched, int32_t selection,
                            int32_t walk, hipStream_t stream);
// Sort every row of P by value, descending, ties by city ascending: the
// first sorted_prefix(n, walk) entries of each row (all n when that is n).
hipError_t launch_sort_rows(const float* P, int32_t n, int32_t ld, int32_t walk, float* Ps,
                            uint16_t* Js, hipStream_t stream);
int32_t sorted_prefix(int32_t n, int32_t walk);
// Zero `count` (<= 64) 64-bit counters with a kernel (safe under graph capture).
hipError_t launch_clear_counters(unsigned long long* c, int32_t count, hipStream_t stream);
// Whether schedule `sched` can run the Roulette Wheel at n cities: the
// running totals of the ceil(ceil(n/4)/G) chunks of a row live one per lane.
bool roulette_fits(int32_t n, int32_t sched);
// Deposit weights of the m ants (elite set of Sec. 2.3) and the best-so-far
// record, one launch.
hipError_t launch_ants(const Buffers& B, int32_t n, int32_t m, uint32_t iter, int32_t elite_k,
                       float Q, int32_t S, hipStream_t stream);
hipError_t launch_clear_best(BestRecord* best, int32_t count, hipStream_t stream);
// tau_min, tau_max: MAX-MIN bounds applied after the update (0, +inf: none).
hipError_t launch_rows(const Buffers& B, int32_t n, int32_t ld, int32_t m, int32_t m_max,
                       bool apply_deposit, bool use_eta, float alpha, float beta, float rho,
                       int32_t S, float gamma, float tau_min, float tau_max,
                       hipStream_t stream);
hipError_t launch_uniforms(uint64_t seed, uint32_t iter, uint32_t ant, uint32_t step,
                           int32_t count, float* out, hipStream_t stream);
hipError_t prepare_kernels();
hipError_t prepare_sort_kernel();

// Error reporting shared by the C ABI files (thread-local message).
aco_status fail(aco_status st, const char* fmt, ...);
aco_status hip_fail(hipError_t e, const char* where);
void clear_error();
size_t align_up(size_t x, size_t a);
bool finite_positive(float x);

#define ACO_HIP(call, where)                                       \
    do {                                                           \
        hipError_t e_ = (call);                                    \
        if (e_ != hipSuccess) return ::aco::hip_fail(e_, where);   \
    } while (0)

// Largest S with m_max * Q / L_lb * 2^S < 2^62 (no pheromone cell can then
// overflow a signed 64-bit sum: a cell gets at most one weight per ant).
int32_t quantisation_exponent(double lower_bound, int32_t m_max, float Q);

}  // namespace aco
