// Descriptors shared by the construct kernels, the batched engine and the C ABI.
#pragma once

#include "internal.hpp"
#include "philox.hpp"

namespace aco {

// One instance as the construct code sees it (single instance or one member
// of a batch).
struct InstanceView {
    const float* P;      // n x ld transition matrix
    const float* dist;   // n x ld distances
    int32_t n, ld;
    int32_t* tours;      // ants x n
    float* lengths;      // ants
    int32_t* succ;       // n x m_stride
    int32_t* pred;       // n x m_stride
    int32_t m_stride;
    uint32_t key0, key1, iter;
    const float* Ps;     // n x ld rows of P sorted by value (sorted walk only)
    const uint16_t* Js;  // n x ld city of each sorted entry
    int32_t sorted_ld;   // row stride of Ps / Js: the K entries each row keeps
    int32_t walk;        // sorted batches per step before the scan
    unsigned long long* walk_stats;  // sorted walk: entries read, steps scanned, blocks scanned
};

// Per-step selection rules (the ACO_SELECT_* codes of the C ABI).
enum : int32_t { kSelAdaIR = 0, kSelRoulette = 1, kSelSorted = 2 };

// Construct schedules: lanes per ant and whether the live-block list is kept.
// The numeric codes are the ACO_SCHED_* values of the C ABI.
enum : int32_t {
    kSched16 = 0,      // 16 lanes per ant, 4 ants per wave
    kSched32 = 1,      // 32 lanes per ant, 2 ants per wave
    kSched32Live = 2,  // 32 lanes per ant, live-block list
    kSched64 = 3,      // one ant per wave
    kSched64Live = 4,  // one ant per wave, live-block list
    kSchedSorted = ACO_SCHED_SORTED,  // batch only: OR'd into 16, 32, 64 for the sorted walk
};

__host__ __device__ constexpr int32_t mask_words(int32_t nblk) { return (nblk + 7) >> 3; }

// LDS words one ant of a group of `lanes` lanes needs: the window of edge
// lengths (one double per lane), a guard word with every bit set (the
// visited mark of "city -1", an empty entry of the sorted walk), the visited
// marks -- one bit per city, or one byte per city (`bytes`, the sorted walk
// without a live list: its test is then one byte load) -- then (optionally)
// the u16 list of live blocks; rounded up to 16 bytes, so that every group's
// window is aligned for 16-byte reads.
__host__ __device__ constexpr int32_t group_lds_words(int32_t n, bool live, int32_t lanes,
                                                      bool bytes = false) {
    return (2 * lanes + 1 + (bytes ? (n + 3) >> 2 : mask_words((n + 3) >> 2)) +
            (live ? (((n + 3) >> 2) + 1) / 2 : 0) + 3) & ~3;
}

int32_t schedule_lanes(int32_t sched);
bool schedule_live(int32_t sched);
bool schedule_valid(int32_t sched);
int32_t default_schedule(int32_t n);
// Schedule of the sorted walk for m ants when none is forced: no live list
// (the walk decides almost every step), and the narrowest group (fewest
// instructions per ant-step) that still leaves two wavefronts per SIMD to
// hide the latency of each step's chain.
int32_t sorted_default_schedule(int32_t m);
size_t wave_lds_bytes(int32_t n, int32_t sched);

// ---- batched engine --------------------------------------------------------
struct BatchInstance {
    int32_t n, ld, m, elite_k;
    int64_t off_mat;     // element offset into the dist / tau / P / eta pools (n x ld)
    int64_t off_tours;   // into the tours pool (m x n)
    int64_t off_succ;    // into the succ / pred pools (n x m)
    int64_t off_ants;    // into the lengths / weights pools (m)
    int64_t off_cities;  // into the best-tour pool (n)
    int64_t off_sorted;  // into the sorted-row pools (n x n), if `sorted`
    uint32_t key0, key1;
    int32_t S;           // deposit quantisation exponent
    int32_t sorted;      // 1: constructs with the sorted walk; its rows are sorted each iteration
};

struct BatchTask {
    int32_t instance, ant0, nants, schedule;
};

struct RowTask {
    int32_t instance, row;
};

// Iteration counters read by the kernels of a captured iteration and
// advanced on the device by its last kernel.
struct IterState {
    uint32_t iter;        // generator iteration word of the current iteration
    int32_t t;            // index into the run's gamma schedule
    int32_t T;            // iterations in the run
    float gamma_next;     // gamma for the P built at the end of this iteration
};

struct BatchPools {
    float* dist;
    float* tau;
    float* P;
    int32_t* tours;
    float* lengths;
    int32_t* succ;
    int32_t* pred;
    int64_t* weight;
    int32_t* best_tour;
    BestRecord* best;
    float* sorted_p;     // rows of P sorted by value, whole (instances with `sorted`)
    uint16_t* sorted_j;  // their cities
    unsigned long long* walk_stats;  // 3 counters of the sorted walks, as a single instance's
};

// Sorted batches a batch member's walk reads before it scans (the default of
// a single instance).
constexpr int32_t kBatchWalk = 8;

// Construct task queues of the batched engine: one per XCD.  Persistent
// wave w drains queue w mod kQueues first (workgroups are dispatched to the
// XCDs in turn), then helps the others, so an instance's rows stay in the
// L2 of the XCD that runs its ants.
constexpr int32_t kQueues = 8;

struct BatchDevice {
    BatchInstance* insts;
    BatchTask* tasks;        // queue by queue
    int32_t* queue_start;    // kQueues + 1: first task of each queue, then the total
    RowTask* rows;
    RowTask* sort_rows;      // the rows of the members on the sorted walk
    uint32_t* queue;         // kQueues counters
    IterState* state;
    float* gammas;  // T + 1 entries
    BatchPools pools;
};

hipError_t launch_construct_view(const InstanceView& I, int32_t m, int32_t sched,
                                 int32_t selection, hipStream_t stream);
hipError_t launch_batch_construct(const BatchDevice& BD, int32_t ntasks, size_t lds_bytes,
                                  int32_t grid, hipStream_t stream);
// Sort the rows of P of the batch members marked `sorted` (the first `nrows`
// entries of BD.sort_rows; members with n <= ACO_BATCH_SORTED_MAX_N).
hipError_t launch_batch_sort_rows(const BatchDevice& BD, int32_t nrows, hipStream_t stream);
hipError_t launch_batch_rows(const BatchDevice& BD, int32_t nrows, int32_t max_ld,
                             const float* gamma_ptr, bool apply_deposit, float alpha, float beta,
                             float rho, hipStream_t stream);
hipError_t launch_batch_ants(const BatchDevice& BD, int32_t count, float Q, hipStream_t stream);
hipError_t launch_batch_advance(const BatchDevice& BD, hipStream_t stream);
hipError_t launch_batch_arm(const BatchDevice& BD, uint32_t iter0, int32_t T,
                            hipStream_t stream);

}  // namespace aco
