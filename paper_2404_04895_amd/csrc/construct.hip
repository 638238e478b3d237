// Tour construction by Adaptive Independent Roulette (Sec. 2.2, Sec. 2.4).
//
// An ant is a group of G lanes of one wavefront (G = 64: one ant per wave;
// G = 32 or 16: two or four ants share a wave, for small instances).  The
// ants of Sec. 2.2's function mapping are independent, so no group ever waits
// on another.  At every step a group streams the current city's row of P as
// one float4 per lane, draws the four deviates of each 4-city block with one
// Philox call per lane, scores each unvisited city by fl32(P[c,j] * r_j) and
// reduces the lane winners to the group's argmax.
//
// Per-group LDS: the visited bitmask (one bit per city; cities at or past n
// are pre-set) and, when the live-block list is on, the sorted indices of the
// 4-city blocks that still hold an unvisited city.  A block leaves the list
// when its last city is taken, so a step scans only live blocks.  The
// generator is keyed by block index, not list position or lane, so the group
// width and the list change no result.
//
// The Roulette Wheel baseline (the proportional rule that IR replaces; the
// ablation of Sec. 3) runs in the same skeleton with another per-step
// selection: the inverse of the cumulative distribution of the unvisited
// cities in ascending order, in FP64, with one deviate per step.
//
// Outputs per ant: the tour (m x n int32), its closed length (FP64 sum in
// tour order, rounded once to FP32 -- the fitness f of Eq. (3)), and the
// successor / predecessor of every city, stored city-major so that the
// update kernel reads one contiguous row of each per city (Eq. (2)'s index
// matrix, held as two maps).  They are written once per G steps from a
// register window, so no scattered store or distance gather sits between
// one step's decision and the next step's loads.
#include "construct.hpp"

namespace aco {

namespace {

constexpr int kWave = 64;

// Key of one candidate: the FP32 bit pattern of fl32(P[c,j] * r_j) with the
// city's visited bit in the sign position.  Scores are >= +0, so unvisited
// keys are >= 0 and order like the scores, while visited keys are negative
// and can never beat the initial -1.
__device__ __forceinline__ int32_t score_key(float p, uint32_t word, uint32_t taken_sign) {
    // 0x3F800000 | (word >> 9): the funnel shift brings 0x7F in above the top
    // 23 bits of the word, i.e. 1 + k*2^-23; minus (1 - 2^-24) gives the
    // deviate (2k+1)*2^-24 exactly.
    const float unit = __uint_as_float(__builtin_amdgcn_alignbit(0x7Fu, word, 9)) - 0x1.fffffep-1f;
    const float score = p * unit;
    return static_cast<int32_t>(__float_as_uint(score) | taken_sign);
}

// All-reduce over the G lanes of a group (every lane gets the result):
// quad butterflies, rotations by 4 and 8 within each 16-lane row, then the
// permlane swaps that pair rows (G >= 32) and wave halves (G = 64).
// The DPP moves take the operation's identity as their old value: every
// source lane of these patterns lies in the same row, so the identity is only
// ever seen from a lane that exec has switched off, and it lets the compiler
// fold each move into the max / min itself (one DPP instruction per stage).
template <int G, bool IS_MAX>
__device__ __forceinline__ int32_t group_reduce(int32_t v) {
    auto op = [](int32_t a, int32_t b) { return IS_MAX ? max(a, b) : min(a, b); };
    constexpr int32_t id = IS_MAX ? INT32_MIN : INT32_MAX;
    v = op(v, __builtin_amdgcn_update_dpp(id, v, 0xB1, 0xF, 0xF, false));   // quad_perm [1,0,3,2]
    v = op(v, __builtin_amdgcn_update_dpp(id, v, 0x4E, 0xF, 0xF, false));   // quad_perm [2,3,0,1]
    v = op(v, __builtin_amdgcn_update_dpp(id, v, 0x124, 0xF, 0xF, false));  // row_ror:4
    v = op(v, __builtin_amdgcn_update_dpp(id, v, 0x128, 0xF, 0xF, false));  // row_ror:8
    if constexpr (G >= 32) {
        const auto sw = __builtin_amdgcn_permlane16_swap(static_cast<uint32_t>(v),
                                                         static_cast<uint32_t>(v), false, false);
        v = op(static_cast<int32_t>(sw[0]), static_cast<int32_t>(sw[1]));
    }
    if constexpr (G == 64) {
        const auto sw = __builtin_amdgcn_permlane32_swap(static_cast<uint32_t>(v),
                                                         static_cast<uint32_t>(v), false, false);
        v = op(static_cast<int32_t>(sw[0]), static_cast<int32_t>(sw[1]));
    }
    return v;
}

template <int G>
__device__ __forceinline__ int32_t group_sum(int32_t v) {
    v += __builtin_amdgcn_update_dpp(0, v, 0xB1, 0xF, 0xF, false);
    v += __builtin_amdgcn_update_dpp(0, v, 0x4E, 0xF, 0xF, false);
    v += __builtin_amdgcn_update_dpp(0, v, 0x124, 0xF, 0xF, false);
    v += __builtin_amdgcn_update_dpp(0, v, 0x128, 0xF, 0xF, false);
    if constexpr (G >= 32) {
        const auto sw = __builtin_amdgcn_permlane16_swap(static_cast<uint32_t>(v),
                                                         static_cast<uint32_t>(v), false, false);
        v = static_cast<int32_t>(sw[0] + sw[1]);
    }
    if constexpr (G == 64) {
        const auto sw = __builtin_amdgcn_permlane32_swap(static_cast<uint32_t>(v),
                                                         static_cast<uint32_t>(v), false, false);
        v = static_cast<int32_t>(sw[0] + sw[1]);
    }
    return v;
}

// The value is the same on every lane of the group; for G = 64 that makes it
// wave-uniform, which lets the compiler keep it in a scalar register.
template <int G>
__device__ __forceinline__ int32_t group_uniform(int32_t v) {
    if constexpr (G == 64) return __builtin_amdgcn_readfirstlane(v);
    return v;
}

// ---- roulette wheel helpers ----------------------------------------------

__device__ __forceinline__ double f64_from_halves(uint32_t lo, uint32_t hi) {
    return __longlong_as_double(static_cast<long long>((static_cast<uint64_t>(hi) << 32) | lo));
}

__device__ __forceinline__ uint32_t f64_lo(double v) {
    return static_cast<uint32_t>(static_cast<uint64_t>(__double_as_longlong(v)));
}

__device__ __forceinline__ uint32_t f64_hi(double v) {
    return static_cast<uint32_t>(static_cast<uint64_t>(__double_as_longlong(v)) >> 32);
}

// v from the lane CTRL names within the 16-lane row; lanes without a source
// in the row get +0.
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
    const uint32_t lo = static_cast<uint32_t>(
        __builtin_amdgcn_update_dpp(0, static_cast<int>(f64_lo(v)), CTRL, 0xF, 0xF, false));
    const uint32_t hi = static_cast<uint32_t>(
        __builtin_amdgcn_update_dpp(0, static_cast<int>(f64_hi(v)), CTRL, 0xF, 0xF, false));
    return f64_from_halves(lo, hi);
}

__device__ __forceinline__ double readlane_f64(double v, int32_t lane) {
    const uint32_t lo =
        static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(f64_lo(v)), lane));
    const uint32_t hi =
        static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(f64_hi(v)), lane));
    return f64_from_halves(lo, hi);
}

// Inclusive prefix sum over the G lanes of a group, in a fixed association:
// shifts by 1, 2, 4, 8 within each 16-lane row, then the row totals.
template <int G>
__device__ __forceinline__ double group_scan_f64(double v) {
    v += dpp_f64<0x111>(v);  // row_shr:1
    v += dpp_f64<0x112>(v);  // row_shr:2
    v += dpp_f64<0x114>(v);  // row_shr:4
    v += dpp_f64<0x118>(v);  // row_shr:8
    const int32_t lane = threadIdx.x & (kWave - 1);
    if constexpr (G >= 32) {
        const double r15 = readlane_f64(v, 15);
        const double r47 = readlane_f64(v, 47);
        if ((lane & 31) >= 16) v += (lane < 32) ? r15 : r47;
    }
    if constexpr (G == 64) {
        const double r31 = readlane_f64(v, 31);
        if (lane >= 32) v += r31;
    }
    return v;
}

// The value of the group's last lane, on every lane of the group.
template <int G>
__device__ __forceinline__ double group_last_f64(double v) {
    if constexpr (G == 64) {
        return readlane_f64(v, 63);
    } else {
        const int32_t g = (threadIdx.x & (kWave - 1)) / G;
        double r = 0.0;
#pragma unroll
        for (int32_t k = 0; k < kWave / G; ++k) {
            const double t = readlane_f64(v, k * G + G - 1);
            if (g == k) r = t;
        }
        return r;
    }
}

// Block b of the row with the visited cities' weights set to +0.
__device__ __forceinline__ float4 masked_block(const float* row, const uint32_t* visited,
                                               int32_t b) {
    float4 p = *reinterpret_cast<const float4*>(row + 4 * b);
    const uint32_t taken = visited[b >> 3] >> ((b & 7) << 2);
    p.x = (taken & 1u) ? 0.0f : p.x;
    p.y = (taken & 2u) ? 0.0f : p.y;
    p.z = (taken & 4u) ? 0.0f : p.z;
    p.w = (taken & 8u) ? 0.0f : p.w;
    return p;
}

// Weight of a block: its four entries summed in city order in FP64.
__device__ __forceinline__ double block_weight(float4 p) {
    return ((static_cast<double>(p.x) + static_cast<double>(p.y)) + static_cast<double>(p.z)) +
           static_cast<double>(p.w);
}

// One Roulette Wheel step of group g: city j with probability P[c,j] over
// the sum of P[c,k] for the unvisited k.  Pass 1 streams the live blocks in
// ascending order, G blocks (one chunk) at a time; lane k of the group keeps
// the running total before and after chunk k (nblk <= G*G is required).
// The deviate of counter (0, s, ant, iter) sets x = v * total; pass 2
// re-reads the first chunk whose closing total exceeds x and takes the first
// city of positive weight whose running sum exceeds x.  All sums are FP64;
// they are associated per chunk rather than strictly left to right, so a
// different city than a sequential sum's can only come from an x within
// rounding of a boundary.  With no positive weight left, the smallest
// unvisited city is taken.
template <int G, bool LIVE>
__device__ __forceinline__ int32_t roulette_select(const InstanceView& I, const float* row,
                                                   const uint32_t* visited,
                                                   const uint16_t* live, int32_t span,
                                                   int32_t gl, int32_t g, int32_t s,
                                                   int32_t ant) {
    double run = 0.0;
    double chunk_lo = 0.0;
    double chunk_hi = 0.0;
    int32_t nchunks = 0;
    for (int32_t base = 0; base < span; base += G, ++nchunks) {
        const int32_t pos = base + gl;
        double w = 0.0;
        if (pos < span) w = block_weight(masked_block(row, visited, LIVE ? live[pos] : pos));
        const double total = group_last_f64<G>(group_scan_f64<G>(w));
        if (gl == nchunks) chunk_lo = run;
        run += total;
        if (gl == nchunks) chunk_hi = run;
    }
    // the smallest unvisited city (one exists: fewer than n cities are taken)
    auto smallest_free = [&]() {
        int32_t first = 0x7FFFFFFF;
        for (int32_t base = 0; base < span; base += G) {
            const int32_t pos = base + gl;
            if (pos < span) {
                const int32_t b = LIVE ? static_cast<int32_t>(live[pos]) : pos;
                const uint32_t free = ~(visited[b >> 3] >> ((b & 7) << 2)) & 0xFu;
                if (free) first = min(first, 4 * b + __builtin_ctz(free));
            }
        }
        return group_reduce<G, false>(first);
    };
    if (!(run > 0.0)) return smallest_free();
    const PhiloxOut d = philox10(0u, static_cast<uint32_t>(s), static_cast<uint32_t>(ant), I.iter,
                                 I.key0, I.key1);
    const double x = static_cast<double>(unit_from_word(d.w0)) * run;
    // x < run (the deviate is below 1), so the last chunk's closing total
    // exceeds it; the guard below only keeps C in range
    const uint64_t group_bits = (G == 64) ? ~0ull : ((1ull << (G & 63)) - 1ull);
    const uint64_t over = (__ballot(gl < nchunks && chunk_hi > x) >> (g * G)) & group_bits;
    const int32_t C = over ? __builtin_ctzll(over) : nchunks - 1;
    const double lo = __shfl(chunk_lo, g * G + C);
    const int32_t pos = C * G + gl;
    float4 p = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    int32_t b = 0;
    if (pos < span) {
        b = LIVE ? static_cast<int32_t>(live[pos]) : pos;
        p = masked_block(row, visited, b);
    }
    const double incl = group_scan_f64<G>(block_weight(p));
    double excl = __shfl_up(incl, 1, G);
    if (gl == 0) excl = 0.0;
    int32_t pick = 0x7FFFFFFF;
    int32_t last = -1;
    if (pos < span) {
        const float q[4] = {p.x, p.y, p.z, p.w};
        double acc = 0.0;
#pragma unroll
        for (int32_t k = 0; k < 4; ++k) {
            acc = (k == 0) ? static_cast<double>(q[0]) : acc + static_cast<double>(q[k]);
            const bool positive = __float_as_uint(q[k]) != 0u;
            if (positive) last = 4 * b + k;
            if (pick == 0x7FFFFFFF && positive && lo + (excl + acc) > x) pick = 4 * b + k;
        }
    }
    pick = group_reduce<G, false>(pick);
    // rounding can leave x past the last running sum of the chunk: its last
    // city of positive weight then takes the draw (the chunk has one)
    if (pick == 0x7FFFFFFF) pick = group_reduce<G, true>(last);
    if (pick < 0) pick = smallest_free();
    return pick;
}

// Build the tours of up to 64/G ants of one instance: group g of this wave
// builds ant ant0 + g if g < nants.  `lds` is this wave's LDS region of
// (64/G) * group_lds_words(n, LIVE, G) words.
// Offset of row c of a matrix with leading dimension ld.  Both are below
// 2^15 (at most 16384 cities, padded), so a 24-bit multiply, which runs at
// the full VALU rate, gives the exact product.
__device__ __forceinline__ size_t row_offset(int32_t c, int32_t ld) {
    const uint32_t e = __umul24(static_cast<uint32_t>(c), static_cast<uint32_t>(ld));
    return static_cast<size_t>(e);
}

// Chunks of the row a scanning step loads before it scores the first: four
// where a scan is latency-bound (the small instances of a batch, the batch's
// walk fallbacks), eight for the rare fallback of one large instance's walk
// (its row is long: fewer round trips per scanned step; the batch kernel
// would pay for the registers everywhere), one for the full scan of one large
// instance, which is bound by HBM and slowed by the extra loads in flight.
constexpr int32_t kScanAhead = 4;
constexpr int32_t kWalkScanAhead = 8;

// ---- per-window output -----------------------------------------------------

// Lane k of the calling lane's group (k the same on every lane of the wave).
template <int G>
__device__ __forceinline__ int32_t group_lane(int32_t v, int32_t k) {
    if constexpr (G == kWave) {
        return __builtin_amdgcn_readlane(v, k);
    } else {
        const int32_t g = (threadIdx.x & (kWave - 1)) / G;
        int32_t r = 0;
#pragma unroll
        for (int32_t q = 0; q < kWave / G; ++q) {
            const int32_t t = __builtin_amdgcn_readlane(v, q * G + k);
            if (g == q) r = t;
        }
        return r;
    }
}

// Write out a window of the tour: lane l of the group holds entry base + l
// (l < cnt); `prev` is the entry before the window (-1 for the first).  Each
// lane writes its entry and the successor / predecessor maps of the edge
// that ends at it, and gathers that edge's length into the group's LDS
// window (+0 where there is no edge).  The group's first lane then adds the
// window to `len` entry by entry in tour order, so the FP64 sum is the
// sequential one (adding +0 to a sum of non-negative terms changes nothing).
// Runs once per G steps, which keeps scattered stores and the random
// distance gathers out of the per-step chain.
template <int G>
__device__ __forceinline__ void flush_window(const InstanceView& I, int32_t* tour, int32_t ant,
                                             int32_t base, int32_t cnt, int32_t win,
                                             int32_t prev, int32_t gl, double* window,
                                             double& len) {
    int32_t from = __shfl_up(win, 1, G);
    if (gl == 0) from = prev;
    float d = 0.0f;
    if (gl < cnt) {
        tour[base + gl] = win;
        if (from >= 0) {
            I.succ[static_cast<size_t>(from) * I.m_stride + ant] = win;
            I.pred[static_cast<size_t>(win) * I.m_stride + ant] = from;
            d = I.dist[static_cast<size_t>(from) * I.ld + win];
        }
    }
    window[gl] = static_cast<double>(d);
    // the group's first lane reads what the other lanes just wrote
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    if (gl == 0) {
        double acc = len;
#pragma unroll
        for (int32_t k = 0; k < G; k += 2) {
            const double2 pair = *reinterpret_cast<const double2*>(window + k);
            acc += pair.x;
            acc += pair.y;
        }
        len = acc;
    }
    // the window is written again G steps later; no lane may get there first
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// The sorted rows as buffer resources: a load then takes one 32-bit offset in
// a VGPR (the base and the range sit in SGPRs), and an offset past the range
// reads zero.  Rows are K entries apart, K the prefix each keeps, so that the
// first batches of all rows lie close together.
constexpr int32_t kBufferWord3 = 0x00020000;  // raw 32-bit loads on gfx9-family chips

struct SortedRows {
    __amdgpu_buffer_rsrc_t p;  // FP32 values
    __amdgpu_buffer_rsrc_t j;  // uint16 cities
};

__device__ __forceinline__ SortedRows sorted_rows(const InstanceView& I) {
    const int32_t elems = I.n * I.sorted_ld;  // at most 2^28
    return {__builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(I.Ps), 0, 4 * elems, kBufferWord3),
            __builtin_amdgcn_make_buffer_rsrc(const_cast<uint16_t*>(I.Js), 0, 2 * elems,
                                              kBufferWord3)};
}

__device__ __forceinline__ float sorted_p(const SortedRows& R, uint32_t e) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(R.p, 4 * e, 0, 0));
}

__device__ __forceinline__ int32_t sorted_j(const SortedRows& R, uint32_t e) {
    return static_cast<int32_t>(__builtin_amdgcn_raw_buffer_load_b16(R.j, 2 * e, 0, 0));
}

// The transition matrix as a buffer resource (n x ld FP32), and block b of
// row c through it: one 16-byte load from a 32-bit offset.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t matrix_rows(const InstanceView& I) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(I.P), 0, 4 * (I.n * I.ld),
                                             kBufferWord3);
}

__device__ __forceinline__ float4 matrix_block(__amdgpu_buffer_rsrc_t R, uint32_t row_e,
                                               int32_t b) {
    return __builtin_bit_cast(
        float4, __builtin_amdgcn_raw_buffer_load_b128(R, 4 * (row_e + 4 * static_cast<uint32_t>(b)), 0, 0));
}

// The first batch of one row's sorted entries, loaded one step ahead for
// the city most likely to be taken next (`city` is -1 when there is none).
struct SortedSpec {
    int32_t city;  // same on every lane of the group
    float p;       // this lane's entry of the batch
    int32_t j;     // its city; -1 (with p = 0) for a lane past the row's end
};

// -1 if x has a bit set, else 0.  For wave-uniform x (a ballot), so the
// compare and the select stay on the scalar unit.
__device__ __forceinline__ uint32_t scalar_any(uint32_t x) {
    uint32_t r;
    asm("s_cmp_lg_u32 %1, 0\n\ts_cselect_b32 %0, -1, 0" : "=s"(r) : "s"(x) : "scc");
    return r;
}

// Lane mask of the groups (G lanes each) that have a bit set in `ballot`.
template <int G>
__device__ __forceinline__ uint64_t groups_with_any(uint64_t ballot) {
    const uint32_t lo = static_cast<uint32_t>(ballot);
    const uint32_t hi = static_cast<uint32_t>(ballot >> 32);
    if constexpr (G == kWave) {
        const uint64_t a = scalar_any(lo | hi);
        return a | (a << 32);
    } else if constexpr (G == 32) {
        return static_cast<uint64_t>(scalar_any(lo)) | (static_cast<uint64_t>(scalar_any(hi)) << 32);
    } else {
        static_assert(G == 16, "groups of 16, 32 or 64 lanes");
        const uint32_t l = (scalar_any(lo & 0xFFFFu) & 0xFFFFu) | (scalar_any(lo >> 16) & 0xFFFF0000u);
        const uint32_t h = (scalar_any(hi & 0xFFFFu) & 0xFFFFu) | (scalar_any(hi >> 16) & 0xFFFF0000u);
        return static_cast<uint64_t>(l) | (static_cast<uint64_t>(h) << 32);
    }
}

// Whether any lane of the calling lane's group has its bit set in `ballot`.
template <int G>
__device__ __forceinline__ bool group_any(uint64_t ballot) {
    return __builtin_amdgcn_inverse_ballot_w64(groups_with_any<G>(ballot));
}

// v of the first lane of the calling lane's group whose bit is set in
// `ballot`, or -1 if none is set.  The lane indices are wave-uniform: per
// group a scalar find-first and one readlane, then a select by group.
template <int G>
__device__ __forceinline__ int32_t group_first(uint64_t ballot, int32_t v) {
    if constexpr (G == kWave) {
        const int32_t t = __builtin_amdgcn_readlane(v, __builtin_ctzll(ballot | (1ull << 63)));
        return t | static_cast<int32_t>(~scalar_any(static_cast<uint32_t>(ballot) |
                                                    static_cast<uint32_t>(ballot >> 32)));
    } else {
        constexpr int32_t kGroups = kWave / G;
        constexpr uint32_t kMask = (G == 32) ? 0xFFFFFFFFu : ((1u << (G & 31)) - 1u);
        int32_t r = 0;
#pragma unroll
        for (int32_t q = 0; q < kGroups; ++q) {
            const uint32_t bits = static_cast<uint32_t>(ballot >> (q * G)) & kMask;
            // an empty group reads its last lane; the OR then makes it -1
            const int32_t first = __builtin_ctz(bits | (1u << (G - 1)));
            const int32_t t = __builtin_amdgcn_readlane(v, q * G + first) |
                              static_cast<int32_t>(~scalar_any(bits));
            const uint64_t group_q = (G == 32 ? 0xFFFFFFFFull : ((1ull << G) - 1ull)) << (q * G);
            r = (q == 0 || __builtin_amdgcn_inverse_ballot_w64(group_q)) ? t : r;
        }
        return r;
    }
}

// Sorted walk of one step of group g: read the row's entries in descending
// P order, G per batch (one per lane), score the unvisited ones and keep each
// lane's best (largest key, then smallest city).  Every deviate is below 1,
// so no city scores above its P: once the smallest P of a batch is below the
// best score so far, no later entry can reach it and the step is decided.
// The walk reads at most 64 * walk entries.  Returns the city, or -1 if that
// did not decide the step; `entries_read` counts the entries read.
//
// The first unvisited entry of the first batch is the likeliest next city
// (it has the largest P left).  The first batch of its row is loaded as soon
// as that entry is known, while the deviates are still being drawn; the next
// step uses it if that city is taken.  Only where the data comes from
// changes, not the result.
template <int G, bool BYTES>
__device__ __forceinline__ int32_t sorted_walk(const InstanceView& I, int32_t cur,
                                               const uint32_t* visited, int32_t gl, int32_t s,
                                               const PhiloxAnt& pant, uint32_t& entries_read,
                                               SortedSpec& spec) {
    const SortedRows R = sorted_rows(I);
    // the deviates' counter words shared by every candidate of this step
    const PhiloxStep pstep = philox_step(pant, static_cast<uint32_t>(s), I.key1);
    const uint32_t iter_k1 = I.iter ^ I.key1;
    const uint32_t off = __umul24(static_cast<uint32_t>(cur), static_cast<uint32_t>(I.sorted_ld));
    int32_t best_key = -1;
    int32_t best_j = 0x7FFFFFFF;
    // 64 * walk is a multiple of G, so a batch is partial only when the limit
    // is n itself; its empty lanes then read P = 0 and nothing follows them
    const int32_t limit = min(64 * I.walk, I.n);
    const bool ahead = spec.city == cur;
    for (int32_t base = 0; base < limit; base += G) {
        // the step's first entries, their visited bits and the next
        // speculative load form the chain every step waits on: issue them
        // ahead of other wavefronts' deviates
        if (base == 0) __builtin_amdgcn_s_setprio(2);
        const int32_t pos = base + gl;
        float p = 0.0f;
        int32_t j = -1;
        if (base == 0 && ahead) {
            // a lane at or past the limit never loads a speculative entry and
            // keeps the empty one (0, -1)
            p = spec.p;
            j = spec.j;
        } else if (pos < limit) {
            p = sorted_p(R, off + pos);
            j = sorted_j(R, off + pos);
        }
        // an empty lane (j = -1) reads the last mark of the guard word, which
        // is set, so the test needs no branch and no range check
        bool cand;
        if constexpr (BYTES) {
            cand = reinterpret_cast<const uint8_t*>(visited)[j] == 0;
        } else {
            cand = !((visited[j >> 5] >> (j & 31)) & 1u);
        }
        if (base == 0) {
            spec.city = group_first<G>(__builtin_amdgcn_ballot_w64(cand), j);
            if (spec.city >= 0 && gl < limit) {
                const uint32_t next =
                    __umul24(static_cast<uint32_t>(spec.city), static_cast<uint32_t>(I.sorted_ld)) + gl;
                spec.p = sorted_p(R, next);
                spec.j = sorted_j(R, next);
            }
            __builtin_amdgcn_s_setprio(0);
        }
        if (cand) {
            const PhiloxOut r = philox10_candidate(static_cast<uint32_t>(j >> 2), pstep,
                                                   iter_k1, I.key0, I.key1);
            // word j mod 4 of the block's four, picked without a branch
            const uint32_t w01 = (j & 1) ? r.w1 : r.w0;
            const uint32_t w23 = (j & 1) ? r.w3 : r.w2;
            const uint32_t w = (j & 2) ? w23 : w01;
            const int32_t key = score_key(p, w, 0u);
            // a lane's first candidate needs no compare: scores are >= +0
            if (base == 0 || key > best_key || (key == best_key && j < best_j)) {
                best_key = key;
                best_j = j;
            }
        }
        entries_read += static_cast<uint32_t>(G);
        // the decision gates the next step: ahead of other deviates too
        __builtin_amdgcn_s_setprio(1);
        const int32_t top = group_reduce<G, true>(best_key);
        // the batch's last entry has its smallest P, so some entry below the
        // best score is the same as the last one below it; an empty lane
        // (P = 0, only at the end of a row) is below any positive score, as
        // the missing entries after it are
        const bool below = group_any<G>(__builtin_amdgcn_ballot_w64(p < __int_as_float(top)));
        if (top >= 0 && below)
            return group_reduce<G, false>(best_key == top ? best_j : 0x7FFFFFFF);
    }
    return -1;
}

template <int G, bool LIVE, int SEL = kSelAdaIR, int AHEAD = kScanAhead>
__device__ void construct_group(const InstanceView& I, int32_t ant0, int32_t nants,
                                uint32_t* __restrict__ lds) {
    const int32_t lane = threadIdx.x & (kWave - 1);
    const int32_t g = lane / G;
    const int32_t gl = lane % G;
    if (g >= nants) return;  // whole groups idle; no lane of an active group depends on them
    const int32_t n = I.n;
    const int32_t ant = ant0 + g;
    // the sorted walk without a live list marks visited cities by bytes
    constexpr bool kBytes = SEL == kSelSorted && !LIVE;
    const int32_t nblk = (n + 3) >> 2;
    const int32_t nwords = kBytes ? nblk : mask_words(nblk);
    uint32_t* area = lds + g * group_lds_words(n, LIVE, G, kBytes);
    double* lengths_window = reinterpret_cast<double*>(area);
    uint32_t* visited = area + 2 * G + 1;  // visited[-1] is the guard word
    uint8_t* vmap = reinterpret_cast<uint8_t*>(visited);  // the byte marks (kBytes)
    uint16_t* live = reinterpret_cast<uint16_t*>(visited + nwords);

    for (int32_t w = gl - 1; w < nwords; w += G) {
        uint32_t bits = 0u;
        if constexpr (kBytes) {
            // word w holds the marks of cities 4w .. 4w+3; cities at or past n
            // (and the guard) are marked
            if (w < 0) {
                bits = 0x80808080u;
            } else {
#pragma unroll
                for (int32_t k = 0; k < 4; ++k)
                    if (4 * w + k >= n) bits |= 0x80u << (8 * k);
            }
        } else {
            const int32_t j0 = w * 32;
            if (w < 0 || j0 + 32 > n)
                bits = (w < 0 || j0 >= n) ? 0xFFFFFFFFu : (0xFFFFFFFFu << (n - j0));
        }
        visited[w] = bits;
    }
    if constexpr (LIVE) {
        for (int32_t i = gl; i < nblk; i += G) live[i] = static_cast<uint16_t>(i);
    }
    int32_t nlive = nblk;
    uint32_t walk_entries = 0, scanned_steps = 0, scanned_blocks = 0;
    SortedSpec spec{-1, 0.0f, -1};
    const PhiloxAnt pant = philox_ant(static_cast<uint32_t>(ant), I.key0);
    __builtin_amdgcn_wave_barrier();

    // Start city (Sec. 2.2 initialization): word 0 of counter (0, 0, ant, iter).
    const PhiloxOut s0 = philox10(0u, 0u, static_cast<uint32_t>(ant), I.iter, I.key0, I.key1);
    const int32_t start = static_cast<int32_t>(__umulhi(s0.w0, static_cast<uint32_t>(n)));

    int32_t* tour = I.tours + static_cast<size_t>(ant) * n;
    int32_t cur = start;
    int32_t next = start;
    double len = 0.0;
    int32_t win = 0;     // lane (s mod G) keeps tour entry s until its window is written
    int32_t prev = -1;   // last entry of the previous window

    for (int32_t s = 0; s < n; ++s) {
        int32_t walked = -1;
        if constexpr (SEL == kSelSorted) {
            if (s > 0) {
                walked = group_uniform<G>(sorted_walk<G, kBytes>(I, cur, visited, gl, s, pant,
                                                                  walk_entries, spec));
            }
        }
        if (SEL == kSelRoulette && s > 0) {
            const float* row = I.P + row_offset(cur, I.ld);
            next = group_uniform<G>(roulette_select<G, LIVE>(I, row, visited, live,
                                                              LIVE ? nlive : nblk, gl, g, s, ant));
        } else if (walked >= 0) {
            next = walked;
        } else if (s > 0) {
            if constexpr (SEL == kSelSorted) {
                // the walk left this step undecided
                ++scanned_steps;
                scanned_blocks += static_cast<uint32_t>(LIVE ? nlive : nblk);
            }
            const __amdgpu_buffer_rsrc_t rows = matrix_rows(I);
            const uint32_t row_e = __umul24(static_cast<uint32_t>(cur), static_cast<uint32_t>(I.ld));
            int32_t best_key = -1;
            int32_t best_j = 0x7FFFFFFF;
            const int32_t span = LIVE ? nlive : nblk;
            // one block of the row: its four scores, the block's winner, then
            // the lane's (a lane's blocks arrive in increasing order)
            auto score_block = [&](int32_t b, float4 p) {
                const PhiloxOut r = philox10_block(static_cast<uint32_t>(b),
                                                   static_cast<uint32_t>(s),
                                                   static_cast<uint32_t>(ant), I.iter,
                                                   I.key0, I.key1);
                int32_t k0, k1, k2, k3;
                if constexpr (kBytes) {
                    // the block's four marks, 0x80 where visited
                    const uint32_t taken = visited[b];
                    k0 = score_key(p.x, r.w0, (taken << 24) & 0x80000000u);
                    k1 = score_key(p.y, r.w1, (taken << 16) & 0x80000000u);
                    k2 = score_key(p.z, r.w2, (taken << 8) & 0x80000000u);
                    k3 = score_key(p.w, r.w3, taken & 0x80000000u);
                } else {
                    const uint32_t taken = visited[b >> 3] >> ((b & 7) << 2);
                    k0 = score_key(p.x, r.w0, taken << 31);
                    k1 = score_key(p.y, r.w1, (taken << 30) & 0x80000000u);
                    k2 = score_key(p.z, r.w2, (taken << 29) & 0x80000000u);
                    k3 = score_key(p.w, r.w3, (taken << 28) & 0x80000000u);
                }
                // block winner: strict compares keep the smaller city on ties
                const int32_t e01 = (k1 > k0) ? 1 : 0;
                const int32_t m01 = max(k0, k1);
                const int32_t e23 = (k3 > k2) ? 3 : 2;
                const int32_t m23 = max(k2, k3);
                const int32_t eb = (m23 > m01) ? e23 : e01;
                const int32_t mb = max(m01, m23);
                if (mb > best_key) {
                    best_key = mb;
                    best_j = 4 * b + eb;
                }
            };
            if constexpr (AHEAD == 1) {
                for (int32_t base = 0; base < span; base += G) {
                    const int32_t pos = base + gl;
                    if (pos < span) {
                        const int32_t b = LIVE ? static_cast<int32_t>(live[pos]) : pos;
                        score_block(b, matrix_block(rows, row_e, b));
                    }
                }
            } else {
                // AHEAD chunks of G blocks are loaded before any is scored, so
                // that a lane waits for memory once per AHEAD chunks
                // (the loads at a higher priority than other wavefronts'
                // scoring, the group's decision between the two)
                for (int32_t base = 0; base < span; base += AHEAD * G) {
                    float4 pv[AHEAD];
                    int32_t bv[AHEAD];
                    __builtin_amdgcn_s_setprio(2);
#pragma unroll
                    for (int32_t u = 0; u < AHEAD; ++u) {
                        const int32_t pos = base + u * G + gl;
                        bv[u] = -1;
                        if (pos < span) {
                            bv[u] = LIVE ? static_cast<int32_t>(live[pos]) : pos;
                            pv[u] = matrix_block(rows, row_e, bv[u]);
                        }
                    }
                    __builtin_amdgcn_s_setprio(0);
#pragma unroll
                    for (int32_t u = 0; u < AHEAD; ++u) {
                        if (bv[u] >= 0) score_block(bv[u], pv[u]);
                    }
                }
                __builtin_amdgcn_s_setprio(1);
            }
            // Group argmax: the largest key, and among equal keys the smallest city.
            const int32_t top = group_reduce<G, true>(best_key);
            next = group_uniform<G>(group_reduce<G, false>(best_key == top ? best_j : 0x7FFFFFFF));
        }
        // record the step: visited bit now; tour entry, maps and length per window
        const int32_t word = next >> 5;
        uint32_t bits = 0u;
        if constexpr (LIVE) {
            // the live list needs the block's bits after this step
            bits = visited[word] | (1u << (next & 31));
            __builtin_amdgcn_wave_barrier();
            if (gl == 0) visited[word] = bits;
        } else if constexpr (kBytes) {
            // one byte store; the wave's later LDS reads see it
            if (gl == 0) vmap[next] = 0x80u;
        } else {
            // an LDS OR with no return value: nothing on the step's chain
            // waits for it, and the wave's later LDS reads see it
            if (gl == 0)
                __hip_atomic_fetch_or(visited + word, 1u << (next & 31), __ATOMIC_RELAXED,
                                      __HIP_MEMORY_SCOPE_WAVEFRONT);
        }
        if (gl == (s & (G - 1))) win = next;
        if ((s & (G - 1)) == G - 1 || s == n - 1) {
            const int32_t base = s & ~(G - 1);
            const int32_t cnt = s - base + 1;
            flush_window<G>(I, tour, ant, base, cnt, win, prev, gl, lengths_window, len);
            prev = group_lane<G>(win, cnt - 1);
        }
        cur = next;
        if constexpr (LIVE) {
            // drop the block from the live list once its last city is taken
            const int32_t nb = next >> 2;
            if (((bits >> ((nb & 7) << 2)) & 0xFu) == 0xFu) {
                int32_t below = 0;  // live blocks before nb = its position in the list
                for (int32_t i = gl; i < nlive; i += G) below += (live[i] < nb) ? 1 : 0;
                const int32_t at = group_uniform<G>(group_sum<G>(below));
                for (int32_t base = at; base < nlive - 1; base += G) {
                    const int32_t i = base + gl;
                    uint16_t v = 0;
                    if (i < nlive - 1) v = live[i + 1];
                    __builtin_amdgcn_wave_barrier();
                    if (i < nlive - 1) live[i] = v;
                    __builtin_amdgcn_wave_barrier();
                }
                --nlive;
            }
        }
        __builtin_amdgcn_wave_barrier();
    }
    // the closing edge, added last
    if (gl == 0) {
        I.succ[static_cast<size_t>(cur) * I.m_stride + ant] = start;
        I.pred[static_cast<size_t>(start) * I.m_stride + ant] = cur;
        len += static_cast<double>(I.dist[static_cast<size_t>(cur) * I.ld + start]);
        I.lengths[ant] = static_cast<float>(len);
        if constexpr (SEL == kSelSorted) {
            if (I.walk_stats) {
                atomicAdd(I.walk_stats + 0, static_cast<unsigned long long>(walk_entries));
                atomicAdd(I.walk_stats + 1, static_cast<unsigned long long>(scanned_steps));
                atomicAdd(I.walk_stats + 2, static_cast<unsigned long long>(scanned_blocks));
            }
        }
    }
}

template <int G, bool LIVE, int SEL>
__global__ __launch_bounds__(kWave) void construct_kernel(InstanceView I, int32_t m) {
    extern __shared__ uint32_t lds[];
    constexpr int32_t kGroups = kWave / G;
    const int32_t ant0 = static_cast<int32_t>(blockIdx.x) * kGroups;
    constexpr int32_t kAhead =
        SEL == kSelAdaIR ? 1 : (SEL == kSelSorted ? kWalkScanAhead : kScanAhead);
    construct_group<G, LIVE, SEL, kAhead>(I, ant0, min(kGroups, m - ant0), lds);
}

__global__ void uniforms_kernel(uint32_t key0, uint32_t key1, uint32_t iter, uint32_t ant,
                                uint32_t step, int32_t count, float* __restrict__ out) {
    const int32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= count) return;
    const PhiloxOut r = philox10(static_cast<uint32_t>(j >> 2), step, ant, iter, key0, key1);
    const uint32_t words[4] = {r.w0, r.w1, r.w2, r.w3};
    out[j] = unit_from_word(words[j & 3]);
}

template <int G, bool LIVE>
hipError_t launch_one(const InstanceView& I, int32_t m, int32_t selection, hipStream_t stream) {
    constexpr int32_t kGroups = kWave / G;
    const size_t lds = sizeof(uint32_t) * static_cast<size_t>(kGroups) *
                       static_cast<size_t>(group_lds_words(I.n, LIVE, G,
                                                           selection == kSelSorted && !LIVE));
    const dim3 grid((m + kGroups - 1) / kGroups);
    if (selection == kSelRoulette) {
        hipLaunchKernelGGL((construct_kernel<G, LIVE, kSelRoulette>), grid, dim3(kWave), lds,
                           stream, I, m);
    } else if (selection == kSelSorted) {
        hipLaunchKernelGGL((construct_kernel<G, LIVE, kSelSorted>), grid, dim3(kWave), lds,
                           stream, I, m);
    } else {
        hipLaunchKernelGGL((construct_kernel<G, LIVE, kSelAdaIR>), grid, dim3(kWave), lds,
                           stream, I, m);
    }
    return hipGetLastError();
}

// ---- persistent construct over a batch of instances -----------------------

template <int G, bool LIVE, bool SORTED = false>
__device__ __forceinline__ void run_task(const BatchInstance& inst, const BatchPools& pools,
                                         uint32_t iter, int32_t ant0, int32_t nants,
                                         uint32_t* lds) {
    InstanceView I;
    I.P = pools.P + inst.off_mat;
    I.dist = pools.dist + inst.off_mat;
    I.n = inst.n;
    I.ld = inst.ld;
    I.tours = pools.tours + inst.off_tours;
    I.lengths = pools.lengths + inst.off_ants;
    I.succ = pools.succ + inst.off_succ;
    I.pred = pools.pred + inst.off_succ;
    I.m_stride = inst.m;
    I.key0 = inst.key0;
    I.key1 = inst.key1;
    I.iter = iter;
    I.walk_stats = nullptr;
    if constexpr (SORTED) {
        // whole rows, sorted by the update that built this P
        I.Ps = pools.sorted_p + inst.off_sorted;
        I.Js = pools.sorted_j + inst.off_sorted;
        I.sorted_ld = inst.n;
        I.walk = kBatchWalk;
        I.walk_stats = pools.walk_stats;
        construct_group<G, false, kSelSorted>(I, ant0, nants, lds);
    } else {
        I.Ps = nullptr;
        I.Js = nullptr;
        I.sorted_ld = 0;
        I.walk = 0;
        construct_group<G, LIVE>(I, ant0, nants, lds);
    }
}

// Each wave takes tasks (instance, first ant, ant count, schedule) from its
// home queue (its workgroup index mod kQueues) until that is empty.  Then
// lanes 0..kQueues-1 read the queue counters at once and the wave moves to
// the first queue that still looks open, until none does.  A counter only
// grows, so a stale read can only make a queue look open; the atomic then
// finds it empty, and the wave probes again.  Every wave reaches the exit:
// the tasks are finite and each is bounded by its instance size.
__global__ __launch_bounds__(kWave) void batch_construct_kernel(
    const BatchInstance* __restrict__ insts, const BatchTask* __restrict__ tasks,
    const int32_t* __restrict__ queue_start, uint32_t* __restrict__ queues,
    const IterState* __restrict__ state, BatchPools pools) {
    extern __shared__ uint32_t lds[];
    const uint32_t iter = state->iter;
    const int32_t lane = static_cast<int32_t>(threadIdx.x);
    const int32_t home = static_cast<int32_t>(blockIdx.x % kQueues);
    int32_t q = home;
    for (;;) {
        const int32_t begin = queue_start[q];
        const uint32_t size = static_cast<uint32_t>(queue_start[q + 1] - begin);
        for (;;) {
            uint32_t t = 0;
            if (lane == 0) t = atomicAdd(queues + q, 1u);
            t = __builtin_amdgcn_readfirstlane(t);
            if (t >= size) break;
            const BatchTask task = tasks[begin + static_cast<int32_t>(t)];
            const BatchInstance inst = insts[task.instance];
            switch (task.schedule) {
                case kSched16: run_task<16, false>(inst, pools, iter, task.ant0, task.nants, lds); break;
                case kSched32: run_task<32, false>(inst, pools, iter, task.ant0, task.nants, lds); break;
                case kSched32Live: run_task<32, true>(inst, pools, iter, task.ant0, task.nants, lds); break;
                case kSched64: run_task<64, false>(inst, pools, iter, task.ant0, task.nants, lds); break;
                case kSched16 | kSchedSorted:
                    run_task<16, false, true>(inst, pools, iter, task.ant0, task.nants, lds);
                    break;
                case kSched32 | kSchedSorted:
                    run_task<32, false, true>(inst, pools, iter, task.ant0, task.nants, lds);
                    break;
                case kSched64 | kSchedSorted:
                    run_task<64, false, true>(inst, pools, iter, task.ant0, task.nants, lds);
                    break;
                default: run_task<64, true>(inst, pools, iter, task.ant0, task.nants, lds); break;
            }
            __syncthreads();
        }
        bool open = false;
        if (lane < kQueues) {
            const int32_t p = (home + lane) % kQueues;
            const uint32_t taken =
                __hip_atomic_load(queues + p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            open = taken < static_cast<uint32_t>(queue_start[p + 1] - queue_start[p]);
        }
        const uint64_t any = __ballot(open);
        if (any == 0ull) break;
        q = (home + __builtin_ctzll(any)) % kQueues;
    }
}

}  // namespace

int32_t schedule_lanes(int32_t sched) {
    switch (sched) {
        case kSched16: return 16;
        case kSched32:
        case kSched32Live: return 32;
        default: return 64;
    }
}

bool schedule_live(int32_t sched) { return sched == kSched32Live || sched == kSched64Live; }

bool schedule_valid(int32_t sched) { return sched >= kSched16 && sched <= kSched64Live; }

int32_t default_schedule(int32_t n) {
    const int32_t nblk = (n + 3) >> 2;
    if (nblk <= 16) return kSched16;
    if (nblk <= 32) return kSched32;
    if (nblk <= 64) return kSched64;
    return kSched64Live;
}

int32_t sorted_default_schedule(int32_t m) {
    // at least two wavefronts of ants per SIMD (1024 SIMDs)
    if (m >= 8192) return kSched16;
    if (m >= 4096) return kSched32;
    return kSched64;
}

size_t wave_lds_bytes(int32_t n, int32_t sched) {
    const bool sorted = (sched & kSchedSorted) != 0;
    const int32_t base = sched & ~kSchedSorted;
    return sizeof(uint32_t) * static_cast<size_t>(kWave / schedule_lanes(base)) *
           static_cast<size_t>(group_lds_words(n, schedule_live(base), schedule_lanes(base),
                                               sorted && !schedule_live(base)));
}

bool roulette_fits(int32_t n, int32_t sched) {
    const int32_t G = schedule_lanes(sched);
    const int32_t nblk = (n + 3) >> 2;
    return (nblk + G - 1) / G <= G;
}

hipError_t launch_construct_view(const InstanceView& I, int32_t m, int32_t sched,
                                 int32_t selection, hipStream_t stream) {
    switch (sched) {
        case kSched16: return launch_one<16, false>(I, m, selection, stream);
        case kSched32: return launch_one<32, false>(I, m, selection, stream);
        case kSched32Live: return launch_one<32, true>(I, m, selection, stream);
        case kSched64: return launch_one<64, false>(I, m, selection, stream);
        default: return launch_one<64, true>(I, m, selection, stream);
    }
}

hipError_t launch_construct(const Buffers& B, int32_t n, int32_t ld, int32_t m, int32_t m_max,
                            uint64_t seed, uint32_t iter, int32_t sched, int32_t selection,
                            int32_t walk, hipStream_t stream) {
    InstanceView I;
    I.P = B.P;
    I.dist = B.dist;
    I.n = n;
    I.ld = ld;
    I.tours = B.tours;
    I.lengths = B.lengths;
    I.succ = B.succ;
    I.pred = B.pred;
    I.m_stride = m_max;
    I.key0 = static_cast<uint32_t>(seed);
    I.key1 = static_cast<uint32_t>(seed >> 32);
    I.iter = iter;
    I.Ps = B.Ps;
    I.Js = B.Js;
    I.sorted_ld = sorted_prefix(n, walk);
    I.walk = walk;
    I.walk_stats = B.walk_stats;
    return launch_construct_view(I, m, sched, selection, stream);
}

hipError_t launch_batch_construct(const BatchDevice& BD, int32_t ntasks, size_t lds_bytes,
                                  int32_t grid, hipStream_t stream) {
    (void)ntasks;
    hipLaunchKernelGGL(batch_construct_kernel, dim3(grid), dim3(kWave), lds_bytes, stream,
                       BD.insts, BD.tasks, BD.queue_start, BD.queue, BD.state, BD.pools);
    return hipGetLastError();
}

hipError_t launch_uniforms(uint64_t seed, uint32_t iter, uint32_t ant, uint32_t step,
                           int32_t count, float* out, hipStream_t stream) {
    if (count <= 0) return hipSuccess;
    const int threads = 256;
    hipLaunchKernelGGL(uniforms_kernel, dim3((count + threads - 1) / threads), dim3(threads), 0,
                       stream, static_cast<uint32_t>(seed), static_cast<uint32_t>(seed >> 32),
                       iter, ant, step, count, out);
    return hipGetLastError();
}

}  // namespace aco
