// Rows of the transition matrix sorted by value, for the sorted walk of the
// AdaIR selection (Sec. 2.4): a step reads a row from its largest entries
// down and stops once no later entry can win.
//
// One workgroup per row.  The walk reads at most `walk` batches of 64, so a
// row needs only its first K = 64 * walk entries (rounded up to a power of
// two) in order; when K < n a radix select finds them first.  The entries,
// with their city indices, sit in LDS as (P bits, city) pairs; P >= +0, so
// the FP32 bit patterns order like the values.  A bitonic network over a
// power of two puts them in descending order of P, ties by ascending city;
// empty slots sort last.  The network is data-oblivious, so the order is the
// same on every run.  The kept rows are written K entries apart (row r at
// r * K), so that the hot first entries of all rows share pages.  Each compare-exchange step reads and writes LDS only,
// with one barrier between steps.
#include "construct.hpp"

namespace aco {

namespace {

constexpr int32_t kSortThreads = 1024;

// True if (ka, ja) comes before (kb, jb): larger P first, then smaller city.
__device__ __forceinline__ bool before(uint32_t ka, uint32_t ja, uint32_t kb, uint32_t jb) {
    return ka > kb || (ka == kb && ja < jb);
}

// Bitonic network over the n2 (a power of two) LDS slots, descending by
// (key, then ascending city).
__device__ __forceinline__ void bitonic_lds(uint32_t* key, uint16_t* city, int32_t n2) {
    const int32_t tid = threadIdx.x;
    const int32_t nt = blockDim.x;
    const int32_t pairs = n2 >> 1;
    for (int32_t size = 2; size <= n2; size <<= 1) {
        for (int32_t stride = size >> 1; stride > 0; stride >>= 1) {
            for (int32_t t = tid; t < pairs; t += nt) {
                const int32_t lo = 2 * t - (t & (stride - 1));
                const int32_t hi = lo + stride;
                const bool down = (lo & size) == 0;
                const uint32_t ka = key[lo], kb = key[hi];
                const uint32_t ja = city[lo], jb = city[hi];
                const bool swap = down ? before(kb, jb, ka, ja) : before(ka, ja, kb, jb);
                if (swap) {
                    key[lo] = kb;
                    key[hi] = ka;
                    city[lo] = static_cast<uint16_t>(jb);
                    city[hi] = static_cast<uint16_t>(ja);
                }
            }
            __syncthreads();
        }
    }
}

__global__ __launch_bounds__(kSortThreads) void sort_rows_kernel(
    const float* __restrict__ P, int32_t n, int32_t ld, int32_t n2, float* __restrict__ Ps,
    uint16_t* __restrict__ Js) {
    extern __shared__ uint32_t sh[];
    uint32_t* key = sh;                                         // n2 words
    uint16_t* city = reinterpret_cast<uint16_t*>(sh + n2);      // n2 halves
    const size_t row = static_cast<size_t>(blockIdx.x) * static_cast<size_t>(ld);
    const int32_t tid = threadIdx.x;
    const int32_t nt = blockDim.x;
    for (int32_t i = tid; i < n2; i += nt) {
        key[i] = i < n ? __float_as_uint(P[row + i]) : 0u;
        city[i] = static_cast<uint16_t>(i < n ? i : 0xFFFF);
    }
    __syncthreads();
    bitonic_lds(key, city, n2);
    const size_t out = static_cast<size_t>(blockIdx.x) * static_cast<size_t>(n);  // K = n
    for (int32_t i = tid; i < n; i += nt) {
        Ps[out + i] = __uint_as_float(key[i]);
        Js[out + i] = city[i];
    }
}

constexpr int32_t kTopThreads = 256;
constexpr int32_t kWave = 64;

// Sum of v over this lane and every lane above it in the wavefront.
__device__ __forceinline__ uint32_t wave_suffix_sum(uint32_t v) {
    const int32_t lane = threadIdx.x & (kWave - 1);
#pragma unroll
    for (int32_t off = 1; off < kWave; off <<= 1) {
        const uint32_t u = __shfl_down(v, off, kWave);
        if (lane + off < kWave) v += u;
    }
    return v;
}

// Sum of v over this lane and every lane below it in the wavefront.
__device__ __forceinline__ uint32_t wave_prefix_sum(uint32_t v) {
    const int32_t lane = threadIdx.x & (kWave - 1);
#pragma unroll
    for (int32_t off = 1; off < kWave; off <<= 1) {
        const uint32_t u = __shfl_up(v, off, kWave);
        if (lane >= off) v += u;
    }
    return v;
}

// v of lane (lane ^ S), S a power of two below 64, without going through
// LDS: quad permutations for 1 and 2; row rotations for 4 and 8 (row_ror:N
// gives lane l the value of lane (l - N) mod 16 of its row of 16, so lane l
// takes l - 4 when bit 2 of l is set and l + 4 = l - 12 otherwise); the
// permlane16 / permlane32 swaps for 16 and 32 (swapping v with itself, the
// first result holds, in the upper row or half of each pair, the lower
// one's values, and the second result the other way round).
template <int S>
__device__ __forceinline__ uint32_t xor_lane(uint32_t v) {
    const int32_t lane = threadIdx.x & 63;
    const int32_t x = static_cast<int32_t>(v);
    if constexpr (S == 1) {
        return static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, x, 0xB1, 0xF, 0xF, false));
    } else if constexpr (S == 2) {
        return static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, x, 0x4E, 0xF, 0xF, false));
    } else if constexpr (S == 4) {
        const int32_t down = __builtin_amdgcn_update_dpp(0, x, 0x124, 0xF, 0xF, false);  // l - 4
        const int32_t up = __builtin_amdgcn_update_dpp(0, x, 0x12C, 0xF, 0xF, false);    // l + 4
        return static_cast<uint32_t>((lane & 4) ? down : up);
    } else if constexpr (S == 8) {
        return static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, x, 0x128, 0xF, 0xF, false));
    } else if constexpr (S == 16) {
        const auto sw = __builtin_amdgcn_permlane16_swap(v, v, false, false);
        return (lane & 16) ? sw[0] : sw[1];
    } else {
        static_assert(S == 32, "S is a power of two below 64");
        const auto sw = __builtin_amdgcn_permlane32_swap(v, v, false, false);
        return (lane & 32) ? sw[0] : sw[1];
    }
}

template <int S>
__device__ __forceinline__ uint64_t xor_lane64(uint64_t v) {
    const uint32_t lo = xor_lane<S>(static_cast<uint32_t>(v));
    const uint32_t hi = xor_lane<S>(static_cast<uint32_t>(v >> 32));
    return (static_cast<uint64_t>(hi) << 32) | lo;
}

// Bitonic network over N = 64 * REGS entries held in registers: entry e sits
// in register e / 64 of lane e mod 64.  An entry is one 64-bit key, the
// value's bits above (0xFFFF - city), so that the larger key is the one that
// comes first (value descending, then city ascending, as in bitonic_lds) and
// an empty slot (key 0) comes last.  Partners at a stride of 64 or more are in
// the same lane; nearer ones are exchanged across lanes.
// One stage of the network: compare-exchange at distance STRIDE within
// bitonic runs of SIZE entries (SIZE and STRIDE are template arguments, so
// every lane exchange has its permutation as an immediate).
template <int REGS, int SIZE, int STRIDE>
__device__ __forceinline__ void bitonic_stage(uint64_t (&v)[REGS]) {
    const int32_t lane = threadIdx.x & 63;
    if constexpr (STRIDE >= 64) {
        constexpr int32_t rs = STRIDE / 64;
#pragma unroll
        for (int32_t r = 0; r < REGS; ++r) {
            if (r & rs) continue;  // r holds the lower entry of the pair (r, r | rs)
            const int32_t r2 = r | rs;
            const bool down = ((r * 64 + lane) & SIZE) == 0;
            const uint64_t hi = max(v[r], v[r2]), lo = min(v[r], v[r2]);
            v[r] = down ? hi : lo;
            v[r2] = down ? lo : hi;
        }
    } else {
        const bool lower = (lane & STRIDE) == 0;
#pragma unroll
        for (int32_t r = 0; r < REGS; ++r) {
            const uint64_t p = xor_lane64<STRIDE>(v[r]);
            const bool down = ((r * 64 + lane) & SIZE) == 0;
            // the lower entry of a descending pair keeps the larger key:
            // take the partner's if it is on the wanted side (when the keys
            // are equal, either is the same)
            const bool keeps_larger = lower == down;
            if ((p > v[r]) == keeps_larger) v[r] = p;
        }
    }
}

template <int REGS, int SIZE, int STRIDE>
__device__ __forceinline__ void bitonic_merge(uint64_t (&v)[REGS]) {
    bitonic_stage<REGS, SIZE, STRIDE>(v);
    if constexpr (STRIDE > 1) bitonic_merge<REGS, SIZE, STRIDE / 2>(v);
}

template <int REGS, int SIZE>
__device__ __forceinline__ void bitonic_sizes(uint64_t (&v)[REGS]) {
    bitonic_merge<REGS, SIZE, SIZE / 2>(v);
    if constexpr (SIZE < 64 * REGS) bitonic_sizes<REGS, SIZE * 2>(v);
}

template <int REGS>
__device__ __forceinline__ void bitonic_wave(uint64_t (&v)[REGS]) {
    bitonic_sizes<REGS, 2>(v);
}

// The K = 64 * REGS (key, city) slots in LDS sorted by one wavefront (value
// descending, then city ascending, as bitonic_lds orders them) and written out.
template <int REGS>
__device__ __forceinline__ void sort_slots_wave(const uint32_t* key, const uint16_t* city,
                                                float* __restrict__ out_p,
                                                uint16_t* __restrict__ out_j) {
    const int32_t lane = threadIdx.x & 63;
    uint64_t v[REGS];
#pragma unroll
    for (int32_t r = 0; r < REGS; ++r) {
        const int32_t e = r * 64 + lane;
        v[r] = (static_cast<uint64_t>(key[e]) << 32) |
               static_cast<uint64_t>(0xFFFFu - static_cast<uint32_t>(city[e]));
    }
    bitonic_wave<REGS>(v);
#pragma unroll
    for (int32_t r = 0; r < REGS; ++r) {
        const int32_t e = r * 64 + lane;
        out_p[e] = __uint_as_float(static_cast<uint32_t>(v[r] >> 32));
        out_j[e] = static_cast<uint16_t>(0xFFFFu - static_cast<uint32_t>(v[r] & 0xFFFFu));
    }
}

// Largest K that one wavefront sorts in registers (16 entries per lane).
constexpr int32_t kTopWaveSortMax = 1024;

// Radix digits of the top-K select, most significant first: 9 + 8 + 8 + 7
// bits.  The first digit is the sign and the whole exponent, so that the
// entries of a row, whose values span many binades, spread over many bins.
constexpr int32_t kTopBins = 512;
constexpr int32_t kDigitShift[4] = {23, 15, 7, 0};
constexpr int32_t kDigitBits[4] = {9, 8, 8, 7};

// LDS bytes of topk_rows_kernel before the row itself: histogram, segment
// counts, scalars, then the K (key, city) slots.
constexpr size_t topk_lds_bytes(int32_t K) {
    return sizeof(uint32_t) * (kTopBins + kTopThreads + 4) +
           static_cast<size_t>(K) * (sizeof(uint32_t) + sizeof(uint16_t));
}
static_assert(topk_lds_bytes(8) % 16 == 0, "the staged row must start on a 16-byte boundary");

// LDS bytes of the staged row: n entries rounded up to whole 16-byte blocks.
constexpr size_t topk_staged_bytes(int32_t n) {
    return sizeof(uint32_t) * static_cast<size_t>((n + 3) & ~3);
}

// 16-byte loads in flight per thread while a row is staged.
constexpr int32_t kStageLoads = 8;
// Largest dynamic LDS a top-K launch asks for (the full sort's 16384 slots
// use as much); rows that would need more are read from global memory.
constexpr size_t kTopStagedMax = 16384 * (sizeof(uint32_t) + sizeof(uint16_t)) +
                                 sizeof(uint32_t) * (kTopBins + kTopThreads + 4);

// The first K entries of the full sort of a row, for K < n (K a power of two):
// every entry whose key exceeds the K-th largest key T, and the entries equal
// to T with the smallest cities, then sorted.  T is found by a radix select,
// most significant byte first: four 256-bin LDS histograms over the entries
// that match the bytes chosen so far.  The entries equal to T are ranked in
// city order through per-thread contiguous segments and a prefix sum.  With
// STAGED the row is first copied to LDS (one coalesced pass), and every later
// pass reads it there.
template <bool STAGED>
__global__ __launch_bounds__(kTopThreads) void topk_rows_kernel(const float* __restrict__ P,
                                                                int32_t n, int32_t ld,
                                                                int32_t K,
                                                                float* __restrict__ Ps,
                                                                uint16_t* __restrict__ Js) {
    extern __shared__ uint32_t sh[];
    uint32_t* hist = sh;                                          // kTopBins
    uint32_t* seg_count = sh + kTopBins;                          // one per wavefront
    uint32_t* misc = sh + kTopBins + kTopThreads;                 // 4
    uint32_t* key = sh + kTopBins + kTopThreads + 4;              // K
    uint16_t* city = reinterpret_cast<uint16_t*>(key + K);        // K
    const size_t row = static_cast<size_t>(blockIdx.x) * static_cast<size_t>(ld);
    const int32_t tid = threadIdx.x;
    const uint32_t* bits = reinterpret_cast<const uint32_t*>(P + row);
    if constexpr (STAGED) {
        // 16-byte blocks: the row starts on a 256-byte boundary and its
        // padding (P = 0) reaches at least the next multiple of 4 entries; the
        // staged copy starts on a 16-byte boundary (K is a multiple of 8) and
        // has room for that many.  Each thread issues all its loads before
        // its first LDS store, so it waits for memory once per kStageLoads.
        uint32_t* staged = reinterpret_cast<uint32_t*>(city + K);
        const int32_t nq = (n + 3) >> 2;
        const uint4* src = reinterpret_cast<const uint4*>(bits);
        uint4* dst = reinterpret_cast<uint4*>(staged);
        for (int32_t q0 = tid; q0 < nq; q0 += kTopThreads * kStageLoads) {
            uint4 v[kStageLoads];
#pragma unroll
            for (int32_t u = 0; u < kStageLoads; ++u) {
                const int32_t q = q0 + u * kTopThreads;
                if (q < nq) v[u] = src[q];
            }
#pragma unroll
            for (int32_t u = 0; u < kStageLoads; ++u) {
                const int32_t q = q0 + u * kTopThreads;
                if (q < nq) dst[q] = v[u];
            }
        }
        bits = staged;
        __syncthreads();
    }

    uint32_t prefix = 0u, mask = 0u;
    uint32_t need = static_cast<uint32_t>(K);
#pragma unroll
    for (int32_t pass = 0; pass < 4; ++pass) {
        const int32_t shift = kDigitShift[pass];
        const int32_t nbins = 1 << kDigitBits[pass];
        const uint32_t digit_mask = static_cast<uint32_t>(nbins - 1);
        for (int32_t i = tid; i < nbins; i += kTopThreads) hist[i] = 0u;
        __syncthreads();
        for (int32_t i = tid; i < n; i += kTopThreads) {
            const uint32_t k = bits[i];
            if ((k & mask) == prefix) atomicAdd(&hist[(k >> shift) & digit_mask], 1u);
        }
        __syncthreads();
        if (tid < kWave) {
            // the digit d holding the need-th largest, counting from the top
            // bin down: lane l holds bins B*l .. B*l+B-1; the last lane whose
            // bins and all above reach `need` holds d
            constexpr int32_t kMaxPerLane = kTopBins / kWave;
            const int32_t per_lane = nbins / kWave;
            uint32_t h[kMaxPerLane];
            uint32_t own = 0u;
#pragma unroll
            for (int32_t q = 0; q < kMaxPerLane; ++q) {
                h[q] = q < per_lane ? hist[tid * per_lane + q] : 0u;
                own += h[q];
            }
            const uint32_t from_here = wave_suffix_sum(own);
            const uint64_t reach = __ballot(from_here >= need);
            if (tid == 63 - __builtin_clzll(reach)) {
                uint32_t above = from_here - own;  // entries in the bins above lane tid's
                int32_t q = per_lane - 1;
                for (; q > 0; --q) {
                    if (above + h[q] >= need) break;
                    above += h[q];
                }
                misc[0] = static_cast<uint32_t>(tid * per_lane + q);
                misc[1] = above;
                misc[3] = h[q];  // entries in the chosen bin
            }
        }
        __syncthreads();
        prefix |= misc[0] << shift;
        mask |= digit_mask << shift;
        need -= misc[1];
        __syncthreads();
    }
    const uint32_t T = prefix;  // `need` (>= 1) entries equal to T complete the top K
    const int32_t lane = tid & (kWave - 1);
    if (misc[3] == need) {
        // every entry equal to T is kept (the usual case: T is unique), so no
        // ranking is needed: all entries >= T take slots, a wavefront's at a
        // time from one counter, in any order (the sort below orders them)
        if (tid == 0) misc[2] = 0u;
        __syncthreads();
        for (int32_t i0 = 0; i0 < n; i0 += kTopThreads) {
            const int32_t i = i0 + tid;
            const uint32_t k = i < n ? bits[i] : 0u;
            const bool kept = i < n && k >= T;
            const uint64_t took = __ballot(kept);
            uint32_t base = 0u;
            if (lane == 0 && took) base = atomicAdd(&misc[2], static_cast<uint32_t>(__popcll(took)));
            base = static_cast<uint32_t>(__shfl(static_cast<int32_t>(base), 0));
            if (kept) {
                const uint32_t slot = base + __builtin_amdgcn_mbcnt_hi(
                    static_cast<uint32_t>(took >> 32),
                    __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(took), 0u));
                if (slot < static_cast<uint32_t>(K)) {
                    key[slot] = k;
                    city[slot] = static_cast<uint16_t>(i);
                }
            }
        }
    } else {
        // rank the entries equal to T in city order: contiguous segments per thread
        const int32_t seg = (n + kTopThreads - 1) / kTopThreads;
        const int32_t lo = min(n, tid * seg), hi = min(n, lo + seg);
        uint32_t eq = 0u;
        for (int32_t i = lo; i < hi; ++i) eq += (bits[i] == T) ? 1u : 0u;
        // exclusive prefix sum of the segment counts in thread order: within each
        // wavefront, then the totals of the wavefronts before it
        const uint32_t incl = wave_prefix_sum(eq);
        if ((tid & (kWave - 1)) == kWave - 1) seg_count[tid / kWave] = incl;
        if (tid == 0) misc[2] = 0u;
        __syncthreads();
        uint32_t rank = incl - eq;
        for (int32_t w = 0; w < tid / kWave; ++w) rank += seg_count[w];
        // entries above T take slots need .. K-1 (their order is fixed by the sort
        // below), a wavefront's at a time from one counter; the equal ones of
        // rank < need take slots 0 .. need-1
        for (int32_t u = 0; u < seg; ++u) {
            const int32_t i = lo + u;
            const uint32_t k = i < hi ? bits[i] : 0u;
            const bool above = i < hi && k > T;
            const uint64_t took = __ballot(above);
            uint32_t base = 0u;
            if (lane == 0 && took) base = atomicAdd(&misc[2], static_cast<uint32_t>(__popcll(took)));
            base = static_cast<uint32_t>(__shfl(static_cast<int32_t>(base), 0));
            int32_t slot = -1;
            if (above) {
                const uint32_t below = __builtin_amdgcn_mbcnt_hi(
                    static_cast<uint32_t>(took >> 32),
                    __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(took), 0u));
                slot = static_cast<int32_t>(need + base + below);
            } else if (i < hi && k == T) {
                if (rank < need) slot = static_cast<int32_t>(rank);
                ++rank;
            }
            if (slot >= 0 && slot < K) {
                key[slot] = k;
                city[slot] = static_cast<uint16_t>(i);
            }
        }
    }
    __syncthreads();
    const size_t out = static_cast<size_t>(blockIdx.x) * static_cast<size_t>(K);
    if (K <= kTopWaveSortMax) {
        // one wavefront sorts the K slots in registers, with no barrier
        if (tid < kWave) {
            float* op = Ps + out;
            uint16_t* oj = Js + out;
            switch (K) {
                case 64: sort_slots_wave<1>(key, city, op, oj); break;
                case 128: sort_slots_wave<2>(key, city, op, oj); break;
                case 256: sort_slots_wave<4>(key, city, op, oj); break;
                case 512: sort_slots_wave<8>(key, city, op, oj); break;
                default: sort_slots_wave<16>(key, city, op, oj); break;
            }
        }
        return;
    }
    bitonic_lds(key, city, K);
    for (int32_t i = tid; i < K; i += kTopThreads) {
        Ps[out + i] = __uint_as_float(key[i]);
        Js[out + i] = city[i];
    }
}

// One whole row (n <= 64 * REGS) sorted in one wavefront and written n
// entries apart; slots past n sort last and are not written.
template <int REGS>
__device__ __forceinline__ void sort_row_wave(const float* __restrict__ P, int32_t n,
                                              float* __restrict__ out_p,
                                              uint16_t* __restrict__ out_j) {
    const int32_t lane = threadIdx.x & 63;
    uint64_t v[REGS];
#pragma unroll
    for (int32_t r = 0; r < REGS; ++r) {
        const int32_t e = r * 64 + lane;
        v[r] = e < n ? (static_cast<uint64_t>(__float_as_uint(P[e])) << 32) |
                           static_cast<uint64_t>(0xFFFFu - static_cast<uint32_t>(e))
                     : 0ull;
    }
    bitonic_wave<REGS>(v);
#pragma unroll
    for (int32_t r = 0; r < REGS; ++r) {
        const int32_t e = r * 64 + lane;
        if (e < n) {
            out_p[e] = __uint_as_float(static_cast<uint32_t>(v[r] >> 32));
            out_j[e] = static_cast<uint16_t>(0xFFFFu - static_cast<uint32_t>(v[r] & 0xFFFFu));
        }
    }
}

// Whole rows of the batch members that construct with the sorted walk: one
// wavefront per row of the task list (those members' rows only; n <=
// ACO_BATCH_SORTED_MAX_N), written n entries apart into the sorted pools.
__global__ __launch_bounds__(64) void batch_sort_rows_kernel(const BatchInstance* __restrict__ insts,
                                                             const RowTask* __restrict__ rows,
                                                             BatchPools pools) {
    const RowTask task = rows[blockIdx.x];
    const BatchInstance in = insts[task.instance];
    if (!in.sorted) return;
    const int32_t n = in.n;
    const float* P = pools.P + in.off_mat + static_cast<int64_t>(task.row) * in.ld;
    const int64_t out = in.off_sorted + static_cast<int64_t>(task.row) * n;
    float* op = pools.sorted_p + out;
    uint16_t* oj = pools.sorted_j + out;
    if (n <= 64) {
        sort_row_wave<1>(P, n, op, oj);
    } else if (n <= 128) {
        sort_row_wave<2>(P, n, op, oj);
    } else if (n <= 256) {
        sort_row_wave<4>(P, n, op, oj);
    } else if (n <= 512) {
        sort_row_wave<8>(P, n, op, oj);
    } else {
        sort_row_wave<16>(P, n, op, oj);  // n <= ACO_BATCH_SORTED_MAX_N = 1024
    }
}

static_assert(ACO_BATCH_SORTED_MAX_N <= 16 * 64, "the batch row sort holds at most 16 entries per lane");

__global__ void clear_counters_kernel(unsigned long long* __restrict__ c, int32_t count) {
    const int32_t i = threadIdx.x;
    if (i < count) c[i] = 0ull;
}

}  // namespace

hipError_t launch_batch_sort_rows(const BatchDevice& BD, int32_t nrows, hipStream_t stream) {
    if (nrows <= 0) return hipSuccess;
    hipLaunchKernelGGL(batch_sort_rows_kernel, dim3(nrows), dim3(64), 0, stream, BD.insts,
                       BD.sort_rows, BD.pools);
    return hipGetLastError();
}

hipError_t launch_clear_counters(unsigned long long* c, int32_t count, hipStream_t stream) {
    hipLaunchKernelGGL(clear_counters_kernel, dim3(1), dim3(64), 0, stream, c, count);
    return hipGetLastError();
}

int32_t sorted_prefix(int32_t n, int32_t walk) {
    int32_t k = 64;
    while (k < 64 * walk) k <<= 1;
    return k < n ? k : n;
}

hipError_t launch_sort_rows(const float* P, int32_t n, int32_t ld, int32_t walk, float* Ps,
                            uint16_t* Js, hipStream_t stream) {
    const int32_t K = sorted_prefix(n, walk);
    if (K < n) {
        const size_t lds = topk_lds_bytes(K);
        const size_t staged = lds + topk_staged_bytes(n);
        if (staged <= kTopStagedMax) {
            hipLaunchKernelGGL(topk_rows_kernel<true>, dim3(n), dim3(kTopThreads), staged, stream,
                               P, n, ld, K, Ps, Js);
        } else {
            hipLaunchKernelGGL(topk_rows_kernel<false>, dim3(n), dim3(kTopThreads), lds, stream,
                               P, n, ld, K, Ps, Js);
        }
        return hipGetLastError();
    }
    int32_t n2 = 2;
    while (n2 < n) n2 <<= 1;
    const int32_t threads = min(kSortThreads, max(64, n2 >> 1));
    const size_t lds = static_cast<size_t>(n2) * (sizeof(uint32_t) + sizeof(uint16_t));
    hipLaunchKernelGGL(sort_rows_kernel, dim3(n), dim3(threads), lds, stream, P, n, ld, n2, Ps,
                       Js);
    return hipGetLastError();
}

hipError_t prepare_sort_kernel() {
    // n2 <= 16384: 96 KB of slots; a top-K launch asks for at most as much
    const int bytes = static_cast<int>(kTopStagedMax);
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(sort_rows_kernel),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    if (e != hipSuccess) return e;
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(topk_rows_kernel<true>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    if (e != hipSuccess) return e;
    return hipFuncSetAttribute(reinterpret_cast<const void*>(topk_rows_kernel<false>),
                               hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
}

}  // namespace aco
