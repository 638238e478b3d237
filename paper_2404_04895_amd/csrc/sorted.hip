// Rows of the transition matrix sorted by value, for the sorted walk of the
// AdaIR selection (Sec. 2.4): a step reads a row from its largest entries
// down and stops once no later entry can win.
//
// One workgroup per row.  The row's n entries, with their city indices, are
// loaded into LDS as (P bits, city) pairs; P >= +0, so the FP32 bit patterns
// order like the values.  A bitonic network over the next power of two puts
// them in descending order of P, ties by ascending city.  Empty slots sort
// last.  The network is data-oblivious, so the order is the same on every
// run.  Each compare-exchange step reads and writes LDS only, with one
// barrier between steps.
#include "internal.hpp"

namespace aco {

namespace {

constexpr int32_t kSortThreads = 1024;

// True if (ka, ja) comes before (kb, jb): larger P first, then smaller city.
__device__ __forceinline__ bool before(uint32_t ka, uint32_t ja, uint32_t kb, uint32_t jb) {
    return ka > kb || (ka == kb && ja < jb);
}

__global__ __launch_bounds__(kSortThreads) void sort_rows_kernel(
    const float* __restrict__ P, int32_t n, int32_t ld, int32_t n2, float* __restrict__ Ps,
    uint16_t* __restrict__ Js, unsigned long long* __restrict__ walk_stats) {
    extern __shared__ uint32_t sh[];
    uint32_t* key = sh;                                         // n2 words
    uint16_t* city = reinterpret_cast<uint16_t*>(sh + n2);      // n2 halves
    const size_t row = static_cast<size_t>(blockIdx.x) * static_cast<size_t>(ld);
    const int32_t tid = threadIdx.x;
    const int32_t nt = blockDim.x;
    if (blockIdx.x == 0 && tid < 3) walk_stats[tid] = 0ull;
    for (int32_t i = tid; i < n2; i += nt) {
        key[i] = i < n ? __float_as_uint(P[row + i]) : 0u;
        city[i] = static_cast<uint16_t>(i < n ? i : 0xFFFF);
    }
    __syncthreads();
    const int32_t pairs = n2 >> 1;
    for (int32_t size = 2; size <= n2; size <<= 1) {
        for (int32_t stride = size >> 1; stride > 0; stride >>= 1) {
            for (int32_t t = tid; t < pairs; t += nt) {
                const int32_t lo = 2 * t - (t & (stride - 1));
                const int32_t hi = lo + stride;
                // the final merge (size = n2) is descending everywhere
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
    for (int32_t i = tid; i < n; i += nt) {
        Ps[row + i] = __uint_as_float(key[i]);
        Js[row + i] = city[i];
    }
}

}  // namespace

hipError_t launch_sort_rows(const float* P, int32_t n, int32_t ld, float* Ps, uint16_t* Js,
                            unsigned long long* walk_stats, hipStream_t stream) {
    int32_t n2 = 2;
    while (n2 < n) n2 <<= 1;
    const int32_t threads = min(kSortThreads, max(64, n2 >> 1));
    const size_t lds = static_cast<size_t>(n2) * (sizeof(uint32_t) + sizeof(uint16_t));
    hipLaunchKernelGGL(sort_rows_kernel, dim3(n), dim3(threads), lds, stream, P, n, ld, n2, Ps,
                       Js, walk_stats);
    return hipGetLastError();
}

hipError_t prepare_sort_kernel() {
    // n2 <= 16384: 96 KB of LDS
    return hipFuncSetAttribute(reinterpret_cast<const void*>(sort_rows_kernel),
                               hipFuncAttributeMaxDynamicSharedMemorySize,
                               static_cast<int>(16384 * (sizeof(uint32_t) + sizeof(uint16_t))));
}

}  // namespace aco
