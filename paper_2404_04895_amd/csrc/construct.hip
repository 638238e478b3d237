// Tour construction by Adaptive Independent Roulette (Sec. 2.2, Sec. 2.4).
//
// One 64-lane wavefront per ant: the ants of Sec. 2.2's function mapping are
// independent, so each gets its own wave and no wave ever waits on another.
// At every step the wave streams the current city's row of P with one float4
// per lane (coalesced, 1 KiB per wave-wide load), draws the four deviates of
// that city block with one Philox call per lane, scores each unvisited city
// by fl32(P[c,j] * r_j) and reduces the lane winners to the wave's argmax.
// The visited set is a bitmask in LDS (one bit per city); cities at or past
// n are pre-marked so the ragged last block needs no extra test.
//
// Outputs per ant: the tour (m x n int32), its closed length (FP64 sum in
// tour order, rounded once to FP32 -- the fitness f of Eq. (3)), and the
// successor / predecessor of every city, stored city-major so that the
// update kernel reads one contiguous row of each per city (Eq. (2)'s index
// matrix, held as two maps).
#include "internal.hpp"
#include "philox.hpp"

namespace aco {

namespace {

constexpr int kWave = 64;

// Score one candidate.  key = FP32 bit pattern of fl32(P[c,j] * r_j) with the
// city's visited bit in the sign position: scores are >= +0, so unvisited keys
// are >= 0 and order like the scores, while visited keys are negative and can
// never beat the initial -1.  Within a lane candidates arrive in increasing j,
// so a strict compare keeps the smallest j among equal scores.  The winner is
// recorded as `id` = j - 4*lane, which is the same for every lane of the wave
// (a scalar operand).
__device__ __forceinline__ void consider(float p, uint32_t word, uint32_t taken_sign, int32_t id,
                                         int32_t& best_key, int32_t& best_id) {
    // 0x3F800000 | (word >> 9): the funnel shift brings 0x7F in above the top
    // 23 bits of the word, i.e. 1 + k*2^-23; minus (1 - 2^-24) gives the
    // deviate (2k+1)*2^-24 exactly.
    const float unit = __uint_as_float(__builtin_amdgcn_alignbit(0x7Fu, word, 9)) - 0x1.fffffep-1f;
    const float score = p * unit;
    const int32_t key = static_cast<int32_t>(__float_as_uint(score) | taken_sign);
    if (key > best_key) {
        best_key = key;
        best_id = id;
    }
}

__global__ __launch_bounds__(kWave) void construct_kernel(
    const float* __restrict__ P, const float* __restrict__ dist, int32_t n, int32_t ld,
    int32_t m_max, uint32_t key0, uint32_t key1, uint32_t iter, int32_t* __restrict__ tours,
    float* __restrict__ lengths, int32_t* __restrict__ succ, int32_t* __restrict__ pred) {
    extern __shared__ uint32_t visited[];
    const int32_t ant = blockIdx.x;
    const int32_t lane = threadIdx.x;
    const int32_t nblk = (n + 3) >> 2;       // 4-city blocks (one Philox call each)
    const int32_t nwords = (nblk + 7) >> 3;  // 32 cities per mask word

    for (int32_t w = lane; w < nwords; w += kWave) {
        const int32_t j0 = w * 32;
        uint32_t bits = 0u;
        if (j0 + 32 > n) bits = (j0 >= n) ? 0xFFFFFFFFu : (0xFFFFFFFFu << (n - j0));
        visited[w] = bits;
    }
    // Start city (Sec. 2.2 initialization): word 0 of counter (0, 0, ant, iter).
    const PhiloxOut s0 = philox10(0u, 0u, static_cast<uint32_t>(ant), iter, key0, key1);
    const int32_t start = static_cast<int32_t>(__umulhi(s0.w0, static_cast<uint32_t>(n)));
    __syncthreads();
    if (lane == 0) visited[start >> 5] |= 1u << (start & 31);
    __syncthreads();

    int32_t* tour = tours + static_cast<size_t>(ant) * n;
    if (lane == 0) tour[0] = start;
    int32_t cur = start;
    double len = 0.0;

    const int32_t nchunk = (nblk + kWave - 1) / kWave;
    for (int32_t s = 1; s < n; ++s) {
        const float* row = P + static_cast<size_t>(cur) * ld;
        int32_t best_key = -1;
        int32_t best_id = 0;
        for (int32_t k = 0; k < nchunk; ++k) {
            const int32_t b = k * kWave + lane;
            if (b < nblk) {
                const float4 p = *reinterpret_cast<const float4*>(row + 4 * b);
                const PhiloxOut r = philox10_block(static_cast<uint32_t>(b),
                                                   static_cast<uint32_t>(s),
                                                   static_cast<uint32_t>(ant), iter, key0, key1);
                const uint32_t taken = visited[b >> 3] >> ((b & 7) << 2);
                const int32_t base = 4 * kWave * k;  // j = 4*lane + base + e
                consider(p.x, r.w0, taken << 31, base + 0, best_key, best_id);
                consider(p.y, r.w1, (taken << 30) & 0x80000000u, base + 1, best_key, best_id);
                consider(p.z, r.w2, (taken << 29) & 0x80000000u, base + 2, best_key, best_id);
                consider(p.w, r.w3, (taken << 28) & 0x80000000u, base + 3, best_key, best_id);
            }
        }
        int32_t best_j = (best_key >= 0) ? 4 * lane + best_id : 0x7FFFFFFF;
        // Wave argmax: larger key wins, equal keys go to the smaller city.
#pragma unroll
        for (int off = kWave / 2; off > 0; off >>= 1) {
            const int32_t ok = __shfl_xor(best_key, off);
            const int32_t oj = __shfl_xor(best_j, off);
            if (ok > best_key || (ok == best_key && oj < best_j)) {
                best_key = ok;
                best_j = oj;
            }
        }
        const int32_t next = __builtin_amdgcn_readfirstlane(best_j);
        if (lane == 0) {
            visited[next >> 5] |= 1u << (next & 31);
            tour[s] = next;
            succ[static_cast<size_t>(cur) * m_max + ant] = next;
            pred[static_cast<size_t>(next) * m_max + ant] = cur;
        }
        len += static_cast<double>(dist[static_cast<size_t>(cur) * ld + next]);
        cur = next;
        __syncthreads();
    }
    if (lane == 0) {
        succ[static_cast<size_t>(cur) * m_max + ant] = start;
        pred[static_cast<size_t>(start) * m_max + ant] = cur;
        len += static_cast<double>(dist[static_cast<size_t>(cur) * ld + start]);
        lengths[ant] = static_cast<float>(len);
    }
}

__global__ void uniforms_kernel(uint32_t key0, uint32_t key1, uint32_t iter, uint32_t ant,
                                uint32_t step, int32_t count, float* __restrict__ out) {
    const int32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= count) return;
    const PhiloxOut r = philox10(static_cast<uint32_t>(j >> 2), step, ant, iter, key0, key1);
    const uint32_t words[4] = {r.w0, r.w1, r.w2, r.w3};
    out[j] = unit_from_word(words[j & 3]);
}

}  // namespace

hipError_t launch_construct(const Buffers& B, int32_t n, int32_t ld, int32_t m, int32_t m_max,
                            uint64_t seed, uint32_t iter, hipStream_t stream) {
    const int32_t nblk = (n + 3) >> 2;
    const size_t lds = sizeof(uint32_t) * static_cast<size_t>((nblk + 7) >> 3);
    hipLaunchKernelGGL(construct_kernel, dim3(m), dim3(kWave), lds, stream, B.P, B.dist, n, ld,
                       m_max, static_cast<uint32_t>(seed), static_cast<uint32_t>(seed >> 32),
                       iter, B.tours, B.lengths, B.succ, B.pred);
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
