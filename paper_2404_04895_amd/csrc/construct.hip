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

// Cross-lane maximum of a wave (row shifts within each 16-lane row, then the
// two row broadcasts); the result is read from lane 63.  Lanes without a
// source keep their own value (max is idempotent).
__device__ __forceinline__ int32_t wave_max_i32(int32_t v) {
    v = max(v, __builtin_amdgcn_update_dpp(v, v, 0x111, 0xF, 0xF, false));  // row_shr:1
    v = max(v, __builtin_amdgcn_update_dpp(v, v, 0x112, 0xF, 0xF, false));  // row_shr:2
    v = max(v, __builtin_amdgcn_update_dpp(v, v, 0x114, 0xF, 0xF, false));  // row_shr:4
    v = max(v, __builtin_amdgcn_update_dpp(v, v, 0x118, 0xF, 0xF, false));  // row_shr:8
    v = max(v, __builtin_amdgcn_update_dpp(v, v, 0x142, 0xA, 0xF, false));  // row_bcast:15
    v = max(v, __builtin_amdgcn_update_dpp(v, v, 0x143, 0xC, 0xF, false));  // row_bcast:31
    return __builtin_amdgcn_readlane(v, 63);
}

__device__ __forceinline__ int32_t wave_min_i32(int32_t v) {
    v = min(v, __builtin_amdgcn_update_dpp(v, v, 0x111, 0xF, 0xF, false));
    v = min(v, __builtin_amdgcn_update_dpp(v, v, 0x112, 0xF, 0xF, false));
    v = min(v, __builtin_amdgcn_update_dpp(v, v, 0x114, 0xF, 0xF, false));
    v = min(v, __builtin_amdgcn_update_dpp(v, v, 0x118, 0xF, 0xF, false));
    v = min(v, __builtin_amdgcn_update_dpp(v, v, 0x142, 0xA, 0xF, false));
    v = min(v, __builtin_amdgcn_update_dpp(v, v, 0x143, 0xC, 0xF, false));
    return __builtin_amdgcn_readlane(v, 63);
}

// LDS layout per ant: the visited bitmask (one bit per city, cities >= n
// pre-set) followed by the live-block list: the indices of the 4-city blocks
// that still hold an unvisited city, in increasing order.  A block leaves the
// list when its last city is taken, so a step scans only live blocks; the
// generator is keyed by block index, not list position, so this changes no
// result.
__host__ __device__ constexpr int32_t mask_words(int32_t nblk) { return (nblk + 7) >> 3; }

__global__ __launch_bounds__(kWave) void construct_kernel(
    const float* __restrict__ P, const float* __restrict__ dist, int32_t n, int32_t ld,
    int32_t m_max, uint32_t key0, uint32_t key1, uint32_t iter, int32_t* __restrict__ tours,
    float* __restrict__ lengths, int32_t* __restrict__ succ, int32_t* __restrict__ pred) {
    extern __shared__ uint32_t lds[];
    const int32_t ant = blockIdx.x;
    const int32_t lane = threadIdx.x;
    const int32_t nblk = (n + 3) >> 2;  // 4-city blocks (one Philox call each)
    const int32_t nwords = mask_words(nblk);
    uint32_t* visited = lds;
    uint16_t* live = reinterpret_cast<uint16_t*>(lds + nwords);

    for (int32_t w = lane; w < nwords; w += kWave) {
        const int32_t j0 = w * 32;
        uint32_t bits = 0u;
        if (j0 + 32 > n) bits = (j0 >= n) ? 0xFFFFFFFFu : (0xFFFFFFFFu << (n - j0));
        visited[w] = bits;
    }
    for (int32_t i = lane; i < nblk; i += kWave) live[i] = static_cast<uint16_t>(i);
    int32_t nlive = nblk;

    // Start city (Sec. 2.2 initialization): word 0 of counter (0, 0, ant, iter).
    const PhiloxOut s0 = philox10(0u, 0u, static_cast<uint32_t>(ant), iter, key0, key1);
    const int32_t start = static_cast<int32_t>(__umulhi(s0.w0, static_cast<uint32_t>(n)));
    __syncthreads();

    int32_t* tour = tours + static_cast<size_t>(ant) * n;
    int32_t cur = start;
    int32_t next = start;
    double len = 0.0;
    float edge = 0.0f;  // length of the previous step's edge, added one step late

    for (int32_t s = 0; s < n; ++s) {
        if (s > 0) {
            const float* row = P + static_cast<size_t>(cur) * ld;
            int32_t best_key = -1;
            int32_t best_j = 0x7FFFFFFF;
            const int32_t nchunk = (nlive + kWave - 1) >> 6;
            for (int32_t k = 0; k < nchunk; ++k) {
                const int32_t pos = (k << 6) + lane;
                if (pos < nlive) {
                    const int32_t b = live[pos];
                    const float4 p = *reinterpret_cast<const float4*>(row + 4 * b);
                    const PhiloxOut r = philox10_block(static_cast<uint32_t>(b),
                                                       static_cast<uint32_t>(s),
                                                       static_cast<uint32_t>(ant), iter, key0,
                                                       key1);
                    const uint32_t taken = visited[b >> 3] >> ((b & 7) << 2);
                    const int32_t k0 = score_key(p.x, r.w0, taken << 31);
                    const int32_t k1 = score_key(p.y, r.w1, (taken << 30) & 0x80000000u);
                    const int32_t k2 = score_key(p.z, r.w2, (taken << 29) & 0x80000000u);
                    const int32_t k3 = score_key(p.w, r.w3, (taken << 28) & 0x80000000u);
                    // block winner: strict compares keep the smaller city on ties
                    const int32_t e01 = (k1 > k0) ? 1 : 0;
                    const int32_t m01 = max(k0, k1);
                    const int32_t e23 = (k3 > k2) ? 3 : 2;
                    const int32_t m23 = max(k2, k3);
                    const int32_t eb = (m23 > m01) ? e23 : e01;
                    const int32_t mb = max(m01, m23);
                    // lane winner: blocks arrive in increasing order
                    if (mb > best_key) {
                        best_key = mb;
                        best_j = 4 * b + eb;
                    }
                }
            }
            // Wave argmax: the largest key, and among equal keys the smallest city.
            const int32_t top = wave_max_i32(best_key);
            const uint64_t holders = __ballot(best_key == top);
            if (__popcll(holders) == 1) {
                next = __builtin_amdgcn_readlane(best_j, __ffsll(static_cast<long long>(holders)) - 1);
            } else {
                next = wave_min_i32(best_key == top ? best_j : 0x7FFFFFFF);
            }
        }
        // record the step: visited bit, tour entry, successor/predecessor maps
        const int32_t nb = next >> 2;
        const int32_t word = next >> 5;
        uint32_t bits = 0u;
        if (lane == 0) {
            bits = visited[word] | (1u << (next & 31));
            visited[word] = bits;
            tour[s] = next;
            if (s > 0) {
                succ[static_cast<size_t>(cur) * m_max + ant] = next;
                pred[static_cast<size_t>(next) * m_max + ant] = cur;
            }
        }
        bits = __builtin_amdgcn_readfirstlane(bits);
        len += static_cast<double>(edge);
        if (s > 0) edge = dist[static_cast<size_t>(cur) * ld + next];
        cur = next;
        // drop the block from the live list once its last city is taken
        if (((bits >> ((nb & 7) << 2)) & 0xFu) == 0xFu) {
            int32_t at = 0;
            for (int32_t base = 0; base < nlive; base += kWave) {
                const int32_t i = base + lane;
                const uint64_t hit = __ballot(i < nlive && live[i] == nb);
                if (hit) {
                    at = base + __ffsll(static_cast<long long>(hit)) - 1;
                    break;
                }
            }
            for (int32_t base = at; base < nlive - 1; base += kWave) {
                const int32_t i = base + lane;
                uint16_t v = 0;
                if (i < nlive - 1) v = live[i + 1];
                __builtin_amdgcn_wave_barrier();
                if (i < nlive - 1) live[i] = v;
                __builtin_amdgcn_wave_barrier();
            }
            --nlive;
        }
        __builtin_amdgcn_wave_barrier();
    }
    len += static_cast<double>(edge);
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
    const size_t lds = sizeof(uint32_t) * static_cast<size_t>(mask_words(nblk)) +
                       sizeof(uint16_t) * static_cast<size_t>(nblk + 1);
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
