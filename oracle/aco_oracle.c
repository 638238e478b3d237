/*
 * aco_oracle.c -- CPU oracle for Tensorized Ant Colony Optimization on the
 * Euclidean TSP (Yang, Jiang & Cheng, "Tensorized Ant Colony Optimization for
 * GPU Acceleration", GECCO'24 Companion).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file.  Only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark use it.  It shares no code, header, table or helper with
 * the GPU path: its Philox generator, its selection, its deposit and its
 * transition are written here from their definitions.
 *
 * Precision: the paper does not fix it.  Matrices are FP32 at rest; every
 * intermediate that is not an FP32 input or output is FP64.  Built with
 * -ffp-contract=off and no fast-math, so every float operation below is the
 * IEEE operation it is written as.
 *
 * Notation: n cities, m ants (the definition in Sec. 2 of the paper; later
 * passages of Sec. 2.2-2.4 swap the two letters, read here with n = cities).
 * All matrices are dense, row-major, n x n.
 *
 * Readings taken where the paper is silent or ambiguous (each one is listed
 * with its reason in the design notes of the repository):
 *   R1  the AdaIR exponent is folded into P: argmax_j p_j*u_j^g equals
 *       argmax_j p_j^(1/g)*u_j because x -> x^(1/g) is increasing (Eq. 4);
 *   R2  r in Sec. 2.4 has one entry per city (length n), keyed by city index;
 *   R3  ties in the argmax go to the smallest city index;
 *   R4  the fitness f of Eq. 3 is the closed tour length, and the increment is
 *       Q/f (Q = 1 gives Eq. 3 exactly);
 *   R5  evaporation tau <- (1-rho) tau + dTau (standard Ant System, which the
 *       paper cites but does not write out);
 *   R6  the deposit weight Q/L is quantised to an integer multiple of 2^-S so
 *       that the sum over ants is exact in any order;
 *   R7  gamma follows a cosine annealing schedule from gamma_max to gamma_min
 *       over the run (Sec. 2.4 names the schedule but gives no constants);
 *   R8  the Roulette Wheel baseline of Sec. 2.4 / Sec. 3 draws one deviate per
 *       step, word 0 of counter (0, s, a, t), and inverts the cumulative
 *       distribution of the unvisited cities in ascending city order in FP64.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_API __attribute__((visibility("default")))

/* ------------------------------------------------------------------------ */
/* Counter-based generator: Philox4x32 with 10 rounds, as published by       */
/* Salmon, Moraes, Dror & Shaw, "Parallel random numbers: as easy as 1, 2,   */
/* 3", SC'11.  One round multiplies words 0 and 2 by the two round           */
/* multipliers, keeps the low halves as the new words 1 and 3, and folds the */
/* high halves with the other two words and the round key into the new      */
/* words 0 and 2.  The key advances by the two Weyl constants between       */
/* rounds.                                                                  */
/* ------------------------------------------------------------------------ */
static const uint32_t PHILOX_MUL_A = 0xD2511F53u; /* multiplies word 0 */
static const uint32_t PHILOX_MUL_B = 0xCD9E8D57u; /* multiplies word 2 */
static const uint32_t PHILOX_WEYL_A = 0x9E3779B9u;
static const uint32_t PHILOX_WEYL_B = 0xBB67AE85u;

ORACLE_API void oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2],
                                     uint32_t out[4]) {
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += PHILOX_WEYL_A;
            k1 += PHILOX_WEYL_B;
        }
        uint64_t prod_a = (uint64_t)PHILOX_MUL_A * (uint64_t)x0;
        uint64_t prod_b = (uint64_t)PHILOX_MUL_B * (uint64_t)x2;
        uint32_t n0 = (uint32_t)(prod_b >> 32) ^ x1 ^ k0;
        uint32_t n1 = (uint32_t)prod_b;
        uint32_t n2 = (uint32_t)(prod_a >> 32) ^ x3 ^ k1;
        uint32_t n3 = (uint32_t)prod_a;
        x0 = n0; x1 = n1; x2 = n2; x3 = n3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* A 32-bit word to a uniform deviate in the open interval (0,1), as required
 * by Sec. 2.4 (r_i uniform on (0,1)): the top 23 bits k give (2k+1)/2^24,
 * which is exact in FP32 and never 0 or 1. */
ORACLE_API float oracle_to_unit(uint32_t w) {
    uint32_t k = w >> 9;
    float odd = (float)(2u * k + 1u); /* < 2^24: exact */
    return odd * 0x1p-24f;            /* power-of-two scale: exact */
}

static void seed_to_key(uint64_t seed, uint32_t key[2]) {
    key[0] = (uint32_t)(seed & 0xFFFFFFFFu);
    key[1] = (uint32_t)(seed >> 32);
}

/* The random deviate r_j of Sec. 2.4 that ant a draws for city j at step s of
 * iteration t (reading R2): counter (j/4, s, a, t), word j mod 4. */
ORACLE_API float oracle_uniform(uint64_t seed, uint32_t t, uint32_t a, uint32_t s,
                                uint32_t j) {
    uint32_t key[2], ctr[4], out[4];
    seed_to_key(seed, key);
    ctr[0] = j / 4u; ctr[1] = s; ctr[2] = a; ctr[3] = t;
    oracle_philox4x32_10(ctr, key, out);
    return oracle_to_unit(out[j % 4u]);
}

/* Initialization of Sec. 2.2: each ant gets a random start city.  Word 0 of
 * counter (0, 0, a, t) is scaled to [0, n) by a 32x32->64 multiply. */
ORACLE_API int32_t oracle_start_city(uint64_t seed, uint32_t t, uint32_t a, int32_t n) {
    uint32_t key[2], ctr[4] = {0u, 0u, a, t}, out[4];
    seed_to_key(seed, key);
    oracle_philox4x32_10(ctr, key, out);
    return (int32_t)(((uint64_t)out[0] * (uint64_t)(uint32_t)n) >> 32);
}

/* ------------------------------------------------------------------------ */
/* Preprocessing, Sec. 2.1 Eq. (1), with the AdaIR exponent of Eq. (4)       */
/* folded in (reading R1):                                                  */
/*   W_ij = tau_ij^alpha * eta_ij^beta  (j != i),  eta = 1/d unless given    */
/*   P_ij = (W_ij / sum_k W_ik)^(1/gamma),  P_ii = 0                         */
/* Logs are used so that tau^alpha and eta^beta cannot overflow; the row is  */
/* shifted by its maximum before exponentiation (same quotient).  The sum    */
/* runs over k in ascending order.                                          */
/* ------------------------------------------------------------------------ */
static void transition_row(const float* tau, const float* dist, const float* eta, int32_t n,
                           float alpha, float beta, float gamma, int32_t i, float* P_row) {
    double* lnw = (double*)malloc(sizeof(double) * (size_t)n);
    double row_max = -INFINITY;
    for (int32_t j = 0; j < n; ++j) {
        if (j == i) continue;
        size_t ij = (size_t)i * (size_t)n + (size_t)j;
        double ln_eta = eta ? log((double)eta[ij]) : -log((double)dist[ij]);
        lnw[j] = (double)alpha * log((double)tau[ij]) + (double)beta * ln_eta;
        if (lnw[j] > row_max) row_max = lnw[j];
    }
    double sum = 0.0;
    for (int32_t j = 0; j < n; ++j) {
        if (j == i) continue;
        sum += exp(lnw[j] - row_max);
    }
    double ln_sum = row_max + log(sum);
    for (int32_t j = 0; j < n; ++j)
        P_row[j] = (j == i) ? 0.0f : (float)exp((lnw[j] - ln_sum) / (double)gamma);
    free(lnw);
}

ORACLE_API void oracle_transition(const float* tau, const float* dist, const float* eta,
                                  int32_t n, float alpha, float beta, float gamma,
                                  float* P) {
#pragma omp parallel for schedule(static)
    for (int32_t i = 0; i < n; ++i)
        transition_row(tau, dist, eta, n, alpha, beta, gamma, i, P + (size_t)i * (size_t)n);
}

/* The same for the listed rows only (count rows, P_rows is count x n). */
ORACLE_API void oracle_transition_rows(const float* tau, const float* dist, const float* eta,
                                       int32_t n, float alpha, float beta, float gamma,
                                       const int32_t* rows, int32_t count, float* P_rows) {
#pragma omp parallel for schedule(static)
    for (int32_t k = 0; k < count; ++k)
        transition_row(tau, dist, eta, n, alpha, beta, gamma, rows[k],
                       P_rows + (size_t)k * (size_t)n);
}

/* ------------------------------------------------------------------------ */
/* Selection, Sec. 2.4: v = argmax_j (r_j * p_u,j) over the unvisited j.    */
/* row = P[c, :] already carries the 1/gamma exponent (reading R1).  The    */
/* score is the FP32 product; visited cities are not candidates; ties go to */
/* the smallest j (reading R3).                                              */
/* ------------------------------------------------------------------------ */
ORACLE_API int32_t oracle_select(const float* row, const uint8_t* visited, int32_t n,
                                 uint64_t seed, uint32_t t, uint32_t a, uint32_t s) {
    int32_t best = -1;
    float best_score = 0.0f;
    for (int32_t j = 0; j < n; ++j) {
        if (visited && visited[j]) continue;
        float r = oracle_uniform(seed, t, a, s, (uint32_t)j);
        float score = row[j] * r;
        if (best < 0 || score > best_score) {
            best = j;
            best_score = score;
        }
    }
    return best;
}

/* Eq. (4) taken literally: score_j = p_j * r_j^gamma in FP64, with p the
 * row-normalised M_p of Eq. (1) (no exponent folded in).  Used only to check
 * in distribution that the folded form selects with the same law. */
ORACLE_API int32_t oracle_select_literal(const double* p, const uint8_t* visited,
                                         int32_t n, double gamma, uint64_t seed,
                                         uint32_t t, uint32_t a, uint32_t s) {
    int32_t best = -1;
    double best_score = 0.0;
    for (int32_t j = 0; j < n; ++j) {
        if (visited && visited[j]) continue;
        double r = (double)oracle_uniform(seed, t, a, s, (uint32_t)j);
        double score = p[j] * pow(r, gamma);
        if (best < 0 || score > best_score) {
            best = j;
            best_score = score;
        }
    }
    return best;
}

/* ------------------------------------------------------------------------ */
/* Roulette Wheel (RW) selection: the proportional rule that the IR of      */
/* Sec. 2.4 replaces and that the ablation of Sec. 3 measures against.      */
/* City j is drawn with probability p_j / sum of p_k over the unvisited k,  */
/* p being the row of M_p (Eq. 1; gamma = 1 gives it exactly).  Reading R8: */
/* one deviate v per step, x = v * total, and the first unvisited city in   */
/* ascending order whose running FP64 sum exceeds x.  A city of weight 0 is */
/* never drawn; if every unvisited city has weight 0, the smallest one is   */
/* taken (the same fallback as the argmax rule's tie-break).                */
/* ------------------------------------------------------------------------ */
ORACLE_API float oracle_roulette_deviate(uint64_t seed, uint32_t t, uint32_t a, uint32_t s) {
    uint32_t key[2], ctr[4] = {0u, s, a, t}, out[4];
    seed_to_key(seed, key);
    oracle_philox4x32_10(ctr, key, out);
    return oracle_to_unit(out[0]);
}

ORACLE_API int32_t oracle_select_roulette(const float* row, const uint8_t* visited, int32_t n,
                                          uint64_t seed, uint32_t t, uint32_t a, uint32_t s) {
    double total = 0.0;
    int32_t first_free = -1;
    for (int32_t j = 0; j < n; ++j) {
        if (visited && visited[j]) continue;
        if (first_free < 0) first_free = j;
        total += (double)row[j];
    }
    if (!(total > 0.0)) return first_free;
    double x = (double)oracle_roulette_deviate(seed, t, a, s) * total;
    double running = 0.0;
    int32_t last_positive = first_free;
    for (int32_t j = 0; j < n; ++j) {
        if (visited && visited[j]) continue;
        running += (double)row[j];
        if (row[j] > 0.0f) last_positive = j;
        if (running > x) return j;
    }
    return last_positive; /* not reached: x < total and the running sum ends at total */
}

/* Fitness f of Eq. (3) (reading R4): closed tour length, summed in FP64 in
 * tour order (closing edge last) and rounded once to FP32. */
ORACLE_API float oracle_tour_length(const int32_t* tour, const float* dist, int32_t n) {
    double len = 0.0;
    for (int32_t s = 0; s < n; ++s) {
        int32_t i = tour[s], j = tour[(s + 1) % n];
        len += (double)dist[(size_t)i * (size_t)n + (size_t)j];
    }
    return (float)len;
}

/* Tensorization of the ant system, Sec. 2.2, as the function it maps over
 * ants: ant a starts at its random city and takes n-1 selections (Sec. 2.4,
 * or the Roulette Wheel when roulette != 0) from the shared P.  Ants are
 * independent, so they run in parallel.  tours is count x n, lengths is
 * count. */
static void construct_ants(const float* P, const float* dist, int32_t n, uint64_t seed,
                           uint32_t t, const int32_t* ants, int32_t count, int32_t roulette,
                           int32_t* tours, float* lengths) {
#pragma omp parallel for schedule(dynamic, 1)
    for (int32_t idx = 0; idx < count; ++idx) {
        uint32_t a = (uint32_t)ants[idx];
        uint8_t* visited = (uint8_t*)calloc((size_t)n, 1);
        int32_t* tour = tours + (size_t)idx * (size_t)n;
        int32_t c = oracle_start_city(seed, t, a, n);
        tour[0] = c;
        visited[c] = 1;
        for (int32_t s = 1; s < n; ++s) {
            const float* row = P + (size_t)c * (size_t)n;
            c = roulette ? oracle_select_roulette(row, visited, n, seed, t, a, (uint32_t)s)
                         : oracle_select(row, visited, n, seed, t, a, (uint32_t)s);
            tour[s] = c;
            visited[c] = 1;
        }
        lengths[idx] = oracle_tour_length(tour, dist, n);
        free(visited);
    }
}

ORACLE_API void oracle_construct(const float* P, const float* dist, int32_t n,
                                 uint64_t seed, uint32_t t, const int32_t* ants,
                                 int32_t count, int32_t* tours, float* lengths) {
    construct_ants(P, dist, n, seed, t, ants, count, 0, tours, lengths);
}

ORACLE_API void oracle_construct_roulette(const float* P, const float* dist, int32_t n,
                                          uint64_t seed, uint32_t t, const int32_t* ants,
                                          int32_t count, int32_t* tours, float* lengths) {
    construct_ants(P, dist, n, seed, t, ants, count, 1, tours, lengths);
}

/* ------------------------------------------------------------------------ */
/* Tensorization of the ant path, Sec. 2.3.                                  */
/* ------------------------------------------------------------------------ */

/* A lower bound on every tour length: each city leaves along an edge at least
 * as long as its nearest neighbour.  Summed in FP64 in ascending city order. */
ORACLE_API double oracle_length_lower_bound(const float* dist, int32_t n) {
    double total = 0.0;
    for (int32_t i = 0; i < n; ++i) {
        float best = INFINITY;
        for (int32_t j = 0; j < n; ++j) {
            if (j == i) continue;
            float d = dist[(size_t)i * (size_t)n + (size_t)j];
            if (d < best) best = d;
        }
        total += (double)best;
    }
    return total;
}

/* Quantisation exponent of reading R6: the largest S with
 * m_max * Q / L_lb * 2^S < 2^62, so that no pheromone cell (which receives at
 * most one weight per ant when n >= 3) can overflow a signed 64-bit sum. */
ORACLE_API int32_t oracle_deposit_scale(double length_lower_bound, int32_t m_max, float Q) {
    double x = (double)m_max * (double)Q / length_lower_bound;
    int32_t S = (int32_t)floor(62.0 - log2(x));
    while (ldexp(x, S) >= 0x1p62) --S;
    while (ldexp(x, S + 1) < 0x1p62) ++S;
    return S;
}

/* Quantised deposit weight Q/f(s_l) of Eq. (3) for one ant. */
ORACLE_API int64_t oracle_deposit_weight(float length, float Q, int32_t S) {
    return (int64_t)llrint(ldexp((double)Q / (double)length, S));
}

typedef struct {
    float len;
    int32_t ant;
} ranked_ant;

static int compare_ranked(const void* pa, const void* pb) {
    const ranked_ant* x = (const ranked_ant*)pa;
    const ranked_ant* y = (const ranked_ant*)pb;
    if (x->len < y->len) return -1;
    if (x->len > y->len) return 1;
    return (x->ant < y->ant) ? -1 : (x->ant > y->ant);
}

/* Sec. 2.3: sort the solution set and keep the top k paths.  Order is by
 * length, then by ant index.  k <= 0 or k >= m keeps every ant. */
ORACLE_API void oracle_elite(const float* lengths, int32_t m, int32_t k, uint8_t* elite) {
    if (k <= 0 || k >= m) {
        for (int32_t a = 0; a < m; ++a) elite[a] = 1;
        return;
    }
    ranked_ant* order = (ranked_ant*)malloc(sizeof(ranked_ant) * (size_t)m);
    for (int32_t a = 0; a < m; ++a) {
        order[a].len = lengths[a];
        order[a].ant = a;
        elite[a] = 0;
    }
    qsort(order, (size_t)m, sizeof(ranked_ant), compare_ranked);
    for (int32_t r = 0; r < k; ++r) elite[order[r].ant] = 1;
    free(order);
}

/* The sequential path update that the paper's index mapping replaces
 * (Sec. 1 and Sec. 2.3): walk every elite tour edge by edge and add the
 * ant's weight to both orientations of the edge.  The result is Eq. (3)'s A
 * summed over the elite set (the total increment dTau), in integer units of
 * 2^-S.  delta is n x n and is overwritten. */
ORACLE_API void oracle_deposit(const int32_t* tours, const float* lengths,
                               const uint8_t* elite, int32_t m, int32_t n, float Q,
                               int32_t S, int64_t* delta) {
    memset(delta, 0, sizeof(int64_t) * (size_t)n * (size_t)n);
    for (int32_t a = 0; a < m; ++a) {
        if (elite && !elite[a]) continue;
        int64_t q = oracle_deposit_weight(lengths[a], Q, S);
        const int32_t* tour = tours + (size_t)a * (size_t)n;
        for (int32_t s = 0; s < n; ++s) {
            int32_t i = tour[s], j = tour[(s + 1) % n];
            delta[(size_t)i * (size_t)n + (size_t)j] += q;
            delta[(size_t)j * (size_t)n + (size_t)i] += q;
        }
    }
}

/* Evaporation then deposit (reading R5):
 *   tau_ij <- fl32((1 - rho) * tau_ij + delta_ij * 2^-S)   (j != i)
 * evaluated as one FP64 fused multiply-add. */
ORACLE_API void oracle_evaporate(float* tau, const int64_t* delta, int32_t n, float rho,
                                 int32_t S) {
    double keep = 1.0 - (double)rho;
    for (int32_t i = 0; i < n; ++i) {
        for (int32_t j = 0; j < n; ++j) {
            if (j == i) continue;
            size_t ij = (size_t)i * (size_t)n + (size_t)j;
            double add = delta ? ldexp((double)delta[ij], -S) : 0.0;
            tau[ij] = (float)fma(keep, (double)tau[ij], add);
        }
    }
}

/* MAX-MIN bounds on the pheromone (the MAX-MIN Ant System of Stuetzle and
 * Hoos; not in the paper): after evaporation and deposit every off-diagonal
 * tau is clamped into [tau_min, tau_max].  tau_min = 0 and tau_max = +inf
 * leave tau unchanged. */
ORACLE_API void oracle_clamp(float* tau, int32_t n, float tau_min, float tau_max) {
    for (int32_t i = 0; i < n; ++i) {
        for (int32_t j = 0; j < n; ++j) {
            if (j == i) continue;
            size_t ij = (size_t)i * (size_t)n + (size_t)j;
            if (tau[ij] < tau_min) tau[ij] = tau_min;
            if (tau[ij] > tau_max) tau[ij] = tau_max;
        }
    }
}

/* Cosine annealing of gamma (reading R7), from gamma_max at t = 0 down to
 * gamma_min at t = T-1, rounded to FP32. */
ORACLE_API float oracle_gamma(int32_t t, int32_t T, float gamma_max, float gamma_min) {
    if (T <= 1) return gamma_max;
    if (t > T - 1) t = T - 1;
    const double pi = 3.14159265358979323846;
    double g = (double)gamma_min + 0.5 * ((double)gamma_max - (double)gamma_min) *
                                       (1.0 + cos(pi * (double)t / (double)(T - 1)));
    return (float)g;
}

/* One whole run: P from tau with gamma_0, then per iteration t: every ant
 * constructs (Sec. 2.2, 2.4), the best-so-far is kept (smallest length, ties
 * to the earlier iteration then the smaller ant), the elite deposit
 * (Sec. 2.3) and evaporation update tau, and P is rebuilt with gamma_{t+1}
 * (Sec. 2.1).  roulette != 0 selects by the Roulette Wheel instead of AdaIR;
 * tau is clamped into [tau_min, tau_max] after each update.
 * tau (n x n) is in/out; P (n x n) is out. */
ORACLE_API int32_t oracle_run(const float* dist, const float* eta, int32_t n, int32_t m,
                              int32_t m_max, float alpha, float beta, float rho, float Q,
                              int32_t elite_k, float gamma_max, float gamma_min,
                              int32_t roulette, float tau_min, float tau_max, uint64_t seed,
                              uint32_t iter0, int32_t iters, float* tau,
                              float* P, int32_t* best_tour, float* best_len,
                              int32_t* best_iter, float* iter_best_len) {
    size_t nn = (size_t)n * (size_t)n;
    int32_t S = oracle_deposit_scale(oracle_length_lower_bound(dist, n), m_max, Q);
    int32_t* tours = (int32_t*)malloc(sizeof(int32_t) * (size_t)m * (size_t)n);
    float* lengths = (float*)malloc(sizeof(float) * (size_t)m);
    int32_t* ants = (int32_t*)malloc(sizeof(int32_t) * (size_t)m);
    uint8_t* elite = (uint8_t*)malloc((size_t)m);
    int64_t* delta = (int64_t*)malloc(sizeof(int64_t) * nn);
    if (!tours || !lengths || !ants || !elite || !delta) {
        free(tours); free(lengths); free(ants); free(elite); free(delta);
        return -1;
    }
    for (int32_t a = 0; a < m; ++a) ants[a] = a;
    *best_len = INFINITY;
    *best_iter = -1;
    oracle_transition(tau, dist, eta, n, alpha, beta,
                      oracle_gamma(0, iters, gamma_max, gamma_min), P);
    for (int32_t it = 0; it < iters; ++it) {
        uint32_t t = iter0 + (uint32_t)it;
        construct_ants(P, dist, n, seed, t, ants, m, roulette, tours, lengths);
        float round_best = INFINITY;
        int32_t round_ant = -1;
        for (int32_t a = 0; a < m; ++a) {
            if (lengths[a] < round_best) {
                round_best = lengths[a];
                round_ant = a;
            }
        }
        if (iter_best_len) iter_best_len[it] = round_best;
        if (round_best < *best_len) {
            *best_len = round_best;
            *best_iter = (int32_t)t;
            memcpy(best_tour, tours + (size_t)round_ant * (size_t)n, sizeof(int32_t) * (size_t)n);
        }
        oracle_elite(lengths, m, elite_k, elite);
        oracle_deposit(tours, lengths, elite, m, n, Q, S, delta);
        oracle_evaporate(tau, delta, n, rho, S);
        oracle_clamp(tau, n, tau_min, tau_max);
        oracle_transition(tau, dist, eta, n, alpha, beta,
                          oracle_gamma(it + 1, iters, gamma_max, gamma_min), P);
    }
    free(tours); free(lengths); free(ants); free(elite); free(delta);
    return S;
}

/* ------------------------------------------------------------------------ */
/* Exact TSP for tiny n (Held-Karp dynamic programme over subsets), used to  */
/* check that the method never reports a tour shorter than the optimum and  */
/* how often it reaches it.  Edge lengths are summed in FP64.  n <= 16.      */
/* ------------------------------------------------------------------------ */
ORACLE_API double oracle_tsp_exact(const float* dist, int32_t n, int32_t* tour_out) {
    if (n < 2 || n > 16) return -1.0;
    int32_t rest = n - 1; /* city 0 is fixed as the start */
    size_t subsets = (size_t)1 << rest;
    double* cost = (double*)malloc(sizeof(double) * subsets * (size_t)rest);
    int8_t* parent = (int8_t*)malloc(subsets * (size_t)rest);
    for (size_t i = 0; i < subsets * (size_t)rest; ++i) {
        cost[i] = INFINITY;
        parent[i] = -1;
    }
    for (int32_t k = 0; k < rest; ++k)
        cost[((size_t)1 << k) * (size_t)rest + (size_t)k] = (double)dist[(size_t)(k + 1)];
    for (size_t set = 1; set < subsets; ++set) {
        for (int32_t last = 0; last < rest; ++last) {
            if (!(set & ((size_t)1 << last))) continue;
            double here = cost[set * (size_t)rest + (size_t)last];
            if (here == INFINITY) continue;
            for (int32_t nxt = 0; nxt < rest; ++nxt) {
                if (set & ((size_t)1 << nxt)) continue;
                size_t grown = set | ((size_t)1 << nxt);
                double cand = here + (double)dist[(size_t)(last + 1) * (size_t)n + (size_t)(nxt + 1)];
                if (cand < cost[grown * (size_t)rest + (size_t)nxt]) {
                    cost[grown * (size_t)rest + (size_t)nxt] = cand;
                    parent[grown * (size_t)rest + (size_t)nxt] = (int8_t)last;
                }
            }
        }
    }
    size_t full = subsets - 1;
    double best = INFINITY;
    int32_t best_last = -1;
    for (int32_t last = 0; last < rest; ++last) {
        double cand = cost[full * (size_t)rest + (size_t)last] +
                      (double)dist[(size_t)(last + 1) * (size_t)n];
        if (cand < best) {
            best = cand;
            best_last = last;
        }
    }
    if (tour_out) {
        size_t set = full;
        int32_t cur = best_last;
        for (int32_t pos = n - 1; pos >= 1; --pos) {
            tour_out[pos] = cur + 1;
            int32_t prev = parent[set * (size_t)rest + (size_t)cur];
            set &= ~((size_t)1 << cur);
            cur = prev;
        }
        tour_out[0] = 0;
    }
    free(cost);
    free(parent);
    return best;
}

/* ------------------------------------------------------------------------ */
/* Batch helpers for the statistical and exhaustive checks of the above.     */
/* ------------------------------------------------------------------------ */
ORACLE_API void oracle_to_unit_many(const uint32_t* w, int64_t count, float* out) {
    for (int64_t i = 0; i < count; ++i) out[i] = oracle_to_unit(w[i]);
}

ORACLE_API void oracle_start_cities(uint64_t seed, uint32_t t, int32_t n, int32_t count,
                                    int32_t* out) {
    for (int32_t a = 0; a < count; ++a) out[a] = oracle_start_city(seed, t, (uint32_t)a, n);
}

/* One selection step for each of `count` ants a = 0..count-1 at step s from
 * the same row and visited set (folded form when literal == 0, Eq. (4)
 * taken literally on p when literal != 0). */
ORACLE_API void oracle_select_many(const float* row, const double* p, const uint8_t* visited,
                                   int32_t n, double gamma, int32_t literal, uint64_t seed,
                                   uint32_t t, uint32_t s, int32_t count, int32_t* out) {
#pragma omp parallel for schedule(static)
    for (int32_t a = 0; a < count; ++a) {
        out[a] = literal ? oracle_select_literal(p, visited, n, gamma, seed, t, (uint32_t)a, s)
                         : oracle_select(row, visited, n, seed, t, (uint32_t)a, s);
    }
}

/* One Roulette Wheel step for each of `count` ants a = 0..count-1 at step s
 * from the same row and visited set. */
ORACLE_API void oracle_select_roulette_many(const float* row, const uint8_t* visited, int32_t n,
                                            uint64_t seed, uint32_t t, uint32_t s,
                                            int32_t count, int32_t* out) {
#pragma omp parallel for schedule(static)
    for (int32_t a = 0; a < count; ++a)
        out[a] = oracle_select_roulette(row, visited, n, seed, t, (uint32_t)a, s);
}
