/*
 * sanitize_check.c -- drives every exported function of the CPU oracle
 * (aco_oracle.c, mlp_oracle.c) on small inputs, for a build with
 * AddressSanitizer and UndefinedBehaviorSanitizer.  TEST INFRASTRUCTURE ONLY,
 * like the oracle itself; tests/test_oracle_sanitized_cpu.py builds and runs it.
 *
 * Every buffer is a heap allocation of exactly the size the function's
 * contract names, so a read or write past it is reported.  Beside the
 * sanitizers' own checks it asserts a few invariants that must hold whatever
 * the inputs: tours are permutations, the deposit is symmetric and totals
 * 2 n sum(q), pheromone after evaporation is finite and positive, the exact
 * optimum is no longer than any constructed tour.  Exit status 0 and the
 * last line "sanitize_check: ok" mean all of it passed.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

void oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
float oracle_to_unit(uint32_t w);
float oracle_uniform(uint64_t seed, uint32_t t, uint32_t a, uint32_t s, uint32_t j);
int32_t oracle_start_city(uint64_t seed, uint32_t t, uint32_t a, int32_t n);
void oracle_transition(const float* tau, const float* dist, const float* eta, int32_t n,
                       float alpha, float beta, float gamma, float* P);
void oracle_transition_rows(const float* tau, const float* dist, const float* eta, int32_t n,
                            float alpha, float beta, float gamma, const int32_t* rows,
                            int32_t count, float* P_rows);
int32_t oracle_select(const float* row, const uint8_t* visited, int32_t n, uint64_t seed,
                      uint32_t t, uint32_t a, uint32_t s);
int32_t oracle_select_literal(const double* p, const uint8_t* visited, int32_t n, double gamma,
                              uint64_t seed, uint32_t t, uint32_t a, uint32_t s);
float oracle_roulette_deviate(uint64_t seed, uint32_t t, uint32_t a, uint32_t s);
int32_t oracle_select_roulette(const float* row, const uint8_t* visited, int32_t n,
                               uint64_t seed, uint32_t t, uint32_t a, uint32_t s);
float oracle_tour_length(const int32_t* tour, const float* dist, int32_t n);
void oracle_construct(const float* P, const float* dist, int32_t n, uint64_t seed, uint32_t t,
                      const int32_t* ants, int32_t count, int32_t* tours, float* lengths);
void oracle_construct_roulette(const float* P, const float* dist, int32_t n, uint64_t seed,
                               uint32_t t, const int32_t* ants, int32_t count, int32_t* tours,
                               float* lengths);
double oracle_length_lower_bound(const float* dist, int32_t n);
int32_t oracle_deposit_scale(double length_lower_bound, int32_t m_max, float Q);
int64_t oracle_deposit_weight(float length, float Q, int32_t S);
void oracle_elite(const float* lengths, int32_t m, int32_t k, uint8_t* elite);
void oracle_deposit(const int32_t* tours, const float* lengths, const uint8_t* elite, int32_t m,
                    int32_t n, float Q, int32_t S, int64_t* delta);
void oracle_evaporate(float* tau, const int64_t* delta, int32_t n, float rho, int32_t S);
void oracle_clamp(float* tau, int32_t n, float tau_min, float tau_max);
float oracle_gamma(int32_t t, int32_t T, float gamma_max, float gamma_min);
int32_t oracle_run(const float* dist, const float* eta, int32_t n, int32_t m, int32_t m_max,
                   float alpha, float beta, float rho, float Q, int32_t elite_k,
                   float gamma_max, float gamma_min, int32_t roulette, float tau_min,
                   float tau_max, uint64_t seed, uint32_t iter0, int32_t iters, float* tau,
                   float* P, int32_t* best_tour, float* best_len, int32_t* best_iter,
                   float* iter_best_len);
double oracle_tsp_exact(const float* dist, int32_t n, int32_t* tour_out);
void oracle_to_unit_many(const uint32_t* w, int64_t count, float* out);
void oracle_start_cities(uint64_t seed, uint32_t t, int32_t n, int32_t count, int32_t* out);
void oracle_select_many(const float* row, const double* p, const uint8_t* visited, int32_t n,
                        double gamma, int32_t literal, uint64_t seed, uint32_t t, uint32_t s,
                        int32_t count, int32_t* out);
void oracle_select_roulette_many(const float* row, const uint8_t* visited, int32_t n,
                                 uint64_t seed, uint32_t t, uint32_t s, int32_t count,
                                 int32_t* out);
int32_t oracle_mlp_param_count(void);
float oracle_bf16_round(float x);
void oracle_edge_ranks(const float* dist, int32_t n, int32_t* rank);
double oracle_mean_nn(const float* dist, int32_t n);
void oracle_edge_features(const float* dist, const int32_t* rank, int32_t n, double mean_nn,
                          float* feats);
void oracle_mlp_forward(const double* params, const float* feats, int64_t count,
                        int32_t round_bf16, double kappa, double lambda, double* z_out,
                        double* eta_out);
double oracle_mlp_loss_grad(const double* params, const float* feats, const float* y,
                            int64_t count, int32_t round_bf16, double* grad);
void oracle_adam_step(double* params, double* m, double* v, const double* grad, int32_t count,
                      int32_t t, double lr, double b1, double b2, double eps);

static int failures = 0;

#define CHECK(cond)                                                          \
    do {                                                                     \
        if (!(cond)) {                                                       \
            fprintf(stderr, "sanitize_check: %s:%d: %s\n", __FILE__, __LINE__, #cond); \
            ++failures;                                                      \
        }                                                                    \
    } while (0)

static void* xmalloc(size_t bytes) {
    void* p = malloc(bytes ? bytes : 1);
    if (!p) {
        fprintf(stderr, "sanitize_check: out of memory\n");
        exit(2);
    }
    return p;
}

/* Input points from a 64-bit linear congruential sequence (input data only;
 * none of the method's arithmetic). */
static uint64_t lcg_state = 0x9E3779B97F4A7C15ull;
static double lcg_unit(void) {
    lcg_state = lcg_state * 6364136223846793005ull + 1442695040888963407ull;
    return (double)(lcg_state >> 11) * 0x1.0p-53;
}

static float* distances(int32_t n) {
    double* xy = (double*)xmalloc(sizeof(double) * 2 * (size_t)n);
    for (int32_t i = 0; i < 2 * n; ++i) xy[i] = lcg_unit();
    float* D = (float*)xmalloc(sizeof(float) * (size_t)n * (size_t)n);
    for (int32_t i = 0; i < n; ++i)
        for (int32_t j = 0; j < n; ++j) {
            double dx = xy[2 * i] - xy[2 * j], dy = xy[2 * i + 1] - xy[2 * j + 1];
            D[(size_t)i * n + j] = (i == j) ? 0.0f : (float)sqrt(dx * dx + dy * dy) + 1e-6f;
        }
    free(xy);
    return D;
}

static int is_permutation(const int32_t* tour, int32_t n) {
    uint8_t* seen = (uint8_t*)calloc((size_t)n, 1);
    int ok = seen != NULL;
    for (int32_t s = 0; ok && s < n; ++s) {
        if (tour[s] < 0 || tour[s] >= n || seen[tour[s]]) ok = 0;
        else seen[tour[s]] = 1;
    }
    free(seen);
    return ok;
}

static void check_generator(void) {
    uint32_t ctr[4] = {0, 0, 0, 0}, key[2] = {0, 0}, out[4];
    oracle_philox4x32_10(ctr, key, out);
    CHECK(out[0] == 0x6627e8d5u && out[3] == 0x9b00dbd8u);  /* published known answer */
    uint32_t* w = (uint32_t*)xmalloc(sizeof(uint32_t) * 1000);
    float* u = (float*)xmalloc(sizeof(float) * 1000);
    for (int i = 0; i < 1000; ++i) w[i] = (uint32_t)(i * 4294967u);
    oracle_to_unit_many(w, 1000, u);
    for (int i = 0; i < 1000; ++i) CHECK(u[i] > 0.0f && u[i] < 1.0f && u[i] == oracle_to_unit(w[i]));
    CHECK(oracle_uniform(7, 1, 2, 3, 4) > 0.0f);
    int32_t* starts = (int32_t*)xmalloc(sizeof(int32_t) * 33);
    oracle_start_cities(5, 2, 17, 33, starts);
    for (int i = 0; i < 33; ++i) CHECK(starts[i] == oracle_start_city(5, 2, (uint32_t)i, 17));
    CHECK(oracle_roulette_deviate(1, 2, 3, 4) > 0.0f);
    free(w); free(u); free(starts);
}

static void check_iteration(int32_t n, int32_t m, int32_t elite_k) {
    const size_t nn = (size_t)n * (size_t)n;
    float* D = distances(n);
    float* tau = (float*)xmalloc(sizeof(float) * nn);
    float* P = (float*)xmalloc(sizeof(float) * nn);
    for (size_t k = 0; k < nn; ++k) tau[k] = (k % ((size_t)n + 1) == 0) ? 0.0f : 1.0f;
    oracle_transition(tau, D, NULL, n, 1.0f, 2.0f, 1.5f, P);
    float* eta = (float*)xmalloc(sizeof(float) * nn);
    for (size_t k = 0; k < nn; ++k) eta[k] = (k % ((size_t)n + 1) == 0) ? 0.0f : 0.5f;
    float* P2 = (float*)xmalloc(sizeof(float) * nn);
    oracle_transition(tau, D, eta, n, 1.0f, 2.0f, 1.0f, P2);
    int32_t rows[2] = {0, n - 1};
    float* Prows = (float*)xmalloc(sizeof(float) * 2 * (size_t)n);
    oracle_transition_rows(tau, D, NULL, n, 1.0f, 2.0f, 1.5f, rows, 2, Prows);
    CHECK(memcmp(Prows, P, sizeof(float) * (size_t)n) == 0);

    int32_t* ants = (int32_t*)xmalloc(sizeof(int32_t) * (size_t)m);
    for (int32_t a = 0; a < m; ++a) ants[a] = a;
    int32_t* tours = (int32_t*)xmalloc(sizeof(int32_t) * (size_t)m * (size_t)n);
    float* lengths = (float*)xmalloc(sizeof(float) * (size_t)m);
    oracle_construct(P, D, n, 11, 0, ants, m, tours, lengths);
    for (int32_t a = 0; a < m; ++a) {
        CHECK(is_permutation(tours + (size_t)a * n, n));
        CHECK(lengths[a] == oracle_tour_length(tours + (size_t)a * n, D, n));
    }
    oracle_construct_roulette(P, D, n, 11, 0, ants, m, tours, lengths);
    for (int32_t a = 0; a < m; ++a) CHECK(is_permutation(tours + (size_t)a * n, n));

    /* single selections from a half-visited row */
    uint8_t* visited = (uint8_t*)xmalloc((size_t)n);
    for (int32_t j = 0; j < n; ++j) visited[j] = (uint8_t)(j % 2);
    double* p64 = (double*)xmalloc(sizeof(double) * (size_t)n);
    for (int32_t j = 0; j < n; ++j) p64[j] = (double)P[j];
    int32_t j1 = oracle_select(P, visited, n, 3, 1, 2, 3);
    CHECK(j1 >= 0 && j1 < n && !visited[j1]);
    int32_t j2 = oracle_select_literal(p64, visited, n, 1.5, 3, 1, 2, 3);
    CHECK(j2 >= 0 && j2 < n && !visited[j2]);
    int32_t j3 = oracle_select_roulette(P, visited, n, 3, 1, 2, 3);
    CHECK(j3 >= 0 && j3 < n && !visited[j3]);
    int32_t* picks = (int32_t*)xmalloc(sizeof(int32_t) * 9);
    oracle_select_many(P, p64, visited, n, 1.0, 0, 3, 1, 3, 9, picks);
    for (int i = 0; i < 9; ++i) CHECK(picks[i] >= 0 && picks[i] < n && !visited[picks[i]]);
    oracle_select_many(P, p64, visited, n, 1.5, 1, 3, 1, 3, 9, picks);
    for (int i = 0; i < 9; ++i) CHECK(picks[i] >= 0 && picks[i] < n && !visited[picks[i]]);
    oracle_select_roulette_many(P, visited, n, 3, 1, 3, 9, picks);
    for (int i = 0; i < 9; ++i) CHECK(picks[i] >= 0 && picks[i] < n && !visited[picks[i]]);

    /* elite, deposit, evaporation, clamp */
    uint8_t* elite = (uint8_t*)xmalloc((size_t)m);
    oracle_elite(lengths, m, elite_k, elite);
    int32_t kept = 0;
    for (int32_t a = 0; a < m; ++a) kept += elite[a];
    CHECK(kept == ((elite_k == 0 || elite_k > m) ? m : elite_k));
    const double lb = oracle_length_lower_bound(D, n);
    const int32_t S = oracle_deposit_scale(lb, m, 1.0f);
    /* the largest S at which m weights of at most 2^S / lb stay below 2^62 */
    CHECK(S > 0 && ldexp((double)m / lb, S) < 0x1.0p62 && ldexp((double)m / lb, S + 1) >= 0x1.0p62);
    int64_t* delta = (int64_t*)xmalloc(sizeof(int64_t) * nn);
    oracle_deposit(tours, lengths, elite, m, n, 1.0f, S, delta);
    __int128 total = 0, want = 0;
    for (int32_t a = 0; a < m; ++a)
        if (elite[a]) want += (__int128)oracle_deposit_weight(lengths[a], 1.0f, S);
    for (int32_t i = 0; i < n; ++i)
        for (int32_t j = 0; j < n; ++j) {
            total += delta[(size_t)i * n + j];
            CHECK(delta[(size_t)i * n + j] == delta[(size_t)j * n + i]);
        }
    CHECK(total == 2 * (__int128)n * want);
    oracle_evaporate(tau, delta, n, 0.3f, S);
    oracle_evaporate(tau, NULL, n, 0.3f, S);
    oracle_clamp(tau, n, 0.05f, 2.0f);
    for (int32_t i = 0; i < n; ++i)
        for (int32_t j = 0; j < n; ++j)
            if (i != j) CHECK(isfinite(tau[(size_t)i * n + j]) && tau[(size_t)i * n + j] >= 0.05f);

    free(D); free(tau); free(P); free(eta); free(P2); free(Prows); free(ants); free(tours);
    free(lengths); free(visited); free(p64); free(picks); free(elite); free(delta);
}

static void check_run(int32_t n, int32_t m, int32_t roulette) {
    const size_t nn = (size_t)n * (size_t)n;
    float* D = distances(n);
    float* tau = (float*)xmalloc(sizeof(float) * nn);
    float* P = (float*)xmalloc(sizeof(float) * nn);
    for (size_t k = 0; k < nn; ++k) tau[k] = (k % ((size_t)n + 1) == 0) ? 0.0f : 1.0f;
    int32_t* best = (int32_t*)xmalloc(sizeof(int32_t) * (size_t)n);
    float best_len = 0.0f;
    int32_t best_iter = -1;
    const int32_t iters = 6;
    float* per_iter = (float*)xmalloc(sizeof(float) * iters);
    int32_t S = oracle_run(D, NULL, n, m, m, 1.0f, 2.0f, 0.2f, 1.0f, m / 2, 1.5f, 1.0f,
                           roulette, 0.0f, INFINITY, 21, 0, iters, tau, P, best, &best_len,
                           &best_iter, per_iter);
    CHECK(S > 0);
    CHECK(is_permutation(best, n) && best_iter >= 0 && best_iter < iters);
    CHECK(best_len == oracle_tour_length(best, D, n));
    if (n <= 12) {
        int32_t* opt = (int32_t*)xmalloc(sizeof(int32_t) * (size_t)n);
        double L = oracle_tsp_exact(D, n, opt);
        CHECK(is_permutation(opt, n));
        CHECK((float)L <= best_len * (1.0f + 1e-6f));
        free(opt);
    }
    CHECK(oracle_gamma(0, iters, 1.5f, 1.0f) == 1.5f && oracle_gamma(iters - 1, iters, 1.5f, 1.0f) == 1.0f);
    free(D); free(tau); free(P); free(best); free(per_iter);
}

static void check_mlp(int32_t n) {
    const int32_t np = oracle_mlp_param_count();
    float* D = distances(n);
    int32_t* rank = (int32_t*)xmalloc(sizeof(int32_t) * (size_t)n * (size_t)n);
    oracle_edge_ranks(D, n, rank);
    for (int32_t i = 0; i < n; ++i) CHECK(rank[(size_t)i * n + i] == 0);
    const double mean = oracle_mean_nn(D, n);
    CHECK(mean > 0.0);
    float* feats = (float*)xmalloc(sizeof(float) * 3 * (size_t)n * (size_t)n);
    oracle_edge_features(D, rank, n, mean, feats);
    const int64_t count = (int64_t)n * n;
    double* params = (double*)xmalloc(sizeof(double) * (size_t)np);
    for (int32_t k = 0; k < np; ++k) params[k] = 0.2 * (lcg_unit() - 0.5);
    double* z = (double*)xmalloc(sizeof(double) * (size_t)count);
    double* eta = (double*)xmalloc(sizeof(double) * (size_t)count);
    oracle_mlp_forward(params, feats, count, 1, 1.4, 1.0, z, eta);
    for (int64_t e = 0; e < count; ++e) CHECK(isfinite(z[e]));
    float* y = (float*)xmalloc(sizeof(float) * (size_t)count);
    for (int64_t e = 0; e < count; ++e) y[e] = (float)lcg_unit();
    double* grad = (double*)xmalloc(sizeof(double) * (size_t)np);
    double* m = (double*)calloc((size_t)np, sizeof(double));
    double* v = (double*)calloc((size_t)np, sizeof(double));
    CHECK(m && v);
    double loss = oracle_mlp_loss_grad(params, feats, y, count, 1, grad);
    CHECK(isfinite(loss) && loss > 0.0);
    oracle_adam_step(params, m, v, grad, np, 1, 1e-3, 0.9, 0.999, 1e-8);
    for (int32_t k = 0; k < np; ++k) CHECK(isfinite(params[k]));
    CHECK(oracle_bf16_round(1.0f) == 1.0f);
    free(D); free(rank); free(feats); free(params); free(z); free(eta); free(y); free(grad);
    free(m); free(v);
}

int main(void) {
    check_generator();
    const int32_t sizes[][3] = {{3, 1, 0}, {4, 4, 2}, {7, 5, 0}, {31, 9, 3}, {64, 64, 0},
                                {65, 20, 7}, {130, 17, 0}};
    for (size_t k = 0; k < sizeof(sizes) / sizeof(sizes[0]); ++k)
        check_iteration(sizes[k][0], sizes[k][1], sizes[k][2]);
    check_run(9, 9, 0);
    check_run(9, 6, 1);
    check_run(40, 25, 0);
    check_mlp(3);
    check_mlp(37);
    if (failures) {
        fprintf(stderr, "sanitize_check: %d failures\n", failures);
        return 1;
    }
    printf("sanitize_check: ok\n");
    return 0;
}
