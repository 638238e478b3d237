/*
 * mlp_oracle.c -- CPU oracle for the learned edge heuristic that may replace
 * eta = 1/d in Eq. (1) (Sec. 2.1): features, the 3-64-64-1 edge MLP, its
 * loss gradient and the Adam update.  None of this is in the paper; it is the
 * learned extension of the method, written from its definition below.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; it shares no code with the GPU path.
 *
 * Definitions (all sums in FP64 unless stated):
 *   rank_i(j)  1-based position of city j among the other cities sorted by
 *              distance from i, ties to the smaller index; rank_i(i) = 0.
 *   dNN        mean over cities of the nearest-neighbour distance, summed in
 *              ascending city order.
 *   features   f1 = fl32(d_ij / dNN), f2 = fl32(log2(1 + rank_i(j))),
 *              f3 = fl32(log2(1 + rank_j(i))).
 *   parameters 4481 values in this order: W1[64][3], b1[64], W2[64][64]
 *              (W2[u][k]: unit u of layer 2 from unit k of layer 1), b2[64],
 *              W3[64], b3.
 *   forward    a1 = W1 f + b1, h1 = relu(a1), a2 = W2 r(h1) + b2,
 *              h2 = relu(a2), z = W3 h2 + b3.
 *   heuristic  eta = sigmoid(z)^kappa / f1^lambda: the network's edge
 *              probability, raised to kappa, times the plain heuristic
 *              1/d (up to the constant dNN, which cancels in the row
 *              normalisation of Eq. (1)) raised to lambda; in FP64 through
 *              log sigmoid(z) = -softplus(-z).
 *              With rounding on, every parameter is first rounded to BF16
 *              (round to nearest even) and r() rounds h1 to BF16; with it off
 *              r() is the identity and parameters are used as given.
 *   loss       mean over edges of BCE-with-logits: softplus(z) - y z.
 *   gradient   exact FP64 derivative of the loss, with each rounding point
 *              passed through as the identity (straight-through), so the
 *              gradient with rounding off is the true gradient.
 *   Adam       m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2,
 *              w -= lr (m / (1-b1^t)) / (sqrt(v / (1-b2^t)) + eps).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_API __attribute__((visibility("default")))

enum { H = 64, NPARAM = 64 * 3 + 64 + 64 * 64 + 64 + 64 + 1 };
enum { OFF_W1 = 0, OFF_B1 = 192, OFF_W2 = 256, OFF_B2 = 4352, OFF_W3 = 4416, OFF_B3 = 4480 };

ORACLE_API int32_t oracle_mlp_param_count(void) { return NPARAM; }

/* Round an FP32 value to the nearest BF16 value (ties to even), returned as
 * FP32: keep the top 16 bits of the bit pattern after adding half an ulp of
 * BF16 plus the tie-breaking bit.  NaN stays NaN. */
ORACLE_API float oracle_bf16_round(float x) {
    uint32_t u;
    memcpy(&u, &x, 4);
    if ((u & 0x7F800000u) == 0x7F800000u && (u & 0x007FFFFFu)) return x; /* NaN */
    uint32_t lsb = (u >> 16) & 1u;
    u = (u + 0x7FFFu + lsb) & 0xFFFF0000u;
    float r;
    memcpy(&r, &u, 4);
    return r;
}

typedef struct {
    float d;
    int32_t j;
} by_distance;

static int compare_distance(const void* pa, const void* pb) {
    const by_distance* a = (const by_distance*)pa;
    const by_distance* b = (const by_distance*)pb;
    if (a->d < b->d) return -1;
    if (a->d > b->d) return 1;
    return (a->j > b->j) - (a->j < b->j);
}

/* rank is n x n int32. */
ORACLE_API void oracle_edge_ranks(const float* dist, int32_t n, int32_t* rank) {
#pragma omp parallel for schedule(static)
    for (int32_t i = 0; i < n; ++i) {
        by_distance* row = (by_distance*)malloc(sizeof(by_distance) * (size_t)n);
        int32_t k = 0;
        for (int32_t j = 0; j < n; ++j) {
            if (j == i) continue;
            row[k].d = dist[(size_t)i * (size_t)n + (size_t)j];
            row[k].j = j;
            ++k;
        }
        qsort(row, (size_t)k, sizeof(by_distance), compare_distance);
        rank[(size_t)i * (size_t)n + (size_t)i] = 0;
        for (int32_t p = 0; p < k; ++p) rank[(size_t)i * (size_t)n + (size_t)row[p].j] = p + 1;
        free(row);
    }
}

ORACLE_API double oracle_mean_nn(const float* dist, int32_t n) {
    double total = 0.0;
    for (int32_t i = 0; i < n; ++i) {
        float best = INFINITY;
        for (int32_t j = 0; j < n; ++j)
            if (j != i && dist[(size_t)i * (size_t)n + (size_t)j] < best)
                best = dist[(size_t)i * (size_t)n + (size_t)j];
        total += (double)best;
    }
    return total / (double)n;
}

/* feats is (n*n) x 3; the diagonal rows are left zero. */
ORACLE_API void oracle_edge_features(const float* dist, const int32_t* rank, int32_t n,
                                     double mean_nn, float* feats) {
    for (int32_t i = 0; i < n; ++i) {
        for (int32_t j = 0; j < n; ++j) {
            size_t ij = (size_t)i * (size_t)n + (size_t)j;
            float* f = feats + 3 * ij;
            if (i == j) {
                f[0] = f[1] = f[2] = 0.0f;
                continue;
            }
            f[0] = (float)((double)dist[ij] / mean_nn);
            f[1] = (float)log2(1.0 + (double)rank[ij]);
            f[2] = (float)log2(1.0 + (double)rank[(size_t)j * (size_t)n + (size_t)i]);
        }
    }
}

static void effective_params(const double* params, int32_t round_bf16, double* out) {
    for (int32_t p = 0; p < NPARAM; ++p)
        out[p] = round_bf16 ? (double)oracle_bf16_round((float)params[p]) : params[p];
}

static double sigmoid(double z) { return 1.0 / (1.0 + exp(-z)); }

static double softplus(double z) { return (z > 0 ? z : 0.0) + log1p(exp(-fabs(z))); }

/* One edge forward; fills the activations the backward pass needs. */
static double edge_forward(const double* w, const float* f, int32_t round_bf16, double* a1,
                           double* h1r, double* a2, double* h2) {
    for (int32_t u = 0; u < H; ++u) {
        double s = w[OFF_B1 + u];
        for (int32_t c = 0; c < 3; ++c) s += w[OFF_W1 + 3 * u + c] * (double)f[c];
        a1[u] = s;
        double h = s > 0.0 ? s : 0.0;
        h1r[u] = round_bf16 ? (double)oracle_bf16_round((float)h) : h;
    }
    double z = w[OFF_B3];
    for (int32_t u = 0; u < H; ++u) {
        double s = w[OFF_B2 + u];
        for (int32_t k = 0; k < H; ++k) s += w[OFF_W2 + H * u + k] * h1r[k];
        a2[u] = s;
        h2[u] = s > 0.0 ? s : 0.0;
        z += w[OFF_W3 + u] * h2[u];
    }
    return z;
}

ORACLE_API void oracle_mlp_forward(const double* params, const float* feats, int64_t count,
                                   int32_t round_bf16, double kappa, double lambda,
                                   double* z_out, double* eta_out) {
    double w[NPARAM];
    effective_params(params, round_bf16, w);
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < count; ++e) {
        double a1[H], h1r[H], a2[H], h2[H];
        const float* f = feats + 3 * e;
        double z = edge_forward(w, f, round_bf16, a1, h1r, a2, h2);
        if (z_out) z_out[e] = z;
        if (eta_out) {
            double log_sig = -softplus(-z);
            eta_out[e] = exp(kappa * log_sig - lambda * log((double)f[0]));
        }
    }
}

/* Mean BCE-with-logits loss over `count` edges and its gradient (grad has
 * NPARAM entries, overwritten).  Sequential over edges. */
ORACLE_API double oracle_mlp_loss_grad(const double* params, const float* feats, const float* y,
                                       int64_t count, int32_t round_bf16, double* grad) {
    double w[NPARAM];
    effective_params(params, round_bf16, w);
    memset(grad, 0, sizeof(double) * NPARAM);
    double loss = 0.0;
    const double inv = 1.0 / (double)count;
    for (int64_t e = 0; e < count; ++e) {
        const float* f = feats + 3 * e;
        double a1[H], h1r[H], a2[H], h2[H], g2[H];
        double z = edge_forward(w, f, round_bf16, a1, h1r, a2, h2);
        loss += softplus(z) - (double)y[e] * z;
        double dz = (sigmoid(z) - (double)y[e]) * inv;
        grad[OFF_B3] += dz;
        for (int32_t u = 0; u < H; ++u) {
            grad[OFF_W3 + u] += dz * h2[u];
            g2[u] = a2[u] > 0.0 ? dz * w[OFF_W3 + u] : 0.0;
            grad[OFF_B2 + u] += g2[u];
            for (int32_t k = 0; k < H; ++k) grad[OFF_W2 + H * u + k] += g2[u] * h1r[k];
        }
        for (int32_t k = 0; k < H; ++k) {
            if (!(a1[k] > 0.0)) continue;
            double g1 = 0.0;
            for (int32_t u = 0; u < H; ++u) g1 += g2[u] * w[OFF_W2 + H * u + k];
            grad[OFF_B1 + k] += g1;
            for (int32_t c = 0; c < 3; ++c) grad[OFF_W1 + 3 * k + c] += g1 * (double)f[c];
        }
    }
    return loss * inv;
}

ORACLE_API void oracle_adam_step(double* params, double* m, double* v, const double* grad,
                                 int32_t count, int32_t t, double lr, double b1, double b2,
                                 double eps) {
    const double c1 = 1.0 - pow(b1, (double)t);
    const double c2 = 1.0 - pow(b2, (double)t);
    for (int32_t p = 0; p < count; ++p) {
        m[p] = b1 * m[p] + (1.0 - b1) * grad[p];
        v[p] = b2 * v[p] + (1.0 - b2) * grad[p] * grad[p];
        params[p] -= lr * (m[p] / c1) / (sqrt(v[p] / c2) + eps);
    }
}
