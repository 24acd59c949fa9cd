/*
 * Driver for the AddressSanitizer / UndefinedBehaviorSanitizer build of the CPU oracle
 * (oracle/wsr_oracle.c): every entry point on seeded inputs of many shapes (empty, d = 1, ties,
 * non-finite weights, many uneven segments over several threads, invalid arguments), with the
 * invariants of the prox checked on the results (the sum of the weights is kept, the order of
 * the weights is kept, |u_i - w_i| <= lam).  Exits 1 on a failed invariant; the sanitizers abort
 * on any memory or undefined-behaviour error.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int wsr_oracle_prox_f64(int64_t d, const double* w, double lam, double* u, int64_t* perm, uint8_t* start);
int wsr_oracle_prox_l1_f64(int64_t d, const double* w, double lam, double beta, double rho, double* u);
int wsr_oracle_prox_segments_f32(int64_t n_seg, const int64_t* offsets, const float* w, const float* lam,
                                 int per_seg_lam, double* u, int32_t* perm_local, uint8_t* start, int n_threads);
int wsr_oracle_prox_l1_segments_f32(int64_t n_seg, const int64_t* offsets, const float* w, const float* lam,
                                    int per_seg_lam, float beta, float rho, double* out, int n_threads);
int wsr_oracle_grad_step_f32(int64_t n, const float* w, const float* grad, float eta, float* z);
int wsr_oracle_prox_step_segments_f32(int64_t n_seg, const int64_t* offsets, const float* w, const float* grad,
                                      float eta, const float* alpha, int per_seg_alpha, float beta, float rho,
                                      int eta_in_displacement, double* out, int n_threads);
int wsr_oracle_segment_stats(int64_t n_seg, const int64_t* offsets, const float* w, double* penalty,
                             int64_t* distinct, int64_t* nonzero);
int wsr_oracle_vjp(int64_t n_seg, const int64_t* offsets, const int32_t* perm_local, const uint8_t* start,
                   const double* g, double* out);

static uint64_t rng_state = 0x2311030960ull;
static double uniform(void) { /* 53-bit uniform in [0, 1), splitmix64 */
    uint64_t z = (rng_state += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    return (double)(z >> 11) * (1.0 / 9007199254740992.0);
}
static double normal(void) {
    double a = uniform(), b = uniform();
    return sqrt(-2.0 * log(a + 1e-300)) * cos(6.283185307179586 * b);
}

static int failures = 0;
#define CHECK(cond, ...)                        \
    do {                                        \
        if (!(cond)) {                          \
            fprintf(stderr, "FAIL: " __VA_ARGS__); \
            fprintf(stderr, "\n");              \
            ++failures;                         \
        }                                       \
    } while (0)

/* sum kept, order kept, displacement at most lam */
static void check_prox(int64_t d, const double* w, const double* u, double lam, const char* what) {
    double sw = 0.0, su = 0.0, sa = 0.0;
    for (int64_t i = 0; i < d; ++i) {
        sw += w[i];
        su += u[i];
        sa += fabs(w[i]);
        CHECK(fabs(u[i] - w[i]) <= lam * (1.0 + 1e-12) + 1e-12, "%s: displacement at %lld", what, (long long)i);
    }
    CHECK(fabs(sw - su) <= 1e-9 * (1.0 + sa), "%s: sum %.17g vs %.17g", what, sw, su);
    for (int64_t i = 0; i + 1 < d && i < 200; ++i)
        for (int64_t j = 0; j < d && j < 200; ++j)
            if (w[i] < w[j]) CHECK(u[i] <= u[j] + 1e-12, "%s: order %lld %lld", what, (long long)i, (long long)j);
}

static void single_segments(void) {
    const int64_t sizes[] = {0, 1, 2, 3, 5, 7, 64, 100, 1000, 4097};
    const double lams[] = {0.0, 0.05, 1.0, 50.0};
    for (size_t a = 0; a < sizeof(sizes) / sizeof(sizes[0]); ++a)
        for (size_t b = 0; b < sizeof(lams) / sizeof(lams[0]); ++b)
            for (int ties = 0; ties < 2; ++ties) {
                const int64_t d = sizes[a];
                double* w = malloc(sizeof(double) * (size_t)(d + 1));
                double* u = malloc(sizeof(double) * (size_t)(d + 1));
                int64_t* perm = malloc(sizeof(int64_t) * (size_t)(d + 1));
                uint8_t* start = malloc((size_t)(d + 1));
                for (int64_t i = 0; i < d; ++i) w[i] = ties ? (double)(int)(8.0 * uniform()) / 4.0 : normal();
                CHECK(wsr_oracle_prox_f64(d, w, lams[b], u, perm, start) == 0, "prox_f64 rc d=%lld", (long long)d);
                check_prox(d, w, u, lams[b], "prox_f64");
                CHECK(wsr_oracle_prox_l1_f64(d, w, lams[b], 0.1, 0.5, u) == 0, "prox_l1_f64 rc");
                if (d > 0) {
                    w[d / 2] = NAN;  /* a non-finite weight: NaN output, no fault */
                    CHECK(wsr_oracle_prox_f64(d, w, lams[b], u, perm, start) == 0, "prox_f64 NaN rc");
                }
                free(w);
                free(u);
                free(perm);
                free(start);
            }
    double w1[3] = {1.0, 2.0, 3.0}, u1[3];
    CHECK(wsr_oracle_prox_f64(3, w1, -1.0, u1, NULL, NULL) == -1, "negative lambda accepted");
    CHECK(wsr_oracle_prox_f64(-1, w1, 1.0, u1, NULL, NULL) == -1, "negative length accepted");
    CHECK(wsr_oracle_prox_f64(3, w1, INFINITY, u1, NULL, NULL) == -1, "infinite lambda accepted");
}

static void batched(void) {
    const int64_t lens[] = {0, 1, 2, 3000, 17, 0, 4096, 9000, 5, 1};
    const int64_t ns = sizeof(lens) / sizeof(lens[0]);
    int64_t off[sizeof(lens) / sizeof(lens[0]) + 1];
    off[0] = 0;
    for (int64_t s = 0; s < ns; ++s) off[s + 1] = off[s] + lens[s];
    const int64_t n = off[ns];
    float* w = malloc(sizeof(float) * (size_t)n);
    float* g32 = malloc(sizeof(float) * (size_t)n);
    float* z = malloc(sizeof(float) * (size_t)n);
    float lam[sizeof(lens) / sizeof(lens[0])];
    double* u = malloc(sizeof(double) * (size_t)n);
    double* g = malloc(sizeof(double) * (size_t)n);
    double* vo = malloc(sizeof(double) * (size_t)n);
    int32_t* perm = malloc(sizeof(int32_t) * (size_t)n);
    uint8_t* start = malloc((size_t)n);
    double pen[sizeof(lens) / sizeof(lens[0])];
    int64_t dist[sizeof(lens) / sizeof(lens[0])], nz[sizeof(lens) / sizeof(lens[0])];
    for (int64_t i = 0; i < n; ++i) {
        w[i] = (float)normal();
        g32[i] = (float)normal();
        g[i] = g32[i];
    }
    for (int64_t s = 0; s < ns; ++s) lam[s] = (float)(0.01 * (double)s);
    for (int threads = 1; threads <= 3; ++threads) {
        CHECK(wsr_oracle_prox_segments_f32(ns, off, w, lam, 1, u, perm, start, threads) == 0, "segments rc");
        for (int64_t s = 0; s < ns; ++s) {
            double* ws = malloc(sizeof(double) * (size_t)(lens[s] + 1));
            for (int64_t i = 0; i < lens[s]; ++i) ws[i] = w[off[s] + i];
            check_prox(lens[s], ws, u + off[s], lam[s], "segments");
            free(ws);
        }
        CHECK(wsr_oracle_vjp(ns, off, perm, start, g, vo) == 0, "vjp rc");
        CHECK(wsr_oracle_prox_l1_segments_f32(ns, off, w, lam, 1, 0.05f, 0.98f, u, threads) == 0, "l1 rc");
        CHECK(wsr_oracle_prox_step_segments_f32(ns, off, w, g32, 0.1f, lam, 1, 0.01f, 0.5f, threads & 1, u,
                                                threads) == 0, "step rc");
    }
    CHECK(wsr_oracle_grad_step_f32(n, w, g32, 0.5f, z) == 0, "grad step rc");
    CHECK(wsr_oracle_segment_stats(ns, off, w, pen, dist, nz) == 0, "stats rc");
    int64_t bad[3] = {0, 5, 2};
    CHECK(wsr_oracle_segment_stats(2, bad, w, pen, dist, nz) == -1, "decreasing offsets accepted");
    CHECK(wsr_oracle_prox_l1_segments_f32(ns, off, w, lam, 1, -1.0f, 0.5f, u, 1) == -1, "negative beta accepted");
    free(w);
    free(g32);
    free(z);
    free(u);
    free(g);
    free(vo);
    free(perm);
    free(start);
}

int main(void) {
    single_segments();
    batched();
    if (failures) {
        fprintf(stderr, "%d failures\n", failures);
        return 1;
    }
    printf("oracle sanitizer driver: ok\n");
    return 0;
}
