/*
 * wsr_oracle.c -- CPU oracle for the proximal map of the weight-sharing penalty.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously correct
 * reference that the GPU library is checked against.  Only the test suite, the
 * smoke check and the benchmark's CPU-baseline leg may load it; the GPU library
 * never links, calls or includes anything from here, and this file includes
 * nothing from the GPU library.
 *
 * What it computes (paper: "Weight-Sharing Regularization", AISTATS 2024):
 *   R(w)        = 1/(d-1) * sum_{i>j} |w_i - w_j|                 (Sec. 1, eq. reg)
 *   prox_{lR}(w) = argmin_u  l*R(u) + 1/2 ||u - w||^2             (Sec. 1; App. A.1)
 * computed by the textbook sequential route the paper describes:
 *   1. sort w ascending (x = sorted w), keeping the permutation     (Sec. 4 preamble;
 *                                                                    Alg. prox, "sort")
 *   2. give the particle of rank k (0-based) the velocity
 *        v_k = l * (d-1-2k)/(d-1)  = -l * grad R at the sorted point (Sec. 2, eq. hyperplane;
 *                                                                    Alg. prox, "v <- ...")
 *   3. destinations y = x + v; pool adjacent violators: keep a stack of blocks and
 *      merge the top two while avg_y(lower) >= avg_y(upper)           (Sec. 4.1: a collision
 *      is detected when y_i >= y_{i+1}; merging is the sticky-particle collision,
 *      Sec. 3 particle model and Alg. search_collisions PerformCollisions)
 *   4. every rank in a block takes the block's y-average; scatter back to the
 *      original order                                                  (Alg. prox, last
 *                                                                    two steps)
 * All arithmetic is FP64.  Block sums of x use Neumaier compensated summation;
 * the block sum of v has the closed form  sum_{k=a}^{b} v_k = l*(b-a+1)*(d-1-a-b)/(d-1),
 * so a block's y-average is  sum_x/n + l*(d-1-a-b)/(d-1).
 *
 * Readings of the paper taken here (each is listed with its justification in the
 * design notes of the repository):
 *   - rank-shift indexing: v runs from +l (rank 0) to -l (rank d-1) so that the
 *     velocities sum to zero (conservation of momentum, Sec. 3 proposition);
 *   - merge on ">=" (coarsest partition: equal neighbouring outputs form one cluster);
 *   - sort ties broken by original index (any tie-break gives the same values);
 *   - d <= 1 or l == 0: identity, every element its own cluster;
 *   - a segment containing a non-finite weight yields NaN for the whole segment.
 *
 * Full Alg. prox (wsr_oracle_prox_l1_*): the same collisions, then the algorithm's
 * l1 and rewinding lines applied per cluster (prox of lam*R + beta*l1, rewinding rho).
 * Proximal-gradient step (wsr_oracle_prox_step_*): the gradient step in FP32, then the full
 * Alg. prox with eta in the coefficients or, as a variant, on the rewinding line.
 * Segment statistics (wsr_oracle_segment_stats): R(w) from the sorted order and the counts of
 * the weight-sharing measure.
 *
 * Gradient: the prox is piecewise affine; on the piece selected by the partition
 * its Jacobian averages within each cluster (symmetric, idempotent).  The
 * vector-Jacobian product is therefore the per-cluster mean of the cotangent.
 * (Not in the paper; follows from step 4 and the fact that the partition is
 * locally constant.)
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    double v;
    int64_t i;
} keyed_t;

static int cmp_keyed(const void* pa, const void* pb) {
    const keyed_t* a = (const keyed_t*)pa;
    const keyed_t* b = (const keyed_t*)pb;
    if (a->v < b->v) return -1;
    if (a->v > b->v) return 1;
    if (a->i < b->i) return -1;
    if (a->i > b->i) return 1;
    return 0;
}

/* Neumaier compensated accumulation: (*s + *c) += x */
static void nsum_add(double* s, double* c, double x) {
    double t = *s + x;
    if (fabs(*s) >= fabs(x))
        *c += (*s - t) + x;
    else
        *c += (x - t) + *s;
    *s = t;
}

/* y-average of the block of ranks [a, a+n-1] whose x-sum is (s + c). */
static double block_avg_y(double s, double c, int64_t a, int64_t n, int64_t d, double lam) {
    int64_t b = a + n - 1;
    return (s + c) / (double)n + lam * (double)(d - 1 - a - b) / (double)(d - 1);
}

/*
 * Single segment, FP64 in and out.
 *   w[d]      input weights (original order)
 *   lam       prox scale (step size x penalty), must be >= 0 and finite
 *   u[d]      output prox values (original order)
 *   perm[d]   optional: perm[k] = original index of rank k
 *   start[d]  optional: start[k] = 1 iff rank k begins a cluster
 * Returns 0, or -1 on bad arguments / allocation failure.
 */
int wsr_oracle_prox_f64(int64_t d, const double* w, double lam, double* u, int64_t* perm,
                        uint8_t* start) {
    if (d < 0 || !(lam >= 0.0) || isinf(lam)) return -1;
    if (d == 0) return 0;
    int finite = 1;
    for (int64_t i = 0; i < d; ++i)
        if (!isfinite(w[i])) finite = 0;
    if (!finite) {
        for (int64_t i = 0; i < d; ++i) {
            u[i] = NAN;
            if (perm) perm[i] = i;
            if (start) start[i] = 1;
        }
        return 0;
    }
    if (d == 1 || lam == 0.0) {
        for (int64_t i = 0; i < d; ++i) {
            u[i] = w[i];
            if (perm) perm[i] = i;
            if (start) start[i] = 1;
        }
        return 0;
    }

    keyed_t* xs = (keyed_t*)malloc(sizeof(keyed_t) * (size_t)d);
    int64_t* bstart = (int64_t*)malloc(sizeof(int64_t) * (size_t)d);
    int64_t* blen = (int64_t*)malloc(sizeof(int64_t) * (size_t)d);
    double* bs = (double*)malloc(sizeof(double) * (size_t)d);
    double* bc = (double*)malloc(sizeof(double) * (size_t)d);
    if (!xs || !bstart || !blen || !bs || !bc) {
        free(xs); free(bstart); free(blen); free(bs); free(bc);
        return -1;
    }
    for (int64_t i = 0; i < d; ++i) {
        xs[i].v = w[i];
        xs[i].i = i;
    }
    /* step 1: sort by (value, original index) */
    qsort(xs, (size_t)d, sizeof(keyed_t), cmp_keyed);

    /* step 3: stack pool-adjacent-violators on y = x + v */
    int64_t top = -1;
    for (int64_t k = 0; k < d; ++k) {
        ++top;
        bstart[top] = k;
        blen[top] = 1;
        bs[top] = xs[k].v;
        bc[top] = 0.0;
        while (top >= 1) {
            double lo = block_avg_y(bs[top - 1], bc[top - 1], bstart[top - 1], blen[top - 1], d, lam);
            double hi = block_avg_y(bs[top], bc[top], bstart[top], blen[top], d, lam);
            if (lo < hi) break;
            /* collision: the upper block sticks to the lower one */
            nsum_add(&bs[top - 1], &bc[top - 1], bs[top]);
            bc[top - 1] += bc[top];
            blen[top - 1] += blen[top];
            --top;
        }
    }

    /* step 4: every rank takes its block's y-average; scatter back */
    for (int64_t b = 0; b <= top; ++b) {
        double val = block_avg_y(bs[b], bc[b], bstart[b], blen[b], d, lam);
        for (int64_t k = bstart[b]; k < bstart[b] + blen[b]; ++k) {
            u[xs[k].i] = val;
            if (perm) perm[k] = xs[k].i;
            if (start) start[k] = (uint8_t)(k == bstart[b]);
        }
    }
    free(xs); free(bstart); free(blen); free(bs); free(bc);
    return 0;
}

/*
 * Alg. prox in full: the proximal map of  lam*R + beta*l1  with rewinding rho
 * (Sec. 1, prox of the combined penalty; App. "combining weight-sharing and
 * sparsity"; Sec. "rewinding").  The collisions give the clusters of prox_{lam R};
 * the algorithm then works per cluster C with
 *     x_C = mean of the weights of C        (what the collisions leave in x),
 *     v_C = mean velocity of C = lam*(d-1-a-b)/(d-1) for C = ranks [a, b],
 * and, in this order:
 *     zero  = |x_C + v_C| < beta           (x_C + v_C is the prox_{lam R} value)
 *     v_C  -= beta * sign(x_C + v_C)
 *     x_C = v_C = 0 where zero
 *     x_C  += (1 - rho) * v_C               (rewinding scales the remaining displacement)
 * and every rank of C takes x_C.  rho = 0 is prox_{lam R + beta l1}, which equals the
 * soft-thresholding of prox_{lam R} (the decomposition proposition); rho = 1 keeps the
 * cluster means of the surviving clusters.  The strict "<" of the zero test is the
 * algorithm's.  d <= 1 or lam == 0: every weight its own cluster with v_C = 0.
 * A segment containing a non-finite weight yields NaN for the whole segment.
 *   lam, beta >= 0 and finite; 0 <= rho <= 1.   out[d]: original order.
 * Returns 0, or -1 on bad arguments / allocation failure.
 */
static int prox_l1_kappa(int64_t d, const double* w, double lam, double beta, double rho,
                         double kappa, double* out);

int wsr_oracle_prox_l1_f64(int64_t d, const double* w, double lam, double beta, double rho,
                           double* out) {
    return prox_l1_kappa(d, w, lam, beta, rho, 1.0, out);
}

/*
 * The same with the rewinding line scaled by kappa:  x_C += kappa * (1 - rho) * v_C.  kappa = 1
 * is Alg. prox; kappa = eta is the variant of the experiments appendix (MNIST on a torus) that
 * multiplies the learning rate into v on that line instead of into alpha and beta.
 */
static int prox_l1_kappa(int64_t d, const double* w, double lam, double beta, double rho,
                         double kappa, double* out) {
    if (d < 0 || !(lam >= 0.0) || isinf(lam) || !(beta >= 0.0) || isinf(beta) ||
        !(rho >= 0.0) || !(rho <= 1.0) || !(kappa >= 0.0) || isinf(kappa))
        return -1;
    if (d == 0) return 0;
    double* u = (double*)malloc(sizeof(double) * (size_t)d);
    int64_t* perm = (int64_t*)malloc(sizeof(int64_t) * (size_t)d);
    uint8_t* start = (uint8_t*)malloc((size_t)d);
    if (!u || !perm || !start) {
        free(u); free(perm); free(start);
        return -1;
    }
    int rc = wsr_oracle_prox_f64(d, w, lam, u, perm, start);
    if (rc == 0) {
        int finite = 1;
        for (int64_t i = 0; i < d; ++i)
            if (!isfinite(w[i])) finite = 0;
        if (!finite) {
            for (int64_t i = 0; i < d; ++i) out[i] = NAN;
        } else {
            int64_t k = 0;
            while (k < d) {
                int64_t e = k + 1;
                while (e < d && !start[e]) ++e;
                /* cluster C = ranks [k, e-1] */
                double acc = 0.0, comp = 0.0;
                for (int64_t j = k; j < e; ++j) nsum_add(&acc, &comp, w[perm[j]]);
                double x = (acc + comp) / (double)(e - k);
                double v = (d <= 1 || lam == 0.0)
                               ? 0.0
                               : lam * (double)(d - 1 - k - (e - 1)) / (double)(d - 1);
                double y = x + v;
                int zero = fabs(y) < beta;
                double sgn = (double)((y > 0.0) - (y < 0.0));
                v = v - beta * sgn;
                if (zero) {
                    x = 0.0;
                    v = 0.0;
                }
                x = x + kappa * (1.0 - rho) * v;
                for (int64_t j = k; j < e; ++j) out[perm[j]] = x;
                k = e;
            }
        }
    }
    free(u); free(perm); free(start);
    return rc;
}

/* ---------------- flat buffer of FP32 segments (what the GPU library consumes) ---------------- */

typedef struct {
    int64_t seg_lo, seg_hi; /* segment range handled by this worker */
    const int64_t* offsets;
    const float* w;
    const float* lam;
    int per_seg_lam;
    double* u;
    int32_t* perm_local;
    uint8_t* start;
    int l1;            /* 1: Alg. prox with its l1 and rewinding lines (u receives its output) */
    double beta, rho;
    double kappa;      /* rewinding-line scale (1, or eta in the eta-in-displacement step) */
    const float* grad; /* non-NULL: the input is the gradient step fmaf(-eta, grad, w) */
    float eta;
    int lam_times_eta; /* the segment's lambda is the FP32 product eta * lambda */
    int rc;
} seg_job_t;

static void* seg_worker(void* arg) {
    seg_job_t* job = (seg_job_t*)arg;
    job->rc = 0;
    for (int64_t s = job->seg_lo; s < job->seg_hi; ++s) {
        int64_t o = job->offsets[s];
        int64_t d = job->offsets[s + 1] - o;
        float lam32 = job->per_seg_lam ? job->lam[s] : job->lam[0];
        if (job->lam_times_eta) lam32 = job->eta * lam32; /* one FP32 rounding */
        double lam = (double)lam32;
        double* w64 = (double*)malloc(sizeof(double) * (size_t)(d > 0 ? d : 1));
        int64_t* p64 = (int64_t*)malloc(sizeof(int64_t) * (size_t)(d > 0 ? d : 1));
        if (!w64 || !p64) {
            free(w64); free(p64);
            job->rc = -1;
            return NULL;
        }
        for (int64_t i = 0; i < d; ++i) {
            float x = job->w[o + i];
            if (job->grad) x = fmaf(-job->eta, job->grad[o + i], x); /* gradient step, one rounding */
            w64[i] = (double)x; /* exact promotion */
        }
        int rc = job->l1 ? prox_l1_kappa(d, w64, lam, job->beta, job->rho, job->kappa, job->u + o)
                         : wsr_oracle_prox_f64(d, w64, lam, job->u + o, p64,
                                               job->start ? job->start + o : NULL);
        if (rc) job->rc = rc;
        if (job->perm_local && !job->l1)
            for (int64_t k = 0; k < d; ++k) job->perm_local[o + k] = (int32_t)p64[k];
        free(w64);
        free(p64);
    }
    return NULL;
}

/*
 * Flat FP32 buffer split into segments offsets[0..n_seg] (offsets[0] = 0, non-decreasing).
 * Segment s gets prox_{lam_s R_{d_s}} with R normalised by its own 1/(d_s - 1).
 *   lam: one value (per_seg_lam = 0) or n_seg values (per_seg_lam = 1), promoted exactly to FP64
 *   u: FP64 output, original order;  perm_local: rank -> segment-local original index
 *   start: 1 at ranks that begin a cluster.  perm_local and start may be NULL.
 *   n_threads: segments are split across this many POSIX threads (>= 1).
 */
typedef struct {
    int l1;
    double beta, rho, kappa;
    const float* grad;
    float eta;
    int lam_times_eta;
} seg_opts_t;

static int run_segments(int64_t n_seg, const int64_t* offsets, const float* w, const float* lam,
                        int per_seg_lam, double* u, int32_t* perm_local, uint8_t* start,
                        int n_threads, seg_opts_t opt) {
    if (n_seg < 0 || !offsets || offsets[0] != 0) return -1;
    for (int64_t s = 0; s < n_seg; ++s) {
        if (offsets[s + 1] < offsets[s]) return -1;
        float l = per_seg_lam ? lam[s] : lam[0];
        if (!(l >= 0.0f) || isinf(l)) return -1;
    }
    if (n_threads < 1) n_threads = 1;
    if ((int64_t)n_threads > n_seg) n_threads = (int)(n_seg > 0 ? n_seg : 1);
    seg_job_t* jobs = (seg_job_t*)calloc((size_t)n_threads, sizeof(seg_job_t));
    pthread_t* th = (pthread_t*)calloc((size_t)n_threads, sizeof(pthread_t));
    if (!jobs || !th) {
        free(jobs); free(th);
        return -1;
    }
    /* balance by element count, not segment count */
    int64_t total = offsets[n_seg];
    int64_t s = 0;
    for (int t = 0; t < n_threads; ++t) {
        int64_t target = total * (t + 1) / n_threads;
        jobs[t].seg_lo = s;
        while (s < n_seg && (offsets[s] < target || t == n_threads - 1)) ++s;
        jobs[t].seg_hi = s;
        jobs[t].offsets = offsets;
        jobs[t].w = w;
        jobs[t].lam = lam;
        jobs[t].per_seg_lam = per_seg_lam;
        jobs[t].u = u;
        jobs[t].perm_local = perm_local;
        jobs[t].start = start;
        jobs[t].l1 = opt.l1;
        jobs[t].beta = opt.beta;
        jobs[t].rho = opt.rho;
        jobs[t].kappa = opt.kappa;
        jobs[t].grad = opt.grad;
        jobs[t].eta = opt.eta;
        jobs[t].lam_times_eta = opt.lam_times_eta;
    }
    int rc = 0;
    if (n_threads == 1) {
        seg_worker(&jobs[0]);
        rc = jobs[0].rc;
    } else {
        for (int t = 0; t < n_threads; ++t) pthread_create(&th[t], NULL, seg_worker, &jobs[t]);
        for (int t = 0; t < n_threads; ++t) {
            pthread_join(th[t], NULL);
            if (jobs[t].rc) rc = jobs[t].rc;
        }
    }
    free(jobs);
    free(th);
    return rc;
}

int wsr_oracle_prox_segments_f32(int64_t n_seg, const int64_t* offsets, const float* w,
                                 const float* lam, int per_seg_lam, double* u,
                                 int32_t* perm_local, uint8_t* start, int n_threads) {
    seg_opts_t opt = {0, 0.0, 0.0, 1.0, NULL, 0.0f, 0};
    return run_segments(n_seg, offsets, w, lam, per_seg_lam, u, perm_local, start, n_threads, opt);
}

/*
 * Alg. prox in full (wsr_oracle_prox_l1_f64) on every segment of a flat FP32 buffer, with the
 * segment's lam (as in wsr_oracle_prox_segments_f32) and one beta and rho for all segments,
 * promoted exactly to FP64.  out: FP64, original order.
 */
int wsr_oracle_prox_l1_segments_f32(int64_t n_seg, const int64_t* offsets, const float* w,
                                    const float* lam, int per_seg_lam, float beta, float rho,
                                    double* out, int n_threads) {
    if (!(beta >= 0.0f) || isinf(beta) || !(rho >= 0.0f) || !(rho <= 1.0f)) return -1;
    seg_opts_t opt = {1, (double)beta, (double)rho, 1.0, NULL, 0.0f, 0};
    return run_segments(n_seg, offsets, w, lam, per_seg_lam, out, NULL, NULL, n_threads, opt);
}

/* The gradient step alone: z[i] = fmaf(-eta, grad[i], w[i]) in FP32 (one rounding). */
int wsr_oracle_grad_step_f32(int64_t n, const float* w, const float* grad, float eta, float* z) {
    if (n < 0 || (n > 0 && (!w || !grad || !z))) return -1;
    for (int64_t i = 0; i < n; ++i) z[i] = fmaf(-eta, grad[i], w[i]);
    return 0;
}

/*
 * One proximal-gradient step (Sec. 1 update with Alg. prox in full): every weight first takes
 * the gradient step z = fmaf(-eta, grad, w) in FP32 (one rounding), then each segment gets
 *   eta_in_displacement == 0:  Alg. prox of z with lambda = eta*alpha_s (FP32 product),
 *                              beta' = eta*beta (FP32 product) and rho, i.e. the prox of
 *                              eta*(alpha R + beta l1) with rewinding;
 *   eta_in_displacement == 1:  Alg. prox of z with alpha_s and beta unscaled and the rewinding
 *                              line x += eta (1 - rho) v (experiments appendix, MNIST on a torus).
 * alpha: one value or n_seg values (per_seg_alpha).  out: FP64, original order.
 */
int wsr_oracle_prox_step_segments_f32(int64_t n_seg, const int64_t* offsets, const float* w,
                                      const float* grad, float eta, const float* alpha,
                                      int per_seg_alpha, float beta, float rho,
                                      int eta_in_displacement, double* out, int n_threads) {
    if (!grad || !(eta >= 0.0f) || isinf(eta)) return -1;
    if (!(beta >= 0.0f) || isinf(beta) || !(rho >= 0.0f) || !(rho <= 1.0f)) return -1;
    seg_opts_t opt;
    opt.l1 = 1;
    opt.rho = (double)rho;
    opt.grad = grad;
    opt.eta = eta;
    if (eta_in_displacement) {
        opt.beta = (double)beta;
        opt.kappa = (double)eta;
        opt.lam_times_eta = 0;
    } else {
        float b = eta * beta; /* one FP32 rounding */
        opt.beta = (double)b;
        opt.kappa = 1.0;
        opt.lam_times_eta = 1;
    }
    return run_segments(n_seg, offsets, w, alpha, per_seg_alpha, out, NULL, NULL, n_threads, opt);
}

static int cmp_double(const void* pa, const void* pb) {
    double a = *(const double*)pa, b = *(const double*)pb;
    return (a > b) - (a < b);
}

/*
 * Per-segment statistics of a flat FP32 buffer, each from the sorted segment x_0 <= ... <= x_{d-1}:
 *   penalty[s]  = R(w_s) = 1/(d-1) * sum_k (2k - d + 1) x_k      (App. B: R in O(d log d) from the
 *                 sorted order, each pair counted once with the larger element positive); 0 for d <= 1
 *   distinct[s] = number of distinct non-zero values               (numerator of the weight-sharing
 *   nonzero[s]  = number of non-zero weights                        measure of the CIFAR10 table)
 * -0 counts as zero.  A segment with a non-finite weight gets penalty NaN and counts -1.
 * FP64, Neumaier summation.
 */
int wsr_oracle_segment_stats(int64_t n_seg, const int64_t* offsets, const float* w, double* penalty,
                             int64_t* distinct, int64_t* nonzero) {
    if (n_seg < 0 || !offsets || offsets[0] != 0) return -1;
    for (int64_t s = 0; s < n_seg; ++s)
        if (offsets[s + 1] < offsets[s]) return -1;
    for (int64_t s = 0; s < n_seg; ++s) {
        int64_t o = offsets[s];
        int64_t d = offsets[s + 1] - o;
        double* x = (double*)malloc(sizeof(double) * (size_t)(d > 0 ? d : 1));
        if (!x) return -1;
        int finite = 1;
        for (int64_t i = 0; i < d; ++i) {
            x[i] = (double)w[o + i];
            if (!isfinite(x[i])) finite = 0;
        }
        if (!finite) {
            penalty[s] = NAN;
            distinct[s] = -1;
            nonzero[s] = -1;
            free(x);
            continue;
        }
        qsort(x, (size_t)d, sizeof(double), cmp_double);
        double acc = 0.0, comp = 0.0;
        int64_t nd = 0, nz = 0;
        for (int64_t k = 0; k < d; ++k) {
            nsum_add(&acc, &comp, (double)(2 * k - d + 1) * x[k]);
            if (x[k] != 0.0) {
                ++nz;
                if (k == 0 || x[k] != x[k - 1]) ++nd;
            }
        }
        penalty[s] = d > 1 ? (acc + comp) / (double)(d - 1) : 0.0;
        distinct[s] = nd;
        nonzero[s] = nz;
        free(x);
    }
    return 0;
}

/*
 * Vector-Jacobian product of the prox at the point whose partition is (perm_local, start):
 * out[i] = mean of g over the cluster containing i.  FP64, per segment, sums in rank order.
 */
int wsr_oracle_vjp(int64_t n_seg, const int64_t* offsets, const int32_t* perm_local,
                   const uint8_t* start, const double* g, double* out) {
    if (n_seg < 0 || !offsets || offsets[0] != 0) return -1;
    for (int64_t s = 0; s < n_seg; ++s) {
        int64_t o = offsets[s];
        int64_t d = offsets[s + 1] - o;
        int64_t k = 0;
        while (k < d) {
            int64_t e = k + 1;
            while (e < d && !start[o + e]) ++e;
            double acc = 0.0, comp = 0.0;
            for (int64_t j = k; j < e; ++j) nsum_add(&acc, &comp, g[o + perm_local[o + j]]);
            double mean = (acc + comp) / (double)(e - k);
            for (int64_t j = k; j < e; ++j) out[o + perm_local[o + j]] = mean;
            k = e;
        }
    }
    return 0;
}
