/*
 * CPU oracle for the all-families regression scores -- TEST INFRASTRUCTURE.
 *
 * Only the tests, the smoke check and the benchmark's CPU-baseline leg may load
 * this code.  It shares nothing with the GPU library: no headers, tables or
 * helpers.  It is deliberately plain and slow: every family is solved on its
 * own, the way the paper's brute-force baseline does it (Sec. 1.1: solve the
 * regression of each child on each parent set independently, via a QR of that
 * family's data, cost O(2 n k^2) per family).
 *
 * Definitions written out here (the readings are listed in the design notes):
 *   family (c, S): child c in {0..m-1}, parent set S a subset of the other m-1
 *                  variables, the empty set included -- m * 2^(m-1) families
 *                  (Sec. 1: "a total of m 2^(m-1) candidate families").
 *   RSS(c, S)    = min_beta || x_c - X_S beta ||^2, no intercept, X as given.
 *   BIC(c, S)    = n ln(RSS/n) + (|S| + 2) ln n   (the paper leaves the score
 *                  as "a function of the regression"; this is the reading).
 *   index(c, S)  = c * 2^(m-1) + compress(S, c), compress drops bit c and shifts
 *                  the higher bits down by one.
 * All arithmetic is IEEE double.  RSS comes from textbook Householder QR of
 * [X_S (ascending labels) | x_c]: after the |S| reflections that triangularise
 * X_S, RSS is the squared norm of the transformed x_c below row |S| -- the
 * squared last diagonal entry of R, which is the QRD-to-regression identity of
 * Sec. 2 ([A,B,C] gives [A,B] -> C).
 *
 * A second, independent route (or_score_all_gram) solves the normal equations, the
 * covariance / Cholesky brute force of Table 1: with G = X^T X accumulated in
 * x87 extended precision, RSS(c, S) is the last pivot of the Cholesky elimination of
 * the Gram matrix of [X_S | x_c], i.e. the Schur complement G_cc - G_cS G_SS^-1 G_Sc.
 * It costs O(|S|^3) per family instead of O(n |S|^2), which makes whole tables of
 * mid-size problems cheap to check.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_OUT_BIC 0
#define OR_OUT_RSS 1

int64_t or_num_families(int m) {
    if (m < 1 || m > 40) return -1;
    return (int64_t)m << (m - 1);
}

int64_t or_family_index(int m, int child, uint64_t mask) {
    if (m < 1 || m > 40 || child < 0 || child >= m) return -1;
    if ((mask >> child) & 1ull) return -1;
    if (m < 64 && (mask >> m) != 0) return -1;
    uint64_t low = mask & ((1ull << child) - 1ull);
    uint64_t high = (mask >> (child + 1)) << child;
    return ((int64_t)child << (m - 1)) + (int64_t)(low | high);
}

int or_family_decode(int m, int64_t idx, int *child, uint64_t *mask) {
    if (m < 1 || m > 40 || idx < 0 || idx >= ((int64_t)m << (m - 1))) return -1;
    int c = (int)(idx >> (m - 1));
    uint64_t comp = (uint64_t)idx & ((1ull << (m - 1)) - 1ull);
    uint64_t low = comp & ((1ull << c) - 1ull);
    uint64_t high = (comp >> c) << (c + 1);
    *child = c;
    *mask = low | high;
    return 0;
}

double or_bic(double rss, int64_t n, int nparents) {
    double dn = (double)n;
    return dn * log(rss / dn) + (double)(nparents + 2) * log(dn);
}

/* RSS of x_child on the columns in mask (Householder, column-major work copy). */
static double rss_householder(const double *X, int64_t n, int m, int64_t ldx, int child,
                              uint64_t mask, double *work) {
    int cols[64];
    int s = 0;
    for (int v = 0; v < m; ++v)
        if ((mask >> v) & 1ull) cols[s++] = v;
    cols[s] = child;
    const int w = s + 1;
    /* work: column-major n x w */
    for (int j = 0; j < w; ++j) {
        double *dst = work + (int64_t)j * n;
        const double *src = X + cols[j];
        for (int64_t i = 0; i < n; ++i) dst[i] = src[i * ldx];
    }
    const int steps = s < n ? s : (int)n;
    for (int j = 0; j < steps; ++j) {
        double *a = work + (int64_t)j * n;
        double normx2 = 0.0;
        for (int64_t i = j; i < n; ++i) normx2 += a[i] * a[i];
        if (normx2 == 0.0) continue; /* column already zero below the diagonal */
        double normx = sqrt(normx2);
        double alpha = a[j] >= 0.0 ? -normx : normx;
        double v0 = a[j] - alpha;
        /* v = (v0, a[j+1..n-1]);  v^T v = normx2 - a[j]^2 + v0^2 */
        double vtv = normx2 - a[j] * a[j] + v0 * v0;
        for (int c = j + 1; c < w; ++c) {
            double *b = work + (int64_t)c * n;
            double dot = v0 * b[j];
            for (int64_t i = j + 1; i < n; ++i) dot += a[i] * b[i];
            double f = 2.0 * dot / vtv;
            b[j] -= f * v0;
            for (int64_t i = j + 1; i < n; ++i) b[i] -= f * a[i];
        }
        a[j] = alpha;
        for (int64_t i = j + 1; i < n; ++i) a[i] = 0.0;
    }
    const double *y = work + (int64_t)s * n;
    double rss = 0.0;
    for (int64_t i = steps; i < n; ++i) rss += y[i] * y[i];
    return rss;
}

double or_rss(const double *X, int64_t n, int m, int64_t ldx, int child, uint64_t mask) {
    if (m < 1 || m > 40 || child < 0 || child >= m || ((mask >> child) & 1ull)) return NAN;
    int s = __builtin_popcountll(mask);
    double *work = (double *)malloc(sizeof(double) * (size_t)n * (size_t)(s + 1));
    if (!work) return NAN;
    double r = rss_householder(X, n, m, ldx, child, mask, work);
    free(work);
    return r;
}

typedef struct {
    const double *X;
    int64_t n;
    int m;
    int64_t ldx;
    const int64_t *idx; /* NULL: all families */
    int64_t begin, end;
    double *out;
    int what;
    int status;
} job_t;

static void *run_job(void *p) {
    job_t *jb = (job_t *)p;
    double *work = (double *)malloc(sizeof(double) * (size_t)jb->n * (size_t)(jb->m + 1));
    if (!work) {
        jb->status = -3;
        return NULL;
    }
    for (int64_t t = jb->begin; t < jb->end; ++t) {
        int64_t id = jb->idx ? jb->idx[t] : t;
        int c;
        uint64_t mask;
        if (or_family_decode(jb->m, id, &c, &mask) != 0) {
            jb->out[t] = NAN;
            jb->status = -1;
            continue;
        }
        double rss = rss_householder(jb->X, jb->n, jb->m, jb->ldx, c, mask, work);
        jb->out[t] = jb->what == OR_OUT_RSS ? rss : or_bic(rss, jb->n, __builtin_popcountll(mask));
    }
    free(work);
    return NULL;
}

static int run_parallel(const double *X, int64_t n, int m, int64_t ldx, const int64_t *idx,
                        int64_t count, double *out, int what, int nthreads) {
    if (!X || !out || n < 1 || m < 1 || m > 40 || ldx < m) return -1;
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    if (count < nthreads) nthreads = count > 0 ? (int)count : 1;
    pthread_t th[256];
    job_t jobs[256];
    for (int t = 0; t < nthreads; ++t) {
        jobs[t] = (job_t){X, n, m, ldx, idx, count * t / nthreads, count * (t + 1) / nthreads,
                          out, what, 0};
        if (nthreads > 1) {
            if (pthread_create(&th[t], NULL, run_job, &jobs[t]) != 0) {
                run_job(&jobs[t]);
                th[t] = 0;
            }
        } else {
            run_job(&jobs[t]);
        }
    }
    int st = 0;
    for (int t = 0; t < nthreads; ++t) {
        if (nthreads > 1 && th[t]) pthread_join(th[t], NULL);
        if (jobs[t].status) st = jobs[t].status;
    }
    return st;
}

/* ---- normal-equations route ------------------------------------------------------ */

#define OR_GRAM_MAXW 41

/* RSS of x_child on the columns in mask from the Gram matrix G (m x m, long double):
 * Cholesky elimination of the Gram matrix of [X_S (ascending labels) | x_c]; the last
 * pivot, before its square root, is the squared residual. */
static double rss_gram(const long double *G, int m, int child, uint64_t mask) {
    int cols[64];
    int s = 0;
    for (int v = 0; v < m; ++v)
        if ((mask >> v) & 1ull) cols[s++] = v;
    cols[s] = child;
    const int w = s + 1;
    long double L[OR_GRAM_MAXW][OR_GRAM_MAXW];
    for (int j = 0; j < w; ++j) {
        long double d = G[cols[j] * m + cols[j]];
        for (int k = 0; k < j; ++k) d -= L[j][k] * L[j][k];
        if (j == w - 1) return (double)d;
        const long double ljj = sqrtl(d);
        L[j][j] = ljj;
        for (int i = j + 1; i < w; ++i) {
            long double a = G[cols[i] * m + cols[j]];
            for (int k = 0; k < j; ++k) a -= L[i][k] * L[j][k];
            L[i][j] = a / ljj;
        }
    }
    return NAN; /* not reached: w >= 1 */
}

typedef struct {
    const long double *G;
    int64_t n;
    int m;
    const int64_t *idx;
    int64_t begin, end;
    double *out;
    int what;
    int status;
} gramjob_t;

static void *run_gram_job(void *p) {
    gramjob_t *jb = (gramjob_t *)p;
    for (int64_t t = jb->begin; t < jb->end; ++t) {
        int64_t id = jb->idx ? jb->idx[t] : t;
        int c;
        uint64_t mask;
        if (or_family_decode(jb->m, id, &c, &mask) != 0) {
            jb->out[t] = NAN;
            jb->status = -1;
            continue;
        }
        double rss = rss_gram(jb->G, jb->m, c, mask);
        jb->out[t] = jb->what == OR_OUT_RSS ? rss : or_bic(rss, jb->n, __builtin_popcountll(mask));
    }
    return NULL;
}

static int run_gram(const double *X, int64_t n, int m, int64_t ldx, const int64_t *idx,
                    int64_t count, double *out, int what, int nthreads) {
    if (!X || !out || n < 1 || m < 1 || m > OR_GRAM_MAXW - 1 || ldx < m) return -1;
    long double *G = (long double *)malloc(sizeof(long double) * (size_t)m * (size_t)m);
    if (!G) return -3;
    for (int i = 0; i < m; ++i)
        for (int j = 0; j < m; ++j) {
            long double acc = 0.0L;
            for (int64_t r = 0; r < n; ++r)
                acc += (long double)X[r * ldx + i] * (long double)X[r * ldx + j];
            G[i * m + j] = acc;
        }
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    if (count < nthreads) nthreads = count > 0 ? (int)count : 1;
    pthread_t th[256];
    gramjob_t jobs[256];
    for (int t = 0; t < nthreads; ++t) {
        jobs[t] = (gramjob_t){G, n, m, idx, count * t / nthreads, count * (t + 1) / nthreads,
                              out, what, 0};
        if (nthreads > 1) {
            if (pthread_create(&th[t], NULL, run_gram_job, &jobs[t]) != 0) {
                run_gram_job(&jobs[t]);
                th[t] = 0;
            }
        } else {
            run_gram_job(&jobs[t]);
        }
    }
    int st = 0;
    for (int t = 0; t < nthreads; ++t) {
        if (nthreads > 1 && th[t]) pthread_join(th[t], NULL);
        if (jobs[t].status) st = jobs[t].status;
    }
    free(G);
    return st;
}

/* Every family by the normal-equations route, table order. */
int or_score_all_gram(const double *X, int64_t n, int m, int64_t ldx, double *out, int what,
                      int nthreads) {
    return run_gram(X, n, m, ldx, NULL, or_num_families(m), out, what, nthreads);
}

/* Every family, table order.  out has m * 2^(m-1) doubles. */
int or_score_all(const double *X, int64_t n, int m, int64_t ldx, double *out, int what, int nthreads) {
    return run_parallel(X, n, m, ldx, NULL, or_num_families(m), out, what, nthreads);
}

/* Selected table indices. */
int or_score_indices(const double *X, int64_t n, int m, int64_t ldx, const int64_t *idx,
                     int64_t count, double *out, int what, int nthreads) {
    if (!idx && count > 0) return -1;
    return run_parallel(X, n, m, ldx, idx, count, out, what, nthreads);
}

/* ---------------------------------------------------------------------------------
 * Gradient oracle.  For RSS(c,S) = min_beta ||x_c - X_S beta||^2 the envelope theorem
 * gives d RSS / d X = 2 r w^T with r = X w the residual and w = e_c - beta (beta placed
 * at the rows of S).  For any loss L of the table with gbar(c,S) = dL/dRSS(c,S):
 *     dL/dX = 2 X A,   A = sum_{c,S} gbar(c,S) w w^T   (m x m).
 * beta comes from the same Householder QR as the RSS (back-substitution on R_SS).
 * ------------------------------------------------------------------------------- */

/* beta of x_child on the columns in mask: QR of [X_S | x_c], then R_SS beta = (Q^T x_c)_S. */
static void beta_householder(const double *X, int64_t n, int m, int64_t ldx, int child,
                             uint64_t mask, double *work, double *beta_full) {
    int cols[64];
    int s = 0;
    for (int v = 0; v < m; ++v)
        if ((mask >> v) & 1ull) cols[s++] = v;
    cols[s] = child;
    const int w = s + 1;
    for (int j = 0; j < w; ++j) {
        double *dst = work + (int64_t)j * n;
        const double *src = X + cols[j];
        for (int64_t i = 0; i < n; ++i) dst[i] = src[i * ldx];
    }
    for (int j = 0; j < s; ++j) {
        double *a = work + (int64_t)j * n;
        double normx2 = 0.0;
        for (int64_t i = j; i < n; ++i) normx2 += a[i] * a[i];
        if (normx2 == 0.0) continue;
        double normx = sqrt(normx2);
        double alpha = a[j] >= 0.0 ? -normx : normx;
        double v0 = a[j] - alpha;
        double vtv = normx2 - a[j] * a[j] + v0 * v0;
        for (int c = j + 1; c < w; ++c) {
            double *b = work + (int64_t)c * n;
            double dot = v0 * b[j];
            for (int64_t i = j + 1; i < n; ++i) dot += a[i] * b[i];
            double f = 2.0 * dot / vtv;
            b[j] -= f * v0;
            for (int64_t i = j + 1; i < n; ++i) b[i] -= f * a[i];
        }
        a[j] = alpha;
        for (int64_t i = j + 1; i < n; ++i) a[i] = 0.0;
    }
    /* back-substitution: R_SS beta = y_S, R_SS[i][j] = work[j*n + i] */
    const double *y = work + (int64_t)s * n;
    double bl[64];
    for (int i = s - 1; i >= 0; --i) {
        double acc = y[i];
        for (int j = i + 1; j < s; ++j) acc -= work[(int64_t)j * n + i] * bl[j];
        bl[i] = acc / work[(int64_t)i * n + i];
    }
    for (int v = 0; v < m; ++v) beta_full[v] = 0.0;
    for (int i = 0; i < s; ++i) beta_full[cols[i]] = bl[i];
}

/* Coefficients of every family, table order: out[idx * m + v] = beta_v of family idx
 * (zero for v outside the parent set, and for v = the child). */
typedef struct {
    const double *X;
    int64_t n;
    int m;
    int64_t ldx;
    int64_t begin, end;
    double *out;
    int status;
} bjob_t;

static void *run_bjob(void *p) {
    bjob_t *jb = (bjob_t *)p;
    double *work = (double *)malloc(sizeof(double) * (size_t)jb->n * (size_t)(jb->m + 1));
    if (!work) {
        jb->status = -3;
        return NULL;
    }
    for (int64_t t = jb->begin; t < jb->end; ++t) {
        int c;
        uint64_t mask;
        or_family_decode(jb->m, t, &c, &mask);
        beta_householder(jb->X, jb->n, jb->m, jb->ldx, c, mask, work, jb->out + t * jb->m);
    }
    free(work);
    return NULL;
}

int or_beta_all(const double *X, int64_t n, int m, int64_t ldx, double *out, int nthreads) {
    if (!X || !out || n < 1 || m < 1 || m > 40 || ldx < m) return -1;
    const int64_t N = or_num_families(m);
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 64) nthreads = 64;
    if (N < nthreads) nthreads = (int)N;
    pthread_t th[64];
    bjob_t jobs[64];
    for (int t = 0; t < nthreads; ++t) {
        jobs[t] = (bjob_t){X, n, m, ldx, N * t / nthreads, N * (t + 1) / nthreads, out, 0};
        if (nthreads > 1) {
            if (pthread_create(&th[t], NULL, run_bjob, &jobs[t]) != 0) {
                run_bjob(&jobs[t]);
                th[t] = 0;
            }
        } else {
            run_bjob(&jobs[t]);
        }
    }
    int st = 0;
    for (int t = 0; t < nthreads; ++t) {
        if (nthreads > 1 && th[t]) pthread_join(th[t], NULL);
        if (jobs[t].status) st = jobs[t].status;
    }
    return st;
}

typedef struct {
    const double *X;
    int64_t n;
    int m;
    int64_t ldx;
    const double *gbar;
    int64_t begin, end;
    double A[64 * 64];
    int status;
} gjob_t;

static void *run_gjob(void *p) {
    gjob_t *jb = (gjob_t *)p;
    const int m = jb->m;
    double *work = (double *)malloc(sizeof(double) * (size_t)jb->n * (size_t)(m + 1));
    if (!work) {
        jb->status = -3;
        return NULL;
    }
    double w[64];
    for (int i = 0; i < m * m; ++i) jb->A[i] = 0.0;
    for (int64_t t = jb->begin; t < jb->end; ++t) {
        const double g = jb->gbar[t];
        if (g == 0.0) continue;
        int c;
        uint64_t mask;
        or_family_decode(m, t, &c, &mask);
        beta_householder(jb->X, jb->n, m, jb->ldx, c, mask, work, w);
        for (int v = 0; v < m; ++v) w[v] = -w[v];
        w[c] = 1.0;
        for (int i = 0; i < m; ++i)
            for (int j = 0; j < m; ++j) jb->A[i * m + j] += g * w[i] * w[j];
    }
    free(work);
    return NULL;
}

/* A = sum_{c,S} gbar(c,S) w w^T over the whole table (gbar in table order), then
 * dX = 2 X A (n x m, row stride m).  Threads reduce their partial A in a fixed order. */
int or_grad_from_gbar(const double *X, int64_t n, int m, int64_t ldx, const double *gbar,
                      double *A_out, double *dX, int nthreads) {
    if (!X || !gbar || n < 1 || m < 1 || m > 40 || ldx < m) return -1;
    const int64_t N = or_num_families(m);
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 64) nthreads = 64;
    gjob_t *jobs = (gjob_t *)calloc((size_t)nthreads, sizeof(gjob_t));
    pthread_t th[64];
    if (!jobs) return -3;
    for (int t = 0; t < nthreads; ++t) {
        jobs[t].X = X;
        jobs[t].n = n;
        jobs[t].m = m;
        jobs[t].ldx = ldx;
        jobs[t].gbar = gbar;
        jobs[t].begin = N * t / nthreads;
        jobs[t].end = N * (t + 1) / nthreads;
        if (nthreads > 1) {
            if (pthread_create(&th[t], NULL, run_gjob, &jobs[t]) != 0) {
                run_gjob(&jobs[t]);
                th[t] = 0;
            }
        } else {
            run_gjob(&jobs[t]);
        }
    }
    double A[64 * 64];
    for (int i = 0; i < m * m; ++i) A[i] = 0.0;
    int st = 0;
    for (int t = 0; t < nthreads; ++t) {
        if (nthreads > 1 && th[t]) pthread_join(th[t], NULL);
        if (jobs[t].status) st = jobs[t].status;
        for (int i = 0; i < m * m; ++i) A[i] += jobs[t].A[i];
    }
    free(jobs);
    if (A_out)
        for (int i = 0; i < m * m; ++i) A_out[i] = A[i];
    if (dX) {
        for (int64_t r = 0; r < n; ++r)
            for (int j = 0; j < m; ++j) {
                double acc = 0.0;
                for (int i = 0; i < m; ++i) acc += X[r * ldx + i] * A[i * m + j];
                dX[r * m + j] = 2.0 * acc;
            }
    }
    return st;
}
