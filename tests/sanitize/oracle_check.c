/* The CPU oracle under AddressSanitizer and UndefinedBehaviorSanitizer (test
 * infrastructure, built with gcc by tests/test_sanitizers.py).  Runs every entry
 * point on small seeded data and checks the two RSS routes against each other and
 * the gradient's symmetry. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int64_t or_num_families(int m);
int or_score_all(const double *X, int64_t n, int m, int64_t ldx, double *out, int what, int nt);
int or_score_indices(const double *X, int64_t n, int m, int64_t ldx, const int64_t *idx,
                     int64_t count, double *out, int what, int nt);
int or_score_all_gram(const double *X, int64_t n, int m, int64_t ldx, double *out, int what,
                      int nt);
int or_grad_from_gbar(const double *X, int64_t n, int m, int64_t ldx, const double *gbar,
                      double *A_out, double *dX, int nt);
double or_rss(const double *X, int64_t n, int m, int64_t ldx, int child, uint64_t mask);

static uint64_t state = 88172645463325252ull;
static double unif(void) {  /* xorshift64, for test data only */
    state ^= state << 13;
    state ^= state >> 7;
    state ^= state << 17;
    return (double)(state >> 11) * (1.0 / 9007199254740992.0) - 0.5;
}

int main(void) {
    int failures = 0;
    for (int m = 1; m <= 9; ++m) {
        const int64_t n = 3 * m + 5, ldx = m + 2, N = or_num_families(m);
        double *X = malloc(sizeof(double) * (size_t)(n * ldx));
        double *a = malloc(sizeof(double) * (size_t)N), *b = malloc(sizeof(double) * (size_t)N);
        double *g = malloc(sizeof(double) * (size_t)N), *dX = malloc(sizeof(double) * (size_t)(n * m));
        double A[64 * 64];
        int64_t idx[3] = {0, N - 1, N / 2};
        double c3[3];
        for (int64_t i = 0; i < n * ldx; ++i) X[i] = unif();
        for (int what = 0; what < 2; ++what) {
            failures += or_score_all(X, n, m, ldx, a, what, 3) != 0;
            failures += or_score_all_gram(X, n, m, ldx, b, what, 2) != 0;
            for (int64_t i = 0; i < N; ++i) {
                const double d = what ? fabs(a[i] - b[i]) / a[i] : fabs(a[i] - b[i]);
                if (!(d <= 1e-9)) ++failures;
            }
            failures += or_score_indices(X, n, m, ldx, idx, 3, c3, what, 2) != 0;
            for (int t = 0; t < 3; ++t) failures += c3[t] != a[idx[t]];
        }
        failures += fabs(or_rss(X, n, m, ldx, 0, 0) - a[0]) > 1e-12 * a[0];
        for (int64_t i = 0; i < N; ++i) g[i] = unif();
        failures += or_grad_from_gbar(X, n, m, ldx, g, A, dX, 4) != 0;
        for (int i = 0; i < m; ++i)
            for (int j = 0; j < m; ++j) failures += fabs(A[i * m + j] - A[j * m + i]) > 1e-9;
        free(X);
        free(a);
        free(b);
        free(g);
        free(dX);
    }
    printf("oracle checks: %d failures\n", failures);
    return failures ? 1 : 0;
}
