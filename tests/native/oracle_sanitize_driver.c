/* Host sanitizer run of the oracle (test infrastructure): built with gcc
 * -fsanitize=address,undefined together with oracle/rhg_oracle.c by
 * tests/test_oracle_sanitize.py, it calls every whole-graph routine on a
 * small graph, with output buffers sized exactly, so that any out-of-bounds
 * access or undefined behaviour in the oracle ends the run with an error. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int orc_solve_R(double n, double kbar, double gamma, double *alpha_out, double *R_out);
int64_t orc_sample(uint64_t seed, double alpha, double R, int64_t i0, int64_t count, double *r, double *theta,
                   int nthreads);
void orc_degrees(int64_t n, const double *r, const double *theta, double R, int32_t *deg, int nthreads,
                 int64_t stats[2]);
void orc_csr_fill(int64_t n, const double *r, const double *theta, double R, const int64_t *row_ptr, int32_t *col,
                  int nthreads);
int64_t orc_rows(int64_t n, const double *r, const double *theta, double R, const int64_t *rows, int64_t nrows,
                 int64_t *out_ptr, int32_t *out, int64_t cap, int nthreads, int64_t stats[2]);
void orc_pair_scan(int64_t n, const double *r, const double *theta, double R, int32_t *deg, uint64_t fp[2],
                   int nthreads, int64_t stats[2], double *loop_s);
void orc_lr_candidates(uint64_t seed, int64_t j0, int64_t count, int64_t n, int64_t *a, int64_t *b);
int64_t orc_temp_edges(int64_t n, const double *r, const double *theta, double R, double T, uint64_t seed,
                       int64_t *out_i, int64_t *out_j, int64_t cap, int nthreads, int64_t stats[2]);
int64_t orc_temp_rows(int64_t n, const double *r, const double *theta, double R, double T, uint64_t seed,
                      const int64_t *rows, int64_t nrows, int64_t *out_ptr, int32_t *out, int64_t cap,
                      int nthreads, int64_t stats[2]);

#define CHECK(c) do { if (!(c)) { fprintf(stderr, "check failed: %s\n", #c); return 1; } } while (0)

int main(void)
{
    const int64_t n = 1500;
    double alpha, R;
    CHECK(orc_solve_R((double)n, 8.0, 2.4, &alpha, &R) == 0);
    double *r = malloc(n * sizeof(double)), *t = malloc(n * sizeof(double));
    orc_sample(7, alpha, R, 0, n, r, t, 2);
    int32_t *deg = malloc(n * sizeof(int32_t));
    int64_t st[2] = {0, 0};
    orc_degrees(n, r, t, R, deg, 2, st);
    int64_t *rp = malloc((n + 1) * sizeof(int64_t));
    rp[0] = 0;
    for (int64_t i = 0; i < n; ++i) rp[i + 1] = rp[i] + deg[i];
    int32_t *col = malloc((size_t)(rp[n] > 0 ? rp[n] : 1) * sizeof(int32_t));
    orc_csr_fill(n, r, t, R, rp, col, 2);
    int64_t rows[5] = {0, 1, 17, 700, n - 1};
    int64_t optr[6];
    int64_t need = 0;
    for (int a = 0; a < 5; ++a) need += deg[rows[a]];
    int32_t *ocol = malloc((size_t)(need > 0 ? need : 1) * sizeof(int32_t));
    CHECK(orc_rows(n, r, t, R, rows, 5, optr, ocol, need, 2, st) == need);
    for (int a = 0; a < 5; ++a) CHECK(optr[a + 1] - optr[a] == deg[rows[a]]);
    int32_t *deg2 = malloc(n * sizeof(int32_t));
    uint64_t fp[2];
    double loop_s;
    orc_pair_scan(n, r, t, R, deg2, fp, 2, st, &loop_s);
    for (int64_t i = 0; i < n; ++i) CHECK(deg2[i] == deg[i]);
    int64_t la[64], lb[64];
    orc_lr_candidates(3, 0, 64, n, la, lb);
    for (int a = 0; a < 64; ++a) CHECK(0 <= la[a] && la[a] <= lb[a] && lb[a] < n);
    /* temperature: count first with a zero-capacity list, then fill exactly */
    const int64_t m = orc_temp_edges(n, r, t, R, 0.3, 7, NULL, NULL, 0, 2, st);
    int64_t *ei = malloc((size_t)(m > 0 ? m : 1) * sizeof(int64_t)), *ej = malloc((size_t)(m > 0 ? m : 1) * sizeof(int64_t));
    CHECK(orc_temp_edges(n, r, t, R, 0.3, 7, ei, ej, m, 2, st) == m);
    int64_t tptr[6];
    const int64_t tm = orc_temp_rows(n, r, t, R, 0.3, 7, rows, 5, tptr, NULL, 0, 2, st);
    CHECK(tm == -1 || tm == 0);
    int32_t *tcol = malloc((size_t)(tptr[5] > 0 ? tptr[5] : 1) * sizeof(int32_t));
    CHECK(orc_temp_rows(n, r, t, R, 0.3, 7, rows, 5, tptr, tcol, tptr[5], 2, st) == tptr[5]);
    printf("ok edges %lld temperature edges %lld\n", (long long)(rp[n] / 2), (long long)m);
    free(r); free(t); free(deg); free(rp); free(col); free(ocol); free(deg2); free(ei); free(ej); free(tcol);
    return 0;
}
