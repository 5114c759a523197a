/* kf_oracle.c -- plain FP64 CPU reference (test infrastructure only).
 *
 * Each routine is the textbook definition of the call it names, as the paper
 * uses it: BLAS-1 calls are maps or a map followed by a reduction, BLAS-2
 * calls are a map over rows (or columns) of a reduction over a row (Section
 * 3.3, equations (1) and (2)). The six sequences are those of Table 1, each
 * written as the composition of the elementary calls, with every intermediate
 * kept in double. Nothing here is blocked, fused or reordered.
 *
 * The same source compiled with OpenMP is the all-core build used to time the
 * oracle on the host's cores: the outer loop of each map (over entries, over
 * rows, and for GEMTV over columns) is split among threads, but every output
 * entry is still computed by one thread in the order written here, so the
 * results are bit-identical to the one-thread build. DOT, a single sum, stays
 * serial.
 */
#include "kf_oracle.h"
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#define KFO_PARALLEL_FOR _Pragma("omp parallel for schedule(static)")
#else
#define KFO_PARALLEL_FOR
#endif

/* Threads of the all-core build (1 in the one-thread build). */
int kfo_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void kfo_set_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

void kfo_f2d(int64_t n, const float* src, double* dst) {
    KFO_PARALLEL_FOR
    for (int64_t i = 0; i < n; ++i) dst[i] = (double)src[i];
}

void kfo_mat_f2d(int64_t m, int64_t n, int64_t ld, const float* a, double* dst) {
    KFO_PARALLEL_FOR
    for (int64_t i = 0; i < m; ++i)
        for (int64_t j = 0; j < n; ++j) dst[i * n + j] = (double)a[i * ld + j];
}

/* SCAL: map of x -> alpha x (Section 3.3, BLAS-1 as map). */
void kfo_scal(int64_t n, double alpha, const double* x, double* y) {
    KFO_PARALLEL_FOR
    for (int64_t i = 0; i < n; ++i) y[i] = alpha * x[i];
}

/* AXPY: map of (x, y) -> alpha x + y. */
void kfo_axpy(int64_t n, double alpha, const double* x, const double* y, double* z) {
    KFO_PARALLEL_FOR
    for (int64_t i = 0; i < n; ++i) z[i] = alpha * x[i] + y[i];
}

/* DOT: map of products followed by a sum reduction (Section 3.3). */
double kfo_dot(int64_t n, const double* x, const double* y) {
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i) s += x[i] * y[i];
    return s;
}

/* GEMV: y_i = alpha * sum_j A_ij x_j + beta * y0_i, a map over rows of a
 * reduction over the row (equation (2)). A is m x n, dense row-major. */
void kfo_gemv(int64_t m, int64_t n, double alpha, const double* a, const double* x,
              double beta, const double* y0, double* y) {
    KFO_PARALLEL_FOR
    for (int64_t i = 0; i < m; ++i) {
        double s = 0.0;
        for (int64_t j = 0; j < n; ++j) s += a[i * n + j] * x[j];
        y[i] = alpha * s + (y0 ? beta * y0[i] : 0.0);
    }
}

/* GEMTV: y_j = alpha * sum_i A_ij x_i + beta * y0_j, the same with the matrix
 * viewed as a list of columns (Section 3.3, last paragraph). */
void kfo_gemtv(int64_t m, int64_t n, double alpha, const double* a, const double* x,
               double beta, const double* y0, double* y) {
    KFO_PARALLEL_FOR
    for (int64_t j = 0; j < n; ++j) {
        double s = 0.0;
        for (int64_t i = 0; i < m; ++i) s += a[i * n + j] * x[i];
        y[j] = alpha * s + (y0 ? beta * y0[j] : 0.0);
    }
}

/* GER: B_ij = A_ij + alpha u_i v_j (the rank-1 update of GEMVER, Table 1). */
void kfo_ger(int64_t m, int64_t n, double alpha, const double* a, const double* u,
             const double* v, double* b) {
    KFO_PARALLEL_FOR
    for (int64_t i = 0; i < m; ++i)
        for (int64_t j = 0; j < n; ++j) b[i * n + j] = a[i * n + j] + alpha * u[i] * v[j];
}

static double* dvec(int64_t n) { return (double*)malloc((size_t)(n > 0 ? n : 1) * sizeof(double)); }

static double* dcopy_vec(int64_t n, const float* x) {
    double* d = dvec(n);
    kfo_f2d(n, x, d);
    return d;
}

static double* dcopy_mat(int64_t m, int64_t n, int64_t ld, const float* a) {
    double* d = dvec(m * n);
    kfo_mat_f2d(m, n, ld, a, d);
    return d;
}

/* AXPYDOT (Table 1): z = w - alpha v ; r = z^T u. */
void kfo_axpydot(int64_t n, double alpha, const float* w, const float* v, const float* u,
                 double* z, double* r) {
    double *wd = dcopy_vec(n, w), *vd = dcopy_vec(n, v), *ud = dcopy_vec(n, u);
    kfo_axpy(n, -alpha, vd, wd, z);
    *r = kfo_dot(n, z, ud);
    free(wd); free(vd); free(ud);
}

/* WAXPBY (Table 1): w = alpha x + beta y. */
void kfo_waxpby(int64_t n, double alpha, const float* x, double beta, const float* y,
                double* w) {
    double *xd = dcopy_vec(n, x), *yd = dcopy_vec(n, y), *t = dvec(n);
    kfo_scal(n, beta, yd, t);
    kfo_axpy(n, alpha, xd, t, w);
    free(xd); free(yd); free(t);
}

/* BiCGK (Table 1, Section 4.4): q = A p ; s = A^T r. A is m x n, so p and s
 * have n entries and q and r have m. */
void kfo_bicgk(int64_t m, int64_t n, int64_t ld, const float* a, const float* p,
               const float* r, double* q, double* s) {
    double *ad = dcopy_mat(m, n, ld, a), *pd = dcopy_vec(n, p), *rd = dcopy_vec(m, r);
    kfo_gemv(m, n, 1.0, ad, pd, 0.0, NULL, q);
    kfo_gemtv(m, n, 1.0, ad, rd, 0.0, NULL, s);
    free(ad); free(pd); free(rd);
}

/* ATAX (Table 1): y = A^T (A x), with A x an intermediate. */
void kfo_atax(int64_t m, int64_t n, int64_t ld, const float* a, const float* x, double* y) {
    double *ad = dcopy_mat(m, n, ld, a), *xd = dcopy_vec(n, x), *t = dvec(m);
    kfo_gemv(m, n, 1.0, ad, xd, 0.0, NULL, t);
    kfo_gemtv(m, n, 1.0, ad, t, 0.0, NULL, y);
    free(ad); free(xd); free(t);
}

/* GESUMMV (Table 1): y = alpha A x + beta B x. */
void kfo_gesummv(int64_t m, int64_t n, int64_t lda, const float* a, int64_t ldb,
                 const float* b, double alpha, double beta, const float* x, double* y) {
    double *ad = dcopy_mat(m, n, lda, a), *bd = dcopy_mat(m, n, ldb, b);
    double *xd = dcopy_vec(n, x), *t = dvec(m);
    kfo_gemv(m, n, alpha, ad, xd, 0.0, NULL, t);
    kfo_gemv(m, n, beta, bd, xd, 1.0, t, y);
    free(ad); free(bd); free(xd); free(t);
}

/* GEMVER (Table 1): B = A + u1 v1^T + u2 v2^T ; x = beta B^T y + z ;
 * w = alpha B x. Every stage uses the double B and x of the previous one. */
void kfo_gemver(int64_t m, int64_t n, int64_t ld, const float* a, const float* u1,
                const float* v1, const float* u2, const float* v2, double alpha,
                double beta, const float* y, const float* z, double* bmat, double* x,
                double* w) {
    double *ad = dcopy_mat(m, n, ld, a), *b1 = dvec(m * n);
    double *b = bmat ? bmat : dvec(m * n);
    double *u1d = dcopy_vec(m, u1), *v1d = dcopy_vec(n, v1);
    double *u2d = dcopy_vec(m, u2), *v2d = dcopy_vec(n, v2);
    double *yd = dcopy_vec(m, y), *zd = dcopy_vec(n, z);
    kfo_ger(m, n, 1.0, ad, u1d, v1d, b1);
    kfo_ger(m, n, 1.0, b1, u2d, v2d, b);
    kfo_gemtv(m, n, beta, b, yd, 1.0, zd, x);
    kfo_gemv(m, n, alpha, b, x, 0.0, NULL, w);
    free(ad); free(b1); if (!bmat) free(b);
    free(u1d); free(v1d); free(u2d); free(v2d); free(yd); free(zd);
}

/* Selected rows of A x: out[k] = sum_j A_{idx[k], j} x_j. */
void kfo_gemv_rows(int64_t m, int64_t n, int64_t ld, const float* a, const double* x,
                   const int64_t* idx, int64_t cnt, double* out) {
    (void)m;
    for (int64_t k = 0; k < cnt; ++k) {
        const float* row = a + idx[k] * ld;
        double s = 0.0;
        for (int64_t j = 0; j < n; ++j) s += (double)row[j] * x[j];
        out[k] = s;
    }
}

/* Selected columns of A^T x: out[k] = sum_i A_{i, idx[k]} x_i. */
void kfo_gemtv_cols(int64_t m, int64_t n, int64_t ld, const float* a, const double* x,
                    const int64_t* idx, int64_t cnt, double* out) {
    (void)n;
    for (int64_t k = 0; k < cnt; ++k) {
        double s = 0.0;
        for (int64_t i = 0; i < m; ++i) s += (double)a[i * ld + idx[k]] * x[i];
        out[k] = s;
    }
}
