/* kf_oracle.h -- plain FP64 CPU reference for the fused BLAS-1/BLAS-2 sequences.
 *
 * TEST INFRASTRUCTURE ONLY. This library is the yardstick the HIP path is
 * checked against; only the test-suite, the smoke check and the benchmark's
 * CPU-baseline leg may load it. It shares no code with the GPU library.
 *
 * Every routine computes the plain mathematical definition in double precision,
 * one loop per definition, with no blocking, fusion or reordering. Matrices are
 * row-major with a leading dimension `ld` (element (i, j) at a[i*ld + j]).
 * Stored operands are float (the exact values the GPU sees); every product and
 * sum is formed in double, which is exact for the products of two floats.
 */
#ifndef KF_ORACLE_H
#define KF_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Threads of the library: 1 in the one-thread build; the OpenMP build (the
 * same source with -fopenmp, used to time the oracle on all host cores)
 * reports and sets its thread count. */
int    kfo_threads(void);
void   kfo_set_threads(int n);

/* ---- elementary calls on double operands (Section 3.3: BLAS as map/reduce) */
void   kfo_f2d(int64_t n, const float* src, double* dst);
void   kfo_mat_f2d(int64_t m, int64_t n, int64_t ld, const float* a, double* dst);
void   kfo_scal(int64_t n, double alpha, const double* x, double* y);            /* y = a x        */
void   kfo_axpy(int64_t n, double alpha, const double* x, const double* y,
                double* z);                                                      /* z = a x + y    */
double kfo_dot(int64_t n, const double* x, const double* y);                     /* x^T y          */
void   kfo_gemv(int64_t m, int64_t n, double alpha, const double* a, const double* x,
                double beta, const double* y0, double* y);                       /* a A x + b y0   */
void   kfo_gemtv(int64_t m, int64_t n, double alpha, const double* a, const double* x,
                 double beta, const double* y0, double* y);                      /* a A^T x + b y0 */
void   kfo_ger(int64_t m, int64_t n, double alpha, const double* a, const double* u,
               const double* v, double* b);                                      /* A + a u v^T    */

/* ---- Table 1 sequences on float storage (A is m x n, row-major, leading dim ld) */
void kfo_axpydot(int64_t n, double alpha, const float* w, const float* v, const float* u,
                 double* z, double* r);
void kfo_waxpby(int64_t n, double alpha, const float* x, double beta, const float* y,
                double* w);
void kfo_bicgk(int64_t m, int64_t n, int64_t ld, const float* a, const float* p,
               const float* r, double* q, double* s);
void kfo_atax(int64_t m, int64_t n, int64_t ld, const float* a, const float* x, double* y);
void kfo_gesummv(int64_t m, int64_t n, int64_t lda, const float* a, int64_t ldb,
                 const float* b, double alpha, double beta, const float* x, double* y);
/* bmat may be NULL (then B is not returned); it is m x n with leading dim n. */
void kfo_gemver(int64_t m, int64_t n, int64_t ld, const float* a, const float* u1,
                const float* v1, const float* u2, const float* v2, double alpha,
                double beta, const float* y, const float* z, double* bmat, double* x,
                double* w);

/* ---- selected outputs, for checks at full size where the whole result is
 * not wanted: rows idx[0..cnt) of A x, and columns idx[..] of A^T x. */
void kfo_gemv_rows(int64_t m, int64_t n, int64_t ld, const float* a, const double* x,
                   const int64_t* idx, int64_t cnt, double* out);
void kfo_gemtv_cols(int64_t m, int64_t n, int64_t ld, const float* a, const double* x,
                    const int64_t* idx, int64_t cnt, double* out);

#ifdef __cplusplus
}
#endif
#endif
