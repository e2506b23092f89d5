/*
 * ks_testing.h -- test hooks of libks.so.  They expose single stages of the
 * solve (the matrix-core GEMM, the Cholesky factorisation, the tridiagonal
 * divide-and-conquer eigensolver and the raw layout of one MFMA instruction)
 * so that the GPU tests can check each stage against the oracle in isolation.
 * Same conventions as ks.h: row-major, device pointers owned by the caller,
 * synchronous on the given stream (the hooks synchronize before returning).
 * They return a ks_status value (0 on success).
 */
#ifndef KS_TESTING_H
#define KS_TESTING_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* C = alpha op(A) op(B) + beta C; dtype 0 real / 1 complex (FP64), 2 real /
 * 3 complex (FP32 on the FP32 matrix cores, FP32 accumulation); op 0 = N, 1 = T,
 * 2 = conjugate transpose; lower != 0 writes only the lower triangle of C. */
int32_t ks_test_gemm(int32_t dtype, int32_t opa, int32_t opb, int32_t m, int32_t n, int32_t k,
                     double alpha, const void* A, int32_t lda, const void* B, int32_t ldb, double beta,
                     void* C, int32_t ldc, int32_t lower, void* stream);

/* In-place Cholesky of the n x n lower triangle of A (upper left untouched)
 * and, if Linv is not NULL, the inverse factor into Linv (n x n, row stride n,
 * zeros above the diagonal); *info = failing 1-based column or 0. */
int32_t ks_test_potrf(int32_t dtype, int32_t n, void* A, int32_t lda, void* Linv, int32_t* info,
                      void* stream);

/* Eigen-decomposition of the symmetric tridiagonal (d[n], e[n-1]) by divide
 * and conquer: lam[n] ascending, Z[n][n] eigenvectors as columns. */
int32_t ks_test_stedc(int32_t n, const double* d, const double* e, double* lam, double* Z,
                      int32_t* info, void* stream);

/* Householder tridiagonalisation of the n x n Hermitian matrix A (full storage,
 * overwritten): d[n], e[n-1] of T with A = Q T Q^H, then Q X for the n x ncols
 * real matrix X (row stride n) into Y (dtype, row stride ncols). */
int32_t ks_test_hetrd(int32_t dtype, int32_t n, void* A, double* d, double* e, const double* X,
                      int32_t ncols, void* Y, void* stream);

/* The same with the two-stage reduction (KS_PLAN_TWOSTAGE): A = Q T Q^H with
 * Q = Q1 Q2 (panel reflectors, then bulge-chasing reflectors), Y = Q X. */
int32_t ks_test_hetrd2(int32_t dtype, int32_t n, void* A, double* d, double* e, const double* X,
                       int32_t ncols, void* Y, void* stream);

/* The first stage alone: A (full storage, overwritten) becomes B = Q1^H A Q1,
 * Hermitian with half-bandwidth 32 (its lower triangle is written: the band,
 * zeros below it; the upper triangle is left undefined), and Y = Q1 X for the
 * n x ncols real X (row stride n), Y of the dtype with row stride ncols. */
int32_t ks_test_he2hb(int32_t dtype, int32_t n, void* A, const double* X, int32_t ncols, void* Y, void* stream);

/* Iteration caps of the divide-and-conquer eigensolver for every later call in
 * this process: Jacobi sweeps of the leaves (default 40) and iterations of the
 * secular-equation solver (default 120); a value <= 0 restores the default.
 * A step that reaches its cap records KS_ERR_NO_CONVERGENCE in the plan's info
 * word and finishes normally (its outputs are then undefined).  Host-only; it
 * lets a test drive that failure path with ordinary inputs. */
int32_t ks_test_set_iteration_caps(int32_t leaf_sweeps, int32_t secular_iters);

/* One v_mfma_f64_16x16x4_f64 where lane l feeds A[l%16][l/16] and B[l/16][l%16]
 * with A[i][0] = 100 i, A[i][1] = 1, B[0][j] = 1, B[1][j] = j (other k zero), so
 * D[i][j] = 100 i + j; out[lane * 4 + r] = accumulator register r of each lane. */
int32_t ks_test_mfma_layout(double* out, void* stream);

/* The same probe for one v_mfma_f32_16x16x4_f32 (FP32 values, D[i][j] = 100 i + j). */
int32_t ks_test_mfma_layout32(float* out, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* KS_TESTING_H */
