// ks_testhooks.hip -- single-stage entry points for the GPU tests
// (declared in include/ks_testing.h).
#include "ks_internal.hpp"
#include "../../include/ks_testing.h"

using namespace ks;

typedef double d4 __attribute__((ext_vector_type(4)));

__global__ void mfma_layout_kernel(double* out) {
    int l = threadIdx.x;
    int ii = l % 16, kk = l / 16;
    double a = (kk == 0) ? 100.0 * ii : (kk == 1 ? 1.0 : 0.0);
    double b = (kk == 0) ? 1.0 : (kk == 1 ? (double)ii : 0.0);
    d4 c = {0.0, 0.0, 0.0, 0.0};
    c = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    for (int r = 0; r < 4; ++r) out[l * 4 + r] = c[r];
}

typedef float f4 __attribute__((ext_vector_type(4)));

__global__ void mfma_layout32_kernel(float* out) {
    int l = threadIdx.x;
    int ii = l % 16, kk = l / 16;
    float a = (kk == 0) ? 100.f * ii : (kk == 1 ? 1.f : 0.f);
    float b = (kk == 0) ? 1.f : (kk == 1 ? (float)ii : 0.f);
    f4 c = {0.f, 0.f, 0.f, 0.f};
    c = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    for (int r = 0; r < 4; ++r) out[l * 4 + r] = c[r];
}

static int32_t finish(hipStream_t s) {
    if (hipStreamSynchronize(s) != hipSuccess) return KS_ERR_HIP;
    if (hipGetLastError() != hipSuccess) return KS_ERR_HIP;
    return KS_OK;
}

extern "C" {

int32_t ks_test_mfma_layout(double* out, void* stream) {
    if (!out) return KS_ERR_INVALID_ARG;
    hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(mfma_layout_kernel, dim3(1), dim3(64), 0, s, out);
    return finish(s);
}

int32_t ks_test_mfma_layout32(float* out, void* stream) {
    if (!out) return KS_ERR_INVALID_ARG;
    hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(mfma_layout32_kernel, dim3(1), dim3(64), 0, s, out);
    return finish(s);
}

int32_t ks_test_gemm(int32_t dtype, int32_t opa, int32_t opb, int32_t m, int32_t n, int32_t k,
                     double alpha, const void* A, int32_t lda, const void* B, int32_t ldb, double beta,
                     void* C, int32_t ldc, int32_t lower, void* stream) {
    if (!A || !B || !C || m < 0 || n < 0 || k < 0 || opa < 0 || opa > 2 || opb < 0 || opb > 2)
        return KS_ERR_INVALID_ARG;
    hipStream_t s = (hipStream_t)stream;
    Uplo u = lower ? UPLO_LOWER : UPLO_FULL;
    if (dtype == 1)
        gemm<cplx>(s, (Op)opa, (Op)opb, m, n, k, alpha, (const cplx*)A, lda, 0, (const cplx*)B, ldb, 0,
                   beta, (cplx*)C, ldc, 0, 1, nullptr, 0, u);
    else if (dtype == 2)
        gemm<float>(s, (Op)opa, (Op)opb, m, n, k, alpha, (const float*)A, lda, 0, (const float*)B, ldb, 0,
                    beta, (float*)C, ldc, 0, 1, nullptr, 0, u);
    else if (dtype == 3)
        gemm<cplx32>(s, (Op)opa, (Op)opb, m, n, k, alpha, (const cplx32*)A, lda, 0, (const cplx32*)B, ldb, 0,
                     beta, (cplx32*)C, ldc, 0, 1, nullptr, 0, u);
    else
        gemm<double>(s, (Op)opa, (Op)opb, m, n, k, alpha, (const double*)A, lda, 0, (const double*)B, ldb,
                     0, beta, (double*)C, ldc, 0, 1, nullptr, 0, u);
    return finish(s);
}

int32_t ks_test_potrf(int32_t dtype, int32_t n, void* A, int32_t lda, void* Linv, int32_t* info, void* stream) {
    if (!A || !info || n < 1 || lda < n) return KS_ERR_INVALID_ARG;
    hipStream_t s = (hipStream_t)stream;
    const size_t es = dtype == 1 ? 16 : 8;
    const size_t nn = (size_t)n * n, nw = nn / 4 + 1;
    char* buf = nullptr;
    if (hipMalloc((void**)&buf, 256 + (nn + nw) * es) != hipSuccess) return KS_ERR_ALLOC;
    int* dinfo = (int*)buf;
    void* Li = buf + 256;
    void* work = buf + 256 + nn * es;
    (void)hipMemsetAsync(dinfo, 0, 2 * sizeof(int), s);
    if (dtype == 1)
        potrf_inv<cplx>(s, n, (cplx*)A, lda, 0, (cplx*)Li, n, 0, (cplx*)work, 0, 1, dinfo);
    else
        potrf_inv<double>(s, n, (double*)A, lda, 0, (double*)Li, n, 0, (double*)work, 0, 1, dinfo);
    if (Linv) (void)hipMemcpyAsync(Linv, Li, nn * es, hipMemcpyDeviceToDevice, s);
    int h[2] = {0, 0};
    int32_t st = finish(s);
    (void)hipMemcpy(h, dinfo, sizeof(h), hipMemcpyDeviceToHost);
    (void)hipFree(buf);
    *info = h[0] ? h[1] : 0;
    return st;
}

int32_t ks_test_stedc(int32_t n, const double* d, const double* e, double* lam, double* Z, int32_t* info,
                      void* stream) {
    if (!d || !lam || !Z || !info || n < 1 || (n > 1 && !e)) return KS_ERR_INVALID_ARG;
    ks_plan_desc desc = {n, 1, KS_REAL64, KS_COLLINEAR, KS_FP64, n, n, stream, 0};
    ks_plan* p = nullptr;
    ks_status st = ks_plan_create(&desc, &p);
    if (st != KS_OK) return st;
    // the plan's tree and scratch drive the same stedc the solve uses
    ks_internal_stedc(p, d, e, lam, Z);
    int32_t inf = 0;
    ks_status s2 = ks_plan_get_info(p, &inf);
    *info = (s2 == KS_OK) ? 0 : (inf ? inf : -(int)s2);
    ks_plan_destroy(p);
    return KS_OK;
}

int32_t ks_test_hetrd(int32_t dtype, int32_t n, void* A, double* d, double* e, const double* X,
                      int32_t ncols, void* Y, void* stream) {
    if (!A || !d || !e || !X || !Y || n < 1 || ncols < 1) return KS_ERR_INVALID_ARG;
    ks_plan_desc desc = {n, 1, dtype == 1 ? KS_COMPLEX128 : KS_REAL64, KS_COLLINEAR, KS_FP64, n, n, stream, 0};
    ks_plan* p = nullptr;
    ks_status st = ks_plan_create(&desc, &p);
    if (st != KS_OK) return st;
    ks_internal_hetrd(p, A, d, e, X, ncols, Y);
    int32_t inf = 0;
    ks_status s2 = ks_plan_get_info(p, &inf);
    ks_plan_destroy(p);
    return s2;
}

int32_t ks_test_hetrd2(int32_t dtype, int32_t n, void* A, double* d, double* e, const double* X,
                       int32_t ncols, void* Y, void* stream) {
    if (!A || !d || !e || !X || !Y || n < 1 || ncols < 1) return KS_ERR_INVALID_ARG;
    ks_plan_desc desc = {n, 1, dtype == 1 ? KS_COMPLEX128 : KS_REAL64, KS_COLLINEAR, KS_FP64, n, n, stream,
                         KS_PLAN_TWOSTAGE};
    ks_plan* p = nullptr;
    ks_status st = ks_plan_create(&desc, &p);
    if (st != KS_OK) return st;
    ks_internal_hetrd(p, A, d, e, X, ncols, Y);
    int32_t inf = 0;
    ks_status s2 = ks_plan_get_info(p, &inf);
    ks_plan_destroy(p);
    return s2;
}

int32_t ks_test_he2hb(int32_t dtype, int32_t n, void* A, const double* X, int32_t ncols, void* Y, void* stream) {
    if (!A || !X || !Y || n < 1 || ncols < 1) return KS_ERR_INVALID_ARG;
    ks_plan_desc desc = {n, 1, dtype == 1 ? KS_COMPLEX128 : KS_REAL64, KS_COLLINEAR, KS_FP64, n, n, stream,
                         KS_PLAN_TWOSTAGE};
    ks_plan* p = nullptr;
    ks_status st = ks_plan_create(&desc, &p);
    if (st != KS_OK) return st;
    ks_internal_he2hb(p, A, X, ncols, Y);
    int32_t inf = 0;
    ks_status s2 = ks_plan_get_info(p, &inf);
    ks_plan_destroy(p);
    return s2;
}

int32_t ks_test_set_iteration_caps(int32_t leaf_sweeps, int32_t secular_iters) {
    ks::stedc_set_caps(leaf_sweeps, secular_iters);
    return KS_OK;
}

}  // extern "C"
