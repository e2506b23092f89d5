// ks_mixed.hip -- element kernels of the mixed-precision solve.
//
// The mixed form keeps the reduced matrix A = L^-1 H L^-H in FP64 and gives a
// FP32 copy to the tridiagonalisation (trailing matrix stored and updated in
// FP32 on the matrix cores, panel arithmetic in FP64).  The eigenvectors of the
// requested window, back-transformed in FP32, are then refined in FP64:
//   correction sweeps   R = A X - X diag(lam_hat);  X -= Q Z S(Z^T Q^H R),
//                       S scaling row k of window column j by 1/(lam_hat_k - lam_hat_j)
//                       for k outside the window and by 0 inside it (one Newton
//                       step on the components along the other eigenvectors,
//                       with the FP32 decomposition A ~ Q Z diag(lam_hat) Z^T Q^H);
//   Rayleigh-Ritz       G = X^H A X, B = X^H X, G y = theta B y in FP64, X <- X y.
// This file holds the element kernels; the sequence lives with the plan.
#include "ks_internal.hpp"

namespace ks {

// dst (rows x cols, ld ldd, batch stride sd) = src narrowed or widened.
template <typename Src, typename Dst>
__global__ void convert_kernel(int rows, int cols, const Src* src, int lds, long ss, Dst* dst, int ldd, long sd) {
    long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (long)rows * cols) return;
    const int r = (int)(e / cols), c = (int)(e % cols);
    const long b = blockIdx.y;
    const Src v = src[b * ss + (long)r * lds + c];
    if constexpr (sizeof(Dst) < sizeof(Src)) dst[b * sd + (long)r * ldd + c] = narrow(v);
    else dst[b * sd + (long)r * ldd + c] = widen(v);
}

template <typename Src, typename Dst>
void convert(hipStream_t s, int batch, int rows, int cols, const Src* src, int lds, long ss, Dst* dst, int ldd,
             long sd) {
    long tot = (long)rows * cols;
    if (tot <= 0 || batch <= 0) return;
    hipLaunchKernelGGL((convert_kernel<Src, Dst>), dim3(cdiv(tot, 256), batch), dim3(256), 0, s, rows, cols, src,
                       lds, ss, dst, ldd, sd);
}

// R = Y - X diag(lam[c0 + j]) (order x m per matrix, ld m, stride sm; lam stride sl).
template <typename T>
__global__ void residual_kernel(int order, int m, const T* Y, const T* X, long sm, const double* lam, long sl,
                                int c0, T* R) {
    long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (long)order * m) return;
    const long b = blockIdx.y;
    const int j = (int)(e % m);
    const long o = b * sm + e;
    R[o] = Y[o] - lam[b * sl + c0 + j] * X[o];
}

template <typename T>
void residual(hipStream_t s, int batch, int order, int m, const T* Y, const T* X, long sm, const double* lam,
              long sl, int c0, T* R) {
    long tot = (long)order * m;
    hipLaunchKernelGGL((residual_kernel<T>), dim3(cdiv(tot, 256), batch), dim3(256), 0, s, order, m, Y, X, sm,
                       lam, sl, c0, R);
}

// P[k][j] (order x m, FP32, w reals per element: 1 real, 2 complex) scaled by
// 1 / (lam_k - lam_{c0+j}) for k outside the window [c0, c0+m), 0 inside; the
// denominator is kept at least dmin in magnitude.
__global__ void correction_scale_kernel(int order, int m, int w, float* P, long sp, const double* lam, long sl,
                                        int c0, double dmin) {
    long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (long)order * m * w) return;
    const long b = blockIdx.y;
    const int k = (int)(e / ((long)m * w));
    const int j = (int)((e / w) % m);
    const double* lb = lam + b * sl;
    float* p = P + b * sp + e;
    if (k >= c0 && k < c0 + m) {
        *p = 0.f;
        return;
    }
    double den = lb[k] - lb[c0 + j];
    if (fabs(den) < dmin) den = den < 0.0 ? -dmin : dmin;
    *p = (float)((double)(*p) / den);
}

void correction_scale(hipStream_t s, int batch, int order, int m, int w, float* P, long sp, const double* lam,
                      long sl, int c0, double dmin) {
    long tot = (long)order * m * w;
    hipLaunchKernelGGL(correction_scale_kernel, dim3(cdiv(tot, 256), batch), dim3(256), 0, s, order, m, w, P, sp,
                       lam, sl, c0, dmin);
}

// X -= widen(D) elementwise (order x m per matrix, both stride sm).
template <typename T, typename S>
__global__ void sub_widened_kernel(long cnt, T* X, const S* D, long sm) {
    long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= cnt) return;
    const long o = blockIdx.y * sm + e;
    X[o] -= widen(D[o]);
}

template <typename T, typename S>
void sub_widened(hipStream_t s, int batch, long cnt, T* X, const S* D, long sm) {
    hipLaunchKernelGGL((sub_widened_kernel<T, S>), dim3(cdiv(cnt, 256), batch), dim3(256), 0, s, cnt, X, D, sm);
}

// eps[b][c0 + j] = theta[b][j] (the refined window values).
__global__ void put_window_kernel(int m, const double* theta, long st, double* eps, long se, int c0) {
    int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= m) return;
    eps[blockIdx.y * se + c0 + j] = theta[blockIdx.y * st + j];
}

void put_window(hipStream_t s, int batch, int m, const double* theta, long st, double* eps, long se, int c0) {
    hipLaunchKernelGGL(put_window_kernel, dim3(cdiv(m, 256), batch), dim3(256), 0, s, m, theta, st, eps, se, c0);
}

// A device failure recorded by an inner solve becomes the outer plan's (the
// first one wins), and the inner word is cleared.
__global__ void merge_info_kernel(int* inner, int* outer) {
    if (inner[0] != 0 && outer[0] == 0) {
        outer[0] = inner[0];
        outer[1] = inner[1];
    }
    inner[0] = 0;
    inner[1] = 0;
}

void merge_info(hipStream_t s, int* inner, int* outer) {
    hipLaunchKernelGGL(merge_info_kernel, dim3(1), dim3(1), 0, s, inner, outer);
}

#define KS_INST(T, S)                                                                                       \
    template void convert<T, S>(hipStream_t, int, int, int, const T*, int, long, S*, int, long);            \
    template void convert<S, T>(hipStream_t, int, int, int, const S*, int, long, T*, int, long);            \
    template void residual<T>(hipStream_t, int, int, int, const T*, const T*, long, const double*, long, int, \
                              T*);                                                                          \
    template void sub_widened<T, S>(hipStream_t, int, long, T*, const S*, long);
KS_INST(double, float)
KS_INST(cplx, cplx32)
#undef KS_INST

}  // namespace ks
