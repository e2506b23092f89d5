// ks_adjoint.hip -- adjoint of the density matrix rho = C f C^H and of the
// band energy E_band = sum_k w_k sum_i f_i eps_i with respect to H and S.
//
// With all eigenvectors (C^H S_NC C = I), f'_i = -g F(x_i) F(-x_i) / kT,
// x_i = (eps_i - mu)/kT, Gh = (Gbar + Gbar^H)/2 and Gt = C^H Gh C:
//   G1_ij = (f_i - f_j)/(eps_i - eps_j) (G1_ii = f'_i), evaluated through the
//           divided difference of F, stable at (near-)degenerate pairs,
//   G2_ij = (f_i + f_j)/2 + (eps_i + eps_j) G1_ij / 2 (G2_ii = f_i + eps_i f'_i),
//   a_k   = w_k sum_k' sum_i Gt_ii f'_i / sum_k' w_k' sum_i f'_i   (mu coupling),
//   b     = sum w eps f' / sum w f',   w_i = w_k (f_i + (eps_i - b) f'_i),
//   grad_H = C (Gt o G1 - a_k diag f' + ebar diag w) C^H,
//   grad_S = -C (Gt o G2 - a_k diag(f' eps) + ebar diag(w eps)) C^H
// (spinor form: grad_S is the sum of the two diagonal spin blocks).
// These follow from first-order perturbation of H c = eps S c
// (d eps_i = c_i^H (dH - eps_i dS) c_i, dC = C X with
// X_ji = (C^H (dH - eps_i dS) C)_ji / (eps_i - eps_j), X_ii = -(C^H dS C)_ii / 2)
// and of the occupations at fixed electron count (df_i = f'_i (d eps_i - d mu)).
// Six order^3 products run on the matrix cores; the rest is elementwise.
#include "ks_internal.hpp"

namespace ks {

__device__ inline double F_(double x) {
    if (x > 0.0) {
        double e = exp(-x);
        return e / (1.0 + e);
    }
    return 1.0 / (1.0 + exp(x));
}

__device__ inline double sech_(double u) {
    double e = exp(-fabs(u));
    return 2.0 * e / (1.0 + e * e);
}

// (F(x) - F(y)) / (x - y); for |x - y| < 1 through
// F(x) - F(y) = -sinh((x - y)/2) / (2 cosh(x/2) cosh(y/2)).
__device__ inline double Fdd(double x, double y) {
    double dlt = x - y;
    if (fabs(dlt) < 1.0) {
        double h = 0.5 * dlt;
        double shc = (h == 0.0) ? 1.0 : sinh(h) / h;
        return -0.25 * shc * sech_(0.5 * x) * sech_(0.5 * y);
    }
    return (F_(x) - F_(y)) / dlt;
}

template <typename T>
__global__ void herm_half_kernel(int n, const T* G, int ldg, T* Out) {
    long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (long)n * n) return;
    int i = (int)(e / n), j = (int)(e % n);
    Out[e] = 0.5 * (G[(long)i * ldg + j] + conj_(G[(long)j * ldg + i]));
}

template <typename T>
__global__ void diag_re_kernel(int n, const T* A, double* dg) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dg[i] = re_(A[(long)i * n + i]);
}

// scal[0] = sum_k sum_i Gt_ii f'_i / sum_k w_k sum_i f'_i (0 if the
// denominator vanishes), scal[1] = b.
__global__ __launch_bounds__(1024) void adj_reduce_kernel(int batch, int order, const double* eps,
                                                          const double* mu, double kT, double g,
                                                          KWeights kw, const double* dg, int have_g,
                                                          double* scal) {
    __shared__ double red[16];
    double A = 0.0, Z = 0.0, B = 0.0;
    double m = *mu;
    for (int b = 0; b < batch; ++b) {
        double a = 0.0, z = 0.0, bb = 0.0;
        for (int i = threadIdx.x; i < order; i += blockDim.x) {
            double e = eps[(long)b * order + i];
            double x = (e - m) / kT;
            double fp = -g * F_(x) * F_(-x) / kT;
            if (have_g) a += dg[(long)b * order + i] * fp;
            z += fp;
            bb += e * fp;
        }
        A += a;
        Z += kw.w[b] * z;
        B += kw.w[b] * bb;
    }
    A = block_sum(A, red);
    Z = block_sum(Z, red);
    B = block_sum(B, red);
    if (threadIdx.x == 0) {
        scal[0] = (Z != 0.0) ? A / Z : 0.0;
        scal[1] = (Z != 0.0) ? B / Z : 0.0;
    }
}

// P1 = Gt o G1 - a diag f' + ebar diag w ; P2 = Gt o G2 - a diag(f' eps) + ebar diag(w eps).
template <typename T>
__global__ void adj_gamma_kernel(int order, const double* eps, const double* mu, double kT, double g,
                                 double wk, const double* scal, const double* grad_eband, const T* Gt,
                                 int have_g, T* P1, T* P2) {
    long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (long)order * order) return;
    int i = (int)(e / order), j = (int)(e % order);
    double m = *mu;
    double ei = eps[i], ej = eps[j];
    double xi = (ei - m) / kT, xj = (ej - m) / kT;
    double fi = g * F_(xi), fj = g * F_(xj);
    double g1, g2;
    if (i == j) {
        g1 = -g * F_(xi) * F_(-xi) / kT;
        g2 = fi + ei * g1;
    } else {
        g1 = g * Fdd(xi, xj) / kT;
        g2 = 0.5 * (fi + fj) + 0.5 * (ei + ej) * g1;
    }
    T gt = have_g ? Gt[e] : zero_<T>();
    T p1 = gt * g1, p2 = gt * g2;
    if (i == j) {
        double fp = g1;
        double a = wk * scal[0], b = scal[1];
        double eb = grad_eband ? *grad_eband : 0.0;
        double wi = wk * (fi + (ei - b) * fp);
        p1 += from_re<T>(-a * fp + eb * wi);
        p2 += from_re<T>(-a * fp * ei + eb * wi * ei);
    }
    P1[e] = p1;
    P2[e] = p2;
}

template <typename T>
static void gt_for(hipStream_t s, int order, const T* C, int ldc, const T* grad_rho, T* W1, T* W2,
                   T* W3) {
    long tot = (long)order * order;
    hipLaunchKernelGGL((herm_half_kernel<T>), dim3(cdiv(tot, 256)), dim3(256), 0, s, order, grad_rho, ldc,
                       W3);
    gemm<T>(s, OP_N, OP_N, order, order, order, 1.0, W3, order, 0, C, ldc, 0, 0.0, W2, order, 0, 1);
    gemm<T>(s, OP_C, OP_N, order, order, order, 1.0, C, ldc, 0, W2, order, 0, 0.0, W1, order, 0, 1);
}

template <typename T>
void density_backward(hipStream_t s, int n, int nsp, int batch, const double* eps, const T* C, int ldc,
                      const double* mu, double kT, double g, const KWeights& kw, const T* grad_rho,
                      const double* grad_eband, T* grad_H, T* grad_S, int lds, T* W1, T* W2, T* W3,
                      double* scal) {
    int order = n * nsp;
    long mat = (long)order * ldc;
    long tot = (long)order * order;
    double* dg = scal + 2;  // batch * order diagonal of Gt
    int have_g = grad_rho != nullptr;
    if (have_g) {
        for (int b = 0; b < batch; ++b) {
            gt_for<T>(s, order, C + b * mat, ldc, grad_rho + b * mat, W1, W2, W3);
            hipLaunchKernelGGL((diag_re_kernel<T>), dim3(cdiv(order, 256)), dim3(256), 0, s, order, W1,
                               dg + (long)b * order);
        }
    }
    hipLaunchKernelGGL(adj_reduce_kernel, dim3(1), dim3(1024), 0, s, batch, order, eps, mu, kT, g, kw, dg,
                       have_g, scal);
    for (int b = 0; b < batch; ++b) {
        const T* Cb = C + b * mat;
        if (have_g && batch > 1) gt_for<T>(s, order, Cb, ldc, grad_rho + b * mat, W1, W2, W3);
        hipLaunchKernelGGL((adj_gamma_kernel<T>), dim3(cdiv(tot, 256)), dim3(256), 0, s, order,
                           eps + (long)b * order, mu, kT, g, kw.w[b], scal, grad_eband, W1, have_g, W2, W3);
        // grad_H = C P1 C^H
        gemm<T>(s, OP_N, OP_N, order, order, order, 1.0, Cb, ldc, 0, W2, order, 0, 0.0, W1, order, 0, 1);
        gemm<T>(s, OP_N, OP_C, order, order, order, 1.0, W1, order, 0, Cb, ldc, 0, 0.0, grad_H + b * mat,
                ldc, 0, 1);
        // grad_S = -sum over spin blocks of (C P2 C^H)_{blocks}
        gemm<T>(s, OP_N, OP_N, order, order, order, 1.0, Cb, ldc, 0, W3, order, 0, 0.0, W1, order, 0, 1);
        T* gS = grad_S + (long)b * n * lds;
        for (int sp = 0; sp < nsp; ++sp) {
            gemm<T>(s, OP_N, OP_C, n, n, order, -1.0, W1 + (long)sp * n * order, order, 0,
                    Cb + (long)sp * n * ldc, ldc, 0, sp == 0 ? 0.0 : 1.0, gS, lds, 0, 1);
        }
    }
}

template void density_backward<double>(hipStream_t, int, int, int, const double*, const double*, int,
                                       const double*, double, double, const KWeights&, const double*,
                                       const double*, double*, double*, int, double*, double*, double*,
                                       double*);
template void density_backward<cplx>(hipStream_t, int, int, int, const double*, const cplx*, int,
                                     const double*, double, double, const KWeights&, const cplx*,
                                     const double*, cplx*, cplx*, int, cplx*, cplx*, cplx*, double*);

}  // namespace ks
