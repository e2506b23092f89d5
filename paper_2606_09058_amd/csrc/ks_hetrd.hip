// ks_hetrd.hip -- blocked Householder tridiagonalisation A = Q T Q^H of the
// reduced Hermitian matrix (the "diagonalize H'" step, Part 2-4 of the
// collinear flow in Sec. 3.1 and Part 3-5 in Sec. 3.2, whose first half the
// paper identifies as bandwidth-bound matrix-vector work in Sec. 6).
//
// Lower-triangle convention, full Hermitian storage (row-major; both
// triangles are maintained, so a column below the diagonal is read as the
// conjugate of the contiguous row).  Panels of NB columns: for each column k
// of a panel
//   K1 update column k with the panel's previous reflectors (V, W),
//   K2 form the reflector H_k = I - tau v v^H with H_k^H x = beta e_1
//      (beta real, so the off-diagonal of T is real for complex input),
//   K3 y = A_trail v (one pass over the trailing matrix, the memory-bound
//      part) plus the partial products W^H v, V^H v,
//   K4 w = tau (y - V (W^H v) - W (V^H v)) and the partial w^H v,
//   K5 w += alpha v with alpha = -tau (w^H v) / 2;
// after the panel the trailing matrix takes the rank-2NB update
// A -= V W^H + W V^H as one MFMA GEMM with K = 2 NB.
// All reductions are fixed-order (deterministic), no floating-point atomics.
#include "ks_internal.hpp"

namespace ks {

constexpr int HROWS = 16;  // rows per workgroup of the trailing matrix-vector product

template <typename T>
__global__ void fill_zero_kernel(T* p, long n) {
    long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = zero_<T>();
}

template <typename T>
void fill_zero(hipStream_t s, T* p, long n) {
    if (n <= 0) return;
    hipLaunchKernelGGL((fill_zero_kernel<T>), dim3(cdiv(n, 256)), dim3(256), 0, s, p, n);
}

// K1: x[r] = A[r][k] - sum_{i<j} (V[r][i] conj(W[k][i]) + W[r][i] conj(V[k][i])),
// r in [k, n); partial sums of |x[r]|^2 over r >= k+2.
template <typename T>
__global__ __launch_bounds__(256) void colupd_kernel(int n, int k, int j, int nb, const T* A, int lda,
                                                     const T* VW, T* x, double* part) {
    __shared__ T vk[64], wk[64];
    __shared__ double red[4];
    int t = threadIdx.x;
    const int ld2 = 2 * nb;
    if (t < j) {
        vk[t] = VW[(long)k * ld2 + t];
        wk[t] = VW[(long)k * ld2 + nb + t];
    }
    __syncthreads();
    int r = k + blockIdx.x * blockDim.x + t;
    double s2 = 0.0;
    if (r < n) {
        T c = conj_(A[(long)k * lda + r]);
        const T* vr = VW + (long)r * ld2;
        for (int i = 0; i < j; ++i) c -= vr[i] * conj_(wk[i]) + vr[nb + i] * conj_(vk[i]);
        if (r == k) c = from_re<T>(re_(c));
        x[r] = c;
        if (r >= k + 2) s2 = abs2_(c);
    }
    double tot = block_sum(s2, red);
    if (t == 0) part[blockIdx.x] = tot;
}

// K2 (one workgroup): reflector from x[k+1..n), write v (zeros above k+1),
// d[k], e[k], tau[k], and column j of the panel buffers.
template <typename T>
__global__ __launch_bounds__(256) void reflector_kernel(int n, int k, int j, int nb, const T* x,
                                                        const double* part, int nparts, T* v, T* VW,
                                                        T* WV, double* d, double* e, T* tau) {
    __shared__ T sh_s;
    int t = threadIdx.x;
    if (t == 0) {
        double xn2 = 0.0;
        for (int i = 0; i < nparts; ++i) xn2 += part[i];
        T alpha = x[k + 1];
        double ar = re_(alpha), ai = im_(alpha);
        d[k] = re_(x[k]);
        T tv, sc;
        double beta;
        if (xn2 == 0.0 && ai == 0.0) {
            tv = zero_<T>();
            beta = ar;
            sc = zero_<T>();
        } else {
            beta = -copysign(sqrt(ar * ar + ai * ai + xn2), ar);
            if constexpr (is_cplx<T>::value) {
                tv = mk((beta - ar) / beta, -ai / beta);
                sc = inv_(alpha - mk(beta, 0.0));
            } else {
                tv = (beta - ar) / beta;
                sc = 1.0 / (alpha - beta);
            }
        }
        e[k] = beta;
        tau[k] = tv;
        sh_s = sc;
    }
    __syncthreads();
    T sc = sh_s;
    const int ld2 = 2 * nb;
    for (int r = t; r < n; r += blockDim.x) {
        T vr;
        if (r <= k) vr = zero_<T>();
        else if (r == k + 1) vr = from_re<T>(1.0);
        else vr = sc * x[r];
        v[r] = vr;
        VW[(long)r * ld2 + j] = vr;
        WV[(long)r * ld2 + nb + j] = vr;
    }
}

// K3: y[r] = sum_{c > k} A[r][c] v[c] for r in (k, n), HROWS rows per block
// (4 per wave, v read once per column chunk for all 4 rows), and the partial
// P_i = sum_r conj(W[r][i]) v[r], Q_i = sum_r conj(V[r][i]) v[r] (i < j).
template <typename T>
__global__ __launch_bounds__(256) void hemv_kernel(int n, int k, int j, int nb, const T* A, int lda,
                                                   const T* v, const T* VW, T* y, T* partPQ) {
    int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    int r0 = k + 1 + blockIdx.x * HROWS + wave * 4;
    int c0 = k + 1;
    T acc[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[q] = zero_<T>();
    const T* rowp[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) rowp[q] = A + (long)min(r0 + q, n - 1) * lda;
    for (int c = c0 + lane; c < n; c += 64) {
        T vc = v[c];
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[q] += rowp[q][c] * vc;
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        T s = wave_sum(acc[q]);
        if (lane == 0 && r0 + q < n) y[r0 + q] = s;
    }
    // partial panel products over this block's rows
    int t = threadIdx.x;
    if (t < 2 * j) {
        int i = (t < j) ? t : t - j;
        int off = (t < j) ? nb + i : i;  // P uses W (cols nb..), Q uses V
        T s = zero_<T>();
        int rb = k + 1 + blockIdx.x * HROWS;
        for (int q = 0; q < HROWS; ++q) {
            int r = rb + q;
            if (r < n) s += conj_(VW[(long)r * 2 * nb + off]) * v[r];
        }
        partPQ[(long)blockIdx.x * 2 * nb + ((t < j) ? i : nb + i)] = s;
    }
}

// K4: w[r] = tau (y[r] - sum_i V[r][i] P_i - sum_i W[r][i] Q_i), r in (k, n);
// partial sigma = sum conj(w[r]) v[r].
template <typename T>
__global__ __launch_bounds__(256) void correct_kernel(int n, int k, int j, int nb, const T* VW,
                                                      const T* y, const T* partPQ, int nparts,
                                                      const T* v, const T* tau, T* w, double* partS) {
    __shared__ T P[64], Q[64];
    __shared__ double red[4];
    int t = threadIdx.x;
    if (t < 2 * j) {
        int i = (t < j) ? t : t - j;
        int col = (t < j) ? i : nb + i;
        T s = zero_<T>();
        for (int b = 0; b < nparts; ++b) s += partPQ[(long)b * 2 * nb + col];
        if (t < j) P[i] = s;
        else Q[i] = s;
    }
    __syncthreads();
    T tk = tau[k];
    int r = k + 1 + blockIdx.x * blockDim.x + t;
    T sg = zero_<T>();
    if (r < n) {
        const T* vr = VW + (long)r * 2 * nb;
        T yr = y[r];
        for (int i = 0; i < j; ++i) yr -= vr[i] * P[i] + vr[nb + i] * Q[i];
        T wr = tk * yr;
        w[r] = wr;
        sg = conj_(wr) * v[r];
    }
    double sr = block_sum(re_(sg), red);
    double si = block_sum(im_(sg), red);
    if (t == 0) {
        partS[2 * blockIdx.x] = sr;
        partS[2 * blockIdx.x + 1] = si;
    }
}

// K5: w += alpha v, alpha = -tau sigma / 2; store column j of W in both panel buffers.
template <typename T>
__global__ __launch_bounds__(256) void wfinal_kernel(int n, int k, int j, int nb, const double* partS,
                                                     int nparts, const T* v, const T* tau, const T* w,
                                                     T* VW, T* WV) {
    double sr = 0.0, si = 0.0;
    for (int b = 0; b < nparts; ++b) {
        sr += partS[2 * b];
        si += partS[2 * b + 1];
    }
    T sigma;
    if constexpr (is_cplx<T>::value) sigma = mk(sr, si);
    else sigma = sr;
    T alpha = (-0.5) * (tau[k] * sigma);
    int r = k + 1 + blockIdx.x * blockDim.x + threadIdx.x;
    if (r < n) {
        T wr = w[r] + alpha * v[r];
        VW[(long)r * 2 * nb + nb + j] = wr;
        WV[(long)r * 2 * nb + j] = wr;
    }
}

// Copy the panel's reflectors into columns k0 .. k0+jb-1 of Vall (n x n).
template <typename T>
__global__ void store_panel_kernel(int n, int k0, int jb, int nb, const T* VW, T* Vall) {
    long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (long)n * jb) return;
    int r = (int)(e / jb), i = (int)(e % jb);
    Vall[(long)r * n + k0 + i] = VW[(long)r * 2 * nb + i];
}

template <typename T>
__global__ void last_diag_kernel(int n, const T* A, int lda, double* d) {
    d[n - 1] = re_(A[(long)(n - 1) * lda + n - 1]);
}

template <typename T>
void hetrd(hipStream_t s, int n, T* A, int lda, double* d, double* e, T* tau, T* Vall, HetrdWork<T>& w) {
    const int nb = HETRD_NB;
    T* VW = w.VW;
    T* WV = w.WV;
    for (int k0 = 0; k0 < n - 1; k0 += nb) {
        int jb = min(nb, n - 1 - k0);
        fill_zero<T>(s, VW, (long)n * 2 * nb);
        fill_zero<T>(s, WV, (long)n * 2 * nb);
        for (int j = 0; j < jb; ++j) {
            int k = k0 + j;
            int m1 = n - k;  // rows k..n-1
            int nb1 = cdiv(m1, 256);
            hipLaunchKernelGGL((colupd_kernel<T>), dim3(nb1), dim3(256), 0, s, n, k, j, nb, A, lda, VW,
                               w.x, w.part1);
            hipLaunchKernelGGL((reflector_kernel<T>), dim3(1), dim3(256), 0, s, n, k, j, nb, w.x,
                               w.part1, nb1, w.v, VW, WV, d, e, tau);
            int m = n - k - 1;
            int nb3 = cdiv(m, HROWS);
            bool smp = w.prof && w.prof->sample();
            hipEvent_t e0 = smp ? w.prof->begin() : nullptr;
            hipLaunchKernelGGL((hemv_kernel<T>), dim3(nb3), dim3(256), 0, s, n, k, j, nb, A, lda, w.v, VW,
                               w.y, w.partPQ);
            // algorithmic bytes of a Hermitian matrix-vector product: the lower triangle once
            if (smp) w.prof->end(PROF_HEMV, e0, (double)sizeof(T) * m * (m + 1) / 2.0);
            int nb4 = cdiv(m, 256);
            hipLaunchKernelGGL((correct_kernel<T>), dim3(nb4), dim3(256), 0, s, n, k, j, nb, VW, w.y,
                               w.partPQ, nb3, w.v, tau, w.w, w.partS);
            hipLaunchKernelGGL((wfinal_kernel<T>), dim3(nb4), dim3(256), 0, s, n, k, j, nb, w.partS, nb4,
                               w.v, tau, w.w, VW, WV);
        }
        long tot = (long)n * jb;
        hipLaunchKernelGGL((store_panel_kernel<T>), dim3(cdiv(tot, 256)), dim3(256), 0, s, n, k0, jb, nb,
                           VW, Vall);
        int t0 = k0 + jb;
        if (t0 < n) {
            int mt = n - t0;
            gemm<T>(s, OP_N, OP_C, mt, mt, 2 * nb, -1.0, VW + (long)t0 * 2 * nb, 2 * nb, 0,
                    WV + (long)t0 * 2 * nb, 2 * nb, 0, 1.0, A + (long)t0 * lda + t0, lda, 0, 1);
        }
    }
    hipLaunchKernelGGL((last_diag_kernel<T>), dim3(1), dim3(1), 0, s, n, A, lda, d);
}

template void hetrd<double>(hipStream_t, int, double*, int, double*, double*, double*, double*,
                            HetrdWork<double>&);
template void hetrd<cplx>(hipStream_t, int, cplx*, int, double*, double*, cplx*, cplx*,
                          HetrdWork<cplx>&);
template void fill_zero<double>(hipStream_t, double*, long);
template void fill_zero<cplx>(hipStream_t, cplx*, long);
template void fill_zero<int>(hipStream_t, int*, long);

}  // namespace ks
