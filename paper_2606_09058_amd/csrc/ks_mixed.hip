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
//   subspace step       G = X^H A X, B = X^H X (M x M) diagonalised by two
//                       refinement passes in M-space (below), X <- X W.
// This file holds the element kernels; the sequence lives with the plan.
#include "ks_internal.hpp"

namespace ks {

template <typename T>
__device__ inline T mkc_(double re, double im);
template <>
__device__ inline double mkc_<double>(double re, double) { return re; }
template <>
__device__ inline cplx mkc_<cplx>(double re, double im) { return mk(re, im); }

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
// 1 / (lam_k - lam_{c0+j}) for k outside the window [c0, c0+m), 0 inside.  The
// denominator is kept at least dmin in magnitude, dmin derived from the data of
// each matrix: half the gap between the window and the nearest eigenvalue
// outside it (no true denominator is smaller than that gap), but no less than
// 8 u32 max|lam|, the size of the FP32 eigenvalues' own error.
__global__ void correction_scale_kernel(int order, int m, int w, float* P, long sp, const double* lam, long sl,
                                        int c0) {
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
    double gap = INFINITY;
    if (c0 + m < order) gap = lb[c0 + m] - lb[c0 + m - 1];
    if (c0 > 0) gap = fmin(gap, lb[c0] - lb[c0 - 1]);
    const double floor32 = 8.0 * 5.96e-8 * fmax(fabs(lb[0]), fabs(lb[order - 1]));
    const double dmin = fmax(0.5 * gap, floor32);
    double den = lb[k] - lb[c0 + j];
    if (fabs(den) < dmin) den = den < 0.0 ? -dmin : dmin;
    *p = (float)((double)(*p) / den);
}

void correction_scale(hipStream_t s, int batch, int order, int m, int w, float* P, long sp, const double* lam,
                      long sl, int c0) {
    long tot = (long)order * m * w;
    hipLaunchKernelGGL(correction_scale_kernel, dim3(cdiv(tot, 256), batch), dim3(256), 0, s, order, m, w, P, sp,
                       lam, sl, c0);
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

// ---------------------------------------------------------------- subspace refinement
// After the correction sweeps the window vectors X span the wanted invariant
// subspace to FP64 accuracy, but inside it they are still mixed at the FP32
// level.  With G = X^H A X and B = X^H X (M x M, nearly diagonal / identity),
// the window is finished in M-space (Ogita and Aishima's refinement of a
// symmetric eigendecomposition, applied to the subspace): with
// theta_i = Re g_ii / Re b_ii and R = I - B, the correction T = I + E,
//   e_ii = r_ii / 2,
//   e_ij = (g_ij - theta_j b_ij) / (theta_j - theta_i)   for theta's in different clusters,
//   e_ij = r_ij / 2                                        inside a cluster,
// makes X T orthonormal and diagonalises it to second order; G <- T^H G T,
// B <- T^H B T, W <- W T.  Clusters are runs of consecutive theta closer than
// delta (where the first-order formula would divide by a near-zero gap); each
// is then diagonalised exactly by a small Jacobi solve.  Two passes, then
// X <- X W and the window values sorted ascending.

// X = I (M x M, ld M) for every matrix of the batch.
template <typename T>
__global__ void identity_kernel(int M, T* X, long sx) {
    long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (long)M * M) return;
    X[blockIdx.y * sx + e] = (e / M == e % M) ? from_re<T>(1.0) : zero_<T>();
}

// One workgroup per matrix: theta_i = Re g_ii / Re b_ii; the cluster bounds
// cstart_i (first index of i's cluster) and csize_i, clusters being maximal runs
// of consecutive thetas less than delta = max(2e-6 max|theta|, 1e-10) apart.
template <typename T>
__global__ __launch_bounds__(1024) void oa_scan_kernel(int M, const T* G, const T* B, long sMM, double* theta,
                                                       long st, int* cstart, int* csize, long sc) {
    __shared__ double red[16];
    const int z = blockIdx.x, t = threadIdx.x;
    G += z * sMM;
    B += z * sMM;
    theta += z * st;
    cstart += z * sc;
    csize += z * sc;
    double mx = 0.0;
    for (int i = t; i < M; i += 1024) {
        const double th = re_(G[(long)i * M + i]) / re_(B[(long)i * M + i]);
        theta[i] = th;
        mx = fmax(mx, fabs(th));
    }
    mx = wave_max(mx);
    if ((t & 63) == 0) red[t >> 6] = mx;
    __syncthreads();
    double amax = 0.0;
    for (int q = 0; q < 16; ++q) amax = fmax(amax, red[q]);
    const double delta = fmax(2e-6 * amax, 1e-10);
    // contiguous chunks of indices per thread; the start of i's cluster is a
    // prefix maximum of the start indices, the next start after i a suffix minimum
    const int chunk = (M + 1023) / 1024, lo = min(M, t * chunk), hi = min(M, lo + chunk);
    auto starts = [&](int i) { return i == 0 || fabs(theta[i] - theta[i - 1]) >= delta; };
    int last = -1, first = M;
    for (int i = lo; i < hi; ++i)
        if (starts(i)) {
            last = i;
            if (first == M) first = i;
        }
    __shared__ int pre[1024], suf[1024];
    pre[t] = last;
    suf[t] = first;
    __syncthreads();
    if (t == 0) {
        for (int q = 1; q < 1024; ++q) pre[q] = max(pre[q], pre[q - 1]);
        for (int q = 1022; q >= 0; --q) suf[q] = min(suf[q], suf[q + 1]);
    }
    __syncthreads();
    int cur = t > 0 ? pre[t - 1] : -1;
    for (int i = lo; i < hi; ++i) {
        if (starts(i)) cur = i;
        cstart[i] = cur;
    }
    int nxt = t < 1023 ? suf[t + 1] : M;  // first start after this chunk
    for (int i = hi - 1; i >= lo; --i) {
        csize[i] = nxt - cstart[i];
        if (starts(i)) nxt = i;
    }
}

// T = I + E (M x M) from G, B, theta and the clusters.
template <typename T>
__global__ void oa_t_kernel(int M, const T* G, const T* B, long sMM, const double* theta, long st, const int* cstart,
                            long sc, T* Tm) {
    long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (long)M * M) return;
    const long z = blockIdx.y;
    const int i = (int)(e / M), j = (int)(e % M);
    const long o = z * sMM + e;
    T v;
    if (i == j) {
        v = from_re<T>(1.0 + 0.5 * (1.0 - re_(B[o])));
    } else if (cstart[z * sc + i] == cstart[z * sc + j]) {
        v = -0.5 * B[o];
    } else {
        const double ti = theta[z * st + i], tj = theta[z * st + j];
        v = (G[o] - tj * B[o]) * (1.0 / (tj - ti));
    }
    Tm[o] = v;
}

// Exact solve of one cluster (or chunk of CL_MAX of a larger one) per
// workgroup: with Bc = I + D (D ~ 1e-10 after the correction above),
// P = I - D/2 is the inverse Cholesky factor to second order; Jacobi
// (cyclic, round-robin pairs) diagonalises C = P Gc P^H into V; the block
// P^H V goes to rows / columns [i0, i0 + k) of Tm (identity elsewhere).
constexpr int CL_MAX = 64;
template <typename T>
__global__ __launch_bounds__(256) void oa_cluster_kernel(int M, const T* G, const T* B, long sMM, const int* cstart,
                                                         const int* csize, long sc, T* Tm) {
    __shared__ T C[CL_MAX][CL_MAX + 1], V[CL_MAX][CL_MAX + 1];
    __shared__ double cs_[CL_MAX / 2], ph_re[CL_MAX / 2], ph_im[CL_MAX / 2], sn_[CL_MAX / 2];
    __shared__ int pp[CL_MAX / 2], qq[CL_MAX / 2];
    __shared__ double red[4];
    const int i0 = blockIdx.x, z = blockIdx.y, t = threadIdx.x;
    const int c0 = cstart[z * sc + i0], cn = csize[z * sc + i0];
    if (cn < 2 || (i0 - c0) % CL_MAX != 0) return;
    const int k = min(CL_MAX, c0 + cn - i0);
    G += z * sMM;
    B += z * sMM;
    Tm += z * sMM;
    // V = P = I - (Bc - I)/2; C = Gc
    for (int e = t; e < k * k; e += 256) {
        const int a = e / k, b = e % k;
        const T bv = B[(long)(i0 + a) * M + i0 + b];
        V[a][b] = (a == b) ? from_re<T>(1.0 - 0.5 * (re_(bv) - 1.0)) : -0.5 * bv;
        C[a][b] = G[(long)(i0 + a) * M + i0 + b];
    }
    __syncthreads();
    // C <- P C P^H, through Tm's block as scratch-free LDS: first rows (P C), then columns
    {
        T tmp[CL_MAX / 4 + 1];
        // each thread: entries e = t, t + 256, ... of P C (k*k <= 4096 -> 16 per thread)
        int cnt = 0;
        for (int e = t; e < k * k; e += 256, ++cnt) {
            const int a = e / k, b = e % k;
            T acc = zero_<T>();
            for (int l = 0; l < k; ++l) acc += V[a][l] * C[l][b];
            tmp[cnt] = acc;
        }
        __syncthreads();
        cnt = 0;
        for (int e = t; e < k * k; e += 256, ++cnt) C[e / k][e % k] = tmp[cnt];
        __syncthreads();
        cnt = 0;
        for (int e = t; e < k * k; e += 256, ++cnt) {
            const int a = e / k, b = e % k;
            T acc = zero_<T>();
            for (int l = 0; l < k; ++l) acc += C[a][l] * conj_(V[b][l]);
            tmp[cnt] = acc;
        }
        __syncthreads();
        cnt = 0;
        for (int e = t; e < k * k; e += 256, ++cnt) {
            const int a = e / k, b = e % k;
            C[a][b] = tmp[cnt];
        }
        __syncthreads();
    }
    // C Hermitian exactly (diagonal real, lower = conj(upper)); the accumulated
    // rotations start from P^H (so that V ends as P^H V_jacobi)
    for (int e = t; e < k * k; e += 256) {
        const int a = e / k, b = e % k;
        if (a == b) C[a][a] = from_re<T>(re_(C[a][a]));
        else if (a > b) C[a][b] = conj_(C[b][a]);
    }
    __syncthreads();
    {
        T tmp[CL_MAX / 4 + 1];
        int cnt = 0;
        for (int e = t; e < k * k; e += 256, ++cnt) tmp[cnt] = conj_(V[e % k][e / k]);
        __syncthreads();
        cnt = 0;
        for (int e = t; e < k * k; e += 256, ++cnt) V[e / k][e % k] = tmp[cnt];
        __syncthreads();
    }
    const int kk = k + (k & 1);  // players of the round-robin (one idle when k is odd)
    for (int sweep = 0; sweep < 30; ++sweep) {
        double off = 0.0, nrm = 0.0;
        for (int e = t; e < k * k; e += 256) {
            const int a = e / k, b = e % k;
            const double v2 = abs2_(C[a][b]);
            nrm += v2;
            if (a != b) off += v2;
        }
        off = block_sum(off, red);
        nrm = block_sum(nrm, red);
        if (off <= 1e-30 * nrm || off == 0.0) break;
        for (int rd = 0; rd < kk - 1; ++rd) {
            // pairs of this round: position 0 fixed, the others rotate
            if (t < kk / 2) {
                auto player = [&](int pos) { return pos == 0 ? 0 : 1 + (pos - 1 + rd) % (kk - 1); };
                int p = player(t), q = player(kk - 1 - t);
                if (p > q) {
                    const int x = p;
                    p = q;
                    q = x;
                }
                pp[t] = p;
                qq[t] = q;
                double c = 1.0, sn = 0.0, pr = 1.0, pi = 0.0;
                if (q < k) {
                    const T cpq = C[p][q];
                    const double ac = sqrt(abs2_(cpq));
                    if (ac > 0.0) {
                        const double a = re_(C[p][p]), b = re_(C[q][q]);
                        const double zeta = (b - a) / (2.0 * ac);
                        const double tt = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
                        c = 1.0 / sqrt(1.0 + tt * tt);
                        sn = tt * c;
                        pr = re_(cpq) / ac;
                        pi = im_(cpq) / ac;
                    }
                }
                cs_[t] = c;
                sn_[t] = sn;
                ph_re[t] = pr;
                ph_im[t] = pi;
            }
            __syncthreads();
            // columns: col_p' = c col_p - s conj(ph) col_q, col_q' = s col_p + c conj(ph) col_q (C and V)
            for (int e = t; e < (kk / 2) * k; e += 256) {
                const int pr_ = e / k, row = e % k;
                const int p = pp[pr_], q = qq[pr_];
                if (q >= k) continue;
                const double c = cs_[pr_], sn = sn_[pr_];
                const T phc = mkc_<T>(ph_re[pr_], -ph_im[pr_]);
                const T xp = C[row][p], xq = C[row][q];
                C[row][p] = c * xp - sn * (phc * xq);
                C[row][q] = sn * xp + c * (phc * xq);
                const T yp = V[row][p], yq = V[row][q];
                V[row][p] = c * yp - sn * (phc * yq);
                V[row][q] = sn * yp + c * (phc * yq);
            }
            __syncthreads();
            // rows: row_p' = c row_p - s ph row_q, row_q' = s row_p + c ph row_q
            for (int e = t; e < (kk / 2) * k; e += 256) {
                const int pr_ = e / k, col = e % k;
                const int p = pp[pr_], q = qq[pr_];
                if (q >= k) continue;
                const double c = cs_[pr_], sn = sn_[pr_];
                const T ph = mkc_<T>(ph_re[pr_], ph_im[pr_]);
                const T xp = C[p][col], xq = C[q][col];
                C[p][col] = c * xp - sn * (ph * xq);
                C[q][col] = sn * xp + c * (ph * xq);
            }
            __syncthreads();
        }
    }
    for (int e = t; e < k * k; e += 256) Tm[(long)(i0 + e / k) * M + i0 + e % k] = V[e / k][e % k];
}

// Window values sorted ascending (stable) and the columns of X permuted to
// match: rank_i = #{j : theta_j < theta_i} + #{j < i : theta_j = theta_i};
// eps[c0 + rank_i] = theta_i, Xs[:, rank_i] = X[:, i].
__global__ __launch_bounds__(1024) void oa_rank_kernel(int M, const double* theta, long st, int* rank, long sr,
                                                       double* eps, long se, int c0) {
    const int z = blockIdx.x;
    theta += z * st;
    rank += z * sr;
    for (int i = threadIdx.x; i < M; i += 1024) {
        const double ti = theta[i];
        int r = 0;
        for (int j = 0; j < M; ++j) {
            const double tj = theta[j];
            r += (tj < ti) || (tj == ti && j < i);
        }
        rank[i] = r;
        eps[z * se + c0 + r] = ti;
    }
}

template <typename T>
__global__ void permute_cols_kernel(int rows, int M, const T* X, long sx, const int* rank, long sr, T* Y) {
    long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (long)rows * M) return;
    const long z = blockIdx.y;
    const int r = (int)(e / M), c = (int)(e % M);
    Y[z * sx + (long)r * M + rank[z * sr + c]] = X[z * sx + e];
}

template <typename T>
void subspace_refine(hipStream_t s, int batch, int order, int M, T* X, long sX, T* Y, T* G, T* Bm, T* Tm, T* W,
                     T* Tmp, double* theta, long st, int* cstart, int* csize, int* rank, long sc, double* eps,
                     long se, int c0, int passes) {
    const long sMM = (long)M * M;
    const dim3 gmm(cdiv(sMM, 256), batch);
    // G = X^H (A X) is formed by the caller into G (Y = A X there); B = X^H X
    gemm<T>(s, OP_C, OP_N, M, M, order, 1.0, X, M, sX, X, M, sX, 0.0, Bm, M, sMM, batch);
    hipLaunchKernelGGL((identity_kernel<T>), gmm, dim3(256), 0, s, M, W, sMM);
    auto congruence = [&](const T* Tt) {  // G <- T^H G T, B <- T^H B T, W <- W T
        gemm<T>(s, OP_N, OP_N, M, M, M, 1.0, G, M, sMM, Tt, M, sMM, 0.0, Tmp, M, sMM, batch);
        gemm<T>(s, OP_C, OP_N, M, M, M, 1.0, Tt, M, sMM, Tmp, M, sMM, 0.0, G, M, sMM, batch);
        gemm<T>(s, OP_N, OP_N, M, M, M, 1.0, Bm, M, sMM, Tt, M, sMM, 0.0, Tmp, M, sMM, batch);
        gemm<T>(s, OP_C, OP_N, M, M, M, 1.0, Tt, M, sMM, Tmp, M, sMM, 0.0, Bm, M, sMM, batch);
        gemm<T>(s, OP_N, OP_N, M, M, M, 1.0, W, M, sMM, Tt, M, sMM, 0.0, Tmp, M, sMM, batch);
        std::swap(W, Tmp);  // the product is the new W; the old one is scratch
    };
    for (int it = 0; it < passes; ++it) {
        hipLaunchKernelGGL((oa_scan_kernel<T>), dim3(batch), dim3(1024), 0, s, M, (const T*)G, (const T*)Bm, sMM, theta,
                           st, cstart, csize, sc);
        hipLaunchKernelGGL((oa_t_kernel<T>), gmm, dim3(256), 0, s, M, (const T*)G, (const T*)Bm, sMM,
                           (const double*)theta, st, (const int*)cstart, sc, Tm);
        congruence(Tm);
        hipLaunchKernelGGL((identity_kernel<T>), gmm, dim3(256), 0, s, M, Tm, sMM);
        hipLaunchKernelGGL((oa_cluster_kernel<T>), dim3(M, batch), dim3(256), 0, s, M, (const T*)G, (const T*)Bm, sMM,
                           (const int*)cstart, (const int*)csize, sc, Tm);
        congruence(Tm);
    }
    hipLaunchKernelGGL((oa_scan_kernel<T>), dim3(batch), dim3(1024), 0, s, M, (const T*)G, (const T*)Bm, sMM, theta, st,
                       cstart, csize, sc);
    hipLaunchKernelGGL(oa_rank_kernel, dim3(batch), dim3(1024), 0, s, M, (const double*)theta, st, rank, sc, eps, se,
                       c0);
    // X W, then its columns in ascending order into X
    gemm<T>(s, OP_N, OP_N, order, M, M, 1.0, X, M, sX, W, M, sMM, 0.0, Y, M, sX, batch);
    hipLaunchKernelGGL((permute_cols_kernel<T>), dim3(cdiv((long)order * M, 256), batch), dim3(256), 0, s, order, M,
                       (const T*)Y, sX, (const int*)rank, sc, X);
}

#define KS_INST(T, S)                                                                                       \
    template void convert<T, S>(hipStream_t, int, int, int, const T*, int, long, S*, int, long);            \
    template void convert<S, T>(hipStream_t, int, int, int, const S*, int, long, T*, int, long);            \
    template void residual<T>(hipStream_t, int, int, int, const T*, const T*, long, const double*, long, int, \
                              T*);                                                                          \
    template void sub_widened<T, S>(hipStream_t, int, long, T*, const S*, long);                          \
    template void subspace_refine<T>(hipStream_t, int, int, int, T*, long, T*, T*, T*, T*, T*, T*, double*, long, \
                                     int*, int*, int*, long, double*, long, int, int);
KS_INST(double, float)
KS_INST(cplx, cplx32)
#undef KS_INST

}  // namespace ks
