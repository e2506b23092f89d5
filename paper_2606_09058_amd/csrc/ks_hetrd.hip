// ks_hetrd.hip -- blocked Householder tridiagonalisation A = Q T Q^H of the
// reduced Hermitian matrix (the "diagonalize H'" step, Part 2-4 of the
// collinear flow in Sec. 3.1 and Part 3-5 in Sec. 3.2, whose first half the
// paper identifies as bandwidth-bound matrix-vector work in Sec. 6).
//
// Lower-triangle convention: only the lower triangle of the trailing matrix is
// read and kept up to date (row-major).  Panels of NB columns; per column k
// (panel column j) three launches:
//   colupd   (grid) finish column j-1 of W (w += alpha v, alpha = -tau w^H v / 2),
//            update column k with the panel's previous reflectors,
//            x = A[:,k] - V W[k,:]^H - W V[k,:]^H, and per-workgroup partial sums
//            of |x|^2, W^H x and V^H x;
//   symv     (grid over 64 x 64 lower tiles) every workgroup reduces those
//            partials and forms the reflector H_k = I - tau v v^H with
//            H_k^H x = beta e_1 (beta real, so T is real for complex input), then
//            the tiles' share of y = A_trail v (the one pass over the trailing
//            matrix, the memory-bound part, each lower tile read once);
//   wcorrect (grid) y from the tile partials, w = tau (y - V (W^H v) - W (V^H v))
//            and partial w^H v.
// After the panel the lower triangle of the trailing matrix takes the rank-2NB
// update A -= V W^H + W V^H as one MFMA GEMM with K = 2 NB.
// The panel buffers are stored transposed (NB columns of length n each) so
// that the per-row corrections read them coalesced, and the GEMM reads them
// as (V W)^T and conj(W V).  All reductions are fixed-order (deterministic).
#include "ks_internal.hpp"

namespace ks {

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

template <typename T>
__device__ inline T make_c(double re, double im);
template <>
__device__ inline double make_c<double>(double re, double) { return re; }
template <>
__device__ inline cplx make_c<cplx>(double re, double im) { return mk(re, im); }

// alpha = -tau sigma / 2 from the per-workgroup partial sigma = w^H v of the
// previous column (every workgroup sums them in the same order).
template <typename T>
__device__ inline T w_alpha(const double* partS, int nS, T tau, double* red) {
    double sr = 0.0, si = 0.0;
    for (int b = threadIdx.x; b < nS; b += blockDim.x) {
        sr += partS[2 * b];
        si += partS[2 * b + 1];
    }
    sr = block_sum(sr, red);
    si = block_sum(si, red);
    return (-0.5) * (tau * make_c<T>(sr, si));
}

// Layout: VWt[i*n + r] = V[r][i] (i < nb), W[r][i-nb] (nb <= i < 2nb);
//         WVc[i*n + r] = conj W[r][i] (i < nb), conj V[r][i-nb] (nb <= i < 2nb).
// One wavefront per 64 rows.  The per-row products of the partial sums go
// through LDS (lane-major, 16 panel columns per pass) and are summed
// column-wise, so there is no long chain of cross-lane reductions.
// Partials per workgroup: [0] |x|^2, [1+i] (W^H x)_i, [1+nb+i] (V^H x)_i.
constexpr int CU_ROWS = 64;
constexpr int CU_PI = 16;
template <typename T>
__global__ __launch_bounds__(64) void colupd_kernel(int n, int k, int j, int nb, const T* A, int lda,
                                                    T* VWt, T* WVc, T* x, const T* wraw,
                                                    const double* partS, int nS, const T* tau,
                                                    T* partA) {
    __shared__ T sv[64], sw[64];
    __shared__ T prod[CU_ROWS][2 * CU_PI + 2];
    __shared__ double red[1];
    int t = threadIdx.x;
    T alpha = zero_<T>();
    if (j > 0) alpha = w_alpha<T>(partS, nS, tau[k - 1], red);
    if (t < j) {
        sv[t] = VWt[(long)t * n + k];
        if (t < j - 1) sw[t] = VWt[(long)(nb + t) * n + k];
        else sw[t] = wraw[k] + alpha * VWt[(long)(j - 1) * n + k];
    }
    __syncthreads();
    int r = k + blockIdx.x * CU_ROWS + t;
    bool in = r < n;
    T wf = zero_<T>();
    T c = zero_<T>();
    if (in) {
        if (j > 0) {
            wf = wraw[r] + alpha * VWt[(long)(j - 1) * n + r];
            VWt[(long)(nb + j - 1) * n + r] = wf;
            WVc[(long)(j - 1) * n + r] = conj_(wf);
        }
        c = A[(long)r * lda + k];  // column k below the diagonal (lower storage)
        T c0 = zero_<T>(), c1 = zero_<T>();
        int i = 0;
        for (; i + 1 < j - 1; i += 2) {
            c0 += VWt[(long)i * n + r] * conj_(sw[i]) + VWt[(long)(nb + i) * n + r] * conj_(sv[i]);
            c1 += VWt[(long)(i + 1) * n + r] * conj_(sw[i + 1]) +
                  VWt[(long)(nb + i + 1) * n + r] * conj_(sv[i + 1]);
        }
        for (; i < j - 1; ++i)
            c0 += VWt[(long)i * n + r] * conj_(sw[i]) + VWt[(long)(nb + i) * n + r] * conj_(sv[i]);
        if (j > 0) c0 += VWt[(long)(j - 1) * n + r] * conj_(sw[j - 1]) + wf * conj_(sv[j - 1]);
        c -= c0 + c1;
        if (r == k) c = from_re<T>(re_(c));
        x[r] = c;
    }
    T xe = (in && r >= k + 2) ? c : zero_<T>();
    const int ld = 1 + 2 * nb;
    T* out = partA + (long)blockIdx.x * ld;
    int npass = j > 0 ? (j + CU_PI - 1) / CU_PI : 1;
    for (int ps = 0; ps < npass; ++ps) {
        int base = ps * CU_PI;
        if (ps == 0) prod[t][2 * CU_PI] = from_re<T>(abs2_(xe));
#pragma unroll
        for (int q = 0; q < CU_PI; ++q) {
            int i = base + q;
            if (i < j) {
                T vri = in ? VWt[(long)i * n + r] : zero_<T>();
                T wri = (i == j - 1) ? wf : (in ? VWt[(long)(nb + i) * n + r] : zero_<T>());
                prod[t][q] = conj_(wri) * xe;
                prod[t][CU_PI + q] = conj_(vri) * xe;
            }
        }
        __syncthreads();
        bool isP = t < CU_PI && base + t < j;
        bool isQ = t >= CU_PI && t < 2 * CU_PI && base + t - CU_PI < j;
        bool isN = t == 2 * CU_PI && ps == 0;
        if (isP || isQ || isN) {
            T s0 = zero_<T>(), s1 = zero_<T>();
            for (int q = 0; q < CU_ROWS; q += 2) {
                s0 += prod[q][t];
                s1 += prod[q + 1][t];
            }
            int idx = isN ? 0 : (isP ? 1 + base + t : 1 + nb + base + t - CU_PI);
            out[idx] = s0 + s1;
        }
        __syncthreads();
    }
}

// Reflector scalars from the per-workgroup partials of colupd (every workgroup
// reduces them in the same order, so all see identical values).  Only the
// norm |x_{k+2..}|^2 is reduced here; sh[0] = s = 1/(alpha - beta), sh[1] = tau,
// and the writer stores d[k], e[k], tau[k].
template <typename T>
__device__ inline void reflector_scalars(int k, int nb, const T* x, const T* partA, int nA, T* sh,
                                         double* d, double* e, T* taua, bool writer, double* red) {
    int t = threadIdx.x;
    const int ld = 1 + 2 * nb;
    double a = 0.0;
    for (int b = t; b < nA; b += blockDim.x) a += re_(partA[(long)b * ld]);
    double xn2 = block_sum(a, red);
    if (t == 0) {
        T alpha = x[k + 1];
        double ar = re_(alpha), ai = im_(alpha);
        T tv, sc;
        double beta;
        if (xn2 == 0.0 && ai == 0.0) {
            tv = zero_<T>();
            beta = ar;
            sc = zero_<T>();
        } else {
            beta = -copysign(sqrt(ar * ar + ai * ai + xn2), ar);
            tv = make_c<T>((beta - ar) / beta, -ai / beta);
            sc = inv_(alpha - from_re<T>(beta));
        }
        sh[0] = sc;
        sh[1] = tv;
        if (writer) {
            d[k] = re_(x[k]);
            e[k] = beta;
            taua[k] = tv;
        }
    }
    __syncthreads();
}

// The panel corrections p = W^H v and q = V^H v (v_{k+1} = 1, v = s x beyond),
// reduced once per column by one workgroup and stored with s and tau in pq:
// pq[0] = s, pq[1] = tau, pq[2 + i] = p_i, pq[2 + nb + i] = q_i.
template <typename T>
__device__ inline void panel_corrections(int n, int k, int j, int nb, const T* partA, int nA, const T* VWt,
                                         T sc, T tv, T* pq) {
    __shared__ T part4[4][64];
    int t = threadIdx.x, lane = t & 63, g = t >> 6;
    const int ld = 1 + 2 * nb;
    const int nv = 2 * j;
    if (lane < nv) {
        int idx = lane < j ? 1 + lane : 1 + nb + (lane - j);
        T a0 = zero_<T>(), a1 = zero_<T>();
        int b = g;
        for (; b + 4 < nA; b += 8) {
            a0 += partA[(long)b * ld + idx];
            a1 += partA[(long)(b + 4) * ld + idx];
        }
        if (b < nA) a0 += partA[(long)b * ld + idx];
        part4[g][lane] = a0 + a1;
    }
    __syncthreads();
    if (t < nv) {
        T P = (part4[0][t] + part4[1][t]) + (part4[2][t] + part4[3][t]);
        if (t < j) pq[2 + t] = conj_(VWt[(long)(nb + t) * n + k + 1]) + sc * P;
        else pq[2 + nb + (t - j)] = conj_(VWt[(long)(t - j) * n + k + 1]) + sc * P;
    }
    if (t == 0) {
        pq[0] = sc;
        pq[1] = tv;
    }
}

// Trailing Hermitian matrix-vector product y = A_trail v from the LOWER
// triangle only.  The trailing matrix (rows/cols k+1 .. n-1) is cut into
// 64 x 64 tiles; workgroup (c, I) takes tiles J = 8c .. 8c+7 (J <= I) of tile
// row I, staged through LDS 32 rows at a time.  Each tile contributes A_IJ v_J
// to y_I (row sums, accumulated over the workgroup's tiles into prow) and,
// below the diagonal, A_IJ^H v_I to y_J (column sums, one partial per tile in
// pcol); a diagonal tile is expanded from its strict lower part.
constexpr int ST = HETRD_TILE;  // tile edge
constexpr int SCH = HETRD_SCH;  // tiles per workgroup
template <typename T>
struct Stage {
    static constexpr int rows = sizeof(T) == 8 ? 64 : 32;  // tile rows per LDS stage (33 KB)
};

template <typename T>
__global__ __launch_bounds__(256) void symv_tiles_kernel(int n, int k, int j, int nb, const T* A, int lda,
                                                         const T* x, const T* partA, int nA, T* prow,
                                                         T* pcol, int nt, int nch, double* d, double* e,
                                                         T* taua, const T* VWt, T* pq) {
    constexpr int SH = Stage<T>::rows;
    constexpr int NSTG = ST / SH;
    __shared__ T tile[SH][ST + 1];
    __shared__ T vI[ST], vJ[2][ST];
    __shared__ T racc[ST];
    __shared__ T red[8][ST];
    __shared__ T sh[2];
    __shared__ double redd[4];
    int c = blockIdx.x, I = blockIdx.y;
    int J0 = c * SCH;
    if (J0 > I) return;
    int J1 = min(J0 + SCH, I + 1);
    int t = threadIdx.x;
    const int o = k + 1;  // first trailing row / column
    const int col = t & 63, r0 = t >> 6;
    const int nstage = NSTG * (J1 - J0);
    // issue the loads of the first half tile before the scalar prologue
    T ra[SH / 4];
    auto load_stage = [&](int st) {
        int J = J0 + st / NSTG, h = st % NSTG;
        int gc = o + J * ST + col;
#pragma unroll
        for (int q = 0; q < SH / 4; ++q) {
            int rl = r0 + 4 * q;
            int gr = o + I * ST + h * SH + rl;
            T a = zero_<T>();
            if (gr < n && gc < n) a = A[(long)gr * lda + gc];
            if (J == I && col > h * SH + rl) a = zero_<T>();  // diagonal tile: lower part only
            ra[q] = a;
        }
    };
    load_stage(0);
    reflector_scalars<T>(k, nb, x, partA, nA, sh, d, e, taua, c == 0 && I == 0, redd);
    T sc = sh[0];
    if (c == 0 && I == 0) panel_corrections<T>(n, k, j, nb, partA, nA, VWt, sc, sh[1], pq);
    auto vof = [&](int g) -> T {
        if (g >= n) return zero_<T>();
        return (g == o) ? from_re<T>(1.0) : sc * x[g];
    };
    if (t < ST) {
        vI[t] = vof(o + I * ST + t);
        vJ[0][t] = vof(o + J0 * ST + t);
        racc[t] = zero_<T>();
    }
    T cacc = zero_<T>();  // column partial of column t (t < 64) for the current tile
    for (int st = 0; st < nstage; ++st) {
        int J = J0 + st / NSTG, h = st % NSTG;
        __syncthreads();
#pragma unroll
        for (int q = 0; q < SH / 4; ++q) tile[r0 + 4 * q][col] = ra[q];
        if (h == NSTG - 1 && st + 1 < nstage && t < ST) vJ[(J + 1 - J0) & 1][t] = vof(o + (J + 1) * ST + t);
        __syncthreads();
        if (st + 1 < nstage) load_stage(st + 1);  // overlap the next half tile with this one
        const T* vj = vJ[(J - J0) & 1];
        // row sums: thread -> row t % SH, a group of RG columns
        constexpr int RGN = 256 / SH, RG = ST / RGN;
        {
            int rl = t % SH, g = t / SH;
            T sacc = zero_<T>();
#pragma unroll
            for (int q = 0; q < RG; ++q) sacc += tile[rl][g * RG + q] * vj[g * RG + q];
            red[g][rl] = sacc;
        }
        // column sums (strictly below the diagonal): column t%64, rows CG*(t/64) .. +CG-1
        constexpr int CG = SH / 4;
        T cs = zero_<T>();
        {
            int cl = t & 63, g = t >> 6;
#pragma unroll
            for (int q = 0; q < CG; ++q) {
                int rl = g * CG + q;
                T a = tile[rl][cl];
                if (J == I && cl == h * SH + rl) a = zero_<T>();  // diagonal counted once
                cs += conj_(a) * vI[h * SH + rl];
            }
        }
        __syncthreads();
        if (t < SH) {
            T sacc = zero_<T>();
#pragma unroll
            for (int g = 0; g < RGN; ++g) sacc += red[g][t];
            racc[h * SH + t] += sacc;
        }
        __syncthreads();
        red[t >> 6][t & 63] = cs;
        __syncthreads();
        if (t < ST) cacc += (red[0][t] + red[1][t]) + (red[2][t] + red[3][t]);
        if (h == NSTG - 1 && t < ST) {
            if (J == I) racc[t] += cacc;  // A_II^H v_I belongs to y_I as well
            else pcol[((long)J * nt + I) * ST + t] = cacc;
            cacc = zero_<T>();
        }
    }
    __syncthreads();
    if (t < ST) prow[((long)I * nch + c) * ST + t] = racc[t];
}

// y from the tile partials, then w = tau (y - V (W^H v) - W (V^H v)), the new V
// column, and partial w^H v per workgroup.  64 rows per workgroup, four
// threads per row share the partial sums and the correction terms.
constexpr int WC_ROWS = 64;
template <typename T>
__global__ __launch_bounds__(256) void wcorrect_kernel(int n, int k, int j, int nb, const T* x, const T* pq,
                                                       const T* prow, const T* pcol, int nt, int nch,
                                                       T* VWt, T* WVc, T* wraw, double* partS) {
    __shared__ T sp[64], sq[64];
    __shared__ T part[4][WC_ROWS];
    __shared__ double red[4];
    int t = threadIdx.x, lr = t & 63, pp = t >> 6;
    T sc = pq[0], tv = pq[1];
    if (t < j) {
        sp[t] = pq[2 + t];
        sq[t] = pq[2 + nb + t];
    }
    __syncthreads();
    int r = k + 1 + blockIdx.x * WC_ROWS + lr;
    T a0 = zero_<T>(), a1 = zero_<T>();
    if (r < n) {
        int q = r - (k + 1), I = q / ST, i = q % ST;
        int nc = I / SCH + 1;
        for (int c = pp; c < nc; c += 4) a0 += prow[((long)I * nch + c) * ST + i];
        const T* pc = pcol + (long)I * nt * ST + i;
        int I2 = I + 1 + pp;
        for (; I2 + 4 < nt; I2 += 8) {
            a0 += pc[(long)I2 * ST];
            a1 += pc[(long)(I2 + 4) * ST];
        }
        if (I2 < nt) a0 += pc[(long)I2 * ST];
        for (int ii = pp; ii < j; ii += 4)
            a1 -= VWt[(long)ii * n + r] * sp[ii] + VWt[(long)(nb + ii) * n + r] * sq[ii];
    }
    part[pp][lr] = a0 + a1;
    __syncthreads();
    T sig = zero_<T>();
    if (pp == 0 && r < n) {
        T y = (part[0][lr] + part[1][lr]) + (part[2][lr] + part[3][lr]);
        T vr = (r == k + 1) ? from_re<T>(1.0) : sc * x[r];
        T w = tv * y;
        wraw[r] = w;
        sig = conj_(w) * vr;
        VWt[(long)j * n + r] = vr;
        WVc[(long)(nb + j) * n + r] = conj_(vr);
    }
    double sr = block_sum(re_(sig), red);
    double si = block_sum(im_(sig), red);
    if (t == 0) {
        partS[2 * blockIdx.x] = sr;
        partS[2 * blockIdx.x + 1] = si;
    }
}

// Finish the last W column of a panel (w += alpha v) for rows r > k.
template <typename T>
__global__ __launch_bounds__(256) void wfix_kernel(int n, int k, int j, int nb, T* VWt, T* WVc,
                                                   const T* wraw, const double* partS, int nS,
                                                   const T* tau) {
    __shared__ double red[4];
    T alpha = w_alpha<T>(partS, nS, tau[k], red);
    int r = k + 1 + blockIdx.x * blockDim.x + threadIdx.x;
    if (r < n) {
        T wf = wraw[r] + alpha * VWt[(long)j * n + r];
        VWt[(long)(nb + j) * n + r] = wf;
        WVc[(long)j * n + r] = conj_(wf);
    }
}

// Copy the panel's reflectors into columns k0 .. k0+jb-1 of Vall (n x n).
template <typename T>
__global__ void store_panel_kernel(int n, int k0, int jb, const T* VWt, T* Vall) {
    long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (long)n * jb) return;
    int i = (int)(e / n), r = (int)(e % n);
    Vall[(long)r * n + k0 + i] = VWt[(long)i * n + r];
}

template <typename T>
__global__ void last_diag_kernel(int n, const T* A, int lda, double* d) {
    d[n - 1] = re_(A[(long)(n - 1) * lda + n - 1]);
}

template <typename T>
void hetrd(hipStream_t s, int n, T* A, int lda, double* d, double* e, T* tau, T* Vall, HetrdWork<T>& w) {
    const int nb = HETRD_NB;
    T* VWt = w.VW;  // 2nb x n
    T* WVc = w.WV;  // 2nb x n
    for (int k0 = 0; k0 < n - 1; k0 += nb) {
        int jb = min(nb, n - 1 - k0);
        fill_zero<T>(s, VWt, (long)n * 2 * nb);
        fill_zero<T>(s, WVc, (long)n * 2 * nb);
        int nS = 0;
        for (int j = 0; j < jb; ++j) {
            int k = k0 + j;
            int nb1 = cdiv(n - k, CU_ROWS);
            hipLaunchKernelGGL((colupd_kernel<T>), dim3(nb1), dim3(CU_ROWS), 0, s, n, k, j, nb, A, lda, VWt, WVc,
                               w.x, w.w, w.partS, nS, tau, w.partPQ);
            int m = n - k - 1;
            int nt = cdiv(m, ST), nch = cdiv(nt, SCH);
            bool smp = w.prof && w.prof->sample();
            hipEvent_t e0 = smp ? w.prof->begin() : nullptr;
            hipLaunchKernelGGL((symv_tiles_kernel<T>), dim3(nch, nt), dim3(256), 0, s, n, k, j, nb, A, lda,
                               w.x, w.partPQ, nb1, w.prow, w.pcol, nt, nch, d, e, tau, VWt, w.pq);
            // algorithmic bytes of a Hermitian matrix-vector product: the lower triangle once
            if (smp) w.prof->end(PROF_HEMV, e0, (double)sizeof(T) * m * (m + 1) / 2.0);
            int nb4 = cdiv(m, WC_ROWS);
            hipLaunchKernelGGL((wcorrect_kernel<T>), dim3(nb4), dim3(256), 0, s, n, k, j, nb, w.x, w.pq,
                               w.prow, w.pcol, nt, nch, VWt, WVc, w.w, w.partS);
            nS = nb4;
        }
        int kl = k0 + jb - 1;
        hipLaunchKernelGGL((wfix_kernel<T>), dim3(cdiv(n - kl - 1, 256)), dim3(256), 0, s, n, kl, jb - 1, nb,
                           VWt, WVc, w.w, w.partS, nS, tau);
        long tot = (long)n * jb;
        hipLaunchKernelGGL((store_panel_kernel<T>), dim3(cdiv(tot, 256)), dim3(256), 0, s, n, k0, jb, VWt,
                           Vall);
        int t0 = k0 + jb;
        if (t0 < n) {
            int mt = n - t0;
            gemm<T>(s, OP_T, OP_N, mt, mt, 2 * nb, -1.0, VWt + t0, n, 0, WVc + t0, n, 0, 1.0,
                    A + (long)t0 * lda + t0, lda, 0, 1, nullptr, 0, UPLO_LOWER);
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
