// ks_backtr.hip -- back-transform of the tridiagonal eigenvectors,
// C = (I (x) L)^-H Q Z (Part 2-5 / Part 3-6 of the paper's flows, with the
// Cholesky factor in place of the Loewdin V), and the density build with
// Fermi-Dirac occupations (Parts 3-4 of Sec. 3.1, Parts 4-5 of Sec. 3.2).
//
// Q = H_0 H_1 ... H_{n-2} is applied in blocks of BT reflectors in compact-WY
// form, H_b ... H_{b+BT-1} = I - V T V^H (T upper triangular, built once per
// set of reflectors from G = V^H V and tau), so each block is three MFMA GEMMs:
// W1 = V^H X, W2 = T W1 (T^H W1 for Q^H), X -= V W2.  A batch of matrices of one
// order shares every launch (GEMM batch index, or blockIdx.y / z selecting the
// matrix).
#include "ks_internal.hpp"

namespace ks {

// X (n x ncols, ld ldx, type T) = Z[:, c0 : c0 + ncols] (real).
template <typename T>
__global__ void load_z_kernel(int n, int ncols, const double* Z, int c0, T* X, int ldx, long sX) {
    Z += (long)blockIdx.y * n * n;
    X += blockIdx.y * sX;
    long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (long)n * ncols) return;
    int r = (int)(e / ncols), c = (int)(e % ncols);
    X[(long)r * ldx + c] = from_re<T>(Z[(long)r * n + c0 + c]);
}

// The triangular factors of the BACKTR_SUB-reflector sub-blocks ("quarters"
// of a 256-reflector block) of every block at once (blockIdx.x = block x
// sub-blocks per block + sub-block, blockIdx.y = matrix): T_q solves
// (diag(1/tau) + striu(G_qq)) T_q = I for the quarter's reflectors, by back
// substitution on the identity, column c by thread c.  G_b (= V_b^H V_b) and
// T_b share storage (leading dimension BT): each quarter reads its diagonal
// block of G into LDS before writing T_q over it, and zeroes the blocks to its
// left (T_b is upper triangular); the blocks above the diagonal still hold
// V_p^H V_q for the coupling terms.
constexpr int TF_Q = BACKTR_SUB;
template <typename T>
__global__ __launch_bounds__(TF_Q) void t_factors_kernel(int n, int B, const T* tau, T* Tall, long sT) {
    constexpr int H = TF_Q;
    const int nq = B / H;
    const int b = blockIdx.x / nq, qd = blockIdx.x % nq, z = blockIdx.y;
    const int b0 = b * B, jb = min(B, n - 1 - b0), o = qd * H, jh = min(H, jb - o);
    if (jh <= 0) return;
    T* Tb = Tall + z * sT + (long)b * B * B;
    T* Th = Tb + (long)o * B + o;
    tau += (long)z * n + b0 + o;
    __shared__ T sg[H][H + 1];
    __shared__ T st[H];
    for (int e = threadIdx.x; e < jh * jh; e += blockDim.x) sg[e / jh][e % jh] = Th[(long)(e / jh) * B + e % jh];
    if ((int)threadIdx.x < jh) st[threadIdx.x] = tau[threadIdx.x];
    __syncthreads();  // the quarter's block of G is in LDS before T_q overwrites it
    const int c = threadIdx.x;
    for (int i = 0; i < jh; ++i)
        for (int cc = c; cc < o; cc += H) Tb[(long)(o + i) * B + cc] = zero_<T>();  // left of the quarter
    if (c >= jh) return;
    T w[H];
#pragma unroll
    for (int i = H - 1; i >= 0; --i) {
        if (i < jh) {
            T acc = (i == c) ? from_re<T>(1.0) : zero_<T>();
#pragma unroll
            for (int l = i + 1; l < H; ++l)
                if (l < jh) acc -= sg[i][l] * w[l];
            w[i] = st[i] * acc;
            Th[(long)i * B + c] = w[i];
        }
    }
}

// The compact-WY factors T_b (jb x jb, row-major with leading dimension BT, at
// Tall + b BT^2 per matrix) of every block of BT reflectors.  The reflector
// matrix is zero above each block, so G_b = V_b^H V_b can run over all n rows:
// one split-K GEMM batched over the full blocks (a ragged last block takes its
// own).  One launch forms the triangular factors of the quarters of every
// block; then pairs of neighbouring factors are joined, quarters into halves
// and halves into the block, by the coupling T_12 = -T_1 (V_1^H V_2) T_2 (the
// product of two compact-WY forms), two batched GEMMs per pair position.
template <typename T>
void backtransform_prepare(hipStream_t s, int n, int batch, const T* Vall, const T* tau, BacktrWork<T>& w) {
    const int bt = w.bt;
    const int nref = n - 1;
    if (nref <= 0) return;
    const int nblk = cdiv(nref, bt), nfull = nref / bt;
    const long sV = (long)n * n, bb = (long)bt * bt;
    for (int z = 0; z < batch; ++z) {
        const T* V = Vall + z * sV;
        // G_b is staged where T_b goes
        T* Gz = w.Tall + z * w.sTall;
        if (nfull > 0)
            gemm_splitk<T>(s, OP_C, OP_N, bt, bt, n, 1.0, V, n, V, n, 0.0, Gz, bt, w.P, w.pelems, nfull, bt, bt, bb);
        if (nblk > nfull) {
            const int b0 = nfull * bt, jb = nref - b0;
            gemm_splitk<T>(s, OP_C, OP_N, jb, jb, n, 1.0, V + b0, n, V + b0, n, 0.0, Gz + (long)nfull * bb, bt,
                           w.P, w.pelems);
        }
    }
    hipLaunchKernelGGL((t_factors_kernel<T>), dim3((bt / TF_Q) * nblk, batch), dim3(TF_Q), 0, s, n, bt, tau, w.Tall,
                       w.sTall);
    // join pairs: Y = G_12 T_2 (in W1), then T_12 = -T_1 Y over G_12
    const int jl = nref - nfull * bt;  // order of a ragged last block (0 if none)
    for (int z = 0; z < batch; ++z) {
        T* Tz = w.Tall + z * w.sTall;
        for (int hb = TF_Q; hb < bt; hb *= 2) {
            for (int po = 0; po < bt; po += 2 * hb) {
                T* T1 = Tz + (long)po * bt + po;
                T* G12 = T1 + hb;
                T* T2 = T1 + (long)hb * bt + hb;
                if (nfull > 0) {
                    gemm<T>(s, OP_N, OP_N, hb, hb, hb, 1.0, G12, bt, bb, T2, bt, bb, 0.0, w.W1, hb, (long)hb * hb,
                            nfull);
                    gemm<T>(s, OP_N, OP_N, hb, hb, hb, -1.0, T1, bt, bb, w.W1, hb, (long)hb * hb, 0.0, G12, bt, bb,
                            nfull);
                }
                const int h2 = std::min(hb, jl - po - hb);  // the ragged block's second factor of this pair
                if (nblk > nfull && h2 > 0) {
                    const long lo = (long)nfull * bb;
                    gemm<T>(s, OP_N, OP_N, hb, h2, h2, 1.0, G12 + lo, bt, 0, T2 + lo, bt, 0, 0.0, w.W1, h2, 0, 1);
                    gemm<T>(s, OP_N, OP_N, hb, h2, hb, -1.0, T1 + lo, bt, 0, w.W1, h2, 0, 0.0, G12 + lo, bt, 0, 1);
                }
            }
        }
    }
}

template <typename T>
void backtransform_q(hipStream_t s, int n, int batch, const T* Vall, int ncols, T* X, int ldx, long sX,
                     BacktrWork<T>& w, bool adjoint) {
    const int bt = w.bt;
    const int B = batch;
    const long sV = (long)n * n;
    int nref = n - 1;
    if (nref <= 0 || ncols <= 0) return;
    int nblk = cdiv(nref, bt);
    // Q X applies the blocks last to first; Q^H X = (H_{n-2}^H ... H_0^H) X applies them first to last
    for (int q = 0; q < nblk; ++q) {
        const int b = adjoint ? q : nblk - 1 - q;
        int b0 = b * bt;
        int jb = min(bt, nref - b0);
        int m = n - b0 - 1;
        const T* Vb = Vall + (long)(b0 + 1) * n + b0;
        const T* Tb = w.Tall + (long)b * bt * bt;
        T* Xb = X + (long)(b0 + 1) * ldx;
        gemm_splitk<T>(s, OP_C, OP_N, jb, ncols, m, 1.0, Vb, n, Xb, ldx, 0.0, w.W1, ncols, w.P, w.pelems, B, sV,
                       sX, (long)jb * ncols);
        gemm<T>(s, adjoint ? OP_C : OP_N, OP_N, jb, ncols, jb, 1.0, Tb, bt, w.sTall, w.W1, ncols, (long)jb * ncols,
                0.0, w.W2, ncols, (long)jb * ncols, B);
        gemm<T>(s, OP_N, OP_N, m, ncols, jb, -1.0, Vb, n, sV, w.W2, ncols, (long)jb * ncols, 1.0, Xb, ldx, sX, B);
    }
}

template <typename T>
void load_z(hipStream_t s, int n, int batch, int ncols, const double* Z, int c0, T* X, int ldx, long sX) {
    long tot = (long)n * ncols;
    hipLaunchKernelGGL((load_z_kernel<T>), dim3(cdiv(tot, 256), batch), dim3(256), 0, s, n, ncols, Z, c0, X, ldx,
                       sX);
}

// ---------------------------------------------------------------- Fermi level
__device__ inline double fermi_F(double x) {
    if (x > 0.0) {
        double e = exp(-x);
        return e / (1.0 + e);
    }
    return 1.0 / (1.0 + exp(x));
}

// One workgroup: mu by bisection on sum_k w_k sum_i g F((eps_ik - mu)/kT) = ne over
// [min eps - 50 kT, max eps + 50 kT] until hi - lo <= 1e-14 max(1, |mu|) (at most
// 200 halvings), mu = midpoint; then occ, E_band and the window check.
__global__ __launch_bounds__(1024) void fermi_kernel(int batch, int order, const double* eps,
                                                     KWeights kw, double g, double ne, double kT,
                                                     int il, int iu, double* occ, double* mu_out,
                                                     double* eband_out, int* kwin, int* info) {
    __shared__ double red[16];
    __shared__ int lastw[16];
    int t = threadIdx.x;
    long tot = (long)batch * order;
    double mn = INFINITY, mx = -INFINITY;
    for (long i = t; i < tot; i += blockDim.x) {
        mn = fmin(mn, eps[i]);
        mx = fmax(mx, eps[i]);
    }
    mn = wave_min(mn);
    mx = wave_max(mx);
    __shared__ double smn[16], smx[16];
    if ((t & 63) == 0) {
        smn[t >> 6] = mn;
        smx[t >> 6] = mx;
    }
    __syncthreads();
    double lo = INFINITY, hi = -INFINITY;
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) {
        lo = fmin(lo, smn[i]);
        hi = fmax(hi, smx[i]);
    }
    lo -= 50.0 * kT;
    hi += 50.0 * kT;
    for (int it = 0; it < 200; ++it) {
        double mid = 0.5 * (lo + hi);
        if (hi - lo <= 1e-14 * fmax(1.0, fabs(mid))) break;
        double cnt = 0.0;
        for (int b = 0; b < batch; ++b) {
            double sb = 0.0;
            for (int i = t; i < order; i += blockDim.x) sb += fermi_F((eps[(long)b * order + i] - mid) / kT);
            cnt += kw.w[b] * g * sb;
        }
        cnt = block_sum(cnt, red);
        if (cnt < ne) lo = mid;
        else hi = mid;
    }
    double mu = 0.5 * (lo + hi);
    double eb = 0.0;
    int last = -1;  // last window column (0-based within [il-1, iu-1]) with f > g 1e-15
    for (int b = 0; b < batch; ++b) {
        double sb = 0.0;
        for (int i = t; i < order; i += blockDim.x) {
            double ei = eps[(long)b * order + i];
            double f = g * fermi_F((ei - mu) / kT);
            occ[(long)b * order + i] = f;
            sb += f * ei;
            bool occd = f > g * 1e-15;
            if ((i < il - 1 || i > iu - 1) && occd) set_info(info, KS_ERR_WINDOW, i + 1);
            if (occd && i >= il - 1 && i <= iu - 1) last = max(last, i - (il - 1));
        }
        eb += kw.w[b] * sb;
    }
    eb = block_sum(eb, red);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) last = max(last, __shfl_xor(last, o, 64));
    if ((t & 63) == 0) lastw[t >> 6] = last;
    __syncthreads();
    if (t == 0) {
        int lw = -1;
        for (int i = 0; i < (int)(blockDim.x >> 6); ++i) lw = max(lw, lastw[i]);
        *kwin = lw + 1;
        *mu_out = mu;
        *eband_out = eb;
    }
}

void fermi(hipStream_t s, int batch, int order, const double* eps, const KWeights& kw, double g,
           double ne, double kT, int il, int iu, double* occ, double* mu, double* eband, int* kwin,
           int* info) {
    hipLaunchKernelGGL(fermi_kernel, dim3(1), dim3(1024), 0, s, batch, order, eps, kw, g, ne, kT, il, iu,
                       occ, mu, eband, kwin, info);
}

#define KS_INST(T)                                                                                 \
    template void backtransform_q<T>(hipStream_t, int, int, const T*, int, T*, int, long,            \
                                     BacktrWork<T>&, bool);                                       \
    template void backtransform_prepare<T>(hipStream_t, int, int, const T*, const T*, BacktrWork<T>&); \
    template void load_z<T>(hipStream_t, int, int, int, const double*, int, T*, int, long);
KS_INST(double)
KS_INST(cplx)
KS_INST(float)
KS_INST(cplx32)
#undef KS_INST

}  // namespace ks
