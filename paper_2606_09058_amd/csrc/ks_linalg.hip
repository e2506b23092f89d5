// ks_linalg.hip -- Cholesky factorisation of S, triangular solves, and the
// reduction A = L^-1 H L^-H of the generalized problem to standard form.
//
// Cholesky and the triangular solves are recursive: the diagonal 32 x 32
// blocks are factored/solved by LDS-resident single-workgroup kernels and
// everything else is an MFMA GEMM (ks_gemm.hip), so the O(n^3) work runs on
// the matrix cores.  The inverse factor L^-1 is formed once per overlap (and
// cached with L), so the reduction and the final back-substitution of every
// solve are plain triangular-aware GEMMs.  The spinor form applies L^-1 to each
// spin block, i.e. (I2 (x) L)^-1 H (I2 (x) L)^-H, by treating the 2n x 2n
// matrix as two n-row (then n-column) blocks: a batch of 2 with a block stride.
#include "ks_internal.hpp"

namespace ks {

constexpr int TB = 32;  // leaf block of the recursive Cholesky / solves

static int split_point(int n) {
    int n1 = ((n / 2 + TB - 1) / TB) * TB;
    if (n1 >= n) n1 = n - TB;
    return n1;
}

// ---------------------------------------------------------------- Cholesky
// Factor the n x n (n <= 32) lower block at A in place; column failures go to
// info with the global 1-based column col0 + j + 1.
template <typename T>
__global__ __launch_bounds__(64) void potrf_leaf_kernel(int n, T* A, int lda, long sa, int col0,
                                                        int* info) {
    __shared__ T L[TB][TB + 1];
    __shared__ int bad;
    A += blockIdx.x * sa;
    int t = threadIdx.x;
    if (t == 0) bad = 0;
    for (int e = t; e < n * n; e += 64) {
        int i = e / n, j = e % n;
        L[i][j] = (j <= i) ? A[(long)i * lda + j] : zero_<T>();
    }
    __syncthreads();
    for (int j = 0; j < n; ++j) {
        if (t == 0) {
            double d = re_(L[j][j]);
            for (int k = 0; k < j; ++k) d -= abs2_(L[j][k]);
            if (!(d > 0.0) || !isfinite(d)) {
                if (!bad) set_info(info, KS_ERR_NOT_POSDEF, col0 + j + 1);
                bad = 1;
                d = 1.0;
            }
            L[j][j] = from_re<T>(sqrt(d));
        }
        __syncthreads();
        double ljj = re_(L[j][j]);
        for (int i = j + 1 + t; i < n; i += 64) {
            T s = L[i][j];
            for (int k = 0; k < j; ++k) s -= L[i][k] * conj_(L[j][k]);
            L[i][j] = s * (1.0 / ljj);
        }
        __syncthreads();
    }
    for (int e = t; e < n * n; e += 64) {
        int i = e / n, j = e % n;
        if (j <= i) A[(long)i * lda + j] = L[i][j];
    }
}

// X L^H = B for X (rows x nl, nl <= 32), in place in B; one thread per row.
template <typename T>
__global__ __launch_bounds__(256) void trsm_right_leaf_kernel(int rows, int nl, const T* L, int ldl,
                                                              long sl, T* B, int ldb, long sb) {
    __shared__ T sL[TB][TB + 1];
    L += blockIdx.y * sl;
    B += blockIdx.y * sb;
    for (int e = threadIdx.x; e < nl * nl; e += blockDim.x) {
        int i = e / nl, j = e % nl;
        sL[i][j] = (j <= i) ? L[(long)i * ldl + j] : zero_<T>();
    }
    __syncthreads();
    int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= rows) return;
    T x[TB];
    T* b = B + (long)r * ldb;
#pragma unroll
    for (int j = 0; j < TB; ++j) {
        if (j < nl) {
            T s = b[j];
#pragma unroll
            for (int i = 0; i < j; ++i) s -= x[i] * conj_(sL[j][i]);
            x[j] = s * (1.0 / re_(sL[j][j]));
        }
    }
#pragma unroll
    for (int j = 0; j < TB; ++j)
        if (j < nl) b[j] = x[j];
}

// L X = B (conjt = 0) or L^H X = B (conjt = 1) for X (nl x cols, nl <= 32),
// in place in B; one thread per column.
template <typename T, int CONJT>
__global__ __launch_bounds__(256) void trsm_left_leaf_kernel(int nl, int cols, const T* L, int ldl,
                                                             long sl, T* B, int ldb, long sb) {
    __shared__ T sL[TB][TB + 1];
    L += blockIdx.y * sl;
    B += blockIdx.y * sb;
    for (int e = threadIdx.x; e < nl * nl; e += blockDim.x) {
        int i = e / nl, j = e % nl;
        sL[i][j] = (j <= i) ? L[(long)i * ldl + j] : zero_<T>();
    }
    __syncthreads();
    int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= cols) return;
    T x[TB];
    if constexpr (CONJT == 0) {
#pragma unroll
        for (int i = 0; i < TB; ++i) {
            if (i < nl) {
                T s = B[(long)i * ldb + c];
#pragma unroll
                for (int j = 0; j < i; ++j) s -= sL[i][j] * x[j];
                x[i] = s * (1.0 / re_(sL[i][i]));
            }
        }
    } else {
#pragma unroll
        for (int i = TB - 1; i >= 0; --i) {
            if (i < nl) {
                T s = B[(long)i * ldb + c];
#pragma unroll
                for (int j = i + 1; j < TB; ++j)
                    if (j < nl) s -= conj_(sL[j][i]) * x[j];
                x[i] = s * (1.0 / re_(sL[i][i]));
            }
        }
    }
#pragma unroll
    for (int i = 0; i < TB; ++i)
        if (i < nl) B[(long)i * ldb + c] = x[i];
}

template <typename T>
static void trsm_right_lh(hipStream_t s, int rows, int nl, const T* L, int ldl, long sl, T* B,
                          int ldb, long sb, int batch) {
    if (rows <= 0 || nl <= 0) return;
    if (nl <= TB) {
        dim3 grid(cdiv(rows, 256), batch);
        hipLaunchKernelGGL((trsm_right_leaf_kernel<T>), grid, dim3(256), 0, s, rows, nl, L, ldl, sl,
                           B, ldb, sb);
        return;
    }
    int n1 = split_point(nl), n2 = nl - n1;
    trsm_right_lh(s, rows, n1, L, ldl, sl, B, ldb, sb, batch);
    gemm<T>(s, OP_N, OP_C, rows, n2, n1, -1.0, B, ldb, sb, L + (long)n1 * ldl, ldl, sl, 1.0, B + n1,
            ldb, sb, batch);
    trsm_right_lh(s, rows, n2, L + (long)n1 * ldl + n1, ldl, sl, B + n1, ldb, sb, batch);
}

template <typename T>
void trsm_left(hipStream_t s, bool conjt, int nl, int cols, const T* L, int ldl, long sl, T* B,
               int ldb, long sb, int batch) {
    if (cols <= 0 || nl <= 0) return;
    if (nl <= TB) {
        dim3 grid(cdiv(cols, 256), batch);
        if (conjt)
            hipLaunchKernelGGL((trsm_left_leaf_kernel<T, 1>), grid, dim3(256), 0, s, nl, cols, L, ldl,
                               sl, B, ldb, sb);
        else
            hipLaunchKernelGGL((trsm_left_leaf_kernel<T, 0>), grid, dim3(256), 0, s, nl, cols, L, ldl,
                               sl, B, ldb, sb);
        return;
    }
    int n1 = split_point(nl), n2 = nl - n1;
    const T* L21 = L + (long)n1 * ldl;
    const T* L22 = L21 + n1;
    T* B2 = B + (long)n1 * ldb;
    if (!conjt) {
        trsm_left(s, false, n1, cols, L, ldl, sl, B, ldb, sb, batch);
        gemm<T>(s, OP_N, OP_N, n2, cols, n1, -1.0, L21, ldl, sl, B, ldb, sb, 1.0, B2, ldb, sb, batch);
        trsm_left(s, false, n2, cols, L22, ldl, sl, B2, ldb, sb, batch);
    } else {
        trsm_left(s, true, n2, cols, L22, ldl, sl, B2, ldb, sb, batch);
        gemm<T>(s, OP_C, OP_N, n1, cols, n2, -1.0, L21, ldl, sl, B2, ldb, sb, 1.0, B, ldb, sb, batch);
        trsm_left(s, true, n1, cols, L, ldl, sl, B, ldb, sb, batch);
    }
}

template <typename T>
static void potrf_rec(hipStream_t s, int n, T* A, int lda, long sa, int batch, int col0, int* info) {
    if (n <= TB) {
        hipLaunchKernelGGL((potrf_leaf_kernel<T>), dim3(batch), dim3(64), 0, s, n, A, lda, sa, col0,
                           info);
        return;
    }
    int n1 = split_point(n), n2 = n - n1;
    T* A21 = A + (long)n1 * lda;
    T* A22 = A21 + n1;
    potrf_rec(s, n1, A, lda, sa, batch, col0, info);
    trsm_right_lh(s, n2, n1, A, lda, sa, A21, lda, sa, batch);
    gemm<T>(s, OP_N, OP_C, n2, n2, n1, -1.0, A21, lda, sa, A21, lda, sa, 1.0, A22, lda, sa, batch,
            nullptr, 0, UPLO_LOWER);
    potrf_rec(s, n2, A22, lda, sa, batch, col0 + n1, info);
}

template <typename T>
void potrf(hipStream_t s, int n, T* A, int lda, long sa, int batch, int* info) {
    potrf_rec(s, n, A, lda, sa, batch, 0, info);
}

// ---------------------------------------------------------------- copies
// dst (n x n, ld ldd) = Hermitian completion of the lower triangle of src;
// flags non-finite entries of the lower triangle.
template <typename T>
__global__ __launch_bounds__(256) void herm_complete_kernel(int n, const T* src, int lds, long ss,
                                                            T* dst, int ldd, long sd, int* info) {
    __shared__ T tile[32][33];
    src += blockIdx.z * ss;
    dst += blockIdx.z * sd;
    int bi = blockIdx.y * 32, bj = blockIdx.x * 32;
    int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
    if (bj > bi) {
        // upper tile: read the mirrored lower tile (bj.., bi..) and conj-transpose
        for (int r = ty; r < 32; r += 8) {
            int i = bj + r, j = bi + tx;
            tile[r][tx] = (i < n && j < n) ? src[(long)i * lds + j] : zero_<T>();
        }
        __syncthreads();
        for (int r = ty; r < 32; r += 8) {
            int i = bi + r, j = bj + tx;
            if (i < n && j < n) dst[(long)i * ldd + j] = conj_(tile[tx][r]);
        }
    } else {
        for (int r = ty; r < 32; r += 8) {
            int i = bi + r, j = bj + tx;
            if (i < n && j < n) {
                T v = src[(long)i * lds + j];
                if (j <= i && !finite_(v)) set_info(info, KS_ERR_NONFINITE, 0);
                if (i == j) v = from_re<T>(re_(v));
                if (j > i) v = conj_(src[(long)j * lds + i]);
                dst[(long)i * ldd + j] = v;
            }
        }
    }
}

template <typename T>
void herm_complete(hipStream_t s, int n, const T* src, int lds, long ss, T* dst, int ldd, long sd,
                   int batch, int* info) {
    dim3 grid(cdiv(n, 32), cdiv(n, 32), batch);
    hipLaunchKernelGGL((herm_complete_kernel<T>), grid, dim3(256), 0, s, n, src, lds, ss, dst, ldd, sd,
                       info);
}

// dst (cols x rows) = src^H (src rows x cols).
template <typename T>
__global__ __launch_bounds__(256) void conj_transpose_kernel(int rows, int cols, const T* src,
                                                             int lds, T* dst, int ldd) {
    __shared__ T tile[32][33];
    int bi = blockIdx.y * 32, bj = blockIdx.x * 32;
    int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    for (int r = ty; r < 32; r += 8) {
        int i = bi + r, j = bj + tx;
        if (i < rows && j < cols) tile[r][tx] = src[(long)i * lds + j];
    }
    __syncthreads();
    for (int r = ty; r < 32; r += 8) {
        int j = bj + r, i = bi + tx;
        if (i < rows && j < cols) dst[(long)j * ldd + i] = conj_(tile[tx][r]);
    }
}

// A <- (A + A^H)/2 in place (n x n).
template <typename T>
__global__ __launch_bounds__(256) void hermitize_kernel(int n, T* A, int lda) {
    long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    long tot = (long)n * n;
    if (e >= tot) return;
    int i = (int)(e / n), j = (int)(e % n);
    if (j > i) return;
    T* a = A + (long)i * lda + j;
    if (i == j) {
        *a = from_re<T>(re_(*a));
        return;
    }
    T* b = A + (long)j * lda + i;
    T v = 0.5 * (*a + conj_(*b));
    *a = v;
    *b = conj_(v);
}

// Explicit inverse of the lower triangular factor, Linv = L^-1 (solve L X = I);
// the upper triangle of Linv comes out exactly zero.
template <typename T>
__global__ void set_identity_kernel(int n, T* X, long sx) {
    long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    X += blockIdx.y * sx;
    if (e >= (long)n * n) return;
    int i = (int)(e / n), j = (int)(e % n);
    X[e] = (i == j) ? from_re<T>(1.0) : zero_<T>();
}

template <typename T>
void tri_inverse(hipStream_t s, int n, const T* L, int ldl, long sl, T* Linv, long si, int batch) {
    long tot = (long)n * n;
    hipLaunchKernelGGL((set_identity_kernel<T>), dim3(cdiv(tot, 256), batch), dim3(256), 0, s, n, Linv, si);
    trsm_left<T>(s, false, n, n, L, ldl, sl, Linv, n, si, batch);
}

// Reduction of H to A = (I (x) L)^-1 H (I (x) L)^-H with the explicit inverse:
// two MFMA GEMMs whose triangular operand lets each tile skip the zero half of
// its K range (~order^3 flops together for real input).  nsp spin blocks of n
// rows; order = nsp * n.  Only the lower triangle of A is used afterwards.
template <typename T>
void reduce_to_standard(hipStream_t s, int n, int nsp, int batch, const T* H, int ldh, long sH, const T* Linv,
                        int ldi, long sL, T* A, T* W, int* info) {
    const int order = n * nsp;
    const long sA = (long)order * order;
    herm_complete<T>(s, order, H, ldh, sH, A, order, sA, batch, info);
    if (nsp == 1) {
        // W = Linv A, A = W Linv^H for every matrix of the batch
        gemm<T>(s, OP_N, OP_N, n, n, n, 1.0, Linv, ldi, sL, A, order, sA, 0.0, W, order, sA, batch, nullptr, 0,
                UPLO_FULL, nullptr, TRI_A_LOWER);
        gemm<T>(s, OP_N, OP_C, n, n, n, 1.0, W, order, sA, Linv, ldi, sL, 0.0, A, order, sA, batch, nullptr, 0,
                UPLO_FULL, nullptr, TRI_B_UPPER);
        return;
    }
    for (int b = 0; b < batch; ++b) {
        const T* Lb = Linv + b * sL;
        T* Ab = A + b * sA;
        T* Wb = W + b * sA;
        // W = (I (x) Linv) A : spin row-block r of W is Linv times row-block r of A
        gemm<T>(s, OP_N, OP_N, n, order, n, 1.0, Lb, ldi, 0, Ab, order, (long)n * order, 0.0, Wb, order,
                (long)n * order, nsp, nullptr, 0, UPLO_FULL, nullptr, TRI_A_LOWER);
        // A = W (I (x) Linv)^H : spin column-block r of A is column-block r of W times Linv^H
        gemm<T>(s, OP_N, OP_C, order, n, n, 1.0, Wb, order, n, Lb, ldi, 0, 0.0, Ab, order, n, nsp, nullptr, 0,
                UPLO_FULL, nullptr, TRI_B_UPPER);
    }
}

#define KS_INST(T)                                                                                 \
    template void potrf<T>(hipStream_t, int, T*, int, long, int, int*);                            \
    template void trsm_left<T>(hipStream_t, bool, int, int, const T*, int, long, T*, int, long, int); \
    template void herm_complete<T>(hipStream_t, int, const T*, int, long, T*, int, long, int, int*); \
    template void reduce_to_standard<T>(hipStream_t, int, int, int, const T*, int, long, const T*, int, \
                                        long, T*, T*, int*);                                        \
    template void tri_inverse<T>(hipStream_t, int, const T*, int, long, T*, long, int);
KS_INST(double)
KS_INST(cplx)
#undef KS_INST

}  // namespace ks
