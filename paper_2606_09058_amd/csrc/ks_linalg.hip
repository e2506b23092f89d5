// ks_linalg.hip -- Cholesky factorisation of S, triangular solves, and the
// reduction A = L^-1 H L^-H of the generalized problem to standard form.
//
// Cholesky is recursive and forms the inverse factor alongside: an
// LDS-resident workgroup factors and inverts each 64 x 64 diagonal block and
// everything else is an MFMA GEMM (ks_gemm.hip), so the O(n^3) work runs on
// the matrix cores.  L^-1 is formed once per overlap and cached with L, so the
// reduction and the final back-substitution of every solve are plain
// triangular-aware GEMMs.  The spinor form applies L^-1 to each
// spin block, i.e. (I2 (x) L)^-1 H (I2 (x) L)^-H, by treating the 2n x 2n
// matrix as two n-row (then n-column) blocks: a batch of 2 with a block stride.
#include "ks_internal.hpp"

namespace ks {

// ---------------------------------------------------------------- Cholesky
// Recursive with explicit inverse: for S = [S11 S12; S21 S22],
//   L11, inv11 from S11;  L21 = S21 inv11^H;  S22 -= L21 L21^H;
//   L22, inv22 from S22;  inv21 = -inv22 L21 inv11,
// down to 64 x 64 diagonal blocks that one workgroup factors and inverts in
// LDS.  Every product is an MFMA GEMM with a large inner dimension, the
// triangular operands skipping their zero half.
constexpr int CB = 64;

// Factor the nb x nb (nb <= CB) lower block at A in place and write its inverse
// (lower, zero above) at D.  Column j of the factorisation and of the inverse
// (right-looking forward substitution of L X = I) share one step with one
// barrier: every thread reads the pivot itself; row i > j, entry c <= i takes
//   c >  j:  S[i][c] -= S[i][j] conj(S[c][j]) / d_j      (factor)
//   c <= j:  Y[i][c] -= S[i][j] Y[j][c] / d_j            (inverse)
// with the columns of S and rows of Y left unscaled until the end
// (L[i][j] = S[i][j] / sqrt(d_j), X[i][c] = Y[i][c] / sqrt(d_i)).  One wavefront
// per row (rows j+1+w, j+1+w+LW, ... for LW = 16 wavefronts), one lane per
// column: no index division, four rows per thread and step.
// A non-positive or non-finite pivot records the global 1-based column
// col0 + j + 1 and continues with pivot 1.
constexpr int LW = 16;  // wavefronts of the leaf kernel
template <typename T>
__global__ __launch_bounds__(64 * LW) void potrf_inv_leaf_kernel(int nb, T* A, int lda, long sa, T* D, int ldd,
                                                             long sd, int col0, int* info) {
    __shared__ T sL[CB][CB + 1];
    __shared__ T sY[CB][CB + 1];
    __shared__ double rl[CB];
    A += blockIdx.x * sa;
    D += blockIdx.x * sd;
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    for (int i = w; i < CB; i += LW) {
        sL[i][lane] = (i < nb && lane <= i) ? A[(long)i * lda + lane] : zero_<T>();
        sY[i][lane] = (i == lane) ? from_re<T>(1.0) : zero_<T>();
    }
    __syncthreads();
    for (int j = 0; j < nb; ++j) {
        const double d = re_(sL[j][j]);
        const bool bad = !(d > 0.0) || !isfinite(d);
        const double dj = bad ? 1.0 : d;
        const double inv_d = 1.0 / dj;
        if (t == 0) {
            if (bad) set_info(info, KS_ERR_NOT_POSDEF, col0 + j + 1);
            rl[j] = 1.0 / sqrt(dj);
        }
        const int c = lane;
        const T scj = conj_(sL[c][j]) * inv_d;  // factor part (c > j)
        const T ycj = sY[j][c] * inv_d;          // inverse part (c <= j)
        // all reads of this step first (they cannot alias its writes), then the writes
        constexpr int RPW = CB / LW;  // rows per wavefront
        T sij[RPW], cur[RPW];
#pragma unroll
        for (int q = 0; q < RPW; ++q) {
            const int i = j + 1 + w + LW * q;
            if (i < nb) {
                sij[q] = sL[i][j];
                cur[q] = (c > j) ? sL[i][c] : sY[i][c];
            }
        }
#pragma unroll
        for (int q = 0; q < RPW; ++q) {
            const int i = j + 1 + w + LW * q;
            if (i < nb) {
                if (c > j && c <= i) sL[i][c] = cur[q] - sij[q] * scj;
                else if (c <= j) sY[i][c] = cur[q] - sij[q] * ycj;
            }
        }
        __syncthreads();
    }
    for (int i = w; i < nb; i += LW) {
        const int c = lane;
        if (c < nb) {
            T lv = zero_<T>(), xv = zero_<T>();
            if (c < i) lv = sL[i][c] * rl[c];
            else if (c == i) lv = from_re<T>(1.0 / rl[i]);
            if (c <= i) xv = sY[i][c] * rl[i];
            if (c <= i) A[(long)i * lda + c] = lv;
            D[(long)i * ldd + c] = xv;
        }
    }
}

// dst (rows x cols, ld ldd) = src (ld lds) for a batch.
template <typename T>
__global__ void copy_block_kernel(int rows, int cols, const T* src, int lds, long ss, T* dst, int ldd, long sd) {
    long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (long)rows * cols) return;
    int r = (int)(e / cols), c = (int)(e % cols);
    dst[blockIdx.y * sd + (long)r * ldd + c] = src[blockIdx.y * ss + (long)r * lds + c];
}

template <typename T>
static void potrf_inv_rec(hipStream_t s, int n, T* L, int ldl, long sl, T* Li, int ldi, long si, T* Tw, long st,
                          int batch, int col0, int* info) {
    if (n <= CB) {
        hipLaunchKernelGGL((potrf_inv_leaf_kernel<T>), dim3(batch), dim3(64 * LW), 0, s, n, L, ldl, sl, Li, ldi, si,
                           col0, info);
        return;
    }
    int n1 = ((n / 2 + CB - 1) / CB) * CB;
    if (n1 >= n) n1 = n - CB;
    const int n2 = n - n1;
    T* L21 = L + (long)n1 * ldl;
    T* L22 = L21 + n1;
    T* Li21 = Li + (long)n1 * ldi;
    T* Li22 = Li21 + n1;
    potrf_inv_rec(s, n1, L, ldl, sl, Li, ldi, si, Tw, st, batch, col0, info);
    // L21 = S21 inv11^H (through Tw: a tile reads whole rows of S21)
    gemm<T>(s, OP_N, OP_C, n2, n1, n1, 1.0, L21, ldl, sl, Li, ldi, si, 0.0, Tw, n1, st, batch, nullptr, 0,
            UPLO_FULL, nullptr, TRI_B_UPPER);
    long tot = (long)n2 * n1;
    hipLaunchKernelGGL((copy_block_kernel<T>), dim3(cdiv(tot, 256), batch), dim3(256), 0, s, n2, n1, Tw, n1, st,
                       L21, ldl, sl);
    gemm<T>(s, OP_N, OP_C, n2, n2, n1, -1.0, L21, ldl, sl, L21, ldl, sl, 1.0, L22, ldl, sl, batch, nullptr, 0,
            UPLO_LOWER);
    potrf_inv_rec(s, n2, L22, ldl, sl, Li22, ldi, si, Tw, st, batch, col0 + n1, info);
    // inv21 = -inv22 (L21 inv11)
    gemm<T>(s, OP_N, OP_N, n2, n1, n1, 1.0, L21, ldl, sl, Li, ldi, si, 0.0, Tw, n1, st, batch, nullptr, 0,
            UPLO_FULL, nullptr, TRI_B_LOWER);
    gemm<T>(s, OP_N, OP_N, n2, n1, n2, -1.0, Li22, ldi, si, Tw, n1, st, 0.0, Li21, ldi, si, batch, nullptr, 0,
            UPLO_FULL, nullptr, TRI_A_LOWER);
}

template <typename T>
__global__ void zero_upper_kernel(int n, T* X, int ldx, long sx) {
    long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (long)n * n) return;
    int i = (int)(e / n), j = (int)(e % n);
    if (j > i) X[blockIdx.y * sx + (long)i * ldx + j] = zero_<T>();
}

template <typename T>
void potrf_inv(hipStream_t s, int n, T* L, int ldl, long sl, T* Li, int ldi, long si, T* work, long sw,
               int batch, int* info) {
    long tot = (long)n * n;
    hipLaunchKernelGGL((zero_upper_kernel<T>), dim3(cdiv(tot, 256), batch), dim3(256), 0, s, n, Li, ldi, si);
    potrf_inv_rec<T>(s, n, L, ldl, sl, Li, ldi, si, work, sw, batch, 0, info);
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

// The strictly upper triangle of each n x n matrix X (row stride ldx, matrix
// stride sx) from its lower one, in place: X[i][j] = conj(X[j][i]) for j > i,
// and the diagonal made real, so that X is exactly Hermitian.  One workgroup
// per 32 x 32 tile on or above the diagonal; each element is read once (into
// LDS) before the tile writes it.
template <typename T>
__global__ __launch_bounds__(256) void mirror_lower_kernel(int n, T* X, int ldx, long sx) {
    __shared__ T tile[32][33];
    const int bi = blockIdx.y * 32, bj = blockIdx.x * 32;
    if (bj < bi) return;
    X += blockIdx.z * sx;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
    for (int r = ty; r < 32; r += 8) {
        const int i = bj + r, j = bi + tx;  // the mirrored tile, lower part only
        tile[r][tx] = (i < n && j < n && j <= i) ? X[(long)i * ldx + j] : zero_<T>();
    }
    __syncthreads();
    for (int r = ty; r < 32; r += 8) {
        const int i = bi + r, j = bj + tx;
        if (i < n && j < n && j > i) X[(long)i * ldx + j] = conj_(tile[tx][r]);
        if (i < n && j == i) X[(long)i * ldx + j] = from_re<T>(re_(tile[tx][r]));  // real diagonal
    }
}

template <typename T>
void mirror_lower(hipStream_t s, int n, T* X, int ldx, long sx, int batch) {
    if (n <= 0 || batch <= 0) return;
    dim3 grid(cdiv(n, 32), cdiv(n, 32), batch);
    hipLaunchKernelGGL((mirror_lower_kernel<T>), grid, dim3(256), 0, s, n, X, ldx, sx);
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
// Reduction of H to A = (I (x) L)^-1 H (I (x) L)^-H with the explicit inverse:
// two MFMA GEMMs whose triangular operand lets each tile skip the zero half of
// its K range (~order^3 flops together for real input).  nsp spin blocks of n
// rows; order = nsp * n.  Only the lower triangle of A is used afterwards.
template <typename T>
void reduce_to_standard(hipStream_t s, int n, int nsp, int batch, const T* H, int ldh, long sH, const T* Linv,
                        int ldi, long sL, T* A, T* W, int* info, bool lower_only) {
    const int order = n * nsp;
    const long sA = (long)order * order;
    const Uplo up = lower_only ? UPLO_LOWER : UPLO_FULL;
    herm_complete<T>(s, order, H, ldh, sH, A, order, sA, batch, info);
    if (nsp == 1) {
        // W = Linv A, A = W Linv^H for every matrix of the batch
        gemm<T>(s, OP_N, OP_N, n, n, n, 1.0, Linv, ldi, sL, A, order, sA, 0.0, W, order, sA, batch, nullptr, 0,
                UPLO_FULL, nullptr, TRI_A_LOWER);
        gemm<T>(s, OP_N, OP_C, n, n, n, 1.0, W, order, sA, Linv, ldi, sL, 0.0, A, order, sA, batch, nullptr, 0, up,
                nullptr, TRI_B_UPPER);
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
        if (!lower_only) {
            gemm<T>(s, OP_N, OP_C, order, n, n, 1.0, Wb, order, n, Lb, ldi, 0, 0.0, Ab, order, n, nsp, nullptr, 0,
                    UPLO_FULL, nullptr, TRI_B_UPPER);
        } else {
            // lower triangle: column-block 0 over all rows, column-block 1 over its own rows only
            gemm<T>(s, OP_N, OP_C, order, n, n, 1.0, Wb, order, 0, Lb, ldi, 0, 0.0, Ab, order, 0, 1, nullptr, 0,
                    UPLO_LOWER, nullptr, TRI_B_UPPER);
            const long d = (long)n * order + n;
            gemm<T>(s, OP_N, OP_C, n, n, n, 1.0, Wb + d, order, 0, Lb, ldi, 0, 0.0, Ab + d, order, 0, 1, nullptr, 0,
                    UPLO_LOWER, nullptr, TRI_B_UPPER);
        }
    }
}

// dst = Re of the symmetric completion of src's lower triangle (tiles of 32
// x 32 through LDS, as in herm_complete); the lower triangle's imaginary
// parts must be zero.
__global__ __launch_bounds__(256) void real_sym_complete_kernel(int n, const cplx* src, int lds, long ss,
                                                                double* dst, int ldd, long sd, int* info) {
    __shared__ double tile[32][33];
    src += blockIdx.z * ss;
    dst += blockIdx.z * sd;
    const int bi = blockIdx.y * 32, bj = blockIdx.x * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
    if (bj > bi) {
        // upper tile: the mirrored lower tile (bj.., bi..), transposed
        for (int r = ty; r < 32; r += 8) {
            const int i = bj + r, j = bi + tx;
            tile[r][tx] = (i < n && j < n) ? src[(long)i * lds + j].x : 0.0;
        }
        __syncthreads();
        for (int r = ty; r < 32; r += 8) {
            const int i = bi + r, j = bj + tx;
            if (i < n && j < n) dst[(long)i * ldd + j] = tile[tx][r];
        }
    } else {
        for (int r = ty; r < 32; r += 8) {
            const int i = bi + r, j = bj + tx;
            if (i < n && j < n) {
                const int a = max(i, j), b = min(i, j);
                const cplx v = src[(long)a * lds + b];
                if (j <= i) {
                    if (!finite_(v)) set_info(info, KS_ERR_NONFINITE, 0);
                    else if (v.y != 0.0) set_info(info, KS_ERR_INVALID_ARG, i + 1);
                }
                dst[(long)i * ldd + j] = v.x;
            }
        }
    }
}

void real_sym_complete(hipStream_t s, int n, const cplx* src, int lds, long ss, double* dst, int ldd, long sd,
                       int batch, int* info) {
    dim3 grid(cdiv(n, 32), cdiv(n, 32), batch);
    hipLaunchKernelGGL(real_sym_complete_kernel, grid, dim3(256), 0, s, n, src, lds, ss, dst, ldd, sd, info);
}

// dst = src^H for a batch of n x n matrices (32 x 32 tiles through LDS).
template <typename T>
__global__ __launch_bounds__(256) void conj_transpose_kernel(int n, const T* src, int lds, long ss, T* dst,
                                                             int ldd, long sd) {
    __shared__ T tile[32][33];
    src += blockIdx.z * ss;
    dst += blockIdx.z * sd;
    const int bi = blockIdx.y * 32, bj = blockIdx.x * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    for (int r = ty; r < 32; r += 8) {
        const int i = bj + r, j = bi + tx;  // source tile (bj.., bi..)
        tile[r][tx] = (i < n && j < n) ? src[(long)i * lds + j] : zero_<T>();
    }
    __syncthreads();
    for (int r = ty; r < 32; r += 8) {
        const int i = bi + r, j = bj + tx;
        if (i < n && j < n) dst[(long)i * ldd + j] = conj_(tile[tx][r]);
    }
}

void reduce_to_standard_real(hipStream_t s, int n, int nsp, int batch, const cplx* H, int ldh, long sH,
                             const double* Linv, int ldi, long sL, cplx* A, cplx* W, int* info,
                             bool lower_only) {
    const int order = n * nsp;
    const long sA = (long)order * order;
    const int ro = 2 * order;  // row length of an order x order complex matrix seen as real
    // W = H (Hermitian completion of its lower triangle)
    herm_complete<cplx>(s, order, H, ldh, sH, W, order, sA, batch, info);
    for (int b = 0; b < batch; ++b) {
        const double* Lb = Linv + b * sL;
        // A = M W: spin row-block r of A is Linv times row-block r of W
        gemm<double>(s, OP_N, OP_N, n, ro, n, 1.0, Lb, ldi, 0, (const double*)(W + b * sA), ro, (long)n * ro, 0.0,
                     (double*)(A + b * sA), ro, (long)n * ro, nsp, nullptr, 0, UPLO_FULL, nullptr, TRI_A_LOWER);
    }
    // W = A^H = H M^T
    hipLaunchKernelGGL((conj_transpose_kernel<cplx>), dim3(cdiv(order, 32), cdiv(order, 32), batch), dim3(256), 0,
                       s, order, A, order, sA, W, order, sA);
    for (int b = 0; b < batch; ++b) {
        const double* Lb = Linv + b * sL;
        const double* Wb = (const double*)(W + b * sA);
        double* Ab = (double*)(A + b * sA);
        if (!lower_only) {
            gemm<double>(s, OP_N, OP_N, n, ro, n, 1.0, Lb, ldi, 0, Wb, ro, (long)n * ro, 0.0, Ab, ro, (long)n * ro,
                         nsp, nullptr, 0, UPLO_FULL, nullptr, TRI_A_LOWER);
            continue;
        }
        // lower triangle of A = M W: row-block 0 over its own columns, and
        // for spinors row-block 1 over all of column-block 0 and its own
        // columns of column-block 1
        gemm<double>(s, OP_N, OP_N, n, 2 * n, n, 1.0, Lb, ldi, 0, Wb, ro, 0, 0.0, Ab, ro, 0, 1, nullptr, 0,
                     UPLO_LOWER2, nullptr, TRI_A_LOWER);
        if (nsp == 2) {
            const long r1 = (long)n * ro;  // first element of row-block 1
            gemm<double>(s, OP_N, OP_N, n, 2 * n, n, 1.0, Lb, ldi, 0, Wb + r1, ro, 0, 0.0, Ab + r1, ro, 0, 1,
                         nullptr, 0, UPLO_FULL, nullptr, TRI_A_LOWER);
            gemm<double>(s, OP_N, OP_N, n, 2 * n, n, 1.0, Lb, ldi, 0, Wb + r1 + 2 * n, ro, 0, 0.0, Ab + r1 + 2 * n,
                         ro, 0, 1, nullptr, 0, UPLO_LOWER2, nullptr, TRI_A_LOWER);
        }
    }
}

#define KS_INST(T)                                                                                 \
    template void herm_complete<T>(hipStream_t, int, const T*, int, long, T*, int, long, int, int*); \
    template void reduce_to_standard<T>(hipStream_t, int, int, int, const T*, int, long, const T*, int, \
                                        long, T*, T*, int*, bool);                                  \
    template void potrf_inv<T>(hipStream_t, int, T*, int, long, T*, int, long, T*, long, int, int*);    \
    template void mirror_lower<T>(hipStream_t, int, T*, int, long, int);
KS_INST(double)
KS_INST(cplx)
#undef KS_INST

}  // namespace ks
