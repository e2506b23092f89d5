// ks_gemm.hip -- matrix-core (MFMA) GEMM for gfx950, real and complex, FP64
// and (for the mixed-precision path) FP32 with FP32 accumulation.
//
// Every dense contraction of the eigensolver goes through this kernel: the
// Cholesky trailing update, the triangular-solve updates of the reduction
// L^-1 H L^-H, the two-sided rank-2k trailing update of the Householder
// tridiagonalisation, the divide-and-conquer merge products, the compact-WY
// back-transform and the density C f C^H.
//
// Tile: 64 x 64 outputs per 256-thread workgroup, K step 16, staged through
// LDS with a register prefetch of the next K step.  Each of the 4 waves owns
// a 32 x 32 quadrant = 2 x 2 blocks of v_mfma_f64_16x16x4_f64.  Lane l of an
// MFMA supplies A[l%16][l/16] and B[l/16][l%16] of the 16x4 / 4x16 operands
// and receives D[l/16 + 4r][l%16] in accumulator register r.  The FP32 tile
// uses v_mfma_f32_16x16x4_f32 with the same operand layout; its lane l receives
// D[4 (l/16) + r][l%16].  A complex product uses four real MFMAs
// (re*re - im*im, re*im + im*re) into separate real and imaginary accumulators.
#include <algorithm>
#include <type_traits>

#include "ks_internal.hpp"

namespace ks {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int BM = 64, BN = 64, BK = 16, LPAD = 2;

__device__ inline d4 mfma(double a, double b, d4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ inline f4 mfma(float a, float b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// Row (within a 16 x 16 block) of accumulator register r of a lane.
template <typename T>
__device__ inline int out_row(int lane, int r) {
    if constexpr (sizeof(T) == 8 && !is_cplx<T>::value) return (lane >> 4) + 4 * r;  // f64 MFMA
    else if constexpr (is_cplx<T>::value && sizeof(T) == 16) return (lane >> 4) + 4 * r;
    else return 4 * (lane >> 4) + r;  // f32 MFMA
}

template <typename T, int OP>
__device__ inline T ld_op(const T* p) {
    T v = *p;
    if constexpr (OP == OP_C) v = conj_(v);
    return v;
}

// Load the BM x BK tile of op(A) starting at (m0, k0) into registers.
// Mapping A: element (m, k) of op(A) is A[m*lda + k] for OP_N, A[k*lda + m]
// otherwise.  The four elements a thread loads are contiguous in memory.
template <typename T, int OPA>
__device__ inline void load_a(T (&r)[4], const T* A, int lda, int m, int K, int m0, int k0,
                              const double* ks) {
    int t = threadIdx.x;
    if constexpr (OPA == OP_N) {
        int mm = m0 + (t >> 2), kk = k0 + (t & 3) * 4;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            bool ok = mm < m && kk + i < K;
            r[i] = ok ? ld_op<T, OPA>(A + (long)mm * lda + kk + i) : zero_<T>();
            if (ks && ok) r[i] = r[i] * ks[kk + i];  // (a narrowing multiply for FP32 types)
        }
    } else {
        int kk = k0 + (t >> 4), mm = m0 + (t & 15) * 4;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            bool ok = mm + i < m && kk < K;
            r[i] = ok ? ld_op<T, OPA>(A + (long)kk * lda + mm + i) : zero_<T>();
            if (ks && ok) r[i] = r[i] * ks[kk];
        }
    }
}

template <typename T, int OPA>
__device__ inline void store_a(const T (&r)[4], T (*sA)[BM + LPAD]) {
    int t = threadIdx.x;
    if constexpr (OPA == OP_N) {
        int mm = t >> 2, kk = (t & 3) * 4;
#pragma unroll
        for (int i = 0; i < 4; ++i) sA[kk + i][mm] = r[i];
    } else {
        int kk = t >> 4, mm = (t & 15) * 4;
#pragma unroll
        for (int i = 0; i < 4; ++i) sA[kk][mm + i] = r[i];
    }
}

// op(B) is K x N: element (k, n) is B[k*ldb + n] for OP_N, B[n*ldb + k] otherwise.
template <typename T, int OPB>
__device__ inline void load_b(T (&r)[4], const T* B, int ldb, int n, int K, int n0, int k0) {
    int t = threadIdx.x;
    if constexpr (OPB == OP_N) {
        int kk = k0 + (t >> 4), nn = n0 + (t & 15) * 4;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            bool ok = nn + i < n && kk < K;
            r[i] = ok ? B[(long)kk * ldb + nn + i] : zero_<T>();
        }
    } else {
        int nn = n0 + (t >> 2), kk = k0 + (t & 3) * 4;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            bool ok = nn < n && kk + i < K;
            r[i] = ok ? ld_op<T, OPB>(B + (long)nn * ldb + kk + i) : zero_<T>();
        }
    }
}

template <typename T, int OPB>
__device__ inline void store_b(const T (&r)[4], T (*sB)[BN + LPAD]) {
    int t = threadIdx.x;
    if constexpr (OPB == OP_N) {
        int kk = t >> 4, nn = (t & 15) * 4;
#pragma unroll
        for (int i = 0; i < 4; ++i) sB[kk][nn + i] = r[i];
    } else {
        int nn = t >> 2, kk = (t & 3) * 4;
#pragma unroll
        for (int i = 0; i < 4; ++i) sB[kk + i][nn] = r[i];
    }
}

template <typename T>
struct Acc;
template <>
struct Acc<double> {
    d4 c[2][2];
};
// FP64 complex tiles take three real products per complex one (p1 = Re a Re b,
// p2 = Im a Im b, p3 = (Re a + Im a)(Re b + Im b); Re = p1 - p2,
// Im = p3 - p1 - p2), a quarter fewer MFMAs than the four-product form with
// the same normwise error bound.
template <>
struct Acc<cplx> {
    d4 p1[2][2], p2[2][2], p3[2][2];
};
template <>
struct Acc<float> {
    f4 c[2][2];
};
template <>
struct Acc<cplx32> {
    f4 re[2][2], im[2][2];
};

__device__ inline void acc_zero(Acc<double>& a) {
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) a.c[i][j] = d4{0.0, 0.0, 0.0, 0.0};
}
__device__ inline void acc_zero(Acc<cplx>& a) {
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            a.p1[i][j] = d4{0.0, 0.0, 0.0, 0.0};
            a.p2[i][j] = d4{0.0, 0.0, 0.0, 0.0};
            a.p3[i][j] = d4{0.0, 0.0, 0.0, 0.0};
        }
}

__device__ inline void acc_zero(Acc<float>& a) {
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) a.c[i][j] = f4{0.f, 0.f, 0.f, 0.f};
}
__device__ inline void acc_zero(Acc<cplx32>& a) {
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            a.re[i][j] = f4{0.f, 0.f, 0.f, 0.f};
            a.im[i][j] = f4{0.f, 0.f, 0.f, 0.f};
        }
}

// Real tile product (FP64 or FP32 MFMA, the same operand layout).
template <typename R, typename V>
__device__ inline void tile_mma_real(V (&c)[2][2], R (*sA)[BM + LPAD], R (*sB)[BN + LPAD]) {
    int lane = threadIdx.x & 63, w = threadIdx.x >> 6, wm = w >> 1, wn = w & 1;
    int li = lane & 15, lk = lane >> 4;
#pragma unroll
    for (int ks = 0; ks < BK / 4; ++ks) {
        int kr = ks * 4 + lk;
        R a0 = sA[kr][wm * 32 + li], a1 = sA[kr][wm * 32 + 16 + li];
        R b0 = sB[kr][wn * 32 + li], b1 = sB[kr][wn * 32 + 16 + li];
        c[0][0] = mfma(a0, b0, c[0][0]);
        c[0][1] = mfma(a0, b1, c[0][1]);
        c[1][0] = mfma(a1, b0, c[1][0]);
        c[1][1] = mfma(a1, b1, c[1][1]);
    }
}

// Complex tile product: four real MFMAs per block.
template <typename C, typename V>
__device__ inline void tile_mma_cplx(V (&re)[2][2], V (&im)[2][2], C (*sA)[BM + LPAD], C (*sB)[BN + LPAD]) {
    int lane = threadIdx.x & 63, w = threadIdx.x >> 6, wm = w >> 1, wn = w & 1;
    int li = lane & 15, lk = lane >> 4;
#pragma unroll
    for (int ks = 0; ks < BK / 4; ++ks) {
        int kr = ks * 4 + lk;
        C a[2] = {sA[kr][wm * 32 + li], sA[kr][wm * 32 + 16 + li]};
        C b[2] = {sB[kr][wn * 32 + li], sB[kr][wn * 32 + 16 + li]};
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                re[i][j] = mfma(a[i].x, b[j].x, re[i][j]);
                re[i][j] = mfma(-a[i].y, b[j].y, re[i][j]);
                im[i][j] = mfma(a[i].x, b[j].y, im[i][j]);
                im[i][j] = mfma(a[i].y, b[j].x, im[i][j]);
            }
    }
}

__device__ inline void tile_mma(Acc<float>& acc, float (*sA)[BM + LPAD], float (*sB)[BN + LPAD]) {
    tile_mma_real<float, f4>(acc.c, sA, sB);
}
__device__ inline void tile_mma(Acc<cplx32>& acc, cplx32 (*sA)[BM + LPAD], cplx32 (*sB)[BN + LPAD]) {
    tile_mma_cplx<cplx32, f4>(acc.re, acc.im, sA, sB);
}
__device__ inline float acc_get(const Acc<float>& a, int i, int j, int r) { return a.c[i][j][r]; }
__device__ inline cplx32 acc_get(const Acc<cplx32>& a, int i, int j, int r) {
    return mk32(a.re[i][j][r], a.im[i][j][r]);
}

__device__ inline void tile_mma(Acc<double>& acc, double (*sA)[BM + LPAD], double (*sB)[BN + LPAD]) {
    int lane = threadIdx.x & 63, w = threadIdx.x >> 6, wm = w >> 1, wn = w & 1;
    int li = lane & 15, lk = lane >> 4;
#pragma unroll
    for (int ks = 0; ks < BK / 4; ++ks) {
        int kr = ks * 4 + lk;
        double a0 = sA[kr][wm * 32 + li], a1 = sA[kr][wm * 32 + 16 + li];
        double b0 = sB[kr][wn * 32 + li], b1 = sB[kr][wn * 32 + 16 + li];
        acc.c[0][0] = mfma(a0, b0, acc.c[0][0]);
        acc.c[0][1] = mfma(a0, b1, acc.c[0][1]);
        acc.c[1][0] = mfma(a1, b0, acc.c[1][0]);
        acc.c[1][1] = mfma(a1, b1, acc.c[1][1]);
    }
}

__device__ inline void tile_mma(Acc<cplx>& acc, cplx (*sA)[BM + LPAD], cplx (*sB)[BN + LPAD]) {
    int lane = threadIdx.x & 63, w = threadIdx.x >> 6, wm = w >> 1, wn = w & 1;
    int li = lane & 15, lk = lane >> 4;
#pragma unroll 2
    for (int ks = 0; ks < BK / 4; ++ks) {
        int kr = ks * 4 + lk;
        cplx a[2] = {sA[kr][wm * 32 + li], sA[kr][wm * 32 + 16 + li]};
        cplx b[2] = {sB[kr][wn * 32 + li], sB[kr][wn * 32 + 16 + li]};
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                acc.p1[i][j] = mfma(a[i].x, b[j].x, acc.p1[i][j]);
                acc.p2[i][j] = mfma(a[i].y, b[j].y, acc.p2[i][j]);
                acc.p3[i][j] = mfma(a[i].x + a[i].y, b[j].x + b[j].y, acc.p3[i][j]);
            }
    }
}

__device__ inline double acc_get(const Acc<double>& a, int i, int j, int r) { return a.c[i][j][r]; }
__device__ inline cplx acc_get(const Acc<cplx>& a, int i, int j, int r) {
    const double p1 = a.p1[i][j][r], p2 = a.p2[i][j][r];
    return mk(p1 - p2, a.p3[i][j][r] - p1 - p2);
}

// One 64 x 64 output tile at (m0, n0).
template <typename T, int OPA, int OPB>
__device__ inline void gemm_tile(int m, int n, int K, double alpha, const T* A, int lda, const T* B,
                                 int ldb, double beta, T* C, int ldc, const double* kscale, int uplo,
                                 int m0, int n0, int klo = 0) {
    __shared__ T sA[BK][BM + LPAD];
    __shared__ T sB[BK][BN + LPAD];
    Acc<T> acc;
    acc_zero(acc);
    T ra[4], rb[4];
    if (K > klo) {
        load_a<T, OPA>(ra, A, lda, m, K, m0, klo, kscale);
        load_b<T, OPB>(rb, B, ldb, n, K, n0, klo);
    }
    for (int k0 = klo; k0 < K; k0 += BK) {
        __syncthreads();
        store_a<T, OPA>(ra, sA);
        store_b<T, OPB>(rb, sB);
        __syncthreads();
        if (k0 + BK < K) {
            load_a<T, OPA>(ra, A, lda, m, K, m0, k0 + BK, kscale);
            load_b<T, OPB>(rb, B, ldb, n, K, n0, k0 + BK);
        }
        tile_mma(acc, sA, sB);
    }
    int lane = threadIdx.x & 63, w = threadIdx.x >> 6, wm = w >> 1, wn = w & 1;
    // with beta != 0 a row of blocks' C values are all requested before any is
    // written back (see the large-tile kernel); complex tiles read C in place,
    // which keeps their register budget
    const bool acc_c = beta != 0.0;
    constexpr bool pre = !is_cplx<T>::value;
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        T cv[2][4];
        if (pre && acc_c) {
#pragma unroll
            for (int j = 0; j < 2; ++j)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int row = m0 + wm * 32 + i * 16 + out_row<T>(lane, r);
                    const int col = n0 + wn * 32 + j * 16 + (lane & 15);
                    const bool ok = row < m && col < n && in_uplo(uplo, row, col);
                    cv[j][r] = ok ? C[(long)row * ldc + col] : zero_<T>();
                }
        }
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                int row = m0 + wm * 32 + i * 16 + out_row<T>(lane, r);
                int col = n0 + wn * 32 + j * 16 + (lane & 15);
                if (row < m && col < n && in_uplo(uplo, row, col)) {
                    T v = alpha * acc_get(acc, i, j, r);
                    T* pc = C + (long)row * ldc + col;
                    if (acc_c) v += beta * (pre ? cv[j][r] : *pc);
                    *pc = v;
                }
            }
    }
}

template <typename T, int OPA, int OPB>
__global__ __launch_bounds__(256) void gemm_kernel(int m, int n, int K, double alpha, const T* A,
                                                   int lda, long sa, const T* B, int ldb, long sb,
                                                   double beta, T* C, int ldc, long sc,
                                                   const double* kscale, long sk, int uplo,
                                                   const int* kdev, int tri) {
    int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
    if (!in_uplo(uplo, m0 + BM - 1, n0)) return;  // tile strictly above the diagonal
    long b = blockIdx.z;
    if (kdev) K = min(K, *kdev);  // inner size decided on the device (occupied window)
    // triangular operands: skip the K range where the operand is known to be zero
    int klo = 0;
    if (tri == TRI_A_LOWER) K = min(K, m0 + BM);
    if (tri == TRI_B_UPPER) K = min(K, n0 + BN);
    if (tri == TRI_A_UPPER) klo = (m0 / BK) * BK;
    if (tri == TRI_B_LOWER) klo = (n0 / BK) * BK;
    gemm_tile<T, OPA, OPB>(m, n, K, alpha, A + b * sa, lda, B + b * sb, ldb, beta, C + b * sc, ldc,
                           kscale ? kscale + b * sk : nullptr, uplo, m0, n0, klo);
}


// ---------------------------------------------------------------- large tiles
// Large tiles only where they pay: enough k steps to amortise the tile's
// prologue and epilogue, and enough tiles to keep two workgroups on every CU
// (measured: rank-64 updates and 6656 x 1414 x 6656 FP64 products run faster
// on 64 x 64 tiles).
constexpr long BIG_MIN_TILES = 512;
constexpr int BIG_MIN_K = 256;
// The smallest k for the large tiles, set per plan call (the autotuner's
// knob) on the calling thread: launches are enqueued by the thread that calls
// the entry point, so a plan's setting holds for exactly its own launches.
static thread_local int g_big_min_k = BIG_MIN_K;
void gemm_set_big_min_k(int k) { g_big_min_k = k; }
int gemm_big_min_k() { return g_big_min_k; }
// Output tiles of BM x BN (128 x 128; 64 x 64 for FP64 complex) with one
// wave tile of BM/2 x BN/2 per wavefront (2 x 2 wavefronts), so that each k
// step feeds (BM/32)(BN/32) MFMA blocks per wavefront per operand fragment
// pair: half the L2 traffic per flop of the 64 x 64 tile.  The LDS stages are
// double-buffered (one barrier per k step) and each thread prefetches its
// share of the next stage into registers while the current one is used.
template <typename T>
struct Big;
// accumulator vector of one 16 x 16 MFMA block, and a complex value from its parts
template <typename T>
struct AccVec {
    using type = d4;
};
template <>
struct AccVec<float> {
    using type = f4;
};
template <>
struct AccVec<cplx32> {
    using type = f4;
};
__device__ inline cplx from_parts(double re, double im, const cplx*) { return mk(re, im); }
__device__ inline cplx32 from_parts(float re, float im, const cplx32*) { return mk32(re, im); }
template <>
struct Big<double> {
    static constexpr int BM = 128, BN = 128, BK = 16;
};
template <>
struct Big<float> {
    static constexpr int BM = 128, BN = 128, BK = 32;
};
template <>
struct Big<cplx> {
    static constexpr int BM = 64, BN = 64, BK = 16;  // (two workgroups per CU fit in LDS)
};
template <>
struct Big<cplx32> {
    static constexpr int BM = 128, BN = 128, BK = 16;
};

// Load an R x C block of memory (row stride ld, C contiguous) starting at
// (r0, c0), zero outside rows < nr and columns < nc; every thread takes one
// contiguous run of R C / 256 elements.
template <typename T, int R, int C, int OP>
__device__ inline void big_load(T (&v)[R * C / 256], const T* P, int ld, int nr, int nc, int r0, int c0,
                                int t) {
    constexpr int E = R * C / 256, TPR = C / E;
    static_assert(E * 256 == R * C && TPR * E == C && 256 / TPR == R, "block shape");
    const int rr = r0 + t / TPR, cc = c0 + (t % TPR) * E;
#pragma unroll
    for (int i = 0; i < E; ++i) {
        const bool ok = rr < nr && cc + i < nc;
        v[i] = ok ? ld_op<T, OP>(P + (long)rr * ld + cc + i) : zero_<T>();
    }
}

template <typename T, int OPA, int OPB>
__global__ __launch_bounds__(256, 2) void gemm_big_kernel(int m, int n, int K, double alpha, const T* A, int lda,
                                                       long sa, const T* B, int ldb, long sb, double beta, T* C,
                                                       int ldc, long sc, int uplo, const int* kdev, int tri) {
    constexpr int BM = Big<T>::BM, BN = Big<T>::BN, BKb = Big<T>::BK;
    constexpr int WM = BM / 2, WN = BN / 2, MI = WM / 16, NI = WN / 16;
    constexpr int EA = BM * BKb / 256, EB = BN * BKb / 256;
    __shared__ T sA[2][BKb][BM + LPAD];
    __shared__ T sB[2][BKb][BN + LPAD];
    const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
    if (!in_uplo(uplo, m0 + BM - 1, n0)) return;  // tile strictly above the diagonal
    const long b = blockIdx.z;
    A += b * sa;
    B += b * sb;
    C += b * sc;
    if (kdev) K = min(K, *kdev);
    int klo = 0;
    if (tri == TRI_A_LOWER) K = min(K, m0 + BM);
    if (tri == TRI_B_UPPER) K = min(K, n0 + BN);
    if (tri == TRI_A_UPPER) klo = (m0 / BKb) * BKb;
    if (tri == TRI_B_LOWER) klo = (n0 / BKb) * BKb;
    const int t = threadIdx.x;
    T ra[EA], rb[EB];
    // op(A) tile BM x BK: A is m x K (OP_N) or K x m; op(B) tile BK x BN: B is K x n (OP_N) or n x K
    auto load = [&](int k0) {
        if constexpr (OPA == OP_N) big_load<T, BM, BKb, OPA>(ra, A, lda, m, K, m0, k0, t);
        else big_load<T, BKb, BM, OPA>(ra, A, lda, K, m, k0, m0, t);
        if constexpr (OPB == OP_N) big_load<T, BKb, BN, OPB>(rb, B, ldb, K, n, k0, n0, t);
        else big_load<T, BN, BKb, OPB>(rb, B, ldb, n, K, n0, k0, t);
    };
    auto store = [&](int buf) {
        if constexpr (OPA == OP_N) {
            constexpr int TPR = BKb / EA;
            const int mm = t / TPR, kk = (t % TPR) * EA;
#pragma unroll
            for (int i = 0; i < EA; ++i) sA[buf][kk + i][mm] = ra[i];
        } else {
            constexpr int TPR = BM / EA;
            const int kk = t / TPR, mm = (t % TPR) * EA;
#pragma unroll
            for (int i = 0; i < EA; ++i) sA[buf][kk][mm + i] = ra[i];
        }
        if constexpr (OPB == OP_N) {
            constexpr int TPR = BN / EB;
            const int kk = t / TPR, nn = (t % TPR) * EB;
#pragma unroll
            for (int i = 0; i < EB; ++i) sB[buf][kk][nn + i] = rb[i];
        } else {
            constexpr int TPR = BKb / EB;
            const int nn = t / TPR, kk = (t % TPR) * EB;
#pragma unroll
            for (int i = 0; i < EB; ++i) sB[buf][kk + i][nn] = rb[i];
        }
    };
    const int lane = t & 63, w = t >> 6, wm = w >> 1, wn = w & 1;
    const int li = lane & 15, lk = lane >> 4;
    using V = typename AccVec<T>::type;
    // complex: cre, cim and c3 hold the three real products of Acc<cplx>
    constexpr int CX = is_cplx<T>::value ? 1 : 0;
    V cre[MI][NI], cim[CX ? MI : 1][CX ? NI : 1], c3[CX ? MI : 1][CX ? NI : 1];
#pragma unroll
    for (int i = 0; i < MI; ++i)
#pragma unroll
        for (int j = 0; j < NI; ++j) {
            cre[i][j] = V{};
            if constexpr (CX) {
                cim[i][j] = V{};
                c3[i][j] = V{};
            }
        }
    if (K > klo) {
        load(klo);
        store(0);
    }
    __syncthreads();
    int cur = 0;
    for (int k0 = klo; k0 < K; k0 += BKb) {
        const bool more = k0 + BKb < K;
        if (more) load(k0 + BKb);
#pragma unroll
        for (int ks = 0; ks < BKb / 4; ++ks) {
            const int kr = ks * 4 + lk;
            T a[MI], bb[NI];
#pragma unroll
            for (int i = 0; i < MI; ++i) a[i] = sA[cur][kr][wm * WM + 16 * i + li];
#pragma unroll
            for (int j = 0; j < NI; ++j) bb[j] = sB[cur][kr][wn * WN + 16 * j + li];
#pragma unroll
            for (int i = 0; i < MI; ++i)
#pragma unroll
                for (int j = 0; j < NI; ++j) {
                    if constexpr (CX) {
                        cre[i][j] = mfma(a[i].x, bb[j].x, cre[i][j]);
                        cim[i][j] = mfma(a[i].y, bb[j].y, cim[i][j]);
                        c3[i][j] = mfma(a[i].x + a[i].y, bb[j].x + bb[j].y, c3[i][j]);
                    } else {
                        cre[i][j] = mfma(a[i], bb[j], cre[i][j]);
                    }
                }
        }
        if (more) store(cur ^ 1);
        __syncthreads();
        cur ^= 1;
    }
    // With beta != 0, one row of blocks at a time: its C values are all
    // requested before any of them is written back (a read of C placed after a
    // write to C would wait for the memory once per element, since the
    // compiler cannot tell that the addresses differ).
    const bool acc_c = beta != 0.0;
#pragma unroll
    for (int i = 0; i < MI; ++i) {
        T cv[NI][4];
        if (acc_c) {
#pragma unroll
            for (int j = 0; j < NI; ++j)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int row = m0 + wm * WM + i * 16 + out_row<T>(lane, r);
                    const int col = n0 + wn * WN + j * 16 + li;
                    const bool ok = row < m && col < n && in_uplo(uplo, row, col);
                    cv[j][r] = ok ? C[(long)row * ldc + col] : zero_<T>();
                }
        }
#pragma unroll
        for (int j = 0; j < NI; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = m0 + wm * WM + i * 16 + out_row<T>(lane, r);
                const int col = n0 + wn * WN + j * 16 + li;
                if (row < m && col < n && in_uplo(uplo, row, col)) {
                    T v;
                    if constexpr (CX) {
                        const auto p1 = cre[i][j][r], p2 = cim[i][j][r];
                        v = from_parts(p1 - p2, c3[i][j][r] - p1 - p2, (const T*)nullptr);
                    } else {
                        v = cre[i][j][r];
                    }
                    v = alpha * v;
                    if (acc_c) v += beta * cv[j][r];
                    C[(long)row * ldc + col] = v;
                }
            }
    }
}

template <typename T, int OPA, int OPB>
static void launch(hipStream_t s, int m, int n, int k, double alpha, const T* A, int lda, long sa,
                   const T* B, int ldb, long sb, double beta, T* C, int ldc, long sc, int batch,
                   const double* kscale, long sk, Uplo uplo, const int* kdev, Tri tri) {
    constexpr int BBM = Big<T>::BM, BBN = Big<T>::BN;
    const long big_tiles = (long)cdiv(m, BBM) * cdiv(n, BBN) * batch / (uplo != UPLO_FULL ? 2 : 1);
    // FP32 gains from large tiles at one round of workgroups, FP64 from two
    const long min_tiles = (sizeof(T) == 4 || std::is_same<T, cplx32>::value) ? BIG_MIN_TILES : 2 * BIG_MIN_TILES;
    if (!kscale && k >= g_big_min_k && big_tiles >= min_tiles) {
        dim3 grid(cdiv(n, BBN), cdiv(m, BBM), batch);
        hipLaunchKernelGGL((gemm_big_kernel<T, OPA, OPB>), grid, dim3(256), 0, s, m, n, k, alpha, A, lda, sa, B,
                           ldb, sb, beta, C, ldc, sc, (int)uplo, kdev, (int)tri);
        return;
    }
    dim3 grid(cdiv(n, BN), cdiv(m, BM), batch);
    hipLaunchKernelGGL((gemm_kernel<T, OPA, OPB>), grid, dim3(256), 0, s, m, n, k, alpha, A, lda, sa,
                       B, ldb, sb, beta, C, ldc, sc, kscale, sk, (int)uplo, kdev, (int)tri);
}

template <typename T>
void gemm(hipStream_t s, Op opa, Op opb, int m, int n, int k, double alpha, const T* A, int lda,
          long sa, const T* B, int ldb, long sb, double beta, T* C, int ldc, long sc, int batch,
          const double* kscale, long sk, Uplo uplo, const int* kdev, Tri tri) {
    if (m <= 0 || n <= 0 || batch <= 0) return;
#define KS_GEMM_CASE(OA, OB)                                                                      \
    if (opa == OA && opb == OB)                                                                   \
        return launch<T, OA, OB>(s, m, n, k, alpha, A, lda, sa, B, ldb, sb, beta, C, ldc, sc, batch, \
                                 kscale, sk, uplo, kdev, tri);
    KS_GEMM_CASE(OP_N, OP_N)
    KS_GEMM_CASE(OP_N, OP_T)
    KS_GEMM_CASE(OP_N, OP_C)
    KS_GEMM_CASE(OP_T, OP_N)
    KS_GEMM_CASE(OP_C, OP_N)
#undef KS_GEMM_CASE
}

template void gemm<double>(hipStream_t, Op, Op, int, int, int, double, const double*, int, long,
                           const double*, int, long, double, double*, int, long, int, const double*,
                           long, Uplo, const int*, Tri);
template void gemm<cplx>(hipStream_t, Op, Op, int, int, int, double, const cplx*, int, long,
                         const cplx*, int, long, double, cplx*, int, long, int, const double*, long,
                         Uplo, const int*, Tri);
template void gemm<float>(hipStream_t, Op, Op, int, int, int, double, const float*, int, long,
                          const float*, int, long, double, float*, int, long, int, const double*, long,
                          Uplo, const int*, Tri);
template void gemm<cplx32>(hipStream_t, Op, Op, int, int, int, double, const cplx32*, int, long,
                           const cplx32*, int, long, double, cplx32*, int, long, int, const double*, long,
                           Uplo, const int*, Tri);

// ---------------------------------------------------------------- split K
// Partial products over K chunks: P[b][z] = op(A_b)[:, Kz] op(B_b)[Kz, :] for
// chunk z of matrix b of the batch (blockIdx.z = b * nz + z).
template <typename T, int OPA, int OPB>
__global__ __launch_bounds__(256) void gemm_splitk_kernel(int m, int n, int K, int kc, int nz, const T* A,
                                                          int lda, long sa, const T* B, int ldb, long sb, T* P) {
    int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
    int z = blockIdx.z % nz, b = blockIdx.z / nz;
    int k0 = z * kc;
    int kz = min(kc, K - k0);
    A += b * sa;
    B += b * sb;
    const T* Az = (OPA == OP_N) ? A + k0 : A + (long)k0 * lda;
    const T* Bz = (OPB == OP_N) ? B + (long)k0 * ldb : B + k0;
    gemm_tile<T, OPA, OPB>(m, n, kz, 1.0, Az, lda, Bz, ldb, 0.0, P + (long)blockIdx.z * m * n, n, nullptr,
                           UPLO_FULL, m0, n0);
}

// C_b = alpha sum_z P[b][z] + beta C_b, summed in chunk order (deterministic).
template <typename T>
__global__ void splitk_reduce_kernel(int m, int n, int nz, const T* P, double alpha, double beta, T* C,
                                     int ldc, long sc) {
    long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (long)m * n) return;
    const int b = blockIdx.y;
    P += (long)b * nz * m * n;
    int i = (int)(e / n), j = (int)(e % n);
    T s = zero_<T>();
    for (int z = 0; z < nz; ++z) s += P[(long)z * m * n + e];
    T v = alpha * s;
    T* pc = C + b * sc + (long)i * ldc + j;
    if (beta != 0.0) v += beta * (*pc);
    *pc = v;
}

template <typename T>
void gemm_splitk(hipStream_t s, Op opa, Op opb, int m, int n, int k, double alpha, const T* A, int lda,
                 const T* B, int ldb, double beta, T* C, int ldc, T* work, long work_elems, int batch, long sa,
                 long sb, long sc) {
    if (m <= 0 || n <= 0 || batch <= 0) return;
    // the chunking depends on one matrix's shape only, so a batched product
    // rounds exactly like the same product on its own
    long tiles = (long)cdiv(m, BM) * cdiv(n, BN);
    int nz = (int)std::max<long>(1, std::min<long>(cdiv(1024, tiles), cdiv(k, 256)));
    while (nz > 1 && (long)nz * m * n * batch > work_elems) --nz;
    int kc = ((cdiv(k, nz) + BK - 1) / BK) * BK;
    nz = cdiv(k, kc);
    if (nz <= 1 || k <= 0) {
        gemm<T>(s, opa, opb, m, n, k, alpha, A, lda, sa, B, ldb, sb, beta, C, ldc, sc, batch);
        return;
    }
    dim3 grid(cdiv(n, BN), cdiv(m, BM), nz * batch);
#define KS_SK_CASE(OA, OB)                                                                            \
    if (opa == OA && opb == OB)                                                                      \
        hipLaunchKernelGGL((gemm_splitk_kernel<T, OA, OB>), grid, dim3(256), 0, s, m, n, k, kc, nz, A, lda, sa, \
                           B, ldb, sb, work);
    KS_SK_CASE(OP_N, OP_N)
    KS_SK_CASE(OP_C, OP_N)
    KS_SK_CASE(OP_T, OP_N)
#undef KS_SK_CASE
    long tot = (long)m * n;
    hipLaunchKernelGGL((splitk_reduce_kernel<T>), dim3(cdiv(tot, 256), batch), dim3(256), 0, s, m, n, nz, work,
                       alpha, beta, C, ldc, sc);
}

template void gemm_splitk<double>(hipStream_t, Op, Op, int, int, int, double, const double*, int, const double*,
                                  int, double, double*, int, double*, long, int, long, long, long);
template void gemm_splitk<cplx>(hipStream_t, Op, Op, int, int, int, double, const cplx*, int, const cplx*, int,
                                double, cplx*, int, cplx*, long, int, long, long, long);
template void gemm_splitk<float>(hipStream_t, Op, Op, int, int, int, double, const float*, int, const float*,
                                 int, double, float*, int, float*, long, int, long, long, long);
template void gemm_splitk<cplx32>(hipStream_t, Op, Op, int, int, int, double, const cplx32*, int,
                                  const cplx32*, int, double, cplx32*, int, cplx32*, long, int, long, long, long);

// ---------------------------------------------------------------- grouped
__global__ __launch_bounds__(256) void gemm_grouped_dc_kernel(int nm, int part, const int* lo, const int* mid,
                                                              const int* hi, const int* kk, const int* kk1,
                                                              const double* A, const double* B, double* C,
                                                              int ld) {
    const int G = blockIdx.z, g = G % nm;  // merge g of matrix G / nm of a batch
    const int l = lo[g], md = mid[g], K = kk[G], K1 = kk1[G];
    // part 0: rows l .. md-1; part 1: rows md .. hi-1; inner range [k0, k1)
    const int r0 = part == 0 ? l : md, rows = part == 0 ? md - l : hi[g] - md;
    const int k0 = (K1 >= 0 && part == 1) ? K1 : 0, k1 = (K1 >= 0 && part == 0) ? K1 : K;
    const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
    if (m0 >= rows || n0 >= K) return;
    const long base = (long)(G / nm) * ld * ld;
    gemm_tile<double, OP_N, OP_N>(rows, K, k1 - k0, 1.0, A + base + (long)r0 * ld + l + k0, ld,
                                  B + base + (long)(l + k0) * ld + l, ld, 0.0, C + base + (long)r0 * ld + l, ld,
                                  nullptr, UPLO_FULL, m0, n0);
}

void gemm_grouped_dc(hipStream_t s, int ngroups, int batch, int max_rows, const int* d_lo, const int* d_mid,
                     const int* d_hi, const int* d_kk, const int* d_kk1, const double* A, const double* B,
                     double* C, int ld) {
    if (ngroups <= 0 || max_rows <= 0 || batch <= 0) return;
    // each part covers at most max_rows - max_rows / 2 rows (the tear splits a merge in halves)
    const int half = max_rows - max_rows / 2;
    dim3 grid(cdiv(max_rows, BN), cdiv(half, BM), ngroups * batch);
    for (int part = 0; part < 2; ++part)
        hipLaunchKernelGGL(gemm_grouped_dc_kernel, grid, dim3(256), 0, s, ngroups, part, d_lo, d_mid, d_hi, d_kk,
                           d_kk1, A, B, C, ld);
}

}  // namespace ks
