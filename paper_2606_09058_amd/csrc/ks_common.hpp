// ks_common.hpp -- element types, small device helpers and the internal
// launch interface shared by the gfx950 kernels of the eigensolver.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <math.h>

#include "../../include/ks.h"

namespace ks {

// ---------------------------------------------------------------- complex
struct cplx {
    double x, y;  // re, im (layout of double complex / torch.complex128)
};

__host__ __device__ inline cplx mk(double r, double i) { cplx c; c.x = r; c.y = i; return c; }
__host__ __device__ inline cplx operator+(cplx a, cplx b) { return mk(a.x + b.x, a.y + b.y); }
__host__ __device__ inline cplx operator-(cplx a, cplx b) { return mk(a.x - b.x, a.y - b.y); }
__host__ __device__ inline cplx operator-(cplx a) { return mk(-a.x, -a.y); }
__host__ __device__ inline cplx operator*(cplx a, cplx b) {
    return mk(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__host__ __device__ inline cplx operator*(double s, cplx a) { return mk(s * a.x, s * a.y); }
__host__ __device__ inline cplx operator*(cplx a, double s) { return mk(s * a.x, s * a.y); }
__host__ __device__ inline cplx& operator+=(cplx& a, cplx b) { a.x += b.x; a.y += b.y; return a; }
__host__ __device__ inline cplx& operator-=(cplx& a, cplx b) { a.x -= b.x; a.y -= b.y; return a; }

// Uniform helpers over double and cplx.
__host__ __device__ inline double conj_(double a) { return a; }
__host__ __device__ inline cplx conj_(cplx a) { return mk(a.x, -a.y); }
__host__ __device__ inline double re_(double a) { return a; }
__host__ __device__ inline double re_(cplx a) { return a.x; }
__host__ __device__ inline double im_(double) { return 0.0; }
__host__ __device__ inline double im_(cplx a) { return a.y; }
__host__ __device__ inline double abs2_(double a) { return a * a; }
__host__ __device__ inline double abs2_(cplx a) { return a.x * a.x + a.y * a.y; }
template <typename T> __host__ __device__ inline T zero_();
template <> __host__ __device__ inline double zero_<double>() { return 0.0; }
template <> __host__ __device__ inline cplx zero_<cplx>() { return mk(0.0, 0.0); }
template <typename T> __host__ __device__ inline T from_re(double r);
template <> __host__ __device__ inline double from_re<double>(double r) { return r; }
template <> __host__ __device__ inline cplx from_re<cplx>(double r) { return mk(r, 0.0); }
__host__ __device__ inline bool finite_(double a) { return isfinite(a); }
__host__ __device__ inline bool finite_(cplx a) { return isfinite(a.x) && isfinite(a.y); }
// 1/a for complex a (Smith's algorithm not needed at these magnitudes).
__host__ __device__ inline cplx inv_(cplx a) {
    double d = a.x * a.x + a.y * a.y;
    return mk(a.x / d, -a.y / d);
}
__host__ __device__ inline double inv_(double a) { return 1.0 / a; }

// ---------------------------------------------------------------- single precision
// Storage and arithmetic type of the mixed-precision trailing updates and
// back-transform (FP32 on the matrix cores, FP32 accumulation).
struct cplx32 {
    float x, y;
};
__host__ __device__ inline cplx32 mk32(float r, float i) { cplx32 c; c.x = r; c.y = i; return c; }
__host__ __device__ inline cplx32 operator+(cplx32 a, cplx32 b) { return mk32(a.x + b.x, a.y + b.y); }
__host__ __device__ inline cplx32 operator-(cplx32 a, cplx32 b) { return mk32(a.x - b.x, a.y - b.y); }
__host__ __device__ inline cplx32 operator-(cplx32 a) { return mk32(-a.x, -a.y); }
__host__ __device__ inline cplx32 operator*(cplx32 a, cplx32 b) {
    return mk32(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__host__ __device__ inline cplx32 operator*(double s, cplx32 a) { return mk32((float)s * a.x, (float)s * a.y); }
__host__ __device__ inline cplx32 operator*(cplx32 a, double s) { return mk32((float)s * a.x, (float)s * a.y); }
__host__ __device__ inline cplx32& operator+=(cplx32& a, cplx32 b) { a.x += b.x; a.y += b.y; return a; }
__host__ __device__ inline cplx32& operator-=(cplx32& a, cplx32 b) { a.x -= b.x; a.y -= b.y; return a; }
__host__ __device__ inline float conj_(float a) { return a; }
__host__ __device__ inline cplx32 conj_(cplx32 a) { return mk32(a.x, -a.y); }
__host__ __device__ inline double re_(float a) { return a; }
__host__ __device__ inline double re_(cplx32 a) { return a.x; }
__host__ __device__ inline double im_(float) { return 0.0; }
__host__ __device__ inline double im_(cplx32 a) { return a.y; }
template <> __host__ __device__ inline float zero_<float>() { return 0.f; }
template <> __host__ __device__ inline cplx32 zero_<cplx32>() { return mk32(0.f, 0.f); }
template <> __host__ __device__ inline float from_re<float>(double r) { return (float)r; }
template <> __host__ __device__ inline cplx32 from_re<cplx32>(double r) { return mk32((float)r, 0.f); }

// FP64 <-> FP32 element conversions (round to nearest).
__host__ __device__ inline float narrow(double a) { return (float)a; }
__host__ __device__ inline cplx32 narrow(cplx a) { return mk32((float)a.x, (float)a.y); }
__host__ __device__ inline double widen(float a) { return (double)a; }
__host__ __device__ inline cplx widen(cplx32 a) { return mk((double)a.x, (double)a.y); }
__host__ __device__ inline double widen(double a) { return a; }
__host__ __device__ inline cplx widen(cplx a) { return a; }

// The FP32 counterpart of an FP64 element type.
template <typename T> struct Lo;
template <> struct Lo<double> { using type = float; };
template <> struct Lo<cplx> { using type = cplx32; };

template <typename T> struct is_cplx { static constexpr bool value = false; };
template <> struct is_cplx<cplx> { static constexpr bool value = true; };
template <> struct is_cplx<cplx32> { static constexpr bool value = true; };

// ---------------------------------------------------------------- wavefront
constexpr int WAVE = 64;

__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, WAVE);
    return v;
}
__device__ inline cplx wave_sum(cplx v) { return mk(wave_sum(v.x), wave_sum(v.y)); }
__device__ inline double shfl_xor_(double v, int m) { return __shfl_xor(v, m, WAVE); }
__device__ inline cplx shfl_xor_(cplx v, int m) { return mk(__shfl_xor(v.x, m, WAVE), __shfl_xor(v.y, m, WAVE)); }
// A store that goes through to memory (an agent-scope relaxed atomic store):
// the line is not left dirty in the writer's L2, so a reader on another XCD
// needs no write-back of it.
__device__ __forceinline__ void store_through(double* p, double v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void store_through(cplx* p, cplx v) {
    __hip_atomic_store(&p->x, v.x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(&p->y, v.y, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Select field by field: a ternary on the whole struct keeps an array of it
// out of registers.
__device__ inline double pick(bool c, double a, double b) { return c ? a : b; }
__device__ inline cplx pick(bool c, cplx a, cplx b) { return mk(c ? a.x : b.x, c ? a.y : b.y); }
__device__ inline double wave_prod(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v *= __shfl_xor(v, o, WAVE);
    return v;
}
__device__ inline double wave_max(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, WAVE));
    return v;
}
__device__ inline double wave_min(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, WAVE));
    return v;
}

// Deterministic block-wide sum of one double (fixed tree order).  `scratch`
// must hold blockDim.x/64 doubles; all threads receive the result.
__device__ inline double block_sum(double v, double* scratch) {
    v = wave_sum(v);
    int w = threadIdx.x / WAVE, l = threadIdx.x % WAVE, nw = blockDim.x / WAVE;
    __syncthreads();
    if (l == 0) scratch[w] = v;
    __syncthreads();
    double t = 0.0;
    for (int i = 0; i < nw; ++i) t += scratch[i];
    __syncthreads();
    return t;
}

// Record a device failure in the plan's info word: the first one wins.
// info layout: info[0] = status code, info[1] = detail (e.g. failing column).
__device__ inline void set_info(int* info, int code, int detail) {
    if (atomicCAS(info, 0, code) == 0) info[1] = detail;
}

// ---------------------------------------------------------------- two-stage reduction
// Half-bandwidth of the band form between the two stages, and the grouping of
// the bulge-chasing reflectors for the back-transform: the reflectors of NB
// consecutive sweeps at one step form a group, each shifted down a row from
// the previous (KB + NB - 1 rows in all).  The back-transform keeps a group's
// rows of one column in a lane's registers: NB = 32 for real data, 16 for
// complex (48 complex rows are 192 registers).
constexpr int KB = 32;
template <typename T>
struct Q2NB {
    static constexpr int v = 32;
};
template <>
struct Q2NB<cplx> {
    static constexpr int v = 16;
};
inline int q2_nb(bool complex_data) { return complex_data ? 16 : 32; }
// Panel rows per workgroup of the stage-1 panel QR (held in registers: 32 per
// thread of 512 for real data, 16 for complex; twice as many rows, in half as
// many workgroups, made the two-stage reduction slower, 190 -> 223 ms at order 6656).
__host__ __device__ constexpr int panel_rows(bool complex_data) { return complex_data ? 256 : 512; }
// Passes (wavefronts) per workgroup of the stage-2 back-transform: two per
// SIMD for real data; one for complex, whose window and coefficients need the
// accumulation registers as well.
inline int q2_passes(bool complex_data) { return complex_data ? 4 : 8; }
// Steps (tasks) of bulge-chasing sweep s of an order-n band: one per KB rows
// below the subdiagonal entry it starts from.
__host__ __device__ inline int s2_steps(int n, int s) { return (n - 1 - s + KB - 1) / KB; }

// ---------------------------------------------------------------- host side
#define KS_HIP(x)                                   \
    do {                                            \
        hipError_t e_ = (x);                        \
        if (e_ != hipSuccess) return KS_ERR_HIP;    \
    } while (0)

inline int cdiv(long a, long b) { return (int)((a + b - 1) / b); }

enum Op { OP_N = 0, OP_T = 1, OP_C = 2 };
// Part of C a product writes: all of it, its lower triangle (col <= row), or
// the lower triangle of a complex matrix seen as a real one of interleaved
// (re, im) columns (real column c is complex column c / 2: c <= 2 row + 1).
enum Uplo { UPLO_FULL = 0, UPLO_LOWER = 1, UPLO_LOWER2 = 2 };
__host__ __device__ inline bool in_uplo(int uplo, int row, int col) {
    return uplo == UPLO_FULL || (col >> (uplo - 1)) <= row;  // col <= 2 row + 1 iff col / 2 <= row
}
// Known-zero structure of an operand, used to shorten the K loop of a tile:
// op(A) lower triangular (zero for k > m), op(B) upper triangular (zero for
// k > n), op(A) upper triangular (zero for k < m).
// Triangular operand of a GEMM (op applied): the tile loop skips the K range
// where that operand is zero.
enum Tri { TRI_NONE = 0, TRI_A_LOWER = 1, TRI_B_UPPER = 2, TRI_A_UPPER = 3, TRI_B_LOWER = 4 };

// C = alpha op(A) op(B) (diag kscale between them if given) + beta C,
// row-major, for `batch` problems with element strides sa, sb, sc.
template <typename T>
void gemm(hipStream_t s, Op opa, Op opb, int m, int n, int k, double alpha, const T* A, int lda,
          long sa, const T* B, int ldb, long sb, double beta, T* C, int ldc, long sc, int batch = 1,
          const double* kscale = nullptr, long sk = 0, Uplo uplo = UPLO_FULL,
          const int* kdev = nullptr, Tri tri = TRI_NONE);

// Same product for small m x n and long K: K is cut into chunks whose partial
// products go to `work` (room for work_elems elements) and are summed in order.
template <typename T>
void gemm_splitk(hipStream_t s, Op opa, Op opb, int m, int n, int k, double alpha, const T* A, int lda,
                 const T* B, int ldb, double beta, T* C, int ldc, T* work, long work_elems, int batch = 1,
                 long sa = 0, long sb = 0, long sc = 0);

// Grouped real GEMM for the divide-and-conquer merges, C = A B with the
// merge's (rows x K) block of A at (lo, lo), (K x K) block of B and C at
// (lo, lo), row stride ld; K = kk[G] from device memory (deflation count) for
// group G = b * ngroups + g (matrix b of a batch, ld x ld consecutive).  The
// rows split at the tear mid: with kk1[G] = K1 >= 0 the first K1 columns of A
// are zero below mid and the others above it (A's columns grouped by child),
// so rows lo..mid-1 take columns 0..K1-1 only and rows mid..hi-1 columns
// K1..K-1; kk1[G] < 0 takes all K for both.
void gemm_grouped_dc(hipStream_t s, int ngroups, int batch, int max_rows, const int* d_lo, const int* d_mid,
                     const int* d_hi, const int* d_kk, const int* d_kk1, const double* A, const double* B,
                     double* C, int ld);

}  // namespace ks
