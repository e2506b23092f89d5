// ks_hetrd.hip -- blocked Householder tridiagonalisation A = Q T Q^H of the
// reduced Hermitian matrix (the "diagonalize H'" step, Part 2-4 of the
// collinear flow in Sec. 3.1 and Part 3-5 in Sec. 3.2, whose first half the
// paper identifies as bandwidth-bound matrix-vector work in Sec. 6).
//
// Lower-triangle convention: only the lower triangle of the trailing matrix is
// read and kept up to date (row-major).  Panels of NB columns; a panel starts
// with colstart (column k0 as the previous trailing update left it), then per
// column k (panel column j) two launches:
//   symv  (grid over 64 x 64 lower tiles) the tiles' share of z = A_trail x
//         with x the raw column (the one pass over the trailing matrix, the
//         memory-bound part, each lower tile read once) and of x^H A x; one
//         workgroup also reduces the raw panel products W^H x, V^H x.  It needs nothing
//         reduced beforehand, so its tiles stream from the first instruction;
//   wcol  (grid over 64-row blocks) the reflector H_k = I - tau v v^H with
//         H_k^H x = beta e_1 (beta real, so T is real for complex input) from
//         the partial |x|^2; with v = s x + c e_{k+1} (c = 1 - s x_{k+1}) the
//         product is A v = s z + c a_1 (a_1 the trailing matrix's first
//         column) and v^H A v follows from x^H A x, x^H a_1 = conj(z_{k+1})
//         and a_11; then the final W column
//         w = tau (A v - V p - W q) + alpha v, and, inside the panel, the update
//         of column k+1 with the panel's reflectors and its partial sums
//         |x|^2, W^H x, V^H x for the next reflector.
// After the panel the lower triangle of the trailing matrix takes the rank-2NB
// update A -= V W^H + W V^H as one MFMA GEMM with K = 2 NB.
// The panel buffers are stored transposed (NB columns of length n each) so
// that the per-row corrections read them coalesced, and the GEMM reads them
// as (V W)^T and conj(W V).  All reductions are fixed-order (deterministic).
#include <hip/hip_ext.h>

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

// Sum of f(i) for i = i0, i0 + step, ... < cnt, U loads at a time: the loads of
// a batch are all issued before the first is used, so a long sum costs
// cnt / (U step) memory round trips instead of cnt / step.  Fixed order.
template <int U, typename V, typename F>
__device__ inline V batched_sum(int i0, int step, int cnt, F f) {
    V acc = zero_<V>();
    for (int b = i0; b < cnt; b += U * step) {
        V v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int i = b + u * step;
            v[u] = i < cnt ? f(i) : zero_<V>();
        }
#pragma unroll
        for (int u = 0; u < U; ++u) acc += v[u];
    }
    return acc;
}

// Origin of the tiling of column k's trailing matrix (rows and columns k+1 ..
// n-1): k+1 rounded down to a 128-byte boundary of a stored row, so that the
// row segment a workgroup reads starts on a cache line and no line is shared
// by two workgroups (their L2s may be on different XCDs); the rows and columns
// below k+1 inside the first tiles are masked.  The column kernels use the
// same row blocks, so the partials of column k come in
// cdiv(n - tile_origin(k - 1), 64) blocks.
template <typename S>
__host__ __device__ constexpr int tile_origin(int k) {
    return (k + 1) & ~(int)(128 / sizeof(S) - 1);
}
template <typename S>
__host__ __device__ constexpr int partial_blocks(int n, int k) {
    return (n - tile_origin<S>(k - 1) + HETRD_TILE - 1) / HETRD_TILE;
}

// Workgroups (c, I) of the symmetric product with tiles (sch c .. ) on or
// below the diagonal, I = 0 .. nt-1, c = 0 .. I / sch, numbered row by row:
// the first index of tile row I (each of its workgroups leaves one x^H A x
// partial there).
__host__ __device__ inline int tri_index(int I, int sch) {
    const int q = I / sch;
    return I + sch * q * (q - 1) / 2 + q * (I - q * sch);
}

// Start of a panel: column k is already up to date (the trailing update of the
// previous panel has been applied), so x = A[k.., k] and the per-workgroup
// partial |x_{k+2..}|^2 is all the next reflector needs.  One wavefront per
// 64 rows; partials laid out as below ([0] of each workgroup's record), in the
// buffer of column k's parity.
template <typename T, typename S>
__global__ __launch_bounds__(64) void colstart_kernel(int n, int k, int nb, const S* A, int lda, long sA,
                                                      HetrdWork<T> hw) {
    const int z = blockIdx.z;
    A += z * sA;
    T* x = hw.x + z * hw.sx;
    T* partA = hw.partPQ + ((k & 1) ? hw.sbuf : 0) + z * hw.spart;
    int t = threadIdx.x;
    int r = tile_origin<S>(k - 1) + blockIdx.x * 64 + t;
    T c = zero_<T>();
    if (r >= k && r < n) {
        c = widen(A[(long)r * lda + k]);  // column k below the diagonal (lower storage)
        if (r == k) c = from_re<T>(re_(c));
        store_through(&x[r], c);
    }
    double a = (r < n && r >= k + 2) ? abs2_(c) : 0.0;
    a = wave_sum(a);
    if (t == 0) store_through(&partA[(long)blockIdx.x * (1 + 2 * nb)], from_re<T>(a));
}

// The reflector H_k = I - tau v v^H of column k with H_k^H x = beta e_1 from
// alpha = x_{k+1} and the per-workgroup partials of |x_{k+2..}|^2, reduced by
// one wavefront in a fixed order.  s = 1/(alpha - beta) gives v = s x below
// row k+1 (v_{k+1} = 1); a zero column below the subdiagonal with real alpha
// gives tau = 0 and s = 0.
template <typename T>
__device__ inline void reflector(const T* partA, int nA, int ld, T alpha, T& sc, T& tv, double& beta) {
    const int lane = threadIdx.x & 63;
    const double a = batched_sum<2, double>(lane, 64, nA, [&](int b) { return re_(partA[(long)b * ld]); });
    const double xn2 = wave_sum(a);
    const double ar = re_(alpha), ai = im_(alpha);
    if (xn2 == 0.0 && ai == 0.0) {
        tv = zero_<T>();
        beta = ar;
        sc = zero_<T>();
    } else {
        beta = -copysign(sqrt(ar * ar + ai * ai + xn2), ar);
        tv = make_c<T>((beta - ar) / beta, -ai / beta);
        sc = inv_(alpha - from_re<T>(beta));
    }
}

// The raw panel products W^H x and V^H x over rows k+2.. of column k, reduced
// once per column by one workgroup of NW wavefronts from the partials of the
// previous kernel: pq[2 + i] (W) and pq[2 + nb + i] (V), with pq[0] = x_{k+1}.
// For real data its last wavefront also forms the reflector of column k from
// alpha = x_{k+1} and the partial norms, into pq[2 + 2nb .. 4 + 2nb] =
// (s, tau, beta), off the column kernel's critical path (measured: 3 ms of
// 147 at N = 6656; complex data keep it in the column kernel, where the
// longer panel workgroup of their product kernel cost more than it saved).  The reflector's scale and the row
// k+1 terms are applied by the next kernel.
template <typename T, int NW>
__device__ inline void panel_products(int k, int j, int nb, const T* x, const T* partA, int nA, T* pq,
                                      T (*part)[64]) {
    static_assert(NW % 4 == 0, "wavefront count");
    const int t = threadIdx.x, lane = t & 63, g = t >> 6;
    const int ld = 1 + 2 * nb;
    const int nv = 2 * j;
    if (lane < nv) {
        const int idx = lane < j ? 1 + lane : 1 + nb + (lane - j);
        part[g][lane] = batched_sum<8, T>(g, NW, nA, [&](int b) { return partA[(long)b * ld + idx]; });
    }
    if (g == NW - 1) {  // alongside the partial sums of the other wavefronts
        const T alpha = x[k + 1];
        if constexpr (!is_cplx<T>::value) {
            T sc, tv;
            double beta;
            reflector<T>(partA, nA, ld, alpha, sc, tv, beta);
            if (lane == 0) {
                store_through(&pq[2 + 2 * nb], sc);
                store_through(&pq[3 + 2 * nb], tv);
                store_through(&pq[4 + 2 * nb], from_re<T>(beta));
            }
        }
        if (lane == 0) store_through(&pq[0], alpha);
    }
    __syncthreads();
    if (t < nv) {
        T P = zero_<T>();
        for (int q = 0; q < NW; q += 4) P += (part[q][t] + part[q + 1][t]) + (part[q + 2][t] + part[q + 3][t]);
        if (t < j) store_through(&pq[2 + t], P);
        else store_through(&pq[2 + nb + (t - j)], P);
    }
}

// Sum of r[0..R-1] over the 64 lanes for each of the R rows at once
// (reduce-scatter by halving, then a butterfly): lanes (64/R) q .. (64/R) q + 64/R - 1
// end with row q.
template <typename T>
__device__ inline T rows_lane_sum(const T (&r)[4], int lane) {
    const bool b5 = lane & 32, b4 = lane & 16;
    T w[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        T send = pick(b5, r[i], r[i + 2]);
        T keep = pick(b5, r[i + 2], r[i]);
        w[i] = keep + shfl_xor_(send, 32);
    }
    T send = pick(b4, w[0], w[1]);
    T z = pick(b4, w[1], w[0]) + shfl_xor_(send, 16);
    z += shfl_xor_(z, 8);
    z += shfl_xor_(z, 4);
    z += shfl_xor_(z, 2);
    z += shfl_xor_(z, 1);
    return z;
}
template <typename T>
__device__ inline T rows_lane_sum(const T (&r)[8], int lane) {
    const bool b5 = lane & 32, b4 = lane & 16, b3 = lane & 8;
    T w[4], u[2];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        T send = pick(b5, r[i], r[i + 4]);
        T keep = pick(b5, r[i + 4], r[i]);
        w[i] = keep + shfl_xor_(send, 32);
    }
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        T send = pick(b4, w[i], w[i + 2]);
        T keep = pick(b4, w[i + 2], w[i]);
        u[i] = keep + shfl_xor_(send, 16);
    }
    T send = pick(b3, u[0], u[1]);
    T z = pick(b3, u[1], u[0]) + shfl_xor_(send, 8);
    z += shfl_xor_(z, 4);
    z += shfl_xor_(z, 2);
    z += shfl_xor_(z, 1);
    return z;
}

template <typename T>
__device__ inline T rows_lane_sum(const T (&r)[16], int lane) {
    const bool b5 = lane & 32, b4 = lane & 16, b3 = lane & 8, b2 = lane & 4;
    T w[8], u[4], v[2];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        T send = pick(b5, r[i], r[i + 8]);
        T keep = pick(b5, r[i + 8], r[i]);
        w[i] = keep + shfl_xor_(send, 32);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        T send = pick(b4, w[i], w[i + 4]);
        T keep = pick(b4, w[i + 4], w[i]);
        u[i] = keep + shfl_xor_(send, 16);
    }
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        T send = pick(b3, u[i], u[i + 2]);
        T keep = pick(b3, u[i + 2], u[i]);
        v[i] = keep + shfl_xor_(send, 8);
    }
    T send = pick(b2, v[0], v[1]);
    T z = pick(b2, v[1], v[0]) + shfl_xor_(send, 4);
    z += shfl_xor_(z, 2);
    z += shfl_xor_(z, 1);
    return z;
}

// Trailing Hermitian matrix-vector product z = A_trail x from the LOWER
// triangle only, x the raw column k below its diagonal.  The trailing matrix
// (rows/cols k+1 .. n-1) is cut into 64 x 64 tiles; workgroup (c, I) takes
// tiles J = SCH c .. SCH c + SCH-1 (SCH, the tiles per workgroup, is a
// template parameter picked per plan) (J <= I) of tile row I.  Each of its
// threads holds one column and R rows of a tile in registers (R = 8 for real,
// 4 for complex data, so that a thread keeps two tiles' worth in flight
// within 128 registers; the next tile's loads are issued before the current
// one is used): the row sums A_IJ x_J stay in registers across the
// workgroup's tiles and are reduced over the lanes once at the end (into
// prow); the column sums A_IJ^H x_I, one per tile, go to LDS and are reduced
// over the row groups at the end (into pcol).  A diagonal tile is expanded
// from its strict lower part.  Each workgroup also leaves its share of
// x^H A x (2 Re x_I^H A_IJ x_J off the diagonal, x_I^H A_II x_I on it) in
// pvav (at tri_index(I, SCH) + c: the workgroups above the diagonal leave
// nothing), from which the next kernel gets v^H A v and so the W-column
// correction without a pass over w.
constexpr int ST = HETRD_TILE;  // tile edge

template <typename T, typename S>
struct Sy {
    static constexpr int R = 8;             // tile rows per thread
    static constexpr int NG = ST / R;       // row groups = wavefronts
    static constexpr int THREADS = 64 * NG; // 512
    // rows per load step: the thread's whole share of a tile for real data,
    // half of it for complex data, so that a step's values and products fit
    // beside the steps in flight within 128 registers (two workgroups per CU:
    // one's loads cover the other's final reductions)
    static constexpr int RS = is_cplx<T>::value ? 4 : 8;
    static constexpr int NSUB = R / RS;  // steps per tile
    // complex data reduce each step's row sums over the lanes at once (one
    // accumulator per lane and step of a tile instead of one per row); real
    // data keep a row's sum in registers across the tiles and reduce it once
    // at the end (per-step reductions measured 15-25% slower there)
    static constexpr bool LSTEP = is_cplx<T>::value;
    // slots of the register ring of steps: three (two steps in flight) with
    // FP64 storage, five (four in flight: the same bytes and registers) when
    // the trailing matrix is stored in FP32
    static constexpr int NSLOT = sizeof(S) < sizeof(T) ? 5 : 3;
};

template <typename T, typename S, int SCH>
__global__ __launch_bounds__((Sy<T, S>::THREADS), 4) void symv_kernel(int n, int k, int j, int nb, const S* A, int lda,
                                                          long sA, int nA, int nt, int nch, HetrdWork<T> hw) {
    constexpr int SY_R = Sy<T, S>::R, NG = Sy<T, S>::NG, RS = Sy<T, S>::RS, NSUB = Sy<T, S>::NSUB;
    __shared__ T vI[ST], yrow[ST];
    __shared__ T cred[SCH][NG][ST];
    __shared__ T part[NG][64];
    __shared__ double redd[NG];
    const int c = blockIdx.x, I = blockIdx.y, z = blockIdx.z;
    const int J0 = c * SCH;
    const int t = threadIdx.x;
    if (c == nch) {
        // the extra workgroup column: workgroup (nch, 0) reduces the panel
        // products from the start, alongside the tiles
        if (I == 0)
            panel_products<T, NG>(k, j, nb, hw.x + z * hw.sx,
                                  hw.partPQ + ((k & 1) ? hw.sbuf : 0) + z * hw.spart, nA, hw.pq + z * hw.spq, part);
        return;
    }
    double* pvav = hw.pvav + z * hw.spvav;
    if (J0 > I) return;
    A += z * sA;
    const T* x = hw.x + z * hw.sx;
    T* prow = hw.prow + z * hw.sprow;
    T* pcol = hw.pcol + z * hw.spcol;
    const int ntile = min(J0 + SCH, I + 1) - J0;
    const int o = k + 1;                   // first trailing row / column
    const int oa = tile_origin<S>(k);      // first row / column of the tiles
    // the row group is the wavefront index: uniform, so that the row addresses
    // stay scalar and every load takes one 32-bit lane offset
    const int col = t & 63, g = __builtin_amdgcn_readfirstlane(t >> 6);
    const int r0 = oa + I * ST + g * SY_R;  // first row of this thread
    // The workgroup's tiles pass, RS rows per thread at a time (a step),
    // through a register ring of NSLOT slots (as stored: FP64, or FP32 in the
    // mixed form): NSLOT - 1 steps' loads stay in flight while one is used.
    // The step loop is unrolled so that a step's slot is fixed at compile time
    // (moving a register whose load is in flight would wait for it), every
    // load is unconditional (indices clamped into the matrix, the value
    // replaced by zero outside it; a workgroup that reaches the diagonal
    // re-reads its last tile in place of the tiles it does not have), so that
    // each wait counts exactly the loads still needed.
    constexpr int NSLOT = Sy<T, S>::NSLOT, PD = NSLOT - 1, NSTEP = SCH * NSUB;
    S b[NSLOT][RS];
    T xv[NSLOT];  // x on the thread's column of the tiles in use or in flight
    auto xof = [&](int gi) -> T {
        const T v = x[min(gi, n - 1)];
        return (gi >= o && gi < n) ? v : zero_<T>();
    };
    auto load_step = [&](int J, int hs, S(&bt)[RS]) {
        const int gc = oa + J * ST + col;
        const bool cin = gc >= o && gc < n;
        const unsigned off = (unsigned)min(gc, n - 1) * (unsigned)sizeof(S);
#pragma unroll
        for (int q = 0; q < RS; ++q) {
            const int r = r0 + hs * RS + q;
            const char* row = (const char*)(A + (long)min(r, n - 1) * lda);
            const S v = *(const S*)(row + off);
            bt[q] = (cin && r >= o && r < n) ? v : zero_<S>();
        }
    };
    const int Jlast = J0 + ntile - 1;
    // x_I is loaded first and stored to LDS after the first steps' loads are
    // issued, so that the barrier waits for it alone (a wait counts the loads
    // in the order they were issued)
    const T xI = xof(oa + I * ST + (t & (ST - 1)));
    // (the loads of a step are issued by code written out at both places: a
    // helper taking the step as an argument kept the ring out of registers
    // until after unrolling and cost 14-38 registers)
#pragma unroll
    for (int h = 0; h < PD; ++h) {
        if (h < NSTEP) {
            load_step(min(J0 + h / NSUB, Jlast), h % NSUB, b[h % NSLOT]);
            if (h % NSUB == 0) xv[(h / NSUB) % NSLOT] = xof(oa + (J0 + h / NSUB) * ST + col);
        }
    }
    if (t < ST) vI[t] = xI;
    __syncthreads();
    // with LSTEP the row sums of each step are reduced over the lanes at once
    // (lanes LPR q .. LPR q + LPR - 1 end with row q of the step), so one
    // accumulator per lane and step of a tile carries them across the tiles;
    // otherwise one accumulator per row of the thread
    constexpr bool LSTEP = Sy<T, S>::LSTEP;
    constexpr int LPR = 64 / (LSTEP ? RS : SY_R), NACC = LSTEP ? NSUB : SY_R;
    T racc[NACC];
#pragma unroll
    for (int q = 0; q < NACC; ++q) racc[q] = zero_<T>();
    double vav = 0.0;
    T cs = zero_<T>();  // column sums of the current tile
#pragma unroll
    for (int h = 0; h < NSTEP; ++h) {
        const int s = h / NSUB, hs = h % NSUB, J = J0 + s;
        // x_I is re-read from LDS at every step rather than kept in registers
        asm volatile("" ::: "memory");
        if (h + PD < NSTEP) {  // constant once the loop is unrolled
            const int h2 = h + PD, s2 = h2 / NSUB;
            load_step(min(J0 + s2, Jlast), h2 % NSUB, b[h2 % NSLOT]);
            if (h2 % NSUB == 0) xv[s2 % NSLOT] = xof(oa + (J0 + s2) * ST + col);
        }
        if (s < ntile) {
            const S(&bc)[RS] = b[h % NSLOT];
            const T xc = xv[s % NSLOT];
            if (hs == 0) cs = zero_<T>();
            T rp[RS];
#pragma unroll
            for (int q = 0; q < RS; ++q) {
                const int rl = g * SY_R + hs * RS + q;
                const T a = widen(bc[q]);
                const T xq = vI[rl];
                if (J != I) {
                    if constexpr (LSTEP) rp[q] = a * xc;
                    else racc[hs * RS + q] += a * xc;
                    cs += conj_(a) * xq;
                } else {
                    if constexpr (LSTEP) rp[q] = pick(col <= rl, a * xc, zero_<T>());
                    else if (col <= rl) racc[hs * RS + q] += a * xc;
                    if (col < rl) cs += conj_(a) * xq;
                    if (col == rl) vav += re_(a) * abs2_(xq);
                }
            }
            if constexpr (LSTEP) racc[hs] += rows_lane_sum<T>(rp, col);
            if (hs == NSUB - 1) {
                vav += 2.0 * re_(conj_(xc) * cs);
                cred[s][g][col] = cs;
            }
        }
    }
    if constexpr (LSTEP) {
        if (col % LPR == 0) {
#pragma unroll
            for (int hs = 0; hs < NSUB; ++hs) yrow[g * SY_R + hs * RS + col / LPR] = racc[hs];
        }
    } else {
        const T rsum = rows_lane_sum<T>(racc, col);
        if (col % LPR == 0) yrow[g * SY_R + col / LPR] = rsum;
    }
    vav = wave_sum(vav);
    if (col == 0) redd[g] = vav;
    __syncthreads();  // publishes yrow, cred and the x^H A x partials
    // wavefront g reduces the column sums of tile g (SCH <= NG); the last tile
    // is the diagonal one when the workgroup reaches it, whose column sums
    // belong to z_I as well, and its wavefront also stores the row sums
    static_assert(SCH <= NG, "one wavefront per tile");
    if (g < ntile) {
        const int s = g, J = J0 + s;
        T cs = zero_<T>();
#pragma unroll
        for (int q = 0; q < NG; q += 4)
            cs += (cred[s][q][col] + cred[s][q + 1][col]) + (cred[s][q + 2][col] + cred[s][q + 3][col]);
        if (J == I) {
            store_through(&prow[((long)I * nch + c) * ST + col], yrow[col] + cs);
        } else {
            store_through(&pcol[((long)J * nt + I) * ST + col], cs);
            if (s == ntile - 1) store_through(&prow[((long)I * nch + c) * ST + col], yrow[col]);
        }
    }
    if (t == 0) {
        double vsum = 0.0;
        for (int q = 0; q < NG; ++q) vsum += redd[q];
        store_through(&pvav[tri_index(I, SCH) + c], vsum);
    }
}

// Column k of the panel (panel column j) after its symmetric product.  One
// workgroup per 64 trailing rows r = k+1+64b+l, which is exactly tile row b of
// the product, and WC_NW wavefronts that split every gather so that each is a
// single batch of loads:
//   * the reflector (s, tau, beta), for real data formed by the product
//     kernel's panel workgroup, for complex data here from alpha = x_{k+1}
//     and the partial |x_{k+2..}|^2, with p = W^H v and q = V^H v from the raw panel products
//     (row k+1, where v = 1, added here), by one wavefront;
//   * A v = s z + c a_1 with c = 1 - s alpha (v = s x + c e_{k+1}) and
//     v^H A v = |s|^2 x^H A x + 2 Re(conj(s) c x^H a_1) + |c|^2 a_11, where
//     x^H a_1 = conj(z_{k+1}) since row k+1 of A is a_1^H;
//   * alpha_w = -|tau|^2 (v^H A v - 2 Re q^H p) / 2, so
//     w = tau (A v - V p - W q) + alpha_w v is final at once (the usual
//     w += alpha_w v with alpha_w = -tau w^H v / 2, since
//     w^H v = conj(tau) v^H (A - V W^H - W V^H) v);
//   * w_r, stored with v_r in the panel;
//   * unless column k closes the panel, column k+1 is brought up to date with
//     the panel's j+1 reflectors, x_r = A[r][k+1] - V_r W_{k+1}^H - W_r V_{k+1}^H,
//     and the workgroup's partials |x_{k+3..}|^2, W^H x and V^H x are written
//     for the next reflector, into the partial buffer of column k+1's parity
//     (every workgroup reads all of column k's partials, so the two columns'
//     partials cannot share one buffer).
// Row k+1 of W (needed by every row for the update of column k+1) is
// computed by every thread in the same order, so all of them agree.
// Workgroup 0 stores d[k], e[k] = beta and tau[k].
// Partials per workgroup: [0] |x|^2, [1+i] (W^H x)_i, [1+nb+i] (V^H x)_i.
constexpr int WC_ROWS = 64;
static_assert(WC_ROWS == ST, "a row block of wcol is a tile row of the symmetric product");
// wavefronts per workgroup: 16 for real data; 8 for complex, whose larger
// per-thread state would not fit the register budget of 16
template <typename T>
struct Wc {
    static constexpr int NW = is_cplx<T>::value ? 8 : 16;
    static constexpr int MAXU = HETRD_NB / NW;  // panel columns per wavefront
    // loads in flight per lane in the reduction of z's partials: the whole
    // reduction is one round of loads up to 16 (real) or 32 (complex) per
    // lane, i.e. up to 256 tile rows of partials
    static constexpr int ZU = is_cplx<T>::value ? 32 : 16;
    static_assert(2 * HETRD_NB <= 64 && HETRD_NB % NW == 0 && NW % 4 == 0, "panel width");
};
template <typename T, typename S>
__global__ __launch_bounds__(64 * Wc<T>::NW) void wcol_kernel(int n, int k, int j, int nb, int next, const S* A,
                                                          int lda, long sA, int nt, int nch, int sch, int nA,
                                                          double* d, double* e, T* taua, HetrdWork<T> hw) {
    constexpr int WC_NW = Wc<T>::NW, WC_MAXU = Wc<T>::MAXU;
    __shared__ T sp[HETRD_NB], sq[HETRD_NB];  // p = W^H v, q = V^H v
    __shared__ T vk[HETRD_NB], wk[HETRD_NB];  // V and W on row k+1
    __shared__ T party[WC_NW][WC_ROWS], partc[WC_NW][WC_ROWS];
    __shared__ T sh[5];  // s, tau, z_{k+1}, (V p + W q)_{k+1}, alpha
    __shared__ double shd[2];  // a_11, Re q^H p
    __shared__ double red[WC_NW];
    const int t = threadIdx.x, lr = t & 63, pp = t >> 6;
    const int I = blockIdx.x, z = blockIdx.z;
    A += z * sA;
    T* x = hw.x + z * hw.sx;
    const T* pq = hw.pq + z * hw.spq;
    const T* prow = hw.prow + z * hw.sprow;
    const T* pcol = hw.pcol + z * hw.spcol;
    const double* pvav = hw.pvav + z * hw.spvav;
    T* VWt = hw.VW + z * hw.sVW;
    T* WVc = hw.WV + z * hw.sVW;
    const long ldp = 1 + 2 * nb;
    const T* partA = hw.partPQ + ((k & 1) ? hw.sbuf : 0) + z * hw.spart;
    T* partN = hw.partPQ + ((k & 1) ? 0 : hw.sbuf) + z * hw.spart;
    const int oa = tile_origin<S>(k);  // first row of the row blocks (a tile row each)
    const int r = oa + I * WC_ROWS + lr;
    const bool in = r > k && r < n;
    // every thread: its row's x and a_1 entries (column k+1 before the panel's
    // updates) and panel entries for columns i = pp, pp + WC_NW, ... < j
    T xr = zero_<T>(), ar = zero_<T>();
    if (in) {
        xr = x[r];
        ar = widen(A[(long)r * lda + k + 1]);
    }
    T vr[WC_MAXU], wr[WC_MAXU];
#pragma unroll
    for (int u = 0; u < WC_MAXU; ++u) {
        const int i = pp + WC_NW * u;
        const bool ok = in && i < j;
        vr[u] = ok ? VWt[(long)i * n + r] : zero_<T>();
        wr[u] = ok ? VWt[(long)(nb + i) * n + r] : zero_<T>();
    }
    if (pp == 1) {
        // z_{k+1} (row k+1 - oa of tile row 0)
        const int lk = k + 1 - oa;
        const T y0 = prow[lk];
        T ys = batched_sum<4, T>(1 + lr, 64, nt, [&](int I2) { return pcol[(long)I2 * ST + lk]; });
        ys = wave_sum(ys);
        if (lr == 0) sh[2] = y0 + ys;
    } else if (pp == 2) {
        // the reflector and the panel products
        // every load of this wavefront is issued before the reflector's reduction
        const int lj = min(lr, nb - 1);
        const T vkt = VWt[(long)lj * n + k + 1], wkt = VWt[(long)(nb + lj) * n + k + 1];
        const T pw = pq[2 + lj], pv = pq[2 + nb + lj];
        const T xk = x[k];
        const T alpha = pq[0];
        T sc, tv;
        double beta;
        if constexpr (is_cplx<T>::value) {
            reflector<T>(partA, nA, (int)ldp, alpha, sc, tv, beta);
        } else {  // formed by the product kernel's panel workgroup
            sc = pq[2 + 2 * nb];
            tv = pq[3 + 2 * nb];
            beta = re_(pq[4 + 2 * nb]);
        }
        T pl = zero_<T>(), ql = zero_<T>(), cs = zero_<T>();
        double cr = 0.0;
        if (lr < j) {
            pl = conj_(wkt) + sc * pw;
            ql = conj_(vkt) + sc * pv;
            vk[lr] = vkt;
            wk[lr] = wkt;
            sp[lr] = pl;
            sq[lr] = ql;
            cs = vkt * pl + wkt * ql;
            cr = re_(conj_(ql) * pl);
        }
        cs = wave_sum(cs);
        cr = wave_sum(cr);
        if (lr == 0) {
            sh[0] = sc;
            sh[1] = tv;
            sh[3] = cs;
            sh[4] = alpha;
            shd[1] = cr;
            if (I == 0) {
                d[(long)z * n + k] = re_(xk);
                e[(long)z * n + k] = beta;
                taua[(long)z * n + k] = tv;
            }
        }
    } else if (pp == 3 && lr == 0) {
        shd[0] = re_(widen(A[(long)(k + 1) * lda + k + 1]));
    }
    // z_r: row partials of tile row I (items 0 .. nc-1), then column partials
    // of the tiles below (items nc ..), split over the wavefronts
    T zr = zero_<T>();
    if (in) {
        const int nc = I / sch + 1;
        const T* pr = prow + (long)I * nch * ST + lr;
        const T* pc = pcol + ((long)I * nt + I + 1 - nc) * ST + lr;
        zr = batched_sum<Wc<T>::ZU, T>(pp, WC_NW, nc + nt - I - 1,
                               [&](int f) { return f < nc ? pr[(long)f * ST] : pc[(long)f * ST]; });
    }
    // x^H A x from the product's partials (same order in every workgroup)
    double va = batched_sum<4, double>(t, 64 * WC_NW, tri_index(nt, sch), [&](int f) { return pvav[f]; });
    va = wave_sum(va);
    if (lr == 0) red[pp] = va;
    __syncthreads();  // publishes sh, shd, sp, sq, vk, wk, red
    double xAx = 0.0;
#pragma unroll
    for (int q = 0; q < WC_NW; q += 4) xAx += (red[q] + red[q + 1]) + (red[q + 2] + red[q + 3]);
    const T sc = sh[0], tv = sh[1], z1 = sh[2], alpha = sh[4];
    const T c1 = from_re<T>(1.0) - sc * alpha;  // v_{k+1} = s alpha + c1 = 1
    const double a11 = shd[0];
    const double vAv = abs2_(sc) * xAx + 2.0 * re_(conj_(sc) * c1 * conj_(z1)) + abs2_(c1) * a11;
    const double alw = -0.5 * abs2_(tv) * (vAv - 2.0 * shd[1]);
    // W on row k+1 (where v = 1)
    const T w1 = tv * (sc * z1 + c1 * from_re<T>(a11) - sh[3]) + from_re<T>(alw);
    T cy = zero_<T>(), cx = zero_<T>();
#pragma unroll
    for (int u = 0; u < WC_MAXU; ++u) {
        const int i = pp + WC_NW * u;
        if (i < j) {
            cy += vr[u] * sp[i] + wr[u] * sq[i];
            cx += vr[u] * conj_(wk[i]) + wr[u] * conj_(vk[i]);
        }
    }
    party[pp][lr] = sc * zr - cy;
    partc[pp][lr] = cx;
    __syncthreads();
    // every wavefront forms its lanes' rows (the same values in each)
    T v = zero_<T>(), w = zero_<T>(), xn = zero_<T>();
    if (in) {
        T y = zero_<T>(), cc = zero_<T>();
#pragma unroll
        for (int q = 0; q < WC_NW; q += 4) {
            y += (party[q][lr] + party[q + 1][lr]) + (party[q + 2][lr] + party[q + 3][lr]);
            cc += (partc[q][lr] + partc[q + 1][lr]) + (partc[q + 2][lr] + partc[q + 3][lr]);
        }
        y += c1 * ar;
        v = (r == k + 1) ? from_re<T>(1.0) : sc * xr;
        w = (r == k + 1) ? w1 : tv * y + alw * v;
        xn = ar - cc - (v * conj_(w1) + w);
        if (r == k + 1) xn = from_re<T>(re_(xn));
        if (pp == 0) {
            store_through(&VWt[(long)j * n + r], v);
            store_through(&VWt[(long)(nb + j) * n + r], w);
            store_through(&WVc[(long)j * n + r], conj_(w));
            store_through(&WVc[(long)(nb + j) * n + r], conj_(v));
            if (next) store_through(&x[r], xn);
        }
    }
    if (!next) return;
    // partials for the next reflector over the panel columns 0 .. j: this
    // wavefront's columns i = pp + WC_NW u, the W and V products of all of them
    // reduced over the 64 rows at once (reduce-scatter; lane (64 / (2 WC_MAXU)) q
    // ends with product q)
    const T xe = (r >= k + 3) ? xn : zero_<T>();
    T* out = partN + (long)I * ldp;
    if (pp == 1) {
        const double a = wave_sum(abs2_(xe));
        if (lr == 0) store_through(&out[0], from_re<T>(a));
    }
    T prod[2 * WC_MAXU];
#pragma unroll
    for (int u = 0; u < WC_MAXU; ++u) {
        const int i = pp + WC_NW * u;
        const T vi = (i == j) ? v : vr[u];
        const T wi = (i == j) ? w : wr[u];
        prod[2 * u] = (i <= j) ? conj_(wi) * xe : zero_<T>();
        prod[2 * u + 1] = (i <= j) ? conj_(vi) * xe : zero_<T>();
    }
    const T ps = rows_lane_sum<T>(prod, lr);
    constexpr int LPQ = 64 / (2 * WC_MAXU);
    if (lr % LPQ == 0) {
        const int q = lr / LPQ, i = pp + WC_NW * (q >> 1);
        if (i <= j) store_through(&out[(q & 1) ? 1 + nb + i : 1 + i], ps);
    }
}

// Copy the panel's reflectors into columns k0 .. k0+jb-1 of Vall (n x n), with
// the zeros above each reflector's first entry (row k0+i+1, where it is 1):
// the panel buffer holds only the rows its column kernels wrote.
template <typename T>
__global__ void store_panel_kernel(int n, int k0, int jb, const T* VWt, long sVW, T* Vall) {
    VWt += blockIdx.z * sVW;
    Vall += blockIdx.z * (long)n * n;
    long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (long)n * jb) return;
    int i = (int)(e / n), r = (int)(e % n);
    Vall[(long)r * n + k0 + i] = r > k0 + i ? VWt[(long)i * n + r] : zero_<T>();
}

template <typename S>
__global__ void last_diag_kernel(int n, const S* A, int lda, long sA, double* d) {
    const int z = blockIdx.x;
    d[(long)z * n + n - 1] = re_(A[z * sA + (long)(n - 1) * lda + n - 1]);
}

// Launch the symmetric product of column k with sch tiles per workgroup.  With
// events (either may be null), the launch itself records them at the kernel's
// start and end (so the sampled duration is the kernel's own, without the gap
// before it).
template <typename T, typename S>
void symv_launch(hipStream_t s, int sch, int n, int k, int j, const S* A, int lda, long sA, int B, int nA,
                 const HetrdWork<T>& w, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr) {
    const int nt = cdiv(n - tile_origin<S>(k), ST), nch = cdiv(nt, sch), nb = HETRD_NB;
    // one workgroup column beyond the tiles' for the panel products
    const dim3 grid(nch + 1, nt, B), block(Sy<T, S>::THREADS);
    if (ev0 || ev1) {
        if (sch == 2)
            hipExtLaunchKernelGGL((symv_kernel<T, S, 2>), grid, block, 0, s, ev0, ev1, 0, n, k, j, nb, A, lda, sA,
                                  nA, nt, nch, w);
        else if (sch == 8)
            hipExtLaunchKernelGGL((symv_kernel<T, S, 8>), grid, block, 0, s, ev0, ev1, 0, n, k, j, nb, A, lda, sA,
                                  nA, nt, nch, w);
        else
            hipExtLaunchKernelGGL((symv_kernel<T, S, 4>), grid, block, 0, s, ev0, ev1, 0, n, k, j, nb, A, lda, sA,
                                  nA, nt, nch, w);
        return;
    }
    if (sch == 2)
        hipLaunchKernelGGL((symv_kernel<T, S, 2>), grid, block, 0, s, n, k, j, nb, A, lda, sA, nA, nt, nch, w);
    else if (sch == 8)
        hipLaunchKernelGGL((symv_kernel<T, S, 8>), grid, block, 0, s, n, k, j, nb, A, lda, sA, nA, nt, nch, w);
    else
        hipLaunchKernelGGL((symv_kernel<T, S, 4>), grid, block, 0, s, n, k, j, nb, A, lda, sA, nA, nt, nch, w);
}

// Panel buffers in the storage precision of the trailing matrix.
template <typename T, typename S>
__global__ void narrow_panel_kernel(long cnt, const T* src, long ssrc, S* dst, long sdst) {
    long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= cnt) return;
    dst[blockIdx.y * sdst + i] = narrow(src[blockIdx.y * ssrc + i]);
}

// One group of matrices of a batch that hetrd reduces on one stream.
template <typename T, typename S>
struct TrdGroup {
    hipStream_t s;
    int B;
    S* A;
    double* d;
    double* e;
    T* tau;
    T* Vall;
    HetrdWork<T> w;
};

// S: storage type of the trailing matrix A (T, or FP32 in the mixed form, where
// the rank-2NB trailing update runs on the FP32 matrix cores and everything
// else, reflectors included, stays in FP64).
// A batch of two or more matrices with a side stream in the workspace runs as
// two groups, the second half on the side stream (forked from and joined back
// to s by events), their launches issued column by column in turn: one group's
// latency-bound column kernel then runs beside the other group's product.
template <typename T, typename S>
void hetrd(hipStream_t s, int n, S* A, int lda, long sA, int batch, double* d, double* e, T* tau, T* Vall,
           HetrdWork<T>& w) {
    constexpr bool lo = !std::is_same<T, S>::value;
    const int nb = HETRD_NB;
    TrdGroup<T, S> g[2];
    int ng = 1;
    g[0] = {s, batch, A, d, e, tau, Vall, w};
    if (w.side && batch >= 2) {
        const int B0 = (batch + 1) / 2;
        g[0].B = B0;
        HetrdWork<T> w1 = w;
        w1.prof = nullptr;
        w1.VW += B0 * w.sVW;
        w1.WV += B0 * w.sVW;
        w1.x += B0 * w.sx;
        w1.partPQ += B0 * w.spart;
        w1.prow += B0 * w.sprow;
        w1.pcol += B0 * w.spcol;
        w1.pvav += B0 * w.spvav;
        w1.pq += B0 * w.spq;
        if (w.VWlo) w1.VWlo = (S*)w.VWlo + B0 * w.sVW;
        if (w.WVlo) w1.WVlo = (S*)w.WVlo + B0 * w.sVW;
        g[1] = {w.side, batch - B0, A + B0 * sA, d + (long)B0 * n, e + (long)B0 * n, tau + (long)B0 * n,
                Vall + (long)B0 * n * n, w1};
        ng = 2;
        (void)hipEventRecord(w.fork, s);
        (void)hipStreamWaitEvent(w.side, w.fork, 0);
    }
    for (int k0 = 0; k0 < n - 1; k0 += nb) {
        int jb = min(nb, n - 1 - k0);
        for (int q = 0; q < ng; ++q) {
            TrdGroup<T, S>& G = g[q];
            // The column kernels write every panel row the trailing update and
            // the next columns read (rows k+1.. of column k); only a short last
            // panel leaves panel columns unwritten that its update would read.
            if (jb < nb) {
                fill_zero<T>(G.s, G.w.VW, G.w.sVW * G.B);
                fill_zero<T>(G.s, G.w.WV, G.w.sVW * G.B);
            }
            hipLaunchKernelGGL((colstart_kernel<T, S>), dim3(partial_blocks<S>(n, k0), 1, G.B), dim3(64), 0, G.s, n,
                               k0, nb, G.A, lda, sA, G.w);
        }
        for (int j = 0; j < jb; ++j) {
            int k = k0 + j;
            int m = n - k - 1;
            const int sch = w.sch_for(k);
            int nt = cdiv(n - tile_origin<S>(k), ST), nch = cdiv(nt, sch);
            int nA = partial_blocks<S>(n, k);  // workgroups that wrote the partials of column k
            // a sampled column is timed from the start of the first group's
            // product to the end of the last group's (both groups' bytes)
            const bool smp = w.prof && w.prof->sample();
            hipEvent_t e0 = smp ? w.prof->take() : nullptr;
            hipEvent_t e1 = smp ? w.prof->take() : nullptr;
            for (int q = 0; q < ng; ++q) {
                TrdGroup<T, S>& G = g[q];
                symv_launch<T, S>(G.s, sch, n, k, j, G.A, lda, sA, G.B, nA, G.w, q == 0 ? e0 : nullptr,
                                  q == ng - 1 ? e1 : nullptr);
                hipLaunchKernelGGL((wcol_kernel<T, S>), dim3(nt, 1, G.B), dim3(64 * Wc<T>::NW), 0, G.s, n, k, j, nb,
                                   (int)(j + 1 < jb), G.A, lda, sA, nt, nch, sch, nA, G.d, G.e, G.tau, G.w);
            }
            // algorithmic bytes of a Hermitian matrix-vector product: the lower
            // triangle once, in the storage precision
            if (smp) w.prof->push(PROF_HEMV, e0, e1, (double)sizeof(S) * m * (m + 1) / 2.0 * batch);
        }
        for (int q = 0; q < ng; ++q) {
            TrdGroup<T, S>& G = g[q];
            long tot = (long)n * jb;
            hipLaunchKernelGGL((store_panel_kernel<T>), dim3(cdiv(tot, 256), 1, G.B), dim3(256), 0, G.s, n, k0, jb,
                               G.w.VW, G.w.sVW, G.Vall);
            int t0 = k0 + jb;
            if (t0 < n) {
                int mt = n - t0;
                if constexpr (lo) {
                    S* VWs = (S*)G.w.VWlo;
                    S* WVs = (S*)G.w.WVlo;
                    const long cnt = G.w.sVW;
                    hipLaunchKernelGGL((narrow_panel_kernel<T, S>), dim3(cdiv(cnt, 256), G.B), dim3(256), 0, G.s, cnt,
                                       G.w.VW, G.w.sVW, VWs, G.w.sVW);
                    hipLaunchKernelGGL((narrow_panel_kernel<T, S>), dim3(cdiv(cnt, 256), G.B), dim3(256), 0, G.s, cnt,
                                       G.w.WV, G.w.sVW, WVs, G.w.sVW);
                    gemm<S>(G.s, OP_T, OP_N, mt, mt, 2 * nb, -1.0, VWs + t0, n, G.w.sVW, WVs + t0, n, G.w.sVW, 1.0,
                            G.A + (long)t0 * lda + t0, lda, sA, G.B, nullptr, 0, UPLO_LOWER);
                } else {
                    // complex rank-2NB updates take the large tiles whenever there
                    // are enough of them (measured at 2N = 9984: 702 -> 692 ms of
                    // tridiagonalisation); real ones keep the 64 x 64 tiles (large
                    // ones were 0.8 ms slower at N = 6656)
                    GemmPolicy pol(is_cplx<T>::value ? 2 * nb : gemm_big_min_k());
                    gemm<T>(G.s, OP_T, OP_N, mt, mt, 2 * nb, -1.0, G.w.VW + t0, n, G.w.sVW, G.w.WV + t0, n, G.w.sVW,
                            1.0, G.A + (long)t0 * lda + t0, lda, sA, G.B, nullptr, 0, UPLO_LOWER);
                }
            }
        }
    }
    for (int q = 0; q < ng; ++q)
        hipLaunchKernelGGL((last_diag_kernel<S>), dim3(g[q].B), dim3(1), 0, g[q].s, n, g[q].A, lda, sA, g[q].d);
    if (ng == 2) {
        (void)hipEventRecord(w.join, w.side);
        (void)hipStreamWaitEvent(s, w.join, 0);
    }
}


// Time the symmetric product with each candidate tile count at NK columns
// spread evenly over the tridiagonalisation: ms[c] is candidate c's total
// (which estimates the whole solve's product time), and segment q of the
// columns (around sample q) takes the candidate fastest at that sample.
template <typename T, typename S>
int hetrd_tune(hipStream_t s, int n, S* A, int lda, long sA, int batch, double* d, double* e, T* tau,
               HetrdWork<T>& w, int* cand, double* ms, int reps, int* seg_first, int* seg_tiles) {
    int nc = 0;
    cand[nc++] = 2;
    cand[nc++] = 4;
    cand[nc++] = 8;
    constexpr int NK = KS_TUNE_SEGMENTS;
    int ks_[NK];
    for (int q = 0; q < NK; ++q) {
        ks_[q] = std::max(0, std::min((int)((long)q * (n - 1) / NK), n - 2));
        seg_first[q] = q == 0 ? 0 : (ks_[q - 1] + ks_[q] + 1) / 2;
        seg_tiles[q] = HETRD_SCH;
    }
    if (n < 2) {
        for (int c = 0; c < nc; ++c) ms[c] = 0.0;
        return nc;
    }
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return 0;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return 0;
    }
    // every (candidate, segment) pair is timed in TUNE_ROUNDS interleaved
    // rounds of `reps` launches and keeps its fastest round, so that a slow
    // round (clock ramp, another process) does not decide the choice
    constexpr int TUNE_ROUNDS = 3;
    float per[4][NK];
    for (int c = 0; c < nc; ++c)
        for (int q = 0; q < NK; ++q) per[c][q] = 3.0e38f;
    for (int round = 0; round < TUNE_ROUNDS; ++round)
        for (int q = 0; q < NK; ++q)
            for (int c0 = 0; c0 < nc; ++c0) {
                const int c = (c0 + round) % nc;
                const int k = ks_[q];
                const int nA = partial_blocks<S>(n, k);
                symv_launch<T, S>(s, cand[c], n, k, 0, A, lda, sA, batch, nA, w);  // warm
                (void)hipEventRecord(e0, s);
                for (int r = 0; r < reps; ++r)
                    symv_launch<T, S>(s, cand[c], n, k, 0, A, lda, sA, batch, nA, w);
                (void)hipEventRecord(e1, s);
                (void)hipEventSynchronize(e1);
                float t = 0.f;
                (void)hipEventElapsedTime(&t, e0, e1);
                per[c][q] = std::min(per[c][q], t);
            }
    for (int c = 0; c < nc; ++c) {
        float tot = 0.f;
        for (int q = 0; q < NK; ++q) tot += per[c][q];
        ms[c] = tot;
    }
    // a segment leaves the candidate fastest over all samples only for a clear
    // gain (10 %): a sample column timed alone, on a matrix already in the
    // caches, misjudges small differences (measured: a choice scattered by
    // gains of a few per cent cost 1 ms of 139 at N = 6656 against 2 tiles
    // throughout)
    int overall = 0;
    for (int c = 1; c < nc; ++c)
        if (ms[c] < ms[overall]) overall = c;
    for (int q = 0; q < NK; ++q) {
        int best = 0;
        for (int c = 1; c < nc; ++c)
            if (per[c][q] < per[best][q]) best = c;
        seg_tiles[q] = cand[per[best][q] < 0.9f * per[overall][q] ? best : overall];
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return nc;
}

template void hetrd<double, double>(hipStream_t, int, double*, int, long, int, double*, double*, double*,
                                    double*, HetrdWork<double>&);
template void hetrd<cplx, cplx>(hipStream_t, int, cplx*, int, long, int, double*, double*, cplx*, cplx*,
                                HetrdWork<cplx>&);
template void hetrd<double, float>(hipStream_t, int, float*, int, long, int, double*, double*, double*,
                                   double*, HetrdWork<double>&);
template void hetrd<cplx, cplx32>(hipStream_t, int, cplx32*, int, long, int, double*, double*, cplx*, cplx*,
                                  HetrdWork<cplx>&);
template int hetrd_tune<double, double>(hipStream_t, int, double*, int, long, int, double*, double*, double*,
                                        HetrdWork<double>&, int*, double*, int, int*, int*);
template int hetrd_tune<cplx, cplx>(hipStream_t, int, cplx*, int, long, int, double*, double*, cplx*,
                                    HetrdWork<cplx>&, int*, double*, int, int*, int*);
template int hetrd_tune<double, float>(hipStream_t, int, float*, int, long, int, double*, double*, double*,
                                       HetrdWork<double>&, int*, double*, int, int*, int*);
template int hetrd_tune<cplx, cplx32>(hipStream_t, int, cplx32*, int, long, int, double*, double*, cplx*,
                                      HetrdWork<cplx>&, int*, double*, int, int*, int*);
template void fill_zero<double>(hipStream_t, double*, long);
template void fill_zero<cplx>(hipStream_t, cplx*, long);
template void fill_zero<int>(hipStream_t, int*, long);

}  // namespace ks
