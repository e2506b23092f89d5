// ks_band.hip -- two-stage reduction of the reduced Hermitian matrix to real
// symmetric tridiagonal form, the alternative to the one-stage Householder
// tridiagonalisation of ks_hetrd.hip.  The paper attributes the limited
// speed-up of its eigen-solve to the one-stage reduction's bandwidth-bound
// matrix-vector products (Sec. 6), and its CPU runs use a two-stage solver
// (Sec. 4).  Here the dense matrix is first reduced to a band of half-bandwidth
// KB with matrix-core updates (stage 1), then the band is chased to tridiagonal
// form (stage 2); the eigenvectors take the stage-2 reflectors (q2_apply) and
// then the stage-1 ones (the compact-WY back-transform of ks_backtr.hip).
//
// Stage 1, panel k0 (columns k0 .. k0+KB-1, rows k0+KB .. n-1 below the band):
//   * QR of the m x KB panel by Householder reflectors H_j = I - tau_j v_j v_j^H
//     (H_j^H x = beta e_1, beta real), in one launch whose workgroups each hold
//     up to R panel rows in LDS.  Per column j each workgroup forms, over its
//     rows below row j, the products conj(x_i) P[i][c] of the raw column x with
//     every panel column (the norm for c = j, the reflector's application for
//     c > j, the triangular factor's V^H v_j for c < j) and row j itself; the
//     partials of all workgroups are summed in a fixed order by every workgroup
//     after an arrival counter shows all of them written, so one exchange per
//     column suffices and every workgroup forms the same reflector.
//   * The two-sided update A22 <- Q^H A22 Q with Q = I - V T V^H (T from the
//     forward recurrence of the compact-WY form): X = A22 V T,
//     W = X - V (T^H V^H X) / 2, A22 -= V W^H + W V^H, all on the matrix cores;
//     A22 is kept full (both triangles) so that A22 V is a plain product.
// Stage 2, sweep s (s = 0 .. n-2) annihilates column s below the subdiagonal
// and chases the bulge down the band in tasks of KB rows: task 0 forms the
// reflector of column s and applies it to the first diagonal block; task t
// applies the previous reflector from the right to the block below (which
// fills it), annihilates that block's first column with a new reflector
// applied from the left, and applies the new reflector to the next diagonal
// block from both sides.  Task (s, t) may start once sweep s-1 has finished
// task t+1 (the blocks they touch are then disjoint).  One wavefront runs one
// sweep; the Q wavefronts of a workgroup take consecutive sweeps and hand
// progress to each other through LDS, consecutive workgroups through a
// progress word in global memory (agent-scope release / acquire), so that only
// one sweep in Q crosses compute units.
#include "ks_internal.hpp"

#include <utility>

namespace ks {

template <typename T>
__device__ inline T mkc(double re, double im);
template <>
__device__ inline double mkc<double>(double re, double) { return re; }
template <>
__device__ inline cplx mkc<cplx>(double re, double im) { return mk(re, im); }

// Householder scalars from alpha (the entry kept) and the squared norm of the
// entries below it: tau, s = 1/(alpha - beta) (v = s x below the first entry)
// and beta, with beta real.  A zero column below a real alpha gives tau = 0.
template <typename T>
__device__ inline void house(T alpha, double xn2, T& tv, T& sc, double& beta) {
    const double ar = re_(alpha), ai = im_(alpha);
    if (xn2 == 0.0 && ai == 0.0) {
        tv = zero_<T>();
        sc = zero_<T>();
        beta = ar;
    } else {
        beta = -copysign(sqrt(ar * ar + ai * ai + xn2), ar);
        tv = mkc<T>((beta - ar) / beta, -ai / beta);
        sc = inv_(alpha - from_re<T>(beta));
    }
}

// Sum of f(g), g = 0 .. cnt-1, in index order, eight loads in flight at a time.
template <typename V, typename F>
__device__ inline V batched_sum8(int cnt, F f) {
    V acc = zero_<V>();
    for (int b = 0; b < cnt; b += 8) {
        V v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = b + u < cnt ? f(b + u) : zero_<V>();
#pragma unroll
        for (int u = 0; u < 8; ++u) acc += v[u];
    }
    return acc;
}

// Bounded waits: a wait gives up after this many polls (a few seconds), records
// the failure and raises the abort word, which every other wait also watches.
// Polls of LDS take ~0.1 us, polls of global memory ~1-2 us.
constexpr long WAIT_POLLS = 1L << 24;
constexpr long WAIT_POLLS_GLOBAL = 1L << 21;

// ---------------------------------------------------------------- stage 1
// A workgroup's panel rows live in registers: thread (rg, c) holds column c of
// rows rg, rg + PN_RG, ... (NI of them); only the pivot column of each step
// goes through LDS, once, for every thread of its row group.
template <typename T>
struct Pn {
    static constexpr int R = panel_rows(is_cplx<T>::value);  // rows per workgroup
};
constexpr int PN_THREADS = 512;
constexpr int PN_RG = PN_THREADS / KB;  // row groups

// c ? a : b by value, field by field (a select between aggregates through
// their addresses would keep a register array in memory)

template <typename T>
__global__ __launch_bounds__(PN_THREADS) void panel_qr_kernel(int n, int k0, int P, int zoff, T* A, int lda, long sA,
                                                              T* Vall, T* tau, BandWork<T> bw, int* info) {
    constexpr int R = Pn<T>::R;
    constexpr int NI = R / PN_RG;   // rows per thread
    __shared__ T xs[R];              // the pivot column (raw) of this workgroup's rows
    __shared__ T red[PN_RG][KB];
    __shared__ T tot[2 * KB];        // summed partials of column j, then row j
    __shared__ T rowj[KB];           // row j of the panel (when it is one of this workgroup's rows)
    __shared__ T Tl[KB][KB + 1];     // compact-WY factor (workgroup 0)
    __shared__ T taus[KB];
    __shared__ int go;
    const int wg = blockIdx.x, z = zoff + blockIdx.z, t = threadIdx.x;
    A += z * sA;
    Vall += z * (long)n * n;
    tau += (long)z * n;
    T* rec = bw.rec + z * bw.srec;
    int* cnt = bw.cnt + z * bw.scnt + k0 / KB;
    const int m = n - k0 - KB;
    const int nr = min(KB, m);  // reflectors of this panel
    const int i0 = wg * R;      // first panel row held here
    const int nl = min(R, m - i0);
    const int rg = t / KB, c = t % KB;
    T pr[NI];
#pragma unroll
    for (int i = 0; i < NI; ++i) {
        const int li = rg + PN_RG * i;
        const T a = A[(long)(k0 + KB + i0 + min(li, nl - 1)) * lda + k0 + c];
        pr[i] = pick(li < nl, a, zero_<T>());
    }
    if (wg == 0)
        for (int e = t; e < KB * (KB + 1); e += PN_THREADS) Tl[e / (KB + 1)][e % (KB + 1)] = zero_<T>();
    for (int j = 0; j < nr; ++j) {
        const int lj = j - i0;  // row j's index in this workgroup (if 0 <= lj < nl)
        // the pivot column to LDS, and row j (its owners: row group lj % PN_RG, slot lj / PN_RG)
        if (c == j) {
#pragma unroll
            for (int i = 0; i < NI; ++i) xs[rg + PN_RG * i] = pr[i];
        }
        if (lj >= 0 && lj < nl && rg == lj % PN_RG) {
            const int ij = lj / PN_RG;
            T v = zero_<T>();
#pragma unroll
            for (int i = 0; i < NI; ++i) v = pick(i == ij, pr[i], v);
            rowj[c] = v;
        }
        __syncthreads();
        // partials over this workgroup's rows below row j: s_c = sum conj(x_i) P[i][c]
        T s0 = zero_<T>(), s1 = zero_<T>();
#pragma unroll
        for (int i = 0; i < NI; i += 2) {
            const int li = rg + PN_RG * i;
            if (i0 + li > j && li < nl) s0 += conj_(xs[li]) * pr[i];
            if (i0 + li + PN_RG > j && li + PN_RG < nl) s1 += conj_(xs[li + PN_RG]) * pr[i + 1];
        }
        red[rg][c] = s0 + s1;
        __syncthreads();
        const int par = j & 1;
        T* myrec = rec + ((long)par * P + wg) * (2 * KB);
        if (t < 2 * KB) {
            T v;
            if (t < KB) {
                v = zero_<T>();
#pragma unroll
                for (int g = 0; g < PN_RG; g += 4) v += (red[g][t] + red[g + 1][t]) + (red[g + 2][t] + red[g + 3][t]);
            } else {
                v = (lj >= 0 && lj < nl) ? rowj[t - KB] : zero_<T>();
            }
            // a single workgroup's record is the total itself (the exchange
            // would give 0 + v, which is exact)
            if (P > 1) myrec[t] = v;
            else tot[t] = v;
        }
        __syncthreads();
        if (P > 1) {
            if (t == 0) {
                __hip_atomic_fetch_add(cnt, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
                const int want = P * (j + 1);
                long polls = 0;
                int ok = 1;
                // plain polls; one acquire once the count is reached
                while (__hip_atomic_load(cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < want) {
                    if ((++polls & 255) == 0 &&
                        (polls > WAIT_POLLS_GLOBAL ||
                         __hip_atomic_load(bw.abort_, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))) {
                        ok = 0;
                        break;
                    }
                    __builtin_amdgcn_s_sleep(1);
                }
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                if (!ok) {
                    atomicExch(bw.abort_, 1);
                    set_info(info, KS_ERR_NO_CONVERGENCE, -1);
                }
                go = ok;
            }
            __syncthreads();  // thread 0's acquire orders every thread's reads below
            if (!go) return;
            if (t < 2 * KB) {
                const T* r0 = rec + (long)par * P * (2 * KB) + t;
                tot[t] = batched_sum8<T>(P, [&](int g) { return r0[(long)g * 2 * KB]; });
            }
            __syncthreads();
        }
        // the reflector (the same in every workgroup)
        const T alpha = tot[KB + j];
        T tv, sc;
        double beta;
        house<T>(alpha, re_(tot[j]), tv, sc, beta);
        // columns c > j of rows i >= j: P[i][c] -= v_i g_c with g_c = conj(tau) (v^H P[:, c]),
        // v^H P[:, c] = P[j][c] + conj(s) s_c; column j itself becomes v (beta on row j)
        if (c > j) {
            const T gc = conj_(tv) * (tot[KB + c] + conj_(sc) * tot[c]);
            const T sg = sc * gc;
#pragma unroll
            for (int i = 0; i < NI; ++i) {
                const int gi = i0 + rg + PN_RG * i;
                if (gi == j) pr[i] -= gc;
                else if (gi > j) pr[i] -= xs[rg + PN_RG * i] * sg;
            }
        } else if (c == j) {
#pragma unroll
            for (int i = 0; i < NI; ++i) {
                const int gi = i0 + rg + PN_RG * i;
                if (gi == j) pr[i] = from_re<T>(beta);
                else if (gi > j) pr[i] = sc * pr[i];
            }
        }
        // inner products with the earlier reflectors for the triangular factor,
        // vd_q = v_q^H v_j = conj(P[j][q]) + s conj(s_q), kept in the strictly
        // lower part of Tl (Tl[j][q]); the factor itself is formed after the loop
        if (wg == 0) {
            if (t < j) Tl[j][t] = conj_(tot[KB + t]) + sc * conj_(tot[t]);
            else if (t == j) taus[j] = tv;
        }
        __syncthreads();  // xs, rowj and tot are rewritten by the next column
    }
    // upper triangular factor by rows, T[l][j] = -tau_j sum_q T[l][q] vd_q(j)
    // (q = l .. j-1); row l only reads its own entries and the stored products
    if (wg == 0 && t < nr) {
        Tl[t][t] = taus[t];
        for (int j = t + 1; j < nr; ++j) {
            T acc = zero_<T>();
            for (int q = t; q < j; ++q) acc += Tl[t][q] * Tl[j][q];
            Tl[t][j] = -(taus[j] * acc);
        }
    }
    __syncthreads();
    // R into the band (zeros below it), the reflectors into Vall (unit entry
    // explicit, zeros above) and into both V columns of the update buffer
    T* b3 = bw.buf3 + z * bw.sbuf;
#pragma unroll
    for (int i = 0; i < NI; ++i) {
        const int li = rg + PN_RG * i;
        if (li >= nl) continue;
        const int gi = i0 + li;
        const T pv = pr[i];
        const long row = k0 + KB + gi;
        A[row * lda + k0 + c] = (gi <= c) ? pv : zero_<T>();
        const T vv = c < nr ? (gi > c ? pv : (gi == c ? from_re<T>(1.0) : zero_<T>())) : zero_<T>();
        Vall[row * n + k0 + c] = vv;
        b3[(long)gi * 3 * KB + c] = vv;
        b3[(long)gi * 3 * KB + 2 * KB + c] = vv;
    }
    if (wg == 0) {
        if (t < KB) tau[k0 + t] = t < nr ? taus[t] : zero_<T>();
        T* Tf = bw.Tf + z * bw.sTf;
        for (int e = t; e < KB * KB; e += PN_THREADS) {
            const int l = e / KB, jj = e % KB;
            Tf[e] = (l <= jj && jj < nr) ? Tl[l][jj] : zero_<T>();
        }
    }
}

template <typename T>
void he2hb(hipStream_t s, int n, T* A, int lda, long sA, int batch, T* Vall, T* tau, BandWork<T>& w, int* info) {
    const long sV = (long)n * n;
    // the trailing products read the full matrix
    mirror_lower<T>(s, n, A, lda, sA, batch);
    fill_zero<T>(s, Vall, sV * batch);
    fill_zero<T>(s, tau, (long)n * batch);
    fill_zero<int>(s, w.cnt, w.scnt * batch);
    fill_zero<int>(s, w.abort_, 1);
    constexpr int R = Pn<T>::R;
    for (int k0 = 0;; k0 += KB) {
        const int m = n - k0 - KB;
        if (m <= 0) break;
        const int P = cdiv(m, R);
        // all workgroups of one launch wait for each other: a chunk of the batch
        // per launch keeps them resident together (one workgroup per compute unit)
        const int zc = std::max(1, std::min(batch, w.ncu / P));
        for (int z0 = 0; z0 < batch; z0 += zc)
            hipLaunchKernelGGL(panel_qr_kernel<T>, dim3(P, 1, std::min(zc, batch - z0)), dim3(PN_THREADS), 0, s, n, k0,
                               P, z0, A, lda, sA, Vall, tau, w, info);
        const int t0 = k0 + KB;
        T* A22 = A + (long)t0 * lda + t0;
        T* b3 = w.buf3;
        const long kk = (long)KB * KB;
        // X = A22 V; X T into the second third of buf3
        gemm_splitk<T>(s, OP_N, OP_N, m, KB, m, 1.0, A22, lda, b3, 3 * KB, 0.0, w.X, KB, w.P, w.pelems, batch, sA,
                       w.sbuf, w.sX);
        gemm<T>(s, OP_N, OP_N, m, KB, KB, 1.0, w.X, KB, w.sX, w.Tf, KB, w.sTf, 0.0, b3 + KB, 3 * KB, w.sbuf, batch);
        // M = V^H X T, N = T^H M, W = X T - V N / 2 in place
        gemm_splitk<T>(s, OP_C, OP_N, KB, KB, m, 1.0, b3, 3 * KB, b3 + KB, 3 * KB, 0.0, w.M, KB, w.P, w.pelems, batch,
                       w.sbuf, w.sbuf, kk);
        gemm<T>(s, OP_C, OP_N, KB, KB, KB, 1.0, w.Tf, KB, w.sTf, w.M, KB, kk, 0.0, w.N, KB, kk, batch);
        gemm<T>(s, OP_N, OP_N, m, KB, KB, -0.5, b3, 3 * KB, w.sbuf, w.N, KB, kk, 1.0, b3 + KB, 3 * KB, w.sbuf, batch);
        // A22 -= [V W] [W V]^H = V W^H + W V^H
        gemm<T>(s, OP_N, OP_C, m, m, 2 * KB, -1.0, b3, 3 * KB, w.sbuf, b3 + KB, 3 * KB, w.sbuf, 1.0, A22, lda, sA,
                batch);
    }
}

// ---------------------------------------------------------------- stage 2
template <typename T>
struct S2 {
    // sweeps (wavefronts) per workgroup: one per SIMD, since the chase is bound
    // by the latency of its dependent tasks, not by throughput (eight, two per
    // SIMD, ran the chase at half the speed); a workgroup takes a whole compute
    // unit (its LDS is padded at launch)
    static constexpr int Q = 4;
    static constexpr size_t LDS = sizeof(T) * (Q * KB * (KB + 1) + 4 * Q * KB) + Q * sizeof(int);
};

// LDS written by some lanes of a wavefront is read by others: keep the
// compiler from reordering across this point and wait for the LDS operations.
__device__ inline void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ inline double shfl_(double v, int src) { return __shfl(v, src, WAVE); }
__device__ inline cplx shfl_(cplx v, int src) { return mk(__shfl(v.x, src, WAVE), __shfl(v.y, src, WAVE)); }

// Reflector of a column held by the lanes of the first half (lane r holds row
// r, the second half holds zero): every lane gets tau, beta and its row's v_r
// (v_0 = 1).
template <typename T>
__device__ inline void wave_reflector(T x, int r, int h, T& tv, T& vr, double& beta) {
    const T xr = shfl_(x, r);
    const T alpha = shfl_(x, 0);
    const double xn2 = wave_sum((h == 0 && r >= 1) ? abs2_(x) : 0.0);
    T sc;
    house<T>(alpha, xn2, tv, sc, beta);
    vr = (r == 0) ? from_re<T>(1.0) : sc * xr;
}

template <typename T>
__global__ __launch_bounds__(64 * S2<T>::Q) void bulge_kernel(int n, int G, int zoff, T* A, int lda, long sA,
                                                             double* e, BandWork<T> bw, int* info) {
    constexpr int Q = S2<T>::Q;
    constexpr int HC = KB / 2;  // columns per lane: lanes r and r + 32 hold the two halves of row r
    __shared__ T tile[Q][KB][KB + 1];
    __shared__ T vsh[Q][KB], wsh[Q][KB], ush[Q][KB], vpv[Q][KB];
    __shared__ int lp[Q];  // progress of each wavefront's current sweep (key, below)
    const int g = blockIdx.x, z = zoff + blockIdx.z;
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int r = lane & (KB - 1), h = lane >> 5, cb = h * HC;
    A += z * sA;
    e += (long)z * n;
    int* gp = bw.gprog + z * bw.sgp;
    T* Vpk = bw.Vpk + z * bw.sVpk;
    T* taupk = bw.taupk + z * bw.staupk;
    const int ns = n - 1, Tmax = s2_steps(n, 0);
    // progress key of sweep s with `done` tasks finished: s (Tmax + 1) + done + 1,
    // increasing along every wavefront's work (0 = nothing yet)
    const int K = Tmax + 1;
    if (lane == 0) lp[w] = 0;
    __syncthreads();
    T (*tl)[KB + 1] = tile[w];
    for (int round = 0;; ++round) {
        const int s = (round * G + g) * Q + w;
        if (s >= ns) break;
        const int Ts = s2_steps(n, s);
        T tprev = zero_<T>();
        for (int t = 0; t < Ts; ++t) {
            if (s > 0) {
                // sweep s-1 must have finished task t+1 (or all of its tasks)
                const int thr = (s - 1) * K + min(t + 2, s2_steps(n, s - 1)) + 1;
                int ok = 1;
                if (lane == 0) {
                    long polls = 0;
                    if (w > 0) {
                        while (__hip_atomic_load(&lp[w - 1], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP) < thr) {
                            if ((++polls & 1023) == 0 &&
                                (polls > WAIT_POLLS ||
                                 __hip_atomic_load(bw.abort_, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))) {
                                ok = 0;
                                break;
                            }
                            __builtin_amdgcn_s_sleep(1);
                        }
                    } else {
                        const int pg = g == 0 ? G - 1 : g - 1;
                        while (__hip_atomic_load(&gp[pg], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < thr) {
                            if ((++polls & 63) == 0 &&
                                (polls > WAIT_POLLS_GLOBAL ||
                                 __hip_atomic_load(bw.abort_, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))) {
                                ok = 0;
                                break;
                            }
                            __builtin_amdgcn_s_sleep(1);
                        }
                    }
                    if (!ok) {
                        atomicExch(bw.abort_, 1);
                        set_info(info, KS_ERR_NO_CONVERGENCE, -2);
                    }
                }
                ok = __shfl(ok, 0, WAVE);
                if (!ok) return;
            }
            const int R0 = s + 1 + t * KB;  // first row of block t
            const int Lr = min(KB, n - R0);
            // every load of the task at once: the column or block below the
            // previous diagonal block, and the diagonal block D (its upper half
            // read as the conjugate of the lower one)
            T bv[HC], dv[HC];
            T x = zero_<T>();
            if (t == 0) {
                if (h == 0 && r < Lr) x = A[(long)(R0 + r) * lda + s];
            } else {
                const int P0 = R0 - KB;
#pragma unroll
                for (int k = 0; k < HC; ++k) bv[k] = (r < Lr) ? A[(long)(R0 + r) * lda + P0 + cb + k] : zero_<T>();
            }
#pragma unroll
            for (int k = 0; k < HC; ++k) {
                const int c = cb + k;
                T v = zero_<T>();
                if (r < Lr && c < Lr) v = c <= r ? A[(long)(R0 + r) * lda + R0 + c] : conj_(A[(long)(R0 + c) * lda + R0 + r]);
                dv[k] = v;
            }
            T tv, vr;
            double beta;
            if (t == 0) {
                // column s below the subdiagonal
                wave_reflector<T>(x, r, h, tv, vr, beta);
                if (h == 0 && r < Lr) A[(long)(R0 + r) * lda + s] = (r == 0) ? from_re<T>(beta) : zero_<T>();
                if (lane == 0) e[s] = beta;
            } else {
                // block t below the previous diagonal block (columns P0 .. P0+KB-1):
                // B <- B H_prev, then a reflector annihilating B's first column, B <- H^H B
                const int P0 = R0 - KB;
                T y = zero_<T>();
#pragma unroll
                for (int k = 0; k < HC; ++k) y += bv[k] * vpv[w][cb + k];
                y += shfl_xor_(y, 32);
                const T ty = tprev * y;
#pragma unroll
                for (int k = 0; k < HC; ++k) bv[k] -= ty * conj_(vpv[w][cb + k]);
                wave_reflector<T>(h == 0 ? bv[0] : zero_<T>(), r, h, tv, vr, beta);
                // u_c = sum_r conj(v_r) B[r][c], through the wavefront's LDS tile
#pragma unroll
                for (int k = 0; k < HC; ++k) tl[r][cb + k] = conj_(vr) * bv[k];
                wave_lds_sync();
                if (lane < KB) {
                    T u = zero_<T>();
                    for (int q = 0; q < KB; ++q) u += tl[q][lane];
                    ush[w][lane] = u;
                }
                wave_lds_sync();
                const T tvr = conj_(tv) * vr;
#pragma unroll
                for (int k = 0; k < HC; ++k) bv[k] -= tvr * ush[w][cb + k];
                if (h == 0) bv[0] = (r == 0) ? from_re<T>(beta) : zero_<T>();
                if (r < Lr)
#pragma unroll
                    for (int k = 0; k < HC; ++k) A[(long)(R0 + r) * lda + P0 + cb + k] = bv[k];
            }
            // diagonal block t: D <- H^H D H with w = tau D v - (|tau|^2 v^H D v / 2) v,
            // D -= v w^H + w v^H (the lower triangle written back)
            if (h == 0) vsh[w][r] = vr;
            wave_lds_sync();
            T p = zero_<T>();
#pragma unroll
            for (int k = 0; k < HC; ++k) p += dv[k] * vsh[w][cb + k];
            p += shfl_xor_(p, 32);
            const T w0 = tv * p;
            const T kv = wave_sum(h == 0 ? conj_(vr) * w0 : zero_<T>());
            const double alw = -0.5 * re_(conj_(tv) * kv);
            const T wr = w0 + alw * vr;
            if (h == 0) wsh[w][r] = wr;
            wave_lds_sync();
#pragma unroll
            for (int k = 0; k < HC; ++k) {
                const int c = cb + k;
                dv[k] -= vr * conj_(wsh[w][c]) + wr * conj_(vsh[w][c]);
                if (c <= r && r < Lr)
                    A[(long)(R0 + r) * lda + R0 + c] = (c == r) ? from_re<T>(re_(dv[k])) : dv[k];
            }
            // the reflector: kept for the next task, and stored for the
            // back-transform as reflector s % NB of group (s / NB, t)
            if (h == 0) vpv[w][r] = vr;
            tprev = tv;
            {
                constexpr int NB = Q2NB<T>::v;
                const int j = s / NB, q = s % NB;
                T* vg = Vpk + ((long)j * Tmax + t) * NB * KB;
                if (h == 0 && r < Lr) vg[q * KB + r] = vr;
                if (lane == 0) taupk[((long)j * Tmax + t) * NB + q] = tv;
            }
            wave_lds_sync();
            const int key = s * K + t + 2;  // t + 1 tasks done
            if (lane == 0) {
                __hip_atomic_store(&lp[w], key, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
                if (w == Q - 1) __hip_atomic_store(&gp[g], key, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
    }
}

template <typename T>
__global__ void band_diag_kernel(int n, const T* A, int lda, long sA, double* d) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x, z = blockIdx.y;
    if (i < n) d[(long)z * n + i] = re_(A[z * sA + (long)i * lda + i]);
}

template <typename T>
void hb2st(hipStream_t s, int n, T* A, int lda, long sA, int batch, double* d, double* e, BandWork<T>& w,
           int* info) {
    const int ns = n - 1;
    if (ns > 0) {
        constexpr int Q = S2<T>::Q;
        const int Tmax = s2_steps(n, 0);
        fill_zero<T>(s, w.Vpk, w.sVpk * batch);
        fill_zero<T>(s, w.taupk, w.staupk * batch);
        fill_zero<int>(s, w.gprog, w.sgp * batch);
        // about Tmax / 2 sweeps are in flight at once (each starts two tasks
        // after its predecessor and lasts up to Tmax tasks)
        int G = std::min(cdiv(ns, Q), cdiv(Tmax, 2 * Q) + 2);
        G = std::max(1, std::min(G, std::min((int)w.sgp, w.ncu)));
        const int zc = std::max(1, std::min(batch, w.ncu / G));
        // LDS above half a compute unit's: one workgroup (one wavefront per SIMD) per CU
        constexpr size_t want = 82 * 1024;
        const unsigned pad = S2<T>::LDS < want ? (unsigned)(want - S2<T>::LDS) : 0u;
        for (int z0 = 0; z0 < batch; z0 += zc)
            hipLaunchKernelGGL(bulge_kernel<T>, dim3(G, 1, std::min(zc, batch - z0)), dim3(64 * Q), pad, s, n, G, z0,
                               A, lda, sA, e, w, info);
    }
    hipLaunchKernelGGL(band_diag_kernel<T>, dim3(cdiv(n, 256), batch), dim3(256), 0, s, n, (const T*)A, lda, sA, d);
}

// ---------------------------------------------------------------- stage-2 back-transform
// X <- Q2 X with Q2 the product of the stage-2 reflectors in the order the
// chase formed them (sweep by sweep, step by step), so the last one formed acts
// first.  Reflectors on disjoint rows commute; the application goes by groups
// (j, t), the reflectors of sweeps NB j .. NB j + NB - 1 at step t (NB = Q2NB):
// rows r0 = NB j + 1 + 32 t .. r0 + NB + 30, reflector q on rows r0 + q ..
// r0 + q + 31, taken q = NB - 1 down to 0.  Pass j applies its groups
// t = 0, 1, ... in order (each overlaps the next only through reflectors of
// later sweeps), after pass j + 1: group t of pass j brings in the rows
// r0 + NB .. r0 + NB + 31, which pass j + 1 has finished once it has applied
// its own group t (they are the top 32 rows of that group, never touched
// again), and keeps the rows r0 .. r0 + NB - 1 from its previous group (for
// t = 0 they are rows no later pass touches).
//
// One lane per column of X: each lane keeps the KB + NB rows of its column's
// window in registers, so a reflector's inner product is the lane's own sum
// and no lane exchanges anything; the window moves down 32 rows per group (the
// top 32 stored, 32 new ones loaded).  A workgroup takes W consecutive passes
// of one 64-column slice, one wavefront each, handing progress on through LDS;
// the next W passes of the slice follow in another workgroup, through the
// progress word of the pass block in global memory (one word per block and
// slice, written by the block's last wavefront only: a word shared by the
// blocks would let a block's own later progress answer its wait).  Items (pass block, matrix, slice) go to the
// resident workgroups in order, so the earliest unfinished item never waits
// for a later one.
typedef __attribute__((address_space(3))) char* LdsPtr;

template <typename T>
struct Q2S {
    // passes per workgroup (q2_passes): the window takes 128 registers per lane
    // for real data (64 rows), 192 for complex (48 rows)
    static constexpr int W = is_cplx<T>::value ? 4 : 8;
};
constexpr int Q2_COLS = 64;  // columns per item, one per lane

// Between the workgroups of the stage-2 back-transform, rows go through
// memory without cache maintenance: the producing wavefront writes them
// through (agent-scope relaxed atomic stores) and waits for the stores to
// complete before it raises the progress word; the consumer polls the word and
// reads the rows with coherent (agent-scope relaxed atomic) loads.  No
// agent-scope release / acquire, whose L2 write-back and invalidation would
// stall every workgroup on the XCD.
__device__ __forceinline__ double load_coherent(const double* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ cplx load_coherent(const cplx* p) {
    return mk(__hip_atomic_load(&p->x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT),
              __hip_atomic_load(&p->y, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
}

// One reflector of a group on the lane's window: x[Q .. Q+31] -= v (tau v^H x),
// the coefficients read from LDS (broadcast).
template <int Q, int WR, typename T>
__device__ __forceinline__ void q2_reflect(T (&x)[WR], const T* vq, const T* tq) {
    T d0 = zero_<T>(), d1 = zero_<T>(), d2 = zero_<T>(), d3 = zero_<T>();
#pragma unroll
    for (int r = 0; r < KB; r += 4) {
        d0 += conj_(vq[r]) * x[Q + r];
        d1 += conj_(vq[r + 1]) * x[Q + r + 1];
        d2 += conj_(vq[r + 2]) * x[Q + r + 2];
        d3 += conj_(vq[r + 3]) * x[Q + r + 3];
    }
    const T d = tq[0] * ((d0 + d1) + (d2 + d3));
#pragma unroll
    for (int r = 0; r < KB; ++r) x[Q + r] -= vq[r] * d;
}

// The group's reflectors q = NB - 1 down to 0 (each index a constant, so that
// the window stays in registers).
template <typename T, int WR, int... Is>
__device__ __forceinline__ void q2_reflect_all(T (&x)[WR], const T* vb, const T* tb,
                                               std::integer_sequence<int, Is...>) {
    constexpr int NB = (int)sizeof...(Is);
    (q2_reflect<NB - 1 - Is, WR, T>(x, vb + (NB - 1 - Is) * KB, tb + (NB - 1 - Is)), ...);
}

template <typename T>
__global__ __launch_bounds__(64 * Q2S<T>::W) void q2_stream_kernel(int n, int J, int Tmax, int ncols, int batch,
                                                                   int G, T* X, int ldx, long sX,
                                                                   const T* __restrict__ Vpk, long sVpk,
                                                                   const T* __restrict__ taupk, long staupk,
                                                                   int* prog, int* abort_, int* info) {
    constexpr int W = Q2S<T>::W;
    constexpr int NB = Q2NB<T>::v;
    constexpr int WR = KB + NB;  // window rows (the group's KB + NB - 1, and one more)
    // the coefficients of a wavefront's current group and of its next one,
    // which direct global -> LDS loads bring in while the current one is applied
    __shared__ T vs[2][W][NB][KB];
    __shared__ T ts[2][W][NB];
    __shared__ int lp[W];  // groups finished by each wavefront's pass
    __shared__ int stop;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int nsl = (ncols + Q2_COLS - 1) / Q2_COLS;
    const long per_b = (long)batch * nsl;
    const long nitems = (long)((J + W - 1) / W) * per_b;
    for (long it = blockIdx.x; it < nitems; it += G) {
        __syncthreads();  // every wavefront is done with the previous item
        if (threadIdx.x == 0) stop = __hip_atomic_load(abort_, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (threadIdx.x < W) lp[threadIdx.x] = 0;
        __syncthreads();
        if (stop) break;
        const int b = (int)(it / per_b);
        const int z = (int)((it % per_b) / nsl), c = (int)(it % nsl);
        const int j = J - 1 - b * W - w;
        if (j < 0) continue;
        const int col = c * Q2_COLS + lane;
        const bool cv = col < ncols;
        T* Xc = X + z * sX + (cv ? col : 0);
        const T* Vz = Vpk + z * sVpk;
        const T* tz = taupk + z * staupk;
        int* pg = prog + it;  // this item's progress; item it - per_b is the previous block
        const int Ts = s2_steps(n, j * NB);
        const int Tp = j + 1 < J ? s2_steps(n, (j + 1) * NB) : 0;  // groups of pass j + 1
        // Rows past the matrix are read as its last row: their coefficients
        // are zero, so they change nothing and are never stored; lanes past
        // the last column read column 0 and store nothing.
        // stage group t's coefficients (NB x KB values, then NB taus, both
        // contiguous) into buffer t & 1 of this wavefront: 16 bytes per lane
        // per load for the coefficients, 4 for the taus
        auto stage = [&](int t) {
            const long grp = (long)j * Tmax + t;
            const char* src = (const char*)(Vz + grp * NB * KB);
            LdsPtr dst = (LdsPtr)(void*)&vs[t & 1][w][0][0];
#pragma unroll
            for (int i = 0; i < (int)(NB * KB * sizeof(T)) / 1024; ++i)
                __builtin_amdgcn_global_load_lds((const void*)(src + i * 1024 + lane * 16), dst + i * 1024, 16, 0, 0);
            static_assert(NB * sizeof(T) == 256, "taus: 4 bytes per lane");
            __builtin_amdgcn_global_load_lds((const void*)((const char*)(tz + grp * NB) + lane * 4),
                                             (LdsPtr)(void*)&ts[t & 1][w][0], 4, 0, 0);
        };
        stage(0);
        T x[WR];
#pragma unroll
        for (int k = 0; k < NB; ++k) x[k] = Xc[(long)min(j * NB + 1 + k, n - 1) * ldx];
        for (int t = 0; t < Ts; ++t) {
            const int r0 = j * NB + 1 + t * KB;
            if (Tp > 0) {
                const int need = min(t + 1, Tp);
                int ok = 1;
                if (lane == 0) {
                    long polls = 0;
                    if (w > 0) {
                        while (__hip_atomic_load(&lp[w - 1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) < need) {
                            if ((++polls & 1023) == 0 &&
                                (polls > WAIT_POLLS ||
                                 __hip_atomic_load(abort_, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))) {
                                ok = 0;
                                break;
                            }
                            __builtin_amdgcn_s_sleep(1);
                        }
                        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
                    } else {
                        // the previous block's rows were written through to memory and are
                        // read below with coherent loads: no cache invalidation needed
                        const int* pp = pg - per_b;
                        while (__hip_atomic_load(pp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < need) {
                            if ((++polls & 63) == 0 &&
                                (polls > WAIT_POLLS_GLOBAL ||
                                 __hip_atomic_load(abort_, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))) {
                                ok = 0;
                                break;
                            }
                            __builtin_amdgcn_s_sleep(1);
                        }
                        asm volatile("" ::: "memory");
                    }
                    if (!ok) {
                        atomicExch(abort_, 1);
                        set_info(info, KS_ERR_NO_CONVERGENCE, -3);
                    }
                }
                ok = __shfl(ok, 0, WAVE);
                if (!ok) break;
            }
            // the window's 32 new rows (coherent loads where another workgroup wrote them)
            if (w == 0 && b > 0) {
#pragma unroll
                for (int k = NB; k < WR; ++k) x[k] = load_coherent(Xc + (long)min(r0 + k, n - 1) * ldx);
            } else if (r0 + WR <= n) {
                const T* pl = Xc + (long)(r0 + NB) * ldx;
#pragma unroll
                for (int k = NB; k < WR; ++k) {
                    x[k] = *pl;
                    pl += ldx;
                }
            } else {
#pragma unroll
                for (int k = NB; k < WR; ++k) x[k] = Xc[(long)min(r0 + k, n - 1) * ldx];
            }
            // this group's coefficients (staged during the previous group) and the
            // new rows have arrived; the next group's coefficients go to the other
            // buffer, whose reads (the previous group's) are done
            asm volatile("" ::: "memory");
            __builtin_amdgcn_s_waitcnt(0);
            asm volatile("" ::: "memory");
            if (t + 1 < Ts) stage(t + 1);
            // an offset the compiler cannot see through, so that the coefficient
            // addresses are formed here rather than hoisted out of the group loop
            int vo = 0;
            asm volatile("" : "+v"(vo));
            q2_reflect_all<T, WR>(x, &vs[t & 1][w][0][0] + vo, &ts[t & 1][w][0] + vo,
                                  std::make_integer_sequence<int, NB>{});
            // the top 32 rows are final for this pass (all of the window after the last group)
            // (the last pass of the block writes its rows through to memory, for
            // the next block's workgroup)
            if (cv) {
                T* ps = Xc + (long)r0 * ldx;
                const int kend = t == Ts - 1 ? min(WR, n - r0) : min(KB, n - r0);
                const bool wt = w == W - 1;
                if (kend == KB && !wt) {
#pragma unroll
                    for (int k = 0; k < KB; ++k) {
                        *ps = x[k];
                        ps += ldx;
                    }
                } else {
#pragma unroll
                    for (int k = 0; k < WR; ++k) {
                        if (k < kend) {
                            if (wt) store_through(ps, x[k]);
                            else *ps = x[k];
                        }
                        ps += ldx;
                    }
                }
            }
#pragma unroll
            for (int k = 0; k < NB; ++k) x[k] = x[k + KB];
            wave_lds_sync();
            if (w == W - 1) {
                // the written-through stores complete before the progress word
                asm volatile("" ::: "memory");
                __builtin_amdgcn_s_waitcnt(0);
                asm volatile("" ::: "memory");
            }
            if (lane == 0) {
                __hip_atomic_store(&lp[w], t + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
                if (w == W - 1) __hip_atomic_store(pg, t + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
    }
}

template <typename T>
void q2_apply(hipStream_t s, int n, int batch, int ncols, T* X, int ldx, long sX, BandWork<T>& w, int* info) {
    const int ns = n - 1;
    if (ns <= 0 || ncols <= 0) return;
    const int J = cdiv(ns, Q2NB<T>::v), Tmax = s2_steps(n, 0);
    const int nsl = cdiv(ncols, Q2_COLS);
    const long nitems = (long)cdiv(J, Q2S<T>::W) * batch * nsl;
    fill_zero<int>(s, w.q2prog, nitems);
    // every workgroup resident (one per compute unit at most, by registers)
    const int G = (int)std::max(1L, std::min(nitems, (long)w.ncu));
    hipLaunchKernelGGL(q2_stream_kernel<T>, dim3(G), dim3(64 * Q2S<T>::W), 0, s, n, J, Tmax, ncols, batch, G, X,
                       ldx, sX, (const T*)w.Vpk, w.sVpk, (const T*)w.taupk, w.staupk, w.q2prog, w.abort_, info);
}

template void he2hb<double>(hipStream_t, int, double*, int, long, int, double*, double*, BandWork<double>&, int*);
template void he2hb<cplx>(hipStream_t, int, cplx*, int, long, int, cplx*, cplx*, BandWork<cplx>&, int*);
template void hb2st<double>(hipStream_t, int, double*, int, long, int, double*, double*, BandWork<double>&, int*);
template void hb2st<cplx>(hipStream_t, int, cplx*, int, long, int, double*, double*, BandWork<cplx>&, int*);
template void q2_apply<double>(hipStream_t, int, int, int, double*, int, long, BandWork<double>&, int*);
template void q2_apply<cplx>(hipStream_t, int, int, int, cplx*, int, long, BandWork<cplx>&, int*);

}  // namespace ks
