// ks_stedc.hip -- divide-and-conquer eigensolver of the real symmetric
// tridiagonal T = tridiag(e, d, e) (Cuppen's method with Gu-Eisenstat
// eigenvectors), the second half of the "diagonalize H'" step that the paper
// (Sec. 6) describes as dominated by matrix products.
//
// Tree: T is torn at the midpoints down to leaves of at most DC_LEAF rows; the
// tear at m uses T = diag(T1', T2') + |b| w w^T with b = e[m-1],
// w = e_{m-1} + sign(b) e_m and d[m-1], d[m] reduced by |b|.
// Leaves: parallel cyclic Jacobi in LDS (one workgroup per leaf).
// Merge of (D1, Q1), (D2, Q2) into D + rho z z^T, z = [Q1 row m-1;
// sign(b) Q2 row m] / sqrt(2), rho = 2|b|:
//   deflate  sort (D, z); drop |rho z_i| <= tol; rotate away z of nearly equal
//            pairs (tol = 8 eps max(|D|, |z|));
//   secular  one wavefront per root of 1 + rho sum z_i^2/(d_i - x) = 0, origin
//            at the nearer pole, safeguarded two-pole rational iteration with
//            bisection fallback;
//   vectors  z_hat from the computed roots (Gu-Eisenstat), u_j ~ z_hat/(d - x_j);
//   product  Q_new = Q_perm U on the matrix cores (grouped GEMM);
//   order    rank sort of the merged eigenvalues, columns permuted to match.
// Every size that depends on deflation stays on the device: kernels are
// launched for the undeflated size and idle workgroups exit, so the whole
// solve is enqueued without a host synchronisation.
// A batch of tridiagonals of one order shares the tree and every launch: the
// matrix index b is folded into the merge (group) index, G = b * nm + g, and
// selects the matrix's slices of the vectors (stride n) and matrices (n^2).
#include "ks_internal.hpp"

namespace ks {

constexpr double DEPS = 1.1102230246251565e-16;  // unit roundoff 2^-53

// The slices of the merge work arrays that belong to matrix b of a batch
// (kk, nrot and rho are indexed by the folded group index instead).
__device__ inline DcWork dc_slice(DcWork w, int b, int n) {
    long o = (long)b * n;
    w.dw += o;
    w.ds += o;
    w.zs += o;
    w.perm += o;
    w.ndl += o;
    w.dfl += o;
    w.dfval += o;
    w.dnd += o;
    w.znd += o;
    w.rot_idx += 2 * o;
    w.rot_cs += 2 * o;
    w.orig += o;
    w.tau += o;
    w.zhat += o;
    w.cinv += o;
    w.fval += o;
    w.fsrc += o;
    w.gpos += o;
    return w;
}

// ---------------------------------------------------------------- setup
// dw = d with |e[m-1]| taken off both neighbours of every tear m; the tears are
// exactly the leaf starts > 0 (sorted), so each entry looks itself up.
__device__ inline bool is_leaf_start(const int* leaf_lo, int nleaf, int i) {
    int a = 0, b = nleaf;
    while (a < b) {
        int h = (a + b) >> 1;
        if (leaf_lo[h] < i) a = h + 1;
        else b = h;
    }
    return a < nleaf && leaf_lo[a] == i;
}

__global__ void dc_init_kernel(int n, const double* d, const double* e, const int* leaf_lo, int nleaf,
                               double* dw) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const long o = (long)blockIdx.y * n;
    d += o;
    e += o;
    dw += o;
    double v = d[i];
    if (i > 0 && is_leaf_start(leaf_lo, nleaf, i)) v -= fabs(e[i - 1]);
    if (i + 1 < n && is_leaf_start(leaf_lo, nleaf, i + 1)) v -= fabs(e[i]);
    dw[i] = v;
}

// ---------------------------------------------------------------- leaves
// Parallel cyclic Jacobi on the dense leaf (size <= DC_LEAF) in LDS.
__global__ __launch_bounds__(64) void dc_leaf_kernel(int n, const int* leaf_lo, const int* leaf_hi,
                                                     const double* dw, const double* e, double* lam,
                                                     double* Z, int* info, int max_sweeps) {
    constexpr int L = DC_LEAF;
    __shared__ double A[L][L + 1];
    __shared__ double VT[L][L + 1];
    __shared__ double rc[L / 2], rs[L / 2], rpp[L / 2], rqq[L / 2];
    __shared__ int rp[L / 2], rq[L / 2], ract[L / 2];
    __shared__ int any_rot;
    __shared__ double w[L];
    __shared__ int idx[L];
    {
        const long o = (long)blockIdx.y * n;
        dw += o;
        e += o;
        lam += o;
        Z += o * n;
    }
    int lo = leaf_lo[blockIdx.x], hi = leaf_hi[blockIdx.x];
    int s = hi - lo;
    int t = threadIdx.x;
    for (int q = t; q < L * L; q += 64) {
        int i = q / L, j = q % L;
        double v = 0.0;
        if (i < s && j < s) {
            if (i == j) v = dw[lo + i];
            else if (j == i + 1) v = e[lo + i];
            else if (i == j + 1) v = e[lo + j];
        }
        A[i][j] = v;
        VT[i][j] = (i == j) ? 1.0 : 0.0;
    }
    __syncthreads();
    double nrm = 0.0;
    for (int i = 0; i < s; ++i) nrm += A[i][i] * A[i][i] + (i + 1 < s ? 2.0 * A[i][i + 1] * A[i][i + 1] : 0.0);
    nrm = sqrt(nrm);
    double tol = 1e-18 * nrm;
    int m = s + (s & 1);
    int np = m / 2;
    int sweep = 0;
    for (; sweep < max_sweeps && s > 1; ++sweep) {
        if (t == 0) any_rot = 0;
        __syncthreads();
        for (int r = 0; r < m - 1; ++r) {
            if (t < np) {
                int a = (t == 0) ? 0 : 1 + ((t - 1 + r) % (m - 1));
                int b = 1 + ((m - 2 - t + r) % (m - 1));
                int p = min(a, b), q = max(a, b);
                rp[t] = p;
                rq[t] = q;
                ract[t] = 0;
                if (q < s) {
                    double apq = A[p][q], app = A[p][p], aqq = A[q][q];
                    if (fabs(apq) > tol) {
                        double tau = (aqq - app) / (2.0 * apq);
                        double tt = (tau >= 0.0) ? 1.0 / (tau + sqrt(1.0 + tau * tau))
                                                 : -1.0 / (-tau + sqrt(1.0 + tau * tau));
                        double c = 1.0 / sqrt(1.0 + tt * tt);
                        rc[t] = c;
                        rs[t] = tt * c;
                        rpp[t] = app - tt * apq;
                        rqq[t] = aqq + tt * apq;
                        ract[t] = 1;
                        any_rot = 1;
                    } else {
                        A[p][q] = 0.0;
                        A[q][p] = 0.0;
                    }
                }
            }
            __syncthreads();
            // rows: A <- J^T A ; VT <- J^T VT
            for (int q = t; q < np * L; q += 64) {
                int pi = q / L, col = q % L;
                if (!ract[pi] || col >= s) continue;
                int p = rp[pi], qq = rq[pi];
                double c = rc[pi], sn = rs[pi];
                double x = A[p][col], y = A[qq][col];
                A[p][col] = c * x - sn * y;
                A[qq][col] = sn * x + c * y;
                x = VT[p][col];
                y = VT[qq][col];
                VT[p][col] = c * x - sn * y;
                VT[qq][col] = sn * x + c * y;
            }
            __syncthreads();
            // columns: A <- A J
            for (int q = t; q < np * L; q += 64) {
                int pi = q / L, row = q % L;
                if (!ract[pi] || row >= s) continue;
                int p = rp[pi], qq = rq[pi];
                double c = rc[pi], sn = rs[pi];
                double x = A[row][p], y = A[row][qq];
                A[row][p] = c * x - sn * y;
                A[row][qq] = sn * x + c * y;
            }
            __syncthreads();
            if (t < np && ract[t]) {
                int p = rp[t], qq = rq[t];
                A[p][p] = rpp[t];
                A[qq][qq] = rqq[t];
                A[p][qq] = 0.0;
                A[qq][p] = 0.0;
            }
            __syncthreads();
        }
        if (!any_rot) break;
    }
    if (sweep >= max_sweeps && s > 1 && t == 0) set_info(info, KS_ERR_NO_CONVERGENCE, 1);
    // stable ascending rank sort of the diagonal
    if (t < s) w[t] = A[t][t];
    __syncthreads();
    if (t < s) {
        int rk = 0;
        for (int q = 0; q < s; ++q) rk += (w[q] < w[t]) || (w[q] == w[t] && q < t);
        idx[rk] = t;
    }
    __syncthreads();
    if (t < s) lam[lo + t] = w[idx[t]];
    for (int q = t; q < s * s; q += 64) {
        int row = q / s, col = q % s;
        Z[(long)(lo + row) * n + lo + col] = VT[idx[col]][row];
    }
}

// ---------------------------------------------------------------- merges
// The deflation test of two consecutive kept entries (d_p, z_p), (d_j, z_j):
// the Givens rotation (c, s) with c = z_j / tau, s = -z_p / tau, tau =
// hypot(z_p, z_j), zeroes z_p; the pair deflates if the off-diagonal it
// leaves, (d_j - d_p) c s, is at most tol in magnitude.
__device__ inline bool deflate_pair(double dp, double zp, double dj, double zj, double tol, double* c = nullptr,
                                    double* s = nullptr, double* t = nullptr) {
    const double tau = hypot(zj, zp);
    const double cs = zj / tau, sn = -zp / tau;
    if (c) {
        *c = cs;
        *s = sn;
        *t = tau;
    }
    return fabs((dj - dp) * cs * sn) <= tol;
}

// One workgroup per merge: form (D, z), merge-sort, deflate.  With use_lds the
// launch provides K0 doubles of dynamic LDS and the two sorted lists are
// staged there for the merge's binary searches.
constexpr int DEFLATE_LDS_MAX = 8192;  // 64 KB of dynamic LDS
__global__ __launch_bounds__(256) void dc_deflate_kernel(int n, int nm, const int* mlo, const int* mmid,
                                                         const int* mhi, const double* e,
                                                         const double* lam, const double* Z,
                                                         DcWork w, int use_lds) {
    __shared__ double sd[64], sz[64];
    extern __shared__ double slam[];
    const int G = blockIdx.x, g = G % nm, bm = G / nm;
    w = dc_slice(w, bm, n);
    e += (long)bm * n;
    lam += (long)bm * n;
    Z += (long)bm * n * n;
    int lo = mlo[g], mid = mmid[g], hi = mhi[g];
    int K0 = hi - lo, n1 = mid - lo;
    int t = threadIdx.x;
    double b = e[mid - 1];
    double rho = 2.0 * fabs(b);
    double sg = (b >= 0.0) ? 1.0 : -1.0;
    const double rs2 = 0.70710678118654752440;
    double dmax = 0.0, zmax = 0.0;
    if (use_lds) {
        for (int c = t; c < K0; c += blockDim.x) slam[c] = lam[lo + c];
        __syncthreads();
    }
    const double* L = use_lds ? (const double*)slam : lam + lo;  // L[q] = lam[lo + q]
    for (int c = t; c < K0; c += blockDim.x) {
        double D = L[c];
        double z = (c < n1) ? Z[(long)(mid - 1) * n + lo + c] : sg * Z[(long)mid * n + lo + c];
        z *= rs2;
        // rank in the merged order (ties: first list first)
        int rank;
        if (c < n1) {
            int a = 0, bb = K0 - n1;  // count of second-list entries < D
            while (a < bb) {
                int h = (a + bb) >> 1;
                if (L[n1 + h] < D) a = h + 1;
                else bb = h;
            }
            rank = c + a;
        } else {
            int a = 0, bb = n1;  // count of first-list entries <= D
            while (a < bb) {
                int h = (a + bb) >> 1;
                if (L[h] <= D) a = h + 1;
                else bb = h;
            }
            rank = (c - n1) + a;
        }
        w.perm[lo + rank] = c;
        w.ds[lo + rank] = D;
        w.zs[lo + rank] = z;
        dmax = fmax(dmax, fabs(D));
        zmax = fmax(zmax, fabs(z));
    }
    // block max (fixed order)
    dmax = wave_max(dmax);
    zmax = wave_max(zmax);
    __shared__ double mx[2][4];
    if ((t & 63) == 0) {
        mx[0][t >> 6] = dmax;
        mx[1][t >> 6] = zmax;
    }
    __threadfence_block();
    __syncthreads();
    double tol = 0.0;
    for (int i = 0; i < 4; ++i) tol = fmax(tol, fmax(mx[0][i], mx[1][i]));
    tol *= 8.0 * DEPS;
    // Deflation in merged order: entry j deflates if rho |z_j| <= tol, and two
    // consecutive kept entries are rotated together (the rotated one carrying
    // on) if the Givens rotation that zeroes the first one's z leaves an
    // off-diagonal |(d_j - d_p) c s| <= tol.  Without such a pair the outcome
    // is a stable partition into deflated and kept entries, which all threads
    // form at once from contiguous chunks; a merge with a pair takes the
    // sequential scan below (same tests, same arithmetic).
    {
        __shared__ int cnt_d[256], cnt_k[256], cnt_k1[256], last_k[256];
        __shared__ int any_pair;
        const int per = (K0 + (int)blockDim.x - 1) / (int)blockDim.x;
        const int c0 = min(K0, t * per), c1 = min(K0, c0 + per);
        int nd = 0, nk = 0, nk1 = 0, firstk = -1, lastk = -1;
        bool pair = false;
        double dp = 0.0, zp = 0.0;
        for (int j = c0; j < c1; ++j) {
            const double dj = w.ds[lo + j], zj = w.zs[lo + j];
            if (rho * fabs(zj) <= tol) {
                ++nd;
                continue;
            }
            if (lastk >= 0 && deflate_pair(dp, zp, dj, zj, tol)) pair = true;
            if (firstk < 0) firstk = j;
            lastk = j;
            dp = dj;
            zp = zj;
            ++nk;
            nk1 += w.perm[lo + j] < n1;
        }
        cnt_d[t] = nd;
        cnt_k[t] = nk;
        cnt_k1[t] = nk1;
        last_k[t] = lastk;
        if (t == 0) any_pair = 0;
        __syncthreads();
        if (firstk >= 0) {
            // the pair across the chunk boundary: the last kept entry before
            int pk = -1;
            for (int q = t - 1; q >= 0 && pk < 0; --q) pk = last_k[q];
            if (pk >= 0 && deflate_pair(w.ds[lo + pk], w.zs[lo + pk], w.ds[lo + firstk], w.zs[lo + firstk], tol))
                pair = true;
        }
        if (pair) any_pair = 1;
        __syncthreads();
        if (!any_pair) {
            // without rotations every kept column belongs to one child: the
            // merge product takes them grouped by child (first child's first,
            // each group in secular order), which halves its flops
            int od = 0, ok = 0, ok1 = 0, K1 = 0;
            for (int q = 0; q < (int)blockDim.x; ++q) {
                if (q < t) {
                    od += cnt_d[q];
                    ok += cnt_k[q];
                    ok1 += cnt_k1[q];
                }
                K1 += cnt_k1[q];
            }
            for (int j = c0; j < c1; ++j) {
                const double dj = w.ds[lo + j], zj = w.zs[lo + j];
                if (rho * fabs(zj) <= tol) {
                    w.dfl[lo + od] = j;
                    w.dfval[lo + od] = dj;
                    ++od;
                } else {
                    const bool first = w.perm[lo + j] < n1;
                    w.ndl[lo + ok] = j;
                    w.dnd[lo + ok] = dj;
                    w.znd[lo + ok] = zj;
                    w.gpos[lo + ok] = first ? ok1 : K1 + (ok - ok1);
                    ok1 += first;
                    ++ok;
                }
            }
            if (t == (int)blockDim.x - 1) {
                w.kk[G] = ok;
                w.kk1[G] = K1;
                w.nrot[G] = 0;
                w.rho[G] = rho;
            }
            return;
        }
    }
    // sequential deflation scan, streamed through LDS in chunks of 64
    if (t < 64) {
        int K = 0, nd = 0, nrot = 0, pj = -1;
        double dpj = 0.0, zpj = 0.0;
        for (int base = 0; base < K0; base += 64) {
            int cnt = min(64, K0 - base);
            if (t < cnt) {
                sd[t] = w.ds[lo + base + t];
                sz[t] = w.zs[lo + base + t];
            }
            __threadfence_block();
            if (t == 0) {
                for (int q = 0; q < cnt; ++q) {
                    int jj = base + q;
                    double dj = sd[q], zj = sz[q];
                    if (rho * fabs(zj) <= tol) {
                        w.dfl[lo + nd] = jj;
                        w.dfval[lo + nd] = dj;
                        ++nd;
                        continue;
                    }
                    if (pj < 0) {
                        pj = jj;
                        dpj = dj;
                        zpj = zj;
                        continue;
                    }
                    double cs, sn, tau;
                    if (deflate_pair(dpj, zpj, dj, zj, tol, &cs, &sn, &tau)) {
                        w.rot_idx[2 * (lo + nrot)] = pj;
                        w.rot_idx[2 * (lo + nrot) + 1] = jj;
                        w.rot_cs[2 * (lo + nrot)] = cs;
                        w.rot_cs[2 * (lo + nrot) + 1] = sn;
                        ++nrot;
                        double tp = dpj * cs * cs + dj * sn * sn;
                        dj = dpj * sn * sn + dj * cs * cs;
                        w.dfl[lo + nd] = pj;
                        w.dfval[lo + nd] = tp;
                        ++nd;
                        pj = jj;
                        dpj = dj;
                        zpj = tau;
                    } else {
                        w.ndl[lo + K] = pj;
                        w.dnd[lo + K] = dpj;
                        w.znd[lo + K] = zpj;
                        ++K;
                        pj = jj;
                        dpj = dj;
                        zpj = zj;
                    }
                }
            }
            __threadfence_block();
        }
        if (t == 0) {
            if (pj >= 0) {
                w.ndl[lo + K] = pj;
                w.dnd[lo + K] = dpj;
                w.znd[lo + K] = zpj;
                ++K;
            }
            w.kk[G] = K;
            w.kk1[G] = -1;  // rotations may mix the children's columns
            w.nrot[G] = nrot;
            w.rho[G] = rho;
        }
    }
}

// Apply the deflation rotations to the merge's columns of Z, one thread per row.
__global__ __launch_bounds__(256) void dc_rotate_kernel(int n, int nm, const int* mlo, const int* mhi,
                                                        DcWork w, double* Z) {
    const int G = blockIdx.y, g = G % nm, bm = G / nm;
    w = dc_slice(w, bm, n);
    Z += (long)bm * n * n;
    int lo = mlo[g], hi = mhi[g];
    int r = lo + blockIdx.x * blockDim.x + threadIdx.x;
    int nr = w.nrot[G];
    if (r >= hi || nr == 0) return;
    double* zr = Z + (long)r * n + lo;
    for (int q = 0; q < nr; ++q) {
        int pj = w.rot_idx[2 * (lo + q)], jj = w.rot_idx[2 * (lo + q) + 1];
        double c = w.rot_cs[2 * (lo + q)], s = w.rot_cs[2 * (lo + q) + 1];
        int cp = w.perm[lo + pj], cj = w.perm[lo + jj];
        double x = zr[cp], y = zr[cj];
        zr[cp] = c * x + s * y;
        zr[cj] = c * y - s * x;
    }
}

// Secular equation: one wavefront per root.
__global__ __launch_bounds__(256) void dc_secular_kernel(int n, int nm, const int* mlo, DcWork w, int* info,
                                                         int max_iter) {
    const int G = blockIdx.y, g = G % nm;
    w = dc_slice(w, G / nm, n);
    int lo = mlo[g];
    int K = w.kk[G];
    int jr = blockIdx.x * 4 + (threadIdx.x >> 6);
    int lane = threadIdx.x & 63;
    if (jr >= K) return;
    const double* d = w.dnd + lo;
    const double* z = w.znd + lo;
    double rho = w.rho[G];
    if (K == 1) {
        if (lane == 0) {
            w.orig[lo] = 0;
            w.tau[lo] = rho * z[0] * z[0];
        }
        return;
    }
    int o;
    double blo, bhi;
    if (jr < K - 1) {
        double D = d[jr + 1] - d[jr];
        double f = 0.0;
        for (int i = lane; i < K; i += 64) f += z[i] * z[i] / ((d[i] - d[jr]) - 0.5 * D);
        f = 1.0 + rho * wave_sum(f);
        if (f >= 0.0) {
            o = jr;
            blo = 0.0;
            bhi = 0.5 * D;
        } else {
            o = jr + 1;
            blo = -0.5 * D;
            bhi = 0.0;
        }
    } else {
        double zz = 0.0;
        for (int i = lane; i < K; i += 64) zz += z[i] * z[i];
        zz = wave_sum(zz);
        o = K - 1;
        blo = 0.0;
        bhi = rho * zz;
    }
    double dor = d[o];
    double tau = 0.5 * (blo + bhi);
    bool conv = false;
    for (int it = 0; it < max_iter; ++it) {
        double psi = 0.0, phi = 0.0, dpsi = 0.0, dphi = 0.0, eabs = 0.0;
        for (int i = lane; i < K; i += 64) {
            double del = (d[i] - dor) - tau;
            double tm = z[i] * z[i] / del;
            if (i <= jr) {
                psi += tm;
                dpsi += tm / del;
            } else {
                phi += tm;
                dphi += tm / del;
            }
            eabs += fabs(tm);
        }
        psi = wave_sum(psi);
        phi = wave_sum(phi);
        dpsi = wave_sum(dpsi);
        dphi = wave_sum(dphi);
        eabs = wave_sum(eabs);
        double f = 1.0 + rho * (psi + phi);
        double err = 16.0 * DEPS * (1.0 + rho * eabs + fabs(tau) * rho * (dpsi + dphi));
        if (fabs(f) <= err) {
            conv = true;
            break;
        }
        if (f < 0.0) blo = tau;
        else bhi = tau;
        if (bhi - blo <= 2.0 * DEPS * fmax(fabs(blo), fabs(bhi))) {
            conv = true;
            break;
        }
        double tn;
        if (jr < K - 1) {
            double D1 = (d[jr] - dor) - tau, D2 = (d[jr + 1] - dor) - tau;
            double S1 = D1 * D1 * dpsi, S2 = D2 * D2 * dphi;
            double c = f - rho * (S1 / D1 + S2 / D2);
            double a2 = c, a1 = -(c * (D1 + D2) + rho * (S1 + S2)), a0 = D1 * D2 * f;
            double eta;
            if (a2 == 0.0) {
                eta = -a0 / a1;
            } else {
                double disc = fmax(0.0, a1 * a1 - 4.0 * a2 * a0);
                double q = -0.5 * (a1 + copysign(sqrt(disc), a1));
                double e1 = q / a2, e2 = (q != 0.0) ? a0 / q : e1;
                bool in1 = (tau + e1 > blo) && (tau + e1 < bhi);
                bool in2 = (tau + e2 > blo) && (tau + e2 < bhi);
                if (in1 && in2) eta = (fabs(e1) < fabs(e2)) ? e1 : e2;
                else if (in2) eta = e2;
                else eta = e1;
            }
            tn = tau + eta;
        } else {
            double D1 = -tau;
            double S1 = D1 * D1 * dpsi;
            double c = f - rho * S1 / D1;
            tn = (c > 0.0) ? tau + D1 + rho * S1 / c : 0.5 * (blo + bhi);
        }
        if (!(tn > blo && tn < bhi) || it >= max_iter / 2) tn = 0.5 * (blo + bhi);
        tau = tn;
    }
    if (lane == 0) {
        if (!conv) set_info(info, KS_ERR_NO_CONVERGENCE, 2);
        w.orig[lo + jr] = o;
        w.tau[lo + jr] = tau;
    }
}

// Gu-Eisenstat: z_hat_i^2 = prod_j (x_j - d_i) / (rho prod_{j != i} (d_j - d_i)),
// paired so that every factor lies in (0, 1].
__global__ __launch_bounds__(256) void dc_zhat_kernel(int n, int nm, const int* mlo, DcWork w) {
    const int G = blockIdx.y, g = G % nm;
    w = dc_slice(w, G / nm, n);
    int lo = mlo[g];
    int K = w.kk[G];
    int i = blockIdx.x * 4 + (threadIdx.x >> 6);
    int lane = threadIdx.x & 63;
    if (i >= K) return;
    const double* d = w.dnd + lo;
    double di = d[i];
    double p = 1.0;
    for (int j = lane; j < K; j += 64) {
        double xj = (d[w.orig[lo + j]] - di) + w.tau[lo + j];  // x_j - d_i
        if (j < i) p *= xj / (d[j] - di);
        else if (j < K - 1) p *= xj / (d[j + 1] - di);
        else p *= xj;
    }
    p = wave_prod(p);
    if (lane == 0) {
        double zh = sqrt(fabs(p / w.rho[G]));
        w.zhat[lo + i] = copysign(zh, w.znd[lo + i]);
    }
}

// 1/||u_j|| with u_ij = z_hat_i / (d_i - x_j).
__global__ __launch_bounds__(256) void dc_colnorm_kernel(int n, int nm, const int* mlo, DcWork w) {
    const int G = blockIdx.y, g = G % nm;
    w = dc_slice(w, G / nm, n);
    int lo = mlo[g];
    int K = w.kk[G];
    int jr = blockIdx.x * 4 + (threadIdx.x >> 6);
    int lane = threadIdx.x & 63;
    if (jr >= K) return;
    const double* d = w.dnd + lo;
    double dor = d[w.orig[lo + jr]], tj = w.tau[lo + jr];
    double s = 0.0;
    for (int i = lane; i < K; i += 64) {
        double u = w.zhat[lo + i] / ((d[i] - dor) - tj);
        s += u * u;
    }
    s = wave_sum(s);
    if (lane == 0) w.cinv[lo + jr] = 1.0 / sqrt(s);
}

// U block (K x K at (lo, lo), row stride n): U_ij = z_hat_i / (d_i - x_j) / ||u_j||.
__global__ __launch_bounds__(256) void dc_ugen_kernel(int n, int nm, const int* mlo, DcWork w, double* U) {
    const int G = blockIdx.z, g = G % nm, bm = G / nm;
    w = dc_slice(w, bm, n);
    U += (long)bm * n * n;
    int lo = mlo[g];
    int K = w.kk[G];
    int i = blockIdx.y;
    int jr = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= K || jr >= K) return;
    const double* d = w.dnd + lo;
    double u = w.zhat[lo + i] / ((d[i] - d[w.orig[lo + jr]]) - w.tau[lo + jr]);
    // row i of U pairs with column i of the gathered eigenvectors: both in the
    // child-grouped order when the merge has one
    const int gi = w.kk1[G] >= 0 ? w.gpos[lo + i] : i;
    U[(long)(lo + gi) * n + lo + jr] = u * w.cinv[lo + jr];
}

// Gather: Qp columns [0, K) = undeflated columns of Z in secular order, or in
// the child-grouped order gpos when the merge has one (kk1 >= 0); Z2 columns
// [K, K0) = deflated columns (both at the merge's block).
__global__ __launch_bounds__(256) void dc_gather_kernel(int n, int nm, const int* mlo, const int* mhi,
                                                        DcWork w, const double* Z, double* Qp, double* Z2) {
    const int G = blockIdx.z, g = G % nm, bm = G / nm;
    w = dc_slice(w, bm, n);
    const long o = (long)bm * n * n;
    Z += o;
    Qp += o;
    Z2 += o;
    int lo = mlo[g], hi = mhi[g];
    int K0 = hi - lo, K = w.kk[G];
    int r = lo + blockIdx.y;
    int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= hi || c >= K0) return;
    if (c < K) {
        int src = w.perm[lo + w.ndl[lo + c]];
        const int gc = w.kk1[G] >= 0 ? w.gpos[lo + c] : c;
        Qp[(long)r * n + lo + gc] = Z[(long)r * n + lo + src];
    } else {
        int src = w.perm[lo + w.dfl[lo + (c - K)]];
        Z2[(long)r * n + lo + c] = Z[(long)r * n + lo + src];
    }
}

// Final order: value of merged column c is x_c (c < K) or the deflated value;
// stable rank sort; lam[lo + rank] = value, src[lo + rank] = c.  The values
// every thread compares against pass through LDS in chunks, formed once per
// workgroup instead of gathered from memory by every thread.
constexpr int RANK_CHUNK = 2048;
__global__ __launch_bounds__(256) void dc_rank_kernel(int n, int nm, const int* mlo, const int* mhi, DcWork w) {
    __shared__ double sv[RANK_CHUNK];
    const int G = blockIdx.y, g = G % nm;
    w = dc_slice(w, G / nm, n);
    const int lo = mlo[g], hi = mhi[g];
    const int K0 = hi - lo, K = w.kk[G];
    if ((int)(blockIdx.x * blockDim.x) >= K0) return;  // the whole workgroup: no barrier is skipped
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    const bool act = c < K0;
    const double* d = w.dnd + lo;
    auto val = [&](int q) -> double {
        return (q < K) ? d[w.orig[lo + q]] + w.tau[lo + q] : w.dfval[lo + q - K];
    };
    const double v = act ? val(c) : 0.0;
    int rk = 0;
    for (int q0 = 0; q0 < K0; q0 += RANK_CHUNK) {
        const int cnt = min(RANK_CHUNK, K0 - q0);
        __syncthreads();  // the previous chunk has been read
        for (int e = threadIdx.x; e < cnt; e += blockDim.x) sv[e] = val(q0 + e);
        __syncthreads();
        if (act)
            for (int e = 0; e < cnt; ++e) {
                const double u = sv[e];
                rk += (u < v) || (u == v && q0 + e < c);
            }
    }
    if (act) {
        w.fval[lo + rk] = v;
        w.fsrc[lo + rk] = c;
    }
}

__global__ __launch_bounds__(256) void dc_permute_kernel(int n, int nm, const int* mlo, const int* mhi,
                                                         DcWork w, const double* Z2, double* Z, double* lam) {
    const int G = blockIdx.z, g = G % nm, bm = G / nm;
    w = dc_slice(w, bm, n);
    const long o = (long)bm * n * n;
    Z2 += o;
    Z += o;
    lam += (long)bm * n;
    int lo = mlo[g], hi = mhi[g];
    int K0 = hi - lo;
    int r = lo + blockIdx.y;
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= hi || p >= K0) return;
    Z[(long)r * n + lo + p] = Z2[(long)r * n + lo + w.fsrc[lo + p]];
    if (r == lo) lam[lo + p] = w.fval[lo + p];
}

// Iteration caps of the leaf Jacobi sweeps and of the secular-equation
// iterations.  A step that reaches its cap records KS_ERR_NO_CONVERGENCE and
// still finishes normally.  The defaults are far above what any input needs
// (quadratic convergence); a test hook lowers them to exercise that path.
namespace {
int g_leaf_sweeps = 40;
int g_secular_iters = 120;
}  // namespace

void stedc_set_caps(int leaf_sweeps, int secular_iters) {
    g_leaf_sweeps = leaf_sweeps > 0 ? leaf_sweeps : 40;
    g_secular_iters = secular_iters > 0 ? secular_iters : 120;
}

void stedc(hipStream_t s, const DcTree& tr, int batch, const double* d, const double* e, double* lam,
           double* Z, double* Z2, double* U, double* Qp, DcWork& w, int* info) {
    const int n = tr.n, B = batch;
    fill_zero<double>(s, Z, (long)n * n * B);
    hipLaunchKernelGGL(dc_init_kernel, dim3(cdiv(n, 256), B), dim3(256), 0, s, n, d, e, tr.d_leaf_lo, tr.nleaf,
                       w.dw);
    hipLaunchKernelGGL(dc_leaf_kernel, dim3(tr.nleaf, B), dim3(64), 0, s, n, tr.d_leaf_lo, tr.d_leaf_hi,
                       (const double*)w.dw, e, lam, Z, info, g_leaf_sweeps);
    for (int l = tr.depth - 1; l >= 0; --l) {
        const int nm = 1 << l, NG = nm * B;
        const int off = nm - 1;
        const int* mlo = tr.d_mlo + off;
        const int* mmid = tr.d_mmid + off;
        const int* mhi = tr.d_mhi + off;
        const int mk = tr.max_k0[l];
        const int dl = mk <= DEFLATE_LDS_MAX ? 1 : 0;
        hipLaunchKernelGGL(dc_deflate_kernel, dim3(NG), dim3(256), dl ? (size_t)mk * sizeof(double) : 0, s, n, nm,
                           mlo, mmid, mhi, e, lam, Z, w, dl);
        hipLaunchKernelGGL(dc_rotate_kernel, dim3(cdiv(mk, 256), NG), dim3(256), 0, s, n, nm, mlo, mhi, w, Z);
        hipLaunchKernelGGL(dc_secular_kernel, dim3(cdiv(mk, 4), NG), dim3(256), 0, s, n, nm, mlo, w, info,
                           g_secular_iters);
        hipLaunchKernelGGL(dc_zhat_kernel, dim3(cdiv(mk, 4), NG), dim3(256), 0, s, n, nm, mlo, w);
        hipLaunchKernelGGL(dc_colnorm_kernel, dim3(cdiv(mk, 4), NG), dim3(256), 0, s, n, nm, mlo, w);
        hipLaunchKernelGGL(dc_ugen_kernel, dim3(cdiv(mk, 256), mk, NG), dim3(256), 0, s, n, nm, mlo, w, U);
        hipLaunchKernelGGL(dc_gather_kernel, dim3(cdiv(mk, 256), mk, NG), dim3(256), 0, s, n, nm, mlo, mhi, w,
                           (const double*)Z, Qp, Z2);
        gemm_grouped_dc(s, nm, B, mk, mlo, mmid, mhi, w.kk, w.kk1, Qp, U, Z2, n);
        hipLaunchKernelGGL(dc_rank_kernel, dim3(cdiv(mk, 256), NG), dim3(256), 0, s, n, nm, mlo, mhi, w);
        hipLaunchKernelGGL(dc_permute_kernel, dim3(cdiv(mk, 256), mk, NG), dim3(256), 0, s, n, nm, mlo, mhi, w,
                           (const double*)Z2, Z, lam);
    }
}

// Host: the tear tree for order n (depth = smallest with ceil(n / 2^depth) <= leaf,
// leaf <= DC_LEAF).
void dc_tree_host(int n, int leaf, std::vector<int>& mlo, std::vector<int>& mmid, std::vector<int>& mhi,
                  std::vector<int>& leaf_lo, std::vector<int>& leaf_hi, int& depth,
                  std::vector<int>& max_k0) {
    leaf = std::max(2, std::min(leaf, DC_LEAF));
    depth = 0;
    while ((n + (1 << depth) - 1) / (1 << depth) > leaf) ++depth;
    // nodes level by level: level l has 2^l nodes, stored at offset 2^l - 1
    std::vector<int> lo{0}, hi{n};
    mlo.clear();
    mmid.clear();
    mhi.clear();
    max_k0.assign(depth > 0 ? depth : 1, 0);
    for (int l = 0; l < depth; ++l) {
        std::vector<int> nlo, nhi;
        for (size_t q = 0; q < lo.size(); ++q) {
            int a = lo[q], b = hi[q], m = a + (b - a) / 2;
            mlo.push_back(a);
            mmid.push_back(m);
            mhi.push_back(b);
            max_k0[l] = std::max(max_k0[l], b - a);
            nlo.push_back(a);
            nhi.push_back(m);
            nlo.push_back(m);
            nhi.push_back(b);
        }
        lo.swap(nlo);
        hi.swap(nhi);
    }
    leaf_lo = lo;
    leaf_hi = hi;
}

}  // namespace ks
