/*
 * ks_oracle.c -- plain, slow FP64 CPU oracle for the generalized Kohn-Sham
 * eigenproblem and the density build.
 *
 * TEST INFRASTRUCTURE ONLY.  The product path never links, loads or calls this
 * file; only the tests, the smoke entry and the CPU-baseline leg of the
 * benchmark do.  It shares no code, header or table with the HIP library.
 *
 * What it computes (paper, Sec. 2 and Sec. 3):
 *   - the generalized eigenproblem H C = S C eps (Sec. 2, the equation that
 *     follows the basis expansion; per k-point in the Bloch form; and the
 *     noncollinear spinor form whose overlap is diag(S, S), end of Sec. 2 and
 *     the definitions of H_NC, C_NC, S_NC in Sec. 3.2),
 *   - Fermi-Dirac occupations and the chemical potential fixed by the electron
 *     count (Sec. 2, density equation with the factor 2; Part 3 of the
 *     collinear flow of Sec. 3.1 and Part 4 of the noncollinear flow),
 *   - the density matrix (Sec. 2 density-matrix equation, and its spinor form)
 *     returned as rho = C f C^H, the complex conjugate of the paper's
 *     n_lm = sum_i f_i conj(c_li) c_mi,
 *   - the Loewdin route of Sec. 3.1 (Parts 2-1 to 2-5; Parts 3-1 to 3-6 of
 *     Sec. 3.2 for the spinor case) as a second, independent reduction,
 *   - the dense adjoint of rho and of the band energy.
 *
 * Route of the main solve, each step its textbook definition with no blocking
 * or fusion: Cholesky S = L L^H (column algorithm, Golub & Van Loan,
 * "Matrix Computations", Alg. 4.2.1) -> A = L^-1 H L^-H by forward
 * substitution -> cyclic Jacobi on A (Golub & Van Loan Sec. 8.5, symmetric
 * Schur 2x2 rotation; for Hermitian A the phase of a_pq is removed first), in
 * the round-robin ordering of disjoint pairs: the rotations of one round touch
 * disjoint rows and columns and commute, so the result does not depend on the
 * thread count -> stable ascending sort -> C = L^-H V by back substitution.
 *
 * Storage: row-major; complex matrices interleave (re, im) like C99
 * double complex and torch.complex128.  Only the lower triangle of H and S is
 * read; it is mirrored into a full Hermitian matrix.
 *
 * Every routine here is pinned by the CPU tests against closed forms,
 * brute-force characteristic polynomials, invariants and finite differences.
 */
#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex zc;

static void set_threads(int nthreads) {
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
}

void ko_set_threads(int nthreads) { set_threads(nthreads); }

int ko_max_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------ */
/* Hermitian completion from the lower triangle                        */
/* ------------------------------------------------------------------ */
static void herm_from_lower(int n, int cplx, const double* X, int ldx, double* Y) {
    if (!cplx) {
        for (int i = 0; i < n; ++i)
            for (int j = 0; j <= i; ++j) {
                double v = X[(size_t)i * ldx + j];
                Y[(size_t)i * n + j] = v;
                Y[(size_t)j * n + i] = v;
            }
    } else {
        const zc* Xz = (const zc*)X;
        zc* Yz = (zc*)Y;
        for (int i = 0; i < n; ++i) {
            for (int j = 0; j < i; ++j) {
                zc v = Xz[(size_t)i * ldx + j];
                Yz[(size_t)i * n + j] = v;
                Yz[(size_t)j * n + i] = conj(v);
            }
            Yz[(size_t)i * n + i] = creal(Xz[(size_t)i * ldx + i]);
        }
    }
}

/* ------------------------------------------------------------------ */
/* Cholesky S = L L^H.  Returns 0, or the 1-based column whose pivot is */
/* not positive and finite (LAPACK convention).  L is n x n, row-major, */
/* upper triangle zero.  Reads the lower triangle of S only.            */
/* ------------------------------------------------------------------ */
int ko_cholesky(int n, int cplx, const double* S, int lds, double* L) {
    if (!cplx) {
        memset(L, 0, sizeof(double) * (size_t)n * n);
        for (int j = 0; j < n; ++j) {
            double d = S[(size_t)j * lds + j];
            for (int k = 0; k < j; ++k) d -= L[(size_t)j * n + k] * L[(size_t)j * n + k];
            if (!(d > 0.0) || !isfinite(d)) return j + 1;
            double ljj = sqrt(d);
            L[(size_t)j * n + j] = ljj;
            for (int i = j + 1; i < n; ++i) {
                double s = S[(size_t)i * lds + j];
                for (int k = 0; k < j; ++k) s -= L[(size_t)i * n + k] * L[(size_t)j * n + k];
                L[(size_t)i * n + j] = s / ljj;
            }
        }
    } else {
        const zc* Sz = (const zc*)S;
        zc* Lz = (zc*)L;
        memset(L, 0, sizeof(zc) * (size_t)n * n);
        for (int j = 0; j < n; ++j) {
            double d = creal(Sz[(size_t)j * lds + j]);
            for (int k = 0; k < j; ++k) {
                zc l = Lz[(size_t)j * n + k];
                d -= creal(l) * creal(l) + cimag(l) * cimag(l);
            }
            if (!(d > 0.0) || !isfinite(d)) return j + 1;
            double ljj = sqrt(d);
            Lz[(size_t)j * n + j] = ljj;
            for (int i = j + 1; i < n; ++i) {
                zc s = Sz[(size_t)i * lds + j];
                for (int k = 0; k < j; ++k) s -= Lz[(size_t)i * n + k] * conj(Lz[(size_t)j * n + k]);
                Lz[(size_t)i * n + j] = s / ljj;
            }
        }
    }
    return 0;
}

/* B <- L^-1 B by forward substitution; B is n x ncols with row stride ldb. */
void ko_solve_lower(int n, int ncols, int cplx, const double* L, double* B, int ldb) {
    if (!cplx) {
        for (int i = 0; i < n; ++i) {
            double* bi = B + (size_t)i * ldb;
            for (int k = 0; k < i; ++k) {
                double l = L[(size_t)i * n + k];
                const double* bk = B + (size_t)k * ldb;
                for (int c = 0; c < ncols; ++c) bi[c] -= l * bk[c];
            }
            double d = L[(size_t)i * n + i];
            for (int c = 0; c < ncols; ++c) bi[c] /= d;
        }
    } else {
        const zc* Lz = (const zc*)L;
        zc* Bz = (zc*)B;
        for (int i = 0; i < n; ++i) {
            zc* bi = Bz + (size_t)i * ldb;
            for (int k = 0; k < i; ++k) {
                zc l = Lz[(size_t)i * n + k];
                const zc* bk = Bz + (size_t)k * ldb;
                for (int c = 0; c < ncols; ++c) bi[c] -= l * bk[c];
            }
            double d = creal(Lz[(size_t)i * n + i]);
            for (int c = 0; c < ncols; ++c) bi[c] /= d;
        }
    }
}

/* B <- L^-H B by back substitution (solves L^H X = B). */
void ko_solve_lower_h(int n, int ncols, int cplx, const double* L, double* B, int ldb) {
    if (!cplx) {
        for (int i = n - 1; i >= 0; --i) {
            double* bi = B + (size_t)i * ldb;
            for (int k = i + 1; k < n; ++k) {
                double l = L[(size_t)k * n + i];
                const double* bk = B + (size_t)k * ldb;
                for (int c = 0; c < ncols; ++c) bi[c] -= l * bk[c];
            }
            double d = L[(size_t)i * n + i];
            for (int c = 0; c < ncols; ++c) bi[c] /= d;
        }
    } else {
        const zc* Lz = (const zc*)L;
        zc* Bz = (zc*)B;
        for (int i = n - 1; i >= 0; --i) {
            zc* bi = Bz + (size_t)i * ldb;
            for (int k = i + 1; k < n; ++k) {
                zc l = conj(Lz[(size_t)k * n + i]);
                const zc* bk = Bz + (size_t)k * ldb;
                for (int c = 0; c < ncols; ++c) bi[c] -= l * bk[c];
            }
            double d = creal(Lz[(size_t)i * n + i]);
            for (int c = 0; c < ncols; ++c) bi[c] /= d;
        }
    }
}

/* ------------------------------------------------------------------ */
/* Cyclic Jacobi in the round-robin ordering.                           */
/* ------------------------------------------------------------------ */
/* Pairs of round r (0 <= r < m-1) of the circle method for m (even)
 * indices: index 0 stays put and the others rotate one place per round, so
 * every pair p < q meets exactly once per sweep. */
static void rr_pairs(int m, int r, int* P, int* Q) {
    for (int i = 0; i < m / 2; ++i) {
        int a = (i == 0) ? 0 : 1 + ((i - 1 + r) % (m - 1));
        int b = 1 + ((m - 2 - i + r) % (m - 1));
        if (a > b) { int t = a; a = b; b = t; }
        P[i] = a;
        Q[i] = b;
    }
}

/* Symmetric Schur 2x2 (Golub & Van Loan Alg. 8.5.1) for [[app, b], [b, aqq]],
 * b != 0: t = tan(theta), c = cos, s = sin of the rotation that makes
 * J^T A J diagonal with J = [[c, s], [-s, c]]. */
static void sym_schur2(double app, double aqq, double b, double* t, double* c, double* s) {
    double tau = (aqq - app) / (2.0 * b);
    double tt;
    if (!isfinite(tau)) tt = 0.0;
    else if (tau >= 0.0) tt = 1.0 / (tau + sqrt(1.0 + tau * tau));
    else tt = -1.0 / (-tau + sqrt(1.0 + tau * tau));
    double cc = 1.0 / sqrt(1.0 + tt * tt);
    *t = tt;
    *c = cc;
    *s = tt * cc;
}

/* Eigen-decomposition of the Hermitian A (n x n, full storage, overwritten).
 * W: eigenvalues ascending (stable: ties keep index order); V: eigenvectors
 * as columns (row-major n x n, V^H V = I).  Stops when
 * off(A) <= 1e-15 ||A||_F (Weyl: every eigenvalue is then within off(A)) or
 * when a sweep performs no rotation.  Returns the sweep count, or -1 if
 * maxsweeps was reached first.  Complex case: J = [[c, s e^{i phi}],
 * [-s e^{-i phi}, c]] with a_pq = |a_pq| e^{i phi}; this is P R P^H with
 * P = diag(1, e^{-i phi}) removing the phase and R the real rotation. */
int ko_jacobi(int n, int cplx, double* Ain, double* W, double* Vout, int maxsweeps, int nthreads) {
    set_threads(nthreads);
    int m = n + (n & 1);
    int np = m / 2;
    int* P = malloc(sizeof(int) * np);
    int* Q = malloc(sizeof(int) * np);
    /* per pair: c, s, phase (re, im), new app, new aqq, active flag */
    double* rot = malloc(sizeof(double) * 7 * np);
    size_t es = cplx ? 2 : 1;
    double* VT = calloc((size_t)n * n * es, sizeof(double)); /* rows = eigenvectors */
    for (int i = 0; i < n; ++i) VT[((size_t)i * n + i) * es] = 1.0;

    double normA = 0.0, off = 0.0;
    for (size_t i = 0; i < (size_t)n * n * es; ++i) normA += Ain[i] * Ain[i];
    normA = sqrt(normA);
    int sweeps = -1;
    for (int sw = 0; sw <= maxsweeps; ++sw) {
        off = 0.0;
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j)
                if (i != j) {
                    size_t o = ((size_t)i * n + j) * es;
                    off += Ain[o] * Ain[o] + (cplx ? Ain[o + 1] * Ain[o + 1] : 0.0);
                }
        off = sqrt(off);
        if (off <= 1e-15 * normA) { sweeps = sw; break; }
        if (sw == maxsweeps) break;
        int rotations = 0;
        for (int r = 0; r < m - 1; ++r) {
            rr_pairs(m, r, P, Q);
            /* 1. angles, all from the 2x2 blocks before this round */
            for (int i = 0; i < np; ++i) {
                int p = P[i], q = Q[i];
                double* R = rot + 7 * i;
                R[6] = 0.0;
                if (q >= n) continue;
                double app, aqq, b, ph_re = 1.0, ph_im = 0.0;
                if (!cplx) {
                    app = Ain[(size_t)p * n + p];
                    aqq = Ain[(size_t)q * n + q];
                    b = Ain[(size_t)p * n + q];
                } else {
                    zc* Az = (zc*)Ain;
                    app = creal(Az[(size_t)p * n + p]);
                    aqq = creal(Az[(size_t)q * n + q]);
                    zc apq = Az[(size_t)p * n + q];
                    b = cabs(apq);
                    if (b != 0.0) { ph_re = creal(apq) / b; ph_im = cimag(apq) / b; }
                }
                /* Rutishauser's skip rule: a_pq negligible next to both diagonals */
                if (b == 0.0 || fabs(b) <= 1e-17 * fmin(fabs(app), fabs(aqq))) {
                    size_t o1 = ((size_t)p * n + q) * es, o2 = ((size_t)q * n + p) * es;
                    Ain[o1] = Ain[o2] = 0.0;
                    if (cplx) Ain[o1 + 1] = Ain[o2 + 1] = 0.0;
                    continue;
                }
                double t, c, s;
                sym_schur2(app, aqq, b, &t, &c, &s);
                R[0] = c; R[1] = s; R[2] = ph_re; R[3] = ph_im;
                R[4] = app - t * b; R[5] = aqq + t * b; R[6] = 1.0;
                ++rotations;
            }
            /* 2. rows: A <- J^H A, and V^T <- J^T V^T (i.e. V <- V J) */
            #pragma omp parallel for schedule(static)
            for (int i = 0; i < np; ++i) {
                const double* R = rot + 7 * i;
                if (R[6] == 0.0) continue;
                int p = P[i], q = Q[i];
                double c = R[0], s = R[1];
                if (!cplx) {
                    double* ap = Ain + (size_t)p * n;
                    double* aq = Ain + (size_t)q * n;
                    for (int k = 0; k < n; ++k) {
                        double x = ap[k], y = aq[k];
                        ap[k] = c * x - s * y;
                        aq[k] = s * x + c * y;
                    }
                    double* vp = VT + (size_t)p * n;
                    double* vq = VT + (size_t)q * n;
                    for (int k = 0; k < n; ++k) {
                        double x = vp[k], y = vq[k];
                        vp[k] = c * x - s * y;
                        vq[k] = s * x + c * y;
                    }
                } else {
                    zc e = R[2] + I * R[3]; /* e^{i phi} */
                    zc* ap = (zc*)Ain + (size_t)p * n;
                    zc* aq = (zc*)Ain + (size_t)q * n;
                    for (int k = 0; k < n; ++k) {
                        zc x = ap[k], y = aq[k];
                        ap[k] = c * x - s * e * y;
                        aq[k] = s * conj(e) * x + c * y;
                    }
                    zc* vp = (zc*)VT + (size_t)p * n;
                    zc* vq = (zc*)VT + (size_t)q * n;
                    for (int k = 0; k < n; ++k) {
                        zc x = vp[k], y = vq[k];
                        vp[k] = c * x - s * conj(e) * y;
                        vq[k] = s * e * x + c * y;
                    }
                }
            }
            /* 3. columns: A <- A J */
            #pragma omp parallel for schedule(static)
            for (int k = 0; k < n; ++k) {
                for (int i = 0; i < np; ++i) {
                    const double* R = rot + 7 * i;
                    if (R[6] == 0.0) continue;
                    int p = P[i], q = Q[i];
                    double c = R[0], s = R[1];
                    if (!cplx) {
                        double* ak = Ain + (size_t)k * n;
                        double x = ak[p], y = ak[q];
                        ak[p] = c * x - s * y;
                        ak[q] = s * x + c * y;
                    } else {
                        zc e = R[2] + I * R[3];
                        zc* ak = (zc*)Ain + (size_t)k * n;
                        zc x = ak[p], y = ak[q];
                        ak[p] = c * x - s * conj(e) * y;
                        ak[q] = s * e * x + c * y;
                    }
                }
            }
            /* 4. the rotated 2x2 blocks take their exact values */
            for (int i = 0; i < np; ++i) {
                const double* R = rot + 7 * i;
                if (R[6] == 0.0) continue;
                int p = P[i], q = Q[i];
                size_t opp = ((size_t)p * n + p) * es, oqq = ((size_t)q * n + q) * es;
                size_t opq = ((size_t)p * n + q) * es, oqp = ((size_t)q * n + p) * es;
                Ain[opp] = R[4]; Ain[oqq] = R[5];
                Ain[opq] = Ain[oqp] = 0.0;
                if (cplx) Ain[opp + 1] = Ain[oqq + 1] = Ain[opq + 1] = Ain[oqp + 1] = 0.0;
            }
        }
        if (rotations == 0) { sweeps = sw + 1; break; }
    }
    /* eigenvalues from the diagonal; stable ascending sort */
    int* idx = malloc(sizeof(int) * n);
    for (int i = 0; i < n; ++i) { W[i] = Ain[((size_t)i * n + i) * es]; idx[i] = i; }
    for (int i = 1; i < n; ++i) { /* insertion sort: stable */
        int v = idx[i], j = i - 1;
        while (j >= 0 && W[idx[j]] > W[v]) { idx[j + 1] = idx[j]; --j; }
        idx[j + 1] = v;
    }
    double* Ws = malloc(sizeof(double) * n);
    for (int j = 0; j < n; ++j) Ws[j] = W[idx[j]];
    memcpy(W, Ws, sizeof(double) * n);
    #pragma omp parallel for schedule(static)
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            size_t dst = ((size_t)i * n + j) * es, src = ((size_t)idx[j] * n + i) * es;
            Vout[dst] = VT[src];
            if (cplx) Vout[dst + 1] = VT[src + 1];
        }
    free(Ws); free(idx); free(VT); free(rot); free(P); free(Q);
    return sweeps;
}

/* ------------------------------------------------------------------ */
/* Plain matrix product helpers for the Loewdin route and the adjoint  */
/* ------------------------------------------------------------------ */
/* Y = op(A) * B, with op(A) = A (ta == 0) or A^H (ta == 1).  A is ar x ac,
 * B is (rows of op(A))' inner x bc. */
static void zmm(int cplx, int ta, int ar, int ac, const double* A, int bc, const double* B, double* Y) {
    int m = ta ? ac : ar, kk = ta ? ar : ac;
    if (!cplx) {
        #pragma omp parallel for schedule(static)
        for (int i = 0; i < m; ++i)
            for (int j = 0; j < bc; ++j) {
                double s = 0.0;
                for (int k = 0; k < kk; ++k) {
                    double a = ta ? A[(size_t)k * ac + i] : A[(size_t)i * ac + k];
                    s += a * B[(size_t)k * bc + j];
                }
                Y[(size_t)i * bc + j] = s;
            }
    } else {
        const zc* Az = (const zc*)A;
        const zc* Bz = (const zc*)B;
        zc* Yz = (zc*)Y;
        #pragma omp parallel for schedule(static)
        for (int i = 0; i < m; ++i)
            for (int j = 0; j < bc; ++j) {
                zc s = 0.0;
                for (int k = 0; k < kk; ++k) {
                    zc a = ta ? conj(Az[(size_t)k * ac + i]) : Az[(size_t)i * ac + k];
                    s += a * Bz[(size_t)k * bc + j];
                }
                Yz[(size_t)i * bc + j] = s;
            }
    }
}

/* ------------------------------------------------------------------ */
/* Generalized eigenproblem, Cholesky route.                            */
/* nsp = 1: collinear, H is n x n.  nsp = 2: noncollinear, H is 2n x 2n */
/* in spin-block order [[aa, ab], [ba, bb]] and the overlap is          */
/* diag(S, S) with S n x n (paper Sec. 3.2, S_NC).                      */
/* eps: order values ascending; C: order x order, eigenvectors as       */
/* columns, C^H S_NC C = I.  Returns 0, -k for a non-positive pivot in  */
/* column k of S, or 1 if Jacobi did not converge.                      */
/* ------------------------------------------------------------------ */
int ko_gevd(int n, int nsp, int cplx, const double* H, int ldh, const double* S, int lds,
            double* eps, double* C, int nthreads, int* sweeps_out) {
    set_threads(nthreads);
    int order = n * nsp;
    size_t es = cplx ? 2 : 1;
    double* L = malloc(sizeof(double) * (size_t)n * n * es);
    int info = ko_cholesky(n, cplx, S, lds, L);
    if (info) { free(L); return -info; }
    double* A = malloc(sizeof(double) * (size_t)order * order * es);
    double* X = malloc(sizeof(double) * (size_t)order * order * es);
    herm_from_lower(order, cplx, H, ldh, X);
    /* X <- (I (x) L)^-1 X : each spin row-block solves with L */
    for (int b = 0; b < nsp; ++b)
        ko_solve_lower(n, order, cplx, L, X + (size_t)b * n * order * es, order);
    /* A <- X^H, then A <- (I (x) L)^-1 A, giving L^-1 H L^-H */
    for (int i = 0; i < order; ++i)
        for (int j = 0; j < order; ++j) {
            size_t d = ((size_t)i * order + j) * es, s = ((size_t)j * order + i) * es;
            A[d] = X[s];
            if (cplx) A[d + 1] = -X[s + 1];
        }
    for (int b = 0; b < nsp; ++b)
        ko_solve_lower(n, order, cplx, L, A + (size_t)b * n * order * es, order);
    /* A <- (A + A^H)/2 */
    for (int i = 0; i < order; ++i)
        for (int j = 0; j <= i; ++j) {
            size_t o1 = ((size_t)i * order + j) * es, o2 = ((size_t)j * order + i) * es;
            double re = 0.5 * (A[o1] + A[o2]);
            A[o1] = A[o2] = re;
            if (cplx) {
                double im = 0.5 * (A[o1 + 1] - A[o2 + 1]);
                A[o1 + 1] = im;
                A[o2 + 1] = -im;
            }
        }
    int sw = ko_jacobi(order, cplx, A, eps, C, 50, nthreads);
    if (sweeps_out) *sweeps_out = sw;
    /* C <- (I (x) L)^-H V */
    for (int b = 0; b < nsp; ++b)
        ko_solve_lower_h(n, order, cplx, L, C + (size_t)b * n * order * es, order);
    free(A); free(X); free(L);
    return sw < 0 ? 1 : 0;
}

/* Loewdin route (paper Sec. 3.1, Parts 2-1..2-5; Sec. 3.2, Parts 3-1..3-6):
 * U^H S U = s, V = U s^-1/2, V_NC = diag(V, V), H' = V_NC^H H V_NC,
 * H' C' = C' eps, C = V_NC C'.  Same outputs as ko_gevd. */
int ko_gevd_lowdin(int n, int nsp, int cplx, const double* H, int ldh, const double* S, int lds,
                   double* eps, double* C, int nthreads) {
    set_threads(nthreads);
    int order = n * nsp;
    size_t es = cplx ? 2 : 1;
    double* Sf = malloc(sizeof(double) * (size_t)n * n * es);
    double* U = malloc(sizeof(double) * (size_t)n * n * es);
    double* s = malloc(sizeof(double) * n);
    herm_from_lower(n, cplx, S, lds, Sf);
    int sw = ko_jacobi(n, cplx, Sf, s, U, 50, nthreads);
    if (sw < 0) { free(Sf); free(U); free(s); return 1; }
    for (int j = 0; j < n; ++j)
        if (!(s[j] > 0.0)) { free(Sf); free(U); free(s); return -(j + 1); }
    /* V = U s^-1/2 (column scaling) */
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            size_t o = ((size_t)i * n + j) * es;
            double f = 1.0 / sqrt(s[j]);
            U[o] *= f;
            if (cplx) U[o + 1] *= f;
        }
    /* V_NC = diag(V, V) as a full order x order matrix */
    double* VN = calloc((size_t)order * order * es, sizeof(double));
    for (int b = 0; b < nsp; ++b)
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                size_t d = (((size_t)(b * n + i)) * order + (b * n + j)) * es, o = ((size_t)i * n + j) * es;
                VN[d] = U[o];
                if (cplx) VN[d + 1] = U[o + 1];
            }
    double* Hf = malloc(sizeof(double) * (size_t)order * order * es);
    double* T = malloc(sizeof(double) * (size_t)order * order * es);
    double* Hp = malloc(sizeof(double) * (size_t)order * order * es);
    herm_from_lower(order, cplx, H, ldh, Hf);
    zmm(cplx, 0, order, order, Hf, order, VN, T);  /* T = H V_NC */
    zmm(cplx, 1, order, order, VN, order, T, Hp);  /* H' = V_NC^H T */
    for (int i = 0; i < order; ++i)                /* H' <- (H' + H'^H)/2 */
        for (int j = 0; j <= i; ++j) {
            size_t o1 = ((size_t)i * order + j) * es, o2 = ((size_t)j * order + i) * es;
            double re = 0.5 * (Hp[o1] + Hp[o2]);
            Hp[o1] = Hp[o2] = re;
            if (cplx) {
                double im = 0.5 * (Hp[o1 + 1] - Hp[o2 + 1]);
                Hp[o1 + 1] = im;
                Hp[o2 + 1] = -im;
            }
        }
    sw = ko_jacobi(order, cplx, Hp, eps, T, 50, nthreads); /* T = C' */
    zmm(cplx, 0, order, order, VN, order, T, C);          /* C = V_NC C' */
    free(Sf); free(U); free(s); free(VN); free(Hf); free(T); free(Hp);
    return sw < 0 ? 1 : 0;
}

/* ------------------------------------------------------------------ */
/* Fermi-Dirac occupations and the chemical potential                  */
/* ------------------------------------------------------------------ */
/* F(x) = 1/(1+e^x), evaluated without overflow on either side. */
static double fermi_F(double x) {
    if (x > 0.0) { double e = exp(-x); return e / (1.0 + e); }
    return 1.0 / (1.0 + exp(x));
}

/* Electron count N(mu) = sum_k w_k sum_i g F((eps_ik - mu)/kT). */
static double electron_count(int nk, int order, const double* eps, const double* wk, double g,
                             double kT, double mu) {
    double total = 0.0;
    for (int k = 0; k < nk; ++k) {
        double s = 0.0;
        for (int i = 0; i < order; ++i) s += g * fermi_F((eps[(size_t)k * order + i] - mu) / kT);
        total += wk[k] * s;
    }
    return total;
}

/* mu by bisection on N(mu) = ne over [min eps - 50 kT, max eps + 50 kT], until
 * hi - lo <= 1e-14 max(1, |mu|) or 200 halvings; mu is the midpoint.  One mu is
 * common to all k-points.  Then f_ik = g F((eps_ik - mu)/kT),
 * E_band = sum_k w_k sum_i f_ik eps_ik, and the electronic entropy term
 * TS = -kT sum_k w_k sum_i g [F ln F + (1-F) ln(1-F)] (for the Mermin free
 * energy Omega = E_band - TS).  Returns the number of halvings. */
int ko_fermi(int nk, int order, const double* eps, const double* wk, double g, double ne, double kT,
             double* mu_out, double* occ, double* eband_out, double* ts_out) {
    double lo = eps[0], hi = eps[0];
    for (size_t i = 0; i < (size_t)nk * order; ++i) {
        if (eps[i] < lo) lo = eps[i];
        if (eps[i] > hi) hi = eps[i];
    }
    lo -= 50.0 * kT;
    hi += 50.0 * kT;
    int it = 0;
    while (it < 200) {
        double mid = 0.5 * (lo + hi);
        if (hi - lo <= 1e-14 * fmax(1.0, fabs(mid))) break;
        if (electron_count(nk, order, eps, wk, g, kT, mid) < ne) lo = mid;
        else hi = mid;
        ++it;
    }
    double mu = 0.5 * (lo + hi);
    double eb = 0.0, ts = 0.0;
    for (int k = 0; k < nk; ++k) {
        double sb = 0.0, st = 0.0;
        for (int i = 0; i < order; ++i) {
            double e = eps[(size_t)k * order + i];
            double x = (e - mu) / kT;
            double F = fermi_F(x), Fm = fermi_F(-x);
            double f = g * F;
            if (occ) occ[(size_t)k * order + i] = f;
            sb += f * e;
            if (F > 0.0) st += F * log(F);
            if (Fm > 0.0) st += Fm * log(Fm);
        }
        eb += wk[k] * sb;
        ts += wk[k] * (-kT * g * st);
    }
    *mu_out = mu;
    if (eband_out) *eband_out = eb;
    if (ts_out) *ts_out = ts;
    return it;
}

/* rho = C diag(w) C^H over the ncols columns of C (order x ncols, row
 * stride ldc); full Hermitian output order x order. */
void ko_density(int order, int ncols, int cplx, const double* C, int ldc, const double* w, double* rho) {
    if (!cplx) {
        #pragma omp parallel for schedule(static)
        for (int i = 0; i < order; ++i)
            for (int j = 0; j < order; ++j) {
                double s = 0.0;
                for (int k = 0; k < ncols; ++k)
                    s += w[k] * C[(size_t)i * ldc + k] * C[(size_t)j * ldc + k];
                rho[(size_t)i * order + j] = s;
            }
    } else {
        const zc* Cz = (const zc*)C;
        zc* R = (zc*)rho;
        #pragma omp parallel for schedule(static)
        for (int i = 0; i < order; ++i)
            for (int j = 0; j < order; ++j) {
                zc s = 0.0;
                for (int k = 0; k < ncols; ++k)
                    s += w[k] * Cz[(size_t)i * ldc + k] * conj(Cz[(size_t)j * ldc + k]);
                R[(size_t)i * order + j] = s;
            }
    }
}

/* ------------------------------------------------------------------ */
/* Dense adjoint of rho = C f C^H and E_band                            */
/* ------------------------------------------------------------------ */
/* Divided difference (F(x) - F(y))/(x - y) of F(x) = 1/(1+e^x).  For
 * |x - y| < 1 it uses the identity
 *   F(x) - F(y) = -sinh((x-y)/2) / (2 cosh(x/2) cosh(y/2)),
 * i.e. -(1/4) sinhc((x-y)/2) sech(x/2) sech(y/2), whose limit at x = y is F'(x);
 * sech is evaluated as 2 e^-|u| / (1 + e^-2|u|), which cannot overflow. */
static double sech_(double u) {
    double a = fabs(u), e = exp(-a);
    return 2.0 * e / (1.0 + e * e);
}
static double fermi_dd(double x, double y) {
    double d = x - y;
    if (fabs(d) < 1.0) {
        double t = 0.5 * d;
        double shc = (t == 0.0) ? 1.0 : sinh(t) / t;
        return -0.25 * shc * sech_(0.5 * x) * sech_(0.5 * y);
    }
    return (fermi_F(x) - fermi_F(y)) / d;
}

/* Gradients of L(rho, E_band) with respect to H and S.
 * Inputs per k (batch nk): eps (order), C (order x order, all eigenvectors,
 * C^H S_NC C = I), mu, kT, g, weights wk; Gbar = dL/drho (order x order per k,
 * NULL for none), ebar = dL/dE_band.  With f'_i = -f_i (1 - f_i/g)/kT,
 * Gh = (Gbar + Gbar^H)/2 and Gt = C^H Gh C:
 *   G1_ij = (f_i - f_j)/(eps_i - eps_j), G1_ii = f'_i,
 *   G2_ij = (f_i + f_j)/2 + (eps_i + eps_j) G1_ij / 2, G2_ii = f_i + eps_i f'_i,
 *   a_k = w_k sum_k' sum_i Gt_ii f'_i / sum_k' w_k' sum_i f'_i (0 if the
 *   denominator vanishes), from d mu fixed by the electron count,
 *   Hbar = C (Gt o G1 - a_k diag f') C^H,
 *   Sbar = -C (Gt o G2 - a_k diag(f' eps)) C^H,
 * plus, for E_band with b = sum w eps f' / sum w f' and
 * w_i = w_k (f_i + (eps_i - b) f'_i): Hbar += ebar C diag(w) C^H,
 * Sbar -= ebar C diag(w eps) C^H.
 * These follow from d eps_i = c_i^H (dH - eps_i dS) c_i,
 * dC = C X with X_ji = (C^H (dH - eps_i dS) C)_ji / (eps_i - eps_j),
 * X_ii = -(C^H dS C)_ii / 2, and df_i = f'_i (d eps_i - d mu).
 * Hbar is order x order per k; Sbar is n x n per k (for nsp = 2 the
 * gradient of S_NC = diag(S, S) is summed over its two diagonal blocks).
 * Gradients follow the convention dL = Re tr(Hbar^H dH) + Re tr(Sbar^H dS). */
void ko_adjoint(int n, int nsp, int cplx, int nk, const double* eps, const double* C, double mu,
                double kT, double g, const double* wk, const double* Gbar, double ebar,
                double* Hbar, double* Sbar) {
    int order = n * nsp;
    size_t es = cplx ? 2 : 1;
    size_t mat = (size_t)order * order * es;
    double* fp = malloc(sizeof(double) * (size_t)nk * order);
    double* f = malloc(sizeof(double) * (size_t)nk * order);
    double* Gt = calloc(mat * nk, sizeof(double));
    double* T = malloc(sizeof(double) * mat);
    double* P1 = malloc(sizeof(double) * mat);
    double* P2 = malloc(sizeof(double) * mat);
    double* Gh = malloc(sizeof(double) * mat);
    for (size_t i = 0; i < (size_t)nk * order; ++i) {
        double x = (eps[i] - mu) / kT;
        f[i] = g * fermi_F(x);
        fp[i] = -g * fermi_F(x) * fermi_F(-x) / kT;
    }
    /* Gt = C^H Gh C per k, and the mu-coupling sums */
    double Asum = 0.0, Z = 0.0, Bsum = 0.0;
    for (int k = 0; k < nk; ++k) {
        const double* Ck = C + (size_t)k * mat;
        double* Gtk = Gt + (size_t)k * mat;
        if (Gbar) {
            const double* Gk = Gbar + (size_t)k * mat;
            for (int i = 0; i < order; ++i)
                for (int j = 0; j < order; ++j) {
                    size_t o1 = ((size_t)i * order + j) * es, o2 = ((size_t)j * order + i) * es;
                    Gh[o1] = 0.5 * (Gk[o1] + Gk[o2]);
                    if (cplx) Gh[o1 + 1] = 0.5 * (Gk[o1 + 1] - Gk[o2 + 1]);
                }
            zmm(cplx, 0, order, order, Gh, order, Ck, T);   /* T = Gh C */
            zmm(cplx, 1, order, order, Ck, order, T, Gtk);  /* Gt = C^H T */
        }
        for (int i = 0; i < order; ++i) {
            double fpi = fp[(size_t)k * order + i];
            Asum += Gtk[((size_t)i * order + i) * es] * fpi;
            Z += wk[k] * fpi;
            Bsum += wk[k] * eps[(size_t)k * order + i] * fpi;
        }
    }
    double a_glob = (Z != 0.0) ? Asum / Z : 0.0;
    double b = (Z != 0.0) ? Bsum / Z : 0.0;
    for (int k = 0; k < nk; ++k) {
        const double* Ck = C + (size_t)k * mat;
        const double* ek = eps + (size_t)k * order;
        const double* fk = f + (size_t)k * order;
        const double* fpk = fp + (size_t)k * order;
        double* Gtk = Gt + (size_t)k * mat;
        double ak = wk[k] * a_glob;
        /* P1 = Gt o G1 - a diag f' + ebar diag(w);  P2 = Gt o G2 - a diag(f' eps) + ebar diag(w eps) */
        for (int i = 0; i < order; ++i)
            for (int j = 0; j < order; ++j) {
                double g1, g2;
                if (i == j) {
                    g1 = fpk[i];
                    g2 = fk[i] + ek[i] * fpk[i];
                } else {
                    g1 = g * fermi_dd((ek[i] - mu) / kT, (ek[j] - mu) / kT) / kT;
                    g2 = 0.5 * (fk[i] + fk[j]) + 0.5 * (ek[i] + ek[j]) * g1;
                }
                size_t o = ((size_t)i * order + j) * es;
                P1[o] = Gtk[o] * g1;
                P2[o] = Gtk[o] * g2;
                if (cplx) { P1[o + 1] = Gtk[o + 1] * g1; P2[o + 1] = Gtk[o + 1] * g2; }
                if (i == j) {
                    double wi = wk[k] * (fk[i] + (ek[i] - b) * fpk[i]);
                    P1[o] += -ak * fpk[i] + ebar * wi;
                    P2[o] += -ak * fpk[i] * ek[i] + ebar * wi * ek[i];
                }
            }
        /* Hbar = C P1 C^H; Sbar_NC = -C P2 C^H */
        double* CH = malloc(sizeof(double) * mat);
        for (int i = 0; i < order; ++i)
            for (int j = 0; j < order; ++j) {
                size_t d = ((size_t)i * order + j) * es, s = ((size_t)j * order + i) * es;
                CH[d] = Ck[s];
                if (cplx) CH[d + 1] = -Ck[s + 1];
            }
        zmm(cplx, 0, order, order, Ck, order, P1, T);
        zmm(cplx, 0, order, order, T, order, CH, Hbar + (size_t)k * mat);
        zmm(cplx, 0, order, order, Ck, order, P2, T);
        zmm(cplx, 0, order, order, T, order, CH, P1); /* P1 reused: C P2 C^H */
        double* Sk = Sbar + (size_t)k * n * n * es;
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                double re = 0.0, im = 0.0;
                for (int bb = 0; bb < nsp; ++bb) {
                    size_t o = (((size_t)(bb * n + i)) * order + (bb * n + j)) * es;
                    re += P1[o];
                    if (cplx) im += P1[o + 1];
                }
                size_t d = ((size_t)i * n + j) * es;
                Sk[d] = -re;
                if (cplx) Sk[d + 1] = -im;
            }
        free(CH);
    }
    free(fp); free(f); free(Gt); free(T); free(P1); free(P2); free(Gh);
}
