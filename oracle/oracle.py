"""ctypes front end of the plain FP64 CPU oracle (``ks_oracle.c``).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this module.  The product path
(the HIP library and its Python binding) never imports it and shares no code
with it.

Every function takes and returns numpy arrays (float64 / complex128, C order)
and follows the paper's definitions:

* ``gevd``          -- H C = S C eps (Sec. 2; spinor form with S_NC = diag(S, S),
                       Sec. 3.2) by Cholesky + cyclic Jacobi,
* ``gevd_lowdin``   -- the same problem by the Loewdin route of Sec. 3.1
                       (Parts 2-1..2-5) / Sec. 3.2 (Parts 3-1..3-6),
* ``gevd_canonical``-- the Loewdin route with the eigenvectors of S whose
                       eigenvalue is at most tau * max(s) left out (canonical
                       orthogonalisation of an overcomplete basis),
* ``fermi``         -- occupations and the chemical potential by bisection on
                       the electron count (Part 3 of Sec. 3.1),
* ``density``       -- rho = C f C^H (Sec. 2 density matrix, conjugated),
* ``energy_density``-- E = C diag(f eps) C^H (the energy-density matrix),
* ``bloch_sum``     -- X(k) = sum_R X_R exp(i k.R) (the Bloch sums of Sec. 2),
* ``adjoint``       -- dense gradients of L(rho, E_band) w.r.t. H and S,
* ``cholesky``, ``solve_lower``, ``solve_lower_h``, ``jacobi`` -- the steps.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ks_oracle.c")
_LIB = os.path.join(_HERE, "libks_oracle.so")


def build(force: bool = False) -> str:
    """Compile ks_oracle.c with gcc (OpenMP) into oracle/libks_oracle.so."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-march=x86-64-v2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
               "-o", tmp, _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None
_lib_threads = [1]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        I = ctypes.c_int
        D = ctypes.c_double
        L.ko_max_threads.restype = I
        L.ko_set_threads.argtypes = [I]
        L.ko_set_threads.restype = None
        _lib_threads[0] = L.ko_max_threads()
        L.ko_cholesky.argtypes = [I, I, P, I, P]
        L.ko_cholesky.restype = I
        L.ko_solve_lower.argtypes = [I, I, I, P, P, I]
        L.ko_solve_lower_h.argtypes = [I, I, I, P, P, I]
        L.ko_jacobi.argtypes = [I, I, P, P, P, I, I]
        L.ko_jacobi.restype = I
        L.ko_gevd.argtypes = [I, I, I, P, I, P, I, P, P, I, ctypes.POINTER(I)]
        L.ko_gevd.restype = I
        L.ko_gevd_lowdin.argtypes = [I, I, I, P, I, P, I, P, P, I]
        L.ko_gevd_lowdin.restype = I
        L.ko_fermi.argtypes = [I, I, P, P, D, D, D, ctypes.POINTER(D), P, ctypes.POINTER(D),
                               ctypes.POINTER(D)]
        L.ko_fermi.restype = I
        L.ko_density.argtypes = [I, I, I, P, I, P, P]
        L.ko_adjoint.argtypes = [I, I, I, I, P, P, D, D, D, P, P, D, P, P]
        _lib = L
    return _lib


class OracleError(RuntimeError):
    pass


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _dt(a):
    return np.complex128 if np.iscomplexobj(a) else np.float64


def _threads(nthreads, order):
    """Threads for a call: 1 for small orders (OpenMP start-up dominates there)."""
    if nthreads and nthreads > 0:
        return int(nthreads)
    return 1 if order <= 256 else 0


def _set(nthreads, order):
    t = _threads(nthreads, order)
    lib().ko_set_threads(t if t > 0 else _lib_threads[0])


def max_threads() -> int:
    return lib().ko_max_threads()


def cholesky(S):
    """Lower L with S = L L^H (reads the lower triangle of S)."""
    dt = _dt(S)
    S = _c(S, dt)
    n = S.shape[0]
    L = np.zeros((n, n), dt)
    info = lib().ko_cholesky(n, int(dt == np.complex128), _ptr(S), n, _ptr(L))
    if info:
        raise OracleError("S not positive definite at column %d" % info)
    return L


def solve_lower(L, B):
    """L^-1 B by forward substitution."""
    dt = np.complex128 if (np.iscomplexobj(L) or np.iscomplexobj(B)) else np.float64
    L = _c(L, dt)
    X = np.array(B, dtype=dt, order="C", copy=True)
    if X.ndim == 1:
        X = X[:, None]
    lib().ko_solve_lower(L.shape[0], X.shape[1], int(dt == np.complex128), _ptr(L), _ptr(X), X.shape[1])
    return X


def solve_lower_h(L, B):
    """L^-H B by back substitution."""
    dt = np.complex128 if (np.iscomplexobj(L) or np.iscomplexobj(B)) else np.float64
    L = _c(L, dt)
    X = np.array(B, dtype=dt, order="C", copy=True)
    if X.ndim == 1:
        X = X[:, None]
    lib().ko_solve_lower_h(L.shape[0], X.shape[1], int(dt == np.complex128), _ptr(L), _ptr(X), X.shape[1])
    return X


def jacobi(A, maxsweeps=50, nthreads=0):
    """Eigen-decomposition of the Hermitian A (full storage): (w ascending, V, sweeps)."""
    dt = _dt(A)
    A = np.array(A, dtype=dt, order="C", copy=True)
    n = A.shape[0]
    w = np.zeros(n)
    V = np.zeros((n, n), dt)
    sw = lib().ko_jacobi(n, int(dt == np.complex128), _ptr(A), _ptr(w), _ptr(V), maxsweeps,
                         _threads(nthreads, n))
    if sw < 0:
        raise OracleError("Jacobi did not converge in %d sweeps" % maxsweeps)
    return w, V, sw


def gevd(H, S, nsp=1, nthreads=0, route="cholesky"):
    """Solve H C = S_NC C eps; nsp=2 is the spinor form (H is 2n x 2n, S is n x n).

    Returns (eps ascending, C with eigenvectors as columns)."""
    dt = np.complex128 if (np.iscomplexobj(H) or np.iscomplexobj(S)) else np.float64
    H = _c(H, dt)
    S = _c(S, dt)
    n = S.shape[0]
    order = n * nsp
    assert H.shape == (order, order), (H.shape, order)
    eps = np.zeros(order)
    C = np.zeros((order, order), dt)
    cp = int(dt == np.complex128)
    nthreads = _threads(nthreads, order)
    if route == "cholesky":
        sw = ctypes.c_int(0)
        info = lib().ko_gevd(n, nsp, cp, _ptr(H), order, _ptr(S), n, _ptr(eps), _ptr(C), nthreads,
                             ctypes.byref(sw))
    elif route == "lowdin":
        info = lib().ko_gevd_lowdin(n, nsp, cp, _ptr(H), order, _ptr(S), n, _ptr(eps), _ptr(C), nthreads)
    else:
        raise ValueError(route)
    if info < 0:
        raise OracleError("S not positive definite at column %d" % (-info))
    if info > 0:
        raise OracleError("Jacobi did not converge")
    return eps, C


def gevd_lowdin(H, S, nsp=1, nthreads=0):
    return gevd(H, S, nsp=nsp, nthreads=nthreads, route="lowdin")


def gevd_canonical(H, S, tau, nsp=1, nthreads=0):
    """The Loewdin route (Sec. 3.1 Parts 2-1..2-5, Sec. 3.2 Parts 3-1..3-6) on
    the eigenvectors of S that are kept: U^H S U = s (ascending), keep the
    columns with s_j > tau * max(s), V = U_keep s_keep^-1/2, V_NC = diag(V, V),
    H' = V_NC^H H V_NC, H' C' = C' eps, C = V_NC C'.  With tau = 0 every s_j
    must be positive.  H and S in full storage.

    Returns (eps ascending (nsp*m,), C (order, nsp*m), m = number kept)."""
    dt = np.complex128 if (np.iscomplexobj(H) or np.iscomplexobj(S)) else np.float64
    H = _c(H, dt)
    S = _c(S, dt)
    n = S.shape[0]
    assert H.shape == (nsp * n, nsp * n)
    s, U, _ = jacobi(S, nthreads=nthreads)
    if not s[-1] > 0.0:
        raise OracleError("S has no positive eigenvalue")
    keep = s > tau * s[-1]
    if tau == 0.0 and not keep.all():
        raise OracleError("S not positive definite: %d eigenvalues <= 0" % int((~keep).sum()))
    V = U[:, keep] / np.sqrt(s[keep])
    VN = np.kron(np.eye(nsp), V)
    Hp = VN.conj().T @ H @ VN
    Hp = 0.5 * (Hp + Hp.conj().T)
    eps, Cp, _ = jacobi(Hp, nthreads=nthreads)
    return eps, VN @ Cp, int(keep.sum())


def fermi(eps, ne, kT, g, wk=None):
    """Common mu over k-points by bisection.  eps is (nk, order) or (order,).

    Returns dict(mu, occ (same shape as eps), eband, ts, iters)."""
    e = np.atleast_2d(np.ascontiguousarray(eps, dtype=np.float64))
    nk, order = e.shape
    w = np.full(nk, 1.0 / nk) if wk is None else _c(wk, np.float64)
    occ = np.zeros_like(e)
    mu = ctypes.c_double(0)
    eb = ctypes.c_double(0)
    ts = ctypes.c_double(0)
    it = lib().ko_fermi(nk, order, _ptr(e), _ptr(w), float(g), float(ne), float(kT), ctypes.byref(mu),
                        _ptr(occ), ctypes.byref(eb), ctypes.byref(ts))
    return dict(mu=mu.value, occ=occ.reshape(np.shape(eps)), eband=eb.value, ts=ts.value, iters=it)


def density(C, w):
    """rho = C diag(w) C^H over the columns of C (w real, one per column)."""
    dt = _dt(C)
    C = _c(C, dt)
    w = _c(w, np.float64)
    order, ncols = C.shape
    assert w.shape == (ncols,)
    rho = np.zeros((order, order), dt)
    _set(0, order)
    lib().ko_density(order, ncols, int(dt == np.complex128), _ptr(C), ncols, _ptr(w), _ptr(rho))
    return rho


def bloch_sum(XR, R, kvec):
    """Bloch sums X(k) = sum_R X_R exp(i k.R) (Sec. 2, the Bloch-sum equations for
    H(k) and S(k)): XR (nR, n, n), R (nR, 3), kvec (nk, 3) -> (nk, n, n) complex."""
    XR = np.asarray(XR, dtype=np.float64)
    ph = np.exp(1j * (np.asarray(kvec, dtype=np.float64) @ np.asarray(R, dtype=np.float64).T))  # (nk, nR)
    return np.einsum("kr,rij->kij", ph, XR)


def energy_density(C, occ, eps):
    """Energy-density matrix E = C diag(f eps) C^H over the columns of C (the
    Part 4 quantity of Sec. 3.1 used for forces): the density-matrix sum with
    weights f_i eps_i."""
    return density(C, np.asarray(occ, dtype=np.float64) * np.asarray(eps, dtype=np.float64))


def adjoint(eps, C, mu, kT, g, Gbar=None, ebar=0.0, nsp=1, wk=None):
    """Dense gradients (Hbar, Sbar) of L(rho, E_band).

    eps: (nk, order) or (order,); C: (nk, order, order) or (order, order) with all
    eigenvectors; Gbar: dL/drho with C's shape or None; ebar: dL/dE_band.
    Hbar has C's shape; Sbar is (nk, n, n) / (n, n) with n = order / nsp."""
    single = np.ndim(eps) == 1
    dt = _dt(C)
    e = np.atleast_2d(np.ascontiguousarray(eps, dtype=np.float64))
    nk, order = e.shape
    Cc = _c(C, dt).reshape(nk, order, order)
    n = order // nsp
    w = np.full(nk, 1.0 / nk) if wk is None else _c(wk, np.float64)
    G = None if Gbar is None else _c(Gbar, dt).reshape(nk, order, order)
    Hb = np.zeros((nk, order, order), dt)
    Sb = np.zeros((nk, n, n), dt)
    _set(0, order)
    lib().ko_adjoint(n, nsp, int(dt == np.complex128), nk, _ptr(e), _ptr(Cc), float(mu), float(kT),
                     float(g), _ptr(w), None if G is None else _ptr(G), float(ebar), _ptr(Hb), _ptr(Sb))
    if single:
        return Hb[0], Sb[0]
    return Hb, Sb


def solve(H, S, ne, kT, nsp=1, g=None, nthreads=0, route="cholesky"):
    """Whole oracle pass for one k-point: eps, C, mu, occ, eband, rho."""
    if g is None:
        g = 2.0 if nsp == 1 else 1.0
    eps, C = gevd(H, S, nsp=nsp, nthreads=nthreads, route=route)
    fr = fermi(eps, ne, kT, g)
    rho = density(C, fr["occ"])
    return dict(eps=eps, C=C, mu=fr["mu"], occ=fr["occ"], eband=fr["eband"], ts=fr["ts"], rho=rho, g=g)
