"""Stage-by-stage parity of the HIP kernels (through the test hooks of
include/ks_testing.h) against the oracle and closed forms."""
import ctypes
import math

import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2606_09058_amd import inputs as I
from paper_2606_09058_amd import ks
from tests.gpu_helpers import announce, dev, host, stream_handle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    lib = ks.lib()
    V, I32, D = ctypes.c_void_p, ctypes.c_int32, ctypes.c_double
    lib.ks_test_gemm.argtypes = [I32, I32, I32, I32, I32, I32, D, V, I32, V, I32, D, V, I32, I32, V]
    lib.ks_test_gemm.restype = I32
    lib.ks_test_potrf.argtypes = [I32, I32, V, I32, V, ctypes.POINTER(I32), V]
    lib.ks_test_potrf.restype = I32
    lib.ks_test_stedc.argtypes = [I32, V, V, V, V, ctypes.POINTER(I32), V]
    lib.ks_test_stedc.restype = I32
    lib.ks_test_hetrd.argtypes = [I32, I32, V, V, V, V, I32, V, V]
    lib.ks_test_hetrd.restype = I32
    lib.ks_test_mfma_layout.argtypes = [V, V]
    lib.ks_test_mfma_layout.restype = I32
    lib.ks_test_mfma_layout32.argtypes = [V, V]
    lib.ks_test_mfma_layout32.restype = I32
    return lib


def P(t):
    return ctypes.c_void_p(t.data_ptr())


def test_mfma_f64_lane_layout(L):
    announce("mfma layout")
    out = torch.zeros(256, dtype=torch.float64, device="cuda")
    assert L.ks_test_mfma_layout(P(out), stream_handle()) == 0
    o = host(out).reshape(64, 4)
    lane = np.arange(64)[:, None]
    r = np.arange(4)[None, :]
    expect = 100.0 * (lane // 16 + 4 * r) + lane % 16
    assert np.array_equal(o, expect), o


def test_mfma_f32_lane_layout(L):
    """The FP32 MFMA returns rows 4 (lane / 16) + r in register r (the FP64 one
    returns lane / 16 + 4 r); the FP32 GEMM's store depends on this."""
    announce("mfma f32 layout")
    out = torch.zeros(256, dtype=torch.float32, device="cuda")
    assert L.ks_test_mfma_layout32(P(out), stream_handle()) == 0
    o = host(out).reshape(64, 4)
    lane = np.arange(64)[:, None]
    r = np.arange(4)[None, :]
    expect = 100.0 * (4 * (lane // 16) + r) + lane % 16
    assert np.array_equal(o, expect), o


# the last shape has enough output tiles and k steps for the large-tile kernel
# in every precision (ragged in m, n and k for every tile and k-step size)
GEMM_SHAPES = [(1, 1, 1), (64, 64, 16), (65, 130, 17), (200, 77, 300), (5, 300, 64), (130, 1, 2),
               (4100, 4099, 270)]


@pytest.mark.parametrize("cplx", [False, True])
@pytest.mark.parametrize("opa,opb", [(0, 0), (0, 1), (0, 2), (1, 0), (2, 0)])
def test_gemm_matches_numpy(L, cplx, opa, opb):
    rng = np.random.default_rng(opa * 3 + opb)
    for (m, n, k) in GEMM_SHAPES:
        announce("gemm", cplx, opa, opb, m, n, k)
        dt = np.complex128 if cplx else np.float64

        def rnd(*s):
            x = rng.normal(size=s)
            return (x + 1j * rng.normal(size=s)) if cplx else x
        A = rnd(m, k) if opa == 0 else rnd(k, m)
        B = rnd(k, n) if opb == 0 else rnd(n, k)
        C0 = rnd(m, n)
        op = lambda X, o: X if o == 0 else (X.T if o == 1 else X.conj().T)  # noqa: E731
        alpha, beta = -0.7, 0.3
        ref = alpha * op(A, opa) @ op(B, opb) + beta * C0
        Ad, Bd, Cd = dev(A.astype(dt)), dev(B.astype(dt)), dev(C0.astype(dt))
        st = L.ks_test_gemm(int(cplx), opa, opb, m, n, k, alpha, P(Ad), A.shape[1], P(Bd), B.shape[1],
                            beta, P(Cd), n, 0, stream_handle())
        assert st == 0
        got = host(Cd)
        scale = np.abs(A).max() * np.abs(B).max() * k + 1
        assert np.abs(got - ref).max() < 1e-13 * scale, (m, n, k)


@pytest.mark.parametrize("cplx", [False, True])
@pytest.mark.parametrize("opa,opb", [(0, 0), (0, 1), (0, 2), (1, 0), (2, 0)])
def test_gemm_fp32_matches_numpy(L, cplx, opa, opb):
    """FP32 matrix-core GEMM (FP32 accumulation) against a float64 product of the
    same FP32-rounded operands; the bound is a few units of FP32 rounding per
    accumulated term, far below what a wrong lane mapping would give."""
    rng = np.random.default_rng(100 + opa * 3 + opb)
    for (m, n, k) in GEMM_SHAPES:
        announce("gemm fp32", cplx, opa, opb, m, n, k)
        dt = np.complex64 if cplx else np.float32

        def rnd(*s):
            x = rng.normal(size=s)
            return ((x + 1j * rng.normal(size=s)) if cplx else x).astype(dt)
        A = rnd(m, k) if opa == 0 else rnd(k, m)
        B = rnd(k, n) if opb == 0 else rnd(n, k)
        C0 = rnd(m, n)
        op = lambda X, o: X if o == 0 else (X.T if o == 1 else X.conj().T)  # noqa: E731
        alpha, beta = -0.7, 0.3
        wide = np.complex128 if cplx else np.float64
        ref = alpha * op(A.astype(wide), opa) @ op(B.astype(wide), opb) + beta * C0.astype(wide)
        Ad, Bd, Cd = dev(A), dev(B), dev(C0)
        st = L.ks_test_gemm(3 if cplx else 2, opa, opb, m, n, k, alpha, P(Ad), A.shape[1], P(Bd),
                            B.shape[1], beta, P(Cd), n, 0, stream_handle())
        assert st == 0
        got = host(Cd).astype(wide)
        scale = np.abs(A).max() * np.abs(B).max() * k + 1
        assert np.abs(got - ref).max() < 4e-7 * scale, (m, n, k)


@pytest.mark.parametrize("m,k", [(150, 40), (5800, 260)])
def test_gemm_lower_only(L, m, k):
    """Only the lower triangle is written; the second shape takes the large-tile kernel."""
    rng = np.random.default_rng(5)
    A = rng.normal(size=(m, k))
    C0 = rng.normal(size=(m, m))
    Cd = dev(C0)
    Ad = dev(A)
    announce("gemm lower")
    assert L.ks_test_gemm(0, 0, 1, m, m, k, 1.0, P(Ad), k, P(Ad), k, 1.0, P(Cd), m, 1,
                          stream_handle()) == 0
    got = host(Cd)
    ref = C0 + A @ A.T
    low = np.tril(np.ones((m, m), bool))
    assert np.abs(got[low] - ref[low]).max() < 1e-12
    assert np.array_equal(got[~low], C0[~low])


@pytest.mark.parametrize("fp32", [False, True])
@pytest.mark.parametrize("m,n,k", [(150, 150, 64), (1000, 1000, 37), (67, 200, 1), (4100, 4100, 64)])
def test_gemm_rank_update_lower(L, m, n, k, fp32):
    """C = C - A^T B on the lower triangle with k <= 64 (the trailing-update form,
    A and B stored k x m, k x n): ragged tiles, a partial last k step, and the
    upper triangle left untouched."""
    announce("gemm rank update", m, n, k, fp32)
    rng = np.random.default_rng(m + k)
    dt = np.float32 if fp32 else np.float64
    A = rng.normal(size=(k, m)).astype(dt)
    B = rng.normal(size=(k, n)).astype(dt)
    C0 = rng.normal(size=(m, n)).astype(dt)
    Cd = dev(C0)
    assert L.ks_test_gemm(2 if fp32 else 0, 1, 0, m, n, k, -1.0, P(dev(A)), m, P(dev(B)), n, 1.0, P(Cd), n, 1,
                          stream_handle()) == 0
    got = host(Cd).astype(np.float64)
    ref = C0.astype(np.float64) - A.astype(np.float64).T @ B.astype(np.float64)
    low = np.tril(np.ones((m, n), bool))
    tol = (4e-7 if fp32 else 1e-13) * (k + 1) * 16
    assert np.abs(got[low] - ref[low]).max() < tol
    assert np.array_equal(got[~low], C0.astype(np.float64)[~low])


@pytest.mark.parametrize("n", [1, 31, 63, 64, 65, 100, 127, 128, 129, 200, 257, 330])
@pytest.mark.parametrize("cplx", [False, True])
def test_potrf_matches_oracle(L, n, cplx):
    """Blocked Cholesky (64-column blocks, ragged last block) against the oracle's
    column algorithm, and the inverse factor: L^-1 L = I, zeros above the diagonal."""
    announce("potrf", n, cplx)
    rng = np.random.default_rng(n)
    S = I.random_spd(rng, n, cplx)
    A = dev(S)
    Li = torch.full((n, n), 7.0, dtype=A.dtype, device="cuda")
    info = ctypes.c_int32(-1)
    assert L.ks_test_potrf(int(cplx), n, P(A), n, P(Li), ctypes.byref(info), stream_handle()) == 0
    assert info.value == 0
    Lg = np.tril(host(A))
    Lo = O.cholesky(S)
    assert np.abs(Lg - Lo).max() < 1e-12 * np.abs(Lo).max()
    Lih = host(Li)
    assert np.array_equal(np.triu(Lih, 1), np.zeros((n, n)))
    assert np.abs(Lih @ Lo - np.eye(n)).max() < 1e-11 * max(1.0, np.linalg.cond(Lo))


def test_potrf_reports_failing_column(L):
    n = 70
    rng = np.random.default_rng(1)
    S = I.random_spd(rng, n, False)
    S[50, 50] = -5.0
    with pytest.raises(O.OracleError) as ex:
        O.cholesky(S)
    col = int(str(ex.value).split()[-1])
    A = dev(S)
    info = ctypes.c_int32(-1)
    announce("potrf failure")
    assert L.ks_test_potrf(0, n, P(A), n, None, ctypes.byref(info), stream_handle()) == 0
    assert info.value == col


def run_stedc(L, d, e):
    n = len(d)
    dd, ed = dev(d), dev(e if n > 1 else np.zeros(1))
    lam = torch.zeros(n, dtype=torch.float64, device="cuda")
    Z = torch.zeros((n, n), dtype=torch.float64, device="cuda")
    info = ctypes.c_int32(-1)
    st = L.ks_test_stedc(n, P(dd), P(ed), P(lam), P(Z), ctypes.byref(info), stream_handle())
    assert st == 0
    return host(lam), host(Z), info.value


def tridiag(d, e):
    return np.diag(d) + np.diag(e, 1) + np.diag(e, -1)


@pytest.mark.parametrize("n", [1, 2, 31, 32, 33, 64, 100, 1000])
def test_stedc_toeplitz_closed_form(L, n):
    """tridiag(b, a, b): lambda_k = a + 2|b| cos(k pi / (n+1))."""
    announce("stedc toeplitz", n)
    a, b = 0.3, -0.9
    lam, Z, info = run_stedc(L, np.full(n, a), np.full(max(n - 1, 0), b))
    assert info == 0
    k = np.arange(1, n + 1)
    ref = np.sort(a + 2 * abs(b) * np.cos(k * np.pi / (n + 1)))
    assert np.abs(lam - ref).max() < 1e-13 * n
    T = tridiag(np.full(n, a), np.full(n - 1, b))
    assert np.abs(Z.T @ Z - np.eye(n)).max() < 1e-12
    assert np.abs(T @ Z - Z * lam).max() < 1e-12


@pytest.mark.parametrize("n", [10, 100, 401])
def test_stedc_clement_integer_spectrum(L, n):
    announce("stedc clement", n)
    e = np.sqrt(np.arange(1, n) * (n - np.arange(1, n)))
    lam, Z, info = run_stedc(L, np.zeros(n), e)
    assert info == 0
    ref = np.arange(-(n - 1), n, 2, dtype=np.float64)
    assert np.abs(lam - ref).max() < 1e-11 * n


@pytest.mark.parametrize("n,seed", [(50, 0), (333, 1), (1024, 2)])
def test_stedc_random_vs_oracle(L, n, seed):
    announce("stedc random", n)
    rng = np.random.default_rng(seed)
    d = rng.normal(size=n)
    e = rng.normal(size=n - 1)
    lam, Z, info = run_stedc(L, d, e)
    assert info == 0
    T = tridiag(d, e)
    w, V, _ = O.jacobi(T)
    assert np.abs(lam - w).max() < 1e-12 * np.abs(w).max() * 10
    assert np.abs(Z.T @ Z - np.eye(n)).max() < 1e-12
    assert np.abs(T @ Z - Z * lam).max() < 1e-12 * np.abs(w).max() * 10


def test_stedc_exact_deflation_and_clusters(L):
    """Block-diagonal T (zero couplings), repeated diagonal values (clusters) and a
    Wilkinson-type matrix with pairs close to machine precision."""
    announce("stedc deflation")
    n = 300
    rng = np.random.default_rng(3)
    d = np.round(rng.normal(size=n), 1)  # many exact ties
    e = rng.normal(size=n - 1) * 1e-3
    e[::7] = 0.0
    for dd, ee in [(d, e), (np.abs(np.arange(-(n // 2), n - n // 2)).astype(float), np.ones(n - 1))]:
        lam, Z, info = run_stedc(L, dd, ee)
        assert info == 0
        T = tridiag(dd, ee)
        w, _, _ = O.jacobi(T)
        scale = max(1.0, np.abs(w).max())
        assert np.abs(lam - w).max() < 1e-12 * scale * 10
        assert np.abs(Z.T @ Z - np.eye(n)).max() < 1e-12
        assert np.abs(T @ Z - Z * lam).max() < 1e-12 * scale * 10


@pytest.mark.parametrize("n", [1, 2, 3, 33, 100, 130, 333, 600])
@pytest.mark.parametrize("cplx", [False, True])
def test_hetrd_similarity(L, n, cplx):
    """A = Q T Q^H: eig(T) = eig(A) (oracle), Q unitary, Q T Q^H reproduces A."""
    announce("hetrd", n, cplx)
    rng = np.random.default_rng(n + 7)
    A = I.random_hermitian(rng, n, cplx)
    dt = np.complex128 if cplx else np.float64
    Ad = dev(A.astype(dt))
    d = torch.zeros(n, dtype=torch.float64, device="cuda")
    e = torch.zeros(max(n, 1), dtype=torch.float64, device="cuda")
    X = dev(np.eye(n))
    Y = torch.zeros((n, n), dtype=torch.complex128 if cplx else torch.float64, device="cuda")
    st = L.ks_test_hetrd(int(cplx), n, P(Ad), P(d), P(e), P(X), n, P(Y), stream_handle())
    assert st == 0
    dh, eh, Q = host(d), host(e)[:n - 1], host(Y)
    T = tridiag(dh, eh)
    assert np.abs(Q.conj().T @ Q - np.eye(n)).max() < 1e-12
    assert np.abs(Q @ T @ Q.conj().T - A).max() < 1e-12 * max(1.0, np.abs(A).max()) * n
    wT, _, _ = O.jacobi(T)
    wA, _, _ = O.jacobi(A)
    assert np.abs(wT - wA).max() < 1e-12 * n


@pytest.mark.parametrize("n", [4100, 6150])
def test_hetrd_similarity_large_orders(L, n):
    """Orders 4100 and 6150 take 256-reflector compact-WY blocks in the
    back-transform (16 full blocks and a ragged one of 3; 24 and a ragged one
    of 5) and the large-tile GEMMs: Q unitary and Q T Q^H = A (which fix
    eig(T) = eig(A))."""
    announce("hetrd", n)
    rng = np.random.default_rng(11)
    A = I.random_hermitian(rng, n, False)
    Ad = dev(A)
    d = torch.zeros(n, dtype=torch.float64, device="cuda")
    e = torch.zeros(n, dtype=torch.float64, device="cuda")
    X = dev(np.eye(n))
    Y = torch.zeros((n, n), dtype=torch.float64, device="cuda")
    assert L.ks_test_hetrd(0, n, P(Ad), P(d), P(e), P(X), n, P(Y), stream_handle()) == 0
    dh, eh, Q = host(d), host(e)[:n - 1], host(Y)
    T = tridiag(dh, eh)
    assert np.abs(Q.T @ Q - np.eye(n)).max() < 1e-12
    assert np.abs(Q @ T @ Q.T - A).max() < 1e-12 * max(1.0, np.abs(A).max()) * n


@pytest.mark.parametrize("n", [4100, 6150])
def test_hetrd_similarity_large_orders_complex(L, n):
    """Complex Hermitian orders 4100 and 6150: the complex symmetric product and
    column kernels over many panels, 256-reflector complex compact-WY blocks with
    a ragged last block and the complex large-tile GEMMs.  Q unitary and
    Q T Q^H = A (which fix eig(T) = eig(A)), checked with FP64 products on the
    device."""
    announce("hetrd complex", n)
    rng = np.random.default_rng(n + 3)
    A = I.random_hermitian(rng, n, True)
    Ad = dev(A)
    A0 = Ad.clone()
    d = torch.zeros(n, dtype=torch.float64, device="cuda")
    e = torch.zeros(n, dtype=torch.float64, device="cuda")
    X = dev(np.eye(n))
    Y = torch.zeros((n, n), dtype=torch.complex128, device="cuda")
    assert L.ks_test_hetrd(1, n, P(Ad), P(d), P(e), P(X), n, P(Y), stream_handle()) == 0
    torch.cuda.synchronize()
    T = torch.diag(d.to(torch.complex128)) + torch.diag(e[:n - 1].to(torch.complex128), 1) + \
        torch.diag(e[:n - 1].to(torch.complex128), -1)
    Yh = Y.conj().T.contiguous()
    err_u = ((Yh @ Y) - torch.eye(n, dtype=torch.complex128, device="cuda")).abs().max().item()
    err_s = ((Y @ T) @ Yh - A0).abs().max().item()
    assert err_u < 1e-12, err_u
    assert err_s < 1e-12 * max(1.0, A0.abs().max().item()) * n, err_s
