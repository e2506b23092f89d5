"""The two-stage reduction (KS_PLAN_TWOSTAGE): the band stage alone, the whole
tridiagonalisation, and the full solve against the oracle."""
import ctypes

import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2606_09058_amd import inputs as I
from paper_2606_09058_amd import ks
from tests.gpu_helpers import announce, dev, host, residuals, stream_handle

pytestmark = pytest.mark.gpu
KB = 32  # half-bandwidth between the stages


@pytest.fixture(scope="module")
def L():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    lib = ks.lib()
    V, I32 = ctypes.c_void_p, ctypes.c_int32
    lib.ks_test_hetrd2.argtypes = [I32, I32, V, V, V, V, I32, V, V]
    lib.ks_test_hetrd2.restype = I32
    lib.ks_test_he2hb.argtypes = [I32, I32, V, V, I32, V, V]
    lib.ks_test_he2hb.restype = I32
    return lib


def P(t):
    return ctypes.c_void_p(t.data_ptr())


def tridiag(d, e):
    return np.diag(d) + np.diag(e, 1) + np.diag(e, -1)


SIZES = [1, 2, 3, 31, 33, 34, 64, 65, 100, 333, 600, 1100]


@pytest.mark.parametrize("n", SIZES)
@pytest.mark.parametrize("cplx", [False, True])
def test_band_stage(L, n, cplx):
    """Stage 1: B = Q1^H A Q1 has half-bandwidth 32 (exact zeros below the
    band), Q1 is unitary and Q1 B Q1^H = A.  Sizes cross the panel width, and
    600 / 1100 rows spread a panel over several workgroups."""
    announce("he2hb", n, cplx)
    rng = np.random.default_rng(n + 17)
    A = I.random_hermitian(rng, n, cplx)
    dt = np.complex128 if cplx else np.float64
    Ad = dev(A.astype(dt))
    X = dev(np.eye(n))
    Y = torch.zeros((n, n), dtype=torch.complex128 if cplx else torch.float64, device="cuda")
    assert L.ks_test_he2hb(int(cplx), n, P(Ad), P(X), n, P(Y), stream_handle()) == 0
    Bl = np.tril(host(Ad))
    i, j = np.indices((n, n))
    assert np.all(Bl[(i - j) > KB] == 0)
    B = Bl + np.tril(Bl, -1).conj().T
    Q = host(Y)
    assert np.abs(Q.conj().T @ Q - np.eye(n)).max() < 1e-12
    assert np.abs(Q @ B @ Q.conj().T - A).max() < 1e-12 * max(1.0, np.abs(A).max()) * max(n, 1)


@pytest.mark.parametrize("n", SIZES)
@pytest.mark.parametrize("cplx", [False, True])
def test_twostage_similarity(L, n, cplx):
    """Both stages: A = Q T Q^H with T real tridiagonal, Q = Q1 Q2 unitary,
    eig(T) = eig(A) (oracle Jacobi)."""
    announce("hetrd2", n, cplx)
    rng = np.random.default_rng(n + 7)
    A = I.random_hermitian(rng, n, cplx)
    dt = np.complex128 if cplx else np.float64
    Ad = dev(A.astype(dt))
    d = torch.zeros(n, dtype=torch.float64, device="cuda")
    e = torch.zeros(max(n, 1), dtype=torch.float64, device="cuda")
    X = dev(np.eye(n))
    Y = torch.zeros((n, n), dtype=torch.complex128 if cplx else torch.float64, device="cuda")
    assert L.ks_test_hetrd2(int(cplx), n, P(Ad), P(d), P(e), P(X), n, P(Y), stream_handle()) == 0
    dh, eh, Q = host(d), host(e)[:n - 1], host(Y)
    T = tridiag(dh, eh)
    assert np.abs(Q.conj().T @ Q - np.eye(n)).max() < 1e-12
    assert np.abs(Q @ T @ Q.conj().T - A).max() < 1e-12 * max(1.0, np.abs(A).max()) * n
    if n <= 600:
        wT, _, _ = O.jacobi(T)
        wA, _, _ = O.jacobi(A)
        assert np.abs(wT - wA).max() < 1e-12 * n


def test_twostage_already_tridiagonal(L):
    """A tridiagonal input keeps its spectrum, and a diagonal one its diagonal
    (every reflector of both stages is the identity: tau = 0 on zero columns)."""
    announce("hetrd2 diagonal")
    n = 200
    rng = np.random.default_rng(3)
    dd = rng.uniform(-1, 1, n)
    A = np.diag(dd)
    Ad = dev(A)
    d = torch.zeros(n, dtype=torch.float64, device="cuda")
    e = torch.zeros(n, dtype=torch.float64, device="cuda")
    X = dev(np.eye(n))
    Y = torch.zeros((n, n), dtype=torch.float64, device="cuda")
    assert L.ks_test_hetrd2(0, n, P(Ad), P(d), P(e), P(X), n, P(Y), stream_handle()) == 0
    assert np.array_equal(host(d), dd)
    assert np.all(host(e)[:n - 1] == 0)
    assert np.array_equal(host(Y), np.eye(n))


@pytest.mark.parametrize("n,cplx", [(4100, False), (4100, True), (6150, False)])
def test_twostage_similarity_large_orders(L, n, cplx):
    """Orders 4100 / 6150: many panels over several workgroups, hundreds of
    sweeps in flight across workgroups, 256-reflector blocks in the panel
    back-transform.  Q unitary and Q T Q^H = A, in FP64 products on the device."""
    announce("hetrd2 large", n, cplx)
    rng = np.random.default_rng(n + 5)
    A = I.random_hermitian(rng, n, cplx)
    tdt = torch.complex128 if cplx else torch.float64
    Ad = dev(A)
    A0 = Ad.clone()
    d = torch.zeros(n, dtype=torch.float64, device="cuda")
    e = torch.zeros(n, dtype=torch.float64, device="cuda")
    X = dev(np.eye(n))
    Y = torch.zeros((n, n), dtype=tdt, device="cuda")
    assert L.ks_test_hetrd2(int(cplx), n, P(Ad), P(d), P(e), P(X), n, P(Y), stream_handle()) == 0
    torch.cuda.synchronize()
    T = torch.diag(d.to(tdt)) + torch.diag(e[:n - 1].to(tdt), 1) + torch.diag(e[:n - 1].to(tdt), -1)
    Yh = Y.conj().T.contiguous()
    err_u = ((Yh @ Y) - torch.eye(n, dtype=tdt, device="cuda")).abs().max().item()
    err_s = ((Y @ T) @ Yh - A0).abs().max().item()
    assert err_u < 1e-12, err_u
    assert err_s < 1e-12 * max(1.0, A0.abs().max().item()) * n, err_s


# ---------------------------------------------------------------- full solve
from tests.gpu_helpers import solve_gpu  # noqa: E402

TWO = ks.KS_PLAN_TWOSTAGE
EPS_TOL, RES_TOL, ORTH_TOL, RHO_TOL, MU_TOL = 1e-10, 1e-12, 1e-11, 1e-9, 1e-9


def compare(p, g, o):
    assert np.abs(g["eps"] - o["eps"]).max() < EPS_TOL
    res, orth = residuals(p.H, p.S, g["eps"], g["C"], p.nsp)
    assert res < RES_TOL, res
    assert orth < ORTH_TOL, orth
    assert abs(g["eband"] - o["eband"]) < MU_TOL * max(1.0, abs(o["eband"]))
    assert abs(g["mu"] - o["mu"]) < MU_TOL
    assert np.abs(g["rho"] - o["rho"]).max() < RHO_TOL
    assert np.abs(g["occ"] - o["occ"]).max() < 1e-9


@pytest.mark.parametrize("natoms,norb", [(1, 1), (1, 3), (4, 8), (8, 8), (12, 8), (10, 13), (16, 13), (24, 13)])
@pytest.mark.parametrize("cplx", [False, True])
def test_collinear_vs_oracle(natoms, norb, cplx):
    """Orders 1 .. 312 (a single element, exactly one and three bands, ragged
    panels) against the oracle, element by element."""
    announce("twostage collinear", natoms, norb, cplx)
    ne = min(max(1.0, round(0.3 * natoms * norb)) * 2.0, 2.0 * natoms * norb)
    p = I.toy(seed=natoms * 100 + norb + 1, natoms=natoms, norb=norb, edge=10 * (natoms / 8) ** (1 / 3) + 1,
              n_electrons=ne, kT=0.01, phases=cplx)
    g, _ = solve_gpu(p, flags=TWO)
    compare(p, g, O.solve(p.H, p.S, p.n_electrons, p.kT))


@pytest.mark.parametrize("natoms", [2, 7, 20])
def test_noncollinear_vs_oracle(natoms):
    announce("twostage noncollinear", natoms)
    p = I.noncollinear(seed=natoms, nx=natoms, ny=1, nz=1, lam_max=0.2)
    g, _ = solve_gpu(p, flags=TWO)
    compare(p, g, O.solve(p.H, p.S, p.n_electrons, p.kT, nsp=2))


def test_kpoint_batch_common_mu():
    """Six k-points in one plan (every kernel takes the batch; the waiting
    kernels of the band reduction and the chasing take one workgroup set per
    k-point), one common mu, against the oracle per k-point."""
    announce("twostage kpoint batch")
    p = I.kpoint_batch(natoms=6, norb=13, kgrid=(3, 2, 1))
    g, _ = solve_gpu(p, flags=TWO)
    eps_o, Cs = [], []
    for k in range(p.batch):
        e, C = O.gevd(p.H[k], p.S[k])
        eps_o.append(e)
        Cs.append(C)
    fr = O.fermi(np.array(eps_o), p.n_electrons, p.kT, p.g, wk=p.weights)
    assert np.abs(g["eps"] - np.array(eps_o)).max() < EPS_TOL
    assert abs(g["mu"] - fr["mu"]) < MU_TOL
    assert abs(g["eband"] - fr["eband"]) < MU_TOL
    for k in range(p.batch):
        assert np.abs(g["rho"][k] - O.density(Cs[k], fr["occ"][k])).max() < RHO_TOL
        res, orth = residuals(p.H[k], p.S[k], g["eps"][k], g["C"][k])
        assert res < RES_TOL and orth < ORTH_TOL


def _gevd(plan, H, S, il=1, iu=None):
    eps = torch.empty(plan._vshape(), dtype=torch.float64, device="cuda")
    C = torch.zeros(plan._mshape(), dtype=plan.mdtype, device="cuda")
    plan.gevd(H, S, eps, C, il=il, iu=iu)
    plan.check("gevd")
    return host(eps), host(C)


@pytest.mark.parametrize("kind", ["real", "complex", "noncollinear"])
def test_batched_equals_single_solves_bitwise(kind):
    """The batch index only selects the matrix in every launch (and the fixed
    order of every reduction does not depend on it), so batched two-stage
    solves equal the single ones bit for bit, full and windowed."""
    announce("twostage batched vs single", kind)
    if kind == "noncollinear":
        probs = [I.noncollinear(seed=s, nx=3, ny=1, nz=1, lam_max=0.2) for s in (1, 2, 3)]
    else:
        probs = [I.toy(seed=s, natoms=12, norb=13, edge=12.0, n_electrons=40.0, kT=0.01,
                       phases=kind == "complex") for s in (5, 6, 7, 8)]
    p0 = probs[0]
    cplx = np.iscomplexobj(p0.H)
    B = len(probs)
    H = dev(np.stack([p.H for p in probs]))
    S = dev(np.stack([p.S.astype(p0.H.dtype) for p in probs]))
    for il, iu in [(1, None), (3, p0.order // 2)]:
        plan = ks.Plan(p0.n, batch=B, complex=cplx, noncollinear=p0.nsp == 2, flags=TWO)
        eb, Cb = _gevd(plan, H, S, il, iu)
        for b, p in enumerate(probs):
            one = ks.Plan(p.n, batch=1, complex=cplx, noncollinear=p.nsp == 2, flags=TWO)
            e1, C1 = _gevd(one, dev(p.H), dev(p.S.astype(p0.H.dtype)), il, iu)
            assert np.array_equal(eb[b], e1)
            assert np.array_equal(Cb[b], C1)


def test_graph_replay_matches_eager_solves():
    """KS_PLAN_GRAPH | KS_PLAN_TWOSTAGE: replays (with eager work in between and
    new input contents) equal the eager two-stage solves bit for bit; the
    counters and progress words are cleared by fill kernels inside the graph."""
    announce("twostage graph replay")
    stream = torch.cuda.Stream()
    probs = [I.kpoint_batch(natoms=5, norb=13, kgrid=(2, 1, 1), seed=s) for s in (0, 1, 2)]
    p0 = probs[0]
    with torch.cuda.stream(stream):
        gplan = ks.Plan(p0.n, batch=p0.batch, complex=True, stream=stream, flags=ks.KS_PLAN_GRAPH | TWO)
        eplan = ks.Plan(p0.n, batch=p0.batch, complex=True, stream=stream, flags=TWO)
        H = dev(p0.H)
        S = dev(p0.S.astype(p0.H.dtype))
        eps = torch.empty(gplan._vshape(), dtype=torch.float64, device="cuda")
        C = torch.zeros(gplan._mshape(), dtype=torch.complex128, device="cuda")
        for rep in range(4):
            p = probs[rep % len(probs)]
            H.copy_(dev(p.H))
            S.copy_(dev(p.S.astype(p.H.dtype)))
            gplan.gevd(H, S, eps, C)
            _ = (H.abs() * 2.0).sum().item()
            stream.synchronize()
            gplan.check("graph replay")
            ge, gC = host(eps).copy(), host(C).copy()
            ee, eC = _gevd(eplan, H, S)
            assert np.array_equal(ge, ee), rep
            assert np.array_equal(gC, eC), rep
        assert gplan.graph_stats() == (1, 3)


def test_window_and_routes_agree():
    """A window of eigenvectors (the occupied ones and five more) gives the
    same density as all of them; the one-stage and two-stage routes agree."""
    announce("twostage window")
    p = I.toy(seed=5, natoms=12, norb=13, edge=12.0, n_electrons=60.0, kT=0.01, phases=True)
    full, _ = solve_gpu(p, flags=TWO)
    one, _ = solve_gpu(p)
    m = int((full["occ"] > 2e-15).sum()) + 5
    win, _ = solve_gpu(p, il=1, iu=m, flags=TWO)
    assert np.abs(win["rho"] - full["rho"]).max() < RHO_TOL
    assert np.abs(win["eps"] - full["eps"]).max() == 0.0
    assert np.abs(one["eps"] - full["eps"]).max() < EPS_TOL
    assert np.abs(one["rho"] - full["rho"]).max() < RHO_TOL


@pytest.mark.parametrize("nsp", [1, 2])
def test_lowdin_route_vs_oracle(nsp):
    """KS_PLAN_LOWDIN | KS_PLAN_TWOSTAGE: H' = V^H H V reduced in two stages,
    against the oracle's Loewdin route."""
    announce("twostage lowdin", nsp)
    if nsp == 2:
        p = I.noncollinear(seed=4, nx=6, ny=1, nz=1, lam_max=0.2)
    else:
        p = I.toy(seed=44, natoms=14, norb=13, edge=12.0, n_electrons=80.0, kT=0.01, phases=True)
    g, _ = solve_gpu(p, flags=TWO | ks.KS_PLAN_LOWDIN)
    compare(p, g, O.solve(p.H, p.S, p.n_electrons, p.kT, nsp=nsp, route="lowdin"))
