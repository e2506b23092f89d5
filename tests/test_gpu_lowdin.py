"""The Loewdin route (KS_PLAN_LOWDIN; paper Sec. 3.1 Parts 2-1..2-5, Sec. 3.2
Parts 3-1..3-6) against the oracle's Loewdin route and against the GPU's own
Cholesky route, element by element on the same seeded inputs.

Tolerances as for the Cholesky route (FP64): eigenvalues 1e-10 Ha, residual
1e-12, |C^H S C - I| 1e-11, density 1e-9."""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2606_09058_amd import inputs as I
from paper_2606_09058_amd import ks
from tests.gpu_helpers import announce, dev, host, residuals

pytestmark = pytest.mark.gpu

EPS_TOL, RES_TOL, ORTH_TOL, RHO_TOL = 1e-10, 1e-12, 1e-11, 1e-9


@pytest.fixture(scope="module", autouse=True)
def gpu():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    ks.lib()


def lowdin_plan(p, flags=0, stream=None):
    return ks.Plan(p.n, batch=p.batch, complex=np.iscomplexobj(p.H), noncollinear=p.nsp == 2,
                   flags=ks.KS_PLAN_LOWDIN | flags, stream=stream)


def run(plan, p, il=1, iu=None, reuse_s=False, check=True):
    out = plan.solve(dev(p.H), None if reuse_s else dev(p.S.astype(p.H.dtype)), p.n_electrons, p.kT, il=il,
                     iu=iu, kweights=p.weights, reuse_s=reuse_s, check=check)
    return {k: host(v) for k, v in out.items()}


def oracle_lowdin(p):
    """Oracle Loewdin route per k-point, then the common mu and rho."""
    Hs = p.H if p.batch > 1 else p.H[None]
    Ss = p.S if p.batch > 1 else p.S[None]
    es, Cs = [], []
    for k in range(p.batch):
        e, C = O.gevd_lowdin(Hs[k], Ss[k], nsp=p.nsp)
        es.append(e)
        Cs.append(C)
    fr = O.fermi(np.array(es), p.n_electrons, p.kT, p.g, wk=p.weights)
    occ = np.atleast_2d(fr["occ"])
    rho = [O.density(Cs[k], occ[k]) for k in range(p.batch)]
    return np.array(es), np.array(rho), fr


def check_against_oracle(p, g):
    e_o, rho_o, fr = oracle_lowdin(p)
    eps = g["eps"].reshape(p.batch, p.order)
    rho = g["rho"].reshape(p.batch, p.order, p.order)
    C = g["C"].reshape(p.batch, p.order, p.order)
    Hs = p.H.reshape(p.batch, p.order, p.order)
    Ss = p.S.reshape(p.batch, p.n, p.n)
    assert np.abs(eps - e_o).max() < EPS_TOL
    assert np.abs(rho - rho_o).max() < RHO_TOL
    # mu itself is ill-conditioned inside a gap; the band energy and the
    # occupations it decides are not
    assert abs(float(g["eband"][0]) - fr["eband"]) < 1e-9 * max(1.0, abs(fr["eband"]))
    assert np.abs(g["occ"].reshape(p.batch, p.order) - np.atleast_2d(fr["occ"])).max() < 1e-9
    for k in range(p.batch):
        res, orth = residuals(Hs[k], Ss[k], eps[k], C[k], p.nsp)
        assert res < RES_TOL, res
        assert orth < ORTH_TOL, orth


@pytest.mark.parametrize("natoms,norb,cplx", [(1, 1, False), (1, 3, True), (5, 8, False), (11, 13, True),
                                              (24, 13, False), (26, 13, True)])
def test_collinear_lowdin_vs_oracle(natoms, norb, cplx):
    """Sizes from 1 to 338 orbitals: several 64-wide tiles and ragged tails."""
    announce("lowdin collinear", natoms, norb, cplx)
    ne = min(2.0 * natoms * norb, max(2.0, 2.0 * round(0.3 * natoms * norb)))
    p = I.toy(seed=natoms * 7 + norb, natoms=natoms, norb=norb, edge=10 * (natoms / 8) ** (1 / 3) + 1,
              n_electrons=ne, kT=0.01, phases=cplx)
    check_against_oracle(p, run(lowdin_plan(p), p))


@pytest.mark.parametrize("natoms", [2, 9])
def test_noncollinear_lowdin_vs_oracle(natoms):
    """Spinor form: V_NC = diag(V, V) with V from the order-n overlap plan."""
    announce("lowdin noncollinear", natoms)
    p = I.noncollinear(seed=natoms + 40, nx=natoms, ny=1, nz=1, lam_max=0.2)
    check_against_oracle(p, run(lowdin_plan(p), p))


def test_kpoint_batch_lowdin_vs_oracle():
    announce("lowdin kpoints")
    p = I.kpoint_batch(natoms=6, norb=13, kgrid=(2, 2, 1), seed=4)
    check_against_oracle(p, run(lowdin_plan(p), p))


@pytest.mark.parametrize("kind", ["real", "complex", "noncollinear"])
def test_lowdin_route_equals_cholesky_route(kind):
    """Both GPU routes on the same input: eps, mu and rho do not depend on the
    S-orthonormal basis."""
    announce("lowdin vs cholesky", kind)
    if kind == "noncollinear":
        p = I.noncollinear(seed=8, nx=6, ny=1, nz=1, lam_max=0.2)
    else:
        p = I.toy(seed=31, natoms=16, norb=13, edge=12.0, n_electrons=120.0, kT=0.01, phases=kind == "complex")
    gl = run(lowdin_plan(p), p)
    pc = ks.Plan(p.n, complex=np.iscomplexobj(p.H), noncollinear=p.nsp == 2)
    gc = run(pc, p)
    assert np.abs(gl["eps"] - gc["eps"]).max() < EPS_TOL
    assert np.abs(gl["rho"] - gc["rho"]).max() < RHO_TOL
    assert abs(float(gl["eband"][0]) - float(gc["eband"][0])) < 1e-9 * max(1.0, abs(float(gc["eband"][0])))


def test_reuse_of_v_across_cycles():
    """KS_REUSE_S keeps V = U s^-1/2 (the paper's cycles 2 onwards): a new H with
    the same S must give the oracle's answer for that H, and equal a fresh solve
    bit for bit (the same V, the same launches)."""
    announce("lowdin reuse V")
    p = I.toy(seed=12, natoms=12, norb=13, edge=11.0, n_electrons=90.0, kT=0.01, phases=True)
    plan = lowdin_plan(p)
    run(plan, p)
    rng = np.random.default_rng(5)
    D = rng.normal(scale=0.01, size=p.H.shape) + 1j * rng.normal(scale=0.01, size=p.H.shape)
    q = I.Problem(p.H + D + D.conj().T, p.S, p.n_electrons, p.kT)
    g2 = run(plan, q, reuse_s=True)
    check_against_oracle(q, g2)
    fresh = run(lowdin_plan(q), q)
    assert np.array_equal(g2["eps"], fresh["eps"])
    assert np.array_equal(g2["rho"], fresh["rho"])


def test_lowdin_window():
    """Windowed eigenvectors il..iu through V C'."""
    announce("lowdin window")
    p = I.toy(seed=13, natoms=14, norb=13, edge=12.0, n_electrons=100.0, kT=0.01, phases=False)
    e_o, rho_o, fr = oracle_lowdin(p)
    iu = int((np.atleast_2d(fr["occ"])[0] > p.g * 1e-15).sum()) + 3
    g = run(lowdin_plan(p), p, il=1, iu=iu)
    assert np.abs(g["eps"] - e_o[0]).max() < EPS_TOL
    assert np.abs(g["rho"] - rho_o[0]).max() < RHO_TOL
    res, orth = residuals(p.H, p.S, g["eps"][:iu], g["C"][:, :iu], 1)
    assert res < RES_TOL and orth < ORTH_TOL


def test_indefinite_s_reports_count():
    """An S with exactly two negative eigenvalues: KS_ERR_NOT_POSDEF with
    info = 2 (the number of eigenvalues <= 0, counted here by LAPACK)."""
    announce("lowdin indefinite S")
    p = I.toy(seed=2, natoms=5, norb=8)
    w, U = np.linalg.eigh(p.S)
    w = w.copy()
    w[:2] = [-0.5, -0.1]
    S = (U * w) @ U.T
    S = 0.5 * (S + S.T)
    assert int((np.linalg.eigvalsh(S) <= 0).sum()) == 2
    plan = lowdin_plan(p)
    run(plan, I.Problem(p.H, S, p.n_electrons, p.kT), check=False)
    st, info = plan.get_info()
    assert st == 2 and info == 2


def test_lowdin_graph_replay_matches_eager():
    """KS_PLAN_LOWDIN | KS_PLAN_GRAPH: replays (new contents in the same buffers,
    eager work in between) equal the eager Loewdin plan bit for bit."""
    announce("lowdin graph")
    stream = torch.cuda.Stream()
    probs = [I.kpoint_batch(natoms=5, norb=13, kgrid=(2, 1, 1), seed=s) for s in (0, 1)]
    p0 = probs[0]
    with torch.cuda.stream(stream):
        gplan = lowdin_plan(p0, flags=ks.KS_PLAN_GRAPH, stream=stream)
        eplan = lowdin_plan(p0, stream=stream)
        H = dev(p0.H)
        S = dev(p0.S.astype(p0.H.dtype))
        eps = torch.empty(gplan._vshape(), dtype=torch.float64, device="cuda")
        C = torch.zeros(gplan._mshape(), dtype=torch.complex128, device="cuda")
        eps2 = torch.empty_like(eps)
        C2 = torch.zeros_like(C)
        for rep in range(3):
            p = probs[rep % 2]
            H.copy_(dev(p.H))
            S.copy_(dev(p.S.astype(p.H.dtype)))
            gplan.gevd(H, S, eps, C)
            _ = (H.abs() * 2.0).sum().item()
            eplan.gevd(H, S, eps2, C2)
            stream.synchronize()
            assert np.array_equal(host(eps), host(eps2)), rep
            assert np.array_equal(host(C), host(C2)), rep
        gplan.check("graph")
        assert gplan.graph_stats()[1] >= 1


@pytest.mark.parametrize("kind", ["real", "complex", "noncollinear", "batch"])
def test_overlap_cutoff_on_an_overcomplete_basis(kind):
    """Canonical orthogonalisation (ks_plan_set_overlap_cutoff): an n-function
    basis spanning m < n dimensions.  The kept count must be m per k-point, the
    kept eigenvalues the oracle's canonical route and eig(h) (the closed form),
    the placeholders equal, above every kept eigenvalue, with zero
    eigenvectors; rho the oracle's and tr(rho S) = N_e."""
    announce("lowdin overlap cutoff", kind)
    tau = 1e-10
    if kind == "real":
        p = I.overcomplete(seed=1, n=90, ms=(70,))
    elif kind == "complex":
        p = I.overcomplete(seed=2, n=100, ms=(77,), cplx=True)
    elif kind == "noncollinear":
        p = I.overcomplete(seed=3, n=50, ms=(41,), nsp=2)
    else:
        p = I.overcomplete(seed=4, n=80, ms=(60, 70))
    plan = lowdin_plan(p)
    plan.set_overlap_cutoff(tau)
    g = run(plan, p)
    assert plan.overlap_rank() == list(p.meta["m"])
    eps = g["eps"].reshape(p.batch, p.order)
    C = g["C"].reshape(p.batch, p.order, p.order)
    rho = g["rho"].reshape(p.batch, p.order, p.order)
    Hs = p.H.reshape(p.batch, p.order, p.order)
    Ss = p.S.reshape(p.batch, p.n, p.n)
    es_pad = np.full((p.batch, p.order), 1.0e6)  # dropped states: never occupied
    Cos = []
    for k in range(p.batch):
        mk = p.nsp * p.meta["m"][k]
        e_o, C_o, m_o = O.gevd_canonical(Hs[k], Ss[k], tau, nsp=p.nsp)
        assert m_o == p.meta["m"][k]
        scale = max(1.0, np.abs(e_o).max())
        assert np.abs(eps[k, :mk] - e_o).max() < 1e-9 * scale
        assert np.abs(eps[k, :mk] - np.linalg.eigvalsh(p.meta["h"][k])).max() < 1e-9 * scale
        ph = eps[k, mk:]
        assert ph.size == p.order - mk and np.all(ph > eps[k, :mk].max())
        assert np.abs(ph - ph[0]).max() <= 1e-9 * abs(ph[0])
        assert np.abs(C[k][:, mk:]).max() < 1e-9
        es_pad[k, :mk] = e_o
        Cos.append(C_o)
    fr = O.fermi(es_pad, p.n_electrons, p.kT, p.g, wk=p.weights)
    occ = np.atleast_2d(fr["occ"])
    for k in range(p.batch):
        mk = p.nsp * p.meta["m"][k]
        rho_o = O.density(Cos[k], occ[k, :mk])
        assert np.abs(rho[k] - rho_o).max() < RHO_TOL * max(1.0, np.abs(rho_o).max())
    SN = [np.kron(np.eye(p.nsp), Ss[k]) if p.nsp == 2 else Ss[k] for k in range(p.batch)]
    w = [1.0] if p.batch == 1 else list(p.weights)
    tr = sum(w[k] * np.trace(rho[k] @ SN[k]).real for k in range(p.batch))
    assert abs(tr - p.n_electrons) < 1e-8 * p.n_electrons


def test_overlap_cutoff_arguments():
    announce("lowdin cutoff arguments")
    p = I.toy(seed=2, natoms=3, norb=8)
    plan = lowdin_plan(p)
    with pytest.raises(ks.KSError):
        plan.set_overlap_cutoff(1.5)
    with pytest.raises(ks.KSError):
        plan.overlap_rank()  # S not decomposed yet
    run(plan, p)
    assert plan.overlap_rank() == [p.n]
    chol = ks.Plan(p.n)
    with pytest.raises(ks.KSError):
        chol.set_overlap_cutoff(1e-8)


def test_overlap_cutoff_kept_with_the_reused_v():
    """V formed with a cutoff and reused (KS_REUSE_S) after the cutoff is reset:
    the reused V keeps its dropped columns, so the new H must still get the
    placeholders (the cutoff in force when V was formed decides), and the kept
    eigenvalues are eig(h') for the new h'."""
    announce("lowdin cutoff with reused V")
    tau = 1e-10
    p = I.overcomplete(seed=6, n=70, ms=(52,), cplx=True)
    plan = lowdin_plan(p)
    plan.set_overlap_cutoff(tau)
    run(plan, p)
    plan.set_overlap_cutoff(0.0)
    B = p.meta["B"][0]
    h2 = p.meta["h"][0] + 0.1 * np.eye(52)
    H2 = B @ h2 @ B.conj().T
    q = I.Problem(0.5 * (H2 + H2.conj().T), p.S, p.n_electrons, p.kT)
    g = run(plan, q, reuse_s=True)
    m = 52
    e_o, C_o, m_o = O.gevd_canonical(q.H, q.S, tau)
    assert m_o == m and plan.overlap_rank() == [m]
    scale = max(1.0, np.abs(e_o).max())
    assert np.abs(g["eps"][:m] - e_o).max() < 1e-9 * scale
    assert np.abs(g["eps"][:m] - np.linalg.eigvalsh(h2)).max() < 1e-9 * scale
    assert np.all(g["eps"][m:] > g["eps"][:m].max())
    assert abs(np.trace(g["rho"] @ q.S).real - q.n_electrons) < 1e-8 * q.n_electrons
    # the adjoint needs a complete eigenbasis: refused while V has dropped columns
    n = p.n
    z = torch.zeros((n, n), dtype=torch.complex128, device="cuda")
    eps_t = dev(g["eps"])
    with pytest.raises(ks.KSError):
        plan.density_backward(eps_t, dev(g["C"]), dev(g["mu"]), dev(g["occ"]), p.kT, dev(g["rho"]) * 0, None,
                              z.clone(), z.clone())
