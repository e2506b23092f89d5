"""Seeded synthetic inputs shaped like numerical-atomic-orbital Hamiltonians.

This module only draws inputs; it holds none of the eigensolver's or the density
build's arithmetic, and both the HIP path and the CPU oracle read what it
returns.  It imports numpy only.

The paper's workloads are silicon diamond supercells from OpenMX with 13 basis
functions per atom (s2p2d1) and a 2x2x2 k mesh (Sec. 4).  Those structures and
the OpenMX basis data are not available here, so a distance-decay model stands
in for the matrix elements:

* atoms carry ``norb`` orbitals each, ordered per atom as [s, s, p x3, p x3, d x5]
  for 13 orbitals (local d block = indices 8..12),
* H_ij = a_ij exp(-d_ij / 2) with a_ij ~ N(0, 0.3) Ha drawn for the strict upper
  triangle in row-major order and mirrored, diagonal H_ii ~ U(-1, 1) Ha,
* S_ij = 0.4 exp(-d_ij) u_ij with u_ij ~ U(0, 1), diagonal 1,
* d_ij is the distance between the atoms of orbitals i and j (0 on one atom),
  optionally the minimum image in a periodic box and cut off beyond ``cutoff``
  Bohr (the elements are then stored as zeros in a dense matrix),
* S is made positive definite with condition number 1e3 by the smallest
  diagonal shift sigma = max(0, (l_max - 1e3 l_min) / (1e3 - 1)); sigma is
  rounded up to a multiple of 2^-30 so that inputs are bit-identical across
  machines even if the extreme eigenvalues differ in their last bits.

Random numbers come from numpy's PCG64 ``default_rng(seed)``.
"""
from __future__ import annotations

import hashlib
from dataclasses import dataclass, field

import numpy as np

COND_S = 1e3


@dataclass
class Problem:
    """One (batch of) generalized eigenproblem(s) with its physical parameters."""
    H: np.ndarray            # (order, order) or (nk, order, order); Hermitian, full storage
    S: np.ndarray            # (n, n) or (nk, n, n); Hermitian positive definite
    n_electrons: float
    kT: float
    nsp: int = 1             # 1 collinear, 2 noncollinear spinor (H is 2n x 2n)
    weights: np.ndarray | None = None   # k weights (sum 1); None for one matrix
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def g(self) -> float:
        """Spin factor folded into the occupations: 2 collinear, 1 spinor."""
        return 2.0 if self.nsp == 1 else 1.0

    @property
    def order(self) -> int:
        return self.H.shape[-1]

    @property
    def n(self) -> int:
        return self.S.shape[-1]

    @property
    def batch(self) -> int:
        return 1 if self.H.ndim == 2 else self.H.shape[0]

    def digest(self) -> str:
        h = hashlib.sha256()
        for a in (self.H, self.S):
            h.update(np.ascontiguousarray(a).tobytes())
        return h.hexdigest()


# ---------------------------------------------------------------------------
# geometry
# ---------------------------------------------------------------------------
def _pair_distances(pos, box=None):
    """Atom-atom distance matrix; minimum image when ``box`` (3,) is given."""
    d = pos[:, None, :] - pos[None, :, :]
    if box is not None:
        box = np.asarray(box, dtype=np.float64)
        d -= box * np.round(d / box)
    return np.sqrt((d * d).sum(-1))


def _orbital_distances(dat, norb):
    return np.repeat(np.repeat(dat, norb, axis=0), norb, axis=1)


def _upper_values(rng, n, kind, scale=1.0):
    """Values for the strict upper triangle in row-major order."""
    m = n * (n - 1) // 2
    if kind == "normal":
        return rng.normal(0.0, scale, size=m)
    return rng.uniform(0.0, 1.0, size=m)


def _sym_from_upper(n, vals, diag):
    A = np.zeros((n, n))
    iu = np.triu_indices(n, 1)
    A[iu] = vals
    A = A + A.T
    A[np.diag_indices(n)] = diag
    return A


def _shift_sigma(lmin, lmax, cond=COND_S):
    sigma = max(0.0, (lmax - cond * lmin) / (cond - 1.0))
    q = 2.0 ** -30
    return np.ceil(sigma / q) * q


def _extreme_eigs(S):
    w = np.linalg.eigvalsh(S)
    return float(w[0]), float(w[-1])


def collinear_matrices(rng, pos, norb, box=None, cutoff=None, phases=False):
    """H and S (order natoms*norb) of the distance-decay model.

    Draw order: a_ij (upper, normal 0.3), H diagonal U(-1,1), u_ij (upper, U(0,1)),
    then, if ``phases``, one phase phi_ij ~ U(0, 2 pi) per upper pair applied to
    both H_ij and S_ij (their conjugates below the diagonal)."""
    natoms = pos.shape[0]
    n = natoms * norb
    dat = _pair_distances(pos, box)
    d = _orbital_distances(dat, norb)
    iu = np.triu_indices(n, 1)
    a = _upper_values(rng, n, "normal", 0.3)
    hdiag = rng.uniform(-1.0, 1.0, size=n)
    u = _upper_values(rng, n, "uniform")
    du = d[iu]
    hv = a * np.exp(-du / 2.0)
    sv = 0.4 * np.exp(-du) * u
    if cutoff is not None:
        keep = du <= cutoff
        hv = np.where(keep, hv, 0.0)
        sv = np.where(keep, sv, 0.0)
    if phases:
        ph = np.exp(1j * rng.uniform(0.0, 2.0 * np.pi, size=hv.shape[0]))
        H = np.zeros((n, n), np.complex128)
        S = np.zeros((n, n), np.complex128)
        H[iu] = hv * ph
        S[iu] = sv * ph
        H = H + H.conj().T
        S = S + S.conj().T
        H[np.diag_indices(n)] = hdiag
        S[np.diag_indices(n)] = 1.0
    else:
        H = _sym_from_upper(n, hv, hdiag)
        S = _sym_from_upper(n, sv, 1.0)
    return H, S


def shift_overlap(S, cond=COND_S):
    """S + sigma I with the smallest sigma giving cond(S) <= cond (see module doc)."""
    lmin, lmax = _extreme_eigs(S)
    sigma = _shift_sigma(lmin, lmax, cond)
    S = S.copy()
    S[np.diag_indices(S.shape[0])] += sigma
    return S, sigma


def lattice_positions(rng, nx, ny, nz, spacing, jitter):
    g = np.stack(np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij"), -1)
    pos = g.reshape(-1, 3).astype(np.float64) * spacing
    pos += rng.uniform(-jitter, jitter, size=pos.shape)
    box = np.array([nx, ny, nz], dtype=np.float64) * spacing
    return pos, box


# ---------------------------------------------------------------------------
# the workloads
# ---------------------------------------------------------------------------
def toy(seed=0, natoms=8, norb=8, edge=10.0, n_electrons=32.0, kT=0.01, phases=False):
    """Collinear Gamma-point toy: random positions in a cube, no periodicity, no cutoff.

    Default: 8 atoms x 8 orbitals = N 64 real, 32 electrons, kT 0.01 Ha."""
    rng = np.random.default_rng(seed)
    pos = rng.uniform(0.0, edge, size=(natoms, 3))
    H, S = collinear_matrices(rng, pos, norb, phases=phases)
    S, sigma = shift_overlap(S)
    return Problem(H, S, float(n_electrons), float(kT), 1, None, "toy",
                   dict(natoms=natoms, norb=norb, sigma=sigma, seed=seed))


def supercell(seed=0, nx=8, ny=8, nz=8, norb=13, spacing=4.0, jitter=0.2, cutoff=12.0,
              electrons_per_atom=4.0, kT=0.01):
    """Collinear Gamma point of a perturbed cubic lattice with periodic minimum image.

    Default: 512 atoms x 13 orbitals = N 6656 real, 2048 electrons, kT 0.01 Ha."""
    rng = np.random.default_rng(seed)
    pos, box = lattice_positions(rng, nx, ny, nz, spacing, jitter)
    H, S = collinear_matrices(rng, pos, norb, box=box, cutoff=cutoff)
    S, sigma = shift_overlap(S)
    natoms = pos.shape[0]
    return Problem(H, S, electrons_per_atom * natoms, float(kT), 1, None, "supercell",
                   dict(natoms=natoms, norb=norb, sigma=sigma, seed=seed, box=box.tolist()))


def spin_block(rng, natoms, norb, lam_max=0.02, d_lo=8, d_hi=13):
    """Spin off-diagonal block H^{ab}: on each atom's d block, i lam X with
    lam ~ U(0, lam_max) Ha and X = (G + G^T)/2, G ~ N(0,1) (5x5); anti-Hermitian."""
    n = natoms * norb
    B = np.zeros((n, n), np.complex128)
    nd = d_hi - d_lo
    for at in range(natoms):
        lam = rng.uniform(0.0, lam_max)
        G = rng.normal(0.0, 1.0, size=(nd, nd))
        X = 0.5 * (G + G.T)
        o = at * norb
        B[o + d_lo:o + d_hi, o + d_lo:o + d_hi] = 1j * lam * X
    return B


def noncollinear(seed=0, nx=8, ny=8, nz=6, norb=13, spacing=4.0, jitter=0.2, cutoff=12.0,
                 electrons_per_atom=4.0, kT=0.01, lam_max=0.02):
    """Noncollinear spinor problem: H_NC = [[H, B], [B^H, H]] with the collinear H of
    the lattice model and B from ``spin_block``; overlap diag(S, S) (S passed n x n).

    Default: 384 atoms x 13 = n 4992, order 9984 complex, 1536 electrons, kT 0.01."""
    rng = np.random.default_rng(seed)
    pos, box = lattice_positions(rng, nx, ny, nz, spacing, jitter)
    Hc, S = collinear_matrices(rng, pos, norb, box=box, cutoff=cutoff)
    S, sigma = shift_overlap(S)
    natoms = pos.shape[0]
    B = spin_block(rng, natoms, norb, lam_max)
    n = Hc.shape[0]
    H = np.zeros((2 * n, 2 * n), np.complex128)
    H[:n, :n] = Hc
    H[n:, n:] = Hc
    H[:n, n:] = B
    H[n:, :n] = B.conj().T
    return Problem(H, S.astype(np.complex128), electrons_per_atom * natoms, float(kT), 2, None,
                   "noncollinear", dict(natoms=natoms, norb=norb, sigma=sigma, seed=seed))


def kpoint_realspace(seed=0, natoms=100, norb=13, density=1.0 / 64.0, min_dist=2.0, kgrid=(4, 2, 2)):
    """The real-space blocks behind ``kpoint_batch`` (same seed, same numbers):
    dict(HR, SR: (27, n, n) real, R: (27, 3) lattice vectors, k: (nk, 3)), with
    S_0 carrying the unit diagonal and without the overlap shift sigma."""
    rng = np.random.default_rng(seed)
    edge = (natoms / density) ** (1.0 / 3.0)
    box = np.full(3, edge)
    pos = np.zeros((natoms, 3))
    cnt = 0
    while cnt < natoms:
        p = rng.uniform(0.0, edge, size=3)
        if cnt:
            d = pos[:cnt] - p
            d -= box * np.round(d / box)
            if np.sqrt((d * d).sum(-1)).min() < min_dist:
                continue
        pos[cnt] = p
        cnt += 1
    n = natoms * norb
    A = _sym_from_upper(n, _upper_values(rng, n, "normal", 0.3), rng.uniform(-1.0, 1.0, size=n))
    U = _sym_from_upper(n, _upper_values(rng, n, "uniform"), rng.uniform(0.0, 1.0, size=n))
    Rs = [np.array([a, b, c], dtype=np.float64) * edge
          for a in (-1, 0, 1) for b in (-1, 0, 1) for c in (-1, 0, 1)]
    ks = [2.0 * np.pi * np.array([i / kgrid[0], j / kgrid[1], l / kgrid[2]]) / edge
          for i in range(kgrid[0]) for j in range(kgrid[1]) for l in range(kgrid[2])]
    HR = np.zeros((len(Rs), n, n))
    SR = np.zeros((len(Rs), n, n))
    for r, R in enumerate(Rs):
        dv = pos[None, :, :] + R - pos[:, None, :]          # t_j + R - t_i
        dat = np.sqrt((dv * dv).sum(-1))
        d = _orbital_distances(dat, norb)
        HR[r] = A * np.exp(-d / 2.0)
        SR[r] = 0.4 * U * np.exp(-d)
        if not R.any():
            SR[r][np.diag_indices(n)] = 1.0
    return dict(HR=HR, SR=SR, R=np.array(Rs), k=np.array(ks))


def kpoint_batch(seed=0, natoms=100, norb=13, density=1.0 / 64.0, min_dist=2.0,
                 kgrid=(4, 2, 2), electrons_per_atom=4.0, kT=0.01):
    """Bloch-summed k-point problems (paper Sec. 2, the Bloch-sum equations):
    H(k) = sum_R H_R e^{i k.R}, S(k) = sum_R S_R e^{i k.R} over the 27 lattice
    vectors R in {-1,0,1}^3 L of a cubic cell of edge L with ``natoms`` atoms at
    number density ``density``, rejection-sampled with minimum image distance
    ``min_dist``.  H_R,ij = A_ij exp(-|t_j + R - t_i| / 2) and
    S_R,ij = 0.4 U_ij exp(-|t_j + R - t_i|), except S_0,ii = 1, with A and U
    symmetric and shared over R (so H_-R = H_R^T and H(k) is Hermitian).
    k = 2 pi (i/k1, j/k2, l/k3)/L on a Gamma-centred grid, equal weights, one
    shift sigma common to all k.

    Default: 100 atoms x 13 = N 1300 complex, 16 k-points, 400 electrons per cell."""
    rng = np.random.default_rng(seed)
    edge = (natoms / density) ** (1.0 / 3.0)
    box = np.full(3, edge)
    pos = np.zeros((natoms, 3))
    cnt = 0
    while cnt < natoms:
        p = rng.uniform(0.0, edge, size=3)
        if cnt:
            d = pos[:cnt] - p
            d -= box * np.round(d / box)
            if np.sqrt((d * d).sum(-1)).min() < min_dist:
                continue
        pos[cnt] = p
        cnt += 1
    n = natoms * norb
    A = _sym_from_upper(n, _upper_values(rng, n, "normal", 0.3), rng.uniform(-1.0, 1.0, size=n))
    U = _sym_from_upper(n, _upper_values(rng, n, "uniform"), rng.uniform(0.0, 1.0, size=n))
    Rs = [np.array([a, b, c], dtype=np.float64) * edge
          for a in (-1, 0, 1) for b in (-1, 0, 1) for c in (-1, 0, 1)]
    ks = [2.0 * np.pi * np.array([i / kgrid[0], j / kgrid[1], l / kgrid[2]]) / edge
          for i in range(kgrid[0]) for j in range(kgrid[1]) for l in range(kgrid[2])]
    nk = len(ks)
    H = np.zeros((nk, n, n), np.complex128)
    S = np.zeros((nk, n, n), np.complex128)
    for R in Rs:
        dv = pos[None, :, :] + R - pos[:, None, :]          # t_j + R - t_i
        dat = np.sqrt((dv * dv).sum(-1))
        d = _orbital_distances(dat, norb)
        HR = A * np.exp(-d / 2.0)
        SR = 0.4 * U * np.exp(-d)
        if not R.any():
            SR[np.diag_indices(n)] = 1.0
        for ki, k in enumerate(ks):
            ph = np.exp(1j * float(k @ R))
            H[ki] += HR * ph
            S[ki] += SR * ph
    for ki in range(nk):  # exact Hermitian symmetry despite summation rounding
        H[ki] = 0.5 * (H[ki] + H[ki].conj().T)
        S[ki] = 0.5 * (S[ki] + S[ki].conj().T)
    lo, hi = np.inf, -np.inf
    for ki in range(nk):
        w = np.linalg.eigvalsh(S[ki])
        lo, hi = min(lo, w[0]), max(hi, w[-1])
    sigma = _shift_sigma(lo, hi)
    for ki in range(nk):
        S[ki][np.diag_indices(n)] += sigma
    wts = np.full(nk, 1.0 / nk)
    return Problem(H, S, electrons_per_atom * natoms, float(kT), 1, wts, "kpoints",
                   dict(natoms=natoms, norb=norb, sigma=sigma, seed=seed, edge=edge))


def differentiation(seed=0, natoms=256, norb=8, n_electrons=None, kT=0.02):
    """Complex toy for the adjoint: cube of edge 10 (natoms/8)^(1/3) Bohr, phases on
    off-diagonal H and S.  Default: 256 atoms x 8 = N 2048 complex, 1024 electrons,
    kT 0.02 Ha."""
    edge = 10.0 * (natoms / 8.0) ** (1.0 / 3.0)
    ne = 4.0 * natoms if n_electrons is None else n_electrons
    p = toy(seed=seed, natoms=natoms, norb=norb, edge=edge, n_electrons=ne, kT=kT, phases=True)
    p.name = "differentiation"
    return p


def random_hermitian(rng, n, cplx):
    X = rng.normal(size=(n, n))
    if cplx:
        X = X + 1j * rng.normal(size=(n, n))
    return 0.5 * (X + X.conj().T)


def random_spd(rng, n, cplx, cond=COND_S):
    S = random_hermitian(rng, n, cplx) * 0.1
    S[np.diag_indices(n)] += 1.0
    S, _ = shift_overlap(S, cond)
    return S


def overcomplete(seed=0, n=90, ms=(70,), nsp=1, cplx=False, kT=0.01):
    """An overcomplete basis: n functions chi = B phi spanning m < n dimensions
    (phi orthonormal, B n x m Gaussian), so S = B B^H has rank m, and
    H = B_NC h B_NC^H with h a random Hermitian matrix of order nsp m (B_NC =
    diag(B, B) for the spinor form).  One k-point per entry of ms; electrons
    g nsp m / 3 per k-point (g = 2 collinear, 1 spinor).  meta holds B and h
    per k-point for closed-form checks."""
    rng = np.random.default_rng(seed)
    cp = cplx or nsp == 2
    Hs, Ss, Bs, hs = [], [], [], []
    for m in ms:
        B = rng.normal(size=(n, m))
        if cp:
            B = B + 1j * rng.normal(size=(n, m))
        h = random_hermitian(rng, nsp * m, cp)
        BN = np.kron(np.eye(nsp), B)
        S = B @ B.conj().T
        H = BN @ h @ BN.conj().T
        Hs.append(0.5 * (H + H.conj().T))
        Ss.append(0.5 * (S + S.conj().T))
        Bs.append(B)
        hs.append(h)
    g = 2.0 if nsp == 1 else 1.0
    ne = float(sum(round(g * nsp * m / 3.0) for m in ms)) / len(ms)
    one = len(ms) == 1
    p = Problem(Hs[0] if one else np.array(Hs), Ss[0] if one else np.array(Ss), ne, kT, nsp=nsp,
                weights=None if one else np.full(len(ms), 1.0 / len(ms)), name="overcomplete")
    p.meta = {"B": Bs, "h": hs, "m": list(ms)}
    return p


def known_spectrum_spinor(seed=0, n=4992, rank=64, lo=-28.8, hi=21.3, n_electrons=1536.0, kT=0.01,
                          offdiag=0.45, close_pairs=48, ties=16, close_gap=1e-7):
    """A spinor problem of order 2n with a spectrum fixed by construction, for
    full-size checks that need no eigensolver on the host.

    Lambda: 2n values drawn uniformly in [lo, hi] (the range of the 384-atom
    noncollinear workload), with ``close_pairs`` pairs moved to within
    ``close_gap`` Ha of each other and ``ties`` exact duplicates, sorted.
    U: 2n x rank with orthonormal columns (QR of a complex Gaussian matrix);
    Q = I - 2 U U^H is unitary, so A = Q diag(Lambda) Q has eigenvalues Lambda
    and eigenvectors Q e_i; it is formed as
    diag(Lambda) + [U, Lambda U] M [U, Lambda U]^H with M = [[4 U^H Lambda U, -2 I],
    [-2 I, 0]].  L0: unit lower bidiagonal, complex subdiagonal of modulus <=
    ``offdiag``; S = L0 L0^H (n x n) and H = B A B^H with B = diag(L0, L0), so
    H C = diag(S, S) C eps has eps = Lambda and C = B^-H Q.

    Returns a Problem (nsp = 2) whose meta holds Lambda, U and the subdiagonal
    of L0."""
    rng = np.random.default_rng(seed)
    order = 2 * n
    lam = np.sort(rng.uniform(lo, hi, size=order))
    pos = rng.choice(order - 1, size=close_pairs + ties, replace=False)
    for q, i in enumerate(pos):
        lam[i + 1] = lam[i] + (close_gap * rng.uniform(0.1, 1.0) if q < close_pairs else 0.0)
    lam = np.sort(lam)
    G = rng.normal(size=(order, rank)) + 1j * rng.normal(size=(order, rank))
    U, _ = np.linalg.qr(G)
    LU = lam[:, None] * U
    M11 = 4.0 * (U.conj().T @ LU)
    P = np.concatenate([U, LU], axis=1)
    M = np.zeros((2 * rank, 2 * rank), np.complex128)
    M[:rank, :rank] = M11
    M[:rank, rank:] = -2.0 * np.eye(rank)
    M[rank:, :rank] = -2.0 * np.eye(rank)
    A = (P @ M) @ P.conj().T
    A[np.diag_indices(order)] += lam
    a = offdiag * rng.uniform(0.0, 1.0, size=n - 1) * np.exp(2j * np.pi * rng.uniform(size=n - 1))
    # B A B^H with B = diag(L0, L0): row i of B X is X_i + a_{i-1} X_{i-1} within a spin block
    BA = A.copy()
    for b in range(2):
        o = b * n
        BA[o + 1:o + n] += a[:, None] * A[o:o + n - 1]
    H = BA.copy()
    for b in range(2):
        o = b * n
        H[:, o + 1:o + n] += BA[:, o:o + n - 1] * a.conj()[None, :]
    # Hermitian up to rounding (only the lower triangle is read by the solver);
    # the diagonal is made exactly real
    H[np.diag_indices(order)] = H[np.diag_indices(order)].real
    S = np.zeros((n, n), np.complex128)
    S[np.diag_indices(n)] = 1.0
    S[np.arange(1, n), np.arange(1, n)] += np.abs(a) ** 2
    S[np.arange(1, n), np.arange(n - 1)] = a
    S[np.arange(n - 1), np.arange(1, n)] = a.conj()
    return Problem(H, S, float(n_electrons), float(kT), 2, None, "known_spectrum_spinor",
                   dict(lam=lam, U=U, a=a, seed=seed))


# Named workloads: the five configurations and small stand-ins of the same kind.
def workload(name: str, seed: int = 0) -> Problem:
    if name == "toy64":
        return toy(seed)
    if name == "supercell6656":
        return supercell(seed)
    if name == "noncollinear9984":
        return noncollinear(seed)
    if name == "noncollinear4160":
        # 160 atoms on a perturbed 8 x 5 x 4 lattice: order 4160 complex spinor, 640 electrons
        return noncollinear(seed, nx=8, ny=5, nz=4)
    if name == "kpoints16x1300":
        return kpoint_batch(seed)
    if name == "diff2048":
        return differentiation(seed)
    raise KeyError(name)
