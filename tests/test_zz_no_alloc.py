"""ks_density_noalloc (the allocation-free density build) against ks_density:
same kernels, so the same results bit for bit; two calls in a row, the second
on a smaller input, share the static scratch of the GPU."""
import ctypes

import numpy as np
import pytest
import torch

from paper_2606_09058_amd import inputs as I
from paper_2606_09058_amd import ks
from tests.gpu_helpers import announce, dev, host

pytestmark = pytest.mark.gpu
V, I32, D = ctypes.c_void_p, ctypes.c_int32, ctypes.c_double


def _lib():
    L = ks.lib()
    L.ks_density_noalloc.argtypes = [ctypes.POINTER(ks.PlanDesc), V, V, I32, I32, D, D, V, V, V, V, V, V]
    L.ks_density_noalloc.restype = I32
    return L


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _case(p, il, iu, with_occ, with_info):
    """Solve p once, then build the density with ks_density (plan workspace) and
    with ks_density_noalloc (static scratch) from the same eigenpairs."""
    L = _lib()
    cplx = np.iscomplexobj(p.H)
    plan = ks.Plan(p.n, batch=p.batch, complex=cplx, noncollinear=p.nsp == 2)
    H, S = dev(p.H), dev(p.S.astype(p.H.dtype))
    eps = torch.empty(plan._vshape(), dtype=torch.float64, device="cuda")
    C = torch.zeros(plan._mshape(), dtype=plan.mdtype, device="cuda")
    plan.gevd(H, S, eps, C, il=il, iu=iu)
    ref = dict(rho=torch.empty_like(C), mu=torch.empty(1, dtype=torch.float64, device="cuda"),
               eband=torch.empty(1, dtype=torch.float64, device="cuda"),
               occ=torch.empty(plan._vshape(), dtype=torch.float64, device="cuda"))
    plan.density(eps, C, p.n_electrons, p.kT, ref["rho"], ref["mu"], ref["eband"], occ=ref["occ"], il=il, iu=iu,
                 kweights=p.weights)
    plan.check("ks_density")
    got = dict(rho=torch.full_like(C, 7.0), mu=torch.zeros(1, dtype=torch.float64, device="cuda"),
               eband=torch.zeros(1, dtype=torch.float64, device="cuda"))
    occ = torch.zeros(plan._vshape(), dtype=torch.float64, device="cuda") if with_occ else None
    info = torch.full((2,), 5, dtype=torch.int32, device="cuda") if with_info else None
    kw = None
    if p.weights is not None:
        arr = (ctypes.c_double * p.batch)(*[float(x) for x in p.weights])
        kw = ctypes.cast(arr, ctypes.c_void_p)
    st = L.ks_density_noalloc(ctypes.byref(plan.desc), _ptr(eps), _ptr(C), il, iu, float(p.n_electrons),
                              float(p.kT), kw, _ptr(got["rho"]), _ptr(got["mu"]), _ptr(got["eband"]), _ptr(occ),
                              _ptr(info))
    assert st == 0, st
    torch.cuda.synchronize()
    for k in ("rho", "mu", "eband"):
        assert np.array_equal(host(got[k]), host(ref[k])), k
    if with_occ:
        assert np.array_equal(host(occ), host(ref["occ"]))
    if with_info:
        assert host(info).tolist() == [0, 0]
    return host(got["rho"])


def test_noalloc_matches_ks_density_twice_then_smaller():
    """Call 1: a batch of three complex k-points of order 390 (occupations to the
    scratch array); call 2: one real matrix of order 120 with a window (caller's
    occupation and info buffers); call 3 repeats the first: every call equals
    ks_density bit for bit, whatever the previous call left in the scratch."""
    announce("noalloc density")
    big = I.kpoint_batch(natoms=5, norb=13, kgrid=(3, 1, 1), seed=4)
    small = I.toy(seed=9, natoms=10, norb=12, edge=12.0, n_electrons=50.0, kT=0.01)
    r1 = _case(big, 1, big.order, with_occ=False, with_info=False)
    _case(small, 1, 60, with_occ=True, with_info=True)
    r3 = _case(big, 1, big.order, with_occ=False, with_info=False)
    assert np.array_equal(r1, r3)


def test_noalloc_reports_window_failure_and_rejects_oversize():
    """An occupied state outside the window is recorded in the caller's info word
    (KS_ERR_WINDOW); a batch whose occupations would not fit the static scratch
    is refused before any device work (KS_ERR_ALLOC)."""
    announce("noalloc failures")
    L = _lib()
    p = I.toy(seed=9, natoms=10, norb=12, edge=12.0, n_electrons=50.0, kT=0.01)
    plan = ks.Plan(p.n)
    eps = torch.empty(p.order, dtype=torch.float64, device="cuda")
    C = torch.zeros((p.order, p.order), dtype=torch.float64, device="cuda")
    plan.gevd(dev(p.H), dev(p.S), eps, C)
    rho = torch.empty_like(C)
    mu = torch.zeros(1, dtype=torch.float64, device="cuda")
    eb = torch.zeros(1, dtype=torch.float64, device="cuda")
    info = torch.zeros(2, dtype=torch.int32, device="cuda")
    st = L.ks_density_noalloc(ctypes.byref(plan.desc), _ptr(eps), _ptr(C), 1, 3, 50.0, 0.01, None, _ptr(rho),
                              _ptr(mu), _ptr(eb), None, _ptr(info))
    assert st == 0
    torch.cuda.synchronize()
    assert host(info)[0] == 5  # KS_ERR_WINDOW
    desc = ks.PlanDesc(60000, 64, 0, 0, 0, 60000, 60000, None, 0)
    st = L.ks_density_noalloc(ctypes.byref(desc), _ptr(eps), _ptr(C), 1, 10, 50.0, 0.01, None, _ptr(rho), _ptr(mu),
                              _ptr(eb), None, None)
    assert st == 7  # KS_ERR_ALLOC
