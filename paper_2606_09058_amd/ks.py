"""Thin Python binding of include/ks.h (ctypes; argument marshalling only).

Every step of the solve runs in the HIP library ``libks.so``; this module only
checks tensor shapes/dtypes/devices, passes device pointers and the current
torch stream, and maps status codes to exceptions.  If the library is missing
the import of the binding fails loudly; there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

import torch

from . import tune_cache as tune_cache_mod

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libks.so")

KS_REAL64, KS_COMPLEX128 = 0, 1
KS_COLLINEAR, KS_NONCOLLINEAR = 0, 1
KS_FP64, KS_MIXED = 0, 1
KS_PLAN_GRAPH = 1
KS_PLAN_AUTOTUNE = 2
KS_PLAN_LOWDIN = 4
KS_PLAN_TWOSTAGE = 8
KS_PLAN_REAL_OVERLAP = 16
KS_REUSE_S = 1

STATUS = {
    0: "KS_OK", 1: "KS_ERR_INVALID_ARG", 2: "KS_ERR_NOT_POSDEF", 3: "KS_ERR_NO_CONVERGENCE",
    4: "KS_ERR_ELECTRON_COUNT", 5: "KS_ERR_WINDOW", 6: "KS_ERR_NONFINITE", 7: "KS_ERR_ALLOC",
    8: "KS_ERR_HIP", 9: "KS_ERR_NOT_SUPPORTED",
}

EXPORTS = ["ks_plan_create", "ks_plan_destroy", "ks_gevd", "ks_density", "ks_energy_density", "ks_bloch_sum",
           "ks_density_backward",
           "ks_plan_get_info", "ks_status_string", "ks_plan_workspace_bytes", "ks_plan_set_profiling",
           "ks_plan_get_profile", "ks_plan_get_graph_stats", "ks_plan_get_tuning", "ks_plan_set_tuning", "ks_plan_set_refinement",
           "ks_plan_set_overlap_cutoff", "ks_plan_get_overlap_rank"]


class KSError(RuntimeError):
    def __init__(self, status, where="", info=0):
        self.status = int(status)
        self.info = int(info)
        msg = "%s: %s (%s)" % (where, STATUS.get(self.status, "?"), _status_string(self.status))
        if info:
            msg += " info=%d" % info
        super().__init__(msg)


class PlanDesc(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("batch", ctypes.c_int32), ("dtype", ctypes.c_int32),
                ("spin", ctypes.c_int32), ("precision", ctypes.c_int32), ("ld_h", ctypes.c_int32),
                ("ld_s", ctypes.c_int32), ("stream", ctypes.c_void_p), ("flags", ctypes.c_uint32)]


class Profile(ctypes.Structure):
    """ks_profile: per-phase times and the sampled matrix-vector kernel launches."""
    _fields_ = [("phase_ms", ctypes.c_double * 8), ("phase_calls", ctypes.c_int64 * 8),
                ("hemv_ms", ctypes.c_double), ("hemv_launches", ctypes.c_int64),
                ("hemv_bytes", ctypes.c_double)]


class Tuning(ctypes.Structure):
    """ks_tuning: the plan's knobs and, under KS_PLAN_AUTOTUNE, the timings behind them."""
    _fields_ = [("tiles_per_workgroup", ctypes.c_int32), ("ncand", ctypes.c_int32),
                ("cand", ctypes.c_int32 * 4), ("ms", ctypes.c_double * 4), ("nseg", ctypes.c_int32),
                ("seg_first", ctypes.c_int32 * 8), ("seg_tiles", ctypes.c_int32 * 8),
                ("backtr_block", ctypes.c_int32), ("gemm_big_min_k", ctypes.c_int32),
                ("backtr_ms", (ctypes.c_double * 2) * 2), ("dc_leaf", ctypes.c_int32),
                ("dc_ms", ctypes.c_double * 2), ("from_cache", ctypes.c_int32)]


KS_TUNE_NEVER = 0x7FFFFFFF


_lib = None


def lib():
    """Load libks.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("HIP library %s is missing; build it with "
                               "`python -m paper_2606_09058_amd.build`" % LIB_PATH)
        L = ctypes.CDLL(LIB_PATH)
        P, I, U, D = ctypes.c_void_p, ctypes.c_int32, ctypes.c_uint32, ctypes.c_double
        L.ks_plan_create.argtypes = [ctypes.POINTER(PlanDesc), ctypes.POINTER(ctypes.c_void_p)]
        L.ks_plan_create.restype = I
        L.ks_plan_destroy.argtypes = [P]
        L.ks_plan_destroy.restype = None
        L.ks_gevd.argtypes = [P, P, P, P, P, I, I, U]
        L.ks_gevd.restype = I
        L.ks_density.argtypes = [P, P, P, I, I, D, D, P, P, P, P, P]
        L.ks_density.restype = I
        L.ks_energy_density.argtypes = [P, P, P, I, I, P, P]
        L.ks_energy_density.restype = I
        L.ks_bloch_sum.argtypes = [P, I, P, P, P, I, P, I]
        L.ks_bloch_sum.restype = I
        L.ks_plan_set_overlap_cutoff.argtypes = [P, D]
        L.ks_plan_set_overlap_cutoff.restype = I
        L.ks_plan_get_overlap_rank.argtypes = [P, P]
        L.ks_plan_get_overlap_rank.restype = I
        L.ks_density_backward.argtypes = [P, P, P, P, P, D, P, P, P, P]
        L.ks_density_backward.restype = I
        L.ks_plan_get_info.argtypes = [P, ctypes.POINTER(I)]
        L.ks_plan_get_info.restype = I
        L.ks_status_string.argtypes = [I]
        L.ks_status_string.restype = ctypes.c_char_p
        L.ks_plan_workspace_bytes.argtypes = [ctypes.POINTER(PlanDesc)]
        L.ks_plan_workspace_bytes.restype = ctypes.c_uint64
        L.ks_plan_set_profiling.argtypes = [P, I, I]
        L.ks_plan_set_profiling.restype = I
        L.ks_plan_get_profile.argtypes = [P, ctypes.POINTER(Profile)]
        L.ks_plan_get_profile.restype = I
        L.ks_plan_get_graph_stats.argtypes = [P, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)]
        L.ks_plan_get_graph_stats.restype = I
        L.ks_plan_get_tuning.argtypes = [P, ctypes.POINTER(Tuning)]
        L.ks_plan_get_tuning.restype = I
        L.ks_plan_set_tuning.argtypes = [P, ctypes.POINTER(Tuning)]
        L.ks_plan_set_tuning.restype = I
        L.ks_plan_set_refinement.argtypes = [P, I]
        L.ks_plan_set_refinement.restype = I
        _lib = L
    return _lib


def _status_string(st):
    try:
        return lib().ks_status_string(int(st)).decode()
    except Exception:  # noqa: BLE001 - message only
        return "?"


def _check(st, where):
    if st != 0:
        raise KSError(st, where)


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _need(t, name, dtype, shape=None):
    if not isinstance(t, torch.Tensor):
        raise TypeError("%s must be a torch tensor" % name)
    if t.device.type != "cuda":
        raise ValueError("%s must live on the GPU" % name)
    if t.dtype != dtype:
        raise TypeError("%s must be %s, got %s" % (name, dtype, t.dtype))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError("%s has shape %s, expected %s" % (name, tuple(t.shape), tuple(shape)))


class Plan:
    """Owns a ks_plan: workspace for `batch` problems of `n` orbitals per spin block."""

    def __init__(self, n, batch=1, complex=False, noncollinear=False, precision=KS_FP64, stream=None,
                 ld_h=None, ld_s=None, flags=0, tune_cache=None):
        """tune_cache: path of a tuning-cache JSON file.  With KS_PLAN_AUTOTUNE in
        flags, a plan whose key is in the cache takes the stored knobs without
        timing anything (tuning()["from_cache"] is then True); otherwise it is
        tuned and its knobs are added to the cache."""
        self.n = int(n)
        self.batch = int(batch)
        self.nsp = 2 if noncollinear else 1
        self.order = self.n * self.nsp
        self.complex = bool(complex or noncollinear)
        self.g = 1.0 if noncollinear else 2.0
        self.mdtype = torch.complex128 if self.complex else torch.float64
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        handle = stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)
        self.desc = PlanDesc(self.n, self.batch, KS_COMPLEX128 if self.complex else KS_REAL64,
                             KS_NONCOLLINEAR if noncollinear else KS_COLLINEAR, int(precision),
                             int(ld_h or self.order), int(ld_s or self.n), ctypes.c_void_p(handle),
                             int(flags))
        self._h = ctypes.c_void_p()
        entry, key = None, None
        if tune_cache is not None and (flags & KS_PLAN_AUTOTUNE):
            key = self.tune_key(flags)
            entry = tune_cache_mod.lookup(tune_cache, key)
            if entry is not None:
                self.desc.flags = int(flags) & ~KS_PLAN_AUTOTUNE
        _check(lib().ks_plan_create(ctypes.byref(self.desc), ctypes.byref(self._h)), "ks_plan_create")
        self.desc.flags = int(flags)
        if entry is not None:
            self.set_tuning(entry)
        elif key is not None:
            tune_cache_mod.store(tune_cache, key, self.tuning_knobs())

    def tune_key(self, flags=None):
        """The tuning-cache key of this plan's shape on the current device."""
        flags = self.desc.flags if flags is None else flags
        props = torch.cuda.get_device_properties(torch.cuda.current_device())
        arch = "%s-%dcu" % (props.gcnArchName.split(":")[0], props.multi_processor_count)
        route = "twostage" if flags & KS_PLAN_TWOSTAGE else ("lowdin" if flags & KS_PLAN_LOWDIN else "onestage")
        return tune_cache_mod.cache_key(arch, "gevd", "complex128" if self.complex else "real64", self.order,
                                        self.batch, "noncollinear" if self.nsp == 2 else "collinear",
                                        "mixed" if self.desc.precision == KS_MIXED else "fp64", route)

    # shapes --------------------------------------------------------------------------------
    def _mshape(self):
        return (self.batch, self.order, self.order) if self.batch > 1 else (self.order, self.order)

    def _sshape(self):
        return (self.batch, self.n, self.n) if self.batch > 1 else (self.n, self.n)

    def _vshape(self):
        return (self.batch, self.order) if self.batch > 1 else (self.order,)

    # entry points --------------------------------------------------------------------------
    def gevd(self, H, S, eps, C, il=1, iu=None, reuse_s=False):
        iu = self.order if iu is None else iu
        _need(H, "H", self.mdtype, self._mshape())
        if S is not None:
            _need(S, "S", self.mdtype, self._sshape())
        _need(eps, "eps", torch.float64, self._vshape())
        _need(C, "C", self.mdtype, self._mshape())
        st = lib().ks_gevd(self._h, _ptr(H), _ptr(S), _ptr(eps), _ptr(C), int(il), int(iu),
                           KS_REUSE_S if reuse_s else 0)
        _check(st, "ks_gevd")

    def density(self, eps, C, n_electrons, kT, rho, mu, eband, occ=None, il=1, iu=None,
                kweights=None):
        iu = self.order if iu is None else iu
        _need(eps, "eps", torch.float64, self._vshape())
        _need(C, "C", self.mdtype, self._mshape())
        _need(rho, "rho", self.mdtype, self._mshape())
        _need(mu, "mu", torch.float64, (1,))
        _need(eband, "eband", torch.float64, (1,))
        if occ is not None:
            _need(occ, "occ", torch.float64, self._vshape())
        kw = None
        if kweights is not None:
            arr = (ctypes.c_double * self.batch)(*[float(x) for x in kweights])
            kw = ctypes.cast(arr, ctypes.c_void_p)
        st = lib().ks_density(self._h, _ptr(eps), _ptr(C), int(il), int(iu), float(n_electrons),
                              float(kT), kw, _ptr(rho), _ptr(mu), _ptr(eband), _ptr(occ))
        _check(st, "ks_density")

    def energy_density(self, eps, C, occ, edm, il=1, iu=None):
        """ks_energy_density: edm = C diag(occ eps) C^H over the window il..iu (device tensors)."""
        iu = self.order if iu is None else iu
        _need(eps, "eps", torch.float64, self._vshape())
        _need(C, "C", self.mdtype, self._mshape())
        _need(occ, "occ", torch.float64, self._vshape())
        _need(edm, "edm", self.mdtype, self._mshape())
        st = lib().ks_energy_density(self._h, _ptr(eps), _ptr(C), int(il), int(iu), _ptr(occ), _ptr(edm))
        _check(st, "ks_energy_density")

    def bloch_sum(self, R, kvec, XR, Xk):
        """ks_bloch_sum: Xk[q] = sum_r XR[r] exp(i kvec[q].R[r]) (device tensors; XR real
        (nR, n, n), Xk complex (batch, n, n) or (n, n) for one k-point)."""
        nR = int(R.shape[0])
        _need(R, "R", torch.float64, (nR, 3))
        _need(kvec, "kvec", torch.float64, (self.batch, 3))
        _need(XR, "XR", torch.float64, (nR, self.n, self.n))
        _need(Xk, "Xk", torch.complex128, self._mshape())
        st = lib().ks_bloch_sum(self._h, nR, _ptr(R), _ptr(kvec), _ptr(XR), self.n, _ptr(Xk), self.n)
        _check(st, "ks_bloch_sum")

    def density_backward(self, eps, C, mu, occ, kT, grad_rho, grad_eband, grad_H, grad_S):
        _need(eps, "eps", torch.float64, self._vshape())
        _need(C, "C", self.mdtype, self._mshape())
        _need(mu, "mu", torch.float64, (1,))
        _need(occ, "occ", torch.float64, self._vshape())
        if grad_rho is not None:
            _need(grad_rho, "grad_rho", self.mdtype, self._mshape())
        if grad_eband is not None:
            _need(grad_eband, "grad_eband", torch.float64, (1,))
        _need(grad_H, "grad_H", self.mdtype, self._mshape())
        _need(grad_S, "grad_S", self.mdtype, self._sshape())
        st = lib().ks_density_backward(self._h, _ptr(eps), _ptr(C), _ptr(mu), _ptr(occ), float(kT),
                                       _ptr(grad_rho), _ptr(grad_eband), _ptr(grad_H), _ptr(grad_S))
        _check(st, "ks_density_backward")

    def set_overlap_cutoff(self, tau):
        """KS_PLAN_LOWDIN: drop the eigenvectors of S with s <= tau * max(s)."""
        _check(lib().ks_plan_set_overlap_cutoff(self._h, float(tau)), "ks_plan_set_overlap_cutoff")

    def overlap_rank(self):
        """KS_PLAN_LOWDIN: eigenvectors of S kept per k-point by the last decomposition."""
        v = (ctypes.c_int32 * self.batch)()
        _check(lib().ks_plan_get_overlap_rank(self._h, v), "ks_plan_get_overlap_rank")
        return [int(x) for x in v]

    def set_profiling(self, enable, stride=1):
        _check(lib().ks_plan_set_profiling(self._h, int(bool(enable)), int(stride)), "ks_plan_set_profiling")

    def get_profile(self):
        pr = Profile()
        _check(lib().ks_plan_get_profile(self._h, ctypes.byref(pr)), "ks_plan_get_profile")
        return pr

    def set_refinement(self, sweeps):
        """KS_MIXED: correction sweeps before the final Rayleigh-Ritz step."""
        _check(lib().ks_plan_set_refinement(self._h, int(sweeps)), "ks_plan_set_refinement")

    def tuning(self):
        """The plan's knobs and (under KS_PLAN_AUTOTUNE) the timings behind them:
        tiles_per_workgroup, candidates {tiles: ms}, segments [(first column, tiles)],
        backtr_block, gemm_big_min_k (KS_TUNE_NEVER: 64 x 64 tiles only),
        backtr_ms {(block, big_min_k): ms}, dc_leaf, dc_ms {leaf: ms}, from_cache."""
        tu = Tuning()
        _check(lib().ks_plan_get_tuning(self._h, ctypes.byref(tu)), "ks_plan_get_tuning")
        return {"tiles_per_workgroup": int(tu.tiles_per_workgroup),
                "candidates": {int(tu.cand[i]): float(tu.ms[i]) for i in range(tu.ncand)},
                "segments": [(int(tu.seg_first[i]), int(tu.seg_tiles[i])) for i in range(tu.nseg)],
                "backtr_block": int(tu.backtr_block), "gemm_big_min_k": int(tu.gemm_big_min_k),
                "backtr_ms": {(128 << b, KS_TUNE_NEVER if g else 256): float(tu.backtr_ms[b][g])
                              for b in range(2) for g in range(2)},
                "dc_leaf": int(tu.dc_leaf), "dc_ms": {16 << i: float(tu.dc_ms[i]) for i in range(2)},
                "from_cache": bool(tu.from_cache)}

    def tuning_knobs(self):
        """The knobs alone, as a tuning-cache entry."""
        tu = Tuning()
        _check(lib().ks_plan_get_tuning(self._h, ctypes.byref(tu)), "ks_plan_get_tuning")
        return {"tiles_per_workgroup": int(tu.tiles_per_workgroup), "nseg": int(tu.nseg),
                "seg_first": [int(tu.seg_first[i]) for i in range(tu.nseg)],
                "seg_tiles": [int(tu.seg_tiles[i]) for i in range(tu.nseg)],
                "backtr_block": int(tu.backtr_block), "gemm_big_min_k": int(tu.gemm_big_min_k),
                "dc_leaf": int(tu.dc_leaf)}

    def set_tuning(self, knobs):
        """Set the knobs from a tuning-cache entry (ks_plan_set_tuning)."""
        tu = Tuning()
        tu.tiles_per_workgroup = int(knobs["tiles_per_workgroup"])
        tu.nseg = int(knobs["nseg"])
        if not 1 <= tu.nseg <= 8 or len(knobs["seg_first"]) != tu.nseg or len(knobs["seg_tiles"]) != tu.nseg:
            raise ValueError("bad segment list in tuning entry")
        for i in range(tu.nseg):
            tu.seg_first[i] = int(knobs["seg_first"][i])
            tu.seg_tiles[i] = int(knobs["seg_tiles"][i])
        tu.backtr_block = int(knobs["backtr_block"])
        tu.gemm_big_min_k = int(knobs["gemm_big_min_k"])
        tu.dc_leaf = int(knobs["dc_leaf"])
        _check(lib().ks_plan_set_tuning(self._h, ctypes.byref(tu)), "ks_plan_set_tuning")

    def graph_stats(self):
        """(captures, replays) of ks_gevd under KS_PLAN_GRAPH."""
        c, r = ctypes.c_int64(0), ctypes.c_int64(0)
        _check(lib().ks_plan_get_graph_stats(self._h, ctypes.byref(c), ctypes.byref(r)), "ks_plan_get_graph_stats")
        return int(c.value), int(r.value)

    def get_info(self):
        """Synchronize and return (status, info); clears the device info word."""
        v = ctypes.c_int32(0)
        st = lib().ks_plan_get_info(self._h, ctypes.byref(v))
        return int(st), int(v.value)

    def check(self, where="device"):
        st, info = self.get_info()
        if st != 0:
            raise KSError(st, where, info)

    def close(self):
        if self._h:
            lib().ks_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:  # noqa: BLE001 - interpreter teardown
            pass

    # convenience ---------------------------------------------------------------------------
    def empty_matrix(self):
        return torch.empty(self._mshape(), dtype=self.mdtype, device="cuda")

    def solve(self, H, S, n_electrons, kT, il=1, iu=None, kweights=None, reuse_s=False, check=True):
        """ks_gevd + ks_density; returns dict of device tensors."""
        dev = H.device
        eps = torch.empty(self._vshape(), dtype=torch.float64, device=dev)
        C = torch.zeros(self._mshape(), dtype=self.mdtype, device=dev)
        rho = torch.empty(self._mshape(), dtype=self.mdtype, device=dev)
        mu = torch.empty(1, dtype=torch.float64, device=dev)
        eband = torch.empty(1, dtype=torch.float64, device=dev)
        occ = torch.empty(self._vshape(), dtype=torch.float64, device=dev)
        self.gevd(H, S, eps, C, il=il, iu=iu, reuse_s=reuse_s)
        self.density(eps, C, n_electrons, kT, rho, mu, eband, occ=occ, il=il, iu=iu, kweights=kweights)
        if check:
            self.check("solve")
        return dict(eps=eps, C=C, rho=rho, mu=mu, eband=eband, occ=occ)


# Plans of KSDensity, one per (order, element type, spin form, device, stream):
# a self-consistent loop that calls KSDensity every cycle reuses the plan's
# workspace instead of allocating it again, and the Cholesky factor of S while
# S is the same tensor, unmodified (same object, same version counter; the
# plan keeps a reference to it, so its memory cannot be reused meanwhile).
_PLANS = {}


def clear_plan_cache():
    """Destroy the plans KSDensity keeps (frees their device workspace)."""
    for plan, _ in _PLANS.values():
        plan.close()
    _PLANS.clear()


def _density_plan(n, cplx, noncollinear, device):
    stream = torch.cuda.current_stream(device)
    key = (int(n), bool(cplx), bool(noncollinear), device.index, stream.cuda_stream)
    ent = _PLANS.get(key)
    if ent is None:
        ent = [Plan(n, complex=cplx, noncollinear=noncollinear, stream=stream), None]
        _PLANS[key] = ent
    return ent


class KSDensity(torch.autograd.Function):
    """(H, S) -> (rho, E_band) through ks_gevd + ks_density; backward through
    ks_density_backward.  Gradients are the Hermitian matrices grad_H, grad_S with
    dL = Re tr(grad_H^H dH) + Re tr(grad_S^H dS) (torch's convention for real L).
    The plan is cached per shape, type, device and stream, and KS_REUSE_S is
    passed while S is the same unmodified tensor as in the previous call."""

    @staticmethod
    def forward(ctx, H, S, n_electrons, kT, noncollinear=False):
        n = S.shape[-1]
        ent = _density_plan(n, H.is_complex(), noncollinear, H.device)
        plan = ent[0]
        Sc = S.contiguous()
        last = ent[1]
        reuse = last is not None and last[0] is Sc and last[1] == Sc._version
        out = plan.solve(H.contiguous(), None if reuse else Sc, n_electrons, kT, reuse_s=reuse)
        ent[1] = (Sc, Sc._version)
        ctx.plan = plan
        ctx.kT = float(kT)
        ctx.save_for_backward(out["eps"], out["C"], out["mu"], out["occ"])
        return out["rho"], out["eband"]

    @staticmethod
    def backward(ctx, grad_rho, grad_eband):
        eps, C, mu, occ = ctx.saved_tensors
        plan = ctx.plan
        gH = plan.empty_matrix()
        gS = torch.empty(plan._sshape(), dtype=plan.mdtype, device=C.device)
        gr = None if grad_rho is None else grad_rho.contiguous()
        ge = None if grad_eband is None else grad_eband.contiguous().reshape(1).to(torch.float64)
        plan.density_backward(eps, C, mu, occ, ctx.kT, gr, ge, gH, gS)
        plan.check("ks_density_backward")
        return gH, gS, None, None, None
