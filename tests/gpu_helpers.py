"""Helpers shared by the GPU tests (device transfer, invariants, oracle runs)."""
import ctypes
import sys

import numpy as np
import torch

from paper_2606_09058_amd import ks


def announce(*parts):
    """Name the case before its GPU work, so a fault report names it."""
    print("[case]", *parts, flush=True)
    sys.stdout.flush()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def stream_handle():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def solve_gpu(p, il=1, iu=None, check=True, flags=0):
    """Run ks_gevd + ks_density on a Problem; returns numpy results and the plan."""
    plan = ks.Plan(p.n, batch=p.batch, complex=np.iscomplexobj(p.H), noncollinear=p.nsp == 2, flags=flags)
    H = dev(p.H)
    S = dev(p.S.astype(p.H.dtype))
    out = plan.solve(H, S, p.n_electrons, p.kT, il=il, iu=iu, kweights=p.weights, check=check)
    res = {k: host(v) for k, v in out.items()}
    res["mu"] = float(res["mu"][0])
    res["eband"] = float(res["eband"][0])
    return res, plan


def residuals(H, S, eps, C, nsp=1):
    """Frobenius ||H C - S_NC C eps|| / (||H|| ||C||) and max |C^H S_NC C - I|."""
    SN = np.kron(np.eye(nsp), S) if nsp == 2 else S
    R = H @ C - (SN @ C) * eps
    res = np.linalg.norm(R) / (np.linalg.norm(H) * np.linalg.norm(C))
    G = C.conj().T @ SN @ C
    orth = np.abs(G - np.eye(G.shape[0])).max()
    return res, orth
