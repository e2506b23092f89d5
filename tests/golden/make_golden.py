"""Write the oracle's reference outputs for the named workloads into tests/golden/.

Calls only ``oracle/`` (and the seeded input generators).  Nothing here comes from
the HIP path.  Usage:  python tests/golden/make_golden.py toy64 [diff2048 ...]

Each JSON file records the SHA-256 of the generated inputs (so a test can detect
drift of the generator), the eigenvalues, mu, E_band, and the density matrix (all
of it for the 64-orbital toy, a seeded sample of entries for the large ones); for
the differentiation workload it also records a sample of the dense adjoint for
L = Re sum_ij W_ij rho_ij with W ~ N(0, 1) (seed 1).
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from paper_2606_09058_amd import inputs as I  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
NSAMPLE = 4096


def cpack(a):
    a = np.asarray(a)
    if np.iscomplexobj(a):
        return [[float(x.real), float(x.imag)] for x in a.ravel()]
    return [float(x) for x in a.ravel()]


def sample_idx(order, seed=2):
    rng = np.random.default_rng(seed)
    return rng.integers(0, order, size=(NSAMPLE, 2))


def host_cpu():
    for line in open("/proc/cpuinfo"):
        if line.startswith("model name"):
            return line.split(":", 1)[1].strip()
    return "unknown"


def one_k(H, S, nsp, nthreads):
    t = time.time()
    eps, C = O.gevd(H, S, nsp=nsp, nthreads=nthreads)
    return eps, C, time.time() - t


def run(name, nthreads=0):
    p = I.workload(name)
    out = dict(workload=name, inputs_sha256=p.digest(), n_electrons=p.n_electrons, kT=p.kT, host_cpu=host_cpu(),
               g=p.g, nsp=p.nsp, order=p.order, batch=p.batch, oracle_threads=O.max_threads()
               if nthreads <= 0 else nthreads)
    Hs = p.H if p.batch > 1 else p.H[None]
    Ss = p.S if p.batch > 1 else p.S[None]
    eps_all, Cs, secs = [], [], []
    for k in range(p.batch):
        e, C, dt = one_k(Hs[k], Ss[k], p.nsp, nthreads)
        eps_all.append(e)
        Cs.append(C)
        secs.append(dt)
        print(name, "k", k, "gevd %.1f s" % dt, flush=True)
    eps_all = np.array(eps_all)
    fr = O.fermi(eps_all, p.n_electrons, p.kT, p.g, wk=p.weights)
    out.update(eps=[cpack(e) for e in eps_all], mu=fr["mu"], eband=fr["eband"], ts=fr["ts"],
               gevd_seconds=secs)
    occ = np.atleast_2d(fr["occ"])
    if p.order <= 64:
        out["rho"] = [cpack(O.density(Cs[k], occ[k])) for k in range(p.batch)]
    else:
        idx = sample_idx(p.order)
        out["rho_idx"] = idx.tolist()
        vals = []
        for k in range(p.batch):
            C = Cs[k]
            f = occ[k]
            a = C[idx[:, 0]] * f
            b = C[idx[:, 1]].conj()
            vals.append(cpack((a * b).sum(1)))
        out["rho_samples"] = vals
    if name == "diff2048":
        rng = np.random.default_rng(1)
        W = rng.normal(size=(p.order, p.order))
        t = time.time()
        Hb, Sb = O.adjoint(eps_all[0], Cs[0], fr["mu"], p.kT, p.g, Gbar=W.astype(np.complex128),
                           ebar=0.0, nsp=p.nsp)
        out["adjoint_seconds"] = time.time() - t
        idx = sample_idx(p.order, seed=3)
        out["grad_idx"] = idx.tolist()
        out["gradH_samples"] = cpack(Hb[idx[:, 0], idx[:, 1]])
        out["gradS_samples"] = cpack(Sb[idx[:, 0], idx[:, 1]])
        out["gradH_fro"] = float(np.linalg.norm(Hb))
        out["gradS_fro"] = float(np.linalg.norm(Sb))
    with open(os.path.join(HERE, name + ".json"), "w") as fh:
        json.dump(out, fh)
    print("wrote", name, flush=True)


if __name__ == "__main__":
    for nm in sys.argv[1:]:
        run(nm)
