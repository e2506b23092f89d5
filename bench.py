#!/usr/bin/env python3
"""Benchmark of the generalized Kohn-Sham eigensolve + density build on one MI355X.

One step = ks_gevd (Cholesky of S, reduction, Householder tridiagonalisation,
divide and conquer, back-transform; all eigenvectors) + ks_density (Fermi level
by bisection, occupations, band energy, density matrix) for one matrix, with
inputs already resident in HBM.  Prints ONE JSON line.

    python bench.py [--steps K] [--warmup W] [--workload supercell6656]

With --counter-workload it instead runs the short fixed workload that the
memory-traffic counters are taken on (one rocprofv3 --pmc run per counter):
a plain 1 GiB device fill and copy, whose counter readings give each
counter's scale, then one FP64 ks_gevd (all eigenvectors) of --workload.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0       # MI355X HBM3E
PEAK_FP64_TFLOPS = 78.6     # MI355X dense FP64 matrix

WORKLOADS = {
    "supercell6656": "N=6656 real symmetric (512 atoms x 13 orbitals, perturbed 8x8x8 lattice, "
                     "12 Bohr cutoff), 2048 electrons, kT=0.01 Ha, all eigenvectors",
    "noncollinear9984": "2N=9984 complex Hermitian spinor (384 atoms x 13 orbitals), overlap S(x)I2, "
                        "1536 electrons, kT=0.01 Ha, all eigenvectors",
    "toy64": "N=64 real symmetric toy (8 atoms x 8 orbitals), 32 electrons, kT=0.01 Ha",
    "kpoints16x1300": "16 k-points x N=1300 complex Hermitian (100-atom cell, 27 lattice vectors), "
                      "400 electrons, kT=0.01 Ha, one common Fermi level, all k in each launch",
}


def nominal_flops(order, ncols, m_occ, cplx, n_s):
    """LAPACK-style nominal counts of the steps performed (real; complex x4):
    Cholesky n^3/3 (n = order of S), reduction order^3, tridiagonalisation
    4 order^3/3, back-transform 2 order^2 ncols + triangular solve order^2 ncols,
    density order^2 m_occ."""
    f = n_s ** 3 / 3.0 + order ** 3 + 4.0 * order ** 3 / 3.0 + 3.0 * order ** 2 * ncols + order ** 2 * m_occ
    return f * (4.0 if cplx else 1.0)


def measured_traffic(workload):
    """Per-launch memory traffic of symv_kernel from the committed counter summary
    (profiles/symv_kernel_<workload>_traffic.txt: FETCH_SIZE + WRITE_SIZE runs,
    each scaled by a plain copy of known size), or None if there is none for
    this workload or the kernel source has changed since it was taken."""
    path = os.path.join(ROOT, "profiles", "symv_kernel_%s_traffic.txt" % workload)
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        line = line.strip()
        if line and not line.startswith("#") and "=" in line:
            k, v = line.split("=", 1)
            kv[k.strip()] = v.strip()
    src = os.path.join(ROOT, kv.get("source_file", "-"))
    if not os.path.isfile(src):
        return None
    if hashlib.sha256(open(src, "rb").read()).hexdigest() != kv.get("source_sha256"):
        return None
    return {"bytes": float(kv["traffic_bytes_per_launch_avg"]),
            "over_algorithmic": float(kv["traffic_over_algorithmic"]),
            "source": os.path.relpath(path, ROOT)}


def cpu_baseline(p, n_sample):
    """The oracle as it stands, on the leading n_sample x n_sample principal block of
    the same workload (electron count scaled), scaled by (order / n_sample)^3."""
    import numpy as np
    from oracle import oracle as O
    ns = min(n_sample, p.n)
    H = np.ascontiguousarray(p.H[:ns, :ns])
    S = np.ascontiguousarray(p.S[:ns, :ns])
    ne = p.n_electrons * ns / p.n
    t0 = time.perf_counter()
    O.solve(H, S, ne, p.kT, nsp=1)
    dt = time.perf_counter() - t0
    scale = (p.order / ns) ** 3
    return {"value": dt * scale, "unit": "s/solve", "cores": O.max_threads(), "kind": "oracle",
            "sample": "oracle (Cholesky + cyclic Jacobi + back-substitution + Fermi bisection + "
                      "density) on the leading %dx%d principal block of the same workload "
                      "(%.0f electrons) took %.2f s; scaled by (%d/%d)^3" % (ns, ns, ne, dt, p.order, ns)}


COPY_BYTES = 1 << 30


def counter_workload(p):
    """A plain copy of known size (the fill writes 1 GiB, the copy reads 1 GiB and
    writes 1 GiB), then one FP64 solve whose kernels the counters measure."""
    import numpy as np
    import torch
    from paper_2606_09058_amd import ks
    x = torch.empty(COPY_BYTES // 8, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    x.fill_(1.0)
    y.copy_(x)
    torch.cuda.synchronize()
    print("copy_bytes", COPY_BYTES, flush=True)
    del x, y
    plan = ks.Plan(p.n, batch=p.batch, complex=np.iscomplexobj(p.H), noncollinear=p.nsp == 2)
    H = torch.from_numpy(p.H).cuda()
    S = torch.from_numpy(p.S.astype(p.H.dtype)).cuda()
    eps = torch.empty(plan._vshape(), dtype=torch.float64, device="cuda")
    C = torch.empty(plan._mshape(), dtype=plan.mdtype, device="cuda")
    plan.gevd(H, S, eps, C)
    plan.check("counter workload")
    print("solved", p.name, "order", p.order, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="supercell6656", choices=sorted(WORKLOADS))
    ap.add_argument("--stride", type=int, default=16, help="sample every n-th matrix-vector launch")
    ap.add_argument("--cpu-sample", type=int, default=1700)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true",
                    help="skip the FP64-vs-mixed comparison on the occupied window")
    ap.add_argument("--no-lowdin", action="store_true", help="skip the Loewdin-route comparison")
    ap.add_argument("--graph", action="store_true", help="plan with KS_PLAN_GRAPH (capture once, replay)")
    ap.add_argument("--counter-workload", action="store_true",
                    help="run the fixed workload of the rocprofv3 memory-counter runs and exit")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on one GPU only: a single matrix of this solve does not shard, and "
              "k-point sharding across GPUs is not implemented here (--gpus 1)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2606_09058_amd import inputs as I
    from paper_2606_09058_amd import ks

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    p = I.workload(args.workload)
    if args.counter_workload:
        counter_workload(p)
        return
    cplx = np.iscomplexobj(p.H)
    stream = torch.cuda.Stream() if args.graph else torch.cuda.current_stream()
    torch.cuda.set_stream(stream)
    # the plan times its symmetric-product tile shapes at creation (KS_PLAN_AUTOTUNE)
    plan = ks.Plan(p.n, batch=p.batch, complex=cplx, noncollinear=p.nsp == 2, stream=stream,
                   flags=ks.KS_PLAN_AUTOTUNE | (ks.KS_PLAN_GRAPH if args.graph else 0))
    H = torch.from_numpy(p.H).cuda()
    S = torch.from_numpy(p.S.astype(p.H.dtype)).cuda()
    eps = torch.empty(plan._vshape(), dtype=torch.float64, device="cuda")
    C = torch.empty(plan._mshape(), dtype=plan.mdtype, device="cuda")
    rho = torch.empty_like(C)
    mu = torch.empty(1, dtype=torch.float64, device="cuda")
    eband = torch.empty(1, dtype=torch.float64, device="cuda")
    occ = torch.empty(plan._vshape(), dtype=torch.float64, device="cuda")

    def step(reuse=False):
        plan.gevd(H, S, eps, C, reuse_s=reuse)
        plan.density(eps, C, p.n_electrons, p.kT, rho, mu, eband, occ=occ, kweights=p.weights)

    for _ in range(args.warmup):
        step()
    plan.check("warmup")
    plan.get_profile()  # clear
    plan.set_profiling(True, args.stride)

    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(args.steps):
        step()
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1) / args.steps
    prof = plan.get_profile()
    plan.set_profiling(False)
    plan.check("timed steps")

    # warm solves (cached Cholesky factor), the analogue of SCF cycles 2 onwards
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(args.steps):
        step(reuse=True)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_warm = e0.elapsed_time(e1) / args.steps
    plan.check("warm steps")

    # cheap property checks of the last solve
    SN = torch.block_diag(S, S) if p.nsp == 2 else S  # overlap of the spinor basis
    if p.batch == 1:
        tr = float((rho * SN.to(rho.dtype).T).sum().real.item())
    else:
        w = torch.tensor(p.weights, dtype=torch.float64, device="cuda")
        tr = float((w * (rho * S.to(rho.dtype).transpose(1, 2)).sum(dim=(1, 2)).real).sum().item())
    m_occ = int((occ > 2e-15 * p.g).sum(dim=-1).max().item())
    flops = p.batch * nominal_flops(p.order, p.order, m_occ, cplx, p.n)

    # energy-density matrix E = C diag(f eps) C^H of the last solve, over the
    # columns that carry occupation (outside the timed steps: not part of `value`)
    edm = torch.empty_like(rho)
    with torch.cuda.stream(stream):
        plan.energy_density(eps, C, occ, edm, il=1, iu=max(1, m_occ))
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(args.steps):
        plan.energy_density(eps, C, occ, edm, il=1, iu=max(1, m_occ))
    e1.record(stream)
    torch.cuda.synchronize()
    plan.check("energy density")
    ms_edm = e0.elapsed_time(e1) / args.steps
    SNe = torch.block_diag(S, S) if p.nsp == 2 else S
    if p.batch == 1:
        edm_tr = float((edm * SNe.to(edm.dtype).T).sum().real.item())
    else:
        wk = torch.tensor(p.weights, dtype=torch.float64, device="cuda")
        edm_tr = float((wk * (edm * S.to(edm.dtype).transpose(1, 2)).sum(dim=(1, 2)).real).sum().item())
    # lower triangle of an order x order x m_occ product (x4 for complex)
    edm_flops = p.batch * (4.0 if cplx else 1.0) * p.order * p.order * m_occ
    hemv_avg_us = 1e3 * prof.hemv_ms / max(1, prof.hemv_launches)
    hemv_gbs = prof.hemv_bytes / max(1e-12, prof.hemv_ms * 1e-3) / 1e9
    phases = phase_dict(prof, args.steps)
    traffic = measured_traffic(args.workload)
    out = {
        "metric": "GEVD+density s/solve & TFLOP/s, N=6656 real, 2N=9984 cplx; mixed vs FP64",
        "value": ms / 1e3,
        "unit": "s/solve",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": args.workload + ": " + WORKLOADS[args.workload], "form": "fp64",
                   "order": p.order, "batch": p.batch, "electrons": p.n_electrons, "kT": p.kT,
                   "eigenvectors": p.order, "occupied_window": m_occ, "graph": bool(args.graph)},
        "tflops": flops / (ms * 1e-3) / 1e12,
        "tflops_frac_fp64_peak": flops / (ms * 1e-3) / 1e12 / PEAK_FP64_TFLOPS,
        "nominal_flops": flops,
        "warm_s_per_solve": ms_warm / 1e3,
        "wall_s_timed": wall,
        "phases_ms": phases,
        "tuning": {"tiles_per_workgroup": plan.tuning()["tiles_per_workgroup"],
                   "candidates_ms": {str(k): v for k, v in plan.tuning()["candidates"].items()},
                   "segments": plan.tuning()["segments"]},
        "roofline": {"bound": "hbm", "kernel": "symv_kernel (trailing Hermitian matrix-vector "
                                               "product of the tridiagonalisation)",
                     "achieved": hemv_gbs, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": hemv_gbs / PEAK_HBM_GBS,
                     "traffic": traffic["bytes"] if traffic else None,
                     "traffic_over_algorithmic": traffic["over_algorithmic"] if traffic else None,
                     "traffic_source": traffic["source"] if traffic else None,
                     "avg_launch_us": hemv_avg_us, "sampled_launches": int(prof.hemv_launches),
                     "bytes_per_launch_avg": prof.hemv_bytes / max(1, prof.hemv_launches)},
        "checks": {"trace_rho_S_minus_Ne": tr - p.n_electrons, "mu": float(mu.item()),
                   "eband": float(eband.item()),
                   "trace_edm_S_minus_eband": edm_tr - float(eband.item())},
        "energy_density": {"ms": ms_edm, "columns": m_occ,
                           "tflops": edm_flops / (ms_edm * 1e-3) / 1e12},
    }
    if p.batch > 1:
        out["ms_per_kpoint"] = ms / p.batch
    if args.workload == "kpoints16x1300":
        out["bloch_sum"] = bloch_sum_timing(plan, p, stream, args.steps)
    if not args.no_lowdin:
        out["lowdin_route"] = lowdin_timing(p, H, S, eps, rho, stream, args.steps)
    if not args.no_mixed:
        out["precision_comparison"] = compare_precisions(p, H, S, eps, mu, args.steps)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(p, args.cpu_sample)
    print(json.dumps(out), flush=True)


def phase_dict(prof, steps):
    names = ["cholesky", "reduce", "tridiag", "dc", "backtransform", "density", "adjoint", "refine"]
    return {nm: prof.phase_ms[i] / steps for i, nm in enumerate(names)}


def bloch_sum_timing(plan, p, stream, steps):
    """ks_bloch_sum of H(k) and S(k) for every k-point from the workload's 27
    real-space blocks (outside the timed solve steps).  GB/s counts the
    algorithmic bytes: the lower triangles of the real blocks read once, the
    complex k-point matrices written once."""
    import torch
    from paper_2606_09058_amd import inputs as I
    rs = I.kpoint_realspace()
    n, nk, nR = p.n, p.batch, rs["R"].shape[0]
    R = torch.from_numpy(rs["R"]).cuda()
    kv = torch.from_numpy(rs["k"]).cuda()
    HR = torch.from_numpy(rs["HR"]).cuda()
    SR = torch.from_numpy(rs["SR"]).cuda()
    Hk = torch.empty((nk, n, n), dtype=torch.complex128, device="cuda")
    Sk = torch.empty_like(Hk)
    torch.cuda.synchronize()
    with torch.cuda.stream(stream):
        plan.bloch_sum(R, kv, HR, Hk)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        plan.bloch_sum(R, kv, HR, Hk)
        plan.bloch_sum(R, kv, SR, Sk)
    e1.record(stream)
    torch.cuda.synchronize()
    plan.check("bloch sum")
    ms = e0.elapsed_time(e1) / (2 * steps)
    nbytes = nR * n * (n + 1) // 2 * 8 + nk * n * n * 16
    dH = float((Hk - torch.from_numpy(p.H).cuda()).abs().max().item())
    return {"ms_per_matrix_set": ms, "lattice_vectors": nR, "kpoints": nk, "GB_per_s": nbytes / (ms * 1e-3) / 1e9,
            "max_abs_diff_vs_generator_H": dH}


def lowdin_timing(p, H, S, eps_ref, rho_ref, stream, steps):
    """The paper's own route (KS_PLAN_LOWDIN: eigen-decomposition of S, V = U s^-1/2,
    H' = V^H H V, C = V C') on the same input, all eigenvectors, outside the
    timed steps: first-cycle solves (S decomposed) and later-cycle solves (V
    reused), with the phase times and the differences from the Cholesky route."""
    import numpy as np
    import torch
    from paper_2606_09058_amd import ks
    plan = ks.Plan(p.n, batch=p.batch, complex=np.iscomplexobj(p.H), noncollinear=p.nsp == 2, stream=stream,
                   flags=ks.KS_PLAN_AUTOTUNE | ks.KS_PLAN_LOWDIN)
    eps = torch.empty_like(eps_ref)
    C = torch.empty_like(rho_ref)
    rho = torch.empty_like(rho_ref)
    mu = torch.empty(1, dtype=torch.float64, device="cuda")
    eband = torch.empty(1, dtype=torch.float64, device="cuda")

    def step(reuse):
        plan.gevd(H, S, eps, C, reuse_s=reuse)
        plan.density(eps, C, p.n_electrons, p.kT, rho, mu, eband, kweights=p.weights)

    with torch.cuda.stream(stream):
        step(False)
    torch.cuda.synchronize()
    plan.check("lowdin warm-up")
    res = {}
    for name, reuse in (("first_cycle", False), ("later_cycles", True)):
        plan.get_profile()
        plan.set_profiling(True, 1 << 30)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(steps):
            step(reuse)
        e1.record(stream)
        torch.cuda.synchronize()
        prof = plan.get_profile()
        plan.set_profiling(False)
        plan.check("lowdin " + name)
        ph = phase_dict(prof, steps)
        ph["overlap_eig_and_V"] = ph.pop("cholesky")
        res[name] = {"s_per_solve": e0.elapsed_time(e1) / steps / 1e3,
                     "phases_ms": {k: v for k, v in ph.items() if v > 0}}
    res["max_abs_eps_diff_vs_cholesky"] = float((eps - eps_ref).abs().max().item())
    res["max_abs_rho_diff_vs_cholesky"] = float((rho - rho_ref).abs().max().item())
    return res


def compare_precisions(p, H, S, eps_all, mu, steps, buffer_ha=0.4):
    """FP64 and mixed forms on the same window [1, iu]: every state below
    mu + 0.4 Ha (40 kT above the Fermi level, so the refined subspace is
    separated from the rest).  Both solve the window only (eigenvectors
    1..iu) and build the density from it; the mixed eigenvalues and density
    are compared with the FP64 ones of the same GPU."""
    import torch
    from paper_2606_09058_amd import ks
    cplx = torch.is_complex(H)
    iu = int((eps_all < float(mu.item()) + buffer_ha).sum(dim=-1).max().item())
    res = {"window": [1, iu], "buffer_ha": buffer_ha}
    outs = {}
    for form, prec, sweeps in (("fp64", ks.KS_FP64, None), ("mixed", ks.KS_MIXED, 2),
                               ("mixed1", ks.KS_MIXED, 1)):
        plan = ks.Plan(p.n, batch=p.batch, complex=cplx, noncollinear=p.nsp == 2, precision=prec,
                       flags=ks.KS_PLAN_AUTOTUNE)
        if sweeps is not None:
            plan.set_refinement(sweeps)
        eps = torch.empty(plan._vshape(), dtype=torch.float64, device="cuda")
        C = torch.zeros(plan._mshape(), dtype=plan.mdtype, device="cuda")
        rho = torch.empty_like(C)
        m = torch.empty(1, dtype=torch.float64, device="cuda")
        eb = torch.empty(1, dtype=torch.float64, device="cuda")

        def step():
            plan.gevd(H, S, eps, C, il=1, iu=iu)
            plan.density(eps, C, p.n_electrons, p.kT, rho, m, eb, il=1, iu=iu, kweights=p.weights)
        step()
        plan.check(form + " window warm-up")
        plan.get_profile()
        plan.set_profiling(True, 1 << 30)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            step()
        e1.record()
        torch.cuda.synchronize()
        prof = plan.get_profile()
        plan.set_profiling(False)
        plan.check(form + " window steps")
        res[form + "_s_per_solve"] = e0.elapsed_time(e1) / steps / 1e3
        res[form + "_phases_ms"] = phase_dict(prof, steps)
        outs[form] = (eps.clone(), rho.clone(), float(eb.item()))
        del plan
    ef, rf, bf = outs["fp64"]
    res["mixed_sweeps"] = {"mixed": 2, "mixed1": 1}
    for form in ("mixed", "mixed1"):
        em, rm, bm = outs[form]
        res["speedup_%s_vs_fp64" % form] = res["fp64_s_per_solve"] / res[form + "_s_per_solve"]
        res[form + "_max_eig_err_window_vs_fp64"] = float((em[..., :iu] - ef[..., :iu]).abs().max().item())
        res[form + "_max_eig_err_outside_vs_fp64"] = float((em[..., iu:] - ef[..., iu:]).abs().max().item()) \
            if iu < p.order else 0.0
        res[form + "_max_rho_err_vs_fp64"] = float((rm - rf).abs().max().item())
        res[form + "_eband_err_vs_fp64"] = abs(bm - bf)
    return res


if __name__ == "__main__":
    main()
