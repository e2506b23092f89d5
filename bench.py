#!/usr/bin/env python3
"""Benchmark of the generalized Kohn-Sham eigensolve + density build on one MI355X.

One step = ks_gevd (Cholesky of S, reduction, tridiagonalisation, divide and
conquer, back-transform; all eigenvectors) + ks_density (Fermi level by
bisection, occupations, band energy, density matrix) for one matrix (or one
batch of k-points), with inputs already resident in HBM.  Prints ONE JSON line.

    python bench.py [--steps K] [--warmup W] [--workload supercell6656] [--route twostage]

`value` is the main workload's seconds per solve on the chosen tridiagonalisation
route; the line also carries the other route, and (unless --no-configs) the
other two sizes of the metric: the 2N = 9984 spinor problem and the 16 x 1300
k-point batch (both routes, FP64 vs mixed on the occupied window, graph vs
eager launches for the batch), at reduced step counts stated in the line.
A complex workload whose overlap is real (the spinor workload, at the Gamma
point) is solved with KS_PLAN_REAL_OVERLAP (the factor of S in real
arithmetic); the line also times the complex-factor route on it.

With --counter-workload it instead runs the short fixed workload that the
memory-traffic counters are taken on (one rocprofv3 --pmc run per counter):
a plain 1 GiB device fill and copy, whose counter readings give each
counter's scale, then one FP64 ks_gevd (all eigenvectors) of --workload.
"""
import argparse
import hashlib
import json
import math
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
                      "400 electrons, kT=0.01 Ha, one common Fermi level, the whole batch per call",
}
# tridiagonalisation routes: one-stage Householder, or dense -> band -> tridiagonal
ROUTE_FLAGS = {"onestage": 0, "twostage": 8}
# complex workloads whose overlap is real (the spinor workloads at the Gamma
# point) are solved with KS_PLAN_REAL_OVERLAP unless --complex-overlap; the
# line also times the complex-factor route for comparison
REAL_OVERLAP = {"use": True}


def overlap_flags(p):
    """KS_PLAN_REAL_OVERLAP (16) for a complex problem with a real S."""
    import numpy as np
    real_s = np.iscomplexobj(p.H) and not np.any(np.imag(p.S))
    return 16 if (real_s and REAL_OVERLAP["use"]) else 0
DEFAULT_ROUTE = "onestage"


def nominal_flops(order, ncols, m_occ, cplx, n_s):
    """LAPACK-style nominal counts of the steps performed (real; complex x4):
    Cholesky n^3/3 (n = order of S), reduction order^3, tridiagonalisation
    4 order^3/3, back-transform 2 order^2 ncols + triangular solve order^2 ncols,
    density order^2 m_occ.  The same count for both routes (the two-stage
    route performs more flops than it is credited with)."""
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


def host_cpu():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def progress(msg):
    """One line per finished part of the run, on stderr (the JSON line stays alone on stdout)."""
    print("[bench] " + msg, file=sys.stderr, flush=True)


def cpu_baseline(p, sizes):
    """The oracle as it stands (Cholesky + cyclic Jacobi + back-substitution +
    Fermi bisection + density) timed on leading principal blocks of the same
    workload (electron count scaled) at several sizes; the time is extrapolated
    to the full order with the exponent fitted to those sizes (cyclic Jacobi
    needs more sweeps as the order grows, so the exponent exceeds 3).  The line
    also quotes the stored full-size oracle run of the same workload, if the
    fixture records one."""
    import numpy as np
    from oracle import oracle as O
    pts = []
    for ns in sizes:
        ns = min(ns, p.n)
        H = np.ascontiguousarray(p.H[:ns, :ns])
        S = np.ascontiguousarray(p.S[:ns, :ns])
        t0 = time.perf_counter()
        O.solve(H, S, p.n_electrons * ns / p.n, p.kT, nsp=1)
        pts.append((ns, time.perf_counter() - t0))
    x = np.log([a for a, _ in pts])
    y = np.log([b for _, b in pts])
    slope, icpt = np.polyfit(x, y, 1)
    est = math.exp(icpt + slope * math.log(p.order))
    out = {"value": est, "unit": "s/solve", "cores": O.max_threads(), "kind": "oracle",
           "host_cpu": host_cpu(),
           "sample": "oracle on leading principal blocks of the same workload: " +
                     ", ".join("%d: %.2f s" % (a, b) for a, b in pts) +
                     "; time ~ order^%.2f fitted, extrapolated to order %d" % (slope, p.order),
           "fitted_exponent": slope}
    gpath = os.path.join(ROOT, "tests", "golden", p.name + ".json")
    if os.path.exists(gpath):
        g = json.load(open(gpath))
        if g.get("gevd_seconds"):
            out["full_size_oracle_run"] = {
                "gevd_seconds": float(sum(g["gevd_seconds"])), "threads": g.get("oracle_threads"),
                "host_cpu": g.get("host_cpu", "not recorded (the fixture predates the field)"),
                "source": os.path.relpath(gpath, ROOT)}
    return out


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
    plan = ks.Plan(p.n, batch=p.batch, complex=np.iscomplexobj(p.H), noncollinear=p.nsp == 2,
                   flags=overlap_flags(p))
    H = torch.from_numpy(p.H).cuda()
    S = torch.from_numpy(p.S.astype(p.H.dtype)).cuda()
    eps = torch.empty(plan._vshape(), dtype=torch.float64, device="cuda")
    C = torch.empty(plan._mshape(), dtype=plan.mdtype, device="cuda")
    plan.gevd(H, S, eps, C)
    plan.check("counter workload")
    print("solved", p.name, "order", p.order, flush=True)


def phase_dict(prof, steps):
    names = ["cholesky", "reduce", "tridiag", "dc", "backtransform", "density", "adjoint", "refine"]
    return {nm: prof.phase_ms[i] / steps for i, nm in enumerate(names)}


def time_route(p, H, S, route, steps, warmup, stride, stream, graph=False, warm=True, tag="", overlap=None):
    """W warm-up and K timed solves (gevd, all eigenvectors, + density) on one
    plan of the given route; events on the plan's stream.  Returns the timings,
    the sampled symmetric-product launches (one-stage route), the phase times
    and the last solve's outputs."""
    import numpy as np
    import torch
    from paper_2606_09058_amd import ks
    flags = ks.KS_PLAN_AUTOTUNE | ROUTE_FLAGS[route] | (ks.KS_PLAN_GRAPH if graph else 0)
    flags |= overlap_flags(p) if overlap is None else overlap
    with torch.cuda.stream(stream):
        plan = ks.Plan(p.n, batch=p.batch, complex=np.iscomplexobj(p.H), noncollinear=p.nsp == 2, stream=stream,
                       flags=flags)
        eps = torch.empty(plan._vshape(), dtype=torch.float64, device="cuda")
        C = torch.empty(plan._mshape(), dtype=plan.mdtype, device="cuda")
        rho = torch.empty_like(C)
        mu = torch.empty(1, dtype=torch.float64, device="cuda")
        eband = torch.empty(1, dtype=torch.float64, device="cuda")
        occ = torch.empty(plan._vshape(), dtype=torch.float64, device="cuda")

    def step(reuse=False):
        plan.gevd(H, S, eps, C, reuse_s=reuse)
        plan.density(eps, C, p.n_electrons, p.kT, rho, mu, eband, occ=occ, kweights=p.weights)

    for _ in range(warmup):
        step()
    plan.check(tag + route + " warm-up")
    plan.get_profile()  # clear
    plan.set_profiling(True, stride)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(steps):
        step()
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1) / steps
    prof = plan.get_profile()
    plan.set_profiling(False)
    plan.check(tag + route + " timed steps")
    ms_warm = None
    if warm:
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(steps):
            step(reuse=True)
        e1.record(stream)
        torch.cuda.synchronize()
        ms_warm = e0.elapsed_time(e1) / steps
        plan.check(tag + route + " warm steps")
    return dict(plan=plan, eps=eps, C=C, rho=rho, mu=mu, eband=eband, occ=occ, ms=ms, ms_warm=ms_warm,
                prof=prof, wall=wall, phases=phase_dict(prof, steps))


def symv_roofline(prof, traffic):
    hemv_avg_us = 1e3 * prof.hemv_ms / max(1, prof.hemv_launches)
    hemv_gbs = prof.hemv_bytes / max(1e-12, prof.hemv_ms * 1e-3) / 1e9
    return {"bound": "hbm", "kernel": "symv_kernel (trailing Hermitian matrix-vector product of the "
                                      "one-stage tridiagonalisation)",
            "achieved": hemv_gbs, "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": hemv_gbs / PEAK_HBM_GBS,
            "traffic": traffic["bytes"] if traffic else None,
            "traffic_over_algorithmic": traffic["over_algorithmic"] if traffic else None,
            "traffic_source": traffic["source"] if traffic else None,
            "avg_launch_us": hemv_avg_us, "sampled_launches": int(prof.hemv_launches),
            "bytes_per_launch_avg": prof.hemv_bytes / max(1, prof.hemv_launches)}


def occupied_count(occ, p):
    return int((occ > 2e-15 * p.g).sum(dim=-1).max().item())


def trace_check(p, rho, S):
    import torch
    SN = torch.block_diag(S, S) if p.nsp == 2 else S
    if p.batch == 1:
        return float((rho * SN.to(rho.dtype).T).sum().real.item())
    w = torch.tensor(p.weights, dtype=torch.float64, device="cuda")
    return float((w * (rho * S.to(rho.dtype).transpose(1, 2)).sum(dim=(1, 2)).real).sum().item())


def route_summary(r, ref, p, flops):
    out = {"s_per_solve": r["ms"] / 1e3, "tflops": flops / (r["ms"] * 1e-3) / 1e12,
           "phases_ms": {k: v for k, v in r["phases"].items() if v > 0}}
    if r["ms_warm"] is not None:
        out["warm_s_per_solve"] = r["ms_warm"] / 1e3
    if ref is not None:
        out["max_abs_eps_diff_vs_main"] = float((r["eps"] - ref["eps"]).abs().max().item())
        out["max_abs_rho_diff_vs_main"] = float((r["rho"] - ref["rho"]).abs().max().item())
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="supercell6656", choices=sorted(WORKLOADS))
    ap.add_argument("--route", default=DEFAULT_ROUTE, choices=sorted(ROUTE_FLAGS),
                    help="tridiagonalisation route of the main measurement")
    ap.add_argument("--stride", type=int, default=16, help="sample every n-th matrix-vector launch")
    ap.add_argument("--cpu-sizes", default="850,1200,1700",
                    help="orders of the oracle samples behind cpu_baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true",
                    help="skip the FP64-vs-mixed comparison on the occupied window")
    ap.add_argument("--no-lowdin", action="store_true", help="skip the Loewdin-route comparison")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the other sizes of the metric (2N = 9984 spinor, 16 x 1300 k-points)")
    ap.add_argument("--graph", action="store_true", help="plan with KS_PLAN_GRAPH (capture once, replay)")
    ap.add_argument("--complex-overlap", action="store_true",
                    help="factor a real overlap of a complex problem in complex arithmetic too")
    ap.add_argument("--counter-workload", action="store_true",
                    help="run the fixed workload of the rocprofv3 memory-counter runs and exit")
    args = ap.parse_args()
    REAL_OVERLAP["use"] = not args.complex_overlap
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
    H = torch.from_numpy(p.H).cuda()
    S = torch.from_numpy(p.S.astype(p.H.dtype)).cuda()
    r = time_route(p, H, S, args.route, args.steps, args.warmup, args.stride, stream, graph=args.graph)
    plan, eps, C, rho, mu, eband, occ = (r[k] for k in ("plan", "eps", "C", "rho", "mu", "eband", "occ"))
    ms = r["ms"]
    tr = trace_check(p, rho, S)
    m_occ = occupied_count(occ, p)
    flops = p.batch * nominal_flops(p.order, p.order, m_occ, cplx, p.n)

    # energy-density matrix E = C diag(f eps) C^H of the last solve, over the
    # columns that carry occupation (outside the timed steps: not part of `value`)
    edm = torch.empty_like(rho)
    with torch.cuda.stream(stream):
        plan.energy_density(eps, C, occ, edm, il=1, iu=max(1, m_occ))
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(args.steps):
        plan.energy_density(eps, C, occ, edm, il=1, iu=max(1, m_occ))
    e1.record(stream)
    torch.cuda.synchronize()
    plan.check("energy density")
    ms_edm = e0.elapsed_time(e1) / args.steps
    edm_tr = trace_check(p, edm, S)
    edm_flops = p.batch * (4.0 if cplx else 1.0) * p.order * p.order * m_occ
    tu = plan.tuning()
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
                   "route": args.route, "order": p.order, "batch": p.batch, "electrons": p.n_electrons,
                   "kT": p.kT, "eigenvectors": p.order, "occupied_window": m_occ, "graph": bool(args.graph),
                   "overlap": "real" if overlap_flags(p) else "as given"},
        "tflops": flops / (ms * 1e-3) / 1e12,
        "tflops_frac_fp64_peak": flops / (ms * 1e-3) / 1e12 / PEAK_FP64_TFLOPS,
        "nominal_flops": flops,
        "warm_s_per_solve": r["ms_warm"] / 1e3,
        "wall_s_timed": r["wall"],
        "phases_ms": r["phases"],
        "tuning": {"tiles_per_workgroup": tu["tiles_per_workgroup"],
                   "candidates_ms": {str(k): v for k, v in tu["candidates"].items()},
                   "segments": tu["segments"],
                   "backtr_block": tu["backtr_block"],
                   "gemm_big_min_k": ("never" if tu["gemm_big_min_k"] == ks.KS_TUNE_NEVER
                                      else tu["gemm_big_min_k"]),
                   "backtr_ms": {"bt%d_%s" % (b, "never" if g == ks.KS_TUNE_NEVER else "k%d" % g): v
                                 for (b, g), v in tu["backtr_ms"].items()},
                   "dc_leaf": tu["dc_leaf"],
                   "dc_ms": {str(k): v for k, v in tu["dc_ms"].items()}},
        "checks": {"trace_rho_S_minus_Ne": tr - p.n_electrons, "mu": float(mu.item()),
                   "eband": float(eband.item()), "trace_edm_S_minus_eband": edm_tr - float(eband.item())},
        "energy_density": {"ms": ms_edm, "columns": m_occ, "tflops": edm_flops / (ms_edm * 1e-3) / 1e12},
    }
    # the other tridiagonalisation route on the same input (fewer steps)
    other = "twostage" if args.route == "onestage" else "onestage"
    progress("%s route timed (%.3f s/solve); %s route" % (args.route, ms / 1e3, other))
    r2 = time_route(p, H, S, other, max(2, args.steps // 4), 1, args.stride, stream, warm=False)
    out["routes"] = {args.route: route_summary(r, None, p, flops), other: route_summary(r2, r, p, flops)}
    out["routes"][other]["steps"] = max(2, args.steps // 4)
    if overlap_flags(p):
        progress("complex-factor route")
        r3 = time_route(p, H, S, "onestage", max(2, args.steps // 4), 1, args.stride, stream, warm=False,
                        overlap=0)
        out["routes"]["onestage_complex_factor"] = route_summary(r3, r, p, flops)
        out["routes"]["onestage_complex_factor"]["steps"] = max(2, args.steps // 4)
        del r3
    sy = r if args.route == "onestage" else r2
    out["roofline"] = symv_roofline(sy["prof"], measured_traffic(args.workload))
    out["roofline"]["route"] = "onestage"
    del r2
    if p.batch > 1:
        out["ms_per_kpoint"] = ms / p.batch
    if args.workload == "kpoints16x1300":
        out["bloch_sum"] = bloch_sum_timing(plan, p, stream, args.steps)
    if not args.no_lowdin:
        progress("Loewdin route")
        out["lowdin_route"] = lowdin_timing(p, H, S, eps, rho, stream, args.steps)
    if not args.no_mixed:
        progress("FP64 vs mixed on the occupied window")
        out["precision_comparison"] = compare_precisions(p, H, S, eps, mu, args.steps)
    if not args.no_cpu_baseline:
        progress("oracle on the host")
        out["cpu_baseline"] = cpu_baseline(p, [int(x) for x in args.cpu_sizes.split(",")])
    del plan, r, H, S, C, rho, edm
    torch.cuda.empty_cache()
    if not args.no_configs:
        out["configs"] = {}
        for name in ("supercell6656", "noncollinear9984", "kpoints16x1300"):
            if name != args.workload:
                progress("workload " + name)
                out["configs"][name] = other_config(name, stream, args.stride)
                torch.cuda.empty_cache()
    print(json.dumps(out), flush=True)


def other_config(name, stream, stride, steps=3):
    """Another size of the metric at reduced steps: both routes (all
    eigenvectors), the one-stage symmetric product's roofline, FP64 vs mixed on
    the occupied window, and for a k-point batch graph-replayed vs eager launches."""
    import numpy as np
    import torch
    from paper_2606_09058_amd import inputs as I
    p = I.workload(name)
    cplx = np.iscomplexobj(p.H)
    H = torch.from_numpy(p.H).cuda()
    S = torch.from_numpy(p.S.astype(p.H.dtype)).cuda()
    res = {"workload": name + ": " + WORKLOADS[name], "steps": steps, "warmup": 1, "order": p.order,
           "batch": p.batch}
    runs = {}
    for route in ("onestage", "twostage"):
        runs[route] = time_route(p, H, S, route, steps, 1, stride, stream, warm=route == "onestage", tag=name + " ")
    if overlap_flags(p):
        runs["onestage_complex_factor"] = time_route(p, H, S, "onestage", 2, 1, stride, stream, warm=False,
                                                     tag=name + " complex factor ", overlap=0)
        res["overlap"] = "real"
    ref = runs["onestage"]
    m_occ = occupied_count(ref["occ"], p)
    flops = p.batch * nominal_flops(p.order, p.order, m_occ, cplx, p.n)
    res["nominal_flops"] = flops
    res["occupied_window"] = m_occ
    res["routes"] = {rt: route_summary(runs[rt], None if rt == "onestage" else ref, p, flops) for rt in runs}
    res["trace_rho_S_minus_Ne"] = trace_check(p, ref["rho"], S) - p.n_electrons
    res["roofline"] = symv_roofline(ref["prof"], measured_traffic(name))
    if p.batch > 1:
        res["ms_per_kpoint"] = {rt: runs[rt]["ms"] / p.batch for rt in runs}
    mu = ref["mu"]
    eps = ref["eps"]
    del runs, ref
    torch.cuda.empty_cache()
    if p.batch > 1:
        # graph capture needs a stream of its own
        torch.cuda.synchronize()
        g = time_route(p, H, S, "onestage", steps, 1, stride, torch.cuda.Stream(), graph=True, warm=False,
                       tag=name + " graph ")
        res["graph_s_per_batch"] = g["ms"] / 1e3
        res["graph_ms_per_kpoint"] = g["ms"] / p.batch
        res["graph_replays"] = g["plan"].graph_stats()[1]
        del g
    res["precision_comparison"] = compare_precisions(p, H, S, eps, mu, 2)
    return res


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
    res = {"window": [1, iu], "buffer_ha": buffer_ha, "steps": steps}
    outs = {}
    for form, prec, sweeps, flags in (("fp64", ks.KS_FP64, None, 0), ("fp64_twostage", ks.KS_FP64, None, 8),
                                      ("mixed", ks.KS_MIXED, 2, 0), ("mixed1", ks.KS_MIXED, 1, 0)):
        plan = ks.Plan(p.n, batch=p.batch, complex=cplx, noncollinear=p.nsp == 2, precision=prec,
                       flags=ks.KS_PLAN_AUTOTUNE | flags | overlap_flags(p))
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
        res[form + "_phases_ms"] = {k: v for k, v in phase_dict(prof, steps).items() if v > 0}
        # host copies after the device has drained: the next form's plan and
        # tensors reuse this memory
        torch.cuda.synchronize()
        outs[form] = (eps.cpu(), rho.cpu(), float(eb.cpu().item()))
        del plan, C, rho
        torch.cuda.empty_cache()
    ef, rf, bf = outs["fp64"]
    res["mixed_sweeps"] = {"mixed": 2, "mixed1": 1}
    best = min(res["fp64_s_per_solve"], res["fp64_twostage_s_per_solve"])
    res["fastest_fp64_s_per_solve"] = best
    for form in ("fp64_twostage", "mixed", "mixed1"):
        em, rm, bm = outs[form]
        if form != "fp64_twostage":
            res["speedup_%s_vs_fp64" % form] = res["fp64_s_per_solve"] / res[form + "_s_per_solve"]
            res["speedup_%s_vs_fastest_fp64" % form] = best / res[form + "_s_per_solve"]
        res[form + "_max_eig_err_window_vs_fp64"] = float((em[..., :iu] - ef[..., :iu]).abs().max().item())
        if form != "fp64_twostage":
            res[form + "_max_eig_err_outside_vs_fp64"] = float((em[..., iu:] - ef[..., iu:]).abs().max().item()) \
                if iu < p.order else 0.0
        res[form + "_max_rho_err_vs_fp64"] = float((rm - rf).abs().max().item())
        res[form + "_eband_err_vs_fp64"] = abs(bm - bf)
    return res


if __name__ == "__main__":
    main()
