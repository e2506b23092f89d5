"""The widened autotuner: every knob (tiles per workgroup by column segment,
back-transform block, large-GEMM threshold, divide-and-conquer leaf) is timed
at plan creation and reported; each candidate of each knob meets the oracle;
the tuning cache gives a later plan of the same shape the same knobs without
timing, and ks_plan_set_tuning refuses knobs outside their candidates."""
import itertools

import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2606_09058_amd import inputs as I
from paper_2606_09058_amd import ks
from tests.gpu_helpers import announce, dev, host
from tests.test_gpu_parity import compare

pytestmark = pytest.mark.gpu


def problem(cplx, n_atoms=24):
    return I.toy(seed=41, natoms=n_atoms, norb=13, edge=14.0, n_electrons=120.0, kT=0.01, phases=cplx)


def run(plan, p):
    with torch.cuda.stream(plan.stream):
        H = dev(p.H)
        S = dev(p.S.astype(p.H.dtype))
        out = plan.solve(H, S, p.n_electrons, p.kT)
        g = {k: host(v) for k, v in out.items()}
    g["mu"], g["eband"] = float(g["mu"][0]), float(g["eband"][0])
    return g


@pytest.mark.parametrize("cplx", [False, True])
def test_autotune_reports_every_knob(cplx):
    announce("autotune knobs", cplx)
    p = problem(cplx)
    plan = ks.Plan(p.n, complex=cplx, stream=torch.cuda.Stream(), flags=ks.KS_PLAN_AUTOTUNE)
    tu = plan.tuning()
    assert not tu["from_cache"]
    assert tu["backtr_block"] in (128, 256)
    assert tu["gemm_big_min_k"] in (256, ks.KS_TUNE_NEVER)
    assert tu["dc_leaf"] in (16, 32)
    bt = tu["backtr_ms"]
    assert sorted(bt) == [(128, 256), (128, ks.KS_TUNE_NEVER), (256, 256), (256, ks.KS_TUNE_NEVER)]
    assert all(t > 0 for t in bt.values()), bt
    assert bt[(tu["backtr_block"], tu["gemm_big_min_k"])] == min(bt.values())
    assert sorted(tu["dc_ms"]) == [16, 32] and all(t > 0 for t in tu["dc_ms"].values())
    assert tu["dc_ms"][tu["dc_leaf"]] == min(tu["dc_ms"].values())
    compare(p, run(plan, p), O.solve(p.H, p.S, p.n_electrons, p.kT))


@pytest.mark.parametrize("cplx", [False, True])
def test_every_candidate_meets_the_oracle(cplx):
    """Forced knobs: both back-transform blocks, three GEMM thresholds, both
    leaves, a mixed segment list.  (At order 312 the large tiles do not take
    part whatever the threshold, too few tiles; their products are checked on
    their own at order 4100 in the stage tests.)"""
    announce("tuning candidates", cplx)
    p = problem(cplx)
    o = O.solve(p.H, p.S, p.n_electrons, p.kT)
    plan = ks.Plan(p.n, complex=cplx, stream=torch.cuda.Stream())
    base = plan.tuning_knobs()
    assert base["backtr_block"] == 128 and base["dc_leaf"] == 32 and base["gemm_big_min_k"] == 256
    for bt, gk, leaf in itertools.product((128, 256), (16, 256, ks.KS_TUNE_NEVER), (16, 32)):
        knobs = dict(base, backtr_block=bt, gemm_big_min_k=gk, dc_leaf=leaf, nseg=3,
                     seg_first=[0, 50, 200], seg_tiles=[8, 2, 4])
        plan.set_tuning(knobs)
        tu = plan.tuning()
        assert tu["from_cache"] and tu["backtr_block"] == bt and tu["dc_leaf"] == leaf
        compare(p, run(plan, p), o)


def test_tuning_cache_round_trip(tmp_path):
    """A second plan of the same shape takes the first one's knobs from the
    cache (no timing) and gives bit-identical results."""
    announce("tuning cache")
    path = str(tmp_path / "tune.json")
    p = problem(False)
    a = ks.Plan(p.n, stream=torch.cuda.Stream(), flags=ks.KS_PLAN_AUTOTUNE, tune_cache=path)
    ta = a.tuning()
    assert not ta["from_cache"]
    b = ks.Plan(p.n, stream=torch.cuda.Stream(), flags=ks.KS_PLAN_AUTOTUNE, tune_cache=path)
    tb = b.tuning()
    assert tb["from_cache"]
    assert a.tuning_knobs() == b.tuning_knobs()
    assert all(t == 0 for t in tb["candidates"].values()) or not tb["candidates"]
    ga, gb = run(a, p), run(b, p)
    for k in ("eps", "rho", "C"):
        assert np.array_equal(ga[k], gb[k]), k
    # another shape is another key
    c = ks.Plan(p.n, complex=True, stream=torch.cuda.Stream(), flags=ks.KS_PLAN_AUTOTUNE, tune_cache=path)
    assert not c.tuning()["from_cache"]


def test_set_tuning_refusals_leave_the_plan_unchanged():
    announce("set_tuning refusals")
    p = problem(False, n_atoms=8)
    plan = ks.Plan(p.n, stream=torch.cuda.Stream())
    base = plan.tuning_knobs()
    bad = [dict(base, tiles_per_workgroup=3), dict(base, backtr_block=64), dict(base, dc_leaf=8),
           dict(base, gemm_big_min_k=4), dict(base, nseg=2, seg_first=[0, 0], seg_tiles=[2, 2]),
           dict(base, nseg=2, seg_first=[1, 5], seg_tiles=[2, 2]), dict(base, nseg=1, seg_tiles=[5])]
    for knobs in bad:
        with pytest.raises(ks.KSError):
            plan.set_tuning(knobs)
        assert plan.tuning_knobs() == base
    assert not plan.tuning()["from_cache"]


def test_set_tuning_recaptures_the_graph():
    """A graph plan captured with one set of knobs captures again after
    ks_plan_set_tuning; its replays equal an eager plan with the same knobs
    bit for bit, and meet the oracle."""
    announce("set_tuning graph")
    p = problem(True)
    o = O.solve(p.H, p.S, p.n_electrons, p.kT)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        gplan = ks.Plan(p.n, complex=True, stream=stream, flags=ks.KS_PLAN_GRAPH)
        eplan = ks.Plan(p.n, complex=True, stream=stream)
        H = dev(p.H)
        S = dev(p.S.astype(p.H.dtype))
        eps = torch.empty(gplan._vshape(), dtype=torch.float64, device="cuda")
        C = torch.zeros(gplan._mshape(), dtype=torch.complex128, device="cuda")
        for knobs in (None, dict(gplan.tuning_knobs(), dc_leaf=16, backtr_block=256, gemm_big_min_k=16)):
            if knobs is not None:
                gplan.set_tuning(knobs)
                eplan.set_tuning(knobs)
            for rep in range(2):
                gplan.gevd(H, S, eps, C)
                stream.synchronize()
                e2 = torch.empty_like(eps)
                C2 = torch.zeros_like(C)
                eplan.gevd(H, S, e2, C2)
                stream.synchronize()
                assert np.array_equal(host(eps), host(e2))
                assert np.array_equal(host(C), host(C2))
            assert np.abs(host(eps) - o["eps"]).max() < 1e-10
        assert gplan.graph_stats() == (2, 2)
