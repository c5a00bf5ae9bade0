"""Run-to-run repeatability of the HIP path on the same inputs.

What is fixed by construction and checked bitwise: each packet's own history
(its Philox stream and arithmetic), the integer tallies, the NLTE roots (one
wavefront per system, no cross-system reduction), the batched solve and the
fused warm-start inference. What is summed with FP64 atomics in an order the
hardware picks (the estimator table, the directly summed rates, the weight
tallies) must agree to the rounding of a reordered sum.
"""
import sys

import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu

COUNTS = ("n_inter", "n_checks", "n_cross", "n_escaped", "n_killed")


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def ex():
    import paper_2511_07539_amd as ex
    return ex


@pytest.fixture(scope="module")
def ctx(ex):
    return ex.Context(0)


@pytest.fixture(scope="module")
def coupled(ex, ctx):
    w = synth.clumpy(n=16, n_lines=1500, n_packets=300_000, number=2)
    atom = ex.Atom(ctx, w.atom)
    cold, _, _ = ex.nlte_solve(ctx, atom, ex.cells_from_workload(w), max_iter=0)
    tau, fc = ex.line_tau(ctx, atom, cold, w.t_exp)
    return w, atom, cold, ex.grid_from_workload(w, tau_ct=tau, fcorr_ct=fc)


def _reordered_sum(a, b, name, rtol=1e-12):
    a, b = a.cpu().numpy(), b.cpu().numpy()
    nz = b != 0
    assert np.array_equal(a != 0, nz), f"{name}: different nonzero pattern"
    r = float(np.max(np.abs(a[nz] - b[nz]) / np.abs(b[nz]))) if nz.any() else 0.0
    say(f"{name}: max rel {r:.2e} over {int(nz.sum())} entries")
    assert r <= rtol, name


@pytest.mark.parametrize("fp32", [False, True])
def test_transport_repeats(ex, ctx, coupled, fp32):
    w, _, _, grid = coupled
    say(f"case: transport twice, clumpy 16^3, 3e5 packets, fp32={fp32}")
    runs = [ex.transport(ctx, grid, w.seed, w.lambda_lo, w.lambda_hi, w.n_packets,
                         geometry_fp32=fp32, packets_out=True) for _ in range(2)]
    torch.cuda.synchronize()
    (e1, s1, p1), (e2, s2, p2) = runs
    assert torch.equal(p1, p2)  # every packet's own record, bitwise
    d1, d2 = ex.stats_dict(s1), ex.stats_dict(s2)
    for k in COUNTS:
        assert d1[k] == d2[k], k
    for k in ("w_emit", "w_esc", "w_kill", "w_abs"):
        assert d1[k] == pytest.approx(d2[k], rel=1e-13), k
    _reordered_sum(e1, e2, "estimators")


def test_streamed_rates_repeat(ex, ctx, coupled):
    w, atom, cold, grid = coupled
    say("case: streamed transport with rates summed per interaction, twice")
    out = []
    for _ in range(2):
        g, st, _ = ex.transport_streamed(ctx, grid, w.seed, w.lambda_lo, w.lambda_hi, w.n_packets,
                                         atom=atom, pops=cold, t_exp=w.t_exp, geometry_fp32=True,
                                         octant_table=False)
        out.append((g.clone(), ex.stats_dict(st)))
    torch.cuda.synchronize()
    for k in COUNTS:
        assert out[0][1][k] == out[1][1][k], k
    _reordered_sum(out[0][0], out[1][0], "rates")


@pytest.mark.parametrize("mixed", [False, True])
def test_nlte_repeats_bitwise(ex, ctx, coupled, mixed):
    w, atom, cold, grid = coupled
    say(f"case: NLTE solve twice on the rates of one transport, FP32 fixed-point steps {mixed}")
    est, _, _ = ex.transport(ctx, grid, w.seed, w.lambda_lo, w.lambda_hi, w.n_packets,
                             geometry_fp32=True)
    gam = ex.rates(ctx, atom, grid, w.t_exp, est, cold)
    cells = ex.cells_from_workload(w, gamma_pe=gam)
    a = ex.nlte_solve(ctx, atom, cells, tol=1e-8, factor_fp32=mixed)
    b = ex.nlte_solve(ctx, atom, cells, tol=1e-8, factor_fp32=mixed)
    c = ex.nlte_solve(ctx, atom, cells, tol=1e-8, guess=a[0], factor_fp32=mixed)
    d = ex.nlte_solve(ctx, atom, cells, tol=1e-8, guess=a[0], factor_fp32=mixed)
    torch.cuda.synchronize()
    for x, y in ((a, b), (c, d)):
        assert torch.equal(x[0], y[0]) and torch.equal(x[1], y[1]) and torch.equal(x[2], y[2])
    assert int((a[1] <= 1).sum()) >= 0.999 * w.n_cells


def test_batched_repeats_bitwise(ex, ctx):
    b = synth.batched_custom([[20, 30, 25], [60, 5, 1], [120, 80, 40], [7, 7, 7]],
                             T_e=[4000.0, 6000.0, 8000.0, 3000.0], n_e=[1e7, 1e6, 1e8, 1e5],
                             gamma_ion=1e-5)
    say("case: batched FP64 solve twice, 4 ragged cells")
    prob = ex.Batched(b)
    p1, s1 = ex.batched_solve(ctx, prob)
    p2, s2 = ex.batched_solve(ctx, prob)
    torch.cuda.synchronize()
    assert torch.equal(p1, p2) and torch.equal(s1, s2)


def test_warm_start_repeats_bitwise(ex, ctx, coupled):
    from paper_2511_07539_amd import warmstart
    w, atom, _, _ = coupled
    say("case: fused warm-start inference twice (untrained network)")
    params = torch.as_tensor(warmstart.init_params(3), device="cuda:0")
    cells = ex.cells_from_workload(w)
    x = ex.mlp_features(ctx, atom, cells, w.deposition).cpu().numpy().astype(np.float64)
    norm = torch.as_tensor(np.r_[x.mean(0), x.std(0) + 1e-6, np.full(100, -2.0), np.ones(100)]
                           .astype(np.float32), device="cuda:0")
    a = ex.nlte_warm_start(ctx, atom, cells, w.deposition, params, norm)
    b = ex.nlte_warm_start(ctx, atom, cells, w.deposition, params, norm)
    torch.cuda.synchronize()
    assert torch.isfinite(a).all()
    assert torch.equal(a, b)
