"""Streamed transport over velocity octants (extrass_transport_streamed).

Pin: the invariance itself. With the same packets, splitting the cube into 8
octants visited in turn (packets handed between octants through queues) takes
the same events as the unsplit run, so every estimator entry agrees up to the
order of atomic additions:
- against the GPU's unsplit transport, in FP64 and in FP32 geometry
  (the stored packet state converts back exactly, so FP32 near-ties resolve
  the same way): per entry, relative 1e-12, identical event counts;
- against the FP64 oracle (unsplit, serial per packet): per entry 1e-10 on
  the FP64-geometry path;
- rates accumulated visit by visit equal extrass_rates on the unsplit table.
"""
import sys

import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def ex():
    import paper_2511_07539_amd as ex
    return ex


@pytest.fixture(scope="module")
def ctx(ex):
    return ex.Context(0)


def _coupled(ex, ctx, w):
    atom = ex.Atom(ctx, w.atom)
    cells = ex.cells_from_workload(w)
    cold, _, _ = ex.nlte_solve(ctx, atom, cells, max_iter=0)
    tau, fc = ex.line_tau(ctx, atom, cold, w.t_exp)
    return atom, cold, ex.grid_from_workload(w, tau_ct=tau, fcorr_ct=fc)


def _close(a, b, rtol, name):
    a, b = a.cpu().numpy(), b.cpu().numpy()
    nz = np.abs(b) > 0
    assert np.array_equal(a != 0, nz), f"{name}: different nonzero pattern"
    r = float(np.max(np.abs(a[nz] - b[nz]) / np.abs(b[nz]))) if nz.any() else 0.0
    say(f"{name}: max rel {r:.2e} over {int(nz.sum())} entries")
    assert r <= rtol, name


@pytest.mark.parametrize("fp32", [False, True])
def test_streamed_equals_unsplit_coupled_clumpy(ex, ctx, fp32):
    w = synth.clumpy(n=16, n_lines=1500, n_packets=300_000, number=2)
    say(f"case: streamed vs unsplit, clumpy 16^3, coupled lines, fp32={fp32}")
    atom, cold, grid = _coupled(ex, ctx, w)
    est, st_u, _ = ex.transport(ctx, grid, w.seed, w.lambda_lo, w.lambda_hi, w.n_packets,
                                geometry_fp32=fp32)
    gam_u = ex.rates(ctx, atom, grid, w.t_exp, est, cold)
    gam_s, st_s, eg = ex.transport_streamed(ctx, grid, w.seed, w.lambda_lo, w.lambda_hi,
                                            w.n_packets, atom=atom, pops=cold, t_exp=w.t_exp,
                                            geometry_fp32=fp32, est_global=True)
    torch.cuda.synchronize()
    su, ss = ex.stats_dict(st_u), ex.stats_dict(st_s)
    say("unsplit", {k: su[k] for k in ("n_inter", "n_cross", "n_escaped", "n_killed")})
    say("streamed", {k: ss[k] for k in ("n_inter", "n_cross", "n_escaped", "n_killed")})
    for k in ("n_inter", "n_checks", "n_cross", "n_escaped", "n_killed"):
        assert su[k] == ss[k], k
    for k in ("w_emit", "w_esc", "w_kill", "w_abs"):
        assert ss[k] == pytest.approx(su[k], rel=1e-12), k
    assert ss["error_flag"] == 0 and ss["bad_packets"] == 0
    _close(eg, est, 1e-12, "estimators")
    _close(gam_s, gam_u, 1e-12, "rates")


@pytest.mark.parametrize("fp32", [False, True])
def test_direct_rates_equal_table_rates(ex, ctx, fp32):
    """Without an octant table the rates are summed per interaction: the same
    sums in another order, so equal to the table path's rates to 1e-12."""
    w = synth.clumpy(n=16, n_lines=1500, n_packets=300_000, number=2)
    say(f"case: streamed rates without the octant table, clumpy 16^3, fp32={fp32}")
    atom, cold, grid = _coupled(ex, ctx, w)
    gam_t, st_t, _ = ex.transport_streamed(ctx, grid, w.seed, w.lambda_lo, w.lambda_hi,
                                           w.n_packets, atom=atom, pops=cold, t_exp=w.t_exp,
                                           geometry_fp32=fp32)
    gam_d, st_d, _ = ex.transport_streamed(ctx, grid, w.seed, w.lambda_lo, w.lambda_hi,
                                           w.n_packets, atom=atom, pops=cold, t_exp=w.t_exp,
                                           geometry_fp32=fp32, octant_table=False)
    torch.cuda.synchronize()
    a, b = ex.stats_dict(st_d), ex.stats_dict(st_t)
    for k in ("n_inter", "n_checks", "n_cross", "n_escaped", "n_killed"):
        assert a[k] == b[k], k
    assert a["error_flag"] == 0 and a["bad_packets"] == 0
    _close(gam_d, gam_t, 1e-12, "rates")


def test_direct_rates_need_a_consistent_line_map(ex, ctx):
    w = synth.clumpy(n=16, n_lines=1500, n_packets=10_000, number=2)
    atom, cold, grid = _coupled(ex, ctx, w)
    say("case: direct streamed rates with the grid's line map broken")
    lt = grid.line_trans.clone()
    k = int(torch.nonzero(lt >= 0)[0])
    grid.line_trans[k] = -1  # one atom line no longer maps back to its transition
    with pytest.raises(ex.ExtrassError, match="inverse"):
        ex.transport_streamed(ctx, grid, w.seed, w.lambda_lo, w.lambda_hi, w.n_packets,
                              atom=atom, pops=cold, t_exp=w.t_exp,
                              octant_table=False)
    torch.cuda.synchronize()
    grid.line_trans.copy_(lt)
    with pytest.raises(ex.ExtrassError, match="invalid argument"):
        ex.transport_streamed(ctx, grid, w.seed, w.lambda_lo, w.lambda_hi, w.n_packets,
                              atom=atom, pops=cold, t_exp=w.t_exp,
                              octant_table=False, est_global=True)


def test_streamed_fp64_matches_oracle(ex, ctx):
    w = synth.sphere_small()
    say("case: streamed FP64 vs oracle, sphere 16^3, 200 lines, 1e5 packets")
    grid = ex.grid_from_workload(w)
    _, st, eg = ex.transport_streamed(ctx, grid, w.seed, w.lambda_lo, w.lambda_hi, w.n_packets,
                                      est_global=True)
    torch.cuda.synchronize()
    r = oracle.transport(oracle.transport_inputs_from_workload(w))
    ref = oracle.dense_estimator(r["records"], w.n_cells, w.n_lines).ravel()
    got = eg.cpu().numpy().ravel()
    nz = ref != 0
    assert np.array_equal(got != 0, nz)
    rel = np.max(np.abs(got[nz] - ref[nz]) / np.abs(ref[nz]))
    say(f"max rel vs oracle {rel:.2e}; interactions {r['stats']['n_inter']:.0f}")
    assert rel <= 1e-10
    assert ex.stats_dict(st)["n_inter"] == r["stats"]["n_inter"]


def test_queue_overflow_and_bad_arguments(ex, ctx):
    w = synth.clumpy(n=16, n_lines=1500, n_packets=100_000, number=2)
    grid = ex.grid_from_workload(w)
    say("case: streamed transport with a queue of 1 packet per octant")
    with pytest.raises(ex.ExtrassError, match="workspace too small"):
        ex.transport_streamed(ctx, grid, w.seed, w.lambda_lo, w.lambda_hi, w.n_packets,
                              queue_capacity=1)
    torch.cuda.synchronize()
    with pytest.raises(ex.ExtrassError, match="invalid argument"):
        ex.transport_streamed(ctx, grid, w.seed, w.lambda_lo, w.lambda_hi, w.n_packets - 1)
    odd = synth.clumpy(n=15, n_lines=1500, n_packets=10_000, number=2)
    with pytest.raises(ex.ExtrassError, match="invalid argument"):
        ex.transport_streamed(ctx, ex.grid_from_workload(odd), odd.seed, odd.lambda_lo,
                              odd.lambda_hi, odd.n_packets)


@pytest.mark.parametrize("fp32", [False, True])
def test_streamed_equals_unsplit_paper_scale(ex, ctx, fp32):
    """The bench's 50^3 workload (125 000 cells, 5000 lines, 1e7 packets,
    coupled atom lines): the octant-streamed table equals the unsplit one per
    entry, with identical event counts."""
    w = synth.paper_scale()
    say(f"case: streamed vs unsplit, clumpy 50^3, 5000 lines, 1e7 packets, fp32={fp32}")
    atom, cold, grid = _coupled(ex, ctx, w)
    est, st_u, _ = ex.transport(ctx, grid, w.seed, w.lambda_lo, w.lambda_hi, w.n_packets,
                                geometry_fp32=fp32)
    _, st_s, eg = ex.transport_streamed(ctx, grid, w.seed, w.lambda_lo, w.lambda_hi,
                                        w.n_packets, geometry_fp32=fp32, est_global=True)
    torch.cuda.synchronize()
    a, b = ex.stats_dict(st_s), ex.stats_dict(st_u)
    for k in ("n_inter", "n_checks", "n_cross", "n_escaped", "n_killed"):
        assert a[k] == b[k], k
    assert a["error_flag"] == 0 and a["bad_packets"] == 0
    del cold, atom
    # compared on the device, one block of cells at a time
    worst, mism = 0.0, 0
    for c0 in range(0, w.n_cells, 25_000):
        x, y = eg[c0:c0 + 25_000], est[c0:c0 + 25_000]
        nz = y != 0
        mism += int(((x != 0) != nz).sum())
        if bool(nz.any()):
            worst = max(worst, float(((x[nz] - y[nz]).abs() / y[nz].abs()).max()))
    say(f"support mismatches {mism}, max rel {worst:.2e}")
    assert mism == 0
    assert worst <= 1e-12
