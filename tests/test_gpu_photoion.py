"""Photoionisation in the transport (Sec. 2.3.1; Eq. A5): HIP path vs the FP64
oracle on the same inputs.

Bars: FP64 geometry - the same photoionising levels; the opacity table equal
to its definition to 1e-14; per entry within 1e-9 on the line estimators and
on the photoionisation rates of every (cell, level), identical event counts,
the absorbed photons of every packet within 1e-8. FP32 geometry - every
level's total rate within 1e-3, the photons absorbed within 1e-4. Streamed
over octants - equal to the unsplit run up to the order of the additions
(1e-12). NLTE with the rates - populations within 1e-8 of the oracle's.
"""
import math
import sys

import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu

C_LIGHT = 2.99792458e10


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
def medium():
    """Clumped 16^3 cube with the 2 x (20 + 15 + 15)-level atom, 1000 background
    lines, 1e5 packets; level populations drawn log-uniform in 1..100 cm^-3 so
    that the continuum is optically thick over a few cells."""
    w = synth.clumpy(n=16, n_lines=1000, n_packets=100_000, number=12)
    ie = synth.ion_energies(12, w.atom)
    g = np.random.default_rng(5)
    pops = 10 ** g.uniform(0.0, 2.0, (w.n_cells, w.atom.n_levels))
    pl = oracle.pi_levels(oracle.nlte_inputs_from_workload(w), ie, 25)
    return w, ie, pops, pl


def _oracle_run(w, pops, pl, explicit=None, lo=None, hi=None):
    photo = dict(level=pl["level"], sigma0=pl["sigma0"], pops=pops, length=C_LIGHT * w.t_exp,
                 **{"lambda": pl["lambda"]})
    inp = oracle.TransportInputs(w.n, w.beta_max, w.tau_scale, w.cell_photons, w.cell_packets,
                                 w.line_lambda, w.line_tau0,
                                 w.lambda_lo if lo is None else lo,
                                 w.lambda_hi if hi is None else hi, w.seed,
                                 explicit_packets=explicit, photoion=photo)
    return oracle.transport(inp, per_packet=True)


def _volume(w):
    return (2 * w.beta_max / w.n * C_LIGHT * w.t_exp) ** 3


def _gpu_setup(ex, ctx, w, ie, pops):
    atom = ex.Atom(ctx, w.atom)
    plan = ex.PiPlan(ctx, atom, ie, 25)
    pd = torch.as_tensor(pops, device="cuda:0")
    opac = plan.opacity(pd)
    grid = ex.grid_from_workload(w)
    grid.photoion = ex.Photoion(plan, opac, w.t_exp)
    return atom, plan, pd, opac, grid


def _rel(a, b):
    nz = b != 0
    assert np.array_equal(a != 0, nz), "different nonzero pattern"
    return float(np.max(np.abs(a[nz] - b[nz]) / np.abs(b[nz]))) if nz.any() else 0.0


def test_plan_and_opacity_match_definition(ex, ctx, medium):
    w, ie, pops, pl = medium
    _, plan, pd, opac, _ = _gpu_setup(ex, ctx, w, ie, pops)
    say(f"case: {plan.M} photoionising levels of {w.atom.n_levels}")
    assert plan.M == len(pl["level"]) > 20
    order = np.argsort(pl["lambda"], kind="stable")
    assert np.array_equal(plan.level, pl["level"][order])
    np.testing.assert_allclose(plan.lambda_thr, pl["lambda"][order], rtol=1e-15)
    np.testing.assert_allclose(plan.sigma0, pl["sigma0"][order], rtol=1e-15)
    assert np.all(np.diff(plan.lambda_thr) >= 0)
    lo, hi = plan.lambda_thr.min(), plan.lambda_thr.max()
    say(f"thresholds {lo * 1e8:.0f}..{hi * 1e8:.0f} A")
    assert lo < w.lambda_lo < hi  # some thresholds inside the emission band
    torch.cuda.synchronize()
    tab = opac.cpu().numpy()
    M = plan.M
    a = pops[:, plan.level] * plan.sigma0 / plan.lambda_thr ** 3
    S = np.concatenate([np.cumsum(a[:, ::-1], axis=1)[:, ::-1], np.zeros((w.n_cells, 1))], axis=1)
    np.testing.assert_allclose(tab[:, M + 1:], a, rtol=1e-15)
    np.testing.assert_allclose(tab[:, :M + 1], S, rtol=1e-14)


def test_fp64_transport_with_photoionisation_matches_oracle(ex, ctx, medium):
    w, ie, pops, pl = medium
    say("case: oracle, clumpy16 with photoionisation, 1e5 packets (serial)")
    r = _oracle_run(w, pops, pl)
    ref = oracle.dense_estimator(r["records"], w.n_cells, w.n_lines)
    gamma_ref = oracle.pi_rates(r["pi_absorbed"], pops, pl["level"], w.atom.n_levels, _volume(w))
    say(f"oracle: w_pi / w_emit = {r['stats']['w_pi'] / r['stats']['w_emit']:.3f}, "
        f"w_abs / w_emit = {r['stats']['w_abs'] / r['stats']['w_emit']:.3f}")
    assert r["stats"]["w_pi"] > 0.05 * r["stats"]["w_emit"]
    atom, plan, pd, opac, grid = _gpu_setup(ex, ctx, w, ie, pops)
    say("case: GPU, FP64 geometry")
    est, st, pk = ex.transport(ctx, grid, w.seed, w.lambda_lo, w.lambda_hi, w.n_packets,
                               packets_out=True)
    gpi = plan.rates(grid, w.t_exp, grid.photoion.tally)
    torch.cuda.synchronize()
    sd = ex.stats_dict(st)
    assert sd["error_flag"] == 0 and sd["bad_packets"] == 0
    for k in ("n_inter", "n_checks", "n_cross", "n_escaped", "n_killed"):
        assert sd[k] == r["stats"][k], k
    for k in ("w_emit", "w_esc", "w_abs", "w_pi"):
        assert sd[k] == pytest.approx(r["stats"][k], rel=1e-11), k
    rel_est = _rel(est.cpu().numpy(), ref)
    rel_pi = _rel(gpi.cpu().numpy(), gamma_ref)
    say(f"estimators max rel {rel_est:.2e}; photoionisation rates max rel {rel_pi:.2e}")
    assert rel_est <= 1e-9
    assert rel_pi <= 1e-9
    pk = pk.cpu().numpy()
    # per packet: a move cut at a threshold just after its start has a length
    # (D_threshold - D_start) that is a difference of nearly equal numbers,
    # rounded differently on the two sides; 1e-8 covers it (observed 9e-10)
    np.testing.assert_allclose(pk[:, 7], r["packets"][:, 11], rtol=1e-8, atol=1e-300)
    np.testing.assert_allclose(pk[:, 0], r["packets"][:, 0], rtol=1e-10, atol=0)


def test_fp32_geometry_photoionisation_statistics(ex, ctx, medium):
    w, ie, pops, pl = medium
    r = _oracle_run(w, pops, pl)
    gamma_ref = oracle.pi_rates(r["pi_absorbed"], pops, pl["level"], w.atom.n_levels, _volume(w))
    atom, plan, pd, opac, grid = _gpu_setup(ex, ctx, w, ie, pops)
    say("case: GPU, FP32 geometry")
    est, st, _ = ex.transport(ctx, grid, w.seed, w.lambda_lo, w.lambda_hi, w.n_packets,
                              geometry_fp32=True)
    gpi = plan.rates(grid, w.t_exp, grid.photoion.tally).cpu().numpy()
    sd = ex.stats_dict(st)
    assert sd["w_pi"] == pytest.approx(r["stats"]["w_pi"], rel=1e-4)
    assert sd["w_abs"] == pytest.approx(r["stats"]["w_abs"], rel=1e-4)
    per_level = gpi.sum(axis=0)
    ref_level = gamma_ref.sum(axis=0)
    on = ref_level > 0
    worst = float(np.max(np.abs(per_level[on] - ref_level[on]) / ref_level[on]))
    say(f"per-level totals max rel {worst:.2e}")
    assert worst <= 1e-3


@pytest.mark.parametrize("fp32", [False, True])
def test_streamed_photoionisation_equals_unsplit(ex, ctx, medium, fp32):
    w, ie, pops, pl = medium
    say(f"case: streamed vs unsplit with photoionisation, fp32={fp32}")
    atom, plan, pd, opac, grid = _gpu_setup(ex, ctx, w, ie, pops)
    est, st_u, _ = ex.transport(ctx, grid, w.seed, w.lambda_lo, w.lambda_hi, w.n_packets,
                                geometry_fp32=fp32)
    tally_u = grid.photoion.tally.clone()
    grid.photoion.tally.zero_()
    _, st_s, eg = ex.transport_streamed(ctx, grid, w.seed, w.lambda_lo, w.lambda_hi, w.n_packets,
                                        geometry_fp32=fp32, est_global=True)
    torch.cuda.synchronize()
    su, ss = ex.stats_dict(st_u), ex.stats_dict(st_s)
    for k in ("n_inter", "n_checks", "n_cross", "n_escaped", "n_killed"):
        assert su[k] == ss[k], k
    for k in ("w_emit", "w_esc", "w_kill", "w_abs", "w_pi"):
        assert ss[k] == pytest.approx(su[k], rel=1e-12), k
    assert _rel(eg.cpu().numpy(), est.cpu().numpy()) <= 1e-12
    r = _rel(grid.photoion.tally.cpu().numpy(), tally_u.cpu().numpy())
    say(f"tally max rel {r:.2e}")
    assert r <= 1e-12


def test_nlte_with_photoionisation_rates_matches_oracle(ex, ctx, medium):
    w, ie, pops, pl = medium
    atom, plan, pd, opac, grid = _gpu_setup(ex, ctx, w, ie, pops)
    ex.transport(ctx, grid, w.seed, w.lambda_lo, w.lambda_hi, w.n_packets)
    gpi = plan.rates(grid, w.t_exp, grid.photoion.tally)
    torch.cuda.synchronize()
    g = gpi.cpu().numpy()
    active = np.flatnonzero(w.rho > 0)
    cells = active[:: max(1, len(active) // 300)][:300]
    say(f"case: NLTE with photoionisation rates, {len(cells)} cells, tol 1e-10")
    sub = ex.cells_from_workload(w, cells=cells)
    sub.gamma_pi = torch.as_tensor(g[cells], device="cuda:0").contiguous()
    sol, status, _ = ex.nlte_solve(ctx, atom, sub, max_iter=200, tol=1e-10)
    plain, _, _ = ex.nlte_solve(ctx, atom, ex.cells_from_workload(w, cells=cells), max_iter=200,
                                tol=1e-10)
    torch.cuda.synchronize()
    inp = oracle.nlte_inputs_from_workload(w, cells=cells, gamma_pi=g)
    ref, ost, _ = oracle.nlte(inp)
    sol, status = sol.cpu().numpy(), status.cpu().numpy()
    assert np.all(ost == 0) and np.all(status == 0)
    rel = np.abs(sol - ref) / ref
    say(f"max rel vs oracle {rel.max():.2e}")
    assert rel.max() <= 1e-8
    # the photoionisation rates matter: ion fractions move
    moved = np.max(np.abs(plain.cpu().numpy() / sol - 1.0))
    say(f"largest population change from photoionisation {moved:.2e}")
    assert moved > 1e-3


def test_rays_with_photoionisation_match_oracle(ex, ctx, medium):
    """Rays of the first 8 cells towards 3 x 5 viewers, at cold-start populations.
    (2 x 2 viewers would send rays exactly along cell diagonals, where which
    of two tied walls comes first is decided by the last bit of the device's
    and the host's sine and cosine.)"""
    w, ie, pops, pl = medium
    inp = oracle.nlte_inputs_from_workload(w)
    cold, _, _ = oracle.nlte(inp, max_iter=0, first=0, count=w.n_cells)
    V = _volume(w)
    lmin, lmax = 1900e-8, 26000e-8
    nb = int(math.ceil(math.log(lmax / lmin) / math.log(1.001)))
    E, lam, _ = oracle.emission_bins(inp, cold, w.t_exp, V, lmin, lmax, nb)
    n_cells = 8
    nt, nph = 3, 5
    rays = oracle.ray_packets(w.n, w.beta_max, E, lam, nt, nph, first=0, count=n_cells)
    say(f"case: {len(rays)} rays with photoionisation (oracle serial)")
    r = _oracle_run(w, pops, pl, explicit=rays, lo=0.0, hi=0.0)
    ref = oracle.dense_estimator(r["records"], w.n_cells, w.n_lines)
    atom, plan, pd, opac, grid = _gpu_setup(ex, ctx, w, ie, pops)
    eplan = ex.EmissionPlan(ctx, atom, lmin, lmax, nb)
    ph, _ = ex.emission(ctx, eplan, atom, grid, w.t_exp, torch.as_tensor(cold, device="cuda:0"))
    n_rays = n_cells * eplan.n_bins * nt * nph
    est, st, _ = ex.transport_rays(ctx, grid, eplan, ph, nt, nph, first_ray=0, n_rays=n_rays)
    gpi = plan.rates(grid, w.t_exp, grid.photoion.tally)
    torch.cuda.synchronize()
    sd = ex.stats_dict(st)
    for k in ("n_inter", "n_cross", "n_escaped", "n_killed"):
        assert sd[k] == r["stats"][k], k
    assert sd["w_pi"] == pytest.approx(r["stats"]["w_pi"], rel=1e-11)
    assert _rel(est.cpu().numpy(), ref) <= 1e-9
    gamma_ref = oracle.pi_rates(r["pi_absorbed"], pops, pl["level"], w.atom.n_levels, V)
    got = gpi.cpu().numpy()
    assert _rel(got, gamma_ref) <= 1e-9


def test_bad_photoion_arguments(ex, ctx, medium):
    w, ie, pops, pl = medium
    atom, plan, pd, opac, grid = _gpu_setup(ex, ctx, w, ie, pops)
    say("case: photoion with no levels; a plan with no qualifying level")
    bad = ex.Photoion(plan, opac, w.t_exp)
    bad.struct = lambda: ex._Photoion(0, plan.device_lambda, ex._ptr(opac), 1.0,
                                      ex._ptr(bad.tally))
    grid.photoion = bad
    with pytest.raises(ex.ExtrassError, match="invalid argument"):
        ex.transport(ctx, grid, w.seed, w.lambda_lo, w.lambda_hi, 1000)
    with pytest.raises(ex.ExtrassError, match="invalid argument"):
        ex.PiPlan(ctx, atom, np.zeros(w.atom.n_species * 3), 25)
