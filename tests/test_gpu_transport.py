"""Transport, opacity and rates: HIP path vs the FP64 oracle on the same inputs.

Bars: FP64 geometry - per-entry relative difference <= 1e-3 on every
estimator entry (observed ~1e-10), the same set of non-zero entries and
identical event counts; FP32 geometry - per entry within 1e-3 wherever no
contributing packet met a resonance within 1e-5 cell widths of a wall at or
before it (near ties counted and reported), L1 difference <= 1e-3 of the
table, every line's sum within 1e-3, event counts within 1e-5.
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


@pytest.fixture(scope="module")
def small():
    w = synth.sphere_small()
    inp = oracle.transport_inputs_from_workload(w)
    r = oracle.transport(inp, per_packet=True)
    return w, r, oracle.dense_estimator(r["records"], w.n_cells, w.n_lines)


def _run(ex, ctx, w, fp32, grid=None, **kw):
    grid = grid or ex.grid_from_workload(w)
    est, stats, pk = ex.transport(ctx, grid, w.seed, w.lambda_lo, w.lambda_hi, w.n_packets,
                                  geometry_fp32=fp32, **kw)
    torch.cuda.synchronize()
    return est.cpu().numpy(), ex.stats_dict(stats), None if pk is None else pk.cpu().numpy()


def test_fp64_geometry_matches_oracle_per_entry(ex, ctx, small):
    w, r, ref = small
    say("case: sphere16 fp64 geometry, 1e5 packets")
    est, st, pk = _run(ex, ctx, w, False, packets_out=True)
    assert st["error_flag"] == 0
    nz = ref != 0
    assert np.array_equal(est != 0, nz)
    rel = np.abs(est[nz] - ref[nz]) / np.abs(ref[nz])
    say("max rel", rel.max())
    assert rel.max() <= 1e-3
    assert rel.max() <= 1e-9   # observed: rounding-level
    for k in ["n_inter", "n_checks", "n_cross", "n_escaped", "n_killed"]:
        assert st[k] == r["stats"][k], k
    for k in ["w_emit", "w_esc", "w_abs"]:
        assert st[k] == pytest.approx(r["stats"][k], rel=1e-12), k
    assert st["w_kill"] == pytest.approx(r["stats"]["w_kill"], rel=1e-9)
    # per packet: escaped/killed weight and lab wavelength
    opk = r["packets"]
    np.testing.assert_allclose(pk[:, 1], opk[:, 1], rtol=1e-14)
    np.testing.assert_allclose(pk[:, 0], opk[:, 0], rtol=1e-11, atol=0)
    np.testing.assert_allclose(pk[:, 3], opk[:, 3], rtol=1e-11, atol=1e-30)


def _fp32_metric(est, ref, rec, tie=1e-4):
    """Reduced-precision parity (FP32 positions and distances against the FP64
    oracle). Rounding can move a resonance that lies within rounding of a cell
    wall into the neighbouring cell, where another optical depth applies; the
    packet's weight then differs for the rest of its path. The oracle records
    each interaction's margin, min(D_k - D_entry, D_exit - D_k) / h, the
    distance of the resonance from its segment's walls in cell widths. A
    record is a near tie if its margin is below `tie`: D is held in FP32,
    whose unit roundoff 6e-8 times |D| <= sqrt(3) beta_max is 2.6e-6 cell
    widths per rounding at 50^3, and a path takes a few tens of roundings
    (wall crossings, D_k to FP32), so 1e-4. A near tie taints every later
    record of its packet, and its line's entries in the 27 cells around it
    (where the moved resonance can land). Entries with no taint must agree to
    1e-3; the tainted ones are counted, and so are entries the GPU filled where
    the oracle has none, which cannot exceed the near-tie records. The table
    and each line's sum must agree to 1e-3."""
    L = ref.shape[1]
    n = int(round(ref.shape[0] ** (1.0 / 3.0)))
    near = rec["margin"] < tie
    pkt = rec["packet"]
    assert np.all(pkt[1:] >= pkt[:-1]), "records must come in packet order"
    first = np.r_[True, pkt[1:] != pkt[:-1]]
    csum = np.cumsum(near)
    before = (csum - near)[first]                   # near ties before each packet
    tainted = (csum - np.repeat(before, np.diff(np.r_[np.flatnonzero(first), len(pkt)]))) > 0
    idx = rec["cell"].astype(np.int64) * L + rec["line"]
    taint_entry = np.zeros(ref.size, dtype=bool)
    taint_entry[idx[tainted]] = True
    c = rec["cell"][near].astype(np.int64)
    ci = np.stack([c % n, (c // n) % n, c // (n * n)], axis=1)
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                q = ci + np.array([dx, dy, dz])
                ok = np.all((q >= 0) & (q < n), axis=1)
                cc = q[ok, 0] + n * (q[ok, 1] + n * q[ok, 2])
                taint_entry[cc * L + rec["line"][near][ok]] = True
    e, r_ = est.ravel(), ref.ravel()
    clean = (r_ != 0) & ~taint_entry
    rel = np.abs(e[clean] - r_[clean]) / np.abs(r_[clean])
    moved = int(((r_ == 0) & (e != 0)).sum())
    bad = np.flatnonzero(clean)[rel > 1e-3]
    if len(bad):   # diagnostics: the records and packets behind the worst entries
        say(f"clean entries off by > 1e-3: {len(bad)}")
        pmin = np.minimum.reduceat(rec["margin"], np.flatnonzero(first))
        pk_first = np.flatnonzero(first)
        for b in bad[:8]:
            ri = np.flatnonzero(idx == b)
            pk = np.unique(pkt[ri])
            gi = np.searchsorted(pkt[pk_first], pk)
            say(f"  entry {b}: ref {r_[b]:.4e} est {e[b]:.4e} records {len(ri)} "
                f"min margin {rec['margin'][ri].min():.2e} packet min margin {pmin[gi].min():.2e}")
    d = np.abs(est - ref)
    line_ref = ref.sum(0)
    big_l = line_ref > 1e-3 * line_ref.max()
    line_err = np.abs(est.sum(0) - line_ref)
    return dict(l1=d.sum() / np.abs(ref).sum(),
                line=(line_err[big_l] / line_ref[big_l]).max(),
                clean_max_rel=float(rel.max()) if rel.size else 0.0,
                clean_entries=int(clean.sum()), near_tie_records=int(near.sum()),
                tainted_entries=int((taint_entry & (r_ != 0)).sum()), moved_entries=moved,
                nonzero=int((r_ != 0).sum()))


def _assert_fp32(m):
    assert m["l1"] <= 1e-3 and m["line"] <= 1e-3
    assert m["clean_max_rel"] <= 1e-3
    assert m["moved_entries"] <= m["near_tie_records"]


def test_fp32_geometry_matches_oracle_statistically(ex, ctx, small):
    w, r, ref = small
    say("case: sphere16 fp32 geometry, 1e5 packets")
    est, st, _ = _run(ex, ctx, w, True)
    m = _fp32_metric(est, ref, r["records"])
    say(m)
    _assert_fp32(m)
    assert abs(st["n_inter"] - r["stats"]["n_inter"]) <= 1e-3 * r["stats"]["n_inter"]


def test_explicit_packets_and_ragged_ranges(ex, ctx):
    """Explicit-packet mode, a packet range that starts mid-list, an empty range."""
    g = np.random.default_rng(5)
    n, beta, L = 7, 0.03, 333
    lam = np.sort(g.uniform(3000, 9000, L)) * synth.ANGSTROM
    tau0 = (10 ** g.uniform(-5, 3, L)).astype(np.float32)
    scale = g.uniform(0, 3, n ** 3).astype(np.float32)
    P = 5000
    x0 = g.uniform(-beta, beta, (P, 3))
    d = g.standard_normal((P, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    pk = np.column_stack([x0, d, g.uniform(3000, 9000, P) * synth.ANGSTROM, g.uniform(0.5, 2, P)])
    inp = oracle.TransportInputs(n, beta, scale, np.zeros(n ** 3), np.zeros(n ** 3, np.int32), lam,
                                 tau0, 0, 0, 1, explicit_packets=pk)
    first, cnt = 1234, 2717
    ro = oracle.transport(inp, first=first, count=cnt)
    ref = oracle.dense_estimator(ro["records"], n ** 3, L)
    grid = ex.Grid(n, beta, scale, np.zeros(n ** 3), np.zeros(n ** 3, np.int32), lam, tau0)
    say("case: explicit packets 7^3 x 333 lines, range [1234, 3951)")
    est, stats, _ = ex.transport(ctx, grid, 1, 0, 0, cnt, first_packet=first, explicit_packets=pk)
    torch.cuda.synchronize()
    est = est.cpu().numpy()
    nz = ref != 0
    assert np.array_equal(est != 0, nz)
    np.testing.assert_allclose(est[nz], ref[nz], rtol=1e-10)
    say("case: empty packet range")
    est0, st0, _ = ex.transport(ctx, grid, 1, 0, 0, 0, explicit_packets=pk)
    torch.cuda.synchronize()
    assert float(est0.abs().sum()) == 0.0
    assert float(st0[:9].abs().sum()) == 0.0


def test_small_packet_counts_every_packet_once(ex, ctx):
    """Counts below, at and just above the 32 idle lanes that trigger a refill,
    and above one wave: every packet is transported exactly once (per-entry
    estimators and the emitted-weight and event tallies equal the oracle's)."""
    g = np.random.default_rng(11)
    n, beta, L = 5, 0.03, 120
    lam = np.sort(g.uniform(3000, 9000, L)) * synth.ANGSTROM
    tau0 = (10 ** g.uniform(-3, 2, L)).astype(np.float32)
    scale = g.uniform(0.5, 2, n ** 3).astype(np.float32)
    P = 200
    x0 = g.uniform(-beta, beta, (P, 3))
    d = g.standard_normal((P, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    pk = np.column_stack([x0, d, g.uniform(3000, 9000, P) * synth.ANGSTROM, g.uniform(0.5, 2, P)])
    inp = oracle.TransportInputs(n, beta, scale, np.zeros(n ** 3), np.zeros(n ** 3, np.int32), lam,
                                 tau0, 0, 0, 1, explicit_packets=pk)
    grid = ex.Grid(n, beta, scale, np.zeros(n ** 3), np.zeros(n ** 3, np.int32), lam, tau0)
    for first, cnt in ((0, 1), (3, 31), (40, 32), (7, 33), (0, 65), (13, 187)):
        say(f"case: explicit packets 5^3 x 120 lines, range [{first}, {first + cnt})")
        ro = oracle.transport(inp, first=first, count=cnt)
        ref = oracle.dense_estimator(ro["records"], n ** 3, L)
        est, st, _ = ex.transport(ctx, grid, 1, 0, 0, cnt, first_packet=first, explicit_packets=pk)
        torch.cuda.synchronize()
        est = est.cpu().numpy()
        nz = ref != 0
        assert np.array_equal(est != 0, nz)
        np.testing.assert_allclose(est[nz], ref[nz], rtol=1e-10)
        sd = ex.stats_dict(st)
        np.testing.assert_allclose(sd["w_emit"], pk[first:first + cnt, 7].sum(), rtol=1e-12)
        for key in ("n_inter", "n_checks", "n_cross"):
            assert sd[key] == ro["stats"][key], key


def test_unsorted_lines_flagged(ex, ctx):
    n = 3
    lam = np.array([5e-5, 4e-5, 6e-5])
    grid = ex.Grid(n, 0.01, np.ones(27, np.float32), np.ones(27), np.ones(27, np.int32), lam,
                   np.ones(3, np.float32))
    say("case: unsorted line list")
    _, st, _ = ex.transport(ctx, grid, 1, 4e-5, 6e-5, 27)
    torch.cuda.synchronize()
    assert ex.stats_dict(st)["error_flag"] == 1


def test_bad_line_map_is_flagged_not_followed(ex, ctx):
    """A line -> transition entry outside [-1, n_trans) is never used as an
    index: the line acts as a background line and the estimators are flagged
    invalid."""
    w = synth.clumpy(n=8, n_lines=1000, n_packets=20_000, number=2)
    T = w.atom.n_trans
    tau = np.full((w.n_cells, T), 0.5)
    fc = np.ones((w.n_cells, T))
    grid = ex.grid_from_workload(w, tau_ct=tau, fcorr_ct=fc)
    say("case: line map entries beyond the transitions")
    _, st, _ = ex.transport(ctx, grid, w.seed, w.lambda_lo, w.lambda_hi, w.n_packets)
    torch.cuda.synchronize()
    assert ex.stats_dict(st)["error_flag"] == 0
    lt = grid.line_trans.clone()
    k = int(torch.nonzero(lt >= 0)[0])
    for bad in (T, T + 1000, -7):
        grid.line_trans[k] = bad
        _, st, _ = ex.transport(ctx, grid, w.seed, w.lambda_lo, w.lambda_hi, w.n_packets)
        torch.cuda.synchronize()
        assert ex.stats_dict(st)["error_flag"] == 1, bad
    grid.line_trans.copy_(lt)


def test_rates_reject_lines_beyond_the_grid(ex, ctx):
    """An atom whose transitions point past the grid's line list is refused
    before any kernel runs; a negative line index is refused at creation."""
    w = synth.sphere_small()
    atom = ex.Atom(ctx, w.atom)
    small = ex.Grid(w.n, w.beta_max, w.tau_scale, w.cell_photons, w.cell_packets,
                    w.line_lambda[: int(w.atom.trans_line.max())],
                    w.line_tau0[: int(w.atom.trans_line.max())])
    est = torch.zeros((small.n_cells, small.n_lines), dtype=torch.float64, device="cuda:0")
    pops = torch.ones((small.n_cells, atom.n_levels), dtype=torch.float64, device="cuda:0")
    say("case: rates with transition lines beyond the grid's lines")
    with pytest.raises(ex.ExtrassError, match="invalid argument"):
        ex.rates(ctx, atom, small, w.t_exp, est, pops)
    import dataclasses
    neg = dataclasses.replace(w.atom, trans_line=np.where(np.arange(w.atom.n_trans) == 3, -1,
                                                          w.atom.trans_line).astype(np.int32))
    with pytest.raises(ex.ExtrassError, match="invalid argument"):
        ex.Atom(ctx, neg)


def test_line_tau_and_rates_match_oracle(ex, ctx, small):
    w, r, ref = small
    inp = oracle.nlte_inputs_from_workload(w)
    pops = np.zeros((w.n_cells, w.atom.n_levels))
    for c in np.where(w.n_species > 0)[0]:
        pops[c] = oracle.nlte_cold(inp, int(c))
    tau_o, fc_o = oracle.line_tau(pops, w.atom, w.t_exp)
    V = (2 * w.beta_max / w.n * synth.C_CGS * w.t_exp) ** 3
    gam_o = oracle.rates(ref, pops, w.atom, V)
    atom = ex.Atom(ctx, w.atom)
    pd = torch.as_tensor(pops, device="cuda:0")
    say("case: Eq. A2 opacity and rates, sphere16")
    tau, fc = ex.line_tau(ctx, atom, pd, w.t_exp)
    gam = ex.rates(ctx, atom, ex.grid_from_workload(w), w.t_exp,
                   torch.as_tensor(ref, device="cuda:0"), pd)
    torch.cuda.synchronize()
    np.testing.assert_allclose(tau.cpu().numpy().ravel(), tau_o, rtol=1e-13, atol=0)
    np.testing.assert_allclose(fc.cpu().numpy().ravel(), fc_o, rtol=1e-13, atol=1e-15)
    np.testing.assert_allclose(gam.cpu().numpy().ravel(), gam_o, rtol=1e-14, atol=0)


def test_coupled_opacity_transport(ex, ctx):
    """Lines of the atom take tau and f_corr from populations (Eq. A2), the rest
    are background lines; a 12^3 clumpy grid, FP64 geometry."""
    w = synth.clumpy(n=12, n_lines=2000, n_packets=200_000, number=2)
    inp_n = oracle.nlte_inputs_from_workload(w)
    pops = np.stack([oracle.nlte_cold(inp_n, c) for c in range(w.n_cells)])
    tau_o, fc_o = oracle.line_tau(pops, w.atom, w.t_exp)
    inp = oracle.transport_inputs_from_workload(w, tau_ct=tau_o, fcorr_ct=fc_o)
    r = oracle.transport(inp)
    ref = oracle.dense_estimator(r["records"], w.n_cells, w.n_lines)
    grid = ex.grid_from_workload(w, tau_ct=tau_o, fcorr_ct=fc_o)
    say("case: clumpy12 coupled opacity, fp64 geometry")
    est, st, _ = _run(ex, ctx, w, False, grid=grid)
    nz = ref != 0
    assert np.array_equal(est != 0, nz)
    np.testing.assert_allclose(est[nz], ref[nz], rtol=1e-10)
    assert st["n_inter"] == r["stats"]["n_inter"]


@pytest.fixture(scope="module")
def paper_scale():
    """50^3 cells, 5000 lines, 1e7 packets; atom lines take tau from the cold-start
    populations (Eq. A2): the workload and launch bench.py times. The oracle runs
    every packet on the host."""
    w = synth.paper_scale()
    inp_n = oracle.nlte_inputs_from_workload(w)
    pops = np.stack([oracle.nlte_cold(inp_n, c) for c in range(w.n_cells)])
    tau_o, fc_o = oracle.line_tau(pops, w.atom, w.t_exp)
    say("case: clumpy50 oracle on host, 1e7 packets")
    r = oracle.transport(oracle.transport_inputs_from_workload(w, tau_ct=tau_o, fcorr_ct=fc_o))
    rec = r["records"]
    idx = rec["cell"].astype(np.int64) * w.n_lines + rec["line"]
    ref = np.bincount(idx, weights=rec["value"], minlength=w.n_cells * w.n_lines)
    return w, tau_o, fc_o, r, ref.reshape(w.n_cells, w.n_lines)


def test_paper_scale_fp64_full_size_per_entry(ex, ctx, paper_scale):
    w, tau_o, fc_o, r, ref = paper_scale
    grid = ex.grid_from_workload(w, tau_ct=tau_o, fcorr_ct=fc_o)
    say("case: clumpy50 fp64 geometry, 1e7 packets (GPU)")
    est, st, _ = _run(ex, ctx, w, False, grid=grid)
    nz = ref != 0
    support = int(((est != 0) != nz).sum())
    rel = np.abs(est[nz] - ref[nz]) / ref[nz]
    say("support mismatches", support, "max rel", rel.max())
    assert support == 0
    assert rel.max() <= 1e-3
    for k in ["n_inter", "n_checks", "n_cross", "n_escaped", "n_killed"]:
        assert st[k] == r["stats"][k], k


def test_paper_scale_fp32_full_size(ex, ctx, paper_scale):
    w, tau_o, fc_o, r, ref = paper_scale
    grid = ex.grid_from_workload(w, tau_ct=tau_o, fcorr_ct=fc_o)
    say("case: clumpy50 fp32 geometry, 1e7 packets (GPU)")
    est, st, _ = _run(ex, ctx, w, True, grid=grid)
    m = _fp32_metric(est, ref, r["records"])
    say(m)
    _assert_fp32(m)
    assert abs(st["n_inter"] - r["stats"]["n_inter"]) <= 1e-5 * r["stats"]["n_inter"]
    assert st["w_emit"] == pytest.approx(r["stats"]["w_emit"], rel=1e-12)
    assert st["w_abs"] == pytest.approx(r["stats"]["w_abs"], rel=1e-6)
