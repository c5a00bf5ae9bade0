"""NLTE solve: HIP path vs the FP64 oracle on the same inputs.

Bar: componentwise max |n_gpu - n_oracle| / n_oracle <= 1e-8 over every level
of every converged cell (populations span down to ~1e-38 of the largest), and
identical convergence status.
"""
import sys

import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu

TOL = 1e-8


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def ex():
    import paper_2511_07539_amd as ex
    return ex


@pytest.fixture(scope="module")
def ctx(ex):
    return ex.Context(0)


def _oracle_gamma(w):
    """Photoexcitation rates from the oracle's own transport and cold start."""
    inp_n = oracle.nlte_inputs_from_workload(w)
    cold = np.zeros((w.n_cells, w.atom.n_levels))
    S = w.atom.n_species
    for c in np.where(w.n_species.reshape(-1, S).sum(1) > 0)[0]:
        cold[c] = oracle.nlte_cold(inp_n, int(c))
    r = oracle.transport(oracle.transport_inputs_from_workload(w))
    est = oracle.dense_estimator(r["records"], w.n_cells, w.n_lines)
    V = (2 * w.beta_max / w.n * synth.C_CGS * w.t_exp) ** 3
    return oracle.rates(est, cold, w.atom, V)


def _compare(pg, sg, po, so):
    mism = np.where(sg != so)[0]
    if len(mism):
        both = (sg == 0) | (so == 0)
        say("status mismatches", len(mism), "gpu", np.bincount(sg[mism] + 1), "oracle",
            np.bincount(so[mism] + 1))
        for c in mism[:5]:
            say(" cell", c, "gpu", sg[c], "oracle", so[c], "max rel",
                np.max(np.abs(pg[c] - po[c]) / np.abs(po[c])))
    assert np.array_equal(sg, so)
    conv = so == 0
    a, b = pg[conv], po[conv]
    rel = np.abs(a - b) / np.abs(b)
    return rel.max(), (b / b.max(axis=1, keepdims=True)).min()


def test_sphere_small_all_cells(ex, ctx):
    w = synth.sphere_small()
    gpe = _oracle_gamma(w)
    po, so, io = oracle.nlte(oracle.nlte_inputs_from_workload(w, gamma_pe=gpe), tol=1e-13)
    atom = ex.Atom(ctx, w.atom)
    cells = ex.cells_from_workload(w, gamma_pe=gpe)
    say("case: sphere16 NLTE, 4096 cells, 10 levels")
    pg, sg, ig = ex.nlte_solve(ctx, atom, cells, max_iter=200, tol=1e-10)
    torch.cuda.synchronize()
    pg, sg, ig = pg.cpu().numpy(), sg.cpu().numpy(), ig.cpu().numpy()
    assert (so == 0).sum() == 2176 and (so == 3).sum() == 1920
    worst, span = _compare(pg, sg, po, so)
    say("max componentwise rel", worst, "span", span, "iters gpu", ig.max(), "oracle", io.max())
    assert worst <= TOL
    assert np.all(pg[so == 3] == 0)


def test_three_stage_atom_sampled_cells(ex, ctx):
    """2 species x (20+15+15) levels; 3000 cells sampled from the 50^3 workload."""
    w = synth.paper_scale()
    g = np.random.default_rng(0)
    cells = np.sort(g.choice(w.n_cells, 3000, replace=False))
    T = w.atom.n_trans
    gpe = np.abs(g.standard_normal((w.n_cells, T))) * 10 ** g.uniform(-8, 0, (w.n_cells, T))
    inp = oracle.nlte_inputs_from_workload(w, gamma_pe=gpe.ravel(), cells=cells)
    po, so, io = oracle.nlte(inp, tol=1e-13)
    atom = ex.Atom(ctx, w.atom)
    cl = ex.cells_from_workload(w, gamma_pe=gpe, cells=cells)
    say("case: clumpy50 NLTE, 3000 sampled cells, 2x50 levels")
    pg, sg, ig = ex.nlte_solve(ctx, atom, cl, max_iter=200, tol=1e-10)
    torch.cuda.synchronize()
    worst, span = _compare(pg.cpu().numpy(), sg.cpu().numpy(), po, so)
    say("max componentwise rel", worst, "span", span)
    assert (so == 0).mean() >= 0.999   # both sides fail on the same rare cells
    assert worst <= TOL
    assert span < 1e-20


@pytest.mark.parametrize("ion_levels", [(10, 10, 24), (40,)])
def test_other_atom_shapes(ex, ctx, ion_levels):
    """Stage blocks that fill a 24-row block exactly (top stage of 24 levels:
    23 excited levels, no next ground), and a 40-level single-stage species
    whose block exceeds 32 rows (whole-system reduction)."""
    w = synth.clumpy(n=16, n_lines=3000, n_packets=1000, number=2, ion_levels=ion_levels)
    g = np.random.default_rng(1)
    cells = np.sort(g.choice(w.n_cells, 600, replace=False))
    T = w.atom.n_trans
    gpe = np.abs(g.standard_normal((w.n_cells, T))) * 10 ** g.uniform(-8, 0, (w.n_cells, T))
    inp = oracle.nlte_inputs_from_workload(w, gamma_pe=gpe.ravel(), cells=cells)
    po, so, _ = oracle.nlte(inp, tol=1e-13)
    atom = ex.Atom(ctx, w.atom)
    cl = ex.cells_from_workload(w, gamma_pe=gpe, cells=cells)
    say(f"case: NLTE with stages {ion_levels}, 600 sampled cells")
    pg, sg, _ = ex.nlte_solve(ctx, atom, cl, max_iter=200, tol=1e-10)
    torch.cuda.synchronize()
    worst, span = _compare(pg.cpu().numpy(), sg.cpu().numpy(), po, so)
    sgn = sg.cpu().numpy()
    say("max componentwise rel", worst, "span", span, "converged: gpu", (sgn == 0).mean(),
        "oracle", (so == 0).mean())
    # a single 40-level stage with A up to 1e8 s^-1 leaves a few percent of
    # cells unconverged on both sides; compared where both converge
    assert (so == 0).mean() >= 0.95 and (sgn == 0).mean() >= 0.95
    assert worst <= TOL


def test_warm_start_and_iteration_cap(ex, ctx):
    w = synth.sphere_small()
    inp = oracle.nlte_inputs_from_workload(w)
    po, so, _ = oracle.nlte(inp, tol=1e-13)
    atom = ex.Atom(ctx, w.atom)
    cells = ex.cells_from_workload(w)
    say("case: warm start from the oracle's roots")
    pg, sg, ig = ex.nlte_solve(ctx, atom, cells, guess=torch.as_tensor(po, device="cuda:0"))
    torch.cuda.synchronize()
    act = so == 0
    assert np.all(sg.cpu().numpy()[act] == 0)
    assert ig.cpu().numpy()[act].max() <= 3
    worst, _ = _compare(pg.cpu().numpy(), sg.cpu().numpy(), po, so)
    assert worst <= TOL
    say("case: max_iter = 1 reports non-convergence")
    _, s1, _ = ex.nlte_solve(ctx, atom, cells, max_iter=1)
    torch.cuda.synchronize()
    s1 = s1.cpu().numpy()
    assert np.all(s1[act] == 2) and np.all(s1[so == 3] == 3)


def test_tolerance_bounds_the_error(ex, ctx):
    """tol is the population accuracy: solved at tol (both the last Newton
    correction and the fixed-point residual below tol), every converged cell
    is within a small multiple of tol of the oracle's root (tol 1e-13), cold
    and warm-started alike. The bench runs both NLTE passes at 1e-8."""
    w = synth.paper_scale()
    g = np.random.default_rng(1)
    cells = np.sort(g.choice(w.n_cells, 2000, replace=False))
    T = w.atom.n_trans
    gpe = np.abs(g.standard_normal((w.n_cells, T))) * 10 ** g.uniform(-8, 0, (w.n_cells, T))
    inp = oracle.nlte_inputs_from_workload(w, gamma_pe=gpe.ravel(), cells=cells)
    po, so, _ = oracle.nlte(inp, tol=1e-13)
    atom = ex.Atom(ctx, w.atom)
    cl = ex.cells_from_workload(w, gamma_pe=gpe, cells=cells)
    for tol in (1e-6, 1e-8):
        say(f"case: clumpy50 NLTE, 2000 sampled cells, tol {tol:g}, cold and from a perturbed guess")
        pg, sg, ig = ex.nlte_solve(ctx, atom, cl, max_iter=200, tol=tol)
        # a guess off by up to a factor 1.5 per level, as a learned start would be
        guess = torch.as_tensor(po * np.exp(g.uniform(-0.4, 0.4, po.shape)), device="cuda:0")
        pw, sw, iw = ex.nlte_solve(ctx, atom, cl, max_iter=200, tol=tol, guess=guess,
                                   warm_budget=30)
        torch.cuda.synchronize()
        for name, p, s in (("cold", pg, sg), ("warm", pw, sw)):
            p, s = p.cpu().numpy(), s.cpu().numpy()
            ok = (so == 0) & (s <= 1)
            assert ok.sum() >= 0.999 * len(cells)
            rel = np.max(np.abs(p[ok] - po[ok]) / po[ok])
            say(f"  {name}: max rel {rel:.2e}")
            assert rel <= 3 * tol
