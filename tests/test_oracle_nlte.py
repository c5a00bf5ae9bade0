"""Pins for the oracle's NLTE solve: each checks it against something other than itself.

- two-level atom: scalar closed form with Sobolev escape, root by mpmath at 40 digits;
- LTE limit (collisions dominate): Boltzmann populations within an ion;
- ionisation balance of ground-only stages: n_{z+1}/n_z = Gamma_ion / (n_e alpha);
- the 1/3 : 2/3 recombination split, through a three-state chain solved by the
  Markov-chain tree theorem (brute-force enumeration of spanning trees);
- the stationary vector of every solved cell's final rate matrix, recomputed by
  brute-force spanning-tree enumeration (small atoms) or exact rational
  elimination, must reproduce the solution (it is a root);
- GTH against exact rational Gaussian elimination on random generators.
"""
import itertools
import math
from fractions import Fraction

import mpmath
import numpy as np
import pytest

import oracle
import synth

K_B = 1.380649e-16
EV = synth.EV


def make_atom(levels_per_stage, E_ev, g, A, ups, lam, alpha0=None):
    offs, ion = [0], []
    tl, tu = [], []
    for z, nl in enumerate(levels_per_stage):
        first = len(ion)
        ion += [z] * nl
        for lo in range(nl):
            for up in range(lo + 1, nl):
                tl.append(first + lo)
                tu.append(first + up)
    offs.append(len(ion))
    T = len(tl)
    alpha = np.zeros(3)
    if alpha0 is not None:
        alpha[: len(alpha0)] = alpha0
    return synth.Atom(species_offset=np.array(offs, np.int32), level_ion=np.array(ion, np.int32),
                      level_energy=np.array(E_ev, float) * EV, level_g=np.array(g, float),
                      trans_lower=np.array(tl, np.int32), trans_upper=np.array(tu, np.int32),
                      trans_A=np.broadcast_to(np.array(A, float), (T,)).copy(),
                      trans_lambda=np.broadcast_to(np.array(lam, float), (T,)).copy(),
                      trans_upsilon=np.broadcast_to(np.array(ups, float), (T,)).copy(),
                      trans_line=np.arange(T, dtype=np.int32), ion_alpha0=alpha,
                      species_mass=np.array([16.0]))


def one_cell(atom, T, ne, ntot, gion=(0.0, 0.0), gpe=None, t_exp=1.728e7):
    g = np.zeros(3)
    g[: len(gion)] = gion
    return oracle.NLTEInputs(atom, t_exp, np.array([T]), np.array([ne]), np.array([ntot]), g,
                             None if gpe is None else np.array(gpe, float))


@pytest.mark.parametrize("A,lam_A,gpe", [(1e-3, 6300, 0.0), (1e8, 6563, 0.0), (1e8, 6563, 3e-2),
                                         (3e5, 8500, 10.0)])
def test_two_level_closed_form(A, lam_A, gpe):
    T, ne, ntot, ups = 6000.0, 2e6, 3e7, 2.5
    gl, gu, dE = 2.0, 6.0, 1.9
    atom = make_atom([2], [0, dE], [gl, gu], A, ups, lam_A * 1e-8)
    inp = one_cell(atom, T, ne, ntot, gpe=[gpe])
    pops, st, _ = oracle.nlte(inp)
    assert st[0] == 0
    mp = mpmath.mp
    mp.dps = 40
    qul = mpmath.mpf(8.629e-6) * ups / (gu * mpmath.sqrt(T))
    qlu = qul * (gu / gl) * mpmath.exp(-mpmath.mpf(dE) * mpmath.mpf(EV) / (mpmath.mpf(K_B) * T))
    K = mpmath.mpf(A) * mpmath.mpf(lam_A * 1e-8) ** 3 * mpmath.mpf(1.728e7) / (8 * mpmath.pi)

    def beta(tau):
        return 1 if tau <= 0 else -mpmath.expm1(-tau) / tau

    def f(nu):
        nl = ntot - nu
        tau = K * ((gu / gl) * nl - nu)
        return nl * (ne * qlu + gpe) - nu * (A * beta(tau) + ne * qul + (gl / gu) * gpe)

    nu = mpmath.findroot(f, (mpmath.mpf(0), mpmath.mpf(ntot) * gu / (gl + gu)), solver="anderson")
    ref = np.array([float(ntot - nu), float(nu)])
    np.testing.assert_allclose(pops[0], ref, rtol=1e-11)


def test_lte_limit_is_boltzmann():
    g = np.random.default_rng(4)
    N = 8
    E = np.concatenate([[0], np.sort(g.uniform(0, 3, N - 1))])
    gw = g.integers(1, 10, N).astype(float)
    atom = make_atom([N], E, gw, 1e2, 5.0, 5000e-8)
    T = 7000.0
    inp = one_cell(atom, T, 1e22, 1e7)
    pops, st, _ = oracle.nlte(inp)
    assert st[0] == 0
    boltz = gw * np.exp(-E * EV / (K_B * T))
    boltz *= 1e7 / boltz.sum()
    np.testing.assert_allclose(pops[0], boltz, rtol=1e-9)


def test_ionisation_balance_ground_only():
    atom = make_atom([1, 1, 1], [0, 0, 0], [1, 2, 3], 0.0, 0.0, 5000e-8, alpha0=[2e-12, 5e-12])
    T, ne, ntot = 8000.0, 3e6, 1e7
    gion = (4e-5, 2e-6)
    inp = one_cell(atom, T, ne, ntot, gion=gion)
    pops, st, _ = oracle.nlte(inp)
    assert st[0] == 0
    a0 = 2e-12 * (T / 1e4) ** -0.8
    a1 = 5e-12 * (T / 1e4) ** -0.8
    r1 = gion[0] / (ne * a0)
    r2 = r1 * gion[1] / (ne * a1)
    ref = np.array([1, r1, r2]) * ntot / (1 + r1 + r2)
    np.testing.assert_allclose(pops[0], ref, rtol=1e-13)


def tree_theorem(R):
    """Stationary vector of a continuous-time chain by the Markov chain tree
    theorem: pi_i is proportional to the sum over spanning trees directed into
    i of the product of their rates. Brute force over all parent maps."""
    N = len(R)
    w = []
    for root in range(N):
        others = [i for i in range(N) if i != root]
        tot = Fraction(0)
        for parents in itertools.product(range(N), repeat=len(others)):
            par = dict(zip(others, parents))
            if any(par[i] == i for i in others):
                continue
            ok = True
            for i in others:  # every node must reach the root
                seen, j = set(), i
                while j != root:
                    if j in seen:
                        ok = False
                        break
                    seen.add(j)
                    j = par[j]
                if not ok:
                    break
            if not ok:
                continue
            prod = Fraction(1)
            for i in others:
                prod *= Fraction(R[i][par[i]])
            tot += prod
        w.append(tot)
    s = sum(w)
    return np.array([float(x / s) for x in w])


def test_recombination_split_by_tree_theorem():
    # stage 0: ground + one excited level; stage 1: ground
    atom = make_atom([2, 1], [0, 2.0, 0], [2, 4, 1], 3.0e3, 0.7, 7000e-8, alpha0=[4e-12])
    T, ne, ntot = 5000.0, 1e6, 1e6   # low density: the line is thin (tau ~ 0)
    inp = one_cell(atom, T, ne, ntot, gion=(1e-4,), t_exp=1.0)
    pops, st, _ = oracle.nlte(inp)
    assert st[0] == 0
    qul = 8.629e-6 * 0.7 / (4 * math.sqrt(T))
    qlu = qul * 2 * math.exp(-2.0 * EV / (K_B * T))
    K = 3.0e3 * (7000e-8) ** 3 * 1.0 / (8 * math.pi)
    nl, nu = pops[0][0], pops[0][1]
    tau = K * (2 * nl - nu)
    beta = -math.expm1(-tau) / tau
    rec = ne * 4e-12 * (T / 1e4) ** -0.8
    R = [[0, ne * qlu, 1e-4], [3.0e3 * beta + ne * qul, 0, 1e-4], [rec / 3, 2 * rec / 3, 0]]
    ref = tree_theorem(R) * ntot
    np.testing.assert_allclose(pops[0], ref, rtol=1e-12)


def _exact_stationary(R):
    """Exact rational solution of pi Q = 0, sum pi = 1 for the float rates R."""
    N = len(R)
    Q = [[Fraction(R[i][j]) if i != j else Fraction(0) for j in range(N)] for i in range(N)]
    for i in range(N):
        Q[i][i] = -sum(Q[i][j] for j in range(N) if j != i)
    # solve Q^T pi = 0 with the last equation replaced by normalisation
    M = [[Q[j][i] for j in range(N)] for i in range(N)]
    rhs = [Fraction(0)] * N
    M[N - 1] = [Fraction(1)] * N
    rhs[N - 1] = Fraction(1)
    for k in range(N):
        p = next(r for r in range(k, N) if M[r][k] != 0)
        M[k], M[p] = M[p], M[k]
        rhs[k], rhs[p] = rhs[p], rhs[k]
        for r in range(k + 1, N):
            f = M[r][k] / M[k][k]
            if f:
                for c in range(k, N):
                    M[r][c] -= f * M[k][c]
                rhs[r] -= f * rhs[k]
    x = [Fraction(0)] * N
    for k in range(N - 1, -1, -1):
        x[k] = (rhs[k] - sum(M[k][c] * x[c] for c in range(k + 1, N))) / M[k][k]
    return np.array([float(v) for v in x])


def test_gth_exact_on_stiff_random_generators():
    g = np.random.default_rng(11)
    for N in (3, 6, 9):
        R = 10 ** g.uniform(-9, 8, (N, N))
        R[g.random((N, N)) < 0.3] = 0.0
        for i in range(N):
            R[i, (i + 1) % N] = max(R[i, (i + 1) % N], 1e-6)   # irreducible ring
            R[i, i] = 0.0
        np.testing.assert_allclose(oracle.gth(R), _exact_stationary(R), rtol=1e-12)


def test_solutions_are_roots_small_atom():
    """The sphere workload's 10-level atom: the final rate matrix of each solved
    cell has the solution as its exact stationary vector."""
    w = synth.sphere_small()
    inp = oracle.nlte_inputs_from_workload(w)
    pops, st, _ = oracle.nlte(inp)
    active = np.where(st == 0)[0]
    assert len(active) == 2176
    for c in active[:: 50]:
        R = oracle.rate_matrix(inp, int(c), 0, pops[c])
        ref = _exact_stationary(R) * pops[c].sum()
        np.testing.assert_allclose(pops[c], ref, rtol=1e-12)
        assert pops[c].sum() == pytest.approx(w.n_species[c], rel=1e-14)


def test_solutions_are_roots_three_stage_atom():
    """The 2-species x 3-stage (20+15+15 levels) atom on a few clumpy cells:
    conservation, positivity, and the final rates' exact stationary vector."""
    w = synth.clumpy(n=10, n_lines=1000, n_packets=1000, number=2)
    cells = [5, 123, 271, 456, 618, 789, 901, 999]
    inp = oracle.nlte_inputs_from_workload(w, cells=cells)
    pops, st, _ = oracle.nlte(inp)
    assert np.all(st == 0)
    S = w.atom.n_species
    off = w.atom.species_offset
    for ci in range(len(cells)):
        for s in range(S):
            n = pops[ci, off[s]: off[s + 1]]
            assert np.all(n > 0)
            assert n.sum() == pytest.approx(w.n_species.reshape(-1, S)[cells[ci], s], rel=1e-13)
            R = oracle.rate_matrix(inp, ci, s, n)
            ref = _exact_stationary(R) * n.sum()
            np.testing.assert_allclose(n, ref, rtol=1e-11)


def test_four_level_nonlinear_root_by_mpmath():
    """A 4-level ion whose lines are optically thick, so beta_S(tau(n)) makes
    the equations nonlinear in every radiative term: the root found by mpmath
    Newton at 50 digits (started 20 % off the oracle's answer, so it has to
    find the root itself) equals the oracle's populations to 1e-11."""
    E = [0.0, 1.1, 2.3, 3.0]
    g = [2.0, 4.0, 6.0, 2.0]
    A, ups, lam = 5e7, 1.5, 5500e-8
    atom = make_atom([4], E, g, A, ups, lam)
    T, ne, ntot = 6500.0, 5e6, 4e8
    gpe = [1e-3, 3e-4, 2e-2, 5e-5, 1e-2, 7e-4]
    inp = one_cell(atom, T, ne, ntot, gpe=gpe)
    pops, st, _ = oracle.nlte(inp)
    assert st[0] == 0
    mp = mpmath.mp
    mp.dps = 50
    kT = mpmath.mpf(K_B) * T
    pairs = [(l, u) for l in range(4) for u in range(l + 1, 4)]

    def rates(n):
        R = [[mpmath.mpf(0)] * 4 for _ in range(4)]
        for t, (l, u) in enumerate(pairs):
            qul = mpmath.mpf(8.629e-6) * ups / (g[u] * mpmath.sqrt(T))
            qlu = qul * (mpmath.mpf(g[u]) / g[l]) * mpmath.exp(-(mpmath.mpf(E[u]) - E[l]) *
                                                                mpmath.mpf(EV) / kT)
            K = mpmath.mpf(A) * mpmath.mpf(lam) ** 3 * mpmath.mpf(1.728e7) / (8 * mpmath.pi)
            tau = K * ((mpmath.mpf(g[u]) / g[l]) * n[l] - n[u])
            beta = 1 if tau <= 0 else -mpmath.expm1(-tau) / tau
            R[u][l] += A * beta + ne * qul + (mpmath.mpf(g[l]) / g[u]) * gpe[t]
            R[l][u] += ne * qlu + gpe[t]
        return R

    def F(*n):
        R = rates(n)
        eq = [sum(n[j] * R[j][i] for j in range(4) if j != i) -
              n[i] * sum(R[i][j] for j in range(4) if j != i) for i in range(3)]
        return eq + [sum(n) - ntot]

    start = [mpmath.mpf(float(v)) * (1.2 if i % 2 else 0.8) for i, v in enumerate(pops[0])]
    root = mpmath.findroot(F, start, tol=mpmath.mpf(10) ** -40)
    ref = np.array([float(v) for v in root])
    K = A * lam ** 3 * 1.728e7 / (8 * math.pi)
    assert K * 3 * ref[0] > 10   # the ground's lines are optically thick
    np.testing.assert_allclose(pops[0], ref, rtol=1e-11)
