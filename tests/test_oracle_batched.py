"""Pins for the batched NLTE oracle (one element, three ion stages per cell,
frozen rates; Sec. 2.2 rate model).

What fixes the answer independently of the oracle's code:
- LTE limit: when collisions dominate every other process, populations within
  a stage follow the Boltzmann law g exp(-E/kT) (detailed balance of the
  collision rates); g and E come from numpy's own Philox.
- Ground-state-only stages: a birth-death chain whose stationary ratios are
  ionisation over recombination into the ground (1/3 of the total).
- Two-level stage: the stationary ratio is the upward over the downward rate
  of the one pair (this restates the rate definition, with numpy's Philox for
  the draws).
- Structure: stages couple only through ionisation into, and recombination
  out of, the next stage's ground state.
- Exact rational stationary vector of the oracle's own matrix on a small cell,
  and the componentwise balance of inflow and outflow on a full-size cell.
"""
from fractions import Fraction

import numpy as np
import pytest

import oracle
import synth

K_B = 1.380649e-16


def _uniforms(seed, c, z, a, b):
    """Philox4x64-10 block at counter (c, z, a, b), key (seed, 6), from numpy."""
    v = (int(c) | (int(z) << 64) | (int(a) << 128) | (int(b) << 192)) - 1  # numpy pre-increments
    words = np.array([(v >> (64 * k)) & (2 ** 64 - 1) for k in range(4)], dtype=np.uint64)
    bg = np.random.Philox(key=np.array([seed, 6], dtype=np.uint64), counter=words)
    x = bg.random_raw(4)
    return (x >> np.uint64(11)).astype(np.float64) * 2.0 ** -53


def _level(seed, c, z, i, T):
    u = _uniforms(seed, c, z, i, 1 << 63)
    return 1.0 + np.floor(9.0 * u[0]), (0.0 if i == 0 else 69.0 * K_B * T * u[1])


def test_lte_limit_is_boltzmann():
    T = 6000.0
    # n_e q e^-69 must exceed every radiative and photoexcitation rate: n_e ~ 1e60
    b = synth.batched_custom([[12, 0, 0], [7, 0, 0]], T_e=T, n_e=1e60, gamma_ion=0.0)
    inp = oracle.BatchedInputs(b)
    pops, bad = oracle.batched(inp, nthreads=1)
    assert bad == 0
    for c in range(2):
        n = int(b.level_count[3 * c])
        w = np.array([g * np.exp(-E / (K_B * T)) for g, E in
                      (_level(b.seed, c, 0, i, T) for i in range(n))])
        expect = w / w.sum()
        got = pops[b.pop_offset[c]:b.pop_offset[c + 1]]
        assert expect.min() < 1e-20          # the span reaches deep Boltzmann tails
        np.testing.assert_allclose(got, expect, rtol=1e-9, atol=0)


def test_ground_only_stages_birth_death_chain():
    T, ne = 8000.0, 3.0e6
    gion = np.array([[1e-4, 3e-6]])
    b = synth.batched_custom([[1, 1, 1]], T_e=T, n_e=ne, gamma_ion=gion, alpha0=(2e-12, 5e-12))
    pops, bad = oracle.batched(oracle.BatchedInputs(b), nthreads=1)
    assert bad == 0
    rec = ne * np.array([2e-12, 5e-12]) * (T / 1e4) ** -0.8 / 3.0
    r1 = gion[0, 0] / rec[0]
    r2 = r1 * gion[0, 1] / rec[1]
    expect = np.array([1.0, r1, r2]) / (1.0 + r1 + r2)
    np.testing.assert_allclose(pops, expect, rtol=1e-13)


def test_two_level_stage_ratio():
    T, ne = 5000.0, 1e6
    b = synth.batched_custom([[2, 0, 0]] * 40, T_e=T, n_e=ne, gamma_ion=0.0)
    pops, bad = oracle.batched(oracle.BatchedInputs(b), nthreads=1)
    assert bad == 0
    seen_rad = 0
    for c in range(40):
        g0, E0 = _level(b.seed, c, 0, 0, T)
        g1, E1 = _level(b.seed, c, 0, 1, T)
        u = _uniforms(b.seed, c, 0, 0, 1)
        rad = u[0] < 0.2
        seen_rad += rad
        A = 10.0 ** (-3 + 11 * u[1]) if rad else 0.0
        n = len(b.gamma_pe_table)
        gam = b.gamma_pe_table[min(n - 1, int(u[3] * n))] if rad else 0.0
        q = 10.0 ** (-10 + 3 * u[2])
        down = A + ne * q + (g0 / g1) * gam
        up = ne * q * (g1 / g0) * np.exp(-(E1 - E0) / (K_B * T)) + gam
        p = pops[2 * c:2 * c + 2]
        assert p[1] / p[0] == pytest.approx(up / down, rel=1e-13)
    assert seen_rad > 0


def test_stage_coupling_structure():
    b = synth.batched(cells=3)
    inp = oracle.BatchedInputs(b)
    for c in range(3):
        L = b.level_count[3 * c:3 * c + 3]
        off = np.concatenate([[0], np.cumsum(L)])
        R = oracle.batched_matrix(inp, c)
        allowed = np.zeros_like(R, dtype=bool)
        for z in range(3):
            s = slice(off[z], off[z + 1])
            allowed[s, s] = True
            if z < 2 and L[z + 1] > 0:
                allowed[s, off[z + 1]] = True      # ionisation into the next ground
                allowed[off[z + 1], s] = True      # recombination out of it
        np.fill_diagonal(allowed, False)
        assert np.all(R[~allowed] == 0.0)
        assert np.all(R[allowed] > 0.0)


def test_exact_rational_stationary_vector_small_cell():
    b = synth.batched_custom([[3, 2, 2]], T_e=7000.0, n_e=1e5, gamma_ion=[[1e-5, 1e-6]])
    inp = oracle.BatchedInputs(b)
    R = oracle.batched_matrix(inp, 0)
    pops, bad = oracle.batched(inp, nthreads=1)
    assert bad == 0
    N = len(R)
    Q = [[Fraction(R[i, j]) for j in range(N)] for i in range(N)]
    for i in range(N):
        Q[i][i] = -sum(Q[i][j] for j in range(N) if j != i)
    # pi^T Q = 0 with sum(pi) = 1: columns of Q (one replaced by ones), Gauss-Jordan
    M = [[Q[j][i] for j in range(N)] + [Fraction(0)] for i in range(N)]
    M[-1] = [Fraction(1)] * N + [Fraction(1)]
    for k in range(N):
        p = next(r for r in range(k, N) if M[r][k] != 0)
        M[k], M[p] = M[p], M[k]
        for r in range(N):
            if r != k and M[r][k] != 0:
                f = M[r][k] / M[k][k]
                M[r] = [a - f * bb for a, bb in zip(M[r], M[k])]
    exact = np.array([float(M[i][N] / M[i][i]) for i in range(N)])
    np.testing.assert_allclose(pops, exact, rtol=1e-13)


def test_full_size_cell_balances_componentwise():
    """The first three cells of the full problem (634, 563 and 208 levels):
    every level balances its own inflow and outflow to 1e-11, and the
    populations span more than 20 decades (the photoexcitation rates taken
    from the measured table pump some sparse levels, Boltzmann factors down
    to e^-69 keep others deep)."""
    b = synth.batched(cells=3)
    inp = oracle.BatchedInputs(b)
    pops, bad = oracle.batched(inp, nthreads=2)
    assert bad == 0
    deepest = 1.0
    for c in range(3):
        R = oracle.batched_matrix(inp, c)
        p = pops[b.pop_offset[c]:b.pop_offset[c + 1]]
        inflow = p @ R
        outflow = p * R.sum(1)
        assert np.all(p > 0)
        assert np.max(np.abs(inflow - outflow) / (inflow + outflow)) < 1e-11
        deepest = min(deepest, p.min())
    assert deepest < 1e-20
