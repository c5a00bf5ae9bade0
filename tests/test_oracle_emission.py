"""Pins for the oracle's deterministic emission (Sec. 2.3; Eq. A3).

- a two-level atom's emission worked out by hand: A beta_S(tau) N_u h c /
  lambda into the right bin, a line outside the range counted outside;
- the rays of a bin carry its photons exactly once over the sphere (the
  reading E_bin (dOmega_k / 4 pi) / E_phot of the ray weight): the viewers'
  solid angles sum to 4 pi, each ray starts at its cell's centre, points at
  its viewer's bin centre and starts at the bin's reddest line;
- optically thin rays all escape with their full weight, so every viewer
  receives photons in proportion to its solid angle (isotropic emission).
"""
import math

import numpy as np
import pytest

import oracle
import synth

HC = 6.62607015e-27 * 2.99792458e10


def _atom(lams, A, g=(2.0, 4.0)):
    T = len(lams)
    # one stage: level 0 ground; transition t joins 0 -> t+1
    return synth.Atom(species_offset=np.array([0, T + 1], np.int32),
                      level_ion=np.zeros(T + 1, np.int32),
                      level_energy=np.linspace(0, 1e-12, T + 1),
                      level_g=np.array([g[0]] + [g[1]] * T),
                      trans_lower=np.zeros(T, np.int32),
                      trans_upper=np.arange(1, T + 1, dtype=np.int32),
                      trans_A=np.array(A, float), trans_lambda=np.array(lams, float),
                      trans_upsilon=np.ones(T), trans_line=np.arange(T, dtype=np.int32),
                      ion_alpha0=np.zeros(3), species_mass=np.array([16.0]))


def _inputs(atom, C=1):
    return oracle.NLTEInputs(atom, 1.728e7, np.full(C, 5000.0), np.full(C, 1e6), np.full(C, 1e7),
                             np.zeros(3 * C))


def test_two_level_emission_by_hand():
    lam_in, lam_out = 6300e-8, 30000e-8
    atom = _atom([lam_in, lam_out], [2.0e6, 3.0e3])
    inp = _inputs(atom)
    nl, nu1, nu2 = 3.0e6, 2.0e5, 7.0e4
    pops = np.array([[nl, nu1, nu2]])
    V, t = 2.5e45, 1.728e7
    lmin, lmax, nb = 3000e-8, 10000e-8, 1204
    E, lam, out = oracle.emission_bins(inp, pops, t, V, lmin, lmax, nb)
    tau = 2.0e6 / (8 * math.pi) * (4.0 / 2.0) * lam_in ** 3 * t * (nl - (2.0 / 4.0) * nu1)
    beta = (1.0 - math.exp(-tau)) / tau
    e_in = 2.0e6 * beta * nu1 * V * HC / lam_in
    b = int(math.floor(nb * math.log(lam_in / lmin) / math.log(lmax / lmin)))
    assert tau > 1.0                      # optically thick: beta matters
    assert E[0, b] == pytest.approx(e_in, rel=1e-13)
    assert np.count_nonzero(E) == 1 and lam[b] == lam_in and np.count_nonzero(lam) == 1
    tau2 = 3.0e3 / (8 * math.pi) * 2.0 * lam_out ** 3 * t * (nl - 0.5 * nu2)
    e_out = 3.0e3 * (-math.expm1(-tau2) / tau2) * nu2 * V * HC / lam_out
    assert out[0] == pytest.approx(e_out, rel=1e-13)


def _small_workload():
    w = synth.sphere_small()
    inp = oracle.nlte_inputs_from_workload(w)
    pops, st, _ = oracle.nlte(inp, max_iter=0)        # the cold start
    V = (2 * w.beta_max / w.n * synth.C_CGS * w.t_exp) ** 3
    return w, inp, pops, V


def test_ray_weights_carry_each_bin_once():
    w, inp, pops, V = _small_workload()
    lmin, lmax = 2900e-8, 10500e-8
    nb = int(math.ceil(math.log(lmax / lmin) / math.log(1.001)))
    E, lam, _ = oracle.emission_bins(inp, pops, w.t_exp, V, lmin, lmax, nb)
    nt, nph = 5, 7
    act = np.flatnonzero(w.n_species > 0)
    empty = np.flatnonzero(w.n_species == 0)[7]
    assert len(oracle.ray_packets(w.n, w.beta_max, E, lam, nt, nph, first=empty, count=1)) == 0
    for c in act[[100, 900, 2000]]:
        rays = oracle.ray_packets(w.n, w.beta_max, E, lam, nt, nph, first=c, count=1)
        occ = np.flatnonzero(E[c] > 0)
        assert len(rays) == len(occ) * nt * nph
        r = rays.reshape(len(occ), nt * nph, 8)
        # every ray of a bin starts at the bin's reddest line, from the cell centre
        assert np.all(r[:, :, 6] == lam[occ][:, None])
        h = 2 * w.beta_max / w.n
        ci = np.array([c % w.n, (c // w.n) % w.n, c // (w.n * w.n)])
        np.testing.assert_allclose(r[:, :, :3], np.broadcast_to(-w.beta_max + (ci + 0.5) * h,
                                                                r[:, :, :3].shape), rtol=0,
                                   atol=1e-18)
        # the rays of a bin carry its photons once: sum over viewers = E / (h c / lambda)
        np.testing.assert_allclose(r[:, :, 7].sum(1), E[c, occ] / (HC / lam[occ]), rtol=1e-13)
        # directions: unit vectors at the viewer bin centres, theta-major
        d = r[0, :, 3:6]
        np.testing.assert_allclose(np.linalg.norm(d, axis=1), 1.0, rtol=1e-15)
        th = np.arccos(np.clip(d[:, 2], -1, 1))
        ph = np.mod(np.arctan2(d[:, 1], d[:, 0]), 2 * np.pi)
        k = np.arange(nt * nph)
        np.testing.assert_allclose(th, (k // nph + 0.5) * np.pi / nt, atol=1e-12)
        np.testing.assert_allclose(ph, (k % nph + 0.5) * 2 * np.pi / nph, atol=1e-12)
        # weights in proportion to the viewers' solid angles, which sum to 4 pi
        dom = (2 * np.pi / nph) * (np.cos((k // nph) * np.pi / nt) -
                                   np.cos((k // nph + 1) * np.pi / nt))
        assert dom.sum() == pytest.approx(4 * np.pi, rel=1e-14)
        np.testing.assert_allclose(r[0, :, 7] / r[0, :, 7].sum(), dom / (4 * np.pi), rtol=1e-13)


def test_thin_rays_escape_isotropically():
    w, inp, pops, V = _small_workload()
    lmin, lmax = 2900e-8, 10500e-8
    nb = int(math.ceil(math.log(lmax / lmin) / math.log(1.001)))
    E, lam, _ = oracle.emission_bins(inp, pops, w.t_exp, V, lmin, lmax, nb)
    nt, nph = 4, 6
    rays = oracle.ray_packets(w.n, w.beta_max, E, lam, nt, nph, first=1800, count=200)
    assert len(rays) > 10000
    # no line can absorb: every ray escapes with its whole weight
    tp = oracle.TransportInputs(w.n, w.beta_max, np.zeros(w.n_cells, np.float32),
                                np.zeros(w.n_cells), np.zeros(w.n_cells, np.int32),
                                w.line_lambda, np.zeros(w.n_lines, np.float32), 0, 0, 1,
                                explicit_packets=rays)
    r = oracle.transport(tp, per_packet=True, nthreads=2)
    pk = r["packets"]
    np.testing.assert_array_equal(pk[:, 0], rays[:, 7])
    k = np.arange(len(rays)) % (nt * nph)
    per_view = np.bincount(k, weights=pk[:, 0], minlength=nt * nph)
    dom = (2 * np.pi / nph) * (np.cos((np.arange(nt * nph) // nph) * np.pi / nt) -
                               np.cos((np.arange(nt * nph) // nph + 1) * np.pi / nt))
    np.testing.assert_allclose(per_view / dom, per_view.sum() / (4 * np.pi), rtol=1e-12)


def test_emission_with_each_cells_volume():
    """Per-cell volumes (the spherical grid's): the same two-level emission by
    hand with a different volume in each of two cells."""
    lam_in = 6300e-8
    atom = _atom([lam_in], [2.0e6])
    inp = _inputs(atom, C=2)
    nl, nu = 3.0e6, 2.0e5
    pops = np.array([[nl, nu], [nl, nu]])
    V = np.array([2.5e45, 7.0e43])
    t = 1.728e7
    lmin, lmax, nb = 3000e-8, 10000e-8, 1204
    E, _, _ = oracle.emission_bins(inp, pops, t, V, lmin, lmax, nb)
    tau = 2.0e6 / (8 * math.pi) * (4.0 / 2.0) * lam_in ** 3 * t * (nl - (2.0 / 4.0) * nu)
    beta = (1.0 - math.exp(-tau)) / tau
    b = int(math.floor(nb * math.log(lam_in / lmin) / math.log(lmax / lmin)))
    for c in range(2):
        assert E[c, b] == pytest.approx(2.0e6 * beta * nu * V[c] * HC / lam_in, rel=1e-13)
