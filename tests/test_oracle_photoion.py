"""Pins for the oracle's photoionisation (Sec. 2.3.1; Eq. A5), against facts
other than the oracle itself:

- Eq. A5 at threshold against the textbook Kramers cross section of
  hydrogen-like levels, 7.9e-18 n / Z^2 cm^2 at lambda_n = 911.5 n^2 / Z^2 A;
- the absorbed fraction of a packet against 1 - exp(-tau), tau integrated
  numerically along the ray (scipy quad) with the cross section's lambda^3 law
  and the cut where the ray redshifts past the threshold;
- the split among levels in proportion to their optical depths;
- photon-number conservation per packet with lines and photoionisation;
- packets redward of every threshold are not touched (bitwise);
- the NLTE ionisation balance of a two-state atom, n+ / n0 = (gamma + Gamma_PI)
  / (n_e alpha), with the photoionisation rate as a level's extra ionisation.
"""
import numpy as np
import pytest
from scipy import integrate

import oracle
import synth

A = synth.ANGSTROM
EV = synth.EV
HC = 6.62607015e-27 * 2.99792458e10
C_LIGHT = 2.99792458e10
RYD_EV = 13.605693


def _atom(stages):
    """One species; stages: list of per-stage level energies (eV, ground first)."""
    ion, en = [], []
    for z, energies in enumerate(stages):
        ion += [z] * len(energies)
        en += list(np.asarray(energies) * EV)
    N = len(ion)
    empty_i = np.zeros(0, np.int32)
    empty_d = np.zeros(0)
    return synth.Atom(species_offset=np.array([0, N], np.int32), level_ion=np.array(ion, np.int32),
                      level_energy=np.array(en), level_g=np.ones(N), trans_lower=empty_i,
                      trans_upper=empty_i, trans_A=empty_d, trans_lambda=empty_d,
                      trans_upsilon=empty_d, trans_line=empty_i, ion_alpha0=np.zeros(3),
                      species_mass=np.array([1.0]))


def _nlte_inputs(atom, n_cells=1):
    S = atom.n_species
    return oracle.NLTEInputs(atom, 1e7, np.full(n_cells, 1e4), np.full(n_cells, 1e8),
                             np.full(n_cells * S, 1e8), np.zeros(n_cells * S * 3))


def test_hydrogenic_cross_section_is_kramers():
    # H I levels n = 1..5 and He II levels n = 1..4, energies above their ground
    h = [RYD_EV * (1 - 1 / k ** 2) for k in range(1, 6)]
    he = [4 * RYD_EV * (1 - 1 / k ** 2) for k in range(1, 5)]
    atom = _atom([h, he, [0.0]])
    ie = np.array([RYD_EV, 4 * RYD_EV, 0.0]) * EV
    pl = oracle.pi_levels(_nlte_inputs(atom), ie, max_per_stage=3)
    assert list(pl["level"]) == [0, 1, 2, 5, 6, 7]
    for j, lv in enumerate(pl["level"]):
        Z = 1 if lv < 5 else 2
        n = lv + 1 if lv < 5 else lv - 4
        assert pl["sigma0"][j] == pytest.approx(7.9e-18 * n / Z ** 2, rel=1e-12)
        lam_n = HC / (Z ** 2 * RYD_EV * EV / n ** 2)
        assert pl["lambda"][j] == pytest.approx(lam_n, rel=1e-12)
    assert pl["lambda"][0] == pytest.approx(911.27 * A, rel=1e-3)


def _medium(pi, pops, n=4, beta=0.01, t_exp=1e7, n_lines=0, packets=None, lam_lines=None,
            tau0=None):
    C = n ** 3
    if lam_lines is None:
        lam_lines = np.zeros(0)
        tau0 = np.zeros(0, np.float32)
    photo = dict(level=pi["level"], sigma0=pi["sigma0"], pops=pops, length=C_LIGHT * t_exp,
                 **{"lambda": pi["lambda"]})
    return oracle.TransportInputs(n, beta, np.ones(C, np.float32), np.ones(C), np.ones(C, np.int32),
                                  lam_lines, tau0, 3000 * A, 9000 * A, 5,
                                  explicit_packets=packets, photoion=photo)


def _exit_distance(x, d, beta):
    s = np.inf
    for a in range(3):
        if d[a] > 0:
            s = min(s, (beta - x[a]) / d[a])
        elif d[a] < 0:
            s = min(s, (-beta - x[a]) / d[a])
    return s


def test_absorbed_fraction_matches_quadrature_with_threshold_cut():
    lam_t = 5000 * A
    sigma0 = 1e-18
    n_pop = 300.0  # tau of order one across the cube at t = 1e7 s
    pi = {"level": np.array([0]), "lambda": np.array([lam_t]), "sigma0": np.array([sigma0])}
    beta, n, t_exp = 0.01, 4, 1e7
    pops = np.full((n ** 3, 1), n_pop)
    g = np.random.default_rng(3)
    rows = []
    for lam_e in [4700 * A, 4960 * A, 4990 * A, 4999.9 * A, 4800 * A]:
        x = g.uniform(-0.8 * beta, 0.8 * beta, 3)
        d = g.normal(size=3)
        d /= np.linalg.norm(d)
        rows.append([*x, *d, lam_e, 2.0])
    pk = np.array(rows)
    r = oracle.transport(_medium(pi, pops, n, beta, t_exp, packets=pk), per_packet=True)
    L = C_LIGHT * t_exp
    taus = []
    for p, row in enumerate(pk):
        x, d, lam_e, w0 = row[:3], row[3:6], row[6], row[7]
        D0 = float(d @ x)
        lamL = lam_e * (1 - D0)
        s_exit = _exit_distance(x, d, beta)
        s_thr = (1 - lamL / lam_t) - D0  # where lambda(s) reaches the threshold

        def kappa(s):
            lam = lamL / (1 - D0 - s)
            return sigma0 * (lam / lam_t) ** 3 * n_pop * L if lam < lam_t else 0.0
        pts = [s_thr] if 0 < s_thr < s_exit else None
        tau, _ = integrate.quad(kappa, 0.0, s_exit, points=pts, epsabs=0, epsrel=1e-13, limit=200)
        got = r["packets"][p, 11]
        assert got == pytest.approx(w0 * -np.expm1(-tau), rel=1e-9), (p, tau)
        taus.append(tau)
        assert r["packets"][p, 0] == pytest.approx(w0 * np.exp(-tau), rel=1e-9)
    assert max(taus) > 0.3 and min(taus) < 0.05  # optically thick paths and cut ones
    assert r["pi_absorbed"].sum() == pytest.approx(r["packets"][:, 11].sum(), rel=1e-13)
    assert r["stats"]["w_pi"] == pytest.approx(r["packets"][:, 11].sum(), rel=1e-13)


def test_split_in_proportion_to_optical_depth():
    lam_t = 6000 * A
    pi = {"level": np.array([0, 0, 1]), "lambda": np.full(3, lam_t),
          "sigma0": np.array([1e-18, 3e-18, 1e-18])}
    n = 4
    pops = np.zeros((n ** 3, 2))
    pops[:, 0] = 100.0
    pops[:, 1] = 200.0
    g = np.random.default_rng(4)
    rows = []
    for _ in range(20):
        d = g.normal(size=3)
        rows.append([*g.uniform(-0.009, 0.009, 3), *(d / np.linalg.norm(d)), 5000 * A, 1.0])
    r = oracle.transport(_medium(pi, pops, n, packets=np.array(rows)))
    ab = r["pi_absorbed"]
    hit = ab[:, 0] > 0
    assert hit.sum() > 10
    np.testing.assert_allclose(ab[hit, 1] / ab[hit, 0], 3.0, rtol=1e-13)
    np.testing.assert_allclose(ab[hit, 2] / ab[hit, 0], 2.0, rtol=1e-13)


def _sampled_with_lines(pi, pops, n=4, n_packets=3000):
    g = np.random.default_rng(8)
    beta = 0.01
    C = n ** 3
    rho = g.uniform(0.5, 2.0, C)
    lam = np.sort(g.uniform(4000, 6000, 40)) * A
    tau0 = (10 ** g.uniform(-3, 1, 40)).astype(np.float32)
    cp = synth.largest_remainder(rho, n_packets)
    photo = dict(level=pi["level"], sigma0=pi["sigma0"], pops=pops, length=C_LIGHT * 1e7,
                 **{"lambda": pi["lambda"]})
    return oracle.TransportInputs(n, beta, (rho / rho.mean()).astype(np.float32), rho * 1e40, cp,
                                  lam, tau0, 4000 * A, 6000 * A, 91, photoion=photo)


def _three_thresholds():
    return {"level": np.array([0, 1, 2]), "lambda": np.array([4500, 5000, 5600]) * A,
            "sigma0": np.array([2e-18, 1e-18, 5e-19])}


def test_photon_conservation_with_lines_and_photoionisation():
    pi = _three_thresholds()
    g = np.random.default_rng(2)
    pops = 10 ** g.uniform(1, 3, (64, 3))
    r = oracle.transport(_sampled_with_lines(pi, pops), per_packet=True)
    pk = r["packets"]
    w0 = pk[:, 0] + pk[:, 2] + pk[:, 3] + pk[:, 11]
    emitted = r["stats"]["w_emit"]
    assert w0.sum() == pytest.approx(emitted, rel=1e-12)
    assert r["stats"]["w_pi"] > 0.01 * emitted and r["stats"]["w_abs"] > 0.01 * emitted
    assert r["pi_absorbed"].sum() == pytest.approx(r["stats"]["w_pi"], rel=1e-12)


def test_packets_redward_of_every_threshold_are_untouched():
    pi = {"level": np.array([0]), "lambda": np.array([3900 * A]), "sigma0": np.array([1e-16])}
    pops = np.full((64, 1), 1e4)
    with_pi = oracle.transport(_sampled_with_lines(pi, pops), per_packet=True)
    plain = _sampled_with_lines(pi, pops)
    plain.s.pi_levels = 0
    plain.pi_levels = 0
    without = oracle.transport(plain, per_packet=True)
    assert with_pi["stats"]["w_pi"] == 0.0
    assert np.array_equal(with_pi["records"], without["records"])
    assert np.array_equal(with_pi["packets"][:, :11], without["packets"][:, :11])


def test_ionisation_balance_with_photoionisation_rate():
    atom = _atom([[0.0], [0.0], []])
    atom.ion_alpha0 = np.array([3e-13, 0.0, 0.0])
    T, ne, ntot, gamma, gpi = 8000.0, 2e7, 5e6, 1e-5, 3e-5
    inp = oracle.NLTEInputs(atom, 1e7, np.array([T]), np.array([ne]), np.array([ntot]),
                            np.array([gamma, 0.0, 0.0]), gamma_pi=np.array([gpi, 0.0]))
    pops, status, _ = oracle.nlte(inp)
    assert status[0] == 0
    rec = ne * 3e-13 * (T / 1e4) ** -0.8
    ratio = (gamma + gpi) / rec
    assert pops[0, 1] / pops[0, 0] == pytest.approx(ratio, rel=1e-13)
    assert pops[0].sum() == pytest.approx(ntot, rel=1e-14)
