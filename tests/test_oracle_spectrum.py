"""Pins of the oracle's emergent spectra per viewer (Sec. 2.3).

The expected bins below come from how the packets are built, not from the
oracle's binning formula:
- optically thin packets aimed at the centres of chosen (theta, phi) viewer
  bins, with lab wavelengths at the centres of chosen log-wavelength bins,
  land in exactly those bins with their full weight (the thin limit fixes
  w and lambda_L = lambda_e (1 - n.x0) in closed form);
- isotropic emission fills the viewers in proportion to their solid angle,
  2 pi / n_phi (cos theta_lo - cos theta_hi), within binomial errors;
- with absorbing lines, the spectrum holds exactly the escaped weight.
"""
import numpy as np

import oracle
import synth

HC = 6.62607015e-27 * 2.99792458e10


def _thin_inputs(n, beta, pk, n_lines=3):
    lam = np.array([3.0e-5, 5.0e-5, 7.0e-5])[:n_lines]
    return oracle.TransportInputs(n, beta, np.ones(n ** 3, np.float32), np.zeros(n ** 3),
                                  np.zeros(n ** 3, np.int32), lam, np.zeros(n_lines, np.float32),
                                  0, 0, 1, explicit_packets=pk)


def test_bin_centres_land_in_their_bins():
    n_t, n_p, n_l = 20, 20, 50
    lmin, lmax = 3000e-8, 9000e-8
    g = np.random.default_rng(3)
    beta = 0.02
    m = 300
    it = g.integers(0, n_t, m)
    ip = g.integers(0, n_p, m)
    ib = g.integers(0, n_l, m)
    theta = (it + 0.5) * np.pi / n_t
    phi = (ip + 0.5) * 2 * np.pi / n_p
    d = np.column_stack([np.sin(theta) * np.cos(phi), np.sin(theta) * np.sin(phi), np.cos(theta)])
    x0 = g.uniform(-0.9 * beta, 0.9 * beta, (m, 3))
    lam_L = lmin * (lmax / lmin) ** ((ib + 0.5) / n_l)
    lam_e = lam_L / (1.0 - np.sum(d * x0, axis=1))
    w0 = g.uniform(0.5, 2.0, m)
    pk = np.column_stack([x0, d, lam_e, w0])
    r = oracle.transport(_thin_inputs(6, beta, pk), per_packet=True)
    assert r["stats"]["n_escaped"] == m
    ph, en = oracle.spectrum(r["packets"], n_t, n_p, n_l, lmin, lmax)
    want = np.zeros((n_t, n_p, n_l))
    np.add.at(want, (it, ip, ib), w0)
    np.testing.assert_allclose(ph, want, rtol=1e-14, atol=0)
    want_e = np.zeros((n_t, n_p, n_l))
    np.add.at(want_e, (it, ip, ib), w0 * HC / lam_L)
    np.testing.assert_allclose(en, want_e, rtol=1e-12, atol=0)


def test_wavelengths_outside_the_range_are_not_binned():
    beta = 0.02
    d = np.array([[0.0, 0.0, 1.0], [0.0, 0.0, -1.0], [1.0, 0.0, 0.0]])
    x0 = np.zeros((3, 3))
    lam_e = np.array([2000e-8, 9000e-8, 5000e-8])  # below, at the top edge, inside
    pk = np.column_stack([x0, d, lam_e, np.ones(3)])
    r = oracle.transport(_thin_inputs(4, beta, pk), per_packet=True)
    ph, _ = oracle.spectrum(r["packets"], 4, 4, 10, 3000e-8, 9000e-8)
    assert ph.sum() == 1.0
    # the direction (1, 0, 0): theta = pi / 2 -> bin 2 of 4, phi = 0 -> bin 0
    assert ph[2, 0].sum() == 1.0


def test_isotropic_emission_fills_viewers_by_solid_angle():
    w = synth.sphere_small()
    inp = oracle.TransportInputs(w.n, w.beta_max, w.tau_scale, w.cell_photons, w.cell_packets,
                                 w.line_lambda, np.zeros_like(w.line_tau0), w.lambda_lo,
                                 w.lambda_hi, w.seed)
    r = oracle.transport(inp, per_packet=True)
    assert r["stats"]["n_escaped"] == inp.n_packets
    n_t, n_p = 10, 12
    ph, _ = oracle.spectrum(r["packets"], n_t, n_p, 1, 1e-6, 1.0)
    tot = r["packets"][:, 0].sum()
    assert abs(ph.sum() - tot) <= 1e-12 * tot
    # packets carry equal weights within a cell; use counts for the errors
    P = inp.n_packets
    edges = np.linspace(0, np.pi, n_t + 1)
    frac_t = (np.cos(edges[:-1]) - np.cos(edges[1:])) / 2
    got_t = ph.sum(axis=(1, 2)) / tot
    sig_t = np.sqrt(frac_t * (1 - frac_t) / P)
    assert np.all(np.abs(got_t - frac_t) < 5 * sig_t + 2e-3 * frac_t)
    got_p = ph.sum(axis=(0, 2)) / tot
    sig_p = np.sqrt((1 / n_p) * (1 - 1 / n_p) / P)
    assert np.all(np.abs(got_p - 1 / n_p) < 5 * sig_p + 2e-3 / n_p)


def test_spectrum_holds_the_escaped_weight():
    w = synth.sphere_small()
    inp = oracle.transport_inputs_from_workload(w)
    r = oracle.transport(inp, per_packet=True)
    pk = r["packets"]
    lmin, lmax = pk[:, 1].min() * 0.999, pk[:, 1].max() * 1.001
    ph, en = oracle.spectrum(pk, 5, 7, 64, lmin, lmax)
    esc = r["stats"]["w_esc"]
    assert 0 < esc < r["stats"]["w_emit"]
    np.testing.assert_allclose(ph.sum(), esc, rtol=1e-12)
    e = pk[:, 0] > 0
    np.testing.assert_allclose(en.sum(), np.sum(pk[e, 0] * HC / pk[e, 1]), rtol=1e-12)
