"""Pins for the oracle's transport: checks against facts other than the oracle itself.

- Philox4x64-10 against numpy's independent implementation;
- the optically thin limit (no line interacts, every packet escapes unchanged);
- photon-number and comoving-energy bookkeeping per packet;
- the analytic Sobolev result for a uniform, isotropically illuminated sphere
  (resonance rate per volume 4 pi I nu_k / (1 - |x|^2) under first-order
  Doppler; absorbed fraction 1 - e^-tau per resonance);
- brute force on a 4^3 grid: every wall plane and every resonance of a ray
  enumerated, sorted by path length and replayed;
- mirror symmetry on a dyadic grid, bitwise.
"""
import math

import numpy as np
import pytest
from scipy import integrate

import oracle
import synth

A = synth.ANGSTROM


def _numpy_philox(ctr, key):
    # numpy advances the 256-bit counter (word 0 least significant) before each
    # block: start one below, borrowing across words
    v = sum(int(w) << (64 * i) for i, w in enumerate(ctr)) - 1
    v %= 1 << 256
    start = [(v >> (64 * i)) & ((1 << 64) - 1) for i in range(4)]
    bg = np.random.Philox(key=np.array(key, dtype=np.uint64),
                          counter=np.array(start, dtype=np.uint64))
    return bg.random_raw(4)


@pytest.mark.parametrize("ctr,key", [((1, 0, 0, 0), (0, 0)), ((5, 7, 1, 0), (2511075391, 3)),
                                     ((0, 5, 1, 0), (77, 3)),
                                     ((2**63 + 11, 3, 0, 9), (123456789, 987654321))])
def test_philox_matches_numpy(ctr, key):
    assert np.array_equal(oracle.philox4x64(ctr, key), _numpy_philox(ctr, key))


def _tiny_workload(tau_lo, tau_hi, n=4, n_lines=40, n_packets=4000, seed=1):
    g = np.random.default_rng(seed)
    beta = 0.01
    rho = g.uniform(0.5, 2.0, n ** 3)
    lam = np.sort(g.uniform(4000, 6000, n_lines)) * A
    tau0 = 10 ** g.uniform(np.log10(tau_lo), np.log10(tau_hi), n_lines)
    cp = synth.largest_remainder(rho, n_packets)
    return oracle.TransportInputs(n, beta, (rho / rho.mean()).astype(np.float32), rho * 1e40, cp,
                                  lam, tau0.astype(np.float32), 4000 * A, 6000 * A, 77)


def test_thin_limit_every_packet_escapes_unchanged():
    inp = _tiny_workload(1e-9, 5e-5)
    r = oracle.transport(inp, per_packet=True, nthreads=2)
    pk = r["packets"]
    assert len(r["records"]) == 0
    assert r["stats"]["n_inter"] == 0 and r["stats"]["n_killed"] == 0
    w0 = inp.arrays["cell_photons"] / np.maximum(inp.arrays["cell_packets"], 1)
    cells = np.repeat(np.arange(inp.n_cells), inp.arrays["cell_packets"])
    assert np.array_equal(pk[:, 0], w0[cells])
    assert r["stats"]["w_esc"] == pytest.approx(r["stats"]["w_emit"], rel=1e-14)


def test_photon_and_energy_bookkeeping_per_packet():
    w = synth.sphere_small()
    inp = oracle.transport_inputs_from_workload(w)
    r = oracle.transport(inp, count=20000, per_packet=True, nthreads=4)
    pk = r["packets"]
    cells = np.repeat(np.arange(w.n_cells), w.cell_packets)[:20000]
    w0 = (w.cell_photons / np.maximum(w.cell_packets, 1))[cells]
    np.testing.assert_allclose(pk[:, 0] + pk[:, 2] + pk[:, 3], w0, rtol=1e-13)
    per = np.bincount(r["records"]["packet"], weights=r["records"]["value"], minlength=20000)
    np.testing.assert_allclose(per, pk[:, 3], rtol=1e-13, atol=0)
    # emitted comoving energy = absorbed + adiabatic (homologous redshift) + remaining
    np.testing.assert_allclose(pk[:, 4] + pk[:, 5] + pk[:, 7], pk[:, 6], rtol=1e-12)
    assert (pk[:, 5] >= -1e-30).all()


def test_sampled_emission_statistics():
    w = synth.sphere_small()
    inp = oracle.transport_inputs_from_workload(w)
    # all tau below threshold: lambda_L = lambda_e (1 - n.x) is returned per packet
    inp.arrays["line_tau0"][:] = 0
    r = oracle.transport(inp, per_packet=True, nthreads=4)
    lamL = r["packets"][:, 1]
    assert np.all(lamL > w.lambda_lo * (1 - 2 * w.beta_max))
    assert np.all(lamL < w.lambda_hi * (1 + 2 * w.beta_max))
    # Doppler shifts average out for isotropic directions: mean lamL ~ mean band
    assert abs(lamL.mean() / (0.5 * (w.lambda_lo + w.lambda_hi)) - 1) < 2e-4


def _cell_integral(n, beta, f, order=6):
    xg, wg = np.polynomial.legendre.leggauss(order)
    h = 2 * beta / n
    out = np.zeros(n ** 3)
    for c in range(n ** 3):
        i, j, k = c % n, (c // n) % n, c // (n * n)
        lo = -beta + np.array([i, j, k]) * h
        px = lo[0] + (xg + 1) * h / 2
        py = lo[1] + (xg + 1) * h / 2
        pz = lo[2] + (xg + 1) * h / 2
        X, Y, Z = np.meshgrid(px, py, pz, indexing="ij")
        W = np.einsum("i,j,k->ijk", wg, wg, wg) * (h / 2) ** 3
        out[c] = (W * f(X, Y, Z)).sum()
    return out


@pytest.mark.parametrize("tau", [1e-3, 0.3, 3.0, 1e3])
def test_uniform_sphere_sobolev_closed_form(tau):
    """Isotropic, uniform intensity inside a sphere of radius R (in v/c).

    Packets enter through the sphere's surface, cosine-weighted inward, with lab
    frequency flat over [nu_k/(1+R), nu_k/(1-R)], which makes the field inside
    uniform and isotropic up to each photon's single resonance. Then the
    expected estimator of a cell with tau is
      (1 - e^-tau) * P w (1 - R^2) / (2 pi R^3) * int_cell d^3x / (1 - |x|^2).
    Only cells lying entirely inside the sphere carry the line.
    """
    n, beta, R = 10, 0.5, 0.46
    P = 400_000
    g = np.random.default_rng(12345)
    m = g.standard_normal((P, 3))
    m /= np.linalg.norm(m, axis=1, keepdims=True)
    x0 = R * m
    # cosine-weighted direction about the inward normal -m
    mu = np.sqrt(g.random(P))
    ph = 2 * np.pi * g.random(P)
    t1 = np.cross(m, np.where(np.abs(m[:, :1]) < 0.9, [[1, 0, 0]], [[0, 1, 0]]))
    t1 /= np.linalg.norm(t1, axis=1, keepdims=True)
    t2 = np.cross(m, t1)
    st = np.sqrt(1 - mu * mu)
    d = -mu[:, None] * m + st[:, None] * (np.cos(ph)[:, None] * t1 + np.sin(ph)[:, None] * t2)
    lam_k = 5000 * A
    nu_k = 1.0 / lam_k
    nuL = g.uniform(nu_k / (1 + R), nu_k / (1 - R), P)
    lamL = 1.0 / nuL
    D0 = (d * x0).sum(1)
    lam_e = lamL / (1 - D0)
    wgt = 1.0 / P
    pk = np.column_stack([x0, d, lam_e, np.full(P, wgt)])
    h = 2 * beta / n
    corners = np.array([[a, b, c] for a in (0, 1) for b in (0, 1) for c in (0, 1)])
    scale = np.zeros(n ** 3, dtype=np.float32)
    for c in range(n ** 3):
        ijk = np.array([c % n, (c // n) % n, c // (n * n)])
        pts = -beta + (ijk + corners) * h
        if np.all(np.linalg.norm(pts, axis=1) <= R):
            scale[c] = 1.0
    assert scale.sum() >= 20
    inp = oracle.TransportInputs(n, beta, scale, np.zeros(n ** 3), np.zeros(n ** 3, np.int32),
                                 np.array([lam_k]), np.array([tau], np.float32), 0, 0, 1,
                                 explicit_packets=pk)
    r = oracle.transport(inp, nthreads=8)
    est = oracle.dense_estimator(r["records"], n ** 3, 1)[:, 0]
    integ = _cell_integral(n, beta, lambda X, Y, Z: 1.0 / (1.0 - (X * X + Y * Y + Z * Z)))
    a = -math.expm1(-tau)
    expect = a * P * wgt * (1 - R * R) / (2 * np.pi * R ** 3) * integ * (scale > 0)
    inside = scale > 0
    # each resonance contributes w*a; counts are Poisson to a good approximation
    sigma = wgt * a * np.sqrt(expect[inside] / (wgt * a))
    z = (est[inside] - expect[inside]) / sigma
    assert np.abs(z).max() < 5.0
    chi2 = (z * z).sum()
    k = inside.sum()
    assert chi2 < k + 5 * np.sqrt(2 * k)
    tot_z = (est[inside].sum() - expect[inside].sum()) / np.sqrt((sigma ** 2).sum())
    assert abs(tot_z) < 4.0
    assert np.all(est[~inside] == 0)


def _brute_force(inp, packets, tau_cl):
    """Independent replay: all wall-plane crossings and all resonances of a ray,
    merged by path length; the cell of a resonance is found from its position."""
    a = inp.arrays
    n = inp.s.n
    beta = inp.s.beta_max
    h = 2 * beta / n
    lam = a["line_lambda"]
    recs = []
    for p, row in enumerate(packets):
        x0, d, lam_e, w0 = row[:3], row[3:6], row[6], row[7]
        D0 = float(np.dot(d, x0))
        lamL = lam_e * (1 - D0)
        # exit path length from the cube
        s_exit = np.inf
        for ax in range(3):
            if d[ax] > 0:
                s_exit = min(s_exit, (beta - x0[ax]) / d[ax])
            elif d[ax] < 0:
                s_exit = min(s_exit, (-beta - x0[ax]) / d[ax])
        events = []
        for k in range(len(lam)):
            if lam[k] > lam_e:
                Dk = 1 - lamL / lam[k]
                s = Dk - D0
                if s <= s_exit:
                    events.append((s, k))
        events.sort()
        w = w0
        for s, k in events:
            pos = x0 + max(s, 0.0) * d
            ijk = np.clip(np.floor((pos + beta) / h).astype(int), 0, n - 1)
            c = ijk[0] + n * (ijk[1] + n * ijk[2])
            tau = tau_cl[c, k]
            if tau > 1e-4:
                dN = w * -math.expm1(-tau)
                recs.append((p, c, k, dN))
                w = w * math.exp(-tau)
                if w * lam_e < (1e-6 * w0) * lam[k]:
                    break
    return recs


def test_brute_force_4cube():
    g = np.random.default_rng(7)
    n, beta = 4, 0.02
    L = 60
    lam = np.sort(g.uniform(4800, 5200, L)) * A
    tau0 = (10 ** g.uniform(-5, 1.5, L)).astype(np.float32)
    scale = g.uniform(0.0, 2.0, n ** 3).astype(np.float32)
    P = 3000
    x0 = g.uniform(-beta, beta, (P, 3))
    d = g.standard_normal((P, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    lam_e = g.uniform(4800, 5200, P) * A
    pk = np.column_stack([x0, d, lam_e, np.ones(P)])
    inp = oracle.TransportInputs(n, beta, scale, np.zeros(n ** 3), np.zeros(n ** 3, np.int32), lam,
                                 tau0, 0, 0, 1, explicit_packets=pk)
    r = oracle.transport(inp, nthreads=4)
    tau_cl = scale.astype(np.float64)[:, None] * tau0.astype(np.float64)[None, :]
    bf = _brute_force(inp, pk, tau_cl)
    rec = r["records"]
    assert len(rec) == len(bf) and len(bf) > 2000
    got = [(int(a), int(b), int(c)) for a, b, c in zip(rec["packet"], rec["cell"], rec["line"])]
    assert got == [(p, c, k) for p, c, k, _ in bf]
    np.testing.assert_allclose(rec["value"], [v for *_, v in bf], rtol=1e-12)


def test_mirror_symmetry_bitwise():
    g = np.random.default_rng(3)
    n, beta = 4, 0.5          # dyadic grid: every wall coordinate is exact
    L = 30
    lam = np.sort(g.uniform(4000, 9000, L)) * A
    tau0 = (10 ** g.uniform(-3, 2, L)).astype(np.float32)
    scale = g.uniform(0.1, 2.0, n ** 3).astype(np.float32)
    P = 2000
    x0 = g.uniform(-beta, beta, (P, 3)) * 0.999
    d = g.standard_normal((P, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    lam_e = g.uniform(4000, 9000, P) * A
    pk = np.column_stack([x0, d, lam_e, np.ones(P)])
    idx = np.arange(n ** 3)
    i, j, k = idx % n, (idx // n) % n, idx // (n * n)
    mirror = (n - 1 - i) + n * (j + n * k)
    pkm = pk.copy()
    pkm[:, 0] *= -1
    pkm[:, 3] *= -1
    base = dict(cell_photons=np.zeros(n ** 3), cell_packets=np.zeros(n ** 3, np.int32),
                line_lambda=lam, line_tau0=tau0, lambda_lo=0, lambda_hi=0, seed=1)
    e1 = oracle.dense_estimator(oracle.transport(oracle.TransportInputs(
        n, beta, scale, explicit_packets=pk, **base), nthreads=1)["records"], n ** 3, L)
    e2 = oracle.dense_estimator(oracle.transport(oracle.TransportInputs(
        n, beta, scale[mirror], explicit_packets=pkm, **base), nthreads=1)["records"], n ** 3, L)
    assert np.count_nonzero(e1) > 100
    assert np.array_equal(e1, e2[mirror])


def test_thread_count_does_not_change_results():
    w = synth.sphere_small()
    inp = oracle.transport_inputs_from_workload(w)
    a = oracle.dense_estimator(oracle.transport(inp, count=30000, nthreads=1)["records"],
                               w.n_cells, w.n_lines)
    b = oracle.dense_estimator(oracle.transport(inp, count=30000, nthreads=7)["records"],
                               w.n_cells, w.n_lines)
    assert np.array_equal(a, b)


def test_line_tau_eq_a2():
    at = synth.Atom(species_offset=np.array([0, 2], np.int32), level_ion=np.array([0, 0], np.int32),
                    level_energy=np.zeros(2), level_g=np.array([2.0, 6.0]),
                    trans_lower=np.array([0], np.int32), trans_upper=np.array([1], np.int32),
                    trans_A=np.array([8 * np.pi]), trans_lambda=np.array([1.0]),
                    trans_upsilon=np.array([1.0]), trans_line=np.array([0], np.int32),
                    ion_alpha0=np.zeros(3), species_mass=np.array([1.0]))
    pops = np.array([[1.0, 0.0], [2.0, 0.0], [1.0, 3.0], [1.0, 1.5]])
    tau, fc = oracle.line_tau(pops, at, 1.0)
    # A/(8 pi) g_u/g_l lambda^3 n_l (1 - g_l n_u / (g_u n_l)) t = 3 n_l - n_u here
    np.testing.assert_allclose(tau, [3.0, 6.0, 0.0, 1.5], rtol=1e-15, atol=1e-15)
    np.testing.assert_allclose(fc, [1.0, 1.0, 0.0, 0.5], rtol=1e-15, atol=1e-15)


def _u53(x):
    return float(int(x) >> 11) * 2.0 ** -53


def test_sampled_emission_mapping_matches_numpy_philox():
    """Each packet's emitted state, recomputed from numpy's own Philox4x64-10
    and the stated mapping: counters (p, iteration, 0, 0) and (p, iteration,
    1, 0) under key (seed, 3); uniforms u0..u3 of the first block and u4, u5 of
    the second; x = corner + h (u0, u1, u2), mu = 2 u3 - 1, phi = 2 pi u4,
    lambda_e in stratum j of the cell's n_c strata: lambda_lo + (lambda_hi -
    lambda_lo) (j + u5) / n_c, w0 = cell photons / n_c. Cell-major ids: the
    cell owning id p is found from the cumulative packet counts. A swapped
    uniform, axis or stratum formula fails this."""
    inp = _tiny_workload(1e-9, 5e-5, n=4, n_packets=3000, seed=3)
    inp.s.iteration = 5
    cp = inp.arrays["cell_packets"].astype(np.int64)
    start = np.concatenate([[0], np.cumsum(cp)])
    ids = [0, 1, 17, 1499, int(start[-1]) - 1] + list(range(700, 705))
    got = {p: oracle.emission(inp, first=p, count=1)[0] for p in ids}
    n, beta = 4, 0.01
    h = 2 * beta / n
    lo, hi = 4000 * A, 6000 * A
    for p in ids:
        c = int(np.searchsorted(start, p, side="right") - 1)
        j, nc = p - start[c], cp[c]
        i, jj, k = c % n, (c // n) % n, c // (n * n)
        r0 = _numpy_philox((p, 5, 0, 0), (77, 3))
        r1 = _numpy_philox((p, 5, 1, 0), (77, 3))
        u = [_u53(v) for v in r0] + [_u53(v) for v in r1]
        corner = [-beta + i * h, -beta + jj * h, -beta + k * h]
        x = [corner[a] + h * u[a] for a in range(3)]
        mu = 2.0 * u[3] - 1.0
        phi = 2.0 * math.pi * u[4]
        st = math.sqrt(max(0.0, 1.0 - mu * mu))
        d = [st * math.cos(phi), st * math.sin(phi), mu]
        lam = lo + (hi - lo) * ((j + u[5]) / nc)
        w0 = inp.arrays["cell_photons"][c] / nc
        np.testing.assert_array_equal(got[p][:3], x)
        np.testing.assert_allclose(got[p][3:6], d, rtol=0, atol=4e-16)
        assert got[p][6] == lam and got[p][7] == w0
    # the transport follows exactly these packets: in the thin limit each
    # escapes with its emitted direction and lambda_L = lambda_e (1 - n.x)
    r = oracle.transport(inp, per_packet=True, nthreads=1)
    em = oracle.emission(inp)
    np.testing.assert_array_equal(r["packets"][:, 8:11], em[:, 3:6])
    lam_l = em[:, 6] * (1.0 - (em[:, 3:6] * em[:, :3]).sum(1))
    np.testing.assert_allclose(r["packets"][:, 1], lam_l, rtol=1e-15)


def test_rates_hand_computed_two_cells():
    """Gamma_PE = est[c, line(t)] / (n_lower(c) V) on a 2-cell, 3-line,
    3-level toy whose values are worked out by hand; a cell whose lower level
    is empty gets 0."""
    atom = synth.Atom(species_offset=np.array([0, 3], np.int32),
                      level_ion=np.zeros(3, np.int32), level_energy=np.zeros(3),
                      level_g=np.ones(3), trans_lower=np.array([0, 1], np.int32),
                      trans_upper=np.array([2, 2], np.int32), trans_A=np.ones(2),
                      trans_lambda=np.ones(2), trans_upsilon=np.ones(2),
                      trans_line=np.array([2, 0], np.int32), ion_alpha0=np.zeros(3),
                      species_mass=np.array([1.0]))
    est = np.array([[3.0, 5.0, 7.0],
                    [11.0, 13.0, 17.0]])
    pops = np.array([[2.0, 4.0, 1.0],
                     [0.0, 8.0, 1.0]])
    V = 0.5
    got = oracle.rates(est, pops, atom, V).reshape(2, 2)
    # cell 0: t0 lower 0 line 2: 7 / (2 * 0.5) = 7; t1 lower 1 line 0: 3 / (4 * 0.5) = 1.5
    # cell 1: t0 lower level empty -> 0;            t1: 11 / (8 * 0.5) = 2.75
    np.testing.assert_array_equal(got, [[7.0, 1.5], [0.0, 2.75]])
    # each cell's own volume (a spherical grid's): 0.5 and 0.25
    got = oracle.rates(est, pops, atom, np.array([0.5, 0.25])).reshape(2, 2)
    np.testing.assert_array_equal(got, [[7.0, 1.5], [0.0, 5.5]])


def test_line_tau_equals_line_opacity_integrated_along_a_ray():
    """Eq. A2 against its derivation rather than its formula: the textbook
    absorption cross section of a line, sigma(nu) = (g_u/g_l) A lambda^2 / (8
    pi) phi(nu), corrected for stimulated emission by (1 - g_l n_u / (g_u
    n_l)), integrated by quadrature along a ray through homologous flow, where
    the comoving frequency falls as nu_L (1 - s / (c t)), with a narrow
    Gaussian profile phi. The ray starts a fraction D of the way before the
    resonance, so the integral is the Sobolev depth times (1 - D) exactly."""
    c = 2.99792458e10
    lam0 = 5000e-8
    nu0 = c / lam0
    t = 1e6
    A_ul, g_l, g_u = 1e7, 2.0, 4.0
    at = synth.Atom(species_offset=np.array([0, 2], np.int32), level_ion=np.array([0, 0], np.int32),
                    level_energy=np.zeros(2), level_g=np.array([g_l, g_u]),
                    trans_lower=np.array([0], np.int32), trans_upper=np.array([1], np.int32),
                    trans_A=np.array([A_ul]), trans_lambda=np.array([lam0]),
                    trans_upsilon=np.array([1.0]), trans_line=np.array([0], np.int32),
                    ion_alpha0=np.zeros(3), species_mass=np.array([1.0]))
    D = 1e-6
    width = 1e-9 * nu0  # Gaussian sigma in frequency
    nu_L = nu0 / (1.0 - D)
    for n_l, n_u in ((1e3, 10.0), (5.0, 9.0), (2e-3, 0.0)):
        tau_a2, _ = oracle.line_tau(np.array([[n_l, n_u]]), at, t)
        stim = 1.0 - g_l * n_u / (g_u * n_l)

        def alpha(u):
            # u = s - s_res: the comoving frequency nu_L (1 - s / (c t)) is
            # nu0 - nu_L u / (c t) there (nu_L (1 - s_res / (c t)) = nu0)
            x = -nu_L * u / (c * t) / width
            phi = np.exp(-0.5 * x * x) / (width * np.sqrt(2 * np.pi))
            return n_l * (g_u / g_l) * A_ul * (c / nu0) ** 2 / (8 * np.pi) * stim * phi

        ds = width / nu_L * c * t  # the profile's width along the ray
        tau, _ = integrate.quad(alpha, -40 * ds, 40 * ds, points=[0.0], epsabs=0, epsrel=1e-12,
                                limit=400)
        assert tau / (1.0 - D) == pytest.approx(tau_a2[0], rel=1e-10), (n_l, n_u)
