"""Pins for the oracle's transport on the spherical (r, theta, phi) grid (Sec. 2),
against facts other than the oracle's own code:

- cell classification against an independent numpy classification of random
  points;
- the cells a ray visits, from the oracle's surface crossings, against fine
  sampling of the ray classified by numpy, and every crossing against the
  sample where the classification changes;
- cell volumes against the sphere's volume, and sampled emission: every packet
  inside its cell, radii distributed as r^2 within the shell;
- the uniform-sphere Sobolev closed form on the spherical grid, with the cell
  integral of 1 / (1 - |x|^2) done analytically (atanh(r) - r per shell);
- the optically thin limit and photon conservation.
"""
import math

import numpy as np
import pytest

import oracle
import synth

A = synth.ANGSTROM


def _grid(n_r=6, n_theta=5, n_phi=8, R=0.02, seed=0, uniform=False):
    g = np.random.default_rng(seed)
    if uniform:
        r = np.linspace(0.0, R, n_r + 1)
        th = np.linspace(0.0, np.pi, n_theta + 1)
    else:
        r = np.concatenate([[0.0], np.sort(g.uniform(0.05, 0.95, n_r - 1)) * R, [R]])
        th = np.concatenate([[0.0], np.sort(g.uniform(0.05, 0.95, n_theta - 1)) * np.pi, [np.pi]])
    return oracle.Sphere(r, th, n_phi)


def _np_cell(S, x):
    r = np.linalg.norm(x)
    if r >= S.r_edge[-1]:
        return -1
    ir = int(np.searchsorted(S.r_edge, r, side="right") - 1)
    th = math.acos(max(-1.0, min(1.0, x[2] / r))) if r > 0 else 0.0
    it = int(min(np.searchsorted(S.theta_edge, th, side="right") - 1, S.n_theta - 1))
    ph = math.atan2(x[1], x[0]) % (2 * math.pi)
    ip = int(min(ph // (2 * math.pi / S.n_phi), S.n_phi - 1))
    return ir + S.n_r * (it + S.n_theta * ip)


def test_cell_classification_matches_numpy():
    S = _grid()
    g = np.random.default_rng(1)
    for _ in range(3000):
        x = g.uniform(-0.021, 0.021, 3)
        assert S.cell(x) == _np_cell(S, x)


def test_ray_crossings_against_fine_sampling():
    S = _grid(n_r=5, n_theta=4, n_phi=6, seed=2)
    g = np.random.default_rng(3)
    R = S.r_edge[-1]
    for trial in range(60):
        x0 = g.normal(size=3)
        x0 *= g.uniform(0, 0.95) * R / np.linalg.norm(x0)
        d = g.normal(size=3)
        d /= np.linalg.norm(d)
        cuts = S.crossings(x0, d)
        s_end = cuts[-1]
        assert np.linalg.norm(x0 + s_end * d) == pytest.approx(R, rel=1e-12)
        # pieces between crossings, classified at their midpoints by numpy
        bounds = np.concatenate([[0.0], cuts])
        seq = []
        for a, b in zip(bounds[:-1], bounds[1:]):
            if b > a:
                c = _np_cell(S, x0 + 0.5 * (a + b) * d)
                if not seq or seq[-1] != c:
                    seq.append(c)
        # fine sampling of the ray
        s = np.linspace(0.0, s_end, 40001)[:-1] + 0.5 * s_end / 40000
        cells = [_np_cell(S, x0 + si * d) for si in s]
        fine = [cells[0]]
        change = []
        for i in range(1, len(cells)):
            if cells[i] != cells[i - 1]:
                fine.append(cells[i])
                change.append(0.5 * (s[i] + s[i - 1]))
        assert seq == fine, trial
        # every change of cell lies within one sampling step of a crossing
        step = s_end / 40000
        for sc in change:
            assert np.min(np.abs(cuts - sc)) <= step, trial


def test_volumes_and_sampled_emission():
    S = _grid(seed=4)
    R = S.r_edge[-1]
    assert S.volumes().sum() == pytest.approx(4 / 3 * np.pi * R ** 3, rel=1e-13)
    C = S.n_cells
    g = np.random.default_rng(5)
    cp = np.zeros(C, np.int32)
    cp[[0, 7, 31, C // 2, C - 1]] = 4000
    inp = oracle.TransportInputs(1, 1.0, np.ones(C, np.float32), np.ones(C), cp,
                                 np.array([9e-5]), np.array([0.0], np.float32),
                                 4000 * A, 6000 * A, 99, sphere=S)
    e = oracle.emission(inp)
    ids = np.repeat(np.arange(C), cp)
    for p in range(0, len(e), 7):
        assert S.cell(e[p, :3]) == ids[p]
    # radii within the shell follow r^2: r^3 uniform between the shell's edges
    c = C // 2
    ir = c % S.n_r
    ra, rb = S.r_edge[ir], S.r_edge[ir + 1]
    r = np.linalg.norm(e[ids == c, :3], axis=1)
    u = np.sort((r ** 3 - ra ** 3) / (rb ** 3 - ra ** 3))
    ks = np.max(np.abs(u - (np.arange(len(u)) + 0.5) / len(u)))
    assert ks < 1.63 / np.sqrt(len(u))  # 99 % Kolmogorov bound
    np.testing.assert_allclose(np.linalg.norm(e[:, 3:6], axis=1), 1.0, rtol=1e-14)


@pytest.mark.parametrize("tau", [1e-3, 0.3, 3.0])
def test_uniform_sphere_sobolev_closed_form_on_spherical_grid(tau):
    """As the cube's pin: packets enter through the sphere (the grid's outer
    edge), cosine-weighted inward, lab frequency flat over [nu_k/(1+R),
    nu_k/(1-R)]; a cell's expected estimator is (1 - e^-tau) P w (1 - R^2) /
    (2 pi R^3) int_cell d^3x / (1 - |x|^2), and on a spherical cell that
    integral is dphi (cos th_a - cos th_b) [atanh(r) - r]_{r_a}^{r_b}."""
    R = 0.46
    S = oracle.Sphere(np.linspace(0.0, R, 6), np.linspace(0.0, np.pi, 5), 6)
    P = 300_000
    g = np.random.default_rng(12345)
    m = g.standard_normal((P, 3))
    m /= np.linalg.norm(m, axis=1, keepdims=True)
    x0 = R * (1 - 1e-12) * m
    mu = np.sqrt(g.random(P))
    ph = 2 * np.pi * g.random(P)
    t1 = np.cross(m, np.where(np.abs(m[:, :1]) < 0.9, [[1, 0, 0]], [[0, 1, 0]]))
    t1 /= np.linalg.norm(t1, axis=1, keepdims=True)
    t2 = np.cross(m, t1)
    st = np.sqrt(1 - mu * mu)
    d = -mu[:, None] * m + st[:, None] * (np.cos(ph)[:, None] * t1 + np.sin(ph)[:, None] * t2)
    lam_k = 5000 * A
    nu_k = 1.0 / lam_k
    lamL = 1.0 / g.uniform(nu_k / (1 + R), nu_k / (1 - R), P)
    lam_e = lamL / (1 - (d * x0).sum(1))
    wgt = 1.0 / P
    pk = np.column_stack([x0, d, lam_e, np.full(P, wgt)])
    C = S.n_cells
    inp = oracle.TransportInputs(1, 1.0, np.ones(C, np.float32), np.zeros(C), np.zeros(C, np.int32),
                                 np.array([lam_k]), np.array([tau], np.float32), 0, 0, 1,
                                 explicit_packets=pk, sphere=S)
    r = oracle.transport(inp, nthreads=8)
    est = oracle.dense_estimator(r["records"], C, 1)[:, 0]
    F = np.arctanh(S.r_edge) - S.r_edge
    radial = F[1:] - F[:-1]
    ct = np.cos(S.theta_edge[:-1]) - np.cos(S.theta_edge[1:])
    integ = (radial[:, None, None] * ct[None, :, None]
             * np.full(S.n_phi, 2 * np.pi / S.n_phi)).transpose(2, 1, 0).ravel()
    a = -math.expm1(-tau)
    expect = a * P * wgt * (1 - R * R) / (2 * np.pi * R ** 3) * integ
    sigma = wgt * a * np.sqrt(expect / (wgt * a))
    z = (est - expect) / sigma
    assert np.abs(z).max() < 5.0
    chi2 = (z * z).sum()
    assert chi2 < C + 5 * np.sqrt(2 * C)
    assert abs((est.sum() - expect.sum()) / np.sqrt((sigma ** 2).sum())) < 4.0


def test_thin_limit_and_conservation_on_spherical_grid():
    S = _grid(n_r=8, n_theta=6, n_phi=10, R=0.02, seed=6)
    C = S.n_cells
    g = np.random.default_rng(7)
    rho = g.uniform(0.5, 2.0, C)
    cp = synth.largest_remainder(rho, 4000)
    lam = np.sort(g.uniform(4000, 6000, 60)) * A
    for lo, hi in ((1e-9, 5e-5), (1e-3, 10.0)):
        tau0 = (10 ** g.uniform(np.log10(lo), np.log10(hi), 60)).astype(np.float32)
        inp = oracle.TransportInputs(1, 1.0, (rho / rho.mean()).astype(np.float32), rho * 1e40, cp,
                                     lam, tau0, 4000 * A, 6000 * A, 11, sphere=S)
        r = oracle.transport(inp, per_packet=True, nthreads=2)
        pk = r["packets"]
        st = r["stats"]
        assert (pk[:, 0] + pk[:, 2] + pk[:, 3]).sum() == pytest.approx(st["w_emit"], rel=1e-12)
        if hi < 1e-4:
            assert len(r["records"]) == 0 and st["n_escaped"] == 4000
            np.testing.assert_allclose(pk[:, 0] * 4000, (rho * 1e40).sum(), rtol=0.6)
        else:
            assert st["n_inter"] > 1000 and st["n_cross"] > 4000


def test_cell_middles_lie_in_their_cells():
    """The rays' starting points on the spherical grid (mid-radius, mid-angle,
    mid-slice) classified by numpy fall in their own cells."""
    S = _grid(n_r=7, n_theta=5, n_phi=9, seed=8)
    m = S.middles()
    assert m.shape == (S.n_cells, 3)
    for c in range(S.n_cells):
        assert _np_cell(S, m[c]) == c


def test_rays_from_spherical_cells_carry_their_photons_once():
    """Deterministic rays from the middles of spherical cells, through lines of
    zero opacity: every ray escapes unshifted in direction, and the escaped
    photons of each cell equal its bins' photons (the viewers' solid angles
    sum to 4 pi)."""
    S = _grid(n_r=4, n_theta=3, n_phi=4, seed=9)
    C = S.n_cells
    g = np.random.default_rng(10)
    nb = 3
    lam = np.array([4500.0, 5200.0, 6100.0]) * A
    E = g.uniform(0.5, 2.0, (C, nb)) * 1e30
    E[::5, 1] = 0.0  # some empty bins
    rays = oracle.ray_packets(1, 1.0, E, lam, 4, 6, sphere=S)
    photons = E / (6.62607015e-27 * 2.99792458e10 / lam)
    assert rays[:, 7].sum() == pytest.approx(photons.sum(), rel=1e-13)
    inp = oracle.TransportInputs(1, 1.0, np.ones(C, np.float32), np.ones(C), np.zeros(C, np.int32),
                                 np.array([5000 * A]), np.array([0.0], np.float32), 0, 0, 1,
                                 explicit_packets=rays, sphere=S)
    r = oracle.transport(inp, per_packet=True)
    assert r["stats"]["n_escaped"] == len(rays) and len(r["records"]) == 0
    assert r["stats"]["w_esc"] == pytest.approx(photons.sum(), rel=1e-13)
    # each ray starts in the cell whose bins it carries, in cell order
    per_cell = (E > 0).sum(1) * 24
    cells = np.repeat(np.arange(C), per_cell)
    for i in range(0, len(rays), 11):
        assert S.cell(rays[i, :3]) == cells[i]
