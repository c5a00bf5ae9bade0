"""Seeded synthetic inputs shared by the oracle, the HIP path, the tests and the bench.

This module only *creates inputs*: grids, line lists, atoms and cell states,
as plain numpy arrays. It contains none of the method's arithmetic (no
transport, no Doppler shifts, no rates, no level populations). Random numbers
that the method itself draws, i.e. the packet positions, directions and
wavelengths, are not drawn here. Both the oracle and the GPU path compute them
from the same counter-based generator (Philox4x64-10) keyed by packet id.

Inputs stand in for the paper's ejecta models and SUMO atomic data. Those are
not available, so every field here is synthetic, with the shapes and value
ranges that the workloads below state.

Units are CGS throughout. Wavelengths are in cm, energies in erg, densities in
cm^-3, times in s. The velocity coordinate is x = v/c: the cube spans
[-beta_max, beta_max]^3 in x, and cell c = i + n*(j + n*k) has lower corner
-beta_max + (i, j, k)*h, with h = 2*beta_max/n.
"""
from __future__ import annotations

import dataclasses
import os
from typing import Optional

import numpy as np

C_KMS = 299792.458
C_CGS = 2.99792458e10
EV = 1.602176634e-12
M_U = 1.66053906660e-24
M_SUN = 1.98847e33
DAY = 86400.0
ANGSTROM = 1e-8

# Seed base: Philox key word 0 = SEED_BASE + workload number; word 1 = stream.
SEED_BASE = 2511075390
STREAM_GRID, STREAM_LINES, STREAM_ATOM, STREAM_PACKETS, STREAM_CELLS, STREAM_MLP = range(6)
# Key word 1 of the per-level and per-pair draws of the batched NLTE problem.
STREAM_BATCHED = 6
# Key word 1 of the ionisation energies drawn for photoionisation.
STREAM_PHOTOION = 7


def rng(workload: int, stream: int) -> np.random.Generator:
    return np.random.Generator(np.random.Philox(key=[SEED_BASE + workload, stream]))


def packet_seed(workload: int) -> int:
    """Philox key word 0 used by the method for packet sampling (word 1 = stream 3)."""
    return SEED_BASE + workload


@dataclasses.dataclass
class Atom:
    """A fixed atom shared by every cell: species -> ion stages -> levels.

    Levels of all species are numbered globally; species s owns levels
    [species_offset[s], species_offset[s+1]). Within a species the levels of ion
    stage z come before those of stage z+1, and the first level of each stage
    is its ground state (energy 0, measured from that stage's ground).
    Transitions join two levels of the same ion stage, lower < upper.
    """
    species_offset: np.ndarray   # int32 [S+1]
    level_ion: np.ndarray        # int32 [N]  ion stage within its species
    level_energy: np.ndarray     # f64 [N]  erg above its ion's ground state
    level_g: np.ndarray          # f64 [N]  statistical weight
    trans_lower: np.ndarray      # int32 [T] global level index
    trans_upper: np.ndarray      # int32 [T]
    trans_A: np.ndarray          # f64 [T] s^-1
    trans_lambda: np.ndarray     # f64 [T] cm
    trans_upsilon: np.ndarray    # f64 [T] effective collision strength
    trans_line: np.ndarray       # int32 [T] index into the line list
    ion_alpha0: np.ndarray       # f64 [S*3] recombination coefficient into stage z at 1e4 K (cm^3 s^-1); 0 if none
    species_mass: np.ndarray     # f64 [S] atomic mass number

    @property
    def n_species(self) -> int:
        return len(self.species_offset) - 1

    @property
    def n_levels(self) -> int:
        return len(self.level_ion)

    @property
    def n_trans(self) -> int:
        return len(self.trans_A)


@dataclasses.dataclass
class Workload:
    name: str
    number: int
    n: int                       # cells per axis
    beta_max: float              # cube half-width, v/c
    t_exp: float                 # s
    rho: np.ndarray              # f64 [C] g cm^-3
    tau_scale: np.ndarray        # f32 [C] synthetic line-opacity scale (rho/rho_bar)
    cell_photons: np.ndarray     # f64 [C] photons s^-1 emitted by the cell
    cell_packets: np.ndarray     # int32 [C] packets emitted by the cell (sampling plan)
    line_lambda: np.ndarray      # f64 [L] cm, ascending
    line_tau0: np.ndarray        # f32 [L]
    lambda_lo: float             # emission band, cm
    lambda_hi: float
    n_packets: int
    seed: int
    atom: Optional[Atom] = None
    T_e: Optional[np.ndarray] = None        # f64 [C] K
    n_e: Optional[np.ndarray] = None        # f64 [C] cm^-3
    n_species: Optional[np.ndarray] = None  # f64 [C*S] cm^-3
    gamma_ion: Optional[np.ndarray] = None  # f64 [C*S*3] s^-1 (stage z -> z+1, any level)
    deposition: Optional[np.ndarray] = None # f64 [C] erg s^-1 cm^-3 (gamma-ray deposition)
    couple_lines: bool = False              # atom lines take tau from populations

    @property
    def n_cells(self) -> int:
        return self.n ** 3

    @property
    def n_lines(self) -> int:
        return len(self.line_lambda)

    @property
    def h(self) -> float:
        return 2.0 * self.beta_max / self.n


def cell_centres(n: int, beta_max: float) -> np.ndarray:
    """[C,3] cell-centre coordinates in x = v/c, cell = i + n*(j + n*k)."""
    h = 2.0 * beta_max / n
    c = -beta_max + (np.arange(n) + 0.5) * h
    k, j, i = np.meshgrid(c, c, c, indexing="ij")
    return np.stack([i.ravel(), j.ravel(), k.ravel()], axis=1)


def largest_remainder(weights: np.ndarray, total: int) -> np.ndarray:
    """Integer counts proportional to weights that sum to `total` (Hamilton's method)."""
    w = np.asarray(weights, dtype=np.float64)
    s = w.sum()
    if total == 0 or s <= 0:
        return np.zeros(len(w), dtype=np.int32)
    quota = w * (total / s)
    base = np.floor(quota).astype(np.int64)
    short = int(total - base.sum())
    if short > 0:
        frac = quota - base
        order = np.argsort(-frac, kind="stable")
        base[order[:short]] += 1
    return base.astype(np.int32)


def _lognormal_unit_mean(g: np.random.Generator, sd: float, size) -> np.ndarray:
    s = np.sqrt(np.log1p(sd * sd))
    return g.lognormal(mean=-0.5 * s * s, sigma=s, size=size)


def _log_uniform(g, lo, hi, size):
    return 10.0 ** g.uniform(np.log10(lo), np.log10(hi), size=size)


def make_atom(workload: int, ion_levels, masses, e_max_ev, lines_available: int,
              a_range=(1e-3, 1e8), q_range=(1e-10, 1e-7), alpha_range=(1e-13, 1e-11),
              line_lambda: Optional[np.ndarray] = None) -> Atom:
    """Synthetic atom: every species has the given levels per ion stage.

    All level pairs within an ion stage are transitions. A is log-uniform in
    a_range; the collision strength is set so that the downward rate
    coefficient at 5000 K is log-uniform in q_range. Each transition is mapped
    to a distinct line of the line list (its wavelength is that line's).
    """
    g = rng(workload, STREAM_ATOM)
    S = len(masses)
    offs = [0]
    ion, en, gw = [], [], []
    tl, tu = [], []
    for s in range(S):
        base = offs[-1]
        for z, nl in enumerate(ion_levels):
            first = base + sum(ion_levels[:z])
            e = np.sort(g.uniform(0.0, e_max_ev, size=nl - 1)) * EV
            ion += [z] * nl
            en += [0.0] + list(e)
            gw += list(g.integers(1, 10, size=nl).astype(np.float64))
            for lo in range(nl):
                for up in range(lo + 1, nl):
                    tl.append(first + lo)
                    tu.append(first + up)
        offs.append(base + sum(ion_levels))
    T = len(tl)
    A = _log_uniform(g, *a_range, T)
    q5000 = _log_uniform(g, *q_range, T)
    gw_a = np.array(gw)
    ups = q5000 * gw_a[np.array(tu)] * np.sqrt(5000.0) / 8.629e-6
    if T > lines_available:
        raise ValueError("not enough lines for the atom's transitions")
    tline = np.sort(g.choice(lines_available, size=T, replace=False)).astype(np.int32)
    # shuffle which transition owns which line, keyed by the atom stream
    tline = tline[g.permutation(T)]
    alpha = np.zeros(S * 3)
    for s in range(S):
        for z in range(len(ion_levels) - 1):
            alpha[s * 3 + z] = _log_uniform(g, *alpha_range, 1)[0]
    atom = Atom(
        species_offset=np.array(offs, dtype=np.int32),
        level_ion=np.array(ion, dtype=np.int32),
        level_energy=np.array(en, dtype=np.float64),
        level_g=gw_a,
        trans_lower=np.array(tl, dtype=np.int32),
        trans_upper=np.array(tu, dtype=np.int32),
        trans_A=A,
        trans_lambda=np.zeros(T) if line_lambda is None else line_lambda[tline].copy(),
        trans_upsilon=ups,
        trans_line=tline,
        ion_alpha0=alpha,
        species_mass=np.array(masses, dtype=np.float64),
    )
    return atom


def ion_energies(workload: int, atom: Atom, chi_lo_ev: float = 0.5,
                 chi_hi_ev: float = 2.0) -> np.ndarray:
    """Ionisation energy (erg) of each (species, stage) [S*3], from the stage's
    ground to the next stage's ground, for photoionisation: the stage's highest
    level plus a binding energy log-uniform in [chi_lo_ev, chi_hi_ev] eV, so
    that the thresholds of the stage's levels spread from the far ultraviolet
    (the ground) into the optical and near infrared (the highest levels). The
    top stage of each species gets 0 (no ionisation from it). Drawn from its
    own Philox stream, so the other inputs of the workload are unchanged."""
    g = rng(workload, STREAM_PHOTOION)
    S = atom.n_species
    out = np.zeros(S * 3)
    for s in range(S):
        b, e = atom.species_offset[s], atom.species_offset[s + 1]
        ion = atom.level_ion[b:e]
        top = int(ion.max())
        for z in range(top):
            e_top = atom.level_energy[b:e][ion == z].max()
            out[s * 3 + z] = e_top + _log_uniform(g, chi_lo_ev, chi_hi_ev, 1)[0] * EV
    return out


def _cell_states(wl, number, rho, active, atom, T_range, mass_fractions):
    """The atom's per-cell state on workload wl (cube or spherical grid):
    T_e, species and electron densities, non-thermal ionisation rates and
    gamma-ray deposition, drawn from the cell-state stream."""
    S = atom.n_species
    gc = rng(number, STREAM_CELLS)
    C = len(rho)
    lo, hi = T_range
    T_e = np.where(active, 10.0 ** gc.uniform(np.log10(lo), np.log10(hi), size=C), lo)
    # mass fractions vary per cell around the given means (first species
    # uniform within +-0.2 of its mean, the rest in proportion)
    X = np.tile(np.asarray(mass_fractions, float), (C, 1))
    if S > 1:
        x0 = np.clip(X[:, 0] + gc.uniform(-0.2, 0.2, C), 0.05, 0.95)
        rest = X[:, 1:] / X[:, 1:].sum(axis=1, keepdims=True)
        X = np.column_stack([x0, (1.0 - x0)[:, None] * rest])
    n_sp = np.zeros((C, S))
    for s in range(S):
        n_sp[:, s] = X[:, s] * rho / (atom.species_mass[s] * M_U)
    n_e = 0.5 * n_sp.sum(axis=1)
    # gamma-ray deposition ~ rho times lognormal scatter (sigma_ln ~ 1); non-thermal
    # ionisation per atom ~ deposition per atom, with one constant per
    # (species, stage) drawn log-uniformly, scaled so that the rates span
    # about 1e-7..1e-3 s^-1 over the cells
    dep = np.where(active, rho * _lognormal_unit_mean(gc, 1.3, C), 0.0)
    per_atom = np.where(active, dep / np.maximum(n_sp.sum(axis=1), 1e-300), 0.0)
    ref = np.median(per_atom[active]) if active.any() else 1.0
    gam = np.zeros((C, S, 3))
    nz = int(atom.level_ion.max()) + 1
    if nz > 1:
        kz = _log_uniform(gc, 1e-6, 1e-4, (S, nz - 1))
        gam[:, :, : nz - 1] = kz[None, :, :] * (per_atom / ref)[:, None, None]
    dep_scale = 1e-7 / max(np.median(dep[active]) if active.any() else 1.0, 1e-300)
    wl.deposition = dep * dep_scale
    wl.atom = atom
    wl.T_e = T_e
    wl.n_e = n_e
    wl.n_species = n_sp.ravel()
    wl.gamma_ion = gam.ravel()


def _finish(name, number, n, beta_max, t_exp, rho, lines_lo_A, lines_hi_A, n_lines,
            tau_lo, tau_hi, n_packets, photons_total, atom_spec, T_range,
            couple_lines, mass_fractions):
    g_lines = rng(number, STREAM_LINES)
    lam = np.sort(g_lines.uniform(lines_lo_A, lines_hi_A, size=n_lines)) * ANGSTROM
    tau0 = _log_uniform(g_lines, tau_lo, tau_hi, n_lines).astype(np.float32)
    active = rho > 0
    rho_bar = rho[active].mean()
    tau_scale = (rho / rho_bar).astype(np.float32)
    w = rho / rho.sum()
    cell_photons = photons_total * w
    cell_packets = largest_remainder(w, n_packets)
    wl = Workload(name=name, number=number, n=n, beta_max=beta_max, t_exp=t_exp, rho=rho,
                  tau_scale=tau_scale, cell_photons=cell_photons, cell_packets=cell_packets,
                  line_lambda=lam, line_tau0=tau0, lambda_lo=lines_lo_A * ANGSTROM,
                  lambda_hi=lines_hi_A * ANGSTROM, n_packets=n_packets,
                  seed=packet_seed(number), couple_lines=couple_lines)
    if atom_spec is not None:
        atom = make_atom(number, line_lambda=lam, lines_available=n_lines, **atom_spec)
        _cell_states(wl, number, rho, active, atom, T_range, mass_fractions)
    return wl


def sphere_small() -> Workload:
    """16^3 cube around a homologous sphere, v_max 5000 km/s, t = 200 d.

    Cells whose centre lies outside the sphere are empty (2176 active cells).
    rho ~ |v|^-2 times 10 % lognormal noise, 1 M_sun of ejecta. 200 lines in
    3000-10000 A with tau0 log-uniform in 1e-3..1e3 scaled by rho/rho_bar.
    1e5 packets emitted in 3000-10000 A, emissivity proportional to rho*V.
    Atom: one species with one ion stage of 10 levels (45 transitions).
    """
    number = 1
    n = 16
    beta_max = 5000.0 / C_KMS
    t_exp = 200.0 * DAY
    x = cell_centres(n, beta_max)
    r = np.sqrt((x * x).sum(axis=1))
    active = r <= beta_max
    g = rng(number, STREAM_GRID)
    noise = _lognormal_unit_mean(g, 0.10, len(r))
    shape = np.where(active, noise / np.maximum(r, 1e-30) ** 2, 0.0)
    V = (2 * beta_max / n * C_CGS * t_exp) ** 3
    rho = shape * (M_SUN / (shape.sum() * V))
    return _finish("sphere16_l200_p1e5", number, n, beta_max, t_exp, rho, 3000.0, 10000.0, 200,
                   1e-3, 1e3, 100_000, 2.5e52,
                   dict(ion_levels=[10], masses=[16.0], e_max_ev=4.0),
                   (5000.0, 5000.0), False, [1.0])


def clumpy(n: int = 50, n_lines: int = 5000, n_packets: int = 10_000_000, number: int = 2,
           couple_lines: bool = True, ion_levels=(20, 15, 15)) -> Workload:
    """Clumped homologous ejecta on an n^3 cube, v_max 5000 km/s, t = 200 d.

    rho ~ |v|^-2 out to the cube corners; clumps with filling factor 0.2
    (multiplier lognormal, median 10, sigma_ln 0.5), renormalised per radial
    shell to conserve that shell's mass, times 10 % noise. Lines in
    2000-25000 A with tau0 log-uniform in 1e-4..1e4 scaled by rho/rho_bar.
    Atom: two species (mass 16 and 56), three ion stages of 20+15+15 levels.
    """
    beta_max = 5000.0 / C_KMS
    t_exp = 200.0 * DAY
    x = cell_centres(n, beta_max)
    r = np.sqrt((x * x).sum(axis=1))
    g = rng(number, STREAM_GRID)
    base = 1.0 / np.maximum(r, 1e-30) ** 2
    clump = g.random(len(r)) < 0.2
    mult = np.where(clump, 10.0 * np.exp(0.5 * g.standard_normal(len(r))), 1.0)
    shell = np.minimum((r / (np.sqrt(3.0) * beta_max) * 40).astype(int), 39)
    dens = base * mult
    for s in range(40):
        m = shell == s
        if m.any():
            dens[m] *= base[m].sum() / dens[m].sum()
    dens *= _lognormal_unit_mean(g, 0.10, len(r))
    V = (2 * beta_max / n * C_CGS * t_exp) ** 3
    rho = dens * (M_SUN / (dens.sum() * V))
    return _finish(f"clumpy{n}_l{n_lines}_p{n_packets:.0e}".replace("+0", ""), number, n, beta_max,
                   t_exp, rho, 2000.0, 25000.0, n_lines, 1e-4, 1e4, n_packets, 2.5e52,
                   dict(ion_levels=list(ion_levels), masses=[16.0, 56.0],
                        e_max_ev=10.0),
                   (2000.0, 10000.0), couple_lines, [0.7, 0.3])


def paper_scale() -> Workload:
    """Transport at the paper's scale: 50^3 cells, 5000 lines, 1e7 packets."""
    return clumpy(50, 5000, 10_000_000, number=2)


@dataclasses.dataclass
class Batched:
    """Batched NLTE problem: one element with three ion stages per cell.

    Level counts differ from cell to cell; the per-level (g, E) and per-pair
    (A, collision, photoexcitation) values are not stored. Both sides draw
    them from Philox4x64-10 with key (seed, STREAM_BATCHED) by the definition
    each side implements:
      level i of stage z in cell c: counter (c, z, i, 2^63), uniforms u0..u3
        g = 1 + floor(9 u0); E = 0 for i = 0, else 69 k T_e(c) u1
      pair l < u of stage z in cell c: counter (c, z, l, u), uniforms u0..u3
        radiative iff u0 < 0.2 with A = 10^(-3 + 11 u1) s^-1 and
        Gamma_PE = gamma_pe_table[min(n - 1, floor(u3 n))] s^-1 (n entries);
        q_down = 10^(-10 + 3 u2) cm^3 s^-1
    where uniforms are (x >> 11) * 2^-53 of the four 64-bit output words.
    The table holds the photoexcitation rates the oracle measures on the 16^3
    sphere workload (synth/make_photoexcitation_table.py writes it). This
    module holds only the stored inputs below.
    """
    name: str
    n_cells: int
    seed: int
    level_count: np.ndarray   # int32 [C*3] levels of stages 0..2 (stage 0 >= 1; 0 = absent)
    T_e: np.ndarray           # f64 [C] K
    n_e: np.ndarray           # f64 [C] cm^-3
    gamma_ion: np.ndarray     # f64 [C*2] s^-1, any level of stage z -> ground of z+1
    alpha0: np.ndarray        # f64 [2] cm^3 s^-1 at 1e4 K, recombination into stage z
    gamma_pe_table: np.ndarray  # f64 [n] s^-1, photoexcitation rates drawn from (sorted)

    @property
    def pop_offset(self) -> np.ndarray:
        n = self.level_count.reshape(-1, 3).sum(1).astype(np.int64)
        return np.concatenate([[0], np.cumsum(n)])


def photoexcitation_table() -> np.ndarray:
    """The stored photoexcitation rates of the 16^3 sphere workload (sorted,
    positive; written by make_photoexcitation_table.py with the oracle)."""
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "photoexcitation_sphere16.npy")
    return np.load(path, allow_pickle=False)


def batched(n: int = 50, lo: int = 20, hi: int = 300, number: int = 3,
            cells: Optional[int] = None) -> Batched:
    """The batched NLTE solve: cell states (T_e, n_e) of the n^3 clumpy
    workload, level counts per stage uniform in lo..hi, ionisation rates
    log-uniform in 1e-7..1e-3 s^-1. `cells` keeps only the first cells."""
    w = clumpy(n, 1000, 1000, number=2)
    C = w.n_cells if cells is None else int(cells)
    g = rng(number, STREAM_CELLS)
    counts = g.integers(lo, hi + 1, size=(w.n_cells, 3)).astype(np.int32)[:C]
    gion = _log_uniform(g, 1e-7, 1e-3, (w.n_cells, 2))[:C]
    return Batched(name=f"batched{n}_L{lo}-{hi}", n_cells=C, seed=SEED_BASE + number,
                   level_count=counts.ravel().copy(), T_e=w.T_e[:C].copy(),
                   n_e=w.n_e[:C].copy(), gamma_ion=gion.ravel().copy(),
                   alpha0=np.array([2.0e-12, 4.0e-12]), gamma_pe_table=photoexcitation_table())


def batched_custom(level_count, T_e, n_e, gamma_ion, alpha0=(2.0e-12, 4.0e-12),
                   seed: int = SEED_BASE + 3) -> Batched:
    """A batched problem with the given stored inputs (tests: small counts,
    limits)."""
    lc = np.asarray(level_count, dtype=np.int32).reshape(-1, 3)
    C = len(lc)
    return Batched(name="custom", n_cells=C, seed=int(seed), level_count=lc.ravel().copy(),
                   T_e=np.broadcast_to(np.asarray(T_e, float), (C,)).copy(),
                   n_e=np.broadcast_to(np.asarray(n_e, float), (C,)).copy(),
                   gamma_ion=np.broadcast_to(np.asarray(gamma_ion, float).reshape(-1, 2)
                                             if np.ndim(gamma_ion) else
                                             np.full((1, 2), float(gamma_ion)), (C, 2)).ravel().copy(),
                   alpha0=np.asarray(alpha0, float), gamma_pe_table=photoexcitation_table())


def large() -> Workload:
    """The streamed case: 100^3 cells, 30000 lines, 1e8 packets, same recipe."""
    return clumpy(100, 30000, 100_000_000, number=5)


@dataclasses.dataclass
class SphericalWorkload:
    """Inputs on a spherical (r, theta, phi) grid (Sec. 2): shell edges r_edge
    (x = v/c, from 0), polar edges theta_edge, n_phi equal azimuthal slices;
    cell c = i_r + n_r (i_theta + n_theta i_phi). Per-cell arrays have
    n_r n_theta n_phi entries. Without an atom every line is a background
    line; with one (spherical(atom=True)) its transitions take lines of the
    list and the cells carry the atom's state, as on the cube."""
    name: str
    number: int
    r_edge: np.ndarray
    theta_edge: np.ndarray
    n_phi: int
    t_exp: float
    rho: np.ndarray
    tau_scale: np.ndarray
    cell_photons: np.ndarray
    cell_packets: np.ndarray
    line_lambda: np.ndarray
    line_tau0: np.ndarray
    lambda_lo: float
    lambda_hi: float
    n_packets: int
    seed: int
    atom: Optional[Atom] = None
    T_e: Optional[np.ndarray] = None
    n_e: Optional[np.ndarray] = None
    n_species: Optional[np.ndarray] = None
    gamma_ion: Optional[np.ndarray] = None
    deposition: Optional[np.ndarray] = None

    @property
    def n_r(self) -> int:
        return len(self.r_edge) - 1

    @property
    def n_theta(self) -> int:
        return len(self.theta_edge) - 1

    @property
    def n_cells(self) -> int:
        return self.n_r * self.n_theta * self.n_phi

    @property
    def n_lines(self) -> int:
        return len(self.line_lambda)

    def cell_volumes(self) -> np.ndarray:
        """Physical cell volumes (cm^3) in cell order."""
        r3 = (self.r_edge[1:] ** 3 - self.r_edge[:-1] ** 3) / 3.0
        ct = np.cos(self.theta_edge[:-1]) - np.cos(self.theta_edge[1:])
        v = (r3[:, None, None] * ct[None, :, None] * np.full(self.n_phi, 2 * np.pi / self.n_phi))
        return v.transpose(2, 1, 0).ravel() * (C_CGS * self.t_exp) ** 3


def spherical(n_r: int = 40, n_theta: int = 30, n_phi: int = 60, n_lines: int = 5000,
              n_packets: int = 10_000_000, number: int = 8, power: float = 1.5,
              atom: bool = False) -> SphericalWorkload:
    """Clumped homologous ejecta on a spherical grid, v_max 5000 km/s, t = 200 d.

    Shell edges r_i = R (i / n_r)^power (cells grow outwards, as the paper's
    grid does), polar edges uniform in theta, n_phi equal slices. rho ~
    |v|^-2 at the cell's middle radius; clumps with filling factor 0.2
    (multiplier lognormal, median 10, sigma_ln 0.5) renormalised per shell to
    conserve its mass, times 10 % noise; 1 M_sun in all. Lines in
    2000-25000 A with tau0 log-uniform in 1e-4..1e4 scaled by rho/rho_bar;
    emission proportional to mass; packets by largest remainder. With atom,
    the cube workloads' atom (two species of mass 16 and 56, three stages of
    20+15+15 levels) on these lines, and its cell state drawn as on the cube
    (T_e log-uniform in 2000-10000 K, mass fractions 0.7/0.3 +- 0.2)."""
    R = 5000.0 / C_KMS
    t_exp = 200.0 * DAY
    r_edge = R * (np.arange(n_r + 1) / n_r) ** power
    theta_edge = np.linspace(0.0, np.pi, n_theta + 1)
    g = rng(number, STREAM_GRID)
    C = n_r * n_theta * n_phi
    ir = np.arange(C) % n_r
    rm = 0.5 * (r_edge[ir] + r_edge[ir + 1])
    base = 1.0 / rm ** 2
    clump = g.random(C) < 0.2
    mult = np.where(clump, 10.0 * np.exp(0.5 * g.standard_normal(C)), 1.0)
    dens = base * mult
    sw = SphericalWorkload("", number, r_edge, theta_edge, n_phi, t_exp, np.zeros(C),
                           np.zeros(C, np.float32), np.zeros(C), np.zeros(C, np.int32),
                           np.zeros(0), np.zeros(0, np.float32), 2000e-8, 25000e-8, n_packets,
                           packet_seed(number))
    V = sw.cell_volumes()
    for i in range(n_r):
        m = ir == i
        dens[m] *= (base[m] * V[m]).sum() / (dens[m] * V[m]).sum()
    dens *= _lognormal_unit_mean(g, 0.10, C)
    rho = dens * (M_SUN / (dens * V).sum())
    gl = rng(number, STREAM_LINES)
    lam = np.sort(gl.uniform(2000.0, 25000.0, size=n_lines)) * ANGSTROM
    tau0 = _log_uniform(gl, 1e-4, 1e4, n_lines).astype(np.float32)
    mass = rho * V
    sw.name = f"sphere{n_r}x{n_theta}x{n_phi}_l{n_lines}_p{n_packets:.0e}".replace("+0", "")
    sw.rho = rho
    sw.tau_scale = (rho / rho.mean()).astype(np.float32)
    sw.cell_photons = 2.5e52 * mass / mass.sum()
    sw.cell_packets = largest_remainder(mass / mass.sum(), n_packets)
    sw.line_lambda = lam
    sw.line_tau0 = tau0
    if atom:
        a = make_atom(number, line_lambda=lam, lines_available=n_lines, ion_levels=[20, 15, 15],
                      masses=[16.0, 56.0], e_max_ev=10.0)
        _cell_states(sw, number, rho, np.ones(C, bool), a, (2000.0, 10000.0), [0.7, 0.3])
        sw.name += "_atom"
    return sw


def workload_by_name(name: str) -> Workload:
    table = {"sphere16": sphere_small, "clumpy50": paper_scale, "clumpy100": large}
    return table[name]()
