"""FP64 CPU oracle for the ExTraSS hot path: ctypes wrapper over liboracle.so.

TEST INFRASTRUCTURE. Only tests/, __graft_entry__.smoke() and bench.py's
cpu_baseline leg may import this package. The product path (the HIP library
in paper_2511_07539_amd/) never imports it, and the two share no code.

Functions whose parity is not pinned by an independent check say so in their
docstring ("parity unpinned").
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")
_lib = None

PKT_FIELDS = 12
N_STATS = 10
STAT_NAMES = ["w_emit", "w_esc", "w_kill", "w_abs", "n_inter", "n_checks", "n_cross",
              "n_escaped", "n_killed", "w_pi"]


class _Sphere(C.Structure):
    _fields_ = [("n_r", C.c_int32), ("n_theta", C.c_int32), ("n_phi", C.c_int32),
                ("r_edge", C.c_void_p), ("theta_edge", C.c_void_p)]


class _Transport(C.Structure):
    _fields_ = [
        ("n", C.c_int32), ("beta_max", C.c_double),
        ("tau_scale", C.c_void_p), ("cell_photons", C.c_void_p), ("cell_packets", C.c_void_p),
        ("n_lines", C.c_int32), ("line_lambda", C.c_void_p), ("line_tau0", C.c_void_p),
        ("line_trans", C.c_void_p), ("n_trans", C.c_int32), ("tau_ct", C.c_void_p),
        ("fcorr_ct", C.c_void_p), ("lambda_lo", C.c_double), ("lambda_hi", C.c_double),
        ("seed", C.c_uint64), ("iteration", C.c_int32), ("explicit_packets", C.c_void_p),
        ("pi_levels", C.c_int32), ("pi_lambda", C.c_void_p), ("pi_sigma0", C.c_void_p),
        ("pi_level", C.c_void_p), ("pi_nlev", C.c_int32), ("pi_pops", C.c_void_p),
        ("pi_length", C.c_double), ("pi_absorbed", C.c_void_p),
        ("sphere", C.c_void_p),
    ]


class _Record(C.Structure):
    _fields_ = [("packet", C.c_int64), ("cell", C.c_int32), ("line", C.c_int32),
                ("value", C.c_double), ("margin", C.c_double)]


class _Atom(C.Structure):
    _fields_ = [
        ("n_species", C.c_int32), ("species_offset", C.c_void_p), ("n_levels", C.c_int32),
        ("level_ion", C.c_void_p), ("level_energy", C.c_void_p), ("level_g", C.c_void_p),
        ("n_trans", C.c_int32), ("trans_lower", C.c_void_p), ("trans_upper", C.c_void_p),
        ("trans_A", C.c_void_p), ("trans_lambda", C.c_void_p), ("trans_upsilon", C.c_void_p),
        ("ion_alpha0", C.c_void_p),
    ]


class _Cells(C.Structure):
    _fields_ = [
        ("t_exp", C.c_double), ("T_e", C.c_void_p), ("n_e", C.c_void_p),
        ("n_species", C.c_void_p), ("gamma_ion", C.c_void_p), ("gamma_pe", C.c_void_p),
        ("gamma_pi", C.c_void_p),
    ]


class _Batched(C.Structure):
    _fields_ = [("n_cells", C.c_int64), ("seed", C.c_uint64), ("level_count", C.c_void_p),
                ("T_e", C.c_void_p), ("n_e", C.c_void_p), ("gamma_ion", C.c_void_p),
                ("alpha0", C.c_double * 2), ("gpe_table", C.c_void_p), ("n_gpe", C.c_int64)]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from . import build as _b
            _b.build()
        L = C.CDLL(LIB_PATH)
        L.oracle_philox4x64.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p]
        L.oracle_transport.restype = C.c_int64
        L.oracle_transport.argtypes = [C.POINTER(_Transport), C.c_int64, C.c_int64, C.c_int,
                                       C.POINTER(C.POINTER(_Record)), C.c_void_p, C.c_void_p]
        L.oracle_free.argtypes = [C.c_void_p]
        L.oracle_emission.restype = C.c_int
        L.oracle_emission.argtypes = [C.POINTER(_Transport), C.c_int64, C.c_int64, C.c_void_p]
        L.oracle_line_tau.argtypes = [C.c_int64, C.c_int32, C.c_int32] + [C.c_void_p] * 6 + \
            [C.c_double, C.c_void_p, C.c_void_p]
        L.oracle_rates.argtypes = [C.c_int64, C.c_int32, C.c_int32, C.c_int32] + [C.c_void_p] * 4 + \
            [C.c_double, C.c_void_p, C.c_void_p]
        L.oracle_nlte.restype = C.c_int
        L.oracle_nlte.argtypes = [C.POINTER(_Atom), C.POINTER(_Cells), C.c_int64, C.c_int64,
                                  C.c_int, C.c_int, C.c_double, C.c_int, C.c_void_p, C.c_void_p,
                                  C.c_void_p]
        L.oracle_nlte_cold.argtypes = [C.POINTER(_Atom), C.POINTER(_Cells), C.c_int64, C.c_void_p]
        L.oracle_rate_matrix.argtypes = [C.POINTER(_Atom), C.POINTER(_Cells), C.c_int64, C.c_int32,
                                         C.c_void_p, C.c_void_p]
        L.oracle_gth.argtypes = [C.c_int32, C.c_void_p, C.c_void_p]
        L.oracle_emission_bins.argtypes = [C.POINTER(_Atom), C.c_int64, C.c_void_p, C.c_double,
                                           C.c_double, C.c_void_p, C.c_double, C.c_double,
                                           C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p]
        L.oracle_ray_packets.restype = C.c_int64
        L.oracle_ray_packets.argtypes = [C.c_int32, C.c_double, C.c_void_p, C.c_int64, C.c_int64,
                                         C.c_int32, C.c_void_p, C.c_void_p, C.c_int32, C.c_int32,
                                         C.POINTER(C.POINTER(C.c_double))]
        L.oracle_sphere_cell.restype = C.c_int64
        L.oracle_sphere_cell.argtypes = [C.POINTER(_Sphere), C.c_void_p]
        L.oracle_sphere_crossings.restype = C.c_int32
        L.oracle_sphere_crossings.argtypes = [C.POINTER(_Sphere), C.c_void_p, C.c_void_p,
                                              C.c_void_p, C.c_int32]
        L.oracle_pi_levels.restype = C.c_int32
        L.oracle_pi_levels.argtypes = [C.POINTER(_Atom), C.c_void_p, C.c_int32, C.c_void_p,
                                       C.c_void_p, C.c_void_p]
        L.oracle_batched_matrix.argtypes = [C.POINTER(_Batched), C.c_int64, C.c_void_p]
        L.oracle_batched.restype = C.c_int64
        L.oracle_batched.argtypes = [C.POINTER(_Batched), C.c_void_p, C.c_int64, C.c_int64,
                                     C.c_int, C.c_void_p]
        _lib = L
    return _lib


def default_threads():
    """Host threads for the oracle: OMP_NUM_THREADS if set, else at most 16."""
    env = os.environ.get("OMP_NUM_THREADS")
    n = int(env) if env and env.isdigit() else 16
    return max(1, min(n, os.cpu_count() or 1))


def _p(a):
    return None if a is None else a.ctypes.data


def _keep(*arrays):
    return [np.ascontiguousarray(a) if a is not None else None for a in arrays]


def philox4x64(ctr, key):
    c = np.array(ctr, dtype=np.uint64)
    k = np.array(key, dtype=np.uint64)
    out = np.zeros(4, dtype=np.uint64)
    lib().oracle_philox4x64(_p(c), _p(k), _p(out))
    return out


class TransportInputs:
    """Holds contiguous copies of every array the C structure points to."""

    def __init__(self, n, beta_max, tau_scale, cell_photons, cell_packets, line_lambda, line_tau0,
                 lambda_lo, lambda_hi, seed, iteration=0, line_trans=None, tau_ct=None,
                 fcorr_ct=None, explicit_packets=None, photoion=None, sphere=None):
        """photoion: None, or a dict with the photoionising levels of
        pi_levels() (level, lambda, sigma0), the populations pops [C, N] in
        cm^-3 and length = c t_exp; transport() then also returns each
        (cell, level)'s absorbed photons. sphere: None, or a Sphere (the
        spherical grid; n and beta_max are then unused)."""
        self.arrays = dict(
            tau_scale=np.ascontiguousarray(tau_scale, dtype=np.float32),
            cell_photons=np.ascontiguousarray(cell_photons, dtype=np.float64),
            cell_packets=np.ascontiguousarray(cell_packets, dtype=np.int32),
            line_lambda=np.ascontiguousarray(line_lambda, dtype=np.float64),
            line_tau0=np.ascontiguousarray(line_tau0, dtype=np.float32),
            line_trans=None if line_trans is None else np.ascontiguousarray(line_trans, np.int32),
            tau_ct=None if tau_ct is None else np.ascontiguousarray(tau_ct, np.float64),
            fcorr_ct=None if fcorr_ct is None else np.ascontiguousarray(fcorr_ct, np.float64),
            explicit=None if explicit_packets is None else
            np.ascontiguousarray(explicit_packets, np.float64).reshape(-1, 8),
        )
        a = self.arrays
        self.sphere = sphere
        self.n_cells = sphere.n_cells if sphere is not None else n ** 3
        n_trans = 0 if a["tau_ct"] is None else a["tau_ct"].size // self.n_cells
        self.n_lines = len(a["line_lambda"])
        self.s = _Transport(n, beta_max, _p(a["tau_scale"]), _p(a["cell_photons"]),
                            _p(a["cell_packets"]), self.n_lines, _p(a["line_lambda"]),
                            _p(a["line_tau0"]), _p(a["line_trans"]), n_trans, _p(a["tau_ct"]),
                            _p(a["fcorr_ct"]), lambda_lo, lambda_hi, seed, iteration,
                            _p(a["explicit"]))
        if sphere is not None:
            self.s.sphere = C.addressof(sphere.s)
        self.pi_levels = 0
        if photoion is not None:
            a["pi_lambda"] = np.ascontiguousarray(photoion["lambda"], np.float64)
            a["pi_sigma0"] = np.ascontiguousarray(photoion["sigma0"], np.float64)
            a["pi_level"] = np.ascontiguousarray(photoion["level"], np.int32)
            pops = np.ascontiguousarray(photoion["pops"], np.float64).reshape(self.n_cells, -1)
            a["pi_pops"] = pops
            self.pi_levels = len(a["pi_lambda"])
            a["pi_absorbed"] = np.zeros((self.n_cells, self.pi_levels))
            self.s.pi_levels = self.pi_levels
            self.s.pi_lambda = _p(a["pi_lambda"])
            self.s.pi_sigma0 = _p(a["pi_sigma0"])
            self.s.pi_level = _p(a["pi_level"])
            self.s.pi_nlev = pops.shape[1]
            self.s.pi_pops = _p(pops)
            self.s.pi_length = float(photoion["length"])
            self.s.pi_absorbed = _p(a["pi_absorbed"])

    @property
    def n_packets(self):
        if self.arrays["explicit"] is not None:
            return len(self.arrays["explicit"])
        return int(self.arrays["cell_packets"].astype(np.int64).sum())


class Sphere:
    """Spherical grid (the paper's (r, theta, phi) cells): shell edges r_edge
    [n_r + 1] in x = v/c from 0, polar edges theta_edge [n_theta + 1] from 0
    to pi, n_phi equal azimuthal slices; cell i_r + n_r (i_theta + n_theta
    i_phi)."""

    def __init__(self, r_edge, theta_edge, n_phi):
        self.r_edge = np.ascontiguousarray(r_edge, np.float64)
        self.theta_edge = np.ascontiguousarray(theta_edge, np.float64)
        self.n_r, self.n_theta, self.n_phi = len(self.r_edge) - 1, len(self.theta_edge) - 1, int(n_phi)
        self.n_cells = self.n_r * self.n_theta * self.n_phi
        self.s = _Sphere(self.n_r, self.n_theta, self.n_phi, _p(self.r_edge), _p(self.theta_edge))

    def cell(self, x):
        xx = np.ascontiguousarray(x, np.float64)
        return int(lib().oracle_sphere_cell(C.byref(self.s), _p(xx)))

    def crossings(self, x0, n):
        a = np.ascontiguousarray(x0, np.float64)
        b = np.ascontiguousarray(n, np.float64)
        cap = 2 * self.n_r + 2 * self.n_theta + self.n_phi + 4
        out = np.zeros(cap)
        m = lib().oracle_sphere_crossings(C.byref(self.s), _p(a), _p(b), _p(out), cap)
        return out[:m].copy()

    def middles(self):
        """The middle of every cell [C, 3] in cell order: mid-radius, mid-angle
        of the polar bin and mid-slice (where the deterministic rays start)."""
        rm = 0.5 * (self.r_edge[:-1] + self.r_edge[1:])
        tm = 0.5 * (self.theta_edge[:-1] + self.theta_edge[1:])
        pm = (np.arange(self.n_phi) + 0.5) * 2 * np.pi / self.n_phi
        R, T, P = np.meshgrid(rm, tm, pm, indexing="ij")  # [n_r, n_theta, n_phi]
        x = np.stack([R * np.sin(T) * np.cos(P), R * np.sin(T) * np.sin(P), R * np.cos(T)], -1)
        return np.ascontiguousarray(x.transpose(2, 1, 0, 3).reshape(-1, 3))

    def volumes(self, scale=1.0):
        """Cell volumes [C] in (scale x)^3 units: (r_b^3 - r_a^3)/3 (cos th_a -
        cos th_b) dphi."""
        r3 = (self.r_edge[1:] ** 3 - self.r_edge[:-1] ** 3) / 3.0
        ct = np.cos(self.theta_edge[:-1]) - np.cos(self.theta_edge[1:])
        v = r3[:, None, None] * ct[None, :, None] * np.full(self.n_phi, 2 * np.pi / self.n_phi)
        return (v.transpose(2, 1, 0).ravel()) * scale ** 3


def transport_inputs_from_workload(w, iteration=0, tau_ct=None, fcorr_ct=None):
    line_trans = None
    if tau_ct is not None:
        line_trans = np.full(w.n_lines, -1, dtype=np.int32)
        line_trans[w.atom.trans_line] = np.arange(w.atom.n_trans, dtype=np.int32)
    return TransportInputs(w.n, w.beta_max, w.tau_scale, w.cell_photons, w.cell_packets,
                           w.line_lambda, w.line_tau0, w.lambda_lo, w.lambda_hi, w.seed,
                           iteration, line_trans, tau_ct, fcorr_ct)


def transport(inp: TransportInputs, first=0, count=None, nthreads=None, per_packet=False):
    """Runs the oracle over packets [first, first+count).

    Returns dict(records=(packet, cell, line, value) structured array in packet
    order, stats=dict, packets=[count, 12] per-packet results if per_packet,
    pi_absorbed=[C, M] photons absorbed per (cell, photoionising level) when the
    inputs have photoionisation; the run is then serial).
    """
    if count is None:
        count = inp.n_packets - first
    if nthreads is None:
        nthreads = default_threads()
    stats = np.zeros(N_STATS)
    pk = np.zeros((count, PKT_FIELDS)) if per_packet else None
    ptr = C.POINTER(_Record)()
    nrec = lib().oracle_transport(C.byref(inp.s), first, count, nthreads, C.byref(ptr),
                                  _p(stats), _p(pk))
    if nrec < 0:
        raise ValueError("oracle_transport: invalid input")
    dt = np.dtype([("packet", np.int64), ("cell", np.int32), ("line", np.int32),
                   ("value", np.float64), ("margin", np.float64)])
    if nrec > 0:
        buf = (C.c_char * (nrec * dt.itemsize)).from_address(C.addressof(ptr.contents))
        recs = np.frombuffer(buf, dtype=dt).copy()
    else:
        recs = np.zeros(0, dtype=dt)
    lib().oracle_free(ptr)
    out = dict(records=recs, stats=dict(zip(STAT_NAMES, stats)), packets=pk)
    if inp.pi_levels:
        out["pi_absorbed"] = inp.arrays["pi_absorbed"].copy()
        inp.arrays["pi_absorbed"][:] = 0.0
    return out


def emission(inp: TransportInputs, first=0, count=None):
    """Emitted state of packets [first, first+count): [count, 8] rows of
    (x, y, z, n_x, n_y, n_z, lambda_e, w0), as the transport draws them."""
    if count is None:
        count = inp.n_packets - first
    out = np.zeros((count, 8))
    if lib().oracle_emission(C.byref(inp.s), first, count, _p(out)) != 0:
        raise ValueError("oracle_emission: invalid input")
    return out


def pi_levels(inp: "NLTEInputs", ion_energy, max_per_stage=25):
    """Photoionising levels (Sec. 2.3.1; Eq. A5): dict(level, lambda, sigma0)
    as oracle_pi_levels selects them (oracle.h). ion_energy [S*3] erg."""
    ie = np.ascontiguousarray(ion_energy, np.float64)
    n = lib().oracle_pi_levels(C.byref(inp.atom), _p(ie), max_per_stage, None, None, None)
    level = np.zeros(n, np.int32)
    lam = np.zeros(n)
    sig = np.zeros(n)
    lib().oracle_pi_levels(C.byref(inp.atom), _p(ie), max_per_stage, _p(level), _p(lam), _p(sig))
    return {"level": level, "lambda": lam, "sigma0": sig}


def pi_rates(pi_absorbed, pops, level, n_levels, cell_volume):
    """Photoionisation rate of each level, Gamma_PI = N_abs / (n V) (Sec.
    2.3.1): [C, N], zero for levels that do not photoionise."""
    ab = np.asarray(pi_absorbed, np.float64)
    P = np.asarray(pops, np.float64).reshape(len(ab), -1)
    out = np.zeros((len(ab), n_levels))
    for j, lv in enumerate(level):
        n = P[:, lv]
        out[:, lv] = np.where(n > 0, ab[:, j] / np.where(n > 0, n, 1.0) / cell_volume, 0.0)
    return out


def dense_estimator(records, n_cells, n_lines):
    """[C, L] table accumulated in packet order (deterministic)."""
    est = np.zeros(n_cells * n_lines)
    idx = records["cell"].astype(np.int64) * n_lines + records["line"]
    np.add.at(est, idx, records["value"])
    return est.reshape(n_cells, n_lines)


PLANCK_CGS = 6.62607015e-27   # erg s
LIGHT_CGS = 2.99792458e10     # cm s^-1


def spectrum(packets, n_theta, n_phi, n_lambda, lambda_min, lambda_max):
    """Emergent spectra per viewer (Sec. 2.3: rays leave towards viewers spread
    evenly in polar and azimuthal angle, 20 x 20 by default; the emergent
    emission is binned logarithmically in wavelength).

    packets: per-packet results of transport(..., per_packet=True). Every
    escaped packet (field 0, the escaped weight w, > 0) falls in the viewer
    bin of its lab-frame direction (fields 8-10): theta = arccos(n_z) in
    n_theta equal bins of [0, pi], phi = atan2(n_y, n_x) taken into
    [0, 2 pi) in n_phi equal bins; and in the wavelength bin
    floor(n_lambda ln(lambda_L / lambda_min) / ln(lambda_max / lambda_min))
    of its lab wavelength (field 1) when lambda_min <= lambda_L < lambda_max.
    Returns (photons, energy), each [n_theta, n_phi, n_lambda]: the sums of w
    and of w h c / lambda_L (erg s^-1), packets in order."""
    pk = np.asarray(packets, dtype=np.float64)
    photons = np.zeros((n_theta, n_phi, n_lambda))
    energy = np.zeros((n_theta, n_phi, n_lambda))
    inv_dlog = n_lambda / np.log(lambda_max / lambda_min)
    for r in pk:
        w, lam = r[0], r[1]
        if not w > 0.0 or not (lambda_min <= lam < lambda_max):
            continue
        b = min(max(int(np.floor(np.log(lam / lambda_min) * inv_dlog)), 0), n_lambda - 1)
        theta = np.arccos(min(1.0, max(-1.0, r[10])))
        it = min(max(int(np.floor(theta * (n_theta / np.pi))), 0), n_theta - 1)
        phi = np.arctan2(r[9], r[8])
        if phi < 0.0:
            phi += 2.0 * np.pi
        ip = min(max(int(np.floor(phi * (n_phi / (2.0 * np.pi)))), 0), n_phi - 1)
        photons[it, ip, b] += w
        energy[it, ip, b] += w * (PLANCK_CGS * LIGHT_CGS / lam)
    return photons, energy


def line_tau(pops, atom, t_exp):
    """Eq. A2 optical depth and stimulated-emission factor for every (cell, transition)."""
    pops = np.ascontiguousarray(pops, dtype=np.float64)
    C_ = pops.size // atom.n_levels
    tau = np.zeros(C_ * atom.n_trans)
    fc = np.zeros(C_ * atom.n_trans)
    lo, up, A, lam, g = _keep(atom.trans_lower, atom.trans_upper, atom.trans_A, atom.trans_lambda,
                              atom.level_g)
    lib().oracle_line_tau(C_, atom.n_levels, atom.n_trans, _p(pops), _p(lo), _p(up), _p(A),
                          _p(lam), _p(g), t_exp, _p(tau), _p(fc))
    return tau, fc


def rates(est, pops, atom, cell_volume):
    """Photoexcitation rate per atom in the lower level [C*T]: est / (n_l V),
    cell_volume one volume for every cell or an array of each cell's."""
    est = np.ascontiguousarray(est, dtype=np.float64)
    pops = np.ascontiguousarray(pops, dtype=np.float64)
    C_ = pops.size // atom.n_levels
    L = est.size // C_
    out = np.zeros(C_ * atom.n_trans)
    lo, tl = _keep(atom.trans_lower, atom.trans_line)
    vols = np.ascontiguousarray(cell_volume, dtype=np.float64) if np.ndim(cell_volume) else None
    lib().oracle_rates(C_, L, atom.n_levels, atom.n_trans, _p(est), _p(pops), _p(lo), _p(tl),
                       0.0 if vols is not None else float(cell_volume),
                       _p(vols) if vols is not None else None, _p(out))
    return out


class NLTEInputs:
    def __init__(self, atom, t_exp, T_e, n_e, n_species, gamma_ion, gamma_pe=None, gamma_pi=None):
        self.k = dict(
            off=np.ascontiguousarray(atom.species_offset, np.int32),
            ion=np.ascontiguousarray(atom.level_ion, np.int32),
            E=np.ascontiguousarray(atom.level_energy, np.float64),
            g=np.ascontiguousarray(atom.level_g, np.float64),
            lo=np.ascontiguousarray(atom.trans_lower, np.int32),
            up=np.ascontiguousarray(atom.trans_upper, np.int32),
            A=np.ascontiguousarray(atom.trans_A, np.float64),
            lam=np.ascontiguousarray(atom.trans_lambda, np.float64),
            ups=np.ascontiguousarray(atom.trans_upsilon, np.float64),
            alpha=np.ascontiguousarray(atom.ion_alpha0, np.float64),
            T=np.ascontiguousarray(T_e, np.float64), ne=np.ascontiguousarray(n_e, np.float64),
            ns=np.ascontiguousarray(n_species, np.float64),
            gion=np.ascontiguousarray(gamma_ion, np.float64),
            gpe=None if gamma_pe is None else np.ascontiguousarray(gamma_pe, np.float64),
            gpi=None if gamma_pi is None else np.ascontiguousarray(gamma_pi, np.float64),
        )
        k = self.k
        self.n_levels = len(k["ion"])
        self.n_cells = len(k["T"])
        self.atom = _Atom(len(k["off"]) - 1, _p(k["off"]), self.n_levels, _p(k["ion"]), _p(k["E"]),
                          _p(k["g"]), len(k["A"]), _p(k["lo"]), _p(k["up"]), _p(k["A"]),
                          _p(k["lam"]), _p(k["ups"]), _p(k["alpha"]))
        self.cells = _Cells(t_exp, _p(k["T"]), _p(k["ne"]), _p(k["ns"]), _p(k["gion"]),
                            _p(k["gpe"]), _p(k["gpi"]))


def nlte_inputs_from_workload(w, gamma_pe=None, cells=None, gamma_pi=None):
    """NLTE inputs for all cells (or the given cell indices) of a workload."""
    if cells is None:
        return NLTEInputs(w.atom, w.t_exp, w.T_e, w.n_e, w.n_species, w.gamma_ion, gamma_pe,
                          gamma_pi)
    cells = np.asarray(cells)
    S = w.atom.n_species
    T = w.atom.n_trans
    N = w.atom.n_levels
    gpe = None if gamma_pe is None else gamma_pe.reshape(-1, T)[cells].ravel()
    gpi = None if gamma_pi is None else gamma_pi.reshape(-1, N)[cells].ravel()
    return NLTEInputs(w.atom, w.t_exp, w.T_e[cells], w.n_e[cells],
                      w.n_species.reshape(-1, S)[cells].ravel(),
                      w.gamma_ion.reshape(-1, S, 3)[cells].ravel(), gpe, gpi)


def nlte(inp: NLTEInputs, guess=None, max_iter=200, tol=1e-12, nthreads=None, first=0,
         count=None):
    """Solves statistical equilibrium for cells [first, first+count).

    Returns (pops [C, N], status [C], iters [C]).
    """
    if count is None:
        count = inp.n_cells - first
    if nthreads is None:
        nthreads = default_threads()
    pops = np.zeros((inp.n_cells, inp.n_levels)) if guess is None else \
        np.ascontiguousarray(guess, dtype=np.float64).reshape(inp.n_cells, inp.n_levels).copy()
    status = np.full(inp.n_cells, -1, dtype=np.int32)
    iters = np.zeros(inp.n_cells, dtype=np.int32)
    lib().oracle_nlte(C.byref(inp.atom), C.byref(inp.cells), first, count,
                      0 if guess is None else 1, max_iter, tol, nthreads, _p(pops), _p(status),
                      _p(iters))
    return pops, status, iters


def nlte_cold(inp: NLTEInputs, c: int):
    out = np.zeros(inp.n_levels)
    lib().oracle_nlte_cold(C.byref(inp.atom), C.byref(inp.cells), c, _p(out))
    return out


def rate_matrix(inp: NLTEInputs, c: int, s: int, n_local):
    off = inp.k["off"]
    Ns = int(off[s + 1] - off[s])
    n_local = np.ascontiguousarray(n_local, dtype=np.float64)
    R = np.zeros((Ns, Ns))
    lib().oracle_rate_matrix(C.byref(inp.atom), C.byref(inp.cells), c, s, _p(n_local), _p(R))
    return R


def gth(R):
    R = np.ascontiguousarray(R, dtype=np.float64)
    pi = np.zeros(len(R))
    lib().oracle_gth(len(R), _p(R), _p(pi))
    return pi


def emission_bins(inp: "NLTEInputs", pops, t_exp, cell_volume, lambda_min, lambda_max, n_lambda):
    """Line emission per cell and logarithmic wavelength bin (Sec. 2.3, Eq. A3):
    returns (energy [C, n_lambda] erg s^-1, reddest line wavelength per bin
    [n_lambda] (0 where empty), energy outside the range [C]). cell_volume is
    one volume for every cell (cm^3) or an array of each cell's volume."""
    pops = np.ascontiguousarray(pops, dtype=np.float64)
    C_ = pops.size // inp.n_levels
    E = np.zeros((C_, n_lambda))
    lam = np.zeros(n_lambda)
    out = np.zeros(C_)
    vols = None
    if np.ndim(cell_volume):
        vols = np.ascontiguousarray(cell_volume, dtype=np.float64)
        assert vols.size == C_
    lib().oracle_emission_bins(C.byref(inp.atom), C_, _p(pops), t_exp,
                               0.0 if vols is not None else float(cell_volume),
                               _p(vols) if vols is not None else None, lambda_min, lambda_max,
                               n_lambda, _p(E), _p(lam), _p(out))
    return E, lam, out


def ray_packets(n, beta_max, bin_energy, bin_lambda, n_theta, n_phi, first=0, count=None,
                sphere=None):
    """The deterministic rays of cells [first, first+count) as explicit packets
    [R, 8] (x, y, z, n_x, n_y, n_z, lambda_e, w0), cell by cell, bin by bin,
    viewer by viewer (theta-major), from the middle of each cell: the cube's
    cell centre, or with sphere (a Sphere) the middle of the spherical cell."""
    E = np.ascontiguousarray(bin_energy, dtype=np.float64)
    lam = np.ascontiguousarray(bin_lambda, dtype=np.float64)
    n_lambda = lam.size
    if count is None:
        count = E.size // n_lambda - first
    origins = None
    if sphere is not None:
        origins = np.ascontiguousarray(sphere.middles()[first:first + count])
    ptr = C.POINTER(C.c_double)()
    nr = lib().oracle_ray_packets(n, beta_max, _p(origins) if origins is not None else None,
                                  first, count, n_lambda, _p(E), _p(lam), n_theta, n_phi,
                                  C.byref(ptr))
    if nr > 0:
        buf = (C.c_double * (8 * nr)).from_address(C.addressof(ptr.contents))
        out = np.frombuffer(buf, dtype=np.float64).reshape(nr, 8).copy()
    else:
        out = np.zeros((0, 8))
    lib().oracle_free(ptr)
    return out


class BatchedInputs:
    """ctypes view of a synth.Batched problem (keeps the arrays alive)."""

    def __init__(self, b):
        self.k = dict(level_count=np.ascontiguousarray(b.level_count, dtype=np.int32),
                      T_e=np.ascontiguousarray(b.T_e, dtype=np.float64),
                      n_e=np.ascontiguousarray(b.n_e, dtype=np.float64),
                      gamma_ion=np.ascontiguousarray(b.gamma_ion, dtype=np.float64),
                      gpe_table=np.ascontiguousarray(b.gamma_pe_table, dtype=np.float64))
        self.s = _Batched(int(b.n_cells), int(b.seed), _p(self.k["level_count"]),
                          _p(self.k["T_e"]), _p(self.k["n_e"]), _p(self.k["gamma_ion"]),
                          (C.c_double * 2)(*[float(a) for a in b.alpha0]),
                          _p(self.k["gpe_table"]), len(self.k["gpe_table"]))
        self.pop_offset = np.ascontiguousarray(b.pop_offset, dtype=np.int64)
        self.n_cells = int(b.n_cells)


def batched_matrix(inp: BatchedInputs, c: int):
    """Dense rate matrix (i -> j, s^-1) of cell c, levels stage-major, ground first."""
    N = int(inp.pop_offset[c + 1] - inp.pop_offset[c])
    R = np.zeros((N, N))
    lib().oracle_batched_matrix(C.byref(inp.s), c, _p(R))
    return R


def batched(inp: BatchedInputs, first=0, count=None, nthreads=None, pops=None):
    """Stationary populations (sum 1 per cell) of cells [first, first+count),
    at pop_offset; returns (pops, number of cells with a failed reduction)."""
    if count is None:
        count = inp.n_cells - first
    if pops is None:
        pops = np.zeros(int(inp.pop_offset[-1]))
    bad = lib().oracle_batched(C.byref(inp.s), _p(inp.pop_offset), int(first), int(count),
                               int(nthreads or default_threads()), _p(pops))
    return pops, int(bad)
