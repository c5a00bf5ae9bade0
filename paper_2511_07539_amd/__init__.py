"""MI355X (gfx950) hot path of ExTraSS (arXiv 2511.07539): Python binding.

The binding only marshals arguments: it passes device pointers of torch
tensors and the current HIP stream to the C ABI of libextrass.so (declared in
include/extrass.h), where every step of the path runs in hand-written HIP
kernels. PyTorch provides device memory and streams. There is no CPU
fallback: importing this package without the built library raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libextrass.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with "
                      "`python -m paper_2511_07539_amd.build` (hipcc, gfx950)")

_lib = C.CDLL(LIB_PATH)

OK, EINVAL, ENOSPACE, EHIP, EUNSUPPORTED = 0, -1, -2, -3, -4
STATS = 16
PACKET_FIELDS = 8  # doubles per packet record (EXTRASS_PACKET_FIELDS)
STAT_NAMES = ["w_emit", "w_esc", "w_kill", "w_abs", "n_inter", "n_checks", "n_cross",
              "n_escaped", "n_killed", "e_esc", "w_pi"]
STAT_ERROR_FLAG = 15


class _Grid(C.Structure):
    _fields_ = [("n", C.c_int32), ("beta_max", C.c_double), ("tau_scale", C.c_void_p),
                ("cell_photons", C.c_void_p), ("cell_packets", C.c_void_p),
                ("n_lines", C.c_int32), ("line_lambda", C.c_void_p), ("line_tau0", C.c_void_p),
                ("line_trans", C.c_void_p), ("n_trans", C.c_int32), ("tau_ct", C.c_void_p),
                ("fcorr_ct", C.c_void_p), ("photoion", C.c_void_p), ("spherical", C.c_void_p)]


class _Spherical(C.Structure):
    _fields_ = [("n_r", C.c_int32), ("n_theta", C.c_int32), ("n_phi", C.c_int32),
                ("r_edge", C.c_void_p), ("theta_edge", C.c_void_p), ("n_domains", C.c_int32)]


class _Photoion(C.Structure):
    _fields_ = [("n_levels", C.c_int32), ("lambda_thr", C.c_void_p), ("opacity", C.c_void_p),
                ("length", C.c_double), ("tally", C.c_void_p)]


class _SpecBins(C.Structure):
    _fields_ = [("n_theta", C.c_int32), ("n_phi", C.c_int32), ("n_lambda", C.c_int32),
                ("lambda_min", C.c_double), ("lambda_max", C.c_double)]


class _Source(C.Structure):
    _fields_ = [("seed", C.c_uint64), ("iteration", C.c_int32), ("first_packet", C.c_int64),
                ("n_packets", C.c_int64), ("lambda_lo", C.c_double), ("lambda_hi", C.c_double),
                ("explicit_packets", C.c_void_p), ("geometry_fp32", C.c_int32),
                ("rays", C.c_void_p)]


class _Rays(C.Structure):
    _fields_ = [("n_theta", C.c_int32), ("n_phi", C.c_int32), ("n_bins", C.c_int32),
                ("bin_lambda", C.c_void_p), ("bin_photons", C.c_void_p)]


class _AtomDesc(C.Structure):
    _fields_ = [("n_species", C.c_int32), ("species_offset", C.c_void_p),
                ("n_levels", C.c_int32), ("level_ion", C.c_void_p), ("level_energy", C.c_void_p),
                ("level_g", C.c_void_p), ("n_trans", C.c_int32), ("trans_lower", C.c_void_p),
                ("trans_upper", C.c_void_p), ("trans_A", C.c_void_p),
                ("trans_lambda", C.c_void_p), ("trans_upsilon", C.c_void_p),
                ("trans_line", C.c_void_p), ("ion_alpha0", C.c_void_p)]


class _Cells(C.Structure):
    _fields_ = [("n_cells", C.c_int64), ("t_exp", C.c_double), ("T_e", C.c_void_p),
                ("n_e", C.c_void_p), ("n_species", C.c_void_p), ("gamma_ion", C.c_void_p),
                ("gamma_pe", C.c_void_p), ("gamma_pi", C.c_void_p)]


class _Opts(C.Structure):
    _fields_ = [("max_iter", C.c_int32), ("tol", C.c_double), ("use_guess", C.c_int32),
                ("factor_fp32", C.c_int32), ("warm_budget", C.c_int32)]


class _Batched(C.Structure):
    _fields_ = [("n_cells", C.c_int64), ("seed", C.c_uint64), ("level_count", C.c_void_p),
                ("level_count_d", C.c_void_p), ("T_e", C.c_void_p), ("n_e", C.c_void_p),
                ("gamma_ion", C.c_void_p), ("alpha0", C.c_double * 2),
                ("gamma_pe_table", C.c_void_p), ("n_gamma_pe", C.c_int64)]


class _BOpts(C.Structure):
    _fields_ = [("factor_fp32", C.c_int32), ("refine", C.c_int32), ("tol", C.c_double),
                ("panel", C.c_int32), ("per_cu", C.c_int32)]


_vp = C.c_void_p
_lib.extrass_create.argtypes = [C.POINTER(_vp), C.c_int]
_lib.extrass_destroy.argtypes = [_vp]
_lib.extrass_error_string.restype = C.c_char_p
_lib.extrass_error_string.argtypes = [C.c_int]
_lib.extrass_last_error.restype = C.c_char_p
_lib.extrass_last_error.argtypes = [_vp]
_lib.extrass_spectrum.argtypes = [_vp, _vp, C.c_int64, C.POINTER(_SpecBins), _vp, _vp, _vp]
_lib.extrass_transport_workspace.restype = C.c_size_t
_lib.extrass_transport_workspace.argtypes = [C.POINTER(_Grid), C.POINTER(_Source)]
_lib.extrass_transport.argtypes = [_vp, C.POINTER(_Grid), C.POINTER(_Source), _vp, _vp, _vp, _vp,
                                   C.c_size_t, _vp]
_lib.extrass_transport_noalloc.argtypes = [_vp, C.POINTER(_Grid), C.POINTER(_Source), _vp, _vp,
                                           _vp, _vp]
_lib.extrass_emission_plan_create.argtypes = [_vp, _vp, C.c_double, C.c_double, C.c_int32,
                                              C.POINTER(_vp)]
_lib.extrass_emission_plan_destroy.argtypes = [_vp]
_lib.extrass_emission_plan_info.argtypes = [_vp, C.POINTER(C.c_int32), _vp, _vp,
                                            C.POINTER(C.c_void_p)]
_lib.extrass_emission.argtypes = [_vp, _vp, _vp, C.POINTER(_Grid), C.c_double, _vp, _vp, _vp, _vp]
_lib.extrass_pi_plan_create.argtypes = [_vp, _vp, _vp, C.c_int32, C.POINTER(_vp)]
_lib.extrass_pi_plan_destroy.argtypes = [_vp]
_lib.extrass_pi_plan_info.argtypes = [_vp, C.POINTER(C.c_int32), _vp, _vp, _vp,
                                      C.POINTER(C.c_void_p)]
_lib.extrass_pi_opacity.argtypes = [_vp, _vp, C.c_int64, _vp, _vp, _vp]
_lib.extrass_pi_rates.argtypes = [_vp, _vp, C.POINTER(_Grid), C.c_double, _vp, _vp, _vp]
_lib.extrass_line_tau.argtypes = [_vp, _vp, C.c_int64, _vp, C.c_double, _vp, _vp, _vp]
_lib.extrass_rates.argtypes = [_vp, _vp, C.POINTER(_Grid), C.c_double, _vp, _vp, _vp, _vp]
_lib.extrass_atom_create.argtypes = [_vp, C.POINTER(_AtomDesc), C.POINTER(_vp)]
_lib.extrass_atom_destroy.argtypes = [_vp]
_lib.extrass_nlte_workspace.restype = C.c_size_t
_lib.extrass_nlte_workspace.argtypes = [_vp, C.c_int64]
_lib.extrass_nlte_solve.argtypes = [_vp, _vp, C.POINTER(_Cells), C.POINTER(_Opts), _vp, _vp, _vp,
                                    _vp, C.c_size_t, _vp]

_lib.extrass_mlp_param_count.restype = C.c_size_t
_lib.extrass_mlp_workspace.restype = C.c_size_t
_lib.extrass_mlp_workspace.argtypes = [C.c_int64]
_lib.extrass_mlp_forward.argtypes = [_vp, _vp, _vp, _vp, C.c_int64, _vp, C.c_size_t, _vp]
_lib.extrass_mlp_train_step.argtypes = [_vp, _vp, _vp, _vp, C.c_int32, C.c_float, _vp, _vp,
                                        C.c_int64, _vp, _vp, _vp, C.c_size_t, _vp]
_lib.extrass_nlte_warm_start_workspace.restype = C.c_size_t
_lib.extrass_nlte_warm_start_workspace.argtypes = [C.c_int64]
_lib.extrass_transport_streamed_workspace.restype = C.c_size_t
_lib.extrass_transport_streamed_workspace.argtypes = [C.POINTER(_Grid), C.c_int64]
_lib.extrass_transport_streamed.argtypes = [_vp, C.POINTER(_Grid), C.POINTER(_Source), _vp, _vp,
                                            C.c_double, _vp, _vp, _vp, _vp, C.c_int64, _vp,
                                            C.c_size_t, _vp]
_lib.extrass_batched_workspace.argtypes = [_vp, C.POINTER(_Batched), C.POINTER(_BOpts),
                                           C.POINTER(C.c_size_t), C.POINTER(C.c_size_t)]
_lib.extrass_batched_solve.argtypes = [_vp, C.POINTER(_Batched), C.POINTER(_BOpts), _vp, _vp, _vp,
                                       C.c_size_t, _vp]
_lib.extrass_batched_tune.argtypes = [_vp, C.POINTER(_Batched), C.POINTER(_BOpts), _vp, C.c_size_t,
                                      _vp, _vp, _vp]
_lib.extrass_mlp_features.argtypes = [_vp, _vp, C.POINTER(_Cells), _vp, _vp, _vp]
_lib.extrass_nlte_warm_start.argtypes = [_vp, _vp, C.POINTER(_Cells), _vp, _vp, _vp, _vp, _vp,
                                         C.c_size_t, _vp]

SYMBOLS = ["extrass_create", "extrass_destroy", "extrass_error_string", "extrass_last_error",
           "extrass_transport_workspace", "extrass_transport", "extrass_line_tau",
           "extrass_rates", "extrass_atom_create", "extrass_atom_destroy",
           "extrass_nlte_workspace", "extrass_nlte_solve", "extrass_mlp_param_count",
           "extrass_mlp_workspace", "extrass_mlp_forward", "extrass_mlp_train_step",
           "extrass_nlte_warm_start_workspace", "extrass_nlte_warm_start",
           "extrass_batched_workspace", "extrass_batched_solve", "extrass_batched_tune",
           "extrass_transport_streamed_workspace", "extrass_transport_streamed",
           "extrass_mlp_features", "extrass_spectrum", "extrass_transport_noalloc",
           "extrass_emission_plan_create", "extrass_emission_plan_destroy",
           "extrass_emission_plan_info", "extrass_emission", "extrass_pi_plan_create",
           "extrass_pi_plan_destroy", "extrass_pi_plan_info", "extrass_pi_opacity",
           "extrass_pi_rates"]


class ExtrassError(RuntimeError):
    pass


def _ptr(t):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("extrass expects device tensors")
    if not t.is_contiguous():
        raise ValueError("extrass expects contiguous tensors")
    return t.data_ptr()


def _stream():
    return torch.cuda.current_stream().cuda_stream


class Context:
    """A library handle bound to one HIP device."""

    def __init__(self, device: int = 0):
        self.device = device
        h = _vp()
        rc = _lib.extrass_create(C.byref(h), device)
        if rc != OK:
            raise ExtrassError(f"extrass_create: {_lib.extrass_error_string(rc).decode()}")
        self.h = h
        self._ws = None

    def close(self):
        if self.h:
            _lib.extrass_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def check(self, rc, what):
        if rc != OK:
            detail = _lib.extrass_last_error(self.h).decode()
            raise ExtrassError(f"{what}: {_lib.extrass_error_string(rc).decode()} ({detail})")

    def workspace(self, nbytes):
        if self._ws is None or self._ws.numel() < nbytes:
            self._ws = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=f"cuda:{self.device}")
        return self._ws


def _dev(a, dtype, device):
    if a is None:
        return None
    if isinstance(a, torch.Tensor):
        return a.to(device=device, dtype=dtype).contiguous()
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device=device)


class Grid:
    """Device copies of the transport inputs of a workload."""

    def __init__(self, n, beta_max, tau_scale, cell_photons, cell_packets, line_lambda,
                 line_tau0, device="cuda:0", line_trans=None, tau_ct=None, fcorr_ct=None):
        self.n = int(n)
        self.beta_max = float(beta_max)
        self.tau_scale = _dev(tau_scale, torch.float32, device)
        self.cell_photons = _dev(cell_photons, torch.float64, device)
        self.cell_packets = _dev(cell_packets, torch.int32, device)
        self.line_lambda = _dev(line_lambda, torch.float64, device)
        self.line_tau0 = _dev(line_tau0, torch.float32, device)
        self.line_trans = _dev(line_trans, torch.int32, device)
        self.tau_ct = _dev(tau_ct, torch.float64, device)
        self.fcorr_ct = _dev(fcorr_ct, torch.float64, device)
        self.n_cells = self.n ** 3
        self.n_lines = int(self.line_lambda.numel())
        self.n_trans = 0 if self.tau_ct is None else self.tau_ct.numel() // self.n_cells
        self.photoion = None  # a Photoion: the transport then also photoionises
        self.spherical = None  # a Spherical: (r, theta, phi) cells instead of the cube

    def struct(self):
        self._pi = self.photoion.struct() if self.photoion is not None else None
        self._sph = self.spherical.struct() if self.spherical is not None else None
        return _Grid(self.n, self.beta_max, _ptr(self.tau_scale), _ptr(self.cell_photons),
                     _ptr(self.cell_packets), self.n_lines, _ptr(self.line_lambda),
                     _ptr(self.line_tau0), _ptr(self.line_trans), self.n_trans,
                     _ptr(self.tau_ct), _ptr(self.fcorr_ct),
                     C.addressof(self._pi) if self._pi is not None else None,
                     C.addressof(self._sph) if self._sph is not None else None)


class Spherical:
    """A spherical grid (extrass_spherical): shell edges r_edge [n_r + 1] in
    x = v/c from 0, polar edges theta_edge [n_theta + 1] from 0 to pi, n_phi
    equal azimuthal slices; cell i_r + n_r (i_theta + n_theta i_phi)."""

    def __init__(self, r_edge, theta_edge, n_phi, device="cuda:0", n_domains=0):
        self.n_domains = int(n_domains)  # phi subdomains of the streamed transport
        self.r_edge = _dev(r_edge, torch.float64, device)
        self.theta_edge = _dev(theta_edge, torch.float64, device)
        self.n_r = int(self.r_edge.numel()) - 1
        self.n_theta = int(self.theta_edge.numel()) - 1
        self.n_phi = int(n_phi)
        self.n_cells = self.n_r * self.n_theta * self.n_phi

    def struct(self):
        return _Spherical(self.n_r, self.n_theta, self.n_phi, _ptr(self.r_edge),
                          _ptr(self.theta_edge), self.n_domains)


def spherical_grid(r_edge, theta_edge, n_phi, tau_scale, cell_photons, cell_packets, line_lambda,
                   line_tau0, device="cuda:0", line_trans=None, tau_ct=None, fcorr_ct=None,
                   n_domains=0):
    """A Grid whose cells are those of a spherical grid (the per-cell arrays
    have n_r n_theta n_phi entries); n_domains phi subdomains for the
    streamed transport."""
    sph = Spherical(r_edge, theta_edge, n_phi, device, n_domains)
    g = Grid(1, 1.0, tau_scale, cell_photons, cell_packets, line_lambda, line_tau0, device,
             line_trans, tau_ct, fcorr_ct)
    g.spherical = sph
    g.n_cells = sph.n_cells
    g.n_trans = 0 if g.tau_ct is None else g.tau_ct.numel() // g.n_cells
    return g


def grid_from_workload(w, device="cuda:0", tau_ct=None, fcorr_ct=None, n_domains=0):
    """The workload's grid: its cube, or for a workload on a spherical grid
    (w.r_edge) that grid with n_domains phi subdomains."""
    line_trans = None
    if tau_ct is not None:
        lt = np.full(w.n_lines, -1, dtype=np.int32)
        lt[w.atom.trans_line] = np.arange(w.atom.n_trans, dtype=np.int32)
        line_trans = lt
    if getattr(w, "r_edge", None) is not None:
        return spherical_grid(w.r_edge, w.theta_edge, w.n_phi, w.tau_scale, w.cell_photons,
                              w.cell_packets, w.line_lambda, w.line_tau0, device, line_trans,
                              tau_ct, fcorr_ct, n_domains)
    return Grid(w.n, w.beta_max, w.tau_scale, w.cell_photons, w.cell_packets, w.line_lambda,
                w.line_tau0, device, line_trans, tau_ct, fcorr_ct)


class PiPlan:
    """The photoionising levels of an atom (extrass_pi_plan_create; Sec.
    2.3.1, Eq. A5): stages 0 and 1, the first max_per_stage levels of each
    below its ionisation energy ion_energy [S*3] (erg), in threshold order."""

    def __init__(self, ctx: Context, atom, ion_energy, max_per_stage=25):
        ie = np.ascontiguousarray(ion_energy, np.float64)
        h = _vp()
        ctx.check(_lib.extrass_pi_plan_create(ctx.h, atom.h, ie.ctypes.data, int(max_per_stage),
                                              C.byref(h)), "extrass_pi_plan_create")
        self.h = h
        self.ctx = ctx
        self.n_levels_atom = atom.n_levels
        m = C.c_int32(0)
        _lib.extrass_pi_plan_info(h, C.byref(m), None, None, None, None)
        self.M = int(m.value)
        self.level = np.zeros(self.M, np.int32)
        self.lambda_thr = np.zeros(self.M)
        self.sigma0 = np.zeros(self.M)
        dptr = C.c_void_p()
        _lib.extrass_pi_plan_info(h, None, self.level.ctypes.data, self.lambda_thr.ctypes.data,
                                  self.sigma0.ctypes.data, C.byref(dptr))
        self.device_lambda = dptr.value

    def opacity(self, pops, out=None):
        """extrass_pi_opacity: [C, 2M+1] per-cell rows from populations [C, N]."""
        C_ = pops.numel() // self.n_levels_atom
        if out is None:
            out = torch.empty((C_, 2 * self.M + 1), dtype=torch.float64, device=pops.device)
        self.ctx.check(_lib.extrass_pi_opacity(self.ctx.h, self.h, C_, _ptr(pops), _ptr(out),
                                               _stream()), "extrass_pi_opacity")
        return out

    def rates(self, grid: "Grid", t_exp, tally, out=None):
        """extrass_pi_rates: photoionisation rate per atom of each level [C, N]."""
        if out is None:
            out = torch.empty((grid.n_cells, self.n_levels_atom), dtype=torch.float64,
                              device=tally.device)
        g = grid.struct()
        self.ctx.check(_lib.extrass_pi_rates(self.ctx.h, self.h, C.byref(g), float(t_exp),
                                             _ptr(tally), _ptr(out), _stream()), "extrass_pi_rates")
        return out

    def close(self):
        if self.h:
            _lib.extrass_pi_plan_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Photoion:
    """Photoionisation for a grid's transport (extrass_photoion): the plan's
    thresholds, an opacity table and a tally [C, 2M] the transport adds into
    (zeroed here). Set grid.photoion to it."""

    LIGHT = 2.99792458e10

    def __init__(self, plan: PiPlan, opacity, t_exp, tally=None):
        self.plan = plan
        self.opacity = opacity
        self.length = self.LIGHT * float(t_exp)
        C_ = opacity.shape[0]
        self.tally = (torch.zeros((C_, 2 * plan.M), dtype=torch.float64, device=opacity.device)
                      if tally is None else tally)

    def struct(self):
        return _Photoion(self.plan.M, self.plan.device_lambda, _ptr(self.opacity), self.length,
                         _ptr(self.tally))


def transport(ctx: Context, grid: Grid, seed, lambda_lo, lambda_hi, n_packets, first_packet=0,
              iteration=0, geometry_fp32=False, explicit_packets=None, est=None, stats=None,
              packets_out=False):
    """Runs extrass_transport; returns (est [C, L] f64, stats [16] f64, packets [P, 8] or None)."""
    dev = grid.line_lambda.device
    expl = _dev(explicit_packets, torch.float64, dev)
    g = grid.struct()
    s = _Source(int(seed), int(iteration), int(first_packet), int(n_packets), float(lambda_lo),
                float(lambda_hi), _ptr(expl), 1 if geometry_fp32 else 0)
    if est is None:
        est = torch.empty((grid.n_cells, grid.n_lines), dtype=torch.float64, device=dev)
    if stats is None:
        stats = torch.empty(STATS, dtype=torch.float64, device=dev)
    pk = (torch.zeros((n_packets, PACKET_FIELDS), dtype=torch.float64, device=dev)
          if packets_out else None)
    need = _lib.extrass_transport_workspace(C.byref(g), C.byref(s))
    ws = ctx.workspace(need)
    rc = _lib.extrass_transport(ctx.h, C.byref(g), C.byref(s), _ptr(est), _ptr(stats), _ptr(pk),
                                _ptr(ws), ws.numel(), _stream())
    ctx.check(rc, "extrass_transport")
    return est, stats, pk


def transport_noalloc(ctx: Context, grid: Grid, seed, lambda_lo, lambda_hi, n_packets, est, stats,
                      first_packet=0, iteration=0, geometry_fp32=False, packets_out=None):
    """Runs extrass_transport_noalloc (no workspace; the library's per-GPU
    scratch) into the caller's est [C, L], stats [16] and optional per-packet
    records; returns the library's return code (0, or ENOSPACE when the problem
    needs more scratch than it holds) without raising on ENOSPACE."""
    g = grid.struct()
    s = _Source(int(seed), int(iteration), int(first_packet), int(n_packets), float(lambda_lo),
                float(lambda_hi), None, 1 if geometry_fp32 else 0)
    rc = _lib.extrass_transport_noalloc(ctx.h, C.byref(g), C.byref(s), _ptr(est), _ptr(stats),
                                        _ptr(packets_out), _stream())
    if rc not in (OK, ENOSPACE):
        ctx.check(rc, "extrass_transport_noalloc")
    return rc


class EmissionPlan:
    """The wavelength binning of an atom's line emission for deterministic rays
    (extrass_emission_plan_create): n_lambda logarithmic bins over
    [lambda_min, lambda_max); the occupied ones, each with its starting
    (reddest) wavelength."""

    def __init__(self, ctx: Context, atom, lambda_min, lambda_max, n_lambda):
        h = _vp()
        ctx.check(_lib.extrass_emission_plan_create(ctx.h, atom.h, float(lambda_min),
                                                    float(lambda_max), int(n_lambda), C.byref(h)),
                  "extrass_emission_plan_create")
        self.h = h
        nb = C.c_int32(0)
        _lib.extrass_emission_plan_info(h, C.byref(nb), None, None, None)
        self.n_bins = int(nb.value)
        self.bin_number = np.zeros(self.n_bins, dtype=np.int32)
        self.bin_lambda = np.zeros(self.n_bins)
        dptr = C.c_void_p()
        _lib.extrass_emission_plan_info(h, None, self.bin_number.ctypes.data,
                                        self.bin_lambda.ctypes.data, C.byref(dptr))
        self.device_lambda = dptr.value

    def close(self):
        if self.h:
            _lib.extrass_emission_plan_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def emission(ctx: Context, plan: EmissionPlan, atom, grid: Grid, t_exp, pops, bin_photons=None,
             outside=None):
    """Line emission of the grid's cells (extrass_emission): photons s^-1 per
    occupied bin [C, B] and erg s^-1 outside the binned range [C]."""
    dev = pops.device
    if bin_photons is None:
        bin_photons = torch.empty((grid.n_cells, plan.n_bins), dtype=torch.float64, device=dev)
    if outside is None:
        outside = torch.empty(grid.n_cells, dtype=torch.float64, device=dev)
    g = grid.struct()
    ctx.check(_lib.extrass_emission(ctx.h, plan.h, atom.h, C.byref(g), float(t_exp), _ptr(pops),
                                    _ptr(bin_photons), _ptr(outside), _stream()),
              "extrass_emission")
    return bin_photons, outside


def transport_rays(ctx: Context, grid: Grid, plan: EmissionPlan, bin_photons, n_theta, n_phi,
                   first_ray=0, n_rays=None, geometry_fp32=False, est=None, stats=None,
                   packets_out=False):
    """Deterministic rays (extrass_transport with extrass_rays): one ray per
    (cell, occupied bin, viewer). Returns (est [C, L], stats [16], packets [R, 8]
    or None)."""
    dev = grid.line_lambda.device
    total = grid.n_cells * plan.n_bins * int(n_theta) * int(n_phi)
    if n_rays is None:
        n_rays = total - first_ray
    rays = _Rays(int(n_theta), int(n_phi), plan.n_bins, plan.device_lambda, _ptr(bin_photons))
    g = grid.struct()
    s = _Source(0, 0, int(first_ray), int(n_rays), 0.0, 0.0, None, 1 if geometry_fp32 else 0,
                C.cast(C.pointer(rays), C.c_void_p))
    if est is None:
        est = torch.empty((grid.n_cells, grid.n_lines), dtype=torch.float64, device=dev)
    if stats is None:
        stats = torch.empty(STATS, dtype=torch.float64, device=dev)
    pk = (torch.zeros((n_rays, PACKET_FIELDS), dtype=torch.float64, device=dev)
          if packets_out else None)
    ws = ctx.workspace(_lib.extrass_transport_workspace(C.byref(g), C.byref(s)))
    ctx.check(_lib.extrass_transport(ctx.h, C.byref(g), C.byref(s), _ptr(est), _ptr(stats),
                                     _ptr(pk), _ptr(ws), ws.numel(), _stream()), "extrass_transport")
    return est, stats, pk


def spectrum(ctx: Context, packets, n_theta, n_phi, n_lambda, lambda_min, lambda_max,
             photons=None, energy=None):
    """Runs extrass_spectrum on per-packet records [P, 8] (device f64, as transport
    writes them). Adds into photons / energy [n_theta, n_phi, n_lambda] (zeros
    allocated when None); returns (photons, energy)."""
    pk = packets.contiguous()
    dev = pk.device
    shape = (int(n_theta), int(n_phi), int(n_lambda))
    if photons is None:
        photons = torch.zeros(shape, dtype=torch.float64, device=dev)
    if energy is None:
        energy = torch.zeros(shape, dtype=torch.float64, device=dev)
    b = _SpecBins(shape[0], shape[1], shape[2], float(lambda_min), float(lambda_max))
    rc = _lib.extrass_spectrum(ctx.h, _ptr(pk), pk.shape[0], C.byref(b), _ptr(photons),
                               _ptr(energy), _stream())
    ctx.check(rc, "extrass_spectrum")
    return photons, energy


def transport_streamed(ctx: Context, grid: Grid, seed, lambda_lo, lambda_hi, n_packets,
                       atom=None, pops=None, t_exp=None, iteration=0, geometry_fp32=False,
                       est_octant=None, est_global=False, gamma=None, stats=None,
                       queue_capacity=None, octant_table=True):
    """Runs extrass_transport_streamed (8 velocity octants, one estimator table
    of one octant resident). Returns (gamma [C, T] or None, stats [16],
    est_global [C, L] or None). queue_capacity defaults to n_packets / 4 per
    octant (at least 4096). With octant_table=False (rates only, atom given)
    no table is allocated and the rates are summed per interaction."""
    dev = grid.line_lambda.device
    g = grid.struct()
    s = _Source(int(seed), int(iteration), 0, int(n_packets), float(lambda_lo), float(lambda_hi),
                None, 1 if geometry_fp32 else 0)
    sub_cells = (grid.n_cells // max(1, grid.spherical.n_domains) if grid.spherical is not None
                 else (grid.n // 2) ** 3)
    if est_octant is None and octant_table:
        est_octant = torch.empty((sub_cells, grid.n_lines), dtype=torch.float64, device=dev)
    eg = (torch.empty((grid.n_cells, grid.n_lines), dtype=torch.float64, device=dev)
          if est_global else None)
    if stats is None:
        stats = torch.empty(STATS, dtype=torch.float64, device=dev)
    if atom is not None and gamma is None:
        gamma = torch.empty((grid.n_cells, atom.n_trans), dtype=torch.float64, device=dev)
    qcap = int(queue_capacity) if queue_capacity else max(4096, int(n_packets) // 4)
    ws = ctx.workspace(_lib.extrass_transport_streamed_workspace(C.byref(g), qcap))
    rc = _lib.extrass_transport_streamed(
        ctx.h, C.byref(g), C.byref(s), atom.h if atom is not None else None, _ptr(pops),
        float(t_exp or 0.0), _ptr(est_octant), _ptr(eg), _ptr(gamma if atom is not None else None),
        _ptr(stats), qcap, _ptr(ws), ws.numel(), _stream())
    ctx.check(rc, "extrass_transport_streamed")
    return (gamma if atom is not None else None), stats, eg


def stats_dict(stats):
    v = stats.detach().cpu().numpy()
    d = dict(zip(STAT_NAMES, v[: len(STAT_NAMES)]))
    d["error_flag"] = v[STAT_ERROR_FLAG]
    d["bad_packets"] = v[STAT_ERROR_FLAG - 1]
    return d


class Atom:
    """An atom uploaded to the device once (extrass_atom_create)."""

    def __init__(self, ctx: Context, atom):
        self.ctx = ctx
        self.src = atom
        keep = dict(
            off=np.ascontiguousarray(atom.species_offset, np.int32),
            ion=np.ascontiguousarray(atom.level_ion, np.int32),
            E=np.ascontiguousarray(atom.level_energy, np.float64),
            g=np.ascontiguousarray(atom.level_g, np.float64),
            lo=np.ascontiguousarray(atom.trans_lower, np.int32),
            up=np.ascontiguousarray(atom.trans_upper, np.int32),
            A=np.ascontiguousarray(atom.trans_A, np.float64),
            lam=np.ascontiguousarray(atom.trans_lambda, np.float64),
            ups=np.ascontiguousarray(atom.trans_upsilon, np.float64),
            line=np.ascontiguousarray(atom.trans_line, np.int32),
            alpha=np.ascontiguousarray(atom.ion_alpha0, np.float64),
        )
        p = {k: v.ctypes.data for k, v in keep.items()}
        d = _AtomDesc(len(keep["off"]) - 1, p["off"], len(keep["ion"]), p["ion"], p["E"], p["g"],
                      len(keep["A"]), p["lo"], p["up"], p["A"], p["lam"], p["ups"], p["line"],
                      p["alpha"])
        h = _vp()
        ctx.check(_lib.extrass_atom_create(ctx.h, C.byref(d), C.byref(h)), "extrass_atom_create")
        self.h = h
        self.n_species = len(keep["off"]) - 1
        self.n_levels = len(keep["ion"])
        self.n_trans = len(keep["A"])

    def close(self):
        if self.h:
            _lib.extrass_atom_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def line_tau(ctx: Context, atom: Atom, pops, t_exp, tau=None, fcorr=None):
    """Eq. A2 opacity and stimulated-emission factor per (cell, transition),
    written into tau / fcorr when given (contiguous f64 [C, T])."""
    C_ = pops.numel() // atom.n_levels
    if tau is None:
        tau = torch.empty((C_, atom.n_trans), dtype=torch.float64, device=pops.device)
    fc = torch.empty_like(tau) if fcorr is None else fcorr
    for t in (tau, fc):
        if t.dtype != torch.float64 or not t.is_contiguous() or t.numel() != C_ * atom.n_trans:
            raise ValueError("line_tau: outputs must be contiguous float64 [C, T]")
    ctx.check(_lib.extrass_line_tau(ctx.h, atom.h, C_, _ptr(pops), float(t_exp), _ptr(tau),
                                    _ptr(fc), _stream()), "extrass_line_tau")
    return tau, fc


def rates(ctx: Context, atom: Atom, grid: Grid, t_exp, est, pops, out=None):
    """Photoexcitation rates per (cell, transition) of the grid's cells at time
    t_exp (extrass_rates), written into out when given (contiguous f64 [C, T])."""
    C_ = grid.n_cells
    for t, n in ((est, C_ * grid.n_lines), (pops, C_ * atom.n_levels)):
        if t.numel() != n:
            raise ValueError("rates: est must be [C, L] and pops [C, N] of the grid's cells")
    if out is None:
        out = torch.empty((C_, atom.n_trans), dtype=torch.float64, device=pops.device)
    elif out.dtype != torch.float64 or not out.is_contiguous() or out.numel() != C_ * atom.n_trans:
        raise ValueError("rates: out must be contiguous float64 [C, T]")
    g = grid.struct()
    ctx.check(_lib.extrass_rates(ctx.h, atom.h, C.byref(g), float(t_exp), _ptr(est), _ptr(pops),
                                 _ptr(out), _stream()), "extrass_rates")
    return out


class Cells:
    def __init__(self, t_exp, T_e, n_e, n_species, gamma_ion, gamma_pe=None, device="cuda:0",
                 gamma_pi=None):
        self.t_exp = float(t_exp)
        self.T_e = _dev(T_e, torch.float64, device)
        self.n_e = _dev(n_e, torch.float64, device)
        self.n_species = _dev(n_species, torch.float64, device)
        self.gamma_ion = _dev(gamma_ion, torch.float64, device)
        self.gamma_pe = _dev(gamma_pe, torch.float64, device)
        self.gamma_pi = _dev(gamma_pi, torch.float64, device)
        self.n_cells = int(self.T_e.numel())

    def struct(self):
        return _Cells(self.n_cells, self.t_exp, _ptr(self.T_e), _ptr(self.n_e),
                      _ptr(self.n_species), _ptr(self.gamma_ion), _ptr(self.gamma_pe),
                      _ptr(self.gamma_pi))


def cells_from_workload(w, gamma_pe=None, device="cuda:0", cells=None):
    S = w.atom.n_species
    if cells is None:
        return Cells(w.t_exp, w.T_e, w.n_e, w.n_species, w.gamma_ion, gamma_pe, device)
    cells = np.asarray(cells)
    gpe = None
    if gamma_pe is not None:
        gpe = gamma_pe.reshape(-1, w.atom.n_trans)[torch.as_tensor(cells, device=gamma_pe.device)] \
            if isinstance(gamma_pe, torch.Tensor) else gamma_pe.reshape(-1, w.atom.n_trans)[cells]
    return Cells(w.t_exp, w.T_e[cells], w.n_e[cells], w.n_species.reshape(-1, S)[cells],
                 w.gamma_ion.reshape(-1, S, 3)[cells], gpe, device)


def nlte_solve(ctx: Context, atom: Atom, cells: Cells, max_iter=200, tol=1e-10, guess=None,
               factor_fp32=False, pops=None, status=None, iters=None, warm_budget=0,
               use_guess=None):
    """Runs extrass_nlte_solve; returns (pops [C, N], status [C], iters [C])."""
    dev = cells.T_e.device
    if pops is None:
        pops = torch.empty((cells.n_cells, atom.n_levels), dtype=torch.float64, device=dev)
    if guess is not None and guess.data_ptr() != pops.data_ptr():
        pops.copy_(guess)
    if use_guess is None:
        use_guess = guess is not None
    if status is None:
        status = torch.empty(cells.n_cells, dtype=torch.int32, device=dev)
    if iters is None:
        iters = torch.empty(cells.n_cells, dtype=torch.int32, device=dev)
    o = _Opts(int(max_iter), float(tol), 1 if use_guess else 0, 1 if factor_fp32 else 0,
              int(warm_budget))
    cs = cells.struct()
    need = _lib.extrass_nlte_workspace(atom.h, cells.n_cells)
    ws = ctx.workspace(need)
    rc = _lib.extrass_nlte_solve(ctx.h, atom.h, C.byref(cs), C.byref(o), _ptr(pops), _ptr(status),
                                 _ptr(iters), _ptr(ws), ws.numel(), _stream())
    ctx.check(rc, "extrass_nlte_solve")
    return pops, status, iters


MLP_PARAMS = int(_lib.extrass_mlp_param_count())
MLP_IN, MLP_OUT = 6, 100


def mlp_forward(ctx: Context, params, x):
    """y = MLP(x) for normalised features x [B, 6] (FP32 device tensors)."""
    B = x.shape[0]
    y = torch.empty((B, MLP_OUT), dtype=torch.float32, device=x.device)
    ws = ctx.workspace(_lib.extrass_mlp_workspace(B))
    ctx.check(_lib.extrass_mlp_forward(ctx.h, _ptr(params), _ptr(x), _ptr(y), B, _ptr(ws),
                                       ws.numel(), _stream()), "extrass_mlp_forward")
    return y


def mlp_train_step(ctx: Context, params, x, t, adam_m=None, adam_v=None, step=1, lr=1e-3,
                   loss=None, grad=None):
    B = x.shape[0]
    ws = ctx.workspace(_lib.extrass_mlp_workspace(B))
    ctx.check(_lib.extrass_mlp_train_step(ctx.h, _ptr(params), _ptr(adam_m), _ptr(adam_v),
                                          int(step), float(lr), _ptr(x), _ptr(t), B, _ptr(loss),
                                          _ptr(grad), _ptr(ws), ws.numel(), _stream()),
              "extrass_mlp_train_step")


def mlp_features(ctx: Context, atom: Atom, cells: Cells, deposition):
    """The six raw warm-start features of every cell [C, 6] (FP32 device tensor),
    as extrass_nlte_warm_start forms them (extrass_mlp_features)."""
    dep = _dev(deposition, torch.float64, cells.T_e.device)
    x = torch.empty((cells.n_cells, MLP_IN), dtype=torch.float32, device=cells.T_e.device)
    cs = cells.struct()
    ctx.check(_lib.extrass_mlp_features(ctx.h, atom.h, C.byref(cs), _ptr(dep), _ptr(x), _stream()),
              "extrass_mlp_features")
    return x


def nlte_warm_start(ctx: Context, atom: Atom, cells: Cells, deposition, params, norm, pops=None):
    """Populations predicted by the MLP for every cell (extrass_nlte_warm_start)."""
    dev = cells.T_e.device
    if pops is None:
        pops = torch.empty((cells.n_cells, atom.n_levels), dtype=torch.float64, device=dev)
    dep = _dev(deposition, torch.float64, dev)
    cs = cells.struct()
    ws = ctx.workspace(_lib.extrass_nlte_warm_start_workspace(cells.n_cells))
    ctx.check(_lib.extrass_nlte_warm_start(ctx.h, atom.h, C.byref(cs), _ptr(dep), _ptr(params),
                                           _ptr(norm), _ptr(pops), _ptr(ws), ws.numel(),
                                           _stream()), "extrass_nlte_warm_start")
    return pops


class Batched:
    """Device copies of a batched NLTE problem (one element, three ion stages
    per cell); the level counts are kept on the host as well."""

    def __init__(self, b, device="cuda:0"):
        self.n_cells = int(b.n_cells)
        self.seed = int(b.seed)
        self.level_count = np.ascontiguousarray(b.level_count, dtype=np.int32)
        self.level_count_d = torch.as_tensor(self.level_count, device=device)
        self.T_e = _dev(b.T_e, torch.float64, device)
        self.n_e = _dev(b.n_e, torch.float64, device)
        self.gamma_ion = _dev(b.gamma_ion, torch.float64, device)
        self.alpha0 = [float(a) for a in b.alpha0]
        self.gamma_pe_table = _dev(b.gamma_pe_table, torch.float64, device)
        self.n_pops = int(self.level_count.astype(np.int64).sum())
        self.device = device

    def struct(self):
        return _Batched(self.n_cells, self.seed, self.level_count.ctypes.data,
                        _ptr(self.level_count_d), _ptr(self.T_e), _ptr(self.n_e),
                        _ptr(self.gamma_ion), (C.c_double * 2)(*self.alpha0),
                        _ptr(self.gamma_pe_table), self.gamma_pe_table.numel())


def _bopts(factor_fp32, refine, tol, panel, per_cu):
    return _BOpts(1 if factor_fp32 else 0, int(refine), float(tol), int(panel), int(per_cu))


def batched_workspace(ctx: Context, prob: Batched, factor_fp32=False, panel=0, per_cu=0):
    """(min_bytes, all_bytes) of extrass_batched_workspace."""
    mn, al = C.c_size_t(0), C.c_size_t(0)
    ps = prob.struct()
    o = _bopts(factor_fp32, 0, 0.0, panel, per_cu)
    ctx.check(_lib.extrass_batched_workspace(ctx.h, C.byref(ps), C.byref(o), C.byref(mn),
                                             C.byref(al)), "extrass_batched_workspace")
    return mn.value, al.value


def batched_solve(ctx: Context, prob: Batched, factor_fp32=False, refine=2, tol=1e-12, panel=0,
                  per_cu=0, ws_limit=16 << 30, pops=None, status=None):
    """Stationary populations of every cell (extrass_batched_solve); the
    workspace is the smaller of all cells at once and ws_limit (then chunked)."""
    dev = prob.device
    if pops is None:
        pops = torch.empty(prob.n_pops, dtype=torch.float64, device=dev)
    if status is None:
        status = torch.empty(prob.n_cells, dtype=torch.int32, device=dev)
    mn, al = batched_workspace(ctx, prob, factor_fp32, panel, per_cu)
    ws = ctx.workspace(max(mn, min(al, ws_limit)))
    ps = prob.struct()
    o = _bopts(factor_fp32, refine, tol, panel, per_cu)
    ctx.check(_lib.extrass_batched_solve(ctx.h, C.byref(ps), C.byref(o), _ptr(pops), _ptr(status),
                                         _ptr(ws), ws.numel(), _stream()), "extrass_batched_solve")
    return pops, status


def batched_tune(ctx: Context, prob: Batched, factor_fp32=False, ws_limit=2 << 30):
    """Runs extrass_batched_tune on the first cells of prob; returns
    ((panel, per_cu), {(panel, per_cu): ms})."""
    mn, al = batched_workspace(ctx, prob, factor_fp32, 64, 4)
    ws = ctx.workspace(max(mn, min(al, ws_limit)))
    ps = prob.struct()
    o = _bopts(factor_fp32, 0, 0.0, 0, 0)
    choice = (C.c_int32 * 2)()
    times = (C.c_float * 9)()
    ctx.check(_lib.extrass_batched_tune(ctx.h, C.byref(ps), C.byref(o), _ptr(ws), ws.numel(),
                                        _stream(), choice, times), "extrass_batched_tune")
    table = {(p, c): times[3 * i + j] for i, p in enumerate((16, 32, 64))
             for j, c in enumerate((1, 2, 4))}
    return (choice[0], choice[1]), table
