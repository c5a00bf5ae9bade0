"""Global iterations of the method on one GPU: the outer loop of radiative
transfer and statistical equilibrium (Sec. 2.2, 2.3).

One iteration: Eq. A2 line opacities from the current populations ->
packet transport streamed over the 8 velocity octants, with photoexcitation
rates accumulated octant by octant -> NLTE solve of every cell, started from
the previous iteration's populations. The first iteration starts from the
learned warm start (or the cold start). This module only orders library
calls and keeps the tensors; every step runs in the library's kernels.

`GlobalLoop` uploads a workload and allocates every buffer once, so that
repeated runs of the loop do no host-to-device copies and no allocations.

`python -m paper_2511_07539_amd.globalloop` runs the 100^3-cell, 30000-line,
1e8-packet case for 5 iterations and prints one JSON line.
"""
from __future__ import annotations

import json
import sys
import time

import numpy as np
import torch

from . import (Atom, Cells, Context, EmissionPlan, Photoion, PiPlan, cells_from_workload,
               emission, grid_from_workload, line_tau, nlte_solve, nlte_warm_start, rates,
               stats_dict, transport_rays, transport_streamed)

HC = 6.62607015e-27 * 2.99792458e10  # h c, erg cm


class GlobalLoop:
    """The global loop over one workload, with its inputs resident on the GPU.

    tol is the population accuracy each NLTE solve runs to; the streamed
    transport sums the rates per interaction (no octant estimator table)
    unless octant_table is set. With ion_energy [S*3] (erg) the transport also
    photoionises (Sec. 2.3.1): each iteration builds the continuum opacity from
    the current populations, and the NLTE solve takes the photoionisation
    rates the transport measured. A workload on a spherical grid streams over
    n_domains equal phi ranges (the paper's decomposition, Sec. 2.4.1); the
    cube over its 8 velocity octants."""

    def __init__(self, ctx: Context, w, device="cuda:0", geometry_fp32=True, queue_capacity=None,
                 max_iter=200, tol=1e-10, warm_budget=30, octant_table=False, ion_energy=None,
                 pi_levels_per_stage=25, n_domains=8, nlte_fp32=False):
        self.ctx, self.w, self.device = ctx, w, device
        # nlte_fp32: the NLTE solves reduce their fixed-point steps in FP32
        # (residuals and Newton systems stay FP64)
        self.nlte_fp32 = nlte_fp32
        self.geometry_fp32, self.queue_capacity = geometry_fp32, queue_capacity
        self.max_iter, self.tol, self.warm_budget = max_iter, tol, warm_budget
        self.octant_table = octant_table
        self.atom = Atom(ctx, w.atom)
        self.cells0 = cells_from_workload(w, device=device)
        C, T, N = w.n_cells, w.atom.n_trans, w.atom.n_levels
        self.gamma = torch.zeros((C, T), dtype=torch.float64, device=device)
        self.pi_plan = None
        self.gamma_pi = None
        if ion_energy is not None:
            self.pi_plan = PiPlan(ctx, self.atom, ion_energy, pi_levels_per_stage)
            self.gamma_pi = torch.zeros((C, N), dtype=torch.float64, device=device)
        self.cells = Cells(w.t_exp, self.cells0.T_e, self.cells0.n_e, self.cells0.n_species,
                           self.cells0.gamma_ion, self.gamma, device=device,
                           gamma_pi=self.gamma_pi)
        self.deposition = torch.as_tensor(w.deposition, device=device)
        tau = torch.empty((C, T), dtype=torch.float64, device=device)
        self.grid = grid_from_workload(w, device=device, tau_ct=tau, fcorr_ct=torch.empty_like(tau),
                                       n_domains=n_domains)
        del tau
        if self.pi_plan is not None:
            M = self.pi_plan.M
            self.grid.photoion = Photoion(
                self.pi_plan, torch.empty((C, 2 * M + 1), dtype=torch.float64, device=device),
                w.t_exp)
        self.pops = torch.empty((C, N), dtype=torch.float64, device=device)
        self.new = torch.empty_like(self.pops)
        self.status = torch.empty(C, dtype=torch.int32, device=device)
        self.iters = torch.empty(C, dtype=torch.int32, device=device)
        self.stats = torch.empty(16, dtype=torch.float64, device=device)
        sub = C // n_domains if self.grid.spherical is not None else (w.n // 2) ** 3
        self.est_oct = (torch.empty((sub, w.n_lines), dtype=torch.float64, device=device)
                        if octant_table else None)
        lv_species = torch.as_tensor(
            np.repeat(np.arange(w.atom.n_species), np.diff(w.atom.species_offset)), device=device)
        self.ns_lv = self.cells0.n_species.view(C, -1)[:, lv_species]

    def start(self, params=None, norm=None):
        """Populations before the first iteration: the MLP's, or the cold start."""
        if params is not None:
            nlte_warm_start(self.ctx, self.atom, self.cells, self.deposition, params, norm,
                            pops=self.pops)
        else:
            nlte_solve(self.ctx, self.atom, self.cells0, max_iter=0, pops=self.pops,
                       status=self.status, iters=self.iters)

    def iterate(self, k, warm_budget=0, events=None):
        """Global iteration k (0-based) from self.pops; the new populations
        replace self.pops. events, if given, receives 4 recorded HIP events
        (start, after the opacities, after the transport, after the NLTE)."""
        w, s = self.w, torch.cuda.current_stream()
        rec = (lambda i: events[i].record(s)) if events is not None else (lambda i: None)
        rec(0)
        line_tau(self.ctx, self.atom, self.pops, w.t_exp, tau=self.grid.tau_ct,
                 fcorr=self.grid.fcorr_ct)
        pi = self.grid.photoion
        if pi is not None:
            self.pi_plan.opacity(self.pops, out=pi.opacity)
            pi.tally.zero_()
        rec(1)
        transport_streamed(self.ctx, self.grid, w.seed, w.lambda_lo, w.lambda_hi, w.n_packets,
                           atom=self.atom, pops=self.pops, t_exp=w.t_exp, iteration=k,
                           geometry_fp32=self.geometry_fp32, est_octant=self.est_oct,
                           gamma=self.gamma, stats=self.stats,
                           queue_capacity=self.queue_capacity, octant_table=self.octant_table)
        if pi is not None:
            self.pi_plan.rates(self.grid, w.t_exp, pi.tally, out=self.gamma_pi)
        rec(2)
        nlte_solve(self.ctx, self.atom, self.cells, max_iter=self.max_iter, tol=self.tol,
                   guess=self.pops, warm_budget=warm_budget, pops=self.new, status=self.status,
                   iters=self.iters, factor_fp32=self.nlte_fp32)
        rec(3)
        self.pops, self.new = self.new, self.pops

    def run(self, iterations=5, params=None, norm=None, log=None, history=True):
        """Runs the loop; returns (pops [C, N], status [C], history). The first
        iteration starts from the MLP's populations when params/norm are given
        (with the warm budget and cold fallback), else from the cold start.
        With history, each iteration's timings and convergence figures are
        recorded (one device synchronisation per iteration)."""
        self.start(params, norm)
        hist = []
        for k in range(iterations):
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)] if history else None
            prev = self.pops
            self.iterate(k, self.warm_budget if k == 0 and params is not None else 0, ev)
            if history:
                hist.append(self._record(k, ev, prev))
                if log:
                    log(hist[-1])
        return self.pops, self.status, hist

    def _record(self, k, ev, prev):
        torch.cuda.synchronize()
        new, st = self.pops, self.status
        ok = st <= 1
        # change of the populated levels (>= 1e-10 of their species); emptier
        # levels follow the Monte Carlo noise of their photoexcitation rates
        sig = ok[:, None] & (new >= 1e-10 * self.ns_lv)
        d = ((new - prev).abs() / new.clamp_min(1e-300))[sig]
        sd = stats_dict(self.stats)
        return {"iteration": k + 1, "ms_line_tau": ev[0].elapsed_time(ev[1]),
                "ms_transport": ev[1].elapsed_time(ev[2]), "ms_nlte": ev[2].elapsed_time(ev[3]),
                "interactions": sd["n_inter"], "escaped_fraction": sd["w_esc"] / sd["w_emit"],
                "photoionised_fraction": sd["w_pi"] / sd["w_emit"],
                "cells_converged": int(ok.sum()), "fallbacks": int((st == 1).sum()),
                "nlte_iters_mean": float(self.iters.float().mean()),
                "max_rel_change": float(d.max().item()) if d.numel() else None,
                "median_rel_change": float(d.median().item()) if d.numel() else None}


class RayLoop:
    """Global iterations with the paper's own radiative transfer (Sec. 2.3):
    the cells' line emission (Eq. A3) from the current populations, sent as
    deterministic rays, one per (cell, occupied 0.1 % wavelength bin, viewer),
    from each cell's middle (of the cube or the spherical grid) -> estimators
    -> rates -> NLTE. Each iteration
    reports the global convergence figure L_bol / L_dep: the luminosity of the
    escaping rays, plus the emission outside the binned range, plus the
    deposition of cells whose NLTE solve failed, over the total deposition
    (Sec. 2.3; global convergence). The loop stops after `stop_after`
    consecutive iterations above `threshold`, or after `iterations`.

    The synthetic workloads prescribe T_e and deposition (no temperature loop,
    no thermal balance), so the figure is computed as the paper defines it but
    need not approach unity."""

    def __init__(self, ctx: Context, w, n_theta=20, n_phi=20, lambda_min=None, lambda_max=None,
                 bin_ratio=1.001, device="cuda:0", geometry_fp32=False, max_iter=200, tol=1e-8):
        self.ctx, self.w, self.device = ctx, w, device
        self.n_theta, self.n_phi = n_theta, n_phi
        self.geometry_fp32, self.max_iter, self.tol = geometry_fp32, max_iter, tol
        lam = w.atom.trans_lambda
        lo = lambda_min if lambda_min is not None else 0.97 * float(lam.min())
        hi = lambda_max if lambda_max is not None else 1.03 * float(lam.max())
        n_lambda = int(np.ceil(np.log(hi / lo) / np.log(bin_ratio)))
        self.atom = Atom(ctx, w.atom)
        self.plan = EmissionPlan(ctx, self.atom, lo, hi, n_lambda)
        C, T = w.n_cells, w.atom.n_trans
        self.cells0 = cells_from_workload(w, device=device)
        self.gamma = torch.zeros((C, T), dtype=torch.float64, device=device)
        self.cells = Cells(w.t_exp, self.cells0.T_e, self.cells0.n_e, self.cells0.n_species,
                           self.cells0.gamma_ion, self.gamma, device=device)
        tau = torch.empty((C, T), dtype=torch.float64, device=device)
        self.grid = grid_from_workload(w, device=device, tau_ct=tau, fcorr_ct=torch.empty_like(tau))
        self.est = torch.empty((C, w.n_lines), dtype=torch.float64, device=device)
        self.stats = torch.empty(16, dtype=torch.float64, device=device)
        self.bin_photons = torch.empty((C, self.plan.n_bins), dtype=torch.float64, device=device)
        self.outside = torch.empty(C, dtype=torch.float64, device=device)
        self.pops = torch.empty((C, w.atom.n_levels), dtype=torch.float64, device=device)
        self.new = torch.empty_like(self.pops)
        self.status = torch.empty(C, dtype=torch.int32, device=device)
        self.iters = torch.empty(C, dtype=torch.int32, device=device)
        # cell volumes: the cube's, or each spherical cell's (the workload's inputs)
        V = (w.cell_volumes() if getattr(w, "r_edge", None) is not None
             else (2.0 * w.beta_max / w.n * 2.99792458e10 * w.t_exp) ** 3)
        self.dep_cell = torch.as_tensor(w.deposition * V, device=device)   # erg s^-1 per cell
        self.L_dep = float(self.dep_cell.sum())

    @property
    def rays_per_iteration(self):
        return self.w.n_cells * self.plan.n_bins * self.n_theta * self.n_phi

    def iterate(self, k):
        """Iteration k from self.pops; returns its record (times, rays emitted,
        L_bol / L_dep and its parts)."""
        w, s = self.w, torch.cuda.current_stream()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(5)]
        ev[0].record(s)
        line_tau(self.ctx, self.atom, self.pops, w.t_exp, tau=self.grid.tau_ct,
                 fcorr=self.grid.fcorr_ct)
        emission(self.ctx, self.plan, self.atom, self.grid, w.t_exp, self.pops,
                 bin_photons=self.bin_photons, outside=self.outside)
        ev[1].record(s)
        transport_rays(self.ctx, self.grid, self.plan, self.bin_photons, self.n_theta,
                       self.n_phi, geometry_fp32=self.geometry_fp32, est=self.est,
                       stats=self.stats)
        ev[2].record(s)
        rates(self.ctx, self.atom, self.grid, w.t_exp, self.est, self.pops, out=self.gamma)
        ev[3].record(s)
        nlte_solve(self.ctx, self.atom, self.cells, max_iter=self.max_iter, tol=self.tol,
                   guess=self.pops, pops=self.new, status=self.status, iters=self.iters)
        ev[4].record(s)
        torch.cuda.synchronize()
        sd = stats_dict(self.stats)
        failed = self.status == 2
        L_esc = HC * sd["e_esc"]
        L_out = float(self.outside.sum())
        L_nc = float(self.dep_cell[failed].sum())
        rec = {"iteration": k + 1, "ms_emission": ev[0].elapsed_time(ev[1]),
               "ms_rays": ev[1].elapsed_time(ev[2]), "ms_rates": ev[2].elapsed_time(ev[3]),
               "ms_nlte": ev[3].elapsed_time(ev[4]), "rays": self.rays_per_iteration,
               "interactions": sd["n_inter"], "photons_emitted": sd["w_emit"],
               "L_escaping": L_esc, "L_outside_range": L_out, "L_nonconverged_cells": L_nc,
               "L_dep": self.L_dep, "L_bol_over_L_dep": (L_esc + L_out + L_nc) / self.L_dep,
               "cells_converged": int((self.status <= 1).sum())}
        self.pops, self.new = self.new, self.pops
        return rec

    def run(self, iterations=5, threshold=0.95, stop_after=3, log=None):
        """From the cold start; returns (pops, status, history, converged)."""
        nlte_solve(self.ctx, self.atom, self.cells0, max_iter=0, pops=self.pops,
                   status=self.status, iters=self.iters)
        hist, above = [], 0
        for k in range(iterations):
            rec = self.iterate(k)
            hist.append(rec)
            if log:
                log(rec)
            above = above + 1 if rec["L_bol_over_L_dep"] > threshold else 0
            if above >= stop_after:
                return self.pops, self.status, hist, True
        return self.pops, self.status, hist, False


def run(ctx: Context, w, iterations=5, params=None, norm=None, warm_budget=30, geometry_fp32=True,
        queue_capacity=None, max_iter=200, tol=1e-10, device="cuda:0", log=None,
        octant_table=False, ion_energy=None, n_domains=8):
    """Returns (pops [C, N], status [C], history) of `iterations` global
    iterations over workload w (see GlobalLoop)."""
    loop = GlobalLoop(ctx, w, device=device, geometry_fp32=geometry_fp32,
                      queue_capacity=queue_capacity, max_iter=max_iter, tol=tol,
                      warm_budget=warm_budget, octant_table=octant_table, ion_energy=ion_energy,
                      n_domains=n_domains)
    pops, status, hist = loop.run(iterations, params, norm, log=log)
    return pops.clone(), status.clone(), hist


def main(argv=None):
    import argparse

    import synth
    from . import warmstart

    ap = argparse.ArgumentParser()
    ap.add_argument("--iterations", type=int, default=5)
    ap.add_argument("--no-mlp", action="store_true", help="start from the cold start")
    ap.add_argument("--epochs", type=int, default=30)
    ap.add_argument("--queue-capacity", type=int, default=0)
    ap.add_argument("--tol", type=float, default=1e-8)
    args = ap.parse_args(argv)
    ctx = Context(0)
    params = norm = None
    t0 = time.perf_counter()
    if not args.no_mlp:
        params, norm, _ = warmstart.train_on_workload(ctx, synth.paper_scale(), epochs=args.epochs)
        torch.cuda.empty_cache()
    t_train = time.perf_counter() - t0
    w = synth.large()
    print(f"workload {w.name}: {w.n_cells} cells, {w.n_lines} lines, {w.n_packets} packets",
          file=sys.stderr, flush=True)
    t1 = time.perf_counter()
    pops, status, hist = run(ctx, w, args.iterations, params, norm, tol=args.tol,
                             queue_capacity=args.queue_capacity or None,
                             log=lambda r: print(json.dumps(r), file=sys.stderr, flush=True))
    wall = time.perf_counter() - t1
    out = {"workload": w.name, "cells": w.n_cells, "lines": w.n_lines, "packets": w.n_packets,
           "iterations": args.iterations, "start": "cold" if args.no_mlp else "mlp",
           "setup_s": t_train, "wall_s": wall, "history": hist,
           "status_counts": torch.bincount(status, minlength=4).tolist()}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
