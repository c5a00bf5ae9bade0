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

from . import (Atom, Cells, Context, cells_from_workload, grid_from_workload, line_tau,
               nlte_solve, nlte_warm_start, stats_dict, transport_streamed)


class GlobalLoop:
    """The global loop over one workload, with its inputs resident on the GPU.

    tol is the population accuracy each NLTE solve runs to; the streamed
    transport sums the rates per interaction (no octant estimator table)
    unless octant_table is set."""

    def __init__(self, ctx: Context, w, device="cuda:0", geometry_fp32=True, queue_capacity=None,
                 max_iter=200, tol=1e-10, warm_budget=30, octant_table=False):
        self.ctx, self.w, self.device = ctx, w, device
        self.geometry_fp32, self.queue_capacity = geometry_fp32, queue_capacity
        self.max_iter, self.tol, self.warm_budget = max_iter, tol, warm_budget
        self.octant_table = octant_table
        self.atom = Atom(ctx, w.atom)
        self.cells0 = cells_from_workload(w, device=device)
        C, T, N = w.n_cells, w.atom.n_trans, w.atom.n_levels
        self.gamma = torch.zeros((C, T), dtype=torch.float64, device=device)
        self.cells = Cells(w.t_exp, self.cells0.T_e, self.cells0.n_e, self.cells0.n_species,
                           self.cells0.gamma_ion, self.gamma, device=device)
        self.deposition = torch.as_tensor(w.deposition, device=device)
        tau = torch.empty((C, T), dtype=torch.float64, device=device)
        self.grid = grid_from_workload(w, device=device, tau_ct=tau, fcorr_ct=torch.empty_like(tau))
        del tau
        self.pops = torch.empty((C, N), dtype=torch.float64, device=device)
        self.new = torch.empty_like(self.pops)
        self.status = torch.empty(C, dtype=torch.int32, device=device)
        self.iters = torch.empty(C, dtype=torch.int32, device=device)
        self.stats = torch.empty(16, dtype=torch.float64, device=device)
        half = w.n // 2
        self.est_oct = (torch.empty((half ** 3, w.n_lines), dtype=torch.float64, device=device)
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
        rec(1)
        transport_streamed(self.ctx, self.grid, w.seed, w.lambda_lo, w.lambda_hi, w.n_packets,
                           atom=self.atom, pops=self.pops, t_exp=w.t_exp, iteration=k,
                           geometry_fp32=self.geometry_fp32, est_octant=self.est_oct,
                           gamma=self.gamma, stats=self.stats,
                           queue_capacity=self.queue_capacity, octant_table=self.octant_table)
        rec(2)
        nlte_solve(self.ctx, self.atom, self.cells, max_iter=self.max_iter, tol=self.tol,
                   guess=self.pops, warm_budget=warm_budget, pops=self.new, status=self.status,
                   iters=self.iters)
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
                "cells_converged": int(ok.sum()), "fallbacks": int((st == 1).sum()),
                "nlte_iters_mean": float(self.iters.float().mean()),
                "max_rel_change": float(d.max().item()) if d.numel() else None,
                "median_rel_change": float(d.median().item()) if d.numel() else None}


def run(ctx: Context, w, iterations=5, params=None, norm=None, warm_budget=30, geometry_fp32=True,
        queue_capacity=None, max_iter=200, tol=1e-10, device="cuda:0", log=None,
        octant_table=False):
    """Returns (pops [C, N], status [C], history) of `iterations` global
    iterations over workload w (see GlobalLoop)."""
    loop = GlobalLoop(ctx, w, device=device, geometry_fp32=geometry_fp32,
                      queue_capacity=queue_capacity, max_iter=max_iter, tol=tol,
                      warm_budget=warm_budget, octant_table=octant_table)
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
