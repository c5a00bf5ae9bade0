"""Global iterations of the method on one GPU: the outer loop of radiative
transfer and statistical equilibrium (Sec. 2.2, 2.3).

One iteration: Eq. A2 line opacities from the current populations ->
packet transport streamed over the 8 velocity octants, with photoexcitation
rates accumulated octant by octant -> NLTE solve of every cell, started from
the previous iteration's populations. The first iteration starts from the
learned warm start (or the cold start). This module only orders library
calls and keeps the tensors; every step runs in the library's kernels.

`python -m paper_2511_07539_amd.globalloop` runs the 100^3-cell, 30000-line,
1e8-packet case for 5 iterations and prints one JSON line.
"""
from __future__ import annotations

import json
import sys
import time

import numpy as np
import torch

from . import (Atom, Cells, Context, cell_volume, cells_from_workload, grid_from_workload,
               line_tau, nlte_solve, nlte_warm_start, stats_dict, transport_streamed)


def run(ctx: Context, w, iterations=5, params=None, norm=None, warm_budget=30, geometry_fp32=True,
        queue_capacity=None, max_iter=200, tol=1e-10, device="cuda:0", log=None,
        octant_table=False):
    """Returns (pops [C, N], status [C], history). With params/norm the first
    iteration's populations come from the MLP, else from the cold start. The
    streamed transport sums the rates per interaction (no octant estimator
    table) unless octant_table is set."""
    atom = Atom(ctx, w.atom)
    cells0 = cells_from_workload(w, device=device)
    V = cell_volume(w)
    s = torch.cuda.current_stream()
    gamma = torch.zeros((w.n_cells, w.atom.n_trans), dtype=torch.float64, device=device)
    cells = Cells(w.t_exp, cells0.T_e, cells0.n_e, cells0.n_species, cells0.gamma_ion, gamma,
                  device=device)
    if params is not None:
        pops = nlte_warm_start(ctx, atom, cells, torch.as_tensor(w.deposition, device=device),
                               params, norm)
    else:
        pops, _, _ = nlte_solve(ctx, atom, cells0, max_iter=0)
    tau, fc = line_tau(ctx, atom, pops, w.t_exp)
    grid = grid_from_workload(w, device=device, tau_ct=tau, fcorr_ct=fc)
    del tau, fc
    history = []
    status = None
    lv_species = torch.as_tensor(
        np.repeat(np.arange(w.atom.n_species), np.diff(w.atom.species_offset)), device=device)
    ns_lv = cells0.n_species.view(w.n_cells, -1)[:, lv_species]
    half = w.n // 2
    est_oct = (torch.empty((half ** 3, w.n_lines), dtype=torch.float64, device=device)
               if octant_table else None)
    new = torch.empty_like(pops)
    st = torch.empty(w.n_cells, dtype=torch.int32, device=device)
    it_ = torch.empty(w.n_cells, dtype=torch.int32, device=device)
    for k in range(iterations):
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
        ev[0].record(s)
        line_tau(ctx, atom, pops, w.t_exp, tau=grid.tau_ct, fcorr=grid.fcorr_ct)
        ev[1].record(s)
        _, stats, _ = transport_streamed(ctx, grid, w.seed, w.lambda_lo, w.lambda_hi, w.n_packets,
                                         atom=atom, pops=pops, cell_volume=V, iteration=k,
                                         geometry_fp32=geometry_fp32, est_octant=est_oct,
                                         gamma=gamma, queue_capacity=queue_capacity,
                                         octant_table=octant_table)
        ev[2].record(s)
        nlte_solve(ctx, atom, cells, max_iter=max_iter, tol=tol, guess=pops,
                   warm_budget=warm_budget if k == 0 and params is not None else 0,
                   pops=new, status=st, iters=it_)
        ev[3].record(s)
        torch.cuda.synchronize()
        ok = st <= 1
        # change of the populated levels (>= 1e-10 of their species); emptier
        # levels follow the Monte Carlo noise of their photoexcitation rates
        sig = ok[:, None] & (new >= 1e-10 * ns_lv)
        d = ((new - pops).abs() / new.clamp_min(1e-300))[sig]
        change = float(d.max().item()) if d.numel() else None
        change_med = float(d.median().item()) if d.numel() else None
        sd = stats_dict(stats)
        rec = {"iteration": k + 1, "ms_line_tau": ev[0].elapsed_time(ev[1]),
               "ms_transport": ev[1].elapsed_time(ev[2]), "ms_nlte": ev[2].elapsed_time(ev[3]),
               "interactions": sd["n_inter"], "escaped_fraction": sd["w_esc"] / sd["w_emit"],
               "cells_converged": int(ok.sum()), "fallbacks": int((st == 1).sum()),
               "nlte_iters_mean": float(it_.float().mean()), "max_rel_change": change,
               "median_rel_change": change_med}
        history.append(rec)
        if log:
            log(rec)
        pops, new = new, pops
        status = st.clone()
    return pops, status, history


def main(argv=None):
    import argparse

    import synth
    from . import warmstart

    ap = argparse.ArgumentParser()
    ap.add_argument("--iterations", type=int, default=5)
    ap.add_argument("--no-mlp", action="store_true", help="start from the cold start")
    ap.add_argument("--epochs", type=int, default=30)
    ap.add_argument("--queue-capacity", type=int, default=0)
    args = ap.parse_args(argv)
    ctx = Context(0)
    params = norm = None
    t0 = time.perf_counter()
    if not args.no_mlp:
        # the warm start is trained on solves of the 50^3 workload's pipeline
        w2 = synth.paper_scale()
        a2 = Atom(ctx, w2.atom)
        gam = warmstart.photoexcitation_rates(ctx, a2, w2)
        X, Y = warmstart.make_dataset(ctx, a2, w2, n_replicas=8, gamma=gam)
        del gam
        params, norm, _ = warmstart.train(ctx, X, Y, epochs=args.epochs, batch=8192)
        del X, Y, a2, w2
        torch.cuda.empty_cache()
    t_train = time.perf_counter() - t0
    w = synth.large()
    print(f"workload {w.name}: {w.n_cells} cells, {w.n_lines} lines, {w.n_packets} packets",
          file=sys.stderr, flush=True)
    t1 = time.perf_counter()
    pops, status, hist = run(ctx, w, args.iterations, params, norm,
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
