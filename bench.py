"""Benchmark of the hot path on one MI355X.

One step = one global iteration of the method on the 50^3-cell workload
(125 000 cells, 5 000 lines, 1e7 packets, 2 species x 50 levels):
  Eq. A2 line opacities from the previous populations -> packet transport
  (FP32 geometry, FP64 estimators) -> photoexcitation rates -> MLP warm
  start -> NLTE solve of every cell from the MLP's populations (cold-start
  fallback for systems that do not converge within the warm budget).
Every step starts from the same previous populations (the cold start), so the
work per step is fixed. Inputs are resident in HBM before the timed region.
Setup (not timed) trains the warm-start network on solves of replicas of the
workload's cells (temperature, deposition and abundances redrawn).

Prints one JSON line. `value` is packet line-interactions per second of the
whole step; NLTE cell-solves per second of the whole step are reported beside
it, and so is the plain FP64 cold-start NLTE pass on the same rates, timed
after the step loop, with the largest population difference between the two.
Both NLTE passes run to the metric's population accuracy (--nlte-tol, 1e-8);
an untimed solve to 1e-12 then gives the accuracy each pass reached.
The roofline object covers the kernel that dominates the step, timed with HIP
events on the stream the library launches on.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "packet line-interactions/s + NLTE cell-solves/s vs plain FP64 at 1e-8 accuracy"
HBM_PEAK_GBS = 8000.0
FP64_VALU_PEAK_TFLOPS = 78.6


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-fraction", type=float, default=1.0,
                    help="fraction of packets and cells the oracle runs for cpu_baseline")
    ap.add_argument("--geometry-fp64", action="store_true")
    ap.add_argument("--replicas", type=int, default=8)
    ap.add_argument("--epochs", type=int, default=30)
    ap.add_argument("--warm-budget", type=int, default=30)
    ap.add_argument("--nlte-tol", type=float, default=1e-8,
                    help="population accuracy of both NLTE passes (the metric's 1e-8)")
    ap.add_argument("--no-spectrum", action="store_true",
                    help="skip the emergent-spectrum measurement")
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the batched three-stage NLTE measurement")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run one 1 GiB device-to-device copy before the step loop, whose "
                         "FETCH_SIZE/WRITE_SIZE counters calibrate the HBM traffic figures")
    return ap.parse_args()


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(sharding is described in DESIGN.md); run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import paper_2511_07539_amd as ex
    import synth

    dev = "cuda:0"
    torch.cuda.set_device(0)
    w = synth.paper_scale()
    ctx = ex.Context(0)
    atom = ex.Atom(ctx, w.atom)
    V = ex.cell_volume(w)
    cells0 = ex.cells_from_workload(w, device=dev)
    # previous populations: the cold start (not timed)
    prev, _, _ = ex.nlte_solve(ctx, atom, cells0, max_iter=0)
    prev = prev.clone()
    tau, fc = ex.line_tau(ctx, atom, prev, w.t_exp)
    grid = ex.grid_from_workload(w, device=dev, tau_ct=tau, fcorr_ct=fc)
    est = torch.empty((w.n_cells, w.n_lines), dtype=torch.float64, device=dev)
    stats = torch.empty(ex.STATS, dtype=torch.float64, device=dev)
    gamma = torch.empty((w.n_cells, w.atom.n_trans), dtype=torch.float64, device=dev)
    pops = torch.empty_like(prev)
    status = torch.empty(w.n_cells, dtype=torch.int32, device=dev)
    iters = torch.empty(w.n_cells, dtype=torch.int32, device=dev)
    cells = ex.Cells(w.t_exp, cells0.T_e, cells0.n_e, cells0.n_species, cells0.gamma_ion, gamma,
                     device=dev)
    fp32 = not args.geometry_fp64
    # learned warm start: trained on the method's own solves (setup, not timed)
    from paper_2511_07539_amd import warmstart
    t_train = time.perf_counter()
    gamma_train = warmstart.photoexcitation_rates(ctx, atom, w, dev)
    X, Y = warmstart.make_dataset(ctx, atom, w, n_replicas=args.replicas, gamma=gamma_train)
    del gamma_train
    params, norm, hist = warmstart.train(ctx, X, Y, epochs=args.epochs, batch=8192)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t_train
    dep = torch.as_tensor(w.deposition, device=dev)
    guess = torch.empty_like(prev)
    s = torch.cuda.current_stream()
    names = ["line_tau", "transport", "rates", "warm_start", "nlte"]

    def step(ev=None):
        def mark(i):
            if ev is not None:
                ev[i].record(s)
        mark(0)
        ex.line_tau(ctx, atom, prev, w.t_exp, tau=grid.tau_ct, fcorr=grid.fcorr_ct)
        mark(1)
        ex.transport(ctx, grid, w.seed, w.lambda_lo, w.lambda_hi, w.n_packets,
                     geometry_fp32=fp32, est=est, stats=stats)
        mark(2)
        ex.rates(ctx, atom, est, prev, V, out=gamma)
        mark(3)
        ex.nlte_warm_start(ctx, atom, cells, dep, params, norm, pops=pops)
        mark(4)
        ex.nlte_solve(ctx, atom, cells, pops=pops, use_guess=True, warm_budget=args.warm_budget,
                      tol=args.nlte_tol,
                      status=status, iters=iters)
        mark(5)

    if args.copy_calibration:
        src = torch.ones(1 << 27, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)  # reads 1 GiB, writes 1 GiB
        torch.cuda.synchronize()
        del src, dst
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(6)] for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(evs[k])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    parts = {n: 0.0 for n in names}
    for ev in evs:
        for i, n in enumerate(names):
            parts[n] += ev[i].elapsed_time(ev[i + 1])
    parts = {n: v / args.steps for n, v in parts.items()}
    ms = (t1 - t0) * 1e3 / args.steps
    st = ex.stats_dict(stats)
    n_inter = st["n_inter"]
    st_np = status.cpu().numpy()
    conv = int((st_np <= 1).sum())
    fallbacks = int((st_np == 1).sum())
    it_warm = iters.cpu().numpy()
    # the plain FP64 pass from the cold start on the same rates, for comparison
    pops_cold = torch.empty_like(pops)
    st_cold = torch.empty_like(status)
    it_cold = torch.empty_like(iters)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    ex.nlte_solve(ctx, atom, cells, pops=pops_cold, status=st_cold, iters=it_cold,
                  tol=args.nlte_tol)
    e1.record(s)
    torch.cuda.synchronize()
    cold_ms = e0.elapsed_time(e1)
    both = (st_cold == 0) & (status <= 1)
    pw, pc = pops[both], pops_cold[both]
    warm_vs_cold = float(((pw - pc).abs() / pc).max().item()) if int(both.sum()) else None
    # accuracy of both passes against a tight FP64 solve (tol 1e-12, untimed)
    ref, st_ref, _ = ex.nlte_solve(ctx, atom, cells, tol=1e-12, max_iter=400)
    ok_ref = st_ref == 0

    def max_rel(p, st):
        m = ok_ref & (st <= 1)
        return float((((p - ref).abs() / ref)[m]).max().item()) if int(m.sum()) else None
    accuracy = {"tol": args.nlte_tol, "reference_tol": 1e-12,
                "reference_converged": int(ok_ref.sum().item()),
                "warm_max_rel": max_rel(pops, status), "cold_max_rel": max_rel(pops_cold, st_cold)}
    del ref
    value = n_inter / (ms * 1e-3)
    solves = w.n_cells / (ms * 1e-3)

    # roofline of the dominant kernel
    dom = max(parts, key=parts.get)
    if dom == "transport":
        bytes_alg = 8.0 * w.n_cells * w.n_lines + 16.0 * w.n_cells + 16.0 * w.n_lines
        ach = bytes_alg / (parts["transport"] * 1e-3) / 1e9
        roof = {"kernel": "extrass_transport (fill + transport kernels)", "bound": "hbm",
                "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": ach / HBM_PEAK_GBS,
                "traffic": recorded_traffic("extrass_transport"), "algorithmic_bytes": bytes_alg}
    else:
        it_np = it_warm
        S = w.atom.n_species
        Ns = np.diff(w.atom.species_offset)
        # state reductions: about two per iteration (fixed-point or Newton + trial),
        # (2/3) N^3 flops each
        flops = float(sum(2.0 * it_np.sum() * (2.0 / 3.0) * n ** 3 for n in Ns))
        ach = flops / (parts[dom] * 1e-3) / 1e12
        roof = {"kernel": f"extrass_{dom}", "bound": "alu", "achieved": ach,
                "peak": FP64_VALU_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": ach / FP64_VALU_PEAK_TFLOPS, "traffic": recorded_traffic("extrass_nlte"),
                "algorithmic_flops": flops}

    out = {
        "metric": METRIC, "value": value, "unit": "line-interactions/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": w.name, "cells": w.n_cells, "lines": w.n_lines,
                   "packets": w.n_packets, "levels": w.atom.n_levels,
                   "species": w.atom.n_species, "geometry": "fp32" if fp32 else "fp64",
                   "parallelism": "single GPU"},
        "nlte_cell_solves_per_s": solves,
        "interactions_per_step": n_inter,
        "cells_converged": conv,
        "nlte_fallbacks": fallbacks,
        "nlte_iters_mean": {"warm": float(it_warm.mean()), "cold": float(it_cold.float().mean())},
        "nlte_plain_fp64_cold_ms": cold_ms,
        "nlte_warm_vs_cold_max_rel": warm_vs_cold,
        "nlte_accuracy": accuracy,
        "warm_start_training": {"samples": int(X.shape[0]), "epochs": args.epochs,
                                "loss_first": hist[0], "loss_last": hist[-1],
                                "setup_s": t_train},
        "ms_parts": parts,
        "roofline": roof,
    }
    if not args.no_spectrum:
        out["spectrum"] = bench_spectrum(ex, ctx, w, grid, fp32)
    if not args.no_batched:
        del est, grid, gamma
        torch.cuda.empty_cache()
        out["batched_nlte"] = bench_batched(ex, ctx)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, prev.cpu().numpy(), args.cpu_fraction)
    print(json.dumps(out), flush=True)


def bench_spectrum(ex, ctx, w, grid, fp32):
    """Emergent spectra of the step's packets (Sec. 2.3): 20 x 20 viewers and
    0.1 % log-wavelength bins over the band widened by the Doppler shifts. One
    untimed transport writes the per-packet records; the binning of all 1e7
    records (64 B each) is timed with HIP events."""
    import math

    import torch
    _, st, pk = ex.transport(ctx, grid, w.seed, w.lambda_lo, w.lambda_hi, w.n_packets,
                             geometry_fp32=fp32, packets_out=True)
    lo, hi = w.lambda_lo * 0.97, w.lambda_hi * 1.03
    n_lam = int(math.ceil(math.log(hi / lo) / math.log(1.001)))
    bins = (20, 20, n_lam, lo, hi)
    ph, en = ex.spectrum(ctx, pk, *bins)  # warm-up
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 5
    e0.record(s)
    for _ in range(reps):
        ph.zero_()
        en.zero_()
        ex.spectrum(ctx, pk, *bins, photons=ph, energy=en)
    e1.record(s)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    sd = ex.stats_dict(st)
    rec_bytes = pk.numel() * 8
    return {"viewers": [20, 20], "lambda_bins": n_lam,
            "lambda_range_cm": [lo, hi], "ms_binning_incl_zero": ms,
            "record_bytes": rec_bytes, "record_read_tb_per_s": rec_bytes / (ms * 1e-3) / 1e12,
            "escaped_packets": int(sd["n_escaped"]),
            "escaped_photon_fraction": sd["w_esc"] / sd["w_emit"],
            "binned_photons_vs_escaped": float(ph.sum()) / sd["w_esc"]}


def bench_batched(ex, ctx):
    """The batched three-stage NLTE problem (125 000 cells, 20-300 levels per
    stage): tuned launch shape, then one FP64 solve and one FP32-factor solve
    with two FP64 refinement sweeps, each timed with HIP events on the stream
    the library launches on. Not part of the step."""
    import numpy as np
    import torch

    import synth
    b = synth.batched()
    prob = ex.Batched(b)
    L = b.level_count.reshape(-1, 3).astype(np.float64)
    flops = float(((2.0 / 3.0) * np.maximum(L - 1, 0) ** 3).sum())  # excited levels eliminated
    s = torch.cuda.current_stream()
    res = {"workload": b.name, "cells": b.n_cells, "levels_total": int(b.level_count.sum()),
           "flops_per_factorisation_pass": flops}
    for name, f32, refine in (("fp64", False, 0), ("fp32_refine2", True, 2)):
        shape, table = ex.batched_tune(ctx, prob, factor_fp32=f32)
        pops, status = ex.batched_solve(ctx, prob, factor_fp32=f32, refine=refine, tol=1e-10)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s)
        pops, status = ex.batched_solve(ctx, prob, factor_fp32=f32, refine=refine, tol=1e-10,
                                        pops=pops, status=status)
        e1.record(s)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        st = status.cpu().numpy()
        res[name] = {"ms": ms, "cell_solves_per_s": b.n_cells / (ms * 1e-3),
                     "tuned_panel_per_cu": list(shape), "status_counts": np.bincount(st, minlength=3).tolist(),
                     "achieved_tflops_factor_equivalent": flops / (ms * 1e-3) / 1e12}
        del pops, status
    return res


def recorded_traffic(key):
    """HBM bytes per launch of a kernel from the committed FETCH_SIZE/WRITE_SIZE
    counter record (scaled by the copy calibration), or None when the kernel's
    sources have changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "hbm_traffic.json")
    try:
        with open(path) as f:
            rec = json.load(f)["kernels"][key]
        m = hashlib.sha256()
        for src in rec["sources"]:
            with open(os.path.join(ROOT, src), "rb") as f:
                m.update(f.read())
    except (OSError, KeyError, ValueError):
        return None
    return rec["bytes"] if m.hexdigest()[:16] == rec["source_hash"] else None


def cpu_baseline(w, prev, frac):
    """The FP64 oracle on the host, as it stands, on a bounded sample: the first
    `frac` of the packets and of the cells; the whole-step time is scaled up
    from that sample."""
    import numpy as np

    import oracle
    nthreads = oracle.default_threads()
    tau, fc = oracle.line_tau(prev, w.atom, w.t_exp)
    inp = oracle.transport_inputs_from_workload(w, tau_ct=tau, fcorr_ct=fc)
    P = int(w.n_packets * frac)
    t0 = time.perf_counter()
    r = oracle.transport(inp, first=0, count=P, nthreads=nthreads)
    t1 = time.perf_counter()
    Cs = int(w.n_cells * frac)
    cells = np.arange(Cs)
    rec = r["records"]
    sel = rec["cell"] < Cs
    est = np.zeros(Cs * w.n_lines)
    np.add.at(est, rec["cell"][sel].astype(np.int64) * w.n_lines + rec["line"][sel],
              rec["value"][sel])
    V = (2 * w.beta_max / w.n * 2.99792458e10 * w.t_exp) ** 3
    gpe = oracle.rates(est, prev[:Cs], w.atom, V)
    ninp = oracle.nlte_inputs_from_workload(w, gamma_pe=gpe, cells=cells)
    t2 = time.perf_counter()
    oracle.nlte(ninp, guess=prev[:Cs], nthreads=nthreads)
    t3 = time.perf_counter()
    t_step = (t1 - t0) / frac + (t3 - t2) / frac
    inter_step = r["stats"]["n_inter"] / frac
    return {"value": inter_step / t_step, "unit": "line-interactions/s", "cores": nthreads,
            "kind": "oracle", "nlte_cell_solves_per_s": w.n_cells / t_step,
            "sample": f"first {P} packets and first {Cs} cells ({frac:.0%}) of the workload; "
                      f"transport {t1 - t0:.2f} s, NLTE {t3 - t2:.2f} s, scaled to the full step"}


if __name__ == "__main__":
    main()
