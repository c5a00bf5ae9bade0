"""Benchmark of the hot path on one MI355X.

One step = the whole method on the largest single-GPU workload, clumpy100:
100^3 = 1e6 cells, 30 000 lines, 1e8 packets per iteration, 2 species x 50
levels, 5 global iterations. Each iteration: Eq. A2 line opacities from the
current populations -> packet transport streamed over the 8 velocity octants
(FP32 geometry, FP64 weights), photoexcitation rates summed per interaction
-> NLTE solve of every cell to the metric's population accuracy (1e-8). The
first iteration starts from the learned warm start (cold-start fallback past
the warm budget), later ones from the previous iteration's populations.
Every step starts from the same MLP populations, so the work per step is
fixed. Inputs are resident in HBM before the timed region; the step does no
host-to-device copies and no allocations.

Setup (not timed): the warm-start network is trained on solves of replicas of
the 50^3 workload's cells (its own transport, rates and NLTE solves).

Prints one JSON line. `value` is packet line-interactions per second of the
whole step; NLTE cell-solves per second are reported beside it, with the
plain FP64 cold-start NLTE pass and the network-started pass on the last
iteration's rates, timed after the step loop. The accuracy of both NLTE passes is measured against the
oracle (tol 1e-12) on a sample of cells with seeded rates, solved by both.
The roofline object covers the kernel that dominates the step, timed with HIP
events on the stream the library launches on. Extra keys: the one-iteration
50^3 step, emergent spectra, and the batched three-stage NLTE problem.
"""
import argparse
import json
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "packet line-interactions/s + NLTE cell-solves/s vs plain FP64 at 1e-8 accuracy"
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6
ITERATIONS = 5
EXTRAS = ("clumpy50_step", "clumpy100_octant_table", "deterministic_rays", "photoionisation",
          "spherical_grid", "spectrum", "batched_nlte")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-packets", type=int, default=10_000_000,
                    help="packets of the first iteration the oracle transports for cpu_baseline")
    ap.add_argument("--cpu-cells", type=int, default=16_000,
                    help="cells the oracle solves for cpu_baseline and the accuracy check")
    ap.add_argument("--epochs", type=int, default=30)
    ap.add_argument("--warm-budget", type=int, default=30)
    ap.add_argument("--nlte-precision", choices=("mixed", "fp64"), default="mixed",
                    help="the step's NLTE pass: fixed-point steps in FP32 with FP64 residuals "
                         "and Newton systems (mixed), or FP64 throughout; the other is timed "
                         "beside it")
    ap.add_argument("--nlte-tol", type=float, default=1e-8,
                    help="population accuracy of the NLTE solves (the metric's 1e-8)")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the 50^3 step, spectrum and batched measurements")
    ap.add_argument("--extras", default=",".join(EXTRAS),
                    help="comma-separated extra measurements to run (default: all of "
                         + ", ".join(EXTRAS) + ")")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run one 1 GiB device-to-device copy before the step loop, whose "
                         "FETCH_SIZE/WRITE_SIZE counters calibrate the HBM traffic figures")
    return ap.parse_args()


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def nlte_flops_per_iteration(atom):
    """Algorithmic FP64 flops of one NLTE iteration of one system, per species:
    two state reductions (a fixed-point or Newton step and its residual), each
    eliminating the excited levels of every ion stage in its own block,
    (2/3) (L_z - 1)^3 per stage of L_z levels."""
    import numpy as np
    out = []
    for s in range(atom.n_species):
        lv = atom.level_ion[atom.species_offset[s]:atom.species_offset[s + 1]]
        L = np.bincount(lv).astype(np.float64)
        out.append(2.0 * float(((2.0 / 3.0) * np.maximum(L - 1, 0) ** 3).sum()))
    return out


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
    from paper_2511_07539_amd import globalloop, warmstart

    dev = "cuda:0"
    torch.cuda.set_device(0)
    ctx = ex.Context(0)
    t_setup = time.perf_counter()
    w50 = synth.paper_scale()
    say("setup: warm-start training on the 50^3 pipeline")
    params, norm, hist = warmstart.train_on_workload(ctx, w50, epochs=args.epochs)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t_setup
    chosen = set() if args.no_extras else {e for e in args.extras.split(",") if e}
    unknown = chosen - set(EXTRAS)
    if unknown:
        print(f"bench.py: unknown extras {sorted(unknown)}", file=sys.stderr)
        sys.exit(2)
    extras = {}
    if "clumpy50_step" in chosen:
        extras["clumpy50_step"] = bench_clumpy50(ex, ctx, w50, params, norm, args)
        torch.cuda.empty_cache()
    w = synth.large()
    say(f"setup: {w.name} resident on the GPU")
    mixed_step = args.nlte_precision == "mixed"
    loop = globalloop.GlobalLoop(ctx, w, tol=args.nlte_tol, warm_budget=args.warm_budget,
                                 nlte_fp32=mixed_step)
    s = torch.cuda.current_stream()
    inter = torch.zeros(ITERATIONS, dtype=torch.float64, device=dev)
    iters_sum = torch.zeros((ITERATIONS, 2), dtype=torch.float64, device=dev)

    def step(evs=None):
        loop.start(params, norm)
        for k in range(ITERATIONS):
            loop.iterate(k, args.warm_budget if k == 0 else 0,
                         None if evs is None else evs[k])
            inter[k].copy_(loop.stats[4])
            iters_sum[k, 0].copy_(loop.iters.sum())
            iters_sum[k, 1].copy_((loop.status <= 1).sum())

    if args.copy_calibration:
        src = torch.ones(1 << 27, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)  # reads 1 GiB, writes 1 GiB
        torch.cuda.synchronize()
        del src, dst
    say("warm-up steps")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    evs = [[[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(ITERATIONS)]
           for _ in range(args.steps)]
    say("timed steps")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(evs[k])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms = (t1 - t0) * 1e3 / args.steps
    names = ["line_tau", "transport", "nlte"]
    per_it = np.zeros((ITERATIONS, 3))
    for e in evs:
        for k in range(ITERATIONS):
            for i in range(3):
                per_it[k, i] += e[k][i].elapsed_time(e[k][i + 1])
    per_it /= args.steps
    parts = {n: float(per_it[:, i].sum()) for i, n in enumerate(names)}
    inter_np = inter.cpu().numpy()
    n_inter = float(inter_np.sum())
    it_np = iters_sum.cpu().numpy()
    status = loop.status.cpu().numpy()
    value = n_inter / (ms * 1e-3)
    solves = ITERATIONS * w.n_cells / (ms * 1e-3)

    # the plain FP64 pass from the cold start on the last iteration's rates
    say("plain FP64 cold-start NLTE pass")
    pops_c = torch.empty_like(loop.pops)
    st_c = torch.empty_like(loop.status)
    it_c = torch.empty_like(loop.iters)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    ex.nlte_solve(ctx, loop.atom, loop.cells, tol=args.nlte_tol, pops=pops_c, status=st_c,
                  iters=it_c)
    e1.record(s)
    torch.cuda.synchronize()
    cold_ms = e0.elapsed_time(e1)
    cold_iters = float(it_c.float().mean())
    cold_ok = int((st_c == 0).sum())
    # the warm-started pass on the same rates: BF16 network guess (fused
    # inference included in the time), then the FP64 solve from it
    say("MLP-warm-started pass on the same rates")
    e0.record(s)
    ex.nlte_warm_start(ctx, loop.atom, loop.cells, loop.deposition, params, norm, pops=pops_c)
    ex.nlte_solve(ctx, loop.atom, loop.cells, tol=args.nlte_tol, guess=pops_c,
                  warm_budget=args.warm_budget, pops=pops_c, status=st_c, iters=it_c,
                  factor_fp32=mixed_step)
    e1.record(s)
    torch.cuda.synchronize()
    warm_same_ms = e0.elapsed_time(e1)
    warm_same = {"ms": warm_same_ms, "iters_mean": float(it_c.float().mean()),
                 "converged": int((st_c <= 1).sum()), "cold_fallbacks": int((st_c == 1).sum())}
    del pops_c, st_c, it_c

    # the same step with the other NLTE precision (mixed: fixed-point steps
    # reduced in FP32, residuals and Newton systems in FP64)
    other = "fp64" if mixed_step else "mixed"
    say(f"step with the {other} NLTE pass")
    loop.nlte_fp32 = not mixed_step
    ev_m = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(ITERATIONS)]
    step(ev_m)
    torch.cuda.synchronize()
    loop.nlte_fp32 = mixed_step
    nlte_m = [ev_m[k][2].elapsed_time(ev_m[k][3]) for k in range(ITERATIONS)]
    it_m = iters_sum.cpu().numpy()
    other_pass = {"nlte_precision": other, "nlte_ms_per_iteration": nlte_m,
                  "warm_later_iterations_ms": float(np.mean(nlte_m[1:])),
                  "nlte_iters_mean": (it_m[:, 0] / w.n_cells).tolist(),
                  "cells_converged_per_iteration": it_m[:, 1].astype(int).tolist()}

    # roofline of the dominant kernel
    fl = nlte_flops_per_iteration(w.atom)
    flops = float(it_np[:, 0].sum() * sum(fl))   # iteration count is the larger of the species'
    dom = max(parts, key=parts.get)
    if dom == "nlte":
        ach = flops / (parts["nlte"] * 1e-3) / 1e12
        roof = {"kernel": "extrass_nlte_solve (k_nlte<0, 21, %s>)" % ("true" if mixed_step else "false"),
                "bound": "alu", "achieved": ach,
                "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": ach / FP64_PEAK_TFLOPS,
                "traffic": recorded_traffic("extrass_nlte_clumpy100_mixed" if mixed_step
                                            else "extrass_nlte_clumpy100"),
                "algorithmic_flops": flops,
                "flops_per_system_iteration": fl}
    else:
        bytes_alg = ITERATIONS * (16.0 * w.n_cells * w.atom.n_trans + 16.0 * w.n_lines)
        ach = bytes_alg / (parts[dom] * 1e-3) / 1e9
        roof = {"kernel": f"extrass_{dom}", "bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": ach / HBM_PEAK_GBS, "traffic": None,
                "algorithmic_bytes": bytes_alg}
    out = {
        "metric": METRIC, "value": value, "unit": "line-interactions/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": w.name, "cells": w.n_cells, "lines": w.n_lines,
                   "packets_per_iteration": w.n_packets, "global_iterations": ITERATIONS,
                   "subdomains": 8, "levels": w.atom.n_levels, "species": w.atom.n_species,
                   "geometry": "fp32", "nlte_tol": args.nlte_tol,
                   "nlte_precision": ("mixed: fixed-point steps fp32, residuals and Newton fp64"
                                      if mixed_step else "fp64")},
        "nlte_cell_solves_per_s": solves,
        "interactions_per_step": n_inter,
        "interactions_per_iteration": inter_np.tolist(),
        "ms_parts": parts,
        "ms_per_iteration": {n: per_it[:, i].tolist() for i, n in enumerate(names)},
        "nlte_iters_mean": (it_np[:, 0] / w.n_cells).tolist(),
        "cells_converged_per_iteration": it_np[:, 1].astype(int).tolist(),
        "nlte_fallbacks_last": int((status == 1).sum()),
        "nlte_vs_plain_fp64": {
            "warm_first_iteration_ms": float(per_it[0, 2]),
            "warm_later_iterations_ms": float(per_it[1:, 2].mean()),
            "plain_fp64_cold_ms": cold_ms, "plain_fp64_cold_iters_mean": cold_iters,
            "plain_fp64_cold_converged": cold_ok,
            "mlp_warm_same_rates": warm_same,
            "cell_solves_per_s_warm_later": w.n_cells / (per_it[1:, 2].mean() * 1e-3),
            "cell_solves_per_s_plain_fp64": w.n_cells / (cold_ms * 1e-3),
            "step_nlte_precision": args.nlte_precision,
            "same_step_other_precision": other_pass},
        "warm_start_training": {"workload": w50.name, "epochs": args.epochs,
                                "loss_first": hist[0], "loss_last": hist[-1],
                                "setup_s": t_train},
        "roofline": roof,
    }
    say("accuracy sample")
    sample, gpe_s = accuracy_sample(w, args.cpu_cells)
    out["nlte_accuracy"], ref = nlte_accuracy(ex, ctx, loop, w, sample, gpe_s, params, norm, args)
    if "clumpy100_octant_table" in chosen:
        out["clumpy100_octant_table"] = bench_octant_table(ex, ctx, loop, w)
    del loop
    torch.cuda.empty_cache()
    out.update(extras)
    legs = {"deterministic_rays": lambda: bench_rays(ex, ctx, w50),
            "photoionisation": lambda: bench_photoion(ex, ctx, w50),
            "spherical_grid": lambda: bench_spherical(ex, ctx),
            "spectrum": lambda: bench_spectrum(ex, ctx, w50),
            "batched_nlte": lambda: bench_batched(ex, ctx)}
    for name, leg in legs.items():
        if name in chosen:
            out[name] = leg()
            torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        say("cpu_baseline: oracle on a sample")
        out["cpu_baseline"] = cpu_baseline(w, n_inter, sample, gpe_s, ref, args)
    print(json.dumps(out), flush=True)


def bench_octant_table(ex, ctx, loop, w):
    """The 100^3 streamed transport with each octant's [C/8 x L] FP64
    estimator table resident (30 GB at 30 000 lines), flushed into the rates
    after every visit, against the step's table-free mode (rates summed per
    interaction), on the same opacities and populations (the loop's last);
    HIP events, one warm-up call each. Both take the same events, so their
    rates agree up to the order of the additions."""
    import numpy as np
    import torch
    dev = "cuda:0"
    s = torch.cuda.current_stream()
    ex.line_tau(ctx, loop.atom, loop.pops, w.t_exp, tau=loop.grid.tau_ct, fcorr=loop.grid.fcorr_ct)
    half = w.n // 2
    table = torch.empty((half ** 3, w.n_lines), dtype=torch.float64, device=dev)
    g_tab = torch.empty_like(loop.gamma)
    g_dir = torch.empty_like(loop.gamma)
    stats = torch.empty(ex.STATS, dtype=torch.float64, device=dev)
    res = {"workload": w.name, "octant_table_gb": table.numel() * 8 / 1e9}
    for name, est, gam in (("octant_table", table, g_tab), ("direct", None, g_dir)):
        times = []
        for _ in range(2):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(s)
            ex.transport_streamed(ctx, loop.grid, w.seed, w.lambda_lo, w.lambda_hi, w.n_packets,
                                  atom=loop.atom, pops=loop.pops, t_exp=w.t_exp, iteration=0,
                                  geometry_fp32=True, est_octant=est, gamma=gam, stats=stats,
                                  octant_table=est is not None)
            e1.record(s)
            torch.cuda.synchronize()
            times.append(e0.elapsed_time(e1))
        sd = ex.stats_dict(stats)
        res[name] = {"ms": times[-1], "interactions": sd["n_inter"],
                     "line_interactions_per_s": sd["n_inter"] / (times[-1] * 1e-3)}
    on = (g_dir > 0) & (g_tab > 0)
    rel = ((g_tab - g_dir).abs() / g_dir.clamp_min(1e-300))[on]
    res["rates_max_rel_diff"] = float(rel.max()) if rel.numel() else 0.0
    res["rates_zero_pattern_equal"] = bool(torch.equal(g_dir > 0, g_tab > 0))
    del table, g_tab, g_dir
    torch.cuda.empty_cache()
    return res


def accuracy_sample(w, n):
    """Cells (evenly spaced over the grid) and seeded photoexcitation rates for
    the accuracy check; both sides solve exactly these inputs."""
    import numpy as np
    n = min(n, w.n_cells)
    cells = np.linspace(0, w.n_cells - 1, n).astype(np.int64)
    g = np.random.default_rng(2511)
    T = w.atom.n_trans
    gpe = np.abs(g.standard_normal((n, T))) * 10 ** g.uniform(-8, 0, (n, T))
    return cells, gpe


def nlte_accuracy(ex, ctx, loop, w, cells, gpe, params, norm, args):
    """Componentwise max |n - n_oracle| / n_oracle of the GPU's NLTE solves on
    the sample: the plain FP64 cold start and the MLP warm start, each also
    with the fixed-point steps reduced in FP32, all at the bench's tol, against
    the oracle at 1e-12 on the same seeded inputs."""
    import numpy as np
    import torch

    import oracle
    S = w.atom.n_species
    cl = ex.Cells(w.t_exp, w.T_e[cells], w.n_e[cells], w.n_species.reshape(-1, S)[cells],
                  w.gamma_ion.reshape(-1, S, 3)[cells], gpe)
    pc, sc, _ = ex.nlte_solve(ctx, loop.atom, cl, tol=args.nlte_tol)
    guess = ex.nlte_warm_start(ctx, loop.atom, cl, w.deposition[cells], params, norm)
    pw, sw, _ = ex.nlte_solve(ctx, loop.atom, cl, tol=args.nlte_tol, guess=guess,
                              warm_budget=args.warm_budget)
    pcm, scm, _ = ex.nlte_solve(ctx, loop.atom, cl, tol=args.nlte_tol, factor_fp32=True)
    pwm, swm, _ = ex.nlte_solve(ctx, loop.atom, cl, tol=args.nlte_tol, guess=guess,
                                warm_budget=args.warm_budget, factor_fp32=True)
    torch.cuda.synchronize()
    inp = oracle.NLTEInputs(w.atom, w.t_exp, w.T_e[cells], w.n_e[cells],
                            w.n_species.reshape(-1, S)[cells].ravel(),
                            w.gamma_ion.reshape(-1, S, 3)[cells].ravel(), gpe.ravel())
    t0 = time.perf_counter()
    po, so, _ = oracle.nlte(inp, tol=1e-12)
    t_or = time.perf_counter() - t0

    def rel(p, st):
        p, st = p.cpu().numpy(), st.cpu().numpy()
        ok = (so == 0) & (st <= 1)
        r = np.abs(p[ok] - po[ok]) / po[ok]
        return {"max_rel": float(r.max()), "cells_above_tol": int((r.max(1) > args.nlte_tol).sum()),
                "compared": int(ok.sum())}
    acc = {"tol": args.nlte_tol, "reference": "oracle, tol 1e-12", "cells": int(len(cells)),
           "oracle_converged": int((so == 0).sum()),
           "plain_fp64_cold": rel(pc, sc), "mlp_warm": rel(pw, sw),
           "mixed_cold": rel(pcm, scm), "mixed_mlp_warm": rel(pwm, swm)}
    return acc, {"oracle_s": t_or, "status": so}


def host_cpu():
    info = {"os_cpu_count": os.cpu_count()}
    try:
        info["affinity"] = len(os.sched_getaffinity(0))
    except AttributeError:
        pass
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            k, _, v = line.partition(":")
            if k.strip() in ("Model name", "Socket(s)", "Core(s) per socket", "Thread(s) per core"):
                info[k.strip()] = v.strip()
    except (OSError, subprocess.SubprocessError):
        pass
    return info


def cpu_baseline(w, inter_step, sample, gpe, ref, args):
    """The FP64 oracle on the host, as it stands, on a bounded sample of the
    step: its transport on the first packets of the first iteration (line
    opacities from the oracle's own cold-start populations), and its NLTE
    solve (tol 1e-12) of the accuracy sample's cells. The whole step's time is
    scaled up from those rates: the step's interactions at the sample's
    interaction rate, plus ITERATIONS solves of every cell at the sample's
    per-cell time."""
    import numpy as np

    import oracle
    nthreads = oracle.default_threads()
    inp_n = oracle.nlte_inputs_from_workload(w)
    cold, _, _ = oracle.nlte(inp_n, max_iter=0)
    tau, fc = oracle.line_tau(cold, w.atom, w.t_exp)
    del cold, inp_n
    inp = oracle.transport_inputs_from_workload(w, tau_ct=tau, fcorr_ct=fc)
    P = min(args.cpu_packets, w.n_packets)
    t0 = time.perf_counter()
    r = oracle.transport(inp, first=0, count=P, nthreads=nthreads)
    t_tr = time.perf_counter() - t0
    rate = r["stats"]["n_inter"] / t_tr
    t_nlte_cell = ref["oracle_s"] / len(sample)
    t_step = inter_step / rate + ITERATIONS * w.n_cells * t_nlte_cell
    return {"value": inter_step / t_step, "unit": "line-interactions/s", "cores": nthreads,
            "kind": "oracle", "nlte_cell_solves_per_s": 1.0 / t_nlte_cell,
            "transport_interactions_per_s": rate, "host": host_cpu(),
            "sample": f"transport of packets [0, {P}) of iteration 1 ({r['stats']['n_inter']:.3g} "
                      f"interactions, {t_tr:.1f} s); NLTE of {len(sample)} cells at tol 1e-12 "
                      f"({ref['oracle_s']:.1f} s); scaled to the step's {inter_step:.3g} "
                      f"interactions and {ITERATIONS} x {w.n_cells} cell solves"}


def bench_clumpy50(ex, ctx, w, params, norm, args):
    """One global iteration on the 50^3 workload (125 000 cells, 5000 lines,
    1e7 packets) with the dense [C x L] FP64 estimator table: opacities ->
    transport -> rates -> MLP warm start -> NLTE (the step's NLTE precision),
    from the cold-start populations; HIP events per part; the transport's HBM roofline counts the
    table written once (8 C L bytes) plus the per-cell and per-line inputs."""
    import torch
    dev = "cuda:0"
    atom = ex.Atom(ctx, w.atom)
    cells0 = ex.cells_from_workload(w, device=dev)
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
    dep = torch.as_tensor(w.deposition, device=dev)
    s = torch.cuda.current_stream()
    names = ["line_tau", "transport", "rates", "warm_start", "nlte"]

    def step(ev=None):
        mark = (lambda i: ev[i].record(s)) if ev is not None else (lambda i: None)
        mark(0)
        ex.line_tau(ctx, atom, prev, w.t_exp, tau=grid.tau_ct, fcorr=grid.fcorr_ct)
        mark(1)
        ex.transport(ctx, grid, w.seed, w.lambda_lo, w.lambda_hi, w.n_packets,
                     geometry_fp32=True, est=est, stats=stats)
        mark(2)
        ex.rates(ctx, atom, grid, w.t_exp, est, prev, out=gamma)
        mark(3)
        ex.nlte_warm_start(ctx, atom, cells, dep, params, norm, pops=pops)
        mark(4)
        ex.nlte_solve(ctx, atom, cells, pops=pops, use_guess=True, warm_budget=args.warm_budget,
                      tol=args.nlte_tol, status=status, iters=iters,
                      factor_fp32=args.nlte_precision == "mixed")
        mark(5)

    step()
    reps = 10
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(6)] for _ in range(reps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(reps):
        step(evs[k])
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / reps
    parts = {n: sum(e[i].elapsed_time(e[i + 1]) for e in evs) / reps for i, n in enumerate(names)}
    sd = ex.stats_dict(stats)
    bytes_alg = 8.0 * w.n_cells * w.n_lines + 16.0 * w.n_cells + 16.0 * w.n_lines
    ach = bytes_alg / (parts["transport"] * 1e-3) / 1e9
    fl = nlte_flops_per_iteration(w.atom)
    flops = float(iters.double().sum()) * sum(fl)
    return {"workload": w.name, "ms_per_step": ms, "value": sd["n_inter"] / (ms * 1e-3),
            "unit": "line-interactions/s", "interactions_per_step": sd["n_inter"],
            "nlte_cell_solves_per_s": w.n_cells / (ms * 1e-3), "ms_parts": parts,
            "cells_converged": int((status <= 1).sum()),
            "nlte_iters_mean": float(iters.float().mean()),
            "nlte_precision": args.nlte_precision,
            "roofline_transport": {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS,
                                   "unit": "GB/s", "frac": ach / HBM_PEAK_GBS,
                                   "algorithmic_bytes": bytes_alg,
                                   "traffic": recorded_traffic("extrass_transport")},
            "roofline_nlte": {"bound": "alu", "achieved": flops / (parts["nlte"] * 1e-3) / 1e12,
                              "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                              "frac": flops / (parts["nlte"] * 1e-3) / 1e12 / FP64_PEAK_TFLOPS,
                              "algorithmic_flops": flops}}


def bench_photoion(ex, ctx, w):
    """Photoionisation in the transport (Sec. 2.3.1) on the 50^3 workload at
    its cold-start populations: the 70 photoionising levels of the two species
    (stages 0 and 1, hydrogenic cross sections, synthetic ionisation energies),
    the continuum opacity table, the 1e7-packet transport with and without the
    continuum (FP32 geometry, the atom's lines at Eq. A2 opacities), and the
    per-level rates; HIP events, median of 5."""
    import numpy as np
    import torch
    import synth
    dev = "cuda:0"
    atom = ex.Atom(ctx, w.atom)
    cold, _, _ = ex.nlte_solve(ctx, atom, ex.cells_from_workload(w, device=dev), max_iter=0)
    tau, fc = ex.line_tau(ctx, atom, cold, w.t_exp)
    grid = ex.grid_from_workload(w, device=dev, tau_ct=tau, fcorr_ct=fc)
    plan = ex.PiPlan(ctx, atom, synth.ion_energies(w.number, w.atom), 25)
    opac = plan.opacity(cold)
    photo = ex.Photoion(plan, opac, w.t_exp)
    est = torch.empty((w.n_cells, w.n_lines), dtype=torch.float64, device=dev)
    stats = torch.empty(ex.STATS, dtype=torch.float64, device=dev)
    gpi = torch.empty((w.n_cells, w.atom.n_levels), dtype=torch.float64, device=dev)
    s = torch.cuda.current_stream()
    res = {}
    for name, on in (("plain", False), ("photoion", True)):
        grid.photoion = photo if on else None
        times, topac, trates = [], [], []
        for _ in range(6):
            e = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
            e[0].record(s)
            if on:
                plan.opacity(cold, out=opac)
                photo.tally.zero_()
            e[1].record(s)
            ex.transport(ctx, grid, w.seed, w.lambda_lo, w.lambda_hi, w.n_packets,
                         geometry_fp32=True, est=est, stats=stats)
            e[2].record(s)
            if on:
                plan.rates(grid, w.t_exp, photo.tally, out=gpi)
            e[3].record(s)
            torch.cuda.synchronize()
            topac.append(e[0].elapsed_time(e[1]))
            times.append(e[1].elapsed_time(e[2]))
            trates.append(e[2].elapsed_time(e[3]))
        sd = ex.stats_dict(stats)
        res[name] = {"ms_transport": float(np.median(times[1:])),
                     "interactions": sd["n_inter"], "crossings": sd["n_cross"],
                     "photoionised_fraction": sd["w_pi"] / sd["w_emit"],
                     "line_absorbed_fraction": sd["w_abs"] / sd["w_emit"],
                     "escaped_fraction": sd["w_esc"] / sd["w_emit"]}
        if on:
            res[name]["ms_opacity_table"] = float(np.median(topac[1:]))
            res[name]["ms_rates"] = float(np.median(trates[1:]))
    grid.photoion = None
    g = gpi.cpu().numpy()
    res.update({"workload": w.name + " (cold-start populations)", "levels": plan.M,
                "threshold_range_A": [float(plan.lambda_thr.min() * 1e8),
                                      float(plan.lambda_thr.max() * 1e8)],
                "rate_range_s": [float(g[g > 0].min()), float(g.max())] if (g > 0).any() else None,
                "slowdown": res["photoion"]["ms_transport"] / res["plain"]["ms_transport"]})
    return res


def bench_spherical(ex, ctx):
    """Transport on the paper's spherical (r, theta, phi) grid: 48 x 32 x 64 =
    98 304 cells (shells growing outwards), 5000 background lines, 1e7
    sampled packets, FP64 geometry; the estimator table [C x L] written as in
    the cube's step; unsplit, and streamed over 2, 4 and 8 phi domains (the
    paper's decomposition; 8 is the bench's figure). HIP events, median of 5."""
    import numpy as np
    import torch
    import synth
    dev = "cuda:0"
    w = synth.spherical(48, 32, 64, 5000, 10_000_000, number=8)
    est = torch.empty((w.n_cells, w.n_lines), dtype=torch.float64, device=dev)
    stats = torch.empty(ex.STATS, dtype=torch.float64, device=dev)
    s = torch.cuda.current_stream()
    out = {"workload": w.name, "cells": w.n_cells, "lines": w.n_lines, "packets": w.n_packets}
    for nd in (0, 2, 4, 8):
        grid = ex.spherical_grid(w.r_edge, w.theta_edge, w.n_phi, w.tau_scale, w.cell_photons,
                                 w.cell_packets, w.line_lambda, w.line_tau0, device=dev,
                                 n_domains=nd)
        name = "unsplit" if nd == 0 else f"streamed_{nd}_phi_domains"
        times = []
        for _ in range(6):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(s)
            if nd == 0:
                ex.transport(ctx, grid, w.seed, w.lambda_lo, w.lambda_hi, w.n_packets, est=est,
                             stats=stats)
            else:
                ex.transport_streamed(ctx, grid, w.seed, w.lambda_lo, w.lambda_hi, w.n_packets,
                                      stats=stats)
            e1.record(s)
            torch.cuda.synchronize()
            times.append(e0.elapsed_time(e1))
        sd = ex.stats_dict(stats)
        ms = float(np.median(times[1:]))
        out[name] = {"ms": ms, "interactions": sd["n_inter"],
                     "line_interactions_per_s": sd["n_inter"] / (ms * 1e-3),
                     "crossings_per_packet": sd["n_cross"] / w.n_packets,
                     "escaped_fraction": sd["w_esc"] / sd["w_emit"]}
        del grid
        torch.cuda.empty_cache()
    # the paper's rays on its grid: line emission of the small plain
    # workload's 10-level atom at log-uniform populations in every cell, one
    # ray per (cell, occupied 0.1 % bin, 20 x 20 viewer) from the cell's middle
    aw = synth.sphere_small()
    g = np.random.default_rng(21)
    pops = torch.as_tensor(10 ** g.uniform(0.0, 4.0, (w.n_cells, aw.atom.n_levels)), device=dev)
    atom = ex.Atom(ctx, aw.atom)
    lo, hi = 2900e-8, 10500e-8
    plan = ex.EmissionPlan(ctx, atom, lo, hi, int(np.ceil(np.log(hi / lo) / np.log(1.001))))
    grid = ex.spherical_grid(w.r_edge, w.theta_edge, w.n_phi, w.tau_scale, w.cell_photons,
                             w.cell_packets, w.line_lambda, w.line_tau0, device=dev)
    e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    e[0].record(s)
    ph, _ = ex.emission(ctx, plan, atom, grid, w.t_exp, pops)
    e[1].record(s)
    _, st, _ = ex.transport_rays(ctx, grid, plan, ph, 20, 20, est=est, stats=stats)
    e[2].record(s)
    torch.cuda.synchronize()
    sd = ex.stats_dict(st)
    n_rays = w.n_cells * plan.n_bins * 400
    out["deterministic_rays"] = {"occupied_bins": plan.n_bins, "viewers": [20, 20],
                                 "rays": n_rays, "ms_emission": e[0].elapsed_time(e[1]),
                                 "ms_rays": e[1].elapsed_time(e[2]),
                                 "rays_per_s": n_rays / (e[1].elapsed_time(e[2]) * 1e-3),
                                 "interactions": sd["n_inter"],
                                 "escaped_fraction": sd["w_esc"] / sd["w_emit"]}
    del grid, est, plan, atom, pops, ph
    torch.cuda.empty_cache()
    # the global loop on the spherical grid (the cube workloads' 100-level
    # atom in every cell), streamed over 8 phi domains with the rates summed
    # per interaction, from the cold start: two iterations
    from paper_2511_07539_amd import globalloop
    wa = synth.spherical(48, 32, 64, 5000, 10_000_000, number=8, atom=True)
    loop = globalloop.GlobalLoop(ctx, wa, tol=1e-8, n_domains=8)
    _, st_l, hist = loop.run(2)
    out["global_loop_8_phi_domains"] = {
        "workload": wa.name, "iterations": [
            {k: h[k] for k in ("ms_line_tau", "ms_transport", "ms_nlte", "interactions",
                               "cells_converged", "nlte_iters_mean")} for h in hist]}
    del loop
    torch.cuda.empty_cache()
    return out


def bench_rays(ex, ctx, w, n_rays=2_000_000_000):
    """The paper's deterministic rays (Sec. 2.3) on the 50^3 workload at its
    cold-start populations: line emission (Eq. A3) into 0.1 % logarithmic bins
    over the atom's lines, one ray per (cell, occupied bin, viewer) towards
    20 x 20 viewers (FP32 geometry). The first n_rays rays (cell-major, so a
    slab of cells with all their bins and viewers) are timed with HIP events;
    the rate is projected to the whole ray set."""
    import math

    import torch
    atom = ex.Atom(ctx, w.atom)
    cells0 = ex.cells_from_workload(w)
    pops, _, _ = ex.nlte_solve(ctx, atom, cells0, max_iter=0)
    tau, fc = ex.line_tau(ctx, atom, pops, w.t_exp)
    grid = ex.grid_from_workload(w, tau_ct=tau, fcorr_ct=fc)
    lo, hi = 0.97 * float(w.atom.trans_lambda.min()), 1.03 * float(w.atom.trans_lambda.max())
    n_lam = int(math.ceil(math.log(hi / lo) / math.log(1.001)))
    plan = ex.EmissionPlan(ctx, atom, lo, hi, n_lam)
    s = torch.cuda.current_stream()
    e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    e[0].record(s)
    ph, _ = ex.emission(ctx, plan, atom, grid, w.t_exp, pops)
    e[1].record(s)
    total = w.n_cells * plan.n_bins * 400
    n = min(n_rays, total)
    est, st, _ = ex.transport_rays(ctx, grid, plan, ph, 20, 20, n_rays=n, geometry_fp32=True)
    e[2].record(s)
    torch.cuda.synchronize()
    ms_em, ms_rays = e[0].elapsed_time(e[1]), e[1].elapsed_time(e[2])
    sd = ex.stats_dict(st)
    return {"workload": w.name, "viewers": [20, 20], "lambda_bins": n_lam,
            "occupied_bins": plan.n_bins, "rays_total": total, "rays_timed": n,
            "ms_emission": ms_em, "ms_rays_incl_table_fill": ms_rays,
            "rays_per_s": n / (ms_rays * 1e-3), "interactions": sd["n_inter"],
            "projected_s_all_rays": total / (n / (ms_rays * 1e-3)),
            "paper_context": "2.5e10 rays per iteration in about 70 min on 768 CPU cores "
                             "(includes the NLTE solve)"}


def bench_spectrum(ex, ctx, w):
    """Emergent spectra of the 50^3 workload's packets (Sec. 2.3): 20 x 20
    viewers and 0.1 % log-wavelength bins over the band widened by the Doppler
    shifts. One untimed transport writes the per-packet records; the binning of
    all 1e7 records (64 B each) is timed with HIP events."""
    import math

    import torch
    grid = ex.grid_from_workload(w)
    _, st, pk = ex.transport(ctx, grid, w.seed, w.lambda_lo, w.lambda_hi, w.n_packets,
                             geometry_fp32=True, packets_out=True)
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
    return {"workload": w.name + " (background opacities)", "viewers": [20, 20],
            "lambda_bins": n_lam, "lambda_range_cm": [lo, hi], "ms_binning_incl_zero": ms,
            "record_bytes": rec_bytes, "record_read_tb_per_s": rec_bytes / (ms * 1e-3) / 1e12,
            "escaped_packets": int(sd["n_escaped"]),
            "escaped_photon_fraction": sd["w_esc"] / sd["w_emit"],
            "binned_photons_vs_escaped": float(ph.sum()) / sd["w_esc"]}


def bench_batched(ex, ctx):
    """The batched three-stage NLTE problem (125 000 cells, 20-300 levels per
    stage): tuned launch shape, then one FP64 solve and one FP32-factor solve
    with two FP64 refinement sweeps, each timed with HIP events on the stream
    the library launches on."""
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
                     "tuned_panel_per_cu": list(shape),
                     "status_counts": np.bincount(st, minlength=3).tolist(),
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


if __name__ == "__main__":
    main()
