"""Global iterations (opacities -> streamed transport -> rates -> NLTE) on the
GPU against the same loop run entirely in the oracle.

Both sides start from their own cold start; every later input is each side's
own result, so no oracle input comes from the GPU. FP64 geometry on the GPU
keeps the event sequences identical (their rounding differences stay far from
the tau > 1e-4 and kill thresholds), so populations after two iterations
agree componentwise to 1e-8 on every cell both sides converge.
"""
import sys

import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def test_two_global_iterations_match_oracle_loop():
    import paper_2511_07539_amd as ex
    from paper_2511_07539_amd import globalloop
    ctx = ex.Context(0)
    w = synth.clumpy(n=16, n_lines=1500, n_packets=200_000, number=2)
    say("case: two global iterations, clumpy 16^3, 1500 lines, 2e5 packets, streamed FP64")
    pops, status, hist = globalloop.run(ctx, w, iterations=2, geometry_fp32=False,
                                        log=lambda r: say(r))
    torch.cuda.synchronize()
    got, sg = pops.cpu().numpy(), status.cpu().numpy()

    C, L = w.n_cells, w.n_lines
    V = (2 * w.beta_max / w.n * synth.C_CGS * w.t_exp) ** 3
    inp0 = oracle.nlte_inputs_from_workload(w)
    p = np.stack([oracle.nlte_cold(inp0, c) for c in range(C)])
    so = None
    for k in range(2):
        tau, fc = oracle.line_tau(p, w.atom, w.t_exp)
        r = oracle.transport(oracle.transport_inputs_from_workload(w, iteration=k, tau_ct=tau,
                                                                   fcorr_ct=fc))
        est = oracle.dense_estimator(r["records"], C, L)
        gam = oracle.rates(est, p, w.atom, V)
        say(f"oracle iteration {k + 1}: interactions {r['stats']['n_inter']:.0f}, "
            f"GPU {hist[k]['interactions']:.0f}")
        assert r["stats"]["n_inter"] == hist[k]["interactions"]
        p, so, _ = oracle.nlte(oracle.nlte_inputs_from_workload(w, gamma_pe=gam), guess=p)
    both = (sg <= 1) & (so == 0)
    say(f"converged: GPU {(sg <= 1).sum()}, oracle {(so == 0).sum()}, both {both.sum()} of {C}")
    assert both.sum() >= 0.999 * C
    ref = p[both]
    g = got[both]
    pos = ref > 0
    rel = np.max(np.abs(g[pos] - ref[pos]) / ref[pos])
    say(f"populations after 2 iterations: max rel {rel:.2e}")
    assert rel <= 1e-8
