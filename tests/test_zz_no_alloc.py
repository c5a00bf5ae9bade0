"""The allocation-free transport entry point (extrass_transport_noalloc)
against extrass_transport on the same inputs: two calls in a row on one GPU,
the second with a smaller problem, then a problem beyond its scratch."""
import sys

import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def _noalloc(ex, ctx, grid, w, est, stats, n_packets=None):
    return ex.transport_noalloc(ctx, grid, w.seed, w.lambda_lo, w.lambda_hi,
                                n_packets or w.n_packets, est, stats, geometry_fp32=True)


def test_noalloc_transport_equals_transport():
    import paper_2511_07539_amd as ex
    ctx = ex.Context(0)
    for w in (synth.paper_scale(), synth.sphere_small()):
        say(f"case: extrass_transport_noalloc vs extrass_transport, {w.name}")
        grid = ex.grid_from_workload(w)
        ref, st_ref, _ = ex.transport(ctx, grid, w.seed, w.lambda_lo, w.lambda_hi, w.n_packets,
                                      geometry_fp32=True)
        est = torch.full_like(ref, 7.0)          # overwritten by the call
        stats = torch.full_like(st_ref, 7.0)
        rc = _noalloc(ex, ctx, grid, w, est, stats)
        torch.cuda.synchronize()
        assert rc == ex.OK
        a, b = ex.stats_dict(stats), ex.stats_dict(st_ref)
        for k in ("n_inter", "n_checks", "n_cross", "n_escaped", "n_killed"):
            assert a[k] == b[k], k
        assert a["error_flag"] == 0 and a["bad_packets"] == 0
        nz = ref != 0
        assert bool(((est != 0) == nz).all())
        rel = float(((est[nz] - ref[nz]).abs() / ref[nz]).max())
        say(f"  max rel {rel:.2e} over {int(nz.sum())} entries")
        assert rel <= 1e-12   # the same sums, atomics in another order
        del ref, est
        torch.cuda.empty_cache()
    say("case: a problem beyond the scratch is refused before any launch")
    w = synth.sphere_small()
    grid = ex.grid_from_workload(w)
    est = torch.zeros((w.n_cells, w.n_lines), dtype=torch.float64, device="cuda:0")
    stats = torch.zeros(ex.STATS, dtype=torch.float64, device="cuda:0")
    rc = _noalloc(ex, ctx, grid, w, est, stats, n_packets=5_000_000_000)
    torch.cuda.synchronize()
    assert rc == ex.ENOSPACE
    assert float(est.abs().sum()) == 0.0 and float(stats.abs().sum()) == 0.0
