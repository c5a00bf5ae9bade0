"""Learned warm start: HIP MLP kernels vs the FP64 oracle, and the warm-started
NLTE solve vs the cold one.

Bars (BF16 operands, FP32 accumulation over K = 256 terms): the oracle runs in
FP64 on the same BF16-rounded inputs and weights; the GPU additionally rounds
each layer's activations to BF16, which bounds the relative error of an
output or gradient element by ~ sqrt(K) * 2^-8 ~ 6e-2 and of whole tensors far
less. Asserted: per-tensor relative Frobenius error <= 2e-2 and cosine
similarity >= 0.999 for outputs and every parameter gradient.
"""
import sys

import numpy as np
import pytest
import torch

import synth
from oracle import mlp as omlp

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def ex():
    import paper_2511_07539_amd as ex
    return ex


@pytest.fixture(scope="module")
def ctx(ex):
    return ex.Context(0)


def _close(a, b, name, rel=2e-2, cos=0.999):
    a = np.asarray(a, np.float64).ravel()
    b = np.asarray(b, np.float64).ravel()
    r = np.linalg.norm(a - b) / np.linalg.norm(b)
    c = a @ b / (np.linalg.norm(a) * np.linalg.norm(b))
    say(f"{name}: rel {r:.2e} cos {c:.6f}")
    assert r <= rel and c >= cos, name


def _problem(B, seed=0):
    g = np.random.default_rng(seed)
    p = omlp.init_params(seed).astype(np.float32)
    p += (0.02 * g.standard_normal(p.size)).astype(np.float32)
    x = g.standard_normal((B, 6)).astype(np.float32)
    t = g.standard_normal((B, 100)).astype(np.float32)
    return p, x, t


@pytest.mark.parametrize("B", [64, 1000, 8192])
def test_forward_matches_oracle(ex, ctx, B):
    p, x, _ = _problem(B)
    say(f"case: MLP forward, batch {B}")
    y = ex.mlp_forward(ctx, torch.as_tensor(p, device="cuda:0"), torch.as_tensor(x, device="cuda:0"))
    torch.cuda.synchronize()
    yo, _ = omlp.forward(omlp.round_bf16(p), x)   # layer 1 is FP32 on the GPU: x not rounded
    _close(y.cpu().numpy(), yo, "y")


@pytest.mark.parametrize("B", [256, 4096])
def test_gradients_match_oracle(ex, ctx, B):
    p, x, t = _problem(B, seed=3)
    dev = "cuda:0"
    grad = torch.zeros(ex.MLP_PARAMS, dtype=torch.float32, device=dev)
    loss = torch.zeros(1, dtype=torch.float32, device=dev)
    say(f"case: MLP gradients, batch {B}")
    ex.mlp_train_step(ctx, torch.as_tensor(p, device=dev), torch.as_tensor(x, device=dev),
                      torch.as_tensor(t, device=dev), loss=loss, grad=grad)
    torch.cuda.synchronize()
    lo, go = omlp.loss_and_grad(omlp.round_bf16(p), x, t)
    assert abs(loss.item() - lo) <= 1e-2 * lo
    g = grad.cpu().numpy()
    off = 0
    for name, shp in zip(["W1", "b1", "W2", "b2", "W3", "b3", "W4", "b4"], omlp.shapes()):
        n = int(np.prod(shp))
        _close(g[off:off + n], go[off:off + n], name)
        off += n


def test_adam_step_and_training_reduce_loss(ex, ctx):
    g = np.random.default_rng(1)
    B = 2048
    x = g.standard_normal((B, 6)).astype(np.float32)
    W = g.standard_normal((100, 6)) / 3
    t = np.tanh(x @ W.T).astype(np.float32)
    dev = "cuda:0"
    p = torch.as_tensor(omlp.init_params(2).astype(np.float32), device=dev)
    p0 = p.clone()
    m = torch.zeros_like(p)
    v = torch.zeros_like(p)
    grad = torch.zeros_like(p)
    loss = torch.zeros(1, dtype=torch.float32, device=dev)
    xd, td = torch.as_tensor(x, device=dev), torch.as_tensor(t, device=dev)
    say("case: one Adam step against the update rule")
    ex.mlp_train_step(ctx, p, xd, td, m, v, 1, 1e-3, loss, grad)
    torch.cuda.synchronize()
    gd = grad.cpu().numpy().astype(np.float64)
    mh = 0.1 * gd / (1 - 0.9)
    vh = 0.001 * gd * gd / (1 - 0.999)
    expect = p0.cpu().numpy() - 1e-3 * mh / (np.sqrt(vh) + 1e-8)
    np.testing.assert_allclose(p.cpu().numpy(), expect, rtol=1e-5, atol=1e-7)
    losses = []
    for s in range(2, 300):
        loss.zero_()
        ex.mlp_train_step(ctx, p, xd, td, m, v, s, 1e-3, loss)
        losses.append(loss.item())
    say("loss", losses[0], "->", losses[-1])
    assert losses[-1] < 0.1 * losses[0]


def test_warm_start_converges_to_cold_roots(ex, ctx):
    """Train on replicas of a 16^3 clumpy workload's cells, then warm-start
    the workload itself: same roots as the cold start (1e-8), fewer iterations."""
    from paper_2511_07539_amd import warmstart
    w = synth.clumpy(n=16, n_lines=2000, n_packets=400_000, number=2)
    atom = ex.Atom(ctx, w.atom)
    say("case: warm-start training data (8 replicas of 4096 cells)")
    gamma = warmstart.photoexcitation_rates(ctx, atom, w)
    X, Y = warmstart.make_dataset(ctx, atom, w, n_replicas=8, gamma=gamma)
    say("case: training", X.shape)
    params, norm, hist = warmstart.train(ctx, X, Y, epochs=40, batch=1024)
    say("loss", hist[0], "->", hist[-1])
    assert hist[-1] < 0.7 * hist[0]
    cells = ex.cells_from_workload(w, gamma_pe=gamma)
    pc, sc, ic = ex.nlte_solve(ctx, atom, cells)
    guess = ex.nlte_warm_start(ctx, atom, cells, w.deposition, params, norm)
    pw, sw, iw = ex.nlte_solve(ctx, atom, cells, guess=guess, warm_budget=20)
    torch.cuda.synchronize()
    pc, pw = pc.cpu().numpy(), pw.cpu().numpy()
    sc, sw, ic, iw = sc.cpu().numpy(), sw.cpu().numpy(), ic.cpu().numpy(), iw.cpu().numpy()
    assert np.all(sc == 0) and np.all(sw <= 1)
    rel = np.abs(pw - pc) / pc
    say("warm vs cold max rel", rel.max(), "iters cold", ic.mean(), "warm", iw.mean(),
        "fallbacks", int((sw == 1).sum()))
    assert rel.max() <= 1e-8
    assert iw.mean() < ic.mean()


def _features_reference(T_e, n_e, n_species, deposition):
    """The six warm-start features as the header states them: log10 of the
    total species density, T_e, n_e and the deposition, and the two species'
    number fractions."""
    ns = np.asarray(n_species).reshape(len(T_e), -1)
    tot = ns.sum(1)
    safe = np.where(tot > 0, tot, 1.0)
    return np.column_stack([np.log10(safe), np.log10(T_e), np.log10(np.where(n_e > 0, n_e, 1.0)),
                            np.log10(np.where(deposition > 0, deposition, 1e-30)),
                            ns[:, 0] / safe, ns[:, 1] / safe])


def test_features_match_their_definition(ex, ctx):
    w = synth.clumpy(n=13, n_lines=2000, n_packets=10_000, number=3)
    atom = ex.Atom(ctx, w.atom)
    cells = ex.cells_from_workload(w)
    say("case: warm-start features, 2197 cells")
    x = ex.mlp_features(ctx, atom, cells, w.deposition)
    torch.cuda.synchronize()
    ref = _features_reference(w.T_e, w.n_e, w.n_species, w.deposition)
    # the device rounds the FP64 features to FP32 once: within one FP32 ulp
    np.testing.assert_allclose(x.cpu().numpy(), ref, rtol=1.2e-7, atol=1e-38)


def test_fused_warm_start_equals_layer_by_layer(ex, ctx):
    """extrass_nlte_warm_start runs the whole network in one fused kernel. Its
    populations equal those of the layer-by-layer forward (extrass_mlp_forward)
    followed by the per-species normalisation, on 13^3 cells (a ragged last
    work-group of 21 rows). The fused kernel takes K in the same order, so
    the network outputs agree bit for bit (observed: populations to 8e-16;
    a feature whose logarithm rounded differently on host and device could
    move a cell, hence the allowance below)."""
    from paper_2511_07539_amd import warmstart
    dev = "cuda:0"
    w = synth.clumpy(n=13, n_lines=2000, n_packets=10_000, number=3)
    atom = ex.Atom(ctx, w.atom)
    cells = ex.cells_from_workload(w)
    g = np.random.default_rng(7)
    params = torch.as_tensor(warmstart.init_params(3), device=dev)
    X = _features_reference(w.T_e, w.n_e, w.n_species, w.deposition)
    xm, xs = X.mean(0), X.std(0) + 0.1
    ym, ys = g.normal(-4.0, 1.0, 100), g.uniform(0.5, 2.0, 100)
    norm_np = np.concatenate([xm, xs, ym, ys]).astype(np.float32)
    norm = torch.as_tensor(norm_np, device=dev)
    say("case: fused warm start vs layer-by-layer forward, 2197 cells")
    xn = ((X - norm_np[:6].astype(np.float64)) / norm_np[6:12].astype(np.float64)).astype(np.float32)
    y = ex.mlp_forward(ctx, params, torch.as_tensor(xn, device=dev)).cpu().numpy()
    # y * scale + mean in FP32 with one rounding (the device contracts it into
    # an FMA), then FP64
    v = (y.astype(np.float64) * norm_np[112:].astype(np.float64) +
         norm_np[12:112].astype(np.float64)).astype(np.float32).astype(np.float64)
    ns = np.asarray(w.n_species).reshape(w.n_cells, -1)
    ref = np.zeros((w.n_cells, 100))
    off = w.atom.species_offset
    for s in range(2):
        vs = v[:, off[s]:off[s + 1]]
        e = 10.0 ** (vs - vs.max(1, keepdims=True))
        ref[:, off[s]:off[s + 1]] = ns[:, s:s + 1] * e / e.sum(1, keepdims=True)
    pw = ex.nlte_warm_start(ctx, atom, cells, w.deposition, params, norm)
    torch.cuda.synchronize()
    pw = pw.cpu().numpy()
    ok = ref > 0
    rel = np.abs(pw[ok] - ref[ok]) / ref[ok]
    say("max rel", rel.max(), "median", np.median(rel))
    assert np.mean(rel > 1e-13) <= 1e-3
    assert rel.max() <= 1e-3
