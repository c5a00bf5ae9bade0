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
