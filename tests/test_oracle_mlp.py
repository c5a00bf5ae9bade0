"""Pin for the MLP oracle: analytic FP64 gradients against central finite
differences of the loss (the derivative's definition), on a small batch."""
import numpy as np

from oracle import mlp


def test_parameter_layout():
    assert mlp.N_PARAMS == 159076


def test_gradient_matches_central_differences():
    g = np.random.default_rng(0)
    p = mlp.init_params(1) + 0.05 * g.standard_normal(mlp.N_PARAMS)
    x = g.standard_normal((7, 6))
    t = g.standard_normal((7, 100))
    loss, grad = mlp.loss_and_grad(p, x, t)
    idx = np.concatenate([g.choice(np.arange(0, 1536), 20, replace=False),       # W1
                          g.choice(np.arange(1536, 1792), 10, replace=False),    # b1
                          g.choice(np.arange(1792, 67328), 30, replace=False),   # W2
                          g.choice(np.arange(67584, 133120), 30, replace=False), # W3
                          g.choice(np.arange(133376, 158976), 30, replace=False),# W4
                          np.arange(158976, 158986)])                            # b4
    for i in idx:
        h = 1e-5 * max(1.0, abs(p[i]))
        pp, pm = p.copy(), p.copy()
        pp[i] += h
        pm[i] -= h
        fd = (mlp.loss_and_grad(pp, x, t)[0] - mlp.loss_and_grad(pm, x, t)[0]) / (2 * h)
        assert abs(fd - grad[i]) <= 1e-7 * max(abs(fd), 1e-3 * np.abs(grad).max()), i


def test_bf16_rounding():
    v = np.array([1.0, 1.00390625, 1.005859375, -3.3e-5, 65504.0], dtype=np.float32)
    r = mlp.round_bf16(v)
    # 1 + 2^-8 is a tie between 1 and 1 + 2^-7: round to even (1.0)
    assert r[0] == 1.0 and r[1] == 1.0 and r[2] == 1.0078125
    assert np.all(np.abs(r - v) <= np.abs(v) * 2.0 ** -8)
