"""Training data and training loop for the learned NLTE warm start.

The network is trained on solves the method itself produces: cell states are
drawn from the distribution of a workload's cells (temperature, deposition and
abundances redrawn), their photoexcitation rates come from one transport pass
over that workload, and the targets are the converged level populations of
extrass_nlte_solve from the cold start. Training runs the library's own
forward/backward/Adam kernels (extrass_mlp_train_step). This module only
orders those calls and keeps the tensors; the arithmetic runs in the kernels.
"""
from __future__ import annotations

import numpy as np
import torch

from . import (MLP_IN, MLP_OUT, MLP_PARAMS, Atom, Cells, Context, grid_from_workload,
               line_tau, mlp_features, mlp_train_step, nlte_solve, rates, transport)


def replica_states(w, k, seed=97):
    """Replica k of the workload's active cells: T_e log-uniform in 2000-10000 K,
    deposition rescaled by a lognormal factor (sigma_ln 1) with the ionisation
    rates rescaled alike, first-species mass share shifted by up to +-0.2."""
    g = np.random.default_rng([seed, k])
    S = w.atom.n_species
    act = np.where(w.n_species.reshape(-1, S).sum(1) > 0)[0]
    C = len(act)
    T = 10 ** g.uniform(np.log10(2000.0), np.log10(10000.0), C)
    f = np.exp(g.standard_normal(C))
    dep = w.deposition[act] * f
    gion = w.gamma_ion.reshape(-1, S, 3)[act] * f[:, None, None]
    ns = w.n_species.reshape(-1, S)[act].copy()
    m = w.atom.species_mass
    mass = ns * m[None, :]
    rho = mass.sum(1)
    x0 = np.clip(mass[:, 0] / rho + g.uniform(-0.2, 0.2, C), 0.05, 0.95)
    ns[:, 0] = x0 * rho / m[0]
    ns[:, 1] = (1 - x0) * rho / m[1]
    n_e = 0.5 * ns.sum(1)
    return act, T, n_e, ns, gion, dep


def photoexcitation_rates(ctx: Context, atom: Atom, w, device="cuda:0"):
    """Gamma_PE of every cell from one transport pass at cold-start opacities."""
    cells = Cells(w.t_exp, w.T_e, w.n_e, w.n_species, w.gamma_ion, None, device)
    cold, _, _ = nlte_solve(ctx, atom, cells, max_iter=0)
    tau, fc = line_tau(ctx, atom, cold, w.t_exp)
    grid = grid_from_workload(w, device=device, tau_ct=tau, fcorr_ct=fc)
    est, _, _ = transport(ctx, grid, w.seed, w.lambda_lo, w.lambda_hi, w.n_packets,
                          geometry_fp32=True)
    gam = rates(ctx, atom, grid, w.t_exp, est, cold)
    del est
    return gam


def make_dataset(ctx: Context, atom: Atom, w, n_replicas=8, device="cuda:0", gamma=None):
    """Features [M, 6] and targets log10(n_i / n_species) [M, 100] (host FP64)."""
    if gamma is None:
        gamma = photoexcitation_rates(ctx, atom, w, device)
    X, Y = [], []
    off = w.atom.species_offset
    for k in range(n_replicas):
        act, T, n_e, ns, gion, dep = replica_states(w, k)
        gpe = gamma[torch.as_tensor(act, device=gamma.device)]
        cells = Cells(w.t_exp, T, n_e, ns, gion, gpe, device)
        pops, status, _ = nlte_solve(ctx, atom, cells)
        p = pops.cpu().numpy()
        ok = status.cpu().numpy() == 0
        y = np.empty_like(p)
        for s in range(len(off) - 1):
            y[:, off[s]:off[s + 1]] = np.log10(p[:, off[s]:off[s + 1]] / ns[:, s:s + 1])
        X.append(mlp_features(ctx, atom, cells, dep).cpu().numpy().astype(np.float64)[ok])
        Y.append(y[ok])
    return np.concatenate(X), np.concatenate(Y)


def init_params(seed=0):
    g = np.random.default_rng(seed)
    sizes = [MLP_IN, 256, 256, 256, MLP_OUT]
    parts = []
    for i in range(4):
        parts.append((g.standard_normal((sizes[i + 1], sizes[i])) *
                      np.sqrt(2.0 / sizes[i])).ravel())
        parts.append(np.zeros(sizes[i + 1]))
    p = np.concatenate(parts).astype(np.float32)
    assert p.size == MLP_PARAMS
    return p


def train(ctx: Context, X, Y, epochs=30, batch=8192, lr=2e-3, seed=0, device="cuda:0",
          verbose=False):
    """Returns (params [P] f32 device tensor, norm [212] f32 device tensor, loss history)."""
    xm, xs = X.mean(0), X.std(0) + 1e-6
    ym, ys = Y.mean(0), Y.std(0) + 1e-6
    norm = torch.as_tensor(np.concatenate([xm, xs, ym, ys]).astype(np.float32), device=device)
    Xn = torch.as_tensor(((X - xm) / xs).astype(np.float32), device=device)
    Yn = torch.as_tensor(((Y - ym) / ys).astype(np.float32), device=device)
    params = torch.as_tensor(init_params(seed), device=device)
    m = torch.zeros_like(params)
    v = torch.zeros_like(params)
    loss = torch.zeros(1, dtype=torch.float32, device=device)
    M = Xn.shape[0]
    gen = torch.Generator(device="cpu").manual_seed(seed)
    hist = []
    step = 0
    nb = M // batch
    for ep in range(epochs):
        perm = torch.randperm(M, generator=gen).to(device)
        loss.zero_()
        lr_ep = lr * 0.5 * (1 + np.cos(np.pi * ep / epochs))
        for b in range(nb):
            idx = perm[b * batch:(b + 1) * batch]
            xb = Xn[idx].contiguous()
            yb = Yn[idx].contiguous()
            step += 1
            mlp_train_step(ctx, params, xb, yb, m, v, step, lr_ep, loss)
        hist.append(float(loss.item()) / max(nb, 1))
        if verbose:
            print(f"epoch {ep} loss {hist[-1]:.4e}", flush=True)
    return params, norm, hist


def train_on_workload(ctx: Context, w, n_replicas=8, epochs=30, batch=8192, device="cuda:0"):
    """Trains the warm-start network on solves of replicas of workload w's
    cells (photoexcitation rates from one transport pass over w). Returns
    (params, norm, loss history)."""
    atom = Atom(ctx, w.atom)
    gamma = photoexcitation_rates(ctx, atom, w, device)
    X, Y = make_dataset(ctx, atom, w, n_replicas=n_replicas, device=device, gamma=gamma)
    del gamma
    params, norm, hist = train(ctx, X, Y, epochs=epochs, batch=batch, device=device)
    return params, norm, hist
