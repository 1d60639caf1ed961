"""Training of the learned pressure guess on fields the solver generates.

Snapshots: after each recorded time step the library returns the features
(phi, rho/rho_max, normalised right-hand side) and the normalised pressure of
the step's last projection (cdi_guess_features).  Training: mini-batches of
snapshots (random crops when the network is smaller than the grid) through
the library's BF16 forward / backward / Adam kernels.
"""
from __future__ import annotations

import time
from typing import List, Sequence, Tuple

import numpy as np
import torch

import workloads as W

from .learned import GuessNet
from .solver import CDISolver


def collect(cases: Sequence, steps: int, every: int = 1, precision: str = "fp64",
            rtol: float = 1e-10) -> List[Tuple[torch.Tensor, torch.Tensor]]:
    """Run every case for `steps` steps and keep (features, target) of every
    `every`-th step (device tensors, FP32)."""
    out = []
    for c in cases:
        s = CDISolver(c.params, c.phi0, precision=precision, rtol=rtol)
        for k in range(steps):
            s.step(1)
            if (k + 1) % every == 0:
                f, t = s.guess_features()
                out.append((f.clone(), t.clone()))
        s.close()
    return out


def train(net: GuessNet, data, iters: int, lr: float = 1e-3, seed: int = 0,
          log_every: int = 0) -> List[float]:
    """Adam on random mini-batches (and random crops of net.h x net.w).
    Returns the loss of every iteration (each of a different random batch:
    compare means over many iterations, see loss_summary)."""
    rng = np.random.default_rng(seed)
    B, h, w = net.batch, net.h, net.w
    losses = []
    x = torch.empty((B, 3, h, w), dtype=torch.float32, device=net.device)
    t = torch.empty((B, h, w), dtype=torch.float32, device=net.device)
    t0 = time.time()
    dev_losses = []
    for it in range(iters):
        for b in range(B):
            f, tt = data[int(rng.integers(len(data)))]
            H, W = tt.shape
            y0 = int(rng.integers(0, H - h + 1)) if H > h else 0
            x0 = int(rng.integers(0, W - w + 1)) if W > w else 0
            x[b] = f[:, y0:y0 + h, x0:x0 + w]
            t[b] = tt[y0:y0 + h, x0:x0 + w]
        net.forward(x)
        loss = net.backward(t)
        net.adam(lr)
        dev_losses.append(loss.detach().clone().reshape(()))
        if log_every and (it % log_every == 0 or it == iters - 1):
            print(f"iter {it} loss {float(loss.item()):.4e} ({time.time() - t0:.1f} s)", flush=True)
    losses = [float(v) for v in torch.stack(dev_losses).cpu()] if dev_losses else []
    return losses


def loss_summary(losses: Sequence[float], frac: float = 0.1):
    """Mean loss over the first and the last `frac` of the iterations."""
    k = max(1, int(len(losses) * frac))
    return float(np.mean(losses[:k])), float(np.mean(losses[-k:]))


def collect_configs(steps1: int = 500, steps2: int = 4000, every2: int = 4,
                    steps3: int = 2000, crop: int = 256, seed: int = 0,
                    verbose: bool = False) -> dict:
    """Training snapshots from the first three benchmark workloads, kept in
    device memory (FP32): the features and normalised pressure of the last
    projection of each recorded step (cdi_guess_features).

      drop64x32      every step of the 500-step equilibrium drop (full grids)
      couette256x64  every every2-th step of the 4000-step Couette flow (full
                     grids)
      drop1024x512   every step of the four ratio-10 drops (theta_eq 30, 60,
                     120, 150 deg, one batched context) for steps3 steps, one
                     random crop x crop window of each

    Returns {name: (features [N, 3, h, w], targets [N, h, w])}."""
    from .solver import CDISolver
    rng = np.random.default_rng(seed)
    out = {}
    t0 = time.perf_counter()
    # the first workload: every step, full 32 x 64 grids
    c = W.config1()
    s = CDISolver(c.params, c.phi0, rtol=1e-10)
    F = torch.empty((steps1, 3, c.params.ny, c.params.nx), dtype=torch.float32, device=s.device)
    T = torch.empty((steps1, c.params.ny, c.params.nx), dtype=torch.float32, device=s.device)
    for k in range(steps1):
        s.step(1)
        f, t = s.guess_features()
        F[k].copy_(f)
        T[k].copy_(t)
    s.close()
    out[c.name] = (F, T)
    if verbose:
        print(f"collected {steps1} snapshots of {c.name} ({time.perf_counter() - t0:.1f} s)",
              flush=True)
    # the second: every every2-th step, full 64 x 256 grids
    c = W.config2()
    n2 = steps2 // every2
    s = CDISolver(c.params, c.phi0, rtol=1e-10)
    F = torch.empty((n2, 3, c.params.ny, c.params.nx), dtype=torch.float32, device=s.device)
    T = torch.empty((n2, c.params.ny, c.params.nx), dtype=torch.float32, device=s.device)
    for k in range(n2):
        s.step(every2)
        f, t = s.guess_features()
        F[k].copy_(f)
        T[k].copy_(t)
    s.close()
    out[c.name] = (F, T)
    if verbose:
        print(f"collected {n2} snapshots of {c.name} ({time.perf_counter() - t0:.1f} s)",
              flush=True)
    # the third: four angles in one context, a random crop of every step
    cases = [W.config3(th) for th in W.CONFIG3_THETAS]
    s = CDISolver([q.params for q in cases], [q.phi0 for q in cases], rtol=1e-10)
    ny, nx = cases[0].params.ny, cases[0].params.nx
    n3 = steps3 * len(cases)
    F = torch.empty((n3, 3, crop, crop), dtype=torch.float32, device=s.device)
    T = torch.empty((n3, crop, crop), dtype=torch.float32, device=s.device)
    k = 0
    for step in range(steps3):
        s.step(1)
        for idx in range(len(cases)):
            f, t = s.guess_features(idx)
            y0 = int(rng.integers(0, ny - crop + 1))
            x0 = int(rng.integers(0, nx - crop + 1))
            F[k].copy_(f[:, y0:y0 + crop, x0:x0 + crop])
            T[k].copy_(t[y0:y0 + crop, x0:x0 + crop])
            k += 1
        if verbose and (step + 1) % 500 == 0:
            print(f"drop1024x512: {step + 1} of {steps3} steps ({time.perf_counter() - t0:.1f} s)",
                  flush=True)
    s.close()
    out[f"drop{nx}x{ny}_crops"] = (F, T)
    return out


def train_multi(data: dict, seconds: float = 60.0, max_iters: int = 100000,
                batch: int = 8, lr: float = 5e-4, seed: int = 0, params=None,
                verbose: bool = False):
    """Adam on mini-batches of one data set at a time (picked with
    probability proportional to its size), each shape through its own
    network over one shared set of parameters, until `seconds` of training
    or `max_iters` iterations.  Returns (parameters as a NumPy vector, loss of
    every iteration, iterations done)."""
    rng = np.random.default_rng(seed)
    names = sorted(data)
    sizes = np.array([data[n][0].shape[0] for n in names], dtype=np.float64)
    prob = sizes / sizes.sum()
    nets = {}
    primary = None
    for n in names:
        F, _ = data[n]
        h, w = F.shape[2], F.shape[3]
        if primary is None:
            nets[n] = GuessNet(batch, h, w, params=params)
            primary = nets[n]
        else:
            nets[n] = GuessNet(batch, h, w, share=primary)
    stale = set()
    losses = []
    dev = primary.device
    torch.cuda.synchronize(dev)
    t0 = time.perf_counter()
    it = 0
    while it < max_iters and time.perf_counter() - t0 < seconds:
        n = names[int(rng.choice(len(names), p=prob))]
        F, T = data[n]
        idx = torch.as_tensor(rng.integers(0, F.shape[0], batch), device=dev)
        net = nets[n]
        if n in stale:
            net.repack()
            stale.discard(n)
        net.forward(F.index_select(0, idx))
        losses.append(net.backward(T.index_select(0, idx)).detach().clone().reshape(()))
        primary.adam(lr)
        stale.update(m for m in names if nets[m] is not primary)
        it += 1
        if verbose and it % 500 == 0:
            print(f"iteration {it}: loss {float(losses[-1]):.4f} "
                  f"({time.perf_counter() - t0:.0f} s)", flush=True)
    torch.cuda.synchronize(dev)
    vec = primary.params.cpu().numpy().copy()
    for net in nets.values():
        net.close()
    return vec, [float(v) for v in torch.stack(losses).cpu()] if losses else [], it
