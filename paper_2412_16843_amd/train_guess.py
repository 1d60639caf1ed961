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
