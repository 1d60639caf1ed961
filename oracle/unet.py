"""FP64 reference of the learned pressure-guess network (TEST INFRASTRUCTURE).

The network maps per-cell features (phi, rho / rho_max, b / rms(b)) to a
normalised pressure.  Its output is only ever used as the initial guess of the
pressure solve, which still iterates to the requested residual.

Architecture (encoder-decoder with 4 levels, 32/64/128/256 channels):
  e0 = relu(conv3(x, 32))                    H   x W
  e1 = relu(conv3(pool(e0), 64))             H/2
  e2 = relu(conv3(pool(e1), 128))            H/4
  e3 = relu(conv3(pool(e2), 256))            H/8
  d2 = relu(conv3(cat(up(e3), e2), 128))     H/4
  d1 = relu(conv3(cat(up(d2), e1), 64))      H/2
  d0 = relu(conv3(cat(up(d1), e0), 32))      H
  y  = conv1(d0, 1)
conv3: 3x3 cross-correlation with zero padding and a bias; pool: 2x2 mean;
up: nearest-neighbour x2; cat: channel concatenation (upsampled first).
Loss: mean squared error against the normalised target.

Plain NumPy, float64, whole-array operations; forward and backward written
out layer by layer.  Parameters are a dict of arrays; gradients have the same
keys.
"""
from __future__ import annotations

from typing import Dict, Tuple

import numpy as np

CONV3 = (("e0", 3, 32), ("e1", 32, 64), ("e2", 64, 128), ("e3", 128, 256),
         ("d2", 256 + 128, 128), ("d1", 128 + 64, 64), ("d0", 64 + 32, 32))


def init_params(seed: int = 0, in_ch: int = 3) -> Dict[str, np.ndarray]:
    """He-normal weights, zero biases."""
    rng = np.random.default_rng(seed)
    p = {}
    for name, ci, co in CONV3:
        ci = in_ch if name == "e0" else ci
        p[name + ".w"] = rng.standard_normal((co, ci, 3, 3)) * np.sqrt(2.0 / (ci * 9))
        p[name + ".b"] = np.zeros(co)
    p["out.w"] = rng.standard_normal((1, 32)) * np.sqrt(1.0 / 32)
    p["out.b"] = np.zeros(1)
    return p


def conv3(x: np.ndarray, w: np.ndarray, b: np.ndarray) -> np.ndarray:
    """y[b,o,i,j] = bias[o] + sum_{c,ky,kx} w[o,c,ky,kx] x[b,c,i+ky-1,j+kx-1]."""
    B, C, H, W = x.shape
    xp = np.zeros((B, C, H + 2, W + 2))
    xp[:, :, 1:-1, 1:-1] = x
    y = np.zeros((B, w.shape[0], H, W))
    for ky in range(3):
        for kx in range(3):
            y += np.einsum("oc,bchw->bohw", w[:, :, ky, kx], xp[:, :, ky:ky + H, kx:kx + W])
    return y + b[None, :, None, None]


def conv3_backward(x, w, dy):
    """Gradients (dx, dw, db) of conv3 for upstream gradient dy."""
    B, C, H, W = x.shape
    xp = np.zeros((B, C, H + 2, W + 2))
    xp[:, :, 1:-1, 1:-1] = x
    dxp = np.zeros_like(xp)
    dw = np.zeros_like(w)
    for ky in range(3):
        for kx in range(3):
            dw[:, :, ky, kx] = np.einsum("bohw,bchw->oc", dy, xp[:, :, ky:ky + H, kx:kx + W])
            dxp[:, :, ky:ky + H, kx:kx + W] += np.einsum("oc,bohw->bchw", w[:, :, ky, kx], dy)
    return dxp[:, :, 1:-1, 1:-1], dw, dy.sum(axis=(0, 2, 3))


def pool(x):
    B, C, H, W = x.shape
    return x.reshape(B, C, H // 2, 2, W // 2, 2).mean(axis=(3, 5))


def pool_backward(dy):
    return np.repeat(np.repeat(dy, 2, axis=2), 2, axis=3) / 4.0


def up(x):
    return np.repeat(np.repeat(x, 2, axis=2), 2, axis=3)


def up_backward(dy):
    B, C, H, W = dy.shape
    return dy.reshape(B, C, H // 2, 2, W // 2, 2).sum(axis=(3, 5))


def bf16_round(a: np.ndarray) -> np.ndarray:
    """Round to the nearest bfloat16 (8 significand bits, ties to even), via
    the float32 bit pattern: keep the high 16 bits after adding half of the
    dropped part (0x7FFF) plus the lowest kept bit.  Returned as float64."""
    b = np.ascontiguousarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    r = (b + 0x7FFF + ((b >> 16) & 1)) & 0xFFFF0000
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def forward(p: Dict[str, np.ndarray], x: np.ndarray, bf16: bool = False
            ) -> Tuple[np.ndarray, Dict]:
    """Network output (B, 1, H, W) and the cache needed by backward.

    bf16=True evaluates the network as specified for the matrix cores: the
    input planes, the 3x3 weights, every convolution's activation (after
    bias and ReLU) and every pooled tensor rounded to bfloat16, everything
    else (sums, biases, the 1x1 output layer's weights) in float64."""
    r = bf16_round if bf16 else (lambda a: a)
    w = {k: (r(v) if k.endswith(".w") and k != "out.w" else v) for k, v in p.items()}
    c = {"x": x}
    c["e0i"] = r(x)
    c["e0"] = r(np.maximum(conv3(c["e0i"], w["e0.w"], w["e0.b"]), 0.0))
    c["e1i"] = r(pool(c["e0"]))
    c["e1"] = r(np.maximum(conv3(c["e1i"], w["e1.w"], w["e1.b"]), 0.0))
    c["e2i"] = r(pool(c["e1"]))
    c["e2"] = r(np.maximum(conv3(c["e2i"], w["e2.w"], w["e2.b"]), 0.0))
    c["e3i"] = r(pool(c["e2"]))
    c["e3"] = r(np.maximum(conv3(c["e3i"], w["e3.w"], w["e3.b"]), 0.0))
    c["d2i"] = np.concatenate([up(c["e3"]), c["e2"]], axis=1)
    c["d2"] = r(np.maximum(conv3(c["d2i"], w["d2.w"], w["d2.b"]), 0.0))
    c["d1i"] = np.concatenate([up(c["d2"]), c["e1"]], axis=1)
    c["d1"] = r(np.maximum(conv3(c["d1i"], w["d1.w"], w["d1.b"]), 0.0))
    c["d0i"] = np.concatenate([up(c["d1"]), c["e0"]], axis=1)
    c["d0"] = r(np.maximum(conv3(c["d0i"], w["d0.w"], w["d0.b"]), 0.0))
    y = np.einsum("oc,bchw->bohw", w["out.w"], c["d0"]) + w["out.b"][None, :, None, None]
    return y, c


def loss(y: np.ndarray, t: np.ndarray) -> float:
    return float(np.mean((y - t) ** 2))


def backward(p, c, y, t) -> Dict[str, np.ndarray]:
    """Gradients of the mean-squared-error loss with respect to every
    parameter (and the input, under key 'x')."""
    g = {}
    dy = 2.0 * (y - t) / y.size
    g["out.w"] = np.einsum("bohw,bchw->oc", dy, c["d0"])
    g["out.b"] = dy.sum(axis=(0, 2, 3))
    dd0 = np.einsum("oc,bohw->bchw", p["out.w"], dy)

    def layer(name, dout, inp):
        dpre = dout * (c[name] > 0.0)
        dx, g[name + ".w"], g[name + ".b"] = conv3_backward(c[inp], p[name + ".w"], dpre)
        return dx

    dd0i = layer("d0", dd0, "d0i")
    n_up = c["d1"].shape[1]
    dd1 = up_backward(dd0i[:, :n_up])
    de0 = dd0i[:, n_up:].copy()
    dd1i = layer("d1", dd1, "d1i")
    n_up = c["d2"].shape[1]
    dd2 = up_backward(dd1i[:, :n_up])
    de1 = dd1i[:, n_up:].copy()
    dd2i = layer("d2", dd2, "d2i")
    n_up = c["e3"].shape[1]
    de3 = up_backward(dd2i[:, :n_up])
    de2 = dd2i[:, n_up:].copy()
    de3i = layer("e3", de3, "e3i")
    de2 = de2 + pool_backward(de3i)
    de2i = layer("e2", de2, "e2i")
    de1 = de1 + pool_backward(de2i)
    de1i = layer("e1", de1, "e1i")
    de0 = de0 + pool_backward(de1i)
    g["x"] = layer("e0", de0, "e0i")
    return g


def adam(p, g, m, v, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (bias-corrected), in place; step counts from 1."""
    for k in p:
        m[k] = b1 * m[k] + (1 - b1) * g[k]
        v[k] = b2 * v[k] + (1 - b2) * g[k] ** 2
        mh = m[k] / (1 - b1 ** step)
        vh = v[k] / (1 - b2 ** step)
        p[k] -= lr * mh / (np.sqrt(vh) + eps)
