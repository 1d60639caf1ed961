"""Pins of the FP64 network reference (oracle/unet.py): convolution against
SciPy's 2-D correlation, the layer algebra against its definitions, and
every gradient against central finite differences of the loss."""
import numpy as np
import pytest
from scipy.signal import correlate2d

from oracle import unet


def test_conv3_equals_scipy_correlation():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((2, 3, 8, 10))
    w = rng.standard_normal((4, 3, 3, 3))
    b = rng.standard_normal(4)
    y = unet.conv3(x, w, b)
    for bb in range(2):
        for o in range(4):
            ref = sum(correlate2d(x[bb, c], w[o, c], mode="same", boundary="fill")
                      for c in range(3)) + b[o]
            assert np.allclose(y[bb, o], ref, atol=1e-12)


def test_pool_and_up_are_adjoint_up_to_scale():
    rng = np.random.default_rng(1)
    a = rng.standard_normal((1, 2, 8, 8))
    c = rng.standard_normal((1, 2, 4, 4))
    # <pool(a), c> = <a, pool_backward(c)>, <up(c), a> = <c, up_backward(a)>
    assert np.isclose(np.sum(unet.pool(a) * c), np.sum(a * unet.pool_backward(c)))
    assert np.isclose(np.sum(unet.up(c) * a), np.sum(c * unet.up_backward(a)))
    assert np.allclose(unet.pool(unet.up(c)), c)


def test_gradients_match_finite_differences():
    rng = np.random.default_rng(2)
    p = unet.init_params(3)
    for k in p:
        if k.endswith(".b"):
            p[k] = 0.1 * rng.standard_normal(p[k].shape)
    x = rng.standard_normal((2, 3, 16, 16))
    t = rng.standard_normal((2, 1, 16, 16))
    y, c = unet.forward(p, x)
    g = unet.backward(p, c, y, t)

    def L():
        return unet.loss(unet.forward(p, x)[0], t)

    h = 1e-6
    for key in ["e0.w", "e1.w", "e2.w", "e3.w", "d2.w", "d1.w", "d0.w", "out.w",
                "e0.b", "d2.b", "out.b"]:
        arr = p[key]
        for _ in range(3):
            idx = tuple(int(rng.integers(0, s)) for s in arr.shape)
            old = arr[idx]
            arr[idx] = old + h
            lp = L()
            arr[idx] = old - h
            lm = L()
            arr[idx] = old
            fd = (lp - lm) / (2 * h)
            assert abs(fd - g[key][idx]) <= 1e-6 * max(1.0, abs(fd)) + 1e-9, (key, idx, fd, g[key][idx])
    for _ in range(3):
        idx = tuple(int(rng.integers(0, s)) for s in x.shape)
        old = x[idx]
        x[idx] = old + h
        lp = L()
        x[idx] = old - h
        lm = L()
        x[idx] = old
        assert abs((lp - lm) / (2 * h) - g["x"][idx]) < 1e-7


def test_adam_moves_downhill():
    rng = np.random.default_rng(4)
    p = unet.init_params(5)
    x = rng.standard_normal((1, 3, 16, 16))
    t = np.zeros((1, 1, 16, 16))
    m = {k: np.zeros_like(v) for k, v in p.items()}
    v = {k: np.zeros_like(val) for k, val in p.items()}
    losses = []
    for s in range(1, 6):
        y, c = unet.forward(p, x)
        losses.append(unet.loss(y, t))
        unet.adam(p, unet.backward(p, c, y, t), m, v, s, lr=1e-3)
    assert losses[-1] < losses[0]


def test_adam_two_steps_match_hand_computed_values():
    """Adam (Kingma & Ba, bias-corrected moments; beta1 0.9, beta2 0.999,
    eps 1e-8 added to the square root) on one scalar parameter p0 = 1 with
    lr 0.1 and gradients 2, then -1, worked by hand in exact fractions:
      step 1: m = 1/5, v = 1/250, m_hat = 2, v_hat = 4,
              p1 = 1 - 0.1 * 2 / (2 + 1e-8)                = 0.9000000005
      step 2: m = 9/10 * 1/5 - 1/10 = 2/25,
              v = 999/1000 * 1/250 + 1/1000 = 1249/250000,
              m_hat = (2/25) / (1 - 0.81)    = 8/19,
              v_hat = (1249/250000) / (1 - 0.998001) = 4996/1999,
              p2 = p1 - 0.1 * (8/19) / (sqrt(4996/1999) + 1e-8)
                 = 0.8733662967024313
    and the moments carried between the steps are the fractions above."""
    p = {"w": np.array([1.0])}
    m = {"w": np.zeros(1)}
    v = {"w": np.zeros(1)}
    unet.adam(p, {"w": np.array([2.0])}, m, v, 1, lr=0.1)
    assert abs(m["w"][0] / 0.2 - 1) < 1e-14 and abs(v["w"][0] / 0.004 - 1) < 1e-14
    assert abs(p["w"][0] - 0.9000000005) < 2e-15
    unet.adam(p, {"w": np.array([-1.0])}, m, v, 2, lr=0.1)
    assert abs(m["w"][0] / 0.08 - 1) < 1e-14 and abs(v["w"][0] / 0.004996 - 1) < 1e-14
    assert abs(p["w"][0] - 0.8733662967024313) < 2e-15


def test_bf16_rounding_of_the_network_oracle():
    """Round to nearest bfloat16, ties to even, worked by hand: 1 + 2^-8 is
    halfway between 1 and 1 + 2^-7 and goes to the even 1; 1 + 3 2^-8 is
    halfway between 1 + 2^-7 and 1 + 2^-6 and goes to the even 1 + 2^-6;
    1 + 3 2^-9 is nearer 1 + 2^-7; pi -> 3.140625 (0x4049); 65504 -> 65536;
    the sign is kept."""
    v = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, 1.0 + 3 * 2 ** -9, np.pi, 65504.0,
                  -1.0 - 2 ** -7])
    ref = np.array([1.0, 1.0, 1.0 + 2 ** -6, 1.0 + 2 ** -7, 3.140625, 65536.0, -1.0 - 2 ** -7])
    assert np.array_equal(unet.bf16_round(v), ref)
    # rounded forward: the same network with its operands rounded, close to FP64
    rng = np.random.default_rng(9)
    p = unet.init_params(3)
    x = rng.standard_normal((1, 3, 16, 16))
    y, _ = unet.forward(p, x)
    y16, c16 = unet.forward(p, x, bf16=True)
    assert np.array_equal(unet.bf16_round(c16["d1"]), c16["d1"])
    assert np.linalg.norm(y16 - y) / np.linalg.norm(y) < 3e-2
