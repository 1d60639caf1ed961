"""Learned pressure guess on the GPU: BF16 matrix-core forward and backward
against the FP64 network oracle, training, and the gain of the trained guess
over the plain solver.

Tolerances: activations and activation gradients are rounded to BF16 (unit
round-off 2^-9 ~ 2e-3) at each of the 8 layers with FP32 accumulation, so
outputs agree with the FP64 reference to a few 1e-3 relative (bound 3e-2),
parameter gradients to a few percent in norm (bound 6e-2), with cosine
similarity above 0.998.
"""
import numpy as np
import pytest

import workloads as W
from oracle import unet

pytestmark = pytest.mark.gpu


def _torch():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _rand_params(seed):
    from paper_2412_16843_amd import learned
    rng = np.random.default_rng(seed)
    p = learned.unflatten(learned.init_params(seed).astype(np.float64))
    for k in p:
        if k.endswith(".b"):
            p[k] = 0.05 * rng.standard_normal(p[k].shape)
    return p


@pytest.mark.parametrize("B,H,Wd", [(2, 16, 16), (1, 32, 96), (1, 40, 48)])
def test_network_forward_and_gradients_match_fp64_oracle(B, H, Wd):
    """(1, 40, 48): 32 weight-gradient row chunks of 2 rows cover the 40 rows
    of level 0 (the last chunks hold no rows), a split the kernel once
    recomputed inconsistently from the row count."""
    torch = _torch()
    from paper_2412_16843_amd import learned
    rng = np.random.default_rng(7)
    p = _rand_params(1)
    x = rng.standard_normal((B, 3, H, Wd))
    t = rng.standard_normal((B, 1, H, Wd))
    y_ref, cache = unet.forward(p, x)
    g_ref = unet.backward(p, cache, y_ref, t)
    net = learned.GuessNet(B, H, Wd, params=learned.flatten(p))
    y = net.forward(torch.as_tensor(x, dtype=torch.float32)).cpu().numpy()
    assert np.linalg.norm(y - y_ref[:, 0]) / np.linalg.norm(y_ref) < 3e-2
    loss = net.backward(torch.as_tensor(t[:, 0], dtype=torch.float32)).item()
    assert abs(loss - unet.loss(y_ref, t)) < 3e-2 * unet.loss(y_ref, t)
    g = learned.unflatten(net.grads.cpu().numpy())
    for key, _ in learned.param_layout():
        a, b = g[key].reshape(-1).astype(np.float64), g_ref[key].reshape(-1)
        rel = np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30)
        cos = float(a @ b / max(np.linalg.norm(a) * np.linalg.norm(b), 1e-30))
        assert rel < 6e-2 and cos > 0.998, (key, rel, cos)
    net.close()


@pytest.mark.parametrize("B,H,Wd", [(2, 16, 16), (1, 24, 40), (1, 32, 96)])
def test_inference_forward_equals_training_forward(B, H, Wd):
    """The inference net reads cat(up2(lo), skip) in place inside the decoder
    convolutions; the training net additionally stores the concatenation.
    Both must give the same output bit for bit, and match the oracle (widths
    24 and 40 take the unvectorised column path at some level)."""
    torch = _torch()
    from paper_2412_16843_amd import learned
    rng = np.random.default_rng(11)
    p = _rand_params(3)
    x = rng.standard_normal((B, 3, H, Wd))
    tr = learned.GuessNet(B, H, Wd, params=learned.flatten(p))
    inf = learned.GuessNet(B, H, Wd, params=learned.flatten(p), train=False)
    xt = torch.as_tensor(x, dtype=torch.float32)
    y_tr = tr.forward(xt).cpu().numpy()
    y_inf = inf.forward(xt).cpu().numpy()
    tr.close()
    inf.close()
    assert np.array_equal(y_tr, y_inf)
    y_ref, _ = unet.forward(p, x)
    assert np.linalg.norm(y_inf - y_ref[:, 0]) / np.linalg.norm(y_ref) < 3e-2


def test_training_reduces_loss_and_guess_beats_zero():
    torch = _torch()
    from paper_2412_16843_amd import learned, train_guess
    from paper_2412_16843_amd.solver import CDISolver
    cases = [W.drop_case(128, 64, th, 10.0, steps=40) for th in (45.0, 75.0, 105.0)]
    data = train_guess.collect(cases, steps=40, every=1)
    trms = [float(t.square().mean().sqrt()) for _, t in data]
    print("target rms: min %.3e max %.3e" % (min(trms), max(trms)))
    net = learned.GuessNet(8, 64, 128)
    losses = train_guess.train(net, data, iters=300, lr=2e-3, log_every=50)
    first, last = train_guess.loss_summary(losses)   # means over 30 iterations each
    print("loss: first 10 %% %.4f, last 10 %% %.4f" % (first, last))
    assert last < 0.5 * first, (first, last)
    # held-out case: compare the pressure solve from zero and from the network
    case = W.drop_case(128, 64, 60.0, 10.0, steps=10)
    plain = CDISolver(case.params, case.phi0, guess="zero", rtol=1e-10)
    prev = CDISolver(case.params, case.phi0, guess="prev", rtol=1e-10)
    lrn = CDISolver(case.params, case.phi0, guess="learned", rtol=1e-10)
    inf = learned.GuessNet(1, 64, 128, params=net.params.cpu().numpy(), train=False,
                           stream=lrn.stream)
    lrn.attach_guess(inf)
    it_zero, it_prev, it_learn = [], [], []
    for _ in range(case.steps):
        plain.step(1)
        prev.step(1)
        lrn.step(1)
        it_zero.append(plain.diagnostics()["last_iters"])
        it_prev.append(prev.diagnostics()["last_iters"])
        it_learn.append(lrn.diagnostics()["last_iters"])
    print("iterations from zero:", it_zero, "from the extrapolated history:", it_prev,
          "from the network fitted on that history:", it_learn)
    assert np.mean(it_learn) < np.mean(it_zero)
    # the fit spans the plain guess, so it starts no farther (energy norm)
    # from the solution: no more iterations on average
    assert np.mean(it_learn) <= np.mean(it_prev) + 0.5
    a, b = plain.state(), lrn.state()
    # both converge to the same 1e-10 residual: fields agree closely
    assert np.abs(a["phi"] - b["phi"]).max() < 1e-8
    inf.close(); net.close(); plain.close(); prev.close(); lrn.close()


@pytest.mark.parametrize("garbage", ["nan", "huge"])
def test_garbage_network_falls_back_to_the_plain_guess(garbage):
    """Network weights that produce a non-finite output (NaN weights, or
    weights so large that the fit's sums overflow) must not break a solve:
    the fit keeps the plain guess alone, so the run is bit for bit the run
    without the network."""
    torch = _torch()
    from paper_2412_16843_amd import learned
    from paper_2412_16843_amd._lib import lib
    from paper_2412_16843_amd.solver import CDISolver
    case = W.drop_case(128, 64, 60.0, 10.0)
    prev = CDISolver(case.params, case.phi0, guess="prev", rtol=1e-10)
    lrn = CDISolver(case.params, case.phi0, guess="learned", rtol=1e-10)
    n = lib().cdi_net_param_count()
    bad = np.full(n, np.nan if garbage == "nan" else 1e30, dtype=np.float32)
    inf = learned.GuessNet(1, 64, 128, params=bad, train=False, stream=lrn.stream)
    lrn.attach_guess(inf)
    it_prev, it_learn = [], []
    for _ in range(6):
        prev.step(1)
        lrn.step(1)
        it_prev.append(prev.diagnostics()["last_iters"])
        it_learn.append(lrn.diagnostics()["last_iters"])
    a, b = prev.state(), lrn.state()
    print(garbage, "iterations without / with the network:", it_prev, it_learn)
    assert it_learn == it_prev
    for k in ("phi", "u", "v", "p"):
        assert np.array_equal(a[k], b[k]), k
    inf.close(); prev.close(); lrn.close()


# elementwise bound of the GPU forward pass against the oracle evaluated with
# the same bfloat16 rounding points (input planes, 3x3 weights, activations,
# pooled tensors): what remains is the FP32 accumulation order of the
# matrix cores, which moves a pre-rounding value by ~1e-6 relative and so
# flips an occasional activation by one bfloat16 ulp (2^-8) that the next
# layers carry on; relative to |y| + rms(y)
BF16_ELEMENTWISE = 2.0 ** -6


@pytest.mark.parametrize("B,H,Wd", [(2, 16, 16), (1, 32, 96), (1, 40, 48)])
def test_network_forward_elementwise_against_bf16_oracle(B, H, Wd):
    """Every output element of the BF16 / FP32-accumulate GPU forward pass
    (training and inference forms) against the oracle network evaluated with
    the matrix cores' bfloat16 rounding points."""
    torch = _torch()
    from paper_2412_16843_amd import learned
    rng = np.random.default_rng(17)
    p = _rand_params(2)
    x = rng.standard_normal((B, 3, H, Wd))
    y16, _ = unet.forward(p, x, bf16=True)
    y16 = y16[:, 0]
    scale = np.abs(y16) + np.sqrt(np.mean(y16 ** 2))
    for train in (True, False):
        net = learned.GuessNet(B, H, Wd, params=learned.flatten(p), train=train)
        y = net.forward(torch.as_tensor(x, dtype=torch.float32)).cpu().numpy()
        net.close()
        r = np.abs(y - y16) / scale
        print(f"B{B} {H}x{Wd} train={train}: |y - y_bf16| / (|y| + rms): max {r.max():.2e}, "
              f"99th percentile {np.percentile(r, 99):.2e}, median {np.median(r):.2e}")
        assert r.max() <= BF16_ELEMENTWISE, (train, r.max())


def test_gpu_adam_matches_oracle_adam():
    """Three Adam steps of the library kernel (FP32 master parameters and
    moments) against the oracle's Adam in FP64 on the same parameters and
    gradients: the parameters agree to FP32 round-off of the update."""
    torch = _torch()
    from paper_2412_16843_amd import learned
    rng = np.random.default_rng(23)
    p0 = learned.init_params(4).astype(np.float64)
    net = learned.GuessNet(1, 16, 16, params=p0)
    po = {"w": p0.astype(np.float32).astype(np.float64)}
    mo = {"w": np.zeros_like(po["w"])}
    vo = {"w": np.zeros_like(po["w"])}
    # the first moment of |g|: the scale of the terms m is a sum of
    pa, ma, va = {"w": po["w"].copy()}, {"w": np.zeros_like(po["w"])}, {"w": np.zeros_like(po["w"])}
    lr = 1e-3
    for step in range(1, 4):
        g = (rng.standard_normal(p0.size) * 10.0 ** rng.uniform(-4, 0, p0.size)).astype(np.float32)
        net.grads.copy_(torch.as_tensor(g))
        net.adam(lr)
        unet.adam(po, {"w": g.astype(np.float64)}, mo, vo, step, lr=lr)
        unet.adam(pa, {"w": np.abs(g).astype(np.float64)}, ma, va, step, lr=lr)
    pg = net.params.cpu().numpy().astype(np.float64)
    mg = net.m.cpu().numpy().astype(np.float64)
    net.close()
    # each update moves a parameter by at most ~lr; FP32 evaluates it to a
    # few ulps of the update and rounds the parameter (|p| ulp)
    err = np.abs(pg - po["w"])
    bound = 4 * np.finfo(np.float32).eps * (np.abs(po["w"]) + 3 * lr)
    print("Adam: max |dp| / bound", float((err / bound).max()))
    assert (err <= bound).all(), float((err / bound).max())
    assert (np.abs(mg - mo["w"]) <= 8 * np.finfo(np.float32).eps * ma["w"]).all()
