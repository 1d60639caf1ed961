"""Learned pressure guess: PyTorch owns the parameter, gradient, moment and
workspace buffers; the forward pass, the backward pass and Adam run in the
library's BF16 matrix-core kernels (include/cdi.h, cdi_net_*)."""
from __future__ import annotations

import ctypes as C
import math

import numpy as np
import torch

from . import _lib as L

# (name, input channels, output channels) of the 3x3 layers, in parameter order
CONV3 = (("e0", 3, 32), ("e1", 32, 64), ("e2", 64, 128), ("e3", 128, 256),
         ("d2", 384, 128), ("d1", 192, 64), ("d0", 96, 32))


def param_layout():
    """[(key, shape)] in the library's parameter order."""
    out = []
    for name, ci, co in CONV3:
        out.append((name + ".w", (co, ci, 3, 3)))
        out.append((name + ".b", (co,)))
    out.append(("out.w", (1, 32)))
    out.append(("out.b", (1,)))
    return out


def init_params(seed: int = 0) -> np.ndarray:
    """He-normal weights and zero biases, flattened in the library order."""
    g = np.random.default_rng(seed)
    parts = []
    for key, shape in param_layout():
        if key.endswith(".b"):
            parts.append(np.zeros(shape))
        elif key == "out.w":
            parts.append(g.standard_normal(shape) * math.sqrt(1.0 / 32))
        else:
            parts.append(g.standard_normal(shape) * math.sqrt(2.0 / (shape[1] * 9)))
    return np.concatenate([p.reshape(-1) for p in parts]).astype(np.float32)


def flatten(params: dict) -> np.ndarray:
    return np.concatenate([np.asarray(params[k], dtype=np.float32).reshape(-1)
                           for k, _ in param_layout()])


def unflatten(vec: np.ndarray) -> dict:
    out, o = {}, 0
    for key, shape in param_layout():
        n = int(np.prod(shape))
        out[key] = vec[o:o + n].reshape(shape)
        o += n
    return out


class GuessNet:
    """One network instance of fixed batch and image size on one GPU."""

    def __init__(self, batch: int, h: int, w: int, params=None, train: bool = True,
                 device: str = "cuda:0", stream=None, share: "GuessNet | None" = None):
        """share: another network whose parameter, gradient and Adam-moment
        buffers this one uses (the same weights on another image shape);
        after the other network's Adam step, call repack() here."""
        self.lib = L.lib()
        self.device = torch.device(device)
        n = self.lib.cdi_net_param_count()
        if share is not None:
            self.params, self.grads, self.m, self.v = share.params, share.grads, share.m, share.v
        else:
            p = init_params(0) if params is None else np.asarray(params, dtype=np.float32)
            if p.size != n:
                raise ValueError(f"expected {n} parameters, got {p.size}")
            self.params = torch.as_tensor(p, device=self.device).clone()
            self.grads = torch.zeros(n, dtype=torch.float32, device=self.device)
            self.m = torch.zeros_like(self.grads)
            self.v = torch.zeros_like(self.grads)
        self.batch, self.h, self.w, self.train = batch, h, w, train
        nbytes = self.lib.cdi_net_workspace_bytes(batch, h, w, int(train))
        if nbytes == 0:
            raise L.CDIError(-2, "unsupported network shape")
        raw = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        self._raw = raw
        ws = raw.data_ptr() + (-raw.data_ptr()) % 256
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.y = torch.zeros((batch, h, w), dtype=torch.float32, device=self.device)
        self.loss_dev = torch.zeros(1, dtype=torch.float32, device=self.device)
        handle = C.c_void_p()
        L.check_net(self.lib.cdi_net_init(self.params.data_ptr(), self.grads.data_ptr(), batch, h,
                                          w, int(train), ws, nbytes, self.stream.cuda_stream,
                                          C.byref(handle)))
        self.handle = handle
        self.step = 0

    def forward(self, x: torch.Tensor) -> torch.Tensor:
        x = x.to(self.device, torch.float32).contiguous()
        L.check_net(self.lib.cdi_net_forward(self.handle, x.data_ptr(), self.y.data_ptr()))
        return self.y

    def backward(self, target: torch.Tensor) -> torch.Tensor:
        t = target.to(self.device, torch.float32).contiguous()
        self._t = t
        L.check_net(self.lib.cdi_net_backward(self.handle, t.data_ptr(), self.loss_dev.data_ptr()))
        return self.loss_dev

    def adam(self, lr: float = 1e-3):
        self.step += 1
        L.check_net(self.lib.cdi_net_adam(self.handle, self.m.data_ptr(), self.v.data_ptr(),
                                          self.step, lr))

    def repack(self):
        """Re-pack the BF16 weights from the (shared) FP32 parameters."""
        L.check_net(self.lib.cdi_net_repack(self.handle))

    def set_params(self, vec):
        self.params.copy_(torch.as_tensor(np.asarray(vec, dtype=np.float32)))
        L.check_net(self.lib.cdi_net_repack(self.handle))

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            self.lib.cdi_net_destroy(self.handle)
            self.handle = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def main(argv=None):
    """Time the inference forward pass of a randomly initialised network on
    an h x w image (the learned guess's cost per solve), e.g. under a
    profiler:  python -m paper_2412_16843_amd.learned --h 1024 --w 2048"""
    import argparse
    import time
    ap = argparse.ArgumentParser(description=main.__doc__.split("\n")[0])
    ap.add_argument("--h", type=int, default=1024)
    ap.add_argument("--w", type=int, default=2048)
    ap.add_argument("--reps", type=int, default=20)
    a = ap.parse_args(argv)
    net = GuessNet(1, a.h, a.w, train=False)
    x = torch.randn((1, 3, a.h, a.w), dtype=torch.float32, device=net.device)
    net.forward(x)
    torch.cuda.synchronize(net.device)
    t0 = time.perf_counter()
    for _ in range(a.reps):
        net.forward(x)
    torch.cuda.synchronize(net.device)
    ms = (time.perf_counter() - t0) / a.reps * 1e3
    net.close()
    # 3x3 convolutions: 2 * co * ci * 9 per pixel of each level (decoder
    # inputs include the skip channels), plus the 1x1 output layer
    flops, hw = 0.0, a.h * a.w
    for name, ci, co in CONV3:
        lvl = {"e0": 0, "e1": 1, "e2": 2, "e3": 3, "d2": 2, "d1": 1, "d0": 0}[name]
        flops += 2.0 * co * ci * 9 * hw / 4 ** lvl
    flops += 2.0 * 32 * hw
    print(f"forward {a.h}x{a.w}: {ms:.3f} ms, {flops / 1e9:.1f} GFLOP (3 input channels), "
          f"{flops / ms / 1e9:.1f} TFLOP/s", flush=True)


if __name__ == "__main__":
    main()
