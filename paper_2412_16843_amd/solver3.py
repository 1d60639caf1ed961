"""Python wrapper of the three-dimensional C ABI (include/cdi3.h).

Allocates the caller-owned fields and the workspace with PyTorch on the
current HIP device and marshals arguments; every step runs in the library's
kernels.
"""
from __future__ import annotations

import ctypes as C
from typing import Dict

import numpy as np
import torch

from . import _lib as L


class CDISolver3:
    """One 3-D CDI + GNBC problem (x and z periodic, walls normal to y).

    params: a workloads.Params3; phi0: (nz, ny, nx) initial phase field;
    u0, v0, w0: optional initial velocities ((nz, ny, nx), (nz, ny+1, nx),
    (nz, ny, nx))."""

    def __init__(self, params, phi0, u0=None, v0=None, w0=None, guess: str = "prev",
                 rtol: float = 1e-10, maxit: int = 0, device: str = "cuda:0", mg_smooth: int = 0):
        self.lib = L.lib()
        self.device = torch.device(device)
        self.p = params
        nx, ny, nz = params.nx, params.ny, params.nz
        self.shape = (nz, ny, nx)
        dev = self.device
        t = lambda a, shp: (torch.zeros(shp, dtype=torch.float64, device=dev) if a is None
                            else torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64)
                            .to(dev).reshape(shp).contiguous())
        self.fields = {"phi": t(phi0, (nz, ny, nx)), "u": t(u0, (nz, ny, nx)),
                       "v": t(v0, (nz, ny + 1, nx)), "w": t(w0, (nz, ny, nx)),
                       "p": torch.zeros((nz, ny, nx), dtype=torch.float64, device=dev)}
        self.cparams = L.make_params3(params, guess=guess, rtol=rtol, maxit=maxit,
                                     mg_smooth=mg_smooth)
        nbytes = C.c_size_t(0)
        L.check(self.lib.cdi3_workspace_bytes(C.byref(self.cparams), C.byref(nbytes)))
        self.ws = torch.empty(nbytes.value + 256, dtype=torch.uint8, device=dev)
        base = self.ws.data_ptr()
        base = (base + 255) & ~255
        f = self.fields
        self.cfields = L.cdi3_fields(phi=f["phi"].data_ptr(), u=f["u"].data_ptr(),
                                     v=f["v"].data_ptr(), w=f["w"].data_ptr(), p=f["p"].data_ptr())
        torch.cuda.synchronize(dev)
        ctx = C.c_void_p()
        L.check(self.lib.cdi3_init(C.byref(self.cparams), C.byref(self.cfields), C.c_void_p(base),
                                   nbytes.value, None, C.byref(ctx)))
        self.ctx = ctx

    def step(self, nsteps: int = 1) -> None:
        L.check(self.lib.cdi3_step(self.ctx, nsteps))

    def eval_rhs(self) -> Dict[str, np.ndarray]:
        nz, ny, nx = self.shape
        dev = self.device
        z = lambda shp: torch.zeros(shp, dtype=torch.float64, device=dev)
        out = {"Lphi": z((nz, ny, nx)), "Lmx": z((nz, ny, nx)), "Lmy": z((nz, ny + 1, nx)),
               "Lmz": z((nz, ny, nx)), "uYx": z((2, nz, nx)), "uYz": z((2, nz, nx))}
        L.check(self.lib.cdi3_eval_rhs(self.ctx, *[out[k].data_ptr() for k in
                                                   ("Lphi", "Lmx", "Lmy", "Lmz", "uYx", "uYz")]))
        torch.cuda.synchronize(dev)
        return {k: v.cpu().numpy() for k, v in out.items()}

    def kappa_p(self) -> np.ndarray:
        out = torch.zeros(self.shape, dtype=torch.float64, device=self.device)
        L.check(self.lib.cdi3_kappa_p(self.ctx, out.data_ptr()))
        torch.cuda.synchronize(self.device)
        return out.cpu().numpy()

    def diagnostics(self) -> Dict[str, float]:
        d = L.cdi3_diag()
        L.check(self.lib.cdi3_diagnostics(self.ctx, C.byref(d)))
        return dict(t=d.t, step=d.step, mass=d.mass, phi_min=d.phi_min, phi_max=d.phi_max,
                    max_div=d.max_div, max_slip_bot=d.max_slip[0], max_slip_top=d.max_slip[1],
                    max_uY_bot=d.max_uY[0], max_uY_top=d.max_uY[1], ke=d.ke,
                    last_iters=d.last_iters, last_relres=d.last_relres)

    def time_stage(self, reps: int = 10) -> float:
        ms = C.c_double(0.0)
        L.check(self.lib.cdi3_time_stage(self.ctx, reps, C.byref(ms)))
        return ms.value

    def state(self) -> Dict[str, np.ndarray]:
        torch.cuda.synchronize(self.device)
        return {k: v.detach().cpu().numpy().copy() for k, v in self.fields.items()}

    def close(self) -> None:
        if getattr(self, "ctx", None):
            self.lib.cdi3_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
