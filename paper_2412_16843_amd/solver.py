"""Python front end of libcdi: device memory and streams come from PyTorch,
every computation runs in the library's HIP kernels."""
from __future__ import annotations

import ctypes as C
from typing import Dict, List, Sequence

import numpy as np
import torch

from . import _lib as L


def _ptr(t: torch.Tensor) -> int:
    return t.data_ptr()


class CDISolver:
    """One instance, or a batch of independent instances, of the CDI + GNBC
    step on one GPU.

    params: parameter objects (attributes as in workloads.Params);
    phi0:   initial phase fields, arrays of shape (ny, nx).
    """

    def __init__(self, params, phi0, precision: str = "fp64", guess: str = "prev",
                 rtol: float = 0.0, maxit: int = 0, device: str = "cuda:0", u0=None, v0=None,
                 launch: str = "tiled", mg_smooth: int = 0):
        if not torch.cuda.is_available():
            raise RuntimeError("CDISolver needs a GPU (the HIP library has no CPU path)")
        single = not isinstance(params, (list, tuple))
        self.params: List = [params] if single else list(params)
        phis = [phi0] if single else list(phi0)
        us = [u0] if single else (u0 if u0 is not None else [None] * len(phis))
        vs = [v0] if single else (v0 if v0 is not None else [None] * len(phis))
        if len(phis) != len(self.params):
            raise ValueError("one phase field per instance is required")
        self.n = len(self.params)
        self.device = torch.device(device)
        self.lib = L.lib()
        self.cparams = (L.cdi_params * self.n)(*[
            L.make_params(p, precision, guess, rtol, maxit, mg_smooth) for p in self.params])
        self.fields: List[Dict[str, torch.Tensor]] = []
        cf = (L.cdi_fields * self.n)()
        for k, p in enumerate(self.params):
            f = dict(
                phi=torch.as_tensor(np.ascontiguousarray(phis[k], dtype=np.float64),
                                    device=self.device).clone(),
                u=torch.zeros((p.ny, p.nx), dtype=torch.float64, device=self.device),
                v=torch.zeros((p.ny + 1, p.nx), dtype=torch.float64, device=self.device),
                p=torch.zeros((p.ny, p.nx), dtype=torch.float64, device=self.device))
            if us[k] is not None:
                f["u"].copy_(torch.as_tensor(np.asarray(us[k], dtype=np.float64)))
            if vs[k] is not None:
                f["v"].copy_(torch.as_tensor(np.asarray(vs[k], dtype=np.float64)))
            self.fields.append(f)
            cf[k] = L.cdi_fields(_ptr(f["phi"]), _ptr(f["u"]), _ptr(f["v"]), _ptr(f["p"]))
        self.cfields = cf
        nbytes = self.lib.cdi_workspace_bytes(self.cparams, self.n)
        if nbytes == 0:
            raise L.CDIError(-1, self.lib.cdi_last_error().decode())
        raw = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        off = (-raw.data_ptr()) % 256
        self._ws_raw = raw
        self.ws_ptr = raw.data_ptr() + off
        self.ws_bytes = nbytes
        self.stream = torch.cuda.current_stream(self.device)
        ctx = C.c_void_p()
        torch.cuda.synchronize(self.device)
        L.check(self.lib.cdi_init_batch(self.cparams, self.n, self.cfields, self.ws_ptr, nbytes,
                                        self.stream.cuda_stream, C.byref(ctx)))
        self.ctx = ctx
        if launch != "tiled":
            self.set_launch(launch)

    # ------------------------------------------------------------------ run
    def step(self, nsteps: int = 1, allow_noconv: bool = False) -> int:
        return L.check(self.lib.cdi_step(self.ctx, int(nsteps)),
                       allow=(-4,) if allow_noconv else ())

    def cg_iterations(self) -> List[int]:
        """CG iterations each instance has run since the context was set up."""
        out = (C.c_int64 * self.n)()
        L.check(self.lib.cdi_cg_iterations(self.ctx, out))
        return list(out)

    def diagnostics(self, idx: int = 0) -> Dict[str, float]:
        d = L.cdi_diag()
        L.check(self.lib.cdi_diagnostics(self.ctx, idx, C.byref(d)), allow=(-5,))
        return dict(t=d.t, step=d.step, mass=d.mass, mass0=d.mass0, phi_min=d.phi_min,
                    phi_max=d.phi_max, max_div=d.max_div, max_uslip_bot=d.max_uslip[0],
                    max_uslip_top=d.max_uslip[1], max_uY_bot=d.max_uY[0],
                    max_uY_top=d.max_uY[1], ke=d.ke, last_iters=d.last_iters,
                    last_relres=d.last_relres, nonfinite=d.nonfinite,
                    n_contact_bot=d.n_contact[0], n_contact_top=d.n_contact[1],
                    contact_x_bot=[d.contact_x[k] for k in range(min(2, d.n_contact[0]))],
                    contact_x_top=[d.contact_x[2 + k] for k in range(min(2, d.n_contact[1]))],
                    wetted_len_bot=d.wetted_len[0], wetted_len_top=d.wetted_len[1],
                    theta_est_bot=d.theta_est[0], theta_est_top=d.theta_est[1])

    def eval_rhs(self):
        """Stage operator on the current fields of instance 0."""
        p = self.params[0]
        dev = self.device
        lphi = torch.empty((p.ny, p.nx), dtype=torch.float64, device=dev)
        lmx = torch.empty((p.ny, p.nx), dtype=torch.float64, device=dev)
        lmy = torch.empty((p.ny + 1, p.nx), dtype=torch.float64, device=dev)
        uy = torch.empty((2, p.nx), dtype=torch.float64, device=dev)
        us = torch.empty((2, p.nx), dtype=torch.float64, device=dev)
        L.check(self.lib.cdi_eval_rhs(self.ctx, _ptr(lphi), _ptr(lmx), _ptr(lmy), _ptr(uy),
                                      _ptr(us)))
        return lphi, lmx, lmy, uy, us

    def solve_pressure(self, b: torch.Tensor, p0: torch.Tensor | None = None):
        p = self.params[0]
        out = torch.zeros((p.ny, p.nx), dtype=torch.float64, device=self.device)
        if p0 is not None:
            out.copy_(p0)
        info = L.cdi_solve_info()
        bb = b.to(device=self.device, dtype=torch.float64).contiguous()
        st = self.lib.cdi_solve_pressure(self.ctx, _ptr(bb), _ptr(out), C.byref(info))
        L.check(st, allow=(-4,))
        return out, dict(iterations=info.iterations, converged=info.converged,
                         relres=info.relres, bnorm=info.bnorm, ms=info.ms, status=st)

    def set_launch(self, mode: str) -> None:
        """How cdi_step enqueues a step: "tiled", "persistent" or "graph"."""
        L.check(self.lib.cdi_set_launch(self.ctx, L.LAUNCH[mode]))

    def get_launch(self) -> str:
        m = C.c_int32()
        L.check(self.lib.cdi_get_launch(self.ctx, C.byref(m)))
        return {v: k for k, v in L.LAUNCH.items()}[m.value]

    def graph_stats(self) -> Dict[str, int]:
        r, m, b = C.c_int64(), C.c_int64(), C.c_int32()
        L.check(self.lib.cdi_graph_stats(self.ctx, C.byref(r), C.byref(m), C.byref(b)))
        return dict(replays=r.value, redone=m.value, budget=b.value)

    def set_strip_rows(self, rows: int) -> None:
        L.check(self.lib.cdi_set_strip_rows(self.ctx, rows))

    def get_strip_rows(self) -> int:
        r = C.c_int32(0)
        L.check(self.lib.cdi_get_strip_rows(self.ctx, C.byref(r)))
        return r.value

    def set_tile_rows(self, rows: int) -> None:
        """Rows per thread of the wide-tile CG kernels (1 or 4)."""
        L.check(self.lib.cdi_set_tile_rows(self.ctx, int(rows)))

    def set_mg_smooth(self, nu: int) -> None:
        """Red-black sweep pairs of the V-cycle (1 or 2)."""
        L.check(self.lib.cdi_set_mg_smooth(self.ctx, int(nu)))

    def get_mg_smooth(self) -> int:
        m = C.c_int32()
        L.check(self.lib.cdi_get_mg_smooth(self.ctx, C.byref(m)))
        return m.value

    def set_extrapolation(self, order: int) -> None:
        """Order (0..3) of the time extrapolation of the previous steps'
        pressure that starts each solve."""
        L.check(self.lib.cdi_set_extrapolation(self.ctx, int(order)))

    def get_extrapolation(self) -> int:
        m = C.c_int32()
        L.check(self.lib.cdi_get_extrapolation(self.ctx, C.byref(m)))
        return m.value

    def set_coarse_cells(self, cells: int) -> None:
        """Levels with at most `cells` cells run in the one-block coarse kernel."""
        L.check(self.lib.cdi_set_coarse_cells(self.ctx, int(cells)))

    def get_coarse_cells(self) -> int:
        m = C.c_int32()
        L.check(self.lib.cdi_get_coarse_cells(self.ctx, C.byref(m)))
        return m.value

    def get_tile_rows(self) -> int:
        m = C.c_int32()
        L.check(self.lib.cdi_get_tile_rows(self.ctx, C.byref(m)))
        return m.value

    def tune(self, trial_steps: int = 10) -> Dict:
        """Time every launch candidate from the current state (restored
        afterwards) and keep the fastest; returns the choice and timings."""
        nb = self.lib.cdi_tune_bytes(self.ctx)
        scratch = torch.empty(nb + 256, dtype=torch.uint8, device=self.device)
        ptr = scratch.data_ptr() + (-scratch.data_ptr()) % 256
        info = L.cdi_tune_info()
        L.check(self.lib.cdi_tune(self.ctx, int(trial_steps), ptr, nb, C.byref(info)))
        torch.cuda.synchronize(self.device)
        del scratch
        names = {v: k for k, v in L.LAUNCH.items()}
        ms = {}
        for v, nu in enumerate((1, 2)):
            for r, rows in enumerate((1, 4)):
                for q, cc in enumerate((1024, 4096, 16384)):
                    ms[f"tiled_nu{nu}_rows{rows}_coarse{cc}"] = info.ms_per_step[v * 6 + r * 3 + q]
        ms["persistent"] = info.ms_per_step[12]
        ms["graph"] = info.ms_per_step[13]
        return dict(launch=names[info.launch], tile_rows=info.tile_rows,
                    coarse_cells=info.coarse_cells, mg_smooth=info.mg_smooth, ms_per_step=ms)

    def set_guess(self, mode: str) -> None:
        """Initial-guess mode of later solves: "zero", "prev" or "learned"."""
        L.check(self.lib.cdi_set_guess(self.ctx, L.GUESS[mode]))

    def solve_last_rhs(self, p0=None):
        """Re-solve the last projection's pressure equation (b = NULL)."""
        p = self.params[0]
        out = torch.zeros((p.ny, p.nx), dtype=torch.float64, device=self.device)
        if p0 is not None:
            out.copy_(p0)
        info = L.cdi_solve_info()
        st = self.lib.cdi_solve_pressure(self.ctx, None, out.data_ptr(), C.byref(info))
        L.check(st, allow=(-4,))
        return out, dict(iterations=info.iterations, converged=info.converged,
                         relres=info.relres, ms=info.ms, guess_used=info.guess_used)

    def attach_guess(self, net) -> None:
        """Use a GuessNet (batch 1, h = ny, w = nx) for every solve's initial
        guess (context created with guess="learned"); None detaches."""
        L.check(self.lib.cdi_guess_attach(self.ctx, net.handle if net is not None else None))
        self._net = net

    def guess_features(self, idx: int = 0):
        """Features [3, ny, nx] and normalised target [ny, nx] of the last
        projection of instance idx (FP32 device tensors)."""
        p = self.params[idx]
        f = torch.empty((3, p.ny, p.nx), dtype=torch.float32, device=self.device)
        t = torch.empty((p.ny, p.nx), dtype=torch.float32, device=self.device)
        L.check(self.lib.cdi_guess_features(self.ctx, idx, f.data_ptr(), t.data_ptr()))
        return f, t

    def timing_enable(self, kernel: str | None):
        L.check(self.lib.cdi_timing_enable(self.ctx, kernel.encode() if kernel else None))

    def timing_read(self):
        ms = C.c_double()
        n = C.c_int64()
        L.check(self.lib.cdi_timing_read(self.ctx, C.byref(ms), C.byref(n)))
        return ms.value, n.value

    def state(self, idx: int = 0):
        torch.cuda.synchronize(self.device)
        f = self.fields[idx]
        return {k: v.detach().cpu().numpy().copy() for k, v in f.items()}

    def set_state(self, idx: int, phi=None, u=None, v=None, p=None):
        f = self.fields[idx]
        for k, val in (("phi", phi), ("u", u), ("v", v), ("p", p)):
            if val is not None:
                f[k].copy_(torch.as_tensor(np.asarray(val, dtype=np.float64)))
        torch.cuda.synchronize(self.device)

    def close(self):
        if getattr(self, "ctx", None) is not None and self.ctx.value:
            self.lib.cdi_destroy(self.ctx)
            self.ctx = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def split_by_size(cells: Sequence[int], groups: int) -> List[List[int]]:
    """Instance indices split into `groups` lists of nearly equal total size:
    largest first, dealt out in a snake order (0, 1, .., G-1, G-1, .., 0, ..)."""
    order = sorted(range(len(cells)), key=lambda k: (-cells[k], k))
    out: List[List[int]] = [[] for _ in range(groups)]
    for r, k in enumerate(order):
        g = r % groups
        out[g if (r // groups) % 2 == 0 else groups - 1 - g].append(k)
    return [sorted(g) for g in out if g]


class EnsembleSolver:
    """A batch of independent instances split into `groups` contexts of
    nearly equal size, each on its own stream, advanced together
    (cdi_step_concurrent): while one context waits on its latency-bound
    phases (the one-block coarse cycle, the host's convergence test) the
    other's kernels fill the compute units.  Every instance evolves exactly
    as it does alone (the instances of a batch never interact).

    Arguments as CDISolver (lists of parameter objects and phase fields);
    instance k of the argument lists keeps index k in diagnostics / state.
    groups: 4 by default, the fastest measured on the 64-instance ensemble
    (more contexts mean more, smaller launches per step: 6 to 16 contexts were
    slower, also with 8 or 16 hardware queues per process).
    """

    def __init__(self, params, phi0, groups: int = 4, device: str = "cuda:0", u0=None, v0=None,
                 **kw):
        if not torch.cuda.is_available():
            raise RuntimeError("EnsembleSolver needs a GPU (the HIP library has no CPU path)")
        params, phi0 = list(params), list(phi0)
        if len(params) != len(phi0):
            raise ValueError("one phase field per instance is required")
        if groups < 1:
            raise ValueError("groups must be >= 1")
        self.n = len(params)
        self.device = torch.device(device)
        self.lib = L.lib()
        self.groups = split_by_size([p.nx * p.ny for p in params], min(groups, self.n))
        self.where = {}
        self.streams = [torch.cuda.Stream(self.device) for _ in self.groups]
        self.solvers: List[CDISolver] = []
        for g, idx in enumerate(self.groups):
            with torch.cuda.stream(self.streams[g]):
                self.solvers.append(CDISolver(
                    [params[k] for k in idx], [phi0[k] for k in idx], device=device,
                    u0=None if u0 is None else [u0[k] for k in idx],
                    v0=None if v0 is None else [v0[k] for k in idx], **kw))
            for j, k in enumerate(idx):
                self.where[k] = (g, j)
        self._ctxs = (C.c_void_p * len(self.solvers))(*[s.ctx.value for s in self.solvers])

    def _live(self):
        if not self.solvers:
            raise RuntimeError("EnsembleSolver is closed")

    def step(self, nsteps: int = 1, allow_noconv: bool = False) -> int:
        self._live()
        return L.check(self.lib.cdi_step_concurrent(self._ctxs, len(self.solvers), int(nsteps)),
                       allow=(-4,) if allow_noconv else ())

    def tune(self, trial_steps: int = 10) -> Dict:
        """One tiled shape for all contexts, timed with every context
        stepping at once (cdi_tune_concurrent); the state is restored."""
        self._live()
        n = len(self.solvers)
        nbytes = [self.lib.cdi_tune_bytes(s.ctx) for s in self.solvers]
        bufs = [torch.empty(b + 256, dtype=torch.uint8, device=self.device) for b in nbytes]
        ptrs = (C.c_void_p * n)(*[t.data_ptr() + (-t.data_ptr()) % 256 for t in bufs])
        sizes = (C.c_size_t * n)(*nbytes)
        info = L.cdi_tune_info()
        torch.cuda.synchronize(self.device)
        L.check(self.lib.cdi_tune_concurrent(self._ctxs, n, int(trial_steps), ptrs, sizes,
                                             C.byref(info)))
        torch.cuda.synchronize(self.device)
        del bufs
        ms = {}
        for v, nu in enumerate((1, 2)):
            for r, rows in enumerate((1, 4)):
                for q, cc in enumerate((1024, 4096, 16384)):
                    ms[f"tiled_nu{nu}_rows{rows}_coarse{cc}"] = info.ms_per_step[v * 6 + r * 3 + q]
        return dict(launch="tiled", tile_rows=info.tile_rows, coarse_cells=info.coarse_cells,
                    mg_smooth=info.mg_smooth, strip_rows=info.strip_rows, ms_per_step=ms)

    def diagnostics(self, idx: int = 0) -> Dict[str, float]:
        g, j = self.where[idx]
        return self.solvers[g].diagnostics(j)

    def cg_iterations(self) -> List[int]:
        """CG iterations of every instance (argument order) since set-up."""
        per = [s.cg_iterations() for s in self.solvers]
        return [per[self.where[k][0]][self.where[k][1]] for k in range(self.n)]

    def state(self, idx: int = 0):
        g, j = self.where[idx]
        return self.solvers[g].state(j)

    def set_state(self, idx: int, **fields):
        g, j = self.where[idx]
        self.solvers[g].set_state(j, **fields)

    def close(self):
        for s in getattr(self, "solvers", []):
            s.close()
        self.solvers = []
        self._ctxs = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
