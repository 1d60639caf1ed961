"""ctypes binding of libcdi.so (include/cdi.h): argument marshalling only.

Every step of the CDI + GNBC time step runs in the HIP kernels of the
library; this module converts Python values into the C structs and checks
return codes.  It fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcdi.so")

CDI_ABI_VERSION = 3
STATUS = {0: "CDI_OK", -1: "CDI_ERR_ARG", -2: "CDI_ERR_SHAPE", -3: "CDI_ERR_DEVICE",
          -4: "CDI_ERR_NOCONV", -5: "CDI_ERR_NONFINITE", -6: "CDI_ERR_STATE"}
SLIP = {"1A": 0, "1B": 1, "2A": 2, "2B": 3, "3A": 4, "3B": 5, "4A": 6, "4B": 7}
CDI_FP64, CDI_MIXED = 0, 1
GUESS = {"zero": 0, "prev": 1, "learned": 2}
LAUNCH = {"tiled": 0, "persistent": 1, "graph": 2}

EXPORTS = ("cdi_workspace_bytes", "cdi_default_dt", "cdi_init", "cdi_init_batch", "cdi_step",
           "cdi_solve_pressure", "cdi_diagnostics", "cdi_eval_rhs", "cdi_timing_enable",
           "cdi_timing_read", "cdi_destroy", "cdi_last_error", "cdi_net_param_count",
           "cdi_net_workspace_bytes", "cdi_net_init", "cdi_net_repack", "cdi_net_forward",
           "cdi_net_backward", "cdi_net_adam", "cdi_net_destroy", "cdi_net_last_error",
           "cdi_set_guess", "cdi_guess_attach", "cdi_guess_features", "cdi_set_launch",
           "cdi_get_launch", "cdi_set_tile_rows", "cdi_get_tile_rows", "cdi_tune_bytes",
           "cdi_tune", "cdi_graph_stats", "cdi_set_coarse_cells", "cdi_get_coarse_cells",
           "cdi_set_mg_smooth", "cdi_get_mg_smooth", "cdi_set_extrapolation",
           "cdi_get_extrapolation", "cdi_eval_rhs_noalloc", "cdi_set_strip_rows",
           "cdi_get_strip_rows", "cdi_step_concurrent",
           "cdi_tune_concurrent", "cdi_cg_iterations")
EXPORTS3 = ("cdi3_workspace_bytes", "cdi3_init", "cdi3_step", "cdi3_eval_rhs", "cdi3_kappa_p",
            "cdi3_diagnostics", "cdi3_time_stage", "cdi3_destroy")


class cdi_params(C.Structure):
    _fields_ = [("abi_version", C.c_int32), ("nx", C.c_int32), ("ny", C.c_int32),
                ("lx", C.c_double), ("ly", C.c_double), ("eps", C.c_double),
                ("gamma", C.c_double), ("sigma", C.c_double), ("theta_eq", C.c_double),
                ("rho1", C.c_double), ("rho2", C.c_double), ("mu1", C.c_double),
                ("mu2", C.c_double), ("beta1", C.c_double), ("beta2", C.c_double),
                ("u_wall_bot", C.c_double), ("u_wall_top", C.c_double), ("dt", C.c_double),
                ("cfl", C.c_double), ("slip_model", C.c_int32), ("precision", C.c_int32),
                ("guess", C.c_int32), ("poisson_rtol", C.c_double),
                ("poisson_maxit", C.c_int32), ("mg_smooth", C.c_int32),
                ("gamma_factor", C.c_double)]


class cdi_fields(C.Structure):
    _fields_ = [("phi", C.c_void_p), ("u", C.c_void_p), ("v", C.c_void_p), ("p", C.c_void_p)]


class cdi_solve_info(C.Structure):
    _fields_ = [("iterations", C.c_int32), ("converged", C.c_int32), ("guess_used", C.c_int32),
                ("pad", C.c_int32), ("relres", C.c_double), ("bnorm", C.c_double),
                ("ms", C.c_double)]


class cdi_diag(C.Structure):
    _fields_ = [("t", C.c_double), ("step", C.c_int64), ("mass", C.c_double),
                ("mass0", C.c_double), ("phi_min", C.c_double), ("phi_max", C.c_double),
                ("max_div", C.c_double), ("max_uslip", C.c_double * 2),
                ("max_uY", C.c_double * 2), ("ke", C.c_double), ("last_iters", C.c_int32),
                ("nonfinite", C.c_int32), ("last_relres", C.c_double),
                ("n_contact", C.c_int32 * 2), ("contact_x", C.c_double * 4),
                ("wetted_len", C.c_double * 2), ("theta_est", C.c_double * 2)]


class cdi_tune_info(C.Structure):
    _fields_ = [("launch", C.c_int32), ("tile_rows", C.c_int32), ("coarse_cells", C.c_int32),
                ("mg_smooth", C.c_int32), ("ncand", C.c_int32), ("strip_rows", C.c_int32),
                ("ms_per_step", C.c_double * 14)]


class CDIError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class cdi3_params(C.Structure):
    _fields_ = [("base", cdi_params), ("nz", C.c_int32), ("pad", C.c_int32), ("lz", C.c_double),
                ("w_wall_bot", C.c_double), ("w_wall_top", C.c_double)]


class cdi3_fields(C.Structure):
    _fields_ = [("phi", C.c_void_p), ("u", C.c_void_p), ("v", C.c_void_p), ("w", C.c_void_p),
                ("p", C.c_void_p)]


class cdi3_diag(C.Structure):
    _fields_ = [("t", C.c_double), ("step", C.c_int64), ("mass", C.c_double),
                ("phi_min", C.c_double), ("phi_max", C.c_double), ("max_div", C.c_double),
                ("max_slip", C.c_double * 2), ("max_uY", C.c_double * 2), ("ke", C.c_double),
                ("last_iters", C.c_int32), ("pad", C.c_int32), ("last_relres", C.c_double)]


_lib = None


def lib() -> C.CDLL:
    """Load libcdi.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} not found: build it with "
                           "`python -m paper_2412_16843_amd.build` (or __graft_entry__.build())")
    L = C.CDLL(LIB_PATH)
    vp, i32, f64 = C.c_void_p, C.c_int32, C.c_double
    P = C.POINTER
    L.cdi_workspace_bytes.argtypes = [P(cdi_params), i32]
    L.cdi_workspace_bytes.restype = C.c_size_t
    L.cdi_default_dt.argtypes = [P(cdi_params)]
    L.cdi_default_dt.restype = f64
    L.cdi_init.argtypes = [P(cdi_params), P(cdi_fields), vp, C.c_size_t, vp, P(vp)]
    L.cdi_init.restype = i32
    L.cdi_init_batch.argtypes = [P(cdi_params), i32, P(cdi_fields), vp, C.c_size_t, vp, P(vp)]
    L.cdi_init_batch.restype = i32
    L.cdi_step.argtypes = [vp, i32]
    L.cdi_step.restype = i32
    L.cdi_step_concurrent.argtypes = [P(vp), i32, i32]
    L.cdi_step_concurrent.restype = i32
    L.cdi_solve_pressure.argtypes = [vp, vp, vp, P(cdi_solve_info)]
    L.cdi_solve_pressure.restype = i32
    L.cdi_diagnostics.argtypes = [vp, i32, P(cdi_diag)]
    L.cdi_diagnostics.restype = i32
    L.cdi_eval_rhs.argtypes = [vp, vp, vp, vp, vp, vp]
    L.cdi_eval_rhs.restype = i32
    L.cdi_eval_rhs_noalloc.argtypes = [P(cdi_params), P(cdi_fields), vp, vp, vp, vp, vp, vp]
    L.cdi_eval_rhs_noalloc.restype = i32
    L.cdi_timing_enable.argtypes = [vp, C.c_char_p]
    L.cdi_timing_enable.restype = i32
    L.cdi_timing_read.argtypes = [vp, P(f64), P(C.c_int64)]
    L.cdi_timing_read.restype = i32
    L.cdi_net_param_count.argtypes = []
    L.cdi_net_param_count.restype = C.c_size_t
    L.cdi_net_workspace_bytes.argtypes = [i32, i32, i32, i32]
    L.cdi_net_workspace_bytes.restype = C.c_size_t
    L.cdi_net_init.argtypes = [vp, vp, i32, i32, i32, i32, vp, C.c_size_t, vp, P(vp)]
    L.cdi_net_init.restype = i32
    L.cdi_net_repack.argtypes = [vp]
    L.cdi_net_repack.restype = i32
    L.cdi_net_forward.argtypes = [vp, vp, vp]
    L.cdi_net_forward.restype = i32
    L.cdi_net_backward.argtypes = [vp, vp, vp]
    L.cdi_net_backward.restype = i32
    L.cdi_net_adam.argtypes = [vp, vp, vp, i32, f64]
    L.cdi_net_adam.restype = i32
    L.cdi_net_destroy.argtypes = [vp]
    L.cdi_net_destroy.restype = None
    L.cdi_net_last_error.argtypes = []
    L.cdi_net_last_error.restype = C.c_char_p
    L.cdi_set_guess.argtypes = [vp, i32]
    L.cdi_set_guess.restype = i32
    L.cdi_guess_attach.argtypes = [vp, vp]
    L.cdi_guess_attach.restype = i32
    L.cdi_guess_features.argtypes = [vp, i32, vp, vp]
    L.cdi_guess_features.restype = i32
    L.cdi_set_launch.argtypes = [vp, i32]
    L.cdi_set_launch.restype = i32
    L.cdi_get_launch.argtypes = [vp, P(i32)]
    L.cdi_get_launch.restype = i32
    L.cdi_set_strip_rows.argtypes = [vp, i32]
    L.cdi_set_strip_rows.restype = i32
    L.cdi_get_strip_rows.argtypes = [vp, P(i32)]
    L.cdi_get_strip_rows.restype = i32
    L.cdi_set_tile_rows.argtypes = [vp, i32]
    L.cdi_set_tile_rows.restype = i32
    L.cdi_get_tile_rows.argtypes = [vp, P(i32)]
    L.cdi_get_tile_rows.restype = i32
    L.cdi_set_coarse_cells.argtypes = [vp, i32]
    L.cdi_set_coarse_cells.restype = i32
    L.cdi_get_coarse_cells.argtypes = [vp, P(i32)]
    L.cdi_get_coarse_cells.restype = i32
    L.cdi_set_mg_smooth.argtypes = [vp, i32]
    L.cdi_set_mg_smooth.restype = i32
    L.cdi_get_mg_smooth.argtypes = [vp, P(i32)]
    L.cdi_get_mg_smooth.restype = i32
    L.cdi_set_extrapolation.argtypes = [vp, i32]
    L.cdi_set_extrapolation.restype = i32
    L.cdi_get_extrapolation.argtypes = [vp, P(i32)]
    L.cdi_get_extrapolation.restype = i32
    L.cdi_graph_stats.argtypes = [vp, P(C.c_int64), P(C.c_int64), P(i32)]
    L.cdi_graph_stats.restype = i32
    L.cdi_tune_bytes.argtypes = [vp]
    L.cdi_tune_bytes.restype = C.c_size_t
    L.cdi_tune.argtypes = [vp, i32, vp, C.c_size_t, P(cdi_tune_info)]
    L.cdi_tune.restype = i32
    L.cdi_tune_concurrent.argtypes = [P(vp), i32, i32, P(vp), P(C.c_size_t), P(cdi_tune_info)]
    L.cdi_tune_concurrent.restype = i32
    L.cdi_cg_iterations.argtypes = [vp, P(C.c_int64)]
    L.cdi_cg_iterations.restype = i32
    L.cdi_destroy.argtypes = [vp]
    L.cdi_destroy.restype = None
    L.cdi_last_error.argtypes = []
    L.cdi_last_error.restype = C.c_char_p
    L.cdi3_workspace_bytes.argtypes = [P(cdi3_params), P(C.c_size_t)]
    L.cdi3_workspace_bytes.restype = i32
    L.cdi3_init.argtypes = [P(cdi3_params), P(cdi3_fields), vp, C.c_size_t, vp, P(vp)]
    L.cdi3_init.restype = i32
    L.cdi3_step.argtypes = [vp, i32]
    L.cdi3_step.restype = i32
    L.cdi3_eval_rhs.argtypes = [vp, vp, vp, vp, vp, vp, vp]
    L.cdi3_eval_rhs.restype = i32
    L.cdi3_kappa_p.argtypes = [vp, vp]
    L.cdi3_kappa_p.restype = i32
    L.cdi3_diagnostics.argtypes = [vp, P(cdi3_diag)]
    L.cdi3_diagnostics.restype = i32
    L.cdi3_time_stage.argtypes = [vp, i32, P(f64)]
    L.cdi3_time_stage.restype = i32
    L.cdi3_destroy.argtypes = [vp]
    L.cdi3_destroy.restype = None
    _lib = L
    return L


def check(status: int, allow=()) -> int:
    if status != 0 and status not in allow:
        raise CDIError(status, lib().cdi_last_error().decode())
    return status


def check_net(status: int) -> int:
    if status != 0:
        raise CDIError(status, lib().cdi_net_last_error().decode())
    return status


def make_params(p, precision: str = "fp64", guess: str = "prev", rtol: float = 0.0,
                maxit: int = 0, mg_smooth: int = 0) -> cdi_params:
    """Marshal a parameter object (attributes as in workloads.Params)."""
    return cdi_params(
        abi_version=CDI_ABI_VERSION, nx=p.nx, ny=p.ny, lx=p.lx, ly=p.ly, eps=p.eps,
        gamma=p.gamma, sigma=p.sigma, theta_eq=p.theta_eq, rho1=p.rho1, rho2=p.rho2,
        mu1=p.mu1, mu2=p.mu2, beta1=p.beta1, beta2=p.beta2, u_wall_bot=p.u_wall_bot,
        u_wall_top=p.u_wall_top, dt=p.dt, cfl=0.0, slip_model=SLIP[p.slip_model],
        precision=CDI_MIXED if precision == "mixed" else CDI_FP64, guess=GUESS[guess],
        poisson_rtol=rtol, poisson_maxit=maxit, mg_smooth=mg_smooth,
        gamma_factor=getattr(p, "gamma_factor", 0.0))


def make_params3(p, guess: str = "prev", rtol: float = 0.0, maxit: int = 0,
                 mg_smooth: int = 0) -> cdi3_params:
    """Marshal a 3-D parameter object (attributes as in workloads.Params3)."""
    return cdi3_params(base=make_params(p, guess=guess, rtol=rtol, maxit=maxit,
                                        mg_smooth=mg_smooth), nz=p.nz, pad=0,
                       lz=p.lz, w_wall_bot=getattr(p, "w_wall_bot", 0.0),
                       w_wall_top=getattr(p, "w_wall_top", 0.0))
