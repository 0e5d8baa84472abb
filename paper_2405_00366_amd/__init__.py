"""MI355X (gfx950) MF-CIM solver for L0-regularised compressed sensing.

Thin Python binding of ``libl0cim.so`` (C ABI declared in include/l0cim.h).
Every function has the name of the C entry point it calls and only marshals
arguments: torch tensors supply device memory and the HIP stream, and all
computation runs in the library's HIP kernels.  Importing works without a
GPU; calling anything that launches work requires the built library and a
visible device, and raises otherwise (there is no CPU fallback).
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_char_p, c_double, c_int, c_int32, c_int64, c_size_t, c_uint64, c_void_p

import torch

__all__ = [
    "F32", "F64", "BF16", "FP8E4M3", "FIELD_CN", "FIELD_BN", "CDP_JACOBI", "CDP_CHOL_F64",
    "CimParams", "SolveParams", "Stats", "L0cimError", "lib", "library_path",
    "l0cim_version", "l0cim_gram", "l0cim_build_couplings", "l0cim_init_r", "l0cim_init_state", "l0cim_mri_mfcim_run",
    "l0cim_mfcim_run", "l0cim_select_replica", "l0cim_update_r", "l0cim_solve",
    "l0cim_mfcim_run_workspace_bytes", "l0cim_update_r_workspace_bytes",
    "l0cim_solve_workspace_bytes", "l0cim_profile_begin", "l0cim_profile_end",
    "cim_params", "solve_params", "Instance", "l0cim_batch_plan_create", "l0cim_batch_plan_workspace_bytes",
    "l0cim_batch_plan_info", "l0cim_batch_plan_destroy", "l0cim_solve_batched", "pack_instances",
    "l0cim_batch_begin", "l0cim_batch_alternations", "l0cim_batch_finish",
    "Completion", "l0cim_server_request_bytes", "l0cim_server_arena_overhead", "l0cim_server_create",
    "l0cim_server_clock", "l0cim_server_submit", "l0cim_server_step", "l0cim_server_completed",
    "l0cim_server_info", "l0cim_server_destroy", "l0cim_server_set_step_budget",
    "l0cim_solve_many", "l0cim_solve_many_workspace_bytes", "l0cim_refit_f64", "l0cim_mfcim_run_noalloc",
    "l0cim_cac_run", "l0cim_cac_solve", "cac_params", "mri_params", "l0cim_mri_solve", "l0cim_mri_solve_many",
]

F32, F64, BF16, FP8E4M3 = 0, 1, 2, 3
FIELD_CN, FIELD_BN = 0, 1
CDP_JACOBI, CDP_CHOL_F64, CDP_CG = 0, 1, 2
LAUNCH_AUTO, LAUNCH_RESIDENT, LAUNCH_STREAMED, LAUNCH_MATRIX = 0, 1, 2, 3

ST_NONFINITE, ST_BLOWUP, ST_CHOL_RIDGE, ST_TINY_DIAG, ST_TIMEOUT = 1, 2, 4, 8, 16
SOLVE_NO_GRAPH = 1

_HERE = os.path.dirname(os.path.abspath(__file__))
library_path = os.path.join(_HERE, "libl0cim.so")


class CimParams(ctypes.Structure):
    _fields_ = [
        ("dt", c_double), ("n_steps", c_int32), ("field", c_int32),
        ("p_thr", c_double), ("d", c_double), ("t_c", c_double), ("t_w", c_double),
        ("K", c_double), ("j", c_double), ("beta", c_double), ("tau", c_double),
        ("c0_std", c_double), ("linear_j", c_int32), ("launch", c_int32),
        ("spin_limit", c_int64),
    ]


class SolveParams(ctypes.Structure):
    _fields_ = [
        ("eta_init", c_double), ("eta_end", c_double), ("velo", c_int32), ("n_outer", c_int32),
        ("cdp", c_int32), ("cdp_iters", c_int32), ("dtc", c_double),
        ("final_refit_f64", c_int32), ("replicas", c_int32), ("seed", c_uint64),
        ("j_dtype", c_int32), ("flags", c_int32),
    ]


class CacParams(ctypes.Structure):
    _fields_ = [("dt", c_double), ("n_steps", c_int32), ("p_thr", c_double), ("d", c_double), ("t_c", c_double),
                ("t_w", c_double), ("K", c_double), ("j", c_double), ("beta", c_double), ("tau", c_double),
                ("g2", c_double)]


class MriParams(ctypes.Structure):
    _fields_ = [("size", c_int32), ("levels", c_int32), ("gamma", c_double), ("lasso_iters", c_int32),
                ("lasso_lam1", c_double), ("cdp", c_int32), ("cg_max_iter", c_int32), ("cg_tol", c_double)]


class Stats(ctypes.Structure):
    _fields_ = [
        ("status_bits", c_int32), ("selected_replica", c_int32), ("support_size", c_int32),
        ("n_outer_done", c_int32), ("H", c_double), ("E", c_double), ("spin_steps", c_int64),
    ]


STATS_BYTES = ctypes.sizeof(Stats)


class Instance(ctypes.Structure):
    _fields_ = [
        ("m", c_int32), ("n", c_int32), ("a_offset", c_int64), ("lda", c_int64),
        ("y_offset", c_int64), ("x_offset", c_int64), ("seed", c_uint64),
    ]


class Completion(ctypes.Structure):
    _fields_ = [("tag", c_int64), ("n", c_int32), ("m", c_int32), ("t_submit", c_double),
                ("t_admit", c_double), ("t_finish", c_double)]


class L0cimError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str):
        super().__init__(f"{where}: status {status}: {detail}")
        self.status = status


_lib = None


def lib():
    """The loaded library (loaded on first use; raises if it was not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(library_path):
            raise L0cimError(-1, "load", f"{library_path} is missing: build it with "
                                         "python paper_2405_00366_amd/build.py")
        L = ctypes.CDLL(library_path)
        st = c_int
        vp = c_void_p
        L.l0cim_version.restype = c_int
        L.l0cim_status_string.restype = c_char_p
        L.l0cim_status_string.argtypes = [c_int]
        L.l0cim_last_error.restype = c_char_p
        L.l0cim_cim_params_default.argtypes = [POINTER(CimParams)]
        L.l0cim_cim_params_default.restype = None
        L.l0cim_solve_params_default.argtypes = [POINTER(SolveParams)]
        L.l0cim_solve_params_default.restype = None
        L.l0cim_gram.argtypes = [c_int, c_int32, c_int32, vp, c_int64, vp, vp, c_int64, vp, vp]
        L.l0cim_gram.restype = st
        L.l0cim_build_couplings.argtypes = [c_int, c_int32, vp, c_int64, vp, vp, c_int, vp, c_int64,
                                            vp, vp, vp]
        L.l0cim_build_couplings.restype = st
        L.l0cim_init_r.argtypes = [c_int, c_int32, vp, c_int64, vp, vp, vp, vp, vp]
        L.l0cim_init_r.restype = st
        L.l0cim_init_state.argtypes = [c_int, c_int32, c_int32, c_uint64, c_int32, c_double, vp, vp, vp]
        L.l0cim_init_state.restype = st
        L.l0cim_mfcim_run_workspace_bytes.argtypes = [c_int, c_int32, c_int32, c_int]
        L.l0cim_mfcim_run_workspace_bytes.restype = c_size_t
        L.l0cim_mfcim_run.argtypes = [c_int, c_int32, c_int32, c_int, vp, c_int64, vp, vp, c_double,
                                      POINTER(CimParams), vp, vp, vp, vp, vp, c_int32, vp, vp,
                                      c_size_t, vp]
        L.l0cim_mfcim_run.restype = st
        L.l0cim_noalloc_scratch_bytes.argtypes = []
        L.l0cim_noalloc_scratch_bytes.restype = c_size_t
        L.l0cim_mfcim_run_noalloc.argtypes = [c_int, c_int32, c_int32, c_int, vp, c_int64, vp, vp, c_double,
                                              POINTER(CimParams), vp, vp, vp, vp, vp, c_int32, vp, vp]
        L.l0cim_mfcim_run_noalloc.restype = st
        L.l0cim_mri_mfcim_run.argtypes = [c_int32, c_int32, c_int32, vp, vp, vp, c_int64, vp, c_double, c_double,
                                          POINTER(CimParams), vp, vp, vp, vp, vp, c_int32, vp, vp]
        L.l0cim_mri_mfcim_run.restype = st
        L.l0cim_mri_l2_diag.argtypes = [c_int32, c_int32, c_double, vp, c_int64, vp, vp]
        L.l0cim_mri_l2_diag.restype = st
        L.l0cim_mri_lasso.argtypes = [c_int32, c_int32, c_double, vp, vp, c_double, c_int32, vp, vp]
        L.l0cim_mri_lasso.restype = st
        L.l0cim_mri_update_r.argtypes = [c_int32, c_int32, c_double, vp, vp, c_int64, vp, vp, c_int, c_double,
                                         c_int32, c_int32, c_double, vp, vp, vp, vp]
        L.l0cim_mri_update_r.restype = st
        L.l0cim_mri_params_default.argtypes = [POINTER(MriParams)]
        L.l0cim_mri_params_default.restype = None
        L.l0cim_mri_solve_workspace_bytes.argtypes = [c_int32, c_int32, c_int32]
        L.l0cim_mri_solve_workspace_bytes.restype = c_size_t
        L.l0cim_mri_solve.argtypes = [POINTER(MriParams), c_int32, vp, c_int64, vp, vp, POINTER(CimParams),
                                      POINTER(SolveParams), vp, vp, vp, vp, c_size_t, vp]
        L.l0cim_mri_solve.restype = st
        L.l0cim_mri_solve_many_workspace_bytes.argtypes = [c_int32, c_int32, c_int32, c_int32]
        L.l0cim_mri_solve_many_workspace_bytes.restype = c_size_t
        L.l0cim_mri_solve_many.argtypes = [POINTER(MriParams), c_int32, c_int32, vp, c_int64, c_int64, vp, c_int64, vp,
                                           c_int64, vp, POINTER(CimParams), POINTER(SolveParams), vp, vp, vp, vp,
                                           c_size_t, vp]
        L.l0cim_mri_solve_many.restype = st
        L.l0cim_cac_params_default.argtypes = [POINTER(CacParams)]
        L.l0cim_cac_params_default.restype = None
        L.l0cim_cac_run_workspace_bytes.argtypes = [c_int, c_int32, c_int32]
        L.l0cim_cac_run_workspace_bytes.restype = c_size_t
        L.l0cim_cac_run.argtypes = [c_int, c_int32, c_int32, vp, c_int64, vp, c_double, POINTER(CacParams), c_uint64,
                                    c_int32, vp, vp, vp, vp, vp, vp, vp, c_int32, vp, vp, c_size_t, vp]
        L.l0cim_cac_run.restype = st
        L.l0cim_cac_solve_workspace_bytes.argtypes = [c_int, c_int32, c_int32, c_int32]
        L.l0cim_cac_solve_workspace_bytes.restype = c_size_t
        L.l0cim_cac_solve.argtypes = [c_int, c_int32, c_int32, vp, c_int64, vp, POINTER(CacParams),
                                      POINTER(SolveParams), vp, vp, vp, vp, c_size_t, vp]
        L.l0cim_cac_solve.restype = st
        L.l0cim_select_replica.argtypes = [c_int32, c_int32, vp, vp, vp, vp, vp]
        L.l0cim_select_replica.restype = st
        L.l0cim_update_r_workspace_bytes.argtypes = [c_int, c_int32, c_int]
        L.l0cim_update_r_workspace_bytes.restype = c_size_t
        L.l0cim_update_r.argtypes = [c_int, c_int32, vp, c_int64, vp, vp, c_int, c_double, c_int32,
                                     vp, vp, vp, c_size_t, vp]
        L.l0cim_update_r.restype = st
        L.l0cim_solve_many_workspace_bytes.argtypes = [c_int, c_int32, c_int32, c_int32, POINTER(SolveParams)]
        L.l0cim_solve_many_workspace_bytes.restype = c_size_t
        L.l0cim_solve_many.argtypes = [c_int, c_int32, c_int32, c_int32, vp, c_int64, c_int64, vp, c_int64, vp,
                                       POINTER(CimParams), POINTER(SolveParams), vp, vp, vp, vp, c_size_t, vp]
        L.l0cim_solve_many.restype = st
        L.l0cim_refit_f64_workspace_bytes.argtypes = [c_int32, c_int32]
        L.l0cim_refit_f64_workspace_bytes.restype = c_size_t
        L.l0cim_refit_f64.argtypes = [c_int, c_int32, c_int32, vp, c_int64, vp, vp, vp, vp, vp, c_size_t, vp]
        L.l0cim_refit_f64.restype = st
        L.l0cim_solve_workspace_bytes.argtypes = [c_int, c_int32, c_int32, POINTER(CimParams),
                                                  POINTER(SolveParams)]
        L.l0cim_solve_workspace_bytes.restype = c_size_t
        L.l0cim_solve.argtypes = [c_int, c_int32, c_int32, vp, c_int64, vp, vp, POINTER(CimParams),
                                  POINTER(SolveParams), vp, vp, vp, vp, c_size_t, vp]
        L.l0cim_solve.restype = st
        L.l0cim_batch_plan_create.argtypes = [c_int32, POINTER(Instance), POINTER(CimParams),
                                              POINTER(SolveParams), POINTER(c_void_p)]
        L.l0cim_batch_plan_create.restype = st
        L.l0cim_batch_plan_workspace_bytes.argtypes = [c_void_p]
        L.l0cim_batch_plan_workspace_bytes.restype = c_size_t
        L.l0cim_batch_plan_info.argtypes = [c_void_p, POINTER(c_int32), POINTER(c_int32), POINTER(c_int32)]
        L.l0cim_batch_plan_info.restype = st
        L.l0cim_batch_plan_destroy.argtypes = [c_void_p]
        L.l0cim_batch_plan_destroy.restype = st
        L.l0cim_solve_batched.argtypes = [c_void_p, vp, vp, vp, vp, vp, vp, c_size_t, vp]
        L.l0cim_solve_batched.restype = st
        L.l0cim_batch_begin.argtypes = [c_void_p, vp, vp, vp, vp, vp, vp, c_size_t, vp]
        L.l0cim_batch_begin.restype = st
        L.l0cim_batch_alternations.argtypes = [c_void_p, c_int32, c_int32, vp, vp, vp, vp, vp, vp, c_size_t, vp]
        L.l0cim_batch_alternations.restype = st
        L.l0cim_batch_finish.argtypes = [c_void_p, vp, vp, vp, vp, vp, vp, c_size_t, vp]
        L.l0cim_batch_finish.restype = st
        L.l0cim_server_request_bytes.argtypes = [c_int32, c_int32, POINTER(SolveParams)]
        L.l0cim_server_request_bytes.restype = c_size_t
        L.l0cim_server_arena_overhead.argtypes = [c_int32, c_int32, POINTER(SolveParams)]
        L.l0cim_server_arena_overhead.restype = c_size_t
        L.l0cim_server_sim_create.argtypes = [POINTER(SolveParams), c_int32, c_int32, c_size_t, POINTER(c_void_p)]
        L.l0cim_server_sim_create.restype = st
        L.l0cim_server_sim_submit.argtypes = [c_void_p, c_int32, c_int32, c_int64, c_double]
        L.l0cim_server_sim_submit.restype = st
        L.l0cim_server_sim_set_step_budget.argtypes = [c_void_p, c_size_t]
        L.l0cim_server_sim_set_step_budget.restype = st
        L.l0cim_server_sim_tick.argtypes = [c_void_p, c_double, c_double, POINTER(c_int32), POINTER(c_int32)]
        L.l0cim_server_sim_tick.restype = st
        L.l0cim_server_sim_completed.argtypes = [c_void_p, POINTER(Completion), c_int32]
        L.l0cim_server_sim_completed.restype = c_int32
        L.l0cim_server_sim_resident.argtypes = [c_void_p, POINTER(c_int64), POINTER(c_int32), POINTER(c_size_t),
                                                POINTER(c_int32), c_int32]
        L.l0cim_server_sim_resident.restype = c_int32
        L.l0cim_server_sim_info.argtypes = [c_void_p, POINTER(c_int32), POINTER(c_int32), POINTER(c_size_t),
                                            POINTER(c_size_t), POINTER(c_int32)]
        L.l0cim_server_sim_info.restype = st
        L.l0cim_server_sim_destroy.argtypes = [c_void_p]
        L.l0cim_server_sim_destroy.restype = st
        L.l0cim_server_create.argtypes = [POINTER(CimParams), POINTER(SolveParams), c_int32, c_int32, vp,
                                          c_size_t, vp, POINTER(c_void_p)]
        L.l0cim_server_create.restype = st
        L.l0cim_server_clock.argtypes = [c_void_p]
        L.l0cim_server_clock.restype = c_double
        L.l0cim_server_submit.argtypes = [c_void_p, c_int32, c_int32, vp, c_int64, vp, c_uint64, c_int64, vp, vp,
                                          vp]
        L.l0cim_server_submit.restype = st
        L.l0cim_server_set_step_budget.argtypes = [c_void_p, c_size_t]
        L.l0cim_server_set_step_budget.restype = st
        L.l0cim_server_step.argtypes = [c_void_p, POINTER(c_int32)]
        L.l0cim_server_step.restype = st
        L.l0cim_server_completed.argtypes = [c_void_p, POINTER(Completion), c_int32]
        L.l0cim_server_completed.restype = c_int32
        L.l0cim_server_info.argtypes = [c_void_p, POINTER(c_int32), POINTER(c_int32), POINTER(c_size_t),
                                        POINTER(c_size_t), POINTER(c_int64)]
        L.l0cim_server_info.restype = st
        L.l0cim_server_destroy.argtypes = [c_void_p]
        L.l0cim_server_destroy.restype = st
        L.l0cim_matrix_tile_get.argtypes = [c_int32, c_int32, c_int32, c_int32, POINTER(c_int32)]
        L.l0cim_matrix_tile_get.restype = st
        L.l0cim_matrix_tile_set.argtypes = [c_int32, c_int32, c_int32, c_int32, c_int32]
        L.l0cim_matrix_tile_set.restype = st
        L.l0cim_profile_begin.restype = st
        L.l0cim_profile_end.argtypes = [POINTER(c_double), POINTER(c_int64)]
        L.l0cim_profile_end.restype = st
        _lib = L
    return _lib


def _check(status: int, where: str):
    if status != 0:
        L = lib()
        raise L0cimError(status, where, L.l0cim_last_error().decode())


def _ptr(t):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("tensor must live on the GPU")
    return c_void_p(t.data_ptr())


def _dtype_code(t) -> int:
    if t.dtype == torch.float32:
        return F32
    if t.dtype == torch.float64:
        return F64
    raise ValueError(f"unsupported arithmetic dtype {t.dtype}")


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return c_void_p(stream.cuda_stream)


def _ld(t) -> int:
    if t.dim() != 2 or t.stride(1) != 1:
        raise ValueError("matrix must be 2-D with unit column stride")
    return t.stride(0)


def _torch_jdtype(code: int):
    return {F32: torch.float32, F64: torch.float64, BF16: torch.bfloat16,
            FP8E4M3: torch.float8_e4m3fn}[code]


def workspace(nbytes: int, device=None):
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device or "cuda")


def cim_params(**kw) -> CimParams:
    """Paper defaults (random data) with keyword overrides."""
    p = CimParams()
    lib().l0cim_cim_params_default(ctypes.byref(p))
    for k, v in kw.items():
        if k == "field" and isinstance(v, str):
            v = FIELD_BN if v.upper() == "BN" else FIELD_CN
        setattr(p, k, v)
    return p


def solve_params(**kw) -> SolveParams:
    p = SolveParams()
    lib().l0cim_solve_params_default(ctypes.byref(p))
    for k, v in kw.items():
        setattr(p, k, v)
    return p


# ---------------------------------------------------------------------------
# Entry points (same names as the C ABI)
# ---------------------------------------------------------------------------

def l0cim_version() -> int:
    return lib().l0cim_version()


def l0cim_gram(A, y, G=None, b=None, stream=None):
    m, n = A.shape
    dt = _dtype_code(A)
    G = torch.empty((n, n), dtype=A.dtype, device=A.device) if G is None else G
    b = torch.empty(n, dtype=A.dtype, device=A.device) if b is None else b
    _check(lib().l0cim_gram(dt, m, n, _ptr(A), _ld(A), _ptr(y), _ptr(G), _ld(G), _ptr(b),
                            _stream(stream)), "l0cim_gram")
    return G, b


def l0cim_build_couplings(G, b, R, j_dtype: int = None, J=None, row_scale=None, z=None, stream=None):
    n = G.shape[0]
    dt = _dtype_code(G)
    if j_dtype is None:
        j_dtype = dt
    J = torch.empty((n, n), dtype=_torch_jdtype(j_dtype), device=G.device) if J is None else J
    if j_dtype in (BF16, FP8E4M3) and row_scale is None:
        row_scale = torch.empty(n, dtype=torch.float32, device=G.device)
    z = torch.empty(n, dtype=G.dtype, device=G.device) if z is None else z
    _check(lib().l0cim_build_couplings(dt, n, _ptr(G), _ld(G), _ptr(b), _ptr(R), j_dtype, _ptr(J),
                                       _ld(J), _ptr(row_scale), _ptr(z), _stream(stream)),
           "l0cim_build_couplings")
    return J, row_scale, z


def l0cim_init_r(G, b, R=None, D_out=None, status=None, stream=None):
    n = G.shape[0]
    R = torch.empty(n, dtype=G.dtype, device=G.device) if R is None else R
    _check(lib().l0cim_init_r(_dtype_code(G), n, _ptr(G), _ld(G), _ptr(b), _ptr(R), _ptr(D_out), _ptr(status),
                              _stream(stream)), "l0cim_init_r")
    return R


def l0cim_init_state(n: int, P: int, seed: int, alt: int, c0_std: float, c, e, stream=None):
    _check(lib().l0cim_init_state(_dtype_code(c), n, P, seed, alt, c0_std, _ptr(c), _ptr(e),
                                  _stream(stream)), "l0cim_init_state")
    return c, e


def l0cim_mfcim_run_workspace_bytes(dtype: int, n: int, P: int, j_dtype: int) -> int:
    return lib().l0cim_mfcim_run_workspace_bytes(dtype, n, P, j_dtype)


def l0cim_mfcim_run(J, z, eta: float, prm: CimParams, c, e, sigma=None, H=None, trace=None,
                    trace_steps: int = 0, row_scale=None, status=None, ws=None, j_dtype: int = None,
                    stream=None):
    P, n = c.shape
    dt = _dtype_code(c)
    if j_dtype is None:
        j_dtype = {torch.float32: F32, torch.float64: F64, torch.bfloat16: BF16,
                   torch.float8_e4m3fn: FP8E4M3}[J.dtype]
    sigma = torch.empty((P, n), dtype=torch.uint8, device=c.device) if sigma is None else sigma
    need = l0cim_mfcim_run_workspace_bytes(dt, n, P, j_dtype)
    ws = workspace(need, c.device) if ws is None else ws
    _check(lib().l0cim_mfcim_run(dt, n, P, j_dtype, _ptr(J), _ld(J), _ptr(row_scale), _ptr(z), eta,
                                 ctypes.byref(prm), _ptr(c), _ptr(e), _ptr(sigma), _ptr(H),
                                 _ptr(trace), trace_steps, _ptr(status), _ptr(ws), ws.numel(),
                                 _stream(stream)), "l0cim_mfcim_run")
    return sigma


def l0cim_mfcim_run_noalloc(J, z, eta: float, prm: CimParams, c, e, sigma, H=None, trace=None,
                            trace_steps: int = 0, row_scale=None, status=None, j_dtype: int = None, stream=None):
    """l0cim_mfcim_run on the library's own device scratch: nothing is
    allocated here or in the library (sigma is the caller's)."""
    P, n = c.shape
    dt = _dtype_code(c)
    if j_dtype is None:
        j_dtype = {torch.float32: F32, torch.float64: F64, torch.bfloat16: BF16,
                   torch.float8_e4m3fn: FP8E4M3}[J.dtype]
    _check(lib().l0cim_mfcim_run_noalloc(dt, n, P, j_dtype, _ptr(J), _ld(J), _ptr(row_scale), _ptr(z), eta,
                                         ctypes.byref(prm), _ptr(c), _ptr(e), _ptr(sigma), _ptr(H),
                                         _ptr(trace), trace_steps, _ptr(status), _stream(stream)),
           "l0cim_mfcim_run_noalloc")
    return sigma


def l0cim_mri_mfcim_run(size: int, levels: int, mask, R, D, b, eta: float, prm: CimParams, c, e, sigma=None,
                        H=None, trace=None, trace_steps: int = 0, status=None, stream=None, gamma: float = 0.0):
    """D: a vector of G_rr, or G itself (its diagonal is read in place)."""
    P = c.shape[0]
    sigma = torch.empty(c.shape, dtype=torch.uint8, device=c.device) if sigma is None else sigma
    incd = 1 if D.dim() == 1 else D.stride(0) + 1
    _check(lib().l0cim_mri_mfcim_run(size, levels, P, _ptr(mask), _ptr(R), _ptr(D), incd, _ptr(b), gamma, eta,
                                     ctypes.byref(prm), _ptr(c), _ptr(e), _ptr(sigma), _ptr(H), _ptr(trace),
                                     trace_steps, _ptr(status), _stream(stream)), "l0cim_mri_mfcim_run")
    return sigma


def l0cim_mri_l2_diag(size: int, levels: int, gamma: float, D_in, D_out, stream=None):
    incd = D_in.stride(0)
    _check(lib().l0cim_mri_l2_diag(size, levels, gamma, _ptr(D_in), incd, _ptr(D_out), _stream(stream)),
           "l0cim_mri_l2_diag")
    return D_out


def l0cim_mri_lasso(size: int, levels: int, gamma: float, mask, b, lam1: float, iters: int, R_out, stream=None):
    _check(lib().l0cim_mri_lasso(size, levels, gamma, _ptr(mask), _ptr(b), lam1, iters, _ptr(R_out),
                                 _stream(stream)), "l0cim_mri_lasso")
    return R_out


def l0cim_mri_update_r(size: int, levels: int, gamma: float, mask, D, b, sigma, R, cdp: int = CDP_JACOBI,
                       dtc: float = 0.1, iters: int = 100, cg_max_iter: int = 10000, cg_tol: float = 1e-5,
                       iters_out=None, status=None, stream=None):
    incd = 1 if D.dim() == 1 else D.stride(0) + 1
    _check(lib().l0cim_mri_update_r(size, levels, gamma, _ptr(mask), _ptr(D), incd, _ptr(b), _ptr(sigma), cdp, dtc,
                                    iters, cg_max_iter, cg_tol, _ptr(R), _ptr(iters_out), _ptr(status),
                                    _stream(stream)), "l0cim_mri_update_r")
    return R


def cac_params(**kw) -> CacParams:
    """CAC-CIM defaults (random data, noise 0.05) with keyword overrides."""
    p = CacParams()
    lib().l0cim_cac_params_default(ctypes.byref(p))
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def l0cim_cac_run(J, z, eta: float, prm: CacParams, seed: int, alt: int, P: int, H=None, trace=None,
                  trace_steps: int = 0, status=None, ws=None, stream=None):
    """CAC-CIM run; returns (mu, n, m, e, sigma) as new device tensors."""
    n = J.shape[0]
    dt = _dtype_code(J)
    mu, nv, mv, e = (torch.empty((P, n), dtype=J.dtype, device=J.device) for _ in range(4))
    sigma = torch.empty((P, n), dtype=torch.uint8, device=J.device)
    ws = workspace(lib().l0cim_cac_run_workspace_bytes(dt, n, P), J.device) if ws is None else ws
    _check(lib().l0cim_cac_run(dt, n, P, _ptr(J), _ld(J), _ptr(z), eta, ctypes.byref(prm), seed, alt, _ptr(mu),
                               _ptr(nv), _ptr(mv), _ptr(e), _ptr(sigma), _ptr(H), _ptr(trace), trace_steps,
                               _ptr(status), _ptr(ws), ws.numel(), _stream(stream)), "l0cim_cac_run")
    return mu, nv, mv, e, sigma


def l0cim_cac_solve(A, y, prm: CacParams, sp: SolveParams, R_out=None, sigma_out=None, stats=None, ws=None,
                    stream=None):
    """Algorithm 1 with the CAC-CIM.  Returns (R, sigma, stats_bytes_tensor)."""
    m, n = A.shape
    dt = _dtype_code(A)
    R_out = torch.empty(n, dtype=A.dtype, device=A.device) if R_out is None else R_out
    sigma_out = torch.empty(n, dtype=torch.uint8, device=A.device) if sigma_out is None else sigma_out
    stats = torch.zeros(STATS_BYTES, dtype=torch.uint8, device=A.device) if stats is None else stats
    ws = workspace(lib().l0cim_cac_solve_workspace_bytes(dt, m, n, sp.replicas), A.device) if ws is None else ws
    _check(lib().l0cim_cac_solve(dt, m, n, _ptr(A), _ld(A), _ptr(y), ctypes.byref(prm), ctypes.byref(sp),
                                 _ptr(R_out), _ptr(sigma_out), _ptr(stats), _ptr(ws), ws.numel(), _stream(stream)),
           "l0cim_cac_solve")
    return R_out, sigma_out, stats


def mri_params(**kw) -> MriParams:
    p = MriParams()
    lib().l0cim_mri_params_default(ctypes.byref(p))
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def l0cim_mri_solve(mp: MriParams, A, y, mask, cim: CimParams, sp: SolveParams, R_out=None, sigma_out=None,
                    stats=None, ws=None, stream=None):
    """Algorithm 1 on the MRI-shaped operator.  Returns (R, sigma, stats_bytes_tensor)."""
    m, n = A.shape
    R_out = torch.empty(n, dtype=torch.float32, device=A.device) if R_out is None else R_out
    sigma_out = torch.empty(n, dtype=torch.uint8, device=A.device) if sigma_out is None else sigma_out
    stats = torch.zeros(STATS_BYTES, dtype=torch.uint8, device=A.device) if stats is None else stats
    need = lib().l0cim_mri_solve_workspace_bytes(m, sp.replicas, sp.final_refit_f64)
    ws = workspace(need, A.device) if ws is None else ws
    _check(lib().l0cim_mri_solve(ctypes.byref(mp), m, _ptr(A), _ld(A), _ptr(y), _ptr(mask), ctypes.byref(cim),
                                 ctypes.byref(sp), _ptr(R_out), _ptr(sigma_out), _ptr(stats), _ptr(ws), ws.numel(),
                                 _stream(stream)), "l0cim_mri_solve")
    return R_out, sigma_out, stats


def l0cim_mri_solve_many(mp: MriParams, A, y, mask, seeds, cim: CimParams, sp: SolveParams, R_out=None,
                         sigma_out=None, stats=None, ws=None, stream=None):
    """l0cim_mri_solve on stacked instances: A (count, m, n) or (m, n) shared, y (count, m), mask (count, n) or (n,)
    shared, seeds (count ints).  Returns (R (count, n), sigma (count, n), stats bytes)."""
    count, m = y.shape
    n = A.shape[-1]
    shared_a = A.dim() == 2
    R_out = torch.empty((count, n), dtype=torch.float32, device=A.device) if R_out is None else R_out
    sigma_out = torch.empty((count, n), dtype=torch.uint8, device=A.device) if sigma_out is None else sigma_out
    stats = torch.zeros(count * STATS_BYTES, dtype=torch.uint8, device=A.device) if stats is None else stats
    need = lib().l0cim_mri_solve_many_workspace_bytes(count, m, sp.replicas, sp.final_refit_f64)
    ws = workspace(need, A.device) if ws is None else ws
    sd = (ctypes.c_uint64 * count)(*[int(v) for v in seeds])
    lda = A.stride(0) if shared_a else A.stride(1)
    strideA = 0 if shared_a else A.stride(0)
    smask = 0 if mask.dim() == 1 else mask.stride(0)
    _check(lib().l0cim_mri_solve_many(ctypes.byref(mp), count, m, _ptr(A), lda, strideA, _ptr(y), y.stride(0),
                                      _ptr(mask), smask, ctypes.cast(sd, c_void_p), ctypes.byref(cim),
                                      ctypes.byref(sp), _ptr(R_out), _ptr(sigma_out), _ptr(stats), _ptr(ws),
                                      ws.numel(), _stream(stream)), "l0cim_mri_solve_many")
    return R_out, sigma_out, stats


def l0cim_select_replica(H, sigma, sigma_out=None, q_out=None, stream=None):
    P, n = sigma.shape
    sigma_out = torch.empty(n, dtype=torch.uint8, device=sigma.device) if sigma_out is None else sigma_out
    _check(lib().l0cim_select_replica(n, P, _ptr(H), _ptr(sigma), _ptr(sigma_out), _ptr(q_out),
                                      _stream(stream)), "l0cim_select_replica")
    return sigma_out


def l0cim_update_r_workspace_bytes(dtype: int, n: int, cdp: int) -> int:
    return lib().l0cim_update_r_workspace_bytes(dtype, n, cdp)


def l0cim_update_r(G, b, sigma, R, cdp: int = CDP_JACOBI, dtc: float = 0.1, iters: int = 100,
                   status=None, ws=None, stream=None):
    n = G.shape[0]
    dt = _dtype_code(G)
    ws = workspace(l0cim_update_r_workspace_bytes(dt, n, cdp), G.device) if ws is None else ws
    _check(lib().l0cim_update_r(dt, n, _ptr(G), _ld(G), _ptr(b), _ptr(sigma), cdp, dtc, iters, _ptr(R),
                                _ptr(status), _ptr(ws), ws.numel(), _stream(stream)), "l0cim_update_r")
    return R


def l0cim_solve_many_workspace_bytes(dtype: int, count: int, m: int, n: int, sp: SolveParams) -> int:
    return lib().l0cim_solve_many_workspace_bytes(dtype, count, m, n, ctypes.byref(sp))


def l0cim_solve_many(A, y, seeds, cim: CimParams, sp: SolveParams, R_out=None, sigma_out=None, stats=None, ws=None,
                     stream=None):
    """l0cim_solve on count stacked instances: A (count, m, n), y (count, m),
    seeds (count ints).  Returns (R (count, n), sigma (count, n), stats bytes)."""
    count, m, n = A.shape
    dt = _dtype_code(A)
    R_out = torch.empty((count, n), dtype=A.dtype, device=A.device) if R_out is None else R_out
    sigma_out = torch.empty((count, n), dtype=torch.uint8, device=A.device) if sigma_out is None else sigma_out
    stats = torch.zeros(count * STATS_BYTES, dtype=torch.uint8, device=A.device) if stats is None else stats
    need = lib().l0cim_solve_many_workspace_bytes(dt, count, m, n, ctypes.byref(sp))
    ws = workspace(need, A.device) if ws is None else ws
    sd = (ctypes.c_uint64 * count)(*[int(v) for v in seeds])
    _check(lib().l0cim_solve_many(dt, count, m, n, _ptr(A), A.stride(1), A.stride(0), _ptr(y), y.stride(0),
                                  ctypes.cast(sd, c_void_p), ctypes.byref(cim), ctypes.byref(sp), _ptr(R_out),
                                  _ptr(sigma_out), _ptr(stats), _ptr(ws), ws.numel(), _stream(stream)),
           "l0cim_solve_many")
    return R_out, sigma_out, stats


def l0cim_refit_f64_workspace_bytes(m: int, n: int) -> int:
    return lib().l0cim_refit_f64_workspace_bytes(m, n)


def l0cim_refit_f64(A, y, sigma, R, status=None, ws=None, stream=None):
    """FP64 least-squares refit of R on the support, G_SS and b_S from A, y."""
    m, n = A.shape
    dt = _dtype_code(A)
    ws = workspace(l0cim_refit_f64_workspace_bytes(m, n), A.device) if ws is None else ws
    _check(lib().l0cim_refit_f64(dt, m, n, _ptr(A), _ld(A), _ptr(y), _ptr(sigma), _ptr(R), _ptr(status),
                                 _ptr(ws), ws.numel(), _stream(stream)), "l0cim_refit_f64")
    return R


def l0cim_solve_workspace_bytes(dtype: int, m: int, n: int, cim: CimParams, sp: SolveParams) -> int:
    return lib().l0cim_solve_workspace_bytes(dtype, m, n, ctypes.byref(cim), ctypes.byref(sp))


def l0cim_solve(A, y, cim: CimParams, sp: SolveParams, R_init=None, R_out=None, sigma_out=None,
                stats=None, ws=None, stream=None):
    """Algorithm 1 on one instance.  Returns (R, sigma, stats_bytes_tensor)."""
    m, n = A.shape
    dt = _dtype_code(A)
    R_out = torch.empty(n, dtype=A.dtype, device=A.device) if R_out is None else R_out
    sigma_out = torch.empty(n, dtype=torch.uint8, device=A.device) if sigma_out is None else sigma_out
    stats = torch.zeros(STATS_BYTES, dtype=torch.uint8, device=A.device) if stats is None else stats
    need = l0cim_solve_workspace_bytes(dt, m, n, cim, sp)
    ws = workspace(need, A.device) if ws is None else ws
    _check(lib().l0cim_solve(dt, m, n, _ptr(A), _ld(A), _ptr(y), _ptr(R_init), ctypes.byref(cim),
                             ctypes.byref(sp), _ptr(R_out), _ptr(sigma_out), _ptr(stats), _ptr(ws),
                             ws.numel(), _stream(stream)), "l0cim_solve")
    return R_out, sigma_out, stats


def read_stats(stats_tensor) -> Stats:
    """Copy a device stats block to the host (synchronises)."""
    raw = bytes(stats_tensor.cpu().numpy().tobytes())
    return Stats.from_buffer_copy(raw)


# ---------------------------------------------------------------------------
# Batched form
# ---------------------------------------------------------------------------

def l0cim_batch_plan_create(instances, cim: CimParams, sp: SolveParams):
    """instances: sequence of Instance (or dicts with its fields).  Returns the plan handle."""
    arr = (Instance * len(instances))()
    for i, d in enumerate(instances):
        arr[i] = d if isinstance(d, Instance) else Instance(**d)
    h = c_void_p()
    _check(lib().l0cim_batch_plan_create(len(instances), arr, ctypes.byref(cim), ctypes.byref(sp),
                                         ctypes.byref(h)), "l0cim_batch_plan_create")
    return h


def l0cim_batch_plan_workspace_bytes(plan) -> int:
    return lib().l0cim_batch_plan_workspace_bytes(plan)


def l0cim_batch_plan_info(plan):
    rows, tiles, tuned = c_int32(), c_int32(), c_int32()
    _check(lib().l0cim_batch_plan_info(plan, ctypes.byref(rows), ctypes.byref(tiles), ctypes.byref(tuned)),
           "l0cim_batch_plan_info")
    return rows.value, tiles.value, bool(tuned.value)


def l0cim_batch_plan_destroy(plan):
    _check(lib().l0cim_batch_plan_destroy(plan), "l0cim_batch_plan_destroy")


def l0cim_solve_batched(plan, A_pool, y_pool, R_pool, sigma_pool, stats, ws, stream=None):
    _check(lib().l0cim_solve_batched(plan, _ptr(A_pool), _ptr(y_pool), _ptr(R_pool), _ptr(sigma_pool),
                                     _ptr(stats), _ptr(ws), ws.numel(), _stream(stream)),
           "l0cim_solve_batched")


def l0cim_batch_begin(plan, A_pool, y_pool, R_pool, sigma_pool, stats, ws, stream=None):
    _check(lib().l0cim_batch_begin(plan, _ptr(A_pool), _ptr(y_pool), _ptr(R_pool), _ptr(sigma_pool),
                                   _ptr(stats), _ptr(ws), ws.numel(), _stream(stream)),
           "l0cim_batch_begin")


def l0cim_batch_alternations(plan, i0: int, i1: int, A_pool, y_pool, R_pool, sigma_pool, stats, ws, stream=None):
    _check(lib().l0cim_batch_alternations(plan, i0, i1, _ptr(A_pool), _ptr(y_pool), _ptr(R_pool),
                                          _ptr(sigma_pool), _ptr(stats), _ptr(ws), ws.numel(), _stream(stream)),
           "l0cim_batch_alternations")


def l0cim_batch_finish(plan, A_pool, y_pool, R_pool, sigma_pool, stats, ws, stream=None):
    _check(lib().l0cim_batch_finish(plan, _ptr(A_pool), _ptr(y_pool), _ptr(R_pool), _ptr(sigma_pool),
                                    _ptr(stats), _ptr(ws), ws.numel(), _stream(stream)),
           "l0cim_batch_finish")


def pack_instances(As, ys, seeds, device="cuda"):
    """Pack per-instance A (m x n) and y into contiguous FP32 pools and build
    the instance descriptors.  Returns (instances, A_pool, y_pool, R_pool,
    sigma_pool, stats, x_offsets)."""
    insts, a_off, y_off, x_off = [], 0, 0, 0
    for A, y, sd in zip(As, ys, seeds):
        m, n = A.shape
        insts.append(Instance(m=m, n=n, a_offset=a_off, lda=n, y_offset=y_off, x_offset=x_off, seed=sd))
        a_off += m * n
        y_off += m
        x_off += n
    A_pool = torch.cat([torch.as_tensor(A, dtype=torch.float32).reshape(-1) for A in As]).to(device)
    y_pool = torch.cat([torch.as_tensor(y, dtype=torch.float32).reshape(-1) for y in ys]).to(device)
    R_pool = torch.zeros(x_off, dtype=torch.float32, device=device)
    sigma_pool = torch.zeros(x_off, dtype=torch.uint8, device=device)
    stats = torch.zeros(len(insts) * STATS_BYTES, dtype=torch.uint8, device=device)
    return insts, A_pool, y_pool, R_pool, sigma_pool, stats


def read_stats_array(stats_tensor, count):
    raw = bytes(stats_tensor.cpu().numpy().tobytes())
    return [Stats.from_buffer_copy(raw, i * STATS_BYTES) for i in range(count)]


def l0cim_server_request_bytes(m: int, n: int, sp: SolveParams) -> int:
    return lib().l0cim_server_request_bytes(m, n, ctypes.byref(sp))


def l0cim_server_arena_overhead(max_slots: int, max_n: int, sp: SolveParams) -> int:
    return lib().l0cim_server_arena_overhead(max_slots, max_n, ctypes.byref(sp))


def l0cim_server_create(cim: CimParams, sp: SolveParams, max_slots: int, max_n: int, arena, stream=None):
    """arena: a uint8 CUDA tensor (256-byte aligned) that the server uses until destroyed."""
    h = c_void_p()
    _check(lib().l0cim_server_create(ctypes.byref(cim), ctypes.byref(sp), max_slots, max_n, _ptr(arena),
                                     arena.numel() * arena.element_size(), _stream(stream), ctypes.byref(h)),
           "l0cim_server_create")
    return h


def l0cim_server_clock(server) -> float:
    return lib().l0cim_server_clock(server)


def l0cim_server_submit(server, A, y, seed: int, tag: int, R_out, sigma_out, stats_out):
    m, n = A.shape
    _check(lib().l0cim_server_submit(server, m, n, _ptr(A), _ld(A), _ptr(y), seed, tag, _ptr(R_out),
                                     _ptr(sigma_out), _ptr(stats_out)), "l0cim_server_submit")


def l0cim_server_set_step_budget(server, nbytes: int) -> None:
    _check(lib().l0cim_server_set_step_budget(server, int(nbytes)), "l0cim_server_set_step_budget")


def l0cim_server_step(server) -> int:
    done = c_int32()
    _check(lib().l0cim_server_step(server, ctypes.byref(done)), "l0cim_server_step")
    return done.value


def l0cim_server_completed(server, max_records: int = 4096):
    buf = (Completion * max_records)()
    k = lib().l0cim_server_completed(server, buf, max_records)
    return [buf[i] for i in range(k)]


def l0cim_server_info(server):
    a, p, u, h, t = c_int32(), c_int32(), c_size_t(), c_size_t(), c_int64()
    _check(lib().l0cim_server_info(server, ctypes.byref(a), ctypes.byref(p), ctypes.byref(u), ctypes.byref(h),
                                   ctypes.byref(t)), "l0cim_server_info")
    return dict(active=a.value, pending=p.value, bytes_in_use=u.value, heap_bytes=h.value, ticks=t.value)


def l0cim_server_destroy(server):
    _check(lib().l0cim_server_destroy(server), "l0cim_server_destroy")


def _field_code(field) -> int:
    return {"CN": FIELD_CN, "BN": FIELD_BN}.get(field, field)


def l0cim_matrix_tile_get(n: int, P: int, j_dtype: int, field) -> int:
    rows = c_int32()
    _check(lib().l0cim_matrix_tile_get(n, P, j_dtype, _field_code(field), ctypes.byref(rows)),
           "l0cim_matrix_tile_get")
    return rows.value


def l0cim_matrix_tile_set(n: int, P: int, j_dtype: int, field, rows: int):
    _check(lib().l0cim_matrix_tile_set(n, P, j_dtype, _field_code(field), rows), "l0cim_matrix_tile_set")


def l0cim_profile_begin():
    _check(lib().l0cim_profile_begin(), "l0cim_profile_begin")


def l0cim_profile_end():
    ms = c_double(0.0)
    cnt = c_int64(0)
    _check(lib().l0cim_profile_end(ctypes.byref(ms), ctypes.byref(cnt)), "l0cim_profile_end")
    return ms.value, cnt.value
