"""Python binding of the gfx950 DOCH library (``libising.so``, include/ising.h).

The functions below have the C names and the C argument order; they only
marshal arguments (device pointers as integers, torch tensors via
``data_ptr()``, the current torch stream as ``hipStream_t``).  Every step of
the hot path runs in the library's HIP kernels.  Importing this module fails
loudly if the library has not been built: there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

__all__ = [
    "ISING_OK", "ISING_F64", "ISING_F32", "ISING_BF16", "ISING_FP8_E4M3", "ISING_I32", "ISING_I16",
    "IsingError", "ising_params", "ising_stats", "ising_info", "lib", "LIB_PATH",
    "ising_create_csr", "ising_create_dense", "ising_destroy", "ising_get_info",
    "ising_check_symmetric", "ising_default_params", "ising_solve", "ising_get_log",
    "ising_energy", "ising_energy_noalloc", "ising_cut", "ising_tune_eta", "ising_set_geometry", "ising_autotune", "ising_create_batch",
    "ising_default_params_batch", "ising_solve_batch", "ising_energy_batch", "ising_set_batch_shape", "ising_autotune_batch", "ising_set_lowp_shape", "ising_autotune_lowp", "ising_solve_lowp", "ising_get_accept_log", "ising_create_procedural",
    "ising_status_string", "ising_last_error", "ising_version",
    "ptr", "current_stream",
]

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libising.so")

ISING_OK = 0
ISING_E_INVALID_ARG = 1
ISING_E_NONZERO_DIAG = 2
ISING_E_NOT_SYMMETRIC = 3
ISING_E_OUT_OF_MEMORY = 4
ISING_E_HIP = 5
ISING_E_UNSUPPORTED = 6
ISING_E_NONFINITE = 7

ISING_F64 = 0
ISING_F32 = 1
ISING_BF16 = 2
ISING_FP8_E4M3 = 3
ISING_I32 = 4
ISING_I16 = 5


class ising_params(ctypes.Structure):
    _fields_ = [("alpha", ctypes.c_double), ("beta", ctypes.c_double), ("eps", ctypes.c_double),
                ("algo", ctypes.c_int32), ("q", ctypes.c_int32), ("x_dtype", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class ising_stats(ctypes.Structure):
    _fields_ = [("iters_done", ctypes.c_int64), ("converged", ctypes.c_int32),
                ("nonfinite", ctypes.c_int32), ("H_last", ctypes.c_double),
                ("r_last", ctypes.c_double)]


class ising_info(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("n_iter", ctypes.c_int64), ("nnz", ctypes.c_int64),
                ("is_dense", ctypes.c_int32), ("has_field", ctypes.c_int32),
                ("integer_J", ctypes.c_int32), ("val_dtype", ctypes.c_int32),
                ("row_len", ctypes.c_int32), ("geometry", ctypes.c_int32),
                ("step_val_bytes", ctypes.c_int32), ("step_col_bytes", ctypes.c_int32)]


class IsingError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: {ising_status_string(status)} ({status}): {ising_last_error()}")


if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it first (python -m paper_2509_01928_amd.build "
                      "or __graft_entry__.build()); there is no fallback path")

# PyTorch ships its own HIP runtime.  Load it first so that the library binds
# to the same runtime instance (same devices, streams and allocations) rather
# than to a second copy from the system ROCm.
import torch  # noqa: E402,F401

lib = ctypes.CDLL(LIB_PATH)

_p = ctypes.c_void_p
_i64 = ctypes.c_int64
_i32 = ctypes.c_int32
_d = ctypes.c_double
_st = ctypes.c_int

_SIGS = {
    "ising_create_csr": (_st, [_i64, _i64, _p, _p, _p, _i32, _p, _i32, _p, ctypes.POINTER(_p)]),
    "ising_create_dense": (_st, [_i64, _p, _i32, _i64, _p, _i32, _p, ctypes.POINTER(_p)]),
    "ising_destroy": (None, [_p]),
    "ising_get_info": (_st, [_p, ctypes.POINTER(ising_info)]),
    "ising_check_symmetric": (_st, [_p, _p]),
    "ising_default_params": (_st, [_p, _d, _i32, _p, ctypes.POINTER(ising_params), ctypes.POINTER(_d)]),
    "ising_solve": (_st, [_p, _p, _i32, _i64, ctypes.POINTER(ising_params), _p, _p, _p, _p]),
    "ising_get_log": (_st, [_p, _i32, _i64, _i64, _p, _p, _p]),
    "ising_energy": (_st, [_p, _p, _i32, _p, _p, _p]),
    "ising_energy_noalloc": (_st, [_p, _p, _i32, _p, _p, _p]),
    "ising_cut": (_st, [_p, _p, _i32, _p, _p, _p]),
    "ising_tune_eta": (_st, [_p, _p, _i32, _p, _i64, _i32, _p, ctypes.POINTER(ising_params), _p, _p]),
    "ising_set_geometry": (_st, [_p, _i32, _i32]),
    "ising_autotune": (_st, [_p, _p, _i64, ctypes.POINTER(ising_params), _p, _p, _p, _p]),
    "ising_create_batch": (_st, [_i32, _p, _p, _p, _p, _i32, _p, ctypes.POINTER(_p)]),
    "ising_default_params_batch": (_st, [_p, _d, _i32, _p, _p, _p, _p]),
    "ising_solve_batch": (_st, [_p, _p, _i32, _i64, _p, _p, _d, _i32, _p, _p, _p, _p, _p]),
    "ising_energy_batch": (_st, [_p, _p, _i32, _p, _p, _p]),
    "ising_set_batch_shape": (_st, [_p, _i32, _i32, _i32]),
    "ising_set_lowp_shape": (_st, [_p, _i32, _i32, _i32, _i32]),
    "ising_autotune_batch": (_st, [_p, _p, _i32, _i64, _p, _p, _d, _i32, ctypes.c_char_p, _p, _p, _p, _p]),
    "ising_autotune_lowp": (_st, [_p, _p, _i32, _i64, _p, _i32, ctypes.c_char_p, _p, _p, _p, _p]),
    "ising_solve_lowp": (_st, [_p, _p, _i32, _i64, ctypes.POINTER(ising_params), _i32, _p, _p, _p, _p, _p]),
    "ising_get_accept_log": (_st, [_p, _i64, _i64, _p, _p]),
    "ising_create_procedural": (_st, [_i64, _i32, _d, _p, ctypes.POINTER(_p)]),
    "ising_status_string": (ctypes.c_char_p, [_st]),
    "ising_last_error": (ctypes.c_char_p, []),
    "ising_version": (ctypes.c_char_p, []),
}
for _name, (_res, _args) in _SIGS.items():
    _fn = getattr(lib, _name)
    _fn.restype = _res
    _fn.argtypes = _args


def ising_status_string(status: int) -> str:
    return lib.ising_status_string(int(status)).decode()


def ising_last_error() -> str:
    return lib.ising_last_error().decode()


def ising_version() -> str:
    return lib.ising_version().decode()


def ptr(t) -> Optional[int]:
    """Device (or host) address of a torch tensor / numpy array, None for None."""
    if t is None:
        return None
    if hasattr(t, "data_ptr"):
        return t.data_ptr()
    return t.ctypes.data


def current_stream() -> int:
    """hipStream_t of torch's current stream on the current device."""
    import torch
    return torch.cuda.current_stream().cuda_stream


def _check(status: int, where: str) -> int:
    if status != ISING_OK:
        raise IsingError(status, where)
    return status


def ising_create_csr(n, nnz, row_ptr, col, val, vt, h=None, ht=ISING_F32, stream=None):
    """Returns the context handle (int).  row_ptr/col/val/h: device pointers or tensors."""
    out = _p()
    _check(lib.ising_create_csr(int(n), int(nnz), ptr(row_ptr), ptr(col), ptr(val), int(vt),
                                ptr(h), int(ht), stream if stream is not None else current_stream(),
                                ctypes.byref(out)), "ising_create_csr")
    return out.value


def ising_create_dense(n, J, jt, ld, h=None, ht=ISING_F32, stream=None):
    out = _p()
    _check(lib.ising_create_dense(int(n), ptr(J), int(jt), int(ld), ptr(h), int(ht),
                                  stream if stream is not None else current_stream(),
                                  ctypes.byref(out)), "ising_create_dense")
    return out.value


def ising_destroy(ctx) -> None:
    if ctx:
        lib.ising_destroy(ctx)


def ising_get_info(ctx) -> ising_info:
    info = ising_info()
    _check(lib.ising_get_info(ctx, ctypes.byref(info)), "ising_get_info")
    return info


def ising_check_symmetric(ctx, stream=None) -> bool:
    st = lib.ising_check_symmetric(ctx, stream if stream is not None else current_stream())
    if st == ISING_E_NOT_SYMMETRIC:
        return False
    _check(st, "ising_check_symmetric")
    return True


def ising_default_params(ctx, eta=1.0, method=0, stream=None):
    """Returns (ising_params, lambda)."""
    p = ising_params()
    lam = _d(0.0)
    _check(lib.ising_default_params(ctx, float(eta), int(method),
                                    stream if stream is not None else current_stream(),
                                    ctypes.byref(p), ctypes.byref(lam)), "ising_default_params")
    return p, lam.value


def ising_solve(ctx, x0, R, iters, params, x_out=None, s_out=None, want_stats=True,
                stream=None, check=True):
    """Returns a list of ising_stats (empty if want_stats is False)."""
    stats = (ising_stats * int(R))() if want_stats else None
    st = lib.ising_solve(ctx, ptr(x0), int(R), int(iters), ctypes.byref(params), ptr(x_out),
                         ptr(s_out), ctypes.cast(stats, _p) if stats is not None else None,
                         stream if stream is not None else current_stream())
    if check:
        _check(st, "ising_solve")
    return list(stats) if stats is not None else []


def ising_get_log(ctx, restart, first, count, stream=None):
    """Returns (H, r) as numpy arrays."""
    import numpy as np
    H = np.empty(int(count), dtype=np.float64)
    r = np.empty(int(count), dtype=np.float64)
    _check(lib.ising_get_log(ctx, int(restart), int(first), int(count), H.ctypes.data,
                             r.ctypes.data, stream if stream is not None else current_stream()),
           "ising_get_log")
    return H, r


def ising_energy(ctx, s, R, E=None, E_int=None, stream=None):
    _check(lib.ising_energy(ctx, ptr(s), int(R), ptr(E), ptr(E_int),
                            stream if stream is not None else current_stream()), "ising_energy")


def ising_energy_noalloc(ctx, s, R, E=None, E_int=None, stream=None):
    _check(lib.ising_energy_noalloc(ctx, ptr(s), int(R), ptr(E), ptr(E_int),
                                    stream if stream is not None else current_stream()),
           "ising_energy_noalloc")


def ising_tune_eta(ctx, x0, etas, probe_iters, method=0, stream=None):
    """Returns (params of the best eta, best eta, numpy array of probe energies)."""
    import numpy as np
    etas = np.ascontiguousarray(etas, dtype=np.float64)
    energies = np.empty(etas.shape[0], dtype=np.float64)
    best = ising_params()
    best_eta = ctypes.c_double()
    _check(lib.ising_tune_eta(ctx, ptr(x0), int(etas.shape[0]), etas.ctypes.data, int(probe_iters),
                              int(method), stream if stream is not None else current_stream(),
                              ctypes.byref(best), ctypes.byref(best_eta), energies.ctypes.data),
           "ising_tune_eta")
    return best, best_eta.value, energies


def ising_cut(ctx, s, R, cut=None, cut_int=None, stream=None):
    """MAX-CUT value of each spin vector for weights w_ij = -J_ij."""
    _check(lib.ising_cut(ctx, ptr(s), int(R), ptr(cut), ptr(cut_int),
                         stream if stream is not None else current_stream()),
           "ising_cut")


# geometry id of the single-launch (resident) solve
GEOMETRY_RESIDENT = 8


def ising_set_geometry(ctx, geometry, wg_per_cu=0) -> None:
    _check(lib.ising_set_geometry(ctx, int(geometry), int(wg_per_cu)), "ising_set_geometry")


def ising_autotune(ctx, x0, iters, params, stream=None):
    """Returns (best geometry, best workgroups per CU, [best ms/iteration per geometry])."""
    g = ctypes.c_int32(-1)
    w = ctypes.c_int32(-1)
    ms = (ctypes.c_double * (GEOMETRY_RESIDENT + 1))()
    _check(lib.ising_autotune(ctx, ptr(x0), int(iters), ctypes.byref(params),
                              stream if stream is not None else current_stream(),
                              ctypes.byref(g), ctypes.byref(w), ctypes.cast(ms, _p)),
           "ising_autotune")
    return g.value, w.value, list(ms)


def ising_create_batch(n_list, row_ptr, col, val, vt, stream=None):
    """Block-diagonal batch of len(n_list) instances; returns the context handle."""
    import numpy as np
    n_arr = np.ascontiguousarray(np.asarray(n_list, dtype=np.int64))
    out = _p()
    _check(lib.ising_create_batch(int(n_arr.shape[0]), n_arr.ctypes.data, ptr(row_ptr), ptr(col),
                                  ptr(val), int(vt),
                                  stream if stream is not None else current_stream(),
                                  ctypes.byref(out)), "ising_create_batch")
    return out.value


def ising_default_params_batch(ctx, count, eta=1.0, method=0, stream=None):
    """Returns numpy arrays (alpha, beta, lambda) of the batch's instances."""
    import numpy as np
    a = np.empty(int(count), dtype=np.float64)
    b = np.empty(int(count), dtype=np.float64)
    lam = np.empty(int(count), dtype=np.float64)
    _check(lib.ising_default_params_batch(ctx, float(eta), int(method),
                                          stream if stream is not None else current_stream(),
                                          a.ctypes.data, b.ctypes.data, lam.ctypes.data),
           "ising_default_params_batch")
    return a, b, lam


def ising_solve_batch(ctx, x0, R, max_iters, alpha, beta, eps=0.0, x_dtype=ISING_F64, x_out=None,
                      s_out=None, want_stats=True, stream=None, check=True):
    """Returns (stats list of count*R entries, numpy time-to-solution in ms) or ([], None)."""
    import numpy as np
    alpha = np.ascontiguousarray(alpha, dtype=np.float64)
    beta = np.ascontiguousarray(beta, dtype=np.float64)
    count = int(alpha.shape[0])
    stats = (ising_stats * (count * int(R)))() if want_stats else None
    tts = np.empty(count, dtype=np.float64) if want_stats else None
    st = lib.ising_solve_batch(ctx, ptr(x0), int(R), int(max_iters), alpha.ctypes.data,
                               beta.ctypes.data, float(eps), int(x_dtype), ptr(x_out), ptr(s_out),
                               ctypes.cast(stats, _p) if stats is not None else None,
                               tts.ctypes.data if tts is not None else None,
                               stream if stream is not None else current_stream())
    if check:
        _check(st, "ising_solve_batch")
    return (list(stats), tts) if want_stats else ([], None)


def ising_energy_batch(ctx, s, R, E=None, E_int=None, stream=None):
    _check(lib.ising_energy_batch(ctx, ptr(s), int(R), ptr(E), ptr(E_int),
                                  stream if stream is not None else current_stream()),
           "ising_energy_batch")


def ising_set_lowp_shape(ctx, bn, splits=1, stage_bytes=256, depth=2):
    _check(lib.ising_set_lowp_shape(ctx, int(bn), int(splits), int(stage_bytes), int(depth)),
           "ising_set_lowp_shape")


def ising_set_batch_shape(ctx, rj, wg, chunk_rows):
    _check(lib.ising_set_batch_shape(ctx, int(rj), int(wg), int(chunk_rows)), "ising_set_batch_shape")


def ising_autotune_batch(ctx, x0, R, max_iters, alpha, beta, eps=0.0, x_dtype=ISING_F64, cache_path=None,
                         stream=None):
    """Returns ((rj, wg, chunk_rows), milliseconds, from_cache)."""
    import numpy as np
    alpha = np.ascontiguousarray(alpha, dtype=np.float64)
    beta = np.ascontiguousarray(beta, dtype=np.float64)
    shape = (ctypes.c_int32 * 3)()
    ms = ctypes.c_double()
    cached = ctypes.c_int32()
    _check(lib.ising_autotune_batch(ctx, ptr(x0), int(R), int(max_iters), alpha.ctypes.data, beta.ctypes.data,
                                    float(eps), int(x_dtype),
                                    os.fsencode(cache_path) if cache_path is not None else None,
                                    stream if stream is not None else current_stream(),
                                    ctypes.cast(shape, _p), ctypes.byref(ms), ctypes.byref(cached)),
           "ising_autotune_batch")
    return (shape[0], shape[1], shape[2]), ms.value, bool(cached.value)


def ising_autotune_lowp(ctx, x0, R, iters, params, jx_dtype, cache_path=None, stream=None):
    """Returns ((bn, splits, stage_bytes, depth), milliseconds, from_cache)."""
    shape = (ctypes.c_int32 * 4)()
    ms = ctypes.c_double()
    cached = ctypes.c_int32()
    _check(lib.ising_autotune_lowp(ctx, ptr(x0), int(R), int(iters), ctypes.byref(params), int(jx_dtype),
                                   os.fsencode(cache_path) if cache_path is not None else None,
                                   stream if stream is not None else current_stream(),
                                   ctypes.cast(shape, _p), ctypes.byref(ms), ctypes.byref(cached)),
           "ising_autotune_lowp")
    return (shape[0], shape[1], shape[2], shape[3]), ms.value, bool(cached.value)


def ising_solve_lowp(ctx, x0, R, iters, params, jx_dtype, x_out=None, s_out=None, H_final=None,
                     want_stats=True, stream=None, check=True):
    """Dense restarts on the matrix cores in BF16 / FP8; returns the stats list."""
    stats = (ising_stats * int(R))() if want_stats else None
    st = lib.ising_solve_lowp(ctx, ptr(x0), int(R), int(iters), ctypes.byref(params), int(jx_dtype),
                              ptr(x_out), ptr(s_out), ptr(H_final),
                              ctypes.cast(stats, _p) if stats is not None else None,
                              stream if stream is not None else current_stream())
    if check:
        _check(st, "ising_solve_lowp")
    return list(stats) if stats is not None else []


def ising_get_accept_log(ctx, first, count, R=1, stream=None):
    """ADOCH decisions of the last solve (numpy int8: 1 = extrapolated point
    taken); shape (count,) for one restart, (count, R) for R restarts."""
    import numpy as np
    out = np.empty(int(count) * int(R), dtype=np.int8)
    _check(lib.ising_get_accept_log(ctx, int(first), int(count), out.ctypes.data,
                                    stream if stream is not None else current_stream()),
           "ising_get_accept_log")
    return out if R == 1 else out.reshape(int(count), int(R))


def ising_create_procedural(n, kind=1, seed=100.0, stream=None):
    """Dense context with J_ij = sin(i*j + seed) generated on demand (kind 1)."""
    out = _p()
    _check(lib.ising_create_procedural(int(n), int(kind), float(seed),
                                       stream if stream is not None else current_stream(),
                                       ctypes.byref(out)), "ising_create_procedural")
    return out.value
