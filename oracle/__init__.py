"""Python face of the FP64 CPU oracle (``doch_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()``
and the CPU-baseline leg of ``bench.py``.  The product library never imports
it, and it never imports the product.

Every function takes host numpy arrays (or an ``ising_inputs.CSR``) and
returns host numpy arrays.  Paper references: eq:FPE and Alg. 1 (DOCH),
Alg. 2 and eq:BBscheme (ADOCH), eq:Hamilton (H), Remark S2 (r), eq:IsingModel
(energy), Supp. Note 1 (field -> extra spin), eq:alphabeta,
eq:estimate_eig_J and Supp. Note 6 (parameters).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

_i64 = ctypes.c_int64
_i32 = ctypes.c_int32
_dbl = ctypes.c_double
_p = ctypes.c_void_p


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, no FMA contraction, no fast-math)."""
    if force or not os.path.exists(_LIB_PATH):
        src = os.path.join(_HERE, "doch_oracle.c")
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-ffp-contract=off",
                               "-fno-fast-math", "-fPIC", "-shared", src, "-o",
                               tmp, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=True)
        lib = ctypes.CDLL(_LIB_PATH)
        sigs = {
            "ref_augment_field": (None, [_i64, _p, _p, _p, _p, _p, _p, _p]),
            "ref_matvec_csr": (None, [_i64, _p, _p, _p, _p, _p]),
            "ref_matvec_dense": (None, [_i64, _p, _p, _p]),
            "ref_hamiltonian_csr": (_dbl, [_i64, _p, _p, _p, _p, _dbl, _dbl]),
            "ref_hamiltonian_dense": (_dbl, [_i64, _p, _p, _dbl, _dbl]),
            "ref_doch_csr": (_i64, [_i64, _p, _p, _p, _p, _dbl, _dbl, _i64, _dbl, _p, _p, _p]),
            "ref_doch_dense": (_i64, [_i64, _p, _p, _dbl, _dbl, _i64, _dbl, _p, _p, _p]),
            "ref_adoch_csr": (_i64, [_i64, _p, _p, _p, _p, _dbl, _dbl, _i64, _i32, _dbl,
                                     _p, _p, _p, _p, _p, _p]),
            "ref_sign": (None, [_i64, _p, _p]),
            "ref_energy_csr_f64": (_dbl, [_i64, _p, _p, _p, _p, _p]),
            "ref_energy_dense_f64": (_dbl, [_i64, _p, _p, _p]),
            "ref_energy_csr_i64": (ctypes.c_int, [_i64, _p, _p, _p, _p, _p]),
            "ref_bruteforce_dense": (_dbl, [_i64, _p, _p, _p]),
            "ref_offdiag_rowsum_max": (_dbl, [_i64, _p, _p, _p]),
            "ref_wigner_lambda": (_dbl, [_i64, _p, _p, _p]),
            "ref_power_lambda_max_neg": (_dbl, [_i64, _p, _p, _p, _p, _dbl, _i64, _p]),
        }
        for name, (res, args) in sigs.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data


@dataclass
class OracleCSR:
    """CSR in the oracle's own precision: int64 offsets, int32 cols, f64 vals."""
    n: int
    rp: np.ndarray
    col: np.ndarray
    val: np.ndarray


def to_oracle_csr(A) -> OracleCSR:
    """Copy an instance's coupling matrix into the oracle's storage types."""
    return OracleCSR(int(A.n), np.ascontiguousarray(A.row_ptr, dtype=np.int64),
                     np.ascontiguousarray(A.col, dtype=np.int32),
                     np.ascontiguousarray(A.val, dtype=np.float64))


def csr_of_dense(J: np.ndarray) -> OracleCSR:
    """All off-diagonal entries of a dense matrix as CSR (zeros kept)."""
    n = J.shape[0]
    mask = ~np.eye(n, dtype=bool)
    rows, cols = np.nonzero(mask)
    rp = np.arange(0, n * (n - 1) + 1, n - 1, dtype=np.int64) if n > 1 else np.zeros(n + 1, np.int64)
    return OracleCSR(n, rp, cols.astype(np.int32), np.ascontiguousarray(J[rows, cols], dtype=np.float64))


def augment_field(A: OracleCSR, h: np.ndarray) -> OracleCSR:
    """Supp. Note 1: the (n+1)-spin matrix [[J, h], [h^T, 0]]."""
    lib = _load()
    n = A.n
    h = np.ascontiguousarray(h, dtype=np.float64)
    nnz = A.col.shape[0]
    rp = np.empty(n + 2, dtype=np.int64)
    col = np.empty(nnz + 2 * n, dtype=np.int32)
    val = np.empty(nnz + 2 * n, dtype=np.float64)
    lib.ref_augment_field(n, _ptr(A.rp), _ptr(A.col), _ptr(A.val), _ptr(h),
                          _ptr(rp), _ptr(col), _ptr(val))
    return OracleCSR(n + 1, rp, col, val)


def problem_matrix(A) -> OracleCSR:
    """The homogeneous matrix the iteration runs on: J, or Jhat if A.h is set."""
    B = to_oracle_csr(A)
    if getattr(A, "h", None) is not None:
        B = augment_field(B, A.h)
    return B


def matvec(B: OracleCSR, x: np.ndarray) -> np.ndarray:
    lib = _load()
    x = np.ascontiguousarray(x, dtype=np.float64)
    z = np.empty(B.n, dtype=np.float64)
    lib.ref_matvec_csr(B.n, _ptr(B.rp), _ptr(B.col), _ptr(B.val), _ptr(x), _ptr(z))
    return z


def matvec_dense(J: np.ndarray, x: np.ndarray) -> np.ndarray:
    lib = _load()
    J = np.ascontiguousarray(J, dtype=np.float64)
    x = np.ascontiguousarray(x, dtype=np.float64)
    z = np.empty(J.shape[0], dtype=np.float64)
    lib.ref_matvec_dense(J.shape[0], _ptr(J), _ptr(x), _ptr(z))
    return z


def hamiltonian(B: OracleCSR, x: np.ndarray, alpha: float, beta: float) -> float:
    lib = _load()
    x = np.ascontiguousarray(x, dtype=np.float64)
    return lib.ref_hamiltonian_csr(B.n, _ptr(B.rp), _ptr(B.col), _ptr(B.val), _ptr(x),
                                   alpha, beta)


def hamiltonian_dense(J: np.ndarray, x: np.ndarray, alpha: float, beta: float) -> float:
    lib = _load()
    J = np.ascontiguousarray(J, dtype=np.float64)
    x = np.ascontiguousarray(x, dtype=np.float64)
    return lib.ref_hamiltonian_dense(J.shape[0], _ptr(J), _ptr(x), alpha, beta)


@dataclass
class Trajectory:
    x: np.ndarray          # x^(iters_done)
    H: np.ndarray          # H(x^(k)), k < iters_done
    r: np.ndarray          # r^(k),   k < iters_done
    iters: int
    accept: Optional[np.ndarray] = None   # ADOCH only: y^(k) taken
    Hy: Optional[np.ndarray] = None       # ADOCH only: H(y^(k))
    Hmax: Optional[np.ndarray] = None     # ADOCH only: window maximum at k


def doch(B: OracleCSR, x0: np.ndarray, alpha: float, beta: float, iters: int,
         eps: float = 0.0) -> Trajectory:
    """Alg. 1 on a CSR problem matrix (already augmented if there is a field)."""
    lib = _load()
    x0 = np.ascontiguousarray(x0, dtype=np.float64).reshape(-1)
    assert x0.shape[0] == B.n
    x = np.empty(B.n, dtype=np.float64)
    H = np.empty(max(iters, 1), dtype=np.float64)
    r = np.empty(max(iters, 1), dtype=np.float64)
    k = lib.ref_doch_csr(B.n, _ptr(B.rp), _ptr(B.col), _ptr(B.val), _ptr(x0), alpha, beta,
                         iters, eps, _ptr(x), _ptr(H), _ptr(r))
    return Trajectory(x, H[:k].copy(), r[:k].copy(), int(k))


def doch_dense(J: np.ndarray, x0: np.ndarray, alpha: float, beta: float, iters: int,
               eps: float = 0.0) -> Trajectory:
    """Alg. 1 on a dense row-major matrix."""
    lib = _load()
    J = np.ascontiguousarray(J, dtype=np.float64)
    n = J.shape[0]
    x0 = np.ascontiguousarray(x0, dtype=np.float64).reshape(-1)
    assert x0.shape[0] == n
    x = np.empty(n, dtype=np.float64)
    H = np.empty(max(iters, 1), dtype=np.float64)
    r = np.empty(max(iters, 1), dtype=np.float64)
    k = lib.ref_doch_dense(n, _ptr(J), _ptr(x0), alpha, beta, iters, eps, _ptr(x), _ptr(H),
                           _ptr(r))
    return Trajectory(x, H[:k].copy(), r[:k].copy(), int(k))


def adoch(B: OracleCSR, x0: np.ndarray, alpha: float, beta: float, iters: int, q: int,
          eps: float = 0.0) -> Trajectory:
    """Alg. 2 on a CSR problem matrix."""
    lib = _load()
    x0 = np.ascontiguousarray(x0, dtype=np.float64).reshape(-1)
    x = np.empty(B.n, dtype=np.float64)
    H = np.empty(max(iters, 1), dtype=np.float64)
    r = np.empty(max(iters, 1), dtype=np.float64)
    acc = np.empty(max(iters, 1), dtype=np.int8)
    Hy = np.empty(max(iters, 1), dtype=np.float64)
    Hm = np.empty(max(iters, 1), dtype=np.float64)
    k = lib.ref_adoch_csr(B.n, _ptr(B.rp), _ptr(B.col), _ptr(B.val), _ptr(x0), alpha, beta,
                          iters, int(q), eps, _ptr(x), _ptr(H), _ptr(r), _ptr(acc), _ptr(Hy),
                          _ptr(Hm))
    return Trajectory(x, H[:k].copy(), r[:k].copy(), int(k), acc[:k].copy(), Hy[:k].copy(),
                      Hm[:k].copy())


def sign(x: np.ndarray) -> np.ndarray:
    lib = _load()
    x = np.ascontiguousarray(x, dtype=np.float64)
    s = np.empty(x.shape[0], dtype=np.int8)
    lib.ref_sign(x.shape[0], _ptr(x), _ptr(s))
    return s


def spins_with_field(x_hat: np.ndarray) -> np.ndarray:
    """Prop. S1: with the extra spin t = x_hat[n], the answer is t * s_0."""
    s = sign(x_hat)
    return (s[:-1] * s[-1]).astype(np.int8)


def energy(A, s: np.ndarray) -> float:
    """eq:IsingModel for an ``ising_inputs.CSR`` (field included if present)."""
    lib = _load()
    B = to_oracle_csr(A)
    s = np.ascontiguousarray(s, dtype=np.int8)
    h = None if getattr(A, "h", None) is None else np.ascontiguousarray(A.h, dtype=np.float64)
    return lib.ref_energy_csr_f64(B.n, _ptr(B.rp), _ptr(B.col), _ptr(B.val), _ptr(h), _ptr(s))


def energy_csr(B: OracleCSR, s: np.ndarray, h: Optional[np.ndarray] = None) -> float:
    lib = _load()
    s = np.ascontiguousarray(s, dtype=np.int8)
    hh = None if h is None else np.ascontiguousarray(h, dtype=np.float64)
    return lib.ref_energy_csr_f64(B.n, _ptr(B.rp), _ptr(B.col), _ptr(B.val), _ptr(hh), _ptr(s))


def energy_dense(J: np.ndarray, s: np.ndarray, h: Optional[np.ndarray] = None) -> float:
    lib = _load()
    J = np.ascontiguousarray(J, dtype=np.float64)
    s = np.ascontiguousarray(s, dtype=np.int8)
    hh = None if h is None else np.ascontiguousarray(h, dtype=np.float64)
    return lib.ref_energy_dense_f64(J.shape[0], _ptr(J), _ptr(hh), _ptr(s))


def energy_i64(B: OracleCSR, s: np.ndarray) -> int:
    """Exact -1/2 s^T J s for integer J; raises if J is not integral."""
    lib = _load()
    s = np.ascontiguousarray(s, dtype=np.int8)
    out = ctypes.c_int64(0)
    rc = lib.ref_energy_csr_i64(B.n, _ptr(B.rp), _ptr(B.col), _ptr(B.val), _ptr(s),
                                ctypes.addressof(out))
    if rc != 0:
        raise ValueError(f"integer energy unavailable (code {rc})")
    return int(out.value)


def bruteforce(J: np.ndarray, h: Optional[np.ndarray] = None):
    """(E_min, s_min) over all 2^n spin vectors (n <= 26)."""
    lib = _load()
    J = np.ascontiguousarray(J, dtype=np.float64)
    n = J.shape[0]
    if n > 26:
        raise ValueError("bruteforce limited to n <= 26")
    hh = None if h is None else np.ascontiguousarray(h, dtype=np.float64)
    s = np.empty(n, dtype=np.int8)
    E = lib.ref_bruteforce_dense(n, _ptr(J), _ptr(hh), _ptr(s))
    return E, s


def rowsum_max(B: OracleCSR) -> float:
    lib = _load()
    return lib.ref_offdiag_rowsum_max(B.n, _ptr(B.rp), _ptr(B.col), _ptr(B.val))


def wigner_lambda(B: OracleCSR) -> float:
    lib = _load()
    return lib.ref_wigner_lambda(B.n, _ptr(B.rp), _ptr(B.col), _ptr(B.val))


def power_lambda_max_neg(B: OracleCSR, v0: np.ndarray, tol: float = 1e-12,
                         maxit: int = 100000):
    lib = _load()
    v0 = np.ascontiguousarray(v0, dtype=np.float64)
    it = ctypes.c_int64(0)
    lam = lib.ref_power_lambda_max_neg(B.n, _ptr(B.rp), _ptr(B.col), _ptr(B.val), _ptr(v0),
                                       tol, maxit, ctypes.addressof(it))
    return lam, int(it.value)


def default_params(B: OracleCSR, eta: float = 1.0, method: str = "auto",
                   v0: Optional[np.ndarray] = None):
    """eq:alphabeta with Supp. Note 6: (alpha, beta, lambda_hat).

    lambda_hat = lambda_max(-J) by the power method for n < 1e4, else the
    Wigner estimate 2<J>sqrt(n); alpha = eta * lambda_hat;
    beta = n^{3/2} * (alpha + max_i sum_{j!=i} |J_ij|).  ``B`` is the
    homogeneous matrix (n counts the extra spin when there is a field).
    """
    n = B.n
    if method == "auto":
        method = "power" if n < 10000 else "wigner"
    if method == "power":
        if v0 is None:
            v0 = 2.0 * np.random.default_rng([7, n]).random(n) - 1.0
        lam, _ = power_lambda_max_neg(B, v0)
    elif method == "wigner":
        lam = wigner_lambda(B)
    else:
        raise ValueError(method)
    alpha = eta * lam
    beta = float(n) ** 1.5 * (alpha + rowsum_max(B))
    return alpha, beta, lam
