"""The allocation-free energy entry point against ising_energy.

ising_energy_noalloc launches the same kernels as ising_energy with its
partial sums in the library's static device array.  Each case calls both
through the C ABI on the same spins and compares them (int64 energies bit
for bit, FP64 energies to 1e-12 relative, and both against the oracle's
eq:IsingModel), twice in a row, the second call on a smaller input, so the
array's leftovers from the first call must not leak into the second.
"""
import ctypes

import numpy as np
import pytest

import ising_inputs as gen
import oracle as orc
from tests._util import GpuProblem

pytestmark = pytest.mark.gpu


def _spins(n, R, seed):
    rng = np.random.default_rng(seed)
    return np.where(rng.random((n, R)) < 0.5, 1, -1).astype(np.int8)


def _both(L, ctx, S, want_int):
    import torch
    n, R = S.shape
    sd = torch.from_numpy(np.ascontiguousarray(S)).to("cuda:0")
    out = {}
    for name, fn in (("alloc", L.ising_energy), ("noalloc", L.ising_energy_noalloc)):
        E = torch.full((R,), float("nan"), dtype=torch.float64, device="cuda:0")
        Ei = torch.full((R,), -7, dtype=torch.int64, device="cuda:0") if want_int else None
        fn(ctx, sd, R, E, Ei)
        torch.cuda.synchronize()
        out[name] = (E.cpu().numpy(), None if Ei is None else Ei.cpu().numpy())
    return out


def _compare(out, E_ref, Ei_ref, label):
    Ea, Eia = out["alloc"]
    En, Ein = out["noalloc"]
    assert np.all(np.isfinite(En)), label
    np.testing.assert_allclose(En, Ea, rtol=1e-12, atol=1e-9, err_msg=label)
    np.testing.assert_allclose(En, E_ref, rtol=1e-11, atol=1e-9, err_msg=label)
    if Ei_ref is not None:
        assert np.array_equal(Ein, Eia), label
        assert np.array_equal(Ein, Ei_ref), label


def test_noalloc_energy_csr_integer_two_calls():
    """Integer couplings, no field: the generic kernel (R = 13) on the larger
    instance, then the eight-lane kernel (R = 5) on a smaller one."""
    import paper_2509_01928_amd as L
    for n, R, seed in ((70_000, 13, 1201), (5_000, 5, 1202)):
        A = gen.er_csr(n, 6.0, seed)
        B = orc.to_oracle_csr(A)
        S = _spins(n, R, seed + 1)
        P = GpuProblem(A=A)
        try:
            out = _both(L, P.ctx, S, want_int=True)
        finally:
            P.close()
        E_ref = np.array([orc.energy(A, S[:, r]) for r in range(R)])
        Ei_ref = np.array([orc.energy_i64(B, S[:, r]) for r in range(R)])
        _compare(out, E_ref, Ei_ref, f"ER n={n} R={R}")


def test_noalloc_energy_csr_field_two_calls():
    """A lattice with a field (FP64 energy only), R = 1 then R = 1 on a
    smaller lattice."""
    import paper_2509_01928_amd as L
    for Lside, seed in ((300, 1203), (40, 1204)):
        A = gen.torus_csr(Lside, seed, h_std=0.1)
        S = _spins(A.n, 1, seed + 1)
        P = GpuProblem(A=A)
        try:
            out = _both(L, P.ctx, S, want_int=False)
        finally:
            P.close()
        _compare(out, np.array([orc.energy(A, S[:, 0])]), None, f"torus L={Lside}")


def test_noalloc_energy_dense_and_procedural_two_calls():
    """Stored dense couplings with a field (tiled kernel, R = 70), then a
    smaller generated instance sin(ij + 7) (R = 13)."""
    import paper_2509_01928_amd as L
    n, R = 500, 70
    J = gen.sk_dense(n, 1205)
    h = np.random.default_rng(1206).normal(0.0, 0.3, n)
    S = _spins(n, R, 1207)
    P = GpuProblem(J=J, h=h)
    try:
        out = _both(L, P.ctx, S, want_int=False)
    finally:
        P.close()
    _compare(out, np.array([orc.energy_dense(J, S[:, r], h) for r in range(R)]), None, "dense n=500")

    n, R, seed = 333, 13, 7.0
    i = np.arange(n, dtype=np.float64)
    Jp = np.sin(np.outer(i, i) + seed)
    np.fill_diagonal(Jp, 0.0)
    S = _spins(n, R, 1208)
    ctx = L.ising_create_procedural(n, 1, seed)
    try:
        out = _both(L, ctx, S, want_int=False)
    finally:
        L.ising_destroy(ctx)
    _compare(out, np.array([orc.energy_dense(Jp, S[:, r]) for r in range(R)]), None, "procedural n=333")


def test_noalloc_energy_rejects_oversize():
    """More partial sums than the static array holds: refused before any
    launch (R = 171 restarts of a CSR instance with at least 262 144 rows),
    while ising_energy still serves the call."""
    import torch
    import paper_2509_01928_amd as L
    A = gen.torus_csr(520, 1209)
    R = 171
    S = _spins(A.n, R, 1210)
    P = GpuProblem(A=A)
    try:
        sd = torch.from_numpy(S).to("cuda:0")
        E = torch.empty(R, dtype=torch.float64, device="cuda:0")
        st = L.lib.ising_energy_noalloc(P.ctx, ctypes.c_void_p(sd.data_ptr()), R,
                                        ctypes.c_void_p(E.data_ptr()), None, L.current_stream())
        assert st == L.ISING_E_INVALID_ARG
        assert b"static scratch" in L.lib.ising_last_error()
        L.ising_energy(P.ctx, sd, R, E)
        torch.cuda.synchronize()
        Ec = E.cpu().numpy()
    finally:
        P.close()
    for r in (0, R - 1):
        assert Ec[r] == pytest.approx(orc.energy(A, S[:, r]), rel=1e-12, abs=1e-9)
