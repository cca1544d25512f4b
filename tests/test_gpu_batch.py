"""GPU batch path (many instances x many restarts in one persistent launch)
against the oracle, which runs every (instance, restart) on its own.

Bars as for the single-instance FP64 path: iterates within 1e-9 max abs and
relative to |x|_inf, spins identical except |x_i| < 1e-6 |x|_inf, identical
iteration counts under the Remark S2 stopping rule, H within 1e-12 relative,
exact integer energies.  alpha and beta come from the oracle.
"""
import numpy as np
import pytest

import ising_inputs as gen
import oracle as orc
from tests._util import (assert_fp32_storage_parity, assert_iterate_parity, assert_spin_parity,
                         oracle_fp32_storage)

pytestmark = pytest.mark.gpu


def concat_batch(instances):
    """Block-diagonal CSR of a list of instances (global column indices)."""
    rps, cols, vals = [np.zeros(1, np.int64)], [], []
    row0 = 0
    nnz0 = 0
    for A in instances:
        rps.append(A.row_ptr[1:].astype(np.int64) + nnz0)
        cols.append(A.col.astype(np.int64) + row0)
        vals.append(A.val)
        row0 += A.n
        nnz0 += A.nnz
    rp = np.concatenate(rps).astype(np.int32)
    col = np.concatenate(cols).astype(np.int32)
    val = np.concatenate(vals).astype(np.float32)
    return rp, col, val


class GpuBatch:
    def __init__(self, instances, R):
        import torch
        import paper_2509_01928_amd as L
        self.L, self.torch, self.R = L, torch, R
        self.instances = instances
        self.ns = [A.n for A in instances]
        self.offs = np.concatenate([[0], np.cumsum(self.ns)])
        rp, col, val = concat_batch(instances)
        d = "cuda:0"
        self.keep = [torch.from_numpy(rp).to(d), torch.from_numpy(col).to(d),
                     torch.from_numpy(val).to(d)]
        self.ctx = L.ising_create_batch(self.ns, *self.keep, L.ISING_F32)

    def solve(self, X0, alpha, beta, iters, eps, x_dtype=None):
        torch, L = self.torch, self.L
        xd = torch.from_numpy(np.ascontiguousarray(X0)).to("cuda:0")
        xo = torch.empty_like(xd)
        so = torch.empty(xd.shape, dtype=torch.int8, device="cuda:0")
        st, tts = L.ising_solve_batch(self.ctx, xd, self.R, iters, alpha, beta, eps,
                                      L.ISING_F64 if x_dtype is None else x_dtype, xo, so)
        torch.cuda.synchronize()
        return xo.cpu().numpy(), so.cpu().numpy(), st, tts

    def energy(self, S, want_int=True):
        torch = self.torch
        sd = torch.from_numpy(np.ascontiguousarray(S, dtype=np.int8)).to("cuda:0")
        count = len(self.ns)
        E = torch.empty(count * self.R, dtype=torch.float64, device="cuda:0")
        Ei = torch.empty(count * self.R, dtype=torch.int64, device="cuda:0") if want_int else None
        self.L.ising_energy_batch(self.ctx, sd, self.R, E, Ei)
        torch.cuda.synchronize()
        return E.cpu().numpy(), (Ei.cpu().numpy() if want_int else None)

    def close(self):
        self.L.ising_destroy(self.ctx)


def oracle_params(instances):
    out = [orc.default_params(orc.to_oracle_csr(A), 1.0, method="wigner") for A in instances]
    return np.array([o[0] for o in out]), np.array([o[1] for o in out])


def small_batch(count=9, seed=4242, n_lo=300, n_hi=2500):
    return gen.uneven_batch(count=count, seed=seed, n_lo=n_lo, n_hi=n_hi)


@pytest.mark.parametrize("R", [1, 2, 8, 32])
def test_batch_fixed_iterations_parity(R):
    inst = small_batch()
    alpha, beta = oracle_params(inst)
    total = sum(A.n for A in inst)
    X0 = gen.uniform_x0(total, R, 77 + R)
    G = GpuBatch(inst, R)
    try:
        X, S, st, tts = G.solve(X0, alpha, beta, 120, 0.0)
        E, Ei = G.energy(S)
    finally:
        G.close()
    for k, A in enumerate(inst):
        B = orc.to_oracle_csr(A)
        a, b = G.offs[k], G.offs[k + 1]
        for r in range(R):
            tr = orc.doch(B, X0[a:b, r], alpha[k], beta[k], 120)
            lab = f"instance {k} restart {r}"
            assert_iterate_parity(X[a:b, r], tr.x, lab)
            assert_spin_parity(S[a:b, r], tr.x, orc.sign(tr.x), lab)
            s_ = st[k * R + r]
            assert s_.iters_done == 120 and not s_.converged
            assert s_.H_last == pytest.approx(tr.H[-1], rel=1e-12)
            assert s_.r_last == pytest.approx(tr.r[-1], rel=1e-9, abs=1e-12)
            assert int(Ei[k * R + r]) == orc.energy_i64(B, S[a:b, r])
            assert E[k * R + r] == float(Ei[k * R + r])
    assert np.all(tts > 0)


@pytest.mark.parametrize("count", [300, 150, 64, 9])
def test_batch_restart_groups_parity(count):
    """8 restarts per instance, split into jobs of 8, 4, 2 or 1 restarts
    depending on how many instances there are (one job per CU at least):
    every sampled (instance, restart) follows its own oracle run."""
    R = 8
    inst = gen.uneven_batch(count=count, seed=500 + count, n_lo=40, n_hi=160, d_lo=3.0, d_hi=9.0)
    alpha, beta = oracle_params(inst)
    total = sum(A.n for A in inst)
    X0 = gen.uniform_x0(total, R, 600 + count)
    G = GpuBatch(inst, R)
    try:
        X, S, st, tts = G.solve(X0, alpha, beta, 60, 0.0)
    finally:
        G.close()
    for k in sorted({0, count // 3, count // 2, count - 1}):
        A = inst[k]
        B = orc.to_oracle_csr(A)
        a, b = G.offs[k], G.offs[k + 1]
        for r in range(R):
            tr = orc.doch(B, X0[a:b, r], alpha[k], beta[k], 60)
            lab = f"{count} instances: instance {k} restart {r}"
            assert_iterate_parity(X[a:b, r], tr.x, lab)
            assert st[k * R + r].iters_done == 60
            assert st[k * R + r].H_last == pytest.approx(tr.H[-1], rel=1e-12)
    assert np.all(tts > 0)


def test_batch_early_stop_per_restart():
    """Remark S2 per restart: every (instance, restart) stops exactly where
    the oracle run of that restart alone stops."""
    R = 8
    inst = small_batch(count=6, seed=99)
    alpha, beta = oracle_params(inst)
    total = sum(A.n for A in inst)
    X0 = gen.uniform_x0(total, R, 5)
    G = GpuBatch(inst, R)
    try:
        X, S, st, tts = G.solve(X0, alpha, beta, 5000, 1e-3)
    finally:
        G.close()
    for k, A in enumerate(inst):
        B = orc.to_oracle_csr(A)
        a, b = G.offs[k], G.offs[k + 1]
        for r in range(R):
            tr = orc.doch(B, X0[a:b, r], alpha[k], beta[k], 5000, eps=1e-3)
            s_ = st[k * R + r]
            assert s_.iters_done == tr.iters and s_.converged == 1, (k, r)
            assert_iterate_parity(X[a:b, r], tr.x, f"instance {k} restart {r}")
    assert np.all(tts > 0)


def test_batch_fp32_storage_and_replay():
    """FP32 iterate storage, and two solves in a row replay one captured graph
    with identical results."""
    import paper_2509_01928_amd as L
    R = 4
    inst = small_batch(count=5, seed=7)
    alpha, beta = oracle_params(inst)
    total = sum(A.n for A in inst)
    X0 = gen.uniform_x0(total, R, 6)
    G = GpuBatch(inst, R)
    try:
        X1, S1, st1, _ = G.solve(X0, alpha, beta, 80, 0.0, x_dtype=L.ISING_F32)
        X2, S2, st2, _ = G.solve(X0, alpha, beta, 80, 0.0, x_dtype=L.ISING_F32)
    finally:
        G.close()
    np.testing.assert_array_equal(X1, X2)
    np.testing.assert_array_equal(S1, S2)
    for k, A in enumerate(inst):
        B = orc.to_oracle_csr(A)
        a, b = G.offs[k], G.offs[k + 1]
        for r in range(R):
            xe, _ = oracle_fp32_storage(B, X0[a:b, r], alpha[k], beta[k], 80)
            assert_fp32_storage_parity(X1[a:b, r], xe, f"instance {k} restart {r}")


def test_batch_default_params_match_oracle():
    import paper_2509_01928_amd as L
    inst = gen.uneven_batch(count=4, seed=31, n_lo=1500, n_hi=12000)
    G = GpuBatch(inst, 1)
    try:
        a, b, lam = L.ising_default_params_batch(G.ctx, len(inst), 1.0, 0)
    finally:
        G.close()
    for k, A in enumerate(inst):
        B = orc.to_oracle_csr(A)
        if A.n >= 10000:
            a_ref, b_ref, lam_ref = orc.default_params(B, 1.0, method="wigner")
            assert lam[k] == pytest.approx(lam_ref, rel=1e-12)
            assert b[k] == pytest.approx(b_ref, rel=1e-12)
        else:
            lam_true = -np.linalg.eigvalsh(gen.dense_from_csr(A))[0]
            assert lam[k] == pytest.approx(lam_true, rel=1e-6)
        assert a[k] == pytest.approx(lam[k], rel=1e-15)


def test_batch_rejects_cross_block_coupling():
    import torch
    import paper_2509_01928_amd as L
    inst = small_batch(count=2, seed=3)
    rp, col, val = concat_batch(inst)
    col = col.copy()
    col[rp[1] - 1] = inst[0].n + 1   # row 0 of instance 0 couples into instance 1
    d = "cuda:0"
    with pytest.raises(L.IsingError) as e:
        L.ising_create_batch([A.n for A in inst], torch.from_numpy(rp).to(d),
                             torch.from_numpy(col).to(d), torch.from_numpy(val).to(d), L.ISING_F32)
    assert e.value.status == L.ISING_E_INVALID_ARG
