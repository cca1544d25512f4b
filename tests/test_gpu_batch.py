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
    """8 restarts per instance, many small instances (single-workgroup jobs
    of the default shape): every sampled (instance, restart) follows its own
    oracle run."""
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


# --------------------------------------------------- lockstep launch shapes
@pytest.fixture(scope="module")
def team_case():
    """Instances of 20000, 9000, 2600 and 700 rows (mean degrees 20, 12, 8,
    5) x 8 restarts, with the oracle's trajectories of 60 fixed iterations
    and of the eps = 1e-3 stopping rule for every (instance, restart)."""
    sizes = [(20000, 20.0), (9000, 12.0), (2600, 8.0), (700, 5.0)]
    inst = [gen.er_csr(n, d, 7100 + i) for i, (n, d) in enumerate(sizes)]
    alpha, beta = oracle_params(inst)
    R = 8
    total = sum(A.n for A in inst)
    X0 = gen.uniform_x0(total, R, 7200)
    offs = np.concatenate([[0], np.cumsum([A.n for A in inst])])
    fixed, stop = {}, {}
    for k, A in enumerate(inst):
        B = orc.to_oracle_csr(A)
        for r in range(R):
            x0 = X0[offs[k]:offs[k + 1], r]
            fixed[k, r] = orc.doch(B, x0, alpha[k], beta[k], 60)
            stop[k, r] = orc.doch(B, x0, alpha[k], beta[k], 5000, eps=1e-3)
    return dict(inst=inst, alpha=alpha, beta=beta, R=R, X0=X0, fixed=fixed, stop=stop)


@pytest.mark.parametrize("rj,wg,rpm", [(8, 256, 512), (8, 512, 4096), (4, 256, 500), (2, 1024, 2048),
                                       (1, 512, 3000), (8, 256, 100)])
def test_batch_team_shapes_parity(team_case, rj, wg, rpm):
    """Every launch shape: units of rj restarts, rows in chunks of rpm (the
    20000-row instance in 200 chunks at rpm 100, one chunk of 4096 rows
    covering the 700-row instance), spread over the workgroups of an XCD
    that exchange iterate rows through L2 each iteration.  Iterates,
    spins, H and r after 60 iterations follow the oracle per (instance,
    restart); under eps = 1e-3 every restart stops at the oracle's
    iteration; exact energies."""
    import paper_2509_01928_amd as L
    c = team_case
    inst, R = c["inst"], c["R"]
    G = GpuBatch(inst, R)
    try:
        L.ising_set_batch_shape(G.ctx, rj, wg, rpm)
        X, S, st, tts = G.solve(c["X0"], c["alpha"], c["beta"], 60, 0.0)
        E, Ei = G.energy(S)
        X2, S2, st2, tts2 = G.solve(c["X0"], c["alpha"], c["beta"], 5000, 1e-3)
    finally:
        G.close()
    for k, A in enumerate(inst):
        B = orc.to_oracle_csr(A)
        a, b = G.offs[k], G.offs[k + 1]
        for r in range(R):
            lab = f"shape ({rj}, {wg}, {rpm}) instance {k} (n={A.n}) restart {r}"
            tr = c["fixed"][k, r]
            assert_iterate_parity(X[a:b, r], tr.x, lab)
            assert_spin_parity(S[a:b, r], tr.x, orc.sign(tr.x), lab)
            s_ = st[k * R + r]
            assert s_.iters_done == 60 and not s_.converged, lab
            assert s_.H_last == pytest.approx(tr.H[-1], rel=1e-12), lab
            assert s_.r_last == pytest.approx(tr.r[-1], rel=1e-9, abs=1e-12), lab
            assert int(Ei[k * R + r]) == orc.energy_i64(B, S[a:b, r]), lab
            ts = c["stop"][k, r]
            s2 = st2[k * R + r]
            assert s2.iters_done == ts.iters and s2.converged == 1, lab
            assert_iterate_parity(X2[a:b, r], ts.x, lab + " (eps)")
    assert np.all(tts > 0) and np.all(tts2 > 0)


def test_batch_set_shape_rejects_unbuilt():
    import paper_2509_01928_amd as L
    inst = small_batch(count=2, seed=5)
    G = GpuBatch(inst, 8)
    try:
        for rj, wg, rpm in ((8, 1024, 512), (3, 256, 512), (4, 128, 512), (8, 256, 0)):
            with pytest.raises(L.IsingError) as e:
                L.ising_set_batch_shape(G.ctx, rj, wg, rpm)
            assert e.value.status == L.ISING_E_INVALID_ARG
        L.ising_set_batch_shape(G.ctx, 0, 0, 0)      # the default again
    finally:
        G.close()


def test_batch_autotune_and_cache(tmp_path):
    """The autotuner times every built shape, keeps the fastest, and writes
    it to the JSON cache; a second context over the same batch reads it back
    without timing; the tuned shape's solve follows the oracle."""
    import json
    import torch
    import paper_2509_01928_amd as L
    R = 4
    inst = gen.uneven_batch(count=24, seed=77, n_lo=200, n_hi=6000)
    alpha, beta = oracle_params(inst)
    total = sum(A.n for A in inst)
    X0 = gen.uniform_x0(total, R, 78)
    cache = str(tmp_path / "shapes.json")
    G = GpuBatch(inst, R)
    try:
        xd = torch.from_numpy(X0).to("cuda:0")
        shape, ms, cached = L.ising_autotune_batch(G.ctx, xd, R, 5000, alpha, beta, 1e-3, L.ISING_F64, cache)
        assert not cached and ms > 0
        assert shape[0] in (1, 2, 4) and shape[1] in (256, 512, 1024) and shape[2] in (256, 512, 1024, 2048)
        X, S, st, _ = G.solve(X0, alpha, beta, 5000, 1e-3)
    finally:
        G.close()
    with open(cache) as f:
        data = json.load(f)
    assert len(data) == 1
    (entry,) = data.values()
    assert (entry["rj"], entry["wg"], entry["chunk_rows"]) == tuple(shape)
    G2 = GpuBatch(inst, R)
    try:
        xd = torch.from_numpy(X0).to("cuda:0")
        shape2, ms2, cached2 = L.ising_autotune_batch(G2.ctx, xd, R, 5000, alpha, beta, 1e-3, L.ISING_F64,
                                                      cache)
    finally:
        G2.close()
    assert cached2 and tuple(shape2) == tuple(shape) and ms2 == pytest.approx(ms, rel=1e-3)
    for k in (0, 7, 23):
        A = inst[k]
        B = orc.to_oracle_csr(A)
        a, b = G.offs[k], G.offs[k + 1]
        for r in range(R):
            tr = orc.doch(B, X0[a:b, r], alpha[k], beta[k], 5000, eps=1e-3)
            assert st[k * R + r].iters_done == tr.iters, (k, r)
            assert_iterate_parity(X[a:b, r], tr.x, f"tuned shape {shape}: instance {k} restart {r}")
