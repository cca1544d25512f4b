"""The 9-bit integer workload (Supp. Alg. S5) with 16-bit integer coupling
values, and MAX-CUT values (Supp. Note 5) read back through the library."""
import numpy as np
import pytest

import ising_inputs as gen
import oracle as orc
from tests._util import GpuProblem, assert_iterate_parity, assert_log_parity, assert_spin_parity

pytestmark = pytest.mark.gpu


def cut_by_count(A, s):
    """Sum of w_ij = -J_ij over the edges i < j whose ends have opposite spins."""
    rows = np.repeat(np.arange(A.n), np.diff(A.row_ptr.astype(np.int64)))
    cols = A.col.astype(np.int64)
    upper = cols > rows
    cut = (s[rows[upper]] != s[cols[upper]])
    return int(-(A.val[upper].astype(np.int64) * cut).sum())


@pytest.mark.parametrize("geometry", [-1, 3, 4, 6])
def test_s5_int16_parity_energy_and_cut(geometry):
    """int16 values: same iterates as the FP64 oracle (the values are exact
    in both), exact int64 energies, and cut = -S_J / 4 - E / 2 equal to the
    cut counted edge by edge."""
    import paper_2509_01928_amd as L
    A = gen.s5_csr(3000, 1.0, 171)
    assert A.val.min() >= -510 and A.val.max() <= 511
    B = orc.to_oracle_csr(A)
    alpha, beta, _ = orc.default_params(B, 1.0)
    x0 = gen.uniform_x0(A.n, 1, 172)[:, 0]
    tr = orc.doch(B, x0, alpha, beta, 150)
    P = GpuProblem(A=A, val_dtype="i16")
    try:
        assert L.ising_get_info(P.ctx).val_dtype == L.ISING_I16
        assert L.ising_get_info(P.ctx).integer_J == 1
        L.ising_set_geometry(P.ctx, geometry, 0)
        x, s, st = P.solve(x0, alpha, beta, 150)
        H, r = P.log(150)
        rng = np.random.default_rng(173)
        S = np.where(rng.random((A.n, 5)) < 0.5, 1, -1).astype(np.int8)
        S[:, 0] = s[:, 0]
        E, Ei = P.energy(S, want_int=True)
        import torch
        sd = torch.from_numpy(S).to("cuda:0")
        cut = torch.empty(5, dtype=torch.float64, device="cuda:0")
        cut_i = torch.empty(5, dtype=torch.int64, device="cuda:0")
        L.ising_cut(P.ctx, sd, 5, cut, cut_i)
        cut, cut_i = cut.cpu().numpy(), cut_i.cpu().numpy()
    finally:
        P.close()
    assert_iterate_parity(x[:, 0], tr.x, f"S5 int16 geometry {geometry}")
    assert_spin_parity(s[:, 0], tr.x, orc.sign(tr.x), f"S5 int16 geometry {geometry}")
    assert_log_parity(H, r, tr, f"S5 int16 geometry {geometry}")
    for q in range(5):
        assert int(Ei[q]) == orc.energy_i64(B, S[:, q])
        want = cut_by_count(A, S[:, q])
        assert int(cut_i[q]) == want
        assert cut[q] == float(want)
        # Supp. Note 5 with w = -J: cut = W_tot / 2 - E / 2 in these units
        assert 4 * want == -int(A.val.astype(np.int64).sum()) - 2 * int(Ei[q])


def test_int16_lattice_with_field_and_adoch():
    """int16 couplings with an FP32 field (the extra spin), DOCH and ADOCH."""
    import paper_2509_01928_amd as L
    import torch
    A = gen.torus_csr(70, 181, h_std=0.1)
    B = orc.problem_matrix(A)
    alpha, beta, _ = orc.default_params(B, 1.0)
    x0 = gen.uniform_x0(A.n + 1, 1, 182)[:, 0]
    tr = orc.doch(B, x0, alpha, beta, 80)
    tra = orc.adoch(B, x0, alpha, beta, 30, 5)
    P = GpuProblem(A=A, val_dtype="i16")
    try:
        x, s, st = P.solve(x0, alpha, beta, 80)
        p = P.params(alpha, beta)
        p.algo, p.q = 1, 5
        xd = torch.from_numpy(x0).to("cuda:0")
        xo = torch.empty_like(xd)
        L.ising_solve(P.ctx, xd, 1, 30, p, xo, None)
        torch.cuda.synchronize()
        xa = xo.cpu().numpy()
        sd = torch.from_numpy(np.ones((A.n, 1), dtype=np.int8)).to("cuda:0")
        cut = torch.empty(1, dtype=torch.float64, device="cuda:0")
        with pytest.raises(L.IsingError):         # the cut is defined for h = 0
            L.ising_cut(P.ctx, sd, 1, cut)
    finally:
        P.close()
    assert_iterate_parity(x[:, 0], tr.x, "int16 lattice with field")
    assert_iterate_parity(xa, tra.x, "int16 lattice ADOCH")


def test_int16_refused_where_unsupported():
    import paper_2509_01928_amd as L
    import torch
    A = gen.er_csr(200, 4.0, 191)
    rp = torch.from_numpy(A.row_ptr).to("cuda:0")
    col = torch.from_numpy(A.col).to("cuda:0")
    val = torch.from_numpy(A.val.astype(np.int16)).to("cuda:0")
    with pytest.raises(L.IsingError):
        L.ising_create_batch([A.n], rp, col, val, L.ISING_I16)
    P = GpuProblem(A=A)                          # FP32 values that are integers
    try:
        s = torch.ones((A.n, 1), dtype=torch.int8, device="cuda:0")
        ci = torch.empty(1, dtype=torch.int64, device="cuda:0")
        L.ising_cut(P.ctx, s, 1, None, ci)       # all spins equal: no edge is cut
        assert int(ci.cpu()[0]) == 0
    finally:
        P.close()
