"""The single-launch (resident) solve against the launch-per-iteration
kernels and the oracle.

Both paths sum every row in ascending column order in FP64, so their
iterates must agree bit for bit; only the order in which the workgroups'
partial sums of H and r are added differs (H within 1e-12 relative).  Every
case is also held to the oracle's FP64 bar where the oracle is run.
"""
import numpy as np
import pytest

import ising_inputs as gen
import oracle as orc
from tests._util import (GpuProblem, assert_iterate_parity, assert_log_parity,
                         assert_spin_parity)

pytestmark = pytest.mark.gpu

RESIDENT = 8


def solve_with(P, geometry, x0, alpha, beta, iters, eps=0.0, x_dtype=None):
    P.L.ising_set_geometry(P.ctx, geometry, 0)
    x, s, st = P.solve(x0, alpha, beta, iters, eps=eps, x_dtype=x_dtype)
    H, r = P.log(st[0].iters_done)
    return x[:, 0], s[:, 0], st[0], H, r


def compare_paths(P, other, x0, alpha, beta, iters, label, eps=0.0, x_dtype=None):
    """Resident against geometry `other` on the same context."""
    xa, sa, sta, Ha, ra = solve_with(P, RESIDENT, x0, alpha, beta, iters, eps, x_dtype)
    xb, sb, stb, Hb, rb = solve_with(P, other, x0, alpha, beta, iters, eps, x_dtype)
    assert sta.iters_done == stb.iters_done, label
    assert sta.converged == stb.converged, label
    assert np.array_equal(xa, xb), f"{label}: iterates differ, max {np.abs(xa - xb).max():.3e}"
    assert np.array_equal(sa, sb), label
    scale = np.abs(Hb).max()
    assert np.abs(Ha - Hb).max() <= 1e-12 * scale, label
    assert np.abs(ra - rb).max() <= 1e-12 * max(np.abs(rb).max(), 1e-300), label
    return xa, sa, sta, Ha, ra


@pytest.mark.parametrize("x_dtype", ["f64", "f32"])
@pytest.mark.parametrize("case", ["er", "torus_field", "s5_int16", "er_long_rows"])
def test_resident_csr_matches_per_launch_and_oracle(case, x_dtype):
    import paper_2509_01928_amd as L
    xt = L.ISING_F64 if x_dtype == "f64" else L.ISING_F32
    val_dtype = "f32"
    if case == "er":
        A = gen.er_csr(3000, 6.0, 301)
        other, iters = 6, 300
    elif case == "torus_field":
        A = gen.torus_csr(64, 302, h_std=0.1)
        other, iters = 4, 200
    elif case == "s5_int16":
        A = gen.s5_csr(3000, 1.0, 303)
        other, iters, val_dtype = 3, 150, "i16"
    else:
        A = gen.er_csr(2000, 40.0, 304)        # rows longer than one 8-entry batch
        other, iters = 7, 150
    B = orc.problem_matrix(A)
    alpha, beta, _ = orc.default_params(B, 1.0, method="wigner")
    x0 = gen.uniform_x0(B.n, 1, 305)[:, 0]
    P = GpuProblem(A=A, val_dtype=val_dtype)
    try:
        x, s, st, H, r = compare_paths(P, other, x0, alpha, beta, iters, f"{case} {x_dtype}", x_dtype=xt)
    finally:
        P.close()
    if x_dtype == "f64":
        tr = orc.doch(B, x0, alpha, beta, iters)
        assert st.iters_done == tr.iters
        assert_iterate_parity(x, tr.x, case)
        s_ref = orc.spins_with_field(tr.x) if A.h is not None else orc.sign(tr.x)
        assert_spin_parity(s, tr.x, s_ref, case)
        assert_log_parity(H, r, tr, case)


@pytest.mark.parametrize("n,field,x_dtype", [(300, False, "f64"), (1024, False, "f64"),
                                             (1024, True, "f32"), (2048, False, "f64"),
                                             (1500, True, "f64"), (77, False, "f64")])
def test_resident_dense_matches_per_launch_and_oracle(n, field, x_dtype):
    """Dense rows of up to 1024 (16 register chunks) and 2048 (32) entries,
    ragged orders, with and without the extra field spin."""
    import paper_2509_01928_amd as L
    xt = L.ISING_F64 if x_dtype == "f64" else L.ISING_F32
    J = gen.sk_dense(n, 310 + n)
    h = np.random.default_rng(311).standard_normal(n) * 0.5 if field else None
    alpha = -np.linalg.eigvalsh(J)[0]
    rows = np.abs(J).sum(axis=1) + (np.abs(h) if field else 0.0)
    np_ = n + (1 if field else 0)
    rho = max(rows.max(), np.abs(h).sum()) if field else rows.max()
    beta = np_ ** 1.5 * (alpha + rho)
    x0 = gen.uniform_x0(np_, 1, 312)[:, 0]
    iters = 200
    P = GpuProblem(J=J, h=h)
    try:
        x, s, st, H, r = compare_paths(P, 0, x0, alpha, beta, iters, f"dense n={n}", x_dtype=xt)
    finally:
        P.close()
    if x_dtype == "f64":
        B = orc.augment_field(orc.csr_of_dense(J), h) if field else None
        tr = orc.doch(B, x0, alpha, beta, iters) if field else orc.doch_dense(J, x0, alpha, beta, iters)
        assert_iterate_parity(x, tr.x, f"dense n={n}")
        s_ref = orc.spins_with_field(tr.x) if field else orc.sign(tr.x)
        assert_spin_parity(s, tr.x, s_ref, f"dense n={n}")
        assert_log_parity(H, r, tr, f"dense n={n}")


def test_resident_early_stop_same_iteration():
    """The stop is seen one iteration late on the device; the iterate and the
    count must still be those of the iteration that converged."""
    A = gen.er_csr(4000, 8.0, 321)
    B = orc.problem_matrix(A)
    alpha, beta, _ = orc.default_params(B)
    x0 = gen.uniform_x0(4000, 1, 322)[:, 0]
    tr = orc.doch(B, x0, alpha, beta, 3000, eps=1e-3)
    assert tr.iters < 3000
    P = GpuProblem(A=A)
    try:
        x, s, st, H, r = compare_paths(P, 6, x0, alpha, beta, 3000, "eps", eps=1e-3)
        assert st.converged == 1 and st.iters_done == tr.iters
        assert_iterate_parity(x, tr.x, "eps")
        # a second solve on the same context starts clean
        x2, s2, st2, _, _ = solve_with(P, RESIDENT, x0, alpha, beta, 3000, eps=1e-3)
        assert np.array_equal(x, x2) and st2.iters_done == st.iters_done
    finally:
        P.close()


def test_resident_dense_early_stop_and_zero_iterations():
    n = 512
    J = gen.sk_dense(n, 331)
    alpha = -np.linalg.eigvalsh(J)[0]
    beta = n ** 1.5 * (alpha + np.abs(J).sum(axis=1).max())
    x0 = gen.uniform_x0(n, 1, 332)[:, 0]
    tr = orc.doch_dense(J, x0, alpha, beta, 5000, eps=1e-4)
    P = GpuProblem(J=J)
    try:
        x, s, st, H, r = compare_paths(P, 0, x0, alpha, beta, 5000, "dense eps", eps=1e-4)
        assert st.iters_done == tr.iters and st.converged == (1 if tr.iters < 5000 else 0)
        assert_iterate_parity(x, tr.x, "dense eps")
        x0z, _, st0, _, _ = solve_with(P, RESIDENT, x0, alpha, beta, 0)
        assert st0.iters_done == 0 and np.array_equal(x0z, x0)
    finally:
        P.close()


def test_resident_many_rows_per_lane():
    """More rows than lanes of 255 row workgroups: each lane walks several."""
    n = 200_000
    A = gen.er_csr(n, 5.0, 341)
    B = orc.problem_matrix(A)
    alpha, beta, _ = orc.default_params(B, 1.0, method="wigner")
    x0 = gen.uniform_x0(n, 1, 342)[:, 0]
    tr = orc.doch(B, x0, alpha, beta, 40)
    P = GpuProblem(A=A)
    try:
        x, s, st, H, r = compare_paths(P, 6, x0, alpha, beta, 40, "n=2e5")
    finally:
        P.close()
    assert_iterate_parity(x, tr.x, "n=2e5")
    assert_log_parity(H, r, tr, "n=2e5")


def test_resident_geometry_rules():
    import paper_2509_01928_amd as L
    J = gen.sk_dense(64, 351)
    P = GpuProblem(J=J)
    try:
        for g in (-1, 0, RESIDENT):
            L.ising_set_geometry(P.ctx, g, 0)
        with pytest.raises(L.IsingError) as e:
            L.ising_set_geometry(P.ctx, 3, 0)
        assert e.value.status == L.ISING_E_INVALID_ARG
    finally:
        P.close()
    Jb = gen.sk_dense(3000, 352)
    P = GpuProblem(J=Jb)
    try:
        with pytest.raises(L.IsingError) as e:
            L.ising_set_geometry(P.ctx, RESIDENT, 0)
        assert e.value.status == L.ISING_E_UNSUPPORTED
    finally:
        P.close()
