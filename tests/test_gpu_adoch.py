"""ADOCH (Alg. 2) on dense stored and generated couplings and over several
restarts at once, against the oracle's ADOCH run of each restart alone.

The GPU forms J y from J x^(k) and J x^(k-1) (one matvec per iteration),
the oracle by its own matvec, so where H(y^(k)) ties the window maximum to
within rounding either decision is a valid run of Alg. 2; everywhere else
the decisions must be the same, the logs must agree up to the first
decision taken the other way, and both runs must end at the same point.
"""
import numpy as np
import pytest

import ising_inputs as gen
import oracle as orc
from tests._util import H_RTOL, assert_iterate_parity, assert_spin_parity

pytestmark = pytest.mark.gpu

TIE_RTOL = 1e-11


# r^(k) of a run on dense couplings: the GPU sums a dense row lane-strided
# (then across the wavefront), the oracle in ascending column order, and the
# momentum step of Alg. 2 transiently amplifies that rounding difference in
# the step length (about 1e-7 relative at worst in the seeded cases), while
# H, the decisions and the end point agree at the strict bars.
R_RTOL_DENSE = 1e-6


def check_run(label, tr, x, s, H, r, acc, iters, field, end_fixed_point=True, r_rtol=1e-9):
    clear = np.abs(tr.Hy - tr.Hmax) > TIE_RTOL * (np.abs(tr.Hy) + np.abs(tr.Hmax))
    assert acc[0] == tr.accept[0] == 1, label
    np.testing.assert_array_equal(acc[clear], tr.accept[clear], err_msg=label)
    diff = np.nonzero(acc != tr.accept)[0]
    m = int(diff[0]) if diff.size else len(tr.H)
    Hs = float(np.abs(tr.H).max())
    assert np.abs(H[:m + 1] - tr.H[:m + 1]).max() <= H_RTOL * Hs, label
    dr = np.abs(r[:m] - tr.r[:m])
    assert np.all(dr <= 1e-12 + r_rtol * np.abs(tr.r[:m])), label
    if end_fixed_point:
        # both runs at the fixed point, where the iterates no longer carry
        # the amplified rounding of the transient
        assert r[-1] < 1e-10 and tr.r[-1] < 1e-10, (label, r[-1], tr.r[-1])
    if end_fixed_point or m == len(tr.H):
        assert_iterate_parity(x, tr.x, label)
        s_ref = orc.spins_with_field(tr.x) if field else orc.sign(tr.x)
        assert_spin_parity(s, tr.x, s_ref, label)


def run_gpu(ctx, L, x0, R, iters, alpha, beta, q, eps, np_rows, n):
    import torch
    p = L.ising_params()
    p.alpha, p.beta, p.eps, p.algo, p.q, p.x_dtype, p.reserved = alpha, beta, eps, 1, q, L.ISING_F64, 0
    xd = torch.from_numpy(np.ascontiguousarray(x0.reshape(np_rows, R))).to("cuda:0")
    xo = torch.empty_like(xd)
    so = torch.empty((n, R), dtype=torch.int8, device="cuda:0")
    st = L.ising_solve(ctx, xd, R, iters, p, xo, so)
    done = max(s_.iters_done for s_ in st)
    logs = [L.ising_get_log(ctx, rr, 0, done) for rr in range(R)]
    acc = L.ising_get_accept_log(ctx, 0, done, R).reshape(done, R)
    torch.cuda.synchronize()
    return xo.cpu().numpy(), so.cpu().numpy(), st, logs, acc


def dense_case(n, seed, field):
    J = gen.sk_dense(n, seed)
    h = np.random.default_rng(seed + 1).normal(0.0, 0.3, n) if field else None
    B = orc.csr_of_dense(J)
    if field:
        B = orc.augment_field(B, h)
    return J, h, B


@pytest.mark.parametrize("field", [False, True])
@pytest.mark.parametrize("R", [1, 4])
def test_adoch_dense_stored(R, field):
    """Dense SK couplings (n = 500), with and without the field's extra spin,
    one and four restarts."""
    import torch
    import paper_2509_01928_amd as L
    n, iters, q = 500, 400, 5
    J, h, B = dense_case(n, 7301 + R, field)
    alpha, beta, _ = orc.default_params(B, 1.0, method="power")
    npr = B.n
    X0 = gen.uniform_x0(npr, R, 7310 + R)
    Jd = torch.from_numpy(J).to("cuda:0")
    hd = torch.from_numpy(h).to("cuda:0") if field else None
    ctx = L.ising_create_dense(n, Jd, L.ISING_F64, n, hd, L.ISING_F64)
    try:
        x, s, st, logs, acc = run_gpu(ctx, L, X0, R, iters, alpha, beta, q, 0.0, npr, n)
    finally:
        L.ising_destroy(ctx)
    for rr in range(R):
        tr = orc.adoch(B, X0[:, rr], alpha, beta, iters, q)
        assert st[rr].iters_done == iters
        check_run(f"dense n={n} field={field} restart {rr}", tr, x[:, rr], s[:, rr], logs[rr][0], logs[rr][1],
                  acc[:, rr], iters, field, r_rtol=R_RTOL_DENSE)


@pytest.mark.parametrize("n,iters,R", [(1024, 600, 1), (1500, 300, 1), (1024, 300, 8)])
def test_adoch_dense_resident_and_launches(n, iters, R):
    """One restart on stored dense couplings without a field runs resident
    (one cooperative launch: every workgroup takes the acceptance decision
    from the same sums; x^(k+1) = T(y) written before it, T(x) rewritten on
    rejection); geometry 0, and more restarts, take a launch per step.  Both
    against the oracle's ADOCH per restart (n = 1024: 16 row chunks per
    lane; n = 1500: 32, the last one ragged; eight restarts with their own
    windows on the launches)."""
    import torch
    import paper_2509_01928_amd as L
    q = 5
    J, h, B = dense_case(n, 7350 + n, False)
    alpha, beta, _ = orc.default_params(B, 1.0, method="power")
    X0 = gen.uniform_x0(n, R, 7351 + n)
    trs = [orc.adoch(B, X0[:, rr], alpha, beta, iters, q) for rr in range(R)]
    assert any((t.accept == 0).any() for t in trs), "the seeded case should reject y at least once"
    Jd = torch.from_numpy(J).to("cuda:0")
    for geometry in (-1, 0):
        ctx = L.ising_create_dense(n, Jd, L.ISING_F64, n)
        try:
            L.ising_set_geometry(ctx, geometry, 0)
            x, s, st, logs, acc = run_gpu(ctx, L, X0, R, iters, alpha, beta, q, 0.0, n, n)
        finally:
            L.ising_destroy(ctx)
        for rr in range(R):
            assert st[rr].iters_done == iters
            check_run(f"dense n={n} R={R} geometry {geometry} restart {rr}", trs[rr], x[:, rr], s[:, rr],
                      logs[rr][0], logs[rr][1], acc[:, rr], iters, False, r_rtol=R_RTOL_DENSE)


def test_adoch_dense_restarts_stop_each_on_its_own():
    """Four restarts on stored dense couplings under eps = 1e-3: each stops
    at its own oracle iteration and keeps its iterate while the others go
    on."""
    import torch
    import paper_2509_01928_amd as L
    n, R, q = 600, 4, 5
    J, h, B = dense_case(n, 7370, False)
    alpha, beta, _ = orc.default_params(B, 1.0, method="power")
    X0 = gen.uniform_x0(n, R, 7371)
    trs = [orc.adoch(B, X0[:, rr], alpha, beta, 3000, q, eps=1e-3) for rr in range(R)]
    assert len({t.iters for t in trs}) > 1, "the seeded restarts should stop at different iterations"
    Jd = torch.from_numpy(J).to("cuda:0")
    ctx = L.ising_create_dense(n, Jd, L.ISING_F64, n)
    try:
        x, s, st, logs, acc = run_gpu(ctx, L, X0, R, 3000, alpha, beta, q, 1e-3, n, n)
    finally:
        L.ising_destroy(ctx)
    for rr in range(R):
        k = trs[rr].iters
        assert st[rr].iters_done == k and st[rr].converged == 1, rr
        check_run(f"dense restart {rr}", trs[rr], x[:, rr], s[:, rr], logs[rr][0][:k], logs[rr][1][:k],
                  acc[:k, rr], k, False, end_fixed_point=False, r_rtol=R_RTOL_DENSE)


def test_adoch_dense_resident_stops_with_oracle():
    """eps = 1e-3: the resident run stops at the oracle's iteration, every
    workgroup at the same one, and returns that iteration's iterate."""
    import torch
    import paper_2509_01928_amd as L
    n, q = 800, 5
    J, h, B = dense_case(n, 7360, False)
    alpha, beta, _ = orc.default_params(B, 1.0, method="power")
    X0 = gen.uniform_x0(n, 1, 7361)
    tr = orc.adoch(B, X0[:, 0], alpha, beta, 3000, q, eps=1e-3)
    assert tr.iters < 3000
    Jd = torch.from_numpy(J).to("cuda:0")
    ctx = L.ising_create_dense(n, Jd, L.ISING_F64, n)
    try:
        x, s, st, logs, acc = run_gpu(ctx, L, X0, 1, 3000, alpha, beta, q, 1e-3, n, n)
    finally:
        L.ising_destroy(ctx)
    assert st[0].iters_done == tr.iters and st[0].converged == 1
    k = tr.iters
    check_run("dense n=800 eps", tr, x[:, 0], s[:, 0], logs[0][0][:k], logs[0][1][:k], acc[:k, 0], k, False,
              end_fixed_point=False, r_rtol=R_RTOL_DENSE)


@pytest.mark.parametrize("R", [1, 8])
def test_adoch_procedural(R):
    """Couplings sin(i j + 7) generated on the fly (n = 700), against the
    oracle on the materialised matrix."""
    import paper_2509_01928_amd as L
    n, seed, iters, q = 700, 7.0, 400, 5
    i = np.arange(n, dtype=np.float64)
    Jp = np.sin(np.outer(i, i) + seed)
    np.fill_diagonal(Jp, 0.0)
    B = orc.csr_of_dense(Jp)
    alpha, beta, _ = orc.default_params(B, 1.0, method="power")
    X0 = gen.uniform_x0(n, R, 7320 + R)
    ctx = L.ising_create_procedural(n, 1, seed)
    try:
        x, s, st, logs, acc = run_gpu(ctx, L, X0, R, iters, alpha, beta, q, 0.0, n, n)
    finally:
        L.ising_destroy(ctx)
    for rr in range(R):
        tr = orc.adoch(B, X0[:, rr], alpha, beta, iters, q)
        check_run(f"procedural restart {rr}", tr, x[:, rr], s[:, rr], logs[rr][0], logs[rr][1], acc[:, rr],
                  iters, False, r_rtol=R_RTOL_DENSE)


def test_adoch_csr_restarts_stop_each_on_its_own():
    """Four restarts on a sparse random graph under eps = 1e-3: each stops
    at the iteration its own oracle run stops, and keeps its iterate while
    the others go on."""
    import paper_2509_01928_amd as L
    from tests._util import GpuProblem
    A = gen.er_csr(2500, 6.0, 7331)
    B = orc.problem_matrix(A)
    alpha, beta, _ = orc.default_params(B, 1.0)
    R, q = 4, 5
    X0 = gen.uniform_x0(A.n, R, 7332)
    trs = [orc.adoch(B, X0[:, rr], alpha, beta, 3000, q, eps=1e-3) for rr in range(R)]
    assert len({t.iters for t in trs}) > 1, "the seeded restarts should stop at different iterations"
    P = GpuProblem(A=A)
    try:
        x, s, st, logs, acc = run_gpu(P.ctx, L, X0, R, 3000, alpha, beta, q, 1e-3, A.n, A.n)
    finally:
        P.close()
    for rr in range(R):
        assert st[rr].iters_done == trs[rr].iters and st[rr].converged == 1, rr
        k = trs[rr].iters
        check_run(f"ER restart {rr}", trs[rr], x[:, rr], s[:, rr], logs[rr][0][:k], logs[rr][1][:k],
                  acc[:k, rr], k, False, end_fixed_point=False)


def test_adoch_csr_rejections_mixed_across_restarts():
    """The CSR product writes x^(k+1) = T(y) before the acceptance test and
    a second launch repairs only the restarts whose y was rejected.  With
    eta = 0.25 the lattice with its field rejects y often before H settles,
    in different iterations for different restarts: every restart must
    follow its own oracle run through those iterations (field spin
    included) and reach the same fixed point."""
    import paper_2509_01928_amd as L
    from tests._util import GpuProblem
    A = gen.torus_csr(40, 133, h_std=0.1)
    B = orc.problem_matrix(A)
    alpha, beta, _ = orc.default_params(B, 0.25)
    R, q, iters = 4, 5, 300
    X0 = gen.uniform_x0(B.n, R, 135)
    trs = [orc.adoch(B, X0[:, rr], alpha, beta, iters, q) for rr in range(R)]
    clear = [np.abs(t.Hy - t.Hmax) > TIE_RTOL * (np.abs(t.Hy) + np.abs(t.Hmax)) for t in trs]
    rej = np.array([(t.accept == 0) & c for t, c in zip(trs, clear)])
    assert all(rj.sum() >= 10 for rj in rej), "the seeded restarts should reject y often"
    assert (rej.any(axis=0) & ~rej.all(axis=0)).sum() >= 10, "rejections should differ across restarts"
    P = GpuProblem(A=A)
    try:
        x, s, st, logs, acc = run_gpu(P.ctx, L, X0, R, iters, alpha, beta, q, 0.0, B.n, A.n)
    finally:
        P.close()
    for rr in range(R):
        assert st[rr].iters_done == iters, rr
        check_run(f"lattice restart {rr}", trs[rr], x[:, rr], s[:, rr], logs[rr][0], logs[rr][1],
                  acc[:, rr], iters, True)


@pytest.mark.parametrize("values,val_bytes", [("pm1", 1), ("int8", 1), ("frac", 4)])
def test_adoch_lattice_rows_per_lane(values, val_bytes):
    """The lattice with its field at 409 600 rows: the product on rows of 4
    entries runs two (FP32 values), three (8-bit values) or four (8-bit
    values and 16-bit column offsets) workgroups per CU, at most 262 144
    lanes, so every lane walks several rows;
    30 iterations against the oracle's ADOCH (decisions, H and r logs,
    iterates).  Couplings +-1 or integers over [-128, 127] (the product
    streams the library's 8-bit copy), or 0.37 * (+-1) (the FP32 values)."""
    import paper_2509_01928_amd as L
    from tests._util import GpuProblem
    A = gen.torus_csr(640, 7381, h_std=0.1)
    if values == "int8":
        rows = np.repeat(np.arange(A.n, dtype=np.int64), np.diff(A.row_ptr))
        a, b = np.minimum(rows, A.col.astype(np.int64)), np.maximum(rows, A.col.astype(np.int64))
        A.val = ((((a * 2654435761 + b * 40503) >> 9) % 256) - 128).astype(np.float32)
    elif values == "frac":
        A.val = A.val * np.float32(0.37)
    B = orc.problem_matrix(A)
    alpha, beta, _ = orc.default_params(B, 1.0)
    q, iters = 5, 30
    X0 = gen.uniform_x0(B.n, 1, 7382)
    tr = orc.adoch(B, X0[:, 0], alpha, beta, iters, q)
    P = GpuProblem(A=A)
    try:
        info = L.ising_get_info(P.ctx)
        assert info.step_val_bytes == val_bytes and info.step_col_bytes == (2 if val_bytes == 1 else 4)
        x, s, st, logs, acc = run_gpu(P.ctx, L, X0, 1, iters, alpha, beta, q, 0.0, B.n, A.n)
    finally:
        P.close()
    assert st[0].iters_done == iters
    check_run(f"lattice L=640 values {values}", tr, x[:, 0], s[:, 0], logs[0][0], logs[0][1], acc[:, 0], iters, True,
              end_fixed_point=False)


def test_adoch_refused_shapes():
    import torch
    import paper_2509_01928_amd as L
    from tests._util import GpuProblem
    A = gen.er_csr(300, 5.0, 7341)
    P = GpuProblem(A=A)
    try:
        p = P.params(1.0, 1e5)
        p.algo, p.q = 1, 5
        xd = torch.zeros(A.n * 3, dtype=torch.float64, device="cuda:0")
        with pytest.raises(L.IsingError) as e:
            L.ising_solve(P.ctx, xd, 3, 10, p)
        assert e.value.status == L.ISING_E_UNSUPPORTED
        p.x_dtype = L.ISING_F32
        with pytest.raises(L.IsingError) as e:
            L.ising_solve(P.ctx, xd[:A.n], 1, 10, p)
        assert e.value.status == L.ISING_E_UNSUPPORTED
    finally:
        P.close()
