"""Dense restarts on the matrix cores (BF16 / FP8 J, FP32 restarts).

This path solves a quantised problem, so iterates are not compared with the
FP64 oracle element by element.  What is exact is checked exactly: with
J = 0 the products vanish in every format and the trajectory is the closed
form of the attractor (Prop. global_minima_A), up to FP32 storage of u; the
final FP64 objective is eq:Hamilton of the returned iterates; spins are the
signs of the iterates.  Energies are compared with the FP64 oracle on the
same starts by their gap.
"""
import math

import numpy as np
import pytest

import ising_inputs as gen
import oracle as orc

pytestmark = pytest.mark.gpu


def dense_ctx(J):
    import torch
    import paper_2509_01928_amd as L
    Jd = torch.from_numpy(np.ascontiguousarray(J, dtype=np.float64)).to("cuda:0")
    return L.ising_create_dense(J.shape[0], Jd, L.ISING_F64, J.shape[0]), Jd


def run_lowp(J, X0, alpha, beta, iters, prec, eps=0.0, shape=None):
    import torch
    import paper_2509_01928_amd as L
    n, R = X0.shape
    ctx, keep = dense_ctx(J)
    try:
        if shape is not None:
            L.ising_set_lowp_shape(ctx, *shape)
        p = L.ising_params()
        p.alpha, p.beta, p.eps, p.algo, p.q, p.x_dtype, p.reserved = alpha, beta, eps, 0, 5, L.ISING_F64, 0
        xd = torch.from_numpy(np.ascontiguousarray(X0)).to("cuda:0")
        xo = torch.empty_like(xd)
        so = torch.empty((n, R), dtype=torch.int8, device="cuda:0")
        Hf = torch.empty(R, dtype=torch.float64, device="cuda:0")
        st = L.ising_solve_lowp(ctx, xd, R, iters, p, prec, xo, so, Hf)
        E = torch.empty(R, dtype=torch.float64, device="cuda:0")
        L.ising_energy(ctx, so, R, E)
        Hlog = [L.ising_get_log(ctx, r, 0, st[r].iters_done)[0] for r in range(min(R, 3))]
        torch.cuda.synchronize()
        return xo.cpu().numpy(), so.cpu().numpy(), Hf.cpu().numpy(), E.cpu().numpy(), st, Hlog
    finally:
        L.ising_destroy(ctx)


@pytest.mark.parametrize("n,R", [(200, 64), (100, 300)])
@pytest.mark.parametrize("prec_name", ["bf16", "fp8"])
def test_lowp_zero_coupling_closed_form(prec_name, n, R):
    """J = 0: u-space iteration u <- cbrt(alpha u); x = u / sqrt(beta) follows
    x^(k) = sign(x0)(a/b)^((1-3^-k)/2)|x0|^(3^-k) (FP32 storage of u).  The
    second shape has more restart blocks (5) than row tiles (4) and ragged
    edges in both."""
    import paper_2509_01928_amd as L
    prec = L.ISING_BF16 if prec_name == "bf16" else L.ISING_FP8_E4M3
    J = np.zeros((n, n))
    X0 = gen.uniform_x0(n, R, 3)
    a, b = 2.5, 7.0e4
    for k in (1, 3, 25):
        X, S, Hf, E, st, _ = run_lowp(J, X0, a, b, k, prec)
        ref = np.sign(X0) * (a / b) ** ((1 - 3.0 ** -k) / 2) * np.abs(X0) ** (3.0 ** -k)
        np.testing.assert_allclose(X, ref, rtol=3e-6 * k, atol=0)
        np.testing.assert_array_equal(S, np.where(X >= 0, 1, -1))


# (bn, splits, stage_bytes, depth): the fused iteration, a split product,
# the resident fused iteration and J held in LDS (256-byte k slices) that
# fit n = 512 with 32 restarts in both formats
SHAPES = {"fused": (64, 0, 256, 2), "split": (64, 2, 128, 2), "resident": (64, -1, 256, 2),
          "held": (128, -2, 256, 1)}


@pytest.mark.parametrize("shape_name", ["fused", "split", "resident", "held"])
@pytest.mark.parametrize("prec_name", ["bf16", "fp8"])
def test_lowp_energy_gap_and_final_objective(prec_name, shape_name):
    """SK n = 512, 32 restarts.  H_final is eq:Hamilton of the returned
    iterate and the energies are those of its signs (exact checks).  A
    quantised run can settle in another local minimum than the FP64 run from
    the same start, so energies are compared as distributions over the
    restarts: the mean and the best energy within 2 % of the FP64 oracle's.
    sqrt(beta) ~ 2.3e3 here, so u = sqrt(beta) x0 starts far above the FP8
    range: the restart scales must carry it."""
    import paper_2509_01928_amd as L
    prec = L.ISING_BF16 if prec_name == "bf16" else L.ISING_FP8_E4M3
    n, R, iters = 512, 32, 300
    J = gen.sk_dense(n, 4004)
    X0 = gen.uniform_x0(n, R, 5004)
    alpha = -np.linalg.eigvalsh(J)[0]
    beta = n ** 1.5 * (alpha + np.abs(J).sum(axis=1).max())
    assert math.sqrt(beta) * np.abs(X0).max() > 448 * 4
    X, S, Hf, E, st, Hlog = run_lowp(J, X0, alpha, beta, iters, prec, shape=SHAPES[shape_name])
    assert all(s.iters_done == iters and s.nonfinite == 0 for s in st)
    # final FP64 objective of the returned iterates (eq:Hamilton)
    H_np = beta / 4 * (X ** 4).sum(0) - alpha / 2 * (X ** 2).sum(0) - 0.5 * np.einsum("ir,ir->r", X, J @ X)
    np.testing.assert_allclose(Hf, H_np, rtol=1e-10)
    for r in range(R):
        assert E[r] == pytest.approx(orc.energy_dense(J, S[:, r]), rel=1e-12)
    # the logged H of the quantised iteration decreases
    for h in Hlog:
        assert h[-1] <= h[0]
    E64 = np.array([orc.energy_dense(J, orc.sign(orc.doch_dense(J, X0[:, r], alpha, beta, iters).x))
                    for r in range(R)])
    scale = abs(E64.mean())
    assert abs(E.mean() - E64.mean()) < 0.02 * scale, (E.mean(), E64.mean())
    assert E.min() - E64.min() < 0.02 * scale, (E.min(), E64.min())
    assert np.abs(E - E64).max() < 0.15 * scale


@pytest.mark.parametrize("shape_name", ["fused", "resident", "held"])
@pytest.mark.parametrize("prec_name", ["bf16", "fp8"])
def test_lowp_freezes_converged_restarts(prec_name, shape_name):
    """Restarts stop on their own; each returns the iterate of the iteration
    it stopped at: a restart's column of the product depends on that
    restart alone, so a run of exactly iters_done iterations without a
    tolerance gives the same column bit for bit.  The resident run sees a
    stop two iterations late, the launch-per-iteration run one: neither may
    overwrite the stopped restart's last iterate."""
    import paper_2509_01928_amd as L
    prec = L.ISING_BF16 if prec_name == "bf16" else L.ISING_FP8_E4M3
    shape = SHAPES[shape_name]
    n, R = 256, 64
    J = gen.sk_dense(n, 4005)
    X0 = gen.uniform_x0(n, R, 5005)
    alpha = -np.linalg.eigvalsh(J)[0]
    beta = n ** 1.5 * (alpha + np.abs(J).sum(axis=1).max())
    X, S, Hf, E, st, Hlog = run_lowp(J, X0, alpha, beta, 2000, prec, eps=1e-3, shape=shape)
    assert all(s.converged == 1 for s in st)
    assert all(s.iters_done < 2000 for s in st)
    done = np.array([s.iters_done for s in st])
    assert len(set(done.tolist())) > 1       # restarts stop on their own
    for r in (int(np.argmin(done)), int(np.argmax(done))):
        m = int(done[r])
        Xm, Sm, _, _, stm, Hm = run_lowp(J, X0, alpha, beta, m, prec, shape=shape)
        assert stm[r].iters_done == m
        assert np.array_equal(X[:, r], Xm[:, r]), f"restart {r}: final iterate is not iteration {m}'s"
        assert np.array_equal(S[:, r], Sm[:, r])
        if r < 3:
            assert np.array_equal(Hlog[r], Hm[r])


def lowp_shapes(prec_name, n, R):
    """Every shape the library is built for that fits n x R (as ising_solve_lowp pads)."""
    np_ = -(-n // (256 if prec_name == "bf16" else 512)) * (256 if prec_name == "bf16" else 512)
    Rp = -(-R // 64) * 64
    esz = 2 if prec_name == "bf16" else 1
    out = [(64, -1, 256, 2), (64, 0, 256, 2)]
    if prec_name == "bf16" and np_ * esz // 256 >= 3:
        out.append((64, 0, 256, 3))
    for sb in (1024, 512, 256):
        # J held in LDS: 128-row blocks, at most 8 k slices of sb bytes per row
        kb = np_ * esz // sb
        if np_ % 128 == 0 and np_ * esz % sb == 0 and kb <= 8 and Rp <= 128 * (np_ // 128) * kb:
            out.append((128, -2, sb, 1))
    for bn in (128, 64):
        for S in (1, 2, 4, 8):
            for sb in (128, 256):
                for d in (2, 3):
                    stages = np_ * esz // sb
                    if Rp % bn == 0 and stages % S == 0 and stages // S >= d:
                        out.append((bn, S, sb, d))
    return out


@pytest.mark.parametrize("prec_name", ["bf16", "fp8"])
def test_lowp_every_shape_same_step(prec_name):
    """One iteration (SK n = 512, 128 restarts) under every shape that fits.
    The shapes change only the order of the FP32 additions of the product
    (k split across wavefronts, splits, stages), so w = z + alpha u, which
    the cube root takes, differs at most by the order-independent bound
    n 2^-24 sum_k |J_ik q_k| of FP32 summation (written with margin for the
    quantised magnitudes); w is recovered as u'^3 up to the FP32 rounding of
    u' and of the cube root.  Comparing u' itself would not do: the cube
    root amplifies any difference in w where w is near zero."""
    import paper_2509_01928_amd as L
    prec = L.ISING_BF16 if prec_name == "bf16" else L.ISING_FP8_E4M3
    n, R = 512, 128
    J = gen.sk_dense(n, 4006)
    X0 = gen.uniform_x0(n, R, 5006)
    alpha = -np.linalg.eigvalsh(J)[0]
    beta = n ** 1.5 * (alpha + np.abs(J).sum(axis=1).max())
    sb = math.sqrt(beta)
    bound = 3 * n * 2.0 ** -24 * (np.abs(J) @ np.abs(sb * X0))
    shapes = lowp_shapes(prec_name, n, R)
    assert len(shapes) >= 8
    W_ref = (sb * run_lowp(J, X0, alpha, beta, 1, prec, shape=shapes[0])[0]) ** 3
    for sh in shapes[1:]:
        W = (sb * run_lowp(J, X0, alpha, beta, 1, prec, shape=sh)[0]) ** 3
        excess = np.abs(W - W_ref) - (bound + 8 * 2.0 ** -24 * np.abs(W_ref))
        assert excess.max() <= 0.0, (sh, excess.max())


def test_lowp_autotune_and_cache(tmp_path):
    """The tuner picks one of the shapes that fit, stores it, and a second
    call returns it from the cache; the solve then runs under that shape."""
    import torch
    import paper_2509_01928_amd as L
    n, R = 512, 64
    J = gen.sk_dense(n, 4007)
    X0 = gen.uniform_x0(n, R, 5007)
    ctx, keep = dense_ctx(J)
    cache = str(tmp_path / "lowp_shapes.json")
    try:
        p, lam = L.ising_default_params(ctx, 1.0, 0)
        xd = torch.from_numpy(np.ascontiguousarray(X0)).to("cuda:0")
        for prec_name, prec in (("bf16", L.ISING_BF16), ("fp8", L.ISING_FP8_E4M3)):
            shape, ms, cached = L.ising_autotune_lowp(ctx, xd, R, 10, p, prec, cache)
            assert not cached and ms > 0.0
            assert tuple(shape) in lowp_shapes(prec_name, n, R), shape
            shape2, ms2, cached2 = L.ising_autotune_lowp(ctx, xd, R, 10, p, prec, cache)
            assert cached2 and tuple(shape2) == tuple(shape) and ms2 == pytest.approx(ms, rel=1e-3)
            st = L.ising_solve_lowp(ctx, xd, R, 20, p, prec)
            assert all(s.iters_done == 20 and s.nonfinite == 0 for s in st)
        text = open(cache).read()
        assert text.count("lowp-v2|") == 2 and '"splits": ' in text
    finally:
        L.ising_destroy(ctx)


@pytest.mark.parametrize("prec_name", ["bf16", "fp8"])
def test_lowp_resident_matches_launches_bitwise(prec_name):
    """The resident run (one cooperative launch, grid barriers) performs the
    same arithmetic in the same order as one launch per iteration, so 100
    iterations (SK n = 768: a ragged 12 x 3 tile grid in BF16, 12 row tiles
    over a padded order of 1024 in FP8) give identical iterates, spins and
    H / r logs -- which also shows that every barrier published the copy of
    the restarts to every XCD before it was read."""
    import paper_2509_01928_amd as L
    prec = L.ISING_BF16 if prec_name == "bf16" else L.ISING_FP8_E4M3
    n, R, iters = 768, 160, 100
    J = gen.sk_dense(n, 4008)
    X0 = gen.uniform_x0(n, R, 5008)
    alpha = -np.linalg.eigvalsh(J)[0]
    beta = n ** 1.5 * (alpha + np.abs(J).sum(axis=1).max())
    Xa, Sa, Ha, Ea, sta, La = run_lowp(J, X0, alpha, beta, iters, prec, shape=(64, 0, 256, 2))
    Xb, Sb, Hb, Eb, stb, Lb = run_lowp(J, X0, alpha, beta, iters, prec, shape=(64, -1, 256, 2))
    # (a timed-out barrier wait would have raised in the stats read)
    assert [s.iters_done for s in sta] == [s.iters_done for s in stb]
    assert np.array_equal(Xa, Xb)
    assert np.array_equal(Sa, Sb)
    assert np.array_equal(Ha, Hb)
    for a_, b_ in zip(La, Lb):
        assert np.array_equal(a_, b_)


def held_logs(J, X0, alpha, beta, iters, prec, sb):
    """Every restart's (H, r) log of a run with J held in LDS."""
    import torch
    import paper_2509_01928_amd as L
    n, R = X0.shape
    ctx, keep = dense_ctx(J)
    try:
        L.ising_set_lowp_shape(ctx, 128, -2, sb, 1)
        p = L.ising_params()
        p.alpha, p.beta, p.eps, p.algo, p.q, p.x_dtype, p.reserved = alpha, beta, 0.0, 0, 5, L.ISING_F64, 0
        xd = torch.from_numpy(np.ascontiguousarray(X0)).to("cuda:0")
        xo = torch.empty_like(xd)
        st = L.ising_solve_lowp(ctx, xd, R, iters, p, prec, xo)
        logs = [L.ising_get_log(ctx, r, 0, iters) for r in range(R)]
        torch.cuda.synchronize()
        return xo.cpu().numpy(), st, logs
    finally:
        L.ising_destroy(ctx)


@pytest.mark.parametrize("prec_name", ["bf16", "fp8"])
def test_lowp_held_closing_matches_final_close(prec_name):
    """With J held in LDS the workgroups close iteration k - 1 inside the run
    (workgroup b: restarts b, b + G, ...), and the kernel that runs after
    the last iteration closes it alone; both add the row tiles' sums in tile
    order, so iteration m - 1 of a run of m + 1 iterations (closed inside)
    and of a run of m iterations (closed after) log the same H and r bit for
    bit.  n = 512 with 128 restarts and one k slice gives 4 workgroups
    closing 32 restarts each: 1024 staged sums, more than one pass of 512."""
    import paper_2509_01928_amd as L
    prec = L.ISING_BF16 if prec_name == "bf16" else L.ISING_FP8_E4M3
    n, R, m = 512, 128, 12
    sb = 1024 if prec_name == "bf16" else 512
    J = gen.sk_dense(n, 4009)
    X0 = gen.uniform_x0(n, R, 5009)
    alpha = -np.linalg.eigvalsh(J)[0]
    beta = n ** 1.5 * (alpha + np.abs(J).sum(axis=1).max())
    Xa, sta, La = held_logs(J, X0, alpha, beta, m, prec, sb)
    Xb, stb, Lb = held_logs(J, X0, alpha, beta, m + 1, prec, sb)
    assert all(s.iters_done == m for s in sta) and all(s.iters_done == m + 1 for s in stb)
    for r in range(R):
        assert np.array_equal(La[r][0], Lb[r][0][:m]), r
        assert np.array_equal(La[r][1], Lb[r][1][:m]), r
    # H decreases over the run, as the FP64 iteration's does
    H = np.array([l_[0] for l_ in Lb])
    assert (H[:, -1] <= H[:, 0]).all()


@pytest.mark.parametrize("prec_name", ["bf16", "fp8"])
def test_lowp_held_full_size_step(prec_name):
    """The dense n = 4096, 256-restart workload: J held in LDS over 256
    workgroups (32 row blocks x 8 k slices, each row block's slices on one
    XCD) against the fused iteration, one step, within the FP32 summation
    bound of the every-shape test; then 100 iterations of each end at the
    same energies up to the spread that rounding order gives."""
    import paper_2509_01928_amd as L
    prec = L.ISING_BF16 if prec_name == "bf16" else L.ISING_FP8_E4M3
    n, R = 4096, 256
    sb = 1024 if prec_name == "bf16" else 512
    J = gen.sk_dense(n, 4010)
    X0 = gen.uniform_x0(n, R, 5010)
    alpha = float(2.0 * math.sqrt(n) * np.abs(J).mean())
    beta = n ** 1.5 * (alpha + np.abs(J).sum(axis=1).max())
    sq = math.sqrt(beta)
    bound = 3 * n * 2.0 ** -24 * (np.abs(J) @ np.abs(sq * X0))
    W_ref = (sq * run_lowp(J, X0, alpha, beta, 1, prec, shape=(64, 0, 256, 2))[0]) ** 3
    W = (sq * run_lowp(J, X0, alpha, beta, 1, prec, shape=(128, -2, sb, 1))[0]) ** 3
    excess = np.abs(W - W_ref) - (bound + 8 * 2.0 ** -24 * np.abs(W_ref))
    assert excess.max() <= 0.0, excess.max()
    Ea = run_lowp(J, X0, alpha, beta, 100, prec, shape=(64, 0, 256, 2))[3]
    Eb = run_lowp(J, X0, alpha, beta, 100, prec, shape=(128, -2, sb, 1))[3]
    scale = abs(Ea.mean())
    assert abs(Ea.mean() - Eb.mean()) < 0.01 * scale, (Ea.mean(), Eb.mean())
