"""Pins of the FP64 CPU oracle against what the paper and mathematics fix.

Each test checks the oracle against something other than itself: a value the
paper states for a worked example, a closed-form trajectory, a proven
invariant, brute force, or an independent library routine.  The pins are
chosen so that a plausible slip (a dropped term, a wrong sign, beta in the
wrong place, a Gauss-Seidel instead of a Jacobi sweep, a wrong energy factor)
fails at least one of them.
"""
import itertools
import json
import math
import os
from decimal import Decimal, getcontext

import numpy as np
import pytest

import ising_inputs as gen
import oracle as orc

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


def dense_csr(J):
    return orc.csr_of_dense(np.asarray(J, dtype=np.float64))


# --------------------------------------------------------------- P1 two spins
def test_two_spin_antiferromagnet_closed_form():
    """Fig. 3 (fig:2d_ising_dca): J12=-1, alpha=1, beta=2 -> (1,-1) or (-1,1).

    From eq:FPE, x^(k) = (c_k, -c_k) with c_k = sign(d0)|d0/2|^(3^-k),
    d0 = x1^(0) - x2^(0); the paper says the iterates reach a ground state
    after five iterations.
    """
    g = GOLD["two_spin_antiferromagnet"]
    J = np.array([[0.0, g["J12"]], [g["J12"], 0.0]])
    B = dense_csr(J)
    a, b = g["alpha"], g["beta"]
    for x0 in ([0.3, 0.1], [-0.7, 0.9], [0.25, -0.05], [0.6, 0.2]):
        tr = orc.doch(B, np.array(x0), a, b, 12)
        d0 = x0[0] - x0[1]
        for k in range(1, 12):
            trk = orc.doch(B, np.array(x0), a, b, k)
            ck = math.copysign(abs(d0 / 2) ** (3.0 ** -k), d0)
            assert trk.x[0] == pytest.approx(ck, rel=1e-14)
            assert trk.x[1] == pytest.approx(-ck, rel=1e-14)
            # eq:Hamilton at x=(c,-c): beta/2 c^4 - alpha c^2 - c^2
            if k < 11:
                assert tr.H[k] == pytest.approx(b / 2 * ck ** 4 - a * ck ** 2 - ck ** 2, rel=1e-13)
        s = orc.sign(tr.x)
        assert list(s) in g["ground_states"]
        assert s[0] == (1 if d0 > 0 else -1)
        if abs(d0 / 2) >= 0.1:
            x5 = orc.doch(B, np.array(x0), a, b, g["iterations_to_converge"]).x
            assert np.max(np.abs(np.abs(x5) - 1.0)) < 0.01


# ---------------------------------------------------------- P2 attractor only
def test_attractor_only_closed_form():
    """Prop. global_minima_A with J = 0: x_i^(k) = sign(x0)(a/b)^((1-3^-k)/2)|x0|^(3^-k)
    tends to +-sqrt(alpha/beta)."""
    n = 5
    B = orc.OracleCSR(n, np.zeros(n + 1, np.int64), np.zeros(0, np.int32), np.zeros(0))
    x0 = np.array([0.9, -0.2, 0.003, -1.7, 4.0])
    a, b = 0.7, 3.0
    for k in (1, 2, 3, 7, 30):
        x = orc.doch(B, x0, a, b, k).x
        ref = np.sign(x0) * (a / b) ** ((1 - 3.0 ** -k) / 2) * np.abs(x0) ** (3.0 ** -k)
        np.testing.assert_allclose(x, ref, rtol=1e-14)
    x = orc.doch(B, x0, a, b, 60).x
    np.testing.assert_allclose(np.abs(x), math.sqrt(a / b), rtol=1e-15)
    g = GOLD["attractor_minimisers"]
    x2 = orc.doch(orc.OracleCSR(2, np.zeros(3, np.int64), np.zeros(0, np.int32), np.zeros(0)),
                  np.array([0.4, -3.0]), g["alpha"], g["beta"], 60).x
    assert [int(v) for v in np.round(x2)] in g["minimisers_2d"]


# ----------------------------------------------------- P3 complete ferromagnet
@pytest.mark.parametrize("n", [3, 7, 32])
def test_complete_ferromagnet_closed_form(n):
    """J = 11^T - I, alpha = 1 = lambda_max(-J): x^(k) = c_k 1 with
    ln|c_k| = L + (ln|c_1| - L) 3^-(k-1), L = ln(n/beta)/2."""
    J = np.ones((n, n)) - np.eye(n)
    B = dense_csr(J)
    rng = np.random.default_rng(n)
    x0 = 2 * rng.random(n) - 1
    beta = 5.0 * n
    c1 = np.cbrt(x0.sum() / beta)
    L = 0.5 * math.log(n / beta)
    for k in (1, 2, 5, 20):
        x = orc.doch(B, x0, 1.0, beta, k).x
        ck = math.copysign(math.exp(L + (math.log(abs(c1)) - L) * 3.0 ** -(k - 1)), c1)
        np.testing.assert_allclose(x, ck, rtol=1e-13)
        xd = orc.doch_dense(J, x0, 1.0, beta, k).x
        np.testing.assert_allclose(xd, ck, rtol=1e-13)
    s = orc.sign(orc.doch(B, x0, 1.0, beta, 20).x)
    assert abs(int(s.sum())) == n       # all equal: a ground state
    assert orc.energy_csr(B, s) == pytest.approx(-n * (n - 1) / 2)
    # the power method recovers lambda_max(-J) = 1 exactly
    lam, _ = orc.power_lambda_max_neg(B, 2 * rng.random(n) - 1)
    assert lam == pytest.approx(1.0, abs=1e-9)


# ------------------------------------------------------------ P4 scale
def test_beta_scaling_invariance():
    """eq:FPE: DOCH(alpha, beta, x0) = beta^-1/2 DOCH(alpha, 1, sqrt(beta) x0),
    and eq:Hamilton: H(beta^-1/2 u; beta) = H(u; 1) / beta."""
    J = gen.sk_dense(40, 11)
    B = dense_csr(J)
    x0 = gen.uniform_x0(40, 1, 12)[:, 0]
    a, beta = 9.0, 4.0e5
    t1 = orc.doch(B, x0, a, beta, 50)
    t2 = orc.doch(B, math.sqrt(beta) * x0, a, 1.0, 50)
    np.testing.assert_allclose(t1.x, t2.x / math.sqrt(beta), rtol=1e-11, atol=1e-13 * np.abs(t1.x).max())
    np.testing.assert_allclose(t1.H, t2.H / beta, rtol=1e-10)


# --------------------------------------------------- P5 monotone descent
def test_monotone_descent_with_mu_bound():
    """Prop. monotone_descent_H: H(x^k) - H(x^k+1) >= mu/2 |x^k+1 - x^k|^2,
    mu = lambda_min(J) + alpha > 0 (alpha above lambda_max(-J))."""
    n = 64
    J = gen.sk_dense(n, 21)
    ev = np.linalg.eigvalsh(J)
    alpha = 1.2 * (-ev[0])
    mu = ev[0] + alpha
    beta = n ** 1.5 * (alpha + np.abs(J).sum(axis=1).max())
    B = dense_csr(J)
    x = gen.uniform_x0(n, 1, 22)[:, 0]
    H_prev = orc.hamiltonian(B, x, alpha, beta)
    for k in range(150):
        xn = orc.doch(B, x, alpha, beta, 1).x
        H_next = orc.hamiltonian(B, xn, alpha, beta)
        drop = H_prev - H_next
        step2 = float(np.sum((xn - x) ** 2))
        assert drop >= mu / 2 * step2 - 1e-12 * abs(H_prev), (k, drop, mu / 2 * step2)
        x, H_prev = xn, H_next
    # the logged H of a long run is non-increasing too
    tr = orc.doch(B, gen.uniform_x0(n, 1, 22)[:, 0], alpha, beta, 300)
    assert np.all(np.diff(tr.H) <= 1e-12 * np.abs(tr.H[:-1]))


# ------------------------------------------------------- P6 boundedness
def test_bounded_iterates_any_alpha():
    """Prop. bounded_iters_all_alpha: beta >= ||J + alpha I||_inf gives
    |x^(k)|_inf <= max(1, |x^(0)|_inf), even for small alpha."""
    n = 50
    J = gen.sk_dense(n, 31)
    B = dense_csr(J)
    for alpha in (0.05, 1.0, 30.0):
        beta = alpha + np.abs(J).sum(axis=1).max()          # the minimal beta
        for seed, scale in ((32, 1.0), (33, 40.0), (34, 1e-3)):
            x0 = scale * gen.uniform_x0(n, 1, seed)[:, 0]
            bound = max(1.0, np.abs(x0).max())
            x = x0
            for _ in range(40):
                x = orc.doch(B, x, alpha, beta, 1).x
                assert np.abs(x).max() <= bound * (1 + 1e-15)


# ------------------------------------------------ P7 limit is a fixed point
def test_limit_is_critical_point_of_H():
    """Prop. bounded_iterates + Prop. on critical points: r^(k) -> 0 and the
    limit satisfies beta x*^3 = (J + alpha I) x*, i.e. grad H(x*) = 0.
    grad H is taken by central differences of the oracle's own H, so H and
    the map T are checked against each other."""
    n = 30
    J = gen.sk_dense(n, 41)
    ev = np.linalg.eigvalsh(J)
    alpha = 1.0 * (-ev[0])
    beta = n ** 1.5 * (alpha + np.abs(J).sum(axis=1).max())
    B = dense_csr(J)
    tr = orc.doch(B, gen.uniform_x0(n, 1, 42)[:, 0], alpha, beta, 3000)
    assert tr.r[-1] < 1e-12 and tr.r[-1] < tr.r[0]
    x = tr.x
    res = beta * x ** 3 - (J @ x + alpha * x)
    assert np.abs(res).max() <= 1e-12 * np.abs(J @ x + alpha * x).max()
    h = 1e-6 * np.abs(x).max()
    for i in range(0, n, 7):
        e = np.zeros(n)
        e[i] = h
        g = (orc.hamiltonian(B, x + e, alpha, beta) - orc.hamiltonian(B, x - e, alpha, beta)) / (2 * h)
        scale = beta * abs(x[i]) ** 3 + abs(alpha * x[i]) + np.abs(J[i]) @ np.abs(x)
        assert abs(g) <= 1e-6 * scale


def test_jacobi_not_gauss_seidel():
    """eq:FPE applies T to the whole old vector: one step equals the
    componentwise formula evaluated with x^(k) on the right-hand side."""
    J = gen.sk_dense(12, 51)
    x0 = gen.uniform_x0(12, 1, 52)[:, 0]
    a, b = 3.0, 500.0
    x1 = orc.doch(dense_csr(J), x0, a, b, 1).x
    ref = np.cbrt((J @ x0 + a * x0) / b)
    np.testing.assert_allclose(x1, ref, rtol=1e-14)
    # a Gauss-Seidel sweep gives a different vector on this instance
    gs = x0.copy()
    for i in range(12):
        gs[i] = np.cbrt((J[i] @ gs + a * gs[i]) / b)
    assert np.abs(gs - x1).max() > 1e-6


def test_matvec_against_numpy_and_dense_equals_csr():
    J = gen.sk_dense(70, 61)
    x = gen.uniform_x0(70, 1, 62)[:, 0]
    np.testing.assert_allclose(orc.matvec(dense_csr(J), x), J @ x, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(orc.matvec_dense(J, x), J @ x, rtol=1e-12, atol=1e-12)
    A = gen.er_csr(300, 5.0, 63)
    Jd = gen.dense_from_csr(A)
    x = gen.uniform_x0(300, 1, 64)[:, 0]
    np.testing.assert_array_equal(orc.matvec(orc.to_oracle_csr(A), x), orc.matvec_dense(Jd, x))
    tr1 = orc.doch(orc.to_oracle_csr(A), x, 2.0, 1e4, 25)
    tr2 = orc.doch_dense(Jd, x, 2.0, 1e4, 25)
    np.testing.assert_array_equal(tr1.x, tr2.x)
    np.testing.assert_array_equal(tr1.H, tr2.H)


def test_stopping_rule_remark_s2():
    """Remark S2: stop at the first k with r^(k) < eps; r uses |x^(k)| below."""
    J = gen.sk_dense(40, 71)
    alpha = -np.linalg.eigvalsh(J)[0]
    beta = 40 ** 1.5 * (alpha + np.abs(J).sum(axis=1).max())
    B = dense_csr(J)
    x0 = gen.uniform_x0(40, 1, 72)[:, 0]
    full = orc.doch(B, x0, alpha, beta, 400)
    eps = GOLD["stopping_tolerance"]["eps"]
    k_stop = int(np.argmax(full.r < eps)) + 1
    early = orc.doch(B, x0, alpha, beta, 400, eps=eps)
    assert early.iters == k_stop
    np.testing.assert_array_equal(early.r, full.r[:k_stop])
    # r^(k) by its definition from two consecutive iterates
    xk = orc.doch(B, x0, alpha, beta, 5).x
    xk1 = orc.doch(B, x0, alpha, beta, 6).x
    assert full.r[5] == pytest.approx(np.linalg.norm(xk1 - xk) / np.linalg.norm(xk), rel=1e-12)
    # x = 0 is a fixed point: r = 0 (reported as converged)
    z = orc.doch(B, np.zeros(40), alpha, beta, 3, eps=eps)
    assert z.iters == 1 and z.r[0] == 0.0 and np.all(z.x == 0.0)


# --------------------------------------------------------- sign rounding
def test_sign_zero_is_plus_one():
    assert list(orc.sign(np.array([0.0, -0.0, 1e-300, -1e-300, 3.0, -2.0]))) == [1, 1, 1, -1, 1, -1]


# ------------------------------------------------ P8 energy and brute force
def _energy_by_definition(J, h, s):
    """eq:IsingModel term by term in Python floats (independent loop order)."""
    n = len(s)
    e = 0.0
    for i in range(n):
        for j in range(n):
            e -= 0.5 * J[i][j] * s[i] * s[j]
        if h is not None:
            e -= h[i] * s[i]
    return e


def test_bruteforce_matches_enumeration_small():
    for seed, n, with_h in ((81, 6, False), (82, 8, True), (83, 9, True)):
        J = gen.sk_dense(n, seed)
        h = np.random.default_rng(seed).standard_normal(n) if with_h else None
        best = min(_energy_by_definition(J, h, s) for s in itertools.product((-1, 1), repeat=n))
        E, s = orc.bruteforce(J, h)
        assert E == pytest.approx(best, rel=1e-12, abs=1e-12)
        assert orc.energy_dense(J, s, h) == pytest.approx(best, rel=1e-12, abs=1e-12)


def test_energy_matches_definition_and_csr_equals_dense():
    n = 11
    J = gen.sk_dense(n, 91)
    h = np.random.default_rng(92).standard_normal(n)
    A = gen.csr_from_dense(J.astype(np.float32).astype(np.float64), h)
    Jf = gen.dense_from_csr(A)
    hf = A.h.astype(np.float64)
    for s in itertools.islice(itertools.product((-1, 1), repeat=n), 0, 2048, 37):
        s = np.array(s, dtype=np.int8)
        ref = _energy_by_definition(Jf, hf, s)
        assert orc.energy(A, s) == pytest.approx(ref, rel=1e-12, abs=1e-12)
        assert orc.energy_dense(Jf, s, hf) == pytest.approx(ref, rel=1e-12, abs=1e-12)


@pytest.mark.parametrize("n", [12, 16, 20])
def test_doch_never_beats_bruteforce(n):
    J = gen.sk_dense(n, 100 + n)
    E_min, _ = orc.bruteforce(J)
    alpha = -np.linalg.eigvalsh(J)[0]
    beta = n ** 1.5 * (alpha + np.abs(J).sum(axis=1).max())
    B = dense_csr(J)
    best = np.inf
    for r in range(8):
        x = orc.doch(B, gen.uniform_x0(n, 1, 200 + r)[:, 0], alpha, beta, 300).x
        E = orc.energy_csr(B, orc.sign(x))
        assert E >= E_min - 1e-9
        best = min(best, E)
    assert best <= E_min + 0.25 * abs(E_min)   # a good but not necessarily optimal state


def test_homogeneous_reduction_identity_exhaustive():
    """Supp. Note 1 eq:equiv: Ehat((s,t)) = E(t s) for every (s,t), and
    Prop. S1: t0 * s0 of a ground state of Jhat is a ground state of (J,h)."""
    n = 7
    J = gen.sk_dense(n, 111)
    h = np.random.default_rng(112).standard_normal(n)
    A = gen.csr_from_dense(J, h)
    Jf, hf = gen.dense_from_csr(A), A.h.astype(np.float64)
    Bhat = orc.augment_field(orc.to_oracle_csr(A), hf)
    Jhat = np.zeros((n + 1, n + 1))
    for i in range(n + 1):
        for e in range(Bhat.rp[i], Bhat.rp[i + 1]):
            Jhat[i, Bhat.col[e]] = Bhat.val[e]
    assert np.array_equal(Jhat, Jhat.T) and np.all(np.diag(Jhat) == 0)
    for st in itertools.product((-1, 1), repeat=n + 1):
        st = np.array(st, dtype=np.int8)
        lhs = orc.energy_csr(Bhat, st)
        rhs = orc.energy_dense(Jf, (st[:n] * st[n]).astype(np.int8), hf)
        assert lhs == pytest.approx(rhs, rel=1e-12, abs=1e-12)
    E_hat, s_hat = orc.bruteforce(Jhat)
    E_min, _ = orc.bruteforce(Jf, hf)
    s_star = (s_hat[:n] * s_hat[n]).astype(np.int8)
    assert orc.energy_dense(Jf, s_star, hf) == pytest.approx(E_min, rel=1e-12)
    assert E_hat == pytest.approx(E_min, rel=1e-12)


# --------------------------------------------- P9 field-dominated instance
def test_field_dominated_ground_state():
    """|h_i| > sum_j |J_ij| for all i: the unique ground state is sign(h)."""
    n = 14
    J = gen.sk_dense(n, 121) * 0.1
    rng = np.random.default_rng(122)
    h = np.sign(rng.standard_normal(n)) * (np.abs(J).sum(axis=1) + 0.5 + rng.random(n))
    E_min, s_min = orc.bruteforce(J, h)
    assert np.array_equal(s_min, np.sign(h).astype(np.int8))
    # DOCH on the homogeneous (n+1)-spin problem reaches it once eta is tuned
    # (Supp. Note 6: eta in (0, 2] is chosen per instance; here eta = 1/2,
    # a weaker attractor, is the setting that finds it from every start)
    A = gen.csr_from_dense(J, h)
    Bhat = orc.problem_matrix(A)
    alpha, beta, _ = orc.default_params(Bhat, 0.5, method="power")
    for seed in range(123, 128):
        tr = orc.doch(Bhat, gen.uniform_x0(n + 1, 1, seed)[:, 0], alpha, beta, 500)
        s = orc.spins_with_field(tr.x)
        assert np.array_equal(s, np.sign(A.h).astype(np.int8))


# -------------------------------------------------------- P10 ferromagnet
def test_ferromagnet_ground_state():
    n = 13
    rng = np.random.default_rng(131)
    W = np.triu(rng.random((n, n)) + 0.1, 1)
    J = W + W.T
    E_min, s = orc.bruteforce(J)
    assert E_min == pytest.approx(-np.triu(J, 1).sum(), rel=1e-12)
    assert abs(int(s.sum())) == n
    alpha = -np.linalg.eigvalsh(J)[0]
    beta = n ** 1.5 * (alpha + np.abs(J).sum(axis=1).max())
    x = orc.doch(dense_csr(J), gen.uniform_x0(n, 1, 132)[:, 0], alpha, beta, 400).x
    assert orc.energy_dense(J, orc.sign(x)) == pytest.approx(E_min, rel=1e-12)


# ---------------------------------------------------- P11 integer energies
def test_integer_energy_exact():
    for seed in (141, 142):
        A = gen.er_csr(500, 7.0, seed)
        B = orc.to_oracle_csr(A)
        rng = np.random.default_rng(seed)
        for _ in range(5):
            s = np.where(rng.random(500) < 0.5, 1, -1).astype(np.int8)
            Ei = orc.energy_i64(B, s)
            assert float(Ei) == orc.energy_csr(B, s)
        ones = np.ones(500, dtype=np.int8)
        assert orc.energy_i64(B, ones) == -int(A.val.astype(np.int64).sum()) // 2
    with pytest.raises(ValueError):
        orc.energy_i64(orc.csr_of_dense(np.array([[0, 0.5], [0.5, 0]])), np.ones(2, np.int8))


# -------------------------------------------------------- P12 MAX-CUT map
def test_maxcut_identity():
    """Supp. Note 5: with J = -W/2, cut(s) = W_tot/2 - E(s), W_tot = sum_{i<j} W_ij."""
    n = 10
    rng = np.random.default_rng(151)
    W = np.triu(rng.integers(0, 4, (n, n)).astype(float) * (rng.random((n, n)) < 0.6), 1)
    W = W + W.T
    J = -0.5 * W
    Wtot = np.triu(W, 1).sum()
    for s in itertools.islice(itertools.product((-1, 1), repeat=n), 0, 1024, 13):
        s = np.array(s, dtype=np.int8)
        cut = sum(W[i, j] for i in range(n) for j in range(i + 1, n) if s[i] != s[j])
        assert orc.energy_dense(J, s) == pytest.approx(0.5 * Wtot - cut, abs=1e-12)


# --------------------------------------------------------- P13 Wigner c0
def test_wigner_estimate_k2000_c0():
    """eq:s29 / eq:estimate_eig_J: K2000 with J = +-1 gives c0 = 1/(2<J>sqrt(n)) ~ 0.0112."""
    g = GOLD["k2000_coupling_strength"]
    J = gen.pm1_complete(g["n"], 161)
    lam = orc.wigner_lambda(dense_csr(J))     # = 2<J>sqrt(n)
    c0 = 1.0 / lam
    assert round(c0, 4) == g["c0_printed"]
    # closed form of the estimator: variance of the n(n-1) off-diagonal entries
    off = J[~np.eye(g["n"], dtype=bool)]
    assert lam == pytest.approx(2 * np.sqrt(off.var()) * np.sqrt(g["n"]), rel=1e-9)


def test_wigner_counts_unstored_zeros():
    A = gen.er_csr(2000, 6.0, 162)
    Jd = gen.dense_from_csr(A)
    off = Jd[~np.eye(2000, dtype=bool)]
    assert orc.wigner_lambda(orc.to_oracle_csr(A)) == pytest.approx(2 * np.sqrt(off.var()) * np.sqrt(2000), rel=1e-11)


# -------------------------------------------------------- P14 power method
@pytest.mark.parametrize("n,seed", [(64, 171), (200, 172)])
def test_power_method_against_eigvalsh(n, seed):
    J = gen.sk_dense(n, seed)
    lam, it = orc.power_lambda_max_neg(dense_csr(J), gen.uniform_x0(n, 1, seed + 1)[:, 0],
                                       tol=1e-13, maxit=200000)
    assert lam == pytest.approx(-np.linalg.eigvalsh(J)[0], rel=1e-8)


def test_default_params_formula():
    """eq:alphabeta: beta = n sqrt(n) max_j (alpha + sum_{i!=j} |J_ij|)."""
    A = gen.er_csr(20000, 6.0, 1002)
    B = orc.to_oracle_csr(A)
    alpha, beta, lam = orc.default_params(B, 1.0)
    assert lam == pytest.approx(4.90, abs=0.02)          # 2 sqrt(6/19999) sqrt(20000)
    Jd_rowsum = np.zeros(A.n)
    np.add.at(Jd_rowsum, np.repeat(np.arange(A.n), np.diff(A.row_ptr)), np.abs(A.val))
    assert beta == pytest.approx(20000 ** 1.5 * (alpha + Jd_rowsum.max()), rel=1e-14)


# ----------------------------------------------------------------- P15 cbrt
def test_cbrt_is_real_cube_root_correctly_rounded():
    """eq:FPE's phi is the real cube root: with J = 0 and alpha = beta one step
    is x -> cbrt(x).  Compare with a 60-digit Newton cube root: the oracle's
    cube root is rounded once from extended precision, so it is within half
    an ulp up to rare double-rounding ties."""
    getcontext().prec = 60
    rng = np.random.default_rng(181)
    xs = np.concatenate([rng.standard_normal(300) * 10.0 ** rng.integers(-300, 300, 300),
                         1.0 + 7.0 * rng.random(2000),
                         [-8.0, 27.0, -1e-310, 5e-324, 1.0, -1.0]])
    n = xs.shape[0]
    B = orc.OracleCSR(n, np.zeros(n + 1, np.int64), np.zeros(0, np.int32), np.zeros(0))
    y = orc.doch(B, xs, 1.0, 1.0, 1).x
    worst = 0.0
    for xi, yi in zip(xs, y):
        d = Decimal(abs(float(xi)))
        g = Decimal(abs(float(yi))) if yi != 0 else Decimal(0)
        if d != 0:
            for _ in range(6):
                g = g - (g ** 3 - d) / (3 * g * g)
        ref = math.copysign(float(g), xi)
        assert math.copysign(1.0, yi) == math.copysign(1.0, xi) or xi == 0
        sgn = Decimal(1) if xi >= 0 else Decimal(-1)
        err = abs(Decimal(float(yi)) - sgn * g) / Decimal(math.ulp(ref)) if ref else 0
        worst = max(worst, float(err))
    assert worst <= 0.501, worst
    assert y[-6] == -2.0 and y[-5] == 3.0


# ------------------------------------------------------------ ADOCH pins
def test_adoch_first_step_and_nonmonotone_bound():
    """Alg. 2: y^(0) = x^(0) is always accepted; with convex g every new
    iterate satisfies H(x^(k+1)) <= max{H(x^(j)), max(0,k-q) <= j <= k}."""
    n = 80
    J = gen.sk_dense(n, 191)
    alpha = 1.05 * -np.linalg.eigvalsh(J)[0]
    beta = n ** 1.5 * (alpha + np.abs(J).sum(axis=1).max())
    B = dense_csr(J)
    q = 5
    tr = orc.adoch(B, gen.uniform_x0(n, 1, 192)[:, 0], alpha, beta, 200, q)
    assert tr.accept[0] == 1
    for k in range(len(tr.H) - 1):
        window = tr.H[max(0, k - q):k + 1].max()
        assert tr.H[k + 1] <= window + 1e-12 * abs(window)
    assert tr.accept.sum() > 1
    # with J = 0 ADOCH still ends at the attractor minimisers +-sqrt(alpha/beta)
    Z = orc.OracleCSR(3, np.zeros(4, np.int64), np.zeros(0, np.int32), np.zeros(0))
    xa = orc.adoch(Z, np.array([0.5, -0.25, 2.0]), 1.0, 4.0, 200, 5).x
    np.testing.assert_allclose(np.abs(xa), 0.5, rtol=1e-12)


def test_adoch_momentum_coefficients():
    """Alg. 2's momentum sequence t_{k+1} = (1 + sqrt(1 + 4 t_k^2))/2, t_0 = 1, so the
    extrapolation weights (t_k - 1)/t_{k+1} are 0, 0.2818, 0.4340, ...
    On the scalar problem J = [0] with beta = alpha the map is T(v) = cbrt(v),
    and when every y is accepted x^(2) = cbrt(x1 + c1 (x1 - x0))."""
    Z = orc.OracleCSR(1, np.zeros(2, np.int64), np.zeros(0, np.int32), np.zeros(0))
    x0 = 0.001
    tr2 = orc.adoch(Z, np.array([x0]), 1.0, 1.0, 2, 10)
    x1 = np.cbrt(x0)
    c1 = 0.28175
    assert tr2.accept.tolist() == [1, 1]
    assert tr2.x[0] == pytest.approx(np.cbrt(x1 + c1 * (x1 - x0)), rel=2e-5)


def test_adoch_window_holds_q_plus_one_values():
    """Alg. 2's look-back window is x^(max(0,k-q)) .. x^(k): q + 1 values of H.
    Scalar J = [0], alpha = beta = 1: T(v) = cbrt(v) and H(v) = v^4/4 - v^2/2
    in closed form.  From x^(0) = 27: x^(1) = 3, H(x^(0)) = 132495.75,
    H(x^(1)) = 15.75, and the momentum point y^(1) = 3 + c_1 (3 - 27) with
    c_1 = (t_1 - 1)/t_2 = 0.2818 lands at -3.762, H(y^(1)) = 43.00 -- above
    H(x^(1)) and below H(x^(0)).  So y^(1) is accepted exactly when the window
    at k = 1 reaches back to x^(0): with q = 1 (two values) it is, giving
    x^(2) = cbrt(y^(1)); with q = 0 (one value) it is not, giving
    x^(2) = cbrt(3).  A window one value short fails the q = 1 case."""
    t1 = (1.0 + math.sqrt(5.0)) / 2.0
    t2 = (1.0 + math.sqrt(1.0 + 4.0 * t1 * t1)) / 2.0
    y1 = 3.0 + (t1 - 1.0) / t2 * (3.0 - 27.0)
    H = lambda v: v ** 4 / 4.0 - v * v / 2.0  # noqa: E731
    assert H(3.0) < H(y1) < H(27.0)
    Z = orc.OracleCSR(1, np.zeros(2, np.int64), np.zeros(0, np.int32), np.zeros(0))
    tr1 = orc.adoch(Z, np.array([27.0]), 1.0, 1.0, 2, 1)
    assert tr1.accept.tolist() == [1, 1]
    assert tr1.x[0] == pytest.approx(np.cbrt(y1), rel=1e-14)
    assert tr1.Hy[1] == pytest.approx(H(y1), rel=1e-13)
    assert tr1.Hmax[1] == pytest.approx(H(27.0), rel=1e-15)
    tr0 = orc.adoch(Z, np.array([27.0]), 1.0, 1.0, 2, 0)
    assert tr0.accept.tolist() == [1, 0]
    assert tr0.x[0] == pytest.approx(np.cbrt(3.0), rel=1e-15)
    assert tr0.Hmax[1] == pytest.approx(H(3.0), rel=1e-15)
