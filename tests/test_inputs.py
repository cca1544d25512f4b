"""Seeded generators: determinism, symmetry, structure and statistics."""
import numpy as np
import pytest

import ising_inputs as gen


def _triples(A):
    rows = np.repeat(np.arange(A.n), np.diff(A.row_ptr.astype(np.int64)))
    return rows, A.col.astype(np.int64), A.val


def _check_csr_symmetric(A):
    rp = A.row_ptr.astype(np.int64)
    assert rp[0] == 0 and rp[-1] == A.nnz and np.all(np.diff(rp) >= 0)
    rows, cols, vals = _triples(A)
    assert np.all(rows != cols), "diagonal must be zero (not stored)"
    key = rows * A.n + cols
    assert np.all(np.diff(key) > 0), "columns ascending within rows, no duplicates"
    tkey = cols * A.n + rows
    order = np.argsort(tkey)
    assert np.array_equal(tkey[order], key)
    assert np.array_equal(vals[order], vals)


def test_er_deterministic_symmetric_and_degree():
    A = gen.er_csr(20000, 6.0, 1002)
    B = gen.er_csr(20000, 6.0, 1002)
    assert np.array_equal(A.row_ptr, B.row_ptr) and np.array_equal(A.col, B.col)
    assert np.array_equal(A.val, B.val)
    _check_csr_symmetric(A)
    M = 20000 * 19999 // 2
    p = 6.0 / 19999
    edges = A.nnz // 2
    assert abs(edges - M * p) < 4 * np.sqrt(M * p * (1 - p))
    assert set(np.unique(A.val).tolist()) == {-1.0, 1.0}
    assert abs(float(A.val.mean())) < 0.02
    assert A.h is None
    C = gen.er_csr(20000, 6.0, 1003)
    assert not np.array_equal(A.col[:100], C.col[:100])


def test_er_pair_probability_small():
    # every strict-lower pair is kept with probability p: check on many draws
    n, d = 40, 8.0
    hits = np.zeros((n, n))
    T = 300
    for s in range(T):
        hits += gen.dense_from_csr(gen.er_csr(n, d, 5000 + s)) != 0
    p = d / (n - 1)
    freq = hits[np.tril_indices(n, -1)] / T
    assert abs(freq.mean() - p) < 0.01
    assert np.all(np.diag(hits) == 0)


@pytest.mark.parametrize("L", [3, 4, 7, 32])
def test_torus_structure(L):
    A = gen.torus_csr(L, 77, h_std=0.1)
    n = L * L
    assert A.n == n and A.nnz == 4 * n
    _check_csr_symmetric(A)
    assert np.array_equal(np.diff(A.row_ptr), np.full(n, 4))
    J = gen.dense_from_csr(A)
    for i in range(n):
        r, c = divmod(i, L)
        nb = {((r - 1) % L) * L + c, r * L + (c - 1) % L, r * L + (c + 1) % L, ((r + 1) % L) * L + c}
        assert set(np.nonzero(J[i])[0].tolist()) == nb
    assert A.h.dtype == np.float32 and A.h.shape == (n,)


def test_torus_field_and_bond_statistics():
    A = gen.torus_csr(300, 1003, h_std=0.1)
    assert abs(float(A.h.std()) - 0.1) < 0.003
    assert abs(float(A.h.mean())) < 0.003
    assert abs(float(A.val.mean())) < 0.01
    B = gen.torus_csr(300, 1003, h_std=0.1)
    assert np.array_equal(A.val, B.val) and np.array_equal(A.h, B.h)


def test_sk_and_x0():
    J = gen.sk_dense(300, 1001)
    assert np.array_equal(J, J.T) and np.all(np.diag(J) == 0)
    off = J[np.triu_indices(300, 1)]
    assert abs(off.mean()) < 0.02 and abs(off.std() - 1) < 0.02
    assert np.array_equal(J, gen.sk_dense(300, 1001))
    x = gen.uniform_x0(1000, 4, 2001)
    assert x.shape == (1000, 4) and x.min() >= -1 and x.max() < 1
    assert abs(x.mean()) < 0.05


def test_uneven_batch_ranges():
    batch = gen.uneven_batch(count=12)
    ns = [A.n for A in batch]
    assert all(800 <= n <= 20000 for n in ns)
    for A in batch[:4]:
        _check_csr_symmetric(A)
        d = A.nnz / A.n
        assert 2.0 <= d <= 21.0
    again = gen.uneven_batch(count=3)
    assert [A.n for A in again] == ns[:3]
    assert np.array_equal(again[2].col, batch[2].col)


def test_csr_dense_roundtrip():
    J = gen.random_dense_int(25, 9, density=0.4)
    A = gen.csr_from_dense(J)
    assert np.array_equal(gen.dense_from_csr(A), J)


def test_s5_nine_bit_generator():
    """Supp. Alg. S5: keep probability 1022/floor(102300/p), values z - 511 for
    z ~ U{1..1022} (never 0 in storage), symmetric CSR."""
    n, p = 3000, 1.0
    A = gen.s5_csr(n, p, 17)
    _check_csr_symmetric(A)
    Np = int(102300 // p)
    q = 1022 / Np
    M = n * (n - 1) // 2
    edges = A.nnz // 2
    # zero draws (z = 511) are dropped: expected kept edges M q (1 - 1/1022)
    mean = M * q * (1 - 1 / 1022)
    assert abs(edges - mean) < 4 * np.sqrt(M * q)
    v = A.val.astype(np.int64)
    assert v.min() >= -510 and v.max() <= 511 and not np.any(v == 0)
    assert abs(v.mean()) < 10
    assert np.array_equal(A.col, gen.s5_csr(n, p, 17).col)
