"""Parity of the lattice step kernel at the launch shape the throughput
measurement uses: one row per lane, the whole grid sweeping the rows
together, more rows than lanes (every lane takes several trips through the
grid-stride loop), implicit row offsets on constant-degree rows, with the
field's extra spin (Supp. Note 1).

FP64 iterates are compared with the oracle (eq:FPE, Alg. 1) at 1e-9; FP32
iterate storage with the oracle's FP64 step applied to FP32-rounded iterates
(at least 99.9% bit-equal, all within 1e-6 |x|_inf), and its H log within
1e-9 relative.
"""
import numpy as np
import pytest

import ising_inputs as gen
import oracle as orc
from tests._util import (GpuProblem, assert_fp32_storage_parity, assert_iterate_parity,
                         assert_log_parity, assert_spin_parity, oracle_fp32_storage)

pytestmark = pytest.mark.gpu

ITERS = 50


def _case(A, xseed):
    B = orc.problem_matrix(A)
    alpha, beta, _ = orc.default_params(B, 1.0, method="wigner")
    x0 = gen.uniform_x0(B.n, 1, xseed)[:, 0]
    tr = orc.doch(B, x0, alpha, beta, ITERS)
    xe, He = oracle_fp32_storage(B, x0, alpha, beta, ITERS)
    return dict(A=A, B=B, alpha=alpha, beta=beta, x0=x0, tr=tr, xe=xe, He=He)


@pytest.fixture(scope="module")
def torus1024():
    # 1024 x 1024 lattice with field: 1 048 577 rows, 4 per row; at 4
    # workgroups per CU (262 144 lanes) each lane takes four trips
    return _case(gen.torus_csr(1024, 1103, h_std=0.1), 2103)


@pytest.fixture(scope="module")
def circulant6():
    # constant degree 6 (row length known only at run time), no field
    return _case(gen.circulant_csr(600_000, [1, 5, 777], 1104), 2104)


def _run(case, geometry, wg_per_cu, x_dtype):
    P = GpuProblem(A=case["A"])
    try:
        info = P.L.ising_get_info(P.ctx)
        P.L.ising_set_geometry(P.ctx, geometry, wg_per_cu)
        assert P.L.ising_get_info(P.ctx).geometry == geometry
        xt = P.L.ISING_F64 if x_dtype == "f64" else P.L.ISING_F32
        x, s, st = P.solve(case["x0"], case["alpha"], case["beta"], ITERS, x_dtype=xt)
        H, r = P.log(st[0].iters_done)
    finally:
        P.close()
    return info, x[:, 0], s[:, 0], st[0], H, r


def _check(case, label, info, x, s, st, H, r, x_dtype):
    A, tr = case["A"], case["tr"]
    assert st.iters_done == ITERS, label
    if x_dtype == "f64":
        assert_iterate_parity(x, tr.x, label)
        s_ref = orc.spins_with_field(tr.x) if A.h is not None else orc.sign(tr.x)
        assert_spin_parity(s, tr.x, s_ref, label)
        assert_log_parity(H, r, tr, label)
    else:
        assert_fp32_storage_parity(x, case["xe"], label)
        He = case["He"]
        assert np.abs(H - He).max() <= 1e-9 * np.abs(He).max(), label
        s_ref = orc.spins_with_field(case["xe"]) if A.h is not None else orc.sign(case["xe"])
        assert_spin_parity(s, case["xe"], s_ref, label)


@pytest.mark.parametrize("x_dtype", ["f32", "f64"])
@pytest.mark.parametrize("wg_per_cu", [4, 0, 1])
@pytest.mark.parametrize("geometry", [3, 4])
def test_lattice_rowlane_multi_trip(torus1024, geometry, wg_per_cu, x_dtype):
    """geometry 3, FP32 iterate, 4 workgroups per CU is the measured
    configuration of the 10^8-spin lattice."""
    info, x, s, st, H, r = _run(torus1024, geometry, wg_per_cu, x_dtype)
    assert info.row_len == 4          # implicit offsets, compile-time length
    assert info.step_val_bytes == 1 and info.step_col_bytes == 2
    _check(torus1024, f"torus L=1024 geometry {geometry} wg/CU {wg_per_cu} {x_dtype}",
           info, x, s, st, H, r, x_dtype)


@pytest.mark.parametrize("x_dtype", ["f32", "f64"])
@pytest.mark.parametrize("geometry,wg_per_cu", [(3, 1), (4, 4), (4, 0)])
def test_runtime_row_length_multi_trip(circulant6, geometry, wg_per_cu, x_dtype):
    """Rows of 6 entries starting at 6i (half of them not 16-byte aligned):
    geometry 4 loads them as two chunks, geometry 3 takes the element loop."""
    info, x, s, st, H, r = _run(circulant6, geometry, wg_per_cu, x_dtype)
    assert info.row_len == 6
    _check(circulant6, f"circulant geometry {geometry} wg/CU {wg_per_cu} {x_dtype}",
           info, x, s, st, H, r, x_dtype)


def test_read_offsets_multi_trip():
    """Rows of varying length (offsets read) with more rows than lanes."""
    A = gen.er_csr(300_000, 6.0, 1105)
    case = _case(A, 2105)
    for geometry, wpc in ((3, 1), (4, 2)):
        info, x, s, st, H, r = _run(case, geometry, wpc, "f64")
        assert info.row_len == 0
        _check(case, f"ER n=300000 geometry {geometry} wg/CU {wpc}", info, x, s, st, H, r, "f64")


def _symmetric_values(A, fn):
    """Replace the values by fn(min(i, j), max(i, j)), keeping J symmetric."""
    rows = np.repeat(np.arange(A.n, dtype=np.int64), np.diff(A.row_ptr))
    cols = A.col.astype(np.int64)
    A.val = fn(np.minimum(rows, cols), np.maximum(rows, cols)).astype(np.float32)
    return A


@pytest.fixture(scope="module")
def torus600_int8():
    # integer couplings over the whole 8-bit range: the lane-per-row step
    # streams the library's 8-bit copy of them; 360 001 rows, more than the
    # 262 144 lanes at 4 workgroups per CU
    A = gen.torus_csr(600, 1106, h_std=0.1)
    A = _symmetric_values(A, lambda a, b: ((a * 2654435761 + b * 40503) >> 9) % 256 - 128)
    assert A.val.min() == -128 and A.val.max() == 127
    return _case(A, 2106)


@pytest.fixture(scope="module")
def torus600_frac():
    # non-integer couplings: the lane-per-row step streams the FP32 values
    A = gen.torus_csr(600, 1107, h_std=0.1)
    A.val = A.val * np.float32(0.37)
    return _case(A, 2107)


@pytest.mark.parametrize("x_dtype", ["f32", "f64"])
@pytest.mark.parametrize("geometry,wg_per_cu", [(3, 4), (4, 0)])
def test_lattice_rowlane_8bit_values(torus600_int8, geometry, wg_per_cu, x_dtype):
    info, x, s, st, H, r = _run(torus600_int8, geometry, wg_per_cu, x_dtype)
    assert info.row_len == 4 and info.step_val_bytes == 1 and info.step_col_bytes == 2
    _check(torus600_int8, f"torus L=600 values in [-128, 127] geometry {geometry} wg/CU {wg_per_cu} {x_dtype}",
           info, x, s, st, H, r, x_dtype)


@pytest.mark.parametrize("x_dtype", ["f32", "f64"])
@pytest.mark.parametrize("geometry,wg_per_cu", [(3, 4), (4, 0)])
def test_lattice_rowlane_fp32_values(torus600_frac, geometry, wg_per_cu, x_dtype):
    info, x, s, st, H, r = _run(torus600_frac, geometry, wg_per_cu, x_dtype)
    assert info.row_len == 4 and info.step_val_bytes == 4 and info.step_col_bytes == 4
    _check(torus600_frac, f"torus L=600 values 0.37 * (+-1) geometry {geometry} wg/CU {wg_per_cu} {x_dtype}",
           info, x, s, st, H, r, x_dtype)


def test_8bit_copy_only_for_8bit_integers():
    """The 8-bit copy is kept exactly when every value is an integer in
    [-128, 127]; one value outside (128, or 0.5) keeps the stored values."""
    import paper_2509_01928_amd as Lb
    base = gen.er_csr(3000, 5.0, 1108)
    for top, want in ((127.0, 1), (128.0, 4), (-128.0, 1), (0.5, 4)):
        A = gen.er_csr(3000, 5.0, 1108)
        # the first stored pair (i, j) and its mirror (j, i) take the value `top`
        i0 = 0
        j0 = int(base.col[base.row_ptr[0]])
        A.val[base.row_ptr[i0]] = top
        k = base.row_ptr[j0] + int(np.searchsorted(base.col[base.row_ptr[j0]:base.row_ptr[j0 + 1]], i0))
        assert base.col[k] == i0
        A.val[k] = top
        P = GpuProblem(A=A)
        try:
            assert Lb.ising_get_info(P.ctx).step_val_bytes == want, top
        finally:
            P.close()


@pytest.fixture(scope="module")
def circulant_far():
    # 4-entry rows, +-1 values, columns 40 000 away: the 8-bit values are
    # streamed with the int32 column indices (the offsets do not fit 16 bits)
    return _case(gen.circulant_csr(300_000, [1, 40_000], 1109, h_std=0.1), 2109)


@pytest.mark.parametrize("x_dtype", ["f32", "f64"])
@pytest.mark.parametrize("geometry,wg_per_cu", [(3, 4), (4, 0)])
def test_rowlane_8bit_values_int32_columns(circulant_far, geometry, wg_per_cu, x_dtype):
    info, x, s, st, H, r = _run(circulant_far, geometry, wg_per_cu, x_dtype)
    assert info.row_len == 4 and info.step_val_bytes == 1 and info.step_col_bytes == 4
    _check(circulant_far, f"circulant offsets 1, 40000 geometry {geometry} wg/CU {wg_per_cu} {x_dtype}",
           info, x, s, st, H, r, x_dtype)


def test_16bit_column_offsets_only_when_they_fit():
    """Offsets of 32767 (and the wrap-around ones of the lattice) fit 16
    bits; an offset of 32768 does not, since +32768 is out of range."""
    import paper_2509_01928_amd as Lb
    for offs, want in (([1, 32767], 2), ([1, 32768], 4), ([3, 32000], 2)):
        A = gen.circulant_csr(70_000, offs, 1110)
        P = GpuProblem(A=A)
        try:
            info = Lb.ising_get_info(P.ctx)
            assert info.row_len == 4 and info.step_val_bytes == 1
            assert info.step_col_bytes == want, offs
        finally:
            P.close()
