"""Helpers shared by the GPU tests: move seeded instances to the device and
run the library through its C ABI; compare against the oracle."""
from __future__ import annotations

import numpy as np

import ising_inputs as gen
import oracle as orc

# Parity bar for the FP64 path: the oracle and the GPU agree to 1e-9 in max
# abs (as an absolute bound and relative to the iterate's scale) after K
# steps; rounded spins agree except where |x_i| < 1e-6 |x|_inf.
X_ATOL = 1e-9
X_RTOL_SCALE = 1e-9
SPIN_EXEMPT = 1e-6
H_RTOL = 1e-12


def torch_dev():
    import torch
    return torch, torch.device("cuda:0")


class GpuProblem:
    """A context built from an ``ising_inputs.CSR`` or a dense numpy matrix."""

    def __init__(self, A=None, J=None, h=None, val_dtype="f32"):
        import paper_2509_01928_amd as L
        torch, dev = torch_dev()
        self.L = L
        self.torch = torch
        self.keep = []
        if A is not None:
            self.n = A.n
            rp = torch.from_numpy(np.ascontiguousarray(A.row_ptr, dtype=np.int32)).to(dev)
            col = torch.from_numpy(np.ascontiguousarray(A.col, dtype=np.int32)).to(dev)
            if val_dtype == "f32":
                val = torch.from_numpy(np.ascontiguousarray(A.val, dtype=np.float32)).to(dev)
                vt = L.ISING_F32
            elif val_dtype == "i16":
                val = torch.from_numpy(np.ascontiguousarray(A.val, dtype=np.int16)).to(dev)
                vt = L.ISING_I16
            else:
                val = torch.from_numpy(np.ascontiguousarray(A.val, dtype=np.float64)).to(dev)
                vt = L.ISING_F64
            hh, ht = None, L.ISING_F32
            if A.h is not None:
                hh = torch.from_numpy(np.ascontiguousarray(A.h, dtype=np.float32)).to(dev)
            self.ctx = L.ising_create_csr(A.n, A.nnz, rp, col, val, vt, hh, ht)
            self.keep = [rp, col, val, hh]
            self.has_field = A.h is not None
        else:
            self.n = J.shape[0]
            Jd = torch.from_numpy(np.ascontiguousarray(J, dtype=np.float64)).to(dev)
            hh, ht = None, L.ISING_F64
            if h is not None:
                hh = torch.from_numpy(np.ascontiguousarray(h, dtype=np.float64)).to(dev)
            self.ctx = L.ising_create_dense(self.n, Jd, L.ISING_F64, self.n, hh, ht)
            self.keep = [Jd, hh]
            self.has_field = h is not None
        self.np = self.n + (1 if self.has_field else 0)

    def params(self, alpha, beta, eps=0.0, x_dtype=None):
        L = self.L
        p = L.ising_params()
        p.alpha, p.beta, p.eps = float(alpha), float(beta), float(eps)
        p.algo, p.q = 0, 5
        p.x_dtype = L.ISING_F64 if x_dtype is None else x_dtype
        p.reserved = 0
        return p

    def solve(self, x0, alpha, beta, iters, eps=0.0, x_dtype=None, R=1):
        torch = self.torch
        x0 = np.ascontiguousarray(x0, dtype=np.float64).reshape(self.np, R)
        xd = torch.from_numpy(x0).to("cuda:0")
        xo = torch.empty_like(xd)
        so = torch.empty((self.n, R), dtype=torch.int8, device="cuda:0")
        stats = self.L.ising_solve(self.ctx, xd, R, iters, self.params(alpha, beta, eps, x_dtype),
                                   xo, so)
        torch.cuda.synchronize()
        return xo.cpu().numpy(), so.cpu().numpy(), stats

    def log(self, count, restart=0):
        return self.L.ising_get_log(self.ctx, restart, 0, count)

    def energy(self, s, want_int=False):
        torch = self.torch
        s = np.ascontiguousarray(s, dtype=np.int8)
        if s.ndim == 1:
            s = s[:, None]
        R = s.shape[1]
        sd = torch.from_numpy(s).to("cuda:0")
        E = torch.empty(R, dtype=torch.float64, device="cuda:0")
        Ei = torch.empty(R, dtype=torch.int64, device="cuda:0") if want_int else None
        self.L.ising_energy(self.ctx, sd, R, E, Ei)
        torch.cuda.synchronize()
        return E.cpu().numpy(), (Ei.cpu().numpy() if want_int else None)

    def close(self):
        self.L.ising_destroy(self.ctx)
        self.ctx = None


def assert_iterate_parity(x_gpu, x_ref, label=""):
    x_gpu = np.asarray(x_gpu).reshape(-1)
    x_ref = np.asarray(x_ref).reshape(-1)
    scale = float(np.abs(x_ref).max())
    err = float(np.abs(x_gpu - x_ref).max())
    assert err <= X_ATOL, f"{label}: max|dx| = {err:.3e} > {X_ATOL}"
    assert err <= X_RTOL_SCALE * scale, f"{label}: max|dx|/|x|_inf = {err / scale:.3e}"
    return err, scale


def assert_spin_parity(s_gpu, x_ref, s_ref, label=""):
    s_gpu = np.asarray(s_gpu).reshape(-1)
    s_ref = np.asarray(s_ref).reshape(-1)
    scale = float(np.abs(x_ref).max())
    diff = np.nonzero(s_gpu != s_ref)[0]
    xr = np.asarray(x_ref).reshape(-1)[: s_ref.shape[0]]
    bad = [int(i) for i in diff if abs(xr[i]) >= SPIN_EXEMPT * scale]
    assert not bad, f"{label}: spins differ at {bad[:10]} (|x| = {[float(xr[i]) for i in bad[:5]]})"
    return len(diff)


def assert_log_parity(H_gpu, r_gpu, tr, label=""):
    Hs = max(float(np.abs(tr.H).max()), 1e-300)
    dH = float(np.abs(H_gpu - tr.H).max())
    assert dH <= H_RTOL * Hs, f"{label}: max|dH| = {dH:.3e} vs scale {Hs:.3e}"
    dr = np.abs(r_gpu - tr.r)
    tol = 1e-12 + 1e-9 * np.abs(tr.r)
    assert np.all(dr <= tol), f"{label}: r mismatch, worst {float((dr / tol).max()):.3e}"


def seeded_csr_er(n, d, seed):
    return gen.er_csr(n, d, seed)


def oracle_fp32_storage(B, x0, alpha, beta, iters):
    """The oracle's FP64 step with the iterate rounded to FP32 between steps,
    as a path that stores x in FP32 does: x <- fl32(T(fl32(x0)))...  Returns
    the final iterate and the H log (H of each stored iterate)."""
    x = np.asarray(x0, dtype=np.float32).astype(np.float64)
    H = []
    for _ in range(iters):
        tr = orc.doch(B, x, alpha, beta, 1)
        H.append(tr.H[0])
        x = tr.x.astype(np.float32).astype(np.float64)
    return x, np.array(H)


def assert_fp32_storage_parity(x_gpu, x_emu, label=""):
    """Same FP64 arithmetic and the same FP32 rounding of every stored
    iterate: the iterates agree exactly except where an FP64 result fell
    within rounding of an FP32 rounding boundary on one side only."""
    scale = float(np.abs(x_emu).max())
    exact = float(np.mean(x_gpu == x_emu))
    assert exact >= 0.999, f"{label}: only {exact:.5f} of the FP32 iterates agree exactly"
    d = float(np.abs(x_gpu - x_emu).max())
    assert d <= 1e-6 * scale, f"{label}: max|dx| = {d:.3e} vs scale {scale:.3e}"

