#!/usr/bin/env python3
"""Benchmark of the DOCH hot path on one MI355X.

A step is one pass of the whole path over the ultra-large lattice workload:
parameter setting (eq:alphabeta, Wigner estimate), ``iters`` DOCH iterations
(eq:FPE / Alg. 1) with the objective and stopping statistics, sign rounding
and the Ising energy (eq:IsingModel).  Inputs are resident in HBM before the
timed region starts.

Prints one JSON line: edge-updates/s of the whole step, the roofline of the
dominant kernel (the fused CSR step, HBM-bound) and the CPU oracle's rate on
a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6          # FP64 vector peak (FMA = 2 flops)
METHOD_FLOPS_PER_COUPLING = 2.0  # J_ij x_j: one multiply, one add
DENSE_SOURCES = ("kernels_dense.hip", "step_common.h", "device_common.h")
SWEEP_SOURCES = ("kernels_sweep.hip", "step_common.h", "device_common.h")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--s5-n", type=int, default=100_000_000,
                    help="spins of the 9-bit integer instance (mean degree 10)")
    ap.add_argument("--workload", default="torus",
                    choices=["torus", "er20000", "sk1024", "dense4096", "batch512", "s5", "adoch",
                             "procedural", "tune_eta", "adoch_dense", "copy_calib"],
                    help="torus = the 10^8-spin lattice (default line); the others print "
                         "their own JSON line")
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--L", type=int, default=10000, help="lattice side (n = L*L spins)")
    ap.add_argument("--iters", type=int, default=2000)
    ap.add_argument("--x-dtype", choices=["f32", "f64"], default="f32")
    ap.add_argument("--cpu-iters", type=int, default=3,
                    help="oracle iterations timed for the CPU baseline (0 = skip)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--geometry", type=int, default=-2,
                    help="step-kernel geometry (default: autotune)")
    ap.add_argument("--wg-per-cu", type=int, default=0)
    ap.add_argument("--plain-restarts", type=int, default=256,
                    help="dense4096: FP64 restarts run one at a time for the comparison")
    ap.add_argument("--oracle-restarts", type=int, default=0,
                    help="oracle restarts of the dense 4096 workload (0: one per host thread, at most 16)")
    ap.add_argument("--adoch-instance", choices=["sk1024", "procedural"], default="sk1024",
                    help="adoch_dense: the dense instance")
    ap.add_argument("--batch-shape", default="",
                    help="batch512: launch shape 'rj,wg,chunk_rows' instead of the autotuner's")
    ap.add_argument("--lowp-shape", default="",
                    help="dense4096: bn,splits,stage_bytes,depth of the matrix-core product instead of the "
                         "tuned one (splits 0: the fused iteration, -1: resident, -2: J held in LDS); "
                         "'BF16 shape/FP8 shape' to give each format its own")
    ap.add_argument("--tune-cache",
                    default=os.path.join(os.environ.get("XDG_CACHE_HOME", os.path.expanduser("~/.cache")),
                                         "paper_2509_01928_amd", "launch_shapes.json"),
                    help="JSON cache of the launch-shape autotuners (batch512, dense4096)")
    ap.add_argument("--ingest-pmc", nargs=4, metavar="CSV",
                    help="record HBM traffic from rocprofv3 counter files and exit")
    ap.add_argument("--pmc-family", choices=["step", "adoch"], default="step",
                    help="--ingest-pmc: the lattice step kernel, or the ADOCH product (workload adoch)")
    ap.add_argument("--tune-instance", choices=["torus", "s5", "procedural"], default="torus",
                    help="tune_eta: the lattice, the Supp. Alg. S5 instance or the procedural "
                         "sin(ij+100) couplings (--proc-n spins)")
    ap.add_argument("--proc-n", type=int, default=65536,
                    help="spins of the procedural sin(ij+100) instance")
    ap.add_argument("--ingest-flops", metavar="CSV",
                    help="record the FP64 flops per coupling of the procedural step kernel from a "
                         "rocprofv3 counter file (SQ_INSTS_VALU_FLOPS_FP64[_TRANS]) and exit")
    return ap.parse_args()


def kernel_source_hash(names=("kernels_csr.hip", "step_common.h", "device_common.h")) -> str:
    h = hashlib.sha256()
    for name in names:
        with open(os.path.join(ROOT, "paper_2509_01928_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


# the step kernel each launch geometry runs (ising_set_geometry)
_GEOMETRY_KERNEL = {0: ("csr_step_kernel", "1, 1, false"), 1: ("csr_step_kernel", "2, 2, false"),
                    2: ("csr_step_kernel", "4, 2, false"), 3: ("csr_rowlane_kernel", "1, 1"),
                    4: ("csr_rowlane_kernel", "1, 2"), 5: ("csr_step_kernel", "1, 1, true"),
                    6: ("csr_step_kernel", "2, 2, true"), 7: ("csr_step_kernel", "4, 2, true")}


def step_kernel_name(geometry: int, x_dtype: str, implicit_offsets: bool = False,
                     val_bytes: int = 4, col_bytes: int = 4) -> str:
    """Kernel instance timed on the lattice (FP32 couplings and field; the
    lane-per-row kernels read the 8-bit copy of small-integer values and,
    on 4-entry rows, the 16-bit cyclic column offsets)."""
    xt = "float" if x_dtype == "f32" else "double"
    if geometry == 8:                                      # the single-launch solve
        return f"resident_csr_kernel<{xt}, float, float, true>"
    name, tail = _GEOMETRY_KERNEL[geometry]
    vt = "float"
    if name == "csr_rowlane_kernel":
        tail += ", 4" if implicit_offsets else ", 0"      # the lattice's rows hold 4 entries
        vt = "signed char" if val_bytes == 1 else "float"
        if col_bytes == 2:
            tail += ", short"
    return f"{name}<{xt}, {vt}, float, true, {tail}>"


# the sources whose hash a counter record of each kernel family is kept under
STEP_SOURCES = ("kernels_csr.hip", "step_common.h", "device_common.h")
ADOCH_SOURCES = ("kernels_adoch.hip", "adoch_common.h", "device_common.h")


def load_traffic(kernel: str, workload: str, sources=STEP_SOURCES):
    """HBM bytes per launch measured by rocprofv3 counters, if they were taken
    on this kernel instance and on the current kernel source (else None)."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f).get(workload)
    if not rec or rec.get("source_hash") != kernel_source_hash(sources) or kernel not in rec.get("kernel", ""):
        return None
    return rec


def load_flops(kernel: str, workload: str, sources=DENSE_SOURCES):
    """FP64 flops per coupling (per coupling and probe for the sweep) of a
    procedural kernel, measured by rocprofv3 counters on the current kernel
    source (else None)."""
    path = os.path.join(ROOT, "profiles", "flops.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f).get(workload)
    if not rec or rec.get("source_hash") != kernel_source_hash(sources) or kernel not in rec.get("kernel", ""):
        return None
    return rec


def ingest_flops(path, n):
    """FP64 flops per dispatch of the procedural kernels found in a counter
    file, stored in profiles/flops.json: the step kernel per coupling of the
    n(n-1) it generates, the eta sweep kernel per coupling and probe (it
    generates each coupling once for its R probes).  The counters add, over
    the whole device, each executed wavefront instruction's flops per lane
    (a fused multiply-add is two); a wavefront has 64 lanes, all active in
    the row loop, so flops = 64 x (FLOPS_FP64 + FLOPS_FP64_TRANS)."""
    import csv
    import re
    from collections import defaultdict
    vals = defaultdict(lambda: defaultdict(list))
    with open(path) as f:
        for r in csv.DictReader(f):
            vals[r["Kernel_Name"]][r["Counter_Name"]].append(float(r["Counter_Value"]))
    out = os.path.join(ROOT, "profiles", "flops.json")
    data = json.load(open(out)) if os.path.exists(out) else {}
    found = [(k, f"procedural{n}", DENSE_SOURCES, 1) for k in vals
             if "dense_step_kernel" in k and "SinJ" in k]
    for k in vals:
        m = re.search(r"dense_sin_sweep_kernel<(\d+)>", k)
        if m:
            found.append((k, f"sweep_procedural{n}_R{m.group(1)}", SWEEP_SOURCES, int(m.group(1))))
    for name, key, sources, R in found:
        c = vals[name]
        avg = {k: sum(v) / len(v) for k, v in c.items()}
        flops = 64.0 * (avg.get("SQ_INSTS_VALU_FLOPS_FP64", 0.0) + avg.get("SQ_INSTS_VALU_FLOPS_FP64_TRANS", 0.0))
        rec = {"kernel": name, "source_hash": kernel_source_hash(sources), "n": n, "probes": R,
               "dispatches": len(next(iter(c.values()))), "counters_per_dispatch": avg,
               "fp64_flops_per_dispatch": flops, "fp64_flops_per_coupling": flops / (n * (n - 1) * R)}
        data[key] = rec
        print(json.dumps({key: rec}, indent=1))
    with open(out, "w") as f:
        json.dump(data, f, indent=1)


def ingest_pmc(paths, workload, family="step"):
    """Turn four rocprofv3 --pmc counter_collection.csv files (step kernel
    FETCH_SIZE, step kernel WRITE_SIZE, copy kernel FETCH_SIZE, copy kernel
    WRITE_SIZE; values in KiB per dispatch) into HBM bytes per launch of the
    step kernel (family "step") or of the ADOCH product (family "adoch"),
    scaled by what the counters read for a copy of known size, and store them
    in profiles/traffic.json under the hash of that kernel's sources."""
    import csv
    from collections import defaultdict

    def per_kernel(path, counter):
        vals = defaultdict(list)
        with open(path) as f:
            for r in csv.DictReader(f):
                if r["Counter_Name"] == counter:
                    vals[r["Kernel_Name"]].append(float(r["Counter_Value"]))
        return vals

    fetch = per_kernel(paths[0], "FETCH_SIZE")
    write = per_kernel(paths[1], "WRITE_SIZE")
    cf = per_kernel(paths[2], "FETCH_SIZE")
    cw = per_kernel(paths[3], "WRITE_SIZE")
    # the copy of known size: the dispatch reading the most in the copy run
    # (`bench.py --workload copy_calib`: 1 GiB read, 1 GiB written)
    copy_name = max(cf, key=lambda k: sum(cf[k]) / len(cf[k]))
    copy_bytes = float(1024 * 1024 * 1024)
    fetch_scale = copy_bytes / (1024.0 * sum(cf[copy_name]) / len(cf[copy_name]))
    write_scale = copy_bytes / (1024.0 * sum(cw[copy_name]) / len(cw[copy_name]))
    # the timed kernel is the variant of the family dispatched most often
    names = ("adoch_mv_kernel",) if family == "adoch" else ("csr_step_kernel", "csr_rowlane_kernel")
    sources = ADOCH_SOURCES if family == "adoch" else STEP_SOURCES
    steps = [k for k in fetch if any(m in k for m in names)]
    step = max(steps, key=lambda k: len(fetch[k]))
    f_kib = sum(fetch[step]) / len(fetch[step])
    w_kib = sum(write[step]) / len(write[step])
    rec = {
        "kernel": step, "source_hash": kernel_source_hash(sources),
        "fetch_kib_raw": f_kib, "write_kib_raw": w_kib,
        "fetch_scale": fetch_scale, "write_scale": write_scale,
        "hbm_bytes_per_launch": 1024.0 * (f_kib * fetch_scale + w_kib * write_scale),
    }
    path = os.path.join(ROOT, "profiles", "traffic.json")
    data = json.load(open(path)) if os.path.exists(path) else {}
    data[workload] = rec
    with open(path, "w") as f:
        json.dump(data, f, indent=1)
    print(json.dumps(rec, indent=1))


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


# ------------------------------------------------------------------ CPU baselines
def host_info():
    """The host the oracle is timed on: logical CPUs and the CPU model."""
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"host_cpus": os.cpu_count(), "cpu_model": model}


def host_threads():
    """Threads for the concurrent oracle runs: the CPUs this process may use,
    at most 16 (a GPU's share of the host)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def oracle_concurrent(fn, items, threads):
    """fn(item) for every item on `threads` host threads; each call runs the
    single-threaded C oracle (ctypes releases the interpreter lock during the
    call), so `threads` independent oracle runs proceed at once.  Returns the
    results, the wall time and the sum of the calls' own durations."""
    from concurrent.futures import ThreadPoolExecutor

    def timed(item):
        t0 = time.perf_counter()
        r = fn(item)
        return r, time.perf_counter() - t0

    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=threads) as ex:
        res = list(ex.map(timed, items))
    wall = time.perf_counter() - t0
    return [r for r, _ in res], wall, sum(d for _, d in res)


def iterate_parity(x_gpu, x_ref, s_gpu, s_ref):
    """max |dx| (absolute and over |x|_inf) and sign mismatches, with the
    scale-aware exemption |x_i| < 1e-6 |x|_inf."""
    import numpy as np
    x_gpu = np.asarray(x_gpu, dtype=np.float64).reshape(-1)
    x_ref = np.asarray(x_ref, dtype=np.float64).reshape(-1)
    scale = float(np.abs(x_ref).max())
    dx = float(np.abs(x_gpu - x_ref).max())
    mism = np.nonzero(np.asarray(s_gpu).reshape(-1) != np.asarray(s_ref).reshape(-1))[0]
    return {"max_abs_dx": dx, "max_dx_over_xinf": dx / scale if scale > 0 else dx, "x_inf": scale,
            "spin_mismatches": int(mism.size),
            "spin_mismatches_scale_aware": int(np.sum(np.abs(x_ref[mism]) >= 1e-6 * scale))}


# ------------------------------------------------------------------ secondary workloads
def _timed(fn, warmup, steps):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / max(steps, 1)


def bench_er20000(args):
    """Sparse ER n = 20000, mean degree 6, +-1, FP64 iterate, 5000 iterations."""
    import numpy as np
    import torch

    import ising_inputs as gen
    import paper_2509_01928_amd as L
    seed, xseed = gen.SEEDS["er20000"]
    A = gen.er_csr(20000, 6.0, seed)
    x0 = gen.uniform_x0(A.n, 1, xseed)[:, 0]
    d = "cuda:0"
    keep = [torch.from_numpy(a).to(d) for a in (A.row_ptr, A.col, A.val)]
    ctx = L.ising_create_csr(A.n, A.nnz, *keep, L.ISING_F32)
    xd = torch.from_numpy(x0).to(d)
    so = torch.empty(A.n, dtype=torch.int8, device=d)
    E = torch.empty(1, dtype=torch.int64, device=d)
    p, lam = L.ising_default_params(ctx, 1.0, 0)
    g, w, ms = L.ising_autotune(ctx, xd, 200, p)
    iters = 5000

    def step():
        q, _ = L.ising_default_params(ctx, 1.0, 0)
        L.ising_solve(ctx, xd, 1, iters, q, None, so, want_stats=False)
        L.ising_energy(ctx, so, 1, None, E)

    dt = _timed(step, args.warmup, args.steps)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    L.ising_solve(ctx, xd, 1, iters, p, None, so, want_stats=False)
    e1.record()
    torch.cuda.synchronize()
    it_us = 1e3 * e0.elapsed_time(e1) / iters
    # the lane-per-row geometries stream the 8-bit copy of the +-1 values
    vb = L.ising_get_info(ctx).step_val_bytes if g in (3, 4) else 4
    bytes_iter = 4 * (A.n + 1) + (4 + vb) * A.nnz + 16 * A.n
    extra = {}
    if not args.no_cpu_baseline:
        import oracle as orc
        xo = torch.empty_like(xd)
        L.ising_solve(ctx, xd, 1, iters, p, xo, so)
        torch.cuda.synchronize()
        xg, sg, Eg = xo.cpu().numpy(), so.cpu().numpy(), int(E.cpu()[0])
        B = orc.problem_matrix(A)
        t0 = time.perf_counter()
        tr = orc.doch(B, x0, p.alpha, p.beta, iters)
        dt_cpu = time.perf_counter() - t0
        s_ref = orc.sign(tr.x)
        extra["parity"] = iterate_parity(xg, tr.x, sg, s_ref)
        extra["parity"]["energy_int64_gpu"] = Eg
        extra["parity"]["energy_int64_oracle"] = orc.energy_i64(B, s_ref)
        extra["cpu_baseline"] = {"value": A.nnz * iters / dt_cpu, "unit": "edge-updates/s", "cores": 1,
                                 "kind": "oracle",
                                 "sample": f"the whole workload: {iters} DOCH iterations of the "
                                           f"single-threaded FP64 oracle from the same x0 ({dt_cpu:.1f} s)",
                                 **host_info()}
        log(f"parity {extra['parity']}; CPU baseline {extra['cpu_baseline']['value']:.3e} edge-updates/s")
    print(json.dumps({
        "metric": "edge-updates/s", "value": A.nnz * iters / dt, "unit": "edge-updates/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * dt,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic", "config": {"workload": "Erdos-Renyi n=20000 mean degree 6, +-1, "
                                        "5000 DOCH iterations (FP64 iterate)",
                                        "n": A.n, "nnz": A.nnz, "iters": iters,
                                        "kernel_geometry": g, "workgroups_per_cu": w},
        "iteration_us": it_us, "energy_int64": int(E.cpu()[0]),
        "autotune_us_per_iteration": {str(k): round(m * 1e3, 2) for k, m in enumerate(ms) if m > 0},
        "roofline": {"kernel": "resident_csr_kernel" if g == 8 else step_kernel_name(g, "f64", False, vb),
                     "bound": "latency", "achieved": bytes_iter / (it_us * 1e-6) / 1e9,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": bytes_iter / (it_us * 1e-6) / 1e9 / HBM_PEAK_GBS,
                     "algorithmic_bytes_per_launch": bytes_iter},
        **extra,
    }), flush=True)
    L.ising_destroy(ctx)


def bench_sk1024(args):
    """Dense SK n = 1024, FP64, 1000 iterations."""
    import numpy as np
    import torch

    import ising_inputs as gen
    import paper_2509_01928_amd as L
    seed, xseed = gen.SEEDS["sk1024"]
    n = 1024
    J = gen.sk_dense(n, seed)
    x0 = gen.uniform_x0(n, 1, xseed)[:, 0]
    d = "cuda:0"
    Jd = torch.from_numpy(J).to(d)
    ctx = L.ising_create_dense(n, Jd, L.ISING_F64, n)
    xd = torch.from_numpy(x0).to(d)
    so = torch.empty(n, dtype=torch.int8, device=d)
    E = torch.empty(1, dtype=torch.float64, device=d)
    p, lam = L.ising_default_params(ctx, 1.0, 0)
    iters = 1000

    def step():
        L.ising_solve(ctx, xd, 1, iters, p, None, so, want_stats=False)
        L.ising_energy(ctx, so, 1, E)

    dt = _timed(step, args.warmup, args.steps)
    it_us = 1e6 * dt / iters
    geometry = L.ising_get_info(ctx).geometry

    def solve_us(g):
        L.ising_set_geometry(ctx, g, 0)
        L.ising_solve(ctx, xd, 1, iters, p, None, so, want_stats=False)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        L.ising_solve(ctx, xd, 1, iters, p, None, so, want_stats=False)
        e1.record()
        torch.cuda.synchronize()
        return 1e3 * e0.elapsed_time(e1) / iters

    solve_it_us = {"resident": solve_us(8), "launch_per_iteration": solve_us(0)}
    L.ising_set_geometry(ctx, geometry, 0)
    extra = {}
    if not args.no_cpu_baseline:
        import oracle as orc
        xo = torch.empty_like(xd)
        L.ising_solve(ctx, xd, 1, iters, p, xo, so)
        L.ising_energy(ctx, so, 1, E)
        torch.cuda.synchronize()
        xg, sg, Eg = xo.cpu().numpy(), so.cpu().numpy(), float(E.cpu()[0])
        t0 = time.perf_counter()
        tr = orc.doch_dense(J, x0, p.alpha, p.beta, iters)
        dt_cpu = time.perf_counter() - t0
        s_ref = orc.sign(tr.x)
        extra["parity"] = iterate_parity(xg, tr.x, sg, s_ref)
        extra["parity"]["energy_gpu"] = Eg
        extra["parity"]["energy_oracle"] = orc.energy_dense(J, s_ref)
        extra["cpu_baseline"] = {"value": n * (n - 1) * iters / dt_cpu, "unit": "edge-updates/s",
                                 "cores": 1, "kind": "oracle",
                                 "sample": f"the whole workload: {iters} DOCH iterations of the "
                                           f"single-threaded FP64 oracle from the same x0 ({dt_cpu:.2f} s)",
                                 **host_info()}
        log(f"parity {extra['parity']}; CPU baseline {extra['cpu_baseline']['value']:.3e} edge-updates/s")
    print(json.dumps({
        "metric": "edge-updates/s", "value": n * (n - 1) * iters / dt, "unit": "edge-updates/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * dt,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic", "config": {"workload": "dense SK n=1024, J~N(0,1), 1000 DOCH "
                                        "iterations, FP64", "n": n, "iters": iters,
                                        "kernel_geometry": geometry},
        "iteration_us": it_us, "solve_iteration_us": solve_it_us,
        "energy": float(E.cpu()[0]), "lambda_hat": lam,
        "roofline": {"kernel": "resident_dense_kernel" if geometry in (-1, 8) else "dense_step_kernel",
                     "bound": "latency", "achieved": 8 * n * n / (it_us * 1e-6) / 1e9,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": 8 * n * n / (it_us * 1e-6) / 1e9 / HBM_PEAK_GBS,
                     "algorithmic_bytes_per_launch": 8 * n * n},
        **extra,
    }), flush=True)
    L.ising_destroy(ctx)


def bench_dense4096(args):
    """Dense n = 4096, 256 restarts: BF16 and FP8 matrix-core iterations vs
    the plain FP64 path on the same 256 starts run one restart at a time,
    compared at equal best energy; energy gaps per restart against the GPU's
    FP64 path (all starts) and the FP64 oracle (one start per host thread)."""
    import numpy as np
    import torch

    import ising_inputs as gen
    import oracle as orc
    import paper_2509_01928_amd as L
    seed, xseed = gen.SEEDS["sk4096"]
    n, R, iters = 4096, 256, 1000
    J = gen.sk_dense(n, seed)
    d = "cuda:0"
    Jd = torch.from_numpy(J).to(d)
    ctx = L.ising_create_dense(n, Jd, L.ISING_F64, n)
    p, lam = L.ising_default_params(ctx, 1.0, 0)
    log(f"lambda = {lam:.4f}, alpha = {p.alpha:.4f}, beta = {p.beta:.4e}")
    out = {"metric": "restarts/s at equal best energy", "unit": "restarts/s", "n_gpus": 1,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "data": "synthetic", "config": {"workload": "dense SK n=4096, J~N(0,1), 256 restarts "
                                           "x0~U(-1,1), 1000 DOCH iterations", "n": n, "R": R,
                                           "iters": iters}}
    X0 = gen.uniform_x0(n, R, xseed)                     # n x R, restart-interleaved
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)

    # plain FP64 path on the same R starts, one restart at a time (matrix-
    # vector products), timed with device events and no host round trips
    nplain = min(args.plain_restarts, R)
    X0T = torch.from_numpy(np.ascontiguousarray(X0.T)).to(d)      # row r: start r
    S64 = torch.empty((R, n), dtype=torch.int8, device=d)
    E64 = torch.empty(R, dtype=torch.float64, device=d)
    L.ising_solve(ctx, X0T[0], 1, 20, p, None, S64[0], want_stats=False)   # warm-up
    torch.cuda.synchronize()
    e0.record()
    for r in range(nplain):
        L.ising_solve(ctx, X0T[r], 1, iters, p, None, S64[r], want_stats=False)
        L.ising_energy(ctx, S64[r], 1, E64[r:r + 1])
    e1.record()
    torch.cuda.synchronize()
    t_plain = 1e-3 * e0.elapsed_time(e1) / nplain
    E_plain = E64.cpu().numpy()[:nplain]
    best64 = float(E_plain.min())
    out["fp64_plain"] = {"restarts_per_s": 1.0 / t_plain, "best_energy": best64,
                         "restarts": nplain, "ms_per_restart": 1e3 * t_plain}
    log(f"FP64 plain: {1e3 * t_plain:.1f} ms/restart over {nplain} starts, best E {best64:.1f}")

    # the FP64 oracle on the first starts, one single-threaded run per host thread
    n_or = args.oracle_restarts if args.oracle_restarts > 0 else host_threads()
    n_or = min(n_or, nplain)
    E_or = None
    if not args.no_cpu_baseline and n_or > 0:
        trs, wall, busy = oracle_concurrent(
            lambda r: orc.doch_dense(J, X0[:, r], p.alpha, p.beta, iters), range(n_or), n_or)
        E_or = np.array([orc.energy_dense(J, orc.sign(t.x)) for t in trs])
        out["cpu_baseline"] = {"value": n_or / wall, "unit": "restarts/s", "cores": n_or, "kind": "oracle",
                               "sample": f"starts 0..{n_or - 1} of the same 256, {iters} DOCH iterations "
                                         f"each, one single-threaded FP64 oracle run per host thread, "
                                         f"concurrently ({wall:.1f} s wall)",
                               "value_1core": n_or / busy, **host_info()}
        gap = (E_plain[:n_or] - E_or) / np.abs(E_or)
        out["fp64_plain"]["energy_gap_vs_fp64_oracle"] = {"restarts": n_or, "max_abs": float(np.abs(gap).max()),
                                                         "equal": int(np.sum(E_plain[:n_or] == E_or))}
        log(f"oracle: {n_or} restarts in {wall:.1f} s; GPU FP64 vs oracle max |gap| {np.abs(gap).max():.2e}")

    for name, prec, peak in (("bf16", L.ISING_BF16, 2500.0), ("fp8", L.ISING_FP8_E4M3, 5000.0)):
        xd = torch.from_numpy(np.ascontiguousarray(X0)).to(d)
        so = torch.empty((n, R), dtype=torch.int8, device=d)
        Hf = torch.empty(R, dtype=torch.float64, device=d)
        Eb = torch.empty(R, dtype=torch.float64, device=d)
        if args.lowp_shape:
            spec = args.lowp_shape.split("/")
            spec = spec[0] if name == "bf16" or len(spec) == 1 else spec[1]
            shape = tuple(int(v) for v in spec.split(","))
            L.ising_set_lowp_shape(ctx, *shape)
            tune = {"source": "flag"}
        else:
            t0 = time.time()
            os.makedirs(os.path.dirname(args.tune_cache), exist_ok=True)
            shape, tms, cached = L.ising_autotune_lowp(ctx, xd, R, 50, p, prec, args.tune_cache)
            tune = {"source": "cache" if cached else "autotuner", "us_per_iteration": 1e3 * tms / 50,
                    "tuning_s": time.time() - t0}
        log(f"{name} shape {shape} ({tune['source']})")
        L.ising_solve_lowp(ctx, xd, R, 20, p, prec, None, so, Hf)      # warm-up
        torch.cuda.synchronize()
        e0.record()
        L.ising_solve_lowp(ctx, xd, R, iters, p, prec, None, so, Hf, want_stats=False)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        L.ising_energy(ctx, so, R, Eb)
        Eh = Eb.cpu().numpy()
        # equal-energy protocol: the first batch is the same R starts as the
        # FP64 path; further batches of R new starts until the best energy
        # reaches the FP64 path's best (at most 16 batches)
        best = float(Eh.min())
        batches = 1
        t_total = ms * 1e-3
        while best > best64 and batches < 16:
            Xb = gen.uniform_x0(n, R, xseed * 1000 + batches)
            xb = torch.from_numpy(Xb).to(d)
            e0.record()
            L.ising_solve_lowp(ctx, xb, R, iters, p, prec, None, so, Hf, want_stats=False)
            e1.record()
            torch.cuda.synchronize()
            t_total += 1e-3 * e0.elapsed_time(e1)
            L.ising_energy(ctx, so, R, Eb)
            best = min(best, float(Eb.cpu().numpy().min()))
            batches += 1
        flops = 2.0 * n * n * R * iters
        g64 = (Eh[:nplain] - E_plain) / np.abs(E_plain)
        res = {"restarts_per_s": R * batches / t_total, "ms_per_batch_of_256": ms,
               "iteration_us": 1e3 * ms / iters, "best_energy": best,
               "best_energy_first_batch": float(Eh.min()),
               "reached_fp64_best": bool(best <= best64), "batches": batches,
               "energy_gap_vs_gpu_fp64_same_starts": {
                   "restarts": nplain, "mean": float(g64.mean()), "min": float(g64.min()),
                   "max": float(g64.max()), "lower_or_equal_fraction": float(np.mean(g64 <= 0))},
               "launch_shape": {"bn": shape[0], "splits": shape[1], "stage_bytes": shape[2], "depth": shape[3],
                                "kind": LOWP_KIND[min(shape[1], 1)]},
               "autotune": tune,
               "roofline": {"bound": "mfma",
                            "kernel": LOWP_KERNEL[min(shape[1], 1)],
                            "achieved": flops / (ms * 1e-3) / 1e12, "peak": peak,
                            "unit": "TFLOP/s", "frac": flops / (ms * 1e-3) / 1e12 / peak}}
        if E_or is not None:
            go = (Eh[:n_or] - E_or) / np.abs(E_or)
            res["energy_gap_vs_fp64_oracle"] = {"restarts": n_or, "per_restart": [float(v) for v in go],
                                                "mean": float(go.mean())}
        out[name] = res
        log(f"{name}: {1e3 * ms / iters:.1f} us/iteration, {res['roofline']['achieved']:.1f} TFLOP/s, "
            f"best {best:.1f} after {batches} batch(es)")
    out["value"] = out["bf16"]["restarts_per_s"]
    out["dtype"] = "bf16"
    out["vs_fp64_plain"] = out["bf16"]["restarts_per_s"] / out["fp64_plain"]["restarts_per_s"]
    print(json.dumps(out), flush=True)
    L.ising_destroy(ctx)


# launch shapes of the dense low-precision path, by their splits field
LOWP_KIND = {-2: "J held in LDS, resident (split k over the device, two grid barriers per iteration)",
             -1: "fused, resident", 0: "fused (a launch per iteration)", 1: "split product + update"}
LOWP_KERNEL = {-2: "lowp_held_kernel", -1: "lowp_resident_kernel", 0: "lowp_fused_kernel",
               1: "lowp_gemm_kernel + lowp_update_kernel"}


def bench_batch512(args):
    """512 Erdos-Renyi instances, n ~ U{800..20000}, degree ~ U[3,20], 8
    restarts each, eps = 1e-3, at most 5000 iterations, one launch."""
    import numpy as np
    import torch

    import ising_inputs as gen
    import paper_2509_01928_amd as L
    seed, xseed = gen.SEEDS["batch512"]
    R = 8
    t0 = time.time()
    inst = gen.uneven_batch(count=512, seed=seed)
    rps, cols, vals = [np.zeros(1, np.int64)], [], []
    row0 = nnz0 = 0
    for A in inst:
        rps.append(A.row_ptr[1:].astype(np.int64) + nnz0)
        cols.append(A.col.astype(np.int64) + row0)
        vals.append(A.val)
        row0 += A.n
        nnz0 += A.nnz
    rp = np.concatenate(rps).astype(np.int32)
    col = np.concatenate(cols).astype(np.int32)
    val = np.concatenate(vals).astype(np.float32)
    total = row0
    X0 = np.concatenate([gen.uniform_x0(A.n, R, xseed * (1 << 20) + k) for k, A in enumerate(inst)])
    log(f"generated 512 instances: {total} spins, {nnz0} couplings in {time.time() - t0:.1f}s")
    d = "cuda:0"
    keep = [torch.from_numpy(a).to(d) for a in (rp, col, val)]
    ctx = L.ising_create_batch([A.n for A in inst], *keep, L.ISING_F32)
    alpha, beta, lam = L.ising_default_params_batch(ctx, len(inst), 1.0, 0)
    xd = torch.from_numpy(X0).to(d)
    so = torch.empty(X0.shape, dtype=torch.int8, device=d)
    Ei = torch.empty(len(inst) * R, dtype=torch.int64, device=d)
    xdt = L.ISING_F32 if args.x_dtype == "f32" else L.ISING_F64
    # launch shape: the project's autotuner (setup, outside the timed region),
    # its choice kept in a JSON cache
    tune = {}
    if args.batch_shape:
        rj, wg, rpm = (int(v) for v in args.batch_shape.split(","))
        L.ising_set_batch_shape(ctx, rj, wg, rpm)
        tune = {"shape": [rj, wg, rpm], "source": "command line"}
    else:
        os.makedirs(os.path.dirname(args.tune_cache), exist_ok=True)
        t0 = time.perf_counter()
        shape, ms, cached = L.ising_autotune_batch(ctx, xd, R, 5000, alpha, beta, 1e-3, xdt, args.tune_cache)
        tune = {"shape": list(shape), "ms": ms, "source": "cache" if cached else "autotuner",
                "tuning_s": time.perf_counter() - t0}
        log(f"batch shape {shape} ({tune['source']}, {ms:.1f} ms)")

    def step():
        L.ising_solve_batch(ctx, xd, R, 5000, alpha, beta, 1e-3, xdt, None, so, want_stats=False)
        L.ising_energy_batch(ctx, so, R, None, Ei)

    dt = _timed(step, args.warmup, args.steps)
    st, tts = L.ising_solve_batch(ctx, xd, R, 5000, alpha, beta, 1e-3, xdt, None, so)
    iters = np.array([s.iters_done for s in st]).reshape(len(inst), R)
    nnz = np.array([A.nnz for A in inst])
    ns = np.array([A.n for A in inst])
    edge_updates = float((iters * nnz[:, None]).sum())
    xb = 4 if args.x_dtype == "f32" else 8
    # per instance: the couplings are streamed once per iteration for all its
    # restarts (until the slowest stops); each live restart reads and writes
    # its iterate column
    bytes_moved = float(((4 * (ns + 1) + 8 * nnz) * iters.max(axis=1)).sum()
                        + (2 * xb * ns[:, None] * iters).sum())
    extra = {}
    if not args.no_cpu_baseline:
        extra = batch_oracle_sample(args, L, torch, ctx, inst, X0, alpha, beta, R, xd, so, Ei)
    print(json.dumps({
        "metric": "edge-updates/s", "value": edge_updates / dt, "unit": "edge-updates/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * dt,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic", "config": {"workload": "512 Erdos-Renyi instances n~U{800..20000}, "
                                        "degree~U[3,20], +-1, 8 restarts, eps=1e-3, <=5000 "
                                        "iterations, one persistent graph-captured launch",
                                        "spins": int(total), "couplings": int(nnz0), "restarts": R,
                                        "x_storage": args.x_dtype,
                                        "launch_shape": {"restarts_per_job": tune["shape"][0],
                                                         "threads": tune["shape"][1],
                                                         "chunk_rows": tune["shape"][2],
                                                         "chosen_by": tune["source"]}},
        "autotune": tune,
        "tts_ms_p50": float(np.percentile(tts, 50)), "tts_ms_p99": float(np.percentile(tts, 99)),
        "tts_ms_max": float(tts.max()),
        "iterations_mean": float(iters.mean()), "iterations_max": int(iters.max()),
        "converged_fraction": float(np.mean([s.converged for s in st])),
        "energy_int64_sum": int(Ei.cpu().numpy().sum()),
        "roofline": {"bound": "hbm", "achieved": bytes_moved / dt / 1e9, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": bytes_moved / dt / 1e9 / HBM_PEAK_GBS,
                     "algorithmic_bytes": bytes_moved},
        **extra,
    }), flush=True)
    L.ising_destroy(ctx)


def batch_oracle_sample(args, L, torch, ctx, inst, X0, alpha, beta, R, xd, so, Ei):
    """The oracle on the instances with index = 0 mod 8, every restart, to
    the same stopping rule: its rate on the host's threads, and parity of the
    GPU's FP64-iterate solve (iterations to stop and exact energies) on that
    sample."""
    import numpy as np

    import oracle as orc
    ids = list(range(0, len(inst), 8))
    row0 = np.concatenate([[0], np.cumsum([A.n for A in inst])])
    # the GPU with FP64 iterates, outside the timed region
    st64, _ = L.ising_solve_batch(ctx, xd, R, 5000, alpha, beta, 1e-3, L.ISING_F64, None, so)
    L.ising_energy_batch(ctx, so, R, None, Ei)
    torch.cuda.synchronize()
    it64 = np.array([s.iters_done for s in st64]).reshape(len(inst), R)
    E64 = Ei.cpu().numpy().reshape(len(inst), R)
    mats = {k: orc.problem_matrix(inst[k]) for k in ids}
    tasks = [(k, r) for k in ids for r in range(R)]

    def run(task):
        k, r = task
        x0 = X0[row0[k]:row0[k + 1], r]
        tr = orc.doch(mats[k], x0, alpha[k], beta[k], 5000, eps=1e-3)
        return tr.iters, orc.energy_i64(mats[k], orc.sign(tr.x))

    threads = host_threads()
    res, wall, busy = oracle_concurrent(run, tasks, threads)
    edge_updates = float(sum(inst[k].nnz * it for (k, _), (it, _) in zip(tasks, res)))
    same_iters = sum(int(it64[k, r] == it) for (k, r), (it, _) in zip(tasks, res))
    same_energy = sum(int(E64[k, r] == e) for (k, r), (_, e) in zip(tasks, res))
    log(f"oracle sample: {len(tasks)} restarts in {wall:.1f} s on {threads} threads; "
        f"iterations equal {same_iters}, energies equal {same_energy}")
    return {
        "parity": {"sample": f"{len(ids)} instances (index = 0 mod 8) x {R} restarts, FP64 iterates",
                   "restarts": len(tasks), "iterations_equal": same_iters, "energy_int64_equal": same_energy},
        "cpu_baseline": {"value": edge_updates / wall, "unit": "edge-updates/s", "cores": threads,
                         "kind": "oracle",
                         "sample": f"{len(ids)} of the 512 instances (index = 0 mod 8) x {R} restarts, "
                                   f"eps = 1e-3, at most 5000 iterations; one single-threaded FP64 oracle "
                                   f"run per (instance, restart), {threads} at a time ({wall:.1f} s wall)",
                         "value_1core": edge_updates / busy, **host_info()},
    }


def bench_s5(args):
    """Supp. Alg. S5 sparse 9-bit integer instance (the paper's ultra-large
    sparse workload): n spins, mean degree 10, values in {-510..511} stored
    as int16 (6 bytes per stored coupling with its index), h = 0, FP32
    iterate, 500 DOCH iterations per step, exact int64 energy and MAX-CUT
    value (weights w = -J) of the rounded spins."""
    import numpy as np
    import torch

    import ising_inputs as gen
    import paper_2509_01928_amd as L
    n = args.s5_n
    p_percent = 100.0 * 10.0 / (n - 1)
    t0 = time.time()
    A = gen.s5_csr(n, p_percent, 1006)
    x0 = gen.uniform_x0(n, 1, 2006)[:, 0]
    log(f"generated S5 instance: n={A.n} nnz={A.nnz} in {time.time() - t0:.1f}s")
    d = "cuda:0"
    rp = torch.from_numpy(A.row_ptr).to(d)
    col = torch.from_numpy(A.col).to(d)
    val = torch.from_numpy(A.val.astype(np.int16)).to(d)
    ctx = L.ising_create_csr(A.n, A.nnz, rp, col, val, L.ISING_I16)
    del rp, col, val
    torch.cuda.empty_cache()
    xd = torch.from_numpy(x0).to(d)
    so = torch.empty(A.n, dtype=torch.int8, device=d)
    Ei = torch.empty(1, dtype=torch.int64, device=d)
    cut = torch.empty(1, dtype=torch.int64, device=d)
    p0, _ = L.ising_default_params(ctx, 1.0, 0)
    p0.x_dtype = L.ISING_F32
    g, w, tune_ms = L.ising_autotune(ctx, xd, 10, p0)
    iters = 500
    solve_ms = []

    def step():
        p, _ = L.ising_default_params(ctx, 1.0, 0)
        p.x_dtype = L.ISING_F32
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        L.ising_solve(ctx, xd, 1, iters, p, None, so, want_stats=False)
        e1.record()
        L.ising_energy(ctx, so, 1, None, Ei)
        solve_ms.append((e0, e1))

    dt = _timed(step, args.warmup, args.steps)
    L.ising_cut(ctx, so, 1, None, cut)
    torch.cuda.synchronize()
    it_us = 1e3 * float(np.mean([a.elapsed_time(b) for a, b in solve_ms[args.warmup:]])) / iters
    bytes_iter = 4 * (A.n + 1) + 6 * A.nnz + 2 * 4 * A.n
    achieved = bytes_iter / (it_us * 1e-6) / 1e9
    print(json.dumps({
        "metric": "edge-updates/s", "value": A.nnz * iters / dt, "unit": "edge-updates/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * dt,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic", "config": {"workload": f"Supp. Alg. S5 sparse 9-bit integer instance, "
                                        f"n={A.n}, mean degree 10, int16 values, h=0, {iters} "
                                        f"DOCH iterations (FP32 iterate) + parameters + energy",
                                        "n": A.n, "nnz": A.nnz, "iters": iters,
                                        "kernel_geometry": g, "workgroups_per_cu": w},
        "iteration_us": it_us, "energy_int64": int(Ei.cpu()[0]), "maxcut_int64": int(cut.cpu()[0]),
        "roofline": {"kernel": step_kernel_name(g, "f32").replace("float, float, float, true",
                                                                  "float, short, float, false"),
                     "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "algorithmic_bytes_per_launch": bytes_iter},
    }), flush=True)
    L.ising_destroy(ctx)


def _torus_ctx(L_side, x_extra=1):
    """The 10^8-spin lattice context of the main bench (FP32 CSR, FP32 field)."""
    import torch

    import ising_inputs as gen
    import paper_2509_01928_amd as L
    seed, xseed = gen.SEEDS["torus1e4"]
    t0 = time.time()
    A = gen.torus_csr(L_side, seed, h_std=0.1)
    x0 = gen.uniform_x0(A.n + x_extra, 1, xseed)[:, 0]
    log(f"generated torus L={L_side}: n={A.n} nnz={A.nnz} in {time.time() - t0:.1f}s")
    d = "cuda:0"
    rp = torch.from_numpy(A.row_ptr).to(d)
    col = torch.from_numpy(A.col).to(d)
    val = torch.from_numpy(A.val).to(d)
    h = torch.from_numpy(A.h).to(d)
    ctx = L.ising_create_csr(A.n, A.nnz, rp, col, val, L.ISING_F32, h, L.ISING_F32)
    del rp, col, val, h
    torch.cuda.empty_cache()
    return A, x0, ctx


def bench_adoch(args):
    """ADOCH (Alg. 2, NEXT-1) on the 10^8-spin lattice with its field: FP64
    iterates, window q = 5, 100 iterations per step.  Each iteration is two
    launches: the product with H(x) and H(y), x^(k+1) = T(y) written before
    the acceptance test and the test itself, then a repair pass that runs
    only when y was rejected (x^(k+1) = T(x) instead)."""
    import numpy as np
    import torch

    import paper_2509_01928_amd as L
    A, x0, ctx = _torus_ctx(args.L)
    d = "cuda:0"
    xd = torch.from_numpy(x0).to(d)
    so = torch.empty(A.n, dtype=torch.int8, device=d)
    E = torch.empty(1, dtype=torch.float64, device=d)
    iters = 100
    solve_ms = []

    def step():
        p, _ = L.ising_default_params(ctx, 1.0, 0)
        p.algo, p.q = 1, 5
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        L.ising_solve(ctx, xd, 1, iters, p, None, so, want_stats=False)
        e1.record()
        L.ising_energy(ctx, so, 1, E)
        solve_ms.append((e0, e1))

    dt = _timed(step, args.warmup, args.steps)
    torch.cuda.synchronize()
    it_us = 1e3 * float(np.mean([a.elapsed_time(b) for a, b in solve_ms[args.warmup:]])) / iters
    acc = L.ising_get_accept_log(ctx, 0, iters)
    n, nnz, np1 = A.n, A.nnz, A.n + 1
    # one pass over the vectors when y is accepted, a second one only when
    # it is rejected (the acceptance test is a global reduction):
    #   product: indices, values, field, x^(k) (read with its
    #            gathers), x^(k-1), z_(k-1) read, z_k and x^(k+1) = T(y)
    #            written
    #   repair : x^(k), z_k read, x^(k+1) = T(x) written, rejected
    #            iterations only
    rejected = float(np.mean(acc == 0))
    # the product on 4-entry rows computes the row starts and streams the
    # library's 8-bit copy of the +-1 values and 16-bit column offsets
    info = L.ising_get_info(ctx)
    vb, cb = info.step_val_bytes, info.step_col_bytes
    kname = (f"adoch_mv_kernel<{'signed char' if vb == 1 else 'float'}, float, true, 4, 1, true"
             + (", short>" if cb == 2 else ">"))
    traffic = load_traffic(kname, f"adoch_torus{args.L}", ADOCH_SOURCES)
    prod = (cb + vb) * nnz + 4 * n + 5 * 8 * np1
    upd = 3 * 8 * np1
    bytes_iter = prod + rejected * upd
    achieved = bytes_iter / (it_us * 1e-6) / 1e9
    print(json.dumps({
        "metric": "edge-updates/s", "value": nnz * iters / dt, "unit": "edge-updates/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * dt,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic (seeded torus lattice generator)",
        "config": {"workload": f"ADOCH (Alg. 2, q=5) on the 2D periodic lattice {args.L}x{args.L} "
                               f"({n} spins, {nnz} stored couplings +-1, field h~N(0,0.1^2)), "
                               f"{iters} iterations per step + parameters + energy",
                   "n": n, "nnz": nnz, "iters": iters, "x_storage": "f64", "q": 5},
        "iteration_us": it_us, "energy": float(E.cpu()[0]),
        "accepted_fraction": float(np.mean(acc)),
        "roofline": {"kernel": kname + " + adoch_update_kernel<1, true>",
                     "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     # HBM bytes per launch of the product (rocprofv3 counters
                     # scaled by a copy of known size), if taken on this source
                     "traffic": traffic["hbm_bytes_per_launch"] if traffic else None,
                     "algorithmic_bytes_per_iteration": bytes_iter,
                     "bytes_product": prod, "bytes_repair": upd, "rejected_fraction": rejected},
    }), flush=True)
    L.ising_destroy(ctx)


def bench_adoch_dense(args):
    """ADOCH (Alg. 2, q = 5) on dense couplings against DOCH on the same
    starts: the stored SK instance n = 1024 (1000 iterations) or the
    generated couplings sin(i j + 100), n = 65536 (10 iterations), for one
    restart and for 8 restarts at once (each generated coupling or loaded
    J_ij then serves all 8).  Iterations per second, edge-updates/s and the
    energies reached; the oracle's ADOCH as the host baseline with parity of
    the GPU run (SK: the same run; generated: the same rule at n = 4096,
    since the oracle holds J in memory)."""
    import numpy as np
    import torch

    import ising_inputs as gen
    import oracle as orc
    import paper_2509_01928_amd as L
    d = "cuda:0"
    if args.adoch_instance == "sk1024":
        seed, xseed = gen.SEEDS["sk1024"]
        n, iters = 1024, 1000
        J = gen.sk_dense(n, seed)
        Jd = torch.from_numpy(J).to(d)
        ctx = L.ising_create_dense(n, Jd, L.ISING_F64, n)
        label = "dense SK n=1024, J~N(0,1)"
    else:
        n, iters = args.proc_n, 10
        ctx = L.ising_create_procedural(n, 1, 100.0)
        xseed = 2007
        label = f"generated couplings sin(ij+100), n={n}"
    p, lam = L.ising_default_params(ctx, 1.0, 0)
    out = {"metric": "edge-updates/s", "unit": "edge-updates/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f64", "data": "synthetic" if args.adoch_instance == "sk1024" else "procedural",
           "config": {"workload": f"ADOCH (Alg. 2, q=5) vs DOCH on {label}, {iters} iterations, "
                                  f"1 and 8 restarts", "n": n, "iters": iters, "q": 5}}
    runs = {}
    for R in (1, 8):
        X0 = gen.uniform_x0(n, R, xseed)
        xd = torch.from_numpy(np.ascontiguousarray(X0)).to(d)
        so = torch.empty((n, R), dtype=torch.int8, device=d)
        E = torch.empty(R, dtype=torch.float64, device=d)
        for algo in (0, 1):
            if algo == 0 and R > 1:
                continue                     # DOCH on one context runs one restart at a time
            q = L.ising_params()
            q.alpha, q.beta, q.eps, q.algo, q.q, q.x_dtype, q.reserved = p.alpha, p.beta, 0.0, algo, 5, L.ISING_F64, 0

            def step():
                L.ising_solve(ctx, xd, R, iters, q, None, so, want_stats=False)
                L.ising_energy(ctx, so, R, E)

            dt = _timed(step, args.warmup, args.steps)
            key = f"{'adoch' if algo else 'doch'}_R{R}"
            runs[key] = {"ms_per_solve": 1e3 * dt, "iteration_us": 1e6 * dt / iters,
                         "edge_updates_per_s": float(n) * (n - 1) * R * iters / dt,
                         "energies": [float(v) for v in E.cpu().numpy()]}
            log(f"{key}: {1e6 * dt / iters:.1f} us/iteration, best E {min(runs[key]['energies']):.2f}")
    out["runs"] = runs
    out["value"] = runs["adoch_R8"]["edge_updates_per_s"]
    out["ms_per_step"] = runs["adoch_R8"]["ms_per_solve"]
    if not args.no_cpu_baseline:
        # the oracle's ADOCH, and the GPU's on the same start, compared
        if args.adoch_instance == "sk1024":
            Jo, no, it_o, lab = J, n, iters, "the same instance and start"
        else:
            no, it_o = 4096, 10
            i = np.arange(no, dtype=np.float64)
            Jo = np.sin(np.outer(i, i) + 100.0)
            np.fill_diagonal(Jo, 0.0)
            lab = "the same rule at n=4096 (the oracle holds J in memory)"
        log(f"oracle ADOCH on {lab}")
        B = orc.csr_of_dense(Jo)
        x0 = gen.uniform_x0(no, 1, xseed)[:, 0]
        # the sample's parameters by the O(nnz) estimate, on both sides
        a2, b2 = (p.alpha, p.beta) if no == n else orc.default_params(B, 1.0, method="wigner")[:2]
        t0 = time.perf_counter()
        tr = orc.adoch(B, x0, a2, b2, it_o, 5)
        dt_cpu = time.perf_counter() - t0
        ctx2 = ctx if no == n else L.ising_create_procedural(no, 1, 100.0)
        q = L.ising_params()
        q.alpha, q.beta, q.eps, q.algo, q.q, q.x_dtype, q.reserved = a2, b2, 0.0, 1, 5, L.ISING_F64, 0
        xd = torch.from_numpy(x0).to(d)
        xo = torch.empty_like(xd)
        so = torch.empty(no, dtype=torch.int8, device=d)
        L.ising_solve(ctx2, xd, 1, it_o, q, xo, so)
        torch.cuda.synchronize()
        out["parity"] = iterate_parity(xo.cpu().numpy(), tr.x, so.cpu().numpy(), orc.sign(tr.x))
        out["parity"]["sample"] = lab
        if ctx2 is not ctx:
            L.ising_destroy(ctx2)
        out["cpu_baseline"] = {"value": float(no) * (no - 1) * it_o / dt_cpu, "unit": "edge-updates/s",
                               "cores": 1, "kind": "oracle",
                               "sample": f"{it_o} ADOCH iterations of the single-threaded FP64 oracle on "
                                         f"{lab} ({dt_cpu:.2f} s)", **host_info()}
        log(f"parity {out['parity']}")
    print(json.dumps(out), flush=True)
    L.ising_destroy(ctx)


def bench_procedural(args):
    """Procedural dense couplings J_ij = sin(i j + 100) (Supp. Note 9,
    NEXT-3), generated in FP64 on the fly: n = 65536, 10 DOCH iterations per
    step, Wigner parameters, FP64 energy.  Bound by the FP64 arithmetic of
    the sine."""
    import numpy as np
    import torch

    import ising_inputs as gen
    import paper_2509_01928_amd as L
    n = args.proc_n
    ctx = L.ising_create_procedural(n, 1, 100.0)
    x0 = gen.uniform_x0(n, 1, 2007)[:, 0]
    d = "cuda:0"
    xd = torch.from_numpy(x0).to(d)
    so = torch.empty(n, dtype=torch.int8, device=d)
    E = torch.empty(1, dtype=torch.float64, device=d)
    p, lam = L.ising_default_params(ctx, 1.0, 0)
    iters = 10
    solve_ms = []

    def step():
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        L.ising_solve(ctx, xd, 1, iters, p, None, so, want_stats=False)
        e1.record()
        L.ising_energy(ctx, so, 1, E)
        solve_ms.append((e0, e1))

    dt = _timed(step, args.warmup, args.steps)
    torch.cuda.synchronize()
    it_us = 1e3 * float(np.mean([a.elapsed_time(b) for a, b in solve_ms[args.warmup:]])) / iters
    couplings = n * (n - 1)
    flops = load_flops("dense_step_kernel", f"procedural{n}")
    # the method's arithmetic: one multiply and one add per coupling
    # (J_ij x_j); how J_ij is produced is the implementation's, so the
    # counted flops (generator included) are reported as issue efficiency
    achieved = METHOD_FLOPS_PER_COUPLING * couplings / (it_us * 1e-6) / 1e12
    roof = {"kernel": "dense_step_kernel<double, double, false, SinJ>", "bound": "alu",
            "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s", "achieved": achieved,
            "frac": achieved / FP64_PEAK_TFLOPS, "method_flops_per_coupling": METHOD_FLOPS_PER_COUPLING,
            "couplings_per_s": couplings / (it_us * 1e-6)}
    if flops:
        counted = flops["fp64_flops_per_coupling"] * couplings / (it_us * 1e-6) / 1e12
        roof["issue"] = {"fp64_flops_per_coupling_counted": flops["fp64_flops_per_coupling"],
                         "achieved": counted, "frac": counted / FP64_PEAK_TFLOPS}
    print(json.dumps({
        "metric": "edge-updates/s", "value": couplings * iters / dt, "unit": "edge-updates/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * dt,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "procedural (J_ij = sin(i j + 100), generated on the fly)",
        "config": {"workload": f"procedural dense couplings sin(ij+100), n={n}, {iters} DOCH "
                               f"iterations per step + energy (FP64)", "n": n, "iters": iters},
        "iteration_us": it_us, "energy": float(E.cpu()[0]), "lambda_hat": lam,
        "roofline": roof,
    }), flush=True)
    L.ising_destroy(ctx)


def bench_tune_eta(args):
    """eta tuning by short probe runs (Supp. Note 6, NEXT-4): 8 values of eta
    in (0, 2], 10 probe iterations each (FP64 iterates) and the energy of the
    rounded spins; the best eta's parameters are kept.  On a CSR context the
    probes run as restarts of one pass over the couplings; the same probes
    one eta per call give the sequential reference.  --tune-instance picks
    the 10^8-spin lattice (streaming-bound) or the Supp. Alg. S5 instance of
    10^8 spins and ~10^9 couplings (random-gather-bound)."""
    import numpy as np
    import torch

    import ising_inputs as gen
    import paper_2509_01928_amd as L
    d = "cuda:0"
    field = args.tune_instance == "torus"
    if args.tune_instance == "procedural":
        n = args.proc_n

        class _P:                         # shape of the instance for the accounting below
            pass
        A = _P()
        A.n, A.nnz = n, n * (n - 1)
        x0 = gen.uniform_x0(n, 1, 2007)[:, 0]
        ctx = L.ising_create_procedural(n, 1, 100.0)
        label = f"procedural couplings sin(ij+100), n={n}"
    elif args.tune_instance == "s5":
        n = args.s5_n
        A = gen.s5_csr(n, 100.0 * 10.0 / (n - 1), 1006)
        x0 = gen.uniform_x0(n, 1, 2006)[:, 0]
        rp = torch.from_numpy(A.row_ptr).to(d)
        col = torch.from_numpy(A.col).to(d)
        val = torch.from_numpy(A.val.astype(np.int16)).to(d)
        ctx = L.ising_create_csr(A.n, A.nnz, rp, col, val, L.ISING_I16)
        del rp, col, val
        torch.cuda.empty_cache()
        label = f"Supp. Alg. S5 instance n={A.n}, mean degree 10, int16 values, h=0"
    else:
        A, x0, ctx = _torus_ctx(args.L)
        label = f"2D periodic lattice {args.L}x{args.L} with field"
    xd = torch.from_numpy(x0).to(d)
    etas = np.array([0.25, 0.5, 0.75, 1.0, 1.25, 1.5, 1.75, 2.0])
    probe = 10
    out = {}

    def step():
        out["r"] = L.ising_tune_eta(ctx, xd, etas, probe)

    dt = _timed(step, args.warmup, args.steps)
    best, best_eta, energies = out["r"]

    def sequential():
        out["e"] = [L.ising_tune_eta(ctx, xd, etas[k:k + 1], probe)[2][0] for k in range(len(etas))]

    dt_seq = _timed(sequential, 0, 1)
    # the same spins; the energies' field sums may differ in the last bits
    # (the 8-restart energy adds its workgroups' sums in another order)
    assert np.allclose(np.array(out["e"]), energies, rtol=1e-12, atol=1e-6), "batched and sequential probes differ"
    n, nnz = A.n, A.nnz
    # one pass per probe iteration for all 8 probes: offsets (not read with
    # 4-entry rows, whose starts are computed), indices and values (the
    # library's 8-bit copy of the lattice's +-1 on 4-entry rows), the field,
    # and 8 FP64 iterates read and written (the procedural couplings are
    # generated, not read)
    if args.tune_instance == "procedural":
        bytes_iter = 2 * 8 * len(etas) * n
    else:
        info = L.ising_get_info(ctx)
        four = info.row_len == 4
        vb = info.step_val_bytes if four else (2 if args.tune_instance == "s5" else 4)
        cb = 4                  # the sweep keeps the int32 column indices
        bytes_iter = ((0 if four else 4 * (n + 1)) + (cb + vb) * nnz + (4 * n if field else 0)
                      + 2 * 8 * len(etas) * (n + 1))
    sweep_bytes = bytes_iter * probe
    if args.tune_instance == "procedural":
        # FP64 flops per coupling and probe, counted on the sweep kernel, over
        # the wall time of whole sweeps (energies and setup included)
        fl = load_flops("dense_sin_sweep_kernel", f"sweep_procedural{n}_R{len(etas)}", SWEEP_SOURCES)
        cps = nnz * len(etas) * probe / dt
        ach = METHOD_FLOPS_PER_COUPLING * cps / 1e12
        sweep_roof = {"kernel": f"dense_sin_sweep_kernel<{len(etas)}>", "bound": "alu",
                      "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s", "coupling_probes_per_s": cps,
                      "achieved": ach, "frac": ach / FP64_PEAK_TFLOPS,
                      "method_flops_per_coupling_probe": METHOD_FLOPS_PER_COUPLING}
        if fl:
            counted = fl["fp64_flops_per_coupling"] * cps / 1e12
            sweep_roof["issue"] = {"fp64_flops_per_coupling_probe_counted": fl["fp64_flops_per_coupling"],
                                   "achieved": counted, "frac": counted / FP64_PEAK_TFLOPS}
    print(json.dumps({
        "metric": "eta candidates/s", "value": len(etas) / dt, "unit": "candidates/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * dt,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"eta sweep of {len(etas)} values x {probe} probe iterations on the "
                               f"{label} (FP64 iterates), probes as restarts of one pass",
                   "n": n, "nnz": nnz, "etas": etas.tolist(), "probe_iters": probe},
        "sequential_ms_per_sweep": 1e3 * dt_seq, "speedup_vs_sequential": dt_seq / dt,
        "probe_edge_updates_per_s": nnz * probe * len(etas) / dt,
        "best_eta": best_eta, "probe_energies": energies.tolist(),
        # the batched pass's algorithmic bytes over the wall time of whole
        # sweeps (energies and parameter setting included)
        "roofline": (sweep_roof if args.tune_instance == "procedural" else
                     {"kernel": "csr_sweep_kernel" + (f"<signed char, float, true, 8, 4{', short' if cb == 2 else ''}>"
                                                      if field and vb == 1 else ""),
                      "bound": "hbm",
                      "achieved": sweep_bytes / dt / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                      "frac": sweep_bytes / dt / 1e9 / HBM_PEAK_GBS,
                      "algorithmic_bytes_per_iteration": bytes_iter}),
    }), flush=True)
    L.ising_destroy(ctx)


def bench_copy_calib(args):
    """A plain device copy of known size (1 GiB read, 1 GiB written per
    launch, torch's elementwise copy kernel): the reference that scales the
    FETCH_SIZE / WRITE_SIZE counters of the step kernels to bytes, and the
    device's copy bandwidth."""
    import torch
    nbytes = 1 << 30
    src = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda:0").uniform_()
    dst = torch.empty_like(src)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    for _ in range(args.warmup):
        dst.copy_(src)
    torch.cuda.synchronize()
    ev[0].record()
    for _ in range(args.steps):
        dst.copy_(src)
    ev[1].record()
    torch.cuda.synchronize()
    ms = ev[0].elapsed_time(ev[1]) / args.steps
    gbs = 2 * nbytes / (ms * 1e-3) / 1e9
    print(json.dumps({"metric": "copy GB/s (read + write)", "value": gbs, "unit": "GB/s",
                      "bytes_read_per_launch": nbytes, "bytes_written_per_launch": nbytes,
                      "ms_per_launch": ms, "frac_of_hbm_peak": gbs / HBM_PEAK_GBS}), flush=True)


def full_scale_parity(orc, B, x0, alpha, beta, iters, tr, gpu_par):
    """Compare the GPU's first iterations on the whole instance with the
    oracle's: FP64 iterates against the oracle's trajectory; FP32 storage
    against the oracle's FP64 step applied to FP32-rounded iterates (one
    oracle iteration at a time, the iterate rounded to FP32 in between)."""
    import numpy as np
    out = {"iterations": iters}
    for name, (xg, sg, _, _) in gpu_par.items():
        if name == "f64":
            xr = tr.x
        else:
            xr = np.asarray(x0, dtype=np.float32).astype(np.float64)
            for _ in range(iters):
                xr = orc.doch(B, xr, alpha, beta, 1).x.astype(np.float32).astype(np.float64)
        scale = float(np.abs(xr).max())
        dx = np.abs(xg - xr)
        s_ref = orc.spins_with_field(xr)
        diff = np.nonzero(sg != s_ref)[0]
        tiny = np.abs(xr[:-1][diff]) < 1e-6 * scale
        rec = {"max_abs_dx": float(dx.max()), "max_dx_over_xinf": float(dx.max()) / scale,
               "x_inf": scale, "spin_mismatches": int(diff.size),
               "spin_mismatches_scale_aware": int(diff.size - int(tiny.sum()))}
        if name == "f32":
            rec["bit_equal_frac"] = float(np.mean(xg == xr))
        out[name] = rec
    return out


def main():
    args = parse()
    if args.ingest_pmc:
        if args.pmc_family == "adoch":
            ingest_pmc(args.ingest_pmc, f"adoch_torus{args.L}", "adoch")
        else:
            ingest_pmc(args.ingest_pmc, f"torus{args.L}_{args.x_dtype}")
        return
    if args.ingest_flops:
        ingest_flops(args.ingest_flops, args.proc_n)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "the library runs on one GPU only; multi-GPU sharding is a "
                                   "design note, not an implemented path", "n_gpus": args.gpus}))
        sys.exit(2)
    if args.workload != "torus":
        {"er20000": bench_er20000, "sk1024": bench_sk1024, "dense4096": bench_dense4096,
         "batch512": bench_batch512, "s5": bench_s5, "adoch": bench_adoch,
         "procedural": bench_procedural, "tune_eta": bench_tune_eta, "adoch_dense": bench_adoch_dense,
         "copy_calib": bench_copy_calib}[args.workload](args)
        return
    import numpy as np
    import torch

    import ising_inputs as gen
    import paper_2509_01928_amd as L

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    seed, xseed = gen.SEEDS["torus1e4"]
    t0 = time.time()
    A = gen.torus_csr(args.L, seed, h_std=0.1)
    x0 = gen.uniform_x0(A.n + 1, 1, xseed)[:, 0]
    log(f"generated torus L={args.L}: n={A.n} nnz={A.nnz} in {time.time() - t0:.1f}s")

    rp = torch.from_numpy(A.row_ptr).to(dev)
    col = torch.from_numpy(A.col).to(dev)
    val = torch.from_numpy(A.val).to(dev)
    h = torch.from_numpy(A.h).to(dev)
    xd = torch.from_numpy(x0).to(dev)
    ctx = L.ising_create_csr(A.n, A.nnz, rp, col, val, L.ISING_F32, h, L.ISING_F32)
    del rp, col, val, h
    torch.cuda.empty_cache()
    s_out = torch.empty(A.n, dtype=torch.int8, device=dev)
    E = torch.empty(1, dtype=torch.float64, device=dev)
    x_dtype = L.ISING_F32 if args.x_dtype == "f32" else L.ISING_F64
    info = L.ising_get_info(ctx)
    row_len, val_bytes, col_bytes = info.row_len, info.step_val_bytes, info.step_col_bytes
    log(f"context created (constant row length {row_len}, {val_bytes} B per value in the lane-per-row step)")
    # launch-shape tuning is setup, outside the timed region
    if args.geometry >= -1:
        L.ising_set_geometry(ctx, args.geometry, args.wg_per_cu)
        geometry, wg_per_cu = args.geometry, args.wg_per_cu
        if geometry == -1:        # the library's choice from the size and mean row length
            geometry, wg_per_cu = L.ising_get_info(ctx).geometry, 0
    else:
        p0, _ = L.ising_default_params(ctx, 1.0, 0)
        p0.x_dtype = x_dtype
        geometry, wg_per_cu, tune_ms = L.ising_autotune(ctx, xd, 30, p0)
        log(f"autotune: geometry {geometry}, {wg_per_cu} workgroups/CU "
            f"({', '.join(f'{m * 1e3:.0f}' for m in tune_ms)} us/iteration per geometry)")

    solve_ms = []

    def step(record):
        p, lam = L.ising_default_params(ctx, 1.0, 0)          # a1
        p.x_dtype = x_dtype
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        ev0.record()
        L.ising_solve(ctx, xd, 1, args.iters, p, None, s_out, want_stats=False)   # a2-a6
        ev1.record()
        L.ising_energy(ctx, s_out, 1, E)                       # a7
        if record:
            solve_ms.append((ev0, ev1))
        return p, lam

    for _ in range(args.warmup):
        step(False)
    torch.cuda.synchronize()
    log("warmup done")
    t_start = time.perf_counter()
    for _ in range(args.steps):
        p, lam = step(True)
    torch.cuda.synchronize()
    t_end = time.perf_counter()
    elapsed = t_end - t_start
    ms_per_step = 1e3 * elapsed / args.steps
    per_iter_ms = float(np.mean([a.elapsed_time(b) for a, b in solve_ms])) / args.iters
    energy = float(E.cpu()[0])
    log(f"{ms_per_step:.1f} ms/step, {per_iter_ms * 1e3:.1f} us/iteration, E={energy:.1f}")

    n, nnz, np1 = A.n, A.nnz, A.n + 1
    xb = 4 if args.x_dtype == "f32" else 8
    # algorithmic bytes of one fused iteration in the stated CSR format: row
    # offsets, column indices and values once, iterate read once and written
    # once, field once (12 B per edge-update with an FP32 iterate)
    bytes_iter = 4 * (n + 1) + 4 * nnz + 4 * nnz + xb * np1 + xb * np1 + 4 * n
    csr_gbs = bytes_iter / (per_iter_ms * 1e-3) / 1e9
    # with a constant row length the lane-per-row kernels compute the row
    # offsets instead of reading them; with small-integer values (the
    # lattice's +-1) they stream the library's exact 8-bit copy of the
    # values, and on 4-entry rows whose columns lie within 32767 of their row
    # (cyclically) the 16-bit column offsets, so the bytes the step needs
    # are 6 B per edge-update; the headline fraction is taken on those, the
    # CSR-format figure is kept beside it
    rowlane = geometry in (3, 4)
    implicit = row_len > 0 and rowlane
    vb = val_bytes if rowlane else 4
    cb = col_bytes if rowlane else 4
    kernel_bytes = bytes_iter - (4 * (n + 1) if implicit else 0) - (4 - vb) * nnz - (4 - cb) * nnz
    achieved = kernel_bytes / (per_iter_ms * 1e-3) / 1e9
    workload = f"torus{args.L}"
    kernel = step_kernel_name(geometry, args.x_dtype, implicit, vb, cb)
    traffic = load_traffic(kernel, f"{workload}_{args.x_dtype}")
    edge_updates = float(nnz) * args.iters * args.steps
    out = {
        "metric": "edge-updates/s",
        "value": edge_updates / elapsed,
        "unit": "edge-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded torus lattice generator)",
        "config": {
            "workload": f"2D periodic lattice {args.L}x{args.L} ({n} spins, {nnz} stored "
                        f"couplings +-1), field h~N(0,0.1^2) as an extra spin, "
                        f"{args.iters} DOCH iterations per step + parameter setting + "
                        f"sign rounding + Ising energy",
            "n": n, "nnz": nnz, "iters": args.iters, "restarts": 1,
            "x_storage": args.x_dtype, "couplings": "f32 CSR, int32 indices",
            "arithmetic": "f64", "parallelism": "single GPU",
            "kernel_geometry": geometry, "workgroups_per_cu": wg_per_cu,
            "row_offsets": (f"implicit (every row holds {row_len} entries)" if implicit else "read"),
            "values_streamed": ("8-bit copy (every value an integer in [-128, 127])" if vb == 1
                                else "f32 as stored"),
            "columns_streamed": ("16-bit cyclic offsets col - i (every one within 32767)" if cb == 2
                                 else "int32 as stored"),
        },
        "iteration_us": per_iter_ms * 1e3,
        "energy": energy,
        "lambda_hat": lam,
        "roofline": {
            "kernel": kernel,
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": (traffic["hbm_bytes_per_launch"] if traffic else None),
            "algorithmic_bytes_per_launch": kernel_bytes,
            "csr_format_bytes_per_launch": bytes_iter,
            "csr_format_gbs": csr_gbs,
            "csr_format_frac": csr_gbs / HBM_PEAK_GBS,
        },
    }
    # Full-scale parity, outside the timed region: the first cpu_iters
    # iterations of the whole instance on the GPU with the measured launch
    # shape, FP64 iterates and the measured FP32 storage, compared below with
    # the oracle's iterations of the CPU baseline.
    gpu_par = {}
    if not args.no_cpu_baseline and args.cpu_iters > 0:
        p_par, _ = L.ising_default_params(ctx, 1.0, 0)
        for name, xt in (("f64", L.ISING_F64), ("f32", L.ISING_F32)):
            p_par.x_dtype = xt
            xo = torch.empty_like(xd)
            so = torch.empty(A.n, dtype=torch.int8, device=dev)
            L.ising_solve(ctx, xd, 1, args.cpu_iters, p_par, xo, so)
            torch.cuda.synchronize()
            gpu_par[name] = (xo.cpu().numpy(), so.cpu().numpy(), p_par.alpha, p_par.beta)
            del xo, so
        log(f"parity runs: {args.cpu_iters} iterations on the GPU in FP64 and FP32 storage")
    L.ising_destroy(ctx)
    del xd, s_out
    torch.cuda.empty_cache()

    if not args.no_cpu_baseline and args.cpu_iters > 0:
        import oracle as orc
        log("CPU baseline: building the oracle's matrix")
        B = orc.problem_matrix(A)
        del A
        a_ref, b_ref, _ = orc.default_params(B, 1.0, method="wigner")
        # both sides iterate with the same alpha and beta (the library's);
        # the oracle's own estimates are compared with them separately
        a_gpu, b_gpu = gpu_par["f64"][2], gpu_par["f64"][3]
        t0 = time.perf_counter()
        tr = orc.doch(B, x0, a_gpu, b_gpu, args.cpu_iters)
        dt = time.perf_counter() - t0
        out["parity"] = full_scale_parity(orc, B, x0, a_gpu, b_gpu, args.cpu_iters, tr, gpu_par)
        out["parity"]["alpha_rel_diff"] = abs(a_gpu - a_ref) / abs(a_ref)
        out["parity"]["beta_rel_diff"] = abs(b_gpu - b_ref) / abs(b_ref)
        log(f"parity: {out['parity']}")
        out["cpu_baseline"] = {
            "value": float(nnz) * args.cpu_iters / dt,
            "unit": "edge-updates/s",
            "cores": 1,
            "kind": "oracle",
            "sample": f"full {n}-spin instance, {args.cpu_iters} DOCH iterations of the "
                      f"single-threaded FP64 oracle ({dt:.1f} s), iteration loop only",
            "host_cpus": os.cpu_count(),
        }
        log(f"CPU baseline {out['cpu_baseline']['value']:.3e} edge-updates/s")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
