#!/usr/bin/env python3
"""Benchmark of the hot path on one MI355X.

Workload (default): the kite x(t) = (cos t + 0.65 cos 2t - 0.65, 1.5 sin t)
with N = 4096 elements (8192 x 8192 complex128 system), host wavenumber
k0 = 20 and two interior cases, k1 = 30 and lossy k1 = 30 + 0.3i, 16
equispaced plane-wave angles solved as one block by GMRES(100) to a relative
residual of 1e-10, far field at 360 directions; everything in FP64.

One step = both cases, each: derive the geometry tables on the device,
assemble the matrix, build the 16 right-hand sides, solve, evaluate the far
field; the two cases run concurrently, each on its own stream driven by its
own host thread, and start every step together (--sequential-cases: one
after the other; --case-pipeline: each case runs its steps back to back
without that barrier).  The inputs (node
coordinates) are uploaded once before the timed region.  value = solved
right-hand sides per second over the K timed steps.

Also reported: the time of one case (16 solves), the assembly rate, the
roofline record of the dominant kernel measured with the library's HIP events
on the solve stream (and the same kernel with the cases one after another,
two steps after the timed region), the precision path (FP32 products + FP64
refinement on the kite of 16384 elements against the FP64 path), the served
stream (capacity of the mixed and FP64 servers and open-loop p50/p99 latency
on a prefix of the request stream), the disk of 256 elements, and the CPU
oracle: modelled from a timed sample on one core and as one concurrent copy
per available core (at most 16), and the disk's whole solve timed in full.

Other workloads (--workload): disk256 (unit disk, N = 256), sectors (three
material sectors with junctions, about 7500 graded elements), kite16384_mixed
(the precision path: N = 16384, FP32 matrix and products with FP64 residual
refinement, 64 angles; also reports the FP64 path on the same workload and the
far-field error of both against an FP64 solution).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME] [--mode full|matvec]
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
WORKLOAD_FACTORIES = {"kite4096": lambda W: W.workload_kite4096, "disk256": lambda W: W.workload_disk256,
                      "sectors": lambda W: W.workload_sectors,
                      "kite16384_mixed": lambda W: W.workload_kite16384_fp32}
FP32_MFMA_PEAK_TFS = 157.3
VALU_PEAK_FLOPS = 78.6e12  # FP64 vector; also FP32 vector without packed FP32 (the kernels are compiled without it)
METRIC = "solves/s + p50/p99 latency at 1e-6 rel. err vs FP64; assembly FLOP/s, matvec GB/s"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def sources_sha(files):
    h = hashlib.sha256()
    for f in files:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    return h.hexdigest()[:16]


def counter_record(kind, workload):
    """Committed rocprofv3 PMC summary (profiles/<kind>_<workload tag>.json) if
    it was taken on the current kernel sources; else None."""
    path = os.path.join(ROOT, "profiles", f"{kind}_{workload.split('_')[0]}.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("source_sha") != sources_sha(rec.get("source_files", [])):
        return None
    return rec


def traffic_record(workload):
    """HBM bytes per launch of the product kernel (FETCH_SIZE + WRITE_SIZE, each
    scaled by a plain copy of known size), or None."""
    rec = counter_record("matvec_traffic", workload)
    return rec.get("bytes_per_launch") if rec else None


def cpu_model():
    """The host CPU's model name (Linux /proc/cpuinfo), or None."""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def arnoldi_units(rhs_steps, restart, n):
    """(basis vector x row) units of modified Gram-Schmidt that a GMRES(restart)
    solve with these Krylov step counts (one per right-hand side) does: step j
    of a cycle projects on j + 1 basis vectors of n rows."""
    u = 0
    for s in rhs_steps:
        s = int(s)
        while s > 0:
            c = min(restart, s)
            u += c * (c + 1) // 2
            s -= c
    return float(u) * n


def arnoldi_unit_seconds():
    """Seconds per (basis vector x row) unit of the oracle's Gram-Schmidt:
    its GMRES(600) run for 600 steps on an order-1024 matrix (3 I plus a
    scaled random matrix: no early stop), minus its 602 products timed alone
    (the product is the same routine); 180 300 x 1024 units."""
    import oracle as O
    n, m = 1024, 600
    rng = np.random.default_rng(0)
    A = np.asfortranarray(3.0 * np.eye(n) + (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)))
                          / np.sqrt(n))
    b = np.ones(n, dtype=np.complex128)
    x = np.ones(n, dtype=np.complex128)
    O.matvec(A, x)
    t0 = time.perf_counter()
    for _ in range(40):
        O.matvec(A, x)
    t_mv = (time.perf_counter() - t0) / 40
    t0 = time.perf_counter()
    _, it, _, _ = O.gmres(A, b, m, 0.0, m)
    T = time.perf_counter() - t0
    units = m * (m + 1) / 2 * n
    return max(0.0, T - (it + 2) * t_mv) / units, T + 40 * t_mv


def oracle_sample(workload, products, arn_units, rows_per_case=None, start_at=None):
    """Time the oracle (single thread) on a bounded sample of the workload and
    model its whole solve from it: strided matrix rows of each case (48 at
    N = 4096, fewer for larger N) scaled to the full assembly, one product of
    at most 8192 x 8192 scaled to the full product size and to the products
    the GPU solve needed (GMRES steps and restart residuals), and the
    Gram-Schmidt work of those steps (arnoldi_unit_seconds x arn_units).
    start_at: wall-clock time (time.time) to wait for once the inputs are
    prepared, so that concurrent copies time the same interval.  Returns
    (modelled seconds for the workload's solves, seconds spent, rows per
    case, product size, seconds per Gram-Schmidt unit)."""
    import oracle as O
    cases = []
    for spec in workload.problems:
        P = O.Problem(spec)
        n = P.n
        rows_n = min(n, rows_per_case or max(12, int(48 * 8192 / n)))
        rows = np.linspace(0, n - 1, rows_n).round().astype(np.int32)
        mv_n = min(n, 8192)
        cases.append((P, n, rows, mv_n))
    # written, not just allocated: untouched pages of a fresh allocation all
    # map the kernel's one zero page, and a product over them runs from cache
    A = np.empty((cases[0][3], cases[0][3]), dtype=np.complex128, order="F")
    A.fill(0.5 + 0.25j)
    if start_at is not None:
        time.sleep(max(0.0, start_at - time.time()))
    c_arn, spent = arnoldi_unit_seconds()
    t_total = 0.0
    for (P, n, rows, mv_n), nprod, units in zip(cases, products, arn_units):
        t0 = time.perf_counter()
        P.assemble_rows(rows)
        t_rows = time.perf_counter() - t0
        if A.shape[0] != mv_n:
            A = np.empty((mv_n, mv_n), dtype=np.complex128, order="F")
            A.fill(0.5 + 0.25j)
        x = np.ones(mv_n, dtype=np.complex128)
        t0 = time.perf_counter()
        O.matvec(A, x)
        t_mv = time.perf_counter() - t0
        spent += t_rows + t_mv
        t_total += t_rows / len(rows) * n + nprod * t_mv * (n / mv_n) ** 2 + c_arn * units
    return t_total, spent, len(cases[-1][2]), cases[-1][3], c_arn


def oracle_full_solve():
    """The oracle's whole solve of the unit disk as a 256-gon (k0 = 1, k1 = 2,
    one plane wave, 8-point Gauss): assembly of the 512 x 512 system, its
    GMRES(50) to 1e-10 and the far field at 360 directions, single thread,
    timed end to end (no model)."""
    import oracle as O
    import workloads as W
    wl = W.workload_disk256()
    t0 = time.perf_counter()
    po = O.Problem(wl.problems[0])
    A = po.assemble()
    b = po.rhs(wl.angles)[:, 0]
    x, it, rel, ok = O.gmres(A, b, wl.restart, wl.tol)
    po.farfield(x.reshape(-1, 1), wl.far_dirs)
    T = time.perf_counter() - t0
    return {"workload": wl.name, "seconds_per_solve": T, "value": 1.0 / T, "unit": "solves/s", "cores": 1,
            "gmres_iterations": int(it), "converged": bool(ok),
            "what": "oracle assembly + GMRES(50) to 1e-10 + far field at 360 directions, measured end to end"}


def cpu_baseline(workload, wl_key, products, arn_units, gpu_value):
    """The oracle on one core (the record's value), then the same sample in P
    concurrent worker processes, one per available core (at most 16), each
    pinned to its core and started together: their summed rate is the CPU
    throughput on P cores (requests and right-hand sides are independent).
    The workload's solves are modelled from the sample (the full oracle solve
    of the 8192 x 8192 systems would take about an hour); the disk of 256
    elements is solved by the oracle in full."""
    t_total, spent, rows_n, mv_n, c_arn = oracle_sample(workload, products, arn_units)
    solves = len(workload.problems) * len(workload.angles)
    one = solves / t_total
    cores = sorted(os.sched_getaffinity(0))[:16]
    import subprocess
    start = time.time() + 4.0 + 0.5 * len(cores)
    cmd = [sys.executable, os.path.abspath(__file__), "--cpu-worker", "--workload", wl_key,
           "--cpu-iters", ",".join(str(int(i)) for i in products),
           "--cpu-arn", ",".join(repr(float(u)) for u in arn_units), "--cpu-start-at", repr(start)]
    env = dict(os.environ, OMP_NUM_THREADS="1")
    procs = [subprocess.Popen(cmd + ["--cpu-core", str(c)], stdout=subprocess.PIPE, stderr=subprocess.PIPE, env=env)
             for c in cores]
    rates, errs = [], []
    for p in procs:
        out, err = p.communicate(timeout=900)
        if p.returncode == 0:
            rates.append(solves / json.loads(out.decode().strip().splitlines()[-1])["t_total"])
        else:
            errs.append(err.decode()[-300:])
    par = {"processes": len(cores), "completed": len(rates), "value": float(sum(rates)), "unit": "solves/s",
           "per_process_min": float(min(rates)) if rates else None,
           "per_process_max": float(max(rates)) if rates else None}
    if errs:
        par["errors"] = errs
    full = oracle_full_solve()
    return {"value": one, "unit": "solves/s", "cores": 1, "kind": "oracle", "modelled": True,
            "host_cores_available": len(os.sched_getaffinity(0)), "cpu_model": cpu_model(),
            "sample": (f"MODELLED from a timed sample: {rows_n} strided rows per case assembled by the oracle "
                       f"(FP64), scaled to {workload.problems[0].order} rows; one {mv_n} x {mv_n} oracle product, "
                       f"scaled to the full product size and to the {int(sum(products))} products the GPU solves "
                       f"used; the oracle's Gram-Schmidt at {c_arn * 1e9:.2f} ns per (basis vector x row) "
                       f"(its GMRES(600) on an order-1024 matrix minus its products) times the "
                       f"{sum(arn_units):.3g} units of the GPU solves' Krylov steps; {spent:.1f} s of CPU work"),
            "parallel": par,
            "gpu_speedup_modelled": {"vs_1_core": gpu_value / one,
                                     f"vs_{len(rates)}_cores": gpu_value / par["value"] if rates else None},
            "measured_full_solve": full}


def cpu_worker(args):
    """One worker of the parallel CPU baseline: the oracle sample on one
    pinned core, its modelled time printed as a JSON line."""
    import workloads as W
    os.sched_setaffinity(0, {args.cpu_core})
    wl = WORKLOAD_FACTORIES[args.workload](W)()
    products = [int(v) for v in args.cpu_iters.split(",")]
    arn = [float(v) for v in args.cpu_arn.split(",")]
    t_total, spent, _, _, _ = oracle_sample(wl, products, arn, start_at=args.cpu_start_at)
    print(json.dumps({"t_total": t_total, "spent": spent, "core": args.cpu_core}), flush=True)


def peaks_mode(args, torch):
    """HBM bandwidth on this GPU by plain device kernels of known traffic
    (the datasheet's 8 TB/s is the ceiling the rooflines quote): a read of 4
    GiB (a sum), a write of 4 GiB (a fill) and a copy of 2 GiB (2 GiB read +
    2 GiB written), and the streaming read of libbem_diag.so over 1 GiB (the
    kite4096 matrix size) and 4 GiB at its best of 12 launch shapes; each the
    median of --steps timed runs after --warmup."""
    n = 1 << 29  # 4 GiB of float64
    a = torch.empty(n, dtype=torch.float64, device="cuda")
    a.fill_(1.0)
    b = torch.empty(n // 2, dtype=torch.float64, device="cuda")
    st = torch.cuda.current_stream()

    def timed(fn):
        for _ in range(max(1, args.warmup)):
            fn()
        ts = []
        for _ in range(max(3, args.steps)):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(st)
            fn()
            e1.record(st)
            e1.synchronize()
            ts.append(e0.elapsed_time(e1) * 1e-3)
        return float(np.median(ts))

    t_read = timed(lambda: a.sum())
    t_write = timed(lambda: a.fill_(2.0))
    t_copy = timed(lambda: b.copy_(a[: n // 2]))
    gb = 8.0 * n / 1e9
    # the library's streaming read (one contiguous panel per workgroup,
    # non-temporal 16-byte loads) over a buffer of ones, best launch shape
    import ctypes as C
    diag = C.CDLL(os.path.join(ROOT, "paper_2312_12787_amd", "libbem_diag.so"))
    diag.bem_diag_stream_read.restype = C.c_int
    diag.bem_diag_stream_read.argtypes = [C.c_void_p, C.c_size_t, C.c_int, C.c_int, C.c_void_p, C.c_void_p]
    a.fill_(1.0)
    sink = torch.empty(1 << 16, dtype=torch.float64, device="cuda")
    stream_read = {}
    for size in (1 << 30, 1 << 32):
        best = (0.0, None)
        for grid in (1024, 2048, 4096, 8192, 16384, 32768):
            for unroll in (4, 8):
                def rd():
                    rc = diag.bem_diag_stream_read(a.data_ptr(), size, grid, unroll, sink.data_ptr(), st.cuda_stream)
                    if rc != 0:
                        raise RuntimeError(f"bem_diag_stream_read: hip error {rc}")
                rate = size / 1e9 / timed(rd)
                if rate > best[0]:
                    best = (rate, {"grid": grid, "unroll": unroll})
        stream_read[f"{size >> 30}GiB"] = {"GB_per_s": best[0], **best[1]}
    out = {"mode": "peaks", "hbm_read_GB_per_s": gb / t_read, "hbm_write_GB_per_s": gb / t_write,
           "hbm_copy_GB_per_s": gb / t_copy, "hbm_stream_read": stream_read, "datasheet_GB_per_s": 8000.0,
           "kernels": "torch sum (read 4 GiB), fill (write 4 GiB), copy (2 GiB each way); hbm_stream_read: "
                      "bem_diag_stream_read (libbem_diag.so), best of 12 launch shapes; median of timed runs"}
    print(json.dumps(out), flush=True)


def padded_ld(n, prec, P):
    """Leading dimension of the benchmark's matrices: n rounded up so that
    every column starts on a 128-byte line (8 complex128 or 16 complex64
    entries).  With an unaligned column start, each column segment that a
    product workgroup reads touches one line more (+2.7 % of the matrix
    traffic at n = 14970)."""
    per = 16 if prec == P.F32 else 8
    return (n + per - 1) // per * per


def matrix_buffer(g, prec, P, torch):
    """Column-major matrix storage (n columns of padded_ld entries)."""
    ld = padded_ld(g.n, prec, P)
    return torch.empty((g.n, ld), dtype=torch.complex64 if prec == P.F32 else torch.complex128, device="cuda")


def matvec_mode(args, wl, P, torch, prec):
    """Assemble the first case, then time --steps block products with all the
    workload's right-hand sides, then one plain device copy of 1 GiB (a
    kernel of known traffic for scaling hardware counters)."""
    g = P.Problem(wl.problems[0])
    A = matrix_buffer(g, prec, P, torch)
    g.assemble(prec, out=A, lda=A.shape[1])
    tuning = tune_or_import(args, P, g, len(wl.angles))
    g.assemble(prec, out=A, lda=A.shape[1])  # a problem takes the table's shapes when it is assembled
    X = g.rhs(wl.angles)
    if prec == P.F32:
        X = X.to(torch.complex64)
    for _ in range(max(1, args.warmup)):
        g.matvec(X)
    torch.cuda.synchronize()
    g.profile(True)
    g.profile_read(reset=True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        Y = g.matvec(X)
    torch.cuda.synchronize()
    T = time.perf_counter() - t0
    pr = g.profile_read(reset=True)
    src = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    n, nr = g.n, len(wl.angles)
    esz = 8.0 if prec == P.F32 else 16.0
    mv_bytes = esz * n * n + 2 * esz * n * nr
    avg = pr["matvec_ms"] / max(1, pr["matvec_launches"])
    print(json.dumps({"mode": "matvec", "workload": wl.name, "launches": pr["matvec_launches"], "avg_ms": avg,
                      "algorithmic_bytes_per_launch": mv_bytes, "GB_per_s": mv_bytes / (avg * 1e-3) / 1e9,
                      "TFLOP_per_s": 8.0 * n * n * nr / (avg * 1e-3) / 1e12,
                      "wall_ms_per_product": T / args.steps * 1e3, "copy_bytes": 1 << 30, "tuning": tuning}),
          flush=True)
    del Y


def assembly_evals(spec):
    """(H0, H1) evaluations of one assembly: for every domain, each row element
    on its boundary against each other element on its boundary, at every Gauss
    point (single material: 2 N (N - 1) q)."""
    sizes = {}
    for f in spec.interfaces:
        n_el = len(f.xy) if f.closed else len(f.xy) - 1
        for d in (f.dom_left, f.dom_right):
            sizes[d] = sizes.get(d, 0) + n_el
    return float(spec.quad) * sum(e * (e - 1) for e in sizes.values())


def assembly_record(wl, launches, avg_ms, evals):
    """Assembly rate; FLOP/s from the committed VALU-counter summary when it
    matches the current kernel sources (FLOPs per assembly averaged over the
    cases, which the step assembles once each)."""
    out = {"launches": launches, "avg_ms": avg_ms, "evals": evals,
           "evals_per_s": evals / (avg_ms * 1e-3) if launches else None}
    rec = counter_record("assembly_flops", wl.name)
    if rec and launches and len(rec["cases"]) == len(wl.problems):
        fl = sum(c["flops_fp64"] + c["flops_fp32"] for c in rec["cases"]) / len(rec["cases"])
        out.update({"flops_per_assembly": fl, "TFLOP_per_s": fl / (avg_ms * 1e-3) / 1e12,
                    "frac_of_valu_peak": fl / (avg_ms * 1e-3) / VALU_PEAK_FLOPS,
                    "valu_peak_TFLOP_per_s": VALU_PEAK_FLOPS / 1e12,
                    "flops_source": "rocprofv3 SQ_INSTS_VALU_FLOPS_FP64/FP32 x 64 lanes, profiles/assembly_flops_*.json"})
    return out


def max_rel_err(F, Fr):
    """max over right-hand sides of ||F_r - Fr_r|| / ||Fr_r|| (rows = right-hand sides)."""
    import torch
    return float(torch.max(torch.linalg.vector_norm(F - Fr, dim=1) / torch.linalg.vector_norm(Fr, dim=1)))


def tune_or_import(args, P, g, nr):
    """Autotune the product launch shape of g's matrix for nr right-hand sides,
    or import the table of --tune-file when that file exists."""
    if args.no_tune:
        return None
    if args.tune_file and os.path.exists(args.tune_file):
        text = open(args.tune_file).read()
        P.tune_import(text)
        return {"imported": os.path.basename(args.tune_file), "table": text.strip().splitlines()[1:]}
    t = g.tune(nr, reps=3)
    if args.tune_file:
        with open(args.tune_file, "w") as f:
            f.write(P.tune_export())
    return t


def fp64_comparison(wl, probs, P, torch, F_mixed, tune=True):
    """Mixed path only, outside the timed region: the FP64 path on the same
    workload (assembly, right-hand sides, GMRES to the same tolerance, far
    field), timed once per case, and the far-field error of both against an
    FP64 solution to 1e-12."""
    nr = len(wl.angles)
    out = {"solves": 0, "seconds": 0.0, "mixed_rel_err": 0.0, "fp64_rel_err": 0.0}
    for g, Fm in zip(probs, F_mixed):
        A64 = torch.empty((g.n, g.n), dtype=torch.complex128, device="cuda")
        g.assemble(P.F64, out=A64)
        if tune:
            g.tune(nr, reps=3)  # the FP64 path gets its own tuned shape too
        Xr, ir = g.solve(g.rhs(wl.angles), restart=wl.restart, tol=1e-12, max_iter=20000)
        Fr = g.farfield(Xr, wl.far_dirs)
        del Xr
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g.geometry_update()
        g.assemble(P.F64, out=A64)
        X, info = g.solve(g.rhs(wl.angles), restart=wl.restart, tol=wl.tol, max_iter=20000)
        F = g.farfield(X, wl.far_dirs)
        torch.cuda.synchronize()
        out["seconds"] += time.perf_counter() - t0
        out["solves"] += nr
        out["mixed_rel_err"] = max(out["mixed_rel_err"], max_rel_err(Fm, Fr))
        out["fp64_rel_err"] = max(out["fp64_rel_err"], max_rel_err(F, Fr))
        out["fp64_iterations_per_rhs"] = float(info.iters.mean())
        out["reference_converged"] = bool(ir.converged.all())
        del A64, X, F, Fr
        torch.cuda.empty_cache()
    return {"fp64_path_solves_per_s": out["solves"] / out["seconds"],
            "fp64_path_iterations_per_rhs": out["fp64_iterations_per_rhs"],
            "far_field_rel_err_mixed": out["mixed_rel_err"], "far_field_rel_err_fp64_path": out["fp64_rel_err"],
            "reference": f"FP64 assembly and GMRES to 1e-12 (converged: {out['reference_converged']}), "
                         f"{len(wl.far_dirs)} directions, max over right-hand sides of the relative 2-norm error"}


def graphs_mode(args, wl, P, torch, prec):
    """Solve time of the workload's cases with the Krylov steps launched kernel
    by kernel (graph_steps 0) and as captured HIP graphs of 4, 8 and 16 steps:
    each case assembled once, one untimed solve per setting (it captures the
    graphs), then --steps timed solves (library timing off); the solutions of
    every setting are compared with the kernel-by-kernel one bit for bit."""
    settings = [0, 4, 8, 16]
    mixed = prec != P.F64
    cases = []
    for spec in wl.problems:
        g = P.Problem(spec)
        g.assemble(prec)
        B = g.rhs(wl.angles)
        kw = dict(restart=wl.restart, tol=wl.tol, max_iter=20000, inner_tol=wl.inner_tol if mixed else 0.0)
        X0, info0 = g.solve(B, **kw)
        X0 = X0.clone()
        row = {"case": str(spec.k), "iters_per_rhs": float(info0.iters.mean())}
        for S in settings:
            X, info = g.solve(B, graph_steps=S, **kw)
            same = bool(torch.equal(X, X0)) and np.array_equal(info.iters, info0.iters)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.steps):
                X, info = g.solve(B, graph_steps=S, **kw)
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) / args.steps * 1e3
            row[f"graph_steps_{S}"] = {"ms_per_solve_call": ms, "identical_to_kernel_by_kernel": same}
            log(f"  case {row['case']} graph_steps {S}: {ms:.3f} ms per solve call, identical {same}")
        cases.append(row)
    out = {"mode": "graphs", "workload": wl.name, "rhs_per_case": len(wl.angles), "restart": wl.restart,
           "tol": wl.tol, "timed_solves_per_setting": args.steps, "cases": cases}
    print(json.dumps(out), flush=True)


def served_record(args, P, torch, n_requests, open_loop=True):
    """Served stream: requests with Poisson arrivals at 20/s, perturbed circles
    with N log-uniform in [512, 8192], k0 ~ U[1, 50], k1/k0 ~ U[1.2, 3], 1-32
    angles (the first n_requests of the seeded stream).  Capacity: every
    request submitted at once (closed loop), solves/s = right-hand sides /
    wall time, for the mixed server (BEM_MIXED) and the FP64 server; accuracy:
    far field of every request, mixed against FP64, and both against FP64
    solved to 1e-12 on every 10th request.  Latency: the arrivals replayed in
    real time (open loop) on the mixed server, p50/p99 of completion minus
    arrival."""
    import workloads as W
    from paper_2312_12787_amd import serve as S
    reqs = W.request_stream(n_requests)
    dirs = W.equispaced_angles(360)
    arena = int(args.arena_gb * (1 << 30))
    solves = sum(len(r["angles"]) for r in reqs)

    def closed_loop(prec, tol):
        with S.Server(arena, slots=args.slots, prec=prec, tol=tol, restart=args.serve_restart, dirs=dirs,
                      graph_steps=args.graph_steps, fuse=args.fuse) as srv:
            for r in reqs[:8]:  # warm-up: code objects, host paths
                srv.submit(r["spec"], r["angles"])
            srv.drain()
            t0 = time.perf_counter()
            ids = {srv.submit(r["spec"], r["angles"]): i for i, r in enumerate(reqs)}
            out = []
            while len(out) < len(reqs):
                out.extend(srv.poll(wait_ms=1000))
                if len(out) // 250 != (len(out) - 1) // 250 or len(out) == len(reqs):
                    log(f"    {len(out)} / {len(reqs)} done, {time.perf_counter() - t0:.1f} s")
            T = time.perf_counter() - t0
            st = srv.stats()
        res = {ids[o.id]: o for o in out}
        return T, res, st

    def ff_err(a, b):
        return float(np.max(np.linalg.norm(a.far_field - b.far_field, axis=1) / np.linalg.norm(b.far_field, axis=1)))

    log(f"serve: {len(reqs)} requests, {solves} solves, closed loop, mixed ...")
    T32, r32, st32 = closed_loop(P.MIXED, args.serve_tol)
    log(f"  {T32:.1f} s; FP64 ...")
    T64, r64, _ = closed_loop(P.F64, args.serve_tol)
    log(f"  {T64:.1f} s; FP64 reference to 1e-12 on every 10th request ...")
    sample = list(range(0, len(reqs), 10))
    with S.Server(arena, slots=args.slots, prec=P.F64, tol=1e-12, restart=args.serve_restart, dirs=dirs,
                  graph_steps=args.graph_steps, fuse=args.fuse) as srv:
        ids = {srv.submit(reqs[i]["spec"], reqs[i]["angles"]): i for i in sample}
        ref = {ids[o.id]: o for o in srv.drain()}
    bad = [i for i in range(len(reqs)) if r32[i].status != 0 or r64[i].status != 0]
    err = max(ff_err(r32[i], r64[i]) for i in range(len(reqs)))
    err32 = [ff_err(r32[i], ref[i]) for i in sample]
    err64 = [ff_err(r64[i], ref[i]) for i in sample]
    f32 = None
    if getattr(args, "serve_f32", False):
        # the FP32-assembly server (BEM_F32: FP32 matrix, refinement residuals
        # with it) on the same stream: capacity, footprint and its far-field
        # error against the FP64 server and against FP64 to 1e-12
        log("  FP32-assembly server ...")
        Tf, rf, stf = closed_loop(P.F32, args.serve_tol)
        ef = [ff_err(rf[i], r64[i]) for i in range(len(reqs))]
        efr = [ff_err(rf[i], ref[i]) for i in sample]
        f32 = {"solves_per_s": solves / Tf, "requests_per_s": len(reqs) / Tf,
               "over_mixed": T32 / Tf, "arena_high_water_GiB": stf["arena_high_water"] / 2**30,
               "far_field_rel_err_vs_fp64_server": {"max": max(ef), "p50": float(np.median(ef)),
                                                    "p99": float(np.percentile(ef, 99)),
                                                    "requests_above_1e-6": int(sum(e > 1e-6 for e in ef))},
               "vs_fp64_1e-12_sample": {"max": max(efr), "p50": float(np.median(efr)),
                                        "above_1e-6": int(sum(e > 1e-6 for e in efr))},
               "failed_requests": [i for i in range(len(reqs)) if rf[i].status != 0],
               "worst_requests": [{"request": i, "err": ef[i], "N": reqs[i]["spec"].n_elements,
                                   "k0": float(np.real(reqs[i]["spec"].k[0])),
                                   "k1": float(np.real(reqs[i]["spec"].k[1])),
                                   "iters_max_mixed": int(r32[i].iters_max)}
                                  for i in sorted(range(len(reqs)), key=lambda i: -ef[i])[:8]]}
    lat = []
    if open_loop:
        log("  open loop at the arrival times ...")
        with S.Server(arena, slots=args.slots, prec=P.MIXED, tol=args.serve_tol, restart=args.serve_restart,
                      dirs=dirs, graph_steps=args.graph_steps, fuse=args.fuse) as srv:
            for r in reqs[:8]:
                srv.submit(r["spec"], r["angles"])
            srv.drain()
            t0 = time.perf_counter()
            lag = {}
            for r in reqs:
                dt = r["arrival"] - (time.perf_counter() - t0)
                if dt > 0:
                    time.sleep(dt)
                late = (time.perf_counter() - t0) - r["arrival"]
                lag[srv.submit(r["spec"], r["angles"])] = late
                got = srv.poll(0)
                lat.extend(got)
                if got and len(lat) // 250 != (len(lat) - len(got)) // 250:
                    log(f"    {len(lat)} / {len(reqs)} done, {time.perf_counter() - t0:.1f} s")
            lat.extend(srv.drain())
        # latency = completion - arrival: the server's own submit-to-done time
        # plus how late the replay submitted the request
        lat_ms = np.array([(o.t_done - o.t_submit + lag[o.id]) * 1e3 for o in lat])
    rec = {
        "workload": f"served stream: first {len(reqs)} requests of the seeded stream, Poisson 20/s, perturbed "
                    f"circles N 512-8192 log-uniform, k0 U[1,50], k1/k0 U[1.2,3], 1-32 angles",
        "requests": len(reqs), "solves": solves, "slots": args.slots, "arena_GiB": args.arena_gb,
        "tol": args.serve_tol, "restart": args.serve_restart, "far_field_dirs": len(dirs),
        "graph_steps": args.graph_steps, "fuse": args.fuse,
        "capacity": {"mixed_solves_per_s": solves / T32, "fp64_solves_per_s": solves / T64,
                     "mixed_over_fp64": T64 / T32,
                     "mixed_requests_per_s": len(reqs) / T32, "fp64_requests_per_s": len(reqs) / T64,
                     "arena_high_water_GiB": st32["arena_high_water"] / 2**30,
                     "unit": "closed loop: every request submitted at once; right-hand sides solved / wall time"},
        "accuracy": {"far_field_rel_err_mixed_vs_fp64_max": err,
                     "vs_fp64_1e-12_sample": {"requests": len(sample), "mixed_max": max(err32),
                                              "mixed_p50": float(np.median(err32)), "fp64_path_max": max(err64),
                                              "fp64_path_p50": float(np.median(err64))},
                     "measure": "max over right-hand sides of the relative 2-norm far-field error at 360 directions",
                     "failed_requests": bad},
        "precision": {"mixed": "BEM_MIXED: FP64 matrix and its FP32 copy from one assembly; FP32 products, "
                               "FP64 Arnoldi, refinement residuals with the FP64 matrix", "fp64": "BEM_F64"},
        "gmres_iterations_max_per_request": {"p50": float(np.median([r32[i].iters_max for i in r32])),
                                             "max": int(max(r32[i].iters_max for i in r32))},
    }
    if f32:
        rec["f32_server"] = f32
    if lat:
        rec["latency_ms"] = {"p50": float(np.percentile(lat_ms, 50)), "p99": float(np.percentile(lat_ms, 99)),
                             "unit": "open loop at the stream's arrival times: completion - arrival, mixed server"}
    return rec


def serve_mode(args, P, torch):
    """The served stream alone (--workload serve): its record as the bench line,
    value = the mixed server's capacity."""
    rec = served_record(args, P, torch, args.requests, open_loop=not args.no_open_loop)
    out = {
        "metric": METRIC,
        "value": rec["capacity"]["mixed_solves_per_s"],
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": 1,
        "warmup": 1,
        "ms_per_step": rec["solves"] / rec["capacity"]["mixed_solves_per_s"] * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": rec["workload"], "requests": rec["requests"], "solves": rec["solves"],
                   "slots": rec["slots"], "arena_GiB": rec["arena_GiB"], "tol": rec["tol"],
                   "restart": rec["restart"], "far_field_dirs": rec["far_field_dirs"],
                   "graph_steps": rec["graph_steps"], "fuse": rec["fuse"]},
        "roofline": None,
    }
    out.update({k: rec[k] for k in ("capacity", "accuracy", "precision", "gmres_iterations_max_per_request")})
    if "f32_server" in rec:
        out["f32_server"] = rec["f32_server"]
    if "latency_ms" in rec:
        out["latency_ms"] = rec["latency_ms"]
    print(json.dumps(out), flush=True)


def nearfield_mode(args, P, torch):
    """The near field of Sec. 7.1's accuracy measure: unit disk (inscribed
    N-gon), omega = 5, eps2 = 2, solved on the GPU (FP64, GMRES to 1e-10),
    then --steps evaluations of the total field on the 101 x 101 grid of
    [-2.99, 2.99]^2 (bem_nearfield; points and domains resident on the
    device), timed with events on the launch stream."""
    import workloads as W
    n_el = args.nf_elements
    spec = W.disk(n_el, 5.0, 5.0 * np.sqrt(2.0))
    g = P.Problem(spec)
    g.assemble(P.F64)
    X, info = g.solve(g.rhs([0.0]), restart=100, tol=1e-10)
    t = np.linspace(-2.99, 2.99, 101)
    xx, yy = np.meshgrid(t, t, indexing="ij")
    pts = np.stack([xx.ravel(), yy.ravel()], axis=1)
    dom = (np.hypot(pts[:, 0], pts[:, 1]) < 1.0).astype(np.int32)
    pts_t = torch.as_tensor(pts, dtype=torch.float64, device="cuda")
    dom_t = torch.as_tensor(dom, dtype=torch.int32, device="cuda")
    for _ in range(max(1, args.warmup)):
        g.nearfield(X, pts_t, dom_t, [0.0])
    torch.cuda.synchronize()
    st = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(args.steps):
        U = g.nearfield(X, pts_t, dom_t, [0.0])
    e1.record(st)
    e1.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    npts, q = len(pts), spec.quad
    pairs = npts * n_el
    out = {"mode": "nearfield", "workload": f"disk{n_el}_k5-7.07_grid101", "points": npts, "elements": n_el,
           "gmres_iterations": int(info.iters[0]), "calls": args.steps, "avg_ms": ms,
           "point_element_pairs_per_s": pairs / (ms * 1e-3),
           "evals_per_s": pairs * q / (ms * 1e-3),
           "timing": "events on the launch stream around --steps bem_nearfield calls (one launch per domain each)"}
    rec = counter_record("nearfield_flops", out["workload"])
    if rec:
        fl = rec["flops_per_call"]
        out.update({"flops_per_call": fl, "TFLOP_per_s": fl / (ms * 1e-3) / 1e12,
                    "frac_of_valu_peak": fl / (ms * 1e-3) / VALU_PEAK_FLOPS})
    print(json.dumps(out), flush=True)
    del U


def assemble_mode(args, wl, P, torch, prec):
    """Only assemblies: every case of the workload --steps times (after
    --warmup), timed with the library's HIP events (for hardware-counter runs
    of the assembly kernels)."""
    out = []
    for spec in wl.problems:
        g = P.Problem(spec)
        g.geometry()
        A = matrix_buffer(g, prec, P, torch)
        for _ in range(max(1, args.warmup)):
            g.assemble(prec, out=A, lda=A.shape[1])
        torch.cuda.synchronize()
        g.profile(True)
        g.profile_read(reset=True)
        for _ in range(args.steps):
            g.assemble(prec, out=A, lda=A.shape[1])
        pr = g.profile_read(reset=True)
        g.profile(False)
        ev = assembly_evals(spec)
        avg = pr["assemble_ms"] / max(1, pr["assemble_launches"])
        out.append({"case": str(spec.k), "launches": pr["assemble_launches"], "avg_ms": avg, "evals": ev,
                    "evals_per_s": ev / (avg * 1e-3)})
        del A
    print(json.dumps({"mode": "assemble", "workload": wl.name, "precision": wl.precision, "cases": out}), flush=True)


def sectors_far_field_error(wl, F_full, P, torch):
    """Far-field error of the multi-material workload: its solution (h = 1/800)
    against the mesh refined to h = 1/1600, and the observed order from
    h = 1/400 (outside the timed region, FP64, GMRES(100) to 1e-10)."""
    import workloads as W
    spec0 = wl.problems[0]
    F = {800: F_full}
    its = {}
    for inv_h in (400, 1600):
        spec = W.sectors(spec0.k, h=1.0 / inv_h)
        g = P.Problem(spec)
        g.assemble(P.F64)
        X, info = g.solve(g.rhs(wl.angles), restart=wl.restart, tol=wl.tol, max_iter=20000)
        F[inv_h] = g.farfield(X, wl.far_dirs)
        its[inv_h] = (spec.n_elements, int(info.iters.max()))
        del g, X
        torch.cuda.empty_cache()
    d = {h: float(max_rel_err(F[h], F[1600])) for h in (400, 800)}
    ratio = d[400] / d[800]
    order = float(np.log2(max(ratio - 1.0, 1e-3)))
    x = 2.0 ** order
    return {"vs_h_1_1600": d[800], "h_1_400_vs_h_1_1600": d[400], "observed_order": order,
            "estimated_error": d[800] * x / (x - 1.0) if x > 1.0 else None,
            "refined_meshes": {f"h=1/{h}": {"elements": e, "gmres_iterations": i} for h, (e, i) in its.items()},
            "measure": "relative 2-norm of the far-field difference at 360 directions; error estimate "
                       "|F_h - F_h/2| 2^p / (2^p - 1) with p the observed order"}


def run_workload(args, wl, P, torch, steps, warmup, tune=True, graph_steps=0):
    """The full hot path of the workload, K timed steps after W untimed ones:
    each case's device tables, assembly, right-hand sides, GMRES solve and far
    field.  Returns the bench record (without the CPU baseline) and what the
    CPU model needs (GMRES products and per-right-hand-side steps)."""
    mixed = wl.precision == "f32"
    prec = P.F32 if mixed else P.F64
    dirs = wl.far_dirs
    probs, mats = [], []
    nr = len(wl.angles)
    for spec in wl.problems:
        g = P.Problem(spec)
        g.geometry()  # uploads the inputs (nodes, plan) once
        mats.append(matrix_buffer(g, prec, P, torch))
        _, _, wb = g.sizes(P.F64, nr, wl.restart)
        g._workspace(wb)
        probs.append(g)
    torch.cuda.synchronize()

    lat = []
    iters = [0] * len(probs)
    products = [0] * len(probs)
    refine = [0] * len(probs)
    rhs_steps = [None] * len(probs)
    last_F = [None] * len(probs)
    # independent cases run concurrently, each on its own stream driven by
    # its own host thread (the library calls release the interpreter lock):
    # one case's latency-bound Krylov kernels overlap the other's HBM-bound
    # products
    concurrent = len(probs) > 1 and not args.sequential_cases
    mode = {"concurrent": concurrent}
    streams = [torch.cuda.Stream() for _ in probs] if concurrent else [torch.cuda.current_stream()] * len(probs)

    def run_case(ci, record, t0):
        g, A, st = probs[ci], mats[ci], streams[ci]
        with torch.cuda.stream(st):
            g.geometry_update(stream=st)
            g.assemble(prec, out=A, lda=A.shape[1], stream=st)
            B = g.rhs(wl.angles, stream=st)
            X, info = g.solve(B, restart=wl.restart, tol=wl.tol, max_iter=20000,
                              inner_tol=wl.inner_tol if mixed else 0.0, graph_steps=graph_steps, stream=st)
            F = g.farfield(X, dirs, stream=st)
            st.synchronize()
        if record:
            lat.append(time.perf_counter() - t0)
            iters[ci] += int(info.iters.sum())
            refine[ci] += int(info.restarts.sum())
            # products a one-right-hand-side-at-a-time solver needs: one per
            # Arnoldi step plus one residual per cycle
            products[ci] += int(info.iters.sum() + info.restarts.sum()) + nr
            rhs_steps[ci] = info.iters.tolist()
            last_F[ci] = F
        if not info.converged.all():
            raise RuntimeError(f"case {ci} did not converge: {info}")

    def step(record):
        if not mode["concurrent"]:
            for ci in range(len(probs)):
                run_case(ci, record, time.perf_counter())
            return
        import threading
        errs = []

        def body(ci, t0):
            try:
                run_case(ci, record, t0)
            except BaseException as e:  # re-raised on the main thread
                errs.append(e)
        t0 = time.perf_counter()
        th = [threading.Thread(target=body, args=(ci, t0)) for ci in range(len(probs))]
        for t in th:
            t.start()
        for t in th:
            t.join()
        if errs:
            raise errs[0]

    def run_steps(k, record):
        """k steps.  With --case-pipeline the concurrent cases each run their
        k steps back to back on their own stream and host thread, without a
        barrier between steps, so that one case's assembly can run beside the
        other case's solve; otherwise both cases start every step together."""
        if not (mode["concurrent"] and args.case_pipeline):
            for _ in range(k):
                step(record)
            return
        import threading
        errs = []

        def body(ci):
            try:
                for _ in range(k):
                    run_case(ci, record, time.perf_counter())
            except BaseException as e:  # re-raised on the main thread
                errs.append(e)
        th = [threading.Thread(target=body, args=(ci,)) for ci in range(len(probs))]
        for t in th:
            t.start()
        for t in th:
            t.join()
        if errs:
            raise errs[0]

    for _ in range(warmup):
        step(False)
    tuning = None
    if tune and not args.no_tune:
        # launch-shape autotuning of the solve's products (bem_tune), outside the timed region
        if warmup == 0:
            probs[0].geometry_update()
            probs[0].assemble(prec, out=mats[0], lda=mats[0].shape[1])
        log("autotuning the product launch shape ...")
        tuning = tune_or_import(args, P, probs[0], nr)
        log("tuned:", tuning)
    for g in probs:
        g.profile(True)
        g.profile_read(reset=True)
    torch.cuda.synchronize()
    w0 = time.monotonic_ns()  # the clock of rocprofv3's timestamps: lets a trace pick out the timed launches
    t0 = time.perf_counter()
    run_steps(steps, True)
    torch.cuda.synchronize()
    T = time.perf_counter() - t0
    windows = {"timed": [w0, time.monotonic_ns()]}
    prof = [g.profile_read(reset=True) for g in probs]
    iso = None
    if concurrent:
        # the product kernel on its own: two more steps with the cases one
        # after the other (outside the timed region), timed by the same events
        mode["concurrent"] = False
        w1 = time.monotonic_ns()
        for _ in range(2):
            step(False)
        torch.cuda.synchronize()
        windows["isolated"] = [w1, time.monotonic_ns()]
        iso = [g.profile_read(reset=True) for g in probs]
        mode["concurrent"] = True
    for g in probs:
        g.profile(False)

    n = probs[0].n
    N = probs[0].N
    q = wl.problems[0].quad
    esz = 8.0 if mixed else 16.0
    solves = steps * len(probs) * nr
    mv_launch = sum(p["matvec_launches"] for p in prof)
    mv_ms = sum(p["matvec_ms"] for p in prof)
    rs_launch = sum(p["residual_launches"] for p in prof)
    rs_ms = sum(p["residual_ms"] for p in prof)
    as_launch = sum(p["assemble_launches"] for p in prof)
    as_ms = sum(p["assemble_ms"] for p in prof)
    mv_bytes = esz * n * n + 2 * esz * n * nr  # matrix + X + Y per launch (algorithmic)
    mv_flops = 8.0 * n * n * nr
    mv_avg_ms = mv_ms / max(1, mv_launch)
    mv_gbs = mv_bytes / (mv_avg_ms * 1e-3) / 1e9
    mv_tfs = mv_flops / (mv_avg_ms * 1e-3) / 1e12
    as_avg_ms = as_ms / max(1, as_launch)
    evals = sum(assembly_evals(s) for s in wl.problems) / len(wl.problems)
    lat_ms = np.array(lat) * 1e3
    if mixed:
        # more than 16 right-hand sides always run the 3-product form, which
        # issues 6 of the 8 algorithmic flops of a complex multiply-add on the
        # matrix cores: the cores are busy 6/8 of the algorithmic fraction
        g3 = True if nr > 16 else bool(tuning.get("g3", 1)) if isinstance(tuning, dict) else True
        roofline = {"kernel": f"k_matvec_mfma (FP32 MFMA split-K block product, {nr} right-hand sides in one pass "
                              f"over A)", "bound": "mfma", "achieved": mv_tfs, "peak": FP32_MFMA_PEAK_TFS,
                    "unit": "TFLOP/s", "frac": mv_tfs / FP32_MFMA_PEAK_TFS,
                    "mfma_busy_frac": mv_tfs / FP32_MFMA_PEAK_TFS * (0.75 if g3 else 1.0),
                    "note": "achieved counts 8 flops per complex multiply-add (the algorithmic count, so frac "
                            "can reach 1.33); the 3-product form runs 6 of them on the matrix cores, and "
                            "mfma_busy_frac is the matrix cores' share of their peak" if g3 else "4-product form",
                    "traffic": traffic_record(wl.name)}
    else:
        roofline = {"kernel": f"k_matvec_mfma (FP64 MFMA split-K block product, {nr} right-hand sides)"
                    if nr > 4 else f"k_matvec (FP64 VALU split-K product, {nr} right-hand side(s))",
                    "bound": "hbm", "achieved": mv_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": mv_gbs / HBM_PEAK_GBS, "traffic": traffic_record(wl.name)}
    assembly_rec = assembly_record(wl, as_launch, as_avg_ms, evals)
    if iso:
        # the cases' assemblies overlap in the timed region (each then takes
        # about twice as long); the rate is that of one assembly at a time
        ia = sum(p["assemble_launches"] for p in iso)
        assembly_rec = assembly_record(wl, ia, sum(p["assemble_ms"] for p in iso) / max(1, ia), evals)
        assembly_rec["timing"] = "cases one after another, two steps after the timed region (library HIP events)"
        assembly_rec["avg_ms_in_timed_region"] = as_avg_ms
        iso_ms = sum(p["matvec_ms"] for p in iso) / max(1, sum(p["matvec_launches"] for p in iso))
        achieved = (mv_tfs if mixed else mv_gbs) * mv_avg_ms / iso_ms
        roofline["isolated"] = {
            "achieved": achieved, "frac": achieved / roofline["peak"], "avg_ms": iso_ms,
            "launches": sum(p["matvec_launches"] for p in iso),
            "note": "the same kernel with the cases run one after another (two steps after the timed region); in "
                    "the timed region the cases run concurrently, so each product shares the GPU with the other "
                    "case's Krylov kernels and its event-timed duration includes them"}
    out = {
        "metric": METRIC,
        "value": solves / T,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warmup,
        "ms_per_step": T / steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if mixed else "f64",
        "data": "synthetic",
        "config": {"workload": wl.name, "elements": N, "system_order": n,
                   "wavenumbers": [[str(k) for k in s.k] for s in wl.problems], "rhs_per_case": nr,
                   "restart": wl.restart, "tol": wl.tol, "quad": q, "far_field_dirs": len(dirs),
                   "solves_per_step": len(probs) * nr, "precision": wl.precision},
        "case_time_ms": {"p50": float(np.percentile(lat_ms, 50)), "p99": float(np.percentile(lat_ms, 99)),
                         "unit": f"closed loop, from the step's start to one case's end: geometry tables + assembly "
                                 f"+ {nr} solves + far field (served latency: the served record)"},
        "cases_concurrent": concurrent,
        "gmres_iterations_per_rhs": [it / (steps * nr) for it in iters],
        "assembly": assembly_rec,
        "matvec": {"launches": mv_launch, "avg_ms": mv_avg_ms, "GB_per_s": mv_gbs, "TFLOP_per_s": mv_tfs,
                   "share_of_step_time": mv_ms / (T * 1e3)},
        "residual": {"launches": rs_launch, "avg_ms": rs_ms / max(1, rs_launch)},
        "tuning": tuning,
        "graph_steps": graph_steps,
        "roofline": roofline,
        "monotonic_ns": windows,
    }
    if mixed:
        out["refinement_steps_per_rhs"] = [r / (steps * nr) for r in refine]
        log("FP64 path on the same workload (reference solve, then one timed run) ...")
        out["fp64_comparison"] = fp64_comparison(wl, probs, P, torch, last_F, tune=tune and not args.no_tune)
    if wl.name.startswith("sectors"):
        log("far-field error against refined meshes ...")
        out["far_field_error"] = sectors_far_field_error(wl, last_F[0], P, torch)
    model = {"products": [p // steps for p in products],
             "arn_units": [arnoldi_units(st, wl.restart, g.n) for st, g in zip(rhs_steps, probs)]}
    del probs, mats
    torch.cuda.empty_cache()
    return out, model


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="kite4096",
                    choices=["kite4096", "disk256", "sectors", "kite16384_mixed", "serve"])
    ap.add_argument("--requests", type=int, default=2000, help="serve: requests in the stream")
    ap.add_argument("--slots", type=int, default=4, help="serve: requests in flight")
    ap.add_argument("--arena-gb", type=float, default=64.0, help="serve: device arena in GiB")
    ap.add_argument("--serve-tol", type=float, default=1e-8, help="serve: GMRES / refinement tolerance")
    ap.add_argument("--serve-restart", type=int, default=300,
                    help="serve: GMRES restart length (high-frequency requests need many steps)")
    ap.add_argument("--no-open-loop", action="store_true", help="serve: skip the real-time replay")
    ap.add_argument("--serve-f32", action="store_true",
                    help="serve: also run the FP32-assembly server (BEM_F32) on the stream and report its error")
    ap.add_argument("--fuse", type=int, default=1,
                    help="serve: requests a slot admits together and solves as one batch with fused Krylov launches")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="default workload only: skip the precision-path, served-prefix and disk256 records")
    ap.add_argument("--sequential-cases", action="store_true",
                    help="run a workload's cases one after another on one stream (default: concurrently, one "
                         "stream and host thread per case)")
    ap.add_argument("--case-pipeline", action="store_true",
                    help="concurrent cases run their timed steps back to back, each on its own, instead of "
                         "starting every step together")
    ap.add_argument("--serve-prefix", type=int, default=200,
                    help="requests of the stream in the default run's served record")
    ap.add_argument("--graph-steps", type=int, default=0,
                    help="Krylov steps per captured HIP graph in the solves (0: kernel-by-kernel launches); "
                         "takes effect in the serve workload; the full mode times kernels with the library's "
                         "events, which keeps kernel-by-kernel launches (--mode graphs compares both)")
    ap.add_argument("--no-tune", action="store_true", help="skip the launch-shape autotuning (bem_tune) before timing")
    ap.add_argument("--tune-file", default=None,
                    help="launch-shape table: imported if the file exists, else written after tuning "
                         "(so that profiling runs use the same shapes)")
    ap.add_argument("--nf-elements", type=int, default=1024, help="nearfield mode: elements of the disk")
    ap.add_argument("--mode", default="full", choices=["full", "matvec", "assemble", "nearfield", "peaks", "graphs"],
                    help="matvec: assemble case 1 and run only --steps block products with all the workload's "
                         "right-hand sides, then one plain 1 GiB device copy (for hardware-counter runs); "
                         "assemble: only --steps assemblies of every case; graphs: --steps solves per case "
                         "kernel by kernel and as captured HIP graphs")
    ap.add_argument("--cpu-worker", action="store_true", help=argparse.SUPPRESS)
    ap.add_argument("--cpu-iters", default="", help=argparse.SUPPRESS)
    ap.add_argument("--cpu-arn", default="", help=argparse.SUPPRESS)
    ap.add_argument("--cpu-start-at", type=float, default=None, help=argparse.SUPPRESS)
    ap.add_argument("--cpu-core", type=int, default=0, help=argparse.SUPPRESS)
    args = ap.parse_args()
    if args.cpu_worker:
        return cpu_worker(args)
    if args.gpus != 1:
        print("bench.py measures one GPU only; run with --gpus 1 "
              "(the library has no multi-GPU path: sharding by row blocks is a design, not code)", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2312_12787_amd as P
    import workloads as W

    torch.cuda.set_device(0)
    if args.workload == "serve":
        return serve_mode(args, P, torch)
    wl = WORKLOAD_FACTORIES[args.workload](W)()
    prec = P.F32 if wl.precision == "f32" else P.F64
    if args.mode == "matvec":
        return matvec_mode(args, wl, P, torch, prec)
    if args.mode == "assemble":
        return assemble_mode(args, wl, P, torch, prec)
    if args.mode == "nearfield":
        return nearfield_mode(args, P, torch)
    if args.mode == "peaks":
        return peaks_mode(args, torch)
    if args.mode == "graphs":
        return graphs_mode(args, wl, P, torch, prec)
    out, model = run_workload(args, wl, P, torch, args.steps, args.warmup, graph_steps=args.graph_steps)
    if args.workload == "kite4096" and not args.no_extras:
        # the metric's other halves, each outside the headline's timed region
        import copy
        xargs = copy.copy(args)
        xargs.tune_file = None  # the headline's launch-shape file stays the headline's
        log("precision path: kite N = 16384, FP32 products + FP64 refinement, 64 angles ...")
        pp, _ = run_workload(xargs, W.workload_kite16384_fp32(), P, torch, 2, 1)
        fc = pp["fp64_comparison"]
        out["precision_path"] = {
            "workload": pp["config"]["workload"], "mixed_solves_per_s": pp["value"],
            "fp64_path_solves_per_s": fc["fp64_path_solves_per_s"],
            "mixed_over_fp64": pp["value"] / fc["fp64_path_solves_per_s"],
            "far_field_rel_err_mixed": fc["far_field_rel_err_mixed"],
            "far_field_rel_err_fp64_path": fc["far_field_rel_err_fp64_path"], "reference": fc["reference"],
            "gmres_iterations_per_rhs": pp["gmres_iterations_per_rhs"],
            "refinement_steps_per_rhs": pp["refinement_steps_per_rhs"], "steps_timed": 2,
            "assembly": pp["assembly"], "roofline": pp["roofline"]}
        P.tune_reset()  # the served stream runs the built-in launch shapes, as with --workload serve
        log(f"served stream: first {args.serve_prefix} requests ...")
        out["served"] = served_record(xargs, P, torch, args.serve_prefix, open_loop=True)
        log("disk256 (unit disk, N = 256), 20 steps ...")
        dk, _ = run_workload(xargs, W.workload_disk256(), P, torch, 20, 3, tune=False)
        out["disk256"] = {"workload": dk["config"]["workload"], "value": dk["value"], "unit": "solves/s",
                          "case_time_ms": dk["case_time_ms"], "gmres_iterations_per_rhs":
                              dk["gmres_iterations_per_rhs"],
                          "note": "4 MB matrix: launch- and latency-bound, not a roofline case"}
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on a bounded sample ...")
        out["cpu_baseline"] = cpu_baseline(wl, args.workload, model["products"], model["arn_units"], out["value"])
        full = out["cpu_baseline"]["measured_full_solve"]
        if "disk256" in out:
            full["gpu_solves_per_s"] = out["disk256"]["value"]
            full["gpu_speedup_measured"] = out["disk256"]["value"] / full["value"]
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
