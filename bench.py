#!/usr/bin/env python3
"""Benchmark of the F3R hot path on one MI355X.

Default workload: the 3D 7-point Poisson system on a 128^3 grid
(n = 2,097,152, nnz = 14,581,760), x* uniform on [-1, 1] from a seeded
SplitMix64 stream, b = A x*, tolerance 1e-10 on the fp64 relative residual.
One step is one fp16-F3R solve (F100, F8, F4, R2, M; c = 64) from x0 = 0 to
the tolerance with b already in HBM; set-up (scaling, level copies, M,
device format) is timed once and reported beside it.  The same GPU also runs
fp64 FGMRES(64)+M, fp32-F3R and fp64-F3R for the comparison the metric
names.

--workload selects another synthetic system shaped like the paper's
workloads: convdiff_q1_100 (nonsymmetric 27-point, fp16 and bf16 inner
storage compared), elasticity_bonds_64 (3x3 blocks, 61.7M entries),
poisson2d_64 (small), or varcoef2d_batch256 (256 independent systems solved
by one persistent launch, against the same systems solved one at a time).

Prints one JSON line.  --gpus above 1 is refused: the solver runs on one GPU.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import statistics
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "F3R time-to-1e-10 residual vs fp64 FGMRES (s, same GPU); SpMV HBM GB/s"
HBM_PEAK_GBS = 8000.0  # MI355X HBM3E


def log(msg):
    print(msg, file=sys.stderr, flush=True)


KERNEL_SOURCES = ("kernels.hip", "sell.h", "common.h", "kernels.h")


def kernel_source_hash() -> str:
    """sha256 over the sources that define the level kernels."""
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2505_20719_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(kernel: str, workload: str):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary (FETCH_SIZE and WRITE_SIZE, scaled by a plain copy of known size),
    or None when there is none or the kernels changed since it was taken."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_traffic.md")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m = re.search(r"^traffic_bytes_per_launch: (\d+)\s*$", text, re.M)
    h = re.search(r"^kernel_source_sha256: ([0-9a-f]{64})\s*$", text, re.M)
    if not m or not h or h.group(1) != kernel_source_hash():
        return None
    return int(m.group(1))


def csr_model_bytes(A):
    """Algorithmic bytes per launch by the per-unit figures of the hot-path
    scope table (CSR with 4-byte column indices and row pointers; fp16
    values and Richardson vectors, fp32 level-2 vectors; each vector read
    once): SpMV nnz (s_A + 4) + 4 (n + 1) + n s_x + n s_y; one M sweep
    (nnz + n) / 2 (s_M + 4) + 4 n + its vectors (W sweep: input, 3 bytes on
    average over the fp32 basis and the fp16 residual, and t; G sweep: t and
    z); the Richardson residual adds the read of v (fp32 basis); the level-2
    SpMV adds its Gram-Schmidt dots, (j + 1) n s with j + 1 = 2.5 on
    average."""
    n, nnz = A.n, A.nnz
    sweep = (nnz + n) / 2.0 * (2 + 4) + 4.0 * n
    spmv16 = nnz * (2 + 4) + 4.0 * (n + 1)
    return {
        "m_lower": sweep + n * (3 + 2),
        "m_upper": sweep + n * (2 + 2),
        "r_residual": spmv16 + n * 2 + n * 2 + n * 4,
        "spmv_l2": spmv16 + n * 2 + n * 4 + 2.5 * n * 4,
    }


def algorithmic_bytes(A, idx_bits: int, layout: int, width: int):
    """Bytes each probed kernel must move per launch in the device format (the
    data structure it reads once and the vectors it reads/writes once), fp16
    level storage.  SELL (1) also reads one 4-byte offset per slice and a
    2-byte diagonal position per row; the diagonal-aligned format (2) reads
    neither; the slice-offset format (3) reads no per-entry index but one
    4-byte offset per slice and position (width per slice; about half of them
    for a one-sided sweep)."""
    n = A.n
    nnz = A.nnz
    rows = np.repeat(np.arange(n), np.diff(A.row_ptr))
    nl = int(np.count_nonzero(A.col_idx < rows))
    nu = int(np.count_nonzero(A.col_idx > rows))
    sv, si = 2, idx_bits // 8
    ns = (n + 63) // 64
    off = {1: n / 16.0, 2: 0.0}.get(layout, 4.0 * ns * width)
    half = {1: n / 16.0, 2: 0.0}.get(layout, 4.0 * ns * (width - 1) / 2)
    kdb = 2 if layout == 1 else 0  # diagonal positions, 2 bytes per row
    return {
        # W sweep: kd (2n), lower entries, input (fp32 basis at k=1, fp16 r
        # at k=2: 3n on average), t written (2n)
        "m_lower": (5 + kdb) * n + (sv + si) * nl + half,
        # G sweep + update: kd, upper entries, t (2n), z written (2n), z_prev
        # read at k=2 only (n on average)
        "m_upper": (5 + kdb) * n + (sv + si) * nu + half,
        # r = v - A z: all entries, z (2n), fp32 basis (4n), r written (2n)
        "r_residual": 8 * n + (sv + si) * nnz + off,
        # level-2 SpMV + dots: all entries, z (2n), w written (4n), 2.5 fp32
        # basis vectors on average (10n)
        "spmv_l2": 16 * n + (sv + si) * nnz + off,
    }


def timed_solves(fn, steps, warmup):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    out = None
    times = []
    t_all = time.perf_counter()
    for _ in range(steps):
        t = time.perf_counter()
        out = fn()
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t)
    torch.cuda.synchronize()
    total = time.perf_counter() - t_all
    return out, times, total


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(A, b, outer_iters_gpu, tol, budget_s=45.0):
    """The CPU oracle on this host's cores: its OpenMP build (independent loop
    iterations shared among threads; dot order 2, blocks of 1,024 summed
    alone and then in order, which the plain build gives bit for bit) runs
    the whole fp16-F3R solve when one outermost iteration says it fits in
    budget_s, else that iteration is scaled to the GPU's count; one
    single-threaded outermost iteration of the plain build is timed beside
    it and scaled the same way."""
    import oracle as O
    from oracle import build as OB

    def run(path, max_outer):
        p = O.default_params(O.FP16_F3R)
        p.dot_order = 2
        p.max_outer = max_outer
        o = O.Oracle(A.row_ptr, A.col_idx, A.val, p, lib_path=path)
        t = time.perf_counter()
        _, info = o.solve(b, tol)
        dt = time.perf_counter() - t
        threads = o.L.or_threads()
        o.close()
        return dt, info, threads

    dt1, i1, threads = run(OB.LIB_OMP, 1)
    per_outer = dt1 / max(i1.outer_iters, 1)
    if per_outer * outer_iters_gpu <= budget_s:
        dt, info, threads = run(OB.LIB_OMP, 300)
        value = dt
        sample = (f"the whole fp16-F3R solve of this workload by the OpenMP build of the C oracle on "
                  f"{threads} threads: {info.outer_iters} outermost iterations, {info.m_calls} M "
                  f"applications, relres {info.relres_true:.2e}, {dt:.2f} s (measured, not scaled)")
    else:
        value = per_outer * outer_iters_gpu
        sample = (f"one outermost iteration of the OpenMP build of the C oracle on {threads} threads "
                  f"took {dt1:.2f} s; scaled by the {outer_iters_gpu} outermost iterations of the GPU "
                  f"solve (an extrapolation)")
    ds, isg, _ = run(None, 1)
    single = ds / max(isg.outer_iters, 1) * outer_iters_gpu
    return {
        "value": round(value, 4),
        "unit": "s",
        "cores": threads,
        "kind": "oracle",
        "sample": sample,
        "nproc": len(os.sched_getaffinity(0)),
        "cpu_model": _cpu_model(),
        "single_thread": {"value": round(single, 3), "unit": "s",
                          "sample": f"one outermost iteration of the plain single-threaded build took "
                                    f"{ds:.2f} s; scaled by the {outer_iters_gpu} outermost iterations "
                                    f"of the GPU solve (an extrapolation)"},
    }


WORKLOADS = {
    # name: (generator, description, extra variants timed beside fp16-F3R)
    "poisson3d_128": (lambda W: W.poisson3d(128), "3D 7-point Poisson 128^3", ("fp32", "fp64")),
    "convdiff_q1_100": (lambda W: W.convdiff_q1(100),
                        "3D Q1 convection-diffusion 100^3 (27-point, nonsymmetric, lognormal sigma 1.5, "
                        "Peclet 50)", ("bf16", "fp32", "fp64")),
    "elasticity_bonds_64": (lambda W: W.elasticity_bonds(64),
                            "elasticity-like bond model, 3x3 blocks on a jittered 64^3 lattice, 26 neighbours",
                            ("bf16",)),
    "poisson2d_64": (lambda W: W.poisson2d(64), "2D 5-point Poisson 64^2", ("fp32", "fp64")),
    "hpcg_7_7_7": (lambda W: W.build("hpcg_7_7_7"), "HPCG 27-point operator, 128^3 (Table 2)",
                   ("fp32", "fp64")),
    "hpgmp_7_7_7": (lambda W: W.build("hpgmp_7_7_7"), "HPGMP nonsymmetric 27-point operator, 128^3, "
                    "beta 0.5 (Table 2)", ("fp32", "fp64")),
    "varcoef2d_batch256": (None, "256 variable-coefficient 2D 5-point systems, sides U{32..256}", ()),
}
# the larger Table 2 operators (2^x x 2^y x 2^z grids)
for _sz in ("8_7_7", "8_8_7", "8_8_8"):
    WORKLOADS[f"hpcg_{_sz}"] = (lambda W, _s=_sz: W.build(f"hpcg_{_s}"),
                                f"HPCG 27-point operator, 2^({_sz.replace('_', ',')}) grid (Table 2)",
                                ("fp32", "fp64"))
    WORKLOADS[f"hpgmp_{_sz}"] = (lambda W, _s=_sz: W.build(f"hpgmp_{_s}"),
                                 f"HPGMP nonsymmetric 27-point operator, 2^({_sz.replace('_', ',')}) grid, "
                                 "beta 0.5 (Table 2)", ("fp32", "fp64"))


def ablation_settings(P):
    """The parameter studies of Sec. 6 (Table 4 and Figs. 3, 5 and 6) as
    (name, levels, c, omega_init); levels are (kind, m, prec_a, prec_v)."""
    F, R = P.FGMRES, P.RICHARDSON
    D, S, H = P.FP64, P.FP32, P.FP16

    def nest(m2=8, m3=4, m4=2):
        return [(F, 100, D, D), (F, m2, S, S), (F, m3, H, S), (R, m4, H, H)]

    out = [("F3R (F100, F8, F4, R2)", nest(), 64, 1.0)]
    out += [(f"m2={m}", nest(m2=m), 64, 1.0) for m in (2, 4, 16, 32)]
    out += [(f"m3={m}", nest(m3=m), 64, 1.0) for m in (2, 8, 16)]
    out += [(f"m4={m}", nest(m4=m), 64, 1.0) for m in (1, 4, 8)]
    out += [(f"c={c}", nest(), c, 1.0) for c in (1, 8, 512)]
    out += [(f"static w={w}", nest(), 0, w) for w in (0.6, 0.8, 1.0, 1.2)]
    out += [("F2", [(F, 100, D, D), (F, 64, S, S)], 64, 1.0),
            ("fp16-F2", [(F, 100, D, D), (F, 64, H, H)], 64, 1.0),
            ("F3", [(F, 100, D, D), (F, 8, S, S), (F, 8, H, S)], 64, 1.0),
            ("fp16-F3", [(F, 100, D, D), (F, 8, S, S), (F, 8, H, H)], 64, 1.0),
            ("F4", [(F, 100, D, D), (F, 8, S, S), (F, 4, H, S), (F, 2, H, H)], 64, 1.0)]
    return out


def bench_ablation(args, P, W, torch):
    """Time every setting of the parameter studies on the workload (mean of
    --steps solves after --warmup) with its outermost iterations and M
    applications."""
    gen, desc, _ = WORKLOADS[args.workload]
    A = gen(W)
    xs, b = W.rhs(A, args.workload)
    bt = torch.as_tensor(b, device="cuda")
    rows = []
    for name, levels, c, w0 in ablation_settings(P):
        p = P.params_default(P.VARIANT_FP16)
        p.nlev = len(levels)
        for d, (kind, m, pa, pv) in enumerate(levels):
            p.lev[d].kind, p.lev[d].m, p.lev[d].prec_a, p.lev[d].prec_v = kind, m, pa, pv
        p.c, p.omega_init = c, w0
        s = P.Solver(A.row_ptr, A.col_idx, A.val, p)
        (x, info), times, total = timed_solves(lambda: s.solve(bt, raise_on_error=False), args.steps,
                                               args.warmup)
        row = {"setting": name, "ms": round(total / args.steps * 1e3, 3), "status": info.status,
               "outer_iters": info.outer_iters, "m_calls": info.m_calls,
               "relres_true": info.relres_true}
        rows.append(row)
        log(f"[bench] ablation {name}: {row['ms']:.2f} ms, outer {info.outer_iters}, "
            f"M calls {info.m_calls}, status {info.status}")
        s.close()
    return {"ablation": args.workload, "workload": f"{args.workload}: {desc} (n={A.n}, nnz={A.nnz})",
            "tol": 1e-10, "steps": args.steps, "warmup": args.warmup, "rows": rows}


def bench_ilu(args, P, W, torch):
    """Block-Jacobi ILU(0) as M (Sec. 5.1's CPU preconditioner) against the
    two-sweep M on the workload: fp16-F3R with several block counts, fp64-F3R
    and fp64 CG / FGMRES(64) with the paper's 112 blocks; each with its set-up
    time and the duration of one forward sweep (HIP events, probe solve)."""
    gen, desc, _ = WORKLOADS[args.workload]
    A = gen(W)
    xs, b = W.rhs(A, args.workload)
    bt = torch.as_tensor(b, device="cuda")
    rows = []

    def run(label, variant, m_kind, blocks, solver="f3r"):
        p = P.params_default(variant)
        p.m_kind, p.ilu_blocks = m_kind, blocks
        t = time.perf_counter()
        s = P.Solver(A.row_ptr, A.col_idx, A.val, p)
        torch.cuda.synchronize()
        setup_s = time.perf_counter() - t
        if solver == "f3r":
            fn = lambda: s.solve(bt, raise_on_error=False)  # noqa: E731
        elif solver == "cg":
            fn = lambda: s.krylov_solve(bt, P.CG, P.FP64, max_iter=19200, raise_on_error=False)  # noqa: E731
        else:
            fn = lambda: s.fgmres_solve(bt, m=64, raise_on_error=False)  # noqa: E731
        (x, info), times, total = timed_solves(fn, args.steps, args.warmup)
        row = {"setting": label, "ms": round(total / args.steps * 1e3, 3), "status": info.status,
               "iters": info.outer_iters, "m_calls": info.m_calls, "setup_s": round(setup_s, 4),
               "relres_true": info.relres_true}
        if solver == "f3r":
            ov = P.params_default(variant)
            ov.probe_kernel = P.PROBE_M_LOWER
            _, ip = s.solve(bt, override=ov, raise_on_error=False)
            row["m_forward_sweep_us"] = round(ip.probe_ms / max(ip.probe_launches, 1) * 1e3, 2)
        rows.append(row)
        log(f"[bench] {label}: {row['ms']:.2f} ms, iters {info.outer_iters}, M calls {info.m_calls}, "
            f"set-up {setup_s:.3f} s" + (f", forward sweep {row['m_forward_sweep_us']} us"
                                         if "m_forward_sweep_us" in row else ""))
        s.close()

    run("fp16-F3R, two-sweep M", P.VARIANT_FP16, P.M_SGS, 112)
    for nb in (112, 1024, 8192):
        run(f"fp16-F3R, block-Jacobi ILU(0), {nb} blocks", P.VARIANT_FP16, P.M_ILU, nb)
    run("fp64-F3R, block-Jacobi ILU(0), 112 blocks", P.VARIANT_FP64, P.M_ILU, 112)
    Asp = A.to_scipy()
    if abs(Asp - Asp.T).max() == 0.0:  # CG for symmetric matrices only
        run("fp64 CG, block-Jacobi ILU(0), 112 blocks", P.VARIANT_FP16, P.M_ILU, 112, "cg")
    run("fp64 FGMRES(64), block-Jacobi ILU(0), 112 blocks", P.VARIANT_FP16, P.M_ILU, 112, "fgmres")
    return {"ilu": args.workload, "workload": f"{args.workload}: {desc} (n={A.n}, nnz={A.nnz})",
            "tol": 1e-10, "steps": args.steps, "warmup": args.warmup, "rows": rows}


def bench_batch(args, P, W, torch):
    """Batched solve in both modes (one persistent launch; lockstep per-kernel
    path) against the same systems solved one at a time."""
    count = 256
    sizes = W.batch_sizes(count, 32, 256)
    mats = [W.varcoef2d(int(sz), tag=f"batch/{i}") for i, sz in enumerate(sizes)]
    rhss = [W.rhs(A, f"batch/{i}") for i, A in enumerate(mats)]
    ntot = sum(A.n for A in mats)
    log(f"[bench] batch of {count} systems, {ntot} unknowns")
    modes = {}
    for mode, lock in (("persistent", False), ("lockstep", True)):
        t = time.perf_counter()
        bs = P.BatchSolver([(A.row_ptr, A.col_idx, A.val) for A in mats], lockstep=lock)
        torch.cuda.synchronize()
        setup_s = time.perf_counter() - t
        bt = [torch.as_tensor(b, device="cuda") for _, b in rhss]
        (xs, infos, st), times, total = timed_solves(lambda: bs.solve(bt), args.steps, args.warmup)
        assert st == 0, [i.status for i in infos]
        mean_s = total / args.steps
        outs = [i.outer_iters for i in infos]
        modes[mode] = {"setup_s": round(setup_s, 4), "batch_s": round(mean_s, 6),
                       "batch_median_s": round(statistics.median(times), 6),
                       "systems_per_s": round(count / mean_s, 2),
                       "outer_iters_min_mean_max": [min(outs), round(float(np.mean(outs)), 2), max(outs)],
                       "worst_relres_true": max(i.relres_true for i in infos)}
        log(f"[bench] batched ({mode}): {mean_s * 1e3:.1f} ms, {count / mean_s:.1f} systems/s, "
            f"outer {min(outs)}..{max(outs)}, set-up {setup_s:.2f} s")
        bs.close()
    one = 0.0
    one_outer = []
    bt = [torch.as_tensor(b, device="cuda") for _, b in rhss]
    for i, A in enumerate(mats):
        g = P.Solver(A.row_ptr, A.col_idx, A.val)
        g.solve(bt[i])  # records the graphs of this system
        torch.cuda.synchronize()
        t = time.perf_counter()
        _, inf = g.solve(bt[i])
        torch.cuda.synchronize()
        one += time.perf_counter() - t
        assert inf.status == 0
        one_outer.append(inf.outer_iters)
        g.close()
    log(f"[bench] one at a time: {one * 1e3:.1f} ms, {count / one:.1f} systems/s")
    best = min(modes, key=lambda m: modes[m]["batch_s"])
    mean_s = modes[best]["batch_s"]
    cfg = {
        "workload": f"varcoef2d_batch256: {WORKLOADS['varcoef2d_batch256'][1]} "
                    f"({ntot} unknowns in total), k = exp(xi), x* ~ U[-1,1] seeded, b = A x*",
        "tol": 1e-10,
        "solver": "fp16-F3R (F100, F8, F4, R2, M), c=64, per system",
        "modes": {"persistent": "one launch, one 512-thread workgroup per system, largest first",
                  "lockstep": "systems stacked on the diagonal of one matrix, every kernel of the "
                              "per-kernel path covers all systems, sums and state per system"},
        "best_mode": best,
        "persistent": modes["persistent"],
        "lockstep": modes["lockstep"],
        "one_at_a_time_s": round(one, 6),
        "one_at_a_time_systems_per_s": round(count / one, 2),
        "one_at_a_time_outer_mean": round(float(np.mean(one_outer)), 2),
        "speedup_vs_one_at_a_time": round(one / mean_s, 3),
    }
    return {
        "metric": "batched F3R solves to 1e-10 per second (systems/s)",
        "value": round(count / mean_s, 3), "unit": "systems/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(mean_s * 1e3, 4), "higher_is_better": True,
        "scaling": "strong", "vs_baseline": None, "dtype": "f16/f32/f64", "data": "synthetic",
        "config": cfg, "roofline": None, "cpu_baseline": None,
    }


VARIANTS = {"fp32": "VARIANT_FP32", "fp64": "VARIANT_FP64", "bf16": "VARIANT_BF16"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="poisson3d_128", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--ilu", action="store_true",
                    help="block-Jacobi ILU(0) as M against the two-sweep M on the workload")
    ap.add_argument("--ablation", action="store_true",
                    help="time the parameter studies of Sec. 6 on the workload instead of the metric")
    ap.add_argument("--only-f3r", action="store_true", help="time the fp16-F3R solves only (profiling)")
    ap.add_argument("--paper-protocol", action="store_true",
                    help="b uniform on [0,1) and tolerance 1e-8 (the paper's runs, Sec. 5) instead of "
                         "b = A x* and 1e-10")
    ap.add_argument("--layout", choices=("auto", "sell", "diag", "slice"), default="auto",
                    help="device matrix format (default: picked at set-up by padding)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="first run one plain device copy of MIB MiB (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU; --gpus {args.gpus} is not supported "
              "(the solver is single-GPU; the design notes describe how it would shard)",
              file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2505_20719_amd as P
    import workloads as W

    torch.cuda.set_device(0)
    if args.copy_calibration:
        src = torch.ones(args.copy_calibration << 18, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"[bench] calibration copy of {args.copy_calibration} MiB done")
        del src, dst
    name = args.workload
    if name == "varcoef2d_batch256":
        print(json.dumps(bench_batch(args, P, W, torch)), flush=True)
        return
    if args.ablation:
        print(json.dumps(bench_ablation(args, P, W, torch)), flush=True)
        return
    if args.ilu:
        print(json.dumps(bench_ilu(args, P, W, torch)), flush=True)
        return
    gen, desc, extra = WORKLOADS[name]
    A = gen(W)
    if args.paper_protocol:
        tol = 1e-8
        b = W.paper_rhs(A, name)
        xs = None
    else:
        tol = 1e-10
        xs, b = W.rhs(A, name)
    bt = torch.as_tensor(b, device="cuda")
    log(f"[bench] {name} n={A.n} nnz={A.nnz}")

    t = time.perf_counter()
    layout = {"auto": P.LAYOUT_AUTO, "sell": P.LAYOUT_SELL, "diag": P.LAYOUT_DIAG,
              "slice": P.LAYOUT_SLICE}[args.layout]

    def params(variant):
        p = P.params_default(variant)
        p.layout = layout
        return p

    s16 = P.Solver(A.row_ptr, A.col_idx, A.val, params(P.VARIANT_FP16))
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t

    (x16, info16), times, total = timed_solves(lambda: s16.solve(bt, tol=tol), args.steps, args.warmup)
    assert info16.status == 0, info16.as_dict()
    mean_s = total / args.steps
    log(f"[bench] fp16-F3R: {mean_s * 1e3:.2f} ms/solve, outer={info16.outer_iters}, "
        f"relres={info16.relres_true:.3e}, graphs={info16.graph_launches}")
    xh = x16.cpu().numpy()

    def err_of(x):
        return None if xs is None else float(np.linalg.norm(x - xs) / np.linalg.norm(xs))

    err_xstar = err_of(xh)

    result_cfg = {
        "workload": f"{name}: {desc} (n={A.n}, nnz={A.nnz}), "
                    + ("b ~ U[0,1) seeded (the paper's protocol)" if args.paper_protocol
                       else "x* ~ U[-1,1] seeded, b = A x*"),
        "tol": tol,
        "solver": "fp16-F3R (F100, F8, F4, R2, M), c=64, M = two-SpMV truncated SGS inverse",
        "setup_s": round(setup_s, 4),
        "f3r_fp16_median_s": round(statistics.median(times), 6),
        "f3r_fp16_outer_iters": info16.outer_iters,
        "f3r_fp16_m_calls": info16.m_calls,
        "relres_true": info16.relres_true,
        "err_vs_xstar": err_xstar,
        "device_format": {P.LAYOUT_SELL: "SELL-64, ", P.LAYOUT_DIAG: "diagonal-aligned SELL-64, ",
                          P.LAYOUT_SLICE: "diagonal-aligned SELL-64 with column offsets per slice, "}
                         [info16.layout]
                         + (f"{info16.idx_bits}-bit column indices, " if info16.idx_bits
                            else "no per-entry index, ")
                         + f"{info16.padded_nnz / A.nnz:.4f} padded/stored entries",
        "tuned_shapes": {k: f"{info16.rows_per_lane[i]} rows/lane, chunks of {info16.entry_chunk[i]}"
                         for i, k in enumerate(("m_lower", "m_upper", "r_residual"))},
        "tune_ms": round(info16.tune_ms, 3),
    }

    if args.paper_protocol:
        gold = os.path.join(ROOT, "tests", "golden", "table3_f3r_mcalls.txt")
        for line in open(gold):
            f = line.split()
            if f and f[0] == name:
                # M applications the paper reports for its CPU runs (Table 3)
                result_cfg["paper_table3_m_calls"] = {"fp64": f[1], "fp32": f[2], "fp16": f[3]}
    if not args.only_f3r:
        reps = max(1, min(args.steps, 3))
        (xf, infof), tf, totf = timed_solves(lambda: s16.fgmres_solve(bt, tol=tol, m=64), reps, 1)
        assert infof.status == 0, infof.as_dict()
        fg_s = totf / reps
        log(f"[bench] fp64 FGMRES(64): {fg_s * 1e3:.2f} ms/solve, iters={infof.outer_iters}")
        result_cfg.update({"fgmres64_s": round(fg_s, 6), "fgmres64_iters": infof.outer_iters,
                           "fgmres64_err_vs_xstar": err_of(xf.cpu().numpy()),
                           "speedup_vs_fgmres64": round(fg_s / mean_s, 3)})
        for key in extra:
            s = P.Solver(A.row_ptr, A.col_idx, A.val, params(getattr(P, VARIANTS[key])))
            (xv, iv), tv, totv = timed_solves(lambda: s.solve(bt, tol=tol), 2, 1)
            assert iv.status == 0, iv.as_dict()
            result_cfg[f"f3r_{key}_s"] = round(totv / 2, 6)
            result_cfg[f"f3r_{key}_outer_iters"] = iv.outer_iters
            result_cfg[f"f3r_{key}_err_vs_xstar"] = err_of(xv.cpu().numpy())
            result_cfg[f"f3r_{key}_m_calls"] = iv.m_calls
            log(f"[bench] {key}-F3R: {totv / 2 * 1e3:.2f} ms/solve, outer={iv.outer_iters}")
            s.close()
        if "fp64" in extra:
            result_cfg["speedup_fp16_vs_fp64_f3r"] = round(result_cfg["f3r_fp64_s"] / mean_s, 3)
        # the other comparison solvers of Sec. 5: fp64 FGMRES(64) with M stored
        # in fp16, and CG (symmetric matrices) and BiCGStab with M in fp64 and
        # in fp16 ("fp16-CG" = fp64 CG, fp16 preconditioner storage)
        Asp = A.to_scipy()
        runs = [("fp16_fgmres64", lambda: s16.fgmres_solve(bt, tol=tol, m=64, prec_m=P.FP16))]
        methods = [("bicgstab", P.BICGSTAB)]
        if abs(Asp - Asp.T).max() == 0.0:
            methods.insert(0, ("cg", P.CG))
        for key, method in methods:
            for pk, prec in (("fp64", P.FP64), ("fp16", P.FP16)):
                runs.append((f"{pk}_{key}", lambda method=method, prec=prec: s16.krylov_solve(
                    bt, method, prec, tol=tol, max_iter=19200)))
        for key, fn in runs:
            (xk, ik), tk, totk = timed_solves(fn, reps, 1)
            assert ik.status == 0, (key, ik.as_dict())
            result_cfg[f"{key}_s"] = round(totk / reps, 6)
            result_cfg[f"{key}_iters"] = ik.outer_iters
            result_cfg[f"{key}_err_vs_xstar"] = err_of(xk.cpu().numpy())
            result_cfg[f"speedup_vs_{key}"] = round(totk / reps / mean_s, 3)
            log(f"[bench] {key}: {totk / reps * 1e3:.2f} ms/solve, iters={ik.outer_iters}")

    # live per-kernel timing of the hot kernels inside one solve (HIP events
    # on the solve's stream, direct launches)
    width = int(round(info16.padded_nnz / (((A.n + 63) // 64) * 64)))
    ab = algorithmic_bytes(A, info16.idx_bits, info16.layout, width)
    sb = csr_model_bytes(A)
    probes = {"m_lower": P.PROBE_M_LOWER, "m_upper": P.PROBE_M_UPPER,
              "r_residual": P.PROBE_R_RESIDUAL, "spmv_l2": P.PROBE_SPMV_L2}
    kern = {}
    for key, pid in probes.items():
        ov = P.params_default(P.VARIANT_FP16)
        ov.probe_kernel = pid
        _, ip = s16.solve(bt, tol=tol, override=ov)
        avg_ms = ip.probe_ms / max(ip.probe_launches, 1)
        kern[key] = {"total_ms": ip.probe_ms, "launches": ip.probe_launches, "avg_us": avg_ms * 1e3,
                     "gbs": sb[key] / (avg_ms * 1e-3) / 1e9,
                     "gbs_format": ab[key] / (avg_ms * 1e-3) / 1e9}
        log(f"[bench] probe {key}: {ip.probe_launches} launches, avg {avg_ms * 1e3:.2f} us, "
            f"{kern[key]['gbs']:.0f} GB/s ({sb[key] / 1e6:.1f} MB/launch); "
            f"format bytes {ab[key] / 1e6:.1f} MB: {kern[key]['gbs_format']:.0f} GB/s")
    dom = max(kern, key=lambda k: kern[k]["launches"] * kern[k]["avg_us"])
    # achieved = the bytes the device format must move per launch (what the
    # kernel reads once and writes once) / the measured launch duration; the
    # CSR-model price of the scope table (4-byte indices and row pointers
    # that this format does not store) is reported apart as "effective"
    achieved = kern[dom]["gbs_format"]
    traffic = measured_traffic(dom, name)
    roofline = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "bytes_per_launch": int(ab[dom]), "avg_launch_us": round(kern[dom]["avg_us"], 3),
                "bytes_model": "device format: stored values and per-slice offsets read once, "
                               "vectors read and written once",
                # the same launch priced as a CSR kernel with 4-byte indices
                # and row pointers; an effective rate, not a fraction of
                # the peak (this format does not move those bytes)
                "effective_csr_model": {"bytes_per_launch": int(sb[dom]),
                                        "achieved": round(kern[dom]["gbs"], 1)}}
    result_cfg["kernels"] = {k: {kk: round(vv, 3) if isinstance(vv, float) else vv for kk, vv in v.items()}
                             for k, v in kern.items()}
    # standalone level SpMVs, warm (back to back) and cold (a 1 GiB buffer
    # read before every launch evicts the 256 MB last-level cache); bytes of
    # the device format: padded stored values, the per-entry index or the
    # per-slice offsets, x and y once
    scrub = torch.zeros(1 << 27, dtype=torch.float64, device="cuda")
    si = info16.idx_bits // 8
    ns = (A.n + 63) // 64
    idx_bytes = (info16.padded_nnz * si + (4.0 * ns if info16.layout == P.LAYOUT_SELL else 0.0)
                 if si else 4.0 * ns * width)
    spmv = {}
    for level, key, sa, sx, sy in ((0, "l0_fp64", 8, 8, 8), (1, "l1_fp32", 4, 4, 4),
                                   (2, "l2_fp16", 2, 2, 4)):
        nbytes = info16.padded_nnz * sa + idx_bytes + A.n * (sx + sy)
        warm = s16.time_spmv(level, reps=20)
        cold = s16.time_spmv(level, reps=20, scrub=scrub)
        spmv[key] = {"bytes": int(nbytes), "warm_us": round(warm * 1e3, 3),
                     "warm_gbs": round(nbytes / (warm * 1e-3) / 1e9, 1),
                     "cold_us": round(cold * 1e3, 3), "cold_gbs": round(nbytes / (cold * 1e-3) / 1e9, 1)}
        log(f"[bench] standalone SpMV {key}: {nbytes / 1e6:.1f} MB, warm {warm * 1e3:.2f} us "
            f"({spmv[key]['warm_gbs']:.0f} GB/s), cold {cold * 1e3:.2f} us ({spmv[key]['cold_gbs']:.0f} GB/s)")
    # what a plain read of the same 1 GiB buffer reaches (contiguous ranges
    # per workgroup, non-temporal 16-byte loads): the cold rates as a
    # fraction of it
    read_ms = s16.time_read(scrub, reps=10)
    rbytes = scrub.numel() * scrub.element_size()
    read_gbs = rbytes / (read_ms * 1e-3) / 1e9
    for key in spmv:
        spmv[key]["cold_frac_of_read"] = round(spmv[key]["cold_gbs"] / read_gbs, 3)
    result_cfg["read_reference"] = {"bytes": int(rbytes), "us": round(read_ms * 1e3, 3),
                                    "gbs": round(read_gbs, 1),
                                    "kernel": "k_read_ref: one contiguous range per workgroup, "
                                              "16-byte non-temporal loads"}
    log(f"[bench] read reference: {rbytes / 2**30:.0f} GiB in {read_ms * 1e3:.1f} us ({read_gbs:.0f} GB/s)")
    del scrub
    result_cfg["spmv_standalone"] = spmv

    cpu = None
    if not args.no_cpu_baseline:
        log("[bench] CPU oracle sample ...")
        cpu = cpu_baseline(A, b, info16.outer_iters, tol)
        log(f"[bench] CPU oracle on {cpu['cores']} threads: {cpu['value']:.2f} s "
            f"(one thread: about {cpu['single_thread']['value']:.1f} s)")

    out = {
        "metric": METRIC,
        "value": round(mean_s, 6),
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(mean_s * 1e3, 4),
        "higher_is_better": False,
        "scaling": "strong",
        "vs_baseline": None,
        "dtype": "f16/f32/f64",
        "data": "synthetic",
        "config": result_cfg,
        "spmv_gbs": round(kern["spmv_l2"]["gbs_format"], 1),
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
