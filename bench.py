#!/usr/bin/env python3
"""Benchmark: FGMRES time-to-solution of one linearised FSI Newton system.

One step = one full FGMRES(50) solve of A_h x = b to a 1e-8 true relative
residual (x0 = 0), right-preconditioned by the block-LDU algorithm with AMG
V(1,1) sub-inverses, on the 2D 256x64-cell Q2/Q1 FSI Jacobian (seeded,
synthetic), inputs resident in HBM.  The preconditioner build (host AMG setup
+ upload) is reported separately and is not part of a step.

Prints one JSON line.  Extra objects: ``roofline`` for the dominant kernel
(the monolithic A_h CSR product, timed with HIP events on the solver's
stream), ``cpu_baseline`` (the CPU oracle on a bounded sample, rank 0 only).
"""
import argparse
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

# HBM bytes per launch of the A_h product measured with rocprofv3 hardware
# counters (FETCH_SIZE x 2.0 + WRITE_SIZE x 1.0, both scales read off a
# 256 MiB device copy in the same runs); see profiles/c2_spmv_hbm_traffic.md.
# Valid only for the kernel and workload it was measured on.
MEASURED_TRAFFIC = {("c2", 0): 180572657}
METRIC = "FGMRES time-to-solution per Newton solve @1e-8 resid; SpMV/V-cycle HBM GB/s"


def spmv_bytes(sysm) -> float:
    """Algorithmic bytes of y = A_h x (FP64 CSR, int32 columns, int64 row
    pointers): 12 nnz + 8 (N + 1) + 8 N (x once) + 8 N (y)."""
    N, nnz = sysm.N, sysm.nnz
    return 12.0 * nnz + 8.0 * (N + 1) + 8.0 * N + 8.0 * N


def cpu_baseline(sysm, gpu_iters: int, sample_iters: int = 25):
    """The CPU oracle, as it stands, on a bounded sample: its AMG setup and
    `sample_iters` FGMRES iterations; the per-iteration time is scaled to the
    iteration count of a full solve."""
    import numpy as np
    try:
        from threadpoolctl import threadpool_limits
    except ImportError:  # pragma: no cover
        threadpool_limits = None
    from oracle import blocks, krylov, precond
    ctx = threadpool_limits(limits=1) if threadpool_limits else None
    try:
        bs = blocks.BlockSystem(sysm)
        t0 = time.perf_counter()
        H = precond.build_hierarchies(bs)
        t_setup = time.perf_counter() - t0
        P = precond.amg_preconditioner(bs, H)
        t0 = time.perf_counter()
        x, info = krylov.fgmres(bs.matvec, P, sysm.b, tol=1e-30, restart=50, maxit=sample_iters)
        t_iter = (time.perf_counter() - t0) / max(info.iters, 1)
    finally:
        if ctx is not None:
            ctx.__exit__(None, None, None)
    return {
        "value": round(t_iter * gpu_iters * 1e3, 1),
        "unit": "ms",
        "cores": 1,
        "kind": "oracle",
        "sample": f"oracle AMG setup ({t_setup:.1f} s, not counted) + {info.iters} FGMRES iterations "
                  f"on the same system ({t_iter * 1e3:.0f} ms/iteration, numpy/scipy, 1 thread), "
                  f"scaled to the {gpu_iters} iterations of a full solve",
    }


def progress(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="c2")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--precision", default="f64", choices=["f64", "f32"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--pmc-probe", action="store_true",
                    help="only launch the A_h product 20 times and a 256 MiB device copy "
                         "(for hardware byte counters); prints nothing else")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for --gpus {args.gpus}); "
              "the multi-GPU sharding is a design, not an implementation", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import fsigen
    from paper_1801_05648_amd import FsiSolver

    cfg = fsigen.config(args.config)
    progress(f"generating {cfg.name} seed {args.seed}")
    sysm = fsigen.generate(cfg, seed=args.seed)
    progress(f"N={sysm.N} nnz={sysm.nnz}")
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream(dev)
    solver = FsiSolver.from_system(sysm, device=0, stream=stream)
    if args.pmc_probe:
        xs = torch.randn(sysm.N, dtype=torch.float64, device=dev)
        ys = torch.empty_like(xs)
        for _ in range(20):
            solver.spmv(xs, ys)
        src = torch.ones(256 * 2 ** 20 // 8, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"pmc_probe": True, "spmv_bytes": spmv_bytes(sysm), "copy_bytes": 2 * 256 * 2 ** 20}))
        solver.close()
        return
    t0 = time.perf_counter()
    progress("building the preconditioner")
    solver.build_precond(args.precision)
    torch.cuda.synchronize()
    setup_ms = (time.perf_counter() - t0) * 1e3
    progress(f"preconditioner built in {setup_ms:.0f} ms")

    b = torch.from_numpy(sysm.b).to(dev)
    x = torch.zeros_like(b)
    for _ in range(args.warmup):
        x.zero_()
        solver.solve(b, x)
    torch.cuda.synchronize()
    times, iters, resid = [], [], []
    t_pre = t_spmv = t_gs = 0.0
    n_timed = 0
    progress("warm-up done")
    t_all = time.perf_counter()
    for _ in range(args.steps):
        x.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, info = solver.solve(b, x, timing=True)
        torch.cuda.synchronize()
        times.append((time.perf_counter() - t0) * 1e3)
        iters.append(info.iters)
        resid.append(info.true_rel_resid)
        t_pre += info.t_precond_ms
        t_spmv += info.t_spmv_ms
        t_gs += info.t_gs_ms
        n_timed += info.n_timed
        if not info.converged:
            raise SystemExit(f"solve did not converge: {info}")
    t_all = (time.perf_counter() - t_all) * 1e3
    ms = statistics.mean(times)

    # dominant kernel: the A_h CSR product, timed inside the timed solves by
    # HIP events recorded on the solver's stream around every launch of it
    spmv_ms = t_spmv / max(n_timed, 1)
    nbytes = spmv_bytes(sysm)
    achieved = nbytes / (spmv_ms * 1e-3) / 1e9

    # one V(1,1) cycle of the fluid-velocity hierarchy (largest V-cycle),
    # bytes as executed by the level kernels
    nv = int(solver.hierarchy_info("H_A")[0][0])
    bv = torch.randn(nv, dtype=torch.float64, device=dev)
    xv = torch.empty_like(bv)
    for _ in range(5):
        solver.vcycle("H_A", bv, xv)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    reps = 50
    for _ in range(reps):
        solver.vcycle("H_A", bv, xv)
    e1.record(stream)
    e1.synchronize()
    vc_ms = e0.elapsed_time(e1) / reps
    vc_bytes = solver.vcycle_bytes("H_A")

    line = {
        "metric": METRIC,
        "value": round(ms, 3),
        "unit": "ms",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 3),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "f64" else "f64-krylov/f32-precond",
        "data": "synthetic",
        "config": {
            "workload": (f"2D FSI Jacobian {cfg.cells[0]}x{cfg.cells[1]} Q2/Q1 cells" if cfg.dim == 2 else
                         f"3D FSI Jacobian {'x'.join(map(str, cfg.cells))} Q2/Q1 cells"),
            "name": cfg.name, "seed": args.seed, "N": sysm.N, "nnz": sysm.nnz,
            "tol": 1e-8, "restart": 50, "precond": "block-LDU + SA-AMG V(1,1) Jacobi",
        },
        "iters": iters[0],
        "true_rel_resid": max(resid),
        "ms_min": round(min(times), 3),
        "setup_ms": round(setup_ms, 1),
        "timed_wall_ms": round(t_all, 1),
        "phase_ms_per_iter": {"precond": round(t_pre / max(n_timed, 1), 4),
                              "spmv": round(spmv_ms, 4), "gram_schmidt": round(t_gs / max(n_timed, 1), 4)},
        "roofline": {
            "kernel": "csr_rows_kernel (A_h product inside the solve)",
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": MEASURED_TRAFFIC.get((cfg.name, args.seed)),
            "algorithmic_bytes": int(nbytes),
            "kernel_ms": round(spmv_ms, 5),
        },
        "vcycle_H_A": {
            "bytes": int(vc_bytes), "ms": round(vc_ms, 5),
            "GB/s": round(vc_bytes / (vc_ms * 1e-3) / 1e9, 1),
            "frac": round(vc_bytes / (vc_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "levels": int(len(solver.hierarchy_info("H_A")[0])),
        },
    }
    if not args.no_cpu_baseline:
        progress("timing the CPU oracle sample")
        line["cpu_baseline"] = cpu_baseline(sysm, iters[0])
    solver.close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
