#!/usr/bin/env python3
"""Benchmark: FGMRES time-to-solution of one linearised FSI Newton system.

One step = one full FGMRES(50) solve of A_h x = b to a 1e-8 true relative
residual (x0 = 0), right-preconditioned by the block-LDU algorithm with AMG
sub-inverses, inputs resident in HBM.  Default workload: the 3D
128x32x32-cell Q2/Q1 FSI Jacobian (6.2M unknowns, 1.44e9 entries; seeded,
synthetic), FP64 throughout.  The preconditioner build (AMG setup steps on
the host threads, its sparse products on the GPU, uploads) is reported
separately (``setup_ms``) and is not part of a step.

Prints one JSON line.  Extra objects: ``roofline`` for the dominant kernel
(the A_h block product, timed with HIP events on the solver's stream),
``vcycle_H_A`` (one V-cycle of the largest hierarchy), ``alternatives``
(the same solve with the FP32 preconditioner, with and without BF16-stored
smoother diagonals, and with the paper's own forms of the fluid step,
against the FP64 solve), ``gpu_c3`` (the 64x16x16-cell system on
the GPU, the configuration the CPU oracle is timed on) and ``cpu_baseline``
(the CPU oracle on a bounded sample, rank 0 only).
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
# 256 MiB device copy in the same runs); see profiles/a_h_spmv_hbm_traffic.md.
# Valid only for the kernel and workload it was measured on (empty: the
# kernel changed since the counters were taken).
MEASURED_TRAFFIC = {"c2": 155605299, "c3": 1752204761, "c4": 15363719875}
# The same for one H_A V-cycle of the benchmark preconditioner (bench.py
# --pmc-vcycle); see profiles/h_a_vcycle_hbm_traffic.md.
# Keyed by workload: (traffic, the cycle's bytes as stored when measured); a
# hierarchy of other bytes (other AMG options) has no figure.
MEASURED_VCYCLE_TRAFFIC = {"c2": (115217321, 108663072), "c3": (1306569344, 1279777388),
                           "c4": (9351010137, 9096401408)}
DTYPE = {"f64": "f64", "f32": "f64-krylov/f32-precond", "f32-bf16diag": "f64-krylov/f32-precond/bf16-diag"}
METRIC = "FGMRES time-to-solution per Newton solve @1e-8 resid; SpMV/V-cycle HBM GB/s"


def csr_bytes(sysm) -> float:
    """Bytes of y = A_h x in plain CSR (FP64 values, int32 columns, int64 row
    pointers): 12 nnz + 8 (N + 1) + 8 N (x once) + 8 N (y)."""
    N, nnz = sysm.N, sysm.nnz
    return 12.0 * nnz + 8.0 * (N + 1) + 8.0 * N + 8.0 * N


def cpu_baseline(args, gpu_c3=None, sample_iters: int = 2):
    """The CPU oracle, as it stands, on a bounded sample.

    The oracle (numpy/scipy, one thread) cannot build its AMG hierarchies for
    the 128x32x32 system within the benchmark's time, so its sample is the
    64x16x16-cell system (configuration c3, seed 0) with the benchmarked
    preconditioner: the AMG setup (timed, not counted) and `sample_iters`
    FGMRES iterations; the per-iteration time is scaled to the GPU's
    iteration count on that same system (``gpu_c3``), giving ms per c3 solve.
    No scaling across configurations."""
    import platform
    try:
        from threadpoolctl import threadpool_limits
    except ImportError:  # pragma: no cover
        threadpool_limits = None
    import fsigen
    from oracle import blocks, krylov, precond
    cfg = fsigen.config("c3")
    sysm = fsigen.generate(cfg, seed=0)
    ctx = threadpool_limits(limits=1) if threadpool_limits else None
    try:
        bs = blocks.BlockSystem(sysm)
        o = precond_opts(args, cfg.dim)
        t0 = time.perf_counter()
        H = precond.build_hierarchies(bs, eps0=o["strength0"], max_coarse=o["max_coarse"], schur=o["schur"],
                                      x_approx=args.x_approx)
        t_setup = time.perf_counter() - t0
        cheb = {h: o["cheb_degree"] for h in o["cheb"]} if o["cheb_degree"] > 0 else None
        poly = {h: (o["poly_degree"], o["poly_ratio"]) for h in o["poly"]}
        P = precond.amg_preconditioner(bs, H, cheb=cheb, poly=poly, fluid_inner=o["fluid_inner"],
                                       fluid_inner_pc=o["fluid_inner_pc"], x_approx=o["x_approx"],
                                       uzawa_inner=o["uzawa_inner"])
        t0 = time.perf_counter()
        x, info = krylov.fgmres(bs.matvec, P, sysm.b, tol=1e-30, restart=50, maxit=sample_iters)
        t_iter = (time.perf_counter() - t0) / max(info.iters, 1)
    finally:
        if ctx is not None:
            ctx.__exit__(None, None, None)
    cpu = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                cpu = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    iters = gpu_c3["iters"] if gpu_c3 else None
    return {
        "value": round(t_iter * iters * 1e3, 1) if iters else None,
        "unit": "ms",
        "cores": 1,
        "kind": "oracle",
        "config": "c3: 3D FSI Jacobian 64x16x16 Q2/Q1 cells, seed 0 (N=%d, nnz=%d)" % (sysm.N, sysm.nnz),
        "sample": f"oracle AMG setup of c3 ({t_setup:.1f} s, not counted) + {info.iters} FGMRES iterations "
                  f"({t_iter * 1e3:.0f} ms/iteration, numpy/scipy on 1 thread), scaled to the {iters} iterations "
                  f"of the GPU's solve of the same c3 system: ms per c3 solve, compare with gpu_c3.ms",
        "host": {"nproc": os.cpu_count(), "cpu": cpu, "python": platform.python_version()},
    }


_T0 = time.perf_counter()


def progress(msg: str) -> None:
    print(f"[bench {time.perf_counter() - _T0:7.1f} s] {msg}", file=sys.stderr, flush=True)


def cheb_on(args) -> tuple:
    return tuple(h for h in args.cheb_on.split(",") if h and h not in poly_on(args))


def poly_on(args) -> tuple:
    return tuple(h for h in (args.poly_on or "").split(",") if h)


def precond_name(args) -> str:
    poly = poly_on(args)
    ptxt = f"; {'/'.join(poly)} by {args.poly_degree} Chebyshev steps alone" if poly else ""
    ptxt += f"; S_p {args.schur.upper()}"
    if args.x_approx != "F":
        ptxt += "; X by its block-diagonal approximation"
    if args.uzawa_inner > 0:
        ptxt += f"; each inverse of the Uzawa-like step by {args.uzawa_inner} AMG-preconditioned GMRES steps"
    elif args.fluid_inner > 0:
        ptxt += f"; F^-1 by {args.fluid_inner} inner GMRES steps ({args.fluid_inner_pc} step)"
    if args.cheb <= 0:
        return "block-LDU + SA-AMG V(1,1) Jacobi" + ptxt
    on = cheb_on(args)
    off = [h for h in ("H_M", "H_SIG", "H_MS", "H_A", "H_P") if h not in on and h not in poly]
    return (f"block-LDU + SA-AMG V-cycles: Chebyshev({args.cheb}) on {'/'.join(on)}, "
            f"Jacobi V(1,1) on {'/'.join(off)}" + ptxt)


def he_init(k_in: int, hidden: int, d: int, seed: int):
    """Seeded He-style initial weights of the smoother network (the random
    draws are inputs of the training)."""
    import numpy as np
    rng = np.random.default_rng(seed)
    return [(rng.standard_normal((k_in, hidden)) * np.sqrt(2.0 / k_in)).astype(np.float32),
            (rng.standard_normal((hidden, hidden)) * np.sqrt(2.0 / hidden)).astype(np.float32),
            (rng.standard_normal((hidden, d)) * np.sqrt(1.0 / hidden)).astype(np.float32)]


def learned_run(args, cfg):
    """Pseudo-time workload of the learned smoother: record the finest-level
    V-cycle inputs of the H_M and H_SIG cycles over the Newton solves of the
    first `train_steps` pseudo-time steps, train both networks on the device
    (two-grid energy loss), then time the solves of later steps with the plain
    and with the learned cycles, both to a 1e-8 FP64 true residual."""
    import numpy as np
    import torch

    import fsigen
    from paper_1801_05648_amd import FsiSolver

    from concurrent.futures import ThreadPoolExecutor

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream(dev)
    phase = fsigen.pseudo_time_phase
    train = [(k, i) for k in range(args.train_steps) for i in range(3)]
    eval_steps = (list(range(args.train_steps, 50)) if args.eval_steps == ["all"]
                  else [int(k) for k in args.eval_steps])
    evals = [(k, i) for k in eval_steps for i in range(args.eval_solves)]
    progress(f"{cfg.name}: training on {len(train)} Newton systems, evaluating {len(evals)}")
    # the next system is assembled on a host thread while the GPU solves this one
    gen = ThreadPoolExecutor(max_workers=1)
    systems = train + evals
    ahead = {0: gen.submit(fsigen.generate, cfg, seed=args.seed, t_phase=phase(*systems[0]))}

    def system_at(n):
        if n + 1 < len(systems):
            ahead[n + 1] = gen.submit(fsigen.generate, cfg, seed=args.seed, t_phase=phase(*systems[n + 1]))
        return ahead.pop(n).result()

    sysm = system_at(0)
    solver = FsiSolver.from_system(sysm, device=0, stream=stream)
    solver.build_precond(args.precision, **precond_opts(args, cfg.dim))
    d = sysm.dim
    W = he_init(3 ** d * d, 64, d, seed=args.seed)
    for which in ("H_M", "H_SIG"):
        solver.mlp_set_weights(which, *W)
    solver.mlp_collect(max_vectors=args.max_vectors, every=args.record_every)
    t_rec = time.perf_counter()
    for n, (k, i) in enumerate(train):
        if n:
            sysm = system_at(n)
            solver.set_from_system(sysm)
            solver.build_precond(args.precision, **precond_opts(args, cfg.dim))
        b = torch.from_numpy(sysm.b).to(dev)
        _, info = solver.solve(b)
        progress(f"recorded step {k} solve {i}: {info.iters} iterations")
    t_rec = time.perf_counter() - t_rec
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tinfo = solver.mlp_train(steps=args.train_iters, batch=16384, lr=2e-3, seed=args.seed, loss="energy")
    torch.cuda.synchronize()
    train_ms = (time.perf_counter() - t0) * 1e3
    progress(f"trained in {train_ms:.0f} ms: {tinfo}")
    rows = []
    for n, (k, i) in enumerate(evals):
        sysm = system_at(len(train) + n)
        solver.set_from_system(sysm)
        solver.build_precond(args.precision, **precond_opts(args, cfg.dim))
        b = torch.from_numpy(sysm.b).to(dev)
        res = {}
        for mode in ("plain", "learned"):
            for which in ("H_M", "H_SIG"):
                solver.mlp_enable(which, mode == "learned")
            x = torch.zeros_like(b)
            for _ in range(args.warmup):
                x.zero_()
                solver.solve(b, x)
            times = []
            for _ in range(args.steps):
                x.zero_()
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                _, info = solver.solve(b, x)
                torch.cuda.synchronize()
                times.append((time.perf_counter() - t0) * 1e3)
                if not info.converged:
                    raise SystemExit(f"{mode} solve did not converge: {info}")
            res[mode] = (statistics.mean(times), info, x.clone())
        diff = float(torch.linalg.norm(res["learned"][2] - res["plain"][2]) / torch.linalg.norm(res["plain"][2]))
        row = {"step": k, "solve": i,
               "plain_ms": round(res["plain"][0], 3), "plain_iters": res["plain"][1].iters,
               "learned_ms": round(res["learned"][0], 3), "learned_iters": res["learned"][1].iters,
               "learned_fallbacks": res["learned"][1].mlp_fallbacks,
               "learned_true_rel_resid": res["learned"][1].true_rel_resid,
               "solution_rel_diff": diff}
        progress(f"step {k}: {row}")
        rows.append(row)
    solver.close()
    gen.shutdown()
    pm = statistics.mean(r["plain_ms"] for r in rows)
    lm = statistics.mean(r["learned_ms"] for r in rows)
    line = {
        "metric": "FGMRES time-to-solution per Newton solve @1e-8 resid, learned vs plain V-cycle smoothing",
        "value": round(lm, 3), "unit": "ms", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(lm, 3), "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": DTYPE[args.precision],
        "data": "synthetic",
        "config": {"workload": f"pseudo-time FSI Jacobians {'x'.join(map(str, cfg.cells))} cells",
                   "name": cfg.name, "seed": args.seed, "train_systems": len(train),
                   "precond": precond_name(args),
                   "eval_steps": [eval_steps[0], eval_steps[-1]] if args.eval_steps == ["all"] else eval_steps,
                   "eval_solves_per_step": args.eval_solves, "eval_systems": len(evals)},
        "plain_ms": round(pm, 3), "learned_over_plain_time": round(lm / pm, 4),
        "learned_faster_on": sum(r["learned_ms"] < r["plain_ms"] for r in rows),
        "max_solution_rel_diff": max(r["solution_rel_diff"] for r in rows),
        "plain_iters_mean": statistics.mean(r["plain_iters"] for r in rows),
        "learned_iters_mean": statistics.mean(r["learned_iters"] for r in rows),
        "record_s": round(t_rec, 1), "train_ms": round(train_ms, 1), "training": tinfo, "per_system": rows,
    }
    print(json.dumps(line), flush=True)


def precond_opts(args, dim: int) -> dict:
    """build_precond keyword arguments of the benchmarked preconditioner for a
    workload of dimension `dim`: the options given on the command line, the
    defaults of that dimension for the others."""
    def given(name, default):
        v = getattr(args, name + "_arg")
        return default if v is None else v
    # the learned smoother's workload: Jacobi V(1,1) with 500-row coarse grids
    # in 2D; in 3D, where Jacobi sweeps everywhere take about 1300 iterations
    # (64x16x16), Chebyshev(4) on H_P and M_s by Chebyshev steps, H_M and
    # H_SIG left to the Jacobi sweeps the network replaces
    learned2d = args.learned and dim == 2
    # 3D solver: Chebyshev(6) sweeps, M_s by five Chebyshev steps, 4000-row
    # coarse grids and the strength threshold 0.04 cut 64x16x16 from 26 to 15
    # iterations (68.6 -> 38 ms) and 128x32x32 from 28 to 17 (466 -> 268 ms;
    # the larger dense coarse inverses cost about a second of its build).  In
    # 3D two M_s steps raise the iterations from 46 to 78 (64x16x16, the split
    # fluid step); in 2D, with the inner fluid GMRES, three take 17/18/21
    # instead of 19/20/23 (11.5 vs 12.3 ms), and the 3D changes gain nothing
    # there (256x64: 11.4-11.7 ms)
    solver3d = dim == 3 and not args.learned
    cheb = given("cheb", 0 if learned2d else 6 if solver3d else 4)
    max_coarse = given("max_coarse", 500 if learned2d else 4000 if solver3d else 2000)
    poly_on_s = given("poly_on", "" if learned2d else "H_MS")
    poly_degree = given("poly_degree", 5 if solver3d else 3)
    strength = given("strength", 0.04 if solver3d else 0.08)
    cheb_on = (args.cheb_on_arg if args.cheb_on_arg is not None
               else "H_MS,H_SIG" if dim == 2 else "H_P" if args.learned else "H_MS,H_SIG,H_P")
    fluid_inner = (args.fluid_inner_arg if args.fluid_inner_arg is not None
                   else (0 if args.learned else 2))
    poly = tuple(h for h in poly_on_s.split(",") if h)
    # SIMPLEC in 3D: with the inner GMRES on F it cuts 64x16x16 from 33 to 26
    # iterations (85.3 -> 66.8 ms) and 128x32x32 from 31 to 28 (519 -> 467 ms);
    # without the inner GMRES it had raised 128x32x32 from 47 to 68
    schur = args.schur_arg if args.schur_arg is not None else ("simple" if dim == 2 or args.learned else "simplec")
    return dict(max_coarse=max_coarse, strength0=strength, cheb_degree=cheb,
                cheb=tuple(h for h in cheb_on.split(",") if h and h not in poly), poly=poly,
                poly_degree=poly_degree, poly_ratio=args.poly_ratio, schur=schur,
                fluid_inner=0 if args.uzawa_inner > 0 else fluid_inner, fluid_inner_pc=args.fluid_inner_pc,
                uzawa_inner=args.uzawa_inner, x_approx=args.x_approx)


def paper_vs_own(args, opts) -> str:
    """Which parts of the benchmarked preconditioner are the paper's and which
    are this library's choices."""
    own = ["smoothed-aggregation parameters (the paper names only ML)",
           f"{args.schur.upper()} pressure Schur approximation (the paper states none)"]
    if opts["cheb_degree"] > 0 and opts["cheb"]:
        own.append(f"Chebyshev({opts['cheb_degree']}) smoothing on {'/'.join(opts['cheb'])}")
    if opts["poly"]:
        own.append(f"{'/'.join(opts['poly'])} by {opts['poly_degree']} Chebyshev steps alone "
                   "(the paper: an AMG solver)")
    if opts["uzawa_inner"] > 0:
        fluid = (f"the fluid inverse as the paper's Section 4.4 step: GMRES ({opts['uzawa_inner']} steps) on "
                 "each inverse of the Uzawa-like elimination")
    elif opts["fluid_inner"] > 0:
        own.append(f"the fluid inverse as {opts['fluid_inner']} GMRES steps on the whole F preconditioned by the "
                   f"{opts['fluid_inner_pc']} step (the paper puts GMRES on each inverse of the Uzawa-like "
                   "elimination: alternatives.paper_uzawa_gmres2)")
        fluid = None
    else:
        fluid = "the Uzawa-like fluid step with one V-cycle per inverse"
    paper = "the block-LDU algorithm (Section 4.1), the solid algorithm (Section 4.3)"
    if fluid:
        paper += ", " + fluid
    return f"paper's: {paper}; this library's: " + "; ".join(own)


def workload_name(cfg) -> str:
    cells = "x".join(map(str, cfg.cells))
    return f"{cfg.dim}D FSI Jacobian {cells} Q2/Q1 cells"


def cycle_ms(solver, hn, dim, stream, reps=50):
    """Average time of one V-cycle of hierarchy hn, back to back (HIP events
    on the solver's stream)."""
    import torch
    nv = int(solver.hierarchy_info(hn)[0][0]) * (dim if hn == "H_M" else 1)
    bv = torch.randn(nv, dtype=torch.float64, device="cuda:0")
    xv = torch.empty_like(bv)
    for _ in range(5):
        solver.vcycle(hn, bv, xv)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        solver.vcycle(hn, bv, xv)
    e1.record(stream)
    e1.synchronize()
    return e0.elapsed_time(e1) / reps


def stream_ceilings(stream, gib: int = 4):
    """Bandwidth of plain device streams in this run, for scale: a copy of
    `gib` GiB (read + write) and a sum over `gib` GiB (read), timed with
    events on the stream (best of 5 after a warm-up)."""
    import torch
    n = gib * 2 ** 30 // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda:0")
    b = torch.empty_like(a)
    out = {}
    for name, fn, nbytes in (("copy", lambda: b.copy_(a), 16.0 * n), ("read", lambda: a.sum(), 8.0 * n)):
        fn()
        best = None
        for _ in range(5):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            fn()
            e1.record(stream)
            e1.synchronize()
            t = e0.elapsed_time(e1)
            best = t if best is None else min(best, t)
        out[name + "_GBps"] = round(nbytes / (best * 1e-3) / 1e9, 1)
    del a, b
    torch.cuda.empty_cache()
    return out


def timed_solves(solver, b, x, k):
    """k solves from x0 = 0, each bracketed by device synchronisations;
    returns (ms list, last info)."""
    import torch
    times, info = [], None
    for _ in range(k):
        x.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, info = solver.solve(b, x)
        torch.cuda.synchronize()
        times.append((time.perf_counter() - t0) * 1e3)
        if not info.converged:
            raise SystemExit(f"solve did not converge: {info}")
    return times, info


def theta_steps_run(args, dim, stream):
    """One-step-theta time steps (Section 3.2) with the shifted Crank-Nicolson
    theta = 1/2 + dt on the mid-size system of the headline's dimension: the
    system handed to the library carries dt theta, the assembly the scheme's
    previous-level terms; each step is the quasi-Newton loop (SA hierarchies
    kept across reassemblies) followed by the advance of the fields."""
    import torch

    import fsigen
    from paper_1801_05648_amd import FsiSolver
    name = "c3" if dim == 3 else "c2"
    base = fsigen.config(name)
    theta = 0.5 + base.dt
    sysm = fsigen.generate(base.with_(dt=base.dt * theta), seed=0, fe=True)
    solver = FsiSolver.from_system(sysm, device=0, stream=stream)
    solver.fe_setup(base.with_(theta=theta), sysm.fe)
    solver.build_precond("f64", **precond_opts(args, dim))
    steps = []
    for _ in range(args.time_steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        info = solver.time_step(precond="reuse")
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3
        if not info.converged:
            raise SystemExit(f"time step did not converge: {info}")
        steps.append({"ms": round(ms, 1), "newton_steps": info.steps, "reassemblies": info.reassemblies,
                      "gmres_iters": info.lin_iters, "resid_inf": [float("%.4e" % v) for v in info.residuals],
                      "assembly_ms": round(info.t_assemble_ms, 1), "precond_ms": round(info.t_precond_ms, 1),
                      "solve_ms": round(info.t_solve_ms, 1)})
    solver.close()
    return {"workload": workload_name(base), "theta": theta, "dt": base.dt, "steps": steps,
            "note": "shifted Crank-Nicolson; each step: quasi-Newton (Section 6 rule) from the previous "
                    "step's state, then the fields advance"}


def fe_newton_run(r, opts):
    """The steps on either side of the solve (Section 3's residual and
    Jacobian assembled on the GPU, Section 6's quasi-Newton loop) on the
    benchmark system: the headline preconditioner is rebuilt (the other forms
    replaced it), residual and Jacobian assemblies are timed (median of three,
    synchronised calls), then the loop runs from the linearisation state with
    the SA hierarchies kept across reassemblies (the coupling blocks, Schur
    approximations and smoothers follow the new Jacobian)."""
    import torch
    solver = r["solver"]
    solver.build_precond("f64", **opts)
    N = solver.N
    R = torch.empty(N, dtype=torch.float64, device=r["b"].device)

    def med(f):
        ts = []
        for _ in range(3):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            f()
            torch.cuda.synchronize()
            ts.append((time.perf_counter() - t0) * 1e3)
        return round(statistics.median(ts), 2)
    res_ms = med(lambda: solver.fe_residual(None, R))
    r0 = float(R.abs().max())
    jac_ms = med(lambda: solver.fe_jacobian(None, host_blocks=False))
    dU, info = solver.newton(precond="reuse")
    torch.cuda.synchronize()
    rN = float(solver.fe_residual(dU, R).abs().max())
    if not info.converged or not rN < 1e-6 * r0:
        raise SystemExit(f"quasi-Newton loop failed: {info}")
    cells = 1
    for a in range(r["sysm"].dim):
        cells *= int(r["sysm"].cfg.cells[a])
    return {"cells": cells, "residual_ms": res_ms, "jacobian_ms": jac_ms,
            "jacobian_cells_per_s": round(cells / (jac_ms * 1e-3), 0),
            "newton": {"steps": info.steps, "reassemblies": info.reassemblies, "gmres_iters": info.lin_iters,
                       "resid_inf": [float("%.4e" % v) for v in info.residuals],
                       "ms": round(info.t_total_ms, 1), "assembly_ms": round(info.t_assemble_ms, 1),
                       "precond_ms": round(info.t_precond_ms, 1), "solve_ms": round(info.t_solve_ms, 1),
                       "rule": "Section 6: reassemble when ||r_k|| > 0.1 ||r_k-1||, stop at 1e-6 ||r_0||, "
                               "GMRES to 1e-3; SA hierarchies kept across reassemblies"}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="c4",
                    help="workload: c4 (3D 128x32x32, the default), c3 (3D 64x16x16), c2 (2D 256x64), ...")
    ap.add_argument("--seed", type=int, default=0, help="seed of the learned-smoother workload")
    ap.add_argument("--seeds", type=int, nargs="+", default=None,
                    help="seeds of the linearisation state; the timed solves cycle through them "
                         "(default 0 on c4, 0 1 2 otherwise)")
    ap.add_argument("--precision", default="f64", choices=["f64", "f32", "f32-bf16diag"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true",
                    help="skip the other preconditioner forms reported beside the headline solve")
    ap.add_argument("--no-fe", action="store_true",
                    help="skip the finite-element assembly and quasi-Newton loop reported after the solves")
    ap.add_argument("--time-steps", type=int, default=3,
                    help="shifted Crank-Nicolson time steps on the 64x16x16 (3D) or 256x64 (2D) system "
                         "reported after the solves (0: none)")
    ap.add_argument("--cheb", type=int, default=None,
                    help="Chebyshev degree of the sweeps on --cheb-on (0: Jacobi V(1,1) everywhere); "
                         "default 6 in 3D, 4 in 2D, 0 with --learned in 2D")
    ap.add_argument("--max-coarse", type=int, default=None,
                    help="AMG: coarsest level size bound (dense inverse below it); default 4000 in 3D, 2000 in 2D, "
                         "500 with --learned in 2D")
    ap.add_argument("--cheb-on", default=None,
                    help="comma-separated hierarchies that get the Chebyshev sweeps "
                         "(default: H_SIG in 2D, H_SIG and H_P in 3D)")
    ap.add_argument("--poly-on", default=None,
                    help="comma-separated hierarchies inverted by Chebyshev steps alone "
                         "(default H_MS, none with --learned)")
    ap.add_argument("--schur", default=None, choices=["simple", "simplec"],
                    help="pressure Schur approximation -D W^{-1} G: W = diag(A_f) (simple) or its "
                         "absolute row sums (simplec); default simplec in 3D, simple in 2D")
    ap.add_argument("--fluid-inner", type=int, default=None,
                    help="inner flexible GMRES steps for the fluid inverse (0: the Uzawa-like step "
                         "alone; default 2, 0 with --learned)")
    ap.add_argument("--fluid-inner-pc", default="triangular", choices=["uzawa", "triangular"],
                    help="preconditioner of the inner fluid GMRES: the Uzawa-like step or the block "
                         "upper-triangular step (one A_f V-cycle fewer; default)")
    ap.add_argument("--uzawa-inner", type=int, default=0,
                    help="GMRES steps per inverse of the Uzawa-like fluid step (Section 4.4 as written; "
                         "0: one V-cycle per inverse)")
    ap.add_argument("--x-approx", default="F", choices=["F", "blockdiag"],
                    help="fluid operator standing for the Schur complement X (Section 4.1)")
    ap.add_argument("--strength", type=float, default=None,
                    help="SA strength threshold of the finest level (halved per level); default 0.04 in 3D, 0.08 in 2D")
    ap.add_argument("--poly-degree", type=int, default=None,
                    help="Chebyshev-alone steps (default 5 in 3D, 3 in 2D)")
    ap.add_argument("--poly-ratio", type=float, default=8.0,
                    help="Chebyshev-alone inverses: interval [lam/ratio, lam]")
    ap.add_argument("--learned", action="store_true",
                    help="pseudo-time workload of the learned smoother (plain vs learned cycles)")
    ap.add_argument("--train-steps", type=int, default=10)
    ap.add_argument("--eval-steps", nargs="+", default=["all"],
                    help="pseudo-time steps evaluated by --learned ('all': every step after training, to 49)")
    ap.add_argument("--eval-solves", type=int, default=3, choices=[1, 2, 3],
                    help="Newton solves evaluated per step by --learned (3: all of them)")
    ap.add_argument("--train-iters", type=int, default=600)
    ap.add_argument("--max-vectors", type=int, default=192)
    ap.add_argument("--record-every", type=int, default=37)
    ap.add_argument("--pmc-vcycle", nargs="?", const="H_A", default=None,
                    help="counter probe: 25 V-cycles of a hierarchy (default H_A) and a 256 MiB copy, then exit")
    ap.add_argument("--pmc-probe", action="store_true",
                    help="only launch the A_h product 20 times and a 256 MiB device copy "
                         "(for hardware byte counters); prints nothing else")
    args = ap.parse_args()
    args.cheb_on_arg, args.fluid_inner_arg, args.schur_arg = args.cheb_on, args.fluid_inner, args.schur
    args.cheb_arg, args.max_coarse_arg, args.poly_on_arg = args.cheb, args.max_coarse, args.poly_on
    args.poly_degree_arg, args.strength_arg = args.poly_degree, args.strength
    if args.gpus != 1:
        print(f"bench.py: this library runs on one GPU only (asked for --gpus {args.gpus}); "
              "the multi-GPU sharding is a design, not an implementation", file=sys.stderr)
        sys.exit(2)

    import torch

    import fsigen
    from paper_1801_05648_amd import FsiError, FsiSolver

    cfg = fsigen.config(args.config)
    if args.seeds is None:
        args.seeds = [0] if cfg.name == "c4" else [0, 1, 2]
    opts = precond_opts(args, cfg.dim)
    # the resolved options of the main workload, for the line's description
    args.cheb_on = ",".join(opts["cheb"])
    args.fluid_inner = opts["fluid_inner"]
    args.schur = opts["schur"]
    args.cheb, args.max_coarse, args.strength = opts["cheb_degree"], opts["max_coarse"], opts["strength0"]
    args.poly_on, args.poly_degree = ",".join(opts["poly"]), opts["poly_degree"]
    if args.learned:
        learned_run(args, cfg)
        return
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream(dev)
    if args.pmc_vcycle:
        # hardware-counter probe of one hierarchy's V-cycle (default H_A, the
        # largest): the benchmark's preconditioner, 25 cycles (the only kernels
        # of the run after the host-side setup), then a plain 256 MiB copy for
        # the counter scale
        sysm = fsigen.generate(cfg, seed=args.seeds[0])
        solver = FsiSolver.from_system(sysm, device=0, stream=stream)
        solver.build_precond(args.precision, **opts)
        hn = args.pmc_vcycle
        nv = int(solver.hierarchy_info(hn)[0][0]) * (sysm.dim if hn == "H_M" else 1)
        bv = torch.randn(nv, dtype=torch.float64, device=dev)
        xv = torch.empty_like(bv)
        for _ in range(25):
            solver.vcycle(hn, bv, xv)
        src = torch.ones(256 * 2 ** 20 // 8, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"pmc_vcycle": hn, "cycles": 25, "vcycle_bytes": solver.vcycle_bytes(hn),
                          "copy_bytes": 2 * 256 * 2 ** 20}))
        solver.close()
        return
    if args.pmc_probe:
        sysm = fsigen.generate(cfg, seed=args.seeds[0])
        solver = FsiSolver.from_system(sysm, device=0, stream=stream)
        xs = torch.randn(sysm.N, dtype=torch.float64, device=dev)
        ys = torch.empty_like(xs)
        for _ in range(20):
            solver.spmv(xs, ys)
        src = torch.ones(256 * 2 ** 20 // 8, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"pmc_probe": True, "spmv_bytes": solver.spmv_bytes(), "csr_bytes": csr_bytes(sysm),
                          "copy_bytes": 2 * 256 * 2 ** 20}))
        solver.close()
        return
    # one solver per seed of the linearisation state, built and warmed up
    # before the timed region; the timed steps cycle through the seeds
    runs = []
    for sd in args.seeds:
        progress(f"generating {cfg.name} seed {sd}")
        sysm = fsigen.generate(cfg, seed=sd, fe=(sd == args.seeds[0] and not args.no_fe))
        progress(f"N={sysm.N} nnz={sysm.nnz}")
        solver = FsiSolver.from_system(sysm, device=0, stream=stream)
        progress("blocks copied and checked")
        t0 = time.perf_counter()
        solver.build_precond(args.precision, **opts)
        torch.cuda.synchronize()
        setup_ms = (time.perf_counter() - t0) * 1e3
        progress(f"seed {sd}: preconditioner built in {setup_ms:.0f} ms")
        b = torch.from_numpy(sysm.b).to(dev)
        x = torch.zeros_like(b)
        for _ in range(args.warmup):
            x.zero_()
            solver.solve(b, x)
        if args.warmup:  # the instrumented pass's own graphs
            x.zero_()
            solver.solve(b, x, timing=True)
        runs.append({"seed": sd, "sysm": sysm, "solver": solver, "b": b, "x": x, "setup_ms": setup_ms,
                     "N": sysm.N, "nnz": sysm.nnz, "bytes": solver.spmv_bytes(), "csr_bytes": csr_bytes(sysm)})
        sysm.blocks = None  # the host copy of the matrix is no longer needed
    torch.cuda.synchronize()
    sysm = runs[0]["sysm"]
    solver = runs[0]["solver"]
    setup_ms = statistics.mean(r["setup_ms"] for r in runs)
    times, iters, resid = [], [], []
    progress("warm-up done")
    t_all = time.perf_counter()
    for k in range(args.steps):
        r = runs[k % len(runs)]
        r["x"].zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, info = r["solver"].solve(r["b"], r["x"])
        torch.cuda.synchronize()
        times.append((time.perf_counter() - t0) * 1e3)
        iters.append(info.iters)
        resid.append(info.true_rel_resid)
        r["iters"] = info.iters
        if not info.converged:
            raise SystemExit(f"solve did not converge: {info}")
    t_all = (time.perf_counter() - t_all) * 1e3
    ms = statistics.mean(times)
    progress(f"timed: {ms:.3f} ms per solve")

    # The same K solves again with the phases separated by HIP events on the
    # solver's stream (the timed mode splits each step's graph into a
    # preconditioner graph, the A_h product launch and a Gram-Schmidt graph,
    # which costs a few percent per solve, so it stays out of the timed
    # region).  Dominant kernel: the A_h product, every launch of it bracketed.
    t_pre = t_spmv = t_gs = 0.0
    b_pre = b_steps = 0.0
    n_timed = 0
    nbytes_sum = 0.0
    times_instr = []
    for k in range(args.steps):
        r = runs[k % len(runs)]
        nbytes_sum += r["bytes"] * 1.0
        r["x"].zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, info = r["solver"].solve(r["b"], r["x"], timing=True)
        torch.cuda.synchronize()
        times_instr.append((time.perf_counter() - t0) * 1e3)
        if info.iters != r["iters"]:
            raise SystemExit(f"instrumented solve took {info.iters} iterations, timed one {r['iters']}")
        t_pre += info.t_precond_ms
        b_pre += info.bytes_precond
        b_steps += info.bytes_precond / r["solver"].precond_bytes()  # Arnoldi steps launched
        t_spmv += info.t_spmv_ms
        t_gs += info.t_gs_ms
        n_timed += info.n_timed
    spmv_ms = t_spmv / max(n_timed, 1)
    nbytes = nbytes_sum / max(args.steps, 1)  # all seeds share the sparsity pattern
    achieved = nbytes / (spmv_ms * 1e-3) / 1e9

    ceil = stream_ceilings(stream)
    # one V(1,1) cycle of the fluid-velocity hierarchy (largest V-cycle),
    # bytes as executed by the level kernels, and of the solid Schur
    # hierarchy (small, latency-bound levels)
    vc_ms = cycle_ms(solver, "H_A", sysm.dim, stream)
    vc_bytes = solver.vcycle_bytes("H_A")
    vs_ms = cycle_ms(solver, "H_SIG", sysm.dim, stream)
    vs_bytes = solver.vcycle_bytes("H_SIG")
    progress("instrumented solves and V-cycles done")

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
        "dtype": DTYPE[args.precision],
        "data": "synthetic",
        "config": {
            "workload": workload_name(cfg),
            "name": cfg.name, "seeds": list(args.seeds), "N": runs[0]["N"], "nnz": runs[0]["nnz"],
            "tol": 1e-8, "restart": 50, "precond": precond_name(args), "max_coarse": args.max_coarse, "strength": args.strength,
            "paper_vs_own": paper_vs_own(args, opts),
        },
        "iters": {str(r["seed"]): r.get("iters") for r in runs},
        "true_rel_resid": max(resid),
        "ms_min": round(min(times), 3),
        "ms_per_step_instrumented": round(statistics.mean(times_instr), 3),
        "setup_ms": round(setup_ms, 1),
        "timed_wall_ms": round(t_all, 1),
        "phase_ms_per_iter": {"precond": round(t_pre / max(n_timed, 1), 4),
                              "spmv": round(spmv_ms, 4), "gram_schmidt": round(t_gs / max(n_timed, 1), 4)},
        "roofline": {
            "kernel": "csr_segments_kernel (A_h product inside the solve)",
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": MEASURED_TRAFFIC.get(cfg.name),  # the A_h product is FP64 in every precision
            "algorithmic_bytes": int(nbytes),
            "csr_bytes": int(runs[0]["csr_bytes"]),
            "kernel_ms": round(spmv_ms, 5),
            # plain device streams in this run (torch copy and sum of 4 GiB):
            # the practical ceiling next to the 8 TB/s peak
            "stream_ceiling": ceil,
            "frac_of_read_stream": round(achieved / ceil["read_GBps"], 4),
        },
        "precond_phase": {
            # one P^{-1} v per Arnoldi step: bytes as stored (fsi_precond_bytes)
            # over the measured phase time (timed steps; launched-ahead steps
            # that were discarded carry bytes but no time, so bytes are taken
            # per launched step)
            "bytes": int(b_pre / max(b_steps, 1.0)),
            "ms": round(t_pre / max(n_timed, 1), 5),
            "GB/s": round(b_pre / max(b_steps, 1.0) / (t_pre / max(n_timed, 1) * 1e-3) / 1e9, 1),
            "frac": round(b_pre / max(b_steps, 1.0) / (t_pre / max(n_timed, 1) * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        },
        "vcycle_H_A": {
            "bytes": int(vc_bytes), "ms": round(vc_ms, 5),
            "GB/s": round(vc_bytes / (vc_ms * 1e-3) / 1e9, 1),
            "frac": round(vc_bytes / (vc_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "levels": int(len(solver.hierarchy_info("H_A")[0])),
            "traffic": (MEASURED_VCYCLE_TRAFFIC[cfg.name][0]
                        if args.precision == "f64" and cfg.name in MEASURED_VCYCLE_TRAFFIC
                        and int(vc_bytes) == MEASURED_VCYCLE_TRAFFIC[cfg.name][1] else None),
        },
        "vcycle_H_SIG": {
            "bytes": int(vs_bytes), "ms": round(vs_ms, 5),
            "GB/s": round(vs_bytes / (vs_ms * 1e-3) / 1e9, 1),
            "frac": round(vs_bytes / (vs_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "levels": int(len(solver.hierarchy_info("H_SIG")[0])),
        },
    }

    # Other forms of the preconditioner on the same system, timed the same
    # way, each solution compared with the FP64 GPU solve (the oracle is not
    # run at this size): the FP32 preconditioner with and without BF16-stored
    # smoother diagonals and the paper's Section 4.4 fluid step (GMRES on each
    # inverse of the Uzawa-like elimination), from the FP64 build's
    # hierarchies (reuse: only the device copies, smoothers and the fluid
    # solve change); where the headline takes SIMPLEC, the paper's step again
    # with SIMPLE (a build of its own), and the Uzawa-like step with one
    # V-cycle per inverse and SIMPLE (the reading without inner Krylov steps);
    # the headline options with the blocks factorised in the reverse order,
    # and in the order solid, mesh, fluid (one mesh inverse fewer)
    if not args.no_mixed and args.precision == "f64":
        r = runs[0]
        x64 = r["x"].clone()
        alts = {}
        forms = [("f32", "f32", {}, True), ("f32-bf16diag", "f32-bf16diag", {}, True)]
        # the forms that keep the headline's hierarchies come first: a build
        # with another Schur option replaces them
        forms.append(("reverse_block_order", "f64", dict(order="fsm"), True))
        forms.append(("block_order_smf", "f64", dict(order="smf"), True))
        if args.uzawa_inner == 0:
            forms.append(("paper_uzawa_gmres2", "f64", dict(fluid_inner=0, uzawa_inner=2), True))
            if opts["schur"] != "simple":
                forms.append(("paper_uzawa_gmres2_simple", "f64",
                              dict(fluid_inner=0, uzawa_inner=2, schur="simple"), False))
            forms.append(("uzawa_vcycle_simple", "f64", dict(fluid_inner=0, uzawa_inner=0, schur="simple"), True))
        for label, prec, over, reuse in forms:
            o2 = dict(opts)
            o2.update(over)
            t0 = time.perf_counter()
            try:
                r["solver"].build_precond(prec, reuse=reuse, **o2)
            except FsiError as e:  # a refused form is reported; the context keeps its preconditioner
                alts[label] = {"precision": prec, **over, "error": str(e)}
                progress(f"{label}: {alts[label]}")
                continue
            build_ms = (time.perf_counter() - t0) * 1e3
            xm = torch.zeros_like(r["b"])
            timed_solves(r["solver"], r["b"], xm, 1)
            tm, im = timed_solves(r["solver"], r["b"], xm, max(min(args.steps, 3), 1))
            diff = float(torch.linalg.norm(xm - x64) / torch.linalg.norm(x64))
            alts[label] = {"precision": prec, "ms": round(statistics.mean(tm), 3), "iters": im.iters,
                           "true_rel_resid": im.true_rel_resid, "rel_diff_vs_f64_gpu": diff,
                           "speedup_vs_headline": round(ms / statistics.mean(tm), 3), **over,
                           "build_ms": round(build_ms, 1), "hierarchies": "reused" if reuse else "built"}
            progress(f"{label}: {alts[label]}")
        alts["note"] = ("seed %d; hierarchies reused from the previous build where marked; FP64 Krylov, A_h "
                        "products, true residual and coarsest solves in every form; difference measured against "
                        "the FP64 GPU solve (oracle not run at this size)" % r["seed"])
        line["alternatives"] = alts

    if not args.no_fe and args.precision == "f64":
        progress("finite-element assembly and quasi-Newton loop")
        line["fe_newton"] = fe_newton_run(runs[0], opts)
        progress(f"fe_newton: {line['fe_newton']}")

    for r in runs:
        r["solver"].close()
    runs.clear()
    if args.time_steps > 0 and args.precision == "f64":
        progress("one-step-theta time steps")
        line["theta_steps"] = theta_steps_run(args, cfg.dim, stream)
        progress(f"theta_steps: {line['theta_steps']}")
    if not args.no_cpu_baseline:
        gpu_c3 = None
        if cfg.name != "c3":
            # the configuration the oracle is timed on, on the GPU too
            progress("c3 on the GPU (the oracle's sample configuration)")
            c3 = fsigen.config("c3")
            s3 = fsigen.generate(c3, seed=0)
            sol3 = FsiSolver.from_system(s3, device=0, stream=stream)
            sol3.build_precond(args.precision, **precond_opts(args, c3.dim))
            b3 = torch.from_numpy(s3.b).to(dev)
            x3 = torch.zeros_like(b3)
            timed_solves(sol3, b3, x3, 1)
            t3, i3 = timed_solves(sol3, b3, x3, 3)
            gpu_c3 = {"ms": round(statistics.mean(t3), 3), "iters": i3.iters, "N": s3.N, "nnz": s3.nnz}
            sol3.close()
            del s3
            line["gpu_c3"] = gpu_c3
        else:
            gpu_c3 = {"iters": iters[0]}
        progress("timing the CPU oracle sample (c3)")
        line["cpu_baseline"] = cpu_baseline(args, gpu_c3)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
