#!/usr/bin/env python3
"""Throughput of the CDG Poisson solve on one MI355X.

One step = one solve A u = M_0 f from u = 0 to a true FP64 relative residual
<= 1e-10 with FCG(1) preconditioned by the FP32 V(2,2) block-Jacobi cycle on
the agglomerated hierarchy (inputs resident in HBM, setup excluded).  The
same solve with an FP64 V-cycle, the GPU rebuild of all level operators for
a new kappa, the adjoint solve + dL/dkappa, per-kernel HIP-event timings with
the level-0 smoother's roofline, and the CPU oracle on a bounded sample are
reported alongside.  Prints one JSON line on stdout; progress goes to stderr.
"""
import argparse
import hashlib
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_2012_08024_amd.bytemodel import (facet_nodes, iteration_bytes,  # noqa: E402
                                            smoother_bytes, spmv_bytes)

METRIC = "DOFs/s to 1e-10 rel residual: FP32-MG-in-FP64-FCG vs FP64-MG; % HBM peak"
HBM_PEAK_GBS = 8000.0


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def kernels_hash():
    h = hashlib.sha256()
    for name in ("kernels.inl", "kernels.hpp"):
        with open(os.path.join(ROOT, "paper_2012_08024_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def cpu_model():
    """The host CPU as /proc/cpuinfo names it, with family, model, stepping,
    clock and cache of the first processor (a virtualised host may report
    only a short model name)."""
    info = {}
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if not line.strip():
                    break
                k, _, v = line.partition(":")
                info[k.strip()] = v.strip()
    except OSError:
        return platform.processor()
    extra = ", ".join("%s %s" % (k, info[k]) for k in ("cpu family", "model", "stepping", "cpu MHz", "cache size")
                      if k in info)
    return "%s (%s)" % (info.get("model name", platform.processor()), extra) if extra else info.get("model name", "")


def cpu_baseline(cfg, n_sample):
    """The FP64 oracle (same generator, smaller n; same p, levels, cycle and
    outer solver) timed around the solve only, on one thread.  Returns the
    record and (mesh, oracle solution) for the GPU comparison."""
    from threadpoolctl import threadpool_info, threadpool_limits

    from oracle.agglomerate import build_hierarchy
    from oracle.cdg import CDG
    from oracle.krylov import fcg
    from oracle.multigrid import Hierarchy
    from workloads import config_mesh, source_sine

    with threadpool_limits(1):
        m, kappa = config_mesh(cfg, n=n_sample)
        t0 = time.perf_counter()
        cdg = CDG(m.coords, m.e2v, m.face_bc, cfg["p"])
        par = build_hierarchy(m.e2v, cdg.topo.neighbor_pairs(), cfg["levels"] or 50, cfg["agg_seed"],
                              coarse_dofs=cfg.get("coarse_dofs") or None, n_p=cdg.np)
        H = Hierarchy(cdg, par, kappa=kappa, coarsening="primal")
        t_setup = time.perf_counter() - t0
        b = cdg.M0() @ source_sine(cdg.nodes_phys().reshape(-1, cfg["dim"]))
        t0 = time.perf_counter()
        x, it, res = fcg(H.A[0], b, H.vcycle, tol=cfg["tol"])
        t_solve = time.perf_counter() - t0
        pools = [{k: d.get(k) for k in ("internal_api", "num_threads")} for d in threadpool_info()]
    dofs = cdg.N * cdg.np
    rec = {
        "value": dofs / t_solve, "unit": "DOFs/s", "cores": 1, "kind": "oracle",
        "sample": "same generator at n=%d (%d elements, %d DOFs), p=%d, %d levels, FP64 V(2,2) "
                  "block Jacobi in FCG(1) to %.0e; solve only, setup %.1f s excluded"
                  % (n_sample, cdg.N, dofs, cfg["p"], len(H.sizes), cfg["tol"], t_setup),
        "iterations": it, "solve_s": t_solve, "cpu": cpu_model(), "host_cpu_count": os.cpu_count(),
        "threads": "1 process, 1 thread: threadpool_limits(1) on the BLAS pools %s; SciPy sparse products "
                   "are single-threaded" % pools,
    }
    return rec, m, x


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", default="c2")
    ap.add_argument("--cpu-sample-n", type=int, default=112)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--kernel-variant", type=int, default=0,
                    help="V-cycle kernel family (see cdgmg_options.kernel_variant); 0 = auto")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run one plain 1 GiB device copy (calibrates HBM byte counters)")
    ap.add_argument("--outer", choices=["fcg", "pcg", "gmres"], default="fcg",
                    help="outer Krylov solver (the metric is quoted with fcg)")
    ap.add_argument("--restart", type=int, default=50, help="GMRES restart length")
    ap.add_argument("--p-coarse", type=int, default=0, help="1: hp front end (p-multigrid to p = 1 first)")
    ap.add_argument("--p-jump", type=int, default=0, help="with --p-coarse 1: 1 goes from p straight to p = 1")
    ap.add_argument("--coarse-fp64", type=int, default=0,
                    help="1: the FP32 V-cycle keeps its coarsest solve in FP64")
    ap.add_argument("--coarsening", choices=["primal", "flux"], default="primal",
                    help="coarse operators: Galerkin L^T A L (primal, Sec. 3.5) or the flux form (Sec. 4.1)")
    ap.add_argument("--study", choices=["coarsening", "coarsening-paper", "switch", "switch-paper", "convection",
                                        "size"],
                    help="instead of the benchmark: primal vs flux coarsening over mesh size and gamma, "
                         "consistent vs natural switch (workload or the paper's solver settings), or "
                         "convection-diffusion under refinement; prints one JSON line with the table")
    ap.add_argument("--sizes", default="",
                    help="with --study size: comma-separated mesh sizes n (default 100 ... 894)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: the solver runs on one GPU only (multi-GPU domain decomposition is "
              "designed, not implemented)", file=sys.stderr)
        sys.exit(2)
    if args.study:
        import torch

        from paper_2012_08024_amd import studies
        torch.cuda.set_device(0)
        kind, _, setting = args.study.partition("-")
        if kind == "convection":
            rows = studies.study_convection(log=log)
        elif kind == "size":
            kw = {"ns": tuple(int(v) for v in args.sizes.split(","))} if args.sizes else {}
            rows = studies.study_size(log=log, **kw)
        else:
            fn = studies.study_coarsening if kind == "coarsening" else studies.study_switch
            rows = fn(setting=setting or "workload", log=log)
        print(json.dumps({"study": args.study, "data": "synthetic", "rows": rows}), flush=True)
        return

    import numpy as np
    import torch

    import paper_2012_08024_amd as cm
    from workloads import CONFIGS, config_mesh, source_sine

    cfg = CONFIGS[args.config]
    torch.cuda.set_device(0)
    log("config %s: building mesh" % args.config)
    mesh, kappa = config_mesh(cfg)
    parents, sizes = cm.agglomerate(mesh, cfg["levels"] or 50, cfg["agg_seed"], p=cfg["p"],
                                    coarse_dofs=cfg.get("coarse_dofs", 0))
    log("levels %s" % list(sizes))
    kappa_t = torch.tensor(kappa, dtype=torch.float64, device="cuda")

    t0 = time.perf_counter()
    outer = {"fcg": cm.OUTER_FCG, "pcg": cm.OUTER_PCG, "gmres": cm.OUTER_GMRES}[args.outer]
    outer_name = {"fcg": "FCG(1)", "pcg": "PCG", "gmres": "GMRES(%d)" % args.restart}[args.outer]
    hp_desc = ""
    if args.p_coarse == 1 and cfg["p"] >= 2:
        hp_desc = "p-multigrid over degrees %s, then " % (
            "%d, 1" % cfg["p"] if args.p_jump else ", ".join(str(q) for q in range(cfg["p"], 0, -1)))
    coarsening = cm.COARSEN_FLUX if args.coarsening == "flux" else cm.COARSEN_PRIMAL
    s32 = cm.Solver(mesh, cfg["p"], kappa_t, parents, sizes, mg_precision=cm.MG_FP32, tol=cfg["tol"],
                    outer=outer, restart=args.restart, p_coarse=args.p_coarse, p_jump=args.p_jump,
                    kernel_variant=args.kernel_variant, coarsening=coarsening, coarse_fp64=args.coarse_fp64)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    npb = s32.np
    dofs = mesh.n_elem * npb
    ne, nnzb = s32.level_info()
    f = torch.tensor(source_sine(s32.node_coords().reshape(-1, mesh.dim)), device="cuda")
    log("setup %.1f s, %d DOFs, nnzb %s" % (setup_s, dofs, list(nnzb)))

    # GPU rebuild of the operators (kappa assembly, Galerkin coarsening, block inverses, coarsest inverse)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s32.update_kappa(kappa_t)
    torch.cuda.synchronize()
    rebuild_ms = (time.perf_counter() - t0) * 1e3

    u32, hinfo = s32.solve(f, history=True)
    log("FP32-MG residual history: " + " ".join("%.1e" % v for v in hinfo.history[::10]))
    for _ in range(args.warmup):
        u32, info = s32.solve(f)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        u32, info = s32.solve(f)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_per_step = elapsed * 1e3 / args.steps
    value = dofs * args.steps / elapsed
    log("FP32-MG: %.2f ms/solve, %d iterations, rel res %.2e, %.3g DOFs/s"
        % (ms_per_step, info.iterations, info.rel_residual, value))

    # the same timed loop with HIP events around every kernel launch
    s32.set_profile(True)
    kms = {k: 0.0 for k in cm.K_NAMES}
    kcnt = {k: 0 for k in cm.K_NAMES}
    for _ in range(args.steps):
        _, pinfo = s32.solve(f)
        for k in cm.K_NAMES:
            kms[k] += pinfo.kernel_ms[k]
            kcnt[k] += pinfo.kernel_launches[k]
    s32.set_profile(False)
    avg_smooth_ms = kms["smooth0"] / max(kcnt["smooth0"], 1)
    avg_spmv_ms = kms["spmv"] / max(kcnt["spmv"], 1)
    nfn, nf = facet_nodes(mesh.dim, npb), mesh.dim + 1
    sb = smoother_bytes(int(nnzb[0]), mesh.n_elem, npb, 4, nfn, nf)
    achieved = sb / (avg_smooth_ms * 1e-3) / 1e9
    spb = spmv_bytes(int(nnzb[0]), mesh.n_elem, npb, nfn, nf)
    spmv_gbs = spb / (avg_spmv_ms * 1e-3) / 1e9
    itb = iteration_bytes(sizes, nnzb, npb, nfn, nf) if len(nnzb) == len(sizes) else None
    traffic = None
    tpath = os.path.join(ROOT, "profiles", "traffic_%s.json" % args.config)
    if os.path.exists(tpath):
        with open(tpath) as fh:
            tj = json.load(fh)
        ent = tj.get("k_smooth_level0")
        if ent and ent.get("kernels_hash") == kernels_hash():
            traffic = ent["hbm_bytes_per_launch"]

    # adjoint: lambda = A^{-1} M_0 u, then dL/dkappa
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g = s32.apply_mass(u32)
    lam, ainfo = s32.solve_transpose(g)
    gk = s32.grad_kappa(u32, lam)
    torch.cuda.synchronize()
    adjoint_ms = (time.perf_counter() - t0) * 1e3

    out64 = None
    err_vs_64 = None
    if not args.no_fp64:
        s32_bytes = s32.device_bytes()
        s64 = cm.Solver(mesh, cfg["p"], kappa_t, parents, sizes, mg_precision=cm.MG_FP64, tol=cfg["tol"],
                        outer=outer, restart=args.restart, p_coarse=args.p_coarse, p_jump=args.p_jump,
                        kernel_variant=args.kernel_variant, coarsening=coarsening)
        for _ in range(max(1, args.warmup)):
            u64, info64 = s64.solve(f)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            u64, info64 = s64.solve(f)
        torch.cuda.synchronize()
        el64 = time.perf_counter() - t0
        err_vs_64 = float(torch.linalg.norm(u32 - u64) / torch.linalg.norm(u64))
        out64 = {"value": dofs * args.steps / el64, "ms_per_step": el64 * 1e3 / args.steps,
                 "iterations": info64.iterations, "rel_residual": info64.rel_residual,
                 "conv_factor": info64.conv_factor}
        log("FP64-MG: %.2f ms/solve, %d iterations" % (out64["ms_per_step"], info64.iterations))
        s64.close()
    else:
        s32_bytes = s32.device_bytes()

    cpu = None
    if not args.no_cpu_baseline:
        log("CPU oracle sample n=%d" % args.cpu_sample_n)
        cpu, m_s, x_s = cpu_baseline(cfg, args.cpu_sample_n)
        log("CPU oracle: %.3g DOFs/s (%d iterations)" % (cpu["value"], cpu["iterations"]))
        # the same sample solved by the GPU path (FP32 V-cycle, same options)
        ps, ss = cm.agglomerate(m_s, cfg["levels"] or 50, cfg["agg_seed"], p=cfg["p"],
                                coarse_dofs=cfg.get("coarse_dofs", 0))
        _, ks = config_mesh(cfg, n=args.cpu_sample_n)
        sg = cm.Solver(m_s, cfg["p"], ks, ps, ss, mg_precision=cm.MG_FP32, tol=cfg["tol"], outer=outer,
                       restart=args.restart, p_coarse=args.p_coarse, p_jump=args.p_jump)
        ug, ig = sg.solve(source_sine(sg.node_coords().reshape(-1, mesh.dim)))
        sg.close()
        ug = ug.cpu().numpy()
        cpu["gpu_iterations_on_sample"] = ig.iterations
        cpu["error_vs_oracle"] = float(np.linalg.norm(ug - x_s) / np.linalg.norm(x_s))
        cpu["error_vs_oracle_max"] = float(np.abs(ug - x_s).max() / np.abs(x_s).max())
        log("GPU on the sample: %d iterations, relative difference to the oracle %.2e"
            % (ig.iterations, cpu["error_vs_oracle"]))

    result = {
        "metric": METRIC,
        "value": value,
        "unit": "DOFs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "dtype_detail": "V-cycle in f32; outer FCG (operator product, vectors, dots, true residual) in f64",
        "data": "synthetic",
        "config": {
            "p_levels": s32.p_levels,
            "workload": "%s: %dD %s mesh n=%d, %d elements, CDG p=%d, %d DOFs, kappa=%s, %s%d-level "
                        "greedy agglomeration (seed %d), V(%d,%d) damped block Jacobi omega=%.1f, "
                        "%s coarse operators, %s, tol %.0e"
                        % (args.config, cfg["dim"],
                           "uniform right-triangle square (Neumann x=0,1)" if cfg.get("mesh") == "square51"
                           else "jittered Delaunay" if cfg["dim"] == 2 else "jittered Kuhn-tet", cfg["n"],
                           mesh.n_elem, cfg["p"], dofs, cfg["kappa"], hp_desc, len(sizes), cfg["agg_seed"], 2, 2,
                           0.7, "Galerkin (primal)" if args.coarsening == "primal" else "flux-form (Sec. 4.1)",
                           outer_name, cfg["tol"]),
            "coarsening": args.coarsening, "coarse_fp64": args.coarse_fp64,
            "elements": int(mesh.n_elem), "dofs": int(dofs), "p": cfg["p"], "levels": [int(x) for x in sizes],
            "nnzb": [int(x) for x in nnzb],
            "operator_complexity": float(sum(nnzb) / nnzb[0]),
            "parallelism": "single GPU",
        },
        "iterations": info.iterations,
        "residual_history_every_10": [float(v) for v in hinfo.history[::10]],
        "rel_residual": info.rel_residual,
        "conv_factor": info.conv_factor,
        "error_vs_fp64_mg": err_vs_64,
        "fp64_mg": out64,
        "speedup_fp32_mg_vs_fp64_mg": (value / out64["value"]) if out64 else None,
        "setup_s_total": setup_s,
        "operator_rebuild_ms_gpu": rebuild_ms,
        "adjoint_ms": adjoint_ms,
        "adjoint_iterations": ainfo.iterations,
        "device_bytes": s32_bytes,
        "kernel_ms_per_solve": {k: kms[k] / args.steps for k in cm.K_NAMES if kcnt[k]},
        "kernel_launches_per_solve": {k: kcnt[k] / args.steps for k in cm.K_NAMES if kcnt[k]},
        "roofline": {
            "kernel": "level-0 damped block-Jacobi sweep on the facet-trace form (k_sweep0<float,%d,H,%d>, FP32)"
                      % (npb, nf),
            "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
            "algorithmic_bytes_per_launch": sb, "avg_launch_ms": avg_smooth_ms,
        },
        "outer_spmv_roofline": {"kernel": "outer q = A_0 p on the facet-trace form, with dots (k_spmv0<%d,H,%d>, FP64)"
                                          % (npb, nf), "achieved": spmv_gbs,
                                "frac": spmv_gbs / HBM_PEAK_GBS, "algorithmic_bytes_per_launch": spb,
                                "avg_launch_ms": avg_spmv_ms},
        "algorithmic_bytes_per_iteration": itb,
        "achieved_gbs_per_iteration": (itb["total"] / (ms_per_step * 1e-3 / max(info.iterations, 1)) / 1e9
                                       if itb else None),
        "cpu_baseline": cpu,
    }
    s32.close()
    if args.copy_probe:
        # a plain 1 GiB device copy: calibrates the HBM counters and gives the
        # copy bandwidth this device reaches (read + write bytes per second)
        src = torch.empty(1 << 28, dtype=torch.float32, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(10):
            dst.copy_(src)
        e1.record()
        torch.cuda.synchronize()
        nbytes = int(src.numel() * 4)
        result["copy_probe_bytes"] = nbytes
        result["copy_probe_gbs"] = 2 * nbytes * 10 / (e0.elapsed_time(e1) * 1e-3) / 1e9
        # read-only stream of the same 1 GiB (torch's sum)
        acc = torch.zeros((), dtype=torch.float32, device="cuda")
        torch.sum(src, dim=0, out=acc)
        e0.record()
        for _ in range(10):
            torch.sum(src, dim=0, out=acc)
        e1.record()
        torch.cuda.synchronize()
        result["read_probe_gbs"] = nbytes * 10 / (e0.elapsed_time(e1) * 1e-3) / 1e9
        # the last dispatch before the counters are read is the 1 GiB copy
        dst.copy_(src)
        torch.cuda.synchronize()
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
