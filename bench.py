#!/usr/bin/env python3
"""Throughput of the EB viscoplastic RK2 step on one MI355X.

Workload: the 128^3 translating-sphere configuration (sphere r = 0.125 at the centre, walls
moving at (0,0,-1), eta = 1 + 10/(|gamma|+1e-6), rho = 4e-3, dt = 5e-4), uniform start.  W warm-up
steps advance the flow, then K steps are timed with the state resident in HBM; every step runs
the whole path (derived quantities with the MAC projection, the implicit viscous multigrid solve
and the end-of-stage projection, twice).  MLUPS = n^3 * K / t / 1e6.

Also reported: the roofline of the dominant kernel (the finest-level red-black smoother of the
viscous multigrid), timed live with HIP events on the stream it runs on, and the FP64 oracle
timed on the host cores on a bounded sample.  Prints one JSON line.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MLUPS per RK2 step (viscous MG + MAC projection) at 128^3 EB; adjoint/fwd ratio"
HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--precision", choices=["fp64", "mixed"], default="fp64")
    ap.add_argument("--n", type=int, default=128, help="cells per direction (default 128)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--kernel-only", action="store_true",
                    help="only the smoother timing loop (for the profiler)")
    ap.add_argument("--sweeps", type=int, default=40)
    ap.add_argument("--nu", type=int, default=2, help="smoothing pairs before and after")
    ap.add_argument("--nbottom", type=int, default=16)
    ap.add_argument("--adjoint-steps", type=int, default=20,
                    help="steps of the adjoint/forward ratio run (0 skips it)")
    ap.add_argument("--ckpt-every", type=int, default=5)
    return ap.parse_args()


def smoother_bytes_per_launch(N, ncomp, w):
    """Algorithmic bytes of one red-black half sweep (one launch, one colour: N/2 updated cells).

    Per updated cell a Gauss-Seidel sweep must move the iterate once in and once out
    (2 ncomp w), the right-hand side (ncomp w), the cell viscosity the face coefficients are
    formed from (w) and the cell-type flag (1 byte): 10 w + 1 bytes for three components
    (81 in FP64, 41 in FP32)."""
    return (N // 2) * (3 * ncomp * w + w + 1)


def time_smoother(api, ctx, precision, sweeps, torch):
    """Average duration (ms) of the finest-level viscous smoother, measured with HIP events on
    the stream the kernel is launched on (torch's current stream)."""
    f32 = precision == api.EB_MIXED
    dt = torch.float32 if f32 else torch.float64
    b = torch.randn((3,) + ctx.shape, dtype=dt, device=ctx.device)
    x = torch.zeros((3,) + ctx.shape, dtype=dt, device=ctx.device)
    for c in range(4):
        api.eb_mg_sweep(ctx, api.EB_SYS_VISC, c & 1, b, x, precision)
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for c in range(sweeps):
        api.eb_mg_sweep(ctx, api.EB_SYS_VISC, c & 1, b, x, precision)
    e1.record(stream)
    e1.synchronize()
    return e0.elapsed_time(e1) / sweeps


def adjoint_ratio(api, AG, ctx, w, opts, nsteps, every, torch, I):
    """Adjoint run: the 128^3 sphere with tau0_c = Bi theta_c (theta = 1 + 0.05 U(-1,1), seed 1,
    Bi = 10), u starting at the wall velocity, nsteps steps with checkpoints every `every`;
    loss = z-force on the sphere.  Returns wall times of the forward (nsteps steps + drag) and of
    the backward (segment recomputation with tapes + step adjoints + drag adjoint)."""
    import copy

    o = copy.copy(opts)
    o.precision = api.EB_FP64
    rheo = api.make_rheology(w.law, w.mu, w.tau0, w.eps, w.rho)
    dev = ctx.device
    u0 = torch.from_numpy(I.initial_velocity(w)).to(dev)
    p0 = torch.zeros(ctx.shape, dtype=torch.float64, device=dev)
    theta = torch.from_numpy(I.yield_field(w, seed=1)).to(dev).requires_grad_(True)
    bi = torch.tensor(float(w.tau0), dtype=torch.float64, device=dev, requires_grad=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    u, p = AG.rollout(ctx, rheo, w.dt, o, u0, p0, theta, bi, nsteps, ckpt_every=every)
    fz = AG.drag(ctx, rheo, u, p, theta, bi)[2]
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    fz.backward()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    return {"steps": nsteps, "ckpt_every": every, "fwd_s": round(t1 - t0, 4),
            "bwd_s": round(t2 - t1, 4), "ratio": round((t2 - t1) / (t1 - t0), 3),
            "Fz": fz.item(), "dFz_dBi": bi.grad.item(),
            "dFz_dtheta_maxabs": theta.grad.abs().max().item()}


def cpu_baseline(w, u0, p0, n_steps=1):
    """The FP64 oracle (as it stands) on the host cores: one RK2 step of the same workload from
    the same state.  Returns MLUPS and the thread count it used."""
    import numpy as np  # noqa: F401

    from oracle import oracle as O

    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or len(os.sched_getaffinity(0))
    os.environ["OMP_NUM_THREADS"] = str(threads)
    og = O.Geometry(w)
    opts = O.make_opts(w)
    rh = O.make_rheo(w)
    t0 = time.perf_counter()
    u, p = u0, p0
    for _ in range(n_steps):
        u, p, st = og.rk2_step(u, p, rh, w.dt, opts)
    t = time.perf_counter() - t0
    return w.ncell * n_steps / t / 1e6, threads, t


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: this build runs on one GPU only; the step is a single box per GPU "
              "and the multi-GPU domain decomposition is not built (see DESIGN.md).",
              file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import eb_inputs as I
    import paper_1905_07392_amd as pkg
    from paper_1905_07392_amd import api

    w = I.sphere128()
    if args.n != 128:
        w = w.replace(n=(args.n,) * 3, h=1.0 / args.n, name=f"sphere{args.n}")
    prec = api.EB_MIXED if args.precision == "mixed" else api.EB_FP64
    box, body, rheo, opts = pkg.from_workload(w, precision=prec)
    opts.nu1 = opts.nu2 = args.nu
    opts.nbottom = args.nbottom
    dev = torch.device("cuda:0")
    ctx = api.eb_geometry_build(box, body, dev)
    u = torch.from_numpy(I.initial_velocity(w)).to(dev)
    p = torch.zeros(ctx.shape, dtype=torch.float64, device=dev)

    if args.kernel_only:
        # build the viscous operator of the start state, then only the smoother loop
        eta, eta_eb = api.eb_apparent_viscosity(ctx, rheo, u)
        r = torch.zeros_like(u)
        api.eb_mg_vcycle(ctx, api.EB_SYS_VISC, r, opts, precision=prec, rho=w.rho, dt=w.dt,
                         eta=eta, eta_eb=eta_eb)
        ms = time_smoother(api, ctx, prec, args.sweeps, torch)
        print(json.dumps({"kernel": "k_smooth_rb<3> finest level", "avg_ms": ms}))
        return

    print(f"[bench] {w.name} n={w.n} precision={args.precision} warmup={args.warmup} "
          f"steps={args.steps}", file=sys.stderr, flush=True)
    stats = []
    for s in range(args.warmup):
        u, p, st = api.eb_rk2_step(ctx, rheo, w.dt, opts, u, p, inplace=True)
        print(f"[bench] warmup step {s}: {st}", file=sys.stderr, flush=True)
    u0_host = u.cpu().numpy().copy()
    p0_host = p.cpu().numpy().copy()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(args.steps):
        u, p, st = api.eb_rk2_step(ctx, rheo, w.dt, opts, u, p, inplace=True)
        stats.append(st)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    ms_step = 1e3 * t / args.steps
    mlups = w.ncell * args.steps / t / 1e6
    print(f"[bench] timed {args.steps} steps: {ms_step:.2f} ms/step, {mlups:.1f} MLUPS; "
          f"last stats {stats[-1]}", file=sys.stderr, flush=True)

    # roofline of the dominant kernel: the finest-level viscous smoother, with the viscous
    # operator of the final state (one V-cycle builds it)
    eta, eta_eb = api.eb_apparent_viscosity(ctx, rheo, u)
    api.eb_mg_vcycle(ctx, api.EB_SYS_VISC, torch.zeros_like(u), opts, precision=prec, rho=w.rho,
                     dt=w.dt, eta=eta, eta_eb=eta_eb)
    ms_k = time_smoother(api, ctx, prec, args.sweeps, torch)
    wbytes = 4 if prec == api.EB_MIXED else 8
    algo = smoother_bytes_per_launch(ctx.N, 3, wbytes)
    achieved = algo / (ms_k * 1e-3) / 1e9
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                "kernel": "k_smooth_rb (finest level, 3 components, one colour)",
                "kernel_ms": round(ms_k, 5), "bytes_per_launch": int(algo)}

    out = {"metric": METRIC, "value": round(mlups, 3), "unit": "MLUPS", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 3),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f64" if prec == api.EB_FP64 else "f64+f32-mg",
           "data": "synthetic",
           "config": {"workload": f"{w.name}: {w.n[0]}^3 box, EB sphere r=0.125, walls (0,0,-1),"
                                  f" eta=1+10/(|g|+1e-6), rho=4e-3, dt=5e-4, rtol=1e-12",
                      "cells": w.ncell, "precision": args.precision,
                      "iterations_last_step": {k: stats[-1][k] for k in
                                               ("it_mac", "it_visc", "it_proj", "vcycles")}},
           "roofline": roofline}
    if args.adjoint_steps > 0:
        from paper_1905_07392_amd import autograd as AG

        adj = adjoint_ratio(api, AG, ctx, w, opts, args.adjoint_steps, args.ckpt_every, torch, I)
        out["adjoint"] = adj
        print(f"[bench] adjoint: {adj}", file=sys.stderr, flush=True)
    if not args.no_cpu_baseline:
        val, cores, tcpu = cpu_baseline(w, u0_host, p0_host)
        out["cpu_baseline"] = {"value": round(val, 4), "unit": "MLUPS", "cores": cores,
                               "kind": "oracle",
                               "sample": f"one FP64 RK2 step of the same {w.n[0]}^3 workload "
                                         f"from the same state ({tcpu:.1f} s)"}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
