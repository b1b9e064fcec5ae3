#!/usr/bin/env python3
"""Throughput of the EB viscoplastic RK2 step on one MI355X.

Workload: the 128^3 translating-sphere configuration (sphere r = 0.125 at the centre, walls
moving at (0,0,-1), eta = 1 + 10/(|gamma|+1e-6), rho = 4e-3, dt = 5e-4), uniform start.  W warm-up
steps advance the flow, then K steps are timed with the state resident in HBM; every step runs
the whole path (derived quantities with the MAC projection, the implicit viscous multigrid solve
and the end-of-stage projection, twice).  MLUPS = n^3 * K / t / 1e6.

Also reported: the same steps in the other precision (mixed: FP32 multigrid inside the FP64
Krylov iteration) from the same start state, with its difference from the FP64 run; the roofline
of the dominant kernel (the finest-level red-black smoother of the viscous multigrid), timed live
with HIP events on the stream it runs on, and of the whole step from the bytes of the passes it
executed; and the FP64 oracle timed on the host cores on a bounded sample (all threads, and one
thread on the 64^3 version).  Prints one JSON line.
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
    ap.add_argument("--no-single-thread", action="store_true",
                    help="skip the single-thread oracle figure of the CPU baseline")
    ap.add_argument("--single-precision", action="store_true",
                    help="time only the --precision run (default: also the other precision)")
    ap.add_argument("--kernel-only", action="store_true",
                    help="only the smoother timing loop (for the profiler)")
    ap.add_argument("--sweeps", type=int, default=100,
                    help="back-to-back smoother launches timed for the roofline")
    ap.add_argument("--nu", type=int, default=2, help="smoothing pairs before and after")
    ap.add_argument("--nbottom", type=int, default=16)
    ap.add_argument("--adjoint-steps", type=int, default=20,
                    help="steps of the adjoint/forward ratio run (0 skips it)")
    ap.add_argument("--ckpt-every", type=int, default=5)
    ap.add_argument("--adjoint-fd", type=int, default=0,
                    help="also check the adjoint against central finite differences in Bi and "
                         "in this many seeded cells next to the body")
    ap.add_argument("--adjoint-fd-steps", type=int, default=20,
                    help="horizon of the finite-difference check (steps of the same run)")
    return ap.parse_args()


def smoother_bytes_per_launch(N, ncomp, w):
    """Algorithmic bytes of one red-black half sweep (one launch, one colour: N/2 updated cells).

    Per updated cell a Gauss-Seidel sweep must move the iterate once in and once out
    (2 ncomp w), the right-hand side (ncomp w), the cell viscosity the face coefficients are
    formed from (w) and the cell-type flag (1 byte): 10 w + 1 bytes for three components
    (81 in FP64, 41 in FP32)."""
    return (N // 2) * (3 * ncomp * w + w + 1)


# the finest-level viscous smoother per precision: FP64 updates two cells per thread with 16-byte
# pair loads, FP32 four cells per thread with 16-byte quad loads
SMOOTHER_KERNEL = {"fp64": "k_smooth_rb_pair", "mixed": "k_smooth_rb_quad"}


def counted_traffic(tag):
    """HBM bytes per launch of the finest-level smoother from the committed byte-counter summary
    (profiles/), or None when there is none for this precision or the kernel source has changed
    since the counters were taken."""
    import hashlib

    kernel = SMOOTHER_KERNEL[tag]
    path = os.path.join(ROOT, "profiles", f"{kernel}_sphere128_{tag}_counters.md")
    if not os.path.exists(path):
        return None
    fields = {}
    for line in open(path):
        if ":" in line and not line.startswith(("#", "|", " ", "`")):
            key, _, val = line.partition(":")
            fields[key.strip()] = val.strip()
    csrc = os.path.join(ROOT, "paper_1905_07392_amd", "csrc")
    src = b"".join(open(os.path.join(csrc, f), "rb").read()
                   for f in ("eb_mg.hip", "eb_internal.hpp"))
    if fields.get("source_sha256") != hashlib.sha256(src).hexdigest():
        return None
    val = fields.get(f"traffic_bytes_per_launch_{tag}")
    return int(val) if val else None


def time_smoother(api, ctx, precision, sweeps, torch):
    """Average duration (ms) of the finest-level viscous smoother, measured with HIP events on
    the stream the kernel is launched on (torch's current stream).  A GPU spin is enqueued first
    so that the host has queued every sweep before the first one starts: the sweeps then run
    back to back and the figure is the kernels' time, not the host's launch rate (launched one
    by one from Python, the host falls behind a 20 us kernel)."""
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
    torch.cuda._sleep(50_000_000)  # tens of ms of GPU time, far more than queueing the sweeps
    e0.record(stream)
    for c in range(sweeps):
        api.eb_mg_sweep(ctx, api.EB_SYS_VISC, c & 1, b, x, precision)
    e1.record(stream)
    e1.synchronize()
    return e0.elapsed_time(e1) / sweeps


def copy_bandwidth(ctx, torch, reps=20):
    """Bandwidth (GB/s, read + write) of a plain device copy of a 3 x n^3 float64 field, timed
    with HIP events on torch's current stream: the practical ceiling the smoother's figure is also
    set against."""
    src = torch.randn((3,) + ctx.shape, dtype=torch.float64, device=ctx.device)
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(reps):
        dst.copy_(src)
    e1.record(stream)
    e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    return 2 * src.numel() * 8 / (ms * 1e-3) / 1e9


def adjoint_ratio(api, AG, ctx, w, opts, nsteps, every, torch, I, fd_cells=0, fd_steps=5):
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
    out = {"steps": nsteps, "ckpt_every": every, "fwd_s": round(t1 - t0, 4),
           "bwd_s": round(t2 - t1, 4), "ratio": round((t2 - t1) / (t1 - t0), 3),
           "Fz": fz.item(), "dFz_dBi": bi.grad.item(),
           "dFz_dtheta_maxabs": theta.grad.abs().max().item()}
    if fd_cells > 0:
        # the gradient checked is that of the run with the finite differences' tolerance
        o2 = copy.copy(o)
        o2.rtol_visc = o2.rtol_mac = o2.rtol_proj = FD_RTOL
        th2 = theta.detach().clone().requires_grad_(True)
        bi2 = torch.tensor(float(w.tau0), dtype=torch.float64, device=dev, requires_grad=True)
        u, p = AG.rollout(ctx, rheo, w.dt, o2, u0, p0, th2, bi2, fd_steps, ckpt_every=every)
        AG.drag(ctx, rheo, u, p, th2, bi2)[2].backward()
        out["fd"] = adjoint_fd(api, ctx, w, o, rheo, u0, p0, theta.detach(), bi2.grad.item(),
                               th2.grad.detach(), fd_steps, fd_cells, torch, I)
    return out


FD_RTOL = 1e-13   # solves of the differentiated and the finite-difference runs (1e-14 is not
                  # reliably attainable: a stagnating solve changes its stopping iteration)
FD_BI_STEP = 1e-6  # relative step in Bi
FD_CELL_STEP = 1e-3  # relative step in one cell's yield-stress multiplier


def adjoint_fd(api, ctx, w, o, rheo, u0, p0, theta, g_bi, g_theta, nsteps, ncells, torch, I):
    """Central differences of the same loss in Bi and in the yield-stress multiplier of `ncells`
    fluid cells within 3h of the body (drawn with seed 2), against the adjoint.

    The step is smooth only piecewise (upwind sides and limiter branches switch), and the
    adjoint is the derivative on the piece the forward run is on.  So each difference is taken
    twice: plainly, counting the switches each perturbed run took differently from the
    unperturbed one (branch records compared byte by byte), and with the switches replayed from
    the unperturbed run (the derivative the adjoint computes).  Each entry also states the
    floors of the difference: rounding eps |L| / (step |g|) and solver tolerance
    rtol |L| / (step |g|).  One cell moves the loss by |g| step ~ 1e-10 |L| for a 1e-6 step,
    below the solver floor, so cells take a larger step."""
    import copy

    import numpy as np

    fo = copy.copy(o)
    fo.rtol_visc = fo.rtol_mac = fo.rtol_proj = FD_RTOL
    base = ctx.switch_record(2 * nsteps)
    other = ctx.switch_record(2 * nsteps)

    def loss(bi, th, mode, rec):
        r = api.make_rheology(rheo.law, rheo.mu, bi, rheo.eps, rheo.rho)
        u, p = u0.clone(), p0.clone()
        ctx.set_switches(mode, rec)
        try:
            for _ in range(nsteps):
                # near 1e-14 a solve may stagnate one notch above rtol; its result is kept
                api.eb_rk2_step(ctx, r, w.dt, fo, u, p, theta=th, inplace=True,
                                allow_noconv=True)
        finally:
            ctx.set_switches(api.EB_SWITCH_OFF)
        return api.eb_drag(ctx, r, u, p, theta=th)[2]

    L0 = loss(w.tau0, theta, api.EB_SWITCH_RECORD, base)
    eps = 2.2e-16

    def central(args_p, args_m, h, g):
        lp = loss(*args_p, api.EB_SWITCH_RECORD, other)
        flips_p = int((other != base).sum().item())
        lm = loss(*args_m, api.EB_SWITCH_RECORD, other)
        flips_m = int((other != base).sum().item())
        fp = loss(*args_p, api.EB_SWITCH_REPLAY, base)
        fm = loss(*args_m, api.EB_SWITCH_REPLAY, base)
        ga = max(abs(g), 1e-300)
        fd, fdf = (lp - lm) / (2 * h), (fp - fm) / (2 * h)
        return {"adjoint": g, "fd": fd, "rel_err": abs(fd - g) / ga,
                "switches_flipped": [flips_p, flips_m], "fd_frozen": fdf,
                "rel_err_frozen": abs(fdf - g) / ga,
                "floor_round": eps * abs(L0) / (h * ga),
                "floor_solver": FD_RTOL * abs(L0) / (h * ga)}

    h = FD_BI_STEP * w.tau0
    res = {"steps": nsteps, "rtol": FD_RTOL, "bi_step_rel": FD_BI_STEP,
           "cell_step_rel": FD_CELL_STEP,
           "bi": central((w.tau0 + h, theta), (w.tau0 - h, theta), h, g_bi)}
    print(f"[bench] fd Bi: {res['bi']}", file=sys.stderr, flush=True)
    # candidate cells: open, centre within 3h of the sphere surface
    nz, ny, nx = ctx.shape
    zz, yy, xx = np.meshgrid(*[(np.arange(n) + 0.5) * w.h for n in (nz, ny, nx)], indexing="ij")
    c = w.body["center"]
    dist = np.sqrt((xx - c[0]) ** 2 + (yy - c[1]) ** 2 + (zz - c[2]) ** 2) - w.body["radius"]
    _, alpha, _, _, _ = api.eb_geometry_export(ctx)
    cand = np.flatnonzero((alpha.cpu().numpy() > 0).ravel() & (np.abs(dist).ravel() < 3 * w.h))
    picks = I.rng(2).choice(cand, size=ncells, replace=False)
    gt = g_theta.cpu().numpy().ravel()
    cells = []
    for cidx in picks:
        t0 = float(theta.view(-1)[cidx])
        hc = FD_CELL_STEP * t0
        tp, tm = theta.clone().view(-1), theta.clone().view(-1)
        tp[cidx] += hc
        tm[cidx] -= hc
        e = central((w.tau0, tp.view(theta.shape)), (w.tau0, tm.view(theta.shape)), hc,
                    float(gt[cidx]))
        e["cell"] = int(cidx)
        cells.append(e)
        print(f"[bench] fd cell {cidx}: {e}", file=sys.stderr, flush=True)
    res["cells"] = cells
    res["max_rel_err_cells"] = max(x["rel_err"] for x in cells)
    res["max_rel_err_cells_frozen"] = max(x["rel_err_frozen"] for x in cells)
    return res


def cpu_model():
    """The host CPU's model name (lscpu), or the platform's processor string."""
    import platform
    import subprocess

    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                return line.split(":", 1)[1].strip()
    except Exception:  # noqa: BLE001 - a missing lscpu only loses the label
        pass
    return platform.processor() or "unknown"


def cpu_baseline(w, u0, p0, n_steps=1):
    """The FP64 oracle (as it stands) on the host cores: one RK2 step of the same workload from
    the same state.  Returns MLUPS, the thread count it used and the seconds it took."""
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


def cpu_baseline_single_thread(w):
    """The oracle on one host thread, one step of the 64^3 version of the workload (same body,
    law and time step) from the uniform start: about 20 s.  Runs in a child process because the
    oracle's OpenMP runtime fixes its thread count when it first starts."""
    import subprocess

    n = 64
    code = ("import sys, time, json; sys.path.insert(0, %r)\n"
            "import numpy as np, eb_inputs as I\n"
            "from oracle import oracle as O\n"
            "w = I.sphere128().replace(n=(%d,)*3, h=1.0/%d, name='sphere%d')\n"
            "g = O.Geometry(w); u = I.initial_velocity(w); p = np.zeros(g.shape)\n"
            "t = time.perf_counter(); g.rk2_step(u, p, O.make_rheo(w), w.dt, O.make_opts(w))\n"
            "print(json.dumps({'s': time.perf_counter() - t, 'cells': w.ncell}))\n"
            % (ROOT, n, n, n))
    env = dict(os.environ, OMP_NUM_THREADS="1")
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, env=env,
                       timeout=600)
    res = json.loads(r.stdout.strip().splitlines()[-1])
    return res["cells"] / res["s"] / 1e6, res["s"], n


# Algorithmic bytes per fine cell of the passes one step executes (the scope table's byte model,
# with the Krylov vector passes counted as well); w = 8 (FP64) or 4 (FP32).  A multigrid V(2,2)
# over all levels: 553 B (viscous, three components) and 174 B (Poisson) in FP64.  In mixed
# precision the levels of at least 64^3 cells run in FP32 (484 -> 245 and 152 -> 79 B per cell
# of the level) and the smaller ones in FP64, which gives 284 and 91 B at 128^3.  Per BiCGSTAB
# half iteration (one V-cycle): an EB operator application (u in, eta, flag, out: 7w + 1) and
# its share of the vector updates and dot products (s = r - alpha v, x and r updates, p update,
# four dot products over 3-component vectors): 285 B.  Per CG iteration (one V-cycle): the
# Poisson application (2w + 1), x and r updates, p update, two dot products: 121 B.  Per step,
# outside the solves: face extrapolation, the derived quantities, psi assembly and the
# projection wrap of both stages, about 1100 B.
VCYCLE_BYTES = {"fp64": {"visc": 553.0, "poisson": 174.0},
                "mixed": {"visc": 284.0, "poisson": 91.0}}
KRYLOV_BYTES = {"visc": 285.0, "poisson": 121.0}
STEP_FIXED_BYTES = 1100.0


def step_bytes(stats, ncell, tag):
    """Algorithmic bytes of one step from its executed V-cycle counts."""
    n_poisson = sum(stats["it_mac"]) + sum(stats["it_proj"])
    n_visc = stats["vcycles"] - n_poisson
    per_cell = (n_visc * (VCYCLE_BYTES[tag]["visc"] + KRYLOV_BYTES["visc"])
                + n_poisson * (VCYCLE_BYTES[tag]["poisson"] + KRYLOV_BYTES["poisson"])
                + STEP_FIXED_BYTES)
    return per_cell * ncell, n_visc, n_poisson


def run_steps(api, torch, I, pkg, w, prec, args, start=None):
    """Builds a context for `prec`, runs the warm-up steps from the workload's start, then times
    args.steps steps from `start` (the warm-up's end state when None).  Returns the timing, the
    stats of every timed step, the start and end states and the context."""
    box, body, rheo, opts = pkg.from_workload(w, precision=prec)
    opts.nu1 = opts.nu2 = args.nu
    opts.nbottom = args.nbottom
    dev = torch.device("cuda:0")
    ctx = api.eb_geometry_build(box, body, dev)
    u = torch.from_numpy(I.initial_velocity(w)).to(dev)
    p = torch.zeros(ctx.shape, dtype=torch.float64, device=dev)
    tag = "fp64" if prec == api.EB_FP64 else "mixed"
    for s in range(args.warmup):
        u, p, st = api.eb_rk2_step(ctx, rheo, w.dt, opts, u, p, inplace=True)
        print(f"[bench] {tag} warmup step {s}: {st}", file=sys.stderr, flush=True)
    if start is not None:
        u.copy_(start[0])
        p.copy_(start[1])
    u0, p0 = u.clone(), p.clone()
    stats = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(args.steps):
        u, p, st = api.eb_rk2_step(ctx, rheo, w.dt, opts, u, p, inplace=True)
        stats.append(st)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    ms_step = 1e3 * t / args.steps
    mlups = w.ncell * args.steps / t / 1e6
    print(f"[bench] {tag} timed {args.steps} steps: {ms_step:.2f} ms/step, {mlups:.1f} MLUPS; "
          f"last stats {stats[-1]}", file=sys.stderr, flush=True)
    bsum = nv = npo = 0
    for st in stats:
        b, a, c = step_bytes(st, w.ncell, tag)
        bsum, nv, npo = bsum + b, nv + a, npo + c
    bstep = bsum / args.steps
    step_roof = {"bytes_per_step": int(bstep),
                 "vcycles_per_step": {"viscous": nv / args.steps, "poisson": npo / args.steps},
                 "achieved": round(bstep / (ms_step * 1e-3) / 1e9, 1),
                 "peak": HBM_PEAK_GBS, "unit": "GB/s",
                 "frac": round(bstep / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
    return {"ms_step": ms_step, "mlups": mlups, "stats": stats, "u0": u0, "p0": p0, "u": u,
            "p": p, "ctx": ctx, "rheo": rheo, "opts": opts, "step_roofline": step_roof}


def smoother_roofline(api, torch, run, w, prec, args):
    """The finest-level viscous smoother with the operator of the run's final state: average
    launch time (HIP events) and the fraction of HBM peak on algorithmic bytes."""
    ctx, rheo, opts, u = run["ctx"], run["rheo"], run["opts"], run["u"]
    eta, eta_eb = api.eb_apparent_viscosity(ctx, rheo, u)
    api.eb_mg_vcycle(ctx, api.EB_SYS_VISC, torch.zeros_like(u), opts, precision=prec, rho=w.rho,
                     dt=w.dt, eta=eta, eta_eb=eta_eb)
    ms_k = time_smoother(api, ctx, prec, args.sweeps, torch)
    wbytes = 4 if prec == api.EB_MIXED else 8
    algo = smoother_bytes_per_launch(ctx.N, 3, wbytes)
    achieved = algo / (ms_k * 1e-3) / 1e9
    return ms_k, algo, achieved


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: runs on one GPU only; the step is a single box on one GPU and the "
              "multi-GPU domain decomposition is not built.", file=sys.stderr)
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
    dev = torch.device("cuda:0")

    if args.kernel_only:
        # build the viscous operator of the start state, then only the smoother loop
        box, body, rheo, opts = pkg.from_workload(w, precision=prec)
        ctx = api.eb_geometry_build(box, body, dev)
        u = torch.from_numpy(I.initial_velocity(w)).to(dev)
        eta, eta_eb = api.eb_apparent_viscosity(ctx, rheo, u)
        r = torch.zeros_like(u)
        api.eb_mg_vcycle(ctx, api.EB_SYS_VISC, r, opts, precision=prec, rho=w.rho, dt=w.dt,
                         eta=eta, eta_eb=eta_eb)
        ms = time_smoother(api, ctx, prec, args.sweeps, torch)
        # a plain device copy of known size (3N doubles read, 3N written) calibrates the
        # hardware byte counters read by a profiler over this run
        src = torch.randn((3,) + ctx.shape, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        for _ in range(args.sweeps):
            dst.copy_(src)
        torch.cuda.synchronize()
        tag = "mixed" if prec == api.EB_MIXED else "fp64"
        print(json.dumps({"kernel": SMOOTHER_KERNEL[tag] + "<3> finest level", "avg_ms": ms,
                          "copy_bytes_each_way": src.numel() * 8}))
        return

    print(f"[bench] {w.name} n={w.n} precision={args.precision} warmup={args.warmup} "
          f"steps={args.steps}", file=sys.stderr, flush=True)
    main_run = run_steps(api, torch, I, pkg, w, prec, args)
    other_prec = api.EB_FP64 if prec == api.EB_MIXED else api.EB_MIXED
    other = None
    if not args.single_precision:
        # the other precision, timed over the same steps from the same start state
        other = run_steps(api, torch, I, pkg, w, other_prec, args,
                          start=(main_run["u0"], main_run["p0"]))
    u0_host = main_run["u0"].cpu().numpy().copy()
    p0_host = main_run["p0"].cpu().numpy().copy()

    # roofline of the dominant kernel: the finest-level viscous smoother
    ms_k, algo, achieved = smoother_roofline(api, torch, main_run, w, prec, args)
    traffic = counted_traffic("fp64" if prec == api.EB_FP64 else "mixed") if args.n == 128 else None
    copy_gbs = copy_bandwidth(main_run["ctx"], torch)
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": SMOOTHER_KERNEL["fp64" if prec == api.EB_FP64 else "mixed"]
                + " (finest level, 3 components, one colour)",
                "kernel_ms": round(ms_k, 5), "bytes_per_launch": int(algo),
                "device_copy_gbs": round(copy_gbs, 1),
                "frac_of_device_copy": round(achieved / copy_gbs, 4),
                "step": main_run["step_roofline"]}
    st_last = main_run["stats"][-1]
    out = {"metric": METRIC, "value": round(main_run["mlups"], 3), "unit": "MLUPS", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": round(main_run["ms_step"], 3),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f64" if prec == api.EB_FP64 else "f64+f32-mg",
           "data": "synthetic",
           "config": {"workload": f"{w.name}: {w.n[0]}^3 box, EB sphere r=0.125, walls (0,0,-1),"
                                  f" eta=1+10/(|g|+1e-6), rho=4e-3, dt=5e-4, rtol=1e-12",
                      "cells": w.ncell, "precision": args.precision,
                      "dt": w.dt, "dt_stability_rule": st_last["dt_stable"],
                      "iterations_last_step": {k: st_last[k] for k in
                                               ("it_mac", "it_visc", "it_proj", "vcycles")}},
           "roofline": roofline}
    if other is not None:
        # the other precision's line: speed, step roofline, smoother, and its difference from
        # the headline run after the same steps from the same state (relative L2 over open cells)
        ms_o, algo_o, ach_o = smoother_roofline(api, torch, other, w, other_prec, args)
        _, alpha, _, _, _ = api.eb_geometry_export(main_run["ctx"])
        op = alpha > 0
        a, b = (other, main_run) if other_prec == api.EB_MIXED else (main_run, other)
        errs = {}
        for j, name in enumerate("uvw"):
            errs[name] = (torch.linalg.norm((a["u"][j] - b["u"][j])[op])
                          / torch.linalg.norm(b["u"][j][op])).item()
        errs["p"] = (torch.linalg.norm((a["p"] - b["p"])[op]) / torch.linalg.norm(b["p"][op])).item()
        Fa = api.eb_drag(a["ctx"], a["rheo"], a["u"], a["p"])
        Fb = api.eb_drag(b["ctx"], b["rheo"], b["u"], b["p"])
        errs["F_z"] = abs(Fa[2] - Fb[2]) / abs(Fb[2])
        tag = "mixed" if other_prec == api.EB_MIXED else "fp64"
        so = other["stats"][-1]
        out[tag] = {"ms_per_step": round(other["ms_step"], 3), "value": round(other["mlups"], 3),
                    "unit": "MLUPS", "speedup_vs_headline": round(main_run["ms_step"]
                                                                  / other["ms_step"], 4),
                    "step_roofline": other["step_roofline"],
                    "smoother": {"kernel_ms": round(ms_o, 5), "bytes_per_launch": int(algo_o),
                                 "achieved": round(ach_o, 1),
                                 "frac": round(ach_o / HBM_PEAK_GBS, 4)},
                    "rel_err_mixed_vs_fp64": errs, "fp64_fallbacks": so["fp64_fallbacks"],
                    "iterations_last_step": {k: so[k] for k in
                                             ("it_mac", "it_visc", "it_proj", "vcycles")}}
        print(f"[bench] {tag}: {out[tag]}", file=sys.stderr, flush=True)
    ctx = main_run["ctx"]
    if args.adjoint_steps > 0:
        from paper_1905_07392_amd import autograd as AG

        adj = adjoint_ratio(api, AG, ctx, w, main_run["opts"], args.adjoint_steps,
                            args.ckpt_every, torch, I, fd_cells=args.adjoint_fd,
                            fd_steps=args.adjoint_fd_steps)
        out["adjoint"] = adj
        print(f"[bench] adjoint: {adj}", file=sys.stderr, flush=True)
    if not args.no_cpu_baseline:
        val, cores, tcpu = cpu_baseline(w, u0_host, p0_host)
        out["cpu_baseline"] = {"value": round(val, 4), "unit": "MLUPS", "cores": cores,
                               "kind": "oracle",
                               "sample": f"one FP64 RK2 step of the same {w.n[0]}^3 workload "
                                         f"from the same state ({tcpu:.1f} s)",
                               "cpu_model": cpu_model()}
        if not args.no_single_thread:
            v1, t1, n1 = cpu_baseline_single_thread(w)
            out["cpu_baseline"]["single_thread"] = {
                "value": round(v1, 4), "unit": "MLUPS", "cores": 1,
                "sample": f"one FP64 RK2 step of the {n1}^3 version of the workload from the "
                          f"uniform start on one thread ({t1:.1f} s)"}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
