"""Writes the FP64 oracle's reference values for the 128^3 translating-sphere workloads.

Calls only the oracle (oracle/) and the seeded inputs (eb_inputs.py).  Two parts:

* ``history``: the perf workload (sphere r = 0.125, walls (0,0,-1), eta = 1 + 10/(|g| + 1e-6),
  rho = 4e-3, dt = 5e-4, uniform start u = (0,0,-1), p = 0), 100 RK2 steps.  Per step: the force
  on the sphere (Eq. drag-force), the L2 norms of u, v, w and p over open cells, the solver
  iterations; at steps 1, 2, 10, 50 and 100 the values of u, v, w, p at 64 seeded open cells (32
  of them within 3h of the body, where the flow changes most).
  -> tests/golden/sphere128_history_oracle.txt

* ``fd``: the adjoint workload (the same, with tau0_c = Bi theta_c, theta = 1 + 0.05 U(-1,1) seed
  1, Bi = 10), 20 steps each at Bi - h, Bi and Bi + h with h = 1e-6 Bi (solves to rtol 1e-12:
  at 1e-13 the oracle's end-of-stage projection creeps along its rounding floor for 200-300 CG
  iterations per solve, several minutes per step):
  per step F_z of the three runs (so the central difference of F_z in Bi after every step) and
  the max-norm and relative L2 of u(Bi + h) - u(Bi) over open cells (how a perturbation of the
  yield stress grows from step to step).
  -> tests/golden/sphere128_fd_oracle.txt

Usage: OMP_NUM_THREADS=8 python tests/golden/make_sphere128_history.py {history|fd}
About 40 s per oracle step on 8 host threads.
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import eb_inputs as I  # noqa: E402
from oracle import oracle as O  # noqa: E402

SAMPLE_STEPS = (1, 2, 10, 50, 100)


def sample_cells(alpha, flag, h, seed=5, n_near=32, n_far=32):
    """64 seeded open cells: n_near among the cells within 3h of a cut cell, n_far elsewhere."""
    from scipy import ndimage

    cut = flag == 1
    near = ndimage.binary_dilation(cut, iterations=3) & (alpha > 0)
    far = (alpha > 0) & ~near
    rng = I.rng(seed)
    a = rng.choice(np.flatnonzero(near.ravel()), size=n_near, replace=False)
    b = rng.choice(np.flatnonzero(far.ravel()), size=n_far, replace=False)
    return np.sort(np.concatenate([a, b]))


def history(nsteps=100):
    w = I.sphere128()
    g = O.Geometry(w)
    flag, alpha, _ = g.export()
    open_ = alpha > 0
    opts = O.make_opts(w)
    rh = O.make_rheo(w)
    u = I.initial_velocity(w)
    p = np.zeros(g.shape)
    cells = sample_cells(alpha, flag, w.h)
    rows, samples = [], []
    for s in range(1, nsteps + 1):
        t0 = time.time()
        u, p, st = g.rk2_step(u, p, rh, w.dt, opts)
        F = g.drag(u, p, rh)
        norms = [float(np.linalg.norm(u[j][open_])) for j in range(3)]
        norms.append(float(np.linalg.norm(p[open_])))
        rows.append((s, *F, *norms, *st["it_mac"], *st["it_visc"], *st["it_proj"]))
        if s in SAMPLE_STEPS:
            flat = [u[j].ravel()[cells] for j in range(3)] + [p.ravel()[cells]]
            samples.append((s, np.stack(flat, axis=1)))
        print(f"[history] step {s}: F_z {F[2]:.15e} ({time.time() - t0:.1f} s) {st}",
              flush=True)
    out = os.path.join(HERE, "sphere128_history_oracle.txt")
    with open(out, "w") as f:
        f.write("# FP64 oracle, 128^3 sphere (r = 0.125, walls (0,0,-1), eta = 1 + 10/(|g|+1e-6),\n"
                "# rho = 4e-3, dt = 5e-4, rtol 1e-12, uniform start), written by\n"
                "# tests/golden/make_sphere128_history.py from the oracle alone.\n"
                "# Force: Eq. drag-force; norms: L2 over open cells.\n")
        f.write("# step Fx Fy Fz |u| |v| |w| |p| it_mac0 it_mac1 it_visc0 it_visc1 it_proj0 "
                "it_proj1\n")
        for r in rows:
            f.write(" ".join([str(r[0])] + [repr(float(x)) for x in r[1:8]] +
                             [str(int(x)) for x in r[8:]]) + "\n")
        f.write("# samples: step cell u v w p\n")
        for s, vals in samples:
            for c, v in zip(cells, vals):
                f.write("S %d %d %s\n" % (s, c, " ".join(repr(float(x)) for x in v)))
    print(f"wrote {out}")


def fd(nsteps=20):
    w = I.sphere128()
    g = O.Geometry(w)
    _, alpha, _ = g.export()
    open_ = alpha > 0
    theta = I.yield_field(w, seed=1)
    opts = O.make_opts(w, rtol=1e-12, max_iter=1000)
    h = 1e-6 * w.tau0
    runs = {}
    for tag, bi in (("0", w.tau0), ("+", w.tau0 + h), ("-", w.tau0 - h)):
        rh = O.make_rheo(w, tau0=bi)
        u = I.initial_velocity(w)
        p = np.zeros(g.shape)
        fz, us = [], []
        for s in range(1, nsteps + 1):
            t0 = time.time()
            u, p, st = g.rk2_step(u, p, rh, w.dt, opts, theta=theta)
            fz.append(float(g.drag(u, p, rh, theta=theta)[2]))
            if tag in ("0", "+"):
                us.append(u.copy() if tag == "0" else None)
            if tag == "+":
                d = u - runs["0"]["u"][s - 1]
                runs.setdefault("du", []).append(
                    (float(np.abs(d[:, open_]).max()),
                     float(np.linalg.norm(d[:, open_]) / np.linalg.norm(u[:, open_]))))
            print(f"[fd {tag}] step {s}: F_z {fz[-1]:.15e} ({time.time() - t0:.1f} s) {st}",
                  flush=True)
        runs[tag] = {"fz": fz, "u": us if tag == "0" else None}
    out = os.path.join(HERE, "sphere128_fd_oracle.txt")
    with open(out, "w") as f:
        f.write("# FP64 oracle, 128^3 sphere adjoint workload (tau0_c = Bi theta_c, theta seed 1,\n"
                "# Bi = 10, rho = 4e-3, dt = 5e-4, rtol 1e-12, uniform start), written by\n"
                "# tests/golden/make_sphere128_history.py from the oracle alone.\n"
                f"# h = {h!r} (1e-6 Bi).  Columns: step, F_z at Bi, at Bi + h, at Bi - h,\n"
                "# max|u(Bi+h) - u(Bi)| and its relative L2 over open cells.\n")
        for s in range(nsteps):
            du = runs["du"][s]
            f.write(f"{s + 1} {runs['0']['fz'][s]!r} {runs['+']['fz'][s]!r} "
                    f"{runs['-']['fz'][s]!r} {du[0]!r} {du[1]!r}\n")
    print(f"wrote {out}")


if __name__ == "__main__":
    part = sys.argv[1] if len(sys.argv) > 1 else "history"
    {"history": history, "fd": fd}[part]()
