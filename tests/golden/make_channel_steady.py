"""Writes channel64_steady.txt: the oracle's steady plane-Poiseuille profiles of the 64^3 Bingham
channel (EB walls at z = 0.1171875 and 0.8828125, periodic in x and y, Papanastasiou law with
eps = 1e-8, body force (1, 0, 0)), for Bi = 0.5 and 2 with tau0 from the appendix relation
Bi = 2 z0 / (1 - z0)^2 and tau0 = z0 G W (App. B; W the half gap).

The flow is uniform in x and y, so the oracle runs a 4 x 4 x 64 box with the same cells in z;
the GPU tests compare their 64 x 64 x 64 steady state with these profiles.  Only the oracle is
called.  Run from the repository root:  python tests/golden/make_channel_steady.py
"""
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
for p in (ROOT, os.path.join(ROOT, "tests")):
    if p not in sys.path:
        sys.path.insert(0, p)

import numpy as np  # noqa: E402

import analytic as A  # noqa: E402
import eb_inputs as I  # noqa: E402

ZLO, ZHI = 0.1171875, 0.8828125
HALF_GAP = 0.5 * (ZHI - ZLO)
EPS = 1e-8
DT = 1.0          # the steady state does not depend on dt; the lagged viscosity sets the pace
STEADY_TOL = 1e-13  # max |u^{m+1} - u^m| / U at which the run stops
BIS = (0.5, 2.0)
OUT = os.path.join(HERE, "channel64_steady.txt")


def channel_params(bi):
    """(z0, tau0, U) of the Bingham channel at Bingham number bi (G = mu = 1)."""
    z0 = A.z0_from_bi(bi)
    tau0 = z0 * HALF_GAP
    U = HALF_GAP ** 2 * (1.0 - z0) ** 2 / 2.0
    return z0, tau0, U


def workload(bi, nxy):
    _, tau0, _ = channel_params(bi)
    w = I.channel64(tau0=tau0, eps=EPS, n=64, nxy=nxy).replace(dt=DT)
    assert abs(w.body["zlo"] - ZLO) < 1e-15 and abs(w.body["zhi"] - ZHI) < 1e-15
    return w


def run_to_steady(O, w, U, rtol=1e-12, maxsteps=3000):
    """Oracle RK2 steps from rest until max |du| < STEADY_TOL U; returns (u, p, steps)."""
    g = O.Geometry(w)
    opts = O.make_opts(w, rtol=rtol, max_iter=500)
    rh = O.make_rheo(w)
    u = np.zeros((3,) + g.shape)
    p = np.zeros(g.shape)
    for s in range(maxsteps):
        u1, p, _ = g.rk2_step(u, p, rh, w.dt, opts)
        du = np.abs(u1 - u).max()
        u = u1
        if du < STEADY_TOL * U:
            return u, p, s + 1
    raise RuntimeError("no steady state")


def oracle_profiles(O):
    out = {}
    for bi in BIS:
        _, _, U = channel_params(bi)
        u, _, steps = run_to_steady(O, workload(bi, 4), U)
        out[bi] = (u[0, :, 0, 0].copy(), steps)
    return out


def main():
    from oracle import build, oracle as O

    if not os.path.exists(O.LIB_PATH):
        build.build()
    prof = oracle_profiles(O)
    with open(OUT, "w") as f:
        f.write("# Steady x-velocity u(z) of the 64^3 Bingham channel (EB walls at z = 0.1171875 and\n"
                "# 0.8828125, Papanastasiou eps = 1e-8, force (1,0,0)), from the oracle on a 4x4x64 box\n"
                "# (make_channel_steady.py; tau0 from Bi by App. B).  Columns: Bi k u_k\n")
        for bi in BIS:
            f.write(f"# Bi = {bi}: {prof[bi][1]} steps\n")
            for k, v in enumerate(prof[bi][0]):
                f.write(f"{bi!r} {k} {float(v)!r}\n")
    print("wrote", OUT)


if __name__ == "__main__":
    main()
