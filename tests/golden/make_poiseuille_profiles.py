"""Writes poiseuille_profiles.txt: the oracle's steady plane-Poiseuille profiles u(z)/U at the
full resolutions of Table convergence:bingham (Sec. IV.B): N = 64, 128, 256 cells across the gap
2W = 1, z0 = 0.1, 0.2, 0.5, Papanastasiou eps = 0.01 U / W, G = mu = 1, tau0 = z0 G W, walls at
z = 0 and 1, dt = 1e3, run from rest until max |u^{m+1} - u^m| < 1e-15 U.

The flow is uniform in x and y, so the oracle runs a 4 x 4 x N box; the GPU test runs a wider box
and compares its profile with these.  Only the oracle is called.  Run from the repository root:
python tests/golden/make_poiseuille_profiles.py   (about ten minutes on one core)
"""
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
for p in (ROOT, os.path.join(ROOT, "tests")):
    if p not in sys.path:
        sys.path.insert(0, p)

import numpy as np  # noqa: E402

import eb_inputs as I  # noqa: E402

NS = (64, 128, 256)
Z0S = (0.1, 0.2, 0.5)
EPS_HAT = 0.01
STEADY_TOL = 1e-15
OUT = os.path.join(HERE, "poiseuille_profiles.txt")


def steady_profile(O, N, z0, maxsteps=3000):
    W, G, mu = 0.5, 1.0, 1.0
    U = G * W * W * (1 - z0) ** 2 / (2 * mu)
    w = I.Workload(name="poiseuille", n=(4, 4, N), h=1.0 / N, periodic=(1, 1, 0),
                   law=I.LAW_PAPANASTASIOU, mu=mu, tau0=z0 * G * W, eps=EPS_HAT * U / W,
                   rho=1.0, dt=1e3, force=(G, 0.0, 0.0))
    g = O.Geometry(w)
    opts = O.make_opts(w, rtol=1e-12)
    rh = O.make_rheo(w)
    u = np.zeros((3,) + g.shape)
    p = np.zeros(g.shape)
    for s in range(maxsteps):
        u1, p, _ = g.rk2_step(u, p, rh, w.dt, opts)
        du = np.abs(u1 - u).max()
        u = u1
        if du < STEADY_TOL * U:
            return u[0, :, 0, 0] / U, s + 1
    raise RuntimeError("no steady state")


def main():
    from oracle import build, oracle as O

    if not os.path.exists(O.LIB_PATH):
        build.build()
    with open(OUT, "w") as f:
        f.write("# Steady u(z)/U of plane Poiseuille flow with the Papanastasiou law (eps = 0.01 U/W),\n"
                "# from the oracle on a 4x4xN box (make_poiseuille_profiles.py).  Sec. IV.B.\n"
                "# Columns: z0 N k u_k/U\n")
        for N in NS:
            for z0 in Z0S:
                prof, steps = steady_profile(O, N, z0)
                f.write(f"# z0 = {z0}, N = {N}: {steps} steps\n")
                for k, v in enumerate(prof):
                    f.write(f"{z0!r} {N} {k} {float(v)!r}\n")
                f.flush()
                print(f"z0={z0} N={N}: {steps} steps", flush=True)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
