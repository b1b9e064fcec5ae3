"""Seeded synthetic workloads for the embedded-boundary viscoplastic RK2 step.

This module holds plain data and random draws only: box sizes, body shapes, rheology constants,
time steps and seeded fields.  It contains none of the numerical method.  Both the CPU oracle
(tests only) and the HIP path read their inputs from here, so the two sides see identical data.

Every field array is float64, C-contiguous, shaped [3, nz, ny, nx] (vector) or [nz, ny, nx]
(scalar); x is the fastest index.

Workloads (sizes and parameters follow the flow configurations studied in the paper,
Sec. IV.B (plane Poiseuille) and Sec. V (translating sphere), with unit-cube boxes):

* ``sphere32``      32^3, sphere r=0.2 at the centre, walls moving at (0,0,-1),
                    eta = 1 + 1/(|gamma|+1e-6), rho=1, dt=1e-3, noisy start (seed 0).
* ``channel64``     64^3, periodic in x and y, EB planes at z=0.1171875 and 0.8828125,
                    Papanastasiou law, body force along x.
* ``sphere128``     128^3, sphere r=0.125, walls (0,0,-1), eta = 1 + 10/(|gamma|+1e-6),
                    rho=4e-3, dt=5e-4, uniform start.
* ``ellipsoid256``  256^3, rotated ellipsoid (0.15,0.10,0.08), Papanastasiou Bi=100,
                    eps=1e-4, dt=2.5e-4.
"""
from __future__ import annotations

import copy
import math
from dataclasses import dataclass, field

import numpy as np

BODY_NONE, BODY_SPHERE, BODY_ELLIPSOID, BODY_ZSLAB, BODY_PLANE, BODY_CYLINDER = 0, 1, 2, 3, 4, 5
BODY_CAVITY = 6  # fluid inside a sphere (body outside)
LAW_NEWTONIAN, LAW_BINGHAM_REG, LAW_PAPANASTASIOU = 0, 1, 2
LAW_POWER, LAW_HERSCHEL_BULKLEY, LAW_SOUZA_MENDES_DUTRA = 3, 4, 5


@dataclass
class Workload:
    name: str
    n: tuple                      # (nx, ny, nz)
    h: float
    lo: tuple = (0.0, 0.0, 0.0)
    periodic: tuple = (0, 0, 0)
    wall_u: list = field(default_factory=lambda: [[0.0, 0.0, 0.0] for _ in range(6)])
    body: dict = field(default_factory=lambda: {"kind": BODY_NONE})
    law: int = LAW_NEWTONIAN
    mu: float = 1.0
    tau0: float = 0.0
    eps: float = 1e-6
    rho: float = 1.0
    kappa: float = 1.0            # consistency of the power-law laws
    flow_n: float = 1.0           # their flow index n
    eta0: float = 1.0             # Souza Mendes-Dutra zero-strain viscosity
    dt: float = 1e-3
    force: tuple = (0.0, 0.0, 0.0)
    rtol: float = 1e-12
    noise: float = 0.0            # amplitude of the seeded Gaussian start perturbation
    seed: int = 0
    steps: int = 1

    @property
    def shape(self):
        nx, ny, nz = self.n
        return (nz, ny, nx)

    @property
    def ncell(self):
        return int(self.n[0] * self.n[1] * self.n[2])

    def replace(self, **kw):
        w = copy.deepcopy(self)
        for k, v in kw.items():
            setattr(w, k, v)
        return w


def _moving_walls(v):
    return [list(v) for _ in range(6)]


def sphere32() -> Workload:
    return Workload(name="sphere32", n=(32, 32, 32), h=1.0 / 32,
                    wall_u=_moving_walls((0.0, 0.0, -1.0)),
                    body={"kind": BODY_SPHERE, "center": (0.5, 0.5, 0.5), "radius": 0.2},
                    law=LAW_BINGHAM_REG, mu=1.0, tau0=1.0, eps=1e-6, rho=1.0, dt=1e-3,
                    noise=1e-2, seed=0, steps=1)


def channel64(tau0: float = 0.0, eps: float = 1e-8, n: int = 64, nxy: int = None) -> Workload:
    nxy = n if nxy is None else nxy
    return Workload(name="channel64", n=(nxy, nxy, n), h=1.0 / n, periodic=(1, 1, 0),
                    body={"kind": BODY_ZSLAB, "zlo": 0.1171875, "zhi": 0.8828125},
                    law=LAW_PAPANASTASIOU, mu=1.0, tau0=tau0, eps=eps, rho=1.0, dt=1e-3,
                    force=(1.0, 0.0, 0.0), noise=0.0, seed=0, steps=1)


def sphere128() -> Workload:
    return Workload(name="sphere128", n=(128, 128, 128), h=1.0 / 128,
                    wall_u=_moving_walls((0.0, 0.0, -1.0)),
                    body={"kind": BODY_SPHERE, "center": (0.5, 0.5, 0.5), "radius": 0.125},
                    law=LAW_BINGHAM_REG, mu=1.0, tau0=10.0, eps=1e-6, rho=4e-3, dt=5e-4,
                    noise=0.0, seed=0, steps=100)


def ellipsoid256() -> Workload:
    ang = euler_angles(3)
    return Workload(name="ellipsoid256", n=(256, 256, 256), h=1.0 / 256,
                    wall_u=_moving_walls((0.0, 0.0, -1.0)),
                    body={"kind": BODY_ELLIPSOID, "center": (0.5, 0.5, 0.5),
                          "radii": (0.15, 0.10, 0.08), "euler_zyx": tuple(ang)},
                    law=LAW_PAPANASTASIOU, mu=1.0, tau0=100.0, eps=1e-4, rho=1.0, dt=2.5e-4,
                    noise=0.0, seed=3, steps=50)


def cylinder(npd: int, bi: float = 0.0) -> Workload:
    """The cylinder of Sec. V.C with D = U = mu = 1: domain [0, 4D] x [0, D/2] x [0, 6D], periodic
    along the axis (y), u = U e_z at the start and on every other wall, Re = rho U D / mu = 1e-3,
    npd cells per diameter, tau0 = Bi (Papanastasiou, eps = 1e-3; Newtonian for bi = 0).  The
    paper does not state the time step; dt = rho D^2 / mu = 1e-3 is taken, far below the
    convective limit, since the step lags the pressure and in creeping flow the lag decays per
    step by about 1 - rho/(mu dt) (the steady state is the same for any dt)."""
    assert npd % 8 == 0
    h = 1.0 / npd
    return Workload(name=f"cylinder{npd}", n=(4 * npd, npd // 2, 6 * npd), h=h,
                    periodic=(0, 1, 0), wall_u=_moving_walls((0.0, 0.0, 1.0)),
                    body={"kind": BODY_CYLINDER, "center": (2.0, 0.25, 3.0), "radius": 0.5},
                    law=LAW_PAPANASTASIOU if bi > 0 else LAW_NEWTONIAN, mu=1.0, tau0=bi,
                    eps=1e-3, rho=1e-3, dt=1e-3, noise=0.0, seed=0, steps=1)


def taylor_green(n: int) -> Workload:
    """The Taylor-Green vortex of Sec. IV.A (Eq. taylor-green): the unit square periodic in x and
    y, extruded over n/4 cells along z (periodic, uniform), Re = rho U L / mu = 100 with
    rho = U = L = 1; dt = h/(2U), so t = 1 takes 2n steps."""
    return Workload(name=f"taylor_green{n}", n=(n, n, n // 4), h=1.0 / n, periodic=(1, 1, 1),
                    law=LAW_NEWTONIAN, mu=0.01, rho=1.0, dt=0.5 / n, noise=0.0, seed=0,
                    steps=2 * n)


def sphere_n(n: int, radius: float = 0.2, **kw) -> Workload:
    """A sphere32-like workload at another resolution (parity sizes with ragged tiles)."""
    w = sphere32().replace(name=f"sphere{n}", n=(n, n, n), h=1.0 / n)
    w.body = {"kind": BODY_SPHERE, "center": (0.5, 0.5, 0.5), "radius": radius}
    for k, v in kw.items():
        setattr(w, k, v)
    return w


WORKLOADS = {"sphere32": sphere32, "channel64": channel64, "sphere128": sphere128,
             "ellipsoid256": ellipsoid256}


# ----------------------------------------------------------------------------------------------
# seeded draws
# ----------------------------------------------------------------------------------------------
def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def euler_angles(seed: int) -> np.ndarray:
    return rng(seed).uniform(0.0, 2.0 * math.pi, size=3)


def initial_velocity(w: Workload) -> np.ndarray:
    """Start field: the wall velocity of the -z face everywhere plus seeded i.i.d. Gaussian noise.

    The field is not projected here (projection belongs to the method)."""
    nz, ny, nx = w.shape
    u = np.empty((3, nz, ny, nx), dtype=np.float64)
    base = w.wall_u[4]
    for c in range(3):
        u[c] = base[c]
    if w.noise > 0.0:
        u += w.noise * rng(w.seed).standard_normal((3, nz, ny, nx))
    return np.ascontiguousarray(u)


def yield_field(w: Workload, seed: int = 1, amp: float = 0.05) -> np.ndarray:
    """Per-cell yield-stress multiplier theta = 1 + amp*U(-1,1) (tau0_i = tau0*theta_i)."""
    return np.ascontiguousarray(1.0 + amp * rng(seed).uniform(-1.0, 1.0, size=w.shape))


def random_field(shape, seed: int, scale: float = 1.0) -> np.ndarray:
    return np.ascontiguousarray(scale * rng(seed).standard_normal(shape))


def random_faces(n, seed: int, scale: float = 1.0):
    """Three face-centred arrays shaped [nz][ny][nx+1], [nz][ny+1][nx], [nz+1][ny][nx]."""
    nx, ny, nz = n
    g = rng(seed)
    fx = scale * g.standard_normal((nz, ny, nx + 1))
    fy = scale * g.standard_normal((nz, ny + 1, nx))
    fz = scale * g.standard_normal((nz + 1, ny, nx))
    return [np.ascontiguousarray(a) for a in (fx, fy, fz)]
