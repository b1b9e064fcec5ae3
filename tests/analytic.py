"""Closed forms used to pin the oracle (test infrastructure).

* Lambert W in the log domain and the Papanastasiou plane-Poiseuille profile (App. B,
  Eq. poiseuille:papabing) plus the unregularised Bingham profile (Eq. poiseuille:bingham).
* Exact volume of a unit cube below a plane and exact area of a unit square below a line
  (inclusion-exclusion over the corners), used to pin the planar cut-cell geometry.
* Convergence-rate helpers (Eqs. convergence-rate and norms).
"""
from __future__ import annotations

import math
from itertools import product

import numpy as np


# ----------------------------------------------------------------------------------------------
# Lambert W (principal branch) for arguments given by their logarithm
# ----------------------------------------------------------------------------------------------
def lambertw_exp(L):
    """W(exp(L)) for real L (elementwise), i.e. the w > 0 solving w + log(w) = L.

    Halley iterations from a log-based start; valid for very large arguments where exp(L)
    would overflow.  For exp(L) below 1e-12 the series W(x) = x - x^2 + 1.5 x^3 is exact to
    double precision."""
    L = np.atleast_1d(np.asarray(L, dtype=np.float64))
    out = np.empty_like(L)
    small = L < math.log(1e-12)
    x = np.exp(L[small])
    out[small] = x - x * x + 1.5 * x ** 3
    Lb = L[~small]
    eL = np.exp(np.minimum(Lb, 1.0))  # the start below needs exp(L) only where L <= 1
    w = np.where(Lb > 1.0, Lb - np.log(np.maximum(Lb, 1.0)), eL / (1.0 + eL))
    for _ in range(100):
        f = w + np.log(w) - Lb
        fp = 1.0 + 1.0 / w
        fpp = -1.0 / (w * w)
        step = f / (fp - 0.5 * f * fpp / fp)
        w_new = np.maximum(w - step, w * 1e-3)
        done = np.all(np.abs(w_new - w) <= 4e-16 * np.abs(w_new))
        w = w_new
        if done:
            break
    out[~small] = w
    return out


def lambertw(x):
    x = np.asarray(x, dtype=np.float64)
    return lambertw_exp(np.log(x))


# ----------------------------------------------------------------------------------------------
# plane Poiseuille flow (Sec. IV.B and App. B), in units of W (half gap) and U (max velocity)
# ----------------------------------------------------------------------------------------------
def bi_from_z0(z0):
    return 2.0 * z0 / (1.0 - z0) ** 2


def z0_from_bi(bi):
    """Solve Bi = 2 z0/(1-z0)^2 for z0 in (0, 1)."""
    # bi (1 - z)^2 = 2 z  ->  bi z^2 - (2 bi + 2) z + bi = 0, take the root below 1
    if bi == 0.0:
        return 0.0
    a, b, c = bi, -(2.0 * bi + 2.0), bi
    return (-b - math.sqrt(b * b - 4 * a * c)) / (2 * a)


def bingham_profile(zhat, z0):
    """Unregularised Bingham plane-Poiseuille velocity (Eq. poiseuille:bingham), u/U."""
    z = np.abs(np.asarray(zhat, dtype=np.float64))
    return np.where(z <= z0, 1.0, 1.0 - ((z - z0) / (1.0 - z0)) ** 2)


def papanastasiou_profile(zhat, z0, eps):
    """Papanastasiou-regularised plane-Poiseuille velocity (Eq. poiseuille:papabing), u/U.

    eps is the dimensionless regularisation parameter (strain rates scaled by U/W)."""
    z = np.abs(np.asarray(zhat, dtype=np.float64))
    if z0 == 0.0:
        return 1.0 - z * z
    xi = 2.0 * z0 / (eps * (1.0 - z0) ** 2)
    w_z = lambertw_exp(math.log(xi) - xi * (z / z0 - 1.0))
    w_1 = lambertw_exp(math.log(xi) - xi * (1.0 / z0 - 1.0))
    return (1.0 - ((z - z0) / (1.0 - z0)) ** 2
            + z0 * eps / (2.0 * xi) * ((1.0 + w_z) ** 2 - (1.0 + w_1) ** 2))


# ----------------------------------------------------------------------------------------------
# exact cube/square fractions below a hyperplane
# ----------------------------------------------------------------------------------------------
def box_fraction_below(nv, d):
    """Measure of {x in [0,1]^k : nv.x <= d} by inclusion-exclusion over the corners."""
    nv = [float(a) for a in nv]
    d = float(d)
    # reflect negative components: x_i -> 1 - x_i
    for i, a in enumerate(nv):
        if a < 0.0:
            d -= a
            nv[i] = -a
    act = [a for a in nv if a != 0.0]
    k = len(act)
    if k == 0:
        return 1.0 if d >= 0.0 else 0.0
    s = 0.0
    for v in product((0, 1), repeat=k):
        t = d - sum(a * b for a, b in zip(act, v))
        if t > 0.0:
            s += (-1) ** sum(v) * t ** k
    return s / (math.factorial(k) * math.prod(act))


# ----------------------------------------------------------------------------------------------
# error norms and rates (Eqs. norms and convergence-rate), mean-normalised over cells
# ----------------------------------------------------------------------------------------------
def norms(err, weight=None):
    e = np.abs(np.asarray(err, dtype=np.float64)).ravel()
    if weight is None:
        weight = np.ones_like(e)
    wgt = np.asarray(weight, dtype=np.float64).ravel()
    wgt = wgt / wgt.sum()
    return float((wgt * e).sum()), float(np.sqrt((wgt * e * e).sum())), float(e.max())


def rate(e_coarse, e_fine):
    return math.log2(e_coarse / e_fine)
