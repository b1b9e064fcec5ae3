"""Manufactured-solution convergence of the oracle's EB operators (Eq. implicit-viscous with the
wall flux of Eq. dudn; the explicit term of Eq. explicit-viscous; the convective term).

u*(x) = (|x-c|^2 - r^2) sin(pi x) sin(pi y) sin(pi z) vanishes on the sphere and on the domain
walls; with a smooth prescribed viscosity, solving (alpha rho - dt L) u = alpha f with
f = rho u* - dt div(eta grad u*) must converge to u* at second order in L1 and L2 over the open
cells (cut-cell truncation errors are O(1) but confined to a surface).
"""
import math

import numpy as np

import analytic as A
import eb_inputs as I

C0, R0 = 0.5, 0.2


def fields(n):
    h = 1.0 / n
    z, y, x = np.meshgrid((np.arange(n) + 0.5) * h, (np.arange(n) + 0.5) * h,
                          (np.arange(n) + 0.5) * h, indexing="ij")
    return x, y, z


def exact(x, y, z, amp):
    pi = math.pi
    phi = (x - C0) ** 2 + (y - C0) ** 2 + (z - C0) ** 2 - R0 ** 2
    sx, sy, sz = np.sin(pi * x), np.sin(pi * y), np.sin(pi * z)
    cx, cy, cz = np.cos(pi * x), np.cos(pi * y), np.cos(pi * z)
    psi = sx * sy * sz
    gpsi = [pi * cx * sy * sz, pi * sx * cy * sz, pi * sx * sy * cz]
    gphi = [2 * (x - C0), 2 * (y - C0), 2 * (z - C0)]
    u = amp * phi * psi
    gu = [amp * (psi * gphi[d] + phi * gpsi[d]) for d in range(3)]
    lap = amp * (6 * psi + 2 * sum(gphi[d] * gpsi[d] for d in range(3)) - 3 * pi * pi * phi * psi)
    return u, gu, lap


def eta_field(x, y, z):
    s = x + 2 * y + 3 * z
    return 1.0 + 0.5 * np.cos(s), [-0.5 * np.sin(s), -1.0 * np.sin(s), -1.5 * np.sin(s)]


def test_viscous_solve_second_order(oracle_lib):
    O = oracle_lib
    rho, dt = 1.0, 1.0
    amps = (1.0, -0.7, 0.4)
    errs = []
    for n in (16, 32, 64):
        w = I.sphere_n(n, wall_u=[[0.0, 0.0, 0.0] for _ in range(6)], noise=0.0)
        g = O.Geometry(w)
        assert g.err == 0
        _, alpha, _ = g.export()
        cell, data = g.cut()
        x, y, z = fields(n)
        eta, geta = eta_field(x, y, z)
        # viscosity at the EB centroids
        cz, rem = np.divmod(cell, n * n)
        cy, cx = np.divmod(rem, n)
        xb = [(cx + 0.5) / n + data[:, 4] / n, (cy + 0.5) / n + data[:, 5] / n,
              (cz + 0.5) / n + data[:, 6] / n]
        eta_eb, _ = eta_field(*xb)
        ue = np.zeros((3,) + g.shape)
        psi = np.zeros((3,) + g.shape)
        for j in range(3):
            u, gu, lap = exact(x, y, z, amps[j])
            ue[j] = u
            psi[j] = rho * u - dt * (eta * lap + sum(geta[d] * gu[d] for d in range(3)))
        sol, it = g.visc_solve(rho, dt, np.ascontiguousarray(eta), eta_eb, psi,
                               np.zeros_like(psi), O.make_opts(w))
        m = alpha > 0
        e = np.abs(sol - ue)[:, m].max(axis=0)
        errs.append(A.norms(e, alpha[m]))
    r = [[A.rate(errs[i][k], errs[i + 1][k]) for k in range(3)] for i in range(2)]
    assert r[1][0] > 1.8 and r[1][1] > 1.8, (errs, r)
    assert r[1][2] > 1.0, (errs, r)


def test_transpose_term_vanishes_for_solenoidal_newtonian(oracle_lib):
    """div(mu (grad u)^T) = mu grad(div u) = 0 for a divergence-free field: O(h^2) discretely."""
    O = oracle_lib
    errs = []
    for n in (16, 32, 64):
        w = I.Workload(name="tg", n=(n, n, 4), h=1.0 / n, periodic=(1, 1, 1))
        g = O.Geometry(w)
        x, y, z = np.meshgrid((np.arange(n) + 0.5) / n, (np.arange(n) + 0.5) / n,
                              (np.arange(4) + 0.5) / n, indexing="ij")
        x, y = x.transpose(2, 1, 0), y.transpose(2, 1, 0)
        u = np.zeros((3,) + g.shape)
        u[0] = np.sin(2 * np.pi * x) * np.cos(2 * np.pi * y)
        u[1] = -np.cos(2 * np.pi * x) * np.sin(2 * np.pi * y)
        V = g.transpose_term(np.ones(g.shape), np.zeros(1), np.ascontiguousarray(u))
        errs.append(np.abs(V).max())
    assert A.rate(errs[0], errs[1]) > 1.9 and A.rate(errs[1], errs[2]) > 1.9, errs


def test_convective_term_taylor_green(oracle_lib):
    """Taylor-Green (Eq. taylor-green): u.grad u = -grad p_TG, compared cellwise; the
    limited-upwind scheme converges at close to second order in L1."""
    O = oracle_lib
    errs = []
    for n in (16, 32, 64):
        w = I.Workload(name="tg", n=(n, n, 4), h=1.0 / n, periodic=(1, 1, 1))
        g = O.Geometry(w)
        zz, yy, xx = np.meshgrid((np.arange(4) + 0.5) / n, (np.arange(n) + 0.5) / n,
                                 (np.arange(n) + 0.5) / n, indexing="ij")
        u = np.zeros((3,) + g.shape)
        u[0] = np.sin(2 * np.pi * xx) * np.cos(2 * np.pi * yy)
        u[1] = -np.cos(2 * np.pi * xx) * np.sin(2 * np.pi * yy)
        rh = O.make_rheo(w)
        Cv, eta, eta_eb, V = g.derived(np.ascontiguousarray(u), rh, O.make_opts(w))
        # -u.grad u for Taylor-Green: C = (pi sin(4 pi x)/2... ) = grad(p) with
        # p = (cos(4 pi x) + cos(4 pi y))/4  ->  C = -grad(-p) ... evaluated directly:
        cx = -np.pi * np.sin(4 * np.pi * xx)
        cy = -np.pi * np.sin(4 * np.pi * yy)
        e = np.abs(Cv[0] - cx) + np.abs(Cv[1] - cy) + np.abs(Cv[2])
        errs.append(A.norms(e))
    r1 = A.rate(errs[1][0], errs[2][0])
    assert r1 > 1.7, errs
