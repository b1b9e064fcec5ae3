"""Oracle pins for the nodal projection (Sec. III.A.4, Alg. advance NodalProjection; readings N1-N6).

What fixes each operator without retyping it:
* D and G are adjoint: <D(w), q> over the nodes equals sum_c alpha_c h^3 <w_c, G(q)_c> (the weak
  divergence is the transpose of the cell-averaged gradient in the volume-weighted inner
  product), exactly up to rounding;
* the patch test of the finite elements: for a linear q the stiffness matrix gives the weak
  divergence of its constant gradient, L q = D(G q), at every node, cut cells and walls included;
* L is symmetric, annihilates constants and is positive on mean-free fields;
* the discrete divergence theorem: with no net flux through the walls, the sum of D(w) - B over
  the nodes vanishes;
* the projection of a smooth field returns its solenoidal part at second order in h, and a pure
  gradient is removed at second order;
* in the plane Poiseuille flow between face-aligned walls the projection does nothing, so the
  whole step keeps the exact Delta x^2/4 errors of Table convergence:bingham (z0 = 0).
"""
import math

import numpy as np
import pytest

import eb_inputs as I


def _unique(g, a):
    """the nodal array without the periodic copies (last node of a periodic direction)"""
    nz, ny, nx = g.node_shape
    px, py, pz = g.w.periodic
    return a[: nz - pz, : ny - py, : nx - px]


def _workloads():
    w1 = I.sphere_n(16, radius=0.27)
    w2 = I.channel64(n=16, nxy=8)
    w3 = I.cylinder(8)
    return [w1, w2, w3]


@pytest.mark.parametrize("k", [0, 1, 2])
def test_divergence_is_the_transpose_of_the_gradient(oracle_lib, k):
    O = oracle_lib
    w = _workloads()[k]
    g = O.Geometry(w)
    _, alpha, _ = g.export()
    rng = np.random.default_rng(3)
    wf = rng.standard_normal((3,) + g.shape)
    q = rng.standard_normal(g.node_shape)
    # periodic copies hold the first node's value
    if w.periodic[0]:
        q[:, :, -1] = q[:, :, 0]
    if w.periodic[1]:
        q[:, -1, :] = q[:, 0, :]
    if w.periodic[2]:
        q[-1, :, :] = q[0, :, :]
    lhs = np.sum(_unique(g, g.nodal_div(wf)) * _unique(g, q))
    gq = g.nodal_grad(q)
    rhs = np.sum(alpha[None] * w.h ** 3 * wf * gq)
    assert abs(lhs - rhs) <= 1e-13 * np.sum(np.abs(alpha[None] * w.h ** 3 * wf * gq))


@pytest.mark.parametrize("k", [0, 1, 2])
def test_patch_test_linear_fields(oracle_lib, k):
    O = oracle_lib
    w = _workloads()[k]
    g = O.Geometry(w)
    nz, ny, nx = g.node_shape
    z, y, x = np.meshgrid(np.arange(nz) * w.h, np.arange(ny) * w.h, np.arange(nx) * w.h,
                          indexing="ij")
    a = np.array([0.7, -1.3, 0.4])
    for d in range(3):  # a periodic direction admits no linear field across the seam
        if w.periodic[d]:
            a[d] = 0.0
    q = a[0] * x + a[1] * y + a[2] * z + 0.25
    Lq = g.nodal_apply(q)
    _, alpha, _ = g.export()
    gq = g.nodal_grad(q)
    open_ = alpha > 0
    for d in range(3):  # the cell gradient of a linear field is its gradient
        assert np.allclose(gq[d][open_], a[d], rtol=0, atol=1e-12 * (np.abs(a).max()))
    DGq = g.nodal_div(gq)
    scale = np.abs(Lq).max() + np.abs(DGq).max()
    assert np.abs(Lq - DGq).max() <= 1e-12 * scale


def test_stiffness_symmetric_positive_with_constant_null_space(oracle_lib):
    O = oracle_lib
    w = _workloads()[0]
    g = O.Geometry(w)
    rng = np.random.default_rng(5)
    xa = rng.standard_normal(g.node_shape)
    ya = rng.standard_normal(g.node_shape)
    Lx, Ly = g.nodal_apply(xa), g.nodal_apply(ya)
    assert abs(np.sum(Lx * ya) - np.sum(xa * Ly)) <= 1e-13 * np.sum(np.abs(Lx * ya))
    L1 = g.nodal_apply(np.ones(g.node_shape))
    assert np.abs(L1).max() <= 1e-13 * np.abs(Lx).max()
    xm = xa - xa.mean()
    assert np.sum(xm * g.nodal_apply(xm)) > 0.0


def test_discrete_divergence_theorem(oracle_lib):
    """sphere32: walls move at (0,0,-1), so the flux in through the top equals the flux out
    through the bottom; the nodal divergence minus the boundary flux sums to zero."""
    O = oracle_lib
    w = I.sphere32()
    g = O.Geometry(w)
    u = I.initial_velocity(w) + 0.05 * I.random_field((3,) + g.shape, 9)
    d = g.nodal_div(u)
    b = g.nodal_bflux()
    assert abs(np.sum(b)) <= 1e-13 * np.sum(np.abs(b))
    assert abs(np.sum(d - b)) <= 1e-12 * np.sum(np.abs(d) + np.abs(b))


def _tg_fields(n):
    """A periodic box (x, y periodic on the unit square, 4 cells along z, periodic): the
    Taylor-Green velocity (solenoidal) and the gradient of Q = 0.3 sin(2 pi x) sin(4 pi y)."""
    w = I.taylor_green(n).replace(n=(n, n, 4))
    h = w.h
    xc = (np.arange(n) + 0.5) * h
    Y, X = np.meshgrid(xc, xc, indexing="ij")
    tg = np.zeros((3, 4, n, n))
    tg[0] = (np.sin(2 * math.pi * X) * np.cos(2 * math.pi * Y))[None]
    tg[1] = (-np.cos(2 * math.pi * X) * np.sin(2 * math.pi * Y))[None]
    gq = np.zeros_like(tg)
    gq[0] = (0.3 * 2 * math.pi * np.cos(2 * math.pi * X) * np.sin(4 * math.pi * Y))[None]
    gq[1] = (0.3 * 4 * math.pi * np.sin(2 * math.pi * X) * np.cos(4 * math.pi * Y))[None]
    return w, tg, gq


def test_projection_second_order(oracle_lib):
    O = oracle_lib
    err_sol, err_grad = [], []
    for n in (16, 32, 64):
        w, tg, gq = _tg_fields(n)
        g = O.Geometry(w)
        opts = O.make_opts(w, rtol=1e-13, max_iter=4000)
        pn = np.zeros(g.node_shape)
        u, _, _, _ = g.nodal_project(tg + gq, pn, 1.0, opts)
        err_sol.append(np.abs(u - tg).max())
        v, _, _, _ = g.nodal_project(gq, np.zeros(g.node_shape), 1.0, opts)
        err_grad.append(np.abs(v).max())
    r1 = [math.log2(err_sol[i] / err_sol[i + 1]) for i in range(2)]
    r2 = [math.log2(err_grad[i] / err_grad[i + 1]) for i in range(2)]
    print("nodal projection errors", err_sol, err_grad, "rates", r1, r2)
    assert min(r1) > 1.8 and min(r2) > 1.8
    amp = np.abs(gq).max()  # of the last (64^2 x 4) field
    assert err_sol[-1] < 2e-3 * amp and err_grad[-1] < 2e-3 * amp


@pytest.mark.parametrize("N", [16, 32])
def test_poiseuille_table_with_nodal_projection(oracle_lib, N):
    """Newtonian plane Poiseuille between face-aligned walls (the setting of the cell-centred pin
    in test_oracle_poiseuille.py): with the nodal projection in the step the steady error norms
    are still Delta x^2/4, the z0 = 0 rows of Table convergence:bingham, which the paper computed
    with its nodal projection."""
    import analytic as A
    from goldens import table

    O = oracle_lib
    W, G, mu = 0.5, 1.0, 1.0
    U = G * W * W / (2 * mu)
    w = I.Workload(name="poiseuille", n=(4, 4, N), h=1.0 / N, periodic=(1, 1, 0),
                   law=I.LAW_NEWTONIAN, mu=mu, rho=1.0, dt=1e3, force=(G, 0.0, 0.0))
    g = O.Geometry(w)
    opts = O.make_opts(w, rtol=1e-12, projection=O.PROJ_NODAL)
    rh = O.make_rheo(w)
    u = np.zeros((3,) + g.shape)
    pn = np.zeros(g.node_shape)
    for _ in range(3000):
        u1, pn, _ = g.rk2_step(u, pn, rh, w.dt, opts)
        du = np.abs(u1 - u).max()
        u = u1
        if du < 1e-15 * U:
            break
    zh = ((np.arange(N) + 0.5) / N - 0.5) / W
    err = u[0, :, 0, 0] / U - (1 - zh ** 2)
    tab = table("poiseuille_convergence.txt")
    row = tab[(tab[:, 0] == 0) & (tab[:, 1] == N)][0]
    nm = A.norms(err)
    for k in range(3):
        assert abs(nm[k] - row[2 + k]) <= 5e-12
    assert np.abs(u[1:]).max() < 1e-14
