"""Pins of the oracle's reverse mode (adjoint of the RK2 step and of the drag).

The adjoint is fixed by the forward map: for every linear piece <ybar, J v> = <J^T ybar, v>
must hold to rounding for random v, ybar (dot-product test), and for the nonlinear pieces the
adjoint must agree with central finite differences of the forward oracle.  The forward oracle is
pinned to the paper by the other oracle tests, so these tests tie the adjoint to the paper too.
Random directions are seeded; covered cells are excluded (the step never reads them).
"""
import numpy as np
import pytest

import eb_inputs as I


def _rel(a, b):
    return abs(a - b) / max(abs(a), abs(b), 1e-300)


@pytest.fixture(scope="module")
def sph(oracle_lib):
    O = oracle_lib
    w = I.sphere_n(16, 0.25)
    g = O.Geometry(w)
    _, alpha, _ = g.export()
    opts = O.make_opts(w, rtol=1e-14, max_iter=1000)
    rh = O.make_rheo(w)
    u0, p0 = O.prepare_state(w, g, opts)
    u0, p0, _ = g.rk2_step(u0, p0, rh, w.dt, opts)  # developed pressure
    theta = I.yield_field(w)
    return dict(O=O, w=w, g=g, open=alpha > 0, opts=opts, rh=rh, u0=u0, p0=p0, theta=theta)


def _rnd(s, shape, seed):
    a = I.rng(seed).standard_normal(shape)
    if len(shape) == 4:
        a[:, ~s["open"]] = 0.0
    elif len(shape) == 3:
        a[~s["open"]] = 0.0
    return a


def test_linear_pieces_dot_product(sph):
    s = sph
    g, u0, p0 = s["g"], s["u0"], s["p0"]
    v3 = (3,) + g.shape
    v = _rnd(s, v3, 1)
    # wall gradient (Eq. dudn): affine in u
    gb = I.rng(2).standard_normal((g.ncut, 3))
    J = g.wall_gradient(u0 + v) - g.wall_gradient(u0)
    assert _rel((gb * J).sum(), (g.wall_gradient_adj(gb) * v).sum()) < 1e-12
    # one-sided cell gradients: linear in (u, wall gradient)
    gw0 = g.wall_gradient(u0)
    dgw = I.rng(3).standard_normal((g.ncut, 3))
    Gb = _rnd(s, (3, 3) + g.shape, 4)
    J = g.cell_gradient_from(u0 + v, gw0 + dgw) - g.cell_gradient_from(u0, gw0)
    ub, gwb = g.cell_gradient_adj(Gb)
    assert _rel((Gb * J).sum(), (ub * v).sum() + (gwb * dgw).sum()) < 1e-12
    # redistribution (Eqs. divergence_nonconservative ... divergence_final): linear
    DC, Db = _rnd(s, v3, 5), _rnd(s, v3, 6)
    assert _rel((Db * g.redistribute(DC)).sum(), (g.redistribute_adj(Db) * DC).sum()) < 1e-12
    # cell-centred pressure gradient: linear
    pp, gpb = _rnd(s, g.shape, 7), _rnd(s, v3, 8)
    assert _rel((gpb * g.gcc(pp)).sum(), (g.gcc_adj(gpb) * pp).sum()) < 1e-12


@pytest.mark.parametrize("case", ["sphere", "periodic_channel"])
def test_projections_dot_product(oracle_lib, sph, case):
    """Both projections are affine maps once the Poisson solve is exact (rtol 1e-14).  The
    periodic channel stores the faces on the periodic seams twice."""
    s = sph
    if case == "periodic_channel":
        O = oracle_lib
        w = I.channel64(tau0=0.0, n=16, nxy=8)
        g = O.Geometry(w)
        _, alpha, _ = g.export()
        opts = O.make_opts(w, rtol=1e-14, max_iter=1000)
        u0 = I.random_field((3,) + g.shape, 31)
        u0[:, alpha == 0] = 0.0
        s = dict(s, w=w, g=g, open=alpha > 0, opts=opts, u0=u0, p0=np.zeros(g.shape))
    g, w, opts = s["g"], s["w"], s["opts"]
    fw, fv, fb = I.random_faces(w.n, 3), I.random_faces(w.n, 4), I.random_faces(w.n, 6)
    P1 = g.mac_project([a + b for a, b in zip(fw, fv)], 0.7, opts)[0]
    P0 = g.mac_project(fw, 0.7, opts)[0]
    lhs = sum((b * (x - y)).sum() for b, x, y in zip(fb, P1, P0))
    fa, _ = g.mac_project_adj(fb, 0.7, opts)
    assert _rel(lhs, sum((a * b).sum() for a, b in zip(fa, fv))) < 1e-11
    v3 = (3,) + g.shape
    uv, pv = _rnd(s, v3, 9), _rnd(s, g.shape, 10)
    ubar, pbar = _rnd(s, v3, 11), _rnd(s, g.shape, 12)
    ua, pa, _, _ = g.cc_project(s["u0"] + uv, s["p0"] + pv, 0.3, opts)
    ub, pb, _, _ = g.cc_project(s["u0"], s["p0"], 0.3, opts)
    lhs = (ubar * (ua - ub)).sum() + (pbar * (pa - pb)).sum()
    ui, pi, _ = g.cc_project_adj(ubar, pbar, 0.3, opts)
    assert _rel(lhs, (ui * uv).sum() + (pi * pv).sum()) < 1e-11


def test_face_extrap_adjoint_fd(sph):
    """Limited upwind face states: piecewise linear; a 1e-7 step flips no branch."""
    s = sph
    g, u0 = s["g"], s["u0"]
    v = _rnd(s, (3,) + g.shape, 13)
    fb = I.random_faces(s["w"].n, 14)
    e = 1e-7
    F1, F0 = g.face_extrap(u0 + e * v), g.face_extrap(u0 - e * v)
    lhs = sum((b * (x - y)).sum() for b, x, y in zip(fb, F1, F0)) / (2 * e)
    assert _rel(lhs, (g.face_extrap_adj(u0, fb) * v).sum()) < 1e-7


def test_visc_solve_adjoint_fd(sph):
    """Transposed BiCGSTAB solve and the viscosity derivative of the operator."""
    s = sph
    g, w, opts = s["g"], s["w"], s["opts"]
    eta, eta_eb = g.viscosity(s["u0"], s["rh"], s["theta"])
    psi = _rnd(s, (3,) + g.shape, 15)
    x, _ = g.visc_solve(w.rho, w.dt, eta, eta_eb, psi, s["u0"], opts)
    xb = _rnd(s, (3,) + g.shape, 16)
    psib, etab, etaebb, _ = g.visc_solve_adj(w.rho, w.dt, eta, eta_eb, x, xb, opts)
    dpsi = _rnd(s, (3,) + g.shape, 17)
    deta = 0.1 * _rnd(s, g.shape, 18)
    deb = 0.1 * I.rng(19).standard_normal(g.ncut)
    e = 1e-4
    xp, _ = g.visc_solve(w.rho, w.dt, eta + e * deta, eta_eb + e * deb, psi + e * dpsi, x, opts)
    xm, _ = g.visc_solve(w.rho, w.dt, eta - e * deta, eta_eb - e * deb, psi - e * dpsi, x, opts)
    lhs = (xb * (xp - xm)).sum() / (2 * e)
    rhs = (psib * dpsi).sum() + (etab * deta).sum() + (etaebb * deb).sum()
    assert _rel(lhs, rhs) < 1e-7


def _derived_loss(g, u, th, rh, opts, bars):
    Cb, etb, ebb, Vb = bars
    Cv, et, eb, V = g.derived(u, rh, opts, th)
    return (Cb * Cv).sum() + (etb * et).sum() + (ebb * eb).sum() + (Vb * V).sum()


# the power-law family of Table rheology on the channel: the cap of n < 1 kept out of reach
# (eps = 1e-12) where eps is not the yield regularisation; Herschel-Bulkley shear-thickening;
# Souza Mendes-Dutra with eta0 = tau0/0.05, so that eta0 |gamma|/tau0 spans the small-x series
_LAWS = {"power_channel": dict(law=I.LAW_POWER, kappa=1.3, flow_n=0.6, eps=1e-12),
         "herschel_bulkley_channel": dict(law=I.LAW_HERSCHEL_BULKLEY, kappa=0.9, flow_n=1.3),
         "smd_channel": dict(law=I.LAW_SOUZA_MENDES_DUTRA, kappa=1.1, flow_n=0.7, eps=1e-12,
                             eta0=0.8 / 0.05)}


@pytest.mark.parametrize("case", ["bingham_sphere", "papanastasiou_channel"] + list(_LAWS))
def test_derived_adjoint_fd(oracle_lib, sph, case):
    """Derived quantities (Alg. derived): velocity and per-cell yield-stress gradients."""
    O = oracle_lib
    if case == "bingham_sphere":
        s = sph
        g, rh, opts, u0, th = s["g"], s["rh"], s["opts"], s["u0"], s["theta"]
        op = s["open"]
    else:
        # Papanastasiou law with eps such that |gamma|/eps spans both sides of the small-x
        # series of the law derivative
        w = I.channel64(tau0=0.8, eps=0.05, n=16, nxy=8).replace(**_LAWS.get(case, {}))
        g = O.Geometry(w)
        _, alpha, _ = g.export()
        op = alpha > 0
        rh = O.make_rheo(w)
        opts = O.make_opts(w, rtol=1e-14, max_iter=1000)
        # noise whose amplitude falls by four decades along z
        env = 10.0 ** (-4.0 * np.arange(g.shape[0]) / g.shape[0])
        u0 = 0.02 * env[None, :, None, None] * I.random_field((3,) + g.shape, 20)
        u0[:, ~op] = 0.0
        th = I.yield_field(w)
        _, _, sr = g.viscosity(u0, rh, th, with_sr=True)
        scale = w.eta0 / w.tau0 if w.law == I.LAW_SOUZA_MENDES_DUTRA else 1.0 / w.eps
        x = sr[op] * scale
        if w.law != I.LAW_POWER:
            assert (x < 1e-2).any() and (x > 1e-2).any()
    r = I.rng(21)
    bars = [r.standard_normal((3,) + g.shape), r.standard_normal(g.shape),
            r.standard_normal(g.ncut), r.standard_normal((3,) + g.shape)]
    for b in (bars[0], bars[3]):
        b[:, ~op] = 0.0
    bars[1][~op] = 0.0
    ub, tau0b = g.derived_adj(u0, rh, opts, *bars, theta=th)
    v = r.standard_normal((3,) + g.shape)
    v[:, ~op] = 0.0
    if case != "bingham_sphere":
        v *= env[None, :, None, None]  # a perturbation small against the local velocity
    dth = r.standard_normal(g.shape)
    e = 1e-7
    lhs = (_derived_loss(g, u0 + e * v, th, rh, opts, bars)
           - _derived_loss(g, u0 - e * v, th, rh, opts, bars)) / (2 * e)
    assert _rel(lhs, (ub * v).sum()) < 1e-6
    e = 1e-6
    lhs = (_derived_loss(g, u0, th + e * dth, rh, opts, bars)
           - _derived_loss(g, u0, th - e * dth, rh, opts, bars)) / (2 * e)
    assert _rel(lhs, (tau0b * rh.tau0 * dth).sum()) < 1e-6


def test_newtonian_has_no_yield_gradient(oracle_lib, sph):
    s = sph
    g, w = s["g"], s["w"]
    rh = oracle_lib.make_rheo(w.replace(law=I.LAW_NEWTONIAN))
    ubar = _rnd(s, (3,) + g.shape, 22)
    _, _, tb, _ = g.rk2_step_adjoint(s["u0"], s["p0"], rh, w.dt, s["opts"], ubar,
                                     np.zeros(g.shape), s["theta"])
    assert np.all(tb == 0.0)


def test_rk2_step_adjoint_fd(sph):
    """Whole step (Alg. advance): adjoints of u^m, p^m and the per-cell yield stress."""
    s = sph
    g, w, opts, rh, th = s["g"], s["w"], s["opts"], s["rh"], s["theta"]
    u0, p0 = s["u0"], s["p0"]
    ubar, pbar = _rnd(s, (3,) + g.shape, 23), _rnd(s, g.shape, 24)
    ui, pi, tb, st = g.rk2_step_adjoint(u0, p0, rh, w.dt, opts, ubar, pbar, th)
    assert np.all(ui[:, ~s["open"]] == 0.0) and np.all(pi[~s["open"]] == 0.0)

    def L(u, p, t):
        a, b, _ = g.rk2_step(u, p, rh, w.dt, opts, t)
        return (ubar * a).sum() + (pbar * b).sum()

    v, q, dth = _rnd(s, (3,) + g.shape, 25), _rnd(s, g.shape, 26), _rnd(s, g.shape, 27)
    e = 1e-7
    assert _rel((L(u0 + e * v, p0, th) - L(u0 - e * v, p0, th)) / (2 * e), (ui * v).sum()) < 1e-6
    # p enters the predictor linearly and the step only through u* otherwise, so the response
    # to p is nearly linear: a larger step keeps the solvers' tolerance out of the difference
    e = 1e-5
    assert _rel((L(u0, p0 + e * q, th) - L(u0, p0 - e * q, th)) / (2 * e), (pi * q).sum()) < 1e-6
    e = 1e-6
    assert _rel((L(u0, p0, th + e * dth) - L(u0, p0, th - e * dth)) / (2 * e),
                (tb * rh.tau0 * dth).sum()) < 1e-6


def test_drag_adjoint_fd(sph):
    """Drag on the body (Eq. drag-force): linear in p, nonlinear in u through eta_EB."""
    s = sph
    g, rh, th = s["g"], s["rh"], s["theta"]
    u, p = s["u0"], s["p0"]
    Fb = np.array([0.3, -0.2, 1.0])
    ub, pb, tb = g.drag_adj(u, rh, Fb, th)

    def D(uu, pp, t):
        return (Fb * g.drag(uu, pp, rh, t)).sum()

    v, q, dth = _rnd(s, (3,) + g.shape, 28), _rnd(s, g.shape, 29), _rnd(s, g.shape, 30)
    e = 1e-6
    assert _rel((D(u + e * v, p, th) - D(u - e * v, p, th)) / (2 * e), (ub * v).sum()) < 1e-6
    assert _rel((D(u, p + e * q, th) - D(u, p - e * q, th)) / (2 * e), (pb * q).sum()) < 1e-6
    # the yield stress moves the drag by ~1e-3 of its size per unit theta: a 1e-6 step would
    # sit at the rounding floor eps |D| / (e |g|) ~ 1e-5, a 1e-3 step at ~1e-8
    e = 1e-3
    assert _rel((D(u, p, th + e * dth) - D(u, p, th - e * dth)) / (2 * e),
                (tb * rh.tau0 * dth).sum()) < 1e-6


def test_rollout_bingham_number_gradient_fd(oracle_lib, sph):
    """d(z-drag after 2 steps)/d(Bi): adjoint through two steps vs a central difference in Bi
    (relative step 1e-6), and a per-cell yield-stress gradient at cells next to the body."""
    O = oracle_lib
    s = sph
    g, w, opts, th = s["g"], s["w"], s["opts"], s["theta"]
    u0, p0 = s["u0"], s["p0"]
    nsteps = 2

    def fwd(tau0, theta):
        rh = O.make_rheo(w, tau0=tau0)
        us, ps = [u0], [p0]
        for _ in range(nsteps):
            a, b, _ = g.rk2_step(us[-1], ps[-1], rh, w.dt, opts, theta)
            us.append(a)
            ps.append(b)
        return us, ps, g.drag(us[-1], ps[-1], rh, theta)[2]

    bi = w.tau0
    us, ps, _ = fwd(bi, th)
    rh = O.make_rheo(w)
    ub, pb, tb = g.drag_adj(us[-1], rh, [0.0, 0.0, 1.0], th)
    for k in range(nsteps - 1, -1, -1):
        ub, pb, t, _ = g.rk2_step_adjoint(us[k], ps[k], rh, w.dt, opts, ub, pb, th)
        tb += t
    dbi = (th * tb).sum()
    e = 1e-6 * bi
    fd = (fwd(bi + e, th)[2] - fwd(bi - e, th)[2]) / (2 * e)
    assert _rel(fd, dbi) < 1e-5
    # one cut cell's yield stress
    cell, _ = g.cut()
    c = np.unravel_index(int(cell[len(cell) // 2]), g.shape)
    e = 1e-6 * th[c]
    tp, tm = th.copy(), th.copy()
    tp[c] += e
    tm[c] -= e
    fd = (fwd(bi, tp)[2] - fwd(bi, tm)[2]) / (2 * e)
    assert _rel(fd, bi * tb[c]) < 1e-4
