"""Oracle pins from invariants of the method and from brute force.

* Redistribution conserves sum(alpha D) (Eqs. divergence_excess, weights, divergence_final).
* Both projections leave a face field whose divergence is at the solver tolerance, and
  projecting twice changes nothing (Eq. helmholtz; end-of-stage projection).
* The Krylov + multigrid solvers agree with a dense direct solve of the assembled operators,
  and the V-cycle used as the CG preconditioner is symmetric.
* Channel with EB walls on cell centres (Newtonian): the parabola is an exact discrete steady
  state of the full RK2 step, and the wall drag balances the body force.
* tau0 = 0 reproduces the Newtonian step bitwise; the noiseless sphere flow keeps the mirror
  symmetries of the geometry.
"""
import numpy as np
import pytest

import eb_inputs as I


def test_redistribution_conserves(oracle_lib):
    O = oracle_lib
    w = I.sphere32()
    g = O.Geometry(w)
    _, alpha, _ = g.export()
    DC = I.random_field((3,) + g.shape, 11)
    DC[:, alpha == 0] = 0.0
    D = g.redistribute(DC)
    for j in range(3):
        lhs = (alpha * D[j]).sum()
        rhs = (alpha * DC[j]).sum()
        assert abs(lhs - rhs) <= 1e-12 * np.abs(alpha * DC[j]).sum()
    # without an embedded body redistribution is the identity
    w0 = I.Workload(name="box", n=(8, 8, 8), h=1 / 8)
    g0 = O.Geometry(w0)
    d0 = I.random_field((3, 8, 8, 8), 12)
    assert np.array_equal(g0.redistribute(d0), d0)


def test_mac_projection_divergence_and_idempotence(oracle_lib):
    O = oracle_lib
    w = I.sphere32()
    g = O.Geometry(w)
    opts = O.make_opts(w)
    faces = I.random_faces(w.n, 7)
    # no net flux through the (Neumann) domain walls, so the problem is compatible
    faces[0][:, :, [0, -1]] = 0.0
    faces[1][:, [0, -1], :] = 0.0
    faces[2][[0, -1], :, :] = 0.0
    f1, phi, div, it = g.mac_project(faces, 1.0, opts)
    scale = max(np.abs(f).max() for f in faces) / w.h
    assert div <= 2e-12 * scale * 6 and it > 0
    assert np.abs(g.divergence(f1)).max() == pytest.approx(div, rel=1e-12)
    f2, phi2, div2, it2 = g.mac_project(f1, 1.0, opts)
    assert max(np.abs(a - b).max() for a, b in zip(f1, f2)) <= 1e-10 * max(
        np.abs(a).max() for a in f1)


def test_cc_projection(oracle_lib):
    O = oracle_lib
    w = I.sphere32()
    g = O.Geometry(w)
    opts = O.make_opts(w)
    u = I.initial_velocity(w)
    p0 = np.zeros(g.shape)
    u1, p1, div, it = g.cc_project(u, p0, 0.5, opts)
    assert div <= 1e-11 * (np.abs(u).max() / w.h)
    _, alpha, _ = g.export()
    assert abs(p1[alpha > 0].mean()) < 1e-12
    # the cell correction is the averaged face gradient of the new pressure
    gp = g.gcc(p1)
    assert np.abs((u1 - (u - 0.5 * gp))[:, alpha > 0]).max() <= 1e-14
    # with the pressure added back, the same face field projects to the same pressure
    u2, p2, _, _ = g.cc_project(u1, p1, 0.5, opts)
    assert np.abs(p2 - p1).max() <= 1e-9 * np.abs(p1).max()


def dense(apply, n):
    M = np.zeros((n, n))
    e = np.zeros(n)
    for c in range(n):
        e[:] = 0
        e[c] = 1
        M[:, c] = apply(e)
    return M


def test_solvers_match_dense(oracle_lib):
    O = oracle_lib
    w = I.Workload(name="tiny", n=(12, 12, 12), h=1 / 12, wall_u=[[0.2, -0.1, 0.4]] * 6,
                   body={"kind": I.BODY_SPHERE, "center": (0.5, 0.5, 0.5), "radius": 2.5 / 12})
    g = O.Geometry(w)
    assert g.err == 0 and g.ncut > 0
    opts = O.make_opts(w, rtol=1e-13)
    _, alpha, _ = g.export()
    m = (alpha > 0).ravel()
    N = g.N
    rng = np.random.default_rng(0)
    eta = np.ascontiguousarray(1.0 + rng.uniform(0, 50, g.shape))
    eta_eb = 1.0 + rng.uniform(0, 5, g.ncut)
    rho, dt = 0.7, 0.01
    # viscous: component-wise the same scalar operator; dense over the open cells
    def apply_scalar(x):
        u = np.zeros((3, N))
        u[0] = x
        return g.visc_apply(rho, dt, eta, eta_eb, u.reshape((3,) + g.shape),
                            homogeneous=True)[0].ravel()
    A = dense(apply_scalar, N)[np.ix_(m, m)]
    psi = I.random_field((3,) + g.shape, 4)
    x, it = g.visc_solve(rho, dt, eta, eta_eb, psi, np.zeros((3,) + g.shape), opts)
    b0 = g.visc_apply(rho, dt, eta, eta_eb, np.zeros((3,) + g.shape))
    for j in range(3):
        b = (alpha * psi[j]).ravel()[m] - b0[j].ravel()[m]
        xd = np.linalg.solve(A, b)
        assert np.abs(x[j].ravel()[m] - xd).max() <= 1e-10 * np.abs(xd).max()
    # Poisson (singular, symmetric): compare modulo constants
    P = dense(lambda v: g.poisson_apply(0.3, v.reshape(g.shape)).ravel(), N)[np.ix_(m, m)]
    assert np.abs(P - P.T).max() < 1e-12 * np.abs(P).max()
    faces = I.random_faces(w.n, 9)
    f1, phi, div, it = g.mac_project(faces, 0.3, opts)
    div0 = g.divergence(faces).ravel()[m]
    b = -(div0 - div0.mean())
    pd = np.linalg.lstsq(P, b, rcond=None)[0]
    pd -= pd.mean()
    assert np.abs(phi.ravel()[m] - pd).max() <= 1e-9 * np.abs(pd).max()


def test_vcycle_symmetric(oracle_lib):
    O = oracle_lib
    w = I.sphere32()
    g = O.Geometry(w)
    opts = O.make_opts(w)
    _, alpha, _ = g.export()
    a = I.random_field(g.shape, 1) * (alpha > 0)
    b = I.random_field(g.shape, 2) * (alpha > 0)
    Va = g.vcycle(0, a, opts, beta=0.4)
    Vb = g.vcycle(0, b, opts, beta=0.4)
    assert abs((Va * b).sum() - (a * Vb).sum()) <= 1e-12 * abs((Va * b).sum())
    assert (Va * a).sum() > 0


def channel_workload(n=64):
    return I.Workload(name="channel", n=(4, 4, n), h=1.0 / n, periodic=(1, 1, 0),
                      body={"kind": I.BODY_ZSLAB, "zlo": 0.1171875, "zhi": 0.8828125},
                      law=I.LAW_PAPANASTASIOU, mu=1.0, tau0=0.0, eps=1e-8, rho=1.0, dt=1e-3,
                      force=(1.0, 0.0, 0.0))


def test_channel_parabola_is_steady(oracle_lib):
    O = oracle_lib
    w = channel_workload()
    g = O.Geometry(w)
    zlo, zhi = 0.1171875, 0.8828125
    zc = (np.arange(64) + 0.5) * w.h
    prof = np.where((zc >= zlo) & (zc <= zhi), 0.5 * (zc - zlo) * (zhi - zc), 0.0)
    u = np.zeros((3,) + g.shape)
    u[0] = prof[:, None, None]
    p = np.zeros(g.shape)
    opts = O.make_opts(w)
    u1, p1, st = g.rk2_step(u, p, O.make_rheo(w), 0.25, opts)
    assert np.abs(u1 - u).max() <= 1e-11 * prof.max()
    assert np.abs(p1).max() <= 1e-12
    # drag balances the body force: F_x = f * fluid volume
    F = g.drag(u1, p1, O.make_rheo(w))
    vol = (zhi - zlo) * (4 * w.h) * (4 * w.h)
    assert F[0] == pytest.approx(1.0 * vol, rel=1e-10)
    assert abs(F[1]) < 1e-14 and abs(F[2]) < 1e-12


def test_tau0_zero_matches_newtonian_step(oracle_lib):
    O = oracle_lib
    w = I.sphere32()
    g = O.Geometry(w)
    u, p = O.prepare_state(w, g)
    opts = O.make_opts(w)
    ua, pa, _ = g.rk2_step(u, p, O.make_rheo(w, tau0=0.0), w.dt, opts)
    ub, pb, _ = g.rk2_step(u, p, O.make_rheo(w.replace(law=I.LAW_NEWTONIAN)), w.dt, opts)
    assert np.array_equal(ua, ub) and np.array_equal(pa, pb)


def test_sphere_step_symmetry(oracle_lib):
    O = oracle_lib
    w = I.sphere32().replace(noise=0.0)
    g = O.Geometry(w)
    u = I.initial_velocity(w)
    p = np.zeros(g.shape)
    u1, p1, st = g.rk2_step(u, p, O.make_rheo(w), w.dt, O.make_opts(w))
    tol = 1e-9 * np.abs(u1).max()
    # mirror in x: u_x odd, u_y and u_z even (array axes are z, y, x)
    assert np.abs(u1[0] + np.flip(u1[0], 2)).max() < tol
    assert np.abs(u1[1] - np.flip(u1[1], 2)).max() < tol
    assert np.abs(u1[2] - np.flip(u1[2], 2)).max() < tol
    # swapping x and y maps u_x <-> u_y
    assert np.abs(u1[0] - u1[1].transpose(0, 2, 1)).max() < tol
    assert np.abs(p1 - np.flip(p1, 2)).max() < 1e-9 * np.abs(p1).max()
