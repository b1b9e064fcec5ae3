"""Oracle pins for the time-step rule (Sec. II.C.1, Eqs. cfl:dt, cfl:convective, cfl:forcing,
cfl:viscous:new): each constraint alone reduces Eq. cfl:dt to its own classical limit, the
combination lies between the largest single constraint and their sum, and the viscous
coefficient is Kang's for a Newtonian fluid and the Bingham-number-scaled one otherwise."""
import numpy as np
import pytest

import eb_inputs as I


@pytest.fixture(scope="module")
def geo(oracle_lib):
    O = oracle_lib
    w = I.sphere_n(32, 0.2)
    g = O.Geometry(w)
    _, alpha, _ = g.export()
    return O, w, g, alpha > 0


def rheo(O, law, mu, tau0, rho=1.0, eps=1e-6):
    w = I.sphere32().replace(law=law, mu=mu, tau0=tau0, rho=rho, eps=eps)
    return O.make_rheo(w)


def test_viscous_limit(geo):
    O, w, g, op = geo
    u = np.zeros((3,) + g.shape)
    h = w.h
    for law, tau0, bi in [(I.LAW_NEWTONIAN, 5.0, 0.0), (I.LAW_BINGHAM_REG, 10.0, 10.0),
                          (I.LAW_PAPANASTASIOU, 2.0, 2.0)]:
        for mu, rho in [(1.0, 1.0), (0.5, 4e-3)]:
            dt = g.stable_dt(u, rheo(O, law, mu, tau0, rho), c_cfl=0.5)
            # C_C = C_F = 0: dt = C_CFL / C_V, C_V = 2 mu (Bi + 1) / rho * 3 / h^2; for a
            # Newtonian fluid that is Kang's coefficient with eta = mu
            assert dt == pytest.approx(0.5 * rho * h * h / (6.0 * mu * (bi + 1.0)), rel=1e-14)


def test_convective_and_forcing_limits(geo):
    O, w, g, op = geo
    h = w.h
    u = np.zeros((3,) + g.shape)
    idx = np.argwhere(op)
    c0, c1 = tuple(idx[0]), tuple(idx[len(idx) // 2])
    u[0][c0], u[1][c0], u[2][c0] = 0.3, -0.2, 0.1      # |u|+|v|+|w| = 0.6
    u[2][c1] = -0.5
    covered = tuple(np.argwhere(~op)[0])
    u[0][covered] = 50.0                                # covered cells do not count
    r0 = rheo(O, I.LAW_NEWTONIAN, 0.0, 0.0)             # no viscous constraint
    assert g.stable_dt(u, r0, c_cfl=0.7) == pytest.approx(0.7 * h / 0.6, rel=1e-14)
    z = np.zeros_like(u)
    f = (0.0, -2.0, 1.0)
    assert g.stable_dt(z, r0, force=f, c_cfl=0.5) == pytest.approx(0.5 * np.sqrt(h / 3.0),
                                                                   rel=1e-14)


def test_combination_bounds(geo):
    O, w, g, op = geo
    h = w.h
    u = I.initial_velocity(w)
    u = u + 0.1 * I.random_field(u.shape, seed=5)
    f = (1.0, 0.0, 0.0)
    r = rheo(O, I.LAW_BINGHAM_REG, 1.0, 1.0)
    dt = g.stable_dt(u, r, force=f, c_cfl=0.5)
    cc = (np.abs(u).sum(axis=0)[op]).max() / h
    cv = 2.0 * 2.0 * 3.0 / (h * h)
    cf = np.sqrt(1.0 / h)
    # 1/dt = (1/2)(a + sqrt(a^2 + 4 b^2)) / C_CFL with a = C_C + C_V, b = C_F lies in
    # [max(a, b), a + b]
    a = cc + cv
    assert 0.5 / (a + cf) <= dt <= 0.5 / max(a, cf)
    # doubling mu doubles C_V: the bounds move with a = C_C + 2 C_V and dt shrinks
    r2 = rheo(O, I.LAW_BINGHAM_REG, 2.0, 1.0)
    dt2 = g.stable_dt(u, r2, force=f, c_cfl=0.5)
    assert 0.5 / (a + cv + cf) <= dt2 <= 0.5 / max(a + cv, cf)
    assert dt2 < dt


def test_yield_stress_field_counts_open_cells_only(geo):
    O, w, g, op = geo
    u = np.zeros((3,) + g.shape)
    theta = np.ones(g.shape)
    theta[tuple(np.argwhere(~op)[0])] = 100.0           # covered: ignored
    theta[tuple(np.argwhere(op)[3])] = 1.5              # largest open value
    r = rheo(O, I.LAW_BINGHAM_REG, 1.0, 4.0)
    dt = g.stable_dt(u, r, theta=theta, c_cfl=0.5)
    assert dt == pytest.approx(0.5 * w.h ** 2 / (6.0 * (4.0 * 1.5 + 1.0)), rel=1e-14)


def test_bench_workload_exceeds_the_rule(oracle_lib):
    """The 128^3 sphere's dt = 5e-4 with rho = 4e-3 and Bi = 10 is about 2.7e5 times the rule's
    (the viscous coefficient dominates: 2 (Bi + 1) / rho * 3 * 128^2 = 2.7e8)."""
    O = oracle_lib
    w = I.sphere128()
    r = O.make_rheo(w)
    g = O.Geometry(I.sphere_n(32, 0.125).replace(rho=4e-3, tau0=10.0))
    u = np.zeros((3,) + g.shape)
    u[2] = -1.0
    dt32 = g.stable_dt(u, r, c_cfl=0.5)
    # at 128^3 every coefficient scales as computed from the 32^3 ones: C_V by 16, C_C by 4
    h32 = 1.0 / 32
    cv32 = 2.0 * 11.0 / 4e-3 * 3.0 / h32 ** 2
    cc32 = 1.0 / h32
    assert dt32 == pytest.approx(0.5 / (cc32 + cv32), rel=1e-12)
    dt128 = 0.5 / (4 * cc32 + 16 * cv32)
    assert 2.6e5 < w.dt / dt128 < 2.8e5
