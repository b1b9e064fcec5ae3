"""Oracle pins for the power-law family of Table rheology (power law, Herschel-Bulkley, Souza
Mendes-Dutra), Sec. II.B.

* Values fixed by hand: on a uniform shear u = (gamma z, 0, 0) every cell's strain-rate norm is
  gamma exactly, so eta is the law's value at gamma, chosen where it is a short decimal.
* Reductions the table itself implies: n = 1 turns the power law into a Newtonian fluid of
  viscosity kappa and Herschel-Bulkley into the Papanastasiou-regularised Bingham law, bit for
  bit; tau0 = 0 leaves the power-law term; Souza Mendes-Dutra with eta0 = tau0/eps has the
  Papanastasiou exponent.
* The plane Poiseuille flow of a power-law fluid has the closed form
  u = n/(n+1) (G/kappa)^(1/n) (W^(1+1/n) - |z - zc|^(1+1/n)); the oracle's steady state
  converges to it at second order.
* The law derivatives of the adjoint: central differences of the oracle's derived quantities.
"""
import math

import numpy as np
import pytest

import eb_inputs as I


def _shear_box(gamma, n=(4, 4, 8)):
    nz = n[2]
    w = I.Workload(name="shear", n=n, h=1.0 / nz, periodic=(1, 1, 0), law=I.LAW_POWER)
    w.wall_u = [[0.0, 0.0, 0.0] for _ in range(6)]
    w.wall_u[5] = [gamma * 1.0, 0.0, 0.0]
    return w


def _eta_on_shear(O, gamma, **law):
    w = _shear_box(gamma).replace(**law)
    g = O.Geometry(w)
    z = (np.arange(w.n[2]) + 0.5) * w.h
    u = np.zeros((3,) + g.shape)
    u[0] = gamma * z[:, None, None]
    eta, _, sr = g.viscosity(u, O.make_rheo(w), with_sr=True)
    assert np.all(sr == gamma)
    return eta


@pytest.mark.parametrize("law,expect", [
    (dict(law=I.LAW_POWER, kappa=2.0, flow_n=0.5, eps=1e-3), 1.0),           # 2 * 4^-1/2
    (dict(law=I.LAW_POWER, kappa=2.0, flow_n=1.5, eps=1e-3), 4.0),           # 2 * 4^1/2
    (dict(law=I.LAW_HERSCHEL_BULKLEY, kappa=2.0, flow_n=0.5, tau0=1.0, eps=1e-3), 1.25),
    (dict(law=I.LAW_SOUZA_MENDES_DUTRA, kappa=2.0, flow_n=0.5, tau0=1.0,
          eta0=math.log(2.0) / 4.0, eps=1e-3), 1.125),                       # 1 + (1 - 1/2)/4
])
def test_uniform_shear_values(oracle_lib, law, expect):
    eta = _eta_on_shear(oracle_lib, 4.0, **law)
    assert np.allclose(eta, expect, rtol=1e-15, atol=0.0), (eta.min(), eta.max())


@pytest.mark.parametrize("law,expect", [
    (dict(law=I.LAW_POWER, kappa=2.0, flow_n=0.5, eps=1e-2), 20.0),          # 2 * (1e-2)^-1/2
    (dict(law=I.LAW_POWER, kappa=2.0, flow_n=1.5, eps=1e-2), 0.0),
    (dict(law=I.LAW_HERSCHEL_BULKLEY, kappa=2.0, flow_n=0.5, tau0=1.0, eps=1e-2), 120.0),
    (dict(law=I.LAW_SOUZA_MENDES_DUTRA, kappa=2.0, flow_n=0.5, tau0=1.0, eta0=3.0,
          eps=1e-2), 23.0),
])
def test_zero_strain_rate_limits(oracle_lib, law, expect):
    eta = _eta_on_shear(oracle_lib, 0.0, **law)
    assert np.allclose(eta, expect, rtol=1e-14, atol=0.0), (eta.min(), eta.max())


@pytest.fixture(scope="module")
def sph16(oracle_lib):
    O = oracle_lib
    w = I.sphere_n(16, 0.3).replace(eps=1e-3)
    g = O.Geometry(w)
    u, p = O.prepare_state(w, g)
    return w, g, u, p


def _step(O, g, w, u, p, **law):
    wl = w.replace(**law)
    return g.rk2_step(u, p, O.make_rheo(wl), wl.dt, O.make_opts(wl))


def test_flow_index_one_reductions(oracle_lib, sph16):
    """n = 1: power law == Newtonian (mu = kappa), Herschel-Bulkley == Papanastasiou, bitwise,
    for eta and for a whole step."""
    O = oracle_lib
    w, g, u, p = sph16
    # covered cells hold eta = mu under every law, so mu is set alike in each pair
    pairs = [(dict(law=I.LAW_POWER, kappa=1.7, flow_n=1.0, mu=1.7),
              dict(law=I.LAW_NEWTONIAN, mu=1.7)),
             (dict(law=I.LAW_HERSCHEL_BULKLEY, kappa=1.3, flow_n=1.0, tau0=2.0, mu=1.3),
              dict(law=I.LAW_PAPANASTASIOU, mu=1.3, tau0=2.0))]
    for a, b in pairs:
        ea, eba = g.viscosity(u, O.make_rheo(w.replace(**a)))
        eb, ebb = g.viscosity(u, O.make_rheo(w.replace(**b)))
        assert np.array_equal(ea, eb) and np.array_equal(eba, ebb)
        ua, pa, _ = _step(O, g, w, u, p, **a)
        ub, pb, _ = _step(O, g, w, u, p, **b)
        assert np.array_equal(ua, ub) and np.array_equal(pa, pb)


def test_zero_yield_stress_and_smd_exponent(oracle_lib, sph16):
    O = oracle_lib
    w, g, u, p = sph16
    pw = dict(kappa=1.2, flow_n=0.6)
    e0, eb0 = g.viscosity(u, O.make_rheo(w.replace(law=I.LAW_POWER, **pw)))
    for law in (I.LAW_HERSCHEL_BULKLEY, I.LAW_SOUZA_MENDES_DUTRA):
        e, eb = g.viscosity(u, O.make_rheo(w.replace(law=law, tau0=0.0, **pw)))
        assert np.array_equal(e, e0) and np.array_equal(eb, eb0)
    # Souza Mendes-Dutra with eta0 = tau0/eps has the Papanastasiou exponent: it equals
    # Herschel-Bulkley up to the rounding of eta0 sr / tau0 against sr / eps
    tau0, eps = 2.0, 1e-3
    eh, ebh = g.viscosity(u, O.make_rheo(w.replace(law=I.LAW_HERSCHEL_BULKLEY, tau0=tau0,
                                                   eps=eps, **pw)))
    es, ebs = g.viscosity(u, O.make_rheo(w.replace(law=I.LAW_SOUZA_MENDES_DUTRA, tau0=tau0,
                                                   eps=eps, eta0=tau0 / eps, **pw)))
    assert np.allclose(es, eh, rtol=1e-13, atol=0.0)
    assert np.allclose(ebs, ebh, rtol=1e-13, atol=0.0)
    # and the yield term does not vanish: a plain power law differs
    assert np.abs(eh - e0).max() > 1.0


def _steady_power_poiseuille(O, N, nflow, tol=1e-14, maxsteps=2000):
    W, G, kappa = 0.5, 1.0, 1.0
    w = I.Workload(name="poiseuille", n=(4, 4, N), h=1.0 / N, periodic=(1, 1, 0),
                   law=I.LAW_POWER, kappa=kappa, flow_n=nflow, eps=1e-12, rho=1.0, dt=1e3,
                   force=(G, 0.0, 0.0))
    g = O.Geometry(w)
    opts = O.make_opts(w, rtol=1e-13)
    rh = O.make_rheo(w)
    u = np.zeros((3,) + g.shape)
    u[0] = 0.01
    p = np.zeros(g.shape)
    umax = nflow / (nflow + 1) * (G / kappa) ** (1 / nflow) * W ** (1 + 1 / nflow)
    for _ in range(maxsteps):
        u1, p, _ = g.rk2_step(u, p, rh, w.dt, opts)
        du = np.abs(u1 - u).max()
        u = u1
        if du < tol * umax:
            break
    else:
        pytest.fail("no steady state")
    zeta = np.abs((np.arange(N) + 0.5) / N - 0.5)
    exact = nflow / (nflow + 1) * (G / kappa) ** (1 / nflow) * (W ** (1 + 1 / nflow)
                                                                - zeta ** (1 + 1 / nflow))
    assert np.abs(u[1:]).max() < 1e-13 * umax
    return np.abs(u[0, :, 0, 0] - exact).max() / umax


@pytest.mark.parametrize("nflow", [0.5, 1.0])
def test_power_law_poiseuille_closed_form(oracle_lib, nflow):
    """Shear-thinning n = 1/2 (u cubic in |z - zc|) and the Newtonian n = 1 (a parabola): the
    steady state converges to the closed form at second order in both."""
    e = [_steady_power_poiseuille(oracle_lib, N, nflow) for N in (16, 32, 64)]
    rates = [math.log2(e[i] / e[i + 1]) for i in range(2)]
    assert min(rates) > 1.8, (e, rates)
    assert e[-1] < 2e-3, e
