"""Oracle failure codes: a non-finite state is reported (OR_ENAN) instead of being stopped on as
converged, a solve short of iterations is reported (OR_ENOCONV), and a wall-flux stencil that
leaves a non-periodic box is a geometry error (OR_EGEOM)."""
import ctypes as C

import numpy as np

import eb_inputs as I


def _step_code(O, g, w, u, p, opts):
    st = O.OrStats()
    u = np.array(u, dtype=np.float64, copy=True, order="C")
    p = np.array(p, dtype=np.float64, copy=True, order="C")
    return O.lib().or_rk2_step(g.g, C.byref(O.make_rheo(w)), None, w.dt, C.byref(opts),
                               O._ptr(u), O._ptr(p), C.byref(st))


def test_nan_state_is_reported(oracle_lib):
    O = oracle_lib
    w = I.sphere_n(16, radius=0.25)
    g = O.Geometry(w)
    u = I.initial_velocity(w)
    u[0, 8, 8, 1] = np.nan
    assert _step_code(O, g, w, u, np.zeros(g.shape), O.make_opts(w)) == -4
    assert _step_code(O, g, w, I.initial_velocity(w), np.zeros(g.shape), O.make_opts(w)) == 0


def test_unreachable_tolerance_is_reported(oracle_lib):
    O = oracle_lib
    w = I.sphere_n(16, radius=0.25)
    g = O.Geometry(w)
    opts = O.make_opts(w, rtol=1e-300, max_iter=1)
    assert _step_code(O, g, w, I.initial_velocity(w), np.zeros(g.shape), opts) == -3


def test_stencil_outside_the_box_is_a_geometry_error(oracle_lib):
    O = oracle_lib
    w = I.sphere_n(32, radius=0.08)
    w.body = {"kind": I.BODY_SPHERE, "center": (0.5, 0.5, 0.1), "radius": 0.08}
    assert O.Geometry(w).err == -2
