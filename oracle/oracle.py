"""ctypes binding of the plain FP64 CPU oracle (oracle/eb_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by tests/, the smoke check and the CPU-baseline leg of the
bench.  It never imports the product package, and the product never imports it.
All arrays are numpy float64 on the host, laid out as the C header describes.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libeb_oracle.so")

_lib = None


class OrBox(C.Structure):
    _fields_ = [("n", C.c_int * 3), ("h", C.c_double), ("lo", C.c_double * 3),
                ("periodic", C.c_int * 3), ("wall_u", (C.c_double * 3) * 6)]


class OrBody(C.Structure):
    _fields_ = [("kind", C.c_int), ("center", C.c_double * 3), ("radii", C.c_double * 3),
                ("euler_zyx", C.c_double * 3), ("zlo", C.c_double), ("zhi", C.c_double),
                ("plane_n", C.c_double * 3), ("plane_d", C.c_double), ("u_eb", C.c_double * 3)]


class OrRheo(C.Structure):
    _fields_ = [("law", C.c_int), ("mu", C.c_double), ("tau0", C.c_double),
                ("eps", C.c_double), ("rho", C.c_double), ("kappa", C.c_double),
                ("n", C.c_double), ("eta0", C.c_double)]


class OrOpts(C.Structure):
    _fields_ = [("rtol_visc", C.c_double), ("rtol_mac", C.c_double), ("rtol_proj", C.c_double),
                ("max_iter", C.c_int), ("nu1", C.c_int), ("nu2", C.c_int),
                ("nbottom", C.c_int), ("force", C.c_double * 3), ("projection", C.c_int)]


PROJ_CELL, PROJ_NODAL = 0, 1


class OrStats(C.Structure):
    _fields_ = [("it_mac", C.c_int * 2), ("it_visc", C.c_int * 2), ("it_proj", C.c_int * 2),
                ("div_proj", C.c_double * 2)]


_P = C.c_void_p
_D = C.c_double
_I = C.c_int


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from . import build as _b  # type: ignore
            _b.build()
        L = C.CDLL(LIB_PATH)
        sig = {
            "or_geom_build": (_P, [_P, _P, C.POINTER(C.c_int)]),
            "or_geom_free": (None, [_P]),
            "or_geom_ncut": (_I, [_P]),
            "or_geom_nlevels": (_I, [_P]),
            "or_geom_nfallback": (_I, [_P]),
            "or_geom_export": (None, [_P, _P, _P, _P, _P, _P]),
            "or_cut_export": (None, [_P, _P, _P]),
            "or_wall_gradient": (None, [_P, _P, _P]),
            "or_cell_gradient": (None, [_P, _P, _P, _P]),
            "or_viscosity": (None, [_P, _P, _P, _P, _P, _P, _P]),
            "or_visc_apply": (None, [_P, _D, _D, _P, _P, _P, _P, _I]),
            "or_transpose_term": (None, [_P, _P, _P, _P, _P]),
            "or_conv_term": (None, [_P, _P, _P, _P, _P, _P]),
            "or_redistribute": (None, [_P, _I, _P, _P]),
            "or_face_extrap": (None, [_P, _P, _P, _P, _P]),
            "or_divergence": (None, [_P, _P, _P, _P, _P]),
            "or_gcc": (None, [_P, _P, _P]),
            "or_poisson_apply": (None, [_P, _D, _P, _P]),
            "or_vcycle": (None, [_P, _I, _D, _D, _D, _P, _P, _P, _P, _P]),
            "or_visc_solve": (_I, [_P, _D, _D, _P, _P, _P, _P, _D, _I, _P, C.POINTER(C.c_int)]),
            "or_mac_project": (_I, [_P, _D, _P, _P, _P, _P, _D, _I, _P, C.POINTER(_D),
                                    C.POINTER(C.c_int)]),
            "or_cc_project": (_I, [_P, _D, _P, _P, _D, _I, _P, C.POINTER(_D),
                                   C.POINTER(C.c_int)]),
            "or_derived": (_I, [_P, _P, _P, _P, _P, _P, _P, _P, _P, C.POINTER(C.c_int)]),
            "or_rk2_step": (_I, [_P, _P, _P, _D, _P, _P, _P, _P]),
            "or_drag": (None, [_P, _P, _P, _P, _P, _P]),
            "or_stable_dt": (C.c_double, [_P, _P, _P, _P, _P, C.c_double]),
            "or_wall_gradient_adj": (None, [_P, _P, _P]),
            "or_cell_gradient_adj": (None, [_P, _P, _P, _P]),
            "or_redistribute_adj": (None, [_P, _I, _P, _P]),
            "or_face_extrap_adj": (None, [_P, _P, _P, _P, _P, _P]),
            "or_gcc_adj": (None, [_P, _P, _P]),
            "or_mac_project_adj": (_I, [_P, _D, _P, _P, _P, _D, _I, _P, C.POINTER(C.c_int)]),
            "or_cc_project_adj": (_I, [_P, _D, _P, _P, _D, _I, _P, C.POINTER(C.c_int)]),
            "or_visc_solve_adj": (_I, [_P, _D, _D, _P, _P, _P, _P, _D, _I, _P, _P, _P, _P,
                                       C.POINTER(C.c_int)]),
            "or_derived_adj": (_I, [_P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P,
                                    C.POINTER(C.c_int)]),
            "or_rk2_step_adjoint": (_I, [_P, _P, _P, _D, _P, _P, _P, _P, _P, _P, _P]),
            "or_drag_adj": (None, [_P, _P, _P, _P, _P, _P, _P, _P]),
            "or_nodal_div": (None, [_P, _P, _P]),
            "or_nodal_bflux": (None, [_P, _P]),
            "or_nodal_apply": (None, [_P, _P, _P]),
            "or_nodal_grad": (None, [_P, _P, _P]),
            "or_nodal_project": (_I, [_P, _D, _P, _P, _D, _I, C.POINTER(_D), C.POINTER(C.c_int)]),
            "or_drag_nodal": (None, [_P, _P, _P, _P, _P, _P]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _ptr(a):
    if a is None:
        return None
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(C.c_void_p)


def make_box(w) -> OrBox:
    b = OrBox()
    for d in range(3):
        b.n[d] = int(w.n[d])
        b.lo[d] = float(w.lo[d])
        b.periodic[d] = int(w.periodic[d])
    b.h = float(w.h)
    for f in range(6):
        for c in range(3):
            b.wall_u[f][c] = float(w.wall_u[f][c])
    return b


def make_body(w) -> OrBody:
    bd = w.body
    b = OrBody()
    b.kind = int(bd.get("kind", 0))
    cen = bd.get("center", (0.5, 0.5, 0.5))
    radii = bd.get("radii", (bd.get("radius", 0.0),) * 3)
    eul = bd.get("euler_zyx", (0.0, 0.0, 0.0))
    for d in range(3):
        b.center[d] = float(cen[d])
        b.radii[d] = float(radii[d])
        b.euler_zyx[d] = float(eul[d])
    b.zlo = float(bd.get("zlo", 0.0))
    b.zhi = float(bd.get("zhi", 1.0))
    pn = bd.get("plane_n", (0.0, 0.0, 1.0))
    for d in range(3):
        b.plane_n[d] = float(pn[d])
        b.u_eb[d] = float(bd.get("u_eb", (0.0, 0.0, 0.0))[d])
    b.plane_d = float(bd.get("plane_d", 0.0))
    return b


def make_rheo(w, tau0=None) -> OrRheo:
    r = OrRheo()
    r.law = int(w.law)
    r.mu = float(w.mu)
    r.tau0 = float(w.tau0 if tau0 is None else tau0)
    r.eps = float(w.eps)
    r.rho = float(w.rho)
    r.kappa = float(w.kappa)
    r.n = float(w.flow_n)
    r.eta0 = float(w.eta0)
    return r


def make_opts(w=None, rtol=None, max_iter=400, nu1=2, nu2=2, nbottom=16,
              projection=PROJ_CELL) -> OrOpts:
    o = OrOpts()
    o.projection = int(projection)
    rt = rtol if rtol is not None else (w.rtol if w is not None else 1e-12)
    o.rtol_visc = o.rtol_mac = o.rtol_proj = float(rt)
    o.max_iter = int(max_iter)
    o.nu1, o.nu2, o.nbottom = int(nu1), int(nu2), int(nbottom)
    f = w.force if w is not None else (0.0, 0.0, 0.0)
    for d in range(3):
        o.force[d] = float(f[d])
    return o


class OracleError(RuntimeError):
    pass


class Geometry:
    """Oracle geometry and the state needed to run the oracle's step on one box."""

    def __init__(self, w):
        self.w = w
        self.box = make_box(w)
        self.body = make_body(w)
        err = C.c_int(0)
        self.g = lib().or_geom_build(C.byref(self.box), C.byref(self.body), C.byref(err))
        self.err = err.value
        if not self.g:
            raise OracleError(f"or_geom_build failed: {err.value}")
        nx, ny, nz = w.n
        self.n = (nx, ny, nz)
        self.N = nx * ny * nz
        self.shape = (nz, ny, nx)
        self.ncut = lib().or_geom_ncut(self.g)
        self.nlevels = lib().or_geom_nlevels(self.g)
        self.nfallback = lib().or_geom_nfallback(self.g)

    def __del__(self):
        try:
            if getattr(self, "g", None):
                lib().or_geom_free(self.g)
                self.g = None
        except Exception:
            pass

    # ---------------------------------------------------------------- geometry data
    def face_shapes(self):
        nx, ny, nz = self.n
        return [(nz, ny, nx + 1), (nz, ny + 1, nx), (nz + 1, ny, nx)]

    def export(self):
        flag = np.zeros(self.shape, np.uint8)
        alpha = np.zeros(self.shape)
        ap = [np.zeros(s) for s in self.face_shapes()]
        lib().or_geom_export(self.g, _ptr(flag), _ptr(alpha), *[_ptr(a) for a in ap])
        return flag, alpha, ap

    def cut(self):
        cell = np.zeros(max(self.ncut, 1), np.int64)
        data = np.zeros((max(self.ncut, 1), 9))
        lib().or_cut_export(self.g, _ptr(cell), _ptr(data))
        return cell[: self.ncut], data[: self.ncut]

    # ---------------------------------------------------------------- pointwise pieces
    def wall_gradient(self, u):
        gw = np.zeros((max(self.ncut, 1), 3))
        lib().or_wall_gradient(self.g, _ptr(np.ascontiguousarray(u)), _ptr(gw))
        return gw[: self.ncut]

    def cell_gradient(self, u):
        u = np.ascontiguousarray(u, dtype=np.float64)
        gw = np.zeros((max(self.ncut, 1), 3))
        lib().or_wall_gradient(self.g, _ptr(u), _ptr(gw))
        G = np.zeros((3, 3) + self.shape)
        lib().or_cell_gradient(self.g, _ptr(u), _ptr(gw), _ptr(G))
        return G

    def viscosity(self, u, rheo: OrRheo, theta=None, with_sr=False):
        eta = np.zeros(self.shape)
        eta_eb = np.zeros(max(self.ncut, 1))
        sr = np.zeros(self.shape)
        lib().or_viscosity(self.g, C.byref(rheo), _ptr(np.ascontiguousarray(u)),
                           _ptr(theta), _ptr(eta), _ptr(eta_eb), _ptr(sr))
        if with_sr:
            return eta, eta_eb[: self.ncut], sr
        return eta, eta_eb[: self.ncut]

    def _eb(self, eta_eb):
        e = np.zeros(max(self.ncut, 1))
        e[: self.ncut] = eta_eb
        return e

    def visc_apply(self, rho, dt, eta, eta_eb, u, homogeneous=False):
        out = np.zeros((3,) + self.shape)
        lib().or_visc_apply(self.g, rho, dt, _ptr(np.ascontiguousarray(eta)),
                            _ptr(self._eb(eta_eb)), _ptr(np.ascontiguousarray(u)), _ptr(out),
                            int(homogeneous))
        return out

    def transpose_term(self, eta, eta_eb, u):
        V = np.zeros((3,) + self.shape)
        lib().or_transpose_term(self.g, _ptr(np.ascontiguousarray(eta)), _ptr(self._eb(eta_eb)),
                                _ptr(np.ascontiguousarray(u)), _ptr(V))
        return V

    def conv_term(self, u, faces):
        Cv = np.zeros((3,) + self.shape)
        f = [np.ascontiguousarray(a) for a in faces]
        lib().or_conv_term(self.g, _ptr(np.ascontiguousarray(u)), *[_ptr(a) for a in f], _ptr(Cv))
        return Cv

    def redistribute(self, DC):
        DC = np.ascontiguousarray(DC, dtype=np.float64)
        ncomp = DC.size // self.N
        D = np.zeros_like(DC)
        lib().or_redistribute(self.g, ncomp, _ptr(DC), _ptr(D))
        return D

    def face_extrap(self, u):
        f = [np.zeros(s) for s in self.face_shapes()]
        lib().or_face_extrap(self.g, _ptr(np.ascontiguousarray(u)), *[_ptr(a) for a in f])
        return f

    def divergence(self, faces):
        div = np.zeros(self.shape)
        f = [np.ascontiguousarray(a) for a in faces]
        lib().or_divergence(self.g, *[_ptr(a) for a in f], _ptr(div))
        return div

    def gcc(self, p):
        gp = np.zeros((3,) + self.shape)
        lib().or_gcc(self.g, _ptr(np.ascontiguousarray(p)), _ptr(gp))
        return gp

    def poisson_apply(self, beta, p):
        out = np.zeros(self.shape)
        lib().or_poisson_apply(self.g, beta, _ptr(np.ascontiguousarray(p)), _ptr(out))
        return out

    # ---------------------------------------------------------------- solvers
    def vcycle(self, system, r, opts, beta=1.0, rho=1.0, dt=1.0, eta=None, eta_eb=None):
        r = np.ascontiguousarray(r, dtype=np.float64)
        e = np.zeros_like(r)
        lib().or_vcycle(self.g, system, beta, rho, dt, _ptr(eta),
                        _ptr(self._eb(eta_eb) if eta_eb is not None else None), _ptr(r), _ptr(e),
                        C.byref(opts))
        return e

    def visc_solve(self, rho, dt, eta, eta_eb, psi, x0, opts, rtol=None):
        x = np.array(x0, dtype=np.float64, copy=True, order="C")
        it = C.c_int(0)
        rt = opts.rtol_visc if rtol is None else rtol
        e = lib().or_visc_solve(self.g, rho, dt, _ptr(np.ascontiguousarray(eta)),
                                _ptr(self._eb(eta_eb)), _ptr(np.ascontiguousarray(psi)), _ptr(x),
                                rt, opts.max_iter, C.byref(opts), C.byref(it))
        if e:
            raise OracleError(f"or_visc_solve: {e}")
        return x, it.value

    def mac_project(self, faces, beta, opts, phi0=None, rtol=None):
        f = [np.array(a, dtype=np.float64, copy=True, order="C") for a in faces]
        phi = np.zeros(self.shape) if phi0 is None else np.array(phi0, copy=True, order="C")
        div = C.c_double(0)
        it = C.c_int(0)
        rt = opts.rtol_mac if rtol is None else rtol
        e = lib().or_mac_project(self.g, beta, *[_ptr(a) for a in f], _ptr(phi), rt,
                                 opts.max_iter, C.byref(opts), C.byref(div), C.byref(it))
        if e:
            raise OracleError(f"or_mac_project: {e}")
        return f, phi, div.value, it.value

    def cc_project(self, u, p, beta, opts, rtol=None):
        u = np.array(u, dtype=np.float64, copy=True, order="C")
        p = np.array(p, dtype=np.float64, copy=True, order="C")
        div = C.c_double(0)
        it = C.c_int(0)
        rt = opts.rtol_proj if rtol is None else rtol
        e = lib().or_cc_project(self.g, beta, _ptr(u), _ptr(p), rt, opts.max_iter,
                                C.byref(opts), C.byref(div), C.byref(it))
        if e:
            raise OracleError(f"or_cc_project: {e}")
        return u, p, div.value, it.value

    def derived(self, u, rheo, opts, theta=None):
        Cv = np.zeros((3,) + self.shape)
        V = np.zeros((3,) + self.shape)
        eta = np.zeros(self.shape)
        eta_eb = np.zeros(max(self.ncut, 1))
        it = C.c_int(0)
        e = lib().or_derived(self.g, C.byref(rheo), _ptr(theta), _ptr(np.ascontiguousarray(u)),
                             C.byref(opts), _ptr(Cv), _ptr(eta), _ptr(eta_eb), _ptr(V),
                             C.byref(it))
        if e:
            raise OracleError(f"or_derived: {e}")
        return Cv, eta, eta_eb[: self.ncut], V

    def rk2_step(self, u, p, rheo, dt, opts, theta=None):
        u = np.array(u, dtype=np.float64, copy=True, order="C")
        p = np.array(p, dtype=np.float64, copy=True, order="C")
        st = OrStats()
        e = lib().or_rk2_step(self.g, C.byref(rheo), _ptr(theta), dt, C.byref(opts), _ptr(u),
                              _ptr(p), C.byref(st))
        if e:
            raise OracleError(f"or_rk2_step: {e}")
        stats = {"it_mac": list(st.it_mac), "it_visc": list(st.it_visc),
                 "it_proj": list(st.it_proj), "div_proj": list(st.div_proj)}
        return u, p, stats

    def stable_dt(self, u, rheo, force=(0.0, 0.0, 0.0), c_cfl=0.5, theta=None):
        f = np.ascontiguousarray(np.asarray(force, dtype=np.float64))
        return lib().or_stable_dt(self.g, C.byref(rheo), _ptr(theta),
                                  _ptr(np.ascontiguousarray(u)), _ptr(f), float(c_cfl))

    def drag(self, u, p, rheo, theta=None):
        F = np.zeros(3)
        lib().or_drag(self.g, C.byref(rheo), _ptr(theta), _ptr(np.ascontiguousarray(u)),
                      _ptr(np.ascontiguousarray(p)), _ptr(F))
        return F

    # ---------------------------------------------------------------- nodal projection
    @property
    def node_shape(self):
        nz, ny, nx = self.shape
        return (nz + 1, ny + 1, nx + 1)

    def nodal_div(self, w):
        out = np.zeros(self.node_shape)
        lib().or_nodal_div(self.g, _ptr(self._c(w)), _ptr(out))
        return out

    def nodal_bflux(self):
        out = np.zeros(self.node_shape)
        lib().or_nodal_bflux(self.g, _ptr(out))
        return out

    def nodal_apply(self, x):
        out = np.zeros(self.node_shape)
        lib().or_nodal_apply(self.g, _ptr(self._c(x)), _ptr(out))
        return out

    def nodal_grad(self, q):
        out = np.zeros((3,) + self.shape)
        lib().or_nodal_grad(self.g, _ptr(self._c(q)), _ptr(out))
        return out

    def nodal_project(self, u, pn, beta, opts):
        u = self._c(u)
        pn = self._c(pn)
        div = C.c_double(0.0)
        it = C.c_int(0)
        e = lib().or_nodal_project(self.g, float(beta), _ptr(u), _ptr(pn), opts.rtol_proj,
                                   opts.max_iter, C.byref(div), C.byref(it))
        if e:
            raise OracleError(f"or_nodal_project: {e}")
        return u, pn, div.value, it.value

    def drag_nodal(self, u, pn, rheo, theta=None):
        F = np.zeros(3)
        lib().or_drag_nodal(self.g, C.byref(rheo), _ptr(theta), _ptr(np.ascontiguousarray(u)),
                            _ptr(np.ascontiguousarray(pn)), _ptr(F))
        return F


    # ---------------------------------------------------------------- adjoint (reverse mode)
    def _c(self, a):
        return np.array(a, dtype=np.float64, copy=True, order="C")

    def wall_gradient_adj(self, gwb):
        ub = np.zeros((3,) + self.shape)
        g = np.zeros((max(self.ncut, 1), 3))
        g[: self.ncut] = gwb
        lib().or_wall_gradient_adj(self.g, _ptr(g), _ptr(ub))
        return ub

    def cell_gradient_adj(self, Gb):
        """Adjoint of G = cell_gradient(u, gw) for fixed gw input: returns (ub, gwb)."""
        ub = np.zeros((3,) + self.shape)
        gwb = np.zeros((max(self.ncut, 1), 3))
        lib().or_cell_gradient_adj(self.g, _ptr(self._c(Gb)), _ptr(ub), _ptr(gwb))
        return ub, gwb[: self.ncut]

    def cell_gradient_from(self, u, gw):
        G = np.zeros((3, 3) + self.shape)
        g = np.zeros((max(self.ncut, 1), 3))
        g[: self.ncut] = gw
        lib().or_cell_gradient(self.g, _ptr(self._c(u)), _ptr(g), _ptr(G))
        return G

    def redistribute_adj(self, Db):
        Db = self._c(Db)
        DCb = np.zeros_like(Db)
        lib().or_redistribute_adj(self.g, Db.size // self.N, _ptr(Db), _ptr(DCb))
        return DCb

    def face_extrap_adj(self, u, fb):
        ub = np.zeros((3,) + self.shape)
        f = [self._c(a) for a in fb]
        lib().or_face_extrap_adj(self.g, _ptr(self._c(u)), *[_ptr(a) for a in f], _ptr(ub))
        return ub

    def gcc_adj(self, gpb):
        pb = np.zeros(self.shape)
        lib().or_gcc_adj(self.g, _ptr(self._c(gpb)), _ptr(pb))
        return pb

    def mac_project_adj(self, fb, beta, opts, rtol=None):
        f = [self._c(a) for a in fb]
        it = C.c_int(0)
        rt = opts.rtol_mac if rtol is None else rtol
        e = lib().or_mac_project_adj(self.g, beta, *[_ptr(a) for a in f], rt, opts.max_iter,
                                     C.byref(opts), C.byref(it))
        if e:
            raise OracleError(f"or_mac_project_adj: {e}")
        return f, it.value

    def cc_project_adj(self, ub, pb, beta, opts, rtol=None):
        ub = self._c(ub)
        pb = self._c(pb)
        it = C.c_int(0)
        rt = opts.rtol_proj if rtol is None else rtol
        e = lib().or_cc_project_adj(self.g, beta, _ptr(ub), _ptr(pb), rt, opts.max_iter,
                                    C.byref(opts), C.byref(it))
        if e:
            raise OracleError(f"or_cc_project_adj: {e}")
        return ub, pb, it.value

    def visc_solve_adj(self, rho, dt, eta, eta_eb, x, xb, opts, rtol=None):
        psib = np.zeros((3,) + self.shape)
        etab = np.zeros(self.shape)
        etaebb = np.zeros(max(self.ncut, 1))
        it = C.c_int(0)
        rt = opts.rtol_visc if rtol is None else rtol
        e = lib().or_visc_solve_adj(self.g, rho, dt, _ptr(self._c(eta)), _ptr(self._eb(eta_eb)),
                                    _ptr(self._c(x)), _ptr(self._c(xb)), rt, opts.max_iter,
                                    C.byref(opts), _ptr(psib), _ptr(etab), _ptr(etaebb),
                                    C.byref(it))
        if e:
            raise OracleError(f"or_visc_solve_adj: {e}")
        return psib, etab, etaebb[: self.ncut], it.value

    def derived_adj(self, u, rheo, opts, Cb, etab, etaebb, Vb, theta=None):
        ub = np.zeros((3,) + self.shape)
        tau0b = np.zeros(self.shape)
        it = C.c_int(0)
        e = lib().or_derived_adj(self.g, C.byref(rheo), _ptr(theta), _ptr(self._c(u)), None,
                                 C.byref(opts), _ptr(self._c(Cb)), _ptr(self._c(etab)),
                                 _ptr(self._eb(etaebb)), _ptr(self._c(Vb)), _ptr(ub),
                                 _ptr(tau0b), C.byref(it))
        if e:
            raise OracleError(f"or_derived_adj: {e}")
        return ub, tau0b

    def rk2_step_adjoint(self, u0, p0, rheo, dt, opts, ub, pb, theta=None):
        """Adjoint of one step at input (u0, p0): (ub, pb) of the output in, those of the input
        out, plus d loss / d tau0_c per cell (tau0_c = rheo.tau0 * theta_c)."""
        ub = self._c(ub)
        pb = self._c(pb)
        tau0b = np.zeros(self.shape)
        st = OrStats()
        e = lib().or_rk2_step_adjoint(self.g, C.byref(rheo), _ptr(theta), dt, C.byref(opts),
                                      _ptr(self._c(u0)), _ptr(self._c(p0)), _ptr(ub), _ptr(pb),
                                      _ptr(tau0b), C.byref(st))
        if e:
            raise OracleError(f"or_rk2_step_adjoint: {e}")
        stats = {"it_mac": list(st.it_mac), "it_visc": list(st.it_visc),
                 "it_proj": list(st.it_proj)}
        return ub, pb, tau0b, stats

    def drag_adj(self, u, rheo, Fb, theta=None):
        ub = np.zeros((3,) + self.shape)
        pb = np.zeros(self.shape)
        tau0b = np.zeros(self.shape)
        fb = np.ascontiguousarray(np.asarray(Fb, dtype=np.float64))
        lib().or_drag_adj(self.g, C.byref(rheo), _ptr(theta), _ptr(self._c(u)), _ptr(fb),
                          _ptr(ub), _ptr(pb), _ptr(tau0b))
        return ub, pb, tau0b


def prepare_state(w, geom: Geometry, opts=None):
    """Seeded start field of workload w, projected once with beta = 1 (pressure reset to 0)."""
    import eb_inputs
    u0 = eb_inputs.initial_velocity(w)
    opts = opts or make_opts(w)
    p0 = np.zeros(geom.shape)
    if w.noise > 0.0:
        u0, _, _, _ = geom.cc_project(u0, p0, 1.0, opts)
    return u0, p0
