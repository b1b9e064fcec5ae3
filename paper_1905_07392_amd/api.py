"""Python binding of the C ABI (include/eb.h): argument marshalling only.

Every function keeps the name of its C entry point, takes torch tensors on a HIP device (float64,
contiguous) and enqueues on torch's current stream.  Device memory (the geometry workspace and
all outputs) is allocated through torch; all computation happens in libeb.so.
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _lib as L
from ._lib import (EB_FP64, EB_MIXED, EB_OP_HELMHOLTZ, EB_OP_HELMHOLTZ_H, EB_OP_TRANSPOSE,
                   EB_PROJ_CELL, EB_PROJ_NODAL,
                   EB_SWITCH_OFF, EB_SWITCH_RECORD, EB_SWITCH_REPLAY, EB_SYS_POISSON, EB_SYS_VISC,
                   EbBody, EbBox, EbRheology, EbStepOpts, EbStepStats, check)

__all__ = ["EbContext", "make_box", "make_body", "make_rheology", "make_opts",
           "eb_workspace_bytes", "eb_geometry_build", "eb_geometry_export",
           "eb_apparent_viscosity", "eb_viscous_apply", "eb_mg_vcycle", "eb_visc_solve",
           "eb_mac_project", "eb_cc_project", "eb_derived", "eb_rk2_step", "eb_drag",
           "eb_pressure_gradient", "eb_drag_noalloc", "eb_nodal_project", "eb_drag_nodal", "eb_stable_dt", "eb_tape_bytes", "eb_rk2_step_taped",
           "eb_rk2_step_adjoint", "eb_drag_adjoint", "eb_mac_project_adjoint", "eb_cc_project_adjoint",
           "eb_visc_solve_adjoint", "eb_derived_adjoint", "EB_FP64", "EB_MIXED", "EB_OP_HELMHOLTZ",
           "EB_OP_HELMHOLTZ_H", "EB_OP_TRANSPOSE", "EB_SYS_POISSON", "EB_SYS_VISC",
           "EB_SWITCH_OFF", "EB_SWITCH_RECORD", "EB_SWITCH_REPLAY", "EB_PROJ_CELL",
           "EB_PROJ_NODAL"]


def _stream(device=None):
    return C.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _p(t):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        raise TypeError("expected a torch tensor")
    if not t.is_cuda:
        raise ValueError("tensors must live on the GPU")
    if not t.is_contiguous():
        raise ValueError("tensors must be contiguous")
    return C.c_void_p(t.data_ptr())


def _f64(t, shape, name):
    if t.dtype != torch.float64:
        raise TypeError(f"{name} must be float64")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    return _p(t)


# ----------------------------------------------------------------------------------------------
# structs from plain parameters (any object with the workload attributes works)
# ----------------------------------------------------------------------------------------------
def make_box(n, h, lo=(0.0, 0.0, 0.0), periodic=(0, 0, 0), wall_u=None) -> EbBox:
    b = EbBox()
    for d in range(3):
        b.n[d] = int(n[d])
        b.lo[d] = float(lo[d])
        b.periodic[d] = int(periodic[d])
    b.h = float(h)
    wall_u = wall_u or [[0.0, 0.0, 0.0]] * 6
    for f in range(6):
        for c in range(3):
            b.wall_u[f][c] = float(wall_u[f][c])
    return b


def make_body(kind=0, center=(0.5, 0.5, 0.5), radius=None, radii=None, euler_zyx=(0, 0, 0),
              zlo=0.0, zhi=1.0, plane_n=(0.0, 0.0, 1.0), plane_d=0.0, u_eb=(0, 0, 0)) -> EbBody:
    b = EbBody()
    b.kind = int(kind)
    if radii is None:
        radii = (radius or 0.0,) * 3
    for d in range(3):
        b.center[d] = float(center[d])
        b.radii[d] = float(radii[d])
        b.euler_zyx[d] = float(euler_zyx[d])
        b.plane_n[d] = float(plane_n[d])
        b.u_eb[d] = float(u_eb[d])
    b.zlo, b.zhi, b.plane_d = float(zlo), float(zhi), float(plane_d)
    return b


def make_rheology(law, mu, tau0, eps, rho, kappa=1.0, n=1.0, eta0=1.0) -> EbRheology:
    """Law parameters (Table rheology); kappa, n and eta0 serve the power-law laws."""
    r = EbRheology()
    r.law, r.mu, r.tau0, r.eps, r.rho = int(law), float(mu), float(tau0), float(eps), float(rho)
    r.kappa, r.n, r.eta0 = float(kappa), float(n), float(eta0)
    return r


def make_opts(precision=EB_FP64, rtol=1e-12, max_iter=400, nu1=2, nu2=2, nbottom=16,
              force=(0.0, 0.0, 0.0), rtol_visc=None, rtol_mac=None, rtol_proj=None,
              projection=EB_PROJ_CELL) -> EbStepOpts:
    o = EbStepOpts()
    o.precision = int(precision)
    o.projection = int(projection)
    o.rtol_visc = float(rtol if rtol_visc is None else rtol_visc)
    o.rtol_mac = float(rtol if rtol_mac is None else rtol_mac)
    o.rtol_proj = float(rtol if rtol_proj is None else rtol_proj)
    o.max_iter, o.nu1, o.nu2, o.nbottom = int(max_iter), int(nu1), int(nu2), int(nbottom)
    for d in range(3):
        o.force[d] = float(force[d])
    return o


class EbContext:
    """Owns the device workspace tensor and the library context built over it."""

    def __init__(self, box: EbBox, body: EbBody, device="cuda"):
        self.device = torch.device(device)
        self.box, self.body = box, body
        nbytes = L.lib().eb_workspace_bytes(C.byref(box), C.byref(body))
        if nbytes == 0:
            check(L.EB_EINVAL, "eb_workspace_bytes")
        self.workspace = torch.empty(int(nbytes), dtype=torch.uint8, device=self.device)
        self.ptr = C.c_void_p()
        with torch.cuda.device(self.device):
            check(L.lib().eb_geometry_build(C.byref(box), C.byref(body), _p(self.workspace),
                                            C.c_size_t(nbytes), C.byref(self.ptr),
                                            _stream(self.device)), "eb_geometry_build")
        ncut, nlev, nfb = C.c_int(), C.c_int(), C.c_int()
        check(L.lib().eb_ctx_info(self.ptr, C.byref(ncut), C.byref(nlev), C.byref(nfb)),
              "eb_ctx_info")
        self.ncut, self.nlevels, self.nfallback = ncut.value, nlev.value, nfb.value
        nx, ny, nz = box.n[0], box.n[1], box.n[2]
        self.n = (nx, ny, nz)
        self.N = nx * ny * nz
        self.shape = (nz, ny, nx)
        self.face_shapes = [(nz, ny, nx + 1), (nz, ny + 1, nx), (nz + 1, ny, nx)]
        self.node_shape = (nz + 1, ny + 1, nx + 1)
        self.h = box.h

    def close(self):
        if getattr(self, "ptr", None) is not None and self.ptr.value:
            L.lib().eb_ctx_destroy(self.ptr)
            self.ptr = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_graphs(self, enable: bool):
        """Replay captured solver iterations (default) or launch every kernel individually."""
        check(L.lib().eb_ctx_set_graphs(self.ptr, int(bool(enable))), "eb_ctx_set_graphs")

    def switch_record(self, evaluations: int):
        """A zeroed uint8 device buffer for the branch records of `evaluations` derived-
        quantities evaluations (two per RK2 step)."""
        nb = int(L.lib().eb_switch_bytes(self.ptr))
        return torch.zeros(nb * int(evaluations), dtype=torch.uint8, device=self.device)

    def set_switches(self, mode: int, record=None):
        """EB_SWITCH_RECORD / EB_SWITCH_REPLAY the step's switches into / from `record` (from
        its start), or EB_SWITCH_OFF."""
        if mode == L.EB_SWITCH_OFF:
            check(L.lib().eb_ctx_set_switches(self.ptr, 0, None, 0), "eb_ctx_set_switches")
            return
        assert record is not None and record.dtype == torch.uint8 and record.is_contiguous()
        assert record.device == self.device
        check(L.lib().eb_ctx_set_switches(self.ptr, int(mode), C.c_void_p(record.data_ptr()),
                                          record.numel()), "eb_ctx_set_switches")

    def zeros(self, *shape):
        return torch.zeros(shape, dtype=torch.float64, device=self.device)

    def vec(self):
        return self.zeros(3, *self.shape)

    def scalar(self):
        return self.zeros(*self.shape)


def eb_workspace_bytes(box: EbBox, body: EbBody) -> int:
    return int(L.lib().eb_workspace_bytes(C.byref(box), C.byref(body)))


def eb_geometry_build(box: EbBox, body: EbBody, device="cuda") -> EbContext:
    return EbContext(box, body, device)


def eb_geometry_export(ctx: EbContext):
    flag = torch.empty(ctx.shape, dtype=torch.uint8, device=ctx.device)
    alpha = ctx.scalar()
    ap = [ctx.zeros(*s) for s in ctx.face_shapes]
    nc = max(ctx.ncut, 1)
    cell = torch.zeros(nc, dtype=torch.int64, device=ctx.device)
    data = ctx.zeros(nc, 9)
    check(L.lib().eb_geometry_export(ctx.ptr, _p(flag), _p(alpha), _p(ap[0]), _p(ap[1]),
                                     _p(ap[2]), _p(cell), _p(data), _stream(ctx.device)),
          "eb_geometry_export")
    return flag, alpha, ap, cell[: ctx.ncut], data[: ctx.ncut]


def eb_apparent_viscosity(ctx: EbContext, rheo: EbRheology, u, theta=None, with_sr=False):
    eta = ctx.scalar()
    eta_eb = ctx.zeros(max(ctx.ncut, 1))
    sr = ctx.scalar() if with_sr else None
    th = _f64(theta, ctx.shape, "theta") if theta is not None else None
    check(L.lib().eb_apparent_viscosity(ctx.ptr, C.byref(rheo), _f64(u, (3,) + ctx.shape, "u"),
                                        th, _p(eta), _p(eta_eb), _p(sr), _stream(ctx.device)),
          "eb_apparent_viscosity")
    eta_eb = eta_eb[: ctx.ncut]
    return (eta, eta_eb, sr) if with_sr else (eta, eta_eb)


def _eb_arr(ctx, eta_eb):
    if ctx.ncut == 0:
        return ctx.zeros(1)
    return eta_eb.contiguous()


def eb_viscous_apply(ctx: EbContext, mode, rho, dt, eta, eta_eb, u):
    out = ctx.vec()
    check(L.lib().eb_viscous_apply(ctx.ptr, int(mode), float(rho), float(dt),
                                   _f64(eta, ctx.shape, "eta"), _p(_eb_arr(ctx, eta_eb)),
                                   _f64(u, (3,) + ctx.shape, "u"), _p(out), _stream(ctx.device)),
          "eb_viscous_apply")
    return out


def eb_mg_vcycle(ctx: EbContext, system, r, opts: EbStepOpts, precision=EB_FP64, beta=1.0,
                 rho=1.0, dt=1.0, eta=None, eta_eb=None):
    e = torch.zeros_like(r)
    ebp = _p(_eb_arr(ctx, eta_eb)) if eta is not None else None
    check(L.lib().eb_mg_vcycle(ctx.ptr, int(system), int(precision), float(beta), float(rho),
                               float(dt), _p(eta), ebp, _p(r.contiguous()), _p(e),
                               C.byref(opts), _stream(ctx.device)), "eb_mg_vcycle")
    return e


def eb_mg_sweep(ctx: EbContext, system, colour, b, x, precision=EB_FP64):
    """One red-black half sweep on the finest level, in place on x (operator already built)."""
    check(L.lib().eb_mg_sweep(ctx.ptr, int(system), int(precision), int(colour), _p(b), _p(x),
                              _stream(ctx.device)), "eb_mg_sweep")
    return x


def eb_visc_solve(ctx: EbContext, rho, dt, eta, eta_eb, psi, x0, opts: EbStepOpts, rtol=None):
    x = x0.clone().contiguous()
    it = C.c_int(0)
    rt = opts.rtol_visc if rtol is None else rtol
    check(L.lib().eb_visc_solve(ctx.ptr, float(rho), float(dt), _f64(eta, ctx.shape, "eta"),
                                _p(_eb_arr(ctx, eta_eb)), _f64(psi, (3,) + ctx.shape, "psi"),
                                _p(x), float(rt), C.byref(opts), C.byref(it),
                                _stream(ctx.device)), "eb_visc_solve")
    return x, it.value


def eb_mac_project(ctx: EbContext, faces, beta, opts: EbStepOpts, phi0=None, rtol=None):
    f = [a.clone().contiguous() for a in faces]
    for a, s in zip(f, ctx.face_shapes):
        _f64(a, s, "face")
    phi = ctx.scalar() if phi0 is None else phi0.clone().contiguous()
    div = C.c_double(0.0)
    it = C.c_int(0)
    rt = opts.rtol_mac if rtol is None else rtol
    check(L.lib().eb_mac_project(ctx.ptr, float(beta), _p(f[0]), _p(f[1]), _p(f[2]), _p(phi),
                                 float(rt), C.byref(opts), C.byref(div), C.byref(it),
                                 _stream(ctx.device)), "eb_mac_project")
    return f, phi, div.value, it.value


def eb_cc_project(ctx: EbContext, u, p, beta, opts: EbStepOpts, rtol=None):
    u = u.clone().contiguous()
    p = p.clone().contiguous()
    div = C.c_double(0.0)
    it = C.c_int(0)
    rt = opts.rtol_proj if rtol is None else rtol
    check(L.lib().eb_cc_project(ctx.ptr, float(beta), _f64(u, (3,) + ctx.shape, "u"),
                                _f64(p, ctx.shape, "p"), float(rt), C.byref(opts), C.byref(div),
                                C.byref(it), _stream(ctx.device)), "eb_cc_project")
    return u, p, div.value, it.value


def eb_derived(ctx: EbContext, rheo: EbRheology, u, opts: EbStepOpts, theta=None):
    Cv, V = ctx.vec(), ctx.vec()
    eta = ctx.scalar()
    eta_eb = ctx.zeros(max(ctx.ncut, 1))
    it = C.c_int(0)
    th = _f64(theta, ctx.shape, "theta") if theta is not None else None
    check(L.lib().eb_derived(ctx.ptr, C.byref(rheo), th, _f64(u, (3,) + ctx.shape, "u"),
                             C.byref(opts), _p(Cv), _p(eta), _p(eta_eb), _p(V), C.byref(it),
                             _stream(ctx.device)), "eb_derived")
    return Cv, eta, eta_eb[: ctx.ncut], V


def eb_rk2_step(ctx: EbContext, rheo: EbRheology, dt, opts: EbStepOpts, u, p, theta=None,
                inplace=False, allow_noconv=False):
    """One RK2 step.  With inplace=True u and p are updated in place (no allocation)."""
    if not inplace:
        u = u.clone().contiguous()
        p = p.clone().contiguous()
    st = EbStepStats()
    th = _f64(theta, ctx.shape, "theta") if theta is not None else None
    pshape = ctx.node_shape if opts.projection == EB_PROJ_NODAL else ctx.shape
    code = L.lib().eb_rk2_step(ctx.ptr, C.byref(rheo), th, float(dt), C.byref(opts),
                               _f64(u, (3,) + ctx.shape, "u"), _f64(p, pshape, "p"),
                               C.byref(st), _stream(ctx.device))
    if not (allow_noconv and code == L.EB_ENOCONV):
        check(code, "eb_rk2_step")
    return u, p, _stats(st)


def _stats(st):
    return {"it_mac": list(st.it_mac), "it_visc": list(st.it_visc),
            "it_proj": list(st.it_proj), "div_proj": list(st.div_proj),
            "vcycles": st.vcycles, "status": st.status, "fp64_fallbacks": st.fp64_fallbacks,
            "dt_stable": st.dt_stable}


def eb_stable_dt(ctx: EbContext, rheo: EbRheology, u, force=(0.0, 0.0, 0.0), c_cfl=0.5,
                 theta=None):
    """Time step of the paper's stability rule for the state u (host float)."""
    dt = C.c_double(0.0)
    f = (C.c_double * 3)(*[float(x) for x in force])
    th = _f64(theta, ctx.shape, "theta") if theta is not None else None
    check(L.lib().eb_stable_dt(ctx.ptr, C.byref(rheo), th, _f64(u, (3,) + ctx.shape, "u"), f,
                               float(c_cfl), C.byref(dt), _stream(ctx.device)), "eb_stable_dt")
    return dt.value


def eb_drag(ctx: EbContext, rheo: EbRheology, u, p, theta=None):
    F = (C.c_double * 3)()
    th = _f64(theta, ctx.shape, "theta") if theta is not None else None
    check(L.lib().eb_drag(ctx.ptr, C.byref(rheo), th, _f64(u, (3,) + ctx.shape, "u"),
                          _f64(p, ctx.shape, "p"), F, _stream(ctx.device)), "eb_drag")
    return [F[0], F[1], F[2]]


def eb_nodal_project(ctx: EbContext, u, pn, beta, opts: EbStepOpts, rtol=None):
    """Nodal end-of-stage projection of u with the nodal pressure pn (node_shape): returns
    (u, pn, max |D(u) - B| left, CG iterations), new tensors."""
    u = u.clone().contiguous()
    pn = pn.clone().contiguous()
    div = C.c_double(0.0)
    it = C.c_int(0)
    rt = opts.rtol_proj if rtol is None else rtol
    check(L.lib().eb_nodal_project(ctx.ptr, float(beta), _f64(u, (3,) + ctx.shape, "u"),
                                   _f64(pn, ctx.node_shape, "pn"), float(rt), C.byref(opts),
                                   C.byref(div), C.byref(it), _stream(ctx.device)),
          "eb_nodal_project")
    return u, pn, div.value, it.value


def eb_drag_nodal(ctx: EbContext, rheo: EbRheology, u, pn, theta=None):
    """Force on the body with a nodal pressure pn (node_shape)."""
    F = (C.c_double * 3)()
    th = _f64(theta, ctx.shape, "theta") if theta is not None else None
    check(L.lib().eb_drag_nodal(ctx.ptr, C.byref(rheo), th, _f64(u, (3,) + ctx.shape, "u"),
                                _f64(pn, ctx.node_shape, "pn"), F, _stream(ctx.device)),
          "eb_drag_nodal")
    return [F[0], F[1], F[2]]


def eb_drag_noalloc(ctx: EbContext, rheo: EbRheology, u, p, theta=None):
    """eb_drag with the library's static device scratch (no allocation, workspace untouched)."""
    F = (C.c_double * 3)()
    th = _f64(theta, ctx.shape, "theta") if theta is not None else None
    check(L.lib().eb_drag_noalloc(ctx.ptr, C.byref(rheo), th, _f64(u, (3,) + ctx.shape, "u"),
                                  _f64(p, ctx.shape, "p"), F, _stream(ctx.device)),
          "eb_drag_noalloc")
    return [F[0], F[1], F[2]]


def eb_pressure_gradient(ctx: EbContext, p):
    gp = ctx.vec()
    check(L.lib().eb_pressure_gradient(ctx.ptr, _f64(p, ctx.shape, "p"), _p(gp),
                                       _stream(ctx.device)), "eb_pressure_gradient")
    return gp


# ----------------------------------------------------------------------------------------------
# reverse mode
# ----------------------------------------------------------------------------------------------
def eb_tape_bytes(ctx: EbContext) -> int:
    return int(L.lib().eb_tape_bytes(ctx.ptr))


def new_tape(ctx: EbContext):
    return torch.empty(eb_tape_bytes(ctx), dtype=torch.uint8, device=ctx.device)


def eb_rk2_step_taped(ctx: EbContext, rheo: EbRheology, dt, opts: EbStepOpts, u, p, tape,
                      theta=None, inplace=False):
    """eb_rk2_step that records the step's tape (a uint8 tensor of eb_tape_bytes)."""
    if not inplace:
        u = u.clone().contiguous()
        p = p.clone().contiguous()
    if tape.numel() < eb_tape_bytes(ctx):
        raise ValueError("tape smaller than eb_tape_bytes")
    st = EbStepStats()
    th = _f64(theta, ctx.shape, "theta") if theta is not None else None
    check(L.lib().eb_rk2_step_taped(ctx.ptr, C.byref(rheo), th, float(dt), C.byref(opts),
                                    _f64(u, (3,) + ctx.shape, "u"), _f64(p, ctx.shape, "p"),
                                    _p(tape), C.byref(st), _stream(ctx.device)),
          "eb_rk2_step_taped")
    return u, p, _stats(st)


def _host_acc(acc):
    """A float64 numpy array of one element that the library adds d(loss)/d(tau0) into."""
    if acc is None:
        acc = np.zeros(1)
    if not (isinstance(acc, np.ndarray) and acc.dtype == np.float64 and acc.size == 1
            and acc.flags["C_CONTIGUOUS"]):
        raise ValueError("tau0bar must be a contiguous float64 numpy array of one element")
    return acc, acc.ctypes.data_as(C.POINTER(C.c_double))


def eb_rk2_step_adjoint(ctx: EbContext, rheo: EbRheology, dt, opts: EbStepOpts, u0, tape, ub,
                        pb, theta=None, tau0b=None, thetab=None, tau0bar=None):
    """Adjoint of the step taped from u0.  Returns (ub_in, pb_in, tau0b, stats).  The step's
    yield-stress adjoint is added into tau0b (per cell; a new zero tensor when None), into
    thetab (d/d theta per cell, when given) and into tau0bar (a one-element float64 numpy
    array, d/d tau0, when given); stats["tau0bar"] is that array's value after the call."""
    ub = ub.clone().contiguous()
    pb = pb.clone().contiguous()
    tb = ctx.scalar() if tau0b is None else tau0b
    st = EbStepStats()
    th = _f64(theta, ctx.shape, "theta") if theta is not None else None
    thb = _f64(thetab, ctx.shape, "thetab") if thetab is not None else None
    acc, accp = _host_acc(tau0bar)
    check(L.lib().eb_rk2_step_adjoint(ctx.ptr, C.byref(rheo), th, float(dt), C.byref(opts),
                                      _f64(u0, (3,) + ctx.shape, "u0"), _p(tape),
                                      _f64(ub, (3,) + ctx.shape, "ub"),
                                      _f64(pb, ctx.shape, "pb"), _f64(tb, ctx.shape, "tau0b"),
                                      thb, accp, C.byref(st), _stream(ctx.device)),
          "eb_rk2_step_adjoint")
    stats = _stats(st)
    stats["tau0bar"] = float(acc[0])
    return ub, pb, tb, stats


def eb_drag_adjoint(ctx: EbContext, rheo: EbRheology, u, fbar, theta=None, ub=None, pb=None,
                    tau0b=None, thetab=None, tau0bar=None):
    """Adjoint of eb_drag at u; (ub, pb, tau0b) accumulate into the tensors given (or zeros),
    thetab (d/d theta per cell) and tau0bar (one-element float64 numpy array, d/d tau0) when
    given.  Returns (ub, pb, tau0b, d/d tau0 after the call)."""
    ub = ctx.vec() if ub is None else ub
    pb = ctx.scalar() if pb is None else pb
    tb = ctx.scalar() if tau0b is None else tau0b
    fb = (C.c_double * 3)(*[float(x) for x in fbar])
    th = _f64(theta, ctx.shape, "theta") if theta is not None else None
    thb = _f64(thetab, ctx.shape, "thetab") if thetab is not None else None
    acc, accp = _host_acc(tau0bar)
    check(L.lib().eb_drag_adjoint(ctx.ptr, C.byref(rheo), th, _f64(u, (3,) + ctx.shape, "u"), fb,
                                  _f64(ub, (3,) + ctx.shape, "ub"), _f64(pb, ctx.shape, "pb"),
                                  _f64(tb, ctx.shape, "tau0b"), thb, accp,
                                  _stream(ctx.device)),
          "eb_drag_adjoint")
    return ub, pb, tb, float(acc[0])


def eb_mac_project_adjoint(ctx: EbContext, fb, beta, opts: EbStepOpts, rtol=None):
    f = [a.clone().contiguous() for a in fb]
    for a, s in zip(f, ctx.face_shapes):
        _f64(a, s, "face")
    it = C.c_int(0)
    rt = opts.rtol_mac if rtol is None else rtol
    check(L.lib().eb_mac_project_adjoint(ctx.ptr, float(beta), _p(f[0]), _p(f[1]), _p(f[2]),
                                         float(rt), C.byref(opts), C.byref(it),
                                         _stream(ctx.device)), "eb_mac_project_adjoint")
    return f, it.value


def eb_cc_project_adjoint(ctx: EbContext, ub, pb, beta, opts: EbStepOpts, rtol=None):
    ub = ub.clone().contiguous()
    pb = pb.clone().contiguous()
    it = C.c_int(0)
    rt = opts.rtol_proj if rtol is None else rtol
    check(L.lib().eb_cc_project_adjoint(ctx.ptr, float(beta), _f64(ub, (3,) + ctx.shape, "ub"),
                                        _f64(pb, ctx.shape, "pb"), float(rt), C.byref(opts),
                                        C.byref(it), _stream(ctx.device)),
          "eb_cc_project_adjoint")
    return ub, pb, it.value


def eb_visc_solve_adjoint(ctx: EbContext, rho, dt, eta, eta_eb, x, xb, opts: EbStepOpts,
                          rtol=None):
    psib = ctx.vec()
    etab = ctx.scalar()
    etaebb = ctx.zeros(max(ctx.ncut, 1))
    it = C.c_int(0)
    rt = opts.rtol_visc if rtol is None else rtol
    check(L.lib().eb_visc_solve_adjoint(ctx.ptr, float(rho), float(dt),
                                        _f64(eta, ctx.shape, "eta"), _p(_eb_arr(ctx, eta_eb)),
                                        _f64(x, (3,) + ctx.shape, "x"),
                                        _f64(xb, (3,) + ctx.shape, "xb"), float(rt),
                                        C.byref(opts), _p(psib), _p(etab), _p(etaebb),
                                        C.byref(it), _stream(ctx.device)),
          "eb_visc_solve_adjoint")
    return psib, etab, etaebb[: ctx.ncut], it.value


def eb_derived_adjoint(ctx: EbContext, rheo: EbRheology, u, opts: EbStepOpts, Cb, etab, etaebb,
                       Vb, theta=None):
    ub = ctx.vec()
    tb = ctx.scalar()
    it = C.c_int(0)
    th = _f64(theta, ctx.shape, "theta") if theta is not None else None
    check(L.lib().eb_derived_adjoint(ctx.ptr, C.byref(rheo), th, _f64(u, (3,) + ctx.shape, "u"),
                                     _f64(Cb, (3,) + ctx.shape, "Cb"),
                                     _f64(etab, ctx.shape, "etab"), _p(_eb_arr(ctx, etaebb)),
                                     _f64(Vb, (3,) + ctx.shape, "Vb"), _p(ub), _p(tb),
                                     C.byref(opts), C.byref(it), _stream(ctx.device)),
          "eb_derived_adjoint")
    return ub, tb, it.value
