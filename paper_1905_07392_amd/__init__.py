"""MI355X-native embedded-boundary viscoplastic RK2 step (HIP kernels for gfx950 behind a C ABI).

The numerical work lives in libeb.so (csrc/, declared in include/eb.h); this package only
marshals torch tensors to it.  `paper_1905_07392_amd.api` holds one Python function per C
entry point.
"""
from __future__ import annotations


def from_workload(w, precision=0, rtol=None, max_iter=400, projection=0):
    """(box, body, rheology, opts) structs for an object with the workload attributes
    (n, h, lo, periodic, wall_u, body dict, law, mu, tau0, eps, rho, force, rtol)."""
    from . import api

    box = api.make_box(w.n, w.h, w.lo, w.periodic, w.wall_u)
    bd = dict(w.body)
    body = api.make_body(kind=bd.get("kind", 0), center=bd.get("center", (0.5, 0.5, 0.5)),
                         radius=bd.get("radius"), radii=bd.get("radii"),
                         euler_zyx=bd.get("euler_zyx", (0.0, 0.0, 0.0)),
                         zlo=bd.get("zlo", 0.0), zhi=bd.get("zhi", 1.0),
                         plane_n=bd.get("plane_n", (0.0, 0.0, 1.0)),
                         plane_d=bd.get("plane_d", 0.0), u_eb=bd.get("u_eb", (0.0, 0.0, 0.0)))
    rheo = api.make_rheology(w.law, w.mu, w.tau0, w.eps, w.rho, w.kappa, w.flow_n, w.eta0)
    opts = api.make_opts(precision=precision, rtol=w.rtol if rtol is None else rtol,
                         max_iter=max_iter, force=w.force, projection=projection)
    return box, body, rheo, opts
