"""Failure codes of the C ABI on the GPU path, each forced from the host (every kernel still
exits normally): a solve that cannot reach its tolerance (EB_ENOCONV), a non-finite state
(EB_ENAN) and a wall-flux stencil that leaves a non-periodic box (EB_EGEOM).  After a failed
solve the same context must still give the clean result bit for bit."""
import numpy as np
import pytest

import eb_inputs as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _require_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _setup(max_iter=400, rtol=None):
    import paper_1905_07392_amd as pkg
    from paper_1905_07392_amd import api

    _require_gpu()
    w = I.sphere_n(16, radius=0.25)
    box, body, rheo, opts = pkg.from_workload(w, max_iter=max_iter, rtol=rtol)
    ctx = api.eb_geometry_build(box, body, "cuda:0")
    u = torch.from_numpy(I.initial_velocity(w)).to("cuda:0")
    return w, api, ctx, rheo, opts, u


def test_enoconv_when_the_tolerance_is_out_of_reach():
    from paper_1905_07392_amd._lib import EB_ENOCONV, EbError

    w, api, ctx, rheo, opts, u = _setup()
    print("[errors] EB_ENOCONV: viscous solve, max_iter 1, rtol 1e-300", flush=True)
    eta, eta_eb = api.eb_apparent_viscosity(ctx, rheo, u)
    psi = u * w.rho
    tight = api.make_opts(rtol=1e-300, max_iter=1)
    with pytest.raises(EbError) as ei:
        api.eb_visc_solve(ctx, w.rho, w.dt, eta, eta_eb, psi, u, tight)
    assert ei.value.code == EB_ENOCONV and "no convergence" in str(ei.value)
    # a whole step at that setting reports the code in its stats and keeps finite iterates
    p = ctx.scalar()
    u1, p1, st = api.eb_rk2_step(ctx, rheo, w.dt, tight, u, p, allow_noconv=True)
    assert st["status"] == EB_ENOCONV
    assert torch.isfinite(u1).all() and torch.isfinite(p1).all()
    # the context is still sound: a clean step equals one on a fresh context, bit for bit
    ua, pa, _ = api.eb_rk2_step(ctx, rheo, w.dt, opts, u, ctx.scalar())
    _, _, ctx2, _, _, _ = _setup()
    ub, pb, _ = api.eb_rk2_step(ctx2, rheo, w.dt, opts, u, ctx2.scalar())
    assert torch.equal(ua, ub) and torch.equal(pa, pb)


def test_enan_on_a_non_finite_state():
    from paper_1905_07392_amd._lib import EB_ENAN, EbError

    w, api, ctx, rheo, opts, u = _setup()
    print("[errors] EB_ENAN: one open cell of the velocity set to NaN", flush=True)
    bad = u.clone()
    c = ctx.shape[0] // 2
    bad[0, c, c, 1] = float("nan")  # an open cell away from the sphere
    with pytest.raises(EbError) as ei:
        api.eb_rk2_step(ctx, rheo, w.dt, opts, bad, ctx.scalar())
    assert ei.value.code == EB_ENAN and "non-finite" in str(ei.value)
    ua, pa, _ = api.eb_rk2_step(ctx, rheo, w.dt, opts, u, ctx.scalar())
    _, _, ctx2, _, _, _ = _setup()
    ub, pb, _ = api.eb_rk2_step(ctx2, rheo, w.dt, opts, u, ctx2.scalar())
    assert torch.equal(ua, ub) and torch.equal(pa, pb)


def test_egeom_when_a_wall_stencil_leaves_the_box():
    """A sphere touching the lower z wall of a closed box: the cut cells under it have normals
    pointing down, so their stencil planes (one and two cells further down) lie outside the box.
    The oracle refuses the same geometry."""
    import paper_1905_07392_amd as pkg
    from oracle import oracle as O
    from paper_1905_07392_amd import api
    from paper_1905_07392_amd._lib import EB_EGEOM, EbError

    _require_gpu()
    w = I.sphere_n(32, radius=0.08).replace(name="sphere_low")
    w.body = {"kind": I.BODY_SPHERE, "center": (0.5, 0.5, 0.1), "radius": 0.08}
    print("[errors] EB_EGEOM: sphere at z = 0.1, r = 0.08 in a closed 32^3 box", flush=True)
    assert O.Geometry(w).err == -2  # the oracle's wall-stencil error (outside the box)
    box, body, _, _ = pkg.from_workload(w)
    with pytest.raises(EbError) as ei:
        api.eb_geometry_build(box, body, "cuda:0")
    assert ei.value.code == EB_EGEOM and "flags 0x4 " in str(ei.value)
    # the library still builds a valid geometry afterwards
    ok = I.sphere_n(32, radius=0.2)
    box, body, _, _ = pkg.from_workload(ok)
    ctx = api.eb_geometry_build(box, body, "cuda:0")
    assert ctx.ncut == O.Geometry(ok).ncut
