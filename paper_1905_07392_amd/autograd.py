"""torch.autograd bindings of the RK2 step and of the drag on the embedded body.

The reverse sweep is the library's own hand-written adjoint (eb_rk2_step_adjoint,
eb_drag_adjoint); these classes only route tensors.  The yield stress is split as
tau0_c = tau0 * theta_c: `tau0` is a 0-d float64 tensor (the Bingham number when mu, U and L are
1) and `theta` the per-cell multiplier (None means 1 everywhere; its gradient is then None).  The
library itself forms d/d tau0 = sum_c theta_c tau0b_c (into a host accumulator) and
d/d theta_c = tau0 tau0b_c (into a device tensor) from its per-cell yield-stress adjoint tau0b.

* ``EbRK2Step``  one step; keeps that step's tape (eb_tape_bytes of device memory) until backward.
* ``EbRollout``  n steps with step checkpointing: forward keeps (u, p) every ``ckpt_every`` steps;
  backward recomputes each segment from its checkpoint with tapes, then runs the step adjoints
  of the segment in reverse.  Peak memory is ckpt_every tapes plus n/ckpt_every states.
* ``EbDrag``     the force F on the body (Eq. drag-force) as a [3] tensor.
"""
from __future__ import annotations

import numpy as np
import torch

from . import api


def _rheo_with(rheo, tau0: float):
    r = api.EbRheology()
    r.law, r.mu, r.eps, r.rho = rheo.law, rheo.mu, rheo.eps, rheo.rho
    r.kappa, r.n, r.eta0 = rheo.kappa, rheo.n, rheo.eta0
    r.tau0 = float(tau0)
    return r


def _zeros_like_or(g, like):
    return torch.zeros_like(like) if g is None else g.contiguous()


def _yield_outputs(theta, tau0):
    """The buffers the library adds the yield-stress gradients into: d/d theta (a device
    tensor, or None without a theta field) and d/d tau0 (a one-element host array)."""
    thetab = torch.zeros_like(theta) if theta is not None else None
    return thetab, np.zeros(1)


def _tau0_grad(acc, tau0):
    return torch.from_numpy(acc.reshape(())).to(dtype=torch.float64, device=tau0.device)


class EbRK2Step(torch.autograd.Function):
    @staticmethod
    def forward(fctx, u, p, theta, tau0, ectx, rheo, dt, opts):
        rh = _rheo_with(rheo, float(tau0))
        tape = api.new_tape(ectx)
        un, pn, _ = api.eb_rk2_step_taped(ectx, rh, dt, opts, u.contiguous(), p.contiguous(),
                                          tape, theta=theta)
        fctx.save_for_backward(u.contiguous(), theta, tau0)
        fctx.tape, fctx.ectx, fctx.rh, fctx.dt, fctx.opts = tape, ectx, rh, dt, opts
        return un, pn

    @staticmethod
    def backward(fctx, gu, gp):
        u, theta, tau0 = fctx.saved_tensors
        ub = _zeros_like_or(gu, u)
        pb = _zeros_like_or(gp, u[0])
        thetab, acc = _yield_outputs(theta, tau0)
        ub, pb, _, _ = api.eb_rk2_step_adjoint(fctx.ectx, fctx.rh, fctx.dt, fctx.opts, u,
                                               fctx.tape, ub, pb, theta=theta, thetab=thetab,
                                               tau0bar=acc)
        fctx.tape = None
        return ub, pb, thetab, _tau0_grad(acc, tau0), None, None, None, None


class EbRollout(torch.autograd.Function):
    @staticmethod
    def forward(fctx, u0, p0, theta, tau0, ectx, rheo, dt, opts, nsteps, ckpt_every):
        rh = _rheo_with(rheo, float(tau0))
        u, p = u0.contiguous().clone(), p0.contiguous().clone()
        ckpts = []
        for s in range(nsteps):
            if s % ckpt_every == 0:
                ckpts.append((u.clone(), p.clone()))
            api.eb_rk2_step(ectx, rh, dt, opts, u, p, theta=theta, inplace=True)
        fctx.save_for_backward(theta, tau0)
        fctx.ckpts, fctx.ectx, fctx.rh, fctx.dt, fctx.opts = ckpts, ectx, rh, dt, opts
        fctx.nsteps, fctx.every = nsteps, ckpt_every
        return u, p

    @staticmethod
    def backward(fctx, gu, gp):
        theta, tau0 = fctx.saved_tensors
        ectx, rh, dt, opts = fctx.ectx, fctx.rh, fctx.dt, fctx.opts
        n, every = fctx.nsteps, fctx.every
        ub = _zeros_like_or(gu, fctx.ckpts[0][0])
        pb = _zeros_like_or(gp, fctx.ckpts[0][1])
        thetab, acc = _yield_outputs(theta, tau0)
        tb = ectx.scalar()  # per-cell adjoint the library accumulates; not returned
        tapes = [api.new_tape(ectx) for _ in range(min(every, n))]
        for seg in range(len(fctx.ckpts) - 1, -1, -1):
            s0 = seg * every
            s1 = min(s0 + every, n)
            u, p = fctx.ckpts[seg][0].clone(), fctx.ckpts[seg][1].clone()
            inputs = []
            for s in range(s0, s1):  # recompute the segment, recording each step's tape
                inputs.append(u.clone())
                api.eb_rk2_step_taped(ectx, rh, dt, opts, u, p, tapes[s - s0], theta=theta,
                                      inplace=True)
            for s in range(s1 - 1, s0 - 1, -1):
                ub, pb, _, _ = api.eb_rk2_step_adjoint(ectx, rh, dt, opts, inputs[s - s0],
                                                       tapes[s - s0], ub, pb, theta=theta,
                                                       tau0b=tb, thetab=thetab, tau0bar=acc)
        fctx.ckpts = None
        return ub, pb, thetab, _tau0_grad(acc, tau0), None, None, None, None, None, None


class EbDrag(torch.autograd.Function):
    @staticmethod
    def forward(fctx, u, p, theta, tau0, ectx, rheo):
        rh = _rheo_with(rheo, float(tau0))
        F = api.eb_drag(ectx, rh, u.contiguous(), p.contiguous(), theta=theta)
        fctx.save_for_backward(u.contiguous(), theta, tau0)
        fctx.ectx, fctx.rh = ectx, rh
        return torch.tensor(F, dtype=torch.float64, device=u.device)

    @staticmethod
    def backward(fctx, gF):
        u, theta, tau0 = fctx.saved_tensors
        fbar = [float(x) for x in gF.detach().cpu()]
        thetab, acc = _yield_outputs(theta, tau0)
        ub, pb, _, _ = api.eb_drag_adjoint(fctx.ectx, fctx.rh, u, fbar, theta=theta,
                                           thetab=thetab, tau0bar=acc)
        return ub, pb, thetab, _tau0_grad(acc, tau0), None, None


def rk2_step(ectx, rheo, dt, opts, u, p, theta, tau0):
    """One differentiable step: (u, p) -> (u_new, p_new)."""
    return EbRK2Step.apply(u, p, theta, tau0, ectx, rheo, dt, opts)


def rollout(ectx, rheo, dt, opts, u0, p0, theta, tau0, nsteps, ckpt_every=5):
    """nsteps differentiable steps with checkpointing every ckpt_every steps."""
    return EbRollout.apply(u0, p0, theta, tau0, ectx, rheo, dt, opts, int(nsteps),
                           int(ckpt_every))


def drag(ectx, rheo, u, p, theta, tau0):
    """Differentiable force on the body, a [3] float64 tensor on u's device."""
    return EbDrag.apply(u, p, theta, tau0, ectx, rheo)


__all__ = ["EbRK2Step", "EbRollout", "EbDrag", "rk2_step", "rollout", "drag"]
