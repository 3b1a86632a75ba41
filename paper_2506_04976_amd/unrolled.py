"""Differentiable unrolled preconditioned SVRG (Algorithm 1 with the clipped
step of eq. (sgm)) as a torch.autograd.Function over the library's HIP
kernels.

Forward: pet_svrg_epoch per epoch, keeping one checkpoint per epoch (the
iterate at the epoch start and the preconditioner in effect).  Backward:
pet_svrg_epoch_vjp per epoch in reverse order; each call recomputes its epoch
from the checkpoint (memory stays at one epoch of iterates) and returns
dL/dx at the epoch start, while the adjoints of the preconditioner and of the
snapshot table are carried to the previous epoch.  The gradient with respect
to log(beta) is beta dL/dbeta.  eps and delta are constants of the problem.
"""

import math

import torch

from . import _lib as L


class UnrolledProblem:
    """Data and schedule of one unrolled reconstruction.

    orders[e][j], taus[e][j], updates[e][j]: subset, step size and
    preconditioner-update flag of iteration j of epoch e (host values)."""

    def __init__(self, geom, y, add, mult, sens, gamma, eps, alpha, delta, orders, taus, updates, w27=None,
                 kappa=None, omega=2):
        self.geom, self.y, self.add, self.mult, self.sens = geom, y, add, mult, sens
        self.gamma, self.eps, self.alpha, self.delta = float(gamma), float(eps), float(alpha), float(delta)
        self.orders = [[int(v) for v in o] for o in orders]
        self.taus = [[float(v) for v in t] for t in taus]
        self.updates = [[bool(v) for v in u] for u in updates]
        self.n_epochs = len(self.orders)
        self.w27 = w27 if w27 is not None else L.rdp_weights27(geom.cfg["vx"], geom.cfg["vy"], geom.cfg["vz"])
        self.kappa = kappa
        self.omega = int(omega)

    def state(self, beta):
        return L.SvrgStateBuffers(self.geom, self.y, self.add, self.mult, self.sens, beta=beta, gamma=self.gamma,
                                  eps=self.eps, alpha=self.alpha, delta=self.delta, w27=self.w27,
                                  kappa=self.kappa, omega=self.omega)


class UnrolledSVRG(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x0, log_beta, prob):
        beta = math.exp(float(log_beta))
        st = prob.state(beta)
        x = x0.detach().to(torch.float32).contiguous().clone()
        ckpt = []
        for e in range(prob.n_epochs):
            ckpt.append((x.clone(), st.D.clone()))
            L.pet_svrg_epoch(prob.geom, st, x, prob.orders[e], prob.taus[e], prob.updates[e])
        ctx.prob, ctx.beta, ctx.ckpt = prob, beta, ckpt
        ctx.lb_dtype = log_beta.dtype
        return x

    @staticmethod
    def backward(ctx, grad_x):
        prob, beta, ckpt = ctx.prob, ctx.beta, ctx.ckpt
        geom = prob.geom
        n = geom.n_subsets
        st = prob.state(beta)
        bufs = L.VjpBuffers(geom, grad_x.device)
        bufs.xbar.copy_(grad_x)
        period = prob.omega * n
        for e in reversed(range(prob.n_epochs)):
            k0 = e * n
            snap_epoch = (k0 // period) * period // n
            bufs.set_checkpoint(ckpt[e][0], None if k0 % period == 0 else ckpt[snap_epoch][0], ckpt[e][1])
            st.c.k = k0
            L.pet_svrg_epoch_vjp(geom, st, bufs, prob.orders[e], prob.taus[e], prob.updates[e])
        dlb = float(bufs.betabar.item()) * beta
        return bufs.xbar.clone(), torch.tensor(dlb, dtype=ctx.lb_dtype, device=grad_x.device), None


def unrolled_svrg(x0, log_beta, prob):
    """Final image of prob.n_epochs SVRG epochs from x0, differentiable with
    respect to x0 and log_beta (a 0-dim tensor)."""
    return UnrolledSVRG.apply(x0, log_beta, prob)
