"""ORACLE — test infrastructure only.  Unrolled preconditioned SVRG in FP64
torch operations, so that torch autograd gives the reference gradient of a loss
of the final image with respect to the initial image and log(beta).

The forward pass follows Algorithm 1 (Appendix B) with the clipped step of
eq. (sgm) and the estimator exactly as the algorithm states it,
g = n (grad J_i(x) - grad J_i(x_snap)) + sum_j grad J_j(x_snap) with
J_i = D_i + (beta / n) S.  Every operation is a plain definition:

* the Joseph pair of the oracle projector is a linear operator whose adjoint is
  the oracle back projection (and vice versa);
* the image-space resolution model G (Section 3.1; oracle.psf) is a symmetric
  linear operator, its own adjoint, applied before the forward projection and
  after the back projection (A = P G);
* the prior gradient and Hessian diagonal are the closed forms of Appendix A,
  written with grid shifts over the in-grid neighbours;
* the preconditioner is eq. (preconditioner) with the harmonic combination,
  D = 0 where its denominator is 0;
* the clip max(0, u) passes the gradient only where u > 0 (a tie passes none).

The constants eps and delta are fixed inputs (they are computed once from the
initial image and not differentiated).
"""

import numpy as np
import torch
import torch.nn.functional as F

from . import projector, psf, rdp


class _Fwd(torch.autograd.Function):
    """P x for the LORs (p1, p2); adjoint = oracle back projection."""

    @staticmethod
    def forward(ctx, x, cfg, p1, p2):
        ctx.cfg, ctx.p1, ctx.p2 = cfg, p1, p2
        return torch.from_numpy(projector.fwd(cfg, x.detach().numpy(), p1, p2))

    @staticmethod
    def backward(ctx, g):
        img = projector.back(ctx.cfg, g.detach().contiguous().numpy(), ctx.p1, ctx.p2)
        return torch.from_numpy(img), None, None, None


class _Back(torch.autograd.Function):
    """P^T s for the LORs (p1, p2); adjoint = oracle forward projection."""

    @staticmethod
    def forward(ctx, s, cfg, p1, p2):
        ctx.cfg, ctx.p1, ctx.p2 = cfg, p1, p2
        ctx.shape = s.shape
        return torch.from_numpy(projector.back(cfg, s.detach().contiguous().numpy(), p1, p2))

    @staticmethod
    def backward(ctx, g):
        out = projector.fwd(ctx.cfg, g.detach().contiguous().numpy(), ctx.p1, ctx.p2)
        return torch.from_numpy(out).reshape(ctx.shape), None, None, None


class _Blur(torch.autograd.Function):
    """G x (the resolution model of cfg, the identity without one); G is
    symmetric, so the adjoint is G again."""

    @staticmethod
    def forward(ctx, x, cfg):
        ctx.cfg = cfg
        return torch.from_numpy(psf.blur(x.detach().numpy(), cfg))

    @staticmethod
    def backward(ctx, g):
        return torch.from_numpy(psf.blur(g.detach().contiguous().numpy(), ctx.cfg)), None


def _embed(c, shape, I):
    """Place c (the values at slice tuple I) into a zero tensor of `shape`."""
    pads = []
    for n, sl in reversed(list(zip(shape, I))):
        pads += [sl.start, n - sl.stop]
    return F.pad(c, pads)


def prior_grad(x, w, gamma, eps, kappa=None):
    """dS/dx (Appendix A) for x [nz][ny][nx]."""
    k = torch.ones_like(x) if kappa is None else kappa
    g = torch.zeros_like(x)
    for off, wij in w.items():
        I, J = rdp._pairs(tuple(x.shape), off)
        d = x[I] - x[J]
        phi = x[I] + x[J] + gamma * torch.abs(d) + eps
        g = g + _embed(wij * k[I] * k[J] * d * (2 * phi - (d + gamma * torch.abs(d))) / phi ** 2, x.shape, I)
    return g


def prior_hessdiag(x, w, gamma, eps, kappa=None):
    """Diagonal of the Hessian of S (Appendix A)."""
    k = torch.ones_like(x) if kappa is None else kappa
    h = torch.zeros_like(x)
    for off, wij in w.items():
        I, J = rdp._pairs(tuple(x.shape), off)
        phi = x[I] + x[J] + gamma * torch.abs(x[I] - x[J]) + eps
        h = h + _embed(2 * wij * k[I] * k[J] * (2 * x[J] + eps) ** 2 / phi ** 3, x.shape, I)
    return h


def preconditioner(x, sens, beta, w, gamma, eps, alpha, delta, kappa=None):
    """Eq. (preconditioner): (x + delta) / (sens + alpha beta h_S(x) (x + delta))."""
    xd = x + delta
    den = sens + alpha * beta * prior_hessdiag(x, w, gamma, eps, kappa) * xd
    ok = den != 0
    return torch.where(ok, xd / torch.where(ok, den, torch.ones_like(den)), torch.zeros_like(den))


class Unrolled:
    """FP64 torch form of one reconstruction problem (oracle.recon.Problem's
    data and subsets)."""

    def __init__(self, prob):
        self.prob = prob
        self.cfg = prob.cfg
        self.n = prob.n
        self.shape = prob.shape
        self.y = [torch.from_numpy(v) for v in prob.y]
        self.r = [torch.from_numpy(v) for v in prob.r]
        self.a = [torch.from_numpy(v) for v in prob.a]
        self.sens = torch.from_numpy(prob.sens())
        self.kappa = None if prob.kappa is None else torch.from_numpy(prob.kappa)

    def data_grad(self, x, i):
        """grad D_i(x) = G P_i^T [a (1 - y / (a P_i G x + r))]."""
        p1, p2 = self.prob.lors[i]
        yb = self.a[i] * _Fwd.apply(_Blur.apply(x, self.cfg), self.cfg, p1, p2) + self.r[i]
        return _Blur.apply(_Back.apply(self.a[i] * (1.0 - self.y[i] / yb), self.cfg, p1, p2), self.cfg)

    def grad_J(self, x, i, beta):
        p = self.prob
        return self.data_grad(x, i) + beta / self.n * prior_grad(x, p.w, p.gamma, p.eps, self.kappa)

    def svrg(self, x0, log_beta, n_epochs, orders, taus, update_iters, omega=2, clip_masks=None, record=None):
        """Final image after n_epochs epochs of Algorithm 1 (clipped step);
        orders[e][j] is the subset of iteration j of epoch e, taus[e][j] its
        step size, update_iters the iterations that recompute D.

        clip_masks (one boolean image per iteration) replaces the clip by the
        fixed selection u * mask: the map restricted to one smooth piece, whose
        derivative at the run that recorded the masks (record: a list that
        receives [u > 0] per iteration) equals the clipped map's."""
        p = self.prob
        n = self.n
        beta = torch.exp(log_beta)
        x = x0
        D = None
        ghat_i = [None] * n
        ghat = None
        for k in range(n_epochs * n):
            e, j = divmod(k, n)
            if k in update_iters:
                D = preconditioner(x, self.sens, beta, p.w, p.gamma, p.eps, p.alpha, p.delta, self.kappa)
            if k % (omega * n) == 0:
                ghat_i = [self.grad_J(x, i, beta) for i in range(n)]
                ghat = sum(ghat_i)
                g = ghat
            else:
                i = int(orders[e][j])
                g = n * (self.grad_J(x, i, beta) - ghat_i[i]) + ghat
            u = x - float(taus[e][j]) * D * g
            if record is not None:
                record.append((u > 0).detach().clone())
            if clip_masks is not None:
                x = u * clip_masks[k]
            else:
                x = torch.where(u > 0, u, torch.zeros_like(u))
        return x


def loss_and_grads(prob, x0, log_beta, x_target, n_epochs, orders, taus, update_iters, omega=2):
    """L = ||x_final - x_target||^2 and (dL/dx0, dL/dlog beta) by autograd (FP64)."""
    u = Unrolled(prob)
    x0t = torch.tensor(np.asarray(x0, np.float64).reshape(prob.shape), requires_grad=True)
    lb = torch.tensor(float(log_beta), dtype=torch.float64, requires_grad=True)
    xf = u.svrg(x0t, lb, n_epochs, orders, taus, update_iters, omega)
    tgt = torch.from_numpy(np.asarray(x_target, np.float64).reshape(prob.shape))
    L = ((xf - tgt) ** 2).sum()
    L.backward()
    return float(L.detach()), x0t.grad.numpy().copy(), float(lb.grad), xf.detach().numpy()


def loss(prob, x0, log_beta, x_target, n_epochs, orders, taus, update_iters, omega=2, clip_masks=None, record=None):
    """L only (no graph), for finite differences; clip_masks / record as in
    Unrolled.svrg."""
    u = Unrolled(prob)
    with torch.no_grad():
        x0t = torch.from_numpy(np.asarray(x0, np.float64).reshape(prob.shape).copy())
        xf = u.svrg(x0t, torch.tensor(float(log_beta), dtype=torch.float64), n_epochs, orders, taus, update_iters,
                    omega, clip_masks, record)
        tgt = torch.from_numpy(np.asarray(x_target, np.float64).reshape(prob.shape))
        return float(((xf - tgt) ** 2).sum())
