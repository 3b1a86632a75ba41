"""ORACLE — test infrastructure only.  Problem assembly, preconditioners and the
iterative algorithms in FP64, following the paper's notation.

Problem (eq. (template)): min_x sum_i J_i(x) + i_{>=0}(x) with
J_i(x) = D_i(x) + (beta/n) S(x), D_i the KL data term of subset S_i and S the
relative difference prior.  Subsets are interleaved views: S_i holds views
v = i, i + n, i + 2n, ... (Section 2.4).
"""

import numpy as np

from synth import configs
from . import poisson, projector, psf, rdp


class Problem:
    """Data, geometry and prior settings of one reconstruction (FP64)."""

    def __init__(self, cfg, y, r, mult, beta, gamma, eps, w=None, kappa=None, alpha=1.0,
                 delta=None, subset_views=None):
        self.cfg = cfg
        self.n = cfg["n_subsets"]
        T = cfg["n_tof"]
        self.T = T
        if subset_views is None:
            subset_views = [configs.subset_views(cfg, i) for i in range(self.n)]
        self.views = subset_views
        self.lors = [projector.view_lors(cfg, v) for v in self.views]
        y = np.asarray(y)
        self.y = [np.asarray(y[v], np.float64).reshape(-1, T) for v in self.views]
        self.r = [np.asarray(r[v], np.float64).reshape(-1, T) for v in self.views]
        self.a = [np.asarray(mult[v], np.float64).reshape(-1, 1) for v in self.views]
        self.beta, self.gamma, self.eps = float(beta), float(gamma), float(eps)
        self.alpha = float(alpha)
        self.delta = float(delta) if delta is not None else None
        self.kappa = None if kappa is None else np.asarray(kappa, np.float64)
        self.w = w if w is not None else rdp.default_weights(cfg["vx"], cfg["vy"], cfg["vz"], cfg["nz"])
        self.shape = (cfg["nz"], cfg["ny"], cfg["nx"])
        self._sens = None
        self._sens_i = {}

    # --- data term -------------------------------------------------------
    def fwd(self, x, i):
        """P_i G x (G: the resolution model, the identity without one)."""
        p1, p2 = self.lors[i]
        return projector.fwd(self.cfg, psf.blur(np.asarray(x, np.float64).reshape(self.shape), self.cfg), p1, p2)

    def back(self, s, i):
        """G P_i^T s."""
        p1, p2 = self.lors[i]
        return psf.blur(projector.back(self.cfg, s, p1, p2), self.cfg)

    def ybar(self, x, i):
        """Expected data A_i x + r_i of subset i, [N_i, T]."""
        return self.a[i] * self.fwd(x, i) + self.r[i]

    def data_grad(self, x, i):
        """Gradient of D_i: A_i^T (1 - y / ybar) = P_i^T (a (1 - y / ybar))."""
        yb = self.ybar(x, i)
        return self.back(self.a[i] * poisson.kl_grad_s(yb, self.y[i]), i)

    def data_value(self, x):
        return float(sum(np.sum(poisson.kl(self.ybar(x, i), self.y[i])) for i in range(self.n)))

    # --- prior -------------------------------------------------------------
    def prior_grad(self, x):
        """Gradient of beta S."""
        return self.beta * rdp.grad(x, self.w, self.gamma, self.eps, self.kappa)

    def prior_hessdiag(self, x):
        """Diagonal of the Hessian of beta S."""
        return self.beta * rdp.hessdiag(x, self.w, self.gamma, self.eps, self.kappa)

    def prior_value(self, x):
        return self.beta * rdp.value(x, self.w, self.gamma, self.eps, self.kappa)

    # --- smooth objective pieces -------------------------------------------
    def grad_J(self, x, i):
        """Gradient of J_i = D_i + (beta/n) S."""
        return self.data_grad(x, i) + self.prior_grad(x) / self.n

    def full_grad(self, x):
        return sum(self.data_grad(x, i) for i in range(self.n)) + self.prior_grad(x)

    def objective(self, x):
        """D(Ax + r, y) + beta S(x) + i_{>=0}(x)."""
        if np.any(np.asarray(x) < 0):
            return np.inf
        return self.data_value(x) + self.prior_value(x)

    def sens_subset(self, i):
        """A_i^T 1 = P_i^T a (a broadcast over TOF bins)."""
        if i not in self._sens_i:
            self._sens_i[i] = self.back(np.repeat(self.a[i], self.T, axis=1), i)
        return self._sens_i[i]

    def sens(self):
        """A^T 1 over all subsets."""
        if self._sens is None:
            self._sens = sum(self.sens_subset(i) for i in range(self.n))
        return self._sens


# --- preconditioners (Section 2.3) ----------------------------------------
def precond_mlem(x, sens, delta):
    """D_MLEM = (x + delta) / A^T 1."""
    return (np.asarray(x, np.float64) + delta) / sens


def precond_prior(hess_betaS):
    """D_betaS = 1 / diag(H_betaS)."""
    return 1.0 / hess_betaS


def precond_harmonic(x, sens, hess_betaS, alpha, delta):
    """D = (x + delta) / (A^T 1 + alpha diag(H_betaS) (x + delta)), eq. (preconditioner).
    A voxel whose denominator vanishes (no data, no prior curvature) gets D = 0."""
    x = np.asarray(x, np.float64)
    den = sens + alpha * hess_betaS * (x + delta)
    out = np.zeros_like(x)
    nz = den != 0
    out[nz] = (x + delta)[nz] / den[nz]
    return out


# --- stepsize rules (Section 2.2, Table tab:algs) ----------------------------
def stepsize_vanishing(tau0, eta, n):
    return lambda k: tau0 / (1.0 + eta * k / n)


def stepsize_constant(tau):
    return lambda k: tau


def stepsize_alg1(k):
    """Piecewise schedule of ALG1 (Table tab:algs)."""
    if k < 10:
        return 3.0
    if k < 100:
        return 2.0
    if k < 200:
        return 1.5
    if k < 300:
        return 1.0
    return 0.5


# --- classical EM ------------------------------------------------------------
def mlem_step(prob, x):
    """x <- x * A^T(y / ybar) / A^T 1 over all data (0/0 keeps x)."""
    num = sum(prob.back(prob.a[i] * prob.y[i] / prob.ybar(x, i), i) for i in range(prob.n))
    sens = prob.sens()
    out = np.array(x, np.float64)
    m = sens > 0
    out[m] = out[m] * num[m] / sens[m]
    return out


def osem_epoch(prob, x, order=None):
    """One OSEM epoch: for each subset in ``order``,
    x <- x * A_i^T(y_i / ybar_i) / A_i^T 1 (0/0 keeps x)."""
    x = np.array(x, np.float64)
    for i in (range(prob.n) if order is None else order):
        num = prob.back(prob.a[i] * prob.y[i] / prob.ybar(x, i), i)
        s = prob.sens_subset(i)
        m = s > 0
        x[m] = x[m] * num[m] / s[m]
    return x


# --- Algorithm 1: preconditioned SVRG -----------------------------------------
def svrg(prob, x0, n_epochs, subset_rule, stepsize, update_pc_iters, omega=2, callback=None, bb_iters=None,
         weight=None, importance_u=None, record=None):
    """Preconditioned SVRG as in Algorithm 1 (Appendix B) with the
    nonnegativity proximal step of eq. (sgm).

    subset_rule(k) -> subset index; stepsize(k) -> tau; update_pc_iters: set of
    iterations k at which D is recomputed by eq. (preconditioner).

    bb_iters (ALG2/ALG3, Section 2.2): snapshot iterations at which the short
    Barzilai-Borwein step is recomputed from the last two snapshots,
    tau_bb = p.q / q.D q with p the difference of the snapshot images and q the
    difference of their full gradients (D the current preconditioner; the
    paper's p.q / q.q for D = I); it is +inf until first computed and the
    step is min(stepsize(k), tau_bb).
    weight(k): estimator weight w of the sampled subset.  With a weight the
    estimator is w (grad D_i(x) - grad D_i(xhat)) + sum_j grad D_j(xhat)
    + beta grad S(x): the weight applies to the data terms and the prior enters
    exactly, which is eq. (svrg) for w = n and unbiased for w = 1 / p_i.
    importance_u (importance sampling, Section 2.4): one uniform number in
    [0, 1) per iteration; at each snapshot p_i = ||grad J_i|| / sum_j ||grad J_j||,
    and iteration k samples i = min{i : p_0 + ... + p_i > u_k} (with
    replacement) with weight 1 / p_i.  subset_rule and weight are then not
    used.  record (a list) receives ("snapshot", k, norms),
    ("sample", k, i, weight) and ("bb", k, p.q, q.D q, tau_bb) entries.
    """
    n = prob.n
    x = np.array(x0, np.float64)
    D = None
    ghat_i = [None] * n
    ghat = None
    tau_bb = np.inf
    x_prev = g_prev = None
    for k in range(n_epochs * n):
        if k in update_pc_iters:
            D = precond_harmonic(x, prob.sens(), prob.prior_hessdiag(x), prob.alpha, prob.delta)
        if k % (omega * n) == 0:
            for i in range(n):
                ghat_i[i] = prob.grad_J(x, i)
            ghat = sum(ghat_i)
            g = ghat
            if weight is not None or importance_u is not None:
                dhat_i = [prob.data_grad(x, i) for i in range(n)]
                dhat = sum(dhat_i)
            if importance_u is not None:
                norms = [float(np.linalg.norm(gi)) for gi in ghat_i]
                probs = importance_probabilities(norms)
                if record is not None:
                    record.append(("snapshot", k, norms))
            if bb_iters is not None:
                if k in bb_iters and x_prev is not None:
                    p = x - x_prev
                    q = ghat - g_prev
                    pq, qdq = float(np.sum(p * q)), float(np.sum(q * D * q))
                    if pq > 0 and qdq > 0:
                        tau_bb = pq / qdq
                    if record is not None:
                        record.append(("bb", k, pq, qdq, tau_bb))
                x_prev, g_prev = x.copy(), ghat.copy()
        else:
            if importance_u is not None:
                i = sample_inverse_cdf(probs, importance_u[k])
                w = 1.0 / probs[i]
                if record is not None:
                    record.append(("sample", k, i, w))
            else:
                i = subset_rule(k)
                w = None if weight is None else weight(k)
            if w is None:
                g = n * (prob.grad_J(x, i) - ghat_i[i]) + ghat
            else:
                g = w * (prob.data_grad(x, i) - dhat_i[i]) + dhat + prob.prior_grad(x)
        tau = stepsize(k) if bb_iters is None else min(stepsize(k), tau_bb)
        x = np.maximum(0.0, x - tau * D * g)
        if callback is not None and (k + 1) % n == 0:
            callback((k + 1) // n, x)
    return x


def importance_probabilities(norms):
    """p_i = ||grad J_i|| / sum_j ||grad J_j|| (Section 2.4)."""
    total = float(sum(norms))
    return [float(v) / total for v in norms]


def sample_inverse_cdf(probs, u):
    """Smallest i with p_0 + ... + p_i > u (the last index if rounding leaves
    the total below u)."""
    c = 0.0
    for i, p in enumerate(probs):
        c += p
        if c > u:
            return i
    return len(probs) - 1


def saga(prob, x0, n_epochs, subset_rule, stepsize, update_pc_iters, callback=None):
    """Preconditioned proximal SAGA, eq. (saga), table initialised at x0."""
    n = prob.n
    x = np.array(x0, np.float64)
    D = None
    table = [prob.grad_J(x, i) for i in range(n)]
    tsum = sum(table)
    for k in range(n_epochs * n):
        if k in update_pc_iters:
            D = precond_harmonic(x, prob.sens(), prob.prior_hessdiag(x), prob.alpha, prob.delta)
        i = subset_rule(k)
        gi = prob.grad_J(x, i)
        g = n * (gi - table[i]) + tsum
        tsum = tsum + gi - table[i]
        table[i] = gi
        x = np.maximum(0.0, x - stepsize(k) * D * g)
        if callback is not None and (k + 1) % n == 0:
            callback((k + 1) // n, x)
    return x


def sgd(prob, x0, n_epochs, subset_rule, stepsize, update_pc_iters, callback=None):
    """Preconditioned proximal SGD with estimator n grad J_i(x)."""
    n = prob.n
    x = np.array(x0, np.float64)
    D = None
    for k in range(n_epochs * n):
        if k in update_pc_iters:
            D = precond_harmonic(x, prob.sens(), prob.prior_hessdiag(x), prob.alpha, prob.delta)
        g = n * prob.grad_J(x, subset_rule(k))
        x = np.maximum(0.0, x - stepsize(k) * D * g)
        if callback is not None and (k + 1) % n == 0:
            callback((k + 1) // n, x)
    return x


def order_rule(orders):
    """Subset rule from per-epoch permutations: iteration k uses orders[k // n][k % n]."""
    orders = np.asarray(orders)
    n = orders.shape[1]
    return lambda k: int(orders[k // n][k % n])


def pc_update_iters(n, epochs=(1, 2, 3)):
    """Iterations at the start of the given (1-indexed) epochs."""
    return {(e - 1) * n for e in epochs}


def nrmse(x, x_ref, mask, c):
    """sqrt(mean over mask of (x - x_ref)^2) / c (Section 3.1)."""
    d = (np.asarray(x, np.float64) - np.asarray(x_ref, np.float64))[mask]
    return float(np.sqrt(np.mean(d * d)) / c)
