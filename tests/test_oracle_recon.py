"""Pins for the oracle's data term, preconditioner and algorithms: KL special
cases, the harmonic-mean identity and bound of the preconditioner (Section 2.3),
MLEM monotonicity, SVRG unbiasedness, the n = 1 reduction of Algorithm 1, SAGA
and SGD to projected gradient descent, the objective's gradient against finite
differences, SAGA's first step, and convergence of SVRG and SAGA to an
independently computed MAP (scipy L-BFGS-B on a dense system matrix built from
unit images)."""

import os

import numpy as np
import pytest
from scipy.optimize import minimize

from oracle import poisson, projector, rdp, recon
from synth import configs, data

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_kl_special_cases():
    assert poisson.kl(3.0, 0.0) == 3.0
    assert poisson.kl(2.5, 2.5) == 0.0
    assert poisson.kl(0.0, 0.0) == 0.0
    assert np.isinf(poisson.kl(0.0, 1.0)) and np.isinf(poisson.kl(1.0, -1.0)) and np.isinf(poisson.kl(-1.0, 0.0))
    s = np.linspace(0.1, 5, 50)
    assert np.all(poisson.kl(s, 1.3) >= -1e-15)
    # d(s, t) for t > 0 is minimised at s = t
    assert np.argmin(poisson.kl(s, 1.3)) == np.argmin(np.abs(s - 1.3))
    # derivative in s by central differences
    h = 1e-6
    for t in (0.0, 0.7, 4.0):
        fd = (poisson.kl(2.0 + h, t) - poisson.kl(2.0 - h, t)) / (2 * h)
        assert poisson.kl_grad_s(2.0, t) == pytest.approx(float(fd), rel=1e-8)


def test_beta_scaling_golden():
    # beta = beta_tilde * 2e-4 * counts / 3e7 (Section 3.1)
    rows = np.loadtxt(os.path.join(GOLDEN, "beta_scaling.txt"))
    for bt, counts, beta in rows:
        cfg = dict(beta_tilde=bt, counts=counts)
        assert configs.beta_value(cfg) == pytest.approx(beta, rel=1e-12)


def test_alg1_stepsize_golden():
    rows = np.loadtxt(os.path.join(GOLDEN, "alg1_stepsize.txt"))
    for k, tau in rows:
        assert recon.stepsize_alg1(int(k)) == tau


def test_preconditioner_harmonic_identity_and_bound():
    rng = np.random.default_rng(0)
    x = rng.uniform(0, 5, 1000)
    x[:10] = 0
    sens = rng.uniform(0.1, 10, 1000)
    H = rng.uniform(1e-3, 50, 1000)
    alpha, delta = 1.7, 1e-3
    D = recon.precond_harmonic(x, sens, H, alpha, delta)
    Dm = recon.precond_mlem(x, sens, delta)
    Dp = recon.precond_prior(H)
    # D = 1/2 h(D_MLEM, alpha^-1 D_betaS) with h(a, b) = 2 / (1/a + 1/b)
    a, b = Dm, Dp / alpha
    half_h = 0.5 * 2.0 / (1.0 / a + 1.0 / b)
    assert np.allclose(D, half_h, rtol=1e-14)
    assert np.all(D <= np.minimum(Dm, Dp / alpha) * (1 + 1e-15))


def _tiny_problem(seed=0, beta=0.5, n_subsets=3):
    # 8x8 image, 12 views x 15 radial bins: overdetermined, so the MAP is well
    # conditioned; some MAP voxels sit on the nonnegativity bound.
    cfg = configs.get("mini_2d", nx=8, ny=8, n_views=12, n_rad=15, rad_spacing=4.0,
                      n_subsets=n_subsets, seed=seed, phantom="c0_small", counts_total=5e4)
    d = data.make_dataset(cfg)
    x0 = np.ones((1, 8, 8))
    prob = recon.Problem(cfg, d["y"].astype(np.float64), d["r"], d["mult"], beta=beta,
                         gamma=2.0, eps=1e-2, alpha=1.0, delta=1e-3)
    return cfg, d, prob, x0


def _dense(prob):
    """Dense A (all subsets stacked, a folded in) from unit images."""
    nv = int(np.prod(prob.shape))
    rows = []
    for i in range(prob.n):
        cols = []
        for j in range(nv):
            e = np.zeros(nv)
            e[j] = 1.0
            cols.append((prob.a[i] * prob.fwd(e.reshape(prob.shape), i)).ravel())
        rows.append(np.stack(cols, 1))
    return np.concatenate(rows, 0)


def test_mlem_monotone_likelihood(oracle_built):
    cfg, d, prob, x = _tiny_problem()
    prev = -np.inf
    for _ in range(200):
        x = recon.mlem_step(prob, x)
        ll = -prob.data_value(x)
        assert ll >= prev - 1e-12 * abs(ll)
        prev = ll


def test_osem_one_subset_is_mlem(oracle_built):
    cfg, d, prob1, x = _tiny_problem(n_subsets=1)
    a = recon.osem_epoch(prob1, x)
    b = recon.mlem_step(prob1, x)
    assert np.array_equal(a, b)


def test_svrg_estimator_unbiased(oracle_built):
    # (1/n) sum_i [n (grad J_i(x) - ghat_i) + ghat] = sum_i grad J_i(x) for any
    # stored table ghat_i with ghat = sum ghat_i.
    cfg, d, prob, x0 = _tiny_problem()
    xs = x0 * 1.3
    ghat_i = [prob.grad_J(xs, i) for i in range(prob.n)]
    ghat = sum(ghat_i)
    x = np.abs(np.random.default_rng(1).normal(1, 0.3, x0.shape))
    est = [prob.n * (prob.grad_J(x, i) - ghat_i[i]) + ghat for i in range(prob.n)]
    full = prob.full_grad(x)
    assert np.allclose(sum(est) / prob.n, full, rtol=1e-12, atol=1e-12 * np.abs(full).max())


def test_svrg_single_subset_is_projected_gradient(oracle_built):
    cfg, d, prob, x0 = _tiny_problem(n_subsets=1)
    tau = recon.stepsize_constant(0.5)
    x_svrg = recon.svrg(prob, x0, 6, lambda k: 0, tau, {0})
    x = np.array(x0, np.float64)
    D = recon.precond_harmonic(x, prob.sens(), prob.prior_hessdiag(x), 1.0, 1e-3)
    for _ in range(6):
        x = np.maximum(0, x - 0.5 * D * prob.full_grad(x))
    assert np.allclose(x_svrg, x, rtol=1e-12, atol=1e-14)


def xmap_has_bound_voxels(x):
    return np.any(x == 0.0)


def _dense_map(prob):
    """MAP by scipy L-BFGS-B on the dense system (bounds x >= 0), and the
    dense objective evaluated there."""
    A = _dense(prob)
    y = np.concatenate([yi.ravel() for yi in prob.y])
    r = np.concatenate([ri.ravel() for ri in prob.r])
    w = prob.w

    def f(z):
        yb = A @ z + r
        val = np.sum(yb - y) + np.sum(y[y > 0] * np.log(y[y > 0] / yb[y > 0]))
        zz = z.reshape(prob.shape)
        val += prob.beta * rdp.value(zz, w, prob.gamma, prob.eps)
        g = A.T @ (1 - y / yb) + prob.beta * rdp.grad(zz, w, prob.gamma, prob.eps).ravel()
        return val, g

    res = minimize(f, np.ones(A.shape[1]), jac=True, method="L-BFGS-B", bounds=[(0, None)] * A.shape[1],
                   options=dict(maxiter=50000, maxfun=100000, ftol=1e-16, gtol=1e-14))
    return res.x.reshape(prob.shape), f(res.x)[0]


def test_svrg_converges_to_dense_map(oracle_built):
    cfg, d, prob, x0 = _tiny_problem()
    xmap, fmap = _dense_map(prob)
    assert xmap_has_bound_voxels(xmap)
    x_init = recon.osem_epoch(prob, x0)
    orders = data.subset_orders(cfg, 300)
    x = recon.svrg(prob, x_init, 300, recon.order_rule(orders), recon.stepsize_vanishing(1.0, 0.02, prob.n),
                   recon.pc_update_iters(prob.n))
    assert np.linalg.norm(x - xmap) / np.linalg.norm(xmap) < 1e-4
    # the MAP is a fixed point of the iteration (up to the L-BFGS-B accuracy)
    x_fp = recon.svrg(prob, xmap, 4, recon.order_rule(orders), recon.stepsize_constant(1.0),
                      recon.pc_update_iters(prob.n))
    assert np.linalg.norm(x_fp - xmap) / np.linalg.norm(xmap) < 1e-5
    # objective agrees with the dense evaluation
    assert prob.objective(xmap) == pytest.approx(fmap, rel=1e-12)


def test_full_gradient_matches_objective_differences(oracle_built):
    # the sum of the subset gradients grad J_i = grad D_i + (beta/n) grad S
    # (eq. (template)) is the gradient of the objective, checked against
    # central differences of the separately coded objective value
    cfg, d, prob, x0 = _tiny_problem()
    rng = np.random.default_rng(3)
    x = rng.uniform(0.5, 2.0, x0.shape)
    g = sum(prob.grad_J(x, i) for i in range(prob.n))
    for _ in range(3):
        v = rng.standard_normal(x.shape)
        h = 1e-6
        fd = (prob.objective(x + h * v) - prob.objective(x - h * v)) / (2 * h)
        assert float(np.sum(g * v)) == pytest.approx(fd, rel=1e-6)


@pytest.mark.parametrize("algo", ["saga", "sgd"])
def test_single_subset_is_projected_gradient(oracle_built, algo):
    # with one subset every estimator is the full gradient
    cfg, d, prob, x0 = _tiny_problem(n_subsets=1)
    x_alg = getattr(recon, algo)(prob, x0, 6, lambda k: 0, recon.stepsize_constant(0.5), {0})
    x = np.array(x0, np.float64)
    D = recon.precond_harmonic(x, prob.sens(), prob.prior_hessdiag(x), 1.0, 1e-3)
    for _ in range(6):
        x = np.maximum(0, x - 0.5 * D * prob.full_grad(x))
    assert np.allclose(x_alg, x, rtol=1e-12, atol=1e-14)


def test_saga_first_step_is_svrg_first_step(oracle_built):
    # SAGA's table starts at x0, so its first estimator is the full gradient,
    # as at SVRG's first (snapshot) iteration; later steps differ
    cfg, d, prob, x0 = _tiny_problem()
    x0 = recon.osem_epoch(prob, x0)
    orders = data.subset_orders(cfg, 2)
    rule = recon.order_rule(orders)
    only_first = lambda k: 0.7 if k == 0 else 0.0  # noqa: E731
    a = recon.saga(prob, x0, 1, rule, only_first, {0})
    b = recon.svrg(prob, x0, 1, rule, only_first, {0})
    assert np.array_equal(a, b)
    a2 = recon.saga(prob, x0, 2, rule, recon.stepsize_constant(0.7), {0})
    b2 = recon.svrg(prob, x0, 2, rule, recon.stepsize_constant(0.7), {0})
    assert np.linalg.norm(a2 - b2) > 1e-6 * np.linalg.norm(b2)


def test_saga_converges_to_dense_map_with_constant_steps(oracle_built):
    # SAGA converges with a constant stepsize (Section 2.1); SGD with the same
    # constant stepsize stalls at a distance set by its variance
    cfg, d, prob, x0 = _tiny_problem()
    xmap, _ = _dense_map(prob)
    x_init = recon.osem_epoch(prob, x0)
    orders = data.subset_orders(cfg, 400)
    rule = recon.order_rule(orders)
    x = recon.saga(prob, x_init, 400, rule, recon.stepsize_constant(0.5), recon.pc_update_iters(prob.n))
    err_saga = np.linalg.norm(x - xmap) / np.linalg.norm(xmap)
    assert err_saga < 1e-6
    xg = recon.sgd(prob, x_init, 60, rule, recon.stepsize_constant(0.5), recon.pc_update_iters(prob.n))
    assert np.linalg.norm(xg - xmap) / np.linalg.norm(xmap) > 10 * err_saga
    # the MAP is a fixed point of SAGA
    x_fp = recon.saga(prob, xmap, 4, rule, recon.stepsize_constant(1.0), recon.pc_update_iters(prob.n))
    assert np.linalg.norm(x_fp - xmap) / np.linalg.norm(xmap) < 1e-5


@pytest.mark.parametrize("name", ["mini_tof", "mini_nontof"])
def test_zero_count_split_of_data_term(oracle_built, name):
    # d(s, 0) = s (Section 1.2): the subset KL and its gradient split into a part
    # linear in x through the subset sensitivity and a part over bins with y > 0
    # only, D_i = <P_i^T a, x> + sum r - sum y + sum_{y>0} y log(y / ybar) and
    # grad D_i = P_i^T a - P_i^T[a y / ybar] restricted to y > 0 -- the identity
    # the zero-count-aware GPU path computes; here both sides are the oracle's
    # dense sums, so it checks the algebra, not a kernel.
    from oracle import poisson
    cfg = configs.get(name)
    d = data.make_dataset(cfg)
    prob = recon.Problem(cfg, d["y"], d["r"], d["mult"], beta=0.1, gamma=2.0, eps=1e-3)
    x = np.random.default_rng(3).uniform(0.1, 2.0, prob.shape)
    for i in range(cfg["n_subsets"]):
        yb = prob.ybar(x, i)
        y = prob.y[i]
        pos = y > 0
        si = prob.sens_subset(i)
        split = (si * x).sum() + prob.r[i].sum() - y.sum() + np.sum(y[pos] * np.log(y[pos] / yb[pos]))
        assert split == pytest.approx(poisson.kl(yb, y).sum(), rel=1e-12)
        q = np.where(pos, prob.a[i] * y / np.where(pos, yb, 1.0), 0.0)
        g_split = si - prob.back(q, i)
        g = prob.data_grad(x, i)
        assert np.linalg.norm(g_split - g) <= 1e-12 * np.linalg.norm(si)
