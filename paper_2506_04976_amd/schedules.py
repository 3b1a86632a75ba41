"""Host-side schedules of the submitted algorithms (Section 2.2, Section 2.4,
Section 4 and its table of hyperparameters): number of subsets, subset orders,
stepsizes or stepsize caps, preconditioner-update and short-BB iterations.
They produce the per-epoch host arrays that pet_svrg_epoch / _ex take.

Conventions: iterations k = 0, 1, ... and epochs e = 0, 1, ... (epoch e + 1 in
the paper's 1-indexed wording); with omega = 2 the snapshots fall on
k = 0, 2n, 4n, ... (the starts of epochs 1, 3, 5, ...).
"""

import math

import numpy as np


def _factorize(n):
    fs, p = [], 2
    while n > 1 and p * p <= n:
        if n % p:
            p += 1
            continue
        fs.append(p)
        n //= p
    if n > 1:
        fs.append(n)
    return fs


def herman_meyer_order(n):
    """Herman-Meyer permutation over the prime factors of n (ascending): the
    order for n = f * m visits the residues of position k modulo f first,
    subset(k) = (k mod f) * m + order_m[k div f], with order_m the order for
    the remaining factors (built from the last factor back to the first)."""
    order = np.zeros(1, dtype=np.int64)
    for f in reversed(_factorize(n)):
        m = order.size
        k = np.arange(f * m)
        order = (k % f) * m + order[k // f]
    return [int(v) for v in order]


def cofactor_order(n, n_epochs):
    """Cofactor rule: units of Z_n ranked by distance to 0.3 n / 0.7 n (ties to
    the smaller one); epoch e walks the cyclic group with the next unit."""
    units = np.array([g for g in range(1, max(n, 2)) if math.gcd(g, n) == 1] or [1])
    key = np.minimum(np.abs(units - 0.3 * n), np.abs(units - 0.7 * n))
    ranked = units[np.lexsort((units, key))]
    steps = np.arange(n)
    return [((steps * int(ranked[e % ranked.size])) % n).astype(np.int32).tolist() for e in range(n_epochs)]


def uniform_orders(n, n_epochs, rng):
    """Uniform sampling without replacement: one permutation per epoch."""
    return [rng.permutation(n).astype(np.int32).tolist() for _ in range(n_epochs)]


def subsets_for(n_views, target=25.0):
    """Divisor of n_views nearest to target; ties go to the smaller divisor."""
    divs = np.array([d for d in range(1, n_views + 1) if n_views % d == 0], dtype=np.float64)
    return int(divs[np.argmin(np.abs(divs - target))])


def alg1_tau(k):
    """ALG1's piecewise stepsize."""
    for bound, tau in ((10, 3.0), (100, 2.0), (200, 1.5), (300, 1.0)):
        if k < bound:
            return tau
    return 0.5


def alg23_cap(k, n):
    """ALG2 / ALG3 bound on the short-BB stepsize."""
    return 3.0 if k < 10 else (2.2 if k < 2 * n else 1.0)


def algorithm_plan(alg, n, n_epochs, rng=None):
    """Per-epoch host arrays for ALG1, ALG2 or ALG3 with n subsets:
    list of dicts {subset_seq, tau, update_pc, bb_update (None for ALG1)}."""
    alg = alg.upper()
    if alg not in ("ALG1", "ALG2", "ALG3"):
        raise ValueError("alg must be ALG1, ALG2 or ALG3")
    if alg == "ALG3":
        orders = cofactor_order(n, n_epochs)
    else:
        orders = uniform_orders(n, n_epochs, rng if rng is not None else np.random.default_rng(0))
    pc_epochs = (1, 2, 3) if alg == "ALG1" else (1, 2, 4, 6)
    pc_iters = {(e - 1) * n for e in pc_epochs}
    bb_iters = set() if alg == "ALG1" else {2 * n, 4 * n, 6 * n}
    plan = []
    for e in range(n_epochs):
        ks = range(e * n, (e + 1) * n)
        plan.append({
            "subset_seq": orders[e],
            "tau": [alg1_tau(k) if alg == "ALG1" else alg23_cap(k, n) for k in ks],
            "update_pc": [k in pc_iters for k in ks],
            "bb_update": None if alg == "ALG1" else [k in bb_iters for k in ks],
        })
    return plan
