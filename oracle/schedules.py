"""ORACLE — test infrastructure only.  Subset counts, subset orders and the
stepsize caps of the submitted algorithms (Section 2.4, Section 4 and its
table of hyperparameters), written plainly for checking the library's own
schedule code.

Readings where the paper gives only a description:
* Herman-Meyer order: the prime factors of n in ascending order; position k,
  written in the mixed radix of those factors (first factor least
  significant), maps to the subset whose digits are the same read in reverse
  significance.
* cofactor order: generators are the 1 <= g < n coprime with n, ranked by
  min(|g - 0.3 n|, |g - 0.7 n|), ties to the smaller g; epoch e walks
  0, g_e, 2 g_e, ... (mod n) with g_e the (e mod #generators)-th generator.
* number of subsets: the divisor of the view count closest to the target,
  ties to the smaller divisor.
"""

import math


def prime_factors(n):
    """Prime factors of n in ascending order, with multiplicity."""
    out = []
    m = n
    p = 2
    while p * p <= m:
        while m % p == 0:
            out.append(p)
            m //= p
        p += 1
    if m > 1:
        out.append(m)
    return out


def herman_meyer(n):
    """Herman-Meyer permutation of range(n)."""
    factors = prime_factors(n)
    order = []
    for k in range(n):
        # digits of k, least significant first, in the mixed radix `factors`
        digits = []
        rest = k
        for p in factors:
            digits.append(rest % p)
            rest //= p
        # the first digit becomes the most significant one
        value = 0
        weight = n
        for p, d in zip(factors, digits):
            weight //= p
            value += d * weight
        order.append(value)
    return order


def cofactor_generators(n):
    """Generators of the cyclic group Z_n, ranked as the cofactor rule does."""
    gens = [g for g in range(1, n) if math.gcd(g, n) == 1]
    if n == 1:
        gens = [1]
    return sorted(gens, key=lambda g: (min(abs(g - 0.3 * n), abs(g - 0.7 * n)), g))


def cofactor_orders(n, n_epochs):
    """One traversal of Z_n per epoch, the generators taken in ranked order and
    reused from the start once exhausted."""
    gens = cofactor_generators(n)
    return [[(j * gens[e % len(gens)]) % n for j in range(n)] for e in range(n_epochs)]


def n_subsets_closest(n_views, target):
    """Divisor of n_views closest to target (ties: the smaller divisor)."""
    divisors = [d for d in range(1, n_views + 1) if n_views % d == 0]
    best = divisors[0]
    for d in divisors[1:]:
        if abs(d - target) < abs(best - target):
            best = d
    return best


def alg2_cap(k, n):
    """Upper bound on the stepsize of ALG2 and ALG3 at iteration k."""
    if k < 10:
        return 3.0
    if k < 2 * n:
        return 2.2
    return 1.0
