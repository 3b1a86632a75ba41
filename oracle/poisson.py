"""ORACLE — test infrastructure only.  Poisson (KL) data fidelity in FP64.

d(s, t) (Section 1.2):  s - t + t log(t/s) if t > 0, s > 0;  s if t = 0, s >= 0;
infinity otherwise.  With the separable form D(Ax + r, y) = sum_i sum_{j in S_i}
d(A_j x + r_j, y_j) (eq. (separable_datafit)), the subset term
D_i(x) = sum_{j in S_i} d(A_j x + r_j, y_j) has gradient
A_i^T (1 - y / (A_i x + r)), since d/ds d(s, t) = 1 - t/s (also for t = 0).
Here A = diag(a) P, so A_i^T q = P_i^T (a q).
"""

import numpy as np


def kl(s, t):
    s = np.asarray(s, np.float64)
    t = np.asarray(t, np.float64)
    out = np.full(np.broadcast(s, t).shape, np.inf)
    pos = (t > 0) & (s > 0)
    zero = (t == 0) & (s >= 0)
    ss, tt = np.broadcast_arrays(s, t)
    out[pos] = ss[pos] - tt[pos] + tt[pos] * np.log(tt[pos] / ss[pos])
    out[zero] = ss[zero]
    return out


def kl_grad_s(s, t):
    """Derivative of d(s, t) in s: 1 - t/s."""
    return 1.0 - np.asarray(t, np.float64) / np.asarray(s, np.float64)
