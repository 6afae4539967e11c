"""Error bars for GPU-vs-oracle log-likelihood checks on few rows, derived from the arithmetic.

A row's log-weights are 2 C_ji / sigma^2 + log rho_i with C_ji = Re <v_j, R_i a>.  Two roundings
move C_ji: the storage format of the observations (unit roundoff u per entry: each product
v_jd t_d is off by a relative u / sqrt(3) in RMS, independently) and the FP32 accumulation over
the contraction (about one rounding of the running sum per matrix-core k-step, n_k = 2D / 4 of
them: RMS u32 |C| sqrt(n_k / 3)).  A row's log-sum-exp moves by at most the largest change of its
log-weights, and the rows' errors are independent, so six standard deviations of their sum bound
the log-likelihood's error (tests take the larger of this and their relative bar, which is the
tighter one for many rows).  Test infrastructure: uses only the oracle's definitions."""
from __future__ import annotations

import numpy as np

import oracle

U32 = 2.0 ** -24


def loglik_bar(V, a, s2, kbar, L, offs, u_store: float) -> float:
    """Six standard deviations of the summed row errors of the log-likelihood."""
    r = oracle.distances(V, a, kbar, L, offs)
    vn = np.sum(np.abs(V) ** 2, axis=1)
    an = float(np.sum(np.abs(a) ** 2))
    cmax = np.max(np.abs(0.5 * (vn[:, None] + an - r)), axis=1)
    n_k = 2 * V.shape[1] / 4
    acc = 2.0 / s2 * U32 * np.sqrt(n_k / 3.0) * cmax
    store = 2.0 / s2 * u_store / np.sqrt(3.0) * np.sqrt(np.sum(np.abs(a) ** 2 * np.abs(V) ** 2, axis=1))
    return 6.0 * float(np.sqrt(np.sum(acc ** 2 + store ** 2)))
