"""FP64 EM for 2-D MRA in steerable coefficients (oracle; test infrastructure only).

Notation (§I eq. (4), §II-B): observations ``V`` (N x D complex), coefficients ``a`` (D complex),
angular index per entry ``kbar`` (D ints), rotation grid ``theta_l = 2 pi l / L``.  A windowed
search (§III-C) visits the offsets ``o_i = lo + i`` (i = 0..W-1); plain EM is ``lo = 0, W = L``.
``rho`` has one entry per visited offset.  Rotating ``a`` by ``theta`` multiplies entry d by
``exp(-i kbar[d] theta)`` (§I eq. (3)).

Wherever a function takes ``offs`` it also accepts an ``AngleList``: the refined-resolution
window of §III-C, which samples the likely range of rotations more densely than the grid, so the
visited rotations are arbitrary angles ``theta_i`` (radians) instead of ``2 pi o_i / L``.  The
E-step, the M-step and rho are then the same formulas with ``exp(-/+ i kbar theta_i)``; ``L``
still sets the grid of the stopping metric and of the error against the truth.
"""
from __future__ import annotations

import math
from typing import Optional

import numpy as np

__all__ = [
    "AngleList", "offsets", "grid_phase", "rotate", "distances_brute", "distances", "log_weights", "normalize",
    "estep", "loglik", "mstep_a", "mstep_rho", "objective", "stop_metric", "em_iteration",
    "em_run", "relative_error", "relative_error_continuous",
    "grad_loglik", "histogram_prior", "argmax_margin",
    "q_function", "validate",
]


class OracleInvalid(ValueError):
    """Raised for inputs the method is not defined on (mirrors the library's EM_EINVAL)."""


class OracleNonFinite(ValueError):
    """Raised for NaN/Inf observations (mirrors the library's EM_ENONFINITE)."""


class AngleList:
    """Visited rotations given as angles in radians (the refined-resolution window, §III-C)."""

    def __init__(self, theta):
        self.theta = np.asarray(theta, dtype=np.float64).ravel()

    def __len__(self) -> int:
        return len(self.theta)


def offsets(lo: int, W: int) -> np.ndarray:
    """Window offsets lo..lo+W-1 (§III-C: angles -pi BW/L .. pi BW/L in steps of 2 pi/L)."""
    return np.arange(lo, lo + W, dtype=np.int64)


def grid_phase(kbar: np.ndarray, l, L: int, sign: int) -> np.ndarray:
    """exp(sign * i * kbar * 2 pi l / L), evaluated at the exact grid angle 2 pi ((k l) mod L)/L.

    ``l`` may be a scalar or a vector of offsets, or an ``AngleList`` (then the phase is
    exp(sign * i * kbar * theta_i) at the given angles); the result has shape (..., D).
    """
    if isinstance(l, AngleList):
        return np.exp(sign * 1j * np.multiply.outer(l.theta, np.asarray(kbar, dtype=np.float64)))
    l = np.asarray(l, dtype=np.int64)
    m = np.mod(np.multiply.outer(l, np.asarray(kbar, dtype=np.int64)), L)
    return np.exp(sign * 2j * np.pi * m / L)


def rotate(a: np.ndarray, kbar: np.ndarray, l: int, L: int) -> np.ndarray:
    """R_{theta_l} a = a o exp(-i kbar theta_l)  (§I eq. (3) and eq. (4))."""
    return a * grid_phase(kbar, l, L, -1)


def _rotated(a, kbar, offs, i: int, L: int) -> np.ndarray:
    """R_{theta_i} a for the i-th visited rotation: the grid rotation for integer offsets; for an
    ``AngleList``, entry by entry a_d (cos(k theta_i) - i sin(k theta_i)) with scalar math."""
    if isinstance(offs, AngleList):
        th = float(offs.theta[i])
        return np.array([a[d] * complex(math.cos(int(kbar[d]) * th), -math.sin(int(kbar[d]) * th))
                         for d in range(len(a))])
    return rotate(a, kbar, int(offs[i]), L)


def distances_brute(V, a, kbar, L, offs) -> np.ndarray:
    """r[j, i] = || R_{o_i} a - v_j ||^2 with the rotation applied explicitly (§II-B eq. (15)).

    Double loop; only for tiny inputs.
    """
    N, W = V.shape[0], len(offs)
    r = np.empty((N, W))
    for i in range(W):
        t = _rotated(a, kbar, offs, i, L)
        for j in range(N):
            diff = t - V[j]
            r[j, i] = float(np.sum(diff.real ** 2 + diff.imag ** 2))
    return r


def distances(V, a, kbar, L, offs) -> np.ndarray:
    """Same as ``distances_brute`` via ||v||^2 + ||a||^2 - 2 Re<v_j, R_{o_i} a> and one matmul."""
    T = a[:, None] * grid_phase(kbar, offs, L, -1).T            # D x W, column i = R_{o_i} a
    # Re(conj(v_j) . t_i) = Re v . Re t + Im v . Im t; the parts are copied into plain arrays
    # so that numpy hands both products to BLAS (strided views take a slow loop)
    Vr, Vi = np.ascontiguousarray(V.real), np.ascontiguousarray(V.imag)
    Tr, Ti = np.ascontiguousarray(T.real), np.ascontiguousarray(T.imag)
    C = Vr @ Tr + Vi @ Ti
    vn = np.sum(V.real ** 2 + V.imag ** 2, axis=1)
    an = float(np.sum(a.real ** 2 + a.imag ** 2))
    return vn[:, None] + an - 2.0 * C


def log_weights(r: np.ndarray, rho: np.ndarray, sigma2: float, D: int) -> np.ndarray:
    """log of rho[i] * p(v_j | theta = o_i, a) for the complex Gaussian likelihood (§II-B eq. (13)):
    -r/sigma^2 + log rho - D log(pi sigma^2).  A zero entry of rho gives -inf."""
    with np.errstate(divide="ignore"):
        lr = np.log(np.asarray(rho, dtype=np.float64))
    return -r / sigma2 + lr[None, :] - D * math.log(math.pi * sigma2)


def normalize(ell: np.ndarray):
    """Normalise each row of weights (Algorithm "Synch-EM", normalisation step; §II-B eq. (15)).

    Returns (w, lse) with lse_j = log sum_i exp(ell_ji) and w_ji = exp(ell_ji - lse_j).
    """
    m = np.max(ell, axis=1, keepdims=True)
    s = np.sum(np.exp(ell - m), axis=1, keepdims=True)
    lse = m + np.log(s)
    w = np.exp(ell - lse)
    return w, lse[:, 0]


def estep(V, a, rho, sigma2, kbar, L, offs, brute: bool = False):
    """E-step posteriors w[j, i] = P(theta_j = o_i | v_j, a, rho) (§II-B eq. (15)) and the
    per-row marginal log-likelihood lse_j = log p(v_j | a, rho)."""
    r = (distances_brute if brute else distances)(V, a, kbar, L, offs)
    ell = log_weights(r, rho, sigma2, V.shape[1])
    w, lse = normalize(ell)
    return w, lse, r


def loglik(V, a, rho, sigma2, kbar, L, offs) -> float:
    """Marginal log-likelihood sum_j log sum_i rho_i p(v_j | o_i, a) (§II-B eq. (13), rotations
    marginalised over the visited grid)."""
    return float(np.sum(estep(V, a, rho, sigma2, kbar, L, offs)[1]))


def mstep_a(V, w, kbar, L, offs, sigma2, gamma_a_inv: Optional[np.ndarray] = None):
    """Coefficient update (§II-B eq. (17); App. C):
    a = (N I + sigma^2 Gamma_a^{-1})^{-1} sum_j sum_i w_ji exp(+i kbar theta_i) o v_j.

    ``gamma_a_inv`` is the diagonal of Gamma_a^{-1} (None: no image prior).  Returns (a, S) with S
    the double sum.  The sum over j is taken first for each rotation (a matmul), then over i.
    """
    N = V.shape[0]
    Y = w.T @ V                                                  # Y[i] = sum_j w_ji v_j
    back = grid_phase(kbar, offs, L, +1)                         # W x D, exp(+i kbar theta_i)
    S = np.sum(back * Y, axis=0)
    denom = N + (0.0 if gamma_a_inv is None else sigma2 * np.asarray(gamma_a_inv, np.float64))
    return S / denom, S


def mstep_rho(Wt: np.ndarray, rho_bar: Optional[np.ndarray], gamma: float) -> np.ndarray:
    """Rotation-distribution update. gamma = 0: W_t / sum W_t (§II-B eq. (18)); otherwise the
    KL-prior maximiser (W_t + gamma rho_bar) / sum (W_t + gamma rho_bar) (App. C eq. (42);
    Algorithm "Synch-EM", distribution update)."""
    x = np.asarray(Wt, np.float64) + (0.0 if rho_bar is None else gamma * np.asarray(rho_bar))
    return x / np.sum(x)


def objective(ll, rho, rho_bar, gamma, a, gamma_a_inv) -> float:
    """MAP objective up to constants (§II-B: log posterior eq. (12) with the KL prior eq. (23)-(24)
    and the Gaussian image prior): LL + gamma sum rho_bar log rho - sum gamma_a^{-1} |a|^2.
    Terms with rho_bar = 0 contribute 0."""
    J = float(ll)
    if gamma and rho_bar is not None:
        rb = np.asarray(rho_bar, np.float64)
        nz = rb > 0
        with np.errstate(divide="ignore"):
            J += gamma * float(np.sum(rb[nz] * np.log(np.asarray(rho)[nz])))
    if gamma_a_inv is not None:
        J -= float(np.sum(np.asarray(gamma_a_inv) * np.abs(a) ** 2))
    return J


def stop_metric(a_new, a_old, kbar, L) -> float:
    """min over l in [0, L) of || a_new - exp(-2 pi i kbar l / L) o a_old ||^2
    (Algorithm "Synch-EM", stopping rule), by brute force over the L rotations."""
    best = math.inf
    for l in range(L):
        d = a_new - rotate(a_old, kbar, l, L)
        best = min(best, float(np.sum(d.real ** 2 + d.imag ** 2)))
    return best


def q_function(a, rho, w, V, kbar, L, offs, sigma2, rho_bar=None, gamma=0.0,
               gamma_a_inv=None) -> float:
    """Q(a, rho | a_t, rho_t) of §II-B eq. (14), written out term by term (slow; tiny inputs),
    with log p(a) = -a^H Gamma_a^{-1} a and log p(rho) = -gamma KL(rho_bar, rho) up to constants."""
    total = 0.0
    with np.errstate(divide="ignore"):
        for j in range(V.shape[0]):
            for i in range(len(offs)):
                if w[j, i] == 0.0:
                    continue
                d = _rotated(a, kbar, offs, i, L) - V[j]
                total += w[j, i] * (math.log(rho[i]) - float(np.sum(np.abs(d) ** 2)) / sigma2)
    if gamma_a_inv is not None:
        total -= float(np.sum(np.asarray(gamma_a_inv) * np.abs(a) ** 2))
    if gamma and rho_bar is not None:
        for i in range(len(rho)):
            if rho_bar[i] > 0:
                total -= gamma * rho_bar[i] * math.log(rho_bar[i] / rho[i])
    return total


def em_iteration(V, a, rho, sigma2, kbar, L, offs, rho_bar=None, gamma=0.0,
                 gamma_a_inv=None, update_rho=True):
    """One iteration of Algorithm "Synch-EM" (E-step over the window, normalisation, W_t,
    coefficient update, distribution update, stopping metric).

    Returns a dict with the new state (``a``, ``rho``) and the quantities of the state the
    iteration started from: ``ll`` (eq. (13) marginal), ``J`` (MAP objective), posteriors ``w``,
    per-row ``lse``, ``W`` (= W_t), ``S``, and ``stop`` (the stopping metric).
    """
    w, lse, r = estep(V, a, rho, sigma2, kbar, L, offs)
    Wt = w.sum(axis=0)
    a_new, S = mstep_a(V, w, kbar, L, offs, sigma2, gamma_a_inv)
    rho_new = mstep_rho(Wt, rho_bar, gamma) if update_rho else np.asarray(rho, np.float64).copy()
    ll = float(np.sum(lse))
    return {
        "a": a_new, "rho": rho_new, "ll": ll,
        "J": objective(ll, rho, rho_bar, gamma, a, gamma_a_inv),
        "w": w, "lse": lse, "W": Wt, "S": S, "r": r,
        "stop": stop_metric(a_new, a, kbar, L),
    }


def em_run(V, a0, rho0, sigma2, kbar, L, offs, iters, tol=0.0, rho_bar=None, gamma=0.0,
           gamma_a_inv=None, update_rho=True):
    """Algorithm "Synch-EM" from (a0, rho0) for at most ``iters`` iterations; stops after the
    iteration whose stopping metric falls below ``tol`` (tol <= 0: never)."""
    a, rho = np.asarray(a0, np.complex128).copy(), np.asarray(rho0, np.float64).copy()
    hist = []
    for _ in range(iters):
        it = em_iteration(V, a, rho, sigma2, kbar, L, offs, rho_bar, gamma, gamma_a_inv,
                          update_rho)
        hist.append({k: it[k] for k in ("ll", "J", "stop")})
        a, rho = it["a"], it["rho"]
        if tol > 0 and it["stop"] < tol:
            break
    return a, rho, hist


def relative_error(a_hat, a_true, kbar, L) -> float:
    """min over grid rotations of ||R_l a_hat - a_true|| / ||a_true|| (§II-B eq. (19), with the
    minimum over the L grid angles; the steerable basis makes the Frobenius norm of the image equal
    to the coefficient norm for an orthonormal basis)."""
    best = math.inf
    for l in range(L):
        best = min(best, float(np.linalg.norm(rotate(a_hat, kbar, l, L) - a_true)))
    return best / float(np.linalg.norm(a_true))


def relative_error_continuous(a_hat, a_true, kbar, steps: int = 36000) -> float:
    """min over all angles theta of ||a_hat o exp(-i kbar theta) - a_true|| / ||a_true|| (eq. (19)
    over the continuous circle, for estimates whose global rotation is off the grid, as after
    synchronization): the best of `steps` grid angles, then a golden-section refinement within
    one grid step on either side."""
    kb = np.asarray(kbar, np.float64)

    def err(th):
        return float(np.linalg.norm(a_hat * np.exp(-1j * kb * th) - a_true))

    grid = 2 * np.pi * np.arange(steps) / steps
    e = [err(t) for t in grid]
    t0 = grid[int(np.argmin(e))]
    lo, hi = t0 - 2 * np.pi / steps, t0 + 2 * np.pi / steps
    r = (math.sqrt(5) - 1) / 2
    for _ in range(60):
        m1, m2 = hi - r * (hi - lo), lo + r * (hi - lo)
        if err(m1) < err(m2):
            hi = m2
        else:
            lo = m1
    return min(err(0.5 * (lo + hi)), min(e)) / float(np.linalg.norm(a_true))


def grad_loglik(V, a, sigma2, rho, kbar, L, offs):
    """Gradients of LL(a, sigma^2, eta) = sum_j log sum_i rho_i p(v_j | o_i, a, sigma^2) with
    rho = softmax(eta), from the posteriors (Fisher identity applied to eq. (13)):

      dLL/da (as dLL/dRe a + i dLL/dIm a) = (2/sigma^2) (S - N a),  S = sum_ji w_ji e^{+ik theta_i} v_j
      dLL/dsigma^2 = -N D / sigma^2 + sum_ji w_ji r_ji / sigma^4
      dLL/deta     = W - N rho

    Returns (ll, grad_a, grad_sigma2, grad_eta).
    """
    N, D = V.shape
    w, lse, r = estep(V, a, rho, sigma2, kbar, L, offs)
    _, S = mstep_a(V, w, kbar, L, offs, sigma2, None)
    g_a = (2.0 / sigma2) * (S - N * a)
    g_s2 = -N * D / sigma2 + float(np.sum(w * r)) / sigma2 ** 2
    g_eta = w.sum(axis=0) - N * np.asarray(rho, np.float64)
    return float(np.sum(lse)), g_a, g_s2, g_eta


def histogram_prior(errors, L: int, lo: int, W: int):
    """Learned rotation prior (§III-B eq. (22); Algorithm "learning rotation distribution"): the
    empirical distribution of integer rotation errors, each wrapped to [-L/2, L/2) (the floor of
    eq. (22) is the identity on integer errors), restricted to the window offsets lo..lo+W-1 and
    renormalised over it.

    Returns (rho_bar over the window, counts over the window, counts over all L bins indexed by
    e mod L).  Counting is a plain loop over the draws.
    """
    counts_all = np.zeros(L, dtype=np.int64)
    for e in np.asarray(errors, dtype=np.int64):
        counts_all[int(e) % L] += 1
    win = np.array([counts_all[(lo + i) % L] for i in range(W)], dtype=np.int64)
    total = int(win.sum())
    if total == 0:
        raise OracleInvalid("no draw falls inside the window")
    return win / total, win, counts_all


def argmax_margin(w: np.ndarray):
    """Most probable window index per row (lowest index wins ties) and the probability gap
    between the best and the runner-up (with W = 1 there is no runner-up and the gap is w_max)."""
    idx = np.argmax(w, axis=1)                                    # numpy: first maximal index
    if w.shape[1] == 1:
        return idx, w[:, 0].copy()
    top2 = np.sort(w, axis=1)[:, -2:]
    return idx, top2[:, 1] - top2[:, 0]


def validate(N, K, Q, L, lo, W, sigma2, prior=None, V=None):
    """Input checks the method needs (mirrors the library's argument validation)."""
    if N < 1 or K < 1 or Q < 1 or L < 1:
        raise OracleInvalid("sizes must be positive")
    if W < 1 or W > L:
        raise OracleInvalid("window size must be in [1, L]")
    if not (sigma2 > 0 and math.isfinite(sigma2)):
        raise OracleInvalid("sigma^2 must be positive and finite")
    if prior is not None:
        p = np.asarray(prior, np.float64)
        if p.shape != (W,) or np.any(p < 0) or not np.all(np.isfinite(p)) or p.sum() <= 0:
            raise OracleInvalid("prior must be W non-negative finite entries with positive sum")
    if V is not None and not np.all(np.isfinite(V)):
        raise OracleNonFinite("observations contain NaN or Inf")
