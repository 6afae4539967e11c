"""FP64 Synchronize and Match (oracle; test infrastructure only).

The step before the EM path (§II-A, §III-A, Algorithm "Synchronize and Match"): relative rotations
between all pairs of a small subset S_P of the observations, angular synchronization of S_P by the
projected power method, then every observation takes the rotation of its nearest neighbour in S_P
(the members of S_P their nearest neighbour other than themselves), and the observations are
aligned by that rotation.

Conventions (the paper's own signs do not close up; this is the reading used on both sides):
``rel[i, j]`` is the grid rotation l that best maps observation j onto observation i,
``argmax_l Re <v_i, R_l v_j>`` = ``argmin_l || v_i - R_l v_j ||^2`` with ``R_l v = v o
exp(-i kbar 2 pi l / L)``, which estimates theta_i - theta_j; ``H_ij = exp(+i 2 pi rel_ij / L)``;
the power method starts from z = 1 and iterates ``z <- phase(H z)``; ``theta_hat_i = arg z_i``;
the aligned observation is ``v_i o exp(+i kbar theta_hat_i)``, the paper's alignment.  Ties in an
argmax or argmin go to the lowest index.
"""
from __future__ import annotations

import math

import numpy as np

from .em import grid_phase

__all__ = ["relative_rotations", "relative_rotations_brute", "ppm", "nearest_neighbours",
           "synchronize_and_match", "align", "aligned_mean", "global_rotation",
           "centred_error_bins"]


def relative_rotations(Vp: np.ndarray, kbar: np.ndarray, L: int):
    """rel[i, j] = argmax_l Re <v_i, R_l v_j> over the L grid rotations (§II-A, the pairwise
    estimate), through the per-frequency sums c_ijk = sum_q conj(v_ikq) v_jkq, so that
    Re <v_i, R_l v_j> = Re sum_k c_ijk exp(-i k 2 pi l / L).  Returns (rel, f) with f[i, j, l]
    the correlations (P x P x L)."""
    P, D = Vp.shape
    K = int(np.max(kbar)) + 1
    kb = np.asarray(kbar, dtype=np.int64)
    c = np.zeros((P, P, K), dtype=np.complex128)
    for k in range(K):
        Vk = Vp[:, kb == k]                                   # P x Q_k
        c[:, :, k] = np.conj(Vk) @ Vk.T
    ph = grid_phase(np.arange(K), np.arange(L), L, -1)        # L x K: exp(-i k 2 pi l / L)
    f = np.real(c @ ph.T)                                     # P x P x L
    return np.argmax(f, axis=2), f


def relative_rotations_brute(Vp: np.ndarray, kbar: np.ndarray, L: int) -> np.ndarray:
    """The same estimate by rotating v_j explicitly and minimising the distance (tiny inputs)."""
    P = Vp.shape[0]
    rel = np.zeros((P, P), dtype=np.int64)
    for i in range(P):
        for j in range(P):
            best, arg = math.inf, 0
            for l in range(L):
                rot = Vp[j] * np.array([complex(math.cos(2 * math.pi * ((int(k) * l) % L) / L),
                                                -math.sin(2 * math.pi * ((int(k) * l) % L) / L))
                                        for k in kbar])
                d = float(np.sum(np.abs(Vp[i] - rot) ** 2))
                if d < best:
                    best, arg = d, l
            rel[i, j] = arg
    return rel


def ppm(rel: np.ndarray, L: int, iters: int) -> np.ndarray:
    """Projected power method (§II-A): z <- phase(H z) with H_ij = exp(i 2 pi rel_ij / L), from
    z = 1, ``iters`` times; returns theta_hat = arg z in [-pi, pi].  A zero entry of H z keeps
    the previous z_i."""
    m = np.mod(np.asarray(rel, dtype=np.int64), L)
    H = np.exp(2j * np.pi * m / L)
    z = np.ones(H.shape[0], dtype=np.complex128)
    for _ in range(iters):
        y = H @ z
        a = np.abs(y)
        z = np.where(a > 0, y / np.where(a > 0, a, 1.0), z)
    return np.angle(z)


def nearest_neighbours(V: np.ndarray, P: int):
    """For every observation i, the index n in S_P = {0 .. P-1} minimising || v_i - v_n ||^2 (no
    rotation), excluding n = i for the members of S_P (Algorithm "Synchronize and Match").
    Returns (nn, d) with d the N x P squared distances."""
    Vp = V[:P]
    d = (np.sum(np.abs(V) ** 2, axis=1)[:, None] + np.sum(np.abs(Vp) ** 2, axis=1)[None, :]
         - 2.0 * np.real(np.conj(V) @ Vp.T))
    dm = d.copy()
    idx = np.arange(min(P, V.shape[0]))
    dm[idx, idx] = np.inf
    return np.argmin(dm, axis=1), d


def synchronize_and_match(V: np.ndarray, kbar: np.ndarray, L: int, P: int, iters: int):
    """Algorithm "Synchronize and Match": returns (theta_hat (N), phi (P), rel, nn)."""
    rel, _ = relative_rotations(V[:P], kbar, L)
    phi = ppm(rel, L, iters)
    nn, _ = nearest_neighbours(V, P)
    return phi[nn], phi, rel, nn


def align(V: np.ndarray, kbar: np.ndarray, theta: np.ndarray) -> np.ndarray:
    """Aligned observations v_i o exp(+i kbar theta_i) (the steerable alignment of §II-A)."""
    return V * np.exp(1j * np.multiply.outer(np.asarray(theta, np.float64),
                                             np.asarray(kbar, np.float64)))


# ---- learning the distribution of the synchronizer's errors (§III-B, Algorithm "learning
# rotation distribution"; the histogram itself is em.histogram_prior)

def aligned_mean(V: np.ndarray, kbar: np.ndarray, theta: np.ndarray) -> np.ndarray:
    """(1/N) sum_i v_i o exp(+i kbar theta_i): the average of the aligned coefficients (§II-A),
    which also starts the EM after synchronization (§III-A)."""
    return align(V, kbar, theta).mean(axis=0)


def global_rotation(x: np.ndarray, abar: np.ndarray, kbar: np.ndarray, L: int) -> int:
    """The grid rotation theta_c = 2 pi l_c / L minimising || R_theta abar - x ||^2 (the
    algorithm's centring step), i.e. argmax_l Re <x, R_l abar>; returns l_c."""
    best, arg = -math.inf, 0
    for l in range(L):
        v = float(np.real(np.vdot(x, abar * grid_phase(kbar, l, L, -1))))
        if v > best:
            best, arg = v, l
    return arg


def centred_error_bins(theta_hat: np.ndarray, theta_true: np.ndarray, lc: int, L: int):
    """floor((theta_hat - theta - theta_c) L / (2 pi)) mod L: the centred errors of the
    algorithm, binned as in its histogram step (integer bins, then eq. (22) is the identity)."""
    e = np.asarray(theta_hat, np.float64) - np.asarray(theta_true, np.float64) - 2 * np.pi * lc / L
    return np.mod(np.floor(e * L / (2 * np.pi)).astype(np.int64), L)
