"""Polar-pixel brute force for rotations (oracle; test infrastructure only).

§I eq. (2)-(3): an image expanded in a steerable basis u^{k,q}(r, phi) = f^{k,q}(r) e^{i k phi} is
rotated counter-clockwise by theta by evaluating it at phi - theta, which multiplies a_{k,q} by
e^{-i k theta}.  Here the image is sampled on a polar grid (R radii x P angles, P a multiple of the
rotation grid L), so a rotation by 2 pi l / L is an exact circular shift of the angle axis by
l P / L samples.  With orthonormal radial profiles (the columns of an R x Q matrix) and P >= K, the
sampled image's squared norm, scaled by 1/P, equals the squared coefficient norm.  Distances
computed this way never apply the coefficient phase, so they pin the sign convention of the
coefficient-domain code.
"""
from __future__ import annotations

import numpy as np

__all__ = ["PolarGrid", "make_grid", "synthesize", "rotate_pixels", "analyze",
           "distances_pixels"]


class PolarGrid:
    def __init__(self, radial: np.ndarray, P: int, K: int, Q: int):
        self.radial = radial          # R x Q, orthonormal columns: f_q(r_p)
        self.P = P                    # angular samples phi_m = 2 pi m / P
        self.K, self.Q = K, Q


def make_grid(K: int, Q: int, L: int, R: int = None, seed: int = 0) -> PolarGrid:
    """Polar grid with a random orthonormal radial basis and P = the smallest multiple of L that
    is at least max(2K, L)."""
    R = max(Q, 2 * Q) if R is None else R
    rng = np.random.default_rng(seed)
    qmat, _ = np.linalg.qr(rng.standard_normal((R, Q)))
    P = L * max(1, -(-max(2 * K, L) // L))
    return PolarGrid(qmat, P, K, Q)


def synthesize(g: PolarGrid, a: np.ndarray) -> np.ndarray:
    """I(r_p, phi_m) = sum_{k,q} a_{k,q} f_q(r_p) e^{i k phi_m}  (§I eq. (2)); a is k-major."""
    A = np.asarray(a).reshape(g.K, g.Q)
    phi = 2 * np.pi * np.arange(g.P) / g.P
    ang = np.exp(1j * np.outer(np.arange(g.K), phi))             # K x P
    return g.radial @ A.T @ ang                                   # R x P


def rotate_pixels(g: PolarGrid, img: np.ndarray, l: int, L: int) -> np.ndarray:
    """(R_theta I)(r, phi) = I(r, phi - theta), theta = 2 pi l / L: shift the angle axis."""
    return np.roll(img, l * (g.P // L), axis=1)


def analyze(g: PolarGrid, img: np.ndarray) -> np.ndarray:
    """Coefficients of a sampled image (inverse of ``synthesize`` on its range), k-major."""
    phi = 2 * np.pi * np.arange(g.P) / g.P
    ang = np.exp(-1j * np.outer(np.arange(g.K), phi)) / g.P      # K x P
    A = (g.radial.T @ img @ ang.T).T                              # K x Q
    return A.reshape(-1)


def distances_pixels(g: PolarGrid, V: np.ndarray, a: np.ndarray, L: int, offs) -> np.ndarray:
    """r[j, i] = ||R_{o_i} I_a - I_{v_j}||^2 / P on the pixel grid (explicit pixel rotation)."""
    Ia = synthesize(g, a)
    Iv = [synthesize(g, v) for v in V]
    r = np.empty((len(V), len(offs)))
    for i, o in enumerate(offs):
        Ir = rotate_pixels(g, Ia, int(o), L)
        for j in range(len(V)):
            d = Ir - Iv[j]
            r[j, i] = float(np.sum(d.real ** 2 + d.imag ** 2)) / g.P
    return r
