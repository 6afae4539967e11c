"""Seeded synthetic workloads for 2-D multi-reference alignment in steerable coefficients.

This module only draws random inputs. It holds no part of the EM arithmetic; both the
CPU oracle (``oracle/``) and the HIP path are fed from it.

Observation model (§I, eq. (4)): ``v_j = a ∘ exp(-i k̄ θ_j) + ε_j`` with ``ε_j`` circular complex
Gaussian, ``E|ε_jd|^2 = σ²`` (real and imaginary parts each ``N(0, σ²/2)``), and rotations on the
grid ``θ_j = 2π l_j / L`` (§II-B).  Coefficients are stored k-major: entry ``d = k·Q + q`` has
angular index ``k̄[d] = d // Q``.

Random streams (numpy PCG64, one ``SeedSequence([seed, stream, chunk])`` per 65 536-row chunk,
so any row range can be regenerated without the rest):

* 0  image coefficients ``a``
* 1  rotation indices ``l_j``
* 2  noise ``ε_j``
* 3  random EM initialisation ``a_0``
* 4  independent draws of the post-synchronisation rotation error (to learn the prior)

The paper's data (sPCA coefficients of ribosome projection images) is not available; these
draws stand in for it with the sizes, SNRs, rotation grids and error spreads of the paper's
experiments (§IV) scaled to the workloads below.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

CHUNK = 65536
STREAM_IMAGE, STREAM_ROT, STREAM_NOISE, STREAM_INIT, STREAM_PRIOR = 0, 1, 2, 3, 4


@dataclasses.dataclass(frozen=True)
class Workload:
    """Shape and statistics of one synthetic EM workload."""

    name: str
    K: int                      # angular indices k = 0..K-1
    Q: int                      # radial indices q = 0..Q-1
    N: int                      # observations
    L: int                      # rotation grid size
    snr: float                  # ||a||^2 / (D sigma^2)
    var_law: str                # "inv1pk": 1/(1+k); "inv1pk2": 1/(1+k)^2; "decay8": (4 e^{-k/8})^2
    rot_law: str                # "uniform" (l ~ U{0..L-1}) or "gauss" (rint N(0, std^2) wrapped)
    rot_std_deg: float = 0.0    # std of the post-synchronisation error, degrees
    half_window: Optional[int] = None   # window offsets -h..h; None = full search over L
    precision: str = "fp64"
    iters: int = 20
    init: str = "random"        # "random" (stream 3) or "mean" (a_0 = mean of the observations)
    gamma: float = 0.0          # KL-prior weight
    prior_draws: int = 0        # stream-4 draws used to learn the prior histogram

    @property
    def D(self) -> int:
        return self.K * self.Q

    @property
    def kbar(self) -> np.ndarray:
        return np.repeat(np.arange(self.K, dtype=np.int64), self.Q)

    @property
    def window(self) -> tuple[int, int]:
        """(lo, W): offsets lo..lo+W-1; full search is (0, L)."""
        if self.half_window is None:
            return 0, self.L
        return -self.half_window, 2 * self.half_window + 1

    @property
    def rot_std_steps(self) -> float:
        return self.rot_std_deg * self.L / 360.0

    def replace(self, **kw) -> "Workload":
        return dataclasses.replace(self, **kw)


# The five workloads: plain EM in FP64 (small), plain full-search EM in FP32 (the baseline the
# windowed form is compared against), windowed Synch-EM in BF16 (split precision), the
# differentiable log-likelihood on the windowed setup, and a large windowed run in FP16.
WORKLOADS = {
    "c1": Workload("c1", K=16, Q=8, N=1000, L=64, snr=0.5, var_law="inv1pk", rot_law="uniform",
                   precision="fp64", iters=20, init="random", gamma=0.0),
    "c2": Workload("c2", K=32, Q=16, N=100_000, L=360, snr=1 / 8, var_law="inv1pk2",
                   rot_law="uniform", precision="fp32", iters=50, init="random", gamma=0.0),
    "c3": Workload("c3", K=32, Q=16, N=100_000, L=360, snr=1 / 8, var_law="inv1pk2",
                   rot_law="gauss", rot_std_deg=8.0, half_window=24, precision="bf16x3",
                   iters=50, init="mean", gamma=100.0, prior_draws=1_000_000),
    "c4": Workload("c4", K=32, Q=16, N=100_000, L=360, snr=1 / 8, var_law="inv1pk2",
                   rot_law="gauss", rot_std_deg=8.0, half_window=24, precision="fp32",
                   iters=5, init="mean", gamma=100.0, prior_draws=1_000_000),
    "c4fd": Workload("c4fd", K=8, Q=4, N=200, L=16, snr=0.5, var_law="inv1pk2",
                     rot_law="gauss", rot_std_deg=45.0, half_window=None, precision="fp64",
                     iters=5, init="mean", gamma=0.0),
    "c5": Workload("c5", K=64, Q=32, N=1_000_000, L=720, snr=1 / 32, var_law="inv1pk2",
                   rot_law="gauss", rot_std_deg=15.0, half_window=90, precision="fp16",
                   iters=30, init="mean", gamma=100.0, prior_draws=1_000_000),
}


def _rng(seed: int, stream: int, chunk: int = 0) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, stream, chunk])))


def coefficient_variance(w: Workload) -> np.ndarray:
    """Per-entry variance of the image coefficients (length D)."""
    k = w.kbar.astype(np.float64)
    if w.var_law == "inv1pk":
        return 1.0 / (1.0 + k)
    if w.var_law == "inv1pk2":
        return 1.0 / (1.0 + k) ** 2
    if w.var_law == "decay8":           # the signal prior fitted in §IV-B, with beta = 8
        return (4.0 * np.exp(-k / 8.0)) ** 2
    raise ValueError(f"unknown variance law {w.var_law!r}")


def _cn(rng: np.random.Generator, shape, var) -> np.ndarray:
    """Circular complex Gaussian with E|z|^2 = var."""
    s = np.sqrt(np.asarray(var, dtype=np.float64) / 2.0)
    return s * rng.standard_normal(shape) + 1j * (s * rng.standard_normal(shape))


def image(w: Workload, seed: int) -> np.ndarray:
    """Ground-truth coefficients a (complex128, length D), a_kq ~ CN(0, var(k))."""
    return _cn(_rng(seed, STREAM_IMAGE), w.D, coefficient_variance(w))


def noise_variance(a: np.ndarray, snr: float) -> float:
    """sigma^2 = ||a||^2 / (D * SNR) for the realised image."""
    return float(np.vdot(a, a).real / (a.size * snr))


def wrap(l: np.ndarray, L: int) -> np.ndarray:
    """Integer rotation index wrapped to [-L/2, L/2)."""
    return (np.asarray(l, dtype=np.int64) + L // 2) % L - L // 2


def _rotation_draw(w: Workload, rng: np.random.Generator, n: int) -> np.ndarray:
    if w.rot_law == "uniform":
        return rng.integers(0, w.L, size=n, dtype=np.int64)
    if w.rot_law == "gauss":
        e = rng.standard_normal(n) * w.rot_std_steps
        return wrap(np.rint(e).astype(np.int64), w.L)      # rint: round half to even
    raise ValueError(f"unknown rotation law {w.rot_law!r}")


def rotations(w: Workload, seed: int, start: int = 0, stop: Optional[int] = None) -> np.ndarray:
    """Rotation indices l_j of rows [start, stop) (int64)."""
    stop = w.N if stop is None else stop
    out = []
    for c in range(start // CHUNK, (stop - 1) // CHUNK + 1 if stop > start else start // CHUNK):
        c0 = c * CHUNK
        n = min(CHUNK, w.N - c0)
        l = _rotation_draw(w, _rng(seed, STREAM_ROT, c), n)
        lo, hi = max(start, c0) - c0, min(stop, c0 + n) - c0
        out.append(l[lo:hi])
    return np.concatenate(out) if out else np.zeros(0, np.int64)


def observations(w: Workload, seed: int, start: int = 0, stop: Optional[int] = None,
                 dtype=np.complex128, a: Optional[np.ndarray] = None) -> np.ndarray:
    """Noisy rotated observations v_j for rows [start, stop), shape (rows, D).

    The phase exp(-i k θ_l) is evaluated at the exact grid angle 2π((k·l) mod L)/L.
    """
    stop = w.N if stop is None else stop
    a = image(w, seed) if a is None else a
    s2 = noise_variance(a, w.snr)
    kb = w.kbar
    # exp(-2 pi i m / L) for every residue m, looked up per entry (the same values as evaluating
    # it entry by entry)
    phase = np.exp(-2j * np.pi * np.arange(w.L) / w.L)
    out = np.empty((stop - start, w.D), dtype=dtype)
    pos = 0
    for c in range(start // CHUNK, (stop - 1) // CHUNK + 1 if stop > start else start // CHUNK):
        c0 = c * CHUNK
        n = min(CHUNK, w.N - c0)
        lo, hi = max(start, c0) - c0, min(stop, c0 + n) - c0
        l = _rotation_draw(w, _rng(seed, STREAM_ROT, c), n)[lo:hi]
        eps = _cn(_rng(seed, STREAM_NOISE, c), (n, w.D), s2)[lo:hi]
        m = (kb[None, :] * l[:, None]) % w.L
        v = a[None, :] * phase[m] + eps
        out[pos:pos + (hi - lo)] = v
        pos += hi - lo
    return out


def observation_chunks(w: Workload, seed: int, dtype=np.complex64, a: Optional[np.ndarray] = None,
                       workers: int = 1):
    """Yield (first_row, rows) over the generator's chunks in order: the same values as
    observations(), without holding all N rows at once.  workers > 1 generates chunks on that
    many threads (the draws of every chunk come from its own seeded stream, so the values do not
    depend on the thread count)."""
    a = image(w, seed) if a is None else a
    nch = (w.N + CHUNK - 1) // CHUNK
    one = lambda c: observations(w, seed, c * CHUNK, min(w.N, (c + 1) * CHUNK), dtype=dtype, a=a)
    if workers <= 1:
        for c in range(nch):
            yield c * CHUNK, one(c)
        return
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(workers) as ex:
        futs = {}
        for c in range(nch):
            while len(futs) >= 2 * workers:
                c0 = min(futs)
                yield c0 * CHUNK, futs.pop(c0).result()
            futs[c] = ex.submit(one, c)
        for c0 in sorted(futs):
            yield c0 * CHUNK, futs[c0].result()


def random_init(w: Workload, seed: int) -> np.ndarray:
    """Seeded random EM initialisation a_0 ~ CN(0, var(k)) (stream 3)."""
    return _cn(_rng(seed, STREAM_INIT), w.D, coefficient_variance(w))


def prior_error_draws(w: Workload, seed: int, n: Optional[int] = None) -> np.ndarray:
    """Independent draws of the post-synchronisation rotation error (stream 4), int32, wrapped."""
    n = w.prior_draws if n is None else n
    out = np.empty(n, dtype=np.int32)
    for c in range((n + CHUNK - 1) // CHUNK):
        m = min(CHUNK, n - c * CHUNK)
        out[c * CHUNK:c * CHUNK + m] = _rotation_draw(w, _rng(seed, STREAM_PRIOR, c), m)
    return out


def describe(w: Workload) -> dict:
    lo, W = w.window
    return {"workload": w.name, "K": w.K, "Q": w.Q, "D": w.D, "N": w.N, "L": w.L,
            "window_lo": lo, "W": W, "snr": w.snr, "precision": w.precision,
            "rotations": w.rot_law if w.rot_law == "uniform" else f"gauss {w.rot_std_deg} deg",
            "gamma": w.gamma, "iters": w.iters}
