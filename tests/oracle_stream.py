"""One oracle EM iteration over the N = 10^6 large-image workload, streamed over the generator's
65,536-row chunks, so that the full-size GPU steps are checked against the oracle rather than
against the kernel's own posteriors.  Each chunk is generated once: its complex64 rows go to the
GPU (what the library receives), and the same values taken in FP64 go through the oracle's E-step
and M-step; the M-step's double sum S (eq. (17)), the column sums W_t and the log-likelihood are
added over chunks in chunk order, in FP64.  Test infrastructure: calls only oracle/ and
workloads/."""
from __future__ import annotations

from concurrent.futures import ThreadPoolExecutor

import numpy as np

import oracle
import workloads as wl

_CACHE: dict = {}


def large_image_state(w, seed: int = 0):
    """The state the full-size large-image tests start the step from: (a_true, sigma2, rho_bar,
    a_t), with rho_t = rho_bar."""
    a_true = wl.image(w, seed)
    s2 = wl.noise_variance(a_true, w.snr)
    lo, W = w.window
    rb, _, _ = oracle.histogram_prior(wl.prior_error_draws(w, seed), w.L, lo, W)
    rng = np.random.default_rng(11)
    a_t = 0.9 * a_true + 0.05 * np.sqrt(s2) * (rng.standard_normal(w.D)
                                                + 1j * rng.standard_normal(w.D))
    return a_true, s2, rb, a_t


def upload_and_iterate(w, seed: int, obs, a_true, a_t, rho_t, s2, rho_bar, gamma,
                       workers: int = 6):
    """Fill obs (a CUDA complex64 tensor of N x D) with the workload's rows and return the oracle
    iteration from (a_t, rho_t) over all of them: dict(a, rho, ll, S, W)."""
    import torch
    key = (w, seed, a_t.tobytes(), np.asarray(rho_t).tobytes(), float(s2), float(gamma))
    need = key not in _CACHE
    lo, W = w.window
    offs = oracle.offsets(lo, W)

    def one(r0):
        r1 = min(w.N, r0 + wl.CHUNK)
        V32 = wl.observations(w, seed, r0, r1, dtype=np.complex64, a=a_true)
        if not need:
            return r0, V32, None
        V = V32.astype(np.complex128)
        wgt, lse, _ = oracle.estep(V, a_t, rho_t, s2, w.kbar, w.L, offs)
        _, S_c = oracle.mstep_a(V, wgt, w.kbar, w.L, offs, s2)
        return r0, V32, (S_c, wgt.sum(axis=0), float(np.sum(lse)))

    S = np.zeros(w.D, np.complex128)
    Wt = np.zeros(W)
    ll = 0.0
    starts = list(range(0, w.N, wl.CHUNK))
    with ThreadPoolExecutor(workers) as ex:
        futs = {}
        nxt = 0
        for r0 in starts:                      # at most 2 x workers chunks in flight
            while nxt < len(starts) and len(futs) < 2 * workers:
                futs[starts[nxt]] = ex.submit(one, starts[nxt])
                nxt += 1
            _, V32, part = futs.pop(r0).result()
            obs[r0:r0 + len(V32)].copy_(torch.from_numpy(V32))
            if part is not None:               # added in chunk order
                S += part[0]
                Wt += part[1]
                ll += part[2]
    if need:
        _CACHE[key] = {"a": S / w.N, "rho": oracle.mstep_rho(Wt, rho_bar, gamma), "ll": ll,
                       "S": S, "W": Wt}
    return _CACHE[key]
