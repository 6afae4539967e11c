"""em_aligned_mean_noalloc (the entry point that allocates nothing; its partial sums live in the
library's static device array) against em_aligned_mean on the same inputs: bit-identical results
on consecutive calls, each later call smaller than the one before (the array keeps the earlier
call's contents), up to the largest D the library accepts."""
import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu


def _inputs(N, K, Q, seed):
    rng = np.random.default_rng(seed)
    V = (rng.standard_normal((N, K * Q)) + 1j * rng.standard_normal((N, K * Q))).astype(np.complex64)
    th = rng.uniform(-np.pi, np.pi, N)
    return V, th


def test_noalloc_matches_allocating_entry_point(gpu):
    import torch
    from paper_2105_07372_amd import aligned_mean
    # (N, K, Q): the largest D first, then smaller calls; N below and above the 256 workgroups
    for (N, K, Q, seed) in [(3001, 64, 32, 0), (70001, 32, 16, 1), (513, 8, 4, 2), (100, 3, 5, 3)]:
        print(f"noalloc aligned mean N={N} K={K} Q={Q}", flush=True)
        V, th = _inputs(N, K, Q, seed)
        obs = torch.from_numpy(V).to(gpu)
        th_d = torch.from_numpy(th).to(gpu)
        ref = aligned_mean(obs, K, Q, th_d)
        got = aligned_mean(obs, K, Q, th_d, noalloc=True)
        torch.cuda.synchronize()
        assert torch.equal(got, ref), (N, K, Q)
        kbar = np.repeat(np.arange(K), Q)
        ao = oracle.aligned_mean(V.astype(np.complex128), kbar, th)
        assert np.abs(got.cpu().numpy() - ao).max() <= 1e-10 * max(1.0, np.abs(ao).max())
    # twice in a row on the same stream, the second smaller, without a synchronisation between
    V1, th1 = _inputs(40000, 16, 16, 4)
    V2, th2 = _inputs(700, 16, 8, 5)
    o1, t1 = torch.from_numpy(V1).to(gpu), torch.from_numpy(th1).to(gpu)
    o2, t2 = torch.from_numpy(V2).to(gpu), torch.from_numpy(th2).to(gpu)
    r1, r2 = aligned_mean(o1, 16, 16, t1), aligned_mean(o2, 16, 8, t2)
    g1 = aligned_mean(o1, 16, 16, t1, noalloc=True)
    g2 = aligned_mean(o2, 16, 8, t2, noalloc=True)
    torch.cuda.synchronize()
    assert torch.equal(g1, r1) and torch.equal(g2, r2)
