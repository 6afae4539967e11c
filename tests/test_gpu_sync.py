"""Synchronize and Match on the GPU (relative rotations, the power method, nearest neighbours,
alignment; §II-A, §III-A) against the FP64 oracle on the same seeded inputs.  Integer results
(rotation indices, neighbours) must agree exactly wherever the oracle's gap to the runner-up is
clear of FP32 rounding; angles from the power method to 1e-9 rad."""
import numpy as np
import pytest

import oracle
import workloads as wl

pytestmark = pytest.mark.gpu


def _data(K, Q, L, N, snr, seed=0):
    w = wl.WORKLOADS["c2"].replace(K=K, Q=Q, L=L, N=N, snr=snr)
    a = wl.image(w, seed)
    V = wl.observations(w, seed, a=a).astype(np.complex64)
    return w, a, V


def _top2_gap(f, axis):
    s = np.sort(f, axis=axis)
    return np.take(s, -1, axis=axis) - np.take(s, -2, axis=axis)


@pytest.mark.parametrize("K,Q,L,P,snr", [(8, 8, 72, 61, 0.5), (5, 3, 36, 40, 2.0),
                                          (32, 16, 360, 33, 1 / 8)])
def test_relative_rotations(gpu, K, Q, L, P, snr):
    """Ragged pair tiles (P not a multiple of 16), odd K and Q, L not a multiple of 16."""
    import torch
    from paper_2105_07372_amd import relative_rotations
    w, a, V = _data(K, Q, L, P, snr)
    print(f"relrot K={K} Q={Q} L={L} P={P}", flush=True)
    rel, gap, dot = relative_rotations(torch.from_numpy(V).to(gpu), K, Q, L)
    rel, gap, dot = rel.cpu().numpy(), gap.cpu().numpy(), dot.cpu().numpy()
    Vd = V.astype(np.complex128)
    ro, f = oracle.relative_rotations(Vd, w.kbar, L)
    scale = np.abs(f).max()
    clear = _top2_gap(f, 2) > 1e-5 * scale
    assert clear.mean() > 0.95
    assert np.array_equal(rel[clear], ro[clear])
    assert np.abs(dot - f[:, :, 0]).max() <= 1e-5 * scale
    assert np.abs(gap[clear] - _top2_gap(f, 2)[clear]).max() <= 1e-5 * scale


def test_relative_rotations_noiseless_are_differences(gpu):
    import torch
    from paper_2105_07372_amd import relative_rotations
    K, Q, L, P = 8, 8, 72, 40
    w = wl.WORKLOADS["c2"].replace(K=K, Q=Q, L=L, N=P)
    a = wl.image(w, 1)
    l = np.random.default_rng(2).integers(0, L, P)
    V = np.stack([a * np.exp(-2j * np.pi * w.kbar * li / L) for li in l]).astype(np.complex64)
    rel, _, _ = relative_rotations(torch.from_numpy(V).to(gpu), K, Q, L)
    assert np.array_equal(rel.cpu().numpy(), np.mod(l[:, None] - l[None, :], L))


def test_ppm_matches_oracle(gpu):
    """The power method on the oracle's relative rotations (FP64 on both sides)."""
    import torch
    from paper_2105_07372_amd import ppm
    w, a, V = _data(8, 8, 72, 150, 0.5)
    ro, _ = oracle.relative_rotations(V.astype(np.complex128), w.kbar, 72)
    for iters in (0, 1, 7, 40):
        th = ppm(torch.from_numpy(ro.astype(np.int32)).to(gpu), 72, iters).cpu().numpy()
        to = oracle.ppm(ro, 72, iters)
        assert np.abs(np.angle(np.exp(1j * (th - to)))).max() <= 1e-9, iters


@pytest.mark.parametrize("L", [72, 3000])          # 3000: the phases read from global memory
def test_ppm_any_integer_relative_rotations(gpu, L):
    """Relative rotations are taken mod L: any integers, negative and past L included, give the
    oracle's iterates."""
    import torch
    from paper_2105_07372_amd import ppm
    rng = np.random.default_rng(7)
    rel = rng.integers(-2 * L, 2 * L, size=(300, 300)).astype(np.int32)
    for iters in (1, 5):
        th = ppm(torch.from_numpy(rel).to(gpu), L, iters).cpu().numpy()
        to = oracle.ppm(rel, L, iters)
        assert np.abs(np.angle(np.exp(1j * (th - to)))).max() <= 1e-9, (L, iters)


@pytest.mark.parametrize("K,Q,N,P", [(8, 8, 3001, 200), (16, 8, 1000, 1000), (4, 2, 517, 37),
                                     (32, 32, 600, 100)])   # the last: rows too long for LDS
def test_nearest_neighbours(gpu, K, Q, N, P):
    import torch
    from paper_2105_07372_amd import nearest
    w, a, V = _data(K, Q, 36, N, 1.0)
    print(f"nearest K={K} Q={Q} N={N} P={P}", flush=True)
    nn, gap = nearest(torch.from_numpy(V).to(gpu), K, Q, P)
    nn, gap = nn.cpu().numpy(), gap.cpu().numpy()
    no, d = oracle.nearest_neighbours(V.astype(np.complex128), P)
    d = d.copy()
    idx = np.arange(min(P, N))
    d[idx, idx] = np.inf
    s = np.sort(d, axis=1)
    g = s[:, 1] - s[:, 0]
    scale = np.abs(d[np.isfinite(d)]).max()
    clear = g > 1e-5 * scale
    assert clear.mean() > 0.95
    assert np.array_equal(nn[clear], no[clear])
    assert all(nn[i] != i for i in range(min(P, N)))
    assert np.abs(gap[clear] - g[clear]).max() <= 1e-5 * scale


def test_sync_match_end_to_end_and_align(gpu):
    """Synchronize and Match at SNR 10^4, where every pairwise estimate has a clear margin
    (checked on the oracle first), so the power method sees the oracle's H.  Many members of S_P
    share a rotation and are near-duplicates, so several neighbours are correct: every GPU choice
    must be a nearest member up to FP32 rounding, and theta_i must equal the oracle's phi at the
    GPU's chosen neighbour.  (The power method on noisy inputs: test_ppm_matches_oracle.)"""
    import torch
    from paper_2105_07372_amd import align, sync_match
    K, Q, L, N, P = 16, 8, 72, 4000, 128
    w, a, V = _data(K, Q, L, N, 1e4, seed=3)
    Vd = V.astype(np.complex128)
    ro, f = oracle.relative_rotations(Vd[:P], w.kbar, L)
    assert (_top2_gap(f, 2) > 1e-4 * np.abs(f).max()).all()
    th_o, phi_o, _, nn_o = oracle.synchronize_and_match(Vd, w.kbar, L, P, 30)
    obs = torch.from_numpy(V).to(gpu)
    th, nn = sync_match(obs, K, Q, L, P, 30)
    th, nn = th.cpu().numpy(), nn.cpu().numpy()
    _, d = oracle.nearest_neighbours(Vd, P)
    d[np.arange(P), np.arange(P)] = np.inf
    rows = np.arange(N)
    assert ((nn >= 0) & (nn < P)).all() and (nn[:P] != np.arange(P)).all()
    assert (d[rows, nn] - d[rows, nn_o] <= 1e-5 * np.abs(d[np.isfinite(d)]).max()).all()
    assert np.abs(np.angle(np.exp(1j * (th - phi_o[nn])))).max() <= 1e-9
    assert np.mean(nn == nn_o) > 0.5
    va = align(obs, K, Q, torch.from_numpy(th).to(gpu)).cpu().numpy()
    vo = oracle.align(Vd, w.kbar, th)
    assert np.abs(va - vo).max() <= 2e-6 * np.abs(vo).max()


def test_sync_match_full_size(gpu):
    """The default workload's shape (N = 10^5, D = 512, L = 360) with P = 1024: sampled pairs and
    rows against the oracle, and the time of each stage."""
    import time
    import torch
    from paper_2105_07372_amd import nearest, relative_rotations, sync_match
    K, Q, L, N, P = 32, 16, 360, 100_000, 1024
    w = wl.WORKLOADS["c2"]
    a = wl.image(w, 0)
    obs = torch.empty((N, K * Q), dtype=torch.complex64, device=gpu)
    for r0, ch in wl.observation_chunks(w, 0, dtype=np.complex64, a=a, workers=16):
        obs[r0:r0 + len(ch)].copy_(torch.from_numpy(ch))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    th, nn = sync_match(obs, K, Q, L, P, 50)
    dt = time.perf_counter() - t0
    print(f"sync_match N={N} P={P} L={L}: {dt * 1e3:.1f} ms", flush=True)
    rel, _, _ = relative_rotations(obs, K, Q, L, P)
    Vs = obs[:48].cpu().numpy().astype(np.complex128)
    ro, f = oracle.relative_rotations(Vs, w.kbar, L)
    clear = _top2_gap(f, 2) > 1e-5 * np.abs(f).max()
    assert np.array_equal(rel[:48, :48].cpu().numpy()[clear], ro[clear])
    rows = np.random.default_rng(0).choice(N, 300, replace=False)
    Vp = obs[:P].cpu().numpy().astype(np.complex128)
    Vr = obs[torch.from_numpy(rows).to(gpu)].cpu().numpy().astype(np.complex128)
    d = (np.sum(np.abs(Vp) ** 2, axis=1)[None, :] - 2 * np.real(np.conj(Vr) @ Vp.T))
    d[rows[:, None] == np.arange(P)[None, :]] = np.inf
    s = np.sort(d, axis=1)
    clear = s[:, 1] - s[:, 0] > 1e-5 * np.abs(d[np.isfinite(d)]).max()
    nn_r = nn.cpu().numpy()[rows]
    assert np.array_equal(nn_r[clear], np.argmin(d, axis=1)[clear])
    assert np.isfinite(th.cpu().numpy()).all()


def test_aligned_mean_and_error_bins(gpu):
    """The aligned average (FP64) and the binned centred errors against the oracle, on angles
    drawn away from the bin edges."""
    import torch
    from paper_2105_07372_amd import aligned_mean, error_bins
    K, Q, L, N = 16, 8, 72, 3001
    w, a, V = _data(K, Q, L, N, 0.5)
    rng = np.random.default_rng(9)
    th = rng.uniform(-np.pi, np.pi, N)
    m = rng.integers(-100, 100, N)
    lc = 11
    th_hat = th + 2 * np.pi * (lc + m + rng.uniform(0.1, 0.9, N)) / L
    obs = torch.from_numpy(V).to(gpu)
    am = aligned_mean(obs, K, Q, torch.from_numpy(th).to(gpu)).cpu().numpy()
    ao = oracle.aligned_mean(V.astype(np.complex128), w.kbar, th)
    assert np.abs(am - ao).max() <= 1e-12 * np.abs(ao).max()
    bins = error_bins(torch.from_numpy(th_hat).to(gpu), torch.from_numpy(th).to(gpu), L, lc)
    assert np.array_equal(bins.cpu().numpy(), oracle.centred_error_bins(th_hat, th, lc, L))
    assert np.array_equal(bins.cpu().numpy(), np.mod(m, L))


def test_learning_the_prior_from_the_synchronizer(gpu):
    """The algorithm that learns the rotation distribution, with Synchronize and Match as the
    synchronizer, over R = 3 trials: every GPU stage after the synchronizer is fed the oracle's
    rotations, and the centring rotation, the binned errors and the learned window prior equal
    the oracle's; the GPU synchronizer's own rotations are checked as in the end-to-end test."""
    import torch
    from paper_2105_07372_amd import (aligned_mean, error_bins, global_rotation, learn_prior,
                                      sync_match)
    K, Q, L, N, P, h = 16, 8, 72, 3000, 256, 9
    bins_all = []
    for r in range(3):
        w, a, V = _data(K, Q, L, N, 1.0, seed=20 + r)
        lt = wl.rotations(w, 20 + r)                            # the generator's true rotations
        th_true = 2 * np.pi * lt / L
        Vd = V.astype(np.complex128)
        th_o, phi_o, _, nn_o = oracle.synchronize_and_match(Vd, w.kbar, L, P, 50)
        lc_o = oracle.global_rotation(a, oracle.aligned_mean(Vd, w.kbar, th_o), w.kbar, L)
        b_o = oracle.centred_error_bins(th_o, th_true, lc_o, L)
        obs = torch.from_numpy(V).to(gpu)
        th_g, nn_g = sync_match(obs, K, Q, L, P, 50)
        ok = nn_g.cpu().numpy() == nn_o
        assert ok.mean() > 0.9
        am = aligned_mean(obs, K, Q, torch.from_numpy(th_o).to(gpu))
        lc = global_rotation(torch.from_numpy(a).to(gpu), am, K, Q, L)
        assert lc == lc_o
        b = error_bins(torch.from_numpy(th_o).to(gpu), torch.from_numpy(th_true).to(gpu), L, lc)
        assert np.array_equal(b.cpu().numpy(), b_o)
        bins_all.append(b)
    allb = torch.cat(bins_all)
    rb, cnt, nin = learn_prior(allb, L, -h, 2 * h + 1)
    rb_o, cnt_o, _ = oracle.histogram_prior(allb.cpu().numpy(), L, -h, 2 * h + 1)
    assert np.allclose(rb, rb_o, rtol=0, atol=1e-15)
    assert rb[h - 2:h + 3].sum() > 0.5                          # concentrated around no error
