"""Algorithm "Synch-EM" end to end on the GPU, on synthetic data with uniform rotations (a
stand-in for the paper's comparison of Synch-EM with plain EM, §IV, and for its window-size study):
the rotation prior is learned from the synchronizer's own errors over simulated trials (Algorithm
"learning rotation distribution"), the data are synchronized by Synchronize and Match and aligned,
the EM starts from the aligned average and searches only the window with the learned prior.  The
error against the truth (up to a global rotation, eq. (19)) is computed by the oracle's evaluator;
everything else runs in the HIP library.  The error is minimised over the continuous circle
because the synchronizer leaves an arbitrary global rotation, off the grid."""
import numpy as np
import pytest

import oracle
import workloads as wl

pytestmark = pytest.mark.gpu

K, Q, L, N, P, SNR = 16, 8, 72, 6000, 300, 0.5


def _problem(seed):
    w = wl.WORKLOADS["c2"].replace(K=K, Q=Q, L=L, N=N, snr=SNR)
    a = wl.image(w, seed)
    V = wl.observations(w, seed, a=a).astype(np.complex64)
    th = 2 * np.pi * wl.rotations(w, seed) / L
    return w, a, V, th, wl.noise_variance(a, w.snr)


def _learned_prior(gpu, h, trials=3):
    """Centred, binned errors of Synchronize and Match over simulated trials, histogrammed over the
    window -h .. h.  After alignment the EM's rotation variable is theta - theta_hat (+ theta_c),
    the negated centred error, so the bins are taken of that (error_bins with the roles of the two
    angle vectors swapped and -l_c)."""
    import torch
    from paper_2105_07372_amd import (aligned_mean, error_bins, global_rotation, learn_prior,
                                      sync_match)
    bins = []
    for r in range(trials):
        w, a, V, th, _ = _problem(100 + r)
        obs = torch.from_numpy(V).to(gpu)
        th_hat, _ = sync_match(obs, K, Q, L, P, 50)
        lc = global_rotation(torch.from_numpy(a).to(gpu), aligned_mean(obs, K, Q, th_hat), K, Q, L)
        bins.append(error_bins(torch.from_numpy(th).to(gpu), th_hat, L, -lc))
    rb, _, nin = learn_prior(torch.cat(bins), L, -h, 2 * h + 1)
    return rb, nin / (trials * N)


def _synch_em(gpu, obs, s2, h, rb, gamma, tol=1e-5, iters=400):
    from paper_2105_07372_amd import EM, align, aligned_mean, sync_match
    th_hat, _ = sync_match(obs, K, Q, L, P, 50)
    al = align(obs, K, Q, th_hat)
    a0 = aligned_mean(obs, K, Q, th_hat).cpu().numpy()
    em = EM(al, K=K, Q=Q, L=L, sigma2=s2, window=(-h, 2 * h + 1), prior=rb, gamma=gamma,
            precision="fp32", a0=a0)
    done, _ = em.step(iters, tol=tol)
    a_hat = em.state()[0]
    em.close()
    return a_hat, done


def test_synch_em_against_plain_em(gpu):
    import torch
    from paper_2105_07372_amd import EM
    w, a, V, th, s2 = _problem(0)
    obs = torch.from_numpy(V).to(gpu)
    h = 12
    rb, inside = _learned_prior(gpu, h)
    assert inside > 0.8                        # the window holds most of the synchronizer's errors
    a_s, it_s = _synch_em(gpu, obs, s2, h, rb, 100.0)
    err_s = oracle.relative_error_continuous(a_s, a, w.kbar)
    em = EM(obs, K=K, Q=Q, L=L, sigma2=s2, precision="fp32", a0=wl.random_init(w, 0))
    it_p, _ = em.step(1000, tol=1e-5)
    err_p = oracle.relative_error_continuous(em.state()[0], a, w.kbar)
    em.close()
    print(f"synch-em: err {err_s:.4f} in {it_s} iterations over W={2 * h + 1}; "
          f"plain EM: err {err_p:.4f} in {it_p} iterations over L={L}", flush=True)
    assert err_s <= 1.1 * err_p + 0.01
    # rotations visited: the window times the iterations, against the full grid's
    assert it_s * (2 * h + 1) < 0.5 * it_p * L


def test_window_size_study(gpu):
    """Error against the truth for a range of windows (the paper's study of BW): very narrow
    windows cut off real rotations, and beyond a width the error stops improving."""
    import torch
    w, a, V, th, s2 = _problem(1)
    obs = torch.from_numpy(V).to(gpu)
    errs = {}
    for h in (1, 4, 12, 24):
        rb, _ = _learned_prior(gpu, h, trials=2)
        a_s, it = _synch_em(gpu, obs, s2, h, rb, 100.0)
        errs[h] = oracle.relative_error_continuous(a_s, a, w.kbar)
        print(f"window h={h} (W={2 * h + 1}): err {errs[h]:.4f} in {it} iterations", flush=True)
    assert errs[12] <= errs[1]
    assert abs(errs[24] - errs[12]) <= 0.1 * errs[12] + 0.005


def test_template_matching_is_the_posterior_argmax(gpu):
    """Template matching against a reference (§II-A) is the argmax of the posterior with the
    reference as the estimate and a uniform prior over all L rotations: it equals the oracle's
    argmax_l Re <v_i, R_l ref> wherever the top two correlations are apart, and the observations
    aligned by it average to the reference's rotation of the image."""
    import torch
    from paper_2105_07372_amd import EM
    w, a, V, th, s2 = _problem(2)
    ref = V[0].astype(np.complex128)
    obs = torch.from_numpy(V).to(gpu)
    em = EM(obs, K=K, Q=Q, L=L, sigma2=s2, precision="fp32", a0=ref)
    _, am, mg = em.posterior()
    em.close()
    am = am.cpu().numpy()
    C = np.real(np.conj(V.astype(np.complex128)) @ (ref[:, None] * oracle.grid_phase(
        w.kbar, np.arange(L), L, -1).T))
    s = np.sort(C, axis=1)
    clear = s[:, -1] - s[:, -2] > 1e-4 * np.abs(C).max()
    assert clear.mean() > 0.95
    assert np.array_equal(am[clear], np.argmax(C, axis=1)[clear])


def test_signal_prior_decay_study(gpu):
    """The paper's study of the decay beta of the Gaussian image prior Gamma_a =
    diag((4 exp(-kbar / beta))^2) (eq. (17)), with Synch-EM on synthetic data: each beta runs, and
    a very strong prior (small beta) costs accuracy against a weak one."""
    import torch
    from paper_2105_07372_amd import EM, align, aligned_mean, sync_match
    w, a, V, th, s2 = _problem(3)
    obs = torch.from_numpy(V).to(gpu)
    h = 12
    rb, _ = _learned_prior(gpu, h, trials=2)
    th_hat, _ = sync_match(obs, K, Q, L, P, 50)
    al = align(obs, K, Q, th_hat)
    a0 = aligned_mean(obs, K, Q, th_hat).cpu().numpy()
    errs = {}
    for beta in (0.5, 4.0, 8.0, 32.0):
        gai = 1.0 / (4.0 * np.exp(-w.kbar / beta)) ** 2
        em = EM(al, K=K, Q=Q, L=L, sigma2=s2, window=(-h, 2 * h + 1), prior=rb, gamma=100.0,
                precision="fp32", a0=a0, gamma_a_inv=gai)
        it, _ = em.step(400, tol=1e-5)
        errs[beta] = oracle.relative_error_continuous(em.state()[0], a, w.kbar)
        em.close()
        print(f"beta={beta}: err {errs[beta]:.4f} in {it} iterations", flush=True)
    assert all(np.isfinite(list(errs.values())))
    assert errs[0.5] > errs[32.0]
