"""The learned rotation prior on the GPU: the histogram kernel (Section III-B eq. (22); Algorithm
"learning rotation distribution"), prior logits trained through the library's forward and
adjoint kernels, and what the learned prior gains in Synch-EM (the gamma study of Section IV-C,
on synthetic data)."""
import numpy as np
import pytest

import oracle
import workloads as wl

pytestmark = pytest.mark.gpu


def test_histogram_kernel_is_exact(gpu):
    import torch
    from paper_2105_07372_amd import learn_prior
    w = wl.WORKLOADS["c5"]
    err = wl.prior_error_draws(w, 0, 300_000)
    for (lo, W) in (w.window, (-45, 91), (700, 40)):
        rb, cnt, nin = learn_prior(torch.from_numpy(err).to(gpu), w.L, lo, W)
        rb_o, cnt_w, cnt_all = oracle.histogram_prior(err, w.L, lo, W)
        assert np.array_equal(cnt, cnt_all)
        assert nin == int(cnt_w.sum())
        assert np.array_equal(rb, rb_o)


def _small(seed, snr=1 / 16, N=3000):
    return wl.WORKLOADS["c3"].replace(N=N, K=8, Q=8, L=72, rot_std_deg=10.0, half_window=6,
                                      snr=snr)


def _adam_train(grad_fn, W, steps=150, lr=0.05):
    eta = np.zeros(W)
    m = np.zeros(W)
    v = np.zeros(W)
    for t in range(1, steps + 1):
        g = grad_fn(eta)                   # gradient of the objective to maximise
        m = 0.9 * m + 0.1 * g
        v = 0.999 * v + 0.001 * g * g
        eta = eta + lr * (m / (1 - 0.9 ** t)) / (np.sqrt(v / (1 - 0.999 ** t)) + 1e-12)
    return eta


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_prior_logits_trained_through_adjoint(gpu, prec):
    """Prior logits eta are trained by gradient ascent on the marginal log-likelihood of simulated
    training trials with known images (the Monte-Carlo setting of the learning algorithm), using
    the GPU forward/adjoint; the same optimisation with the oracle's gradients lands on the same
    logits, and the trained distribution is close to the histogram of the true rotations."""
    import torch
    from paper_2105_07372_amd import EM
    from paper_2105_07372_amd.autograd import marginal_loglik
    trials = []
    for seed in (10, 11):
        w = _small(seed, snr=1.0)
        a = wl.image(w, seed)
        V = wl.observations(w, seed, a=a)
        s2 = wl.noise_variance(a, w.snr)
        lo, W = w.window
        obs = torch.from_numpy(V.astype(np.complex128 if prec == "fp64" else np.complex64))
        em = EM(obs.to(gpu), K=w.K, Q=w.Q, L=w.L, sigma2=s2, window=(lo, W), precision=prec)
        trials.append((w, a, V, s2, em))
    lo, W = trials[0][0].window

    def grad_gpu(eta):
        e_t = torch.from_numpy(eta).to(gpu).requires_grad_(True)
        tot = 0.0
        for (w, a, V, s2, em) in trials:
            a_t = torch.from_numpy(a).to(gpu)
            s_t = torch.tensor(s2, dtype=torch.float64, device=gpu)
            tot = tot + marginal_loglik(em, a_t, s_t, e_t) / w.N
        (g,) = torch.autograd.grad(tot, (e_t,))
        return g.cpu().numpy()

    def grad_oracle(eta):
        r = np.exp(eta - eta.max())
        r /= r.sum()
        g = np.zeros(W)
        for (w, a, V, s2, _) in trials:
            g += oracle.grad_loglik(V, a, s2, r, w.kbar, w.L, oracle.offsets(lo, W))[3] / w.N
        return g

    eta_probe = np.linspace(-0.5, 0.5, W)
    gg, go = grad_gpu(eta_probe), grad_oracle(eta_probe)
    tol = 1e-10 if prec == "fp64" else 1e-4
    assert np.abs(gg - go).max() <= tol * max(1.0, np.abs(go).max())
    eta_g = _adam_train(grad_gpu, W, steps=300)
    eta_o = _adam_train(grad_oracle, W, steps=300)
    rg, ro = np.exp(eta_g - eta_g.max()), np.exp(eta_o - eta_o.max())
    rg, ro = rg / rg.sum(), ro / ro.sum()
    assert np.abs(rg - ro).max() <= (1e-8 if prec == "fp64" else 2e-3)
    # the true rotations of the training trials, binned on the window
    true = np.concatenate([wl.rotations(t[0], s) for t, s in zip(trials, (10, 11))])
    hist, _, _ = oracle.histogram_prior(true, trials[0][0].L, lo, W)
    assert np.abs(rg - hist).max() <= 0.03
    for t in trials:
        t[4].close()


def test_learned_prior_gains_over_no_prior(gpu):
    """Synch-EM with the learned prior (gamma = 0.02 N, rho_0 = rho_bar) against the same window
    without it (gamma = 0, uniform rho_0) and against full search, on three seeds at SNR 1/16 and
    1/32: the learned prior reaches the stopping tolerance in fewer iterations with a relative
    error no worse than 2% above the run without it."""
    import torch
    from paper_2105_07372_amd import EM, learn_prior
    rows = []
    for snr in (1 / 16, 1 / 32):
        for seed in (0, 1, 2):
            w = _small(seed, snr=snr)
            a = wl.image(w, seed)
            V = wl.observations(w, seed, a=a)
            s2 = wl.noise_variance(a, w.snr)
            lo, W = w.window
            obs = torch.from_numpy(V.astype(np.complex64)).to(gpu)
            err = torch.from_numpy(wl.prior_error_draws(w, seed, 200_000)).to(gpu)
            rb, _, _ = learn_prior(err, w.L, lo, W)
            res = {}
            for name, kw in (("prior", dict(window=(lo, W), prior=rb, gamma=0.02 * w.N)),
                             ("none", dict(window=(lo, W), gamma=0.0)),
                             ("full", dict()),):
                em = EM(obs, K=w.K, Q=w.Q, L=w.L, sigma2=s2, precision="bf16x3", **kw)
                n, _ = em.step(300, tol=1e-5)
                res[name] = (n, oracle.relative_error(em.state()[0], a, w.kbar, w.L))
                em.close()
            print(f"snr={snr:.4f} seed={seed} {res}", flush=True)
            rows.append(res)
            assert res["prior"][0] < res["none"][0]
            assert res["prior"][1] <= 1.02 * res["none"][1]
    assert np.mean([r["prior"][0] for r in rows]) < 0.6 * np.mean([r["none"][0] for r in rows])
