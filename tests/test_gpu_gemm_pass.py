"""The long-window FP32 pass (pass_gm_kernel: the correlation GEMM over all window columns with the
posterior and M-step as its epilogue) against the FP64 oracle: full search over L = 360 and 384
(23 and 24 column tiles) and shorter windows, radial sizes Q = 8 .. 64, row counts around the
128-row tile (including one row and a ragged last tile), posterior queries, the adjoint's stored
and reloaded log-sum-exp, and agreement with the general pass."""
import numpy as np
import pytest

import oracle
import workloads as wl
from bounds import U32, loglik_bar

pytestmark = pytest.mark.gpu

TOL = dict(post=2e-4, a=2e-5, ll=1e-7)


def _problem(N, K, Q, L, h=None, seed=0):
    base = wl.WORKLOADS["c3"] if h is not None else wl.WORKLOADS["c2"]
    w = base.replace(N=N, K=K, Q=Q, L=L, half_window=h)
    a_true = wl.image(w, seed)
    V = wl.observations(w, seed, a=a_true)
    s2 = wl.noise_variance(a_true, w.snr)
    lo, W = w.window
    if h is not None:
        rb, _, _ = oracle.histogram_prior(wl.prior_error_draws(w, seed, 200_000), w.L, lo, W)
    else:
        rb = np.full(W, 1.0 / W)
    return w, a_true, V, s2, lo, W, rb


def _check(gpu, w, a_true, V, s2, lo, W, rb, gamma, rng, **kw):
    import torch
    from paper_2105_07372_amd import EM
    obs = torch.from_numpy(V.astype(np.complex64)).to(gpu)
    em = EM(obs, K=w.K, Q=w.Q, L=w.L, sigma2=s2, window=(lo, W), prior=rb, gamma=gamma,
            precision="fp32", **kw)
    a_t = 0.9 * a_true + 0.1 * a_true * rng.standard_normal(w.D)
    rho_t = rb * rng.uniform(0.5, 1.5, W)
    rho_t /= rho_t.sum()
    em.set_state(a_t, rho_t, 0)
    offs = oracle.offsets(lo, W)
    wg, am, mg = em.posterior()
    wg, am, mg = wg.cpu().numpy().astype(np.float64), am.cpu().numpy(), mg.cpu().numpy()
    wo, _, _ = oracle.estep(V, a_t, rho_t, s2, w.kbar, w.L, offs)
    ao, mo = oracle.argmax_margin(wo)
    assert np.abs(wg - wo).max() <= TOL["post"]
    assert np.linalg.norm(wg - wo) / np.linalg.norm(wo) <= TOL["post"]
    sure = mo > 1e-3
    assert int(np.sum(am[sure] != ao[sure])) == 0
    assert np.abs(mg - mo).max() <= 2 * TOL["post"] + 1e-6
    ll_ref = oracle.loglik(V, a_t, rho_t, s2, w.kbar, w.L, offs)
    ll_bar = max(TOL["ll"] * abs(ll_ref),
                 loglik_bar(V, a_t, s2, w.kbar, w.L, offs, U32) + 1e-12 * abs(ll_ref))
    assert abs(em.loglik() - ll_ref) <= ll_bar
    em.step(1)
    it = oracle.em_iteration(V, a_t, rho_t, s2, w.kbar, w.L, offs, rho_bar=rb, gamma=gamma)
    a1, rho1, _ = em.state()
    a_bar = max(TOL["a"], 3 * 2.0 ** -24 / np.sqrt(3 * V.shape[0]))
    assert np.linalg.norm(a1 - it["a"]) / np.linalg.norm(it["a"]) <= a_bar
    assert np.abs(rho1 - it["rho"]).max() <= a_bar
    st = em.stats()[-1]
    assert abs(st[1] - ll_ref) <= ll_bar
    assert abs(st[2] - it["J"]) <= ll_bar + 1e-12 * abs(it["J"])
    kernel = em.info()["kernel"]
    em.close()
    return kernel


@pytest.mark.parametrize("K,Q,L,h", [(32, 16, 360, None), (32, 16, 384, None), (16, 32, 360, None),
                                      (8, 64, 200, None), (32, 8, 360, None), (32, 16, 360, 24),
                                      (32, 16, 720, 60), (8, 16, 64, 3)])
def test_gemm_pass_shapes(gpu, K, Q, L, h):
    w, a_true, V, s2, lo, W, rb = _problem(9001, K, Q, L, h)
    print(f"gemm pass K={K} Q={Q} L={L} W={W}", flush=True)
    kernel = _check(gpu, w, a_true, V, s2, lo, W, rb, 0.0 if h is None else 30.0,
                    np.random.default_rng(K + Q + L))
    assert kernel == f"pass_gm_kernel<f32,BM=128,NTC={(W + 15) // 16}>", kernel


@pytest.mark.parametrize("N", [1, 127, 128, 129, 32768 + 77])
def test_gemm_pass_row_counts(gpu, N):
    """Row counts around the 128-row tile; the largest gives every workgroup one or two tiles."""
    w, a_true, V, s2, lo, W, rb = _problem(N, 32, 16, 360, seed=1)
    print(f"gemm pass N={N}", flush=True)
    kernel = _check(gpu, w, a_true, V, s2, lo, W, rb, 0.0, np.random.default_rng(N))
    assert kernel.startswith("pass_gm_kernel"), kernel


def test_gemm_pass_matches_general_pass(gpu):
    """The GEMM-epilogue pass and the general pass on the same FP32 inputs: 5 free-running
    iterations each against the oracle's (full search, L = 360)."""
    import torch
    from paper_2105_07372_amd import EM
    w, a_true, V, s2, lo, W, rb = _problem(12001, 32, 16, 360, seed=2)
    a0 = wl.random_init(w, 0)
    a_o, rho_o, _ = oracle.em_run(V, a0, rb, s2, w.kbar, w.L, oracle.offsets(lo, W), 5)
    obs = torch.from_numpy(V.astype(np.complex64)).to(gpu)
    for general in (False, True):
        em = EM(obs, K=w.K, Q=w.Q, L=w.L, sigma2=s2, precision="fp32", a0=a0,
                general_pass=general)
        assert em.info()["kernel"].startswith("pass_kernel" if general else "pass_gm_kernel")
        em.step(5)
        a_g, rho_g, t = em.state()
        assert t == 5
        assert np.linalg.norm(a_g - a_o) / np.linalg.norm(a_o) <= 1e-4, general
        assert np.abs(rho_g - rho_o).max() <= 1e-4, general
        ll = em.stats()[:, 1]
        assert np.all(np.diff(ll) >= -1e-7 * np.abs(ll[1:]))
        em.close()


def test_gemm_pass_adjoint(gpu):
    """em_loglik_fwd (stores the per-row log-sum-exp) and em_loglik_bwd (reloads it) through the
    GEMM-epilogue pass: gradients against the oracle's Fisher-identity gradients."""
    import torch
    from paper_2105_07372_amd import EM
    w, a_true, V, s2, lo, W, rb = _problem(5003, 32, 16, 360, h=40, seed=3)
    em = EM(torch.from_numpy(V.astype(np.complex64)).to(gpu), K=w.K, Q=w.Q, L=w.L, sigma2=s2,
            window=(lo, W), prior=rb, precision="fp32")
    assert em.info()["kernel"].startswith("pass_gm_kernel")
    rng = np.random.default_rng(9)
    a = V.mean(axis=0) + 0.2 * a_true
    eta = np.log(rb) + 0.1 * rng.standard_normal(W)
    a_d = torch.from_numpy(a).to(gpu)
    e_d = torch.from_numpy(eta).to(gpu)
    ll = em.loglik_fwd(a_d, s2 * 1.05, e_d)
    ga = torch.empty_like(a_d)
    ge = torch.empty_like(e_d)
    gs = em.loglik_bwd(1.0, ga, ge)
    r = np.exp(eta - eta.max())
    r /= r.sum()
    ll_o, ga_o, gs_o, ge_o = oracle.grad_loglik(V, a, s2 * 1.05, r, w.kbar, w.L,
                                                oracle.offsets(lo, W))
    assert abs(ll - ll_o) <= 1e-7 * abs(ll_o)
    assert np.linalg.norm(ga.cpu().numpy() - ga_o) <= 2e-4 * np.linalg.norm(ga_o)
    assert abs(gs - gs_o) <= 2e-4 * abs(gs_o)
    assert np.abs(ge.cpu().numpy() - ge_o).max() <= 2e-4 * max(1.0, np.abs(ge_o).max())
    em.close()
