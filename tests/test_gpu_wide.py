"""The wide-row E(+M) pass (rows streamed through an LDS ring; chosen for D = 2048 in fp16/bf16)
against the FP64 oracle: forced on small edge shapes (odd k-step counts, window tile counts that
are not a multiple of four, ragged row tails), on the large-image shape (D = 2048, L = 720, W =
181 and 91) at a size the oracle runs whole, and at full size (N = 10^6) on sampled rows plus the
M-step's consistency with the kernel's own posteriors."""
import numpy as np
import pytest

import oracle
import workloads as wl

pytestmark = pytest.mark.gpu

TOL = {"fp16": dict(post=1e-3, a=2e-4, ll=1e-6), "bf16": dict(post=5e-3, a=1e-3, ll=1e-5)}


def _problem(w, seed=0):
    a_true = wl.image(w, seed)
    V = wl.observations(w, seed, a=a_true)
    s2 = wl.noise_variance(a_true, w.snr)
    lo, W = w.window
    rb, _, _ = oracle.histogram_prior(wl.prior_error_draws(w, seed, 300_000), w.L, lo, W)
    return a_true, V, s2, lo, W, rb


def _post_check(em, V, a, rho, s2, w, lo, W, prec, row0=0):
    """Posterior queries of rows row0 .. row0 + len(V) (V holds exactly those rows)."""
    wg, am, mg = em.posterior(row0, V.shape[0])
    wg, am, mg = wg.cpu().numpy().astype(np.float64), am.cpu().numpy(), mg.cpu().numpy()
    wo, _, _ = oracle.estep(V, a, rho, s2, w.kbar, w.L, oracle.offsets(lo, W))
    ao, mo = oracle.argmax_margin(wo)
    assert np.abs(wg - wo).max() <= TOL[prec]["post"]
    assert np.linalg.norm(wg - wo) / np.linalg.norm(wo) <= TOL[prec]["post"]
    sure = mo > 1e-3
    assert int(np.sum(am[sure] != ao[sure])) == 0
    assert np.abs(mg - mo).max() <= 2 * TOL[prec]["post"] + 1e-6
    return wg


SHAPES = {
    # name: (K, Q, L, half window (None: full search), N)
    "tiny": (8, 8, 72, 6, 1001),          # one slot per K-half, one window tile per wave group
    "oddks": (5, 40, 360, 45, 3001),      # 2D = 400 reals: 13 k-steps (odd), W = 91: 6 tiles
    "full": (6, 7, 40, None, 517),        # full search, W = 40 -> 3 tiles, one ragged tile
    "big": (64, 32, 720, 90, 6000),       # the large-image shape, W = 181
}


@pytest.mark.parametrize("prec", ["fp16", "bf16"])
@pytest.mark.parametrize("shape", list(SHAPES))
def test_wide_teacher_forced_step(gpu, prec, shape):
    import torch
    from paper_2105_07372_amd import EM
    K, Q, L, h, N = SHAPES[shape]
    base = wl.WORKLOADS["c5"] if h is not None else wl.WORKLOADS["c2"]
    w = base.replace(K=K, Q=Q, L=L, N=N, **({"half_window": h} if h is not None else {}))
    a_true, V, s2, lo, W, rb = _problem(w)
    if h is None:
        rb = np.full(W, 1.0 / W)
    rng = np.random.default_rng(3)
    a_t = V.mean(axis=0) + 0.1 * a_true * rng.standard_normal(w.D)
    rho_t = rb * rng.uniform(0.5, 1.5, W)
    rho_t /= rho_t.sum()
    gamma = 0.0 if h is None else 50.0
    print(f"wide shape={shape} prec={prec} N={N} D={w.D} L={L} W={W}", flush=True)
    em = EM(torch.from_numpy(V.astype(np.complex64)).to(gpu), K=K, Q=Q, L=L, sigma2=s2,
            window=(lo, W), prior=rb, gamma=gamma, precision=prec, wide_pass=True)
    assert em.info()["kernel"].startswith("pass_wide_kernel"), em.info()
    em.set_state(a_t, rho_t, 0)
    _post_check(em, V, a_t, rho_t, s2, w, lo, W, prec)
    offs = oracle.offsets(lo, W)
    ll_ref = oracle.loglik(V, a_t, rho_t, s2, w.kbar, L, offs)
    assert abs(em.loglik() - ll_ref) <= TOL[prec]["ll"] * abs(ll_ref)
    done, ll_step = em.step(1)
    assert done == 1 and abs(ll_step - ll_ref) <= TOL[prec]["ll"] * abs(ll_ref)
    it = oracle.em_iteration(V, a_t, rho_t, s2, w.kbar, L, offs, rho_bar=rb, gamma=gamma)
    a1, rho1, _ = em.state()
    assert np.linalg.norm(a1 - it["a"]) / np.linalg.norm(it["a"]) <= TOL[prec]["a"]
    assert np.abs(rho1 - it["rho"]).max() <= TOL[prec]["a"]
    em.close()


@pytest.mark.parametrize("half_window", [90, 45])
def test_large_image_trajectory(gpu, half_window):
    """D = 2048 (K = 64, Q = 32), L = 720, learned prior with gamma = 100, fp16: the library picks
    the wide-row pass by itself; three EM iterations from the mean against the oracle's."""
    import torch
    from paper_2105_07372_amd import EM
    w = wl.WORKLOADS["c5"].replace(N=20000, half_window=half_window)
    a_true, V, s2, lo, W, rb = _problem(w)
    a0 = V.astype(np.complex64).astype(np.complex128).mean(axis=0)
    print(f"large image W={W} N={w.N}", flush=True)
    em = EM(torch.from_numpy(V.astype(np.complex64)).to(gpu), K=w.K, Q=w.Q, L=w.L, sigma2=s2,
            window=(lo, W), prior=rb, gamma=w.gamma, precision="fp16", a0=a0)
    assert em.info()["kernel"].startswith("pass_wide_kernel"), em.info()
    offs = oracle.offsets(lo, W)
    a_o, rho_o = a0, rb
    for t in range(3):
        ref = oracle.em_iteration(V, a_o, rho_o, s2, w.kbar, w.L, offs, rho_bar=rb, gamma=w.gamma)
        em.step(1)
        a, rho, _ = em.state()
        assert np.linalg.norm(a - ref["a"]) / np.linalg.norm(ref["a"]) <= 3e-4, t
        assert np.abs(rho - ref["rho"]).max() <= 3e-4, t
        assert abs(em.stats()[-1, 1] - ref["ll"]) <= 1e-6 * abs(ref["ll"]), t
        a_o, rho_o = ref["a"], ref["rho"]
    em.close()


def test_large_image_adjoint(gpu):
    """The differentiable log-likelihood on the large-image shape (fp16 correlations, FP64
    reductions): value and gradients against the oracle's Fisher-identity gradients."""
    import torch
    from paper_2105_07372_amd import EM
    w = wl.WORKLOADS["c5"].replace(N=8000)
    a_true, V, s2, lo, W, rb = _problem(w)
    rng = np.random.default_rng(5)
    a = V.mean(axis=0) + 0.2 * a_true
    eta = np.log(rb + 1e-3) + 0.1 * rng.standard_normal(W)
    em = EM(torch.from_numpy(V.astype(np.complex64)).to(gpu), K=w.K, Q=w.Q, L=w.L, sigma2=s2,
            window=(lo, W), prior=rb, precision="fp16")
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
    assert abs(ll - ll_o) <= 1e-6 * abs(ll_o)
    assert np.linalg.norm(ga.cpu().numpy() - ga_o) <= 2e-3 * np.linalg.norm(ga_o)
    assert abs(gs - gs_o) <= 2e-3 * abs(gs_o)
    assert np.abs(ge.cpu().numpy() - ge_o).max() <= 2e-3 * max(1.0, np.abs(ge_o).max())
    em.close()


@pytest.mark.timeout(900)
def test_large_image_full_size(gpu):
    """N = 10^6, D = 2048, L = 720, W = 181, fp16, in the launch configuration the library picks:
    posteriors, argmax and margins of 1024 sampled rows (first and last generator chunks) against
    the oracle at a state set by the test; then one EM step, whose estimate, distribution and
    log-likelihood must equal the oracle's iteration from the same state, streamed over all rows
    (tests/oracle_stream.py)."""
    import torch
    from paper_2105_07372_amd import EM
    from oracle_stream import large_image_state, upload_and_iterate
    w = wl.WORKLOADS["c5"]
    lo, W = w.window
    a_true, s2, rb, a_t = large_image_state(w, 0)
    rho_t = rb
    obs = torch.empty((w.N, w.D), dtype=torch.complex64, device=gpu)
    ref = upload_and_iterate(w, 0, obs, a_true, a_t, rho_t, s2, rb, w.gamma)
    print("large image full size: generated, oracle iteration streamed", flush=True)
    em = EM(obs, K=w.K, Q=w.Q, L=w.L, sigma2=s2, window=(lo, W), prior=rb, gamma=w.gamma,
            precision="fp16", timing=True)
    assert em.info()["kernel"].startswith("pass_wide_kernel"), em.info()
    em.set_state(a_t, rho_t, 0)
    for (r0, n) in ((0, 512), (w.N - 512, 512)):
        Vs = wl.observations(w, 0, r0, r0 + n, dtype=np.complex64, a=a_true)
        Vs = Vs.astype(np.complex128)
        _post_check(em, Vs, a_t, rho_t, s2, w, lo, W, "fp16", row0=r0)
    print("large image full size: sampled rows ok", flush=True)
    em.step(1)
    a1, rho1, _ = em.state()
    assert np.linalg.norm(a1 - ref["a"]) / np.linalg.norm(ref["a"]) <= 2e-4
    assert np.abs(rho1 - ref["rho"]).max() <= 2e-4 * ref["rho"].max()
    assert abs(em.stats()[-1, 1] - ref["ll"]) <= 1e-6 * abs(ref["ll"])
    em.pass_time(reset=True)
    em.step(3)
    ms, n = em.pass_time(reset=True)
    print(f"large image full size: {em.info()['kernel']} {1e3 * ms / n:.1f} us per pass", flush=True)
    em.close()
