"""The factored E(+M) pass (correlations through the per-frequency sums c_jk, an exact rewrite of
the contraction; no template) against the FP64 oracle: teacher-forced steps on windowed and
full-search shapes with one to 32 lanes per angular frequency and ragged row tails, every
precision it supports; the large-image shape (D = 2048, 32 entries per lane, fp16 and bf16),
including its full size; a windowed trajectory; the posterior queries and the adjoint."""
import numpy as np
import pytest

import oracle
import workloads as wl

pytestmark = pytest.mark.gpu

TOL = {"fp32": dict(post=2e-4, a=2e-5, ll=1e-7), "bf16x3": dict(post=1e-3, a=1e-4, ll=1e-6),
       "fp16": dict(post=1e-3, a=2e-4, ll=1e-6), "bf16": dict(post=5e-3, a=1e-3, ll=1e-5)}

SHAPES = {
    # name: (K, Q, L, half window (None: full search), N)
    "win16": (32, 16, 360, 24, 4099),      # the windowed workload's shape: W = 49
    "win8": (64, 8, 72, 6, 1001),          # one lane per frequency, W = 13
    "win32": (16, 32, 360, 40, 777),       # four lanes per frequency, W = 81 (L2 path)
    "win128": (4, 128, 72, 6, 1001),       # 16 lanes per frequency: every DPP step of the sum
    "win256": (2, 256, 72, 6, 517),        # 32 lanes per frequency: DPP steps and a shuffle
    "full": (32, 16, 60, None, 2050),      # full search, W = 60
    # windows symmetric about 0 past 64 offsets: EM and log-likelihood passes take the
    # symmetric-window kernel (posterior queries the plain one)
    "full360": (32, 16, 360, None, 3001),  # full search, 181 half-window offsets: 12 tiles
    "fullodd": (32, 16, 75, None, 1001),   # odd L: no offset at L / 2
    "win64": (8, 64, 360, 60, 517),        # W = 121, eight lanes per frequency, 2K = 16
}
FS_SHAPES = {"win32", "full360", "fullodd", "win64"}


def _problem(shape, seed=0):
    K, Q, L, h, N = SHAPES[shape]
    base = wl.WORKLOADS["c3"] if h is not None else wl.WORKLOADS["c2"]
    w = base.replace(K=K, Q=Q, L=L, N=N, **({"half_window": h} if h is not None else {}))
    a_true = wl.image(w, seed)
    V = wl.observations(w, seed, a=a_true)
    s2 = wl.noise_variance(a_true, w.snr)
    lo, W = w.window
    if h is None:
        rb = np.full(W, 1.0 / W)
    else:
        rb, _, _ = oracle.histogram_prior(wl.prior_error_draws(w, seed, 200_000), w.L, lo, W)
    return w, a_true, V, s2, lo, W, rb


@pytest.mark.parametrize("prec", ["fp32", "bf16x3", "fp16", "bf16"])
@pytest.mark.parametrize("shape", list(SHAPES))
def test_factored_teacher_forced_step(gpu, prec, shape):
    import torch
    from paper_2105_07372_amd import EM
    w, a_true, V, s2, lo, W, rb = _problem(shape)
    rng = np.random.default_rng(2)
    a_t = V.mean(axis=0) + 0.1 * a_true * rng.standard_normal(w.D)
    rho_t = rb * rng.uniform(0.5, 1.5, W)
    rho_t /= rho_t.sum()
    gamma = 0.0 if shape == "full" else 50.0
    print(f"factored shape={shape} prec={prec} N={w.N} W={W}", flush=True)
    em = EM(torch.from_numpy(V.astype(np.complex64)).to(gpu), K=w.K, Q=w.Q, L=w.L, sigma2=s2,
            window=(lo, W), prior=rb, gamma=gamma, precision=prec, factored=True)
    want = "pass_fs_kernel" if shape in FS_SHAPES else "pass_fac_kernel"
    assert em.info()["kernel"].startswith(want), em.info()
    em.set_state(a_t, rho_t, 0)
    offs = oracle.offsets(lo, W)
    wg, am, mg = em.posterior()
    wo, _, _ = oracle.estep(V, a_t, rho_t, s2, w.kbar, w.L, offs)
    ao, mo = oracle.argmax_margin(wo)
    wg, am, mg = wg.cpu().numpy().astype(np.float64), am.cpu().numpy(), mg.cpu().numpy()
    assert np.abs(wg - wo).max() <= TOL[prec]["post"]
    assert np.linalg.norm(wg - wo) / np.linalg.norm(wo) <= TOL[prec]["post"]
    # argmax bit-exact where the margin exceeds the posterior error bar (single-plane bf16:
    # twice its 5e-3 bar)
    sure = mo > (1e-2 if prec == "bf16" else 1e-3)
    assert int(np.sum(am[sure] != ao[sure])) == 0
    ll_ref = oracle.loglik(V, a_t, rho_t, s2, w.kbar, w.L, offs)
    assert abs(em.loglik() - ll_ref) <= TOL[prec]["ll"] * abs(ll_ref)
    done, ll_step = em.step(1)
    assert done == 1 and abs(ll_step - ll_ref) <= TOL[prec]["ll"] * abs(ll_ref)
    it = oracle.em_iteration(V, a_t, rho_t, s2, w.kbar, w.L, offs, rho_bar=rb, gamma=gamma)
    a1, rho1, _ = em.state()
    assert np.linalg.norm(a1 - it["a"]) / np.linalg.norm(it["a"]) <= TOL[prec]["a"]
    assert np.abs(rho1 - it["rho"]).max() <= TOL[prec]["a"]
    em.close()


@pytest.mark.parametrize("prec", ["fp32", "fp16"])
@pytest.mark.parametrize("case", ["full_lo_neg", "full_lo_pos", "zero_bins", "gamma0"])
def test_symmetric_window_pass(gpu, prec, case):
    """The symmetric-window factored kernel on the cases its index maps must get right: a full
    search that starts at another offset (the window index of +m and -m wraps), a learned prior
    with empty bins at +m only, at -m only and at 0, and gamma = 0.  Log-likelihood and one step
    against the oracle; three more steps against the oracle's trajectory."""
    import torch
    from paper_2105_07372_amd import EM
    L = 120
    w = wl.WORKLOADS["c3"].replace(N=2001, K=32, Q=16, L=L, half_window=45)
    a_true = wl.image(w, 3)
    V = wl.observations(w, 3, a=a_true)
    s2 = wl.noise_variance(a_true, w.snr)
    if case == "full_lo_neg":
        lo, W = -L // 2, L
    elif case == "full_lo_pos":
        lo, W = 7, L
    else:
        lo, W = w.window
    if W == L:
        rb = np.full(W, 1.0 / W)
        gamma = 0.0
    else:
        rb, _, _ = oracle.histogram_prior(wl.prior_error_draws(w, 3, 200_000), L, lo, W)
        gamma = 0.0 if case == "gamma0" else 30.0
    if case == "zero_bins":
        h = -lo
        rb[[h + 3, h - 7, h, 0, W - 1]] = 0.0        # +3, -7, 0 and both window edges
        rb /= rb.sum()
    print(f"symmetric window {case} {prec} lo={lo} W={W}", flush=True)
    em = EM(torch.from_numpy(V.astype(np.complex64)).to(gpu), K=w.K, Q=w.Q, L=L, sigma2=s2,
            window=(lo, W), prior=rb, gamma=gamma, precision=prec, factored=True)
    assert em.info()["kernel"].startswith("pass_fs_kernel"), em.info()
    offs = oracle.offsets(lo, W)
    a0 = V.astype(np.complex64).astype(np.complex128).mean(axis=0)
    ll_ref = oracle.loglik(V, a0, rb, s2, w.kbar, L, offs)
    assert abs(em.loglik() - ll_ref) <= TOL[prec]["ll"] * abs(ll_ref)
    a_o, rho_o = a0, rb
    for t in range(4):
        ref = oracle.em_iteration(V, a_o, rho_o, s2, w.kbar, L, offs, rho_bar=rb, gamma=gamma)
        em.step(1)
        a, rho, _ = em.state()
        assert np.linalg.norm(a - ref["a"]) / np.linalg.norm(ref["a"]) <= 3 * TOL[prec]["a"], t
        assert np.abs(rho - ref["rho"]).max() <= 3 * TOL[prec]["a"], t
        assert abs(em.stats()[-1, 1] - ref["ll"]) <= TOL[prec]["ll"] * abs(ref["ll"]), t
        if case == "zero_bins":
            assert np.all(rho[rb == 0.0] == 0.0)
        a_o, rho_o = ref["a"], ref["rho"]
    em.close()


def test_factored_windowed_trajectory(gpu):
    """The windowed workload's shape at N = 20000, fp16, 4 iterations from the mean."""
    import torch
    from paper_2105_07372_amd import EM
    w = wl.WORKLOADS["c3"].replace(N=20000)
    a_true = wl.image(w, 1)
    V = wl.observations(w, 1, a=a_true)
    s2 = wl.noise_variance(a_true, w.snr)
    lo, W = w.window
    rb, _, _ = oracle.histogram_prior(wl.prior_error_draws(w, 1), w.L, lo, W)
    a0 = V.astype(np.complex64).astype(np.complex128).mean(axis=0)
    em = EM(torch.from_numpy(V.astype(np.complex64)).to(gpu), K=w.K, Q=w.Q, L=w.L, sigma2=s2,
            window=(lo, W), prior=rb, gamma=w.gamma, precision="fp16", a0=a0, factored=True)
    offs = oracle.offsets(lo, W)
    a_o, rho_o = a0, rb
    for t in range(4):
        ref = oracle.em_iteration(V, a_o, rho_o, s2, w.kbar, w.L, offs, rho_bar=rb, gamma=w.gamma)
        em.step(1)
        a, rho, _ = em.state()
        assert np.linalg.norm(a - ref["a"]) / np.linalg.norm(ref["a"]) <= 3e-4, t
        assert np.abs(rho - ref["rho"]).max() <= 3e-4, t
        a_o, rho_o = ref["a"], ref["rho"]
    em.close()


def test_factored_adjoint(gpu):
    import torch
    from paper_2105_07372_amd import EM
    w, a_true, V, s2, lo, W, rb = _problem("win16")
    rng = np.random.default_rng(4)
    a = V.mean(axis=0) + 0.2 * a_true
    eta = np.log(rb + 1e-3) + 0.1 * rng.standard_normal(W)
    em = EM(torch.from_numpy(V.astype(np.complex64)).to(gpu), K=w.K, Q=w.Q, L=w.L, sigma2=s2,
            window=(lo, W), prior=rb, precision="fp32", factored=True)
    a_d = torch.from_numpy(a).to(gpu)
    e_d = torch.from_numpy(eta).to(gpu)
    ll = em.loglik_fwd(a_d, s2 * 1.1, e_d)
    ga = torch.empty_like(a_d)
    ge = torch.empty_like(e_d)
    gs = em.loglik_bwd(1.0, ga, ge)
    r = np.exp(eta - eta.max())
    r /= r.sum()
    ll_o, ga_o, gs_o, ge_o = oracle.grad_loglik(V, a, s2 * 1.1, r, w.kbar, w.L,
                                                oracle.offsets(lo, W))
    assert abs(ll - ll_o) <= 1e-7 * abs(ll_o)
    assert np.linalg.norm(ga.cpu().numpy() - ga_o) <= 2e-4 * np.linalg.norm(ga_o)
    assert abs(gs - gs_o) <= 2e-4 * abs(gs_o)
    assert np.abs(ge.cpu().numpy() - ge_o).max() <= 2e-4 * max(1.0, np.abs(ge_o).max())
    em.close()


def test_factored_rejects_unsupported_shapes(gpu):
    import torch
    from paper_2105_07372_amd import EM, SynchemError
    V = np.zeros((10, 8 * 6), np.complex64)
    with pytest.raises(SynchemError) as ei:
        EM(torch.from_numpy(V).to(gpu), K=8, Q=6, L=12, sigma2=1.0, precision="fp32",
           factored=True)
    assert ei.value.status == -6


SHAPES2048 = {
    # name: (K, Q, L, half window, N): 16 entries per lane (rows over wave pairs), D = 2048
    "c5": (64, 32, 720, 90, 3001),         # the large-image shape, W = 181
    "c5narrow": (64, 32, 720, 45, 1001),   # W = 91
    "q64": (32, 64, 360, 24, 777),         # two lanes per frequency, 2K = 64, W = 49
}


@pytest.mark.parametrize("prec", ["fp16", "bf16"])
@pytest.mark.parametrize("shape", list(SHAPES2048))
def test_factored_2048_teacher_forced_step(gpu, prec, shape):
    import torch
    from paper_2105_07372_amd import EM
    K, Q, L, h, N = SHAPES2048[shape]
    w = wl.WORKLOADS["c5"].replace(K=K, Q=Q, L=L, N=N, half_window=h)
    a_true = wl.image(w, 0)
    V = wl.observations(w, 0, a=a_true)
    s2 = wl.noise_variance(a_true, w.snr)
    lo, W = w.window
    rb, _, _ = oracle.histogram_prior(wl.prior_error_draws(w, 0, 200_000), w.L, lo, W)
    rng = np.random.default_rng(6)
    a_t = V.mean(axis=0) + 0.1 * a_true * rng.standard_normal(w.D)
    rho_t = rb * rng.uniform(0.5, 1.5, W)
    rho_t /= rho_t.sum()
    print(f"factored D=2048 shape={shape} prec={prec} N={N} W={W}", flush=True)
    em = EM(torch.from_numpy(V.astype(np.complex64)).to(gpu), K=K, Q=Q, L=L, sigma2=s2,
            window=(lo, W), prior=rb, gamma=50.0, precision=prec, factored=True)
    # windows past 64 offsets (symmetric about 0) take the paired-offset kernel for EM steps
    want = "pass_fs_kernel" if W > 64 else "pass_fac_kernel"
    assert em.info()["kernel"].startswith(want) and "E16" in em.info()["kernel"], em.info()
    em.set_state(a_t, rho_t, 0)
    offs = oracle.offsets(lo, W)
    wg, am, mg = em.posterior()
    wo, _, _ = oracle.estep(V, a_t, rho_t, s2, w.kbar, L, offs)
    ao, mo = oracle.argmax_margin(wo)
    wg, am = wg.cpu().numpy().astype(np.float64), am.cpu().numpy()
    assert np.abs(wg - wo).max() <= TOL[prec]["post"]
    assert np.linalg.norm(wg - wo) / np.linalg.norm(wo) <= TOL[prec]["post"]
    sure = mo > (1e-2 if prec == "bf16" else 1e-3)
    assert int(np.sum(am[sure] != ao[sure])) == 0
    ll_ref = oracle.loglik(V, a_t, rho_t, s2, w.kbar, L, offs)
    assert abs(em.loglik() - ll_ref) <= TOL[prec]["ll"] * abs(ll_ref)
    em.step(1)
    it = oracle.em_iteration(V, a_t, rho_t, s2, w.kbar, L, offs, rho_bar=rb, gamma=50.0)
    a1, rho1, _ = em.state()
    assert np.linalg.norm(a1 - it["a"]) / np.linalg.norm(it["a"]) <= TOL[prec]["a"]
    assert np.abs(rho1 - it["rho"]).max() <= TOL[prec]["a"]
    em.close()


@pytest.mark.timeout(900)
def test_factored_2048_full_size(gpu):
    """N = 10^6, D = 2048, L = 720, W = 181, fp16, factored: sampled rows' posteriors against the
    oracle, one EM step against the oracle's iteration from the same state streamed over all rows
    (tests/oracle_stream.py), and the pass time."""
    import torch
    from paper_2105_07372_amd import EM
    from oracle_stream import large_image_state, upload_and_iterate
    w = wl.WORKLOADS["c5"]
    lo, W = w.window
    a_true, s2, rb, a_t = large_image_state(w, 0)
    obs = torch.empty((w.N, w.D), dtype=torch.complex64, device=gpu)
    ref = upload_and_iterate(w, 0, obs, a_true, a_t, rb, s2, rb, w.gamma)
    print("factored full size: generated, oracle iteration streamed", flush=True)
    em = EM(obs, K=w.K, Q=w.Q, L=w.L, sigma2=s2, window=(lo, W), prior=rb, gamma=w.gamma,
            precision="fp16", timing=True, factored=True)
    assert "E16" in em.info()["kernel"], em.info()
    em.set_state(a_t, rb, 0)
    offs = oracle.offsets(lo, W)
    for (r0, n) in ((0, 512), (w.N - 512, 512)):
        Vs = wl.observations(w, 0, r0, r0 + n, dtype=np.complex64, a=a_true).astype(np.complex128)
        wg, am, _ = em.posterior(r0, n)
        wo, _, _ = oracle.estep(Vs, a_t, rb, s2, w.kbar, w.L, offs)
        assert np.abs(wg.cpu().numpy().astype(np.float64) - wo).max() <= TOL["fp16"]["post"]
    em.step(1)
    a1, rho1, _ = em.state()
    assert np.linalg.norm(a1 - ref["a"]) / np.linalg.norm(ref["a"]) <= 2e-4
    assert np.abs(rho1 - ref["rho"]).max() <= 2e-4 * ref["rho"].max()
    assert abs(em.stats()[-1, 1] - ref["ll"]) <= 1e-6 * abs(ref["ll"])
    em.pass_time(reset=True)
    em.step(3)
    ms, n = em.pass_time(reset=True)
    print(f"factored full size: {em.info()['kernel']} {1e3 * ms / n:.1f} us per pass", flush=True)
    em.close()
