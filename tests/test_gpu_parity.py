"""GPU (HIP, through the C ABI) against the FP64 oracle on the same seeded inputs.

Tolerances: FP64 path 1e-10 relative (posterior queries return float32, so 2e-7 there).  Low-precision paths: posteriors <= 1e-3 in max-abs and in
Frobenius-relative error, estimate and log-likelihood relative error <= 1e-3 (tighter where the
arithmetic allows); rotation argmax bit-exact on every row whose two best posteriors differ by
more than 1e-3.  The single-plane bf16 mode is reported against a looser bar (5e-3): its rounding
of the observations alone exceeds 1e-3 on the posteriors.
"""
import numpy as np
import pytest

import oracle
import workloads as wl

pytestmark = pytest.mark.gpu

TOL = {  # posterior max-abs / frob-rel, estimate rel, loglik rel
    "fp64": dict(post=2e-7, a=1e-10, ll=1e-12),     # posteriors are returned as float32
    "fp32": dict(post=2e-4, a=2e-5, ll=1e-7),
    "bf16x3": dict(post=1e-3, a=1e-4, ll=1e-6),
    "fp16": dict(post=1e-3, a=2e-4, ll=1e-6),
    "bf16": dict(post=5e-3, a=1e-3, ll=1e-5),
}


def _obs(V, prec, dev):
    import torch
    return torch.from_numpy(V.astype(np.complex128 if prec == "fp64" else np.complex64)).to(dev)


def _case(name, seed=0):
    """Small cases that span many tiles (and several tiles per workgroup) with a ragged tail."""
    if name == "window":
        w = wl.WORKLOADS["c3"].replace(N=20037, K=8, Q=8, L=72, rot_std_deg=10.0, half_window=6)
        gamma = 50.0
    elif name == "full":
        w = wl.WORKLOADS["c2"].replace(N=9001, K=8, Q=6, L=40)
        gamma = 0.0
    elif name == "odd":
        w = wl.WORKLOADS["c3"].replace(N=997, K=3, Q=5, L=10, rot_std_deg=40.0, half_window=2)
        gamma = 5.0
    elif name == "wide":
        w = wl.WORKLOADS["c3"].replace(N=4099, K=32, Q=16, L=360, half_window=24)
        gamma = 100.0
    elif name == "kodd":
        # D = 507 (Q = 13 odd, D not a multiple of 4) and W = 41: the K-split pass with three
        # column tiles and entries of one M-step lane spanning two frequencies
        w = wl.WORKLOADS["c3"].replace(N=3001, K=39, Q=13, L=180, half_window=20)
        gamma = 20.0
    else:
        raise KeyError(name)
    a_true = wl.image(w, seed)
    V = wl.observations(w, seed, a=a_true)
    s2 = wl.noise_variance(a_true, w.snr)
    lo, W = w.window
    if w.rot_law == "gauss":
        rb, _, _ = oracle.histogram_prior(wl.prior_error_draws(w, seed, 200_000), w.L, lo, W)
    else:
        rb = np.full(W, 1.0 / W)
    return w, a_true, V, s2, lo, W, rb, gamma


def _compare_posteriors(em, V, a, rho, s2, w, lo, W, prec, row0=0, nrows=None):
    nrows = V.shape[0] - row0 if nrows is None else nrows
    wg, am, mg = em.posterior(row0, nrows)
    wg, am, mg = wg.cpu().numpy().astype(np.float64), am.cpu().numpy(), mg.cpu().numpy()
    wo, _, _ = oracle.estep(V[row0:row0 + nrows], a, rho, s2, w.kbar, w.L, oracle.offsets(lo, W))
    ao, mo = oracle.argmax_margin(wo)
    maxabs = np.abs(wg - wo).max()
    frob = np.linalg.norm(wg - wo) / np.linalg.norm(wo)
    sure = mo > 1e-3
    mism = int(np.sum(am[sure] != ao[sure]))
    assert maxabs <= TOL[prec]["post"], (prec, maxabs)
    assert frob <= TOL[prec]["post"], (prec, frob)
    assert mism == 0, (prec, mism)
    assert np.abs(mg - mo).max() <= 2 * TOL[prec]["post"] + 1e-6
    return maxabs, frob


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3", "fp16", "bf16"])
@pytest.mark.parametrize("case", ["window", "full", "odd", "wide", "kodd"])
def test_teacher_forced_step(gpu, prec, case):
    from paper_2105_07372_amd import EM
    w, a_true, V, s2, lo, W, rb, gamma = _case(case)
    gai = 1.0 / (4 * np.exp(-w.kbar / 8.0)) ** 2 if case == "odd" else None
    rng = np.random.default_rng(1)
    a_t = V.mean(axis=0) + 0.1 * a_true * rng.standard_normal(w.D)
    rho_t = rb * rng.uniform(0.5, 1.5, W)
    rho_t /= rho_t.sum()
    print(f"case={case} prec={prec} N={w.N} D={w.D} L={w.L} W={W}", flush=True)
    em = EM(_obs(V, prec, gpu), K=w.K, Q=w.Q, L=w.L, sigma2=s2, window=(lo, W), prior=rb,
            gamma=gamma, precision=prec, gamma_a_inv=gai)
    if case == "kodd" and prec in ("bf16x3", "fp16", "bf16"):
        assert em.info()["kernel"].startswith("pass_ks_kernel"), em.info()
    if case == "wide" and prec in ("bf16x3", "fp16", "bf16"):
        want = "pass_ks_kernel" if prec == "bf16x3" else "pass_kr_kernel"
        assert em.info()["kernel"].startswith(want), em.info()
    em.set_state(a_t, rho_t, 0)
    _compare_posteriors(em, V, a_t, rho_t, s2, w, lo, W, prec)
    ll_ref = oracle.loglik(V, a_t, rho_t, s2, w.kbar, w.L, oracle.offsets(lo, W))
    ll = em.loglik()
    assert abs(ll - ll_ref) <= TOL[prec]["ll"] * abs(ll_ref), (ll, ll_ref)
    done, ll_step = em.step(1)
    assert done == 1 and abs(ll_step - ll_ref) <= TOL[prec]["ll"] * abs(ll_ref)
    it = oracle.em_iteration(V, a_t, rho_t, s2, w.kbar, w.L, oracle.offsets(lo, W), rho_bar=rb,
                             gamma=gamma, gamma_a_inv=gai)
    a1, rho1, t = em.state()
    assert t == 1
    ea = np.linalg.norm(a1 - it["a"]) / np.linalg.norm(it["a"])
    er = np.abs(rho1 - it["rho"]).max()
    assert ea <= TOL[prec]["a"], (prec, ea)
    assert er <= TOL[prec]["a"], (prec, er)
    st = em.stats()
    assert st.shape == (1, 6)
    assert st[0, 0] == 0
    assert abs(st[0, 1] - ll_ref) <= TOL[prec]["ll"] * abs(ll_ref)
    # MAP objective of the starting state (eq. (12) with the priors of eqs. (23)-(24)): the prior
    # terms are exact FP64 functions of (a_t, rho_t), so it carries the log-likelihood's error
    assert abs(st[0, 2] - it["J"]) <= TOL[prec]["ll"] * abs(ll_ref) + 1e-12 * abs(it["J"])
    # ||a_{t+1} - a_t||^2 moves by at most ~2 ||a_{t+1} - a_t|| ||error of a_{t+1}||
    da2 = float(np.sum(np.abs(it["a"] - a_t) ** 2))
    err_a = TOL[prec]["a"] * np.linalg.norm(it["a"])
    assert abs(st[0, 3] - da2) <= 3 * np.sqrt(da2) * err_a + err_a ** 2 + 1e-12 * da2
    # entropy of rho_{t+1}: |dH| <= sum_i |log rho_i + 1| |d rho_i|
    r1 = it["rho"]
    nz = r1 > 0
    ent = -float(np.sum(r1[nz] * np.log(r1[nz])))
    bar = float(np.sum(np.abs(np.log(r1[nz]) + 1))) * TOL[prec]["a"] * 3 + 1e-12
    assert abs(st[0, 5] - ent) <= bar, (st[0, 5], ent)
    # the stopping metric moves by at most ~2 sqrt(metric) ||delta a|| with the estimate's error
    na = np.linalg.norm(a1)
    bar = 3 * np.sqrt(it["stop"]) * TOL[prec]["a"] * na + 1e-12 * na * na
    assert abs(st[0, 4] - it["stop"]) <= bar, (st[0, 4], it["stop"])
    em.close()


def test_fp64_trajectory_plain_em(gpu):
    """Plain EM, FP64, full search over L=64 from a seeded random start, 20 iterations: every
    iterate, every rho and every log-likelihood within 1e-10 of the oracle."""
    from paper_2105_07372_amd import EM
    w = wl.WORKLOADS["c1"]
    a_true = wl.image(w, 0)
    V = wl.observations(w, 0, a=a_true)
    s2 = wl.noise_variance(a_true, w.snr)
    a0 = wl.random_init(w, 0)
    rho0 = np.full(w.L, 1.0 / w.L)
    em = EM(_obs(V, "fp64", gpu), K=w.K, Q=w.Q, L=w.L, sigma2=s2, precision="fp64", a0=a0)
    a, rho = a0.copy(), rho0.copy()
    offs = oracle.offsets(0, w.L)
    for t in range(w.iters):
        it = oracle.em_iteration(V, a, rho, s2, w.kbar, w.L, offs)
        em.step(1)
        ag, rg, tg = em.state()
        assert tg == t + 1
        assert np.linalg.norm(ag - it["a"]) <= 1e-10 * np.linalg.norm(it["a"]), t
        assert np.abs(rg - it["rho"]).max() <= 1e-10 * it["rho"].max(), t
        assert abs(em.stats()[-1, 1] - it["ll"]) <= 1e-10 * abs(it["ll"]), t
        a, rho = it["a"], it["rho"]
    ll = em.stats()[:, 1]
    assert np.all(np.diff(ll) >= -1e-9 * np.abs(ll[1:]))
    em.close()


@pytest.mark.parametrize("prec", ["fp32", "bf16x3", "fp16"])
def test_windowed_trajectory(gpu, prec):
    """Windowed Synch-EM with the learned prior and gamma > 0 for 10 iterations, free-running on
    both sides: the estimate stays within the precision's bar of the oracle's."""
    from paper_2105_07372_amd import EM
    w, a_true, V, s2, lo, W, rb, gamma = _case("window")
    em = EM(_obs(V, prec, gpu), K=w.K, Q=w.Q, L=w.L, sigma2=s2, window=(lo, W), prior=rb,
            gamma=gamma, precision=prec)
    em.step(10)
    a_g, rho_g, t = em.state()
    a_o, rho_o, hist = oracle.em_run(V, V.mean(axis=0), rb, s2, w.kbar, w.L,
                                     oracle.offsets(lo, W), 10, rho_bar=rb, gamma=gamma)
    assert t == 10
    assert np.linalg.norm(a_g - a_o) / np.linalg.norm(a_o) <= 10 * TOL[prec]["a"]
    assert np.abs(rho_g - rho_o).max() <= 10 * TOL[prec]["a"]
    J = em.stats()[:, 2]
    assert np.all(np.diff(J) >= -1e-6 * np.abs(J[1:]))
    em.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp16"])
def test_edge_cases(gpu, prec):
    from paper_2105_07372_amd import EM
    rng = np.random.default_rng(3)
    for (N, K, Q, L, lo, W) in [(1, 4, 4, 12, 0, 12), (17, 2, 3, 8, -1, 1), (33, 1, 7, 6, 0, 6),
                                (50, 5, 2, 1, 0, 1), (129, 6, 6, 20, 17, 9)]:
        D = K * Q
        kbar = np.repeat(np.arange(K), Q)
        a = (rng.standard_normal(D) + 1j * rng.standard_normal(D)) / 2
        V = a[None, :] * np.exp(-2j * np.pi * np.outer(rng.integers(0, L, N), kbar) / L)
        V = V + 0.3 * (rng.standard_normal((N, D)) + 1j * rng.standard_normal((N, D)))
        s2 = 0.18
        rho = rng.uniform(0.5, 1.0, W)
        rho /= rho.sum()
        print(f"edge N={N} K={K} Q={Q} L={L} lo={lo} W={W} prec={prec}", flush=True)
        em = EM(_obs(V, prec, gpu), K=K, Q=Q, L=L, sigma2=s2, window=(lo, W), prior=rho,
                precision=prec)
        wg, am, mg = em.posterior()
        wo, _, _ = oracle.estep(V, V.mean(axis=0), rho, s2, kbar, L, oracle.offsets(lo, W))
        assert np.abs(wg.cpu().numpy() - wo).max() <= TOL[prec]["post"]
        if K == 1:
            assert np.abs(wg.cpu().numpy() - rho[None, :]).max() <= 1e-6
        em.step(2)
        a_o, rho_o, _ = oracle.em_run(V, V.mean(axis=0), rho, s2, kbar, L, oracle.offsets(lo, W), 2)
        a_g, rho_g, _ = em.state()
        assert np.linalg.norm(a_g - a_o) <= 10 * TOL[prec]["a"] * np.linalg.norm(a_o)
        em.close()


def test_determinism_resume_and_stop(gpu):
    from paper_2105_07372_amd import EM
    w, a_true, V, s2, lo, W, rb, gamma = _case("window")
    obs = _obs(V, "bf16x3", gpu)
    kw = dict(K=w.K, Q=w.Q, L=w.L, sigma2=s2, window=(lo, W), prior=rb, gamma=gamma,
              precision="bf16x3")
    e1 = EM(obs, **kw)
    e1.step(6)
    a1, r1, _ = e1.state()
    e2 = EM(obs, **kw)
    e2.step(3)
    a_mid, r_mid, t_mid = e2.state()
    e2.close()
    e3 = EM(obs, **kw)
    e3.set_state(a_mid, r_mid, t_mid)
    e3.step(3)
    a3, r3, t3 = e3.state()
    assert t3 == 6
    assert np.array_equal(a1, a3) and np.array_equal(r1, r3)       # bit-identical
    e4 = EM(obs, **kw)
    e4.step(6)
    assert np.array_equal(e4.state()[0], a1)
    done, _ = e4.step(5, tol=1e30)                                 # stops after one iteration
    assert done == 1
    done, _ = e4.step(5, tol=1e30)
    assert done == 0
    e4.set_state(a1, r1, 0)
    assert e4.step(2)[0] == 2
    for e in (e1, e3, e4):
        e.close()


def test_nonfinite_observations_rejected(gpu):
    import torch
    from paper_2105_07372_amd import EM, SynchemError
    V = np.ones((40, 8), np.complex64)
    V[17, 3] = np.nan
    with pytest.raises(SynchemError) as ei:
        EM(torch.from_numpy(V).to(gpu), K=2, Q=4, L=8, sigma2=1.0)
    assert ei.value.status == -5


@pytest.mark.parametrize("prec,factored", [("bf16x3", False), ("fp16", False), ("fp32", True),
                                           ("fp16", True), ("bf16x3", True)])
def test_full_size_windowed_step(gpu, prec, factored):
    """The windowed workload at full size (N=1e5, D=512, L=360, W=49, gamma=100), with the
    correlation pass and with the factored pass: one EM step from a_0 = mean v, the estimate and
    rho against the oracle on all rows, the posteriors on sampled row blocks."""
    from paper_2105_07372_amd import EM
    w = wl.WORKLOADS["c3"]
    a_true = wl.image(w, 0)
    V = wl.observations(w, 0, a=a_true)
    s2 = wl.noise_variance(a_true, w.snr)
    lo, W = w.window
    rb, _, _ = oracle.histogram_prior(wl.prior_error_draws(w, 0), w.L, lo, W)
    em = EM(_obs(V, prec, gpu), K=w.K, Q=w.Q, L=w.L, sigma2=s2, window=(lo, W), prior=rb,
            gamma=w.gamma, precision=prec, factored=factored)
    a0 = V.astype(np.complex64).astype(np.complex128).mean(axis=0)   # the GPU gets complex64
    a_g0 = em.state()[0]
    assert np.linalg.norm(a_g0 - a0) <= 1e-12 * np.linalg.norm(a0)
    for r0 in (0, 31_337, 99_000):
        _compare_posteriors(em, V, a0, rb, s2, w, lo, W, prec, row0=r0, nrows=1000)
    em.step(1)
    it = oracle.em_iteration(V, a0, rb, s2, w.kbar, w.L, oracle.offsets(lo, W), rho_bar=rb,
                             gamma=w.gamma)
    a1, rho1, _ = em.state()
    assert np.linalg.norm(a1 - it["a"]) / np.linalg.norm(it["a"]) <= 1e-3
    assert np.abs(rho1 - it["rho"]).max() <= 1e-3 * it["rho"].max()
    assert abs(em.stats()[-1, 1] - it["ll"]) <= 1e-6 * abs(it["ll"])
    em.close()


@pytest.mark.parametrize("factored", [False, True])
def test_full_size_full_search_step(gpu, factored):
    """The plain full-search workload at full size (N=1e5, D=512, L=360, FP32): one step, with
    the correlation pass and with the factored pass."""
    from paper_2105_07372_amd import EM
    w = wl.WORKLOADS["c2"]
    a_true = wl.image(w, 0)
    V = wl.observations(w, 0, a=a_true)
    s2 = wl.noise_variance(a_true, w.snr)
    a0 = wl.random_init(w, 0)
    em = EM(_obs(V, "fp32", gpu), K=w.K, Q=w.Q, L=w.L, sigma2=s2, precision="fp32", a0=a0,
            factored=factored)
    rho = np.full(w.L, 1.0 / w.L)
    _compare_posteriors(em, V, a0, rho, s2, w, 0, w.L, "fp32", row0=50_000, nrows=2000)
    em.step(1)
    it = oracle.em_iteration(V, a0, rho, s2, w.kbar, w.L, oracle.offsets(0, w.L))
    a1, rho1, _ = em.state()
    assert np.linalg.norm(a1 - it["a"]) / np.linalg.norm(it["a"]) <= 1e-4
    assert np.abs(rho1 - it["rho"]).max() <= 1e-4 * it["rho"].max()
    em.close()
