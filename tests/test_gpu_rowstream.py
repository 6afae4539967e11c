"""The row-stream correlation pass (pass_kr_kernel: one 16-bit plane, D = 512, windows up to 64)
against the FP64 oracle: teacher-forced steps over every window-tile count and every supported
radial size Q, ragged tails and row counts that give each workgroup one, two, three or many
tiles (the copy pipeline keeps two tiles in flight), posterior queries, free-running
trajectories, the stored / reloaded log-sum-exp of the adjoint, and agreement with the
LDS-staged pass on the same inputs."""
import numpy as np
import pytest

import oracle
import workloads as wl
from bounds import loglik_bar

pytestmark = pytest.mark.gpu

TOL = {"fp16": dict(post=1e-3, a=2e-4, ll=1e-6), "bf16": dict(post=5e-3, a=1e-3, ll=1e-5)}


def _problem(N, K, Q, h, seed=0, L=360):
    w = wl.WORKLOADS["c3"].replace(N=N, K=K, Q=Q, L=L, half_window=h)
    a_true = wl.image(w, seed)
    V = wl.observations(w, seed, a=a_true)
    s2 = wl.noise_variance(a_true, w.snr)
    lo, W = w.window
    rb, _, _ = oracle.histogram_prior(wl.prior_error_draws(w, seed, 200_000), w.L, lo, W)
    return w, a_true, V, s2, lo, W, rb


def _em(gpu, V, w, s2, lo, W, rb, prec, gamma=50.0, **kw):
    import torch
    from paper_2105_07372_amd import EM
    obs = torch.from_numpy(V.astype(np.complex64)).to(gpu)
    return EM(obs, K=w.K, Q=w.Q, L=w.L, sigma2=s2, window=(lo, W), prior=rb, gamma=gamma,
              precision=prec, **kw)


def _check_step(em, V, w, s2, lo, W, rb, prec, gamma, rng):
    # a state near the image, the same whatever N (a state built from the rows themselves would
    # sit on top of a single row for N = 1, where the fp16 rounding of that row dominates)
    a0 = wl.image(w, 0)
    a_t = 0.9 * a0 + 0.1 * a0 * rng.standard_normal(w.D)
    rho_t = rb * rng.uniform(0.5, 1.5, W)
    rho_t /= rho_t.sum()
    em.set_state(a_t, rho_t, 0)
    offs = oracle.offsets(lo, W)
    wg, am, mg = em.posterior()
    wg, am, mg = wg.cpu().numpy().astype(np.float64), am.cpu().numpy(), mg.cpu().numpy()
    wo, _, _ = oracle.estep(V, a_t, rho_t, s2, w.kbar, w.L, offs)
    ao, mo = oracle.argmax_margin(wo)
    assert np.abs(wg - wo).max() <= TOL[prec]["post"]
    assert np.linalg.norm(wg - wo) / np.linalg.norm(wo) <= TOL[prec]["post"]
    sure = mo > (1e-3 if prec == "fp16" else 1e-2)
    assert int(np.sum(am[sure] != ao[sure])) == 0
    assert np.abs(mg - mo).max() <= 2 * TOL[prec]["post"] + 1e-6
    ll_ref = oracle.loglik(V, a_t, rho_t, s2, w.kbar, w.L, offs)
    u = 2.0 ** -11 if prec == "fp16" else 2.0 ** -8        # unit roundoff of the storage
    ll_bar = max(TOL[prec]["ll"] * abs(ll_ref),
                 loglik_bar(V, a_t, s2, w.kbar, w.L, offs, u) + 1e-12 * abs(ll_ref))
    assert abs(em.loglik() - ll_ref) <= ll_bar
    em.step(1)
    it = oracle.em_iteration(V, a_t, rho_t, s2, w.kbar, w.L, offs, rho_bar=rb, gamma=gamma)
    a1, rho1, _ = em.state()
    # the new estimate averages N rounded rows: their rounding alone contributes a relative error
    # of RMS u / sqrt(3 N), which sets the bar for few rows
    a_bar = max(TOL[prec]["a"], 3 * u / np.sqrt(3 * V.shape[0]))
    assert np.linalg.norm(a1 - it["a"]) / np.linalg.norm(it["a"]) <= a_bar
    assert np.abs(rho1 - it["rho"]).max() <= a_bar
    st = em.stats()[-1]
    assert abs(st[1] - ll_ref) <= ll_bar
    assert abs(st[2] - it["J"]) <= ll_bar + 1e-12 * abs(it["J"])


@pytest.mark.parametrize("prec", ["fp16", "bf16"])
@pytest.mark.parametrize("K,Q,h", [(32, 16, 24), (64, 8, 20), (16, 32, 12), (8, 64, 4),
                                    (32, 16, 31), (32, 16, 15)])
def test_rowstream_teacher_forced(gpu, prec, K, Q, h):
    """W = 2h + 1 over 1, 2, 3 and 4 window tiles; Q = 8 .. 64; N = 20037 (ragged last tile,
    about five tiles per workgroup)."""
    w, a_true, V, s2, lo, W, rb = _problem(20037, K, Q, h)
    print(f"row-stream {prec} K={K} Q={Q} W={W}", flush=True)
    em = _em(gpu, V, w, s2, lo, W, rb, prec)
    assert em.info()["kernel"] == f"pass_kr_kernel<{'f16' if prec == 'fp16' else 'bf16'},NT={(W + 15) // 16}>", em.info()
    _check_step(em, V, w, s2, lo, W, rb, prec, 50.0, np.random.default_rng(K + Q + h))
    em.close()


@pytest.mark.parametrize("N", [1, 15, 16, 17, 4096, 4111, 8193, 12289, 12300])
def test_rowstream_tile_counts(gpu, N):
    """Row counts that give the workgroups zero, one, two, three and four tiles (a grid of up to
    256 workgroups of 16-row tiles), with ragged last tiles."""
    w, a_true, V, s2, lo, W, rb = _problem(N, 32, 16, 24, seed=1)
    print(f"row-stream N={N}", flush=True)
    em = _em(gpu, V, w, s2, lo, W, rb, "fp16")
    assert em.info()["kernel"].startswith("pass_kr_kernel"), em.info()
    _check_step(em, V, w, s2, lo, W, rb, "fp16", 50.0, np.random.default_rng(N))
    em.close()


def test_rowstream_matches_staged_pass_and_trajectory(gpu):
    """The row-stream and LDS-staged passes on the same fp16 inputs (they round the same
    products in different orders): 10 free-running iterations each against the oracle's."""
    w, a_true, V, s2, lo, W, rb = _problem(30011, 32, 16, 24, seed=2)
    a_o, rho_o, _ = oracle.em_run(V, V.astype(np.complex64).astype(np.complex128).mean(axis=0),
                                  rb, s2, w.kbar, w.L, oracle.offsets(lo, W), 10, rho_bar=rb,
                                  gamma=100.0)
    out = {}
    for staged in (False, True):
        em = _em(gpu, V, w, s2, lo, W, rb, "fp16", gamma=100.0, staged_pass=staged)
        assert em.info()["kernel"].startswith("pass_ks_kernel" if staged else "pass_kr_kernel")
        em.step(10)
        out[staged] = em.state()
        J = em.stats()[:, 2]
        assert np.all(np.diff(J) >= -1e-6 * np.abs(J[1:]))
        em.close()
    for staged, (a_g, rho_g, t) in out.items():
        assert t == 10
        assert np.linalg.norm(a_g - a_o) / np.linalg.norm(a_o) <= 2e-3, staged
        assert np.abs(rho_g - rho_o).max() <= 2e-3, staged
    a0, a1 = out[False][0], out[True][0]
    assert np.linalg.norm(a0 - a1) / np.linalg.norm(a1) <= 2e-3


def test_rowstream_adjoint_and_lse_checkpoint(gpu):
    """em_loglik_fwd stores the per-row log-sum-exp and em_loglik_bwd reloads it (both leave the
    copy pipeline's exact counts): gradients against the oracle's Fisher-identity gradients."""
    import torch
    w, a_true, V, s2, lo, W, rb = _problem(9001, 32, 16, 24, seed=3)
    em = _em(gpu, V, w, s2, lo, W, rb, "fp16")
    rng = np.random.default_rng(7)
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
    assert abs(ll - ll_o) <= 1e-6 * abs(ll_o)
    assert np.linalg.norm(ga.cpu().numpy() - ga_o) <= 2e-3 * np.linalg.norm(ga_o)
    assert abs(gs - gs_o) <= 2e-3 * abs(gs_o)
    assert np.abs(ge.cpu().numpy() - ge_o).max() <= 2e-3 * max(1.0, np.abs(ge_o).max())
    em.close()
