"""A learned prior with empty bins inside the window (eq. (15) multiplies each posterior by the
prior, so such a rotation gets weight exactly zero; eq. (18) and the KL-prior update then keep
it at zero).  Every pass variant, with gamma = 0 and gamma > 0: the zero columns of the
posteriors and of rho are exactly zero, the rest matches the oracle."""
import numpy as np
import pytest

import oracle
import workloads as wl

pytestmark = pytest.mark.gpu

TOL = {"fp64": dict(post=2e-7, a=1e-10, ll=1e-12), "fp32": dict(post=2e-4, a=2e-5, ll=1e-7),
       "bf16x3": dict(post=1e-3, a=1e-4, ll=1e-6), "fp16": dict(post=1e-3, a=2e-4, ll=1e-6)}

# (precision, EM keyword arguments, kernel family the planner must pick)
PASSES = [("fp64", {}, "pass_kernel"),
          ("fp32", {}, "pass_gm_kernel"),
          ("fp32", {"general_pass": True}, "pass_kernel"),
          ("bf16x3", {"general_pass": True}, "pass_kernel"),
          ("bf16x3", {}, "pass_ks_kernel"),
          ("fp16", {}, "pass_kr_kernel"),
          ("fp16", {"staged_pass": True}, "pass_ks_kernel"),
          ("fp32", {"factored": True}, "pass_fac_kernel"),
          ("bf16x3", {"factored": True}, "pass_fac_kernel"),
          ("fp16", {"wide_pass": True}, "pass_wide_kernel")]


@pytest.mark.parametrize("gamma", [0.0, 40.0])
@pytest.mark.parametrize("prec,kw,kernel", PASSES)
def test_zero_prior_bins(gpu, prec, kw, kernel, gamma):
    import torch
    from paper_2105_07372_amd import EM
    w = wl.WORKLOADS["c3"].replace(N=4099, K=32, Q=16, L=360, half_window=24)
    a_true = wl.image(w, 0)
    V = wl.observations(w, 0, a=a_true)
    s2 = wl.noise_variance(a_true, w.snr)
    lo, W = w.window
    rb, _, _ = oracle.histogram_prior(wl.prior_error_draws(w, 0, 200_000), w.L, lo, W)
    zero = np.array([0, 5, 24, 25, 47])              # empty bins: the edges and the centre
    rb[zero] = 0.0
    rb /= rb.sum()
    print(f"zero prior: {prec} {kw} gamma={gamma}", flush=True)
    cdt = np.complex128 if prec == "fp64" else np.complex64
    obs = torch.from_numpy(V.astype(cdt)).to(gpu)
    em = EM(obs, K=w.K, Q=w.Q, L=w.L, sigma2=s2, window=(lo, W), prior=rb, gamma=gamma,
            precision=prec, **kw)
    assert em.info()["kernel"].startswith(kernel + "<"), em.info()
    a0 = V.astype(cdt).astype(np.complex128).mean(axis=0)      # the GPU's a_0 = mean v
    offs = oracle.offsets(lo, W)
    wg, am, mg = em.posterior()
    wg = wg.cpu().numpy().astype(np.float64)
    wo, _, _ = oracle.estep(V, a0, rb, s2, w.kbar, w.L, offs)
    assert np.all(wg[:, zero] == 0.0)
    assert np.abs(wg - wo).max() <= TOL[prec]["post"]
    ao, mo = oracle.argmax_margin(wo)
    sure = mo > 1e-3
    assert int(np.sum(am.cpu().numpy()[sure] != ao[sure])) == 0
    assert not np.isin(am.cpu().numpy(), zero).any()
    # three free-running iterations on both sides
    a, rho = a0, rb
    for t in range(3):
        it = oracle.em_iteration(V, a, rho, s2, w.kbar, w.L, offs, rho_bar=rb, gamma=gamma)
        em.step(1)
        a1, rho1, _ = em.state()
        assert np.all(rho1[zero] == 0.0), t
        assert np.linalg.norm(a1 - it["a"]) <= 3 * TOL[prec]["a"] * np.linalg.norm(it["a"]), t
        assert np.abs(rho1 - it["rho"]).max() <= 3 * TOL[prec]["a"], t
        st = em.stats()[-1]
        assert abs(st[1] - it["ll"]) <= 3 * TOL[prec]["ll"] * abs(it["ll"]), t
        assert np.isfinite(st[2]) and abs(st[2] - it["J"]) <= 3 * TOL[prec]["ll"] * abs(it["ll"]) + 1e-12 * abs(it["J"]), t
        a, rho = it["a"], it["rho"]
    em.close()
