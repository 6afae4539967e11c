"""The planner over a grid of shapes: every precision at coefficient counts from tiny to the
largest supported, windows from one rotation to a few hundred.  Each context either runs (its
log-likelihood and one EM step against the oracle) or is refused with EM_EUNSUPPORTED for the
documented limit: FP64, FP32 and bf16x3 rows must fit the LDS tile (D <= 512); only the
single-plane 16-bit formats stream longer rows (up to D = 2048) through the wide-row pass."""
import numpy as np
import pytest

import oracle
import workloads as wl

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-10, "fp32": 2e-5, "bf16x3": 1e-4, "fp16": 3e-4, "bf16": 2e-3}     # estimate
LLTOL = {"fp64": 1e-12, "fp32": 1e-7, "bf16x3": 1e-6, "fp16": 1e-6, "bf16": 1e-5}
SHAPES = [(1, 8), (3, 8), (8, 8), (16, 8), (10, 20), (32, 16), (25, 40), (64, 32)]   # (K, Q)
WINDOWS = [1, 7, 49, 181]


def _documented_limit(prec, D):
    return prec in ("fp64", "fp32", "bf16x3") and D > 512


@pytest.mark.parametrize("prec", list(TOL))
@pytest.mark.parametrize("K,Q", SHAPES)
def test_planner_covers_shapes(gpu, prec, K, Q):
    import torch
    from paper_2105_07372_amd import EM, SynchemError
    L = 360
    w = wl.WORKLOADS["c3"].replace(K=K, Q=Q, N=257, L=L, rot_std_deg=20.0)
    a = wl.image(w, 0)
    V = wl.observations(w, 0, a=a)
    s2 = wl.noise_variance(a, w.snr)
    dt = np.complex128 if prec == "fp64" else np.complex64
    obs = torch.from_numpy(V.astype(dt)).to(gpu)
    a_t = V.mean(axis=0) + 0.2 * a
    for W in WINDOWS:
        lo = -(W // 2)
        print(f"shape K={K} Q={Q} prec={prec} W={W}", flush=True)
        try:
            em = EM(obs, K=K, Q=Q, L=L, sigma2=s2, window=(lo, W), precision=prec)
        except SynchemError as e:
            assert "EM_EUNSUPPORTED" in str(e) and _documented_limit(prec, K * Q), str(e)
            continue
        assert not _documented_limit(prec, K * Q)
        rho = np.full(W, 1.0 / W)
        em.set_state(a_t, rho, 0)
        offs = oracle.offsets(lo, W)
        ll_o = oracle.loglik(V.astype(dt).astype(np.complex128), a_t, rho, s2, w.kbar, L, offs)
        assert abs(em.loglik() - ll_o) <= LLTOL[prec] * abs(ll_o), (em.info()["kernel"], W)
        em.step(1)
        it = oracle.em_iteration(V.astype(dt).astype(np.complex128), a_t, rho, s2, w.kbar, L,
                                 offs)
        a1 = em.state()[0]
        assert np.linalg.norm(a1 - it["a"]) <= TOL[prec] * np.linalg.norm(it["a"]), \
            (em.info()["kernel"], W)
        em.close()
