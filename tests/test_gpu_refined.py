"""The refined-resolution window (Section III-C: the likely range of rotations sampled more densely
than the grid 2 pi / L, here at off-grid angles) against the FP64 oracle with the same angle list:
teacher-forced steps through every pass kind (general, K-split, factored) and precision, a
trajectory, and a grid angle list against the offset window it lists."""
import numpy as np
import pytest

import oracle
import workloads as wl

pytestmark = pytest.mark.gpu

TOL = {"fp64": dict(post=2e-7, a=1e-10, ll=1e-12),   # posteriors are returned as float32
       "fp32": dict(post=2e-4, a=2e-5, ll=1e-7),
       "bf16x3": dict(post=1e-3, a=1e-4, ll=1e-6), "fp16": dict(post=1e-3, a=2e-4, ll=1e-6),
       "bf16": dict(post=5e-3, a=1e-3, ll=1e-5)}

CASES = {
    # name: (K, Q, L, rotation std in degrees, W angles, step in grid units, N, factored)
    "small": (8, 8, 72, 6.0, 25, 0.5, 5003, False),        # general pass, W = 25 -> 2 tiles
    "ksplit": (32, 16, 360, 4.0, 49, 0.5, 4099, False),    # D = 512, 49 half-degree angles
    "factored": (32, 16, 360, 4.0, 49, 0.5, 4099, True),   # the factored pass, same angles
    "uneven": (8, 8, 72, 6.0, 21, 0.37, 997, False),       # off-grid step, ragged tail
}


def _angles(L, W, step):
    """W angles centred on 0, `step` grid steps apart (radians)."""
    return (np.arange(W) - W // 2) * step * 2 * np.pi / L


def _problem(case, seed=0):
    K, Q, L, std, W, step, N, fac = CASES[case]
    w = wl.WORKLOADS["c3"].replace(K=K, Q=Q, L=L, N=N, rot_std_deg=std)
    a_true = wl.image(w, seed)
    V = wl.observations(w, seed, a=a_true)
    s2 = wl.noise_variance(a_true, w.snr)
    th = _angles(L, W, step)
    # a prior shaped like the rotation law, evaluated at the angles
    rb = np.exp(-0.5 * (np.degrees(th) / std) ** 2)
    rb /= rb.sum()
    return w, a_true, V, s2, th, rb, fac


def _teacher_forced(gpu, case, prec, staged=False):
    import torch
    from paper_2105_07372_amd import EM
    w, a_true, V, s2, th, rb, fac = _problem(case)
    W = len(th)
    rng = np.random.default_rng(7)
    a_t = V.mean(axis=0) + 0.1 * a_true * rng.standard_normal(w.D)
    rho_t = rb * rng.uniform(0.5, 1.5, W)
    rho_t /= rho_t.sum()
    gamma = 30.0
    dt = np.complex128 if prec == "fp64" else np.complex64
    print(f"refined case={case} prec={prec} N={w.N} D={w.D} W={W}", flush=True)
    em = EM(torch.from_numpy(V.astype(dt)).to(gpu), K=w.K, Q=w.Q, L=w.L, sigma2=s2, prior=rb,
            gamma=gamma, precision=prec, angles=th, factored=fac, staged_pass=staged)
    kern = em.info()["kernel"]
    if fac:
        assert kern.startswith("pass_fac_kernel"), kern
    elif case == "ksplit":
        want = {"fp32": "pass_gm_kernel", "bf16x3": "pass_ks_kernel",
                "fp16": "pass_ks_kernel" if staged else "pass_kr_kernel"}[prec]
        assert kern.startswith(want), kern
    em.set_state(a_t, rho_t, 0)
    ang = oracle.AngleList(th)
    wg, am, mg = em.posterior()
    wo, _, _ = oracle.estep(V, a_t, rho_t, s2, w.kbar, w.L, ang)
    ao, mo = oracle.argmax_margin(wo)
    wg, am, mg = wg.cpu().numpy().astype(np.float64), am.cpu().numpy(), mg.cpu().numpy()
    assert np.abs(wg - wo).max() <= TOL[prec]["post"]
    assert np.linalg.norm(wg - wo) / np.linalg.norm(wo) <= TOL[prec]["post"]
    sure = mo > (1e-2 if prec == "bf16" else 1e-3)
    assert int(np.sum(am[sure] != ao[sure])) == 0
    ll_ref = oracle.loglik(V, a_t, rho_t, s2, w.kbar, w.L, ang)
    assert abs(em.loglik() - ll_ref) <= TOL[prec]["ll"] * abs(ll_ref)
    done, ll_step = em.step(1)
    assert done == 1 and abs(ll_step - ll_ref) <= TOL[prec]["ll"] * abs(ll_ref)
    it = oracle.em_iteration(V, a_t, rho_t, s2, w.kbar, w.L, ang, rho_bar=rb, gamma=gamma)
    a1, rho1, _ = em.state()
    assert np.linalg.norm(a1 - it["a"]) / np.linalg.norm(it["a"]) <= TOL[prec]["a"]
    assert np.abs(rho1 - it["rho"]).max() <= TOL[prec]["a"]
    # the stopping metric stays on the L-point grid
    st = em.stats()
    na = np.linalg.norm(a1)
    bar = 3 * np.sqrt(it["stop"]) * TOL[prec]["a"] * na + 1e-12 * na * na
    assert abs(st[0, 4] - it["stop"]) <= bar
    em.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3", "fp16", "bf16"])
@pytest.mark.parametrize("case", ["small", "uneven"])
def test_refined_teacher_forced_general(gpu, case, prec):
    _teacher_forced(gpu, case, prec)


@pytest.mark.parametrize("prec,staged", [("fp32", False), ("bf16x3", False), ("fp16", False),
                                          ("fp16", True)])
def test_refined_teacher_forced_ksplit(gpu, prec, staged):
    """The default windowed passes on an angle list: the FP32 matrix-core GEMM, the K-split
    pass (bf16 hi + lo, and fp16 when asked for), the row-stream pass (fp16)."""
    _teacher_forced(gpu, "ksplit", prec, staged)


@pytest.mark.parametrize("prec", ["fp32", "fp16"])
def test_refined_teacher_forced_factored(gpu, prec):
    _teacher_forced(gpu, "factored", prec)


def test_refined_trajectory(gpu):
    """49 half-degree angles on the D = 512 shape, bf16x3: four EM iterations from the mean
    against the oracle's, each from its own previous state."""
    import torch
    from paper_2105_07372_amd import EM
    w, a_true, V, s2, th, rb, _ = _problem("ksplit")
    a0 = V.astype(np.complex64).astype(np.complex128).mean(axis=0)
    em = EM(torch.from_numpy(V.astype(np.complex64)).to(gpu), K=w.K, Q=w.Q, L=w.L, sigma2=s2,
            prior=rb, gamma=100.0, precision="bf16x3", angles=th, a0=a0)
    ang = oracle.AngleList(th)
    a_o, rho_o = a0, rb
    for t in range(4):
        ref = oracle.em_iteration(V, a_o, rho_o, s2, w.kbar, w.L, ang, rho_bar=rb, gamma=100.0)
        em.step(1)
        a, rho, _ = em.state()
        assert np.linalg.norm(a - ref["a"]) / np.linalg.norm(ref["a"]) <= 1e-4, t
        assert np.abs(rho - ref["rho"]).max() <= 1e-4, t
        assert abs(em.stats()[-1, 1] - ref["ll"]) <= 1e-6 * abs(ref["ll"]), t
        a_o, rho_o = ref["a"], ref["rho"]
    em.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_grid_angle_list_is_the_offset_window(gpu, prec):
    """Angles 2 pi (lo + i) / L listed explicitly reproduce the offset window lo .. lo + W - 1."""
    import torch
    from paper_2105_07372_amd import EM
    w = wl.WORKLOADS["c3"].replace(N=3001, K=8, Q=8, L=72, half_window=6)
    a_true = wl.image(w, 0)
    V = wl.observations(w, 0, a=a_true)
    s2 = wl.noise_variance(a_true, w.snr)
    lo, W = w.window
    dt = np.complex128 if prec == "fp64" else np.complex64
    obs = torch.from_numpy(V.astype(dt)).to(gpu)
    th = 2 * np.pi * np.arange(lo, lo + W) / w.L
    out = []
    for kw in (dict(window=(lo, W)), dict(angles=th)):
        em = EM(obs, K=w.K, Q=w.Q, L=w.L, sigma2=s2, gamma=0.0, precision=prec, **kw)
        em.step(3)
        a, rho, _ = em.state()
        out.append((a, rho, em.stats()[:, 1].copy()))
        em.close()
    tol = 1e-12 if prec == "fp64" else 2e-5
    assert np.linalg.norm(out[0][0] - out[1][0]) <= tol * np.linalg.norm(out[0][0])
    assert np.abs(out[0][1] - out[1][1]).max() <= tol
    assert np.abs(out[0][2] - out[1][2]).max() <= tol * np.abs(out[0][2]).max()
