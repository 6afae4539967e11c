"""The hand-written adjoint of the marginal log-likelihood (em_loglik_fwd / em_loglik_bwd) and its
torch.autograd.Function, against the oracle's Fisher-identity gradients and FP64 finite
differences."""
import numpy as np
import pytest

import oracle
import workloads as wl

pytestmark = pytest.mark.gpu


def _fd_problem(W):
    w = wl.WORKLOADS["c4fd"]
    a_true = wl.image(w, 0)
    V = wl.observations(w, 0, a=a_true)
    lo = 0 if W == w.L else -(W // 2)
    rng = np.random.default_rng(4)
    eta = rng.standard_normal(W) * 0.3
    a = V.mean(axis=0) + 0.05 * a_true
    s2 = wl.noise_variance(a_true, w.snr) * 1.3
    return w, V, lo, eta, a, s2


def _rho(eta):
    r = np.exp(eta - eta.max())
    return r / r.sum()


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("fp32", 2e-4)])
@pytest.mark.parametrize("W", [16, 7])
def test_adjoint_matches_oracle_fisher_gradient(gpu, prec, tol, W):
    import torch
    from paper_2105_07372_amd import EM
    w, V, lo, eta, a, s2 = _fd_problem(W)
    obs = torch.from_numpy(V.astype(np.complex128 if prec == "fp64" else np.complex64)).to(gpu)
    em = EM(obs, K=w.K, Q=w.Q, L=w.L, sigma2=s2, window=(lo, W), precision=prec)
    a_d = torch.from_numpy(a).to(gpu)
    eta_d = torch.from_numpy(eta).to(gpu)
    ll = em.loglik_fwd(a_d, s2, eta_d)
    ga = torch.empty_like(a_d)
    ge = torch.empty_like(eta_d)
    gs = em.loglik_bwd(1.0, ga, ge)
    ll_o, ga_o, gs_o, ge_o = oracle.grad_loglik(V, a, s2, _rho(eta), w.kbar, w.L,
                                                oracle.offsets(lo, W))
    assert abs(ll - ll_o) <= tol * abs(ll_o)
    assert np.linalg.norm(ga.cpu().numpy() - ga_o) <= tol * np.linalg.norm(ga_o) * 10
    assert abs(gs - gs_o) <= tol * 10 * max(1.0, abs(gs_o))
    assert np.abs(ge.cpu().numpy() - ge_o).max() <= tol * 10 * max(1.0, np.abs(ge_o).max())
    em.close()


def test_adjoint_against_gpu_finite_differences(gpu):
    """FP64: fourth-order central differences of the GPU log-likelihood itself against the GPU
    adjoint.  A difference quotient with step h carries the log-likelihood's rounding error delta
    amplified to about 1.5 delta / h; delta is taken as 64 ulps of |LL| (the FP64 sums of the pass
    and the finalize, with cancellation among terms a few times |LL|), and h = 1e-4 of each
    argument's scale keeps the h^4 truncation term far below that floor."""
    import torch
    from paper_2105_07372_amd import EM
    w, V, lo, eta, a, s2 = _fd_problem(7)
    em = EM(torch.from_numpy(V).to(gpu), K=w.K, Q=w.Q, L=w.L, sigma2=s2, window=(lo, 7),
            precision="fp64")
    ll = lambda a_, s_, e_: em.loglik_fwd(torch.from_numpy(a_).to(gpu), s_,
                                          torch.from_numpy(e_).to(gpu))
    ll0 = ll(a, s2, eta)
    ga = torch.empty(w.D, dtype=torch.complex128, device=gpu)
    ge = torch.empty(7, dtype=torch.float64, device=gpu)
    gs = em.loglik_bwd(1.0, ga, ge)
    ga, ge = ga.cpu().numpy(), ge.cpu().numpy()
    delta = 64 * np.finfo(np.float64).eps * abs(ll0)

    def fd4(f, h):
        return (8 * (f(h) - f(-h)) - (f(2 * h) - f(-2 * h))) / (12 * h)

    def bar(h, g):
        return 1.5 * delta / h + 1e-9 * max(1.0, abs(g))

    h = 1e-4 * float(np.abs(a).max())
    for d in range(0, w.D, 5):
        for unit, comp in ((1.0, ga[d].real), (1j, ga[d].imag)):
            e = np.zeros(w.D, complex)
            e[d] = unit
            fd = fd4(lambda x: ll(a + x * e, s2, eta), h)
            assert abs(fd - comp) <= bar(h, comp), (d, unit, fd, comp)
    hs = 1e-4 * s2
    fd = fd4(lambda x: ll(a, s2 + x, eta), hs)
    assert abs(fd - gs) <= bar(hs, gs), (fd, gs)
    for i in range(7):
        e = np.zeros(7)
        e[i] = 1.0
        fd = fd4(lambda x: ll(a, s2, eta + x * e), 1e-4)
        assert abs(fd - ge[i]) <= bar(1e-4, ge[i]), (i, fd, ge[i])
    em.close()


def test_autograd_function_and_fisher_step(gpu):
    """torch.autograd through MarginalLogLik gives the adjoint's gradients, and a gradient-ascent
    step of size sigma^2 / (2N) on a equals one EM coefficient update (no image prior)."""
    import torch
    from paper_2105_07372_amd import EM
    from paper_2105_07372_amd.autograd import marginal_loglik
    w, V, lo, eta, a, s2 = _fd_problem(16)
    rho = _rho(eta)
    em = EM(torch.from_numpy(V).to(gpu), K=w.K, Q=w.Q, L=w.L, sigma2=s2, window=(lo, 16),
            prior=rho, precision="fp64", update_rho=False)
    a_t = torch.from_numpy(a).to(gpu).requires_grad_(True)
    s_t = torch.tensor(s2, dtype=torch.float64, device=gpu, requires_grad=True)
    e_t = torch.from_numpy(eta).to(gpu).requires_grad_(True)
    ll = marginal_loglik(em, a_t, s_t, e_t)
    ga, gs, ge = torch.autograd.grad(3.0 * ll, (a_t, s_t, e_t))
    ll_o, ga_o, gs_o, ge_o = oracle.grad_loglik(V, a, s2, rho, w.kbar, w.L, oracle.offsets(lo, 16))
    assert abs(ll.item() - ll_o) <= 1e-10 * abs(ll_o)
    assert np.linalg.norm(ga.cpu().numpy() - 3 * ga_o) <= 1e-9 * np.linalg.norm(ga_o)
    assert abs(gs.item() - 3 * gs_o) <= 1e-9 * abs(gs_o)
    assert np.abs(ge.cpu().numpy() - 3 * ge_o).max() <= 1e-9 * max(1.0, np.abs(ge_o).max())
    # Fisher identity: a + s2/(2N) dLL/da == EM update at (a, rho)
    em.set_state(a, rho, 0)
    em.step(1)
    a_em = em.state()[0]
    a_step = a + s2 / (2 * w.N) * (ga.cpu().numpy() / 3.0)
    assert np.linalg.norm(a_step - a_em) <= 1e-10 * np.linalg.norm(a_em)
    em.close()


def test_backward_needs_forward(gpu):
    import torch
    from paper_2105_07372_amd import EM, SynchemError
    w, V, lo, eta, a, s2 = _fd_problem(16)
    em = EM(torch.from_numpy(V).to(gpu), K=w.K, Q=w.Q, L=w.L, sigma2=s2, precision="fp64")
    g = torch.empty(w.D, dtype=torch.complex128, device=gpu)
    with pytest.raises(SynchemError) as ei:
        em.loglik_bwd(1.0, g)
    assert ei.value.status == -4
    em.close()


def test_adjoint_full_size_windowed(gpu):
    """The differentiable log-likelihood on the windowed workload (N=1e5, D=512, W=49, FP32 with
    FP64 reductions) at the state after 5 EM iterations: gradients against the oracle's."""
    import torch
    from paper_2105_07372_amd import EM
    w = wl.WORKLOADS["c4"]
    a_true = wl.image(w, 0)
    V = wl.observations(w, 0, a=a_true)
    s2 = wl.noise_variance(a_true, w.snr)
    lo, W = w.window
    rb, _, _ = oracle.histogram_prior(wl.prior_error_draws(w, 0), w.L, lo, W)
    em = EM(torch.from_numpy(V.astype(np.complex64)).to(gpu), K=w.K, Q=w.Q, L=w.L, sigma2=s2,
            window=(lo, W), prior=rb, gamma=w.gamma, precision="fp32")
    em.step(5)
    a5, rho5, _ = em.state()
    a_d = torch.from_numpy(a5).to(gpu)
    ll = em.loglik_fwd(a_d, s2 * 1.1)
    ga = torch.empty_like(a_d)
    gs = em.loglik_bwd(1.0, ga)
    ll_o, ga_o, gs_o, _ = oracle.grad_loglik(V, a5, s2 * 1.1, rho5, w.kbar, w.L,
                                             oracle.offsets(lo, W))
    assert abs(ll - ll_o) <= 1e-6 * abs(ll_o)
    assert np.linalg.norm(ga.cpu().numpy() - ga_o) <= 1e-3 * np.linalg.norm(ga_o)
    assert abs(gs - gs_o) <= 1e-3 * abs(gs_o)
    em.close()


@pytest.mark.parametrize("between", ["step_keep_lse", "set_state"])
def test_checkpoint_invalidated_between_forward_and_backward(gpu, between):
    """An EM step that stores its own per-row LSE (keep_lse) or a state reset between the forward
    and the backward: the raw backward refuses (EM_ESTATE), and the autograd Function runs the
    forward again, so its gradients are still those of the forward's inputs (oracle)."""
    import torch
    from paper_2105_07372_amd import EM, SynchemError
    from paper_2105_07372_amd.autograd import marginal_loglik
    w, V, lo, eta, a, s2 = _fd_problem(16)
    rho = _rho(eta)
    em = EM(torch.from_numpy(V).to(gpu), K=w.K, Q=w.Q, L=w.L, sigma2=s2, window=(lo, 16),
            prior=rho, precision="fp64", keep_lse=True)

    def disturb():
        if between == "step_keep_lse":
            em.step(2)                       # moves a_t and rewrites the LSE buffer
        else:
            em.set_state(V[3], rho, 0)

    a_d = torch.from_numpy(a).to(gpu)
    em.loglik_fwd(a_d, s2)
    disturb()
    with pytest.raises(SynchemError) as ei:
        em.loglik_bwd(1.0, torch.empty_like(a_d))
    assert ei.value.status == -4
    a_t = torch.from_numpy(a).to(gpu).requires_grad_(True)
    s_t = torch.tensor(s2, dtype=torch.float64, device=gpu, requires_grad=True)
    e_t = torch.from_numpy(eta).to(gpu).requires_grad_(True)
    ll = marginal_loglik(em, a_t, s_t, e_t)
    disturb()
    ga, gs, ge = torch.autograd.grad(ll, (a_t, s_t, e_t))
    ll_o, ga_o, gs_o, ge_o = oracle.grad_loglik(V, a, s2, rho, w.kbar, w.L, oracle.offsets(lo, 16))
    assert abs(ll.item() - ll_o) <= 1e-10 * abs(ll_o)
    assert np.linalg.norm(ga.cpu().numpy() - ga_o) <= 1e-9 * np.linalg.norm(ga_o)
    assert abs(gs.item() - gs_o) <= 1e-9 * abs(gs_o)
    assert np.abs(ge.cpu().numpy() - ge_o).max() <= 1e-9 * max(1.0, np.abs(ge_o).max())
    em.close()
