"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics (CPU only).

Each test checks the oracle against something other than itself: explicit rotation (coefficient
and pixel domain), a density written out term by term, closed forms, optimality conditions,
invariants, or finite differences.
"""
import math

import numpy as np
import pytest

import oracle
import workloads as wl
from oracle.em import OracleInvalid, OracleNonFinite


def _problem(K=4, Q=3, N=7, L=12, snr=0.7, seed=0, window=None):
    rng = np.random.default_rng(seed)
    D = K * Q
    kbar = np.repeat(np.arange(K), Q)
    a = (rng.standard_normal(D) + 1j * rng.standard_normal(D)) / np.sqrt(2 * (1 + kbar))
    s2 = float(np.vdot(a, a).real / (D * snr))
    l = rng.integers(0, L, N)
    V = np.stack([a * np.exp(-2j * np.pi * kbar * li / L) for li in l])
    V = V + np.sqrt(s2 / 2) * (rng.standard_normal((N, D)) + 1j * rng.standard_normal((N, D)))
    lo, W = (0, L) if window is None else window
    offs = oracle.offsets(lo, W)
    rho = rng.uniform(0.2, 1.0, W)
    rho /= rho.sum()
    a0 = a + 0.5 * (rng.standard_normal(D) + 1j * rng.standard_normal(D)) / np.sqrt(2)
    return dict(V=V, a=a, a0=a0, s2=s2, kbar=kbar, L=L, offs=offs, rho=rho, lmb=l, D=D)


# ---------------------------------------------------------------- distances and weights (eq. 15)

@pytest.mark.parametrize("window", [None, (-3, 7), (5, 4)])
def test_vectorised_distances_match_explicit_rotation(window):
    p = _problem(window=window)
    rb = oracle.distances_brute(p["V"], p["a0"], p["kbar"], p["L"], p["offs"])
    rv = oracle.distances(p["V"], p["a0"], p["kbar"], p["L"], p["offs"])
    assert np.max(np.abs(rb - rv)) <= 1e-12 * np.max(np.abs(rb))


# ---------------------------------------------------------------- refined-resolution window (§III-C)

def _refined(L, W, step):
    """W angles centred on 0, `step` grid steps (2 pi / L) apart: a window sampled more densely
    than the grid when step < 1 (§III-C)."""
    return oracle.AngleList((np.arange(W) - W // 2) * step * 2 * np.pi / L)


def test_angle_list_on_the_grid_is_the_offset_window():
    """Angles 2 pi o_i / L listed explicitly give the offset window's posteriors, log-likelihood
    and M-step (the table-free angle path against the exact grid phases)."""
    p = _problem(window=(-3, 7))
    ang = oracle.AngleList(2 * np.pi * p["offs"] / p["L"])
    args = (p["V"], p["a0"], p["rho"], p["s2"], p["kbar"], p["L"])
    w1, l1, _ = oracle.estep(*args, p["offs"])
    w2, l2, _ = oracle.estep(*args, ang)
    assert np.max(np.abs(w1 - w2)) <= 1e-13
    assert np.max(np.abs(l1 - l2)) <= 1e-12 * np.max(np.abs(l1))
    a1, _ = oracle.mstep_a(p["V"], w1, p["kbar"], p["L"], p["offs"], p["s2"])
    a2, _ = oracle.mstep_a(p["V"], w2, p["kbar"], p["L"], ang, p["s2"])
    assert np.max(np.abs(a1 - a2)) <= 1e-13 * np.max(np.abs(a1))


@pytest.mark.parametrize("step", [0.5, 0.37])
def test_angle_list_distances_match_explicit_rotation(step):
    """Off-grid angles: the matmul distances equal those of the rotation applied entry by entry
    with scalar cos/sin (eq. (15))."""
    p = _problem(L=12)
    ang = _refined(12, 9, step)
    rb = oracle.distances_brute(p["V"], p["a0"], p["kbar"], 12, ang)
    rv = oracle.distances(p["V"], p["a0"], p["kbar"], 12, ang)
    assert np.max(np.abs(rb - rv)) <= 1e-12 * np.max(np.abs(rb))


def test_refined_window_noiseless_exact_recovery():
    """Observations rotated by listed off-grid angles, no noise, s2 -> 0 at the true image: each
    posterior row is one-hot on its observation's own angle, and one M-step (eq. (17) with
    exp(+i k theta_i)) returns the image exactly."""
    K, Q, L, N, W = 4, 3, 12, 20, 9
    p = _problem(K=K, Q=Q, N=N, L=L)
    a, kbar = p["a"], p["kbar"]
    ang = _refined(L, W, 0.37)
    c = np.random.default_rng(4).integers(0, W, N)
    V = np.stack([a * np.exp(-1j * kbar * ang.theta[ci]) for ci in c])
    rho = np.full(W, 1.0 / W)
    w, _, _ = oracle.estep(V, a, rho, 1e-8, kbar, L, ang)
    assert np.array_equal(np.argmax(w, axis=1), c)
    assert np.max(np.abs(w.max(axis=1) - 1.0)) <= 1e-12
    a1, _ = oracle.mstep_a(V, w, kbar, L, ang, 1e-8)
    assert np.max(np.abs(a1 - a)) <= 1e-12 * np.max(np.abs(a))


def test_loglik_never_decreases_refined_window():
    """EM over a refined window (half-step angles) never decreases the log-likelihood."""
    p = _problem(K=6, Q=4, N=300, L=24, snr=0.3, seed=5)
    ang = _refined(24, 15, 0.5)
    rho = np.full(15, 1 / 15)
    _, _, hist = oracle.em_run(p["V"], p["a0"], rho, p["s2"], p["kbar"], 24, ang, 30)
    ll = [h["ll"] for h in hist]
    assert all(b >= a - 1e-10 * abs(a) for a, b in zip(ll, ll[1:]))


def test_pixel_rotation_matches_coefficient_phase():
    """Rotating the sampled image by shifting its angle axis equals multiplying a_kq by
    exp(-i k theta) (§I eq. (3)); the pixel-domain distances equal the coefficient ones."""
    K, Q, L = 5, 3, 8
    p = _problem(K=K, Q=Q, N=4, L=L)
    g = oracle.make_grid(K, Q, L, seed=3)
    for l in range(L):
        img = oracle.rotate_pixels(g, oracle.synthesize(g, p["a"]), l, L)
        assert np.allclose(oracle.analyze(g, img), oracle.rotate(p["a"], p["kbar"], l, L),
                           atol=1e-12)
    rp = oracle.distances_pixels(g, p["V"], p["a0"], L, p["offs"])
    rc = oracle.distances(p["V"], p["a0"], p["kbar"], L, p["offs"])
    assert np.max(np.abs(rp - rc)) <= 1e-10 * np.max(np.abs(rc))


def test_loglik_and_weights_match_density_written_out():
    """Per-row marginal likelihood sum_i rho_i (pi s2)^-D exp(-||R_i a - v||^2/s2) and Bayes'
    rule for the weights, with the Gaussian density of eq. (13) evaluated term by term."""
    p = _problem(K=2, Q=2, N=5, L=6, snr=2.0)
    w, lse, _ = oracle.estep(p["V"], p["a0"], p["rho"], p["s2"], p["kbar"], p["L"], p["offs"])
    D = p["D"]
    for j in range(5):
        terms = []
        for i, o in enumerate(p["offs"]):
            th = 2 * math.pi * o / p["L"]
            dist = 0.0
            for d in range(D):
                z = p["a0"][d] * complex(math.cos(p["kbar"][d] * th), -math.sin(p["kbar"][d] * th))
                dist += abs(z - p["V"][j, d]) ** 2
            terms.append(p["rho"][i] * math.exp(-dist / p["s2"]) / (math.pi * p["s2"]) ** D)
        tot = sum(terms)
        assert abs(math.log(tot) - lse[j]) <= 1e-12 * max(1.0, abs(lse[j]))
        assert np.allclose(w[j], np.array(terms) / tot, atol=1e-14)


def test_rows_sum_to_one():
    p = _problem(N=40)
    w, _, _ = oracle.estep(p["V"], p["a0"], p["rho"], p["s2"], p["kbar"], p["L"], p["offs"])
    assert np.max(np.abs(w.sum(axis=1) - 1.0)) <= 1e-15 * 4


def test_k0_only_is_rotation_invariant_so_weights_equal_prior():
    p = _problem(K=1, Q=5, N=9)
    w, _, _ = oracle.estep(p["V"], p["a0"], p["rho"], p["s2"], p["kbar"], p["L"], p["offs"])
    assert np.max(np.abs(w - p["rho"][None, :])) <= 1e-15


def test_huge_noise_weights_tend_to_prior():
    p = _problem(N=6)
    w, _, _ = oracle.estep(p["V"], p["a0"], p["rho"], 1e12, p["kbar"], p["L"], p["offs"])
    assert np.max(np.abs(w - p["rho"][None, :])) <= 1e-9


# ---------------------------------------------------------------- M-step (eq. 17, 18, 42)

def _perturb_dirs(D, rng, n=6):
    return [(rng.standard_normal(D) + 1j * rng.standard_normal(D)) for _ in range(n)]


@pytest.mark.parametrize("with_prior,refined", [(False, False), (True, False), (False, True)])
def test_coefficient_update_maximises_q(with_prior, refined):
    """The closed form of eq. (17) is the maximiser of Q (eq. (14)) over a: Q written out term
    by term is lower at every perturbation and its finite-difference gradient vanishes.  Also for
    a refined window of off-grid angles (Q then rotates by explicit cos/sin of k theta_i)."""
    p = _problem(K=3, Q=2, N=6, L=8, window=(-2, 5))
    if refined:
        p["offs"] = _refined(8, 5, 0.41)
    D = p["D"]
    gai = np.linspace(0.3, 2.0, D) if with_prior else None
    w, _, _ = oracle.estep(p["V"], p["a0"], p["rho"], p["s2"], p["kbar"], p["L"], p["offs"])
    a1, _ = oracle.mstep_a(p["V"], w, p["kbar"], p["L"], p["offs"], p["s2"], gai)
    q = lambda a: oracle.q_function(a, p["rho"], w, p["V"], p["kbar"], p["L"], p["offs"],
                                    p["s2"], gamma_a_inv=gai)
    q0 = q(a1)
    rng = np.random.default_rng(1)
    for dvec in _perturb_dirs(D, rng):
        assert q(a1 + 1e-3 * dvec) < q0
    h = 1e-5
    for d in range(D):
        for unit in (1.0, 1j):
            e = np.zeros(D, complex)
            e[d] = unit * h
            g = (q(a1 + e) - q(a1 - e)) / (2 * h)
            assert abs(g) <= 1e-6 * max(1.0, abs(q0))


def test_rho_update_maximises_its_lagrangian():
    """(W + gamma rho_bar)/sum maximises sum W log rho + gamma sum rho_bar log rho on the simplex
    (App. C), and reduces to W/sum W for gamma = 0 and to rho_bar for gamma -> inf."""
    rng = np.random.default_rng(2)
    Wt = rng.uniform(0, 30, 9)
    rb = rng.uniform(0, 1, 9)
    rb /= rb.sum()
    for gamma in (0.0, 1.0, 100.0):
        r = oracle.mstep_rho(Wt, rb, gamma)
        f = lambda x: float(np.sum(Wt * np.log(x)) + gamma * np.sum(rb * np.log(x)))
        for _ in range(20):
            dlt = rng.standard_normal(9)
            dlt -= dlt.mean()                     # stay on sum = 1
            x = r + 1e-3 * dlt / np.abs(dlt).max() * r.min()
            assert f(x) < f(r)
    assert np.allclose(oracle.mstep_rho(Wt, rb, 0.0), Wt / Wt.sum(), atol=1e-15)
    assert np.allclose(oracle.mstep_rho(Wt, rb, 1e15), rb, atol=1e-12)


def test_single_offset_window_gives_mean():
    p = _problem(N=11, window=(0, 1))
    w, _, _ = oracle.estep(p["V"], p["a0"], [1.0], p["s2"], p["kbar"], p["L"], p["offs"])
    a1, _ = oracle.mstep_a(p["V"], w, p["kbar"], p["L"], p["offs"], p["s2"])
    assert np.allclose(a1, p["V"].mean(axis=0), atol=1e-15)
    p = _problem(N=11, window=(3, 1))
    w, _, _ = oracle.estep(p["V"], p["a0"], [1.0], p["s2"], p["kbar"], p["L"], p["offs"])
    a1, _ = oracle.mstep_a(p["V"], w, p["kbar"], p["L"], p["offs"], p["s2"])
    back = np.exp(2j * np.pi * p["kbar"] * 3 / p["L"])
    assert np.allclose(a1, (back[None, :] * p["V"]).mean(axis=0), atol=1e-14)


def test_noiseless_first_step_closed_form_and_exact_recovery():
    """Noiseless data, full search, uniform rho: every posterior row is a circular shift of
    p_m = softmax_m(2 Re<a, R_m a0>/s2), so a_1 = (sum_m p_m e^{+i k theta_m}) o a.  As s2 -> 0
    this is R_{-m*} a: exact recovery up to a global rotation."""
    K, Q, L, N = 4, 3, 10, 25
    p = _problem(K=K, Q=Q, N=N, L=L)
    a, kbar = p["a"], p["kbar"]
    V = np.stack([a * np.exp(-2j * np.pi * kbar * li / L) for li in p["lmb"][:N]])
    offs = oracle.offsets(0, L)
    rho = np.full(L, 1.0 / L)
    for s2 in (0.3, 1e-6):
        lg = []
        for m in range(L):
            rot = p["a0"] * np.exp(-2j * np.pi * kbar * m / L)
            lg.append(2 * float(np.sum(np.conj(a) * rot).real) / s2)
        lg = np.array(lg)
        pm = np.exp(lg - lg.max())
        pm /= pm.sum()
        expect = sum(pm[m] * np.exp(2j * np.pi * kbar * m / L) for m in range(L)) * a
        w, _, _ = oracle.estep(V, p["a0"], rho, s2, kbar, L, offs)
        a1, _ = oracle.mstep_a(V, w, kbar, L, offs, s2)
        assert np.allclose(a1, expect, atol=1e-12 * np.abs(a).max())
    assert oracle.relative_error(a1, a, kbar, L) <= 1e-12


def test_full_window_in_any_order_is_plain_em():
    """A window covering all L rotations, listed from -L/2, is plain EM over 0..L-1."""
    p = _problem(N=30, L=10)
    rho = np.full(10, 0.1)
    plain = oracle.em_run(p["V"], p["a0"], rho, p["s2"], p["kbar"], 10, oracle.offsets(0, 10), 6)
    shifted = oracle.em_run(p["V"], p["a0"], rho, p["s2"], p["kbar"], 10, oracle.offsets(-5, 10), 6)
    assert np.allclose(plain[0], shifted[0], atol=1e-13)
    assert np.allclose(plain[1], np.roll(shifted[1], -5), atol=1e-13)
    assert all(abs(x["ll"] - y["ll"]) <= 1e-10 * abs(x["ll"]) for x, y in zip(plain[2], shifted[2]))


# ---------------------------------------------------------------- EM monotonicity

def test_loglik_never_decreases_plain_em():
    p = _problem(K=6, Q=4, N=300, L=24, snr=0.3, seed=5)
    rho = np.full(24, 1 / 24)
    _, _, hist = oracle.em_run(p["V"], p["a0"], rho, p["s2"], p["kbar"], 24, oracle.offsets(0, 24), 40)
    ll = [h["ll"] for h in hist]
    assert all(b >= a - 1e-9 * abs(a) for a, b in zip(ll, ll[1:]))
    assert ll[-1] > ll[0]


def test_map_objective_never_decreases_with_priors():
    p = _problem(K=6, Q=4, N=300, L=24, snr=0.3, seed=6, window=(-4, 9))
    rb = np.exp(-0.5 * (np.arange(-4, 5) / 2.0) ** 2)
    rb /= rb.sum()
    gai = 1.0 / (16 * np.exp(-p["kbar"] / 8.0) ** 2)
    _, _, hist = oracle.em_run(p["V"], p["a0"], rb, p["s2"], p["kbar"], 24, p["offs"], 40,
                               rho_bar=rb, gamma=50.0, gamma_a_inv=gai)
    J = [h["J"] for h in hist]
    assert all(b >= a - 1e-9 * abs(a) for a, b in zip(J, J[1:]))


# ---------------------------------------------------------------- stopping rule, error metric

def test_stop_metric_and_relative_error_are_rotation_invariant():
    p = _problem()
    for l in (0, 3, 11):
        ar = oracle.rotate(p["a"], p["kbar"], l, p["L"])
        assert oracle.stop_metric(ar, p["a"], p["kbar"], p["L"]) <= 1e-28
        assert oracle.relative_error(ar, p["a"], p["kbar"], p["L"]) <= 1e-15
    d = 0.01 * np.ones(p["D"])
    m = oracle.stop_metric(p["a"] + d, p["a"], p["kbar"], p["L"])
    assert abs(m - np.sum(d ** 2)) <= 1e-15


# ---------------------------------------------------------------- gradients (Fisher identity)

@pytest.mark.parametrize("W", [16, 7])
def test_gradients_match_central_finite_differences(W):
    """Gradient w.r.t. Re a, Im a, sigma^2 and the prior logits eta (rho = softmax(eta)) against
    FP64 central differences of the log-likelihood, at N=200, D=32, L=16."""
    w4 = wl.WORKLOADS["c4fd"]
    a_true = wl.image(w4, 0)
    V = wl.observations(w4, 0)
    lo = 0 if W == 16 else -(W // 2)
    offs = oracle.offsets(lo, W)
    rng = np.random.default_rng(4)
    eta = rng.standard_normal(W) * 0.3
    rho = np.exp(eta - eta.max())
    rho /= rho.sum()
    a = V.mean(axis=0) + 0.05 * a_true
    s2 = wl.noise_variance(a_true, w4.snr) * 1.3
    kbar = w4.kbar
    ll, ga, gs, ge = oracle.grad_loglik(V, a, s2, rho, kbar, w4.L, offs)

    def LL(a_, s2_, eta_):
        r_ = np.exp(eta_ - eta_.max())
        return oracle.loglik(V, a_, r_ / r_.sum(), s2_, kbar, w4.L, offs)

    h = 1e-6 * float(np.abs(a).max())
    for d in range(0, w4.D, 3):
        for unit, comp in ((1.0, ga[d].real), (1j, ga[d].imag)):
            e = np.zeros(w4.D, complex)
            e[d] = unit * h
            fd = (LL(a + e, s2, eta) - LL(a - e, s2, eta)) / (2 * h)
            assert abs(fd - comp) <= 1e-6 * max(1.0, abs(comp)), (d, unit)
    hs = 1e-6 * s2
    fd = (LL(a, s2 + hs, eta) - LL(a, s2 - hs, eta)) / (2 * hs)
    assert abs(fd - gs) <= 1e-6 * max(1.0, abs(gs))
    for i in range(W):
        e = np.zeros(W)
        e[i] = 1e-6
        fd = (LL(a, s2, eta + e) - LL(a, s2, eta - e)) / 2e-6
        assert abs(fd - ge[i]) <= 1e-5 * max(1.0, abs(ge[i]))


def test_gradient_step_equals_em_step():
    """With no image prior, a + (s2 / 2N) dLL/da is the EM coefficient update."""
    p = _problem(N=50, window=(-3, 7))
    _, ga, _, _ = oracle.grad_loglik(p["V"], p["a0"], p["s2"], p["rho"], p["kbar"], p["L"], p["offs"])
    it = oracle.em_iteration(p["V"], p["a0"], p["rho"], p["s2"], p["kbar"], p["L"], p["offs"])
    assert np.allclose(p["a0"] + p["s2"] / (2 * 50) * ga, it["a"], atol=1e-13)


# ---------------------------------------------------------------- learned prior (eq. 22, Alg.)

def test_histogram_is_categorical_mle():
    w3 = wl.WORKLOADS["c3"]
    err = wl.prior_error_draws(w3, 0, 20000)
    lo, W = w3.window
    rb, cnt, call = oracle.histogram_prior(err, w3.L, lo, W)
    assert abs(rb.sum() - 1.0) <= 1e-15
    bc = np.bincount(np.mod(err.astype(np.int64), w3.L), minlength=w3.L)
    assert np.array_equal(call, bc)
    inside = np.array([(e - lo) % w3.L < W for e in err.astype(np.int64)])
    idx = (err.astype(np.int64)[inside] - lo) % w3.L
    f = lambda x: float(np.sum(np.log(x[idx])))
    rng = np.random.default_rng(0)
    base = f(rb)
    for _ in range(20):
        dlt = rng.standard_normal(W)
        dlt -= dlt.mean()
        assert f(rb + 1e-4 * dlt / np.abs(dlt).max() * rb[rb > 0].min()) < base


# ---------------------------------------------------------------- validation semantics

def test_validation_mirrors_library():
    with pytest.raises(OracleInvalid):
        oracle.validate(0, 4, 4, 10, 0, 10, 1.0)
    with pytest.raises(OracleInvalid):
        oracle.validate(5, 4, 4, 10, 0, 11, 1.0)
    with pytest.raises(OracleInvalid):
        oracle.validate(5, 4, 4, 10, 0, 10, -1.0)
    with pytest.raises(OracleInvalid):
        oracle.validate(5, 4, 4, 10, 0, 3, 1.0, prior=[0.5, -0.1, 0.6])
    with pytest.raises(OracleInvalid):
        oracle.validate(5, 4, 4, 10, 0, 3, 1.0, prior=[0.0, 0.0, 0.0])
    V = np.ones((2, 3), complex)
    V[1, 2] = np.nan
    with pytest.raises(OracleNonFinite):
        oracle.validate(2, 1, 3, 10, 0, 10, 1.0, V=V)


def test_map_objective_is_stationary_at_em_fixed_point():
    """At a fixed point of MAP-EM (image prior Gamma_a and KL prior on rho), the finite-difference
    gradient of the MAP objective J (log posterior up to constants, §II-B eq. (12) with eq. (23)) in
    a and in the logits of rho vanishes."""
    p = _problem(K=3, Q=3, N=80, L=12, snr=3.0, seed=8, window=(-3, 7))
    rb = np.exp(-0.5 * (np.arange(-3, 4) / 1.5) ** 2)
    rb /= rb.sum()
    gai = 1.0 / (0.6 * np.exp(-p["kbar"] / 2.0)) ** 2
    gamma = 20.0
    a, rho, hist = oracle.em_run(p["V"], p["a0"], rb, p["s2"], p["kbar"], p["L"], p["offs"], 3000,
                                 tol=1e-26, rho_bar=rb, gamma=gamma, gamma_a_inv=gai)
    assert hist[-1]["stop"] < 1e-20

    def J(a_, eta_):
        r_ = np.exp(eta_ - eta_.max())
        r_ /= r_.sum()
        ll = oracle.loglik(p["V"], a_, r_, p["s2"], p["kbar"], p["L"], p["offs"])
        return oracle.objective(ll, r_, rb, gamma, a_, gai)

    eta = np.log(rho)
    h = 1e-6
    _, ga, _, _ = oracle.grad_loglik(p["V"], a, p["s2"], rho, p["kbar"], p["L"], p["offs"])
    scale = np.abs(ga).max()          # size of the likelihood part alone (cancelled by the prior)
    assert scale > 1.0
    for d in range(p["D"]):
        for unit in (1.0, 1j):
            e = np.zeros(p["D"], complex)
            e[d] = unit * h
            assert abs(J(a + e, eta) - J(a - e, eta)) / (2 * h) <= 1e-5 * scale
    for i in range(len(eta)):
        e = np.zeros(len(eta))
        e[i] = h
        assert abs(J(a, eta + e) - J(a, eta - e)) / (2 * h) <= 1e-5 * max(1.0, gamma)


# ---------------------------------------------------------------- argmax and top-two margin (eq. 15)

def _argmax_margin_by_definition(w):
    """The most probable rotation and the probability gap, read off each row by a plain scan:
    the first index whose weight is not exceeded by any other (the lowest index wins a tie),
    and that weight minus the largest weight at any other index (0 when the maximum is shared;
    with one rotation there is no other index and the gap is the weight itself)."""
    idx, gap = [], []
    for row in np.asarray(w, dtype=np.float64):
        best = 0
        for i in range(1, len(row)):
            if row[i] > row[best]:
                best = i
        other = [row[i] for i in range(len(row)) if i != best]
        idx.append(best)
        gap.append(row[best] - max(other) if other else row[best])
    return np.array(idx), np.array(gap)


def _argmax_margin_failures(fn):
    """Names of the checks that ``fn`` fails; an empty list means it is a correct argmax/margin."""
    fails = []
    rng = np.random.default_rng(7)

    def agree(name, w):
        i1, g1 = fn(w)
        i2, g2 = _argmax_margin_by_definition(w)
        if not (np.array_equal(np.asarray(i1), i2) and np.allclose(g1, g2, rtol=0, atol=1e-15)):
            fails.append(name)

    # rows of a softmax (what the E-step produces), distinct entries almost surely
    x = rng.standard_normal((40, 9))
    agree("random rows", np.exp(x) / np.exp(x).sum(axis=1, keepdims=True))
    # ties at the maximum: lowest index, zero gap
    agree("two-way tie", np.array([[0.1, 0.4, 0.1, 0.4], [0.45, 0.1, 0.0, 0.45]]))
    agree("uniform row", np.full((3, 5), 0.2))
    # one rotation only (W = 1): the gap is the weight itself
    agree("single rotation", np.array([[1.0], [0.25]]))
    # one-hot rows: the hot index and a gap of one (noiseless posteriors)
    agree("one-hot", np.eye(6)[[3, 0, 5]])
    # a maximum in the last column and a runner-up equal to the next value (sorted-order traps)
    agree("max last", np.array([[0.1, 0.2, 0.3, 0.4], [0.3, 0.3, 0.0, 0.4]]))
    # closed forms that do not go through the scan above
    w = np.array([[0.2, 0.5, 0.3], [0.6, 0.1, 0.3], [0.5, 0.0, 0.5]])
    i, g = fn(w)
    if list(np.asarray(i)) != [1, 0, 0] or not np.allclose(g, [0.2, 0.3, 0.0], atol=1e-15):
        fails.append("closed form")
    return fails


def test_argmax_margin_pinned():
    """Reading of the argmax rule: the lowest window index wins a tie, and the margin is the gap
    between the two largest posteriors (eq. (15) gives the posteriors; a rotation whose weight is
    not exceeded by any other is the most probable one).  The pin is a plain scan of each row plus
    closed forms on hand-made rows."""
    assert _argmax_margin_failures(oracle.argmax_margin) == []


def _highest_index_wins(w):
    w = np.asarray(w)
    idx = w.shape[1] - 1 - np.argmax(w[:, ::-1], axis=1)
    return idx, oracle.argmax_margin(w)[1]


def _ratio_margin(w):
    idx, _ = oracle.argmax_margin(w)
    top2 = np.sort(w, axis=1)[:, -2:] if w.shape[1] > 1 else np.concatenate([w, w], axis=1)
    with np.errstate(divide="ignore", invalid="ignore"):
        return idx, top2[:, 1] / top2[:, 0]


def _single_rotation_zero(w):
    idx, g = oracle.argmax_margin(w)
    return idx, (np.zeros_like(g) if w.shape[1] == 1 else g)


def _distinct_runner_up(w):
    """Takes the runner-up as the largest value below the maximum (a tie would give a gap > 0)."""
    idx = np.argmax(w, axis=1)
    gaps = []
    for row in w:
        m = row.max()
        below = row[row < m]
        gaps.append(m - (below.max() if below.size else 0.0))
    return idx, np.array(gaps)


@pytest.mark.parametrize("planted", [_highest_index_wins, _ratio_margin, _single_rotation_zero,
                                     _distinct_runner_up])
def test_argmax_margin_pin_rejects_planted_mistakes(planted):
    """Plausible mistakes in the argmax rule fail the pin above."""
    assert _argmax_margin_failures(planted) != []
