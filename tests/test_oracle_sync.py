"""Pins of the FP64 Synchronize-and-Match oracle (CPU only): explicit rotation, exact noiseless
relative rotations, recovery up to one global rotation by the power method, brute-force nearest
neighbours."""
import math

import numpy as np
import pytest

import oracle


def _data(K=4, Q=3, N=12, L=12, noise=0.3, seed=0):
    rng = np.random.default_rng(seed)
    D = K * Q
    kbar = np.repeat(np.arange(K), Q)
    a = (rng.standard_normal(D) + 1j * rng.standard_normal(D)) / np.sqrt(2 * (1 + kbar))
    l = rng.integers(0, L, N)
    V = np.stack([a * np.exp(-2j * np.pi * kbar * li / L) for li in l])
    V = V + noise * (rng.standard_normal((N, D)) + 1j * rng.standard_normal((N, D))) / np.sqrt(2)
    return V, a, kbar, l


def test_relative_rotations_match_explicit_rotation():
    V, _, kbar, _ = _data(N=6)
    rel, f = oracle.relative_rotations(V, kbar, 12)
    assert np.array_equal(rel, oracle.relative_rotations_brute(V, kbar, 12))
    # f is the correlation Re <v_i, R_l v_j> written out
    for (i, j, l) in [(0, 1, 3), (2, 5, 11), (4, 4, 0)]:
        rot = V[j] * np.exp(-2j * np.pi * kbar * l / 12)
        assert abs(f[i, j, l] - float(np.real(np.vdot(V[i], rot)))) <= 1e-12 * np.abs(f).max()


def test_noiseless_relative_rotations_are_the_differences():
    V, _, kbar, l = _data(N=10, L=16, noise=0.0)
    rel, _ = oracle.relative_rotations(V, kbar, 16)
    assert np.array_equal(rel, np.mod(l[:, None] - l[None, :], 16))


def test_ppm_recovers_noiseless_rotations_up_to_a_global_rotation():
    V, a, kbar, l = _data(N=15, L=20, noise=0.0)
    rel, _ = oracle.relative_rotations(V, kbar, 20)
    th = oracle.ppm(rel, 20, 5)
    d = np.angle(np.exp(1j * (th - 2 * np.pi * l / 20)))     # theta_hat - theta, wrapped
    assert np.max(np.abs(np.angle(np.exp(1j * (d - d[0]))))) <= 1e-12
    Va = oracle.align(V, kbar, th)                            # all rows are one rotated image
    assert np.max(np.abs(Va - Va[0])) <= 1e-12 * np.abs(a).max()
    c = -d[0]                                                 # ... a rotated by the global shift
    assert np.max(np.abs(Va[0] - a * np.exp(-1j * kbar * c))) <= 1e-12 * np.abs(a).max()


def test_ppm_first_iteration_is_the_phase_of_the_row_sums():
    V, _, kbar, _ = _data(N=9)
    rel, _ = oracle.relative_rotations(V, kbar, 12)
    th = oracle.ppm(rel, 12, 1)
    for i in range(9):
        s = sum(complex(math.cos(2 * math.pi * rel[i, j] / 12), math.sin(2 * math.pi * rel[i, j] / 12))
                for j in range(9))
        assert abs(math.remainder(th[i] - math.atan2(s.imag, s.real), 2 * math.pi)) <= 1e-12


def test_nearest_neighbours_by_brute_force():
    V, _, _, _ = _data(N=20, noise=0.5, seed=3)
    P = 7
    nn, d = oracle.nearest_neighbours(V, P)
    for i in range(20):
        best, arg = math.inf, -1
        for n in range(P):
            if n == i:
                continue
            dist = float(np.sum(np.abs(V[i] - V[n]) ** 2))
            assert abs(dist - d[i, n]) <= 1e-12 * max(1.0, dist)
            if dist < best:
                best, arg = dist, n
        assert nn[i] == arg


def test_synchronize_and_match_noiseless_exact_up_to_global_rotation():
    """Noiseless data whose subset S_P holds every rotation class at least twice: every
    observation matches an identical one and gets its exact rotation up to one global shift."""
    L, P, N = 8, 24, 60
    V, a, kbar, l = _data(N=N, L=L, noise=0.0, seed=5)
    l[:P] = np.arange(P) % L                                  # each class three times in S_P
    V = np.stack([a * np.exp(-2j * np.pi * kbar * li / L) for li in l])
    th, phi, rel, nn = oracle.synchronize_and_match(V, kbar, L, P, 10)
    assert all(nn[i] != i for i in range(P))
    assert np.array_equal(l[nn], l)
    d = np.angle(np.exp(1j * (th - 2 * np.pi * l / L)))
    assert np.max(np.abs(np.angle(np.exp(1j * (d - d[0]))))) <= 1e-12


@pytest.mark.parametrize("l", [0, 3, 7])
def test_align_undoes_a_grid_rotation(l):
    V, a, kbar, _ = _data(N=1, noise=0.0)
    v = a * np.exp(-2j * np.pi * kbar * l / 12)
    assert np.max(np.abs(oracle.align(v[None], kbar, np.array([2 * np.pi * l / 12]))[0] - a)) \
        <= 1e-14 * np.abs(a).max()


def test_global_rotation_and_centred_bins():
    """The centring step finds an injected global rotation exactly; errors placed in the middle
    of known bins come back as those bins (mod L)."""
    V, a, kbar, _ = _data(N=1, noise=0.0, L=24)
    for c in (0, 5, 17):
        abar = a * np.exp(2j * np.pi * kbar * c / 24)          # R_{-c} a
        assert oracle.global_rotation(a, abar, kbar, 24) == c
    rng = np.random.default_rng(1)
    th = rng.uniform(-np.pi, np.pi, 50)
    m = rng.integers(-30, 30, 50)
    th_hat = th + 2 * np.pi * (7 + m + 0.5) / 24
    assert np.array_equal(oracle.centred_error_bins(th_hat, th, 7, 24), np.mod(m, 24))


def test_aligned_mean_of_synchronized_noiseless_data_is_the_rotated_image():
    V, a, kbar, l = _data(N=30, L=12, noise=0.0, seed=2)
    th = 2 * np.pi * l / 12 + 0.3                              # exact up to a global 0.3 rad
    assert np.max(np.abs(oracle.aligned_mean(V, kbar, th) - a * np.exp(0.3j * kbar))) <= 1e-13


def test_continuous_relative_error_removes_any_global_rotation():
    V, a, kbar, _ = _data(N=1, noise=0.0, seed=4)
    for th in (0.0, 0.123456, 2.5, -1.0):
        assert oracle.relative_error_continuous(a * np.exp(-1j * kbar * th), a, kbar) <= 1e-9
    b = a + 0.01 * np.exp(0.3j * kbar)
    assert oracle.relative_error_continuous(b, a, kbar) <= np.linalg.norm(b - a) / np.linalg.norm(a)
