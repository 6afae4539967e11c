"""The seeded generator: determinism, chunk regeneration and the model's statistics (CPU)."""
import numpy as np

import workloads as wl


def test_snr_is_exact_for_realised_image():
    for name in ("c1", "c2", "c5"):
        w = wl.WORKLOADS[name]
        a = wl.image(w, 0)
        s2 = wl.noise_variance(a, w.snr)
        assert abs(np.vdot(a, a).real / (w.D * s2) - w.snr) <= 1e-12


def test_row_ranges_regenerate_identically_across_chunks():
    w = wl.WORKLOADS["c1"].replace(N=140_000, K=2, Q=2)
    full = wl.observations(w, 3, 65_000, 66_100)
    part = wl.observations(w, 3, 65_536, 65_540)
    assert np.array_equal(full[536:540], part)
    l = wl.rotations(w, 3, 65_000, 66_100)
    assert np.array_equal(l[536:540], wl.rotations(w, 3, 65_536, 65_540))


def test_noise_and_rotation_statistics():
    w = wl.WORKLOADS["c3"].replace(N=20000)
    a = wl.image(w, 1)
    V = wl.observations(w, 1, a=a)
    l = wl.rotations(w, 1)
    clean = a[None, :] * np.exp(-2j * np.pi * ((w.kbar[None, :] * l[:, None]) % w.L) / w.L)
    eps = V - clean
    s2 = wl.noise_variance(a, w.snr)
    assert abs(np.mean(np.abs(eps) ** 2) / s2 - 1) < 0.01
    assert abs(np.mean(eps.real ** 2) / (s2 / 2) - 1) < 0.01
    assert abs(np.std(l) / w.rot_std_steps - 1) < 0.03
    assert l.min() >= -w.L // 2 and l.max() < w.L // 2


def test_prior_draws_are_seeded_and_wrapped():
    w = wl.WORKLOADS["c5"]
    e1 = wl.prior_error_draws(w, 0, 70000)
    e2 = wl.prior_error_draws(w, 0, 70000)
    assert np.array_equal(e1, e2) and e1.dtype == np.int32
    assert e1.min() >= -w.L // 2 and e1.max() < w.L // 2
