"""Checks of the seeded input generators (CPU only)."""
import numpy as np
from scipy import integrate

import workloads as wl


def test_sine_load_is_exact_integral():
    n = 15
    h = 1.0 / (n + 1)
    F = wl.sine_load_1d(n)
    for j in (0, 7, 14):
        xj = (j + 1) * h
        hat = lambda x: max(0.0, 1 - abs(x - xj) / h)
        val, _ = integrate.quad(lambda x: np.sin(np.pi * x) * hat(x), xj - h, xj + h, points=[xj])
        assert abs(F[j] - val) < 1e-14


def test_interval_integrals_match_quadrature():
    rng = np.random.default_rng(0)
    a, b = rng.normal(size=9), rng.normal(size=9)
    t = wl.time_grid(50, 1.0)
    th = lambda s: sum((a[m] * np.cos(2 * np.pi * m * s) + b[m] * np.sin(2 * np.pi * m * s)) / (1 + m) ** 2
                       for m in range(9))
    F = wl.trig_series_interval_integrals(a, b, t)
    ref = [integrate.quad(th, t[i], t[i + 1], epsabs=1e-15)[0] for i in range(50)]
    np.testing.assert_allclose(F, ref, rtol=1e-11, atol=1e-16)
    c = rng.normal(size=4)
    G = wl.cubic_interval_integrals(c, t)
    ref = [integrate.quad(lambda s: c[0] + c[1] * s + c[2] * s * s + c[3] * s ** 3, t[i], t[i + 1])[0] for i in range(50)]
    np.testing.assert_allclose(G, ref, rtol=1e-12)


def test_generators_are_seeded_and_shaped():
    w1, w2 = wl.heat_2d_bumps(n=31, nt=64, p=2, seed=2), wl.heat_2d_bumps(n=31, nt=64, p=2, seed=2)
    np.testing.assert_array_equal(w1.F1, w2.F1)
    np.testing.assert_array_equal(w1.F2, w2.F2)
    assert w1.F1.shape == (31 * 31, 2) and w1.F2.shape == (64, 2)
    assert w1.F1.flags.f_contiguous and w1.F2.flags.f_contiguous
    w3 = wl.heat_3d_separable(n=7, nt=8, p=4)
    assert w3.F1.shape == (343, 4)
    c1 = wl.heat_1d_sine()
    assert c1.nh == 127 and c1.nt == 128 and c1.p == 1
