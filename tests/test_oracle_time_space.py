"""Pins of the oracle's discretisation matrices (CPU only)."""
import math

import numpy as np
import pytest

from oracle import fem
from oracle.closed_form import sine_mode_eigs_1d


@pytest.mark.parametrize("tag", ["uniform", "graded"])
def test_time_matrices_match_hand_derivation(golden, tag):
    g = golden("time_matrices.txt")
    t = g[f"nodes_{tag}"][0]
    Dt, Mt = fem.time_matrices(t, window=None)      # every (test, trial) pair integrated
    np.testing.assert_allclose(Dt, g[f"Dt_{tag}"], atol=1e-15)
    np.testing.assert_allclose(Mt, g[f"Mt_{tag}"], atol=1e-15)


def test_time_window_equals_full_quadrature():
    t = np.cumsum(np.r_[0.0, np.random.default_rng(0).uniform(0.5, 1.5, 17)])
    A = fem.time_matrices(t, window=None)
    B = fem.time_matrices(t)
    for a, b in zip(A, B):
        np.testing.assert_array_equal(a, b)
    fem.bidiagonals(*B)                              # raises unless lower bidiagonal


def test_element_matrices_textbook(golden):
    g = golden("p1_element_matrices.txt")
    Ke, Me = fem.p1_interval_element(0.5)
    np.testing.assert_allclose(Ke, g["K_interval_h0.5"], rtol=1e-14)
    np.testing.assert_allclose(Me, g["M_interval_h0.5"], rtol=1e-14)
    h = 0.25
    Kt, Mt = fem.p1_triangle_element(np.array([[0, 0], [h, 0], [h, h]], float))
    np.testing.assert_allclose(Kt, g["K_triangle_h0.25"], atol=1e-15)
    np.testing.assert_allclose(Mt, g["M_triangle_h0.25"], rtol=1e-14)


def test_1d_operators_sine_eigenpairs():
    n, mu = 31, 0.7
    K, M = fem.p1_1d(n, mu)
    x = np.arange(1, n + 1) / (n + 1)
    for m in (1, 2, 7, n):
        q = np.sin(m * np.pi * x)
        kap, nu = sine_mode_eigs_1d(n, mu, m)
        np.testing.assert_allclose(K @ q, kap * q, atol=1e-12 * kap)
        np.testing.assert_allclose(M @ q, nu * q, atol=1e-14)


def test_2d_stiffness_sine_eigenpairs_and_linear_kernel():
    n, mu = 15, 1.3
    K, M = fem.p1_2d_courant(n, mu)
    h = 1.0 / (n + 1)
    x = np.arange(1, n + 1) * h
    X, Y = np.meshgrid(x, x, indexing="xy")
    for m1, m2 in ((1, 1), (2, 5), (n, 3)):
        q = (np.sin(m1 * np.pi * X) * np.sin(m2 * np.pi * Y)).ravel()
        lam = mu * (4 - 2 * math.cos(m1 * np.pi * h) - 2 * math.cos(m2 * np.pi * h))
        np.testing.assert_allclose(K @ q, lam * q, atol=1e-12 * lam)
    # linear functions are annihilated by K and reproduced by M (times h^2) on rows
    # whose stencil does not touch the boundary
    lin = (0.3 + 2.0 * X - 1.5 * Y).ravel()
    inner = np.zeros((n, n), bool)
    inner[1:-1, 1:-1] = True
    inner = inner.ravel()
    np.testing.assert_allclose((K @ lin)[inner], 0.0, atol=1e-12)
    np.testing.assert_allclose((M @ lin)[inner], h * h * lin[inner], rtol=1e-13)
    assert abs(K - K.T).max() == 0 and abs(M - M.T).max() == 0


def _hat2d(s, t):
    """Courant-triangulation hat (SW-NE diagonals) in units of h, centred at 0."""
    return np.maximum(0.0, 1.0 - np.maximum(np.maximum(abs(s), abs(t)), abs(s - t)))


def test_2d_mass_against_brute_force_quadrature():
    """(phi_i, phi_j) from a fine midpoint rule over the hat functions themselves."""
    n = 7
    K, M = fem.p1_2d_courant(n)
    h = 1.0 / (n + 1)
    N = 600                                           # sub-cells per mesh width
    u = (np.arange(-2 * N, 2 * N) + 0.5) / N          # local coordinates in [-2, 2]
    S, T = np.meshgrid(u, u, indexing="xy")
    ci = 3 + n * 3                                    # interior node (3, 3)
    phi_i = _hat2d(S, T)
    for di, dj in ((0, 0), (1, 0), (0, 1), (1, 1), (-1, -1), (1, -1), (-1, 1)):
        val = (phi_i * _hat2d(S - di, T - dj)).sum() * (h / N) ** 2
        np.testing.assert_allclose(M[ci, ci + di + n * dj], val, rtol=2e-5, atol=1e-12)


def test_3d_operators_closed_forms():
    n, mu = 7, 0.9
    K, M = fem.q1_3d_7pt(n, mu)
    h = 1.0 / (n + 1)
    x = np.arange(1, n + 1) * h
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")     # x fastest after ravel
    for m in ((1, 1, 1), (2, 3, 5), (7, 1, 4)):
        q = (np.sin(m[0] * np.pi * X) * np.sin(m[1] * np.pi * Y) * np.sin(m[2] * np.pi * Z)).ravel()
        th = [mi * np.pi * h for mi in m]
        lamK = mu * h * sum(2 - 2 * math.cos(a) for a in th)
        lamM = np.prod([h / 6 * (4 + 2 * math.cos(a)) for a in th])
        np.testing.assert_allclose(K @ q, lamK * q, atol=1e-12 * lamK)
        np.testing.assert_allclose(M @ q, lamM * q, atol=1e-14 * lamM * 1e3)
    assert K.nnz <= 7 * n ** 3
    centre = (n // 2) * (1 + n + n * n)
    assert K[centre, centre] == pytest.approx(6 * mu * h)
