"""Closed-form special cases used to pin the oracle (tests only).

* Rank-one sine mode in 1-D: sin(pi x_j) is a common eigenvector of the P1
  stiffness and mass matrices on a uniform grid, so for F1 = c sin(pi x) the
  space-time solution is U = sin(pi x) w^T with a scalar lower-bidiagonal
  recurrence for w.
* Manufactured continuous solution u(t, x) = sin(pi x) omega(t) of
  u_t - u_xx = f (Sec. 2, heat equation with a(u,v) = (u', v')), used to
  check O(h^2 + dt^2) convergence of the discrete scheme.
"""
from __future__ import annotations

import math

import numpy as np


def sine_mode_eigs_1d(n: int, mu: float = 1.0, m: int = 1):
    """(kappa_m, nu_m): eigenvalues of 1-D P1 stiffness / mass for mode m.

    Textbook eigenvalues of tridiagonal Toeplitz matrices:
    (mu/h) tridiag(-1, 2, -1) -> (2 mu / h)(1 - cos m pi h);
    (h/6) tridiag(1, 4, 1)    -> (h/3)(2 + cos m pi h).
    """
    h = 1.0 / (n + 1)
    c = math.cos(m * math.pi * h)
    return 2.0 * mu / h * (1.0 - c), h / 3.0 * (2.0 + c)


def sine_mode_solution_1d(n: int, mu: float, Dt, Mt, F2, load_scale: float):
    """Exact U for F1 = load_scale * sin(pi x_j) (rank one).

    U = s w^T with s_j = sin(pi x_j) and (nu_1 Dt + kappa_1 Mt) w = load_scale F2.
    """
    kappa, nu = sine_mode_eigs_1d(n, mu, 1)
    h = 1.0 / (n + 1)
    s = np.sin(math.pi * h * np.arange(1, n + 1))
    A = nu * np.asarray(Dt) + kappa * np.asarray(Mt)
    w = np.linalg.solve(A, load_scale * np.asarray(F2)[:, 0])
    return np.outer(s, w)


def manufactured_omega(c: np.ndarray):
    """omega(t) = sum_i c_i t^(i+1) (so omega(0) = 0) and g = omega' + pi^2 omega.

    Returns callables (omega, G) where G is an antiderivative of g, so that
    integrals of g over time intervals are exact.
    """
    c = np.asarray(c, dtype=float)
    pi2 = math.pi ** 2

    def omega(t):
        return sum(c[i] * t ** (i + 1) for i in range(len(c)))

    def G(t):
        # integral of omega' is omega; integral of pi^2 omega is pi^2 sum c_i t^(i+2)/(i+2)
        return omega(t) + pi2 * sum(c[i] * t ** (i + 2) / (i + 2) for i in range(len(c)))

    return omega, G
