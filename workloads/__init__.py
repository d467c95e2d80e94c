"""Seeded synthetic inputs for the space-time heat problem.

This module is shared by the CPU oracle tests, the GPU parity tests and the
benchmark.  It produces only *inputs*: grid descriptions, the spatial load
factor ``F1`` (Nh x P) and the temporal load factor ``F2`` (Nt x P) of the
low-rank right-hand side ``F = F1 F2^T`` (Sec. 3, eq. (EIM) and the load
definition that follows it: ``F[j, l] = sum_p (theta_p, tau^l)(f_p, phi_j)``).
It holds no operator, solver or projection arithmetic: no stiffness or mass
matrix, no time matrix, no Krylov step.

Conventions
-----------
* Uniform grids on the unit interval / square / cube with homogeneous
  Dirichlet conditions; only interior nodes are unknowns, numbered
  lexicographically with x fastest.  ``h = 1/(n+1)``.
* Time grid ``t^l = l * T / Nt``, l = 0..Nt; column l-1 of ``F2`` is the
  integral of ``theta_p`` over ``I^l = (t^{l-1}, t^l)``.
* Random numbers come from ``numpy.random.default_rng(seed)`` (PCG64) and are
  drawn in the order documented in each function.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "Workload", "node_coords", "time_grid", "sine_load_1d",
    "cubic_interval_integrals", "trig_series_interval_integrals",
    "gaussian_bump_field_2d", "heat_1d_sine", "heat_2d_bumps",
    "heat_3d_separable", "heat_2d_separable", "heat_1d_profiles", "batch_2d_uneven",
    "serving_mix", "make_request_workload", "random_spd_pencil",
    "random_reduced_problem",
]


@dataclass
class Workload:
    """One synthetic space-time heat problem (inputs only)."""
    name: str
    dim: int
    n: tuple            # interior nodes per direction (length dim)
    mu: float           # diffusion coefficient: a(u, v) = mu (grad u, grad v)
    T: float            # final time
    nt: int             # number of time intervals
    F1: np.ndarray      # Nh x P, float64, Fortran order
    F2: np.ndarray      # Nt x P, float64, Fortran order
    meta: dict = field(default_factory=dict)

    @property
    def nh(self) -> int:
        return int(np.prod(self.n))

    @property
    def p(self) -> int:
        return int(self.F1.shape[1])

    @property
    def h(self) -> tuple:
        return tuple(1.0 / (ni + 1) for ni in self.n)


def node_coords(n: int) -> np.ndarray:
    """Interior node coordinates of the uniform grid on (0, 1)."""
    h = 1.0 / (n + 1)
    return h * np.arange(1, n + 1, dtype=np.float64)


def time_grid(nt: int, T: float = 1.0) -> np.ndarray:
    """Uniform time nodes t^0..t^Nt."""
    return np.linspace(0.0, T, nt + 1)


def sine_load_1d(n: int) -> np.ndarray:
    """Exact load integrals (sin(pi x), phi_j) for P1 hats on the uniform grid.

    For a hat of half-width h centred at x_j the integral equals
    sin(pi x_j) * 2 (1 - cos(pi h)) / (pi^2 h) (odd part integrates to zero).
    """
    h = 1.0 / (n + 1)
    x = node_coords(n)
    return np.sin(np.pi * x) * (2.0 * (1.0 - math.cos(math.pi * h)) / (math.pi ** 2 * h))


def cubic_interval_integrals(a: np.ndarray, t: np.ndarray) -> np.ndarray:
    """Integrals of g(t) = a0 + a1 t + a2 t^2 + a3 t^3 over each (t^{l-1}, t^l)."""
    def G(s):
        return a[0] * s + a[1] * s ** 2 / 2 + a[2] * s ** 3 / 3 + a[3] * s ** 4 / 4
    return G(t[1:]) - G(t[:-1])


def trig_series_interval_integrals(a: np.ndarray, b: np.ndarray, t: np.ndarray) -> np.ndarray:
    """Integrals of theta(t) = sum_m (a_m cos(2 pi m t) + b_m sin(2 pi m t)) / (1+m)^2.

    Differences of sines/cosines are formed with product identities so that
    short intervals do not lose digits to cancellation.
    """
    t0, t1 = t[:-1], t[1:]
    out = a[0] * (t1 - t0)
    for m in range(1, len(a)):
        w = 2.0 * np.pi * m
        mid, half = 0.5 * w * (t1 + t0), 0.5 * w * (t1 - t0)
        dsin = 2.0 * np.cos(mid) * np.sin(half)     # sin(w t1) - sin(w t0)
        dcos = -2.0 * np.sin(mid) * np.sin(half)    # cos(w t1) - cos(w t0)
        out = out + (a[m] * dsin / w - b[m] * dcos / w) / (1.0 + m) ** 2
    return out


def gaussian_bump_field_2d(n: int, rng: np.random.Generator, nbumps: int = 8) -> np.ndarray:
    """Nodal values (x fastest) of a sum of isotropic Gaussians.

    Draw order per bump: centre (2 x U[0.15, 0.85]), width U[0.03, 0.15],
    amplitude N(0, 1).
    """
    x = node_coords(n)
    X, Y = np.meshgrid(x, x, indexing="xy")      # X varies along axis 1 (fastest)
    f = np.zeros_like(X)
    for _ in range(nbumps):
        c = rng.uniform(0.15, 0.85, size=2)
        w = rng.uniform(0.03, 0.15)
        amp = rng.normal()
        f += amp * np.exp(-((X - c[0]) ** 2 + (Y - c[1]) ** 2) / (2.0 * w * w))
    return f.ravel()


def heat_1d_sine(nx: int = 127, nt: int = 128, seed: int = 1, T: float = 1.0,
                 mu: float = 1.0) -> Workload:
    """1-D heat on (0,1) with f = sin(pi x) g(t), g a seeded random cubic (rank 1).

    Draw order: a0..a3 ~ N(0, 1).  F1 = exact P1 load of sin(pi x);
    F2[l] = integral of g over I^l.
    """
    rng = np.random.default_rng(seed)
    a = rng.normal(size=4)
    t = time_grid(nt, T)
    F1 = np.asfortranarray(sine_load_1d(nx)[:, None])
    F2 = np.asfortranarray(cubic_interval_integrals(a, t)[:, None])
    return Workload("heat1d_sine", 1, (nx,), mu, T, nt, F1, F2,
                    meta={"cubic": a, "seed": seed})


def heat_2d_bumps(n: int = 511, nt: int = 1024, p: int = 2, seed: int = 2,
                  T: float = 1.0, mu: float = 1.0, nbumps: int = 8,
                  nmodes: int = 9) -> Workload:
    """2-D heat on the unit square with a rank-p bump x trig-series right-hand side.

    Spatial factor p: sum of ``nbumps`` Gaussians (gaussian_bump_field_2d); the
    load is the vertex-quadrature value h^2 f_p(x_j) of (f_p, phi_j).
    Temporal factor p: theta_p(t) = sum_{m<nmodes} (a_m cos 2 pi m t +
    b_m sin 2 pi m t)/(1+m)^2; F2 holds its exact interval integrals.
    Draw order: all spatial factors (p = 0..P-1), then for each p the vectors
    a (nmodes normals) and b (nmodes normals).
    """
    rng = np.random.default_rng(seed)
    h = 1.0 / (n + 1)
    F1 = np.empty((n * n, p), order="F")
    for q in range(p):
        F1[:, q] = h * h * gaussian_bump_field_2d(n, rng, nbumps)
    t = time_grid(nt, T)
    F2 = np.empty((nt, p), order="F")
    for q in range(p):
        a = rng.normal(size=nmodes)
        b = rng.normal(size=nmodes)
        F2[:, q] = trig_series_interval_integrals(a, b, t)
    return Workload(f"heat2d_bumps_n{n}", 2, (n, n), mu, T, nt, F1, F2,
                    meta={"seed": seed})


def _profile_1d(x: np.ndarray, rng: np.random.Generator) -> np.ndarray:
    c = rng.normal(size=6)
    c0 = rng.normal()
    x0 = rng.uniform(0.2, 0.8)
    f = sum(c[m - 1] * np.sin(m * np.pi * x) / m ** 2 for m in range(1, 7))
    return f + c0 * np.exp(-(x - x0) ** 2 / 0.02)


def heat_3d_separable(n: int = 31, nt: int = 64, p: int = 4, seed: int = 3,
                      T: float = 1.0, mu: float = 1.0, nmodes: int = 9) -> Workload:
    """3-D heat on the unit cube with a rank-p separable right-hand side.

    f_p(x, y, z) = X_p(x) Y_p(y) Z_p(z), each 1-D profile
    sum_{m=1..6} c_m sin(m pi x)/m^2 + c0 exp(-(x - x0)^2 / 0.02); the load is
    the vertex-quadrature value h^3 f_p(x_j).  Temporal factors as in the 2-D
    recipe.  Draw order: for each p the profiles X, Y, Z (each: c (6 normals),
    c0 (normal), x0 (U[0.2, 0.8])), then the temporal coefficients.
    """
    rng = np.random.default_rng(seed)
    h = 1.0 / (n + 1)
    x = node_coords(n)
    F1 = np.empty((n ** 3, p), order="F")
    for q in range(p):
        fx, fy, fz = (_profile_1d(x, rng) for _ in range(3))
        F1[:, q] = h ** 3 * np.einsum("k,j,i->kji", fz, fy, fx).ravel()
    t = time_grid(nt, T)
    F2 = np.empty((nt, p), order="F")
    for q in range(p):
        a = rng.normal(size=nmodes)
        b = rng.normal(size=nmodes)
        F2[:, q] = trig_series_interval_integrals(a, b, t)
    return Workload(f"heat3d_sep_n{n}", 3, (n, n, n), mu, T, nt, F1, F2,
                    meta={"seed": seed})


def heat_2d_separable(n: int = 127, nt: int = 256, p: int = 2, seed: int = 4000,
                      T: float = 1.0, mu: float = 1.0, nmodes: int = 9) -> Workload:
    """2-D heat on the unit square with a rank-p separable right-hand side.

    f_p(x, y) = X_p(x) Y_p(y), each 1-D profile as in heat_3d_separable; the
    load is the vertex-quadrature value h^2 f_p(x_j).  Temporal factors as in
    the 2-D bump recipe.  Draw order: for each p the profiles X, Y, then the
    temporal coefficients.
    """
    rng = np.random.default_rng(seed)
    h = 1.0 / (n + 1)
    x = node_coords(n)
    F1 = np.empty((n * n, p), order="F")
    for q in range(p):
        fx, fy = (_profile_1d(x, rng) for _ in range(2))
        F1[:, q] = h * h * np.outer(fy, fx).ravel()
    t = time_grid(nt, T)
    F2 = np.empty((nt, p), order="F")
    for q in range(p):
        a = rng.normal(size=nmodes)
        b = rng.normal(size=nmodes)
        F2[:, q] = trig_series_interval_integrals(a, b, t)
    return Workload(f"heat2d_sep_n{n}", 2, (n, n), mu, T, nt, F1, F2,
                    meta={"seed": seed})


def heat_1d_profiles(n: int = 1023, nt: int = 256, p: int = 2, seed: int = 5,
                     T: float = 1.0, mu: float = 1.0, nmodes: int = 9) -> Workload:
    """1-D heat on the unit interval with a rank-p right-hand side: each
    spatial factor a profile as in heat_3d_separable, vertex-quadrature load
    h X_p(x_j); temporal factors as in the 2-D bump recipe.  Draw order: for
    each p the profile, then the temporal coefficients."""
    rng = np.random.default_rng(seed)
    h = 1.0 / (n + 1)
    x = node_coords(n)
    F1 = np.empty((n, p), order="F")
    for q in range(p):
        F1[:, q] = h * _profile_1d(x, rng)
    t = time_grid(nt, T)
    F2 = np.empty((nt, p), order="F")
    for q in range(p):
        a = rng.normal(size=nmodes)
        b = rng.normal(size=nmodes)
        F2[:, q] = trig_series_interval_integrals(a, b, t)
    return Workload(f"heat1d_prof_n{n}", 1, (n,), mu, T, nt, F1, F2, meta={"seed": seed})


def serving_mix(count: int, seed: int = 5, frac_1d: float = 0.5, frac_2d: float = 0.4,
                nx_1d=(1000, 65536), sides_2d=(63, 95, 127, 191, 255, 383, 511),
                sides_3d=(63, 95, 127), nt_range=(128, 2048)) -> list:
    """Request shapes of a serving workload: (dim, n, nt, p, mu, seed) tuples.

    One generator default_rng(seed) draws, per request and in this order: a
    uniform u choosing the dimension (1-D if u < frac_1d, 2-D if below
    frac_1d + frac_2d, else 3-D), Nt = round(exp(U[log a, log b])) over
    nt_range, mu = exp(U[log 0.1, log 10]), P uniform in 1..4, the grid size
    (1-D: log-uniform over nx_1d, rounded; 2-D / 3-D: uniform over the
    sides), and a 31-bit seed for the request's load.
    """
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        u = rng.uniform()
        nt = int(round(np.exp(rng.uniform(np.log(nt_range[0]), np.log(nt_range[1])))))
        mu = float(np.exp(rng.uniform(np.log(0.1), np.log(10.0))))
        p = int(rng.integers(1, 5))
        if u < frac_1d:
            dim = 1
            n = int(round(np.exp(rng.uniform(np.log(nx_1d[0]), np.log(nx_1d[1])))))
        elif u < frac_1d + frac_2d:
            dim = 2
            n = int(sides_2d[rng.integers(len(sides_2d))])
        else:
            dim = 3
            n = int(sides_3d[rng.integers(len(sides_3d))])
        out.append((dim, n, nt, p, mu, int(rng.integers(1 << 31))))
    return out


def make_request_workload(dim: int, n: int, nt: int, p: int, mu: float, seed: int) -> Workload:
    """The load of one serving_mix request."""
    if dim == 1:
        return heat_1d_profiles(n=n, nt=nt, p=p, seed=seed, mu=mu)
    if dim == 2:
        return heat_2d_separable(n=n, nt=nt, p=p, seed=seed, mu=mu)
    return heat_3d_separable(n=n, nt=nt, p=p, seed=seed, mu=mu)


def batch_2d_uneven(count: int = 256, seed0: int = 4000, sides=(63, 127, 255),
                    nts=(128, 256, 512, 1024), ps=(1, 2, 3)) -> list:
    """A batch of independent 2-D problems of uneven size.

    Problem i uses default_rng(seed0 + i) and draws, in this order: the
    diffusion coefficient mu = exp(U[log 0.1, log 10]), the grid side
    (uniform over ``sides``), Nt (uniform over ``nts``), P (uniform over
    ``ps``); its right-hand side is heat_2d_separable with the seed
    seed0 + i + 1000000.
    """
    out = []
    for i in range(count):
        rng = np.random.default_rng(seed0 + i)
        mu = float(np.exp(rng.uniform(np.log(0.1), np.log(10.0))))
        n = int(sides[rng.integers(len(sides))])
        nt = int(nts[rng.integers(len(nts))])
        p = int(ps[rng.integers(len(ps))])
        w = heat_2d_separable(n=n, nt=nt, p=p, seed=seed0 + i + 1000000, mu=mu)
        w.name = f"batch{i}_n{n}_nt{nt}_p{p}"
        w.meta["index"] = i
        out.append(w)
    return out


def random_spd_pencil(k: int, seed: int, spread: float = 6.0):
    """A seeded symmetric positive definite pencil (Km, Mm) of order k.

    Km has eigenvalues log-uniform over ``spread`` decades (as the Ritz values
    of a Laplacian pencil are); Mm = I + E with a small symmetric E, mimicking a
    numerically M-orthonormal basis.  Returned in Fortran order.
    """
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.normal(size=(k, k)))
    lam = 10.0 ** rng.uniform(1.0, 1.0 + spread, size=k)
    Km = (Q * lam) @ Q.T
    Km = 0.5 * (Km + Km.T)
    E = rng.normal(size=(k, k)) * 1e-3 / max(k, 1)
    Mm = np.eye(k) + 0.5 * (E + E.T)
    return np.asfortranarray(Km), np.asfortranarray(Mm)


def random_reduced_problem(k: int, nt: int, p: int, seed: int, T: float = 1.0):
    """Seeded reduced-equation inputs: an SPD pencil plus beta (k x p) and F2 (nt x p)."""
    Km, Mm = random_spd_pencil(k, seed)
    rng = np.random.default_rng(seed + 7919)
    beta = np.asfortranarray(rng.normal(size=(k, p)))
    t = time_grid(nt, T)
    F2 = np.empty((nt, p), order="F")
    for q in range(p):
        F2[:, q] = trig_series_interval_integrals(rng.normal(size=5), rng.normal(size=5), t)
    return Km, Mm, beta, F2
