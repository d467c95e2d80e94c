"""Reference multigrid V-cycle for the tests of the preconditioned inner solver.

The library preconditions its inner Kx solves (2-D P1, Sec. 4's negative
powers) with one geometric multigrid V-cycle; the preconditioner is the
library's choice, not part of the paper's method, so it has no place in
``oracle/``.  This module restates the operator plainly -- assembled sparse
matrices from the oracle's finite elements, a prolongation built by
evaluating coarse P1 hat functions at fine nodes, and a recursive V-cycle --
so that the GPU V-cycle can be compared entry by entry.

V-cycle on level n (interior nodes per direction), right-hand side b:
  exact solve         on the finest level if n <= 63, on a coarser level if
                      n <= 255;
  otherwise           three Chebyshev smoothing steps from zero, restriction of
                      the residual by P^T to n_c = (n - 1) / 2 (n must be odd),
                      V-cycle there, correction u += P e_c, three more
                      Chebyshev steps on the residual equation.
Chebyshev smoothing targets [1/2, 2] of the spectrum of D^{-1} Kx (D its
diagonal, 4 mu): with theta, delta the centre and half-width of the interval
and sigma = theta / delta, the textbook three-term recurrence
  d_0 = r_0 / (theta D),  rho_0 = 1 / sigma,
  rho_k = 1 / (2 sigma - rho_{k-1}),
  d_k = rho_k rho_{k-1} d_{k-1} + (2 rho_k / delta) D^{-1} r_k,
  u_{k+1} = u_k + d_k,  r_k = b - Kx u_k.
"""
from __future__ import annotations

import functools

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle import fem

CHEB_STEPS = 3
CHEB_INTERVAL = (0.5, 2.0)
EXACT_FINEST = 63     # finest level solved exactly up to this size
EXACT_COARSE = 255    # coarser levels solved exactly up to this size


def hat(xi, eta):
    """P1 hat function of a node of the Courant triangulation whose squares are
    cut along the SW-NE diagonal, at offset (xi, eta) in units of the mesh
    width: 1 - max(|xi|, |eta|, |xi - eta|), clipped at zero."""
    return np.maximum(0.0, 1.0 - np.maximum(np.maximum(abs(xi), abs(eta)), abs(xi - eta)))


def prolongation(nc: int) -> sp.csr_matrix:
    """P1 interpolation from the nc x nc interior grid to the (2 nc + 1)^2 one:
    P[f, c] = coarse hat c evaluated at fine node f (fine node 2I+1 coincides
    with coarse node I; nodes numbered with x fastest)."""
    n = 2 * nc + 1
    I, J = np.meshgrid(np.arange(nc), np.arange(nc), indexing="xy")
    I, J = I.ravel(), J.ravel()
    rows, cols, vals = [], [], []
    for dy in (-1, 0, 1):
        for dx in (-1, 0, 1):
            w = float(hat(dx / 2.0, dy / 2.0))
            if w == 0.0:
                continue
            fx, fy = 2 * I + 1 + dx, 2 * J + 1 + dy
            rows.append(fy * n + fx)
            cols.append(J * nc + I)
            vals.append(np.full(I.shape, w))
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(n * n, nc * nc))


def stiffness(n: int, mu: float) -> sp.csr_matrix:
    return fem.spatial_operators(2, n, mu)[0].tocsr()


def chebyshev(K, b, u, steps=CHEB_STEPS):
    """`steps` Chebyshev steps on K u = b from u (see the module docstring)."""
    lo, hi = CHEB_INTERVAL
    theta, delta = 0.5 * (hi + lo), 0.5 * (hi - lo)
    sigma = theta / delta
    dinv = 1.0 / K.diagonal()
    if b.ndim == 2:
        dinv = dinv[:, None]
    rho = 1.0 / sigma
    d = dinv * (b - K @ u) / theta
    u = u + d
    for _ in range(steps - 1):
        rho_new = 1.0 / (2.0 * sigma - rho)
        d = rho_new * rho * d + (2.0 * rho_new / delta) * dinv * (b - K @ u)
        u = u + d
        rho = rho_new
    return u


def mass_stand_in(n: int) -> sp.csr_matrix:
    """The coarsest level's mass in the shifted solve: the 2-D P1 mass without
    its SW-NE coupling, (h^2 / 12) (6; 1 at W, E, S, N), which the sine
    transform diagonalises."""
    w = (1.0 / (n + 1)) ** 2 / 12.0
    e = np.ones(n)
    T1 = sp.diags([e[:-1], e[:-1]], [-1, 1])
    eye = sp.identity(n)
    return (w * (6.0 * sp.identity(n * n) + sp.kron(eye, T1) + sp.kron(T1, eye))).tocsr()


def vcycle(b: np.ndarray, n: int, mu: float, finest: bool = True, shift: float = 0.0) -> np.ndarray:
    """One V-cycle from zero applied to b (length n^2, or n^2 x m) for
    Kx + shift Mx; each level's operator is the Galerkin product of the finer
    one (nested P1 spaces: the coarse Kx + shift Mx)."""
    K = stiffness(n, mu)
    if shift:
        K = (K + shift * fem.spatial_operators(2, n, mu)[1]).tocsr()
    if n <= (EXACT_FINEST if finest else EXACT_COARSE):
        A = stiffness(n, mu) + shift * mass_stand_in(n) if shift else K
        return spla.spsolve(A.tocsc(), b).reshape(b.shape)
    assert n % 2 == 1, "levels that do not fit the exact solve must halve"
    u = chebyshev(K, b, np.zeros_like(b))
    nc = (n - 1) // 2
    P = prolongation(nc)
    u = u + P @ vcycle(P.T @ (b - K @ u), nc, mu, finest=False, shift=shift)
    return chebyshev(K, b, u)


def supported(n: int) -> bool:
    """Grids the library's multigrid accepts: n <= 63, or n odd halving (odd at
    each step) down to at most 255."""
    first = True
    while n > EXACT_COARSE or (first and n > EXACT_FINEST):
        if n % 2 == 0:
            return False
        n = (n - 1) // 2
        first = False
    return n >= 1


# ---------------------------------------------------------------------------
# 3-D: the seven-point stiffness mu h (6; -1 x 6), which is the P1 stiffness
# of the Kuhn triangulation (cubes cut into six tetrahedra around the x+y+z
# diagonal).  Nested Kuhn meshes give P1 interpolation along the seven edge
# directions x, y, z, x+y, x+z, y+z, x+y+z.  Two Chebyshev steps for
# [1/3, 2]; the coarsest level (n <= 63, on any level) is solved exactly by
# the orthonormal DST-I along the three axes.
# ---------------------------------------------------------------------------
CHEB3_STEPS = 2
CHEB3_INTERVAL = (1.0 / 3.0, 2.0)
EXACT3 = 63


def kuhn_hat(xi, eta, zeta):
    """P1 hat of a Kuhn-mesh node at offset (xi, eta, zeta) in mesh widths:
    the tetrahedra of a cube are the orderings of its coordinates, and on the
    one containing the offset the hat is 1 minus the largest of the
    magnitudes of the coordinates and of their pairwise differences (the
    barycentric form of the ordered simplex), clipped at zero."""
    d = np.max(np.abs([xi, eta, zeta, xi - eta, xi - zeta, eta - zeta]), axis=0)
    return np.maximum(0.0, 1.0 - d)


@functools.lru_cache(maxsize=8)
def prolongation3(nc: int) -> sp.csr_matrix:
    """P[f, c] = coarse Kuhn hat c at fine node f, nc^3 -> (2 nc + 1)^3
    (fine node 2I+1 coincides with coarse I; x fastest)."""
    n = 2 * nc + 1
    K, J, I = np.meshgrid(np.arange(nc), np.arange(nc), np.arange(nc), indexing="ij")
    I, J, K = I.ravel(), J.ravel(), K.ravel()
    rows, cols, vals = [], [], []
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                w = float(kuhn_hat(dx / 2.0, dy / 2.0, dz / 2.0))
                if w == 0.0:
                    continue
                fx, fy, fz = 2 * I + 1 + dx, 2 * J + 1 + dy, 2 * K + 1 + dz
                rows.append((fz * n + fy) * n + fx)
                cols.append((K * nc + J) * nc + I)
                vals.append(np.full(I.shape, w))
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(n ** 3, nc ** 3))


@functools.lru_cache(maxsize=8)
def stiffness3(n: int, mu: float) -> sp.csr_matrix:
    """mu h (T (x) I (x) I + I (x) T (x) I + I (x) I (x) T), T = tridiag(-1, 2, -1):
    the oracle's 3-D stiffness written as a Kronecker sum (equal to its
    element assembly, which is too slow for the largest test grids)."""
    h = 1.0 / (n + 1)
    T = sp.diags([-np.ones(n - 1), 2.0 * np.ones(n), -np.ones(n - 1)], [-1, 0, 1])
    eye = sp.identity(n)
    K = sp.kron(sp.kron(T, eye), eye) + sp.kron(sp.kron(eye, T), eye) + sp.kron(sp.kron(eye, eye), T)
    return (mu * h * K).tocsr()


@functools.lru_cache(maxsize=8)
def mass3(n: int) -> sp.csr_matrix:
    """(h/6)^3 Tm (x) Tm (x) Tm, Tm = tridiag(1, 4, 1): the oracle's Q1 mass as a
    Kronecker product (equal to its element assembly)."""
    h = 1.0 / (n + 1)
    Tm = sp.diags([np.ones(n - 1), 4.0 * np.ones(n), np.ones(n - 1)], [-1, 0, 1])
    return ((h / 6.0) ** 3 * sp.kron(sp.kron(Tm, Tm), Tm)).tocsr()


def exact3(b: np.ndarray, n: int, mu: float, shift: float = 0.0) -> np.ndarray:
    """(Kx + shift Mx)^{-1} b for the seven-point stiffness and the Q1 mass by
    the sine transform (both are diagonal in the sine basis)."""
    from scipy.fft import dstn

    h = 1.0 / (n + 1)
    lam = 2.0 - 2.0 * np.cos(np.arange(1, n + 1) * np.pi * h)
    D = mu * h * (lam[:, None, None] + lam[None, :, None] + lam[None, None, :])
    if shift:
        tm = 6.0 - lam
        D = D + shift * (h / 6.0) ** 3 * (tm[:, None, None] * tm[None, :, None] * tm[None, None, :])
    cols = b.reshape(n ** 3, -1)
    out = np.empty_like(cols)
    for j in range(cols.shape[1]):
        B = cols[:, j].reshape(n, n, n)
        out[:, j] = dstn(dstn(B, type=1, norm="ortho") / D, type=1, norm="ortho").ravel()
    return out.reshape(b.shape)


def chebyshev3(K, b, u, steps=CHEB3_STEPS, interval=CHEB3_INTERVAL):
    lo, hi = interval
    theta, delta = 0.5 * (hi + lo), 0.5 * (hi - lo)
    sigma = theta / delta
    dinv = 1.0 / K.diagonal()
    if b.ndim == 2:
        dinv = dinv[:, None]
    rho = 1.0 / sigma
    d = dinv * (b - K @ u) / theta
    u = u + d
    for _ in range(steps - 1):
        rho_new = 1.0 / (2.0 * sigma - rho)
        d = rho_new * rho * d + (2.0 * rho_new / delta) * dinv * (b - K @ u)
        u = u + d
        rho = rho_new
    return u


def vcycle3(b: np.ndarray, n: int, mu: float, shift: float = 0.0) -> np.ndarray:
    """One 3-D V-cycle from zero applied to b (length n^3, or n^3 x m) for
    Kx + shift Mx; the coarse levels rediscretise the Q1 mass."""
    if n <= EXACT3:
        return exact3(b, n, mu, shift)
    assert n % 2 == 1, "levels above the exact size must halve"
    K = stiffness3(n, mu)
    if shift:
        K = (K + shift * mass3(n)).tocsr()
    u = chebyshev3(K, b, np.zeros_like(b))
    nc = (n - 1) // 2
    P = prolongation3(nc)
    # the coarse stiffness is mu (2h) (6; -1 x 6): the same stencil at nc
    u = u + P @ vcycle3(P.T @ (b - K @ u), nc, mu, shift)
    return chebyshev3(K, b, u)


def supported3(n: int) -> bool:
    while n > EXACT3:
        if n % 2 == 0:
            return False
        n = (n - 1) // 2
    return n >= 1
