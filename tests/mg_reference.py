"""Reference multigrid V-cycle for the tests of the preconditioned inner solver.

The library preconditions its inner Kx solves (2-D P1, Sec. 4's negative
powers) with one geometric multigrid V-cycle; the preconditioner is the
library's choice, not part of the paper's method, so it has no place in
``oracle/``.  This module restates the operator plainly -- assembled sparse
matrices from the oracle's finite elements, a prolongation built by
evaluating coarse P1 hat functions at fine nodes, and a recursive V-cycle --
so that the GPU V-cycle can be compared entry by entry.

V-cycle on level n (interior nodes per direction), right-hand side b:
  n == 1           exact solve;
  n even, n > 1    20 damped-Jacobi sweeps from zero (the level does not halve);
  otherwise        two damped-Jacobi sweeps from zero (weight 0.8), restriction
                   of the residual by P^T to n_c = (n - 1) / 2, recursive
                   V-cycle there, correction u += P e_c, two more sweeps.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from oracle import fem

OMEGA = 0.8
BOTTOM_SWEEPS = 20


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


def vcycle(b: np.ndarray, n: int, mu: float) -> np.ndarray:
    """One V-cycle from zero applied to b (length n^2, or n^2 x m)."""
    K = stiffness(n, mu)
    c = OMEGA / K.diagonal()
    if b.ndim == 2:
        c = c[:, None]
    if n == 1:
        return b / K.diagonal()[0]
    if n % 2 == 0:
        u = np.zeros_like(b)
        for _ in range(BOTTOM_SWEEPS):
            u = u + c * (b - K @ u)
        return u
    u = np.zeros_like(b)
    for _ in range(2):
        u = u + c * (b - K @ u)
    nc = (n - 1) // 2
    P = prolongation(nc)
    u = u + P @ vcycle(P.T @ (b - K @ u), nc, mu)
    for _ in range(2):
        u = u + c * (b - K @ u)
    return u


def supported(n: int) -> bool:
    """Grids the library's multigrid accepts: n halves down to at most 63."""
    while n > 63:
        if n % 2 == 0:
            return False
        n = (n - 1) // 2
    return n >= 1
