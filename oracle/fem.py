"""Discretisation matrices of the space-time Petrov-Galerkin scheme (oracle).

Time: trial space S_dt = span{sigma^1..sigma^Nt} (hat functions, sigma^Nt
truncated at T; sigma^0 is absent because u(0) = 0), test space
Q_dt = span{tau^1..tau^Nt} (indicators of I^l = (t^{l-1}, t^l)) -- Sec. 3,
heat-equation paragraph.  The matrices of eq. (par1) are formed by Gauss
quadrature of these functions and returned indexed [test l, trial k]:

    Dt[l, k] = (d/dt sigma^k, tau^l)_{L2(I)},   Mt[l, k] = (sigma^k, tau^l)_{L2(I)}

so that the space-time system reads (Dt kron Mx + Mt kron Kx) vec(U) = vec(F)
(the paper's B_delta^T u = f with D_dt = Dt^T, C_dt = Mt^T).

Space: conforming P1 elements (Sec. 3) on uniform meshes of (0,1)^d with
homogeneous Dirichlet conditions.  Matrices are assembled element by element
from local matrices computed by quadrature of the local shape functions, then
restricted to interior nodes (x fastest).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

# --------------------------------------------------------------------------
# time
# --------------------------------------------------------------------------

_GL2 = (np.array([-1.0, 1.0]) / np.sqrt(3.0), np.array([1.0, 1.0]))


def _hat(k: int, t: np.ndarray, s: np.ndarray):
    """Value and derivative of the trial hat sigma^k (k = 1..Nt) at points s."""
    nt = len(t) - 1
    val = np.zeros_like(s)
    der = np.zeros_like(s)
    left = (s > t[k - 1]) & (s <= t[k])
    hl = t[k] - t[k - 1]
    val[left] = (s[left] - t[k - 1]) / hl
    der[left] = 1.0 / hl
    if k < nt:
        right = (s > t[k]) & (s < t[k + 1])
        hr = t[k + 1] - t[k]
        val[right] = (t[k + 1] - s[right]) / hr
        der[right] = -1.0 / hr
    return val, der


def time_matrices(t: np.ndarray, window: int | None = 2):
    """Dense (Dt, Mt), Nt x Nt, from eq. (par1) by 2-point Gauss quadrature.

    ``t`` holds the time nodes t^0 < ... < t^Nt.  Two Gauss points per interval
    integrate the piecewise-linear integrands exactly.  A hat sigma^k is
    supported on [t^{k-1}, t^{k+1}], so on I^l only hats with |k - l| small can
    be non-zero; ``window`` limits the trial loop to |k - l| <= window (pass
    None to integrate every pair, which the tests do at small Nt).
    """
    t = np.asarray(t, dtype=np.float64)
    nt = len(t) - 1
    xg, wg = _GL2
    Dt = np.zeros((nt, nt))
    Mt = np.zeros((nt, nt))
    for l in range(1, nt + 1):                       # test function tau^l
        a, b = t[l - 1], t[l]
        s = 0.5 * (a + b) + 0.5 * (b - a) * xg
        w = 0.5 * (b - a) * wg
        ks = range(1, nt + 1) if window is None else range(max(1, l - window), min(nt, l + window) + 1)
        for k in ks:                                 # trial function sigma^k
            v, d = _hat(k, t, s)
            Dt[l - 1, k - 1] = np.dot(w, d)
            Mt[l - 1, k - 1] = np.dot(w, v)
    return Dt, Mt


def bidiagonals(Dt: np.ndarray, Mt: np.ndarray):
    """Split lower-bidiagonal Dt, Mt into (diag, sub) arrays.

    ``sub[l]`` is the entry in row l+1, column l (length Nt-1).  Raises if
    anything lies outside the two diagonals.
    """
    for A in (Dt, Mt):
        if np.any(np.triu(A, 1)) or np.any(np.tril(A, -2)):
            raise ValueError("time matrix is not lower bidiagonal")
    return (np.diag(Dt).copy(), np.diag(Dt, -1).copy(),
            np.diag(Mt).copy(), np.diag(Mt, -1).copy())


# --------------------------------------------------------------------------
# space: local element matrices by quadrature
# --------------------------------------------------------------------------

def p1_interval_element(h: float, mu: float = 1.0):
    """Local P1 stiffness and mass on an interval of length h (3-pt Gauss)."""
    xq = 0.5 + 0.5 * np.array([-np.sqrt(0.6), 0.0, np.sqrt(0.6)])
    wq = 0.5 * np.array([5.0, 8.0, 5.0]) / 9.0
    phi = np.stack([1.0 - xq, xq])                   # shape functions on (0,1)
    dphi = np.array([-1.0, 1.0]) / h                 # constant derivatives
    Ke = mu * h * np.outer(dphi, dphi)
    Me = h * (phi * wq) @ phi.T
    return Ke, Me


def p1_triangle_element(verts: np.ndarray, mu: float = 1.0):
    """Local P1 stiffness and mass on a triangle (vertices 3 x 2).

    Gradients of the barycentric functions from the inverse of the affine map;
    mass by the 3-point edge-midpoint rule (exact for quadratics).
    """
    v0, v1, v2 = verts
    J = np.column_stack([v1 - v0, v2 - v0])
    area = 0.5 * abs(np.linalg.det(J))
    Jinv = np.linalg.inv(J)
    ref_grads = np.array([[-1.0, -1.0], [1.0, 0.0], [0.0, 1.0]])
    grads = ref_grads @ Jinv                          # rows: grad lambda_a
    Ke = mu * area * grads @ grads.T
    mids = np.array([[0.5, 0.5, 0.0], [0.0, 0.5, 0.5], [0.5, 0.0, 0.5]])
    Me = area / 3.0 * mids.T @ mids
    return Ke, Me


# --------------------------------------------------------------------------
# space: assembly
# --------------------------------------------------------------------------

def _restrict(A: sp.spmatrix, interior: np.ndarray) -> sp.csr_matrix:
    A = A.tocsr()
    A = A[interior][:, interior].tocsr()
    A.eliminate_zeros()
    return A


def p1_1d(n: int, mu: float = 1.0):
    """P1 stiffness Kx and mass Mx on (0,1) with n interior nodes (Dirichlet)."""
    h = 1.0 / (n + 1)
    nn = n + 2
    Ke, Me = p1_interval_element(h, mu)
    rows, cols, kv, mv = [], [], [], []
    for e in range(n + 1):                           # element [x_e, x_{e+1}]
        dofs = (e, e + 1)
        for a in range(2):
            for b in range(2):
                rows.append(dofs[a]); cols.append(dofs[b])
                kv.append(Ke[a, b]); mv.append(Me[a, b])
    K = sp.coo_matrix((kv, (rows, cols)), shape=(nn, nn))
    M = sp.coo_matrix((mv, (rows, cols)), shape=(nn, nn))
    interior = np.arange(1, n + 1)
    return _restrict(K, interior), _restrict(M, interior)


def p1_2d_courant(n: int, mu: float = 1.0):
    """P1 stiffness Kx and mass Mx on the unit square, Courant triangulation.

    Each mesh square is cut along its SW-NE diagonal.  Interior nodes are
    numbered lexicographically with x fastest.  Element matrices depend only on
    the triangle's shape, so the two reference triangles are integrated once and
    scattered over all squares.
    """
    h = 1.0 / (n + 1)
    nn = n + 2
    sw, se, ne, nw = (np.array(v, dtype=float) * h for v in ((0, 0), (1, 0), (1, 1), (0, 1)))
    KA, MA = p1_triangle_element(np.array([sw, se, ne]), mu)    # lower-right triangle
    KB, MB = p1_triangle_element(np.array([sw, ne, nw]), mu)    # upper-left triangle
    i, j = np.meshgrid(np.arange(n + 1), np.arange(n + 1), indexing="xy")
    i, j = i.ravel(), j.ravel()
    g = lambda ii, jj: ii + nn * jj
    triA = np.stack([g(i, j), g(i + 1, j), g(i + 1, j + 1)], axis=1)
    triB = np.stack([g(i, j), g(i + 1, j + 1), g(i, j + 1)], axis=1)
    rows, cols, kv, mv = [], [], [], []
    for tri, Ke, Me in ((triA, KA, MA), (triB, KB, MB)):
        for a in range(3):
            for b in range(3):
                rows.append(tri[:, a]); cols.append(tri[:, b])
                kv.append(np.full(len(tri), Ke[a, b])); mv.append(np.full(len(tri), Me[a, b]))
    rows, cols = np.concatenate(rows), np.concatenate(cols)
    K = sp.coo_matrix((np.concatenate(kv), (rows, cols)), shape=(nn * nn, nn * nn))
    M = sp.coo_matrix((np.concatenate(mv), (rows, cols)), shape=(nn * nn, nn * nn))
    ii, jj = np.meshgrid(np.arange(1, n + 1), np.arange(1, n + 1), indexing="xy")
    interior = g(ii.ravel(), jj.ravel())
    return _restrict(K, interior), _restrict(M, interior)


def q1_3d_7pt(n: int, mu: float = 1.0):
    """3-D stiffness with a 7-point stencil and the consistent trilinear mass.

    The trilinear (Q1) element on a cube is the tensor product of 1-D P1
    elements.  The mass uses the full tensor product Me x Me x Me (27-point
    stencil).  The stiffness takes, in each direction d, the 1-D stiffness in d
    times the row-sum-lumped 1-D mass in the other two directions, which is the
    Q1 stiffness with lumped transverse mass and gives the 7-point stencil
    mu h (6; -1 on the six faces).  Assembled by a loop over the cubes.
    """
    h = 1.0 / (n + 1)
    nn = n + 2
    K1, M1 = p1_interval_element(h, mu=1.0)
    L1 = np.diag(M1.sum(axis=1))                       # lumped 1-D mass
    # local index a = ax + 2 ay + 4 az  (x fastest) -> kron order (z, y, x)
    Ke = mu * (np.kron(L1, np.kron(L1, K1)) + np.kron(L1, np.kron(K1, L1))
               + np.kron(K1, np.kron(L1, L1)))
    Me = np.kron(M1, np.kron(M1, M1))
    i, j, k = np.meshgrid(np.arange(n + 1), np.arange(n + 1), np.arange(n + 1), indexing="ij")
    i, j, k = i.ravel(), j.ravel(), k.ravel()
    g = lambda a, b, c: a + nn * (b + nn * c)
    corners = [g(i + ax, j + ay, k + az) for az in (0, 1) for ay in (0, 1) for ax in (0, 1)]
    rows, cols, kv, mv = [], [], [], []
    for a in range(8):
        for b in range(8):
            rows.append(corners[a]); cols.append(corners[b])
            kv.append(np.full(len(i), Ke[a, b])); mv.append(np.full(len(i), Me[a, b]))
    rows, cols = np.concatenate(rows), np.concatenate(cols)
    N = nn ** 3
    K = sp.coo_matrix((np.concatenate(kv), (rows, cols)), shape=(N, N))
    M = sp.coo_matrix((np.concatenate(mv), (rows, cols)), shape=(N, N))
    ii, jj, kk = np.meshgrid(np.arange(1, n + 1), np.arange(1, n + 1), np.arange(1, n + 1), indexing="ij")
    interior = np.sort(g(ii.ravel(), jj.ravel(), kk.ravel()))
    return _restrict(K, interior), _restrict(M, interior)


def spatial_operators(dim: int, n: int, mu: float = 1.0):
    """(Kx, Mx) for the uniform-mesh discretisations used by the workloads."""
    if dim == 1:
        return p1_1d(n, mu)
    if dim == 2:
        return p1_2d_courant(n, mu)
    if dim == 3:
        return q1_3d_7pt(n, mu)
    raise ValueError(dim)
