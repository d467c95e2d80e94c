"""Exact discrete space-time solutions (oracle).

The space-time system of Sec. 3 (eq. (par1)-(par2)), written with the test
index first, is

    (Dt kron Mx + Mt kron Kx) vec(U) = vec(F1 F2^T),

and by the vec identity of Sec. 4 ((D kron A) vec X = vec(A X D^T), columns
stacked) it is the generalized Sylvester equation of eq. (Sylv_Heat):

    Kx U Mt^T + Mx U Dt^T = F1 F2^T,   U in R^{Nh x Nt},  U[:, l-1] = u(t^l).

The system is block lower bidiagonal in time with SPD diagonal blocks
Mt[l,l] Kx + Dt[l,l] Mx, so its solution is unique.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def vec(X: np.ndarray) -> np.ndarray:
    """Stack the columns of X (Sec. 4)."""
    return np.asarray(X).reshape(-1, order="F")


def unvec(x: np.ndarray, nrows: int) -> np.ndarray:
    return np.asarray(x).reshape(nrows, -1, order="F")


def kron_system(Kx, Mx, Dt, Mt) -> sp.csc_matrix:
    """The assembled space-time matrix Dt kron Mx + Mt kron Kx (eq. (par1))."""
    Dt = sp.csr_matrix(Dt)
    Mt = sp.csr_matrix(Mt)
    return (sp.kron(Dt, Mx) + sp.kron(Mt, Kx)).tocsc()


def kron_solve(Kx, Mx, Dt, Mt, F1, F2) -> np.ndarray:
    """Sparse-direct solve of the assembled Kronecker system (tiny sizes only)."""
    B = kron_system(Kx, Mx, Dt, Mt)
    f = vec(np.asarray(F1) @ np.asarray(F2).T)
    return unvec(spla.spsolve(B, f), Kx.shape[0])


def crank_nicolson(Kx, Mx, Dt, Mt, F1, F2, steps: int | None = None) -> np.ndarray:
    """Time stepping of the space-time system, one interval at a time.

    Row l of the block-bidiagonal system reads
        (Mt[l,l] Kx + Dt[l,l] Mx) u^l = F[:, l] - (Mt[l,l-1] Kx + Dt[l,l-1] Mx) u^{l-1},
    u^0 = 0.  With the uniform hat/indicator pair this is the Crank-Nicolson
    scheme with the exact-integral load (Sec. 3, final remark of the heat
    paragraph).  A factorisation is reused while the step matrix is unchanged.
    ``steps`` limits the march to the first ``steps`` intervals.
    """
    F1 = np.asarray(F1)
    F2 = np.asarray(F2)
    nt = F2.shape[0] if steps is None else min(steps, F2.shape[0])
    nh = Kx.shape[0]
    U = np.zeros((nh, nt))
    prev = np.zeros(nh)
    key, lu = None, None
    for l in range(nt):
        d, m = Dt[l, l], Mt[l, l]
        if key != (d, m):
            lu = spla.splu((m * Kx + d * Mx).tocsc())
            key = (d, m)
        rhs = F1 @ F2[l]
        if l > 0:
            rhs = rhs - (Mt[l, l - 1] * (Kx @ prev) + Dt[l, l - 1] * (Mx @ prev))
        prev = lu.solve(rhs)
        U[:, l] = prev
    return U


def crank_nicolson_chunks(Kx, Mx, Dt, Mt, F1, F2, chunk: int):
    """The time stepping of ``crank_nicolson`` in pieces: yields (l0, U[:, l0:l0+c])
    for consecutive chunks of at most ``chunk`` intervals, carrying u^{l0} from
    one chunk to the next (Sec. 3, Crank-Nicolson remark), so a long march
    never holds the whole Nh x Nt solution."""
    F1 = np.asarray(F1)
    F2 = np.asarray(F2)
    nt = F2.shape[0]
    nh = Kx.shape[0]
    prev = np.zeros(nh)
    key, lu = None, None
    for l0 in range(0, nt, chunk):
        c = min(chunk, nt - l0)
        U = np.zeros((nh, c))
        for j in range(c):
            l = l0 + j
            d, m = Dt[l, l], Mt[l, l]
            if key != (d, m):
                lu = spla.splu((m * Kx + d * Mx).tocsc())
                key = (d, m)
            rhs = F1 @ F2[l]
            if l > 0:
                rhs = rhs - (Mt[l, l - 1] * (Kx @ prev) + Dt[l, l - 1] * (Mx @ prev))
            prev = lu.solve(rhs)
            U[:, j] = prev
        yield l0, U


def modal_solve_1d_fast(n: int, mu: float, Dt, Mt, F1, F2) -> np.ndarray:
    """The 1-D sine-mode solve of ``modal_solve_1d`` with the transforms done
    by the orthonormal DST-I (a library FFT) and all modes swept together, for
    grids where the O(n^2) mode loop is too slow.  The orthonormal sine vectors
    s_m = sqrt(2 h) sin(m pi x_j) diagonalise Kx = (mu/h) tridiag(-1, 2, -1)
    with kappa_m = (4 mu / h) sin^2(m pi h / 2) and Mx = (h/6) tridiag(1, 4, 1)
    with nu_m = (h/6)(6 - 4 sin^2(m pi h / 2)) (half-angle forms: no
    cancellation for the smooth modes); each mode solves the lower-bidiagonal
    system (nu_m Dt + kappa_m Mt) w_m = F2 (s_m^T F1), by forward substitution
    in time."""
    from scipy.fft import dst

    Dt = np.asarray(Dt, dtype=float)
    Mt = np.asarray(Mt, dtype=float)
    F1 = np.asarray(F1, dtype=float)
    F2 = np.asarray(F2, dtype=float)
    nt = F2.shape[0]
    band = np.tril(np.triu(np.ones((nt, nt)), -1))
    assert not np.any(Dt * (1 - band)) and not np.any(Mt * (1 - band)), "lower bidiagonal in time"
    h = 1.0 / (n + 1)
    s2 = np.sin(np.arange(1, n + 1) * np.pi * h / 2.0) ** 2
    kappa = 4.0 * mu / h * s2
    nu = h / 6.0 * (6.0 - 4.0 * s2)
    fhat = dst(F1, type=1, norm="ortho", axis=0)              # n x P
    W = np.zeros((n, nt))
    prev = np.zeros(n)
    for l in range(nt):
        rhs = fhat @ F2[l]
        if l > 0:
            rhs = rhs - (nu * Dt[l, l - 1] + kappa * Mt[l, l - 1]) * prev
        prev = rhs / (nu * Dt[l, l] + kappa * Mt[l, l])
        W[:, l] = prev
    return dst(W, type=1, norm="ortho", axis=0)


def modal_solve_1d(n: int, mu: float, Dt, Mt, F1, F2) -> np.ndarray:
    """Exact solve for uniform 1-D P1 by sine-mode diagonalisation.

    Kx and Mx are symmetric tridiagonal Toeplitz, so both are diagonalised by
    q_m = sin(m pi x_j): Kx q_m = kappa_m q_m, Mx q_m = nu_m q_m with
    kappa_m = (2 mu / h)(1 - cos m pi h), nu_m = (h/3)(2 + cos m pi h).
    Writing U = sum_m q_m w_m^T and projecting on q_m gives the Nt x Nt
    lower-bidiagonal systems (nu_m Dt + kappa_m Mt) w_m = F2 (F1^T q_m)/|q_m|^2.
    """
    h = 1.0 / (n + 1)
    j = np.arange(1, n + 1)
    U = np.zeros((n, F2.shape[0]))
    for m in range(1, n + 1):
        q = np.sin(m * np.pi * j * h)
        kappa = 2.0 * mu / h * (1.0 - np.cos(m * np.pi * h))
        nu = h / 3.0 * (2.0 + np.cos(m * np.pi * h))
        rhs = np.asarray(F2) @ (np.asarray(F1).T @ q) / (q @ q)
        w = np.linalg.solve(nu * np.asarray(Dt) + kappa * np.asarray(Mt), rhs)
        U += np.outer(q, w)
    return U


def modal_solve_3d(n: int, mu: float, Dt, Mt, F1, F2) -> np.ndarray:
    """Exact solve for the uniform 3-D trilinear-mass / 7-point-stiffness pair
    by sine-mode diagonalisation.  The paper's 3-D heat problem (Sec. 5,
    Example 1) uses linear elements; this trilinear-mass / 7-point-stiffness
    pair is the reading of a 3-D configuration that the paper does not define
    (its 7-point matrix is the P1 stiffness of the Kuhn tetrahedral mesh).

    With T = tridiag(-1, 2, -1) and Tm = tridiag(1, 4, 1) of order n,
    Kx = mu h (T (x) I (x) I + I (x) T (x) I + I (x) I (x) T) and
    Mx = (h/6)^3 Tm (x) Tm (x) Tm.  The orthonormal sine vectors
    s_m = sqrt(2 h) sin(m pi x_j) diagonalise both factors:
    T s_m = (2 - 2 cos m pi h) s_m, Tm s_m = (4 + 2 cos m pi h) s_m.  In the
    tensor basis s_a (x) s_b (x) s_c every mode decouples into the Nt x Nt
    lower-bidiagonal system (nu Dt + kappa Mt) w = F2 f_hat, with
    kappa = mu h (t_a + t_b + t_c), nu = (h/6)^3 m_a m_b m_c and f_hat the
    mode's coefficients of the columns of F1; forward substitution in time,
    all modes at once.  The transform to and from the basis is the
    orthonormal DST-I along each axis (a library FFT).
    """
    from scipy.fft import dstn

    Dt = np.asarray(Dt, dtype=float)
    Mt = np.asarray(Mt, dtype=float)
    F1 = np.asarray(F1, dtype=float)
    F2 = np.asarray(F2, dtype=float)
    nt = F2.shape[0]
    band = np.tril(np.triu(np.ones((nt, nt)), -1))
    assert not np.any(Dt * (1 - band)) and not np.any(Mt * (1 - band)), "lower bidiagonal in time"
    h = 1.0 / (n + 1)
    c = np.cos(np.arange(1, n + 1) * np.pi * h)
    t = 2.0 - 2.0 * c
    m = 4.0 + 2.0 * c
    # axis order (z, y, x) of the nodal array; x is fastest in the numbering
    kappa = mu * h * (t[:, None, None] + t[None, :, None] + t[None, None, :])
    nu = (h / 6.0) ** 3 * (m[:, None, None] * m[None, :, None] * m[None, None, :])
    fhat = np.stack([dstn(F1[:, q].reshape(n, n, n), type=1, norm="ortho")
                     for q in range(F1.shape[1])], axis=-1)    # n x n x n x P
    W = np.zeros((n, n, n, nt))
    prev = np.zeros((n, n, n))
    for l in range(nt):
        rhs = fhat @ F2[l]
        if l > 0:
            rhs = rhs - (nu * Dt[l, l - 1] + kappa * Mt[l, l - 1]) * prev
        prev = rhs / (nu * Dt[l, l] + kappa * Mt[l, l])
        W[..., l] = prev
    U = np.empty((n ** 3, nt))
    for l in range(nt):
        U[:, l] = dstn(W[..., l], type=1, norm="ortho").ravel()
    return U


def sylvester_residual(Kx, Mx, Dt, Mt, F1, F2, U) -> float:
    """Relative Frobenius residual of eq. (Sylv_Heat) for a full U."""
    F = np.asarray(F1) @ np.asarray(F2).T
    R = F - (Kx @ (U @ np.asarray(Mt).T) + Mx @ (U @ np.asarray(Dt).T))
    return float(np.linalg.norm(R) / np.linalg.norm(F))


def relative_error(A: np.ndarray, B: np.ndarray) -> float:
    """||A - B||_F / ||B||_F on nodal coefficients."""
    return float(np.linalg.norm(A - B) / np.linalg.norm(B))
