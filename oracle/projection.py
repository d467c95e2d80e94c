"""Galerkin projection solver of Sec. 4, written plainly (oracle).

Given a basis V (Nh x k) of a spatial subspace, the approximation U_m = V Y is
fixed by the Galerkin condition V^T R = 0 on the residual
R = F1 F2^T - Kx V Y Mt^T - Mx V Y Dt^T, i.e. by the reduced equation

    (V^T Kx V) Y Mt^T + (V^T Mx V) Y Dt^T = (V^T F1) F2^T        (Sec. 4)

(the printed reduced equation carries a stray trailing V_m on the right-hand
side; its dimensions only allow V_m^T F).  The subspace is a rational Krylov
space in the operator A = Mx^{-1} Kx (since (Kx - s Mx)^{-1} Mx = (A - s I)^{-1}),
here with the two poles 0 and infinity (extended Krylov), started from
Mx^{-1} F1 and grown block by block (Sec. 4, rational Krylov paragraph):

    V_1      = orth([Mx^{-1} F1, Kx^{-1} F1])
    V_{j+1}  = orth([A V_j^+, A^{-1} V_j^-])  against all previous blocks,

where V_j^+ / V_j^- are the columns of block j descended from the
positive / negative powers.  Columns are orthonormal in the Mx inner product.
Inner solves are sparse-direct, so every step is exact up to rounding.  The
reduced equation is solved by forward block substitution in time, which is its
definition written out (block lower bidiagonal in time).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.linalg as sla
import scipy.sparse.linalg as spla


def m_orthonormalize(W: np.ndarray, V: np.ndarray, Mx, defl: float = 1e-10):
    """Orthonormalise the columns of W against V and each other in the Mx product.

    Modified Gram-Schmidt, applied twice per column.  A column whose Mx-norm
    after orthogonalisation falls below ``defl`` times its norm before is
    dropped (the space already contains it).  Returns (new columns, kept indices).
    """
    basis = [V[:, i] for i in range(V.shape[1])]
    out, kept = [], []
    for c in range(W.shape[1]):
        w = W[:, c].astype(float).copy()
        n0 = np.sqrt(w @ (Mx @ w))
        if n0 == 0.0:
            continue
        for _ in range(2):
            for v in basis + out:
                w -= (v @ (Mx @ w)) * v
        n1 = np.sqrt(w @ (Mx @ w))
        if n1 <= defl * n0:
            continue
        out.append(w / n1)
        kept.append(c)
    Wn = np.column_stack(out) if out else np.zeros((W.shape[0], 0))
    return Wn, kept


def galerkin_reduced_solve(Km, Mm, Dt, Mt, beta, F2) -> np.ndarray:
    """Solve Km Y Mt^T + Mm Y Dt^T = beta F2^T by forward substitution in time.

    Column l: (Mt[l,l] Km + Dt[l,l] Mm) y_l = beta F2[l] - (Mt[l,l-1] Km + Dt[l,l-1] Mm) y_{l-1}.
    """
    Dt = np.asarray(Dt)
    Mt = np.asarray(Mt)
    k, nt = Km.shape[0], F2.shape[0]
    Y = np.zeros((k, nt))
    for l in range(nt):
        rhs = beta @ F2[l]
        if l > 0:
            rhs = rhs - (Mt[l, l - 1] * Km + Dt[l, l - 1] * Mm) @ Y[:, l - 1]
        Y[:, l] = np.linalg.solve(Mt[l, l] * Km + Dt[l, l] * Mm, rhs)
    return Y


def reduced_eig_sweep(Km, Mm, Dt, Mt, beta, F2):
    """The reduced solve by diagonalising the spatial pencil (Sec. 4, reduced
    small Sylvester equation).

    Km Q = Mm Q diag(lam), Q^T Mm Q = I; with Y = Q Z each row z_i solves the
    scalar lower-bidiagonal system (Dt + lam_i Mt) z_i = (Q^T beta F2^T)[i].
    Returns (Y, lam, Q).
    """
    lam, Q = sla.eigh(Km, Mm)
    G = (Q.T @ beta) @ F2.T
    Z = np.zeros_like(G)
    for i in range(len(lam)):
        Z[i] = sla.solve_banded((1, 0), _bidiag_band(Dt, Mt, lam[i]), G[i])
    return Q @ Z, lam, Q


def _bidiag_band(Dt, Mt, lam):
    A = np.asarray(Dt) + lam * np.asarray(Mt)
    band = np.zeros((2, A.shape[0]))
    band[0] = np.diag(A)
    band[1, :-1] = np.diag(A, -1)
    return band


def galerkin_residual(Kx, Mx, Dt, Mt, F1, F2, V, Y) -> float:
    """Relative Frobenius norm of R = F1 F2^T - Kx V Y Mt^T - Mx V Y Dt^T."""
    U = V @ Y
    F = F1 @ F2.T
    R = F - Kx @ (U @ np.asarray(Mt).T) - Mx @ (U @ np.asarray(Dt).T)
    return float(np.linalg.norm(R) / np.linalg.norm(F))


@dataclass
class ProjectionResult:
    V: np.ndarray
    Y: np.ndarray
    outer: int
    history: list = field(default_factory=list)     # (k, relative residual) per step
    breakdown: bool = False


def extended_krylov_galerkin(Kx, Mx, Dt, Mt, F1, F2, tol: float = 1e-10,
                             max_outer: int = 200, defl: float = 1e-10) -> ProjectionResult:
    """Grow the extended Krylov space until the Galerkin residual is <= tol.

    Each step adds one block, solves the reduced equation on the enlarged
    space and evaluates the residual explicitly (relative Frobenius norm).
    Stops early if a whole block is deflated: the space is then invariant under
    A and A^{-1} and the Galerkin solution is the exact one.
    """
    F1 = np.asarray(F1, dtype=float)
    F2 = np.asarray(F2, dtype=float)
    luK = spla.splu(Kx.tocsc())
    luM = spla.splu(Mx.tocsc())
    p = F1.shape[1]
    X = np.column_stack([luM.solve(F1), luK.solve(F1)])
    tags = ["+"] * p + ["-"] * p
    V, kept = m_orthonormalize(X, np.zeros((Kx.shape[0], 0)), Mx, defl)
    block_tags = [tags[c] for c in kept]
    block = list(range(V.shape[1]))
    history = []
    breakdown = False
    Y = None
    for outer in range(1, max_outer + 1):
        Km = V.T @ (Kx @ V)
        Mm = V.T @ (Mx @ V)
        beta = V.T @ F1
        Y = galerkin_reduced_solve(Km, Mm, Dt, Mt, beta, F2)
        res = galerkin_residual(Kx, Mx, Dt, Mt, F1, F2, V, Y)
        history.append((V.shape[1], res))
        if res <= tol or breakdown:
            return ProjectionResult(V, Y, outer, history, breakdown)
        cols, new_tags = [], []
        for c, tg in zip(block, block_tags):
            v = V[:, c]
            cols.append(luM.solve(Kx @ v) if tg == "+" else luK.solve(Mx @ v))
            new_tags.append(tg)
        Wn, kept = m_orthonormalize(np.column_stack(cols), V, Mx, defl)
        if Wn.shape[1] == 0:
            breakdown = True
            continue
        block = list(range(V.shape[1], V.shape[1] + Wn.shape[1]))
        block_tags = [new_tags[c] for c in kept]
        V = np.column_stack([V, Wn])
    # not converged: the factors of the last reduced solve
    return ProjectionResult(V[:, :Y.shape[0]], Y, max_outer, history, breakdown)


# ---------------------------------------------------------------------------
# Rational Krylov space with adaptive shifts (Sec. 4, rational Krylov paragraph)
# ---------------------------------------------------------------------------
#
# Sec. 4 proposes RK_m = range([F1, (A_h - s_2 M_h)^{-1} M_h F1, ...]) with
# shifts chosen adaptively while the space grows, citing the survey of
# Simoncini for the rule.  In operator form this is the rational Krylov space
# of A = Mx^{-1} Kx with poles -s_j (s_j = -sigma_j > 0 for the SPD pencil),
# so each shifted direction solves (Kx + s Mx) w = Mx v.  Read with the same
# start block as the extended Krylov space ([Mx^{-1} F1, Kx^{-1} F1]: poles
# infinity and 0) and grown block by block (each new block is the shifted
# solve applied to the last one; for distinct shifts this spans the same
# space as the printed partial-fraction form).  The adaptive rule is the
# greedy one of Druskin and Simoncini (2011) for real spectra: with Ritz
# values theta_i of the current projected pencil, earlier shifts s_l and the
# spectral interval [a, b] of A,
#     s_next = argmax_{s in [a, b]}  prod_l |s - s_l| / prod_i |s + theta_i|,
# i.e. the point of the mirrored spectrum where the current rational function
# is largest in modulus.  The interval is the range of the Ritz values seen
# so far (widened as they move), the maximum is taken over a fine logarithmic
# grid of the interval.

def adaptive_shift(ritz, shifts, a: float, b: float, grid: int = 4001) -> float:
    """Next shift by the greedy rule above (log-spaced grid of [a, b], a > 0).

    The objective is evaluated in logarithms; its maximiser over the grid is
    returned (the first one if several tie)."""
    ritz = np.asarray(ritz, dtype=float)
    shifts = np.asarray(shifts, dtype=float)
    s = np.exp(np.linspace(np.log(a), np.log(b), grid))
    logf = np.zeros_like(s)
    for sl in shifts:
        logf += np.log(np.abs(s - sl) + 1e-300)
    for th in ritz:
        logf -= np.log(np.abs(s + th))
    return float(s[int(np.argmax(logf))])


def rational_krylov_galerkin(Kx, Mx, Dt, Mt, F1, F2, tol: float = 1e-10, max_outer: int = 200,
                             defl: float = 1e-10, shifts=None) -> ProjectionResult:
    """Grow the rational Krylov space until the Galerkin residual is <= tol.

    ``shifts``: an explicit list of shifts s_2, s_3, ... (used in order), or
    None for the adaptive rule.  Inner solves are sparse-direct.  The result's
    history holds (k, residual, shift) per step."""
    F1 = np.asarray(F1, dtype=float)
    F2 = np.asarray(F2, dtype=float)
    luK = spla.splu(Kx.tocsc())
    luM = spla.splu(Mx.tocsc())
    X = np.column_stack([luM.solve(F1), luK.solve(F1)])
    V, kept = m_orthonormalize(X, np.zeros((Kx.shape[0], 0)), Mx, defl)
    block = list(range(V.shape[1]))
    used, history = [], []
    lo, hi = np.inf, 0.0
    Y = None
    breakdown = False
    for outer in range(1, max_outer + 1):
        Km = V.T @ (Kx @ V)
        Mm = V.T @ (Mx @ V)
        beta = V.T @ F1
        Y = galerkin_reduced_solve(Km, Mm, Dt, Mt, beta, F2)
        res = galerkin_residual(Kx, Mx, Dt, Mt, F1, F2, V, Y)
        history.append((V.shape[1], res, used[-1] if used else None))
        if res <= tol or breakdown:
            return ProjectionResult(V, Y, outer, history, breakdown)
        theta = sla.eigh(Km, Mm, eigvals_only=True)
        lo, hi = min(lo, theta.min()), max(hi, theta.max())
        if shifts is not None:
            if len(used) >= len(shifts):
                break
            s = float(shifts[len(used)])
        else:
            s = adaptive_shift(theta, used, lo, hi)
        used.append(s)
        lu = spla.splu((Kx + s * Mx).tocsc())
        W = np.column_stack([lu.solve(Mx @ V[:, c]) for c in block])
        Wn, kept = m_orthonormalize(W, V, Mx, defl)
        if Wn.shape[1] == 0:
            breakdown = True
            continue
        block = list(range(V.shape[1], V.shape[1] + Wn.shape[1]))
        V = np.column_stack([V, Wn])
    # not converged: the factors of the last reduced solve
    return ProjectionResult(V[:, :Y.shape[0]], Y, len(history), history, breakdown)
