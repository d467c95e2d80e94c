"""Pins of the oracle's rational Krylov solver with adaptive shifts (Sec. 4,
rational Krylov paragraph): closed-form cases of the greedy shift rule, the
identity between the nested construction and the partial-fraction form of
the space, exactness on an invariant load, and agreement with the exact
Crank-Nicolson solution."""
import numpy as np
import scipy.linalg as sla
import scipy.sparse.linalg as spla

import workloads as wl
from oracle import exact, fem, projection


def test_shift_rule_without_earlier_shifts_takes_the_left_end():
    # prod_i 1 / (s + theta_i) decreases in s > 0: the maximiser is a
    s = projection.adaptive_shift([3.0, 40.0], [], 2.0, 500.0)
    assert s == 2.0


def test_shift_rule_with_one_shift_and_one_ritz_value():
    # f(s) = |s - s1| / (s + theta) decreases left of s1 and increases right
    # of it, so the maximiser is the end point with the larger value
    a, b, s1, th = 1.0, 1000.0, 30.0, 5.0
    fa, fb = (s1 - a) / (a + th), (b - s1) / (b + th)
    s = projection.adaptive_shift([th], [s1], a, b)
    assert s == (a if fa > fb else b)
    # with no Ritz value the farthest end point wins
    assert projection.adaptive_shift([], [900.0], 1.0, 1000.0) == 1.0


def test_shift_rule_avoids_earlier_shifts():
    a, b = 1.0, 1e4
    used = [1.0, 1e4, 100.0]
    s = projection.adaptive_shift([2.0, 50.0, 3000.0], used, a, b)
    assert a < s < b and min(abs(np.log(s / u)) for u in used) > 0.5


def _principal_sines(A, B, M):
    """Largest sine of the principal angles between range(A) and range(B) in
    the M inner product."""
    L = np.linalg.cholesky(M.toarray())
    qa, _ = np.linalg.qr(L.T @ A)
    qb, _ = np.linalg.qr(L.T @ B)
    s = sla.svdvals(qb - qa @ (qa.T @ qb))
    return float(s.max())


def test_nested_construction_spans_the_partial_fraction_space():
    n, nt = 40, 8
    w = wl.heat_1d_profiles(n=n, nt=nt, p=1, seed=3)
    K, M = fem.spatial_operators(1, n, 1.0)
    Dt, Mt = fem.time_matrices(wl.time_grid(nt, 1.0))
    shifts = [7.0, 300.0, 55.0]
    r = projection.rational_krylov_galerkin(K, M, Dt, Mt, w.F1, w.F2, tol=0.0, max_outer=4,
                                            shifts=shifts)
    assert r.V.shape[1] == 5
    F1 = w.F1
    cols = [spla.spsolve(M.tocsc(), F1[:, 0]), spla.spsolve(K.tocsc(), F1[:, 0])]
    cols += [spla.spsolve((K + s * M).tocsc(), F1[:, 0]) for s in shifts]
    P = np.column_stack(cols)
    assert _principal_sines(r.V, P, M) < 1e-8
    # a wrong sign of the shift gives another space
    Pw = np.column_stack(cols[:2] + [spla.spsolve((K - s * M).tocsc(), F1[:, 0])
                                     for s in shifts])
    assert _principal_sines(r.V, Pw, M) > 1e-3


def test_invariant_load_gives_exact_solution():
    w = wl.heat_1d_sine(nx=63, nt=32)
    K, M = fem.spatial_operators(1, 63, 1.0)
    Dt, Mt = fem.time_matrices(wl.time_grid(32, 1.0))
    r = projection.rational_krylov_galerkin(K, M, Dt, Mt, w.F1, w.F2, tol=1e-12)
    U = exact.kron_solve(K, M, Dt, Mt, w.F1, w.F2)
    assert r.V.shape[1] == 1          # the start block deflates to the eigenvector
    assert np.linalg.norm(r.V @ r.Y - U) <= 1e-12 * np.linalg.norm(U)


def test_adaptive_rksm_matches_crank_nicolson_with_a_smaller_basis():
    w = wl.heat_2d_bumps(n=31, nt=32, p=2, seed=4)
    K, M = fem.spatial_operators(2, 31, w.mu)
    Dt, Mt = fem.time_matrices(wl.time_grid(32, 1.0))
    U = exact.crank_nicolson(K, M, Dt, Mt, w.F1, w.F2)
    rk = projection.rational_krylov_galerkin(K, M, Dt, Mt, w.F1, w.F2, tol=1e-10)
    ek = projection.extended_krylov_galerkin(K, M, Dt, Mt, w.F1, w.F2, tol=1e-10)
    assert rk.history[-1][1] <= 1e-10
    assert np.linalg.norm(rk.V @ rk.Y - U) <= 1e-8 * np.linalg.norm(U)
    # one block of P columns per shift instead of 2P per extended step
    assert rk.V.shape[1] < ek.V.shape[1]
    # the shifts stay inside the Ritz interval
    th = sla.eigh(rk.V.T @ (K @ rk.V), rk.V.T @ (M @ rk.V), eigvals_only=True)
    for _, _, s in rk.history[1:]:
        assert th.min() * 0.999 <= s <= th.max() * 1.001
