"""Pins of the oracle's exact space-time solvers and projection method (CPU only).

Every check compares two routes that share no arithmetic, or compares against a
closed form / textbook fact, so a dropped term, wrong sign or transposed
operand in any one route fails a test.
"""
import math

import numpy as np
import pytest
import scipy.sparse as sp

import workloads as wl
from oracle import closed_form, exact, fem, projection


def _setup(w):
    K, M = fem.spatial_operators(w.dim, w.n[0], w.mu)
    Dt, Mt = fem.time_matrices(wl.time_grid(w.nt, w.T))
    return K, M, Dt, Mt


def test_vec_identity_bruteforce():
    """(D kron A) vec X == vec(A X D^T) with column stacking (Sec. 4)."""
    rng = np.random.default_rng(5)
    A, D, X = rng.normal(size=(4, 4)), rng.normal(size=(3, 3)), rng.normal(size=(4, 3))
    np.testing.assert_allclose(np.kron(D, A) @ exact.vec(X), exact.vec(A @ X @ D.T), rtol=1e-13)
    # and the transposed operand ordering is genuinely different
    assert np.linalg.norm(np.kron(A[:3, :3], D) @ exact.vec(X[:3]) - exact.vec(A[:3, :3] @ X[:3] @ D.T)) > 1e-3


def test_c1_kron_equals_crank_nicolson_and_closed_form():
    w = wl.heat_1d_sine()
    K, M, Dt, Mt = _setup(w)
    Uk = exact.kron_solve(K, M, Dt, Mt, w.F1, w.F2)
    Uc = exact.crank_nicolson(K, M, Dt, Mt, w.F1, w.F2)
    h = 1.0 / (w.n[0] + 1)
    scale = 2 * (1 - math.cos(math.pi * h)) / (math.pi ** 2 * h)
    Us = closed_form.sine_mode_solution_1d(w.n[0], w.mu, Dt, Mt, w.F2, scale)
    assert exact.relative_error(Uc, Uk) < 1e-12
    assert exact.relative_error(Us, Uk) < 1e-12
    assert exact.sylvester_residual(K, M, Dt, Mt, w.F1, w.F2, Uk) < 1e-12
    s = np.linalg.svd(Uk, compute_uv=False)
    assert s[1] < 1e-12 * s[0]                         # rank one


def test_modal_solve_matches_kron_on_random_rhs():
    rng = np.random.default_rng(11)
    n, nt = 23, 17
    K, M = fem.p1_1d(n, 0.6)
    t = np.cumsum(np.r_[0.0, rng.uniform(0.02, 0.1, nt)])   # graded time grid
    Dt, Mt = fem.time_matrices(t)
    F1, F2 = rng.normal(size=(n, 3)), rng.normal(size=(nt, 3))
    Uk = exact.kron_solve(K, M, Dt, Mt, F1, F2)
    assert exact.relative_error(exact.modal_solve_1d(n, 0.6, Dt, Mt, F1, F2), Uk) < 1e-12
    assert exact.relative_error(exact.crank_nicolson(K, M, Dt, Mt, F1, F2), Uk) < 1e-12


@pytest.mark.parametrize("n", [1, 2, 23, 100])
def test_modal_solve_1d_fast_matches_kron_and_mode_loop(n):
    """The DST-based 1-D modal solve against the assembled Kronecker system
    (graded time grid, random data) and against the explicit mode loop."""
    rng = np.random.default_rng(40 + n)
    nt = 13
    K, M = fem.p1_1d(n, 0.45)
    t = np.cumsum(np.r_[0.0, rng.uniform(0.02, 0.1, nt)])
    Dt, Mt = fem.time_matrices(t)
    F1, F2 = rng.normal(size=(n, 2)), rng.normal(size=(nt, 2))
    Uf = exact.modal_solve_1d_fast(n, 0.45, Dt, Mt, F1, F2)
    assert exact.relative_error(Uf, exact.kron_solve(K, M, Dt, Mt, F1, F2)) < 1e-12
    assert exact.relative_error(Uf, exact.modal_solve_1d(n, 0.45, Dt, Mt, F1, F2)) < 1e-12


def test_modal_solve_1d_fast_sylvester_residual_at_large_n():
    """At n = 4095 (Kronecker too large) the fast modal solution satisfies
    eq. (Sylv_Heat) to its FP64 rounding level, and Crank-Nicolson agrees."""
    w = wl.heat_1d_profiles(n=4095, nt=64, p=2, seed=7)
    K, M, Dt, Mt = _setup(w)
    Uf = exact.modal_solve_1d_fast(4095, w.mu, Dt, Mt, w.F1, w.F2)
    assert exact.sylvester_residual(K, M, Dt, Mt, w.F1, w.F2, Uf) < 1e-8
    assert exact.relative_error(exact.crank_nicolson(K, M, Dt, Mt, w.F1, w.F2), Uf) < 1e-9


def test_crank_nicolson_chunks_equal_one_march():
    """The chunked march carries u^{l0} exactly: its pieces concatenate to the
    single march bitwise, also for a graded grid and a chunk that leaves a
    ragged tail."""
    rng = np.random.default_rng(3)
    n, nt = 15, 23
    K, M = fem.spatial_operators(2, n, 0.8)
    t = np.cumsum(np.r_[0.0, rng.uniform(0.02, 0.1, nt)])
    Dt, Mt = fem.time_matrices(t)
    F1, F2 = rng.normal(size=(n * n, 2)), rng.normal(size=(nt, 2))
    U = exact.crank_nicolson(K, M, Dt, Mt, F1, F2)
    parts = list(exact.crank_nicolson_chunks(K, M, Dt, Mt, F1, F2, chunk=5))
    assert [l0 for l0, _ in parts] == [0, 5, 10, 15, 20]
    assert np.array_equal(np.hstack([P for _, P in parts]), U)


@pytest.mark.parametrize("n", [1, 4, 7])
def test_modal_solve_3d_matches_kron_on_random_rhs(n):
    rng = np.random.default_rng(12 + n)
    nt, mu = 9, 0.7
    K, M = fem.spatial_operators(3, n, mu)
    t = np.cumsum(np.r_[0.0, rng.uniform(0.02, 0.1, nt)])   # graded time grid
    Dt, Mt = fem.time_matrices(t)
    F1, F2 = rng.normal(size=(n ** 3, 2)), rng.normal(size=(nt, 2))
    Uk = exact.kron_solve(K, M, Dt, Mt, F1, F2)
    assert exact.relative_error(exact.modal_solve_3d(n, mu, Dt, Mt, F1, F2), Uk) < 1e-12


def test_2d_kron_equals_crank_nicolson():
    w = wl.heat_2d_bumps(n=15, nt=24, p=2, seed=3)
    K, M, Dt, Mt = _setup(w)
    Uk = exact.kron_solve(K, M, Dt, Mt, w.F1, w.F2)
    assert exact.relative_error(exact.crank_nicolson(K, M, Dt, Mt, w.F1, w.F2), Uk) < 1e-12
    assert exact.sylvester_residual(K, M, Dt, Mt, w.F1, w.F2, Uk) < 1e-12


def test_crank_nicolson_classic_form():
    """With the uniform pair the step matrix is M + dt/2 K and the history term
    is (M - dt/2 K) u^{l-1} (Sec. 3: the scheme is Crank-Nicolson)."""
    w = wl.heat_1d_sine(nx=31, nt=20, seed=4)
    K, M, Dt, Mt = _setup(w)
    dt = w.T / w.nt
    U = exact.crank_nicolson(K, M, Dt, Mt, w.F1, w.F2)
    import scipy.sparse.linalg as spla
    u = np.zeros(31)
    for l in range(w.nt):
        u = spla.spsolve((M + dt / 2 * K).tocsc(), (M - dt / 2 * K) @ u + w.F1[:, 0] * w.F2[l, 0])
        np.testing.assert_allclose(U[:, l], u, rtol=1e-12, atol=1e-15)


def test_manufactured_second_order():
    """u = sin(pi x) omega(t), omega(t) = t + t^2 - t^3: nodal error O(h^2 + dt^2)."""
    omega, G = closed_form.manufactured_omega([1.0, 1.0, -1.0])
    errs = []
    for n in (15, 31, 63):
        nt = n + 1
        K, M = fem.p1_1d(n)
        t = wl.time_grid(nt)
        Dt, Mt = fem.time_matrices(t)
        F1 = wl.sine_load_1d(n)[:, None]
        F2 = (G(t[1:]) - G(t[:-1]))[:, None]
        U = exact.crank_nicolson(K, M, Dt, Mt, F1, F2)
        x = np.arange(1, n + 1) / (n + 1)
        Uex = np.outer(np.sin(np.pi * x), omega(t[1:]))
        errs.append(exact.relative_error(U, Uex))
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert all(1.9 < r < 2.1 for r in rates), (errs, rates)


@pytest.mark.parametrize("n,nt", [(15, 32), (31, 16)])
def test_projection_converges_to_exact(n, nt):
    w = wl.heat_2d_bumps(n=n, nt=nt, p=2, seed=6)
    K, M, Dt, Mt = _setup(w)
    Uk = exact.kron_solve(K, M, Dt, Mt, w.F1, w.F2)
    r = projection.extended_krylov_galerkin(K, M, Dt, Mt, w.F1, w.F2, tol=1e-11)
    V, Y = r.V, r.Y
    assert r.history[-1][1] <= 1e-11
    assert exact.relative_error(V @ Y, Uk) < 1e-9
    np.testing.assert_allclose(V.T @ (M @ V), np.eye(V.shape[1]), atol=1e-12)
    R = w.F1 @ w.F2.T - K @ (V @ Y @ Mt.T) - M @ (V @ Y @ Dt.T)
    assert np.linalg.norm(V.T @ R) < 1e-10 * np.linalg.norm(w.F1 @ w.F2.T)   # Galerkin condition
    ks = [h[0] for h in r.history]
    assert ks == sorted(ks) and ks[-1] <= 4 * len(ks)


def test_projection_c1_breaks_down_to_rank_one():
    w = wl.heat_1d_sine()
    K, M, Dt, Mt = _setup(w)
    r = projection.extended_krylov_galerkin(K, M, Dt, Mt, w.F1, w.F2, tol=1e-14)
    assert r.V.shape[1] == 1 and r.breakdown
    Uk = exact.kron_solve(K, M, Dt, Mt, w.F1, w.F2)
    assert exact.relative_error(r.V @ r.Y, Uk) < 1e-12


def test_reduced_sweep_equals_block_substitution():
    Km, Mm, beta, F2 = wl.random_reduced_problem(40, 64, 3, seed=9)
    t = np.cumsum(np.r_[0.0, np.random.default_rng(1).uniform(0.005, 0.03, 64)])
    Dt, Mt = fem.time_matrices(t)
    Y1 = projection.galerkin_reduced_solve(Km, Mm, Dt, Mt, beta, F2)
    Y2, lam, Q = projection.reduced_eig_sweep(Km, Mm, Dt, Mt, beta, F2)
    assert exact.relative_error(Y2, Y1) < 1e-10
    np.testing.assert_allclose(Q.T @ Mm @ Q, np.eye(40), atol=1e-12)


# ---- planted mistakes: each pin above must reject a plausible oracle bug ----

def test_pin_rejects_wrong_subdiagonal_sign():
    w = wl.heat_1d_sine(nx=31, nt=32)
    K, M, Dt, Mt = _setup(w)
    Mt_bad = Mt.copy()
    Mt_bad[np.arange(1, 32), np.arange(31)] *= -1
    h = 1.0 / 32
    scale = 2 * (1 - math.cos(math.pi * h)) / (math.pi ** 2 * h)
    Us = closed_form.sine_mode_solution_1d(31, 1.0, Dt, Mt, w.F2, scale)
    assert exact.relative_error(exact.crank_nicolson(K, M, Dt, Mt_bad, w.F1, w.F2), Us) > 1e-3


def test_pin_rejects_transposed_kronecker():
    w = wl.heat_1d_sine(nx=15, nt=16)
    K, M, Dt, Mt = _setup(w)
    Uc = exact.crank_nicolson(K, M, Dt, Mt, w.F1, w.F2)
    B_bad = (sp.kron(sp.csr_matrix(Dt.T), M) + sp.kron(sp.csr_matrix(Mt.T), K)).tocsc()
    import scipy.sparse.linalg as spla
    U_bad = exact.unvec(spla.spsolve(B_bad, exact.vec(w.F1 @ w.F2.T)), 15)
    assert exact.relative_error(U_bad, Uc) > 1e-2


def test_pin_rejects_dropped_mass_term():
    w = wl.heat_1d_sine(nx=31, nt=32)
    K, M, Dt, Mt = _setup(w)
    omega, G = closed_form.manufactured_omega([1.0, 1.0, -1.0])
    t = wl.time_grid(32)
    F2 = (G(t[1:]) - G(t[:-1]))[:, None]
    U_bad = exact.crank_nicolson(K, 0 * M + 1e-30 * sp.identity(31), Dt, Mt, w.F1, F2)
    x = np.arange(1, 32) / 32
    assert exact.relative_error(U_bad, np.outer(np.sin(np.pi * x), omega(t[1:]))) > 0.1
