"""CPU pins of the reference multigrid V-cycle (tests/mg_reference.py).

The reference is checked against facts that do not depend on it: the
Galerkin identity of nested P1 spaces against the oracle's assembled
stiffness, the symmetry and positivity a V-cycle with adjoint smoothing must
have, the bound Bmg <= Kx^{-1} (the error propagator I - Bmg Kx is
Kx-positive semidefinite), and h-independent PCG iteration counts.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import mg_reference as mgr


@pytest.mark.parametrize("nc", [1, 3, 15, 31])
def test_galerkin_coarse_operator_is_the_coarse_stiffness(nc):
    mu = 0.37
    P = mgr.prolongation(nc)
    Kf = mgr.stiffness(2 * nc + 1, mu)
    Kc = mgr.stiffness(nc, mu)
    assert abs(P.T @ Kf @ P - Kc).max() <= 1e-13


def test_prolongation_reproduces_linear_functions():
    """P1 interpolation is exact for functions linear on the coarse mesh."""
    nc = 7
    n = 2 * nc + 1
    xc = np.arange(1, nc + 1) / (nc + 1)
    xf = np.arange(1, n + 1) / (n + 1)
    Xc, Yc = np.meshgrid(xc, xc, indexing="xy")
    Xf, Yf = np.meshgrid(xf, xf, indexing="xy")
    f = lambda x, y: 0.3 + 2.0 * x - 1.5 * y
    got = mgr.prolongation(nc) @ f(Xc, Yc).ravel()
    want = f(Xf, Yf).ravel()
    inner = ((Xf > xf[0]) & (Xf < xf[-1]) & (Yf > xf[0]) & (Yf < xf[-1])).ravel()
    np.testing.assert_allclose(got[inner], want[inner], rtol=0, atol=1e-14)


def test_hat_function_pins():
    assert mgr.hat(0.0, 0.0) == 1.0
    assert mgr.hat(0.5, 0.5) == 0.5 and mgr.hat(-0.5, -0.5) == 0.5     # SW-NE edge
    assert mgr.hat(0.5, -0.5) == 0.0 and mgr.hat(-0.5, 0.5) == 0.0     # no SE-NW edge
    assert mgr.hat(1.0, 0.0) == 0.0 and mgr.hat(0.5, 0.0) == 0.5


@pytest.mark.parametrize("n", [1, 2, 15, 40, 63, 127])
def test_vcycle_is_spd_and_below_the_inverse(n):
    mu = 1.7
    rng = np.random.default_rng(n)
    R = rng.normal(size=(n * n, 3))
    Z = mgr.vcycle(R, n, mu)
    G = R.T @ Z
    np.testing.assert_allclose(G, G.T, rtol=1e-12, atol=1e-14 * abs(G).max())
    assert np.all(np.diag(G) > 0)          # (r, Bmg r) > 0
    # (r, Bmg r) <= (r, Kx^{-1} r)
    K = mgr.stiffness(n, mu)
    X = spla.spsolve(K.tocsc(), R)
    X = X.reshape(R.shape)
    for j in range(3):
        assert R[:, j] @ Z[:, j] <= R[:, j] @ X[:, j] * (1 + 1e-12)


def _pcg(K, b, prec, rtol):
    x = np.zeros_like(b)
    r = b.copy()
    z = prec(r)
    p = z.copy()
    rho = r @ z
    for it in range(1, 200):
        q = K @ p
        a = rho / (p @ q)
        x += a * p
        r -= a * q
        if np.linalg.norm(r) <= rtol * np.linalg.norm(b):
            return x, it
        z = prec(r)
        rho, rho0 = r @ z, rho
        p = z + rho / rho0 * p
    return x, -1


def test_pcg_iterations_do_not_grow_with_refinement():
    its = []
    for n in (63, 127, 255, 511):
        K = mgr.stiffness(n, 1.0)
        b = np.random.default_rng(n).normal(size=n * n)
        x, it = _pcg(K, b, lambda r: mgr.vcycle(r, n, 1.0), 1e-12)
        assert it > 0 and np.linalg.norm(b - K @ x) <= 1e-12 * np.linalg.norm(b)
        its.append(it)
    assert its[0] == 1, its                      # n <= 63: the V-cycle is the exact inverse
    assert max(its[1:]) <= 12 and its[-1] - its[1] <= 2, its


def test_galerkin_coarse_mass_is_the_coarse_mass():
    """The shifted V-cycle relies on P^T Mx_h P = Mx_2h as well (nested P1)."""
    from oracle import fem
    for nc in (1, 3, 15):
        P = mgr.prolongation(nc)
        Mf = fem.spatial_operators(2, 2 * nc + 1)[1]
        Mc = fem.spatial_operators(2, nc)[1]
        assert abs(P.T @ Mf @ P - Mc).max() <= 1e-15


def test_mass_stand_in_is_the_mass_without_the_diagonal_coupling():
    from oracle import fem
    n = 9
    M = fem.spatial_operators(2, n)[1].toarray()
    Ms = mgr.mass_stand_in(n).toarray()
    D = M - Ms
    w = (1.0 / (n + 1)) ** 2 / 12.0
    # what is left is w at the SW and NE neighbours only
    idx = np.arange(n * n)
    x, y = idx % n, idx // n
    for a in range(n * n):
        for b in np.nonzero(abs(D[a]) > 1e-3 * w)[0]:
            assert (x[b] - x[a], y[b] - y[a]) in ((1, 1), (-1, -1))
            assert abs(D[a, b] - w) <= 1e-12 * w
    assert np.all(np.linalg.eigvalsh(Ms) > 0)


@pytest.mark.parametrize("n,shift", [(40, 50.0), (127, 300.0), (127, 2.0e4)])
def test_shifted_vcycle_is_spd_and_converges(n, shift):
    from oracle import fem
    mu = 0.8
    K, M = fem.spatial_operators(2, n, mu)
    A = (K + shift * M).tocsc()
    rng = np.random.default_rng(n)
    R = rng.normal(size=(n * n, 2))
    Z = mgr.vcycle(R, n, mu, shift=shift)
    G = R.T @ Z
    np.testing.assert_allclose(G, G.T, rtol=1e-12, atol=1e-14 * abs(G).max())
    assert np.all(np.diag(G) > 0)
    b = R[:, 0]
    x, it = _pcg(A, b, lambda r: mgr.vcycle(r, n, mu, shift=shift), 1e-12)
    assert it > 0 and np.linalg.norm(b - A @ x) <= 1e-12 * np.linalg.norm(b)
    assert it <= 20, it


def test_supported_grids():
    assert all(mgr.supported(n) for n in (1, 2, 31, 62, 63, 65, 97, 125, 127, 129, 255, 511,
                                          1023, 2047))
    assert not any(mgr.supported(n) for n in (64, 100, 130, 256, 510, 1022))


@pytest.mark.parametrize("n", [1, 2, 7, 16, 31])
def test_mass_spectrum_inside_the_chebyshev_interval(n):
    """The Chebyshev Mx solve relies on spec(diag(Mx)^{-1} Mx) within [1/2, 2]
    (the range of the mass stencil's symbol), checked on the assembled matrix."""
    from oracle import fem
    M = fem.spatial_operators(2, n, 1.0)[1].toarray()
    d = np.diag(M)
    ev = np.linalg.eigvalsh(M / np.sqrt(np.outer(d, d)))
    assert ev.min() >= 0.5 - 1e-12 and ev.max() <= 2.0 + 1e-12, (ev.min(), ev.max())


# ---------------------------------------------------------------------------
# 3-D (seven-point stiffness, Kuhn-mesh interpolation)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("n", [1, 2, 5, 8])
def test_kronecker_stiffness_equals_the_element_assembly(n):
    from oracle import fem
    K = fem.spatial_operators(3, n, 0.45)[0]
    assert abs(mgr.stiffness3(n, 0.45) - K).max() <= 1e-15


@pytest.mark.parametrize("nc", [1, 3, 7])
def test_galerkin_coarse_operator_is_the_coarse_stiffness_3d(nc):
    """P^T K_h P = K_2h: the seven-point stencil with mu h is the P1 stiffness
    of the Kuhn mesh, and the meshes nest."""
    mu = 0.61
    P = mgr.prolongation3(nc)
    assert abs(P.T @ mgr.stiffness3(2 * nc + 1, mu) @ P - mgr.stiffness3(nc, mu)).max() <= 1e-13


def test_prolongation_reproduces_linear_functions_3d():
    nc = 5
    n = 2 * nc + 1
    xc = np.arange(1, nc + 1) / (nc + 1)
    xf = np.arange(1, n + 1) / (n + 1)
    f = lambda x, y, z: 0.3 + 2.0 * x - 1.5 * y + 0.7 * z
    Zc, Yc, Xc = np.meshgrid(xc, xc, xc, indexing="ij")
    Zf, Yf, Xf = np.meshgrid(xf, xf, xf, indexing="ij")
    got = mgr.prolongation3(nc) @ f(Xc, Yc, Zc).ravel()
    want = f(Xf, Yf, Zf).ravel()
    lo, hi = xf[0], xf[-1]
    inner = ((Xf > lo) & (Xf < hi) & (Yf > lo) & (Yf < hi) & (Zf > lo) & (Zf < hi)).ravel()
    np.testing.assert_allclose(got[inner], want[inner], rtol=0, atol=1e-14)


def test_kuhn_hat_pins():
    assert mgr.kuhn_hat(0.0, 0.0, 0.0) == 1.0
    # midpoints of the seven edge directions (both orientations)
    for e in [(1, 0, 0), (0, 1, 0), (0, 0, 1), (1, 1, 0), (1, 0, 1), (0, 1, 1), (1, 1, 1)]:
        v = np.array(e) / 2.0
        assert mgr.kuhn_hat(*v) == 0.5 and mgr.kuhn_hat(*-v) == 0.5
    # mixed-sign diagonals are not edges of the Kuhn mesh
    for v in [(0.5, -0.5, 0.0), (0.5, 0.0, -0.5), (0.0, 0.5, -0.5), (0.5, 0.5, -0.5),
              (0.5, -0.5, 0.5), (-0.5, 0.5, 0.5)]:
        assert mgr.kuhn_hat(*v) == 0.0
    assert mgr.kuhn_hat(1.0, 0.0, 0.0) == 0.0


@pytest.mark.parametrize("n", [1, 2, 9])
def test_exact3_is_the_inverse(n):
    K = mgr.stiffness3(n, 0.8)
    B = np.random.default_rng(n).normal(size=(n ** 3, 2))
    X = spla.spsolve(K.tocsc(), B).reshape(B.shape)
    np.testing.assert_allclose(mgr.exact3(B, n, 0.8), X, rtol=1e-12, atol=1e-13 * abs(X).max())


def test_vcycle3_is_spd_and_below_the_inverse():
    n, mu = 65, 1.3
    R = np.random.default_rng(n).normal(size=(n ** 3, 3))
    Z = mgr.vcycle3(R, n, mu)
    G = R.T @ Z
    np.testing.assert_allclose(G, G.T, rtol=1e-12, atol=1e-14 * abs(G).max())
    assert np.all(np.diag(G) > 0)
    X = mgr.exact3(R, n, mu)
    for j in range(3):
        assert R[:, j] @ Z[:, j] <= R[:, j] @ X[:, j] * (1 + 1e-12)


def test_pcg3_iterations_stay_small():
    its = []
    for n in (31, 65):
        K = mgr.stiffness3(n, 1.0)
        b = np.random.default_rng(n).normal(size=n ** 3)
        x, it = _pcg(K, b, lambda r: mgr.vcycle3(r, n, 1.0), 1e-12)
        assert it > 0 and np.linalg.norm(b - K @ x) <= 1e-12 * np.linalg.norm(b)
        its.append(it)
    assert its[0] == 1, its          # n <= 63: the V-cycle is the exact inverse
    assert its[1] <= 12, its


@pytest.mark.parametrize("n", [1, 2, 5])
def test_kronecker_mass_equals_the_element_assembly(n):
    from oracle import fem
    M = fem.spatial_operators(3, n, 0.45)[1]
    assert abs(mgr.mass3(n) - M).max() <= 1e-14 * abs(M).max()


def test_exact3_shifted_is_the_inverse():
    n, mu, s = 9, 0.8, 120.0
    A = (mgr.stiffness3(n, mu) + s * mgr.mass3(n)).tocsc()
    B = np.random.default_rng(4).normal(size=(n ** 3, 2))
    X = spla.spsolve(A, B).reshape(B.shape)
    np.testing.assert_allclose(mgr.exact3(B, n, mu, s), X, rtol=1e-12, atol=1e-13 * abs(X).max())


@pytest.mark.parametrize("shift", [30.0, 3e3])
def test_shifted_vcycle3_is_spd_and_converges(shift):
    n, mu = 65, 1.1
    A = (mgr.stiffness3(n, mu) + shift * mgr.mass3(n)).tocsr()
    R = np.random.default_rng(9).normal(size=(n ** 3, 2))
    Z = mgr.vcycle3(R, n, mu, shift)
    G = R.T @ Z
    np.testing.assert_allclose(G, G.T, rtol=1e-12, atol=1e-14 * abs(G).max())
    assert np.all(np.diag(G) > 0)
    b = R[:, 0]
    x, it = _pcg(A, b, lambda r: mgr.vcycle3(r, n, mu, shift), 1e-12)
    assert it > 0 and np.linalg.norm(b - A @ x) <= 1e-12 * np.linalg.norm(b)
    assert it <= 20, it


def test_supported_grids_3d():
    assert all(mgr.supported3(n) for n in (1, 2, 40, 63, 95, 127, 191, 255, 511))
    assert not any(mgr.supported3(n) for n in (64, 100, 128, 254))
