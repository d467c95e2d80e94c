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
