"""GPU parity of the multigrid-preconditioned inner solver.

The V-cycle is compared entry by entry with the reference of
``tests/mg_reference.py``; the preconditioned CG solves with the oracle's
sparse direct solve; whole solves with the preconditioner on and off with the
oracle's Crank-Nicolson solution.  All calls go through the C ABI.
"""
import math

import numpy as np
import pytest
import scipy.sparse.linalg as spla

import mg_reference as mgr
import paper_1912_10082_amd as sts
import workloads as wl
from oracle import exact, fem

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    sts.load()


def dev(a):
    return torch.from_numpy(np.asfortranarray(a, dtype=np.float64)).cuda()


def host(t):
    return t.detach().cpu().numpy()


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


# Sizes: exact solves in one work-group alone (1 .. 63, even 62), one tiled
# level above a one-work-group exact solve with a coarse grid that is an
# exact multiple of the tile in x (65 -> 32) or in y (97 -> 48) or ragged
# (81 -> 40, 125 -> 62, 127 -> 63), one tiled level above the many-work-group
# exact solve (129 -> 64, 255 -> 127, 511 -> 255), and two tiled levels
# (1023 -> 511 -> 255).
VC_SIZES = [1, 2, 3, 31, 33, 62, 63, 65, 81, 97, 125, 127, 129, 255, 511, 1023]


@pytest.mark.parametrize("n", VC_SIZES)
def test_vcycle_matches_reference(n):
    mu = 0.25 + 0.1 * (n % 7)
    rng = np.random.default_rng(200 + n)
    R = rng.normal(size=(n * n, 3))
    R[:, 2] = 0.0                                   # a zero column stays zero
    Z = host(sts.mg_vcycle(sts.make_space(2, n, mu), dev(R)))
    Zr = mgr.vcycle(R, n, mu)
    scale = abs(Zr).max()
    # the reference's sparse LU on the 255^2 coarse grid is accurate to about
    # kappa eps (kappa ~ 3e4); two smoothed levels above it amplify that
    tol = 1e-13 if n < 1023 else 1e-11
    np.testing.assert_allclose(Z, Zr, rtol=0, atol=tol * scale)
    assert np.all(Z[:, 2] == 0.0)


def test_vcycle_symmetric_and_below_the_inverse():
    n, mu = 127, 1.3
    rng = np.random.default_rng(5)
    R = rng.normal(size=(n * n, 4))
    Z = host(sts.mg_vcycle(sts.make_space(2, n, mu), dev(R)))
    G = R.T @ Z
    np.testing.assert_allclose(G, G.T, rtol=1e-12, atol=1e-14 * abs(G).max())
    K = fem.spatial_operators(2, n, mu)[0].tocsc()
    X = spla.spsolve(K, R)
    for j in range(4):
        assert 0.0 < R[:, j] @ Z[:, j] <= R[:, j] @ X[:, j] * (1 + 1e-12)


@pytest.mark.parametrize("n,ncols", [(1, 1), (31, 2), (65, 3), (127, 8), (255, 4), (511, 2)])
def test_pcg_matches_sparse_direct(n, ncols):
    mu = 0.7
    rng = np.random.default_rng(300 + n)
    B = rng.normal(size=(n * n, ncols))
    X, its, _ = sts.pcg_mg(sts.make_space(2, n, mu), dev(B), rtol=1e-12)
    X = host(X)
    K = fem.spatial_operators(2, n, mu)[0].tocsc()
    for c in range(ncols):
        assert np.linalg.norm(B[:, c] - K @ X[:, c]) <= 1e-12 * np.linalg.norm(B[:, c])
        x_ref = spla.spsolve(K, B[:, c])
        assert rel(X[:, c], x_ref) < 1e-9, (c, rel(X[:, c], x_ref))
    # mesh-independent convergence (unpreconditioned CG needs ~1900 at n = 511)
    assert max(its) <= 13, its


def test_pcg_zero_rhs_iteration_cap_and_bad_grids():
    space = sts.make_space(2, 127)
    B = np.zeros((127 * 127, 2))
    B[:, 1] = np.random.default_rng(1).normal(size=127 * 127)
    X, its, code = sts.pcg_mg(space, dev(B), rtol=1e-14, maxit=3, check=False)
    assert its[0] == 0 and np.all(host(X)[:, 0] == 0.0)
    assert its[1] == 3 and code == 4                   # STS_E_NOT_CONVERGED (maxit)
    # n <= 63: the V-cycle is the exact inverse, one iteration
    B = np.random.default_rng(2).normal(size=(63 * 63, 1))
    X, its, _ = sts.pcg_mg(sts.make_space(2, 63), dev(B), rtol=1e-12)
    assert its[0] == 1
    for bad in (sts.make_space(2, 100), sts.make_space(2, 130), sts.make_space(1, 127),
                sts.make_space(3, 100), sts.make_space(3, 128)):
        nh = int(np.prod([bad.n[d] for d in range(3)]))
        with pytest.raises(sts.STSError) as e:
            sts.pcg_mg(bad, dev(np.ones((nh, 1))))
        assert e.value.code == 1


@pytest.mark.parametrize("n,shift", [(1, 3.0), (31, 40.0), (65, 300.0), (127, 2e4), (191, 7.0),
                                     (255, 50.0), (511, 1e5)])
def test_shifted_vcycle_matches_reference(n, shift):
    """The V-cycle for Kx + shift Mx (rational Krylov's shifted solves): every
    level's operator carries the mass term, the coarsest solve its stand-in."""
    mu = 0.6
    rng = np.random.default_rng(800 + n)
    R = rng.normal(size=(n * n, 2))
    Z = host(sts.mg_vcycle(sts.make_space(2, n, mu), dev(R), shift=shift))
    Zr = mgr.vcycle(R, n, mu, shift=shift)
    np.testing.assert_allclose(Z, Zr, rtol=0, atol=1e-12 * abs(Zr).max())


@pytest.mark.parametrize("n,shift", [(1, 2.0), (40, 30.0), (65, 3e3), (127, 40.0)])
def test_shifted_vcycle3_matches_reference(n, shift):
    """3-D: every level adds s times its own (rediscretised) Q1 mass; the
    coarsest solve is exact for the shifted operator."""
    mu = 0.9
    R = np.random.default_rng(900 + n).normal(size=(n ** 3, 2))
    Z = host(sts.mg_vcycle(sts.make_space(3, n, mu), dev(R), shift=shift))
    Zr = mgr.vcycle3(R, n, mu, shift)
    np.testing.assert_allclose(Z, Zr, rtol=0, atol=1e-12 * abs(Zr).max())


def test_shifted_vcycle_rejects_bad_arguments():
    with pytest.raises(sts.STSError) as e:
        sts.mg_vcycle(sts.make_space(2, 31), dev(np.ones((31 * 31, 1))), shift=-1.0)
    assert e.value.code == 1
    with pytest.raises(sts.STSError) as e:
        sts.mg_vcycle(sts.make_space(3, 100), dev(np.ones((100 ** 3, 1))), shift=2.0)
    assert e.value.code == 1


# 3-D sizes: the exact sine-transform solve alone (1, 2, 17, 40, 63), one
# smoothed level above it with the fine grid ragged against the 32 x 8 x 4
# tile and the coarse grid against the 16 x 4 x 4 restriction tile (65 -> 32,
# 95 -> 47, 127 -> 63), and two smoothed levels (191 -> 95 -> 47).
VC3_SIZES = [1, 2, 17, 40, 63, 65, 95, 127, 191]


@pytest.mark.parametrize("n", VC3_SIZES)
def test_vcycle3_matches_reference(n):
    mu = 0.25 + 0.1 * (n % 7)
    rng = np.random.default_rng(600 + n)
    R = rng.normal(size=(n ** 3, 3))
    R[:, 1] = 0.0                                   # a zero column stays zero
    Z = host(sts.mg_vcycle(sts.make_space(3, n, mu), dev(R)))
    Zr = mgr.vcycle3(R, n, mu)
    np.testing.assert_allclose(Z, Zr, rtol=0, atol=1e-13 * abs(Zr).max())
    assert np.all(Z[:, 1] == 0.0)


@pytest.mark.parametrize("n,ncols", [(1, 1), (40, 2), (65, 3), (127, 8), (191, 2)])
def test_pcg3_matches_the_sine_transform_solve(n, ncols):
    mu = 0.9
    rng = np.random.default_rng(700 + n)
    B = rng.normal(size=(n ** 3, ncols))
    X, its, _ = sts.pcg_mg(sts.make_space(3, n, mu), dev(B), rtol=1e-12)
    X = host(X)
    Xr = mgr.exact3(B, n, mu)
    for c in range(ncols):
        assert rel(X[:, c], Xr[:, c]) < 1e-10, (c, rel(X[:, c], Xr[:, c]))
    if n <= mgr.EXACT3:
        assert max(its) == 1, its          # the V-cycle is the exact inverse
    else:
        assert max(its) <= 13, its         # plain CG needs ~700 at n = 191


def test_pcg_is_bitwise_deterministic():
    rng = np.random.default_rng(3)
    B = dev(rng.normal(size=(255 * 255, 3)))
    space = sts.make_space(2, 255)
    X1, i1, _ = sts.pcg_mg(space, B)
    X2, i2, _ = sts.pcg_mg(space, B)
    assert i1 == i2 and torch.equal(X1, X2)


@pytest.mark.parametrize("n,ncols", [(1, 1), (2, 2), (31, 3), (64, 2), (100, 8), (511, 2)])
def test_mass_chebyshev_matches_sparse_direct(n, ncols):
    mu = 0.9
    rng = np.random.default_rng(400 + n)
    B = rng.normal(size=(n * n, ncols))
    if ncols > 1:
        B[:, 0] = 0.0
    X, its = sts.mass_solve(sts.make_space(2, n, mu), dev(B), rtol=1e-13)
    X = host(X)
    assert its == math.ceil(math.log(0.5e-13) / math.log(1.0 / 3.0))
    M = fem.spatial_operators(2, n, mu)[1].tocsc()
    for c in range(ncols):
        nb = np.linalg.norm(B[:, c])
        if nb == 0.0:
            assert np.all(X[:, c] == 0.0)
            continue
        # the Chebyshev bound 2 (1/3)^k, with rounding slack
        assert np.linalg.norm(B[:, c] - M @ X[:, c]) <= 2e-13 * nb
        assert rel(X[:, c], spla.spsolve(M, B[:, c])) < 1e-12


def test_mass_solve_rejects_other_spaces():
    bad = sts.make_space(1, 127)
    with pytest.raises(sts.STSError) as e:
        sts.mass_solve(bad, dev(np.ones((127, 1))))
    assert e.value.code == 1


@pytest.mark.parametrize("n,ncols", [(1, 1), (2, 2), (15, 3), (40, 2), (63, 8)])
def test_tensor_mass_solve_3d_matches_sparse_direct(n, ncols):
    """3-D trilinear mass: three passes of tridiagonal solves along the grid lines."""
    rng = np.random.default_rng(500 + n)
    B = rng.normal(size=(n ** 3, ncols))
    X, its = sts.mass_solve(sts.make_space(3, n, 0.6), dev(B))
    X = host(X)
    assert its == 1
    M = fem.spatial_operators(3, n, 0.6)[1].tocsc()
    for c in range(ncols):
        r = B[:, c] - M @ X[:, c]
        assert np.linalg.norm(r) <= 1e-13 * np.linalg.norm(B[:, c])
        if n <= 40:
            assert rel(X[:, c], spla.spsolve(M, B[:, c])) < 1e-12


def _solve(w, **opts):
    t = wl.time_grid(w.nt, w.T)
    dd, ds, md, ms = sts.time_matrices(t)
    prob = sts.Problem(w.dim, w.n[0], w.mu, (dd, ds), (md, ms), dev(w.F1), dev(w.F2))
    info = prob.solve(**opts)
    V, Y = prob.factors()
    prob.close()
    return info, V, Y


@pytest.mark.parametrize("n,nt,p,seed", [(63, 64, 2, 21), (127, 40, 3, 22), (97, 17, 1, 23)])
def test_solve_with_and_without_multigrid_match_crank_nicolson(n, nt, p, seed):
    w = wl.heat_2d_bumps(n=n, nt=nt, p=p, seed=seed)
    K, M = fem.spatial_operators(2, n, w.mu)
    Dt, Mt = fem.time_matrices(wl.time_grid(w.nt, w.T))
    U = exact.crank_nicolson(K, M, Dt, Mt, w.F1, w.F2)
    res = {}
    for pre in (0, 1):
        info, V, Y = _solve(w, tol=1e-10, inner_precond=pre)
        assert info["status"] == "STS_OK", info
        assert info["res_true"] <= 1e-10
        assert rel(V @ Y, U) <= 1e-8, (pre, rel(V @ Y, U))
        res[pre] = info
    # the preconditioned run needs far fewer inner iterations on Kx
    assert res[1]["inner_its_K"] * 4 < res[0]["inner_its_K"], (res[0], res[1])


@pytest.mark.parametrize("n,nt,p,seed", [(65, 24, 2, 41), (95, 12, 3, 42)])
def test_3d_solve_with_and_without_multigrid_match_the_modal_solution(n, nt, p, seed):
    """3-D trilinear mass / seven-point stiffness: direct Mx and multigrid Kx
    inner solves against plain CG for both, and both against the exact
    space-time solution by sine modes."""
    w = wl.heat_3d_separable(n=n, nt=nt, p=p, seed=seed)
    Dt, Mt = fem.time_matrices(wl.time_grid(w.nt, w.T))
    U = exact.modal_solve_3d(n, w.mu, Dt, Mt, w.F1, w.F2)
    res = {}
    for pre in (0, 1):
        info, V, Y = _solve(w, tol=1e-10, inner_precond=pre)
        assert info["status"] == "STS_OK", info
        assert info["res_true"] <= 1e-10
        assert rel(V @ Y, U) <= 1e-8, (pre, rel(V @ Y, U))
        res[pre] = info
    assert res[1]["inner_its_K"] * 10 < res[0]["inner_its_K"], (res[0], res[1])


@pytest.mark.parametrize("dim,n,nt,p", [(2, 127, 64, 2), (3, 65, 24, 3), (1, 2047, 48, 2)])
def test_relaxed_inner_tolerance_keeps_the_solution(dim, n, nt, p):
    """Inner solves stopped at max(inner_rtol, min(1e-4, 10^-j tol / r)), j = 1, 2
    (inexact Krylov): the same tolerance on the exact residual, the same
    accuracy against the oracle, fewer inner iterations."""
    if dim == 1:
        w = wl.heat_1d_profiles(n=n, nt=nt, p=p, seed=51)
    elif dim == 2:
        w = wl.heat_2d_bumps(n=n, nt=nt, p=p, seed=52)
    else:
        w = wl.heat_3d_separable(n=n, nt=nt, p=p, seed=53)
    Dt, Mt = fem.time_matrices(wl.time_grid(w.nt, w.T))
    if dim == 3:
        U = exact.modal_solve_3d(n, w.mu, Dt, Mt, w.F1, w.F2)
    else:
        K, M = fem.spatial_operators(dim, n, w.mu)
        U = exact.crank_nicolson(K, M, Dt, Mt, w.F1, w.F2)
    res = {}
    for relax in (0, 1, 2):
        info, V, Y = _solve(w, tol=1e-10, inner_relax=relax)
        assert info["status"] == "STS_OK", info
        # the 1-D grid's exact residual has an FP64 floor of the order of tol:
        # STS_OK then also means within tol + res_floor (floor_limited)
        assert info["res_true"] <= 1e-10 or (info["floor_limited"] == 1 and
                                             info["res_true"] <= 1e-10 + info["res_floor"]), info
        assert rel(V @ Y, U) <= 1e-8, (relax, rel(V @ Y, U))
        res[relax] = info
    if dim > 1:
        assert res[1]["inner_its_K"] < res[0]["inner_its_K"], (res[0], res[1])
        assert res[2]["inner_its_K"] < res[0]["inner_its_K"], (res[0], res[2])
