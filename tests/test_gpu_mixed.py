"""Mixed precision in the 3-D Kx solves: the multigrid V-cycle stores its
vectors in FP32, the conjugate-gradient iteration around it stays FP64.

Bars, from the arithmetic:
  * V-cycle: every stored value is rounded once to single precision (unit
    roundoff u = 2^-24 ~ 6e-8) at about ten places per level, and the V-cycle
    maps each such perturbation through an operator of norm O(1) relative to
    its output, so Z differs from the FP64 reference by a few u to a few
    hundred u.  The tests take 1e-5 (a wrong index or a dropped term gives
    O(1)) and also require a difference above 1e-10 (the FP32 path ran: the
    FP64 V-cycle matches the reference to 1e-13).
  * PCG: the rounding perturbs the preconditioner only; the operator and the
    residual recurrence are FP64, so the iteration reaches the same rtol and
    the same accuracy against the exact sine-transform solve as the FP64 one,
    at most one iteration later.
  * Whole solve: the same exact-residual tolerance and the same error against
    the space-time solution by sine modes as with FP64 inner solves.
"""
import numpy as np
import pytest

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


# one smoothed level, fine grid ragged against the 32 x 8 x 4 tile and the
# coarse one against the restriction tile (65 -> 32, 95 -> 47, 127 -> 63), and
# two smoothed levels, the second in FP32 on both sides (191 -> 95 -> 47)
@pytest.mark.parametrize("n,shift", [(65, 0.0), (95, 0.0), (127, 0.0), (191, 0.0), (95, 30.0),
                                     (127, 3e3)])
def test_mixed_vcycle3_is_the_fp64_vcycle_to_single_precision(n, shift):
    mu = 0.25 + 0.1 * (n % 7)
    rng = np.random.default_rng(1200 + n)
    R = rng.normal(size=(n ** 3, 3))
    R[:, 1] = 0.0                                   # a zero column stays zero
    space = sts.make_space(3, n, mu)
    Z = host(sts.mg_vcycle(space, dev(R), shift=shift, fp32=True))
    Z64 = host(sts.mg_vcycle(space, dev(R), shift=shift))
    Zr = mgr.vcycle3(R, n, mu, shift)
    assert np.all(Z[:, 1] == 0.0)
    for c in (0, 2):
        e = rel(Z[:, c], Zr[:, c])
        assert 1e-10 < e < 1e-5, (c, e)
        assert rel(Z64[:, c], Zr[:, c]) < 1e-13
        assert rel(Z[:, c], Z64[:, c]) < 1e-5


@pytest.mark.parametrize("n,ncols,shift", [(65, 1, 0.0), (127, 4, 0.0), (191, 2, 0.0),
                                           (127, 2, 40.0)])
def test_mixed_pcg3_reaches_the_fp64_accuracy(n, ncols, shift):
    mu = 0.9
    rng = np.random.default_rng(1300 + n)
    B = rng.normal(size=(n ** 3, ncols))
    space = sts.make_space(3, n, mu)
    X, its, _ = sts.pcg_mg_mixed(space, dev(B), shift=shift, rtol=1e-12)
    X = host(X)
    Xr = mgr.exact3(B, n, mu, shift)
    for c in range(ncols):
        assert rel(X[:, c], Xr[:, c]) < 1e-10, (c, rel(X[:, c], Xr[:, c]))
    if shift:
        _, its64 = sts.shifted_solve(space, shift, dev(B), rtol=1e-12)
    else:
        _, its64, _ = sts.pcg_mg(space, dev(B), rtol=1e-12)
    assert max(its) <= max(its64) + 1, (its, its64)


def test_mixed_pcg3_zero_rhs_and_iteration_cap():
    n = 95
    space = sts.make_space(3, n, 1.0)
    B = np.zeros((n ** 3, 2))
    B[:, 1] = np.random.default_rng(5).normal(size=n ** 3)
    X, its, code = sts.pcg_mg_mixed(space, dev(B), rtol=1e-12)
    assert code == 0 and its[0] == 0 and np.all(host(X)[:, 0] == 0.0)
    _, its, code = sts.pcg_mg_mixed(space, dev(B), rtol=1e-12, maxit=2, check=False)
    assert code == 4 and max(its) == 2                # STS_E_NOT_CONVERGED (maxit)


def _solve(w, **opts):
    t = wl.time_grid(w.nt, w.T)
    dd, ds, md, ms = sts.time_matrices(t)
    prob = sts.Problem(w.dim, w.n[0], w.mu, (dd, ds), (md, ms), dev(w.F1), dev(w.F2))
    info = prob.solve(**opts)
    V, Y = prob.factors()
    prob.close()
    return info, V, Y


@pytest.mark.parametrize("n,nt,p,seed,extra", [(95, 12, 3, 61, {}), (127, 24, 2, 62, {}),
                                               (127, 16, 2, 63, {"inner_relax": 2}),
                                               (95, 12, 2, 64, {"rational": 1})])
def test_mixed_solve_3d_matches_the_modal_solution(n, nt, p, seed, extra):
    """Extended Krylov (and the rational Krylov space, whose shifted solves use
    the shifted FP32 V-cycle) with FP32-storage multigrid in the Kx solves:
    the same tolerance on the exact residual and the same accuracy against the
    exact space-time solution as the FP64 run, with about the same work."""
    w = wl.heat_3d_separable(n=n, nt=nt, p=p, seed=seed)
    Dt, Mt = fem.time_matrices(wl.time_grid(w.nt, w.T))
    U = exact.modal_solve_3d(n, w.mu, Dt, Mt, w.F1, w.F2)
    res = {}
    for f32 in (0, 1):
        info, V, Y = _solve(w, tol=1e-10, precond_fp32=f32, **extra)
        assert info["status"] == "STS_OK", info
        assert info["res_true"] <= 1e-10
        assert rel(V @ Y, U) <= 1e-8, (f32, rel(V @ Y, U))
        res[f32] = info
    assert abs(res[1]["outer_its"] - res[0]["outer_its"]) <= 1, (res[0], res[1])
    assert res[1]["inner_its_K"] <= 1.2 * res[0]["inner_its_K"] + 4, (res[0], res[1])
    # The byte accounting follows the launches: the FP32 V-cycle keeps two
    # post-smoothing launches (u_1 and d_0 stored between them), the FP64 one
    # fuses them, so per iteration the two move about the same bytes.
    if res[1]["inner_its_K"] == res[0]["inner_its_K"]:
        ratio = res[1]["alg_bytes"] / res[0]["alg_bytes"]
        assert 0.9 < ratio < 1.1, (res[0], res[1])


def test_mixed_option_is_ignored_where_it_does_not_apply():
    """2-D spaces and 3-D grids solved exactly on one level keep FP64: the
    option changes nothing there, bit for bit."""
    for w in (wl.heat_2d_bumps(n=63, nt=16, p=2, seed=71),
              wl.heat_3d_separable(n=63, nt=12, p=2, seed=72)):
        a, Va, Ya = _solve(w, tol=1e-10)
        b, Vb, Yb = _solve(w, tol=1e-10, precond_fp32=1)
        assert a["status"] == b["status"] == "STS_OK"
        assert a["outer_its"] == b["outer_its"] and a["inner_its_K"] == b["inner_its_K"]
        assert np.array_equal(Va @ Ya, Vb @ Yb)


def test_mixed_entry_points_with_padded_leading_dimensions():
    """Eight columns (the maximum) in buffers with ld > Nh, through the C ABI:
    the same V-cycle and the same solve as from packed buffers, bit for bit;
    the padding rows of Z and X are left untouched."""
    import ctypes as C
    from paper_1912_10082_amd import binding as b
    n, ncols, pad = 65, 8, 7
    nh, ld = n ** 3, n ** 3 + pad
    space = sts.make_space(3, n, 0.7)
    R = np.random.default_rng(1400).normal(size=(nh, ncols))
    Rp = torch.full((ncols, ld), 3.0, dtype=torch.float64, device="cuda")
    Rp[:, :nh] = torch.from_numpy(R.T.copy()).cuda()
    lib = b.load()
    st = b._stream_handle()
    for shift in (0.0, 25.0):
        Zp = torch.full((ncols, ld), -5.0, dtype=torch.float64, device="cuda")
        assert lib.sts_mg_vcycle_mixed(C.byref(space), shift, C.c_void_p(Rp.data_ptr()), ld,
                                       C.c_void_p(Zp.data_ptr()), ld, ncols, st) == 0
        Z = host(sts.mg_vcycle(space, dev(R), shift=shift, fp32=True))
        Zh = host(Zp)
        assert np.array_equal(Zh[:, :nh].T, Z)
        assert np.all(Zh[:, nh:] == -5.0)
        Xp = torch.full((ncols, ld), -5.0, dtype=torch.float64, device="cuda")
        its = (C.c_int32 * ncols)()
        assert lib.sts_pcg_mg_mixed(C.byref(space), shift, C.c_void_p(Rp.data_ptr()), ld,
                                    C.c_void_p(Xp.data_ptr()), ld, ncols, 1e-12, 100, its,
                                    st) == 0
        X, its2, _ = sts.pcg_mg_mixed(space, dev(R), shift=shift, rtol=1e-12)
        Xh = host(Xp)
        assert np.array_equal(Xh[:, :nh].T, host(X)) and list(its) == its2
        assert np.all(Xh[:, nh:] == -5.0)
