"""FP32 bulk work with FP64 refinement (sts_opts.mixed) in the 3-D solve.

Bars, from the arithmetic:
  * Refined Kx solve: each FP32 round is a correction accumulated in FP64
    whose residual is replaced from that FP64 correction every few
    iterations; the FP64 defect r = b - Kx x is exact to FP64 rounding, so the
    refinement reaches the requested rtol on the FP64 residual, and the error
    against the exact sine-transform solve is then what an FP64 solve to that
    rtol gives: 1e-10 at rtol 1e-12 (the bar of the FP64 PCG test).  With
    the replacement CG keeps its directions, so the FP32 iterations stay
    within 1.5x the FP64 PCG's on the same system.
  * Whole solve: the Galerkin projection, reduced solve and exact residual are
    FP64, so the solve meets the same exact-residual tolerance; the relative
    error against the oracle's sine-mode space-time solution and against the
    FP64 GPU run must be <= 1e-8 (the relative-error target of the mixed
    configuration).
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


# one smoothed level with ragged tiles (65, 95), the 127 -> 63 hierarchy of
# the 255^3 problem's second level, two smoothed levels (191 -> 95 -> 47)
@pytest.mark.parametrize("n,ncols,rtol", [(65, 1, 1e-12), (95, 3, 1e-12), (127, 8, 1e-12),
                                          (191, 2, 1e-12), (127, 4, 1e-4)])
def test_refined_fp32_kx_solve_matches_the_sine_transform_solve(n, ncols, rtol):
    mu = 0.7
    rng = np.random.default_rng(900 + n + ncols)
    B = rng.normal(size=(n ** 3, ncols))
    space = sts.make_space(3, n, mu)
    X, its32, its64, rounds = sts.pcg_mg_refined(space, dev(B), rtol=rtol)
    X = host(X)
    _, its_ref, _ = sts.pcg_mg(space, dev(B), rtol=rtol)
    K = mgr.stiffness3(n, mu)
    Xr = mgr.exact3(B, n, mu)
    for c in range(ncols):
        # the FP64 residual meets rtol (the refinement's stopping test)
        r = np.linalg.norm(B[:, c] - K @ X[:, c]) / np.linalg.norm(B[:, c])
        assert r <= 1.05 * rtol, (c, r)
        if rtol <= 1e-12:
            assert rel(X[:, c], Xr[:, c]) < 1e-10, (c, rel(X[:, c], Xr[:, c]))
    assert its32 > 0 and its64 == 0, (its32, its64, rounds)
    assert its32 <= 1.5 * sum(its_ref) + 2 * ncols, (its32, its_ref)
    if rtol > 1e-6:
        assert rounds == 1, (its32, its64, rounds)


def test_refined_fp32_kx_solve_rejects_grids_without_a_smoothed_level():
    with pytest.raises(sts.STSError):
        sts.pcg_mg_refined(sts.make_space(3, 63, 1.0), dev(np.ones((63 ** 3, 1))))
    with pytest.raises(sts.STSError):
        sts.pcg_mg_refined(sts.make_space(2, 127, 1.0), dev(np.ones((127 ** 2, 1))))


def _solve(w, **opts):
    t = wl.time_grid(w.nt, w.T)
    dd, ds, md, ms = sts.time_matrices(t)
    prob = sts.Problem(w.dim, w.n[0], w.mu, (dd, ds), (md, ms), dev(w.F1), dev(w.F2))
    info = prob.solve(**opts)
    V, Y = prob.factors()
    prob.close()
    return info, V, Y


@pytest.mark.parametrize("n,nt,p,seed,extra", [(95, 12, 3, 81, {}), (127, 24, 2, 82, {}),
                                               (127, 16, 4, 83, {"inner_relax": 2}),
                                               (65, 512, 4, 84, {"inner_relax": 2})])
def test_fp32_bulk_solve_matches_the_oracle_and_the_fp64_run(n, nt, p, seed, extra):
    w = wl.heat_3d_separable(n=n, nt=nt, p=p, seed=seed)
    Dt, Mt = fem.time_matrices(wl.time_grid(w.nt, w.T))
    U = exact.modal_solve_3d(n, w.mu, Dt, Mt, w.F1, w.F2)
    i64, V64, Y64 = _solve(w, tol=1e-10, **extra)
    i32, V32, Y32 = _solve(w, tol=1e-10, mixed=1, **extra)
    keys = ("status", "outer_its", "k", "res_cheap", "res_true", "inner_its_K", "inner_its_fp32",
            "defect_rounds")
    for info in (i64, i32):
        assert info["status"] == "STS_OK", {k: info[k] for k in keys}
        assert info["res_true"] <= 1e-10, {k: info[k] for k in keys}
    U64, U32 = V64 @ Y64, V32 @ Y32
    assert rel(U64, U) <= 1e-8, rel(U64, U)
    assert rel(U32, U) <= 1e-8, rel(U32, U)
    assert rel(U32, U64) <= 1e-8, rel(U32, U64)
    # the FP32 path ran: FP32 iterations and defect corrections counted
    assert i32["inner_its_fp32"] > 0 and i32["defect_rounds"] > 0, i32
    assert i64["inner_its_fp32"] == 0 and i64["defect_rounds"] == 0, i64
    assert abs(i32["outer_its"] - i64["outer_its"]) <= 2, (i32, i64)


def test_fp32_bulk_option_is_ignored_where_it_does_not_apply():
    """2-D spaces and 3-D grids solved exactly on one level keep FP64: the
    option changes nothing there, bit for bit."""
    for w in (wl.heat_2d_bumps(n=63, nt=16, p=2, seed=85),
              wl.heat_3d_separable(n=63, nt=12, p=2, seed=86)):
        a, Va, Ya = _solve(w, tol=1e-10)
        b, Vb, Yb = _solve(w, tol=1e-10, mixed=1)
        assert a["status"] == b["status"] == "STS_OK"
        assert b["inner_its_fp32"] == 0
        assert a["outer_its"] == b["outer_its"] and a["inner_its_K"] == b["inner_its_K"]
        assert np.array_equal(Va @ Ya, Vb @ Yb)


# the FP32 contraction of the first Gram-Schmidt pass against NumPy: the
# lane layout of v_mfma_f32_16x16x4f32 (a transposed operand or a wrong
# accumulator row gives O(1) errors), ragged rows and columns, both load
# widths (ld % 4 != 0 takes the scalar loads), chunked long reductions.
# Bar: FP32 products and sums of rows terms each of size |a||b|, so the error
# is a few 1e-7 * sqrt(rows) * rms|a| rms|b|; the test takes 2e-5 relative to
# |A|^T |B| entrywise.
@pytest.mark.parametrize("rows,m,n,pad", [(1000, 37, 5, 0), (4099, 16, 16, 0), (17, 3, 1, 1),
                                          (70000, 130, 8, 0), (100003, 240, 8, 2),
                                          (261121, 4, 4, 0), (65536, 1, 16, 3)])
def test_fp32_gram_matches_numpy(rows, m, n, pad):
    rng = np.random.default_rng(rows + m + n)
    A = rng.normal(size=(rows, m)).astype(np.float32)
    B = rng.normal(size=(rows, n))
    # column-major FP32 A with leading dimension rows + pad
    At = torch.zeros((m, rows + pad), dtype=torch.float32, device="cuda")
    At[:, :rows] = torch.from_numpy(A.T.copy()).cuda()
    A_dev = At.t()[:rows]
    G = host(sts.binding.gram_fp32(A_dev, dev(B)))
    A64 = A.astype(np.float64)
    want = A64.T @ B
    scale = np.abs(A64).T @ np.abs(B)
    assert np.all(np.abs(G - want) <= 2e-5 * scale + 1e-30), np.max(np.abs(G - want) / scale)
