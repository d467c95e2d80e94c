"""GPU tests of the batch executor (sts_pool_*) and its autotuner.

A pooled solve must give bitwise the factors of the same problem solved
alone, and each factor product must match the oracle's Crank-Nicolson
solution to the 1e-8 gate.  All calls go through the C ABI.
"""
import numpy as np
import pytest

import paper_1912_10082_amd as sts
import workloads as wl
from oracle import exact, fem
from paper_1912_10082_amd import autotune

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


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _make(w, device=True):
    dd, ds, md, ms = sts.time_matrices(wl.time_grid(w.nt, w.T))
    F1, F2 = (dev(w.F1), dev(w.F2)) if device else (w.F1, w.F2)
    return sts.Problem(w.dim, w.n[0], w.mu, (dd, ds), (md, ms), F1, F2)


def test_pool_matches_solo_bitwise_and_oracle():
    batch = wl.batch_2d_uneven(count=10, seed0=77, sides=(31, 63), nts=(16, 64, 128),
                               ps=(1, 2, 3))
    opts = dict(tol=1e-10, max_outer=80)
    pooled = [_make(w, device=(i % 2 == 0)) for i, w in enumerate(batch)]
    with sts.Pool(3) as pool:
        infos = pool.solve(pooled, **opts)
    for w, pr, info in zip(batch, pooled, infos):
        assert info["status"] == "STS_OK", (w.name, info)
        V, Y = pr.factors()
        solo = _make(w)
        assert solo.solve(**opts)["status"] == "STS_OK"
        Vs, Ys = solo.factors()
        assert np.array_equal(V, Vs) and np.array_equal(Y, Ys), w.name
        K, M = fem.spatial_operators(2, w.n[0], w.mu)
        Dt, Mt = fem.time_matrices(wl.time_grid(w.nt, w.T))
        U = exact.crank_nicolson(K, M, Dt, Mt, w.F1, w.F2)
        assert rel(V @ Y, U) <= 1e-8, (w.name, rel(V @ Y, U))
        solo.close()
        pr.close()


def test_pool_at_batch_benchmark_sizes_matches_oracle():
    """Sides 127 and 255 with Nt = 1024, ranks 1..3, mu across [0.1, 10], with
    the batch benchmark's options: every problem against Crank-Nicolson."""
    batch = [wl.heat_2d_separable(n=255, nt=1024, p=3, seed=4101, mu=0.13),
             wl.heat_2d_separable(n=127, nt=1024, p=1, seed=4102, mu=7.5),
             wl.heat_2d_separable(n=255, nt=1024, p=2, seed=4103, mu=1.9),
             wl.heat_2d_separable(n=127, nt=1024, p=2, seed=4104, mu=0.4)]
    opts = dict(tol=1e-9, max_outer=80, inner_relax=1)
    probs = [_make(w) for w in batch]
    with sts.Pool(4) as pool:
        infos = pool.solve(probs, **opts)
    for w, pr, info in zip(batch, probs, infos):
        assert info["status"] == "STS_OK", (w.name, info)
        V, Y = pr.factors()
        K, M = fem.spatial_operators(2, w.n[0], w.mu)
        Dt, Mt = fem.time_matrices(wl.time_grid(w.nt, w.T))
        U = exact.crank_nicolson(K, M, Dt, Mt, w.F1, w.F2)
        assert rel(V @ Y, U) <= 1e-8, (w.name, rel(V @ Y, U))
        pr.close()


def test_pool_per_problem_options_and_failures():
    batch = wl.batch_2d_uneven(count=4, seed0=91, sides=(31,), nts=(32,), ps=(2,))
    probs = [_make(w) for w in batch]
    opts = [dict(tol=1e-10), dict(tol=1e-12, max_outer=2), dict(tol=1e-10), dict(tol=1e-10)]
    with sts.Pool(2) as pool:
        infos = pool.solve(probs, opts)
        assert [d["status"] for d in infos] == ["STS_OK", "STS_E_NOT_CONVERGED", "STS_OK",
                                                "STS_OK"]
        assert "problem 1" in infos[1]["error"]
        assert infos[1]["outer_its"] == 2
        # the unconverged problem continues from where it stopped
        more = pool.solve([probs[1]], tol=1e-10)
        assert more[0]["status"] == "STS_OK"
        assert pool.solve([]) == []
        with pytest.raises(sts.STSError) as e:
            pool.solve([probs[0], probs[0]])
        assert e.value.code == 1
    for pr in probs:
        pr.close()


def test_autotuner_returns_a_measured_candidate():
    batch = wl.batch_2d_uneven(count=6, seed0=5, sides=(31, 63), nts=(32, 64), ps=(1, 2))
    probs = [_make(w) for w in batch]
    best, timings = autotune.tune_workers(probs, candidates=(1, 2), probe=6, tol=1e-9)
    assert best in (1, 2) and set(timings) == {1, 2}
    assert all(t > 0 for t in timings.values())
    for pr in probs:
        pr.close()


def test_joint_autotuner_searches_workers_and_relaxation():
    batch = wl.batch_2d_uneven(count=6, seed0=6, sides=(31, 63), nts=(32, 64), ps=(1, 2))
    probs = [_make(w) for w in batch]
    (w, j), timings = autotune.tune(probs, candidates=(1, 2), relax=(1, 2), probe=4, tol=1e-9)
    assert set(timings) == {(1, 1), (1, 2), (2, 1), (2, 2)}
    assert timings[(w, j)] == min(timings.values())
    for pr in probs:
        pr.close()
