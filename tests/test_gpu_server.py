"""GPU tests of the request server (sts_server_*): results of served requests
equal the same problems solved alone, bitwise, and match the oracle; the
footprint budget bounds the memory held at once."""
import numpy as np
import pytest

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


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _mix():
    out = [wl.heat_1d_sine(nx=511, nt=64, seed=3),
           wl.heat_2d_separable(n=63, nt=40, p=2, seed=7, mu=0.3),
           wl.heat_2d_bumps(n=31, nt=17, p=3, seed=8),
           wl.heat_3d_separable(n=7, nt=20, p=2, seed=9),
           wl.heat_2d_separable(n=95, nt=33, p=1, seed=10, mu=4.0)]
    out[0].F1 = np.asfortranarray(np.random.default_rng(4).normal(size=(511, 2)) / 512)
    out[0].F2 = np.asfortranarray(np.column_stack([out[0].F2[:, 0], np.sin(np.arange(64.0)) / 64]))
    return out


def _submit(server, w, **opts):
    dd, ds, md, ms = sts.time_matrices(wl.time_grid(w.nt, w.T))
    return server.submit(w.dim, w.n[0], w.mu, (dd, ds), (md, ms), w.F1, w.F2, **opts)


def _alone(w, **opts):
    dd, ds, md, ms = sts.time_matrices(wl.time_grid(w.nt, w.T))
    with sts.Problem(w.dim, w.n[0], w.mu, (dd, ds), (md, ms), w.F1, w.F2) as pr:
        info = pr.solve(**opts)
        V, Y = pr.factors()
    return info, V, Y


def test_served_requests_equal_alone_and_oracle():
    mix = _mix()
    opts = dict(tol=1e-10, max_outer=120)
    with sts.Server(workers=3, mem_budget=8 << 30) as server:
        tickets = [_submit(server, w, **opts) for w in mix]
        for w, t in zip(mix, tickets):
            res, prob = server.wait(t)
            assert res["status"] == "STS_OK", (w.name, res)
            assert 0.0 <= res["queued_seconds"] <= res["latency_seconds"]
            V, Y = prob.factors()
            info, Va, Ya = _alone(w, **opts)
            assert np.array_equal(V, Va) and np.array_equal(Y, Ya), w.name
            K, M = fem.spatial_operators(w.dim, w.n[0], w.mu)
            Dt, Mt = fem.time_matrices(wl.time_grid(w.nt, w.T))
            U = exact.crank_nicolson(K, M, Dt, Mt, w.F1, w.F2)
            assert rel(V @ Y, U) <= 1e-8, (w.name, rel(V @ Y, U))
            server.release(t)
        st = server.stats()
        assert st["submitted"] == st["completed"] == st["released"] == len(mix)
        assert st["mem_in_use"] == 0 and st["queued"] == 0 and st["running"] == 0


def test_budget_admission_growth_and_refusal():
    """Admission by the starting footprint; a running request's basis then
    grows, each step waiting for budget (its growth and the transient of its
    copy) unless the request is the oldest running one, so the peak stays
    within the budget plus one request's growth and one transient (the old
    copy of one of its three basis arrays: under a third of its footprint)."""
    mix = [wl.heat_2d_separable(n=63, nt=32, p=2, seed=s) for s in range(6)]
    opts = dict(tol=1e-9, max_outer=60)
    one = sts.footprint(2, 63, 32, 2, **opts)
    assert one > 63 * 63 * 8
    budget = 2 * one + one // 2                       # two requests at their start
    with sts.Server(workers=4, mem_budget=budget) as server:
        tickets = [_submit(server, w, **opts) for w in mix]
        held = []
        for t in tickets:
            res, prob = server.wait(t)
            assert res["status"] == "STS_OK", res
            assert res["footprint"] >= one
            held.append(res["footprint"])
            server.release(t)
        st = server.stats()
        assert max(held) > one                        # the bases grew past the first capacity
        assert one <= st["mem_peak"] <= budget + max(held) - one + max(held) // 3, (st, one, held)
        with pytest.raises(sts.STSError) as e:
            _submit(server, wl.heat_2d_separable(n=127, nt=32, p=2, seed=1), **opts)
        assert e.value.code == 2                      # STS_E_NOMEM: can never fit
        with pytest.raises(sts.STSError) as e:
            server.release(tickets[0])                # already released
        assert e.value.code == 1


def test_serving_sizes_alone_equal_mixed_and_oracle():
    """Requests at the serving mix's sizes in flight together: a 1-D grid of
    32767 nodes, 3-D cubes of side 63 and 127, a 2-D grid of side 255.  Each
    served result equals the same request solved alone, bitwise, and matches
    the oracle (sine-mode solutions in 1-D and 3-D, Crank-Nicolson in 2-D)."""
    mix = [wl.heat_1d_profiles(n=32767, nt=512, p=3, seed=71, mu=2.5),
           wl.heat_3d_separable(n=63, nt=256, p=3, seed=72, mu=0.5),
           wl.heat_3d_separable(n=127, nt=128, p=2, seed=73, mu=3.0),
           wl.heat_2d_separable(n=255, nt=300, p=4, seed=74, mu=0.2)]

    def ropts(w):   # the serving benchmark's options
        return dict(tol=1e-8, max_outer=60, inner_relax=2 if w.dim == 3 else 1)

    with sts.Server(workers=3, mem_budget=64 << 30) as server:
        tickets = [_submit(server, w, **ropts(w)) for w in mix]
        for w, t in zip(mix, tickets):
            res, prob = server.wait(t)
            assert res["status"] == "STS_OK", (w.name, res)
            V, Y = prob.factors()
            server.release(t)
            info, Va, Ya = _alone(w, **ropts(w))
            assert np.array_equal(V, Va) and np.array_equal(Y, Ya), w.name
            Dt, Mt = fem.time_matrices(wl.time_grid(w.nt, w.T))
            if w.dim == 1:
                U = exact.modal_solve_1d_fast(w.n[0], w.mu, Dt, Mt, w.F1, w.F2)
            elif w.dim == 3:
                U = exact.modal_solve_3d(w.n[0], w.mu, Dt, Mt, w.F1, w.F2)
            else:
                K, M = fem.spatial_operators(2, w.n[0], w.mu)
                U = exact.crank_nicolson(K, M, Dt, Mt, w.F1, w.F2)
            assert rel(V @ Y, U) <= 1e-8, (w.name, rel(V @ Y, U))


def test_failed_request_is_reported_and_others_finish():
    mix = _mix()[:3]
    with sts.Server(workers=2, mem_budget=8 << 30) as server:
        t0 = _submit(server, mix[0], tol=1e-14, max_outer=1)
        t1 = _submit(server, mix[1], tol=1e-10)
        t2 = _submit(server, mix[2], tol=1e-10)
        r0, p0 = server.wait(t0)
        assert r0["status"] == "STS_E_NOT_CONVERGED" and p0 is not None
        for t in (t1, t2):
            assert server.wait(t)[0]["status"] == "STS_OK"
        # unreleased requests are freed by close()
