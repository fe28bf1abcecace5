"""GPU tests of the serving path: CG restricted to the training rows of a
joint lattice, the predictive mean (Section 2, eq. gp_pred_mean, computed by
one lattice MVM of [a; 0]), and the continuous-batching server.

Bars: restricted CG with a fixed iteration count matches the oracle's
restricted CG to a per-column relative error of 1e-4 (as the unrestricted CG
parity test) and leaves the test rows exactly zero; the predictive mean from
the GPU's a matches the oracle's MVM of that a to 1e-5 of |K| |a|; results of
requests served together are bitwise equal to the same requests served one at
a time; admission never reserves more than the HBM budget.
"""
import sys

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

CG_TOL = 1e-4
MVM_TOL = 1e-5


def _note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def sgp():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    import paper_2106_06695_amd as sgp
    sgp._lib.load()
    return sgp


def _cuda(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def _colerr(got, ref):
    got = np.asarray(got, dtype=np.float64).reshape(ref.shape[0], -1)
    ref = ref.reshape(ref.shape[0], -1)
    return np.linalg.norm(got - ref, axis=0) / np.maximum(np.linalg.norm(ref, axis=0), 1e-300)


def _assert_mean(olat, a, mu, n):
    """The mean is a sum of kernel-weighted solution entries that can cancel,
    so its error is bounded by the magnitude sum |K| |a| (the oracle's MVM of
    |a|; the lattice weights are positive), not by the mean itself."""
    ref = olat.mvm(a.astype(np.float64))[n:, 0]
    scale = olat.mvm(np.abs(a).astype(np.float64))[n:, 0]
    assert np.all(np.abs(mu - ref) <= MVM_TOL * scale + 1e-30)


def _joint_case(seed, n, n_test, d, C):
    c = workloads.small_case(seed, n + n_test, d, channels=C, kind="mixture")
    B = c.values.astype(np.float64).copy()
    B[n:] = 0.0
    return c, B


# The tiny case has m = 20 lattice points: by iteration 12 its Krylov space
# spans the operator's effective range and the recursive residual is set by
# rounding (a 1e-7 relative change of b moves it by 4% in the oracle itself),
# so it runs 8 iterations, where the same change moves it by 2e-8.
@pytest.mark.parametrize("seed,n,n_test,d,C,its", [(31, 1500, 300, 4, 3, 12),
                                                  (32, 3000, 1111, 9, 8, 12),
                                                  (33, 257, 1, 2, 1, 8)])
def test_restricted_cg_and_predictive_mean(sgp, orc, seed, n, n_test, d, C, its):
    _note(f"restricted cg seed={seed} n={n} n_test={n_test} d={d} C={C}")
    c, B = _joint_case(seed, n, n_test, d, C)
    noise = 0.1
    lat = sgp.lattice_build(_cuda(c.X), c.lengthscales, solve_rows=n)
    olat = orc.Lattice(c.X, c.lengthscales)
    x, iters, rel = sgp.cg_solve(lat, _cuda(B), noise, 0.0, max_iter=its)
    xo, itero, relo, _ = olat.cg(B, noise, 0.0, max_iter=its, rows=n)
    xg = x.cpu().numpy()
    assert np.all(iters == its) and np.all(itero == its)
    assert np.all(xg[n:] == 0.0)
    assert _colerr(xg[:n], xo[:n]).max() <= CG_TOL
    np.testing.assert_allclose(rel, relo, rtol=1e-3)
    # predictive mean at the test rows: K(X*, X) a, from the GPU's own a
    a = np.zeros((n + n_test, 1), dtype=np.float32)
    a[:n, 0] = xg[:n, 0]
    mu = sgp.lattice_mvm(lat, _cuda(a)).cpu().numpy()[n:, 0]
    _assert_mean(olat, a, mu, n)
    lat.free()


def test_restricted_cg_to_tolerance(sgp, orc):
    _note("restricted cg to tolerance")
    n, n_test, d = 2000, 500, 3
    c, B = _joint_case(34, n, n_test, d, 2)
    noise, tol = 0.1, 1e-4
    lat = sgp.lattice_build(_cuda(c.X), c.lengthscales, solve_rows=n)
    olat = orc.Lattice(c.X, c.lengthscales)
    x, iters, rel = sgp.cg_solve(lat, _cuda(B), noise, tol, max_iter=500)
    assert np.all(rel <= tol)
    xg = x.cpu().numpy().astype(np.float64)
    assert np.all(xg[n:] == 0.0)
    # the residual of the training block, with the oracle's fp64 operator
    res = B[:n] - (olat.mvm(xg)[:n] + noise * xg[:n])
    assert np.all(np.linalg.norm(res, axis=0) / np.linalg.norm(B[:n], axis=0) <= 1.05 * tol)
    lat.free()


def test_solve_rows_validation(sgp):
    X = _cuda(np.zeros((10, 2)))
    with pytest.raises(sgp.SGPError):
        sgp.lattice_build(X, [1.0, 1.0], solve_rows=11)
    with pytest.raises(sgp.SGPError):
        sgp.lattice_build(X, [1.0, 1.0], solve_rows=-1)


def _requests(count=14, seed=1105):
    return workloads.ws5_requests(seed=seed, count=count, mean_gap_s=0.002, n_lo=500,
                                  n_hi=20000, d_lo=3, d_hi=12, channels=4, n_test=400)


def test_server_alone_vs_mix_bitwise(sgp):
    from paper_2106_06695_amd import serve
    reqs = _requests()
    _note(f"server alone: {len(reqs)} requests")
    alone = serve.Server(workers=1).run(reqs, realtime=False)
    _note("server mixed: 4 workers, real-time arrivals")
    srv = serve.Server(workers=4)
    mixed = srv.run(reqs, realtime=True)
    assert [r.rid for r in alone] == [r.rid for r in mixed] == [q.rid for q in reqs]
    for a, b in zip(alone, mixed):
        np.testing.assert_array_equal(a.mean, b.mean)
        np.testing.assert_array_equal(a.alpha, b.alpha)
        np.testing.assert_array_equal(a.iters, b.iters)
        np.testing.assert_array_equal(a.rel, b.rel)
        assert np.all((a.rel <= reqs[a.rid].tol) | (a.iters == 1000))
    assert srv.max_reserved <= srv.budget


def test_server_admission_budget(sgp):
    from paper_2106_06695_amd import serve
    reqs = _requests(count=10, seed=1106)
    worst = max(serve.footprint_worst(q) for q in reqs)
    ref = serve.Server(workers=1).run(reqs, realtime=False)
    for budget in (int(2.5 * worst), worst // 2):
        _note(f"admission budget {budget}")
        srv = serve.Server(workers=4, hbm_budget=budget)
        got = srv.run(reqs, realtime=False)
        assert len(got) == len(reqs)
        assert 0 < srv.max_reserved <= budget
        for a, b in zip(ref, got):
            np.testing.assert_array_equal(a.mean, b.mean)
            assert b.reserved_bytes <= budget
    s = serve.latency_summary(ref)
    assert s["requests"] == len(reqs) and s["p99_ms"] >= s["p50_ms"] > 0


def test_server_request_matches_oracle(sgp, orc):
    """One served request against the oracle's joint-lattice pipeline, at a
    fixed iteration count."""
    from paper_2106_06695_amd import serve
    c = workloads.small_case(35, 1800, 5, channels=3, kind="mixture")
    n = 1500
    req = serve.SolveRequest(rid=0, arrival_s=0.0, X=c.X[:n], X_test=c.X[n:],
                             lengthscales=c.lengthscales, values=c.values[:n], noise=0.1,
                             tol=0.0, max_iter=15)
    (res,) = serve.Server(workers=2).run([req], realtime=False)
    olat = orc.Lattice(c.X, c.lengthscales)
    B = np.zeros((1800, 3))
    B[:n] = c.values[:n]
    xo, itero, _, _ = olat.cg(B, 0.1, 0.0, max_iter=15, rows=n)
    assert np.all(res.iters == 15)
    assert _colerr(res.alpha[:, None], xo[:n, :1]).max() <= CG_TOL
    a = np.zeros((1800, 1), dtype=np.float32)
    a[:n, 0] = res.alpha
    _assert_mean(olat, a, res.mean, n)


def test_server_failing_request_releases_its_reservation(sgp):
    """A request that fails after its lattice is built (noise < 0 is rejected
    by cg_solve) surfaces its error from run(), the other requests are
    served, and every reserved byte is released."""
    from paper_2106_06695_amd import serve
    reqs = _requests(count=6, seed=1107)
    reqs[2].noise = -1.0
    srv = serve.Server(workers=3)
    _note("server with one failing request")
    with pytest.raises(sgp.SGPError) as ei:
        srv.run(reqs, realtime=False)
    assert ei.value.code == -1
    assert srv._reserved == 0
    assert 0 < srv.max_reserved <= srv.budget
    assert sorted(r.rid for r in srv._results) == [q.rid for q in reqs if q.rid != 2]
