"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Bars (stated once here, used below):
  * lattice keys, vertex indices and neighbour tables: bit-exact;
  * barycentric weights: bit-exact against the oracle's fp64 weights rounded
    to fp32 (both sides evaluate the same fp64 operation sequence);
  * MVM: per-column relative 2-norm error <= 1e-5 (fp32 accumulation on the
    GPU against fp64 in the oracle) and, element by element,
    |out - ref| <= 1e-5 (|K| |v|), the oracle's MVM of |v| (the operator's
    entries are non-negative: barycentric weights and kernel samples), so a
    few wrong small outputs cannot hide under a column norm;
  * CG with a fixed iteration count: per-column relative 2-norm error of x
    <= 1e-4; CG to a tolerance: the GPU's x, checked with the oracle's fp64
    operator, meets 1.05 * tol.
"""
import concurrent.futures
import os
import sys

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

MVM_TOL = 1e-5
CG_TOL = 1e-4


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


def _build_both(sgp, orc, X, ell, order=1, kernel="rbf", blur="symmetric", outputscale=1.0):
    lat = sgp.lattice_build(_cuda(X), ell, order=order, kernel=kernel, blur=blur,
                            outputscale=outputscale)
    olat = orc.Lattice(X, ell, r=order, kernel=orc.RBF if kernel == "rbf" else orc.MATERN32)
    return lat, olat


def _assert_structure(sgp, lat, olat):
    keys, idx, w, nbr = sgp.lattice_export(lat)
    okeys, oidx, ow, onbr = olat.export()
    assert lat.m == olat.m
    np.testing.assert_array_equal(keys, okeys)
    np.testing.assert_array_equal(idx, oidx)
    np.testing.assert_array_equal(w, ow.astype(np.float32))
    np.testing.assert_array_equal(nbr, onbr)


def _colerr(got, ref):
    got = np.asarray(got, dtype=np.float64).reshape(ref.shape[0], -1)
    ref = ref.reshape(ref.shape[0], -1)
    return np.linalg.norm(got - ref, axis=0) / np.maximum(np.linalg.norm(ref, axis=0), 1e-300)


def _assert_mvm(out, olat, V, mode=0, outputscale=1.0):
    """MVM parity: per-column 2-norm and element-wise against |K| |V|."""
    V = np.asarray(V, dtype=np.float64).reshape(olat.n, -1)
    ref = olat.mvm(V, mode=mode, outputscale=outputscale)
    scale = olat.mvm(np.abs(V), mode=mode, outputscale=outputscale)
    got = np.asarray(out, dtype=np.float64).reshape(ref.shape)
    err = _colerr(got, ref)
    assert err.max() <= MVM_TOL, err
    bad = np.abs(got - ref) > MVM_TOL * scale + 1e-30
    assert not bad.any(), (int(bad.sum()), np.argwhere(bad)[:5].tolist())


def _oracle_cg_columns(olat, B, noise, tol, max_iter, cols, rows=0):
    """The oracle's CG on each listed column, one column per thread (its
    calls release the GIL and share no state); returns x (n x len(cols)),
    iterations and recursive residuals."""
    B = np.asarray(B, dtype=np.float64)
    workers = max(1, min(len(cols), 16, os.cpu_count() or 1))

    def one(c):
        return olat.cg(B[:, c:c + 1], noise, tol, max_iter=max_iter, rows=rows)

    with concurrent.futures.ThreadPoolExecutor(max_workers=workers) as ex:
        res = list(ex.map(one, cols))
    x = np.concatenate([r[0] for r in res], axis=1)
    its = np.concatenate([r[1] for r in res])
    rel = np.concatenate([r[2] for r in res])
    return x, its, rel


STRUCT_CASES = [
    # (seed, n, d, kind, order)
    (1, 1, 3, "normal", 1),
    (2, 7, 2, "normal", 1),
    (3, 1000, 1, "normal", 1),
    (4, 2000, 3, "normal", 1),
    (5, 4097, 5, "mixture", 1),
    (6, 3001, 8, "mixture", 2),
    (7, 2500, 11, "mixture", 1),
    (8, 1500, 16, "uniform", 1),
    (9, 999, 20, "normal", 3),
    (10, 600, 32, "normal", 1),
]


@pytest.mark.parametrize("seed,n,d,kind,order", STRUCT_CASES)
def test_structure_bit_exact(sgp, orc, seed, n, d, kind, order):
    _note(f"structure seed={seed} n={n} d={d} order={order}")
    w = workloads.small_case(seed, n, d, kind=kind)
    lat, olat = _build_both(sgp, orc, w.X, w.lengthscales, order=order)
    _assert_structure(sgp, lat, olat)
    info = sgp.lattice_info(lat)
    assert info["m"] == olat.m <= n * (d + 1)


def test_structure_ties_and_duplicates(sgp, orc):
    _note("structure ties")
    rng = np.random.default_rng(0)
    base = rng.standard_normal((50, 4)).astype(np.float32)
    X = np.concatenate([np.zeros((3, 4), np.float32), base, base[:20], base[::-1]])
    lat, olat = _build_both(sgp, orc, X, np.ones(4))
    _assert_structure(sgp, lat, olat)
    s = np.sqrt(2 * np.pi / 3)
    X1 = (np.arange(-20, 21) * s * 0.5).astype(np.float32)[:, None]
    lat, olat = _build_both(sgp, orc, X1, np.array([0.5]))
    _assert_structure(sgp, lat, olat)
    # exact residual ties at d = 2 and 3: a zero coordinate makes elevated
    # coordinates equal, so the tie rule picks the zero-weight vertex
    for d, cs in ((3, [(1.2, 0, 0), (2.9, 0, 0), (0, 0, 1.7)]), (2, [(0, 0.5), (0, 1.6), (0, -1.6)])):
        j = np.arange(1, d + 1)
        unit = s * np.sqrt(j * (j + 1)) / np.sqrt(d * (d + 1))
        Xt = np.concatenate([(np.asarray(c) * unit)[None, :] for c in cs]
                            + [rng.standard_normal((30, d))]).astype(np.float32)
        lat, olat = _build_both(sgp, orc, Xt, np.ones(d))
        _assert_structure(sgp, lat, olat)


@pytest.mark.parametrize("spread,seed", [(60.0, 5), (8.0, 6), (10.0, 6)])
def test_structure_point_key_widths(sgp, orc, spread, seed):
    """Point sort keys of every layout: at d = 12, x ~ U[-spread, spread]
    needs 86 coordinate bits (only the leading coordinates fit, no ranks;
    every vertex distinct, so the first hash table fills and grows), 51
    (three ranks fit) or 57 (one rank)."""
    _note(f"structure point key spread={spread}")
    rng = np.random.default_rng(seed)
    X = rng.uniform(-spread, spread, size=(3000, 12)).astype(np.float32)
    lat, olat = _build_both(sgp, orc, X, np.ones(12))
    _assert_structure(sgp, lat, olat)


def test_structure_matern(sgp, orc):
    _note("structure matern32")
    w = workloads.small_case(21, 1500, 6, kind="mixture")
    lat, olat = _build_both(sgp, orc, w.X, w.lengthscales, kernel="matern32")
    _assert_structure(sgp, lat, olat)


@pytest.mark.parametrize("blur", ["symmetric", "forward", "reverse"])
@pytest.mark.parametrize("C", [1, 3, 16, 70])
def test_mvm_parity(sgp, orc, blur, C):
    _note(f"mvm blur={blur} C={C}")
    w = workloads.small_case(30 + C, 3001, 6, channels=C, kind="mixture")
    lat, olat = _build_both(sgp, orc, w.X, w.lengthscales, blur=blur, outputscale=1.7)
    out = sgp.lattice_mvm(lat, _cuda(w.values)).cpu().numpy()
    mode = {"symmetric": orc.SYMMETRIC, "forward": orc.FORWARD, "reverse": orc.REVERSE}[blur]
    _assert_mvm(out, olat, w.values, mode=mode, outputscale=1.7)


@pytest.mark.parametrize("d,order,kernel", [(1, 1, "rbf"), (3, 2, "rbf"), (11, 1, "rbf"),
                                            (20, 1, "rbf"), (5, 1, "matern32")])
def test_mvm_parity_dims(sgp, orc, d, order, kernel):
    _note(f"mvm d={d} order={order} kernel={kernel}")
    w = workloads.small_case(50 + d, 2000, d, channels=2, kind="mixture")
    lat, olat = _build_both(sgp, orc, w.X, w.lengthscales, order=order, kernel=kernel)
    out = sgp.lattice_mvm(lat, _cuda(w.values)).cpu().numpy()
    _assert_mvm(out, olat, w.values)


def test_mvm_parity_many_lattice_points(sgp, orc):
    """More than 2^20 lattice points: the tile sort then keys on 64 bits."""
    _note("mvm with m > 2^20")
    w = workloads.small_case(61, 55_000, 20, channels=2, kind="uniform", ell_range=(0.05, 0.1))
    lat, olat = _build_both(sgp, orc, w.X, w.lengthscales)
    assert lat.m == olat.m > (1 << 20)
    out = sgp.lattice_mvm(lat, _cuda(w.values)).cpu().numpy()
    _assert_mvm(out, olat, w.values)


def test_mvm_reuse_and_many_handles(sgp, orc):
    _note("mvm reuse")
    w = workloads.small_case(60, 1000, 4, channels=5, kind="normal")
    lat, olat = _build_both(sgp, orc, w.X, w.lengthscales)
    other = sgp.lattice_build(_cuda(w.X[:500]), w.lengthscales * 2)
    for C in (1, 5, 2):
        V = w.values[:, :C]
        out = sgp.lattice_mvm(lat, _cuda(V)).cpu().numpy()
        _assert_mvm(out, olat, V)
    _ = sgp.lattice_mvm(other, _cuda(w.values[:500, :1]))
    sgp.lattice_free(other)


def test_mvm_symmetry_any_size(sgp):
    _note("mvm symmetry ws2")
    w = workloads.ws2()
    lat = sgp.lattice_build(_cuda(w.X), w.lengthscales)
    rng = np.random.default_rng(1)
    U = rng.standard_normal((w.n, 2)).astype(np.float32)
    KU = sgp.lattice_mvm(lat, _cuda(U)).cpu().numpy().astype(np.float64)
    a = U[:, 0] @ KU[:, 1]
    b = U[:, 1] @ KU[:, 0]
    assert abs(a - b) <= 1e-5 * (abs(a) + abs(b))


def test_cg_fixed_iterations(sgp, orc):
    _note("cg fixed iterations ws1")
    w = workloads.ws1()
    V = np.concatenate([w.values, np.random.default_rng(2).standard_normal((w.n, 2))], axis=1)
    lat, olat = _build_both(sgp, orc, w.X, w.lengthscales)
    x, iters, rel = sgp.cg_solve(lat, _cuda(V), w.noise, 0.0, max_iter=20)
    xo, itero, relo, _ = olat.cg(V.astype(np.float64), w.noise, 0.0, max_iter=20)
    assert np.all(iters == 20) and np.all(itero == 20)
    assert _colerr(x.cpu().numpy(), xo).max() <= CG_TOL
    np.testing.assert_allclose(rel, relo, rtol=1e-3)


@pytest.mark.parametrize("C,d", [(2, 3), (4, 5), (8, 2), (5, 4)])
def test_cg_fixed_iterations_widths(sgp, orc, C, d):
    """Channel counts that change how the tile kernels stage and split rows."""
    _note(f"cg fixed iterations C={C} d={d}")
    c = workloads.small_case(50 + C, 2500, d, channels=C, kind="mixture")
    lat, olat = _build_both(sgp, orc, c.X, c.lengthscales)
    x, iters, rel = sgp.cg_solve(lat, _cuda(c.values), 0.1, 0.0, max_iter=10)
    xo, itero, relo, _ = olat.cg(c.values.astype(np.float64), 0.1, 0.0, max_iter=10)
    assert np.all(iters == 10)
    assert _colerr(x.cpu().numpy(), xo).max() <= CG_TOL


@pytest.mark.parametrize("seed,n,d,C,order,kernel,blur,outputscale,noise,iters", [
    (401, 3000, 4, 3, 2, "rbf", "symmetric", 1.0, 0.1, 10),      # five-tap stencil: unfused blur
    (402, 2500, 5, 2, 1, "matern32", "symmetric", 1.7, 0.2, 10),
    (403, 2500, 3, 40, 1, "rbf", "symmetric", 1.0, 0.1, 10),    # two channel chunks
    (404, 2000, 3, 4, 1, "rbf", "forward", 1.0, 0.5, 4),        # one blur chain, paper order
    (405, 2000, 6, 1, 1, "rbf", "reverse", 2.5, 0.5, 4),
])
def test_cg_operator_variants(sgp, orc, seed, n, d, C, order, kernel, blur, outputscale, noise, iters):
    """Fixed-iteration CG iterates against the oracle's CG for blur orders,
    kernels, output scales and channel counts beyond the default: alpha's
    p.Ap is formed on the lattice (scale u.Bu + noise p.p) and the residual
    moves in the slice for every one of them. FORWARD and REVERSE are not
    symmetric; a few iterations of the same recurrence still compare."""
    _note(f"cg operator variant seed={seed} d={d} C={C} order={order} {kernel} {blur}")
    c = workloads.small_case(seed, n, d, channels=C, kind="mixture")
    lat, olat = _build_both(sgp, orc, c.X, c.lengthscales, order=order, kernel=kernel, blur=blur,
                            outputscale=outputscale)
    mode = {"symmetric": orc.SYMMETRIC, "forward": orc.FORWARD, "reverse": orc.REVERSE}[blur]
    x, it, rel = sgp.cg_solve(lat, _cuda(c.values), noise, 0.0, max_iter=iters)
    xo, ito, relo, _ = olat.cg(c.values.astype(np.float64), noise, 0.0, max_iter=iters, mode=mode,
                                outputscale=outputscale)
    assert np.all(it == iters) and np.all(ito == iters)
    assert _colerr(x.cpu().numpy(), xo).max() <= CG_TOL
    lat.free()


def test_cg_to_tolerance(sgp, orc):
    _note("cg tolerance ws1")
    w = workloads.ws1()
    lat, olat = _build_both(sgp, orc, w.X, w.lengthscales)
    x, iters, rel = sgp.cg_solve(lat, _cuda(w.values), w.noise, w.tol, max_iter=500)
    xo, itero, relo, _ = olat.cg(w.values.astype(np.float64), w.noise, w.tol, max_iter=500)
    assert rel[0] <= w.tol
    # near the tolerance the residual curve is flat; rounding-order changes
    # move the crossing by a few iterations
    assert abs(int(iters[0]) - int(itero[0])) <= max(2, 0.1 * itero[0])
    xg = x.cpu().numpy().astype(np.float64)
    b = w.values.astype(np.float64)
    res = b - (olat.mvm(xg) + w.noise * xg)
    assert np.linalg.norm(res) / np.linalg.norm(b) <= 1.05 * w.tol
    assert _colerr(xg, xo).max() <= 10 * w.tol


def test_cg_columns_stop_independently(sgp, orc):
    _note("cg columns")
    w = workloads.small_case(70, 1500, 3, channels=3, kind="normal")
    V = w.values.copy()
    V[:, 1] = 0.0
    lat = sgp.lattice_build(_cuda(w.X), w.lengthscales)
    x, iters, rel = sgp.cg_solve(lat, _cuda(V), 0.1, 1e-3, max_iter=200)
    assert iters[1] == 0 and rel[1] == 0.0
    assert np.all(x[:, 1].cpu().numpy() == 0.0)
    assert rel[0] <= 1e-3 and rel[2] <= 1e-3
    x1, it1, _ = sgp.cg_solve(lat, _cuda(V[:, :1]), 0.1, 1e-3, max_iter=200)
    assert it1[0] == iters[0]


def test_columns_bitwise_alone_and_batched_on_long_run_lists(sgp):
    """Uniform 16-d points at short lengthscales (m / n(d+1) ~ 0.9): every
    tile touches more lattice points than one staged slice chunk of a
    16-column batch holds (512 rows), but fewer than a single column's
    chunk. A column's MVM and CG iterates are still bitwise the same alone
    and in batches of 8, 16 and 24: the slice adds a point's entries by
    512-run blocks of its tile, then in vertex order, whatever the
    chunk (at most 16 channels: a batch of 24 takes two)."""
    _note("columns alone and batched, long run lists")
    w = workloads.small_case(77, 20000, 16, channels=16, kind="uniform", ell_range=(0.3, 3.0))
    lat = sgp.lattice_build(_cuda(w.X), w.lengthscales)
    try:
        assert lat.m > 0.8 * w.n * 17
        y16 = sgp.lattice_mvm(lat, _cuda(w.values)).cpu().numpy()
        x16, _, _ = sgp.cg_solve(lat, _cuda(w.values), 0.1, 0.0, max_iter=6)
        x16 = x16.cpu().numpy()
        y8 = sgp.lattice_mvm(lat, _cuda(w.values[:, :8])).cpu().numpy()
        x8, _, _ = sgp.cg_solve(lat, _cuda(w.values[:, :8]), 0.1, 0.0, max_iter=6)
        np.testing.assert_array_equal(y8, y16[:, :8])
        np.testing.assert_array_equal(x8.cpu().numpy(), x16[:, :8])
        v24 = np.concatenate([w.values, w.values[:, :8]], axis=1)
        y24 = sgp.lattice_mvm(lat, _cuda(v24)).cpu().numpy()
        x24, _, _ = sgp.cg_solve(lat, _cuda(v24), 0.1, 0.0, max_iter=6)
        x24 = x24.cpu().numpy()
        np.testing.assert_array_equal(y24[:, :16], y16)
        np.testing.assert_array_equal(y24[:, 16:], y16[:, :8])
        np.testing.assert_array_equal(x24[:, :16], x16)
        np.testing.assert_array_equal(x24[:, 16:], x16[:, :8])
        for c in (0, 5, 15):
            v1 = _cuda(w.values[:, c:c + 1])
            y1 = sgp.lattice_mvm(lat, v1).cpu().numpy()
            x1, _, _ = sgp.cg_solve(lat, v1, 0.1, 0.0, max_iter=6)
            np.testing.assert_array_equal(y1[:, 0], y16[:, c])
            np.testing.assert_array_equal(x1.cpu().numpy()[:, 0], x16[:, c])
    finally:
        lat.free()


def test_cg_max_iter_reports_nonconvergence(sgp):
    w = workloads.ws1()
    lat = sgp.lattice_build(_cuda(w.X), w.lengthscales)
    x, iters, rel = sgp.cg_solve(lat, _cuda(w.values), w.noise, 1e-12, max_iter=3)
    assert iters[0] == 3 and rel[0] > 1e-12


def test_build_errors(sgp):
    _note("build errors")
    X = np.random.default_rng(0).standard_normal((100, 3)).astype(np.float32)
    Xn = X.copy()
    Xn[17, 1] = np.nan
    with pytest.raises(sgp.SGPError) as ei:
        sgp.lattice_build(_cuda(Xn), np.ones(3))
    assert ei.value.code == -1
    Xb = X.copy()
    Xb[5, 0] = 3e8
    with pytest.raises(sgp.SGPError) as ei:
        sgp.lattice_build(_cuda(Xb), np.ones(3) * 1e-2)
    assert ei.value.code == -3
    # the library is still usable afterwards
    lat = sgp.lattice_build(_cuda(X), np.ones(3))
    assert lat.m > 0


# ---------------------------------------------------------------------------
# Full-size workloads, in the launch configuration the benchmark times.

def test_ws2_full(sgp, orc):
    _note("full ws2 n=500000 d=8")
    w = workloads.ws2()
    lat, olat = _build_both(sgp, orc, w.X, w.lengthscales)
    _assert_structure(sgp, lat, olat)
    b = w.values.astype(np.float64)
    out = sgp.lattice_mvm(lat, _cuda(w.values)).cpu().numpy()
    _assert_mvm(out, olat, b)
    # a few fixed iterations: iterate parity
    x, iters, rel = sgp.cg_solve(lat, _cuda(w.values), w.noise, 0.0, max_iter=10)
    xo, _, _, _ = olat.cg(b, w.noise, 0.0, max_iter=10)
    assert _colerr(x.cpu().numpy(), xo).max() <= CG_TOL
    # to the tolerance (cond ~2e5, hundreds of iterations): the GPU's answer
    # meets the tolerance under the oracle's operator, in a similar count
    x, iters, rel = sgp.cg_solve(lat, _cuda(w.values), w.noise, w.tol, max_iter=w.max_iter)
    xo, itero, relo, _ = olat.cg(b, w.noise, w.tol, max_iter=w.max_iter)
    assert rel[0] <= w.tol and relo[0] <= w.tol
    assert abs(int(iters[0]) - int(itero[0])) <= 0.1 * itero[0], (iters, itero)
    xg = x.cpu().numpy().astype(np.float64)
    res = b - (olat.mvm(xg) + w.noise * xg)
    assert np.linalg.norm(res) / np.linalg.norm(b) <= 1.05 * w.tol


def _full_step_parity(sgp, orc, w, label):
    """A full-size step as the benchmark runs it: structure bit-exact, the
    fp32 MVM on all C columns (norm and element-wise bars), and the batched
    fp64 CG with a fixed iteration count against the oracle's CG on every
    column."""
    _note(f"full {label} n={w.n} d={w.d} C={w.C}: build + structure")
    lat, olat = _build_both(sgp, orc, w.X, w.lengthscales)
    _assert_structure(sgp, lat, olat)
    V = _cuda(w.values)
    _note(f"full {label}: mvm (m={lat.m})")
    out = sgp.lattice_mvm(lat, V).cpu().numpy()
    _assert_mvm(out, olat, w.values)
    _note(f"full {label}: {w.max_iter} batched CG iterations, oracle on all {w.C} columns")
    x, iters, rel = sgp.cg_solve(lat, V, w.noise, 0.0, max_iter=w.max_iter)
    assert np.all(iters == w.max_iter)
    xo, itero, relo = _oracle_cg_columns(olat, w.values, w.noise, 0.0, w.max_iter, list(range(w.C)))
    assert np.all(itero == w.max_iter)
    err = _colerr(x.cpu().numpy(), xo)
    assert err.max() <= CG_TOL, err
    lat.free()


def test_ws3_full(sgp, orc):
    _full_step_parity(sgp, orc, workloads.ws3(), "ws3")


def test_ws3p_full(sgp, orc):
    """The paper's lattice sparsity (m / n(d+1) ~ 0.04, m ~ 1e6, where the
    blur dominates), at full size: m equals the oracle's lattice size stored
    when the lengthscale factor was chosen, and the step matches the oracle."""
    import json
    w = workloads.ws3p()
    rec = json.load(open(os.path.join(os.path.dirname(workloads.__file__), "ws3p_scale.json")))
    m_stored = round(rec["m_over_L"] * w.n * (w.d + 1))
    lat = sgp.lattice_build(_cuda(w.X), w.lengthscales)
    try:
        assert lat.m == m_stored
    finally:
        lat.free()
    _full_step_parity(sgp, orc, w, "ws3p")


def test_ws4_full_sampled(sgp, orc):
    _note("full ws4 n=1000000 d=16 (sampled points)")
    w = workloads.ws4()
    lat = sgp.lattice_build(_cuda(w.X), w.lengthscales)
    keys, idx, wts, nbr = sgp.lattice_export(lat)
    n, d = w.n, w.d
    assert lat.m <= n * (d + 1)
    # first-occurrence numbering: the running maximum of idx in (point, vertex)
    # order grows by exactly one at every new index
    flat = idx.reshape(-1).astype(np.int64)
    runmax = np.maximum.accumulate(flat)
    assert runmax[0] == 0 and runmax[-1] == lat.m - 1
    assert np.all(np.diff(runmax) <= 1)
    # distinct keys
    assert np.unique(keys, axis=0).shape[0] == lat.m
    # sampled points recomputed one by one by the oracle
    rng = np.random.default_rng(3)
    sample = rng.choice(n, 2000, replace=False)
    okeys, obary, _, _ = orc.simplex(w.X[sample], w.lengthscales)
    np.testing.assert_array_equal(keys[idx[sample]], okeys)
    np.testing.assert_array_equal(wts[sample], obary.astype(np.float32))
    # sampled neighbour entries against a dictionary of all keys
    where = {k.tobytes(): j for j, k in enumerate(keys)}
    for j in rng.choice(lat.m, 300, replace=False):
        for k in range(d + 1):
            for ti, t in enumerate((-1, 1)):
                step = np.full(d, t, dtype=np.int32)
                if k < d:
                    step[k] = -t * d
                target = (keys[j] + step).astype(np.int32).tobytes()
                assert nbr[j, k, ti] == where.get(target, -1)
    # symmetric operator at full size
    U = rng.standard_normal((n, 2)).astype(np.float32)
    KU = sgp.lattice_mvm(lat, _cuda(U)).cpu().numpy().astype(np.float64)
    a, b = U[:, 0] @ KU[:, 1], U[:, 1] @ KU[:, 0]
    assert abs(a - b) <= 1e-5 * (abs(a) + abs(b))


def test_ws4_full_oracle(sgp, orc):
    """The differentiation workload at full size (n = 1M, d = 16, C = 8,
    m ~ 2.4M): structure, the MVM on all 8 columns, and the adjoint with
    respect to X and the log-lengthscales for one column against the
    oracle's k' filtering (Section 4.2)."""
    w = workloads.ws4()
    _note("full ws4 n=1000000 d=16: build + structure")
    lat, olat = _build_both(sgp, orc, w.X, w.lengthscales)
    _assert_structure(sgp, lat, olat)
    _note(f"full ws4: mvm C=8 (m={lat.m})")
    out = sgp.lattice_mvm(lat, _cuda(w.values)).cpu().numpy()
    _assert_mvm(out, olat, w.values)
    del olat
    _note("full ws4: adjoint, one column")
    G = np.random.default_rng(4).standard_normal((w.n, 1)).astype(np.float32)
    V1 = np.ascontiguousarray(w.values[:, :1])
    dX, dl = sgp.lattice_mvm_grad(lat, _cuda(w.X), _cuda(V1), _cuda(G))
    odX, odl = orc.mvm_grad(w.X, w.lengthscales, V1.astype(np.float64), G.astype(np.float64))
    dX = dX.cpu().numpy().astype(np.float64)
    assert np.linalg.norm(dX - odX) / np.linalg.norm(odX) <= 1e-4
    assert np.linalg.norm(dl - odl) / np.linalg.norm(odl) <= 1e-4
    lat.free()


@pytest.mark.parametrize("blur", ["symmetric", "forward", "reverse"])
@pytest.mark.parametrize("seed,n,d,C", [(51, 3000, 3, 4), (52, 2500, 4, 1), (53, 20000, 11, 16),
                                        (54, 777, 2, 3)])
def test_blur_fused_matches_unfused(sgp, blur, seed, n, d, C):
    """Two blur steps fused into one launch give bitwise the same MVM (fp32)
    and CG iterates (fp64) as one launch per step; d + 1 odd leaves a single
    last step."""
    _note(f"blur fusion {blur} seed={seed} n={n} d={d} C={C}")
    c = workloads.small_case(seed, n, d, channels=C, kind="mixture")
    lat = sgp.lattice_build(_cuda(c.X), c.lengthscales, blur=blur)
    V = _cuda(c.values)
    prev = sgp.blur_fuse_enable(False)
    try:
        y0 = sgp.lattice_mvm(lat, V).cpu().numpy()
        x0, it0, rel0 = sgp.cg_solve(lat, V, 0.1, 0.0, max_iter=6)
        x0 = x0.cpu().numpy()
        sgp.blur_fuse_enable(True)
        y1 = sgp.lattice_mvm(lat, V).cpu().numpy()
        x1, it1, rel1 = sgp.cg_solve(lat, V, 0.1, 0.0, max_iter=6)
        np.testing.assert_array_equal(y1, y0)
        np.testing.assert_array_equal(x1.cpu().numpy(), x0)
        np.testing.assert_array_equal(rel1, rel0)
    finally:
        sgp.blur_fuse_enable(prev)
        lat.free()


@pytest.mark.parametrize("seed,n,d,C", [(95, 30000, 11, 16), (96, 9000, 6, 3), (97, 12000, 4, 8)])
def test_blur_sequential_chains_match(sgp, seed, n, d, C):
    """The symmetric blur's two chains run one after the other (as for large
    lattices) give bitwise the same MVM (fp32) and CG iterates (fp64) as both
    chains in one launch, with d + 1 even and odd."""
    _note(f"blur sequential chains seed={seed} n={n} d={d} C={C}")
    c = workloads.small_case(seed, n, d, channels=C, kind="mixture")
    lat = sgp.lattice_build(_cuda(c.X), c.lengthscales)
    V = _cuda(c.values)
    prev = sgp.blur_seq_bytes(-1)
    try:
        y0 = sgp.lattice_mvm(lat, V).cpu().numpy()
        x0, it0, rel0 = sgp.cg_solve(lat, V, 0.1, 0.0, max_iter=6)
        x0 = x0.cpu().numpy()
        sgp.blur_seq_bytes(0)
        y1 = sgp.lattice_mvm(lat, V).cpu().numpy()
        x1, it1, rel1 = sgp.cg_solve(lat, V, 0.1, 0.0, max_iter=6)
        np.testing.assert_array_equal(y1, y0)
        np.testing.assert_array_equal(x1.cpu().numpy(), x0)
        np.testing.assert_array_equal(rel1, rel0)
    finally:
        sgp.blur_seq_bytes(prev)
        lat.free()


@pytest.mark.parametrize("C,fp64", [(5, True), (16, True), (3, False)])
def test_autotune_keeps_results(sgp, C, fp64):
    """Autotuned launch shapes give bitwise the same MVM and CG results, and
    the choice is one of the candidates."""
    _note(f"autotune C={C} fp64={fp64}")
    c = workloads.small_case(71 + C, 20000, 6, channels=C, kind="mixture")
    lat = sgp.lattice_build(_cuda(c.X), c.lengthscales)
    V = _cuda(c.values)
    sgp.autotune_reset()
    try:
        y0 = sgp.lattice_mvm(lat, V).cpu().numpy()
        x0, _, rel0 = sgp.cg_solve(lat, V, 0.1, 0.0, max_iter=6)
        x0 = x0.cpu().numpy()
        ch = sgp.autotune(lat, C, fp64=fp64, reps=2)
        assert ch["chunk"] in (1, 2, 4, 8, 16, 32, 64) and ch["ms_per_mvm"] > 0
        assert ch["splat_blocks_per_cu"] in (0, 1) and ch["slice_blocks_per_cu"] in (0, 1)
        y1 = sgp.lattice_mvm(lat, V).cpu().numpy()
        x1, _, rel1 = sgp.cg_solve(lat, V, 0.1, 0.0, max_iter=6)
        np.testing.assert_array_equal(y1, y0)
        np.testing.assert_array_equal(x1.cpu().numpy(), x0)
        np.testing.assert_array_equal(rel1, rel0)
    finally:
        sgp.autotune_reset()
        lat.free()


@pytest.mark.parametrize("tol,max_iter", [(0.0, 45), (1e-6, 300)])
def test_cg_graph_replay_matches_launches(sgp, tol, max_iter):
    """CG with iteration blocks replayed from a graph equals the launch-by-
    launch solve bitwise, over several solves with other work in between."""
    _note(f"cg graph replay tol={tol} max_iter={max_iter}")
    c = workloads.small_case(41, 6000, 6, channels=5, kind="mixture")
    lat = sgp.lattice_build(_cuda(c.X), c.lengthscales)
    B = _cuda(c.values)
    prev = sgp.cg_graph_enable(False)
    try:
        x_ref, it_ref, rel_ref = sgp.cg_solve(lat, B, 0.05, tol, max_iter=max_iter)
        x_ref = x_ref.cpu().numpy()
        sgp.cg_graph_enable(True)
        for rep in range(3):
            sgp.lattice_mvm(lat, B)  # eager work between the graph solves
            x, it, rel = sgp.cg_solve(lat, B, 0.05, tol, max_iter=max_iter)
            np.testing.assert_array_equal(x.cpu().numpy(), x_ref)
            np.testing.assert_array_equal(it, it_ref)
            np.testing.assert_array_equal(rel, rel_ref)
    finally:
        sgp.cg_graph_enable(prev)
        lat.free()
    if tol > 0:
        assert np.all(it_ref > 20)  # several replayed blocks ran


@pytest.mark.parametrize("seed,n,d,C,tol,max_iter", [(61, 20000, 6, 16, 0.0, 20), (62, 9000, 4, 4, 1e-5, 400),
                                                     (63, 5000, 3, 5, 1e-4, 300), (64, 3000, 5, 1, 0.0, 13),
                                                     (65, 12000, 7, 32, 0.0, 11), (66, 4000, 2, 8, 1e-6, 600),
                                                     (67, 6000, 3, 2, 1e-5, 300)])
def test_cg_fused_direction_update_matches_pass(sgp, seed, n, d, C, tol, max_iter):
    """The CG direction update run inside the next splat gives bitwise the
    same iterates, iteration counts and residuals as its own pass, with
    columns that stop at different iterations, widths that take the fused
    path (C = 4, 8, 16, 32 as 16-byte vectors, C = 1, 2 element by element)
    and a width that falls back to the pass (C = 5: its channel chunk is
    wider than C), and graph replay on."""
    _note(f"cg fused direction update seed={seed} n={n} d={d} C={C} tol={tol}")
    c = workloads.small_case(seed, n, d, channels=C, kind="mixture")
    lat = sgp.lattice_build(_cuda(c.X), c.lengthscales)
    B = _cuda(c.values)
    prev = sgp.cg_fuse_enable(False)
    try:
        x0, it0, rel0 = sgp.cg_solve(lat, B, 0.05, tol, max_iter=max_iter)
        x0 = x0.cpu().numpy()
        sgp.cg_fuse_enable(True)
        for _ in range(2):
            x1, it1, rel1 = sgp.cg_solve(lat, B, 0.05, tol, max_iter=max_iter)
            np.testing.assert_array_equal(x1.cpu().numpy(), x0)
            np.testing.assert_array_equal(it1, it0)
            np.testing.assert_array_equal(rel1, rel0)
    finally:
        sgp.cg_fuse_enable(prev)
        lat.free()


def test_autotune_build_keeps_structure(sgp):
    """Every hash-table shape the build autotuner tries, and the one it keeps,
    give the same lattice bit for bit (numbering by first occurrence)."""
    _note("build autotune")
    c = workloads.small_case(67, 30000, 9, channels=1, kind="mixture")
    X = _cuda(c.X)
    sgp.autotune_reset()
    try:
        lat = sgp.lattice_build(X, c.lengthscales)
        ref = sgp.lattice_export(lat)
        lat.free()
        ch = sgp.autotune_build(X, c.lengthscales, reps=1)
        assert round(ch["load_factor"], 6) in (0.25, 0.5, 0.9) and ch["shrink"] in (0, 2, 3, 4)
        assert ch["ms_per_build"] > 0
        for lf in (0.0, 0.25, 0.9):
            lat = sgp.lattice_build(X, c.lengthscales, load_factor=lf)
            got = sgp.lattice_export(lat)
            lat.free()
            for a, b in zip(ref, got):
                np.testing.assert_array_equal(a, b)
    finally:
        sgp.autotune_reset()
