"""Pins of the CPU oracle against what the paper and mathematics fix.

None of these re-types an oracle formula: each checks a property, a closed
form, a textbook special case, a library routine or a brute force that an
error in the oracle (dropped term, wrong sign or index, transposed operand,
wrong scale) would break.
"""
import os

import numpy as np
import pytest
from scipy import integrate, optimize, special

import workloads

HERE = os.path.dirname(os.path.abspath(__file__))


# ---------------------------------------------------------------------------
# Stencil spacing: the root of the coverage balance (Section 4.1,
# eq. balance_coverage), found here with scipy quadrature and root finding.

def _coverage_root(kernel_fn, r):
    m = 2 * r + 1
    total, _ = integrate.quad(kernel_fn, -np.inf, np.inf)

    def fourier(w):  # real, even kernel: F(w) = 2 int_0^inf k(t) cos(w t) dt
        v, _ = integrate.quad(kernel_fn, 0, np.inf, weight="cos", wvar=w)
        return 2.0 * v

    ftotal = 2.0 * np.pi * kernel_fn(0.0)  # inverse transform at 0

    def gap(s):
        a = s * m / 2.0
        spatial = integrate.quad(kernel_fn, -a, a)[0] / total
        b = np.pi / s
        spectral = 2.0 * integrate.quad(fourier, 0, b, limit=200)[0] / ftotal
        return spatial - spectral

    return optimize.brentq(gap, 0.2, 5.0, xtol=1e-13)


def _rbf(t):
    return np.exp(-0.5 * t * t)


def _matern32(t):
    a = np.sqrt(3.0) * abs(t)
    return (1.0 + a) * np.exp(-a)


@pytest.mark.parametrize("r", [1, 2, 3])
def test_rbf_spacing_is_coverage_root(orc, r):
    s, stencil, _, _ = orc.constants(3, r, orc.RBF)
    # closed form of the balance for the Gaussian: erf(s m / 2 / sqrt2) = erf(pi / s / sqrt2)
    s_erf = optimize.brentq(
        lambda s_: special.erf(s_ * (2 * r + 1) / 2 / np.sqrt(2)) - special.erf(np.pi / s_ / np.sqrt(2)),
        0.1, 10, xtol=1e-15)
    assert abs(s - s_erf) < 1e-12
    assert abs(s - _coverage_root(_rbf, r)) < 1e-6
    t = np.arange(-r, r + 1)
    np.testing.assert_allclose(stencil, np.exp(-0.5 * (t * s) ** 2), rtol=1e-15)
    if r == 1:
        assert abs(stencil[0] - np.exp(-np.pi / 3)) < 1e-15
        assert stencil[1] == 1.0


def test_matern32_spacing_is_coverage_root(orc):
    s, stencil, _, _ = orc.constants(3, 1, orc.MATERN32)
    assert abs(s - _coverage_root(_matern32, 1)) < 1e-6
    assert abs(stencil[0] - _matern32(s)) < 1e-12
    assert stencil[1] == 1.0


# ---------------------------------------------------------------------------
# Elevation (Section 3.2, Splat): an orthogonal triangular basis of H_d.

@pytest.mark.parametrize("d", [1, 2, 5, 11, 20])
def test_elevation_is_scaled_orthogonal_into_hyperplane(orc, d):
    rng = np.random.default_rng(d)
    ell = np.exp(rng.uniform(-1, 1, d))
    E = orc.embed(np.eye(d, dtype=np.float32), ell).T  # (d+1) x d, column j = image of e_j
    s, _, alpha, _ = orc.constants(d, 1, orc.RBF, ell)
    np.testing.assert_allclose(np.ones(d + 1) @ E, 0.0, atol=1e-12 * alpha)
    G = E.T @ E
    np.testing.assert_allclose(G, np.diag(alpha ** 2 / ell ** 2), rtol=1e-12, atol=1e-10 * alpha ** 2)
    # Reading: one lattice step along any direction covers s lengthscale units.
    for k in range(d + 1):
        step = np.ones(d + 1)
        step[k] -= d + 1
        delta, *_ = np.linalg.lstsq(E, step, rcond=None)
        np.testing.assert_allclose(E @ delta, step, atol=1e-9)
        assert abs(np.linalg.norm(delta / ell) - s) < 1e-9


# ---------------------------------------------------------------------------
# Keys and barycentric weights (Section 3.2, eq. canon_simplex).

def _golden_simplex():
    rows = {}
    with open(os.path.join(HERE, "golden", "canonical_simplex.txt")) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            v = [int(t) for t in line.split()]
            rows.setdefault(v[0], {})[v[1]] = np.array(v[2:])
    return rows


def _full_keys(r0, rank, d):
    """All d+1 coordinates of each vertex from the remainder-0 point and ranks."""
    D = d + 1
    k = np.arange(D)
    # vertex k: r0 + k, minus (d+1) where rank > d - k
    return r0[:, None, :] + k[None, :, None] - D * (rank[:, None, :] > (d - k)[None, :, None])


@pytest.mark.parametrize("d", [2, 3, 4])
def test_canonical_simplex_golden(orc, d):
    """A point just inside the canonical simplex gets exactly its vertices."""
    gold = _golden_simplex()[d]
    # barycentre of the canonical simplex, then solve for x (l = 1)
    verts = np.array([gold[k] for k in range(d + 1)], dtype=np.float64)
    ybar = verts.mean(axis=0)
    E = orc.embed(np.eye(d, dtype=np.float32), np.ones(d)).T
    x, *_ = np.linalg.lstsq(E, ybar, rcond=None)
    keys, bary, r0, rank = orc.simplex(x[None, :].astype(np.float32), np.ones(d))
    full = _full_keys(r0, rank, d)[0]
    for k in range(d + 1):
        np.testing.assert_array_equal(full[k], gold[k])
        np.testing.assert_array_equal(keys[0, k], gold[k][:d])
    np.testing.assert_allclose(bary[0], 1.0 / (d + 1), atol=1e-6)


@pytest.mark.parametrize("d,kind", [(1, "normal"), (2, "normal"), (3, "mixture"), (8, "mixture"),
                                    (11, "uniform"), (20, "normal")])
def test_simplex_invariants(orc, d, kind):
    w = workloads.small_case(7 + d, 400, d, kind=kind)
    keys, bary, r0, rank = orc.simplex(w.X, w.lengthscales)
    y = orc.embed(w.X, w.lengthscales)
    D = d + 1
    full = _full_keys(r0, rank, d)
    np.testing.assert_array_equal(full[:, :, :d], keys)
    # lattice points: coordinates sum to zero, all congruent to k mod d+1
    assert np.all(full.sum(axis=2) == 0)
    for k in range(D):
        assert np.all(np.mod(full[:, k, :], D) == k)
    # ranks are permutations
    assert np.all(np.sort(rank, axis=1) == np.arange(D))
    # consecutive vertices differ by one lattice direction 1 - (d+1) e_j
    for k in range(d):
        diff = full[:, k + 1, :] - full[:, k, :]
        assert np.all(np.sort(diff, axis=1)[:, 0] == -d)
        assert np.all(np.sort(diff, axis=1)[:, 1:] == 1)
    # the vertex set, shifted by r0, is a permutation of the canonical simplex
    canon = np.array([[k] * (D - k) + [k - D] * k for k in range(D)])
    for i in range(0, len(full), 37):
        for k in range(D):
            np.testing.assert_array_equal(np.sort(full[i, k] - r0[i])[::-1], canon[k])
    # barycentric: non-negative, sum to one, reproduce the point
    assert np.all(bary >= -1e-12)
    np.testing.assert_allclose(bary.sum(axis=1), 1.0, atol=1e-12)
    recon = np.einsum("nk,nkj->nj", bary, full.astype(np.float64))
    scale = np.linalg.norm(y, axis=1, keepdims=True) + 1.0
    assert np.all(np.abs(recon - y) <= 1e-9 * scale)


def test_ties_zero_rows_and_grid_points(orc):
    """Exact ties: the origin and points exactly on the d=1 grid."""
    d = 3
    keys, bary, r0, rank = orc.simplex(np.zeros((2, d), np.float32), np.ones(d))
    # all residuals tie at 0: ranks follow the index order, weight 1 on vertex 0
    np.testing.assert_array_equal(rank[0], np.arange(d + 1))
    np.testing.assert_array_equal(bary[0], [1.0, 0, 0, 0])
    np.testing.assert_array_equal(keys[0, 0], 0)
    s, _, _, _ = orc.constants(1, 1, orc.RBF)
    x = (np.arange(-3, 4) * s).astype(np.float32)[:, None]
    keys, bary, _, _ = orc.simplex(x, np.ones(1))
    assert np.all(bary >= 0) and np.allclose(bary.sum(1), 1)


# Exact residual ties at d >= 2. Zero input coordinates make elevated
# coordinates exactly equal: x = (t, 0, 0) elevates to y = (c, -c, 0, 0) and
# x = (0, t) to y = (c, c, -2c), where c = t sqrt(d(d+1)) / (s sqrt(j(j+1)))
# for the nonzero coordinate j and unit lengthscales (the triangular basis of
# the elevation, scaled so that one lattice step spans s lengthscales;
# Section 3.2, Splat). The tie rule (ties
# ranked by lower coordinate index first, rounding half to even) then fixes
# which vertex of the shared face the point's zero-weight vertex is. The
# vertices below were worked out by hand from eq. canon_simplex:
#  (a) d=3, c ~ 1.2: r0 = 0, residuals (c, -c, 0, 0), ranks (0, 3, 1, 2);
#      vertex k = r0 + k - (d+1) [rank > d-k]: (0,0,0,0), (1,-3,1,1),
#      (2,-2,2,-2), (3,-1,-1,-1); weights (1 - c/2, c/4, 0, c/4). The
#      opposite tie order would give vertex 2 = (2,-2,-2,2).
#  (b) d=2, c ~ 0.5: r0 = 0, residuals (c, c, -2c), ranks (0, 1, 2);
#      vertices (0,0,0), (1,1,-2), (2,-1,-1); weights (1 - c, c, 0). The
#      opposite order gives vertex 2 = (-1,2,-1).
#  (c) d=2, c ~ 1.6: rounding y/3 gives (1, 1, -1), so r0 = (3, 3, -3) with
#      excess 1; residuals (c-3, c-3, 3-2c) rank (1, 2, 0) before the sum
#      fix, which lowers the coordinate of rank 2 (index 1): r0 = (3, 0, -3),
#      ranks (2, 0, 1); vertices (3,0,-3), (1,1,-2), (2,2,-4); vertex 0 has
#      weight 1 + (c-3)/3 - c/3 = 0 (up to one rounding of the residuals).
#      The opposite order lowers index 0 instead and gives vertex 0 =
#      (0,3,-3).
TIE_CASES = [
    (3, (1.2, 0.0, 0.0), [[0, 0, 0], [1, -3, 1], [2, -2, 2], [3, -1, -1]], 2),
    (2, (0.0, 0.5), [[0, 0], [1, 1], [2, -1]], 2),
    (2, (0.0, 1.6), [[3, 0], [1, 1], [2, 2]], 0),
]


@pytest.mark.parametrize("d,c,expected,zero_vertex", TIE_CASES)
def test_exact_ties_at_higher_dimension(orc, d, c, expected, zero_vertex):
    s, _, _, _ = orc.constants(d, 1, orc.RBF)
    j = np.arange(1, d + 1)
    x = (np.asarray(c) * s * np.sqrt(j * (j + 1)) / np.sqrt(d * (d + 1))).astype(np.float32)[None, :]
    y = orc.embed(x, np.ones(d))[0]
    cval = y[0]
    assert abs(cval - max(c)) < 1e-6
    # the zero coordinates produce exact ties in the elevated point
    if d == 3:
        assert y[2] == 0.0 and y[3] == 0.0 and y[0] == -y[1]
    else:
        assert y[0] == y[1] and y[2] == -2 * y[0]
    keys, bary, r0, rank = orc.simplex(x, np.ones(d))
    np.testing.assert_array_equal(keys[0], np.asarray(expected, dtype=np.int32))
    assert abs(bary[0, zero_vertex]) <= 1e-15
    assert np.all(bary[0] >= -1e-15) and abs(bary[0].sum() - 1.0) < 1e-12
    full = _full_keys(r0, rank, d)[0].astype(np.float64)
    np.testing.assert_allclose(bary[0] @ full, y, atol=1e-12)
    # the same points inside a lattice: the zero-weight vertex is inserted
    # (it counts in m), as a vertex of its own
    lat = orc.Lattice(x, np.ones(d))
    assert lat.m == d + 1


# ---------------------------------------------------------------------------
# d = 1: the lattice is a grid of spacing s*l, W is linear interpolation and
# both blur directions are the same 1-D stencil (Section 3.2; Section 4.1).

def _d1_reference(X, ell, V, s):
    u = X[:, 0].astype(np.float64) / (s * ell[0])
    lo = np.floor(u).astype(np.int64)
    frac = u - lo
    nodes = np.unique(np.concatenate([lo, lo + 1]))
    pos = {v: i for i, v in enumerate(nodes)}
    W = np.zeros((len(X), len(nodes)))
    for i in range(len(X)):
        W[i, pos[lo[i]]] += 1 - frac[i]
        W[i, pos[lo[i] + 1]] += frac[i]
    w1 = np.exp(-0.5 * s * s)
    S = np.eye(len(nodes))
    for a in range(len(nodes) - 1):
        if nodes[a + 1] == nodes[a] + 1:
            S[a, a + 1] = S[a + 1, a] = w1
    return W, S, nodes


@pytest.mark.parametrize("seed", [0, 1])
def test_d1_is_linear_interpolation_and_toeplitz_blur(orc, seed):
    rng = np.random.default_rng(seed)
    n = 300
    X = (rng.standard_normal((n, 1)) * 3).astype(np.float32)
    ell = np.array([0.7])
    s = np.sqrt(2 * np.pi / 3)
    lat = orc.Lattice(X, ell)
    keys, idx, w, nbr = lat.export()
    W, S, nodes = _d1_reference(X, ell, None, s)
    # same grid nodes; map oracle lattice index -> node position
    assert sorted(keys[:, 0].tolist()) == nodes.tolist()
    Wo = np.zeros((n, lat.m))
    for i in range(n):
        for k in range(2):
            Wo[i, idx[i, k]] += w[i, k]
    perm = np.array([np.searchsorted(nodes, keys[j, 0]) for j in range(lat.m)])
    Wref = W[:, perm]
    np.testing.assert_allclose(Wo, Wref, atol=1e-12)
    Sref = S[np.ix_(perm, perm)]
    V = rng.standard_normal((n, 3))
    Kref = Wref @ Sref @ Sref @ Wref.T
    for mode in (orc.SYMMETRIC, orc.FORWARD, orc.REVERSE):
        np.testing.assert_allclose(lat.mvm(V, mode=mode), Kref @ V, rtol=1e-12, atol=1e-12)


# ---------------------------------------------------------------------------
# Canonical numbering, neighbours and blur by brute force on tiny inputs.

def _brute_lattice(orc, X, ell, r):
    keys, bary, _, _ = orc.simplex(X, ell, r=r)
    n, D, d = keys.shape
    seen = []  # O(L^2) first-occurrence scan
    idx = np.zeros((n, D), dtype=np.int64)
    for i in range(n):
        for k in range(D):
            key = keys[i, k].tolist()
            j = next((q for q, kk in enumerate(seen) if kk == key), None)
            if j is None:
                j = len(seen)
                seen.append(key)
            idx[i, k] = j
    return np.array(seen, dtype=np.int64), idx, bary


def _direction(d, k):
    step = np.ones(d + 1, dtype=np.int64)
    step[k] -= d + 1
    return step[:d]


@pytest.mark.parametrize("d", [2, 3, 5])
def test_canonical_order_and_neighbours_brute_force(orc, d):
    w = workloads.small_case(40 + d, 60, d, kind="mixture")
    keys_b, idx_b, bary_b = _brute_lattice(orc, w.X, w.lengthscales, 2)
    lat = orc.Lattice(w.X, w.lengthscales, r=2)
    keys, idx, wts, nbr = lat.export()
    assert lat.m == len(keys_b) <= w.n * (d + 1)
    np.testing.assert_array_equal(keys, keys_b)
    np.testing.assert_array_equal(idx, idx_b)
    np.testing.assert_array_equal(wts, bary_b)
    where = {tuple(k): j for j, k in enumerate(keys_b.tolist())}
    for j in range(lat.m):
        for k in range(d + 1):
            for ti, t in enumerate([-2, -1, 1, 2]):
                target = tuple((keys_b[j] + t * _direction(d, k)).tolist())
                assert nbr[j, k, ti] == where.get(target, -1)


def _dense_operator(orc, lat, X, ell, s, r, mode):
    """W S_k ... W^T from keys by coordinate arithmetic and the scipy-pinned stencil."""
    keys, idx, w, _ = lat.export()
    n, D = idx.shape
    d = D - 1
    m = lat.m
    where = {tuple(k): j for j, k in enumerate(keys.tolist())}
    stencil = {t: np.exp(-0.5 * (t * s) ** 2) for t in range(-r, r + 1)}
    S = []
    for k in range(D):
        Sk = np.zeros((m, m))
        for j in range(m):
            for t in range(-r, r + 1):
                nb = where.get(tuple((keys[j] + t * _direction(d, k)).tolist()))
                if nb is not None:
                    Sk[j, nb] += stencil[t]
        S.append(Sk)
    W = np.zeros((n, m))
    for i in range(n):
        for k in range(D):
            W[i, idx[i, k]] += w[i, k]
    B = np.eye(m)
    order = range(D) if mode == orc.FORWARD else range(D - 1, -1, -1)
    for k in order:
        B = S[k] @ B
    return W @ B @ W.T, W, S


@pytest.mark.parametrize("d,r", [(2, 1), (3, 1), (3, 2), (4, 1)])
def test_blur_brute_force_and_adjoint(orc, d, r):
    w = workloads.small_case(70 + d, 120, d, kind="mixture")
    lat = orc.Lattice(w.X, w.lengthscales, r=r)
    s = _coverage_root(_rbf, r) if r > 1 else np.sqrt(2 * np.pi / 3)
    Kf, W, S = _dense_operator(orc, lat, w.X, w.lengthscales, s, r, orc.FORWARD)
    Kr, _, _ = _dense_operator(orc, lat, w.X, w.lengthscales, s, r, orc.REVERSE)
    I = np.eye(w.n)
    Kf_o = lat.mvm(I, mode=orc.FORWARD)
    Kr_o = lat.mvm(I, mode=orc.REVERSE)
    Ks_o = lat.mvm(I, mode=orc.SYMMETRIC)
    np.testing.assert_allclose(Kf_o, Kf, rtol=1e-9, atol=1e-9 * np.abs(Kf).max())
    np.testing.assert_allclose(Kr_o, Kr, rtol=1e-9, atol=1e-9 * np.abs(Kf).max())
    # every S_k is symmetric, so REVERSE is the transpose of FORWARD
    for Sk in S:
        np.testing.assert_array_equal(Sk, Sk.T)
    np.testing.assert_allclose(Kr_o, Kf_o.T, atol=1e-12 * np.abs(Kf).max())
    # SYMMETRIC averages the two chains and is exactly symmetric
    np.testing.assert_allclose(Ks_o, 0.5 * (Kf_o + Kr_o), atol=1e-12 * np.abs(Kf).max())
    np.testing.assert_allclose(Ks_o, Ks_o.T, atol=1e-12 * np.abs(Kf).max())
    # the pieces: splat is W^T, slice is W
    V = np.random.default_rng(0).standard_normal((w.n, 2))
    np.testing.assert_allclose(lat.splat(V), W.T @ V, atol=1e-12)
    U = np.random.default_rng(1).standard_normal((lat.m, 2))
    np.testing.assert_allclose(lat.slice(U), W @ U, atol=1e-12)


def test_mvm_linearity_and_outputscale(orc):
    w = workloads.small_case(5, 500, 6, channels=3, kind="mixture")
    lat = orc.Lattice(w.X, w.lengthscales)
    rng = np.random.default_rng(3)
    A, B = rng.standard_normal((w.n, 3)), rng.standard_normal((w.n, 3))
    lhs = lat.mvm(2.0 * A - 3.0 * B)
    rhs = 2.0 * lat.mvm(A) - 3.0 * lat.mvm(B)
    np.testing.assert_allclose(lhs, rhs, rtol=1e-10, atol=1e-10 * np.abs(rhs).max())
    np.testing.assert_allclose(lat.mvm(A, outputscale=2.5), 2.5 * lat.mvm(A), rtol=1e-14)
    # columns are independent
    np.testing.assert_allclose(lat.mvm(A)[:, 1], lat.mvm(A[:, 1])[:, 0], rtol=1e-14)
    # u.Kv = v.Ku for the symmetric operator
    u, v = A[:, 0], B[:, 0]
    assert abs(u @ lat.mvm(v)[:, 0] - v @ lat.mvm(u)[:, 0]) < 1e-10 * abs(u @ lat.mvm(v)[:, 0])


# ---------------------------------------------------------------------------
# Approximation quality against the exact RBF MVM (Section 5.1, cosine error).
# Bounds stated after measuring at n = 2,000 (d = 3, l = 1): 0.060 against
# the exact kernel and 0.022 against the RBF with lengthscale l sqrt((d+1)/d),
# the scale a product of d+1 one-dimensional blurs produces.

def _cos_err(a, b):
    return 1 - (a @ b) / np.linalg.norm(a) / np.linalg.norm(b)


def test_cosine_error_against_exact_rbf(orc):
    w = workloads.ws1()
    lat = orc.Lattice(w.X, w.lengthscales)
    assert lat.m <= w.n * (w.d + 1)
    v = w.values[:, 0].astype(np.float64)
    z = lat.mvm(v)[:, 0]
    Z = w.X.astype(np.float64) / w.lengthscales
    D2 = ((Z[:, None, :] - Z[None, :, :]) ** 2).sum(-1)
    exact = np.exp(-0.5 * D2) @ v
    wide = np.exp(-0.5 * D2 / ((w.d + 1) / w.d)) @ v
    assert _cos_err(z, exact) < 0.08
    assert _cos_err(z, wide) < 0.03
    # a lattice with the wrong scale would be far off
    far = np.exp(-0.5 * D2 * 4.0) @ v
    assert _cos_err(z, far) > 0.1


# ---------------------------------------------------------------------------
# Conjugate gradients: the dense solve (library routine) and the Krylov
# characterisation of the iterates.

def test_cg_matches_dense_solve(orc):
    w = workloads.ws1(n=800)
    lat = orc.Lattice(w.X, w.lengthscales)
    A = lat.mvm(np.eye(w.n)) + w.noise * np.eye(w.n)
    b = w.values.astype(np.float64)
    x_ref = np.linalg.solve(A, b)
    x, iters, rel, rel_true = lat.cg(b, w.noise, 1e-10, max_iter=2000)
    assert iters[0] < 2000 and rel[0] <= 1e-10
    np.testing.assert_allclose(x, x_ref, rtol=0, atol=1e-8 * np.abs(x_ref).max())
    assert rel_true[0] < 1e-9


def test_cg_iterates_minimise_energy_over_krylov_space(orc):
    w = workloads.small_case(11, 300, 4, channels=1, kind="mixture")
    lat = orc.Lattice(w.X, w.lengthscales)
    noise = 0.05
    A = lat.mvm(np.eye(w.n)) + noise * np.eye(w.n)
    b = w.values[:, 0].astype(np.float64)
    for k in (1, 3, 6):
        x, iters, _, _ = lat.cg(b, noise, 0.0, max_iter=k)
        assert iters[0] == k
        Kry = np.stack([np.linalg.matrix_power(A, p) @ b for p in range(k)], axis=1)
        Q, _ = np.linalg.qr(Kry)
        yk = np.linalg.solve(Q.T @ A @ Q, Q.T @ b)
        np.testing.assert_allclose(x[:, 0], Q @ yk, rtol=1e-7, atol=1e-9 * np.abs(Q @ yk).max())


def test_cg_columns_independent_and_stop_rule(orc):
    w = workloads.small_case(12, 400, 3, channels=3, kind="normal")
    lat = orc.Lattice(w.X, w.lengthscales)
    B = w.values.astype(np.float64)
    B[:, 2] = 0.0  # zero right-hand side: zero iterations, x = 0
    X, iters, rel, rel_true = lat.cg(B, 0.1, 1e-3)
    x0, it0, _, _ = lat.cg(B[:, :1], 0.1, 1e-3)
    np.testing.assert_array_equal(X[:, :1], x0)
    assert iters[0] == it0[0]
    assert iters[2] == 0 and np.all(X[:, 2] == 0)
    assert rel[0] <= 1e-3 and rel[1] <= 1e-3
    # one iteration fewer would not have met the tolerance
    _, _, rel_m1, _ = lat.cg(B[:, :1], 0.1, 0.0, max_iter=int(iters[0]) - 1)
    assert rel_m1[0] > 1e-3


# ---------------------------------------------------------------------------
# MVM gradient (Section 4.2). A finite difference of the lattice operator is
# no pin (K_lat jumps when a point changes simplex), so the chain is:
# (1) central differences of the dense exact objective confirm the analytic
#     gradient of L = sum G * (K V) for the RBF kernel;
# (2) the four-channel k' rewrite with a dense k' matrix reproduces that
#     gradient exactly (sign and channel layout);
# (3) the oracle equals the same rewrite evaluated with its own lattice
#     operator (materialised column by column), so it implements (2) on the
#     lattice;
# (4) the lattice gradient points along the exact one.

def _dense_objective(Z, V, G):
    D2 = ((Z[:, None, :] - Z[None, :, :]) ** 2).sum(-1)
    return float((G * (np.exp(-0.5 * D2) @ V)).sum())


def _dense_grad_z(Z, V, G):
    """dL/dz_n = 2 sum_j k'_nj (z_n - z_j) (g_n . v_j + v_n . g_j), k' = -k/2."""
    D2 = ((Z[:, None, :] - Z[None, :, :]) ** 2).sum(-1)
    kp = -0.5 * np.exp(-0.5 * D2)
    S = G @ V.T + V @ G.T               # s_nj = g_n . v_j + v_n . g_j
    Wm = kp * S
    return 2.0 * (Wm.sum(1)[:, None] * Z - Wm @ Z)


def _rewrite_grad_z(Z, V, G, Kp):
    """Section 4.2 rewrite: one filtering of [v, z*v, g, z*g] with K'."""
    n, d = Z.shape
    out = np.zeros((n, d))
    for c in range(V.shape[1]):
        v, g = V[:, c:c + 1], G[:, c:c + 1]
        Kv, Kzv = Kp @ v, Kp @ (Z * v)
        Kg, Kzg = Kp @ g, Kp @ (Z * g)
        out += 2.0 * (g * (Z * Kv - Kzv) + v * (Z * Kg - Kzg))
    return out


def test_gradient_chain_dense_fd_and_rewrite():
    rng = np.random.default_rng(5)
    n, d, C = 40, 4, 2
    Z = rng.standard_normal((n, d))
    V, G = rng.standard_normal((n, C)), rng.standard_normal((n, C))
    g_an = _dense_grad_z(Z, V, G)
    h = 1e-3
    g_fd = np.zeros_like(Z)
    for i in range(n):
        for p in range(d):
            Zp, Zm = Z.copy(), Z.copy()
            Zp[i, p] += h
            Zm[i, p] -= h
            g_fd[i, p] = (_dense_objective(Zp, V, G) - _dense_objective(Zm, V, G)) / (2 * h)
    np.testing.assert_allclose(g_an, g_fd, rtol=1e-5, atol=1e-6 * np.abs(g_fd).max())
    D2 = ((Z[:, None, :] - Z[None, :, :]) ** 2).sum(-1)
    Kp = -0.5 * np.exp(-0.5 * D2)
    np.testing.assert_allclose(_rewrite_grad_z(Z, V, G, Kp), g_an, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("d", [2, 4])
def test_oracle_gradient_is_the_rewrite_on_the_lattice(orc, d):
    w = workloads.small_case(90 + d, 150, d, channels=2, kind="mixture")
    rng = np.random.default_rng(d)
    V = rng.standard_normal((w.n, 2))
    G = rng.standard_normal((w.n, 2))
    dX, dl = orc.mvm_grad(w.X, w.lengthscales, V, G)
    lat = orc.Lattice(w.X, w.lengthscales)
    Kp = -0.5 * lat.mvm(np.eye(w.n))      # the lattice operator, k' = -k/2
    Z = w.X.astype(np.float64) / w.lengthscales
    gz = _rewrite_grad_z(Z, V, G, Kp)
    np.testing.assert_allclose(dX, gz / w.lengthscales, rtol=1e-9, atol=1e-9 * np.abs(gz).max())
    np.testing.assert_allclose(dl, -(Z * gz).sum(0), rtol=1e-9, atol=1e-9 * np.abs(gz).max())


def test_lattice_gradient_tracks_exact_gradient(orc):
    w = workloads.ws1()
    rng = np.random.default_rng(9)
    V = rng.standard_normal((w.n, 1))
    G = rng.standard_normal((w.n, 1))
    dX, dl = orc.mvm_grad(w.X, w.lengthscales, V, G)
    Z = w.X.astype(np.float64) / w.lengthscales
    # the lattice approximates an RBF widened by sqrt((d+1)/d) (reading R4)
    s2 = (w.d + 1) / w.d
    gz = _dense_grad_z(Z / np.sqrt(s2), V, G) / np.sqrt(s2)
    cos = (dX.ravel() @ gz.ravel()) / np.linalg.norm(dX) / np.linalg.norm(gz)
    assert cos > 0.95, cos  # measured 0.981 at n = 2000, d = 3


def test_cg_restricted_rows_is_the_submatrix_solve(orc):
    """CG on the first n_train points of a lattice built on [X; X*] solves
    with the submatrix of the joint operator (reading for the predictive
    mean, Section 2 eq. gp_pred_mean)."""
    w = workloads.small_case(13, 500, 3, channels=1, kind="mixture")
    n_train = 380
    lat = orc.Lattice(w.X, w.lengthscales)
    K = lat.mvm(np.eye(w.n))
    A = K[:n_train, :n_train] + 0.1 * np.eye(n_train)
    b = np.zeros((w.n, 1))
    b[:n_train] = w.values[:n_train]
    x, iters, rel, rel_true = lat.cg(b, 0.1, 1e-11, max_iter=3000, rows=n_train)
    np.testing.assert_allclose(x[:n_train, 0], np.linalg.solve(A, b[:n_train, 0]), rtol=0,
                               atol=1e-8 * np.abs(x).max())
    assert np.all(x[n_train:] == 0.0)
    # predictive mean: one MVM of [alpha; 0], test rows
    mu = lat.mvm(np.concatenate([x[:n_train], np.zeros((w.n - n_train, 1))]))[n_train:, 0]
    np.testing.assert_allclose(mu, K[n_train:, :n_train] @ x[:n_train, 0], rtol=1e-10,
                               atol=1e-12)
