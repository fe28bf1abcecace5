"""CPU oracle for the Simplex-GP lattice MVM and CG (test infrastructure).

Only tests, the smoke check and the benchmark's CPU-baseline leg use this
package; the GPU library never imports, links or calls it. The arithmetic
lives in ``sgp_oracle.cpp`` (single-threaded fp64 C++, std::unordered_map),
built with g++ and -ffp-contract=off; this module only marshals numpy arrays.

Each function below names the passage of the paper (arXiv:2106.06695) that
defines what it computes; the C++ source carries the detailed steps.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sgp_oracle.cpp")
_LIB = os.path.join(_HERE, "libsgp_oracle.so")

RBF, MATERN32 = 0, 1
SYMMETRIC, FORWARD, REVERSE = 0, 1, 2

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with g++ (no fast-math, no FMA contraction)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        cmd = ["g++", "-std=c++17", "-O2", "-ffp-contract=off", "-fno-fast-math",
               "-fPIC", "-shared", "-o", tmp, _SRC]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build()
    lib = ctypes.CDLL(_LIB)
    P = ctypes.c_void_p
    I64, I32, D = ctypes.c_int64, ctypes.c_int, ctypes.c_double
    sig = {
        "orc_constants": (I32, [I32, I32, I32, P, P, P, P, P]),
        "orc_embed": (I32, [P, I64, I32, P, I32, I32, P]),
        "orc_simplex": (I32, [P, I64, I32, P, I32, I32, P, P, P, P]),
        "orc_build": (P, [P, I64, I32, P, I32, I32]),
        "orc_num_vertices": (I64, [P]),
        "orc_export": (I32, [P, P, P, P, P]),
        "orc_free": (None, [P]),
        "orc_mvm": (I32, [P, P, I32, I32, D, P]),
        "orc_splat": (I32, [P, P, I32, P]),
        "orc_slice": (I32, [P, P, I32, P]),
        "orc_blur": (I32, [P, P, I32, I32]),
        "orc_cg": (I32, [P, P, I32, I32, D, D, D, I32, P, P, P, P]),
        "orc_cg_rows": (I32, [P, P, I32, I32, D, D, D, I32, I64, P, P, P, P]),
        "orc_mvm_grad": (I32, [P, I64, I32, P, I32, I32, I32, P, P, I32, P, P]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _x(X):
    X = np.ascontiguousarray(X, dtype=np.float32)
    if X.ndim != 2:
        raise ValueError("X must be n x d")
    return X


def _ell(ell, d):
    ell = np.ascontiguousarray(ell, dtype=np.float64)
    if ell.shape != (d,):
        raise ValueError("lengthscales must have d entries")
    return ell


def _check(rc, what):
    if rc != 0:
        raise ValueError(f"oracle {what} failed with code {rc}")


def constants(d: int, r: int = 1, kernel: int = RBF, ell=None):
    """Spacing s, stencil k(t s) for t=-r..r, alpha and elevation factors
    (Section 4.1, eq. balance_coverage; Section 3.2 Splat)."""
    ell = np.ones(d) if ell is None else _ell(ell, d)
    s, alpha = ctypes.c_double(), ctypes.c_double()
    st = np.zeros(2 * r + 1)
    f = np.zeros(d)
    _check(_load().orc_constants(d, r, kernel, _p(ell), ctypes.byref(s), _p(st),
                                 ctypes.byref(alpha), _p(f)), "constants")
    return s.value, st, alpha.value, f


def embed(X, ell, r: int = 1, kernel: int = RBF):
    """Elevated points in H_d (Section 3.2, Splat)."""
    X = _x(X)
    n, d = X.shape
    y = np.zeros((n, d + 1))
    _check(_load().orc_embed(_p(X), n, d, _p(_ell(ell, d)), r, kernel, _p(y)), "embed")
    return y


def simplex(X, ell, r: int = 1, kernel: int = RBF):
    """Per point: vertex keys (n, d+1, d), barycentric weights (n, d+1),
    remainder-0 point and ranks (n, d+1) (Section 3.2, eq. canon_simplex)."""
    X = _x(X)
    n, d = X.shape
    keys = np.zeros((n, d + 1, d), dtype=np.int32)
    bary = np.zeros((n, d + 1))
    r0 = np.zeros((n, d + 1), dtype=np.int32)
    rank = np.zeros((n, d + 1), dtype=np.int32)
    rc = _load().orc_simplex(_p(X), n, d, _p(_ell(ell, d)), r, kernel, _p(keys), _p(bary),
                             _p(r0), _p(rank))
    _check(rc, "simplex")
    return keys, bary, r0, rank


class Lattice:
    """The oracle's lattice: W (idx, w), lattice keys and neighbour table."""

    def __init__(self, X, ell, r: int = 1, kernel: int = RBF):
        X = _x(X)
        self.n, self.d = X.shape
        self.r = r
        self.kernel = kernel
        lib = _load()
        self._h = lib.orc_build(_p(X), self.n, self.d, _p(_ell(ell, self.d)), r, kernel)
        if not self._h:
            raise ValueError("oracle lattice build failed")
        self.m = int(lib.orc_num_vertices(self._h))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            _load().orc_free(h)
            self._h = None

    def export(self):
        d, D, T = self.d, self.d + 1, 2 * self.r
        keys = np.zeros((self.m, d), dtype=np.int32)
        idx = np.zeros((self.n, D), dtype=np.int32)
        w = np.zeros((self.n, D))
        nbr = np.zeros((self.m, D, T), dtype=np.int32)
        _check(_load().orc_export(self._h, _p(keys), _p(idx), _p(w), _p(nbr)), "export")
        return keys, idx, w, nbr

    def _v(self, V):
        V = np.ascontiguousarray(V, dtype=np.float64)
        if V.ndim == 1:
            V = V[:, None]
        if V.shape[0] != self.n:
            raise ValueError("values must have n rows")
        return V

    def mvm(self, V, mode: int = SYMMETRIC, outputscale: float = 1.0):
        """outputscale * W B W^T V (eq. ski_to_bf)."""
        V = self._v(V)
        out = np.zeros_like(V)
        _check(_load().orc_mvm(self._h, _p(V), V.shape[1], mode, outputscale, _p(out)), "mvm")
        return out

    def splat(self, V):
        V = self._v(V)
        U = np.zeros((self.m, V.shape[1]))
        _check(_load().orc_splat(self._h, _p(V), V.shape[1], _p(U)), "splat")
        return U

    def slice(self, U):
        U = np.ascontiguousarray(U, dtype=np.float64)
        out = np.zeros((self.n, U.shape[1]))
        _check(_load().orc_slice(self._h, _p(U), U.shape[1], _p(out)), "slice")
        return out

    def blur(self, U, mode: int = SYMMETRIC):
        U = np.array(U, dtype=np.float64, order="C", copy=True)
        _check(_load().orc_blur(self._h, _p(U), U.shape[1], mode), "blur")
        return U

    def cg(self, B, noise: float, tol: float, max_iter: int = 500, mode: int = SYMMETRIC,
           outputscale: float = 1.0, rows: int = 0):
        """Per-column CG on outputscale*K_lat + noise*I (Section 2, Krylov
        methods), optionally restricted to the first `rows` points. Returns x,
        iterations, recursive and true relative residuals."""
        B = self._v(B)
        C = B.shape[1]
        X = np.zeros_like(B)
        iters = np.zeros(C, dtype=np.int32)
        rel = np.zeros(C)
        rel_true = np.zeros(C)
        _check(_load().orc_cg_rows(self._h, _p(B), C, mode, outputscale, noise, tol, max_iter,
                                   int(rows), _p(X), _p(iters), _p(rel), _p(rel_true)), "cg")
        return X, iters, rel, rel_true


def mvm_grad(X, ell, V, G, r: int = 1, mode: int = SYMMETRIC):
    """Gradient of sum(G * (K_lat V)) with respect to X and log-lengthscales,
    by one filtering with k' of the concatenated channels (Section 4.2)."""
    X = _x(X)
    n, d = X.shape
    V = np.ascontiguousarray(V, dtype=np.float64).reshape(n, -1)
    G = np.ascontiguousarray(G, dtype=np.float64).reshape(n, -1)
    C = V.shape[1]
    dX = np.zeros((n, d))
    dl = np.zeros(d)
    _check(_load().orc_mvm_grad(_p(X), n, d, _p(_ell(ell, d)), r, RBF, mode, _p(V), _p(G), C,
                                _p(dX), _p(dl)), "mvm_grad")
    return dX, dl
