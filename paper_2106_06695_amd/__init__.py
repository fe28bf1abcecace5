"""Python binding of libsimplexgp (the MI355X permutohedral-lattice library).

Argument marshalling only: every step of the lattice build, MVM and CG runs
in the library's HIP kernels. Tensors are torch CUDA (ROCm) tensors, used
here for device memory and streams; the functions mirror the C ABI in
include/simplexgp.h:

    lattice_build(X, lengthscales, ...) -> Lattice
    lattice_mvm(lat, values, out=None)  -> out = outputscale * W K_UU W^T values
    cg_solve(lat, rhs, noise, tol, max_iter=500, x=None) -> (x, iters, rel_residual)
    lattice_info(lat), lattice_export(lat), lattice_free(lat)

If the compiled library is missing, every call raises: there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

from . import _lib

__all__ = [
    "SGPError", "Lattice", "lattice_build", "lattice_mvm", "cg_solve", "lattice_mvm_grad",
    "lattice_info", "lattice_export", "lattice_free", "lattice_kernel_mvm", "profile",
    "library_path", "cg_graph_enable", "blur_fuse_enable", "blur_seq_bytes", "autotune", "autotune_reset",
    "set_allocator", "use_torch_allocator",
]

SYMMETRIC, FORWARD, REVERSE = 0, 1, 2
RBF, MATERN32 = 0, 1
_BLUR = {"symmetric": SYMMETRIC, "forward": FORWARD, "reverse": REVERSE}
_KERNEL = {"rbf": RBF, "matern32": MATERN32}


class SGPError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"[{code}] {msg}")
        self.code = code


def library_path() -> str:
    return _lib.LIB_PATH


def _check(rc: int):
    if rc != 0:
        raise SGPError(rc, _lib.load().sgp_last_error().decode())


def _stream(dev=None):
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)


def _dev_f32(t, name: str, rows: Optional[int] = None):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA tensor")
    if t.dtype != torch.float32:
        raise TypeError(f"{name} must be float32")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if rows is not None and (t.dim() not in (1, 2) or t.shape[0] != rows):
        raise ValueError(f"{name} must have {rows} rows")
    return ctypes.c_void_p(t.data_ptr())


def _cols(t) -> int:
    return 1 if t.dim() == 1 else int(t.shape[1])


class Lattice:
    """Handle of a lattice built on the device (owned by the library)."""

    def __init__(self, handle: ctypes.c_void_p, n: int, d: int, order: int, blur: int,
                 kernel: int, outputscale: float, device):
        self._h = handle
        self.n, self.d, self.order = n, d, order
        self.blur, self.kernel, self.outputscale = blur, kernel, outputscale
        self.device = device
        m = ctypes.c_int64()
        _check(_lib.load().lattice_info(self._h, None, None, ctypes.byref(m), None))
        self.m = int(m.value)

    def free(self):
        if getattr(self, "_h", None):
            _lib.load().lattice_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass

    @property
    def handle(self):
        if not self._h:
            raise ValueError("lattice already freed")
        return self._h

    def mvm(self, values, out=None):
        return lattice_mvm(self, values, out)

    def cg(self, rhs, noise: float, tol: float, max_iter: int = 500, x=None):
        return cg_solve(self, rhs, noise, tol, max_iter, x)


def lattice_build(X, lengthscales: Sequence[float], order: int = 1, kernel: str = "rbf",
                  blur: str = "symmetric", outputscale: float = 1.0,
                  load_factor: float = 0.0, solve_rows: int = 0) -> Lattice:
    """Build the lattice of X (n x d fp32 CUDA tensor); see lattice_build in
    include/simplexgp.h (Section 3.2 of the paper: Splat and Blur)."""
    lib = _lib.load()
    if X.dim() != 2:
        raise ValueError("X must be n x d")
    n, d = int(X.shape[0]), int(X.shape[1])
    px = _dev_f32(X, "X")
    ell = np.ascontiguousarray(np.asarray(lengthscales, dtype=np.float64).reshape(-1))
    if ell.shape[0] != d:
        raise ValueError("lengthscales must have d entries")
    opts = _lib.Opts()
    lib.sgp_opts_default(ctypes.byref(opts))
    opts.order = int(order)
    opts.kernel = _KERNEL[kernel]
    opts.blur = _BLUR[blur]
    opts.outputscale = float(outputscale)
    opts.load_factor = float(load_factor)
    opts.solve_rows = int(solve_rows)
    h = ctypes.c_void_p()
    _check(lib.lattice_build(px, n, d, ell.ctypes.data_as(ctypes.c_void_p), ctypes.byref(opts),
                             _stream(X.device), ctypes.byref(h)))
    return Lattice(h, n, d, int(order), opts.blur, opts.kernel, float(outputscale), X.device)


def lattice_mvm(lat: Lattice, values, out=None):
    """out = outputscale * W K_UU W^T values (eq. ski_to_bf), asynchronous."""
    import torch
    pv = _dev_f32(values, "values", lat.n)
    C = _cols(values)
    if out is None:
        out = torch.empty_like(values)
    po = _dev_f32(out, "out", lat.n)
    if out.shape != values.shape:
        raise ValueError("out must have the shape of values")
    _check(_lib.load().lattice_mvm(lat.handle, pv, C, po, _stream(values.device)))
    return out


def lattice_mvm_noalloc(lat: Lattice, values, out):
    """lattice_mvm whose work memory is the library's fixed per-device
    scratch array (no device allocation in the call); out must be given."""
    pv = _dev_f32(values, "values", lat.n)
    C = _cols(values)
    po = _dev_f32(out, "out", lat.n)
    if out.shape != values.shape:
        raise ValueError("out must have the shape of values")
    _check(_lib.load().lattice_mvm_noalloc(lat.handle, pv, C, po, _stream(values.device)))
    return out


NOALLOC_SCRATCH_BYTES = 64 << 20


def cg_solve(lat: Lattice, rhs, noise: float, tol: float, max_iter: int = 500, x=None):
    """Solve (outputscale*K + noise*I) x = rhs per column by CG (Section 2).
    Returns (x, iterations per column, recursive relative residual per column)."""
    import torch
    pb = _dev_f32(rhs, "rhs", lat.n)
    C = _cols(rhs)
    if x is None:
        x = torch.empty_like(rhs)
    px = _dev_f32(x, "x", lat.n)
    iters = np.zeros(C, dtype=np.int32)
    rel = np.zeros(C, dtype=np.float32)
    _check(_lib.load().cg_solve(lat.handle, pb, C, float(noise), float(tol), int(max_iter), px,
                                iters.ctypes.data_as(ctypes.c_void_p),
                                rel.ctypes.data_as(ctypes.c_void_p), _stream(rhs.device)))
    return x, iters, rel


def lattice_mvm_grad(lat: Lattice, X, V, G):
    """Gradient of sum(G * (outputscale K V)) with respect to X (n x d) and the
    log-lengthscales (d,), by k' filtering of [v, z v, g, z g] (Section 4.2).
    Returns (dX tensor, dlogell numpy array)."""
    import torch
    px = _dev_f32(X, "X", lat.n)
    pv = _dev_f32(V, "V", lat.n)
    pg = _dev_f32(G, "G", lat.n)
    C = _cols(V)
    if _cols(G) != C:
        raise ValueError("V and G must have the same columns")
    dX = torch.empty_like(X)
    dl = np.zeros(lat.d, dtype=np.float64)
    _check(_lib.load().lattice_mvm_grad(lat.handle, px, pv, pg, C, ctypes.c_void_p(dX.data_ptr()),
                                        dl.ctypes.data_as(ctypes.c_void_p), _stream(X.device)))
    return dX, dl


def _autograd_fn():
    import torch

    class LatticeKernelMVM(torch.autograd.Function):
        """out = outputscale * K_lat(X, l) V with the hand-written adjoint:
        dV = K G (the symmetric operator), dX and dlog l by k' filtering."""

        @staticmethod
        def forward(ctx, X, log_ell, V, opts):
            ell = log_ell.detach().double().exp().cpu().numpy()
            Xc = X.detach().contiguous()
            Vc = V.detach().contiguous()
            lat = lattice_build(Xc, ell, **opts)
            out = lattice_mvm(lat, Vc)
            ctx.lat = lat
            ctx.log_ell_meta = (log_ell.dtype, log_ell.device)
            ctx.save_for_backward(Xc, Vc)
            return out

        @staticmethod
        def backward(ctx, G):
            Xc, Vc = ctx.saved_tensors
            lat = ctx.lat
            Gc = G.detach().float().contiguous()
            dV = lattice_mvm(lat, Gc) if ctx.needs_input_grad[2] else None
            dX = dlog = None
            if ctx.needs_input_grad[0] or ctx.needs_input_grad[1]:
                gX, gl = lattice_mvm_grad(lat, Xc, Vc, Gc)
                dX = gX if ctx.needs_input_grad[0] else None
                if ctx.needs_input_grad[1]:
                    dtype, device = ctx.log_ell_meta
                    dlog = torch.from_numpy(gl).to(device=device, dtype=dtype)
            return dX, dlog, dV, None

    return LatticeKernelMVM


_FN = None


def lattice_kernel_mvm(X, log_lengthscales, V, **opts):
    """Differentiable lattice MVM for torch autograd (RBF kernel): gradients
    flow to X, the log-lengthscales and V."""
    global _FN
    if _FN is None:
        _FN = _autograd_fn()
    squeeze = V.dim() == 1
    Vm = V.unsqueeze(1) if squeeze else V
    out = _FN.apply(X, log_lengthscales, Vm, opts)
    return out.squeeze(1) if squeeze else out


def lattice_info(lat: Lattice) -> dict:
    n, d, m, b = ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int64(), ctypes.c_int64()
    _check(_lib.load().lattice_info(lat.handle, ctypes.byref(n), ctypes.byref(d), ctypes.byref(m),
                                    ctypes.byref(b)))
    return {"n": n.value, "d": d.value, "m": m.value, "device_bytes": b.value}


def lattice_export(lat: Lattice):
    """Host copies of keys (m x d), idx (n x d+1), w (n x d+1), nbr (m x d+1 x 2r)."""
    D, T = lat.d + 1, 2 * lat.order
    keys = np.zeros((lat.m, lat.d), dtype=np.int32)
    idx = np.zeros((lat.n, D), dtype=np.int32)
    w = np.zeros((lat.n, D), dtype=np.float32)
    nbr = np.zeros((lat.m, D, T), dtype=np.int32)
    P = lambda a: a.ctypes.data_as(ctypes.c_void_p)
    _check(_lib.load().lattice_export(lat.handle, P(keys), P(idx), P(w), P(nbr)))
    return keys, idx, w, nbr


def lattice_free(lat: Lattice):
    lat.free()


def cache_info() -> dict:
    """Bytes and blocks in the library's idle-block cache (current device)."""
    b, k = ctypes.c_int64(), ctypes.c_int32()
    _check(_lib.load().sgp_cache_info(ctypes.byref(b), ctypes.byref(k)))
    return {"bytes": int(b.value), "blocks": int(k.value)}


def debug_inject_oom(count: int) -> None:
    """Test hook: the next `count` pool allocations report out-of-memory."""
    _check(_lib.load().sgp_debug_inject_oom(int(count)))


def cg_graph_enable(on: bool) -> bool:
    """Turn graph replay of CG iterations on or off (process-wide); returns
    the previous setting. Results do not depend on it."""
    return bool(_lib.load().sgp_cg_graph_enable(1 if on else 0))


def cg_fuse_enable(on: bool) -> bool:
    """Switch the CG direction update between the splat (on, default) and a
    pass of its own; returns the previous setting. Results are identical."""
    return bool(_lib.load().sgp_cg_fuse_enable(1 if on else 0))


def blur_fuse_enable(on: bool) -> bool:
    """Turn fused two-step blur launches on or off (process-wide); returns
    the previous setting. Results do not depend on it."""
    return bool(_lib.load().sgp_blur_fuse_enable(1 if on else 0))


def blur_seq_bytes(nbytes: int) -> int:
    """Set the size of the four lattice value arrays above which the
    symmetric blur runs its two chains one after the other (process-wide;
    negative: never); returns the previous threshold. Results do not depend
    on it."""
    return int(_lib.load().sgp_blur_seq_bytes(int(nbytes)))


def autotune(lat: Lattice, C: int, fp64: bool = True, reps: int = 3) -> dict:
    """Time the MVM's launch-shape candidates on this lattice for C columns
    and keep the fastest for lattices of the same shape class; see
    sgp_autotune in include/simplexgp.h. Results do not depend on it."""
    lib = _lib.load()
    choice = (ctypes.c_int32 * 3)()
    ms = ctypes.c_float()
    _check(lib.sgp_autotune(lat.handle, int(C), 1 if fp64 else 0, int(reps), _stream(),
                            ctypes.cast(choice, ctypes.c_void_p), ctypes.cast(ctypes.pointer(ms), ctypes.c_void_p)))
    return {"chunk": choice[0], "splat_blocks_per_cu": choice[1], "slice_blocks_per_cu": choice[2],
            "ms_per_mvm": ms.value}


def autotune_build(X, lengthscales: Sequence[float], reps: int = 2, order: int = 1,
                   kernel: str = "rbf", blur: str = "symmetric") -> dict:
    """Time lattice builds of X for each hash-table shape (load factor and
    first-attempt reduction) and keep the fastest for builds of the same d
    and size class whose load_factor is 0 (the default); see
    sgp_autotune_build in include/simplexgp.h. Results do not depend on it."""
    lib = _lib.load()
    n, d = int(X.shape[0]), int(X.shape[1])
    px = _dev_f32(X, "X")
    ell = np.ascontiguousarray(np.asarray(lengthscales, dtype=np.float64).reshape(-1))
    if ell.shape[0] != d:
        raise ValueError("lengthscales must have d entries")
    opts = _lib.Opts()
    lib.sgp_opts_default(ctypes.byref(opts))
    opts.order = int(order)
    opts.kernel = _KERNEL[kernel]
    opts.blur = _BLUR[blur]
    lf, sh, ms = ctypes.c_float(), ctypes.c_int32(), ctypes.c_float()
    _check(lib.sgp_autotune_build(px, n, d, ell.ctypes.data_as(ctypes.c_void_p), ctypes.byref(opts),
                                  int(reps), _stream(X.device), ctypes.byref(lf), ctypes.byref(sh),
                                  ctypes.byref(ms)))
    return {"load_factor": lf.value, "shrink": int(sh.value), "ms_per_build": ms.value}


def autotune_reset() -> None:
    """Forget every autotuned choice (MVM launch shapes and build shapes)."""
    _check(_lib.load().sgp_autotune_reset())


_allocator_hooks = None  # the installed ctypes callbacks, kept alive while set


def set_allocator(alloc=None, free=None) -> None:
    """Take the library's device memory from alloc(nbytes, stream) -> device
    pointer (int; 0 on failure) and give it back with free(ptr, stream),
    stream being a hipStream_t as an int; both None restores the built-in
    pool (sgp_set_allocator). Raises SGPError while a lattice is alive. The
    hooks must not call into this module's functions."""
    global _allocator_hooks
    lib = _lib.load()
    if (alloc is None) != (free is None):
        raise ValueError("set_allocator: give both alloc and free, or neither")
    if alloc is None:
        _check(lib.sgp_set_allocator(None, None))
        _allocator_hooks = None
        return

    def _alloc(nbytes, stream):
        try:
            return int(alloc(int(nbytes), int(stream or 0))) or None
        except Exception:  # a failed allocation is reported by the library
            return None

    def _free(ptr, stream):
        free(int(ptr), int(stream or 0))

    hooks = (_lib.ALLOC_FN(_alloc), _lib.FREE_FN(_free))
    _check(lib.sgp_set_allocator(*(ctypes.cast(h, ctypes.c_void_p) for h in hooks)))
    _allocator_hooks = hooks


def use_torch_allocator() -> None:
    """Take the library's device memory from torch's caching allocator on
    the current device (it then shows in torch.cuda.memory_allocated)."""
    import torch

    dev = torch.cuda.current_device()
    set_allocator(lambda n, s: torch.cuda.caching_allocator_alloc(n, dev, s),
                  lambda p, s: torch.cuda.caching_allocator_delete(p))


class profile:
    """Context manager: per-kernel HIP-event timings of library launches.

    with profile() as prof: ...;  prof.results -> {kind: (launches, total_ms)}
    """

    def __enter__(self):
        lib = _lib.load()
        _check(lib.sgp_profile_reset())
        _check(lib.sgp_profile_enable(1))
        self.results = {}
        return self

    def __exit__(self, *exc):
        lib = _lib.load()
        _check(lib.sgp_profile_enable(0))
        self.results = read_profile()
        return False


def read_profile() -> dict:
    lib = _lib.load()
    out = {}
    for k in range(lib.sgp_profile_kinds()):
        launches, ms = ctypes.c_int64(), ctypes.c_double()
        _check(lib.sgp_profile_read(k, ctypes.byref(launches), ctypes.byref(ms)))
        out[lib.sgp_profile_name(k).decode()] = (int(launches.value), float(ms.value))
    return out
