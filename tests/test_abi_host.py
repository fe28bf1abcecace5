"""Host-side checks of the C-ABI library (no GPU needed).

The library must load, export every function include/simplexgp.h declares,
and reject bad arguments on the host before touching the device.
"""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "simplexgp.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\**\s*([a-z_][a-z0-9_]*)\s*\(",
                       text, flags=re.M)
    return sorted(set(n for n in names if n not in ("defined",)))


@pytest.fixture(scope="module")
def lib():
    from paper_2106_06695_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("libsimplexgp.so is not built; run __graft_entry__.build()")
    return _lib.load()


def test_header_declares_the_boundary():
    names = _declared_functions()
    for required in ("lattice_build", "lattice_mvm", "cg_solve", "lattice_info", "lattice_export",
                     "lattice_free", "sgp_last_error", "sgp_opts_default"):
        assert required in names


def test_every_declared_symbol_is_exported(lib):
    from paper_2106_06695_amd import _lib
    names = _declared_functions()
    assert len(names) >= 8
    for name in names:
        assert hasattr(lib, name), name
        assert name in _lib.SIGNATURES, f"binding lacks a signature for {name}"


def test_opts_defaults(lib):
    from paper_2106_06695_amd import _lib
    o = _lib.Opts()
    lib.sgp_opts_default(ctypes.byref(o))
    assert (o.order, o.kernel, o.blur) == (1, 0, 0)
    assert o.outputscale == 1.0 and o.load_factor == 0.0  # automatic table shape


FAKE = ctypes.c_void_p(0x1000)  # never dereferenced: validation fails first


def _build(lib, X, n, d, ell, opts=None):
    h = ctypes.c_void_p()
    rc = lib.lattice_build(X, n, d, ell, opts, None, ctypes.byref(h))
    return rc, h


def test_build_argument_errors(lib):
    from paper_2106_06695_amd import _lib
    ell = np.ones(4)
    pe = ell.ctypes.data_as(ctypes.c_void_p)
    assert _build(lib, None, 10, 4, pe)[0] == -1
    assert b"non-NULL" in lib.sgp_last_error()
    assert _build(lib, FAKE, 0, 4, pe)[0] == -1
    assert _build(lib, FAKE, 10, 0, pe)[0] == -1
    assert _build(lib, FAKE, 10, 33, pe)[0] == -1
    assert _build(lib, FAKE, 1 << 29, 4, pe)[0] == -1  # n(d+1) > 2^30
    for bad in (0.0, -1.0, np.nan, np.inf):
        e2 = np.ones(4)
        e2[2] = bad
        rc, _ = _build(lib, FAKE, 10, 4, e2.ctypes.data_as(ctypes.c_void_p))
        assert rc == -1 and b"lengthscale 2" in lib.sgp_last_error()
    o = _lib.Opts()
    for field, value in (("order", 0), ("order", 9), ("kernel", 5), ("blur", 3),
                         ("load_factor", -0.1), ("load_factor", 0.95), ("outputscale", float("inf"))):
        lib.sgp_opts_default(ctypes.byref(o))
        setattr(o, field, value)
        rc, _ = _build(lib, FAKE, 10, 4, pe, ctypes.byref(o))
        assert rc == -1, (field, value)
    rc = lib.lattice_build(FAKE, 10, 4, pe, None, None, None)
    assert rc == -1


def test_mvm_and_cg_argument_errors(lib):
    assert lib.lattice_mvm(None, FAKE, 1, FAKE, None) == -1
    assert lib.cg_solve(None, FAKE, 1, 0.1, 1e-3, 10, FAKE, None, None, None) == -1
    assert lib.lattice_info(None, None, None, None, None) == -1
    assert lib.lattice_export(None, None, None, None, None) == -1
    lib.lattice_free(None)


def test_profiler_kinds(lib):
    kinds = lib.sgp_profile_kinds()
    names = [lib.sgp_profile_name(k).decode() for k in range(kinds)]
    for needed in ("splat", "blur", "slice", "simplex_insert", "cg_alpha"):
        assert needed in names
    assert lib.sgp_profile_read(kinds, None, None) == -1
    launches, ms = ctypes.c_int64(), ctypes.c_double()
    assert lib.sgp_profile_reset() == 0
    assert lib.sgp_profile_read(0, ctypes.byref(launches), ctypes.byref(ms)) == 0
    assert launches.value == 0 and ms.value == 0.0


def test_python_binding_rejects_cpu_tensors():
    import torch
    import paper_2106_06695_amd as sgp
    with pytest.raises(TypeError):
        sgp.lattice_build(torch.zeros(4, 2), [1.0, 1.0])


def test_ws3p_scale_matches_paper_sparsity():
    """The stored lengthscale factor of ws3p (written from the oracle's lattice
    by workloads/paper_sparsity.py) gives the paper's Houseelectric ratio
    m / (n (d+1)) = 1,000,190 / (2,049,280 * 12) to within 0.5%."""
    import json
    import os
    import workloads
    path = os.path.join(os.path.dirname(workloads.__file__), "ws3p_scale.json")
    rec = json.load(open(path))
    target = 1_000_190 / (2_049_280 * 12)
    assert abs(rec["target"] - target) < 1e-12
    assert abs(rec["m_over_L"] - target) <= 0.005 * target
    assert 0.5 < rec["scale"] < 1.0 and workloads.ws3p_scale() == rec["scale"]


def test_set_allocator_needs_both_hooks(lib):
    from paper_2106_06695_amd import _lib
    hook = _lib.ALLOC_FN(lambda n, s: None)
    assert lib.sgp_set_allocator(ctypes.cast(hook, ctypes.c_void_p), None) == -1  # SGP_EINVAL
    assert b"both" in lib.sgp_last_error()
    assert lib.sgp_set_allocator(None, None) == 0  # the built-in pool, nothing held
