"""The caller's allocator (sgp_set_allocator): a lattice's buffers, the
build's temporaries and the gradient's work buffers come from it and go
back to it, and results equal the built-in pool's bit for bit."""
import gc

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


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


def _run(sgp, w, G):
    lat = sgp.lattice_build(_cuda(w.X), w.lengthscales)
    V = _cuda(w.values)
    y = sgp.lattice_mvm(lat, V).cpu().numpy()
    x, _, _ = sgp.cg_solve(lat, V, 0.1, 0.0, max_iter=12)
    dX, dl = sgp.lattice_mvm_grad(lat, _cuda(w.X), V, _cuda(G))
    return lat, [y, x.cpu().numpy(), dX.cpu().numpy(), np.asarray(dl)]


def test_user_allocator_matches_pool(sgp):
    import torch
    print("allocator: torch caching allocator hooks, n=6000 d=5 C=4", flush=True)
    w = workloads.small_case(77, 6000, 5, channels=4, kind="mixture")
    G = np.random.default_rng(7).standard_normal(w.values.shape).astype(np.float32)
    lat, ref = _run(sgp, w, G)
    lat.free()
    del lat
    gc.collect()

    dev = torch.cuda.current_device()
    live, counts = {}, {"alloc": 0, "free": 0, "unknown": 0}

    def alloc(nbytes, stream):
        p = torch.cuda.caching_allocator_alloc(nbytes, dev, stream)
        live[p] = nbytes
        counts["alloc"] += 1
        return p

    def free(ptr, stream):
        counts["free"] += 1
        if live.pop(ptr, None) is None:
            counts["unknown"] += 1
        torch.cuda.caching_allocator_delete(ptr)

    sgp.set_allocator(alloc, free)
    try:
        lat, got = _run(sgp, w, G)
        assert counts["alloc"] > 0 and live
        with pytest.raises(sgp.SGPError):
            sgp.set_allocator(None, None)  # the lattice still holds blocks
        lat.free()
        del lat
        torch.cuda.synchronize()
    finally:
        gc.collect()
        sgp.set_allocator(None, None)
    assert not live and counts["unknown"] == 0 and counts["alloc"] == counts["free"]
    for a, b in zip(ref, got):
        np.testing.assert_array_equal(a, b)

    # the built-in pool serves again
    lat, again = _run(sgp, w, G)
    lat.free()
    for a, b in zip(ref, again):
        np.testing.assert_array_equal(a, b)


def test_use_torch_allocator_shows_in_torch(sgp):
    import torch
    print("allocator: use_torch_allocator, n=20000 d=6", flush=True)
    w = workloads.small_case(78, 20000, 6, channels=2, kind="mixture")
    X, V = _cuda(w.X), _cuda(w.values)
    gc.collect()
    torch.cuda.synchronize()
    base = torch.cuda.memory_allocated()
    sgp.use_torch_allocator()
    try:
        lat = sgp.lattice_build(X, w.lengthscales)
        sgp.lattice_mvm(lat, V)
        torch.cuda.synchronize()
        held = sgp.lattice_info(lat)["device_bytes"]
        assert torch.cuda.memory_allocated() - base >= held > 0
        lat.free()
        del lat
        torch.cuda.synchronize()
    finally:
        gc.collect()
        sgp.set_allocator(None, None)
    assert torch.cuda.memory_allocated() == base


def test_out_of_memory_flushes_idle_cache_and_retries(sgp):
    """An allocation from the built-in pool that runs out of memory returns
    the idle-block cache to the pool and tries once more: one injected
    failure is absorbed (results bitwise as without it), two surface as
    SGP_ENOMEM, and the library stays usable."""
    print("allocator: out-of-memory retry", flush=True)
    w = workloads.small_case(78, 5000, 4, channels=3, kind="mixture")
    G = np.random.default_rng(8).standard_normal(w.values.shape).astype(np.float32)
    lat, ref = _run(sgp, w, G)
    lat.free()
    # the freed lattice's blocks are idle in the cache now
    assert sgp.cache_info()["blocks"] > 0
    # a build of another size misses the cache, hits the injected failure,
    # flushes the cache and succeeds on the retry
    other = workloads.small_case(79, 40000, 6, channels=1, kind="mixture")
    sgp.debug_inject_oom(1)
    try:
        lat2 = sgp.lattice_build(_cuda(other.X), other.lengthscales)
    finally:
        sgp.debug_inject_oom(0)
    assert lat2.m > 0
    lat2.free()
    # both attempts fail: the error is reported, nothing leaks (a larger
    # build than any before, so that its blocks cannot come from the cache)
    lat, _ = _run(sgp, w, G)
    lat.free()
    big = workloads.small_case(80, 150000, 7, channels=1, kind="mixture")
    sgp.debug_inject_oom(2)
    try:
        with pytest.raises(sgp.SGPError) as ei:
            sgp.lattice_build(_cuda(big.X), big.lengthscales)
        assert ei.value.code == -2
    finally:
        sgp.debug_inject_oom(0)
    lat, got = _run(sgp, w, G)
    for a, b in zip(ref, got):
        np.testing.assert_array_equal(a, b)
    lat.free()
