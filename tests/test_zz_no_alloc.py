"""lattice_mvm_noalloc: the MVM with its work memory in the library's fixed
per-device scratch array. Its results equal lattice_mvm's bit for bit (same
kernels, same order of every sum), on two calls in a row, the second with a
smaller lattice and fewer columns; it makes no device allocation (checked
with counting allocator hooks); sizes beyond the array are refused."""
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


CASES = [  # (seed, n, d, C, kind): the second is smaller in n, m and C
    (91, 60000, 8, 7, "mixture"),
    (92, 3000, 3, 2, "normal"),
]


def test_noalloc_matches_lattice_mvm(sgp, orc):
    import torch
    lats = []
    for seed, n, d, C, kind in CASES:
        print(f"noalloc seed={seed} n={n} d={d} C={C}", flush=True)
        w = workloads.small_case(seed, n, d, channels=C, kind=kind)
        lat = sgp.lattice_build(_cuda(w.X), w.lengthscales)
        V = _cuda(w.values)
        ref = sgp.lattice_mvm(lat, V).cpu().numpy()
        out = torch.full_like(V, float("nan"))
        sgp.lattice_mvm_noalloc(lat, V, out)
        got = out.cpu().numpy()
        np.testing.assert_array_equal(got, ref)
        # and against the oracle, to the MVM parity bar
        olat = orc.Lattice(w.X, w.lengthscales)
        o = olat.mvm(w.values.astype(np.float64))
        scale = olat.mvm(np.abs(w.values).astype(np.float64))
        assert np.all(np.abs(got - o) <= 1e-5 * scale + 1e-30)
        lats.append((lat, V, ref))
    # repeated calls alternate between the two lattices: the shared array
    # keeps the previous call's contents, which must not leak into a result
    for lat, V, ref in lats[::-1] + lats:
        out = torch.empty_like(V)
        sgp.lattice_mvm_noalloc(lat, V, out)
        np.testing.assert_array_equal(out.cpu().numpy(), ref)
    for lat, _, _ in lats:
        lat.free()


def test_noalloc_makes_no_device_allocation(sgp):
    import torch
    print("noalloc with counting allocator hooks", flush=True)
    gc.collect()
    dev = torch.cuda.current_device()
    counts = {"alloc": 0, "free": 0}
    live = {}

    def alloc(nbytes, stream):
        p = torch.cuda.caching_allocator_alloc(nbytes, dev, stream)
        live[p] = nbytes
        counts["alloc"] += 1
        return p

    def free(ptr, stream):
        counts["free"] += 1
        live.pop(ptr, None)
        torch.cuda.caching_allocator_delete(ptr)

    w = workloads.small_case(93, 20000, 5, channels=4, kind="mixture")
    sgp.set_allocator(alloc, free)
    try:
        lat = sgp.lattice_build(_cuda(w.X), w.lengthscales)
        V = _cuda(w.values)
        out = torch.empty_like(V)
        torch.cuda.synchronize()
        before = dict(counts)
        for _ in range(3):
            sgp.lattice_mvm_noalloc(lat, V, out)
        torch.cuda.synchronize()
        assert counts == before, (before, counts)
        # the allocating entry point does take its work buffer from the hooks
        ref = sgp.lattice_mvm(lat, V).cpu().numpy()
        assert counts["alloc"] > before["alloc"]
        np.testing.assert_array_equal(out.cpu().numpy(), ref)
        lat.free()
        del lat
        gc.collect()
        torch.cuda.synchronize()
    finally:
        sgp.set_allocator(None, None)
    assert not live


def test_noalloc_refuses_sizes_beyond_the_array(sgp):
    import torch
    print("noalloc size limit", flush=True)
    w = workloads.small_case(94, 200000, 11, channels=1, kind="mixture")
    lat = sgp.lattice_build(_cuda(w.X), w.lengthscales)
    # work memory 4 (4m + runs) C bytes, m = 51,971 here: at C = 96 even the
    # lattice values alone (76 MiB) exceed the 64 MiB array
    V1 = _cuda(w.values)
    out1 = torch.empty_like(V1)
    sgp.lattice_mvm_noalloc(lat, V1, out1)
    np.testing.assert_array_equal(out1.cpu().numpy(), sgp.lattice_mvm(lat, V1).cpu().numpy())
    C = 96
    V = _cuda(np.random.default_rng(0).standard_normal((w.n, C)))
    out = torch.empty_like(V)
    with pytest.raises(sgp.SGPError) as ei:
        sgp.lattice_mvm_noalloc(lat, V, out)
    assert ei.value.code == -1 and "no-allocation" in str(ei.value)
    lat.free()
