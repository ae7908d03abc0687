"""tagi_direct_noalloc (the allocation-free direct sum, for callers that cannot
allocate) through the C ABI against tagi_direct on the same inputs: two calls in
a row, the second with a smaller input, both equal to tagi_direct's results
(same kernels, chunking and summation order); sizes beyond its scratch are
rejected before any work."""
import ctypes

import numpy as np
import pytest
import torch

from workloads.configs import uniform_cube
from workloads.rng import SplitMix64

pytestmark = pytest.mark.gpu

KERNELS = {"yukawa_ss": 0, "coulomb_ss": 1, "yukawa": 2, "coulomb": 3}


def _lib():
    from paper_2003_01833_amd import binding
    lib = binding.load_library()
    vp, i64, i32, dbl = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_double
    lib.tagi_direct_noalloc.argtypes = [vp, vp, vp, vp, vp, i64, vp, vp, vp, vp, i64, i32, dbl,
                                        dbl, vp, vp]
    lib.tagi_direct_noalloc.restype = ctypes.c_int
    return lib


def _call(fn, src, tgt, kernel, kappa, out):
    p = lambda t: ctypes.c_void_p(t.data_ptr())  # noqa: E731
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    return fn(*(p(a) for a in src), src[0].numel(), *(p(a) for a in tgt), tgt[0].numel(),
              KERNELS[kernel], float(kappa), 1.0, p(out), stream)


def _case(ns, nt, seed):
    x, y, z, f, w = uniform_cube(ns, seed=seed)
    g = SplitMix64(seed + 1)
    tx, ty, tz, tf = (g.uniform(nt, -1.0, 1.0) for _ in range(4))
    tx[:7], ty[:7], tz[:7] = x[:7], y[:7], z[:7]  # targets on sources
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()  # noqa: E731
    return [d(a) for a in (x, y, z, f, w)], [d(a) for a in (tx, ty, tz, tf)]


@pytest.mark.parametrize("kernel", ["yukawa_ss", "coulomb_ss"])
def test_noalloc_direct_matches_tagi_direct_twice(kernel):
    lib = _lib()
    for ns, nt, seed in ((40000, 9000, 3), (5000, 777, 4)):
        src, tgt = _case(ns, nt, seed)
        ref = torch.empty(nt, dtype=torch.float64, device="cuda")
        got = torch.full((nt,), np.nan, dtype=torch.float64, device="cuda")
        assert _call(lib.tagi_direct, src, tgt, kernel, 1.3, ref) == 0
        assert _call(lib.tagi_direct_noalloc, src, tgt, kernel, 1.3, got) == 0, \
            lib.tagi_last_error()
        torch.cuda.synchronize()
        assert torch.equal(got, ref), (ns, nt, float((got - ref).abs().max()))


def test_noalloc_direct_rejects_sizes_beyond_its_scratch():
    lib = _lib()
    src, tgt = _case(64, 64, 5)
    # only the sizes are read before the rejection: 8 ns bytes of charges alone
    # exceed the 32 MiB scratch
    p = lambda t: ctypes.c_void_p(t.data_ptr())  # noqa: E731
    out = torch.empty(64, dtype=torch.float64, device="cuda")
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = lib.tagi_direct_noalloc(*(p(a) for a in src), 5_000_000, *(p(a) for a in tgt), 64,
                                 KERNELS["yukawa"], 1.0, 1.0, p(out), stream)
    assert rc == -1
    assert b"scratch" in lib.tagi_last_error()
