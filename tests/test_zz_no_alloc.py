"""The allocation-free entry point rsvd_truncate_noalloc (through the C ABI)
against rsvd_truncate on the same inputs: the same kernels run in the same
order on the library's static scratch array instead of a plan workspace, so
every output must be bit-identical.  Two calls in a row on one GPU, the
second smaller (the scratch keeps the first call's contents), then a third
call larger again, and a problem too large for the scratch."""
import ctypes

import numpy as np
import pytest
import torch

import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    import paper_1710_01463_amd as P
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return P


def same(a, b):
    torch.cuda.synchronize()
    return torch.equal(a, b)


@pytest.mark.parametrize("dtype,prec", [(torch.float64, "f64"), (torch.float32, "f32"), (torch.float32, "bf16")])
def test_noalloc_matches_rsvd_truncate(lib, dtype, prec):
    cases = [(300, 220, 40, 12, 2, 0.0, 31), (90, 130, 20, 8, 1, 1e-6, 32), (520, 140, 30, 10, 3, 0.0, 33)]
    for m, n, k, p, q, delta, seed in cases:
        s = wl.spectrum_exp(min(m, n), 0.05)
        A = torch.from_numpy(wl.make_matrix(m, n, s, seed=seed + 500)).to(dtype).cuda()
        ref = lib.rsvd_truncate(A, k, p, q, seed, delta, prec)
        got = lib.rsvd_truncate_noalloc(A, k, p, q, seed, delta, prec)
        torch.cuda.synchronize()
        assert int(got[5].item()) == 0, (m, n)
        for r, g, name in zip(ref, got[:5], ("U", "S", "VT", "w", "k_kept")):
            assert same(r, g), (m, n, prec, name)


def test_noalloc_through_graph_capture(lib):
    """Captured once (the wrapper allocates nothing either), replayed with
    other work in between; every replay equals the eager result."""
    m, n, k = 200, 160, 24
    A = torch.from_numpy(wl.make_matrix(m, n, wl.spectrum_power(160, 1.2), seed=41)).cuda()
    ref = lib.rsvd_truncate(A, k, 10, 2, 7)
    out = (torch.empty((m, k), dtype=A.dtype, device="cuda"), torch.empty(k, dtype=A.dtype, device="cuda"),
           torch.empty((k, n), dtype=A.dtype, device="cuda"), torch.empty(1, dtype=torch.float64, device="cuda"),
           torch.empty(1, dtype=torch.int64, device="cuda"), torch.empty(1, dtype=torch.int32, device="cuda"))
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        lib.rsvd_truncate_noalloc(A, k, 10, 2, 7, out=out)  # warm-up outside capture
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        lib.rsvd_truncate_noalloc(A, k, 10, 2, 7, out=out)
    B = torch.from_numpy(wl.make_matrix(90, 70, wl.spectrum_exp(70, 0.1), seed=42)).cuda()
    for rep in range(3):
        for t in out:
            t.zero_()
        g.replay()
        torch.cuda.synchronize()
        assert int(out[5].item()) == 0
        for r, o in zip(ref, out[:5]):
            assert same(r, o), rep
        # another call on the same scratch between replays
        other = lib.rsvd_truncate_noalloc(B, 10, 5, 1, 9)
        torch.cuda.synchronize()
        assert int(other[5].item()) == 0


def test_noalloc_rejects_a_problem_beyond_the_scratch(lib):
    from paper_1710_01463_amd._lib import RSVD_ERR_INVALID, lib as clib
    m = n = 4096
    A = torch.zeros((1, 1), dtype=torch.float64, device="cuda")  # never read: the size check comes first
    U = torch.zeros(1, dtype=torch.float64, device="cuda")
    st = clib().rsvd_truncate_noalloc(A.data_ptr(), 0, m, n, n, 1000, 24, 2, ctypes.c_uint64(1), 0.0, 0,
                                      U.data_ptr(), 1000, U.data_ptr(), U.data_ptr(), n, U.data_ptr(),
                                      U.data_ptr(), U.data_ptr(), None)
    assert st == RSVD_ERR_INVALID
    assert b"scratch" in clib().rsvd_last_error()
    torch.cuda.synchronize()
