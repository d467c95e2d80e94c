"""sts_gram_noalloc (the contraction of block Gram-Schmidt with its partial
products in the library's device-resident scratch array) against sts_gram,
which allocates its scratch per call: two calls in a row, the second on a
smaller input, through the C ABI."""
import ctypes as C
import math

import numpy as np
import pytest

from paper_1912_10082_amd import binding as b

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    return torch


def _dev(torch, a):
    # column-major float64 device copy
    return torch.from_numpy(np.asfortranarray(a)).cuda().t().contiguous().t()


def _ld(t):
    # leading dimension of a column-major matrix (a single column may report
    # any stride for its size-1 dimension)
    return t.stride(1) if t.shape[1] > 1 else max(t.shape[0], 1)


def _call(fn, torch, A, B, Cm):
    lib = b.load()
    rc = getattr(lib, fn)(A.shape[0], A.shape[1], B.shape[1], C.c_void_p(A.data_ptr()), _ld(A),
                          C.c_void_p(B.data_ptr()), _ld(B), C.c_void_p(Cm.data_ptr()), _ld(Cm),
                          C.c_void_p(torch.cuda.current_stream().cuda_stream))
    return rc


@pytest.mark.parametrize("first,second", [((200003, 300, 8), (1000, 37, 5)),
                                          ((4099, 512, 16), (17, 3, 1))])
def test_noalloc_matches_allocating_entry_point(first, second):
    torch = _torch()
    rng = np.random.default_rng(first[0] + second[0])
    cases = []
    for rows, m, n in (first, second):
        A, B = rng.normal(size=(rows, m)), rng.normal(size=(rows, n))
        dA, dB = _dev(torch, A), _dev(torch, B)
        out = b.dev_empty(m, n)
        cases.append((A, B, dA, dB, out))
    torch.cuda.synchronize()
    before = torch.cuda.memory_allocated()
    for A, B, dA, dB, out in cases:          # two calls in a row, the second smaller
        assert _call("sts_gram_noalloc", torch, dA, dB, out) == b.STS_OK, \
            b.load().sts_last_error().decode()
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() == before
    for A, B, dA, dB, out in cases:
        ref = b.dev_empty(A.shape[1], B.shape[1])
        assert _call("sts_gram", torch, dA, dB, ref) == b.STS_OK
        torch.cuda.synchronize()
        got, want = out.cpu().numpy(), ref.cpu().numpy()
        # same kernels and work split: the same bits
        assert np.array_equal(got, want)
        np.testing.assert_allclose(got, A.T @ B, rtol=1e-12, atol=1e-12 * math.sqrt(A.shape[0]))


def test_noalloc_empty_rows_and_limits():
    torch = _torch()
    lib = b.load()
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    dA, dB = b.dev_zeros(1, 40), b.dev_zeros(1, 3)
    out = b.dev_empty(40, 3)
    out.fill_(7.0)
    # no rows: C = 0
    rc = lib.sts_gram_noalloc(0, 40, 3, C.c_void_p(dA.data_ptr()), 1, C.c_void_p(dB.data_ptr()), 1,
                              C.c_void_p(out.data_ptr()), 40, stream)
    assert rc == b.STS_OK
    torch.cuda.synchronize()
    assert float(out.abs().max()) == 0.0
    # beyond the scratch: refused on the host, nothing launched
    big, w, c = b.dev_zeros(64, 513), b.dev_zeros(64, 2), b.dev_zeros(513, 2)
    rc = lib.sts_gram_noalloc(64, 513, 2, C.c_void_p(big.data_ptr()), 64, C.c_void_p(w.data_ptr()),
                              64, C.c_void_p(c.data_ptr()), 513, stream)
    assert rc == b.STS_E_INVALID
    assert "513" in lib.sts_last_error().decode()
