"""The allocation-free entry point (cholmod_update_noalloc): workspace in the
library's fixed device array, called through the C ABI.  Its result must
equal cholmod_update_async's (same kernels, caller workspace) bit for bit,
on two calls in a row, the second on a smaller problem (the array keeps the
first call's contents, which the second must not depend on)."""
import ctypes

import pytest
import torch

from gpu_util import inputs, print_case

pytestmark = pytest.mark.gpu


def _lib():
    from paper_1011_1173_amd import _native
    return _native, _native.load()


def _call_async(lib, L, V, sigma, stream):
    n, k = V.shape
    ws = torch.empty(lib.cholmod_workspace_bytes(n, k, 0), dtype=torch.uint8, device="cuda")
    info = torch.empty(1, dtype=torch.int64, device="cuda")
    st = lib.cholmod_update_async(ctypes.c_void_p(L.data_ptr()), ctypes.c_void_p(V.data_ptr()),
                                  n, k, L.stride(0), sigma, ctypes.c_void_p(ws.data_ptr()),
                                  ws.numel(), ctypes.c_void_p(info.data_ptr()),
                                  ctypes.c_void_p(stream.cuda_stream))
    assert st == 0
    stream.synchronize()
    return int(info.item())


def _call_noalloc(lib, L, V, sigma, stream):
    n, k = V.shape
    info = torch.empty(1, dtype=torch.int64, device="cuda")
    st = lib.cholmod_update_noalloc(ctypes.c_void_p(L.data_ptr()),
                                    ctypes.c_void_p(V.data_ptr()), n, k, L.stride(0), sigma,
                                    ctypes.c_void_p(info.data_ptr()),
                                    ctypes.c_void_p(stream.cuda_stream))
    assert st == 0
    stream.synchronize()
    return int(info.item())


def test_noalloc_equals_async_twice_second_smaller():
    nat, lib = _lib()
    stream = torch.cuda.Stream()
    # second call smaller than the first, and a downdate after an update
    for n, k, ldl, sigma, seed in ((3000, 16, 3001, 1, 81), (700, 5, 700, -1, 82)):
        print_case("noalloc", n=n, k=k, ldl=ldl, sigma=sigma)
        L = inputs.spd_factor(n, seed, device="cuda", ldl=ldl)
        V = inputs.update_vectors(n, k, seed, device="cuda")
        if sigma < 0:  # a factor that contains V V^T
            assert _call_async(lib, L, V, +1, stream) == nat.INFO_NONE
        torch.cuda.synchronize()
        a, b = L.clone(), L.clone()
        torch.cuda.synchronize()
        ia = _call_async(lib, a, V, sigma, stream)
        ib = _call_noalloc(lib, b, V, sigma, stream)
        assert ia == nat.INFO_NONE and ib == nat.INFO_NONE
        assert torch.equal(a, b), "max |diff| = %g" % float((a - b).abs().max())


def test_noalloc_reports_failures_like_async():
    nat, lib = _lib()
    stream = torch.cuda.Stream()
    n, r = 300, 130
    print_case("noalloc-fail", n=n, row=r)
    L = inputs.spd_factor(n, 83, device="cuda")
    V = torch.zeros(n, 2, dtype=torch.float64, device="cuda")
    V[:, 0] = 2.0 * L[r, :n]
    torch.cuda.synchronize()
    ia = _call_async(lib, L.clone(), V, -1, stream)
    ib = _call_noalloc(lib, L.clone(), V, -1, stream)
    assert ia == ib
    assert nat.decode_info(ib, 2) == (nat.ERR_NOT_PD, r, 0)


def test_noalloc_rejects_sizes_beyond_its_array():
    nat, lib = _lib()
    cap = lib.cholmod_noalloc_max_bytes()
    n, k = 60000, 16
    assert lib.cholmod_workspace_bytes(n, k, 0) > cap
    info = torch.empty(1, dtype=torch.int64, device="cuda")
    L = torch.empty(1, dtype=torch.float64, device="cuda")
    st = lib.cholmod_update_noalloc(ctypes.c_void_p(L.data_ptr()), ctypes.c_void_p(L.data_ptr()),
                                    n, k, n, 1, ctypes.c_void_p(info.data_ptr()), None)
    assert st == nat.ERR_ARG
