"""The allocation-free top-k entry point (tqc_topk_noalloc) against tqc_topk
through the C-ABI: equal indices and values bit for bit, on two calls in a
row, the second with a smaller input, and the stated size limit enforced
before any device work."""
import ctypes

import numpy as np
import pytest
import torch

import paper_2502_03445_amd as tqc

pytestmark = pytest.mark.gpu


def _call(name, probs, k, stream):
    L = tqc.lib()
    f = getattr(L, name)
    f.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_uint64, ctypes.c_int32, ctypes.c_void_p,
                  ctypes.c_void_p, ctypes.c_void_p]
    f.restype = ctypes.c_int
    idx = torch.empty(k, dtype=torch.int64, device="cuda")
    val = torch.empty(k, dtype=torch.float64, device="cuda")
    dt = 1 if probs.dtype == torch.float32 else 0
    st = f(ctypes.c_void_p(probs.data_ptr()), dt, probs.numel(), k, ctypes.c_void_p(idx.data_ptr()),
           ctypes.c_void_p(val.data_ptr()), ctypes.c_void_p(stream.cuda_stream))
    return st, idx, val


def test_noalloc_topk_equals_topk_twice_second_smaller():
    s = torch.cuda.current_stream()
    g = torch.Generator(device="cuda").manual_seed(5)
    big = torch.rand(1 << 26, device="cuda", generator=g)
    big[1 << 25] = 2.0
    big[17] = 2.0                      # a tie: smaller index first
    small = torch.rand(300001, device="cuda", dtype=torch.float64, generator=g) ** 2
    small[4] = small[9] = small[123] = 0.5
    cases = [(big, 4096), (small, 777)]
    got = []
    for probs, k in cases:             # two calls in a row, no synchronisation between
        st, i, v = _call("tqc_topk_noalloc", probs, k, s)
        assert st == 0, tqc.lib().tqc_last_error()
        got.append((i, v))
    torch.cuda.synchronize()
    for (probs, k), (i, v) in zip(cases, got):
        st, ri, rv = _call("tqc_topk", probs, k, s)
        assert st == 0
        torch.cuda.synchronize()
        assert torch.equal(i, ri) and torch.equal(v, rv)
        # against a host sort of the same vector: value desc, index asc
        h = probs.double().cpu().numpy()
        order = np.lexsort((np.arange(h.size), -h))[:k]
        assert np.array_equal(i.cpu().numpy(), order)


def test_noalloc_topk_rejects_vectors_beyond_its_scratch():
    s = torch.cuda.current_stream()
    probs = torch.zeros(16, device="cuda")
    L = tqc.lib()
    f = L.tqc_topk_noalloc
    f.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_uint64, ctypes.c_int32, ctypes.c_void_p,
                  ctypes.c_void_p, ctypes.c_void_p]
    idx = torch.empty(8, dtype=torch.int64, device="cuda")
    val = torch.empty(8, dtype=torch.float64, device="cuda")
    # length 2^34 claimed for a 16-entry buffer: the host check rejects it
    # before any kernel could read the buffer
    st = f(ctypes.c_void_p(probs.data_ptr()), 1, 1 << 34, 8, ctypes.c_void_p(idx.data_ptr()),
           ctypes.c_void_p(val.data_ptr()), ctypes.c_void_p(s.cuda_stream))
    assert st == 1
    assert b"scratch" in L.tqc_last_error()
