"""drMlpSoftmaxXentNoAlloc (the allocation-free per-view softmax cross-entropy)
against drMlpSoftmaxXent, through the C ABI: two calls in a row, the second
on fewer views and rows, with and without a target, plus the size limit."""
import ctypes

import numpy as np
import pytest
import torch

from paper_1904_12228_amd import _lib

pytestmark = pytest.mark.gpu


def _p(t):
    return ctypes.c_void_p(0 if t is None else t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _case(rng, sizes, dev):
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int32)
    n = int(off[-1])
    z = torch.as_tensor((rng.normal(size=n) * 3).astype(np.float32), device=dev)
    t = np.abs(rng.normal(size=n)).astype(np.float32)
    if len(sizes) > 2:
        t[off[1]:off[2]] = 0.0      # a view whose target sums to zero
    return z, torch.as_tensor(t, device=dev), torch.as_tensor(off, device=dev)


def _run(z, t, off, no_alloc):
    lib = _lib.load()
    nv = int(off.numel()) - 1
    prob = torch.full_like(z, float("nan"))
    dz = torch.full_like(z, float("nan")) if t is not None else None
    vl = torch.full((nv,), float("nan"), device=z.device) if t is not None else None
    if no_alloc:
        st = lib.drMlpSoftmaxXentNoAlloc(_p(z), _p(t), _p(off), nv, _p(prob), _p(dz), _p(vl), _stream())
    else:
        scratch = torch.empty(max(nv, 1), dtype=torch.float32, device=z.device)
        st = lib.drMlpSoftmaxXent(_p(z), _p(t), _p(off), nv, _p(prob), _p(dz), _p(vl), _p(scratch), _stream())
    _lib.check(st, "softmax cross-entropy")
    torch.cuda.synchronize()
    return prob, dz, vl


def test_no_alloc_softmax_matches_allocating_entry_point():
    dev = "cuda:0"
    rng = np.random.default_rng(11)
    big = [300, 57, 0, 1, 1000, 250, 33] * 40          # 280 views, uneven, some empty
    small = [5, 200, 17]                                # fewer views and rows
    for sizes in (big, small):
        z, t, off = _case(rng, sizes, dev)
        for target in (t, None):
            ref = _run(z, target, off, no_alloc=False)
            got = _run(z, target, off, no_alloc=True)
            for a, b in zip(ref, got):
                if a is None:
                    assert b is None
                    continue
                # same kernels on the same inputs: identical results
                assert torch.equal(a, b), (a - b).abs().max()
                assert torch.isfinite(b).all()


def test_no_alloc_softmax_rejects_too_many_views():
    lib = _lib.load()
    nv = 65536 + 1
    off = torch.zeros(nv + 1, dtype=torch.int32, device="cuda:0")
    z = torch.zeros(1, device="cuda:0")
    st = lib.drMlpSoftmaxXentNoAlloc(_p(z), None, _p(off), nv, _p(z), None, None, _stream())
    assert st == 1          # DR_ERROR_INVALID_VALUE, nothing queued
