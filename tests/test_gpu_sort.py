"""The setup's own stable radix sort and exclusive scan against numpy's
stable argsort and cumulative sum (integer work: bit for bit).  Sizes span
one tile, several tiles and a ragged tail, duplicate keys (stability), and
the scan's multi-level recursion."""
import ctypes as C

import numpy as np
import pytest
import torch

from paper_1108_1310_amd import lamg

pytestmark = pytest.mark.gpu


def _lib():
    L = lamg.lib()
    vp, i64, i32 = C.c_void_p, C.c_int64, C.c_int32
    for name, args in (("lamg_t_sort_pairs64", [i64, vp, vp, vp, vp, i32]),
                       ("lamg_t_sort_pairs32", [i64, vp, vp, vp, vp, i32]),
                       ("lamg_t_sort_f64", [i64, vp, vp]),
                       ("lamg_t_excl_scan", [i64, vp, vp])):
        f = getattr(L, name)
        f.restype = C.c_int
        f.argtypes = args
    return L


def _p(t):
    return C.c_void_p(t.data_ptr())


@pytest.mark.parametrize("n", [1, 4095, 4096, 4097, 100003, 3_000_000])
def test_sort_pairs64(n):
    L = _lib()
    rng = np.random.default_rng(n)
    keys = rng.integers(0, 1 << 40, n, dtype=np.uint64)
    dup = rng.random(n) < 0.25
    keys[dup] = keys[rng.integers(0, n, dup.sum())]
    vals = rng.standard_normal(n)
    k = torch.tensor(keys.view(np.int64), device="cuda")
    v = torch.tensor(vals, device="cuda")
    ko, vo = torch.empty_like(k), torch.empty_like(v)
    assert L.lamg_t_sort_pairs64(n, _p(k), _p(v), _p(ko), _p(vo), 40) == 0
    o = np.argsort(keys, kind="stable")
    assert np.array_equal(ko.cpu().numpy().view(np.uint64), keys[o])
    assert np.array_equal(vo.cpu().numpy().view(np.uint64), vals[o].view(np.uint64))
    # inputs untouched
    assert np.array_equal(k.cpu().numpy().view(np.uint64), keys)


@pytest.mark.parametrize("n,bits", [(7, 3), (4097, 12), (250001, 17), (1 << 20, 32)])
def test_sort_pairs32(n, bits):
    L = _lib()
    rng = np.random.default_rng(bits)
    keys = rng.integers(0, 1 << bits, n, dtype=np.uint64).astype(np.uint32)
    vals = np.arange(n, dtype=np.int32)
    k = torch.tensor(keys.view(np.int32), device="cuda")
    v = torch.tensor(vals, device="cuda")
    ko, vo = torch.empty_like(k), torch.empty_like(v)
    assert L.lamg_t_sort_pairs32(n, _p(k), _p(v), _p(ko), _p(vo), bits) == 0
    o = np.argsort(keys, kind="stable")
    assert np.array_equal(ko.cpu().numpy().view(np.uint32), keys[o])
    assert np.array_equal(vo.cpu().numpy(), vals[o])


def test_sort_f64_order_and_bits():
    L = _lib()
    rng = np.random.default_rng(3)
    x = rng.standard_normal(50000)
    x[:100] = 0.0
    x[100:200] = -0.0
    x[200:210] = np.inf
    x[210:220] = -np.inf
    x[220:1000] = x[1000:1780]  # duplicates
    rng.shuffle(x)
    d = torch.tensor(x, device="cuda")
    o = torch.empty_like(d)
    assert L.lamg_t_sort_f64(x.size, _p(d), _p(o)) == 0
    got = o.cpu().numpy()
    # expected: ascending, -0 before +0 (order of the IEEE bit patterns mapped
    # to unsigned integers: negatives reversed below the positives)
    u = x.view(np.uint64)
    enc = np.where(u >> np.uint64(63), ~u, u | np.uint64(1 << 63))
    want = x[np.argsort(enc, kind="stable")]
    assert np.array_equal(got.view(np.uint64), want.view(np.uint64))
    assert np.all(got[1:] >= got[:-1])


@pytest.mark.parametrize("n", [0, 1, 2047, 2048, 2049, 5_000_000])
def test_exclusive_scan(n):
    L = _lib()
    rng = np.random.default_rng(n + 1)
    a = rng.integers(0, 7, n).astype(np.int32)
    d = torch.tensor(a, device="cuda") if n else torch.zeros(1, dtype=torch.int32, device="cuda")
    o = torch.full((n + 1,), -1, dtype=torch.int32, device="cuda")
    assert L.lamg_t_excl_scan(n, _p(d), _p(o)) == 0
    want = np.concatenate([[0], np.cumsum(a, dtype=np.int64)]).astype(np.int32)
    assert np.array_equal(o.cpu().numpy(), want)


def test_invalid_arguments():
    L = _lib()
    d = torch.zeros(4, dtype=torch.int64, device="cuda")
    assert L.lamg_t_sort_pairs64(4, _p(d), _p(d), _p(d), _p(d), 0) == lamg.E_INVALID_ARG
    assert L.lamg_t_sort_pairs64(4, _p(d), _p(d), _p(d), _p(d), 65) == lamg.E_INVALID_ARG
    assert L.lamg_t_sort_pairs32(-1, _p(d), _p(d), _p(d), _p(d), 8) == lamg.E_INVALID_ARG
    assert L.lamg_t_excl_scan(-1, _p(d), _p(d)) == lamg.E_INVALID_ARG
