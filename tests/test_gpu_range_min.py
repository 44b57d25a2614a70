"""GPU parity of hrr_range_min against the oracle (bit-exact argmin and min).

Both the paper's sweep (Section 2, Algorithms 2 and 3) and the O(1) ablation
are checked.  Inputs are the seeded range-query workloads of ``synth``.
"""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

M32 = 0xFFFFFFFF
METHODS = [0, 1, 2, 3, 4]   # paper (default), closed form, unpruned sweep, pruned loop sweep,
                            # aligned blocks


@pytest.fixture(scope="module")
def ctx():
    import paper_1907_12343_amd as hrr
    c = hrr.Context(synth.dither_tile(100))
    yield c
    c.close()


def _run(ctx, a, b, r, method):
    import paper_1907_12343_amd as hrr
    import torch
    dev = ctx.torch_device
    ta, tb, tr = (hrr.u32_tensor(x, dev) for x in (a, b, r))
    bad = torch.zeros(1, dtype=torch.int64, device=dev)
    k, v = ctx.range_min(ta, tb, tr, method=method, n_invalid=bad)
    torch.cuda.synchronize()
    return hrr.as_u32_numpy(k), hrr.as_u32_numpy(v), int(bad.item())


@pytest.mark.parametrize("method", METHODS)
def test_tiny_queries(ctx, orc, method):
    a, b, r = synth.tiny_queries()
    k, v, bad = _run(ctx, a, b, r, method)
    ek, ev = orc.rmq_scan(a, b, r)
    assert bad == 0
    assert np.array_equal(k, ek)
    assert np.array_equal(v, ev)


@pytest.mark.parametrize("method", METHODS)
def test_check_subset_against_scan(ctx, orc, method):
    # 2^16 queries with b - a <= 2^16, brute-force scan of every range
    a, b, r = synth.rangemin_check_queries()
    k, v, bad = _run(ctx, a, b, r, method)
    if method != 1:
        ek, ev = orc.rmq_scan(a, b, r)
    else:
        ek, ev = orc.rmq_dyadic(a, b, r)   # pinned to the scan by the CPU tests
    assert bad == 0
    assert np.array_equal(k, ek) and np.array_equal(v, ev)


def test_full_microbenchmark_against_dyadic_form(ctx, orc):
    """2^28 uniform queries, the benchmark launch shape: every output against
    the oracle's dyadic closed form (threaded over the host cores; the form is
    pinned to the scan by the CPU tests)."""
    import os
    import paper_1907_12343_amd as hrr
    import torch
    a, b, r = synth.rangemin_queries()
    dev = ctx.torch_device
    ta, tb, tr = (hrr.u32_tensor(x, dev) for x in (a, b, r))
    bad = torch.zeros(1, dtype=torch.int64, device=dev)
    k, v = ctx.range_min(ta, tb, tr, method=0, n_invalid=bad)
    torch.cuda.synchronize()
    assert int(bad.item()) == 0
    del ta, tb, tr
    threads = len(os.sched_getaffinity(0))
    chunk = 1 << 24
    for s0 in range(0, a.size, chunk):
        s1 = min(s0 + chunk, a.size)
        ek, ev = orc.rmq_dyadic(a[s0:s1], b[s0:s1], r[s0:s1], threads=threads)
        ks = hrr.as_u32_numpy(k[s0:s1])
        vs = hrr.as_u32_numpy(v[s0:s1])
        bad_k = np.flatnonzero(ks != ek)
        bad_v = np.flatnonzero(vs != ev)
        assert bad_k.size == 0 and bad_v.size == 0, \
            "queries %s differ" % (s0 + np.concatenate([bad_k, bad_v])[:8]).tolist()


def _edge_queries(orc):
    pts = [0, 1, 2, 3, 7, 8, 9, 255, 256, 257, (1 << 16) - 1, 1 << 16, (1 << 16) + 1,
           (1 << 31) - 1, 1 << 31, (1 << 31) + 1, M32 - 2, M32 - 1, M32]
    A, B, R = [], [], []
    shifts = [0, 1, 1 << 31, M32, 0x12345678]
    for a in pts:
        for b in pts:
            if a >= b:
                continue
            for r in shifts:
                A.append(a); B.append(b); R.append(r)
            # shifts that put k_r at a - 1, a, b - 1, b
            for kk in (a - 1, a, b - 1, b):
                kk &= M32
                A.append(a); B.append(b); R.append((-orc.bitrev(kk, 32)) & M32)
        if a < M32:
            A.append(a); B.append(a + 1); R.append(0xDEADBEEF)   # single element
    return (np.array(A, np.uint32), np.array(B, np.uint32), np.array(R, np.uint32))


@pytest.mark.parametrize("method", METHODS)
def test_edge_cases(ctx, orc, method):
    a, b, r = _edge_queries(orc)
    long_ = (b.astype(np.int64) - a) > (1 << 18)
    k, v, bad = _run(ctx, a, b, r, method)
    assert bad == 0
    ek = np.empty_like(a)
    ev = np.empty_like(a)
    ek[~long_], ev[~long_] = orc.rmq_scan(a[~long_], b[~long_], r[~long_])
    ek[long_], ev[long_] = orc.rmq_dyadic(a[long_], b[long_], r[long_])
    assert np.array_equal(k, ek) and np.array_equal(v, ev)


@pytest.mark.parametrize("method", METHODS)
def test_empty_ranges_marked_invalid(ctx, method):
    a = np.array([5, 9, 0, M32, 7], np.uint32)
    b = np.array([5, 3, 0, M32, 8], np.uint32)
    r = np.array([1, 2, 3, 4, 5], np.uint32)
    k, v, bad = _run(ctx, a, b, r, method)
    assert bad == 4
    assert k[:4].tolist() == b[:4].tolist()
    assert v[:4].tolist() == [M32] * 4
    assert k[4] == 7


@pytest.mark.parametrize("n", [1, 2, 3, 5, 7, 1023, 1025, 4099])
def test_ragged_sizes_and_unaligned_views(ctx, orc, n):
    import paper_1907_12343_amd as hrr
    import torch
    a, b, r = synth.range_queries(n + 1, 700 + n, max_len=300)
    dev = ctx.torch_device
    for off in (0, 1):   # off = 1: 4-byte aligned views take the scalar path
        ta, tb, tr = (hrr.u32_tensor(x, dev)[off:off + n] for x in (a, b, r))
        k, v = ctx.range_min(ta.contiguous() if off == 0 else ta, tb, tr, method=0)
        torch.cuda.synchronize()
        ek, ev = orc.rmq_scan(a[off:off + n], b[off:off + n], r[off:off + n])
        assert np.array_equal(hrr.as_u32_numpy(k), ek)
        assert np.array_equal(hrr.as_u32_numpy(v), ev)


def test_zero_queries(ctx):
    import torch
    e = torch.empty(0, dtype=torch.int32, device=ctx.torch_device)
    k, v = ctx.range_min(e, e, e)
    assert k.numel() == 0 and v.numel() == 0


def test_traversal_only_method_rejected(ctx):
    import paper_1907_12343_amd as hrr
    a = np.array([0, 3], np.uint32)
    with pytest.raises(hrr.HrrError):
        _run(ctx, a, a + 5, a, hrr.RMQ_PAPER_NO_REUSE)
    with pytest.raises(hrr.HrrError):
        _run(ctx, a, a + 5, a, 6)
