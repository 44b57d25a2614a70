"""GPU test of hrr_traverse_noalloc, the traversal that allocates nothing
(for callers that cannot allocate: code under graph capture, tight serving
loops): its result must equal hrr_traverse's on the same inputs, bit for bit
as pair sets, on consecutive calls that reuse the device's fixed scratch --
the second with a smaller input, then with other shapes, weights and an
output that overflows."""
import numpy as np
import pytest

import synth
from _helpers import pair_keys_from_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hrr():
    import paper_1907_12343_amd as m
    return m


def _noalloc(ctx, h, eyes, s, width, capacity, **kw):
    import torch
    pairs = torch.full((max(capacity, 1), 2), -1, dtype=torch.int32, device=eyes.device)
    weights = (torch.zeros((max(capacity, 1),), dtype=torch.float32, device=eyes.device)
               if kw.pop("with_weights", False) else None)
    res = torch.full((2,), -7, dtype=torch.int64, device=eyes.device)
    ctx.traverse_noalloc(h, eyes, s, width, pairs, res, weights=weights, capacity=capacity, **kw)
    torch.cuda.synchronize()
    count, status = (int(x) for x in res.cpu())
    return pairs, weights, count, status


def test_noalloc_equals_traverse_on_consecutive_calls(hrr):
    import torch
    fr = synth.frame()
    tiny = synth.tiny()
    ctx = hrr.Context(fr["tile"])
    try:
        big = ctx.build_hierarchy(fr["lights"], leaf_size=1, split="pow2")
        e_big = torch.from_numpy(np.ascontiguousarray(fr["eyes"][:1 << 16])).to(ctx.torch_device)
        small = ctx.build_hierarchy(tiny["lights"], leaf_size=1)
        e_small = torch.from_numpy(tiny["eyes"]).to(ctx.torch_device)
        cases = [
            # (hierarchy, eyes, s, width, options): the second smaller than the first
            (big, e_big, fr["s"], fr["width"], {}),
            (small, e_small, tiny["s"], tiny["width"], {}),
            (small, e_small, tiny["s"], tiny["width"], dict(eyes_per_wave=8, stack_entries=256)),
            (big, e_big[:5000], fr["s"], fr["width"], dict(n_samples=3, psi_s0=0x1234567)),
        ]
        for q, (h, e, s, w, kw) in enumerate(cases):
            ref, n, _ = ctx.traverse_all(h, e, s, w, **kw)
            want = pair_keys_from_gpu(ref)
            pairs, _, count, status = _noalloc(ctx, h, e, s, w, n, **kw)
            assert status == 0 and count == n, (q, count, n, status)
            assert np.array_equal(pair_keys_from_gpu(pairs[:n]), want), q
            del ref, pairs
        # weights: the same pairs with the same weights
        ref, n, _, rw = ctx.traverse_all(small, e_small, tiny["s"], tiny["width"], with_weights=True)
        pairs, weights, count, status = _noalloc(ctx, small, e_small, tiny["s"], tiny["width"], n,
                                                 with_weights=True)
        assert status == 0 and count == n

        def keyed(p, wt):
            k = pair_keys_from_gpu(p)
            u = p[:, 0].to(torch.int64) & 0xFFFFFFFF
            i = p[:, 1].to(torch.int64) & 0xFFFFFFFF
            order = torch.argsort((u << 32) | i)
            return k, wt[order].cpu().numpy().view(np.uint32)

        k1, w1 = keyed(ref, rw)
        k2, w2 = keyed(pairs[:n], weights[:n])
        assert np.array_equal(k1, k2) and np.array_equal(w1, w2)
        # an output that overflows: the true count, distinct accepted pairs in front
        cap = n // 3
        pairs, _, count, status = _noalloc(ctx, small, e_small, tiny["s"], tiny["width"], cap)
        assert status == 0 and count == n
        got = pair_keys_from_gpu(pairs[:cap])
        assert got.size == cap and np.unique(got).size == cap
        assert np.isin(got, k1).all()
        # a count-only call (no output at all)
        _, _, count, status = _noalloc(ctx, big, e_big, fr["s"], fr["width"], 0)
        assert status == 0 and count == ctx.count(big, e_big, fr["s"], fr["width"])
        # options that need a readback are refused
        with pytest.raises(hrr.HrrError):
            _noalloc(ctx, small, e_small, tiny["s"], tiny["width"], n, stats=True)
        big.free()
        small.free()
    finally:
        ctx.close()
