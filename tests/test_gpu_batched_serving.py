"""GPU tests of the batched launch, the autotuner and the serving loop.

Every item of a batched launch, and every served request, must return the
same pair set as a plain hrr_traverse of that item alone, which in turn must
equal the all-pairs oracle (checked here on sampled eyes of each item).
"""
import threading

import numpy as np
import pytest

import synth
from _helpers import (pair_keys_from_gpu, pair_keys_from_oracle, per_eye_fingerprints,
                      select_pairs_of_eyes)

pytestmark = pytest.mark.gpu

TILE_SEED = 100


@pytest.fixture(scope="module")
def hrr():
    import paper_1907_12343_amd as m
    return m


@pytest.fixture(scope="module")
def ctx(hrr):
    c = hrr.Context(synth.dither_tile(TILE_SEED))
    yield c
    c.close()


def _dev(ctx, a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, np.float32)).to(ctx.torch_device)


def _oracle_keys(orc, lights, eyes, sel, width, offset, s):
    ls = lights[orc.morton_order(lights)]
    out = orc.accept_eyes(eyes, sel, width, offset, synth.dither_tile(TILE_SEED), ls, s,
                          lists=True)
    return pair_keys_from_oracle(out, sel)


def _plain_keys(ctx, h, eyes_t, s, width, offset=0):
    pairs, n, _ = ctx.traverse_all(h, eyes_t, s, width, shift_offset=offset)
    return pair_keys_from_gpu(pairs)


def _pairs_with_weights(pairs, weights):
    """Sorted (eye, light, weight bits) tuples of a GPU result."""
    p = pairs.cpu().numpy().astype(np.int64) & 0xFFFFFFFF
    w = weights.cpu().numpy().view(np.uint32).astype(np.int64)
    order = np.lexsort((p[:, 1], p[:, 0]))
    return [tuple(x) for x in np.stack([p[order, 0], p[order, 1], w[order]], 1).tolist()]


def _small_cache(c, max_lights=1 << 16, max_eyes=1 << 12):
    """Cache c of the batched workload, cut to sizes the oracle samples fast."""
    d = synth.batched_cache(c)
    return dict(lights=d["lights"][:max_lights], eyes=d["eyes"][:max_eyes], width=d["width"],
                s=d["s"])


# ---------------------------------------------------------------------------
# batched launch
# ---------------------------------------------------------------------------

def test_batched_items_equal_plain_and_oracle(ctx, orc):
    import torch
    caches = [_small_cache(c) for c in range(10)]
    hs = [ctx.build_hierarchy(d["lights"]) for d in caches]
    eyes = [_dev(ctx, d["eyes"]) for d in caches]
    counts = [ctx.count(h, e, d["s"], d["width"]) for h, e, d in zip(hs, eyes, caches)]
    offs = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    pairs = torch.empty((max(int(offs[-1]), 1), 2), dtype=torch.int32, device=ctx.torch_device)
    items = [dict(h=h, eyes=e, s=d["s"], width=d["width"], out_offset=int(offs[k]),
                  out_capacity=int(counts[k]))
             for k, (h, e, d) in enumerate(zip(hs, eyes, caches))]
    got, st = ctx.traverse_batched(items, pairs)
    assert [int(x) for x in got] == counts
    rng = np.random.default_rng(7)
    for k, d in enumerate(caches):
        sl = pairs[offs[k]:offs[k + 1]]
        keys = pair_keys_from_gpu(sl)
        assert np.array_equal(keys, _plain_keys(ctx, hs[k], eyes[k], d["s"], d["width"]))
        sel = np.sort(rng.choice(d["eyes"].shape[0], 12, replace=False)).astype(np.uint32)
        want = _oracle_keys(orc, d["lights"], d["eyes"], sel, d["width"], 0, d["s"])
        assert np.array_equal(select_pairs_of_eyes(sl, sel), want)
    for h in hs:
        h.free()


def test_batched_groups_by_hierarchy_size(ctx, hrr):
    """Items whose hierarchies want different eyes per wave (8 below 2^16
    lights, 4 below 2^17, else 1) run as one launch per group; every item
    equals a plain launch of its group's shape pair for pair and weight for
    weight, work statistics add up exactly (one-eye-per-wave walks start at
    the hierarchy's top, several eyes per wave at the root, so the shapes
    must agree for the counts to), and an overflow stays per item."""
    import torch
    sizes = [1 << 11, (1 << 17) + 5, 1 << 16, 1 << 12, 1 << 18, 1 << 11]
    caches = []
    for c, nl in enumerate(sizes):
        d = synth.batched_cache(20 + c)
        lights = d["lights"]
        if lights.shape[0] < nl:
            lights = synth.mixture_points(nl, np.random.default_rng(900 + c).random((64, 3)), 910 + c)
        caches.append(dict(lights=np.ascontiguousarray(lights[:nl]), eyes=d["eyes"][:1 << 12],
                           width=d["width"], s=d["s"]))
    hs = [ctx.build_hierarchy(d["lights"]) for d in caches]
    eyes = [_dev(ctx, d["eyes"]) for d in caches]
    def group_epw(n):
        return 1 if n >= 1 << 17 else (4 if n >= 1 << 16 else 8)
    plain = [ctx.traverse_all(h, e, d["s"], d["width"], eyes_per_wave=group_epw(d["lights"].shape[0]),
                              stack_entries=512, with_weights=True, stats=True)
             for h, e, d in zip(hs, eyes, caches)]
    counts = [p[1] for p in plain]
    offs = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    pairs = torch.empty((int(offs[-1]), 2), dtype=torch.int32, device=ctx.torch_device)
    weights = torch.empty((int(offs[-1]),), dtype=torch.float32, device=ctx.torch_device)
    items = [dict(h=h, eyes=e, s=d["s"], width=d["width"], out_offset=int(offs[k]),
                  out_capacity=int(counts[k]))
             for k, (h, e, d) in enumerate(zip(hs, eyes, caches))]
    got, st = ctx.traverse_batched(items, pairs, weights=weights, stats=True, timing=True)
    assert [int(x) for x in got] == counts
    for k in range(len(caches)):
        sl = slice(int(offs[k]), int(offs[k + 1]))
        assert _pairs_with_weights(pairs[sl], weights[sl]) == \
            _pairs_with_weights(plain[k][0], plain[k][3]), k
    for key in ("node_visits", "rmq_calls", "leaf_tests", "eyes"):
        assert st[key] == sum(p[2][key] for p in plain), key
    assert st["pairs"] == sum(counts) and st["kernel_ms"] > 0
    # one item of the 8-eye group over its capacity: the others stay complete
    caps = list(counts)
    caps[3] = counts[3] // 2
    offs2 = np.concatenate([[0], np.cumsum(caps)]).astype(np.int64)
    items2 = [dict(it, out_offset=int(offs2[k]), out_capacity=int(caps[k])) for k, it in enumerate(items)]
    pairs.fill_(-1)
    with pytest.raises(hrr.OverflowResult) as ei:
        ctx.traverse_batched(items2, pairs)
    assert [int(x) for x in ei.value.counts] == counts
    for k in range(len(caches)):
        keys = pair_keys_from_gpu(pairs[int(offs2[k]):int(offs2[k + 1])])
        full = pair_keys_from_gpu(plain[k][0])
        if k == 3:
            assert keys.size == caps[3] and np.unique(keys).size == keys.size and np.isin(keys, full).all()
        else:
            assert np.array_equal(keys, full), k
    for h in hs:
        h.free()


def test_batched_overflow_is_per_item(ctx, hrr):
    import torch
    caches = [_small_cache(c, 1 << 12, 1 << 10) for c in range(3)]
    hs = [ctx.build_hierarchy(d["lights"]) for d in caches]
    eyes = [_dev(ctx, d["eyes"]) for d in caches]
    counts = [ctx.count(h, e, d["s"], d["width"]) for h, e, d in zip(hs, eyes, caches)]
    assert min(counts) > 10
    caps = [counts[0], counts[1] // 3, counts[2]]
    offs = np.concatenate([[0], np.cumsum(caps)]).astype(np.int64)
    pairs = torch.full((int(offs[-1]), 2), -1, dtype=torch.int32, device=ctx.torch_device)
    items = [dict(h=h, eyes=e, s=d["s"], width=d["width"], out_offset=int(offs[k]),
                  out_capacity=int(caps[k]))
             for k, (h, e, d) in enumerate(zip(hs, eyes, caches))]
    with pytest.raises(hrr.OverflowResult) as ei:
        ctx.traverse_batched(items, pairs)
    assert [int(x) for x in ei.value.counts] == counts
    for k in (0, 2):   # items within capacity are complete
        keys = pair_keys_from_gpu(pairs[offs[k]:offs[k + 1]])
        assert np.array_equal(keys, _plain_keys(ctx, hs[k], eyes[k], caches[k]["s"], 64))
    # the overflowing item's slice holds distinct pairs of its true set
    part = pair_keys_from_gpu(pairs[offs[1]:offs[2]])
    full = _plain_keys(ctx, hs[1], eyes[1], caches[1]["s"], 64)
    assert part.size == caps[1] and np.unique(part).size == part.size
    assert np.isin(part, full).all()
    for h in hs:
        h.free()


def test_batched_with_empty_items(ctx):
    import torch
    d = _small_cache(3, 1 << 12, 1 << 10)
    h = ctx.build_hierarchy(d["lights"])
    h0 = ctx.build_hierarchy(np.zeros((0, 3), np.float32))
    e = _dev(ctx, d["eyes"])
    e0 = torch.zeros((0, 3), dtype=torch.float32, device=ctx.torch_device)
    n = ctx.count(h, e, d["s"], 64)
    pairs = torch.empty((2 * n + 1, 2), dtype=torch.int32, device=ctx.torch_device)
    items = [dict(h=h, eyes=e0, s=d["s"], width=64, out_offset=0, out_capacity=0),
             dict(h=h, eyes=e, s=d["s"], width=64, out_offset=0, out_capacity=n),
             dict(h=h0, eyes=e, s=d["s"], width=64, out_offset=n, out_capacity=1),
             dict(h=h, eyes=e, s=d["s"], width=64, shift_offset=12345, out_offset=n + 1,
                  out_capacity=n)]
    ctx_counts, _ = ctx.traverse_batched(items, pairs)
    assert int(ctx_counts[0]) == 0 and int(ctx_counts[1]) == n and int(ctx_counts[2]) == 0
    assert np.array_equal(pair_keys_from_gpu(pairs[:n]), _plain_keys(ctx, h, e, d["s"], 64))
    m = int(ctx_counts[3])
    assert m <= n
    assert np.array_equal(pair_keys_from_gpu(pairs[n + 1:n + 1 + m]),
                          _plain_keys(ctx, h, e, d["s"], 64, offset=12345))
    h.free()
    h0.free()


def test_batched_interleaved_queues_equal_plain_and_oracle(ctx, orc, hrr):
    """A launch of several items with 2^19 or more tasks hands the XCD queues
    interleaved chunks of tasks (and lets a wave leave an item up to eight
    times); every item must still equal its plain launch, also when one item
    overflows its slice."""
    import torch
    caches = []
    for c in range(18):
        d = _small_cache(c, 1 << 12, 1 << 15)
        reps = -(-(1 << 15) // d["eyes"].shape[0])
        d["eyes"] = np.ascontiguousarray(np.tile(d["eyes"], (reps, 1))[:1 << 15])
        caches.append(d)
    assert sum(d["eyes"].shape[0] for d in caches) >= 1 << 19
    hs = [ctx.build_hierarchy(d["lights"]) for d in caches]
    eyes = [_dev(ctx, d["eyes"]) for d in caches]
    counts = [ctx.count(h, e, d["s"], d["width"]) for h, e, d in zip(hs, eyes, caches)]
    caps = list(counts)
    caps[5] = counts[5] // 2       # overflows
    caps[9] = counts[9] + 777      # room to spare
    offs = np.concatenate([[0], np.cumsum(caps)]).astype(np.int64)
    pairs = torch.full((int(offs[-1]), 2), -1, dtype=torch.int32, device=ctx.torch_device)
    weights = torch.full((int(offs[-1]),), -1.0, dtype=torch.float32, device=ctx.torch_device)
    items = [dict(h=h, eyes=e, s=d["s"], width=d["width"], out_offset=int(offs[k]),
                  out_capacity=int(caps[k]))
             for k, (h, e, d) in enumerate(zip(hs, eyes, caches))]
    with pytest.raises(hrr.OverflowResult) as ei:
        ctx.traverse_batched(items, pairs, weights=weights)
    assert [int(x) for x in ei.value.counts] == counts
    rng = np.random.default_rng(11)
    for k, d in enumerate(caches):
        sl = pairs[offs[k]:offs[k] + min(caps[k], counts[k])]
        keys = pair_keys_from_gpu(sl)
        full = _plain_keys(ctx, hs[k], eyes[k], d["s"], d["width"])
        if k == 5:
            assert keys.size == caps[5] and np.unique(keys).size == keys.size
            assert np.isin(keys, full).all()
            continue
        assert np.array_equal(keys, full)
        # the weights moved with their pairs: (pair, 1/p) tuples equal a plain launch's
        if k % 3 == 0:
            pp, _, _, pw = ctx.traverse_all(hs[k], eyes[k], d["s"], d["width"], with_weights=True)
            got_w = _pairs_with_weights(sl, weights[offs[k]:offs[k] + counts[k]])
            assert got_w == _pairs_with_weights(pp, pw)
        if k % 6 == 0:
            sel = np.sort(rng.choice(d["eyes"].shape[0], 8, replace=False)).astype(np.uint32)
            want = _oracle_keys(orc, d["lights"], d["eyes"], sel, d["width"], 0, d["s"])
            assert np.array_equal(select_pairs_of_eyes(sl, sel), want)
    for h in hs:
        h.free()


def test_batched_256_caches_counts_match_plain(ctx):
    """The 256-cache workload at its real sizes: per-item counts of one
    counting launch equal those of 256 plain launches."""
    caches = [synth.batched_cache(c) for c in range(256)]
    hs = [ctx.build_hierarchy(d["lights"]) for d in caches]
    eyes = [_dev(ctx, d["eyes"]) for d in caches]
    items = [dict(h=h, eyes=e, s=d["s"], width=d["width"], out_offset=0, out_capacity=0)
             for h, e, d in zip(hs, eyes, caches)]
    import paper_1907_12343_amd as hrr
    with pytest.raises(hrr.OverflowResult) as ei:
        ctx.traverse_batched(items, None)
    got = [int(x) for x in ei.value.counts]
    want = [ctx.count(h, e, d["s"], d["width"]) for h, e, d in zip(hs, eyes, caches)]
    assert got == want
    for h in hs:
        h.free()


def test_batched_256_caches_sampled_parity(ctx, orc):
    """The 256-cache workload at its real sizes in the benchmark's launch
    configuration (shape left to the library: one launch per eyes-per-wave
    group, leaf 1), all 1.35e9 pairs stored: counts equal plain counts, and
    sampled eyes of items from every group equal the oracle pair for pair."""
    import torch
    caches = [synth.batched_cache(c) for c in range(256)]
    hs = [ctx.build_hierarchy(d["lights"]) for d in caches]
    eyes = [_dev(ctx, d["eyes"]) for d in caches]
    counts = [ctx.count(h, e, d["s"], d["width"]) for h, e, d in zip(hs, eyes, caches)]
    offs = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    pairs = torch.empty((int(offs[-1]), 2), dtype=torch.int32, device=ctx.torch_device)
    items = [dict(h=h, eyes=e, s=d["s"], width=d["width"], out_offset=int(offs[k]),
                  out_capacity=int(counts[k]))
             for k, (h, e, d) in enumerate(zip(hs, eyes, caches))]
    got, _ = ctx.traverse_batched(items, pairs)
    assert [int(x) for x in got] == counts
    sizes = np.array([d["lights"].shape[0] for d in caches])
    order = np.argsort(sizes, kind="stable")
    band = lambda lo, hi: [int(k) for k in order if lo <= sizes[k] < hi][:2]
    pick = [int(k) for k in order[:2]] + band(1 << 13, 1 << 16) + band(1 << 16, 1 << 17) + \
        band(1 << 17, 1 << 18) + [int(k) for k in order[-2:]]
    rng = np.random.default_rng(11)
    for k in pick:
        d = caches[k]
        sl = pairs[int(offs[k]):int(offs[k + 1])]
        sel = np.sort(rng.choice(d["eyes"].shape[0], 6, replace=False)).astype(np.uint32)
        want = _oracle_keys(orc, d["lights"], d["eyes"], sel, d["width"], 0, d["s"])
        assert np.array_equal(select_pairs_of_eyes(sl, sel), want), (k, sizes[k])
    del pairs
    for h in hs:
        h.free()


# ---------------------------------------------------------------------------
# autotuner
# ---------------------------------------------------------------------------

def test_autotune_choice_is_valid_and_results_unchanged(hrr):
    ctx = hrr.Context(synth.dither_tile(TILE_SEED))
    try:
        d = _small_cache(5, 1 << 15, 1 << 13)
        hs = [ctx.build_hierarchy(d["lights"], leaf_size=L) for L in (1, 2, 4, 8)]
        e = _dev(ctx, d["eyes"])
        best = ctx.autotune(hs, e, d["s"], d["width"], max_probe_eyes=4096)
        assert best["eyes_per_wave"] in (1, 2, 4, 8)
        assert best["stack_entries"] in ((192, 256, 512) if best["eyes_per_wave"] == 1 else (256, 512, 1024))
        assert best["leaf_size"] in (1, 2, 4, 8)
        assert best["ms"] > 0
        assert ctx.tuned_leaf_size(d["lights"].shape[0]) == best["leaf_size"]
        ref = _plain_keys(ctx, hs[0], e, d["s"], d["width"])
        for h in hs:   # tuned shape (eyes_per_wave = stack_entries = 0) on every leaf size
            pairs, n, _ = ctx.traverse_all(h, e, d["s"], d["width"], eyes_per_wave=0,
                                           stack_entries=0)
            assert np.array_equal(pair_keys_from_gpu(pairs), ref)
        for h in hs:
            h.free()
    finally:
        ctx.close()


def test_autotune_batched_choice_is_applied_and_results_unchanged(hrr):
    """The batched tuner times one launch of all items per (leaf set, shape);
    afterwards a batched call with eyes_per_wave = stack_entries = 0 runs
    every item in the remembered shape, with the pairs of plain launches."""
    ctx = hrr.Context(synth.dither_tile(TILE_SEED))
    try:
        import torch
        ds = [_small_cache(c, 1 << 14, 1 << 11) for c in (7, 8, 9)]
        es = [_dev(ctx, d["eyes"]) for d in ds]
        sets = [[dict(h=ctx.build_hierarchy(d["lights"], leaf_size=L), eyes=e, s=d["s"],
                      width=d["width"]) for d, e in zip(ds, es)] for L in (1, 2)]
        best = ctx.autotune_batched(sets)
        assert best["eyes_per_wave"] in (1, 2, 4, 8)
        assert best["stack_entries"] in ((192, 256, 512) if best["eyes_per_wave"] == 1 else (256, 512, 1024))
        assert best["leaf_size"] in (1, 2) and best["ms"] > 0
        for d in ds:
            assert ctx.tuned_leaf_size(d["lights"].shape[0]) == best["leaf_size"]
        q = (1, 2).index(best["leaf_size"])
        items = sets[q]
        refs = [_plain_keys(ctx, it["h"], it["eyes"], it["s"], it["width"]) for it in items]
        offs = np.concatenate([[0], np.cumsum([r.size for r in refs])]).astype(np.int64)
        pairs = torch.empty((max(int(offs[-1]), 1), 2), dtype=torch.int32, device=ctx.torch_device)
        bi = [dict(it, out_offset=int(offs[k]), out_capacity=int(refs[k].size)) for k, it in enumerate(items)]
        counts, _ = ctx.traverse_batched(bi, pairs, eyes_per_wave=0, stack_entries=0)
        for k in range(len(items)):
            assert int(counts[k]) == refs[k].size
            got = pair_keys_from_gpu(pairs[offs[k]:offs[k + 1]])
            assert np.array_equal(got, refs[k]), k
        # a set whose items differ from set 0 is refused
        bad = [sets[0], [dict(sets[1][0], eyes=es[0][:100])] + sets[1][1:]]
        with pytest.raises(hrr.HrrError):
            ctx.autotune_batched(bad)
        del pairs
        for st in sets:
            for it in st:
                it["h"].free()
    finally:
        ctx.close()


# ---------------------------------------------------------------------------
# serving loop
# ---------------------------------------------------------------------------

def _served_setup(ctx, sizes=(1 << 12, 1 << 14, 1 << 16)):
    scenes = []
    for k, n in enumerate(sizes):
        rng = np.random.default_rng(700 + k)
        centers = rng.random((64, 3))
        lights = synth.mixture_points(n, centers, 710 + k)
        scenes.append(dict(lights=lights, centers=centers, h=ctx.build_hierarchy(lights)))
    return scenes


def _requests(scenes, n_req, seed, lo=6.0, hi=11.0):
    rng = np.random.default_rng(seed)
    out = []
    for q in range(n_req):
        k = int(rng.integers(len(scenes)))
        n = int(np.floor(2.0 ** rng.uniform(lo, hi)))
        eyes = synth.request_eyes(scenes[k]["centers"], n, int(rng.integers(1 << 31)))
        out.append(dict(scene=k, eyes=eyes, offset=int(rng.integers(0, 1 << 32)), width=64,
                        s=1e-4))
    return out


def test_served_requests_equal_plain_and_oracle(ctx, orc):
    scenes = _served_setup(ctx)
    reqs = _requests(scenes, 48, 720)
    ctx.server_start(hbm_budget_bytes=1 << 30, max_inflight=2, max_batch_items=16,
                     pairs_per_eye_guess=64.0)
    try:
        tickets = [ctx.submit(scenes[r["scene"]]["h"], r["eyes"], r["width"], r["offset"], r["s"])
                   for r in reqs]
        assert len(set(tickets)) == len(tickets)
        for t in tickets:
            assert ctx.wait(t, 60000)
        rng = np.random.default_rng(721)
        for q, (t, r) in enumerate(zip(tickets, reqs)):
            got = pair_keys_from_gpu(ctx.result(t))
            sc = scenes[r["scene"]]
            want = _plain_keys(ctx, sc["h"], _dev(ctx, r["eyes"]), r["s"], r["width"], r["offset"])
            assert np.array_equal(got, want), "request %d" % q
            _, n, info = ctx.poll(t)
            assert n == got.size and info["n_pairs"] == n and info["launches"] >= 1
            assert info["submit_s"] <= info["start_s"] <= info["done_s"]
            if q % 12 == 0:
                sel = np.sort(rng.choice(r["eyes"].shape[0], 8, replace=False)).astype(np.uint32)
                o = _oracle_keys(orc, sc["lights"], r["eyes"], sel, r["width"], r["offset"], r["s"])
                assert np.array_equal(select_pairs_of_eyes(ctx.result(t), sel), o)
            ctx.release(t)
        st = ctx.server_stats()
        assert st["submitted"] == st["completed"] == len(reqs)
        assert 1 <= st["launches"] <= len(reqs) + st["retries"]
        assert st["p99_ms"] >= st["p50_ms"] > 0
    finally:
        ctx.server_stop()
    for sc in scenes:
        sc["h"].free()


def test_served_at_the_served_configs_sizes(ctx, orc):
    """Requests of 2^16..2^18 eyes against hierarchies of the served workload's
    largest sizes (2^20.8, 2^21.2 and 2^22 lights, power-of-two splits, the
    benchmark's build) mixed with small ones, served together: every result
    equals the plain launch of the same request (one eye per wave for the
    large hierarchies, several for the small ones, each group with its own
    stack size) and sampled eyes equal the oracle."""
    import torch
    big = [12, 13, 15]                       # synth.served_hierarchy(h): 2^(16 + 6h/15) lights
    scenes = []
    for h in big:
        sc = synth.served_hierarchy(h)
        scenes.append(dict(lights=sc["lights"], centers=sc["centers"],
                           h=ctx.build_hierarchy(sc["lights"], split="pow2")))
    assert scenes[-1]["h"].n_lights == 1 << 22
    small = _served_setup(ctx, sizes=(1 << 12, 1 << 15))
    scenes += small
    rng = np.random.default_rng(777)
    reqs = []
    for q, (k, lg) in enumerate([(0, 16.0), (1, 17.0), (2, 18.0), (2, 16.5), (1, 17.5),
                                 (3, 10.0), (4, 12.0), (3, 11.0)]):
        n = int(np.floor(2.0 ** lg))
        eyes = synth.request_eyes(scenes[k]["centers"], n, int(rng.integers(1 << 31)))
        reqs.append(dict(scene=k, eyes=eyes, offset=int(rng.integers(0, 1 << 32)), width=64, s=1e-4))
    ctx.server_start(hbm_budget_bytes=64 << 30, max_inflight=2, max_batch_items=16,
                     max_batch_eyes=1 << 20, pairs_per_eye_guess=2000.0)
    try:
        tickets = [ctx.submit(scenes[r["scene"]]["h"], r["eyes"], r["width"], r["offset"], r["s"])
                   for r in reqs]
        for t in tickets:
            assert ctx.wait(t, 120000)
        for q, (t, r) in enumerate(zip(tickets, reqs)):
            sc = scenes[r["scene"]]
            res = ctx.result(t)
            ne = r["eyes"].shape[0]
            # billions of pairs: compared by per-eye count and two 64-bit hash sums
            got = per_eye_fingerprints(res, ne)
            plain, n_plain, _ = ctx.traverse_all(sc["h"], _dev(ctx, r["eyes"]), r["s"], r["width"],
                                                 shift_offset=r["offset"])
            want = per_eye_fingerprints(plain, ne)
            assert res.shape[0] == n_plain or (n_plain == 0 and res.shape[0] == 1), "request %d" % q
            for a_, b_ in zip(got, want):
                assert np.array_equal(a_, b_), "request %d" % q
            del plain
            torch.cuda.empty_cache()
            sel = np.sort(rng.choice(r["eyes"].shape[0], 6, replace=False)).astype(np.uint32)
            o = _oracle_keys(orc, sc["lights"], r["eyes"], sel, r["width"], r["offset"], r["s"])
            assert np.array_equal(select_pairs_of_eyes(res, sel), o), "request %d" % q
            del res
            ctx.release(t)
        st = ctx.server_stats()
        assert st["completed"] == len(reqs)
    finally:
        ctx.server_stop()
    for sc in scenes:
        sc["h"].free()
    torch.cuda.empty_cache()


def test_served_overflow_is_retried_exactly(ctx):
    scenes = _served_setup(ctx, sizes=(1 << 14,))
    reqs = _requests(scenes, 6, 730, lo=9.0, hi=10.0)
    ctx.server_start(hbm_budget_bytes=1 << 28, max_inflight=1, pairs_per_eye_guess=1e-6)
    try:
        ts = [ctx.submit(scenes[0]["h"], r["eyes"], 64, r["offset"], r["s"]) for r in reqs]
        for t, r in zip(ts, reqs):
            assert ctx.wait(t, 60000)
            want = _plain_keys(ctx, scenes[0]["h"], _dev(ctx, r["eyes"]), r["s"], 64, r["offset"])
            assert np.array_equal(pair_keys_from_gpu(ctx.result(t)), want)
            if want.size > 4096 * 2:
                assert ctx.poll(t)[2]["launches"] == 2 or ctx.server_stats()["retries"] >= 1
            ctx.release(t)
        assert ctx.server_stats()["retries"] >= 1
    finally:
        ctx.server_stop()
    scenes[0]["h"].free()


def test_served_admission_cancel_and_release(ctx, hrr):
    """A held result blocks a request whose output reservation needs the whole
    budget; that request stays queued (so it can be cancelled) until the
    result is released.  The blocked requests use a second hierarchy that no
    request has finished on, so their reservation is the configured guess."""
    rng = np.random.default_rng(740)
    lights = rng.random((1 << 12, 3)).astype(np.float32)
    h = ctx.build_hierarchy(lights)
    h2 = ctx.build_hierarchy(lights)
    small = rng.random((64, 3)).astype(np.float32)
    big = rng.random((1000, 3)).astype(np.float32)
    budget = 8 << 20
    ctx.server_start(hbm_budget_bytes=budget, max_inflight=1, pairs_per_eye_guess=1e4)
    try:
        ta = ctx.submit(h, small, 64, 0, 1e-3)
        assert ctx.wait(ta, 60000)
        assert ctx.poll(ta)[1] > 0
        tb = ctx.submit(h2, big, 64, 0, 1e-3)
        assert not ctx.wait(tb, 300)           # queued behind the held result
        assert ctx.cancel(tb) == hrr.HRR_OK
        with pytest.raises(hrr.HrrError) as ei:
            ctx.poll(tb)
        assert ei.value.status == hrr.HRR_E_CANCELLED
        ctx.release(tb)
        tc = ctx.submit(h2, big, 64, 0, 1e-3)
        assert not ctx.wait(tc, 300)
        with pytest.raises(hrr.HrrError) as ei:
            ctx.release(tc)                    # still queued
        assert ei.value.status == hrr.HRR_E_BUSY
        ctx.release(ta)                        # frees the arena: tc runs
        assert ctx.wait(tc, 60000)
        want = _plain_keys(ctx, h2, _dev(ctx, big), 1e-3, 64)
        assert np.array_equal(pair_keys_from_gpu(ctx.result(tc)), want)
        assert ctx.cancel(tc) == hrr.HRR_E_BUSY    # already complete
        ctx.release(tc)
        # eyes that can never fit are rejected at submit
        with pytest.raises(hrr.HrrError) as ei:
            ctx.submit(h, rng.random((budget // 12 + 1, 3)).astype(np.float32), 64, 0, 1e-3)
        assert ei.value.status == hrr.HRR_E_NOMEM
        # a result larger than the whole budget fails the request, not the server
        huge = rng.random((1 << 16, 3)).astype(np.float32)
        td = ctx.submit(h, huge, 64, 0, 1.0)   # p = 1 for most pairs: ~2^28 pairs
        with pytest.raises(hrr.HrrError) as ei:
            ctx.wait(td, 60000)
        assert ei.value.status == hrr.HRR_E_NOMEM
        with pytest.raises(hrr.HrrError) as ei:
            ctx.poll(td)
        assert ei.value.status == hrr.HRR_E_NOMEM
        ctx.release(td)
        # the server still serves
        te = ctx.submit(h, small, 64, 7, 1e-3)
        assert ctx.wait(te, 60000)
        want = _plain_keys(ctx, h, _dev(ctx, small), 1e-3, 64, offset=7)
        assert np.array_equal(pair_keys_from_gpu(ctx.result(te)), want)
        ctx.release(te)
        st = ctx.server_stats()
        assert st["cancelled"] == 1 and st["rejected"] == 1 and st["peak_bytes"] <= budget
    finally:
        ctx.server_stop()
    h.free()
    h2.free()


def test_served_from_many_threads(ctx):
    scenes = _served_setup(ctx, sizes=(1 << 13, 1 << 15))
    reqs = _requests(scenes, 40, 750, lo=6.0, hi=10.0)
    ctx.server_start(hbm_budget_bytes=1 << 30, max_inflight=3, max_batch_items=8)
    results = {}
    errors = []

    def client(part):
        try:
            for q in part:
                r = reqs[q]
                t = ctx.submit(scenes[r["scene"]]["h"], r["eyes"], 64, r["offset"], r["s"])
                assert ctx.wait(t, 60000)
                results[q] = pair_keys_from_gpu(ctx.result(t))
                ctx.release(t)
        except Exception as ex:   # reported below
            errors.append(ex)

    try:
        ths = [threading.Thread(target=client, args=(list(range(k, len(reqs), 4)),))
               for k in range(4)]
        for t in ths:
            t.start()
        for t in ths:
            t.join()
        assert not errors, errors
        for q, r in enumerate(reqs):
            want = _plain_keys(ctx, scenes[r["scene"]]["h"], _dev(ctx, r["eyes"]), r["s"], 64,
                               r["offset"])
            assert np.array_equal(results[q], want), "request %d" % q
    finally:
        ctx.server_stop()
    for sc in scenes:
        sc["h"].free()


def test_server_lifecycle_errors(ctx, hrr):
    h = ctx.build_hierarchy(np.random.default_rng(1).random((256, 3)).astype(np.float32))
    eyes = np.random.default_rng(2).random((16, 3)).astype(np.float32)
    with pytest.raises(hrr.HrrError) as ei:
        ctx.submit(h, eyes, 64, 0, 1e-3)
    assert ei.value.status == hrr.HRR_E_BUSY
    with pytest.raises(hrr.HrrError) as ei:
        ctx.server_start(hbm_budget_bytes=1 << 10)
    assert ei.value.status == hrr.HRR_E_INVALID
    ctx.server_start(hbm_budget_bytes=1 << 24)
    try:
        with pytest.raises(hrr.HrrError) as ei:
            ctx.server_start(hbm_budget_bytes=1 << 24)
        assert ei.value.status == hrr.HRR_E_BUSY
        with pytest.raises(hrr.HrrError) as ei:
            ctx.poll(987654321)
        assert ei.value.status == hrr.HRR_E_INVALID
        bad = eyes.copy()
        bad[3, 1] = np.nan
        with pytest.raises(hrr.HrrError) as ei:
            ctx.submit(h, bad, 64, 0, 1e-3)
        assert ei.value.status == hrr.HRR_E_INVALID
        with pytest.raises(hrr.HrrError) as ei:
            ctx.submit(h, eyes, 64, 0, 0.0)
        assert ei.value.status == hrr.HRR_E_INVALID
        t = ctx.submit(h, np.zeros((0, 3), np.float32), 64, 0, 1e-3)
        assert ctx.wait(t, 60000) and ctx.poll(t)[1] == 0
        ctx.release(t)
    finally:
        ctx.server_stop()
    ctx.server_stop()          # stopping twice is fine
    with pytest.raises(hrr.HrrError) as ei:
        ctx.server_stats()
    assert ei.value.status == hrr.HRR_E_BUSY
    h.free()
