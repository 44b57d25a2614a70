"""GPU parity of hrr_traverse against the all-pairs oracle.

The accepted (j, i) set must equal, element for element after sorting, the
set of pairs whose own rotated radical inverse passes their own acceptance
test (Section 1's hierarchical Russian roulette must never drop or add a
pair).  Bit-exact: xi is an integer and the fp32 acceptance test uses the
same rounding on both sides.
"""
import numpy as np
import pytest

import synth
from _helpers import (per_eye_fingerprints, pair_keys_from_gpu, pair_keys_from_oracle,
                      select_pairs_of_eyes)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_1907_12343_amd as hrr
    c = hrr.Context(synth.dither_tile(100))
    yield c
    c.close()


@pytest.fixture(scope="module")
def tiny():
    return synth.tiny()


@pytest.fixture(scope="module")
def tiny_oracle(orc, tiny):
    perm = orc.morton_order(tiny["lights"])
    ls = tiny["lights"][perm]
    sel = np.arange(tiny["eyes"].shape[0])
    out = orc.accept_eyes(tiny["eyes"], sel, tiny["width"], 0, tiny["tile"], ls, tiny["s"],
                          lists=True)
    return dict(perm=perm, lights_sorted=ls, keys=pair_keys_from_oracle(out, sel), out=out)


def _eyes_t(ctx, eyes):
    import torch
    return torch.from_numpy(np.ascontiguousarray(eyes, np.float32)).to(ctx.torch_device)


def test_light_order_matches_oracle(ctx, orc, tiny, tiny_oracle):
    for leaf in (1, 2, 4, 8):
        h = ctx.build_hierarchy(tiny["lights"], leaf_size=leaf)
        assert np.array_equal(h.permutation(), tiny_oracle["perm"])
        assert np.array_equal(h.sorted_lights(), tiny_oracle["lights_sorted"])
        h.free()


@pytest.mark.parametrize("method", [0, 1, 2, 3, 4, 5])
@pytest.mark.parametrize("leaf", [1, 2, 4, 8])
@pytest.mark.parametrize("epw", [1, 2, 4, 8])
def test_tiny_full_parity(ctx, tiny, tiny_oracle, method, leaf, epw):
    h = ctx.build_hierarchy(tiny["lights"], leaf_size=leaf)
    eyes = _eyes_t(ctx, tiny["eyes"])
    # one eye per wave on the smallest stack (record area beside it in LDS)
    pairs, n, st = ctx.traverse_all(h, eyes, tiny["s"], tiny["width"], rmq_method=method,
                                    eyes_per_wave=epw, stack_entries=192 if epw == 1 else 512,
                                    stats=True)
    got = pair_keys_from_gpu(pairs)
    assert n == tiny_oracle["keys"].size
    assert np.array_equal(got, tiny_oracle["keys"])
    assert st["eyes"] == tiny["eyes"].shape[0]
    h.free()


@pytest.mark.parametrize("method", [0, 1, 4])
@pytest.mark.parametrize("leaf", [1, 2, 8])
@pytest.mark.parametrize("epw", [1, 8])
def test_tiny_full_parity_pow2_split(ctx, tiny, tiny_oracle, method, leaf, epw):
    """The accepted set does not depend on how the hierarchy splits its index
    ranges: power-of-two splits (aligned blocks) give the oracle's set too."""
    h = ctx.build_hierarchy(tiny["lights"], leaf_size=leaf, split="pow2")
    assert h.split == "pow2"
    pairs, n, _ = ctx.traverse_all(h, _eyes_t(ctx, tiny["eyes"]), tiny["s"], tiny["width"],
                                   rmq_method=method, eyes_per_wave=epw, stack_entries=512)
    assert n == tiny_oracle["keys"].size
    assert np.array_equal(pair_keys_from_gpu(pairs), tiny_oracle["keys"])
    h.free()


@pytest.mark.parametrize("cap,epw", [(192, 1), (256, 1), (320, 1), (192, 4)])
def test_stack_spills_to_device_memory(ctx, orc, cap, epw):
    # a wide survivor front (large s) against a small LDS stack ring (any
    # multiple of 64 entries from 192 on; 64-entry units move to device memory)
    lights = synth.uniform_points(1 << 15, 801)
    eyes = synth.uniform_points(512, 802)
    tile = synth.dither_tile(100)
    s = 2e-2
    h = ctx.build_hierarchy(lights, leaf_size=1)
    pairs, n, st = ctx.traverse_all(h, _eyes_t(ctx, eyes), s, 64, stack_entries=cap,
                                    eyes_per_wave=epw, stats=True)
    assert st["spills"] > 0, st
    assert st["max_stack"] > cap
    assert st["max_stack"] <= 128 * (h.depth + 1)
    sel = np.arange(0, 512, 5)
    out = orc.accept_eyes(eyes, sel, 64, 0, tile, h.sorted_lights(), s, lists=True)
    assert np.array_equal(select_pairs_of_eyes(pairs, sel), pair_keys_from_oracle(out, sel))
    # same set with a roomy stack and several eyes per wave, and in index order
    p2, n2, st2 = ctx.traverse_all(h, _eyes_t(ctx, eyes), s, 64, stack_entries=2048,
                                   eyes_per_wave=4, stats=True)
    assert n2 == n
    assert np.array_equal(pair_keys_from_gpu(p2), pair_keys_from_gpu(pairs))
    p3, n3, _ = ctx.traverse_all(h, _eyes_t(ctx, eyes), s, 64, reorder=False)
    assert n3 == n
    assert np.array_equal(pair_keys_from_gpu(p3), pair_keys_from_gpu(pairs))
    h.free()


@pytest.fixture(scope="module")
def ordered_case(orc):
    """A launch with enough work to be ordered (8192 eyes x 2^14 lights: cost
    8192 x (2^14)^0.6 = 2.8e6, above the 2^21 at which the library orders)."""
    lights = synth.uniform_points(1 << 14, 811)
    eyes = synth.uniform_points(8192, 812)
    tile = synth.dither_tile(100)
    sel = np.arange(eyes.shape[0])
    ls = lights[orc.morton_order(lights)]
    out = orc.accept_eyes(eyes, sel, 64, 0, tile, ls, 1e-3, lists=True)
    return dict(lights=lights, eyes=eyes, keys=pair_keys_from_oracle(out, sel))


@pytest.mark.parametrize("epw", [1, 2, 4, 8])
def test_processing_order_does_not_change_the_set(ctx, ordered_case, epw):
    """Eye ordering on and off give the oracle's set (leaf size 2)."""
    h = ctx.build_hierarchy(ordered_case["lights"], leaf_size=2)
    eyes = _eyes_t(ctx, ordered_case["eyes"])
    for reorder in (True, False):
        pairs, n, st = ctx.traverse_all(h, eyes, 1e-3, 64, eyes_per_wave=epw,
                                        reorder=reorder, stats=True)
        assert np.array_equal(pair_keys_from_gpu(pairs), ordered_case["keys"]), reorder
        assert st["eyes"] == ordered_case["eyes"].shape[0]
    h.free()


@pytest.mark.parametrize("leaf", [1, 4])
def test_weights_are_exact_reciprocals(ctx, orc, tiny, tiny_oracle, leaf):
    import torch
    h = ctx.build_hierarchy(tiny["lights"], leaf_size=leaf)
    eyes = _eyes_t(ctx, tiny["eyes"])
    pairs, n, st, w = ctx.traverse_all(h, eyes, tiny["s"], tiny["width"], with_weights=True)
    pj = pairs.cpu().numpy().view(np.uint32)
    wn = w.cpu().numpy()
    ls = tiny_oracle["lights_sorted"]
    rng = np.random.default_rng(5)
    pick = rng.choice(n, size=min(n, 3000), replace=False)
    for q in pick:
        j, i = pj[q]
        exp = orc.accept_weight(tiny["eyes"][j], ls[i], tiny["s"])
        assert np.float32(wn[q]) == np.float32(exp)
    h.free()


def test_multi_sample(ctx, orc, tiny, tiny_oracle):
    ns, s0 = 3, 0x51ED270B
    h = ctx.build_hierarchy(tiny["lights"], leaf_size=1)
    eyes = _eyes_t(ctx, tiny["eyes"])
    pairs, n, _ = ctx.traverse_all(h, eyes, tiny["s"], tiny["width"], n_samples=ns, psi_s0=s0)
    sel = np.arange(tiny["eyes"].shape[0])
    out = orc.accept_eyes(tiny["eyes"], sel, tiny["width"], 0, tiny["tile"],
                          tiny_oracle["lights_sorted"], tiny["s"], n_samples=ns, psi_s0=s0,
                          lists=True)
    assert np.array_equal(pair_keys_from_gpu(pairs), pair_keys_from_oracle(out, sel, ns))
    h.free()


def test_shift_offset_and_pixel_base(ctx, orc, tiny, tiny_oracle):
    off, base, W = 0x9E3779B9, 37, 50
    h = ctx.build_hierarchy(tiny["lights"], leaf_size=2)
    ne = tiny["eyes"].shape[0]
    pairs, n, _ = ctx.traverse_all(h, _eyes_t(ctx, tiny["eyes"]), tiny["s"], W,
                                   shift_offset=off, pixel_base=base)
    # the oracle places eye j at pixel j: pad the eye array by `base`
    padded = np.concatenate([np.zeros((base, 3), np.float32), tiny["eyes"]])
    sel = np.arange(base, base + ne)
    out = orc.accept_eyes(padded, sel, W, off, tiny["tile"], tiny_oracle["lights_sorted"],
                          tiny["s"], lists=True)
    exp = pair_keys_from_oracle(out, sel)
    exp = np.sort(exp - (np.uint64(base) << np.uint64(32)))
    assert np.array_equal(pair_keys_from_gpu(pairs), exp)
    h.free()


@pytest.mark.parametrize("kind", ["zero", "random", "odd"])
def test_any_tile_values(orc, tiny, tiny_oracle, kind):
    """The eye order groups eyes by the low significant bits of their tile
    value; tiles without the permutation-times-2^20 structure (all zero: no
    class bits; full 32-bit values; odd values) must give the same set as
    the oracle."""
    import paper_1907_12343_amd as hrr
    rng = np.random.default_rng(7)
    if kind == "zero":
        tile = np.zeros(4096, np.uint32)
    elif kind == "random":
        tile = rng.integers(0, 2**32, 4096, dtype=np.uint64).astype(np.uint32)
    else:
        tile = (2 * rng.integers(0, 2**20, 4096) + 1).astype(np.uint32)
    c = hrr.Context(tile)
    try:
        h = c.build_hierarchy(tiny["lights"], leaf_size=1)
        sel = np.arange(tiny["eyes"].shape[0])
        exp = pair_keys_from_oracle(
            orc.accept_eyes(tiny["eyes"], sel, tiny["width"], 0, tile, tiny_oracle["lights_sorted"],
                            tiny["s"], lists=True), sel)
        for reorder in (True, False):
            pairs, n, _ = c.traverse_all(h, _eyes_t(c, tiny["eyes"]), tiny["s"], tiny["width"],
                                         reorder=reorder)
            assert np.array_equal(pair_keys_from_gpu(pairs), exp)
        h.free()
    finally:
        c.close()


def test_overflow_reports_true_count(ctx, tiny, tiny_oracle):
    import paper_1907_12343_amd as hrr
    import torch
    h = ctx.build_hierarchy(tiny["lights"], leaf_size=1)
    eyes = _eyes_t(ctx, tiny["eyes"])
    total = tiny_oracle["keys"].size
    cap = total // 3
    buf = torch.full((cap, 2), -1, dtype=torch.int32, device=ctx.torch_device)
    with pytest.raises(hrr.OverflowResult) as ei:
        ctx.traverse(h, eyes, tiny["s"], tiny["width"], pairs=buf)
    assert str(total) in str(ei.value)
    assert ctx.count(h, eyes, tiny["s"], tiny["width"]) == total
    stored = pair_keys_from_gpu(buf)
    assert stored.size == cap and np.unique(stored).size == cap
    assert np.isin(stored, tiny_oracle["keys"]).all()
    h.free()


@pytest.mark.parametrize("extra", [1, 77, 1000, 100003, -1])
def test_capacity_above_the_count(ctx, tiny, tiny_oracle, extra):
    """Capacity larger than the count: output chunks straddle the capacity
    and the pairs past it live in the slack area until compaction; the first
    count positions must hold exactly the accepted set (with weights)."""
    import torch
    h = ctx.build_hierarchy(tiny["lights"], leaf_size=1)
    eyes = _eyes_t(ctx, tiny["eyes"])
    total = tiny_oracle["keys"].size
    cap = 2 * total if extra < 0 else total + extra
    buf = torch.full((cap, 2), -7, dtype=torch.int32, device=ctx.torch_device)
    w = torch.full((cap,), -7.0, dtype=torch.float32, device=ctx.torch_device)
    pairs, n, _, wt = ctx.traverse(h, eyes, tiny["s"], tiny["width"], pairs=buf, weights=w)
    assert n == total
    assert np.array_equal(pair_keys_from_gpu(pairs), tiny_oracle["keys"])
    assert bool((wt >= 1.0).all())
    h.free()


@pytest.mark.parametrize("n_l,leaf", [(1, 1), (2, 1), (3, 1), (5, 8), (8, 8), (9, 8), (17, 4)])
def test_small_and_root_leaf_hierarchies(ctx, orc, n_l, leaf):
    lights = synth.uniform_points(n_l, 900 + n_l)
    eyes = synth.uniform_points(300, 901)
    eyes[7] = lights[0]                      # eye on a light: d = 0, p = 1
    tile = synth.dither_tile(100)
    h = ctx.build_hierarchy(lights, leaf_size=leaf)
    for epw in (1, 8):
        pairs, n, _ = ctx.traverse_all(h, _eyes_t(ctx, eyes), 0.05, 64, eyes_per_wave=epw)
        sel = np.arange(300)
        out = orc.accept_eyes(eyes, sel, 64, 0, tile, h.sorted_lights(), 0.05, lists=True)
        assert np.array_equal(pair_keys_from_gpu(pairs), pair_keys_from_oracle(out, sel))
    h.free()


@pytest.mark.parametrize("split", ["radix", "pow2"])
@pytest.mark.parametrize("n_l,leaf", [(33, 1), (64, 1), (65, 1), (100, 3), (127, 1), (128, 3), (129, 1),
                                      (200, 3), (300, 8)])
def test_walk_start_at_the_hierarchy_top(ctx, orc, n_l, leaf, split):
    """One-eye-per-wave walks start from the hierarchy's top (the nodes of
    depth 6 and the leaves above it).  Light counts around 2^6 with leaf sizes
    1, 3 and 8 make tops that mix leaves of every depth with internal nodes,
    in both split rules; the accepted set equals the oracle's all-pairs set
    and the several-eyes-per-wave walk, which starts at the root."""
    lights = synth.mixture_points(n_l, np.random.default_rng(700 + n_l).random((4, 3)), 710 + n_l)
    eyes = synth.uniform_points(500, 720 + n_l)
    tile = synth.dither_tile(100)
    h = ctx.build_hierarchy(lights, leaf_size=leaf, split=split)
    sel = np.arange(500)
    out = orc.accept_eyes(eyes, sel, 64, 0, tile, h.sorted_lights(), 0.02, lists=True)
    want = pair_keys_from_oracle(out, sel)
    for epw in (1, 8):
        pairs, n, _ = ctx.traverse_all(h, _eyes_t(ctx, eyes), 0.02, 64, eyes_per_wave=epw)
        assert np.array_equal(pair_keys_from_gpu(pairs), want), epw
    h.free()


def test_keep_decisions_at_the_threshold(ctx, orc):
    """s chosen so that p 2^32 lands within a few units of a pair's xi: the
    fast reciprocal band must hand every such case to the exact division."""
    import torch
    tile = synth.dither_tile(100)
    lights = np.array([[0.25, 0.0, 0.0], [0.0, 0.5, 0.0], [0.1, 0.2, 0.3]], np.float32)
    eyes = np.zeros((1, 3), np.float32)
    e_t = _eyes_t(ctx, eyes)
    r0 = orc.eye_shift(tile, 0, 64)
    for leaf in (1, 8):                      # internal node with leaf children / root leaf
        h = ctx.build_hierarchy(lights, leaf_size=leaf)
        ls = h.sorted_lights()
        for i in range(3):
            xi = orc.phi(i, r0, 32)
            d = ls[i].astype(np.float32)
            d2 = np.float32(np.float32(np.float32(d[0] * d[0]) + np.float32(d[1] * d[1]))
                            + np.float32(d[2] * d[2]))
            for delta in (-3.0, -1.0, -0.5, -1e-3, 0.0, 1e-3, 0.5, 1.0, 3.0):
                p_target = (xi + delta) / 2.0 ** 32
                if not (0.0 < p_target < 1.0):
                    continue
                s = float(np.float32(p_target * float(d2)))
                for ds in (-1, 0, 1):           # neighbouring floats of s
                    s2 = float(np.nextafter(np.float32(s), np.float32(np.inf if ds > 0 else -np.inf))) if ds else s
                    pairs, n, _ = ctx.traverse_all(h, e_t, s2, 64)
                    got = sorted(int(x) for x in pairs[:, 1].cpu().numpy())
                    exp = [k for k in range(3) if orc.accept(eyes[0], ls[k], s2, orc.phi(k, r0, 32))]
                    assert got == exp, (leaf, i, delta, ds, s2)
        h.free()


@pytest.mark.parametrize("s", [3.4028235e38, 1e30, 2.0 ** 61, 2.0 ** 60, 2.0 ** -60, 2.0 ** -61, 1e-30,
                               1.4e-45])
def test_extreme_s(ctx, orc, tiny, s):
    """Values of s at and beyond the range of the kernel's product-form test
    (2^-60 .. 2^60) and up to accepting the whole product set: the decisions
    then come from the IEEE division alone and must still equal the oracle's.
    Two eyes sit exactly on a light (d^2 = 0, p = 1)."""
    h = ctx.build_hierarchy(tiny["lights"], leaf_size=1)
    ls = h.sorted_lights()
    eyes = np.ascontiguousarray(tiny["eyes"][:512]).copy()
    eyes[7] = ls[5]
    eyes[300] = ls[1000]
    pairs, n, _ = ctx.traverse_all(h, _eyes_t(ctx, eyes), s, tiny["width"])
    sel = np.arange(eyes.shape[0])
    out = orc.accept_eyes(eyes, sel, tiny["width"], 0, tiny["tile"], ls, s, lists=True)
    exp = pair_keys_from_oracle(out, sel)
    assert n == exp.size
    assert np.array_equal(pair_keys_from_gpu(pairs), exp)
    if s >= 1e30:
        assert n == eyes.shape[0] * ls.shape[0]          # every pair is kept
    for j, i in ((7, 5), (300, 1000)):                   # a light under the eye is always kept
        assert (np.uint64(j) << np.uint64(32)) | np.uint64(i) in set(exp.tolist())
    h.free()


def test_coincident_lights_split_at_midpoint(ctx, orc):
    base = synth.uniform_points(40, 950)
    lights = np.repeat(base, 25, axis=0)            # 25 copies each: equal Morton codes
    eyes = synth.uniform_points(200, 951)
    tile = synth.dither_tile(100)
    h = ctx.build_hierarchy(lights, leaf_size=1)
    assert np.array_equal(h.permutation(), orc.morton_order(lights))
    pairs, n, _ = ctx.traverse_all(h, _eyes_t(ctx, eyes), 0.01, 16)
    sel = np.arange(200)
    out = orc.accept_eyes(eyes, sel, 16, 0, tile, h.sorted_lights(), 0.01, lists=True)
    assert np.array_equal(pair_keys_from_gpu(pairs), pair_keys_from_oracle(out, sel))
    h.free()


def test_empty_inputs(ctx, tiny):
    import torch
    h = ctx.build_hierarchy(tiny["lights"], leaf_size=1)
    e0 = torch.empty((0, 3), dtype=torch.float32, device=ctx.torch_device)
    pairs, n, _ = ctx.traverse(h, e0, 1e-3, 64, capacity=16)
    assert n == 0
    h0 = ctx.build_hierarchy(np.zeros((0, 3), np.float32))
    pairs, n, _ = ctx.traverse(h0, _eyes_t(ctx, tiny["eyes"]), 1e-3, 64, capacity=16)
    assert n == 0
    h.free()
    h0.free()


def test_invalid_arguments(ctx, tiny):
    import paper_1907_12343_amd as hrr
    with pytest.raises(hrr.HrrError):
        ctx.build_hierarchy(np.array([[0.0, np.nan, 0.0]], np.float32))
    with pytest.raises(hrr.HrrError):
        ctx.build_hierarchy(tiny["lights"], leaf_size=9)
    h = ctx.build_hierarchy(tiny["lights"], leaf_size=1)
    e = _eyes_t(ctx, tiny["eyes"])
    for bad_s in (0.0, -1.0, float("inf"), float("nan")):
        with pytest.raises(hrr.HrrError):
            ctx.traverse(h, e, bad_s, 64, capacity=8)
    with pytest.raises(hrr.HrrError):
        ctx.traverse(h, e, 1e-3, 0, capacity=8)
    with pytest.raises(hrr.HrrError):
        ctx.traverse(h, e, 1e-3, 64, capacity=8, eyes_per_wave=3)
    for bad_cap in (300, 128, 160, 4160):   # not a multiple of 64 in [192, 4096]
        with pytest.raises(hrr.HrrError):
            ctx.traverse(h, e, 1e-3, 64, capacity=8, stack_entries=bad_cap)
    h.free()


def _bitrev32(x):
    """Bit reversal of u32 values held in an int64 tensor (Section 2's radical
    inverse in 32-bit fixed point), by the usual swap of halves, bytes, ..."""
    x = ((x >> 1) & 0x55555555) | ((x & 0x55555555) << 1)
    x = ((x >> 2) & 0x33333333) | ((x & 0x33333333) << 2)
    x = ((x >> 4) & 0x0F0F0F0F) | ((x & 0x0F0F0F0F) << 4)
    x = ((x >> 8) & 0x00FF00FF) | ((x & 0x00FF00FF) << 8)
    return ((x >> 16) & 0xFFFF) | ((x & 0xFFFF) << 16)


def _assert_every_pair_passes_its_test(pairs, fr, perm, chunk=1 << 27):
    """Soundness over the whole launch: every emitted (j, i) has valid indices
    and xi_ij < ceil(min(1, s / d^2) 2^32), with d^2 = (dx dx + dy dy) + dz dz
    in separately rounded binary32 operations (plain torch ops, one per
    kernel) and xi_ij = bitreverse(i) + r_j mod 2^32."""
    import torch
    dev = pairs.device
    eyes = torch.from_numpy(fr["eyes"]).to(dev)
    lights = torch.from_numpy(np.ascontiguousarray(fr["lights"][perm])).to(dev)
    tile = torch.from_numpy(fr["tile"].astype(np.int64)).to(dev)
    W = fr["width"]
    s = torch.tensor(fr["s"], dtype=torch.float32, device=dev)
    two32 = float(2 ** 32)
    for at in range(0, pairs.shape[0], chunk):
        pc = pairs[at:at + chunk].to(torch.int64) & 0xFFFFFFFF
        j, i = pc[:, 0], pc[:, 1]
        assert int(j.max()) < eyes.shape[0] and int(i.max()) < lights.shape[0]
        e = eyes[j]
        lt = lights[i]
        dx = lt[:, 0] - e[:, 0]
        dy = lt[:, 1] - e[:, 1]
        dz = lt[:, 2] - e[:, 2]
        d2 = (dx * dx + dy * dy) + dz * dz
        p = torch.clamp(s / d2, max=1.0)
        r = tile[(j % W & 63) * 64 + (j // W & 63)]
        xi = (_bitrev32(i) + r) & 0xFFFFFFFF
        assert bool((xi.to(torch.float64) < torch.ceil(p.to(torch.float64) * two32)).all())
        del pc, j, i, e, lt, dx, dy, dz, d2, p, r, xi


def test_frame_scale_sampled_pow2_split(ctx, orc):
    """The frame against the power-of-two hierarchy of its 2^20 lights (every
    node an aligned block): sampled eyes pair for pair against the oracle, and
    every eye's pair fingerprint equal to the radix hierarchy's (the accepted
    set does not depend on the hierarchy) and to the aligned-block closed
    form's on the same hierarchy."""
    import torch
    fr = synth.frame()
    hr = ctx.build_hierarchy(fr["lights"], leaf_size=1)
    hp = ctx.build_hierarchy(fr["lights"], leaf_size=1, split="pow2")
    perm = orc.morton_order(fr["lights"])
    assert np.array_equal(hp.permutation(), perm)
    eyes = _eyes_t(ctx, fr["eyes"])
    n_eyes = fr["eyes"].shape[0]
    n = ctx.count(hr, eyes, fr["s"], fr["width"])
    assert ctx.count(hp, eyes, fr["s"], fr["width"]) == n
    pairs, n1, _ = ctx.traverse(hp, eyes, fr["s"], fr["width"], capacity=n)
    assert n1 == n
    sel = np.unique(np.concatenate([np.arange(7, n_eyes, 4099), [n_eyes - 1]]))
    out = orc.accept_eyes(fr["eyes"], sel, fr["width"], 0, fr["tile"], fr["lights"][perm],
                          fr["s"], lists=True)
    assert np.array_equal(select_pairs_of_eyes(pairs, sel), pair_keys_from_oracle(out, sel))
    f0 = per_eye_fingerprints(pairs, n_eyes)
    del pairs
    torch.cuda.empty_cache()
    for h, method in ((hr, 0), (hp, 4)):
        p2, n2, _ = ctx.traverse(h, eyes, fr["s"], fr["width"], capacity=n, rmq_method=method)
        assert n2 == n
        f2 = per_eye_fingerprints(p2, n_eyes)
        for a, b in zip(f0, f2):
            assert np.array_equal(a, b), method
        del p2
        torch.cuda.empty_cache()
    hr.free()
    hp.free()


def test_frame_scale_multi_sample_sampled(ctx, orc):
    """Section 3's several samples per eye at the benchmark's shape (the first
    270 pixel rows x 4 samples, about one frame of virtual eyes, power-of-two
    hierarchy): sampled eyes, all four samples each, pair for pair against
    the oracle."""
    import torch
    ns, s0 = 4, 0x6A09E667
    fr = synth.frame()
    rows = 1080 // ns
    eyes_np = np.ascontiguousarray(fr["eyes"][:rows * fr["width"]])
    h = ctx.build_hierarchy(fr["lights"], leaf_size=1, split="pow2")
    perm = orc.morton_order(fr["lights"])
    eyes = _eyes_t(ctx, eyes_np)
    n = ctx.count(h, eyes, fr["s"], fr["width"], n_samples=ns, psi_s0=s0)
    pairs, n1, _ = ctx.traverse(h, eyes, fr["s"], fr["width"], capacity=n, n_samples=ns, psi_s0=s0)
    assert n1 == n
    n_eyes = eyes_np.shape[0]
    sel = np.unique(np.concatenate([np.arange(3, n_eyes, 2039), [n_eyes - 1]])).astype(np.uint32)
    out = orc.accept_eyes(eyes_np, sel, fr["width"], 0, fr["tile"], fr["lights"][perm], fr["s"],
                          n_samples=ns, psi_s0=s0, lists=True)
    virt = (sel.astype(np.int64)[:, None] * ns + np.arange(ns)[None, :]).ravel()
    assert np.array_equal(select_pairs_of_eyes(pairs, virt), pair_keys_from_oracle(out, sel, ns))
    del pairs
    torch.cuda.empty_cache()
    h.free()


def test_frame_scale_weights_sampled(ctx, orc):
    """The frame with 1/p weights (power-of-two hierarchy, the benchmark's
    --weights run): sampled eyes pair for pair against the oracle, and the
    weight of every pair of those eyes bit for bit against the oracle's
    correctly rounded reciprocal."""
    import torch
    fr = synth.frame()
    h = ctx.build_hierarchy(fr["lights"], leaf_size=1, split="pow2")
    perm = orc.morton_order(fr["lights"])
    ls = fr["lights"][perm]
    eyes = _eyes_t(ctx, fr["eyes"])
    n_eyes = fr["eyes"].shape[0]
    n = ctx.count(h, eyes, fr["s"], fr["width"])
    pairs, n1, _, w = ctx.traverse(h, eyes, fr["s"], fr["width"], capacity=n, with_weights=True)
    assert n1 == n
    sel = np.unique(np.concatenate([np.arange(11, n_eyes, 8209), [n_eyes - 1]])).astype(np.uint32)
    out = orc.accept_eyes(fr["eyes"], sel, fr["width"], 0, fr["tile"], ls, fr["s"], lists=True)
    # the selected eyes' pairs with their weights, from the huge output in chunks
    sel_t = torch.as_tensor(sel.astype(np.int64), device=pairs.device)
    keys, wts = [], []
    for at in range(0, n, 1 << 27):
        pc = pairs[at:at + (1 << 27)].to(torch.int64) & 0xFFFFFFFF
        m = torch.isin(pc[:, 0], sel_t)
        if m.any():
            keys.append((pc[m, 0] << 32) | pc[m, 1])
            wts.append(w[at:at + (1 << 27)][m])
        del pc, m
    k = torch.cat(keys)
    order = torch.argsort(k)
    k = k[order].cpu().numpy().view(np.uint64)
    wv = torch.cat(wts)[order].cpu().numpy()
    assert np.array_equal(k, pair_keys_from_oracle(out, sel))
    j = (k >> np.uint64(32)).astype(np.int64)
    i = (k & np.uint64(0xFFFFFFFF)).astype(np.int64)
    for q in range(k.size):
        assert np.float32(wv[q]) == np.float32(orc.accept_weight(fr["eyes"][j[q]], ls[i[q]], fr["s"])), q
    del pairs, w
    torch.cuda.empty_cache()
    h.free()


def test_frame_scale_sampled(ctx, orc):
    """1920x1080 eyes against 2^20 Gaussian-mixture lights in one launch (the
    benchmark shape); sampled eyes compared pair for pair with the oracle,
    every emitted pair checked against its own test, and every eye's
    fingerprint (count and two 64-bit hash sums of its lights) identical
    between the paper's method, the O(1) ablation and the aligned-block
    closed form (a separate range-minimum implementation)."""
    import torch
    fr = synth.frame()
    h = ctx.build_hierarchy(fr["lights"], leaf_size=1)
    perm = orc.morton_order(fr["lights"])
    assert np.array_equal(h.permutation(), perm)
    eyes = _eyes_t(ctx, fr["eyes"])
    n_eyes = fr["eyes"].shape[0]
    n = ctx.count(h, eyes, fr["s"], fr["width"])
    pairs, n1, _ = ctx.traverse(h, eyes, fr["s"], fr["width"], capacity=n)
    assert n1 == n
    sel = np.unique(np.concatenate([np.arange(0, n_eyes, 1021), [n_eyes - 1]]))
    out = orc.accept_eyes(fr["eyes"], sel, fr["width"], 0, fr["tile"], fr["lights"][perm],
                          fr["s"], lists=True)
    assert np.array_equal(select_pairs_of_eyes(pairs, sel), pair_keys_from_oracle(out, sel))
    f0 = per_eye_fingerprints(pairs, n_eyes)
    assert int(f0[0].sum()) == n
    assert np.array_equal(f0[0][sel], out["count"].astype(np.int64))
    _assert_every_pair_passes_its_test(pairs, fr, perm)
    del pairs
    torch.cuda.empty_cache()
    for method in (1, 4):
        p2, n2, _ = ctx.traverse(h, eyes, fr["s"], fr["width"], capacity=n, rmq_method=method)
        assert n2 == n
        f2 = per_eye_fingerprints(p2, n_eyes)
        for a, b in zip(f0, f2):
            assert np.array_equal(a, b), method
        del p2
        torch.cuda.empty_cache()
    h.free()
