"""GPU hierarchy build: the same hierarchy as the host builder, record for
record (order, splits, exact fp32 boxes, record numbering), and traversals
on it equal the all-pairs oracle."""
import numpy as np
import pytest

import synth
from _helpers import pair_keys_from_gpu, pair_keys_from_oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hrr():
    import paper_1907_12343_amd as m
    return m


@pytest.fixture(scope="module")
def ctx(hrr):
    c = hrr.Context(synth.dither_tile(100))
    yield c
    c.close()


def _dev(ctx, a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, np.float32).reshape(-1, 3)).to(ctx.torch_device)


def _same(h_host, h_dev):
    assert (h_host.n_lights, h_host.leaf_size, h_host.n_nodes, h_host.depth) == \
        (h_dev.n_lights, h_dev.leaf_size, h_dev.n_nodes, h_dev.depth)
    assert np.array_equal(np.array(h_host.box, np.float32).view(np.uint32),
                          np.array(h_dev.box, np.float32).view(np.uint32))
    assert np.array_equal(h_host.permutation(), h_dev.permutation())
    assert np.array_equal(h_host.sorted_lights().view(np.uint32), h_dev.sorted_lights().view(np.uint32))
    rh, rd = h_host.records(), h_dev.records()
    assert rh.tobytes() == rd.tobytes()


def _cases():
    rng = np.random.default_rng(11)
    cases = {
        "one": rng.random((1, 3)),
        "two": rng.random((2, 3)),
        "seven": rng.random((7, 3)),
        "uniform_1000": rng.random((1000, 3)),
        "tiny": synth.tiny()["lights"],
        "mixture_70k": synth.mixture_points(70000, synth.mixture_centers(12), 13),
        "coincident": np.repeat(rng.random((9, 3)), 37, axis=0),
        "signed_zeros": np.array([[0.0, -0.0, 0.5], [-0.0, 0.0, 0.5], [0.25, 0.0, -0.0],
                                  [0.0, 0.0, 0.0], [-0.0, -0.0, -0.0]] * 7),
        "outside_box": rng.normal(0.5, 1.0, (3000, 3)),
    }
    return {k: np.ascontiguousarray(v, np.float32) for k, v in cases.items()}


@pytest.mark.parametrize("split", ["radix", "pow2"])
@pytest.mark.parametrize("leaf", [1, 2, 4, 8])
def test_device_build_equals_host_build(ctx, leaf, split):
    for name, lights in _cases().items():
        hh = ctx.build_hierarchy(lights, leaf_size=leaf, split=split)
        hd = ctx.build_hierarchy_device(_dev(ctx, lights), leaf_size=leaf, split=split)
        assert hh.split == hd.split == split
        try:
            _same(hh, hd)
        except AssertionError as ex:
            raise AssertionError("case %s leaf %d %s: %s" % (name, leaf, split, ex))
        hh.free()
        hd.free()


def test_device_build_with_a_box_and_empty(ctx):
    rng = np.random.default_rng(12)
    lights = (rng.random((5000, 3)) * 4.0 - 1.0).astype(np.float32)
    box = np.array([-1, -1, -1, 3, 3, 3], np.float32)
    hh = ctx.build_hierarchy(lights, leaf_size=1, box=box)
    hd = ctx.build_hierarchy_device(_dev(ctx, lights), leaf_size=1, box=box)
    _same(hh, hd)
    e0 = ctx.build_hierarchy_device(_dev(ctx, np.zeros((0, 3), np.float32)))
    assert e0.n_lights == 0 and e0.n_nodes == 0
    for h in (hh, hd, e0):
        h.free()


@pytest.mark.parametrize("split", ["radix", "pow2"])
def test_device_build_frame_scale(ctx, split):
    fr = synth.frame()
    hh = ctx.build_hierarchy(fr["lights"], leaf_size=1, split=split)
    hd = ctx.build_hierarchy_device(_dev(ctx, fr["lights"]), leaf_size=1, split=split)
    _same(hh, hd)
    hh.free()
    hd.free()


@pytest.mark.parametrize("split", ["radix", "pow2"])
def test_device_build_largest_served_hierarchy(ctx, split):
    """The served workload's largest hierarchy (2^22 lights of a Gaussian
    mixture, radix depth about 40, many single-internal-child nodes): record
    for record equal to the host build, holes of the sibling pairs included."""
    sc = synth.served_hierarchy(15)
    assert sc["lights"].shape[0] == 1 << 22
    hh = ctx.build_hierarchy(sc["lights"], leaf_size=1, split=split)
    hd = ctx.build_hierarchy_device(_dev(ctx, sc["lights"]), leaf_size=1, split=split)
    _same(hh, hd)
    if split == "pow2":
        assert hh.n_nodes == 1 << 22   # a perfect tree fills every pair
    hh.free()
    hd.free()


def test_device_build_rejects_bad_input(ctx, hrr):
    bad = np.random.default_rng(13).random((100, 3)).astype(np.float32)
    bad[57, 2] = np.inf
    with pytest.raises(hrr.HrrError) as ei:
        ctx.build_hierarchy_device(_dev(ctx, bad))
    assert ei.value.status == hrr.HRR_E_INVALID
    with pytest.raises(hrr.HrrError):
        ctx.build_hierarchy_device(_dev(ctx, bad[:10]), leaf_size=0)
    for arg in (0x200 | 1, 0x100, 9 | 0x100, 1 << 31):   # unknown flag bits, leaf size 0 or 9
        with pytest.raises(hrr.HrrError):
            ctx.build_hierarchy_device(_dev(ctx, bad[:10]), leaf_size=arg)
        with pytest.raises(hrr.HrrError):
            ctx.build_hierarchy(bad[:10], leaf_size=arg)


def test_traversal_on_device_built_hierarchy(ctx, orc):
    t = synth.tiny()
    hd = ctx.build_hierarchy_device(_dev(ctx, t["lights"]), leaf_size=1)
    pairs, n, _ = ctx.traverse_all(hd, _dev(ctx, t["eyes"]), t["s"], t["width"])
    ls = t["lights"][orc.morton_order(t["lights"])]
    sel = np.arange(t["eyes"].shape[0])
    out = orc.accept_eyes(t["eyes"], sel, t["width"], 0, t["tile"], ls, t["s"], lists=True)
    assert np.array_equal(pair_keys_from_gpu(pairs), pair_keys_from_oracle(out, sel))
    hd.free()
