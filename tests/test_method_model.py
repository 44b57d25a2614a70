"""Exhaustive check, on tiny inputs, that hierarchical culling is exact.

A plain Python model of hierarchical Russian roulette (Section 1 of the
paper): lights in sequence order, every binary hierarchy whose nodes are
contiguous index ranges, a node culled when the minimum of its eye's rotated
sequence over the node's range (the paper's v(a,b), here from the oracle's
scan) is not below the node's acceptance bound.  The node bound is built from
the node's fp32 bounding box the way the GPU path builds it (per-axis
distance to the box, same summation order, same rounding, times 1 + 2^-20).

For every hierarchy shape and leaf size the culled traversal must return
exactly the all-pairs set of the oracle.  This pins the argument that lets
the GPU path be bit-exact: every fp32 step of the box bound is monotone, so
the bound can never fall below the bound of a light inside the box.
"""
import itertools

import numpy as np
import pytest

F = np.float32
MARGIN = F(1.0) + F(2.0 ** -20)


def _threshold(p):
    """Smallest integer xi that is rejected: ceil(p * 2^32), or 2^32."""
    if p >= F(1.0):
        return 1 << 32
    t = float(p * F(4294967296.0))
    return int(np.ceil(t))


def _node_bound(e, lo, hi, s):
    d = [max(max(F(lo[k] - e[k]), F(e[k] - hi[k])), F(0.0)) for k in range(3)]
    d2 = F(F(F(d[0] * d[0]) + F(d[1] * d[1])) + F(d[2] * d[2]))
    with np.errstate(divide="ignore"):
        q = F(F(s) / d2)
    q = F(q * MARGIN)
    return _threshold(min(q, F(1.0)))


def _trees(a, b, leaf):
    """Every binary hierarchy over [a,b) with leaves of at most ``leaf``."""
    if b - a <= leaf:
        yield ("leaf", a, b)
        return
    for c in range(a + 1, b):
        for left in _trees(a, c, leaf):
            for right in _trees(c, b, leaf):
                yield ("node", a, b, left, right)


def _traverse(tree, e, R, lights, s, orc):
    out = []
    stack = [tree]
    while stack:
        t = stack.pop()
        a, b = t[1], t[2]
        k, v = orc.rmq_scan_one(a, b, R, 32)
        lo = lights[a:b].min(axis=0)
        hi = lights[a:b].max(axis=0)
        if v >= _node_bound(e, lo, hi, s):
            continue
        if t[0] == "leaf":
            for i in range(a, b):
                xi = orc.phi(i, R, 32)
                if orc.accept(e, lights[i], s, xi):
                    out.append(i)
        else:
            stack.append(t[3])
            stack.append(t[4])
    return sorted(out)


@pytest.mark.parametrize("n_l,leaf", [(5, 1), (6, 1), (7, 2), (8, 3), (6, 4)])
def test_every_hierarchy_returns_the_all_pairs_set(orc, n_l, leaf):
    rng = np.random.default_rng(1000 + n_l * 10 + leaf)
    lights = rng.random((n_l, 3), dtype=np.float32)
    lights = lights[orc.morton_order(lights)]
    eyes = rng.random((3, 3), dtype=np.float32)
    eyes[0] = lights[n_l // 2]                  # an eye on top of a light
    shifts = [0, 1, 1 << 31, (1 << 32) - 1, int(rng.integers(0, 1 << 32))]
    trees = list(_trees(0, n_l, leaf))
    assert len(trees) > 1
    for s in (0.02, 0.2):
        for e in eyes:
            for R in shifts:
                want = [i for i in range(n_l)
                        if orc.accept(e, lights[i], s, orc.phi(i, R, 32))]
                for t in trees:
                    assert _traverse(t, e, R, lights, s, orc) == want


def test_margin_never_needed_for_exactness(orc):
    # Sanity of the monotonicity argument without the 1 + 2^-20 factor: for
    # a point box the node bound equals the leaf threshold bit for bit.
    rng = np.random.default_rng(77)
    for _ in range(2000):
        e = rng.random(3, dtype=np.float32)
        l = rng.random(3, dtype=np.float32)
        s = F(10.0 ** rng.uniform(-5, 0))
        d = [max(max(F(l[k] - e[k]), F(e[k] - l[k])), F(0.0)) for k in range(3)]
        d2 = F(F(F(d[0] * d[0]) + F(d[1] * d[1])) + F(d[2] * d[2]))
        with np.errstate(divide="ignore"):
            p = min(F(s / d2), F(1.0))
        assert p == F(orc.accept_prob(e, l, float(s)))
