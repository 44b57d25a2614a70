"""Pins of the CPU oracle to facts fixed by the paper and by mathematics.

Each test checks the oracle against something other than itself: values the
paper prints (tests/golden/), closed forms, textbook special cases, exact
counting properties, or an independent computation (string-based bit
reversal, trailing-zero scans).  None of these tests uses the GPU.
"""
import math
import os
from fractions import Fraction

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
M32 = (1 << 32) - 1


def _rows(name):
    out = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if line:
                out.append(line.split())
    return out


def _kv(name):
    return {k: int(v, 0) for k, v in _rows(name)}


def _rev_str(i, B):
    """Bit reversal through a string: an independent way to get Phi_2."""
    return int(format(i, "0%db" % B)[::-1], 2)


def _ctz(x):
    return (x & -x).bit_length() - 1


# -- radical inverse -----------------------------------------------------------

def test_van_der_corput_fixture(orc):
    for i, num, den in _rows("van_der_corput.txt"):
        i, num, den = int(i), int(num), int(den)
        for B in (4, 8, 16, 32):
            assert Fraction(orc.bitrev(i, B), 1 << B) == Fraction(num, den)


def test_bitrev_matches_string_reversal(orc):
    rng = np.random.default_rng(7)
    for B in (1, 5, 13, 32):
        for i in rng.integers(0, 1 << B, size=200):
            assert orc.bitrev(int(i), B) == _rev_str(int(i), B)


def test_radical_inverse_shift_identity(orc):
    # Section 4: Phi_2(l + n 2^d) = 2^-d Phi_2(n) + Phi_2(l) for l < 2^d,
    # exact in 32-bit fixed point while n < 2^(32-d).
    rng = np.random.default_rng(11)
    for d in range(0, 32):
        for _ in range(20):
            l = int(rng.integers(0, 1 << d)) if d else 0
            n = int(rng.integers(0, 1 << (32 - d)))
            lhs = orc.bitrev(l + (n << d), 32)
            rhs = (orc.bitrev(n, 32) >> d) + orc.bitrev(l, 32)
            assert lhs == rhs


def test_shifted_sequence_is_a_bijection(orc):
    rng = np.random.default_rng(3)
    for B in range(1, 11):
        for r in (0, 1, (1 << B) - 1, int(rng.integers(0, 1 << B))):
            vals = sorted(orc.phi(i, r, B) for i in range(1 << B))
            assert vals == list(range(1 << B))


# -- range minimum --------------------------------------------------------------

def test_paper_worked_query(orc):
    g = _kv("paper_worked_query.txt")
    B = g["B"]
    # r follows from k_r = Phi_2^{-1}(1 - r)
    R = ((1 << B) - orc.bitrev(g["k_r"], B)) % (1 << B)
    assert R == g["R"]
    k, v = orc.rmq_scan_one(g["a"], g["b"], R, B)
    assert k & 1 == g["argmin_low_bit"]
    assert (k, v) == (g["argmin"], g["min"])


def test_zero_at_kr(orc):
    # Section 2, first case: if k_r = Phi_2^{-1}(1 - r) lies in [a,b) the
    # minimum is 0 and is taken at k_r.
    rng = np.random.default_rng(5)
    for _ in range(300):
        a = int(rng.integers(0, M32 - 5000))
        b = a + int(rng.integers(1, 4000))
        k = int(rng.integers(a, b))
        R = (-orc.bitrev(k, 32)) & M32
        assert orc.rmq_scan_one(a, b, R, 32) == (k, 0)
    B = 6
    for a in range(0, 1 << B):
        for b in range(a + 1, (1 << B) + 1):
            for k in (a, b - 1, (a + b) // 2):
                R = (-orc.bitrev(k, B)) % (1 << B)
                assert orc.rmq_scan_one(a, b, R, B) == (k, 0)


def test_unshifted_minimum_has_most_trailing_zeros(orc):
    # Section 2 (Algorithm 1's problem): with no shift, the argmin is the
    # number in [a,b) with the most trailing zeros (0 if a == 0).
    def most_tz(a, b):
        if a == 0:
            return 0
        return max(range(a, b), key=_ctz)

    B = 7
    for a in range(0, 1 << B):
        for b in range(a + 1, (1 << B) + 1):
            assert orc.rmq_scan_one(a, b, 0, B)[0] == most_tz(a, b)
    rng = np.random.default_rng(9)
    for _ in range(200):
        a = int(rng.integers(1, M32 - 3000))
        b = a + int(rng.integers(1, 2048))
        assert orc.rmq_scan_one(a, b, 0, 32)[0] == most_tz(a, b)


def test_scan_against_independent_brute(orc):
    rng = np.random.default_rng(13)
    for _ in range(150):
        B = int(rng.integers(1, 33))
        a = int(rng.integers(0, (1 << B) - 1))
        b = min(a + int(rng.integers(1, 300)), 1 << B)
        r = int(rng.integers(0, 1 << B))
        vals = [(_rev_str(i, B) + r) % (1 << B) for i in range(a, b)]
        j = int(np.argmin(vals))
        assert orc.rmq_scan_one(a, b, r, B) == (a + j, vals[j])


def test_single_element_and_empty_ranges(orc):
    rng = np.random.default_rng(17)
    for _ in range(100):
        a = int(rng.integers(0, M32))
        r = int(rng.integers(0, M32 + 1))
        assert orc.rmq_scan_one(a, a + 1, r, 32) == (a, (_rev_str(a, 32) + r) & M32)
        assert orc.rmq_scan_one(a, a, r, 32) == (a, M32)
        assert orc.rmq_dyadic_one(a, a, r, 32) == (a, M32)


def test_dyadic_equals_scan_exhaustive_small_words(orc):
    for B in range(1, 8):
        n = 1 << B
        a, b = np.triu_indices(n + 1, k=1)
        keep = a < n
        a, b = a[keep], b[keep]
        a = np.repeat(a, n).astype(np.uint32)
        b = np.repeat(b, n).astype(np.uint32)
        r = np.tile(np.arange(n), a.size // n).astype(np.uint32)
        k1, v1 = orc.rmq_scan(a, b, r, B=B)
        k2, v2 = orc.rmq_dyadic(a, b, r, B=B)
        assert np.array_equal(k1, k2) and np.array_equal(v1, v2), B


def test_dyadic_equals_scan_32bit(orc):
    rng = np.random.default_rng(19)
    n = 4000
    a = rng.integers(0, M32 - (1 << 13), size=n, dtype=np.uint64)
    a[:200] = rng.integers(0, 64, size=200)
    a[200:400] = M32 - (1 << 13) - rng.integers(0, 64, size=200)
    ln = rng.integers(1, 1 << 13, size=n, dtype=np.uint64)
    b = (a + ln).astype(np.uint32)
    a = a.astype(np.uint32)
    r = rng.integers(0, 1 << 32, size=n, dtype=np.uint64).astype(np.uint32)
    r[:50] = 0
    r[50:100] = M32
    k1, v1 = orc.rmq_scan(a, b, r)
    k2, v2 = orc.rmq_dyadic(a, b, r)
    assert np.array_equal(k1, k2) and np.array_equal(v1, v2)


# -- light order ----------------------------------------------------------------

def test_morton_octant_fixture(orc):
    for cx, cy, cz, code in _rows("morton_octants.txt"):
        pt = [(int(c) + 0.5) / (1 << 21) for c in (cx, cy, cz)]
        assert orc.morton(*pt) == int(code)


def test_morton_order_is_z_order_with_stable_ties(orc):
    rows = _rows("morton_octants.txt")[:8]
    pts = np.array([[(int(c) + 0.5) / 2.0 for c in r[:3]] for r in rows],
                   np.float32)  # the eight octant centres, in Z order
    rng = np.random.default_rng(23)
    shuffle = rng.permutation(8)
    dup = np.concatenate([pts[shuffle], pts[shuffle]])
    perm = orc.morton_order(dup)
    # expected: octants in Z order; each octant's two copies by original index
    inv = np.argsort(shuffle)
    exp = []
    for z in range(8):
        exp += [inv[z], inv[z] + 8]
    assert perm.tolist() == exp


def test_morton_clamps_outside_unit_cube(orc):
    assert orc.morton(-3.0, -0.0, -1e-30) == 0
    assert orc.morton(2.0, 5.0, 1.0) == (1 << 63) - 1
    box = np.array([-1, -1, -1, 1, 1, 1], np.float32)
    assert orc.morton(0.0, 0.0, 0.0, box) == orc.morton(0.5, 0.5, 0.5)


# -- shifts ------------------------------------------------------------------------

def test_tile_lookup_fixture(orc):
    tile = np.arange(4096, dtype=np.uint32)
    for W, j, e in _rows("tile_lookup.txt"):
        assert orc.eye_shift(tile, int(j), int(W)) == int(e)
        assert orc.eye_shift(tile, int(j), int(W), M32) == (int(e) - 1) & M32


def test_golden_alpha_is_rounded_inverse_golden_ratio(orc):
    # 2^32 / phi = 2^31 (sqrt 5 - 1); bracket sqrt(5) * 2^80 with integers
    s = math.isqrt(5 << 160)
    lo = Fraction(s, 1 << 80)
    hi = Fraction(s + 1, 1 << 80)
    exact_lo = (lo - 1) * (1 << 31)
    exact_hi = (hi - 1) * (1 << 31)
    a = orc.golden_alpha()
    assert abs(Fraction(a) - exact_lo) <= Fraction(1, 2)
    assert abs(Fraction(a) - exact_hi) <= Fraction(1, 2)


def test_psi_three_gap_theorem(orc):
    # Section 3's lattice psi(n) = s + n alpha mod 1: any N points of a
    # rotation on the circle split it into gaps of at most three lengths.
    for s0 in (0, 12345, M32):
        for N in (2, 3, 5, 8, 13, 100, 987, 1000):
            pts = sorted(orc.psi(n, s0) for n in range(N))
            gaps = {(pts[(t + 1) % N] - pts[t]) % (1 << 32) for t in range(N)}
            assert len(gaps) <= 3
        assert orc.psi(0, s0) == s0
        assert orc.psi(1, s0) == (s0 + orc.golden_alpha()) & M32


# -- acceptance test -----------------------------------------------------------

def test_accept_prob_exact_cases(orc):
    e = [0.0, 0.0, 0.0]
    assert orc.accept_prob(e, [0.5, 0.0, 0.0], 0.0625) == 0.25
    assert orc.accept_prob(e, [0.0, -0.5, 0.0], 0.0625) == 0.25
    assert orc.accept_prob(e, [0.0, 0.0, 0.5], 0.0625) == 0.25
    assert orc.accept_prob(e, [0.5, 0.5, 0.0], 0.125) == 0.25
    assert orc.accept_prob(e, [0.5, 0.5, 0.5], 0.1875) == 0.25
    assert orc.accept_prob(e, e, 1e-4) == 1.0          # d = 0
    assert orc.accept_prob(e, [0.25, 0, 0], 0.0625) == 1.0   # s = d^2
    assert orc.accept_prob(e, [0.25, 0, 0], 0.125) == 1.0    # s > d^2


def test_accept_threshold_reading(orc):
    e = [0.0, 0.0, 0.0]
    l = [0.5, 0.0, 0.0]
    # p = 1/4: keep xi / 2^32 < 1/4
    assert orc.accept(e, l, 0.0625, (1 << 30) - 1)
    assert not orc.accept(e, l, 0.0625, 1 << 30)
    # p = 1 keeps every xi
    assert orc.accept(e, e, 1.0, M32)
    # p * 2^32 not an integer: p = 5 * 2^-33 keeps xi in {0, 1, 2}
    l1 = [1.0, 0.0, 0.0]
    s = 5.0 * 2.0 ** -33
    assert [orc.accept(e, l1, s, x) for x in range(5)] == [True, True, True,
                                                           False, False]
    s = 3.0 * 2.0 ** -35   # p * 2^32 = 3/8: only xi = 0
    assert [orc.accept(e, l1, s, x) for x in range(3)] == [True, False, False]


def _round_binary32(x):
    """Round a positive Fraction to the nearest IEEE binary32 value, ties to
    even (normal range only), with exact rational arithmetic: an independent
    way to get a correctly rounded reciprocal."""
    assert x > 0
    e = x.numerator.bit_length() - x.denominator.bit_length()
    if Fraction(2) ** e > x:
        e -= 1
    assert Fraction(2) ** e <= x < Fraction(2) ** (e + 1)
    m = x / Fraction(2) ** (e - 23)            # in [2^23, 2^24)
    n = m.numerator // m.denominator
    rem = m - n
    if rem > Fraction(1, 2) or (rem == Fraction(1, 2) and n % 2 == 1):
        n += 1
    if n == 1 << 24:
        n, e = 1 << 23, e + 1
    assert -126 <= e <= 127
    return float(Fraction(n) * Fraction(2) ** (e - 23))


def test_accept_weight_pins(orc):
    """The roulette weight 1/p of a kept pair (Section 1: a pair survives with
    probability p and is reweighted by its inverse): exact powers of two,
    p = 1 for d^2 <= s (weight 1, never above p's clamp), a hand-checked
    non-representable case, and random pairs against an exact rational
    reciprocal rounded to binary32 by an independent routine."""
    e = [0.0, 0.0, 0.0]
    l1 = [1.0, 0.0, 0.0]
    for k in range(0, 60):
        assert orc.accept_weight(e, l1, 2.0 ** -k) == 2.0 ** k
    # p clamped to 1: d = 0, d^2 = s, d^2 < s
    assert orc.accept_weight(e, e, 1e-4) == 1.0
    assert orc.accept_weight(e, [0.25, 0.0, 0.0], 0.0625) == 1.0
    assert orc.accept_weight(e, [0.25, 0.0, 0.0], 3.0) == 1.0
    # p = 3/4: 1/p = 4/3 is not a binary32 value; the nearest is 0x3FAAAAAB
    w = orc.accept_weight(e, l1, 0.75)
    assert np.float32(w).view(np.uint32) == 0x3FAAAAAB
    assert _round_binary32(Fraction(4, 3)) == w
    # random pairs: weight == RN32(1 / p) exactly, p the oracle's own binary32 p
    rng = np.random.default_rng(41)
    diffs = 0
    for _ in range(3000):
        ev = rng.random(3, dtype=np.float32)
        lv = rng.random(3, dtype=np.float32)
        s = float(np.float32(10.0 ** rng.uniform(-7, 0)))
        p = orc.accept_prob(ev, lv, s)
        w = orc.accept_weight(ev, lv, s)
        assert w == _round_binary32(1 / Fraction(p)), (ev, lv, s, p, w)
        # a reciprocal of the margin-inflated bound would differ
        infl = float(np.float32(np.float32(p) * np.float32(1.0 + 2.0 ** -20)))
        if p < 1.0 and _round_binary32(1 / Fraction(infl)) != w:
            diffs += 1
    assert diffs > 2500


def _single_eye(orc, light, n_l, s, R):
    tile = np.full(4096, R, np.uint32)
    eyes = np.zeros((1, 3), np.float32)
    lights = np.tile(np.asarray(light, np.float32), (n_l, 1))
    return orc.accept_eyes(eyes, [0], 64, 0, tile, lights, s, lists=True)


def test_stratified_count_is_exact(orc):
    # 2^m copies of one light, p = 2^-k: the shifted van der Corput points
    # i < 2^m are a lattice of step 2^(32-m), so exactly 2^(m-k) of them fall
    # below p whatever the shift.
    for m in (4, 8, 11):
        for k in range(0, m + 1):
            for R in (0, 1, 1 << 31, M32, 0x9E3779B9):
                out = _single_eye(orc, [1.0, 0.0, 0.0], 1 << m, 2.0 ** -k, R)
                assert int(out["count"][0]) == 1 << (m - k)


def test_stratified_count_any_probability(orc):
    # general p: the count is floor or ceil of N * T / 2^32, T = ceil(p 2^32)
    rng = np.random.default_rng(29)
    for _ in range(40):
        m = int(rng.integers(3, 12))
        s = float(np.float32(rng.uniform(0.001, 0.99)))
        R = int(rng.integers(0, 1 << 32))
        out = _single_eye(orc, [1.0, 0.0, 0.0], 1 << m, s, R)
        T = math.ceil(Fraction(float(np.float32(s))) * (1 << 32))
        q = Fraction(T * (1 << m), 1 << 32)
        assert math.floor(q) <= int(out["count"][0]) <= math.ceil(q)
        # and the listed indices are exactly those whose xi is below T
        xi = [(orc.bitrev(i, 32) + R) & M32 for i in range(1 << m)]
        assert out["idx"].tolist() == [i for i in range(1 << m) if xi[i] < T]


def test_accepted_sets_grow_with_s(orc):
    rng = np.random.default_rng(31)
    eyes = rng.random((8, 3), dtype=np.float32)
    lights = rng.random((300, 3), dtype=np.float32)
    tile = (rng.permutation(4096).astype(np.uint32) << np.uint32(20))
    prev = None
    for s in (1e-4, 1e-3, 1e-2, 1e-1, 10.0):
        out = orc.accept_eyes(eyes, np.arange(8), 4, 0, tile, lights, s,
                              lists=True)
        sets = [set(out["idx"][out["offsets"][q]:out["offsets"][q + 1]].tolist())
                for q in range(8)]
        if prev is not None:
            assert all(p <= c for p, c in zip(prev, sets))
        prev = sets
    assert all(len(c) == 300 for c in prev)   # s = 10 > every d^2 <= 3


def test_fingerprint_hash_reference_vector(orc):
    # SplitMix64 (Steele, Lea, Flood 2014): first output for seed 0.
    assert orc.fingerprint_hash(0) == 0xE220A8397B1DCDAF


def test_multi_sample_uses_extra_rotation(orc):
    # Section 3: sample n is the one-sample problem with shift r + psi(n).
    rng = np.random.default_rng(37)
    eyes = rng.random((3, 3), dtype=np.float32)
    lights = rng.random((200, 3), dtype=np.float32)
    tile = (rng.permutation(4096).astype(np.uint32) << np.uint32(20))
    multi = orc.accept_eyes(eyes, np.arange(3), 2, 0, tile, lights, 0.01,
                            n_samples=4, psi_s0=99, lists=True)
    for n in range(4):
        one = orc.accept_eyes(eyes, np.arange(3), 2, orc.psi(n, 99), tile,
                              lights, 0.01, lists=True)
        for q in range(3):
            a, b = multi["offsets"][q], multi["offsets"][q + 1]
            got = multi["idx"][a:b][multi["sample"][a:b] == n]
            exp = one["idx"][one["offsets"][q]:one["offsets"][q + 1]]
            assert got.tolist() == exp.tolist()
