"""CPU-only checks of the library boundary and its host-side logic.

* libhrr.so loads and exports every function include/hrr.h declares, and the
  Python binding declares exactly those (no GPU call is made).
* The host hierarchy builder (compiled here for the CPU, with no HIP) orders
  lights exactly like the oracle's own Morton sort and produces a valid
  hierarchy: children partition their parent's range at the radix split, the
  boxes are the exact bounds of their lights, records sit in sibling pairs.
"""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hrr.h")
LIB = os.path.join(ROOT, "paper_1907_12343_amd", "libhrr.so")
CSRC = os.path.join(ROOT, "paper_1907_12343_amd", "csrc")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    names = set(re.findall(r"\b(hrr_[a-z0-9_]+)\s*\(", txt))
    return names


def test_header_declares_the_boundary():
    names = _declared()
    for must in ("hrr_build_hierarchy", "hrr_range_min", "hrr_traverse", "hrr_submit", "hrr_poll",
                 "hrr_traverse_batched", "hrr_autotune", "hrr_release"):
        assert must in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libhrr.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in sorted(_declared()) if not hasattr(lib, n)]
    assert not missing, missing
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True).stdout
    exported = {ln.split()[-1] for ln in out.splitlines() if " T " in ln}
    public = {n for n in exported if n.startswith("hrr_")}
    assert public == _declared(), public ^ _declared()


def test_binding_constants_equal_the_header():
    """Status codes, range-minimum methods, split rules and launch flags of
    the Python binding are the values include/hrr.h defines."""
    import paper_1907_12343_amd as hrr
    text = open(HEADER).read()
    defines = {m.group(1): int(m.group(2), 0)
               for m in re.finditer(r"#define (HRR_\w+) (0x[0-9a-fA-F]+|\d+)u", text)}
    enum = {m.group(1): int(m.group(2)) for m in re.finditer(r"(HRR_(?:OK|E_\w+)) = (\d+)", text)}
    pairs = {"HRR_RMQ_PAPER": hrr.RMQ_PAPER, "HRR_RMQ_DIRECT": hrr.RMQ_DIRECT,
             "HRR_RMQ_PAPER_FULL": hrr.RMQ_PAPER_FULL, "HRR_RMQ_PAPER_LOOP": hrr.RMQ_PAPER_LOOP,
             "HRR_RMQ_DYADIC": hrr.RMQ_DYADIC, "HRR_RMQ_PAPER_NO_REUSE": hrr.RMQ_PAPER_NO_REUSE,
             "HRR_SPLIT_RADIX": hrr.SPLIT_RADIX, "HRR_SPLIT_POW2": hrr.SPLIT_POW2,
             "HRR_F_STATS": hrr.F_STATS, "HRR_F_NO_REORDER": hrr.F_NO_REORDER,
             "HRR_F_TIMING": hrr.F_TIMING}
    for name, value in pairs.items():
        assert defines[name] == value, name
    for name in ("HRR_OK", "HRR_E_INVALID", "HRR_E_NOMEM", "HRR_E_OVERFLOW", "HRR_E_DEVICE",
                 "HRR_E_NOTREADY", "HRR_E_CANCELLED", "HRR_E_BUSY"):
        assert enum[name] == getattr(hrr, name), name


def test_binding_signatures_cover_the_header():
    import importlib.util
    spec = importlib.util.spec_from_file_location(
        "hrr_binding_probe", os.path.join(ROOT, "paper_1907_12343_amd", "__init__.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    assert set(mod.SIGNATURES) == _declared()


HARNESS = r"""
#include <cstdio>
#include <cstdlib>
#include <vector>
#include "hrr_build.hpp"
// reads: n leaf pow2 then 3n floats on stdin; writes perm, then nodes, then depth
int main() {
    unsigned n, leaf, pow2;
    if (scanf("%u %u %u", &n, &leaf, &pow2) != 3) return 2;
    std::vector<float> xyz(3 * (size_t)n);
    for (auto& v : xyz) if (scanf("%a", &v) != 1) return 3;
    hrr::HostHierarchy H;
    if (!hrr::build_hierarchy(xyz.data(), n, leaf, pow2 != 0, nullptr, H)) return 4;
    printf("%zu %u\n", H.nodes.size(), H.depth);
    for (unsigned i = 0; i < n; ++i) printf("%u\n", H.perm[i]);
    for (auto& d : H.nodes) {
        printf("%u %u %u %u", d.a, d.c, d.b, d.first);
        for (int k = 0; k < 3; ++k) printf(" %a %a %a %a", d.lo_l[k], d.hi_l[k], d.lo_r[k], d.hi_r[k]);
        printf("\n");
    }
    return 0;
}
"""


@pytest.fixture(scope="module")
def build_harness(tmp_path_factory):
    d = tmp_path_factory.mktemp("host_build")
    src = d / "harness.cpp"
    src.write_text(HARNESS)
    exe = d / "harness"
    cxx = "/opt/rocm/llvm/bin/clang++" if os.path.exists("/opt/rocm/llvm/bin/clang++") else "g++"
    subprocess.run([cxx, "-O1", "-std=c++17", "-ffp-contract=off", "-I", CSRC, str(src),
                    os.path.join(CSRC, "hrr_build.cpp"), "-o", str(exe)], check=True)
    return str(exe)


def _run_builder(exe, lights, leaf, pow2=False):
    inp = "%d %d %d\n" % (lights.shape[0], leaf, int(pow2)) + "\n".join(
        " ".join(float(v).hex() for v in row) for row in lights) + "\n"
    out = subprocess.run([exe], input=inp, capture_output=True, text=True, check=True).stdout
    lines = out.splitlines()
    n_nodes, depth = map(int, lines[0].split())
    n = lights.shape[0]
    perm = np.array([int(x) for x in lines[1:1 + n]], np.uint32)
    nodes = []
    for ln in lines[1 + n:1 + n + n_nodes]:
        f = ln.split()
        a, c, b, first = (int(x) for x in f[:4])
        vals = [float.fromhex(x) for x in f[4:]]
        lo_l = vals[0::4]; hi_l = vals[1::4]; lo_r = vals[2::4]; hi_r = vals[3::4]
        nodes.append((a, c, b, first, lo_l, hi_l, lo_r, hi_r))
    return perm, nodes, depth


@pytest.mark.parametrize("pow2", [False, True])
@pytest.mark.parametrize("n,leaf,seed", [(1, 1, 1), (2, 1, 2), (300, 1, 3), (300, 3, 4),
                                         (1000, 8, 5), (64, 2, 6), (1024, 1, 7)])
def test_host_builder_matches_oracle_order_and_is_valid(orc, build_harness, n, leaf, seed, pow2):
    """Order = the oracle's Morton order; every split follows its rule (radix:
    the highest differing code bit, midpoint for equal codes; power of two:
    the left child holds the largest power of two below the length); exact
    child boxes; sibling-pair records (a node with an internal child owns
    the aligned pair first, first + 1, pairs in preorder of their owners,
    unused slots all zero); the recorded depth."""
    if seed == 6:   # many coincident lights: equal codes split at the midpoint
        lights = np.repeat(synth.uniform_points(8, seed), 8, axis=0)
    else:
        lights = synth.mixture_points(n, synth.mixture_centers(seed), seed + 100)
    perm, nodes, depth = _run_builder(build_harness, lights, leaf, pow2)
    assert np.array_equal(perm, orc.morton_order(lights))
    ls = lights[perm]
    codes = [orc.morton(*p) for p in ls]
    if n <= leaf:
        assert nodes == []
        return
    # sibling pairs: the root is record 0, record 1 unused; an owner's pair
    # is the next one in preorder of the owners
    seen = set()
    owners = []

    def walk(idx, a, b, d):
        assert idx not in seen
        seen.add(idx)
        na, c, nb, first, lo_l, hi_l, lo_r, hi_r = nodes[idx]
        assert (na, nb) == (a, b) and a < c < b
        if pow2:
            k = 1 << ((b - a - 1).bit_length() - 1)   # largest power of two below b - a
            assert c - a == k and k < b - a <= 2 * k
            assert a % k == 0 or n & (n - 1)          # aligned blocks when n is a power of two
        elif codes[a] == codes[b - 1]:
            assert c == a + (b - a) // 2
        else:
            h = (codes[a] ^ codes[b - 1]).bit_length() - 1
            assert all(((codes[t] >> h) & 1) == 0 for t in range(a, c))
            assert all(((codes[t] >> h) & 1) == 1 for t in range(c, b))
        for (lo, hi, s, e) in ((lo_l, hi_l, a, c), (lo_r, hi_r, c, b)):
            assert np.array_equal(np.array(lo, np.float32), ls[s:e].min(axis=0))
            assert np.array_equal(np.array(hi, np.float32), ls[s:e].max(axis=0))
        dd = d
        if c - a > leaf or b - c > leaf:
            owners.append(idx)
            assert first == 2 * len(owners)
        else:
            assert first == 0xFFFFFFFF
        for (child, s, e) in ((first, a, c), (first + 1, c, b)):
            if e - s > leaf:
                dd = max(dd, walk(child, s, e, d + 1))
            elif first != 0xFFFFFFFF:
                assert nodes[child][:4] == (0, 0, 0, 0) and not any(any(v) for v in nodes[child][4:])
                seen.add(child)
        return dd

    assert walk(0, 0, n, 0) == depth
    assert nodes[1][:4] == (0, 0, 0, 0) and not any(any(v) for v in nodes[1][4:])
    seen.add(1)
    assert len(seen) == len(nodes) == 2 * (1 + len(owners))


ARENA_HARNESS = r"""
#include <cstdio>
#include <cstring>
#include <map>
#include "hrr_arena.hpp"
// stdin: size, then ops "a id bytes" | "f id" | "s id bytes"; stdout: one line per op
int main() {
    unsigned long long size;
    if (scanf("%llu", &size) != 1) return 2;
    hrr::Arena A;
    A.init(size);
    std::map<long, std::pair<unsigned long long, unsigned long long>> blocks;
    char op[4];
    long id;
    unsigned long long bytes;
    while (scanf("%3s %ld", op, &id) == 2) {
        if (op[0] == 'a' || op[0] == 's') {
            if (scanf("%llu", &bytes) != 1) return 3;
        }
        if (op[0] == 'a') {
            uint64_t off = 0;
            if (A.alloc(bytes, &off)) {
                blocks[id] = {off, bytes};
                printf("%llu\n", (unsigned long long)off);
            } else {
                printf("-1\n");
            }
        } else if (op[0] == 'f') {
            A.release(blocks[id].first, blocks[id].second);
            blocks.erase(id);
            printf("ok\n");
        } else {
            A.shrink(blocks[id].first, blocks[id].second, bytes);
            blocks[id].second = bytes;
            printf("ok\n");
        }
    }
    printf("%llu %llu %llu %zu\n", (unsigned long long)A.used(), (unsigned long long)A.peak(),
           (unsigned long long)A.largest_free(), A.free_blocks());
    return 0;
}
"""


@pytest.fixture(scope="module")
def arena_harness(tmp_path_factory):
    d = tmp_path_factory.mktemp("arena")
    src = d / "arena.cpp"
    src.write_text(ARENA_HARNESS)
    exe = d / "arena"
    subprocess.run(["g++", "-O1", "-std=c++17", "-I", CSRC, str(src), "-o", str(exe)], check=True)
    return str(exe)


class _UnitModel:
    """First fit over a bitmap of 256-byte units: the lowest run of free units."""

    def __init__(self, size):
        self.units = [False] * (size // 256)
        self.peak = 0

    @staticmethod
    def n_units(b):
        return max(1, (b + 255) // 256)

    def alloc(self, b):
        k = self.n_units(b)
        run = 0
        for u, used in enumerate(self.units):
            run = 0 if used else run + 1
            if run == k:
                start = u - k + 1
                for v in range(start, u + 1):
                    self.units[v] = True
                self.peak = max(self.peak, sum(self.units))
                return start * 256
        return -1

    def free(self, off, b):
        for v in range(off // 256, off // 256 + self.n_units(b)):
            assert self.units[v]
            self.units[v] = False

    def largest(self):
        best = run = 0
        for used in self.units:
            run = 0 if used else run + 1
            best = max(best, run)
        return best * 256

    def blocks(self):
        n, prev = 0, True
        for used in self.units:
            if not used and prev:
                n += 1
            prev = used
        return n


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_server_arena_is_first_fit_and_coalesces(arena_harness, seed):
    rng = np.random.default_rng(900 + seed)
    size = 256 * 400 + (seed * 37)      # a size that is not a multiple of 256 on purpose
    model = _UnitModel(size)
    live = {}
    ops, expect = ["%d" % size], []
    nid = 0
    for _ in range(600):
        u = rng.random()
        if u < 0.5 or not live:
            b = int(rng.integers(0, 256 * 24))
            off = model.alloc(b)
            ops.append("a %d %d" % (nid, b))
            expect.append(str(off))
            if off >= 0:
                live[nid] = (off, b)
            nid += 1
        elif u < 0.85:
            k = list(live)[int(rng.integers(len(live)))]
            off, b = live.pop(k)
            model.free(off, b)
            ops.append("f %d" % k)
            expect.append("ok")
        else:
            k = list(live)[int(rng.integers(len(live)))]
            off, b = live[k]
            nb = int(rng.integers(0, b + 1))
            keep = model.n_units(nb)
            model.free(off + keep * 256, b - keep * 256) if model.n_units(b) > keep else None
            live[k] = (off, nb)
            ops.append("s %d %d" % (k, nb))
            expect.append("ok")
    # free everything: one block of the whole (rounded-down) size remains
    for k, (off, b) in list(live.items()):
        model.free(off, b)
        ops.append("f %d" % k)
        expect.append("ok")
    out = subprocess.run([arena_harness], input="\n".join(ops) + "\n", capture_output=True,
                         text=True, check=True).stdout.split("\n")
    assert out[:len(expect)] == expect
    used, peak, largest, nblocks = map(int, out[len(expect)].split())
    assert used == 0 and nblocks == 1 and largest == size // 256 * 256
    assert peak == model.peak * 256


COMPACT_HARNESS = r"""
#include <cstdio>
#include <cstdlib>
#include <random>
#include <set>
#include <vector>
#include "hrr_compact.hpp"
// Simulates the kernel's chunked emission by W virtual waves (each leaving the
// item `leaves` times), then applies the planned moves and checks the result.
// args: count capacity shift waves leaves seed
int main(int argc, char** argv) {
    const unsigned long long count = strtoull(argv[1], 0, 10), cap = strtoull(argv[2], 0, 10);
    const unsigned shift = atoi(argv[3]);
    const unsigned waves = atoi(argv[4]), leaves = atoi(argv[5]);
    std::mt19937_64 rng(strtoull(argv[6], 0, 10));
    const unsigned long long C = 1ull << shift;
    const unsigned long long pcap = (unsigned long long)waves * leaves;
    const unsigned long long slack = cap ? 2 * pcap * C : 0;
    std::vector<long long> buf(cap, -1), sl(slack, -1);
    // split the pairs into (wave, visit) runs, then into bursts of <= 128
    std::vector<std::vector<unsigned long long>> runs(pcap);
    for (unsigned long long p = 0; p < count; ++p) runs[rng() % pcap].push_back(p);
    struct W { long long chunk = -1; unsigned long long fill = 0; size_t run = 0, at = 0; };
    std::vector<W> ws(waves);
    for (unsigned w = 0; w < waves; ++w) ws[w].run = w * leaves;
    unsigned long long K = 0;
    std::vector<unsigned long long> partials;
    auto store = [&](unsigned long long pos, unsigned long long id) {
        if (pos < cap) buf[pos] = (long long)id;
        else if (pos - cap < slack) sl[pos - cap] = (long long)id;
    };
    std::vector<unsigned> live;
    for (unsigned w = 0; w < waves; ++w) live.push_back(w);
    while (!live.empty()) {
        const size_t li = rng() % live.size();
        W& x = ws[live[li]];
        std::vector<unsigned long long>& r = runs[x.run];
        if (x.at >= r.size()) {   // leave the item: publish the partial chunk
            if (x.chunk >= 0 && x.fill > 0) { partials.push_back(x.chunk); partials.push_back(x.fill); }
            x.chunk = -1; x.fill = 0; x.at = 0;
            if (++x.run % leaves == 0) { live.erase(live.begin() + li); }
            continue;
        }
        const unsigned long long b = std::min<unsigned long long>(1 + rng() % 128, r.size() - x.at);
        if (cap == 0) { x.at += b; continue; }
        if (x.chunk < 0) { x.chunk = (long long)K++; x.fill = 0; }
        long long next = -1;
        if (x.fill + b > C) next = (long long)K++;
        for (unsigned long long q = 0; q < b; ++q) {
            const unsigned long long pos = x.fill + q;
            store(pos < C ? x.chunk * C + pos : next * C + (pos - C), r[x.at + q]);
        }
        x.at += b;
        x.fill += b;
        if (x.fill >= C) { x.fill -= C; x.chunk = next; if (x.fill == 0) x.chunk = -1; }
    }
    // the device compaction (compact_plan_kernel, then compact_move_kernel),
    // emulated with the functions those kernels use
    const unsigned long long listed = partials.size() / 2;
    const hrr::CompactGeom g = hrr::compact_geom(count, K, listed, pcap, cap, slack, shift);
    const unsigned long long target = g.target;
    if (g.nd > 2 * pcap + 2) {
        printf("data chunks %llu above the bound %llu\n", g.nd, 2 * pcap + 2);
        return 1;
    }
    std::vector<unsigned long long> Hs(g.P + 1), Ds(g.nd + 1), fill(g.nd, C);
    unsigned long long run = 0;
    for (unsigned long long q = 0; q < g.P; ++q) {
        Hs[q] = run;
        run += hrr::hole_len(g, partials[2 * q], partials[2 * q + 1]);
    }
    Hs[g.P] = run;
    for (unsigned long long q = 0; q < g.P; ++q) {
        const unsigned long long c = partials[2 * q];
        if (c >= g.c0 && c - g.c0 < g.nd) fill[c - g.c0] = partials[2 * q + 1];
    }
    run = 0;
    for (unsigned long long i = 0; i < g.nd; ++i) {
        Ds[i] = run;
        run += hrr::data_len(g, i, fill[i]);
    }
    Ds[g.nd] = run;
    const unsigned long long moved = std::min(Hs[g.P], Ds[g.nd]);
    const unsigned long long unfilled = Hs[g.P] - moved;
    // element e: from the e-th data position to the e-th hole position (sources
    // are never destinations, so the order of the moves does not matter)
    for (unsigned long long e = 0; e < moved; ++e) {
        unsigned long long q = hrr::prefix_rank(Hs.data(), g.P, e);
        unsigned long long i = hrr::prefix_rank(Ds.data(), g.nd, e);
        while (Hs[q + 1] <= e) ++q;
        while (Ds[i + 1] <= e) ++i;
        const unsigned long long dst = hrr::hole_lo(g, partials[2 * q], partials[2 * q + 1]) + (e - Hs[q]);
        const unsigned long long src = hrr::data_lo(g, i) + (e - Ds[i]);
        if (dst >= target || src < target || src >= cap + slack) {
            printf("move out of place: %llu -> %llu\n", src, dst);
            return 1;
        }
        buf[dst] = src < cap ? buf[src] : sl[src - cap];
    }
    std::set<long long> seen;
    for (unsigned long long p = 0; p < target; ++p) {
        if (buf[p] < 0 || buf[p] >= (long long)count || !seen.insert(buf[p]).second) {
            printf("bad position %llu (value %lld)\n", p, buf[p]);
            return 1;
        }
    }
    printf("ok unfilled=%llu moved=%llu partials=%zu chunks=%llu\n", unfilled, moved, partials.size() / 2, K);
    return unfilled ? 1 : 0;
}
"""


@pytest.fixture(scope="module")
def compact_harness(tmp_path_factory):
    d = tmp_path_factory.mktemp("compact")
    src = d / "compact.cpp"
    src.write_text(COMPACT_HARNESS)
    exe = d / "compact"
    subprocess.run(["g++", "-O2", "-std=c++17", "-I", CSRC, str(src), "-o", str(exe)], check=True)
    return str(exe)


@pytest.mark.parametrize("count,extra,shift,waves,leaves", [
    (0, 10, 7, 4, 1), (1, 0, 7, 4, 1), (1000, 0, 7, 16, 1), (1000, 1, 7, 16, 1),
    (1000, 77, 7, 16, 2), (5000, 5000, 8, 64, 2), (20000, 0, 9, 200, 2), (20000, 300, 7, 300, 1),
    (3000, -1000, 7, 40, 2), (3000, -2999, 7, 40, 1), (100000, -50000, 10, 512, 2),
    (100000, 12345, 13, 512, 2), (70000, 0, 13, 3, 2)])
def test_output_compaction_fills_every_position(compact_harness, count, extra, shift, waves, leaves):
    """The plan for making an item's output dense, against a simulation of the
    kernel's chunked emission (random interleaving of waves, capacity above,
    equal to and below the count, one or two departures per wave)."""
    cap = count + extra
    for seed in range(3):
        r = subprocess.run([compact_harness, str(count), str(cap), str(shift), str(waves), str(leaves),
                            str(seed)], capture_output=True, text=True)
        assert r.returncode == 0, r.stdout + r.stderr


MOVEMAP_HARNESS = r"""
#include <cstdio>
#include <vector>
#include "hrr_compact.hpp"
// args: lanes threads run moved; walks every thread's elements exactly as
// compact_move_kernel does and checks that each e in [0, moved) is visited once
int main(int argc, char** argv) {
    if (argc != 5) return 2;
    const bool lanes = atoi(argv[1]) != 0;
    const unsigned long long threads = strtoull(argv[2], 0, 10), run = strtoull(argv[3], 0, 10),
                             moved = strtoull(argv[4], 0, 10);
    std::vector<unsigned char> seen(moved, 0);
    for (unsigned long long t = 0; t < threads; ++t) {
        const hrr::MoveMap m = hrr::move_map(lanes, t, threads, run);
        for (unsigned long long e0 = m.first; e0 < moved; e0 += m.step) {
            const unsigned long long e1 = hrr::move_run_end(m, e0, moved);
            for (unsigned long long e = e0; e < e1; e += m.stride) {
                if (seen[e]++) { printf("element %llu visited twice (thread %llu)\n", e, t); return 1; }
            }
        }
    }
    for (unsigned long long e = 0; e < moved; ++e)
        if (!seen[e]) { printf("element %llu never visited\n", e); return 1; }
    printf("ok\n");
    return 0;
}
"""


@pytest.fixture(scope="module")
def movemap_harness(tmp_path_factory):
    d = tmp_path_factory.mktemp("movemap")
    src = d / "movemap.cpp"
    src.write_text("#include <cstdlib>\n" + MOVEMAP_HARNESS)
    exe = d / "movemap"
    subprocess.run(["g++", "-O2", "-std=c++17", "-I", CSRC, str(src), "-o", str(exe)], check=True)
    return str(exe)


@pytest.mark.parametrize("lanes", [0, 1])
@pytest.mark.parametrize("threads", [256, 1024, 4096, 256 * 23])
@pytest.mark.parametrize("moved", [0, 1, 63, 64, 65, 1023, 1024, 1025, 16383, 16384, 16385, 100003, 1 << 18])
def test_compaction_move_mapping_visits_each_element_once(movemap_harness, lanes, threads, moved):
    """Both thread mappings of compact_move_kernel (per-lane runs for small
    chunks, lane-interleaved blocks for chunks of 2^10 pairs or more) hand
    every moved element to exactly one thread, for grids of 1 to 23 blocks
    per item and moved counts around the run and block sizes."""
    r = subprocess.run([movemap_harness, str(lanes), str(threads), "16", str(moved)],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stdout + r.stderr


BITS_HARNESS = r"""
#include <cstdio>
#include "hrr_rmq.hpp"
// args: b k_r; prints b_h = fls(b), k_p = ffs(k_r), k_q = top bit of the lowest
// run of ones of k_r, and m = k_r with the bits above b_h cleared, using the
// bit primitives of the range-minimum code
int main(int argc, char** argv) {
    if (argc != 3) return 2;
    const uint32_t b = (uint32_t)strtoul(argv[1], 0, 0), kr = (uint32_t)strtoul(argv[2], 0, 0);
    const int bh = hrr::top_bit(b);
    const int kp = hrr::bottom_bit(kr);
    const int kq = hrr::bottom_bit(~kr & ~hrr::low_mask(kp)) - 1;
    const uint32_t m = kr & hrr::low_mask(bh + 1);
    printf("%d %d %d %u\n", bh, kp, kq, m);
    return 0;
}
"""


def test_section2_bit_example_fixes_fls_and_ffs(tmp_path):
    """Section 2's worked bit pattern (tests/golden/paper_bit_example.txt):
    b = 010010 has b_h = 4 and k_r = 100110 has k_p = 1, k_q = 2; the
    highest / lowest set-bit primitives of the range-minimum code are 0-based
    and reproduce every printed value, and so does clearing k_r above b_h."""
    clang = "/opt/rocm/llvm/bin/clang++"
    if not os.path.exists(clang):
        pytest.skip("clang++ with __builtin_bitreverse32 is not available")
    kv = {}
    with open(os.path.join(ROOT, "tests", "golden", "paper_bit_example.txt")) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if line:
                k, v = line.split()
                kv[k] = int(v, 0)
    src = tmp_path / "bits.cpp"
    src.write_text("#include <cstdlib>\n" + BITS_HARNESS)
    exe = tmp_path / "bits"
    subprocess.run([clang, "-O1", "-std=c++17", "-I", CSRC, str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe), str(kv["b"]), str(kv["k_r"])], capture_output=True, text=True,
                         check=True).stdout.split()
    assert [int(x) for x in out] == [kv["b_h"], kv["k_p"], kv["k_q"], kv["m"]]
    assert kv["B"] == 6 and kv["b"] < 1 << kv["B"] and kv["k_r"] < 1 << kv["B"]


RMQ_HARNESS = r"""
#include <cstdio>
#include "hrr_rmq.hpp"
// stdin: n, then n lines "a b R"; stdout per query: argmin of each method 0..4
int main() {
    unsigned n;
    if (scanf("%u", &n) != 1) return 2;
    for (unsigned q = 0; q < n; ++q) {
        unsigned a, b, R;
        if (scanf("%u %u %u", &a, &b, &R) != 3) return 3;
        const unsigned kr = hrr::threshold_index(R);
        printf("%u %u %u %u %u\n", hrr::rmq<0>(a, b, kr), hrr::rmq<1>(a, b, kr), hrr::rmq<2>(a, b, kr),
               hrr::rmq<3>(a, b, kr), hrr::rmq<4>(a, b, kr));
    }
    return 0;
}
"""


@pytest.fixture(scope="module")
def rmq_harness(tmp_path_factory):
    clang = "/opt/rocm/llvm/bin/clang++"
    if not os.path.exists(clang):
        pytest.skip("clang++ with __builtin_bitreverse32 is not available")
    d = tmp_path_factory.mktemp("rmq")
    src = d / "rmq.cpp"
    src.write_text(RMQ_HARNESS)
    exe = d / "rmq"
    subprocess.run([clang, "-O2", "-std=c++17", "-I", CSRC, str(src), "-o", str(exe)], check=True)
    return str(exe)


def test_device_range_minimum_code_on_the_host(orc, rmq_harness):
    """The range-minimum functions the kernels run (host-compiled) against the
    oracle's scan: random ranges of every length class, node-like aligned
    ranges, ranges at both ends of the index space, shifts 0 / 2^31 / 2^32-1
    and shifts that put k_r just inside, at and just outside the range."""
    rng = np.random.default_rng(77)
    qs = []
    for t in range(6000):
        L = int(2 ** rng.uniform(0, 12))
        mode = t % 6
        if mode == 0:
            a = int(rng.integers(0, 64))
        elif mode == 1:
            a = (1 << 32) - 1 - L - int(rng.integers(0, 64))
        elif mode == 2:
            a = int(rng.integers(0, 1 << 20)) // L * L      # node-like, aligned
        else:
            a = int(rng.integers(0, (1 << 32) - 1 - L))
        b = a + L
        R = int(rng.integers(0, 1 << 32))
        if t % 7 == 0:
            R = 0
        elif t % 11 == 0:
            R = (1 << 32) - 1
        elif t % 13 == 0:
            R = 1 << 31
        elif t % 17 == 0:      # k_r at a - 1, a .. b - 1 or b
            k = (a - 1 + int(rng.integers(0, L + 2))) & 0xFFFFFFFF
            R = (-int(orc.bitrev(k))) & 0xFFFFFFFF
        qs.append((a, b, R))
    a = np.array([q[0] for q in qs], np.uint32)
    b = np.array([q[1] for q in qs], np.uint32)
    r = np.array([q[2] for q in qs], np.uint32)
    inp = "%d\n" % len(qs) + "\n".join("%d %d %d" % q for q in qs) + "\n"
    out = subprocess.run([rmq_harness], input=inp, capture_output=True, text=True, check=True).stdout
    got = np.array([[int(x) for x in ln.split()] for ln in out.splitlines()], np.uint64)
    want, _ = orc.rmq_scan(a, b, r)
    for m in range(5):
        assert np.array_equal(got[:, m], want.astype(np.uint64)), "method %d" % m


LAYOUT_HARNESS = r"""
#include <cstdio>
#include "hrr_layout.hpp"
// stdin lines: "o n virtual_eyes tile_bits" | "q n tasks" | "c capacity waves" | "e n_lights" | "p cost" | "s epw"
int main() {
    char op;
    unsigned long long a, b, c;
    while (scanf(" %c", &op) == 1) {
        if (op == 'o' && scanf("%llu %llu %llu", &a, &b, &c) == 3) {
            uint32_t bits, rbits;
            hrr::order_key_bits(a, b, (uint32_t)c, &bits, &rbits);
            printf("%u %u\n", bits, rbits);
        } else if (op == 'q' && scanf("%llu %llu", &a, &b) == 2) {
            const uint32_t s = hrr::queue_interleave_shift(a, b);
            printf("%u %llu\n", s, (unsigned long long)hrr::departures_per_wave(a, s));
        } else if (op == 'c' && scanf("%llu %llu", &a, &b) == 2) {
            printf("%u\n", hrr::chunk_shift_for(a, b));
        } else if (op == 'e' && scanf("%llu", &a) == 1) {
            printf("%u\n", hrr::default_eyes_per_wave((uint32_t)a));
        } else if (op == 'p' && scanf("%llu", &a) == 1) {
            printf("%d\n", hrr::order_pays((double)a) ? 1 : 0);
        } else if (op == 's' && scanf("%llu", &a) == 1) {
            uint32_t c[3];
            hrr::tune_stack_candidates((uint32_t)a, c);
            printf("%u %u %u %u\n", hrr::default_stack_entries((uint32_t)a), c[0], c[1], c[2]);
        } else {
            return 1;
        }
    }
    return 0;
}
"""


@pytest.fixture(scope="module")
def layout_harness(tmp_path_factory):
    d = tmp_path_factory.mktemp("layout")
    src = d / "layout.cpp"
    src.write_text(LAYOUT_HARNESS)
    exe = d / "layout"
    subprocess.run(["g++", "-O1", "-std=c++17", "-I", CSRC, str(src), "-o", str(exe)], check=True)
    return str(exe)


def _ask(exe, lines):
    out = subprocess.run([exe], input="\n".join(lines) + "\n", capture_output=True, text=True,
                         check=True).stdout.split("\n")
    return [tuple(map(int, o.split())) for o in out if o]


def test_launch_layout_choices(layout_harness):
    """Eye-order key widths, queue layout, departures per wave, chunk size and
    default eyes per wave of a launch, for the benchmark shapes and the
    boundaries of each rule."""
    ask = lambda lines: _ask(layout_harness, lines)
    # order key: frame (3 bits per axis, 9 class bits), 256 caches (2, 6), a
    # small item (2, 9), the bucket budget, tiles without class bits
    assert ask(["o 1 2073600 12", "o 256 4034935 12", "o 1 4096 12", "o 16384 1000000 12",
                "o 131073 1000000 12", "o 1 2073600 0", "o 1 2073600 3", "o 1 0 12",
                "o 1 4294967295 12"]) == [
        (3, 9), (2, 6), (2, 9), (2, 0), (0, 0), (3, 0), (3, 3), (0, 0), (0, 0)]
    # the budget always holds and cells keep two bits per axis where it allows
    lines, cases = [], []
    for n in (1, 2, 3, 7, 64, 255, 1024, 4096, 16383, 16384, 16385, 131072):
        for ve in (1, 100, 2 ** 11, 2 ** 14, 2 ** 20, 2 ** 24, 2 ** 31):
            for tb in (0, 1, 12, 32):
                lines.append("o %d %d %d" % (n, ve, tb))
                cases.append((n, ve, tb))
    for (n, ve, tb), (bits, rbits) in zip(cases, ask(lines)):
        if bits:
            assert n << (3 * bits + rbits) <= 1 << 20
            assert rbits <= min(9, tb)
        assert bits >= min(2, max(b for b in range(3) if n << (3 * b) <= 1 << 20))
    # queues: interleaved 2^13-task chunks for several items with >= 2^19 tasks
    assert ask(["q 1 10000000", "q 2 524287", "q 2 524288", "q 256 4034935", "q 1 1"]) == [
        (0, 1), (0, 2), (13, 8), (13, 8), (0, 1)]
    # chunks: about sixteen per touching wave, 2^7 .. 2^13 pairs
    w = 7168
    assert ask(["c 0 1", "c %d 1" % (1 << 40), "c 4829514196 %d" % w, "c %d %d" % (16 * w * 256, w),
                "c %d %d" % (16 * w * 256 - 1, w)]) == [(7,), (13,), (13,), (8,), (7,)]
    # eyes per wave by hierarchy size: 8 below 2^16 lights, 4 below 2^17, then 1
    assert ask(["e 0", "e 1024", "e 65535", "e 65536", "e 131071", "e 131072", "e 1048576",
                "e 4294967295"]) == [(8,), (8,), (8,), (4,), (4,), (1,), (1,), (1,)]
    # eye ordering only for launches with enough work: the 4096 x 1024 case (cost 4096 x
    # 1024^0.6 = 262144) goes unordered, 4096 frame eyes x 2^20 lights (16777216) ordered
    assert ask(["p 262144", "p 2097151", "p 2097152", "p 16777216"]) == [(0,), (0,), (1,), (1,)]
    # stack entries: 192 for one eye per wave (its LDS record area leaves room
    # for 7 waves per SIMD), 512 otherwise; the default is the first candidate,
    # every candidate a multiple of 64 in [192, 4096] (the launch's rule)
    got = ask(["s 1", "s 2", "s 4", "s 8"])
    assert got == [(192, 192, 256, 512), (512, 512, 256, 1024), (512, 512, 256, 1024), (512, 512, 256, 1024)]
    for row in got:
        assert all(c % 64 == 0 and 192 <= c <= 4096 for c in row)
