"""Admission policy of the serving loop (hrr_admit.hpp), on the CPU.

A small event simulation drives the same admit_batch() the server calls
under its lock: synthetic requests arrive at given times, W workers each run
one batch at a time for a service time that grows with the batch's eyes, and
every batch holds its requests' eye copies and output reservations in the
arena until it ends.  The tests check the policy's promises on the recorded
schedule: batch limits, the memory budget, no overtaking of a request that
has waited overtake_ms, strict FIFO order when that bound is 0, a bounded wait
for a large request behind a stream of small ones, and that passing over a
request that does not fit lowers the median latency when the head of the
queue blocks.
"""
import os
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1907_12343_amd", "csrc")

SIM = r"""
#include <algorithm>
#include <cstdio>
#include <deque>
#include <vector>
#include "hrr_admit.hpp"
// stdin: budget workers max_items max_eyes overtake_s c0 c1 n, then n lines
// "t eyes eye_bytes out_bytes" (arrival order).  Simulates the workers and
// prints "B worker t_start t_end n_items eyes bytes_in_use_after_admission ids..."
// per batch and "R id t_arrive t_admit t_done" per request.
struct Req { double t; unsigned long long eyes, eb, ob; double admit = -1, done = -1; };
struct Run { double end; std::vector<int> ids; std::vector<unsigned long long> eo, oo; };
int main() {
    unsigned long long budget, max_eyes; int W, n; unsigned max_items; double overtake, c0, c1;
    if (scanf("%llu %d %u %llu %lf %lf %lf %d", &budget, &W, &max_items, &max_eyes, &overtake, &c0, &c1, &n) != 8)
        return 2;
    std::vector<Req> R(n);
    for (auto& r : R)
        if (scanf("%lf %llu %llu %llu", &r.t, &r.eyes, &r.eb, &r.ob) != 4) return 3;
    hrr::Arena A;
    A.init(budget);
    hrr::AdmitLimits L{max_items, max_eyes, overtake, 256};
    std::deque<int> q;
    std::vector<Run> running(W);
    std::vector<bool> busy(W, false);
    size_t next = 0;
    double now = 0;
    int done = 0;
    std::vector<hrr::Admitted> picked;
    while (done < n) {
        // next event: an arrival or the end of a running batch
        double t_ev = 1e300;
        if (next < R.size()) t_ev = R[next].t;
        for (int w = 0; w < W; ++w) if (busy[w]) t_ev = std::min(t_ev, running[w].end);
        now = t_ev;
        for (int w = 0; w < W; ++w) {
            if (busy[w] && running[w].end <= now) {
                for (size_t k = 0; k < running[w].ids.size(); ++k) {
                    Req& r = R[running[w].ids[k]];
                    if (r.eb) A.release(running[w].eo[k], r.eb);
                    if (r.ob) A.release(running[w].oo[k], r.ob);
                    r.done = running[w].end;
                    ++done;
                }
                busy[w] = false;
            }
        }
        while (next < R.size() && R[next].t <= now) q.push_back((int)next++);
        for (int w = 0; w < W; ++w) {
            if (busy[w] || q.empty()) continue;
            hrr::admit_batch(A, L, now, q.size(), [&](size_t i) {
                const Req& r = R[q[i]];
                return hrr::AdmitView{r.eyes, r.eb, r.ob, r.t};
            }, picked);
            if (picked.empty()) break;   // nothing fits now; a later event frees memory
            Run run;
            unsigned long long eyes = 0;
            for (auto& a : picked) {
                run.ids.push_back(q[a.pos]);
                run.eo.push_back(a.eye_off);
                run.oo.push_back(a.out_off);
                R[q[a.pos]].admit = now;
                eyes += R[q[a.pos]].eyes;
            }
            for (auto it = picked.rbegin(); it != picked.rend(); ++it) q.erase(q.begin() + (long)it->pos);
            run.end = now + c0 + c1 * (double)eyes;
            printf("B %d %.9f %.9f %zu %llu %llu", w, now, run.end, run.ids.size(), eyes, A.used());
            for (int id : run.ids) printf(" %d", id);
            printf("\n");
            running[w] = run;
            busy[w] = true;
        }
    }
    for (int i = 0; i < n; ++i) printf("R %d %.9f %.9f %.9f\n", i, R[i].t, R[i].admit, R[i].done);
    return 0;
}
"""


@pytest.fixture(scope="module")
def sim(tmp_path_factory):
    d = tmp_path_factory.mktemp("admit")
    src = d / "sim.cpp"
    src.write_text(SIM)
    exe = d / "sim"
    subprocess.run(["g++", "-O2", "-std=c++17", "-I", CSRC, str(src), "-o", str(exe)], check=True)
    return str(exe)


def run_sim(exe, reqs, budget, workers=2, max_items=64, max_eyes=1 << 20, overtake_s=0.1,
            c0=1e-3, c1=1e-7):
    head = "%d %d %d %d %.9f %.9f %.12f %d\n" % (budget, workers, max_items, max_eyes, overtake_s, c0, c1,
                                                len(reqs))
    body = "".join("%.9f %d %d %d\n" % r for r in reqs)
    out = subprocess.run([exe], input=head + body, capture_output=True, text=True, check=True).stdout
    batches, R = [], {}
    for line in out.splitlines():
        f = line.split()
        if f[0] == "B":
            batches.append(dict(worker=int(f[1]), t0=float(f[2]), t1=float(f[3]), n=int(f[4]),
                                eyes=int(f[5]), used=int(f[6]), ids=[int(x) for x in f[7:]]))
        else:
            R[int(f[1])] = dict(t=float(f[2]), admit=float(f[3]), done=float(f[4]))
    return batches, R


def _mix(seed, n, rate, budget):
    """Poisson arrivals of 2^U[8,18]-eye requests with ~600 pairs per eye reserved."""
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate, n))
    eyes = np.floor(2.0 ** rng.uniform(8, 18, n)).astype(np.int64)
    reqs = []
    for k in range(n):
        eb = int(eyes[k]) * 12
        ob = min(int(eyes[k]) * 600 * 8, budget // 2)
        reqs.append((float(t[k]), int(eyes[k]), eb, ob))
    return reqs


def _check_common(batches, R, reqs, budget, max_items, max_eyes):
    assert len(R) == len(reqs)
    for k, r in R.items():
        assert r["admit"] >= r["t"] - 1e-12 and r["done"] > r["admit"], k
    seen = set()
    for b in batches:
        assert 1 <= b["n"] <= max_items
        assert b["n"] == 1 or b["eyes"] <= max_eyes
        assert b["used"] <= budget
        assert not (set(b["ids"]) & seen)
        seen |= set(b["ids"])
        assert b["ids"] == sorted(b["ids"])   # queue order inside a batch
    assert seen == set(range(len(reqs)))


@pytest.mark.parametrize("seed", [0, 1, 2])
@pytest.mark.parametrize("overtake_s", [0.0, 0.02, 0.1])
def test_limits_budget_and_no_overtaking_of_overdue_requests(sim, seed, overtake_s):
    budget = 1 << 30
    reqs = _mix(seed, 400, 300.0, budget)
    batches, R = run_sim(sim, reqs, budget, overtake_s=overtake_s, max_items=16, max_eyes=1 << 19)
    _check_common(batches, R, reqs, budget, 16, 1 << 19)
    for b in batches:
        t = b["t0"]
        first_admitted = min(b["ids"])
        last_admitted = max(b["ids"])
        for y in range(last_admitted):
            ry = R[y]
            if y in b["ids"] or not (ry["t"] <= t < ry["admit"]):
                continue   # not waiting in the queue at this admission
            # y was passed over by a later request of this batch: only while young
            assert y < last_admitted
            assert t - ry["t"] < overtake_s + 1e-9, (y, t, ry, overtake_s)
        if overtake_s == 0.0:
            # strict FIFO: nothing older than the batch's first request is still queued
            assert all(not (R[y]["t"] <= t < R[y]["admit"]) for y in range(first_admitted))


def test_strict_fifo_admits_in_arrival_order(sim):
    budget = 1 << 30
    reqs = _mix(5, 300, 400.0, budget)
    _, R = run_sim(sim, reqs, budget, overtake_s=0.0, max_items=8, max_eyes=1 << 19)
    admits = [R[k]["admit"] for k in range(len(reqs))]
    assert all(a <= b + 1e-12 for a, b in zip(admits, admits[1:]))


def test_small_requests_pass_a_blocked_head_then_it_runs_in_bounded_time(sim):
    """A request that needs most of the arena arrives while a long batch holds
    half of it; small requests arriving behind it run meanwhile, until it has
    waited overtake_ms; then the queue drains for it and it starts within one
    service time of the batches already running."""
    budget = 64 << 20
    c0, c1 = 1e-3, 1e-7
    reqs = [(0.0, 200000, 2400000, 30 << 20)]            # holds ~32 MiB for 21 ms
    reqs.append((0.001, 1000, 12000, 40 << 20))          # needs 40 MiB: blocked
    for k in range(400):                                 # then a stream of small requests
        reqs.append((0.002 + k * 2e-4, 300, 3600, 1 << 20))
    overtake = 0.05
    batches, R = run_sim(sim, reqs, budget, overtake_s=overtake, max_items=4, max_eyes=1 << 20, c0=c0, c1=c1)
    _check_common(batches, R, reqs, budget, 4, 1 << 20)
    big = R[1]
    # small requests behind it were admitted before it
    assert sum(1 for k in range(2, len(reqs)) if R[k]["admit"] < big["admit"]) > 20
    # but it waited at most the age bound plus one service time of what was running
    longest = max(b["t1"] - b["t0"] for b in batches)
    assert big["admit"] - big["t"] <= overtake + longest + 1e-9
    # with strict FIFO nothing passes it
    _, F = run_sim(sim, reqs, budget, overtake_s=0.0, max_items=4, max_eyes=1 << 20, c0=c0, c1=c1)
    assert all(F[k]["admit"] >= F[1]["admit"] for k in range(2, len(reqs)))
    # and the small requests' median latency is lower when they may pass
    lat = lambda D: np.median([D[k]["done"] - D[k]["t"] for k in range(2, len(reqs))])
    assert lat(R) < lat(F)
