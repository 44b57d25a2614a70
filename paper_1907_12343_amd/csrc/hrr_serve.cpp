// hrr_serve.cpp -- serving loop: eye tiles from many clients against
// hierarchies resident on the GPU, batched continuously into persistent
// traversal launches.
//
// Design.  One device arena (the HBM budget) is allocated at start and
// carved by a first-fit allocator into request eye copies and result pair
// arrays.  max_inflight worker threads each own a HIP stream and a launch
// scratch set.  A free worker takes, under the server lock, the queued
// requests that fit its limits and the free arena (hrr_admit.hpp: in arrival
// order, passing over a request that does not fit until it has waited
// overtake_ms), enqueues the eye uploads and the traversal of that batch --
// one persistent launch per eyes-per-wave group of its requests, one item per
// request -- and waits for it on its own stream; meanwhile another worker is
// already batching whatever arrived since.  Results stay in the arena until
// released; a request whose output overflowed its reservation is put back at
// the head of the queue with its exact count reserved.
#include <hip/hip_runtime_api.h>
#include <math.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "hrr_admit.hpp"
#include "hrr_arena.hpp"
#include "hrr_ctx.hpp"

#define HRR_EXPORT extern "C" __attribute__((visibility("default")))

namespace hrr {

namespace {

constexpr uint64_t kAlign = Arena::kAlign;
constexpr uint64_t kEyeBytes = 3 * sizeof(float);
constexpr uint64_t kPairBytes = 2 * sizeof(uint32_t);
constexpr uint32_t kAdmitScan = 256;   // queue entries the admission looks at per batch

uint64_t round_up(uint64_t x) { return Arena::round_up(x); }

double now_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

enum class RState { Queued, Running, Done, Cancelled, Failed };

struct Request {
    uint64_t ticket = 0;
    const hrr_hierarchy* h = nullptr;
    std::vector<float> eyes;       // host copy, 3 per eye
    uint32_t n = 0, width = 1, offset = 0;
    float s = 1.0f;
    RState state = RState::Queued;
    hrr_status status = HRR_OK;
    std::string err;
    uint64_t reserve = 0;          // pairs reserved for the next launch
    bool exact = false;            // reserve is the known count
    uint64_t out_off = 0, out_bytes = 0;   // result block (out_bytes 0: none)
    uint64_t eye_off = 0, eye_bytes = 0;   // eye block while running
    uint64_t n_pairs = 0;
    double submit_s = 0, start_s = 0, done_s = 0;
    uint32_t launches = 0;
    uint32_t copying = 0;          // result copies in progress
};

using ReqPtr = std::shared_ptr<Request>;

struct Slot {
    hipStream_t stream = nullptr;
    LaunchScratch S[4];            // one per eyes-per-wave group of a batch
    std::vector<uint64_t> counts;  // pair count of every request of the last batch
    std::vector<hrr_status> status;   // outcome of every request of the last batch
    std::vector<std::string> errs;    // and its message when it failed
    std::thread th;
    float* h_stage = nullptr;      // pinned eye staging
    size_t h_stage_bytes = 0;
};

}  // namespace

struct Server {
    hrr_ctx* ctx = nullptr;
    hrr_server_config cfg{};
    char* base = nullptr;          // arena base (device)
    Arena arena;
    std::mutex mu;
    std::condition_variable cv_work;   // queue or arena changed
    std::condition_variable cv_done;   // a request left the queued/running states
    std::deque<ReqPtr> queue;
    std::unordered_map<uint64_t, ReqPtr> tickets;
    std::vector<std::unique_ptr<Slot>> slots;
    std::map<const hrr_hierarchy*, double> ppe;   // observed pairs per eye
    bool stopping = false;
    uint64_t next_ticket = 1;
    int running_launches = 0;
    double busy_from = 0;
    hrr_server_stats st{};
    std::vector<double> lat_ms;
};

namespace {

uint64_t reservation_for(Server& sv, const Request& r) {
    if (r.exact) return r.reserve;
    auto it = sv.ppe.find(r.h);
    const double per_eye = it != sv.ppe.end() ? it->second : (double)sv.cfg.pairs_per_eye_guess;
    const double want = ceil((double)r.n * per_eye * 1.25) + 4096.0;
    return (uint64_t)std::min(want, 1e18);
}

// Mark a request finished (any final state) and wake its waiters.
void finish_request(Server& sv, Request& r, RState state, hrr_status status, const char* msg) {
    r.state = state;
    r.status = status;
    if (msg) r.err = msg;
    r.done_s = now_s();
    r.eyes.clear();
    r.eyes.shrink_to_fit();
    if (state == RState::Done) {
        sv.st.completed++;
        sv.st.pairs += r.n_pairs;
        sv.lat_ms.push_back((r.done_s - r.submit_s) * 1e3);
    } else if (state == RState::Cancelled) {
        sv.st.cancelled++;
    }
}

// Requests whose exact reservation (known after an overflow) can never fit
// beside their eyes fail; then the admission policy picks the batch.  Called
// with sv.mu held.
void take_batch(Server& sv, std::vector<ReqPtr>& batch) {
    const uint64_t budget = sv.arena.size();
    auto room_of = [&](const Request& r) {
        const uint64_t ebytes = (uint64_t)r.n * kEyeBytes;
        return budget > round_up(ebytes) + kAlign ? (budget - round_up(ebytes) - kAlign) / kPairBytes : 0;
    };
    bool failed = false;
    for (auto it = sv.queue.begin(); it != sv.queue.end();) {
        Request& r = **it;
        if (r.exact && r.reserve > room_of(r)) {
            finish_request(sv, r, RState::Failed, HRR_E_NOMEM, "result does not fit the server's device budget");
            it = sv.queue.erase(it);
            failed = true;
        } else {
            ++it;
        }
    }
    if (failed) sv.cv_done.notify_all();
    // output reservation per queued request: the estimate, never more than
    // could ever fit beside its eyes
    std::vector<uint64_t> want;
    want.reserve(std::min<size_t>(sv.queue.size(), kAdmitScan));
    AdmitLimits L{sv.cfg.max_batch_items, sv.cfg.max_batch_eyes, (double)sv.cfg.overtake_ms * 1e-3, kAdmitScan};
    std::vector<Admitted> picked;
    admit_batch(sv.arena, L, now_s(), sv.queue.size(),
                [&](size_t i) {
                    const Request& r = *sv.queue[i];
                    if (want.size() <= i) want.resize(i + 1, 0);
                    want[i] = std::min(reservation_for(sv, r), room_of(r));
                    return AdmitView{r.n, (uint64_t)r.n * kEyeBytes, want[i] * kPairBytes, r.submit_s};
                },
                picked);
    for (const Admitted& a : picked) {
        const ReqPtr& r = sv.queue[a.pos];
        r->eye_off = a.eye_off;
        r->eye_bytes = (uint64_t)r->n * kEyeBytes;
        r->out_off = a.out_off;
        r->out_bytes = want[a.pos] * kPairBytes;
        r->reserve = want[a.pos];
        r->state = RState::Running;
        if (r->launches == 0) r->start_s = now_s();
        r->launches++;
        batch.push_back(r);
    }
    for (auto it = picked.rbegin(); it != picked.rend(); ++it) sv.queue.erase(sv.queue.begin() + (ptrdiff_t)it->pos);
}

// Enqueue uploads and one traversal launch for `batch`, wait for it and
// finish the items.  Called without the lock.
hrr_status run_batch(Server& sv, Slot& slot, const std::vector<ReqPtr>& batch) {
    hrr_ctx* ctx = sv.ctx;
    hipError_t e;
    size_t stage = 0;
    for (auto& r : batch) stage += (size_t)r->n * kEyeBytes;
    if (stage > slot.h_stage_bytes) {
        if (slot.h_stage) (void)hipHostFree(slot.h_stage);
        slot.h_stage = nullptr;
        slot.h_stage_bytes = 0;
        if ((e = hipHostMalloc((void**)&slot.h_stage, stage, hipHostMallocDefault)) != hipSuccess)
            return hip_fail(e, "server eye staging");
        slot.h_stage_bytes = stage;
    }
    std::vector<HostItem> items;
    items.reserve(batch.size());
    size_t at = 0;
    for (auto& r : batch) {
        const size_t bytes = (size_t)r->n * kEyeBytes;
        float* dev_eyes = bytes ? reinterpret_cast<float*>(sv.base + r->eye_off) : nullptr;
        if (bytes) {
            memcpy(reinterpret_cast<char*>(slot.h_stage) + at, r->eyes.data(), bytes);
            if ((e = hipMemcpyAsync(dev_eyes, reinterpret_cast<char*>(slot.h_stage) + at, bytes,
                                    hipMemcpyHostToDevice, slot.stream)) != hipSuccess)
                return hip_fail(e, "server eye upload");
        }
        at += bytes;
        hrr_eyes E{dev_eyes, r->n, r->width, r->offset, 0};
        items.push_back(HostItem{r->h, E, r->s, r->out_off / kPairBytes, r->reserve});
    }
    hrr_traverse_opts o{};
    o.eyes_per_wave = sv.cfg.eyes_per_wave;
    // requests grouped by the eyes per wave of their own hierarchy (as a
    // batched call does), unless the configuration fixes the shape; each
    // group with the stack size of its own items
    std::vector<LaunchGroup> groups;
    group_by_shape(ctx, &o, items, o.eyes_per_wave == 0 && items.size() > 1, groups);
    uint32_t* pairs = reinterpret_cast<uint32_t*>(sv.base);
    std::vector<HostItem> sub;
    std::vector<hrr_status> gst(groups.size(), HRR_OK);
    std::vector<std::string> gmsg(groups.size());
    for (size_t g = 0; g < groups.size(); ++g) {
        sub.clear();
        for (size_t k : groups[g].items) sub.push_back(items[k]);
        gst[g] = launch_items(ctx, slot.S[g], sub, groups[g].epw, groups[g].cap, HRR_RMQ_PAPER, 1, 0, false, true,
                              pairs, nullptr, slot.stream);
        if (gst[g] != HRR_OK) gmsg[g] = hrr_last_error(ctx);
    }
    // launches that were enqueued run to the end even when another failed
    if ((e = hipStreamSynchronize(slot.stream)) != hipSuccess) return hip_fail(e, "server traversal");
    // a group's failure fails only that group's requests
    slot.counts.assign(items.size(), 0);
    slot.status.assign(items.size(), HRR_OK);
    slot.errs.assign(items.size(), std::string());
    for (size_t g = 0; g < groups.size(); ++g) {
        hrr_status st = gst[g];
        if (st == HRR_OK) {
            st = finish_items(ctx, slot.S[g]);
            if (st == HRR_OK && slot.S[g].error)
                st = fail(HRR_E_DEVICE, "traversal kernel reported error %u", slot.S[g].error);
            if (st != HRR_OK) gmsg[g] = hrr_last_error(ctx);
        }
        for (size_t q = 0; q < groups[g].items.size(); ++q) {
            const size_t k = groups[g].items[q];
            slot.status[k] = st;
            if (st == HRR_OK) slot.counts[k] = slot.S[g].counts[q];
            else slot.errs[k] = gmsg[g];
        }
    }
    return HRR_OK;
}

void worker(Server* sv, Slot* slot) {
    (void)hipSetDevice(sv->ctx->device);
    std::vector<ReqPtr> batch;
    for (;;) {
        batch.clear();
        {
            std::unique_lock<std::mutex> lk(sv->mu);
            for (;;) {
                if (sv->stopping) return;
                take_batch(*sv, batch);
                if (!batch.empty()) break;
                sv->cv_work.wait(lk);
            }
            if (sv->running_launches++ == 0) sv->busy_from = now_s();
            sv->st.launches++;
        }
        const hrr_status rc = run_batch(*sv, *slot, batch);
        const std::string msg = rc == HRR_OK ? std::string() : std::string(hrr_last_error(sv->ctx));
        {
            std::lock_guard<std::mutex> g(sv->mu);
            if (--sv->running_launches == 0) sv->st.busy_s += now_s() - sv->busy_from;
            std::vector<ReqPtr> retry;
            for (size_t k = 0; k < batch.size(); ++k) {
                Request& r = *batch[k];
                if (r.eye_bytes) sv->arena.release(r.eye_off, r.eye_bytes);
                r.eye_bytes = 0;
                const hrr_status rk = rc != HRR_OK ? rc : slot->status[k];
                if (rk != HRR_OK) {
                    if (r.out_bytes) sv->arena.release(r.out_off, r.out_bytes);
                    r.out_bytes = 0;
                    finish_request(*sv, r, RState::Failed, rk, rc != HRR_OK ? msg.c_str() : slot->errs[k].c_str());
                    continue;
                }
                const uint64_t cnt = slot->counts[k];
                if (r.n) {
                    double& e = sv->ppe[r.h];
                    const double obs = (double)cnt / r.n;
                    // follow increases at once, decreases by halves
                    e = e > 0 ? std::max(obs, 0.5 * e + 0.5 * obs) : obs;
                }
                if (cnt > r.reserve) {
                    // overflow: run again with the exact count reserved
                    if (r.out_bytes) sv->arena.release(r.out_off, r.out_bytes);
                    r.out_bytes = 0;
                    r.reserve = cnt;
                    r.exact = true;
                    r.state = RState::Queued;
                    sv->st.retries++;
                    retry.push_back(batch[k]);
                    continue;
                }
                if (cnt == 0) {
                    if (r.out_bytes) sv->arena.release(r.out_off, r.out_bytes);
                    r.out_bytes = 0;
                } else {
                    sv->arena.shrink(r.out_off, r.out_bytes, cnt * kPairBytes);
                    r.out_bytes = cnt * kPairBytes;
                }
                r.n_pairs = cnt;
                finish_request(*sv, r, RState::Done, HRR_OK, nullptr);
            }
            for (auto it = retry.rbegin(); it != retry.rend(); ++it) sv->queue.push_front(*it);
            sv->st.peak_bytes = std::max<uint64_t>(sv->st.peak_bytes, sv->arena.peak());
        }
        sv->cv_done.notify_all();
        sv->cv_work.notify_all();
    }
}

hrr_status result_of(const Request& r) {
    switch (r.state) {
        case RState::Queued:
        case RState::Running: return HRR_E_NOTREADY;
        case RState::Done: return HRR_OK;
        case RState::Cancelled: return fail(HRR_E_CANCELLED, "request %llu was cancelled", (unsigned long long)r.ticket);
        case RState::Failed: return fail(r.status, "request %llu failed: %s", (unsigned long long)r.ticket, r.err.c_str());
    }
    return HRR_E_INVALID;
}

void stop_server(hrr_ctx* ctx) {
    Server* sv = ctx->server;
    if (!sv) return;
    {
        std::lock_guard<std::mutex> g(sv->mu);
        sv->stopping = true;
        for (auto& r : sv->queue) finish_request(*sv, *r, RState::Cancelled, HRR_E_CANCELLED, nullptr);
        sv->queue.clear();
    }
    sv->cv_work.notify_all();
    sv->cv_done.notify_all();
    for (auto& s : sv->slots)
        if (s->th.joinable()) s->th.join();
    (void)hipSetDevice(ctx->device);
    for (auto& s : sv->slots) {
        if (s->stream) (void)hipStreamSynchronize(s->stream);
        for (auto& S : s->S) release_scratch(S);
        if (s->h_stage) (void)hipHostFree(s->h_stage);
        if (s->stream) (void)hipStreamDestroy(s->stream);
    }
    if (sv->base) (void)hipFree(sv->base);
    ctx->server = nullptr;
    delete sv;
}

}  // namespace

}  // namespace hrr

using namespace hrr;

void hrr_server_shutdown(hrr_ctx* ctx) {
    if (!ctx) return;
    std::lock_guard<std::mutex> g(ctx->server_mu);
    stop_server(ctx);
}

HRR_EXPORT hrr_status hrr_server_start(hrr_ctx* ctx, const hrr_server_config* cfg) {
    if (!ctx || !cfg) return fail(HRR_E_INVALID, "hrr_server_start: null argument");
    if (cfg->hbm_budget_bytes < (1ull << 20)) return fail(HRR_E_INVALID, "hbm_budget_bytes must be >= 1 MiB");
    if (cfg->max_inflight < 1 || cfg->max_inflight > 8) return fail(HRR_E_INVALID, "max_inflight must be in [1, 8]");
    if (cfg->max_batch_eyes < 1) return fail(HRR_E_INVALID, "max_batch_eyes must be >= 1");
    if (!(cfg->overtake_ms >= 0.0f) || !isfinite(cfg->overtake_ms))
        return fail(HRR_E_INVALID, "overtake_ms must be finite and >= 0");
    if (cfg->max_batch_items < 1 || cfg->max_batch_items > kMaxItemsPerLaunch)
        return fail(HRR_E_INVALID, "max_batch_items must be in [1, %u]", kMaxItemsPerLaunch);
    const uint32_t epw = cfg->eyes_per_wave;
    if (!(epw == 0 || epw == 1 || epw == 2 || epw == 4 || epw == 8))
        return fail(HRR_E_INVALID, "eyes_per_wave must be 0, 1, 2, 4 or 8");
    if (!(cfg->pairs_per_eye_guess > 0.0f) || !isfinite(cfg->pairs_per_eye_guess))
        return fail(HRR_E_INVALID, "pairs_per_eye_guess must be finite and > 0");
    std::lock_guard<std::mutex> g(ctx->server_mu);
    if (ctx->server) return fail(HRR_E_BUSY, "a server already runs on this context");
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    Server* sv = new Server();
    sv->ctx = ctx;
    sv->cfg = *cfg;
    const uint64_t budget = cfg->hbm_budget_bytes / kAlign * kAlign;
    if ((e = hipMalloc((void**)&sv->base, budget)) != hipSuccess) {
        delete sv;
        return hip_fail(e, "server arena");
    }
    sv->arena.init(budget);
    for (uint32_t k = 0; k < cfg->max_inflight; ++k) {
        auto s = std::make_unique<Slot>();
        if ((e = hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking)) != hipSuccess) {
            ctx->server = sv;
            stop_server(ctx);
            return hip_fail(e, "server stream");
        }
        sv->slots.push_back(std::move(s));
    }
    ctx->server = sv;
    for (auto& s : sv->slots) s->th = std::thread(worker, sv, s.get());
    return HRR_OK;
}

HRR_EXPORT hrr_status hrr_server_stop(hrr_ctx* ctx) {
    if (!ctx) return fail(HRR_E_INVALID, "hrr_server_stop: null context");
    hrr_server_shutdown(ctx);
    return HRR_OK;
}

// The server pointer only changes under server_mu, which the client calls
// below do not take: they are not meant to race with start/stop.
static Server* running(hrr_ctx* ctx) { return ctx ? ctx->server : nullptr; }

HRR_EXPORT hrr_status hrr_submit(hrr_ctx* ctx, const hrr_hierarchy* h, const float* eyes_xyz, uint32_t n_eyes,
                                 uint32_t width, uint32_t shift_offset, float s, uint64_t* ticket) {
    if (!ctx || !h || !ticket) return fail(HRR_E_INVALID, "hrr_submit: null argument");
    Server* sv = running(ctx);
    if (!sv) return fail(HRR_E_BUSY, "hrr_submit: server not running");
    if (h->owner != ctx) return fail(HRR_E_INVALID, "hrr_submit: hierarchy belongs to another context");
    if (n_eyes && !eyes_xyz) return fail(HRR_E_INVALID, "hrr_submit: null eye positions");
    if (width == 0) return fail(HRR_E_INVALID, "hrr_submit: width must be >= 1");
    if (!(s > 0.0f) || !isfinite(s)) return fail(HRR_E_INVALID, "hrr_submit: s must be finite and > 0");
    for (uint64_t q = 0; q < 3ull * n_eyes; ++q)
        if (!isfinite(eyes_xyz[q])) return fail(HRR_E_INVALID, "hrr_submit: non-finite eye coordinate");
    auto r = std::make_shared<Request>();
    r->h = h;
    r->n = n_eyes;
    r->width = width;
    r->offset = shift_offset;
    r->s = s;
    r->eyes.assign(eyes_xyz, eyes_xyz + 3ull * n_eyes);
    {
        std::lock_guard<std::mutex> g(sv->mu);
        if (sv->stopping) return fail(HRR_E_BUSY, "hrr_submit: server stopping");
        sv->st.submitted++;
        if (round_up((uint64_t)n_eyes * kEyeBytes) + kAlign > sv->arena.size()) {
            sv->st.rejected++;
            return fail(HRR_E_NOMEM, "hrr_submit: %u eyes exceed the server's device budget", n_eyes);
        }
        r->ticket = sv->next_ticket++;
        r->submit_s = now_s();
        sv->tickets[r->ticket] = r;
        sv->queue.push_back(r);
        *ticket = r->ticket;
    }
    sv->cv_work.notify_one();
    return HRR_OK;
}

HRR_EXPORT hrr_status hrr_poll(hrr_ctx* ctx, uint64_t ticket, const uint32_t** pairs_dev, uint64_t* n_pairs,
                               hrr_ticket_info* info) {
    Server* sv = running(ctx);
    if (!sv) return fail(HRR_E_BUSY, "hrr_poll: server not running");
    std::lock_guard<std::mutex> g(sv->mu);
    auto it = sv->tickets.find(ticket);
    if (it == sv->tickets.end()) return fail(HRR_E_INVALID, "hrr_poll: unknown ticket %llu", (unsigned long long)ticket);
    const Request& r = *it->second;
    if (info) {
        info->submit_s = r.submit_s;
        info->start_s = r.start_s;
        info->done_s = r.done_s;
        info->n_pairs = r.n_pairs;
        info->launches = r.launches;
    }
    const hrr_status st = result_of(r);
    if (st == HRR_OK) {
        if (pairs_dev) *pairs_dev = r.out_bytes ? reinterpret_cast<const uint32_t*>(sv->base + r.out_off) : nullptr;
        if (n_pairs) *n_pairs = r.n_pairs;
    }
    return st;
}

HRR_EXPORT hrr_status hrr_wait(hrr_ctx* ctx, uint64_t ticket, uint32_t timeout_ms) {
    Server* sv = running(ctx);
    if (!sv) return fail(HRR_E_BUSY, "hrr_wait: server not running");
    std::unique_lock<std::mutex> lk(sv->mu);
    auto it = sv->tickets.find(ticket);
    if (it == sv->tickets.end()) return fail(HRR_E_INVALID, "hrr_wait: unknown ticket %llu", (unsigned long long)ticket);
    ReqPtr r = it->second;
    const auto until = std::chrono::steady_clock::now() + std::chrono::milliseconds(timeout_ms);
    while (r->state == RState::Queued || r->state == RState::Running) {
        if (sv->cv_done.wait_until(lk, until) == std::cv_status::timeout &&
            (r->state == RState::Queued || r->state == RState::Running))
            return HRR_E_NOTREADY;
    }
    return result_of(*r);
}

HRR_EXPORT hrr_status hrr_result_copy(hrr_ctx* ctx, uint64_t ticket, uint32_t* dst, uint64_t capacity, void* stream) {
    Server* sv = running(ctx);
    if (!sv) return fail(HRR_E_BUSY, "hrr_result_copy: server not running");
    ReqPtr r;
    {
        std::lock_guard<std::mutex> g(sv->mu);
        auto it = sv->tickets.find(ticket);
        if (it == sv->tickets.end())
            return fail(HRR_E_INVALID, "hrr_result_copy: unknown ticket %llu", (unsigned long long)ticket);
        r = it->second;
        const hrr_status st = result_of(*r);
        if (st != HRR_OK) return st;
        if (r->n_pairs && capacity && !dst) return fail(HRR_E_INVALID, "hrr_result_copy: null destination");
        r->copying++;
    }
    const uint64_t n = std::min(r->n_pairs, capacity);
    hipError_t e = hipSuccess;
    if (n) {
        e = hipSetDevice(ctx->device);
        if (e == hipSuccess)
            e = hipMemcpyAsync(dst, sv->base + r->out_off, n * kPairBytes, hipMemcpyDeviceToDevice, (hipStream_t)stream);
        if (e == hipSuccess) e = hipStreamSynchronize((hipStream_t)stream);
    }
    {
        std::lock_guard<std::mutex> g(sv->mu);
        r->copying--;
    }
    if (e != hipSuccess) return hip_fail(e, "hrr_result_copy");
    if (r->n_pairs > capacity)
        return fail(HRR_E_OVERFLOW, "hrr_result_copy: %llu pairs exceed capacity %llu",
                    (unsigned long long)r->n_pairs, (unsigned long long)capacity);
    return HRR_OK;
}

HRR_EXPORT hrr_status hrr_cancel(hrr_ctx* ctx, uint64_t ticket) {
    Server* sv = running(ctx);
    if (!sv) return fail(HRR_E_BUSY, "hrr_cancel: server not running");
    {
        std::lock_guard<std::mutex> g(sv->mu);
        auto it = sv->tickets.find(ticket);
        if (it == sv->tickets.end())
            return fail(HRR_E_INVALID, "hrr_cancel: unknown ticket %llu", (unsigned long long)ticket);
        Request& r = *it->second;
        if (r.state != RState::Queued)
            return fail(HRR_E_BUSY, "hrr_cancel: request %llu is %s", (unsigned long long)ticket,
                        r.state == RState::Running ? "running" : "already finished");
        for (auto q = sv->queue.begin(); q != sv->queue.end(); ++q)
            if ((*q)->ticket == ticket) {
                sv->queue.erase(q);
                break;
            }
        finish_request(*sv, r, RState::Cancelled, HRR_E_CANCELLED, nullptr);
    }
    sv->cv_done.notify_all();
    sv->cv_work.notify_all();
    return HRR_OK;
}

HRR_EXPORT hrr_status hrr_release(hrr_ctx* ctx, uint64_t ticket) {
    Server* sv = running(ctx);
    if (!sv) return fail(HRR_E_BUSY, "hrr_release: server not running");
    {
        std::lock_guard<std::mutex> g(sv->mu);
        auto it = sv->tickets.find(ticket);
        if (it == sv->tickets.end())
            return fail(HRR_E_INVALID, "hrr_release: unknown ticket %llu", (unsigned long long)ticket);
        Request& r = *it->second;
        if (r.state == RState::Queued || r.state == RState::Running)
            return fail(HRR_E_BUSY, "hrr_release: request %llu has not finished", (unsigned long long)ticket);
        if (r.copying) return fail(HRR_E_BUSY, "hrr_release: request %llu is being copied", (unsigned long long)ticket);
        if (r.out_bytes) sv->arena.release(r.out_off, r.out_bytes);
        r.out_bytes = 0;
        sv->tickets.erase(it);
    }
    sv->cv_work.notify_all();
    return HRR_OK;
}

HRR_EXPORT hrr_status hrr_server_get_stats(hrr_ctx* ctx, hrr_server_stats* out) {
    if (!out) return fail(HRR_E_INVALID, "hrr_server_get_stats: null argument");
    Server* sv = running(ctx);
    if (!sv) return fail(HRR_E_BUSY, "hrr_server_get_stats: server not running");
    std::lock_guard<std::mutex> g(sv->mu);
    *out = sv->st;
    out->peak_bytes = std::max<uint64_t>(out->peak_bytes, sv->arena.peak());
    if (sv->running_launches) out->busy_s += now_s() - sv->busy_from;
    std::vector<double> v = sv->lat_ms;
    if (!v.empty()) {
        std::sort(v.begin(), v.end());
        auto pct = [&](double q) {
            const size_t i = (size_t)std::min<double>((double)v.size() - 1, floor(q * (double)(v.size() - 1) + 0.5));
            return v[i];
        };
        out->p50_ms = pct(0.50);
        out->p99_ms = pct(0.99);
        double sum = 0;
        for (double x : v) sum += x;
        out->mean_ms = sum / (double)v.size();
    }
    return HRR_OK;
}
