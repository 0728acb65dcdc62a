// Serving loop: continuous batching of independent products.
//
// Clients submit descriptors (thread-safe) and receive tickets. One
// scheduler thread per server
//   1. retires finished groups (hipEventQuery on each busy slot), releasing
//      their bytes and marking their requests done;
//   2. admits waiting requests in arrival order while the bytes held by
//      in-flight requests stay within the HBM budget (first-come first-served:
//      a request that does not fit yet blocks those behind it, so none
//      starves), up to max_group per group;
//   3. enqueues each admitted group on a free slot's stream as one grouped
//      launch sequence (moa_gemm_grouped's path) and records a completion
//      event behind it.
// Requests that arrive while groups run are admitted as soon as a slot and
// budget are free, so their work overlaps the running groups on other
// streams. A request's bytes are its operands, its result and its scratch.
#include <sys/prctl.h>

#include <chrono>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "moa_internal.h"

namespace {

int64_t now_ns() {
    return std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

struct Request {
    moa_gemm_desc d;
    uint64_t ticket = 0;
    int64_t bytes = 0;
    moa_req_info info{};
    bool done = false;
};

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    std::vector<Request *> members;
    int64_t bytes = 0;
    bool busy = false;
};

int64_t request_bytes(const moa_gemm_desc &d) {
    const int64_t es = d.dtype == MOA_F64 ? 8 : 4;
    int64_t b = (d.m * d.n + d.n * d.p + d.m * d.p) * es;
    moa::Plan pl;
    if (d.m > 0 && d.p > 0 && moa::make_plan(d, &pl) == MOA_OK) b += pl.workspace_bytes;
    return b;
}

}  // namespace

struct moa_server {
    moa_serve_cfg cfg{};
    std::mutex mu;
    std::condition_variable cv_work;    // scheduler: new submissions / stop
    std::condition_variable cv_done;    // drain: completions
    std::deque<Request *> waiting;
    std::unordered_map<uint64_t, Request *> all;
    std::vector<Slot> slots;
    uint64_t next_ticket = 1;
    int64_t held_bytes = 0;
    int64_t outstanding = 0;            // submitted and not done
    bool stop = false;
    std::thread sched;

    void run();
    bool retire_locked();
};

bool moa_server::retire_locked() {
    bool any = false;
    for (Slot &s : slots) {
        if (!s.busy) continue;
        const hipError_t q = hipEventQuery(s.done);
        if (q == hipErrorNotReady) continue;
        const int64_t t = now_ns();
        for (Request *r : s.members) {
            r->info.t_done_ns = t;
            if (q != hipSuccess) r->info.status = MOA_ERR_DEVICE;
            r->done = true;
        }
        outstanding -= (int64_t)s.members.size();
        held_bytes -= s.bytes;
        s.members.clear();
        s.bytes = 0;
        s.busy = false;
        any = true;
    }
    return any;
}

void moa_server::run() {
    (void)hipSetDevice(cfg.device);
    // the completion polls below wait 20 us; the default timer slack of a
    // thread (50 us) would stretch each of them to about 70 us
    (void)prctl(PR_SET_TIMERSLACK, 1000UL, 0UL, 0UL, 0UL);
    std::unique_lock<std::mutex> lk(mu);
    std::vector<moa_gemm_desc> descs;
    for (;;) {
        if (retire_locked()) cv_done.notify_all();
        // admit and launch while there is a free slot and admissible work
        bool launched = false;
        for (Slot &s : slots) {
            if (s.busy || waiting.empty()) continue;
            if (held_bytes + waiting.front()->bytes > cfg.hbm_budget_bytes) break;
            const int64_t t_admit = now_ns();
            while (!waiting.empty() && (int)s.members.size() < cfg.max_group &&
                   held_bytes + s.bytes + waiting.front()->bytes <= cfg.hbm_budget_bytes) {
                Request *r = waiting.front();
                waiting.pop_front();
                r->info.t_admit_ns = t_admit;
                s.bytes += r->bytes;
                s.members.push_back(r);
            }
            held_bytes += s.bytes;
            s.busy = true;
            descs.clear();
            for (Request *r : s.members) descs.push_back(r->d);
            const int64_t t_start = now_ns();
            for (Request *r : s.members) {
                r->info.t_start_ns = t_start;
                r->info.group_size = (int32_t)s.members.size();
            }
            lk.unlock();   // enqueue without blocking submitters
            moa_status st = moa::run_grouped(descs.data(), (int64_t)descs.size(), s.stream);
            hipError_t e = hipEventRecord(s.done, s.stream);
            lk.lock();
            if (st != MOA_OK || e != hipSuccess)
                for (Request *r : s.members) r->info.status = st != MOA_OK ? st : MOA_ERR_DEVICE;
            launched = true;
        }
        if (stop && outstanding == 0) break;
        bool busy = false;
        for (const Slot &s : slots) busy = busy || s.busy;
        if (launched) continue;
        if (busy) {
            // groups in flight: poll their events at a fine interval
            cv_work.wait_for(lk, std::chrono::microseconds(20));
        } else if (waiting.empty()) {
            cv_work.wait(lk, [&] { return stop || !waiting.empty(); });
        } else {
            cv_work.wait_for(lk, std::chrono::microseconds(20));
        }
    }
}

using namespace moa;

extern "C" {

moa_status moa_serve_create(const moa_serve_cfg *cfg, moa_server **out) {
    try {
        if (!cfg || !out) return fail(MOA_ERR_INVALID, "null argument");
        *out = nullptr;
        if (cfg->slots < 1 || cfg->max_group < 1 || cfg->hbm_budget_bytes <= 0)
            return fail(MOA_ERR_INVALID, "slots and max_group must be >= 1 and the budget positive");
        int ndev = 0;
        hipError_t e = hipGetDeviceCount(&ndev);
        if (e != hipSuccess) return hip_fail(e, "hipGetDeviceCount");
        if (cfg->device < 0 || cfg->device >= ndev) return fail(MOA_ERR_INVALID, "no device %d", cfg->device);
        auto *srv = new moa_server();
        srv->cfg = *cfg;
        int prev = 0;
        (void)hipGetDevice(&prev);
        (void)hipSetDevice(cfg->device);
        srv->slots.resize((size_t)cfg->slots);
        for (Slot &s : srv->slots) {
            if ((e = hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking)) != hipSuccess ||
                (e = hipEventCreateWithFlags(&s.done, hipEventDisableTiming)) != hipSuccess) {
                for (Slot &t : srv->slots) {
                    if (t.stream) (void)hipStreamDestroy(t.stream);
                    if (t.done) (void)hipEventDestroy(t.done);
                }
                (void)hipSetDevice(prev);
                delete srv;
                return hip_fail(e, "slot stream/event");
            }
        }
        (void)hipSetDevice(prev);
        srv->sched = std::thread([srv] { srv->run(); });
        *out = srv;
        return MOA_OK;
    } catch (...) {
        return fail(MOA_ERR_DEVICE, "internal error");
    }
}

moa_status moa_serve_submit(moa_server *srv, const moa_gemm_desc *desc, uint64_t *ticket) {
    try {
        if (!srv || !desc || !ticket) return fail(MOA_ERR_INVALID, "null argument");
        moa_status s = validate(*desc, true);
        if (s != MOA_OK) return s;
        Plan pl;
        if (desc->m > 0 && desc->p > 0 && (s = make_plan(*desc, &pl)) != MOA_OK) return s;
        auto *r = new Request();
        r->d = *desc;
        r->bytes = request_bytes(*desc);
        r->info.t_submit_ns = now_ns();
        r->info.status = MOA_OK;
        if (r->bytes > srv->cfg.hbm_budget_bytes) {
            const long long need = (long long)r->bytes;
            delete r;
            return fail(MOA_ERR_NOMEM, "request needs %lld bytes, budget is %lld", need,
                        (long long)srv->cfg.hbm_budget_bytes);
        }
        {
            std::lock_guard<std::mutex> lk(srv->mu);
            if (srv->stop) {
                delete r;
                return fail(MOA_ERR_INVALID, "server is shutting down");
            }
            r->ticket = srv->next_ticket++;
            srv->all[r->ticket] = r;
            srv->waiting.push_back(r);
            ++srv->outstanding;
            *ticket = r->ticket;
        }
        srv->cv_work.notify_one();
        return MOA_OK;
    } catch (...) {
        return fail(MOA_ERR_DEVICE, "internal error");
    }
}

moa_status moa_serve_poll(moa_server *srv, uint64_t ticket, moa_req_info *out) {
    if (!srv || !out) return fail(MOA_ERR_INVALID, "null argument");
    std::lock_guard<std::mutex> lk(srv->mu);
    auto it = srv->all.find(ticket);
    if (it == srv->all.end()) return fail(MOA_ERR_INVALID, "unknown ticket %llu", (unsigned long long)ticket);
    if (!it->second->done) return MOA_NOT_READY;
    *out = it->second->info;
    return MOA_OK;
}

moa_status moa_serve_release(moa_server *srv, uint64_t ticket) {
    if (!srv) return fail(MOA_ERR_INVALID, "null server");
    std::lock_guard<std::mutex> lk(srv->mu);
    auto it = srv->all.find(ticket);
    if (it == srv->all.end()) return fail(MOA_ERR_INVALID, "unknown ticket %llu", (unsigned long long)ticket);
    if (!it->second->done) return MOA_NOT_READY;
    // a done request is referenced by no queue or slot any more
    delete it->second;
    srv->all.erase(it);
    return MOA_OK;
}

moa_status moa_serve_drain(moa_server *srv) {
    if (!srv) return fail(MOA_ERR_INVALID, "null server");
    std::unique_lock<std::mutex> lk(srv->mu);
    srv->cv_done.wait(lk, [&] { return srv->outstanding == 0; });
    return MOA_OK;
}

moa_status moa_serve_destroy(moa_server *srv) {
    if (!srv) return MOA_OK;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->stop = true;
    }
    srv->cv_work.notify_all();
    if (srv->sched.joinable()) srv->sched.join();
    for (Slot &s : srv->slots) {
        (void)hipStreamSynchronize(s.stream);
        (void)hipStreamDestroy(s.stream);
        (void)hipEventDestroy(s.done);
    }
    for (auto &kv : srv->all) delete kv.second;
    delete srv;
    return MOA_OK;
}

}  // extern "C"
