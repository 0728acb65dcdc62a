// Host-only test of the serving scheduler (paper_2306_11148_amd/csrc/serve_core.cpp)
// against a fake device: failures of launches, completion markers and the
// device itself, memory exhaustion, the HBM budget, first-come first-served
// admission, the batching window and the pool's block handling. Built with
// g++ and run by tests/test_serve_host.py; no GPU and no HIP involved.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "serve_core.h"

using moa::serve::Backend;
using moa::serve::Pool;
using moa::serve::Server;

namespace {

int g_failures = 0;

#define CHECK(cond, ...)                                                              \
    do {                                                                              \
        if (!(cond)) {                                                                \
            std::printf("FAIL %s:%d: %s: ", __FILE__, __LINE__, #cond);               \
            std::printf(__VA_ARGS__);                                                 \
            std::printf("\n");                                                        \
            ++g_failures;                                                             \
        }                                                                             \
    } while (0)

struct Fake final : Backend {
    std::mutex mu;
    int64_t device_cap = int64_t(1) << 40;   // bytes the fake device can hand out
    int64_t device_used = 0;
    int device_allocs = 0;
    std::map<char *, int64_t> chunks;         // live device allocations
    int64_t scratch_per_member = 256;         // scratch model: this + 4 m p per member
    struct SlotState {
        bool pending = false;
        int polls_left = 0;
        moa_status outcome = MOA_OK;
    };
    std::vector<SlotState> slots;
    int polls_to_finish = 2;
    std::atomic<bool> hold{false};            // no completion while set
    int launches = 0;
    int fail_launch_at = -1, fail_mark_at = -1, fail_query_at = -1;
    std::vector<int> group_sizes;
    struct FillRec { float *x; int64_t count; uint64_t seed; uint32_t tag; };
    std::vector<FillRec> fills;
    std::vector<std::string> errors;

    explicit Fake(int nslots) : slots((size_t)nslots) {}

    void *device_alloc(int64_t bytes) override {
        std::lock_guard<std::mutex> lk(mu);
        if (device_used + bytes > device_cap) return nullptr;
        char *p = static_cast<char *>(std::aligned_alloc(256, (size_t)((bytes + 255) / 256 * 256)));
        if (!p) return nullptr;
        chunks[p] = bytes;
        device_used += bytes;
        ++device_allocs;
        return p;
    }
    void device_free(void *p) override {
        std::lock_guard<std::mutex> lk(mu);
        auto it = chunks.find(static_cast<char *>(p));
        if (it == chunks.end()) {
            errors.push_back("free of unknown chunk");
            return;
        }
        device_used -= it->second;
        chunks.erase(it);
        std::free(p);
    }
    bool inside(const void *p, int64_t bytes) {
        for (auto &kv : chunks)
            if (static_cast<const char *>(p) >= kv.first && static_cast<const char *>(p) + bytes <= kv.first + kv.second)
                return true;
        return false;
    }
    int64_t group_scratch_bytes(const moa_gemm_desc *d, int64_t count) override {
        int64_t s = 0;
        for (int64_t g = 0; g < count; ++g) s += scratch_per_member + 4 * d[g].m * d[g].p;
        return s;
    }
    moa_status fill(int, float *x, int64_t count, uint64_t seed, uint32_t tag) override {
        std::lock_guard<std::mutex> lk(mu);
        if (count > 0 && !inside(x, 4 * count)) errors.push_back("fill outside the pool");
        fills.push_back({x, count, seed, tag});
        return MOA_OK;
    }
    moa_status launch(int slot, const moa_gemm_desc *d, int64_t count, void *scratch, int64_t bytes) override {
        std::lock_guard<std::mutex> lk(mu);
        const int seq = launches++;
        group_sizes.push_back((int)count);
        if (bytes > 0 && !inside(scratch, bytes)) errors.push_back("scratch outside the pool");
        for (int64_t g = 0; g < count; ++g)
            if (d[g].m * d[g].p > 0 && !d[g].C) errors.push_back("member without C");
        slots[(size_t)slot].pending = true;
        slots[(size_t)slot].polls_left = polls_to_finish;
        slots[(size_t)slot].outcome = seq == fail_query_at ? MOA_ERR_DEVICE : MOA_OK;
        return seq == fail_launch_at ? MOA_ERR_DEVICE : MOA_OK;
    }
    moa_status mark(int) override {
        std::lock_guard<std::mutex> lk(mu);
        return launches - 1 == fail_mark_at ? MOA_ERR_DEVICE : MOA_OK;
    }
    moa_status query(int slot) override {
        std::lock_guard<std::mutex> lk(mu);
        SlotState &s = slots[(size_t)slot];
        if (hold) return MOA_NOT_READY;
        if (s.polls_left > 0) {
            --s.polls_left;
            return MOA_NOT_READY;
        }
        s.pending = false;
        return s.outcome;
    }
    void wait(int slot) override {
        std::lock_guard<std::mutex> lk(mu);
        slots[(size_t)slot].pending = false;
        slots[(size_t)slot].polls_left = 0;
    }
};

moa_serve_cfg cfg(int64_t budget, int slots, int max_group, int window_us = 0) {
    moa_serve_cfg c{};
    c.hbm_budget_bytes = budget;
    c.slots = slots;
    c.max_group = max_group;
    c.device = 0;
    c.batch_window_us = window_us;
    return c;
}

moa_synth_request synth(int64_t m, int64_t n, int64_t p, uint64_t seed) {
    moa_synth_request r{};
    r.m = m;
    r.n = n;
    r.p = p;
    r.path = MOA_PATH_SPLIT_BF16;
    r.seed = seed;
    return r;
}

int64_t a256(int64_t x) { return (x + 255) / 256 * 256; }
// bytes a synthetic request reserves under the fake scratch model
int64_t reserve_of(const Fake &f, int64_t m, int64_t n, int64_t p) {
    return a256(4 * m * n) + a256(4 * n * p) + a256(4 * m * p) + a256(f.scratch_per_member + 4 * m * p);
}

moa_req_info info_of(Server &s, uint64_t t) {
    moa_req_info i{};
    const moa_status st = s.poll(t, &i);
    CHECK(st == MOA_OK, "poll of ticket %llu gave %d", (unsigned long long)t, (int)st);
    return i;
}

void test_pool_blocks() {
    Fake f(1);
    Pool pool(&f, int64_t(4) << 20);
    void *a = pool.alloc(1000), *b = pool.alloc(3000), *c = pool.alloc(256);
    CHECK(a && b && c, "small allocations");
    CHECK(pool.live_bytes() == 1024 + 3072 + 256, "live %lld", (long long)pool.live_bytes());
    CHECK(pool.chunk_bytes() == (int64_t(4) << 20), "one chunk clipped to the cap: %lld", (long long)pool.chunk_bytes());
    CHECK((uintptr_t)b % 256 == 0 && (uintptr_t)c % 256 == 0, "256-byte alignment");
    pool.release(b);
    pool.release(a);                      // a and b merge into one 4 KiB hole
    void *d = pool.alloc(4096);
    CHECK(d == a, "merged hole reused first-fit");
    pool.trim();                          // blocks live: no-op
    CHECK(pool.chunk_bytes() > 0 && f.device_used > 0, "trim keeps chunks with live blocks");
    void *big = pool.alloc(int64_t(8) << 20);
    CHECK(!big, "beyond the cap");
    pool.release(c);
    pool.release(d);
    CHECK(pool.live_bytes() == 0, "all released");
    pool.trim();
    CHECK(pool.chunk_bytes() == 0 && f.device_used == 0, "trim returns every chunk");
    std::printf("ok pool_blocks\n");
}

void test_synthetic_lifecycle() {
    Fake f(2);
    const int64_t r1 = reserve_of(f, 16, 24, 8);
    {
        Server s(cfg(int64_t(1) << 20, 2, 4), &f);
        std::vector<uint64_t> t(10);
        for (int k = 0; k < 10; ++k) CHECK(s.submit_synthetic(synth(16, 24, 8, 100 + k), &t[k]) == MOA_OK, "submit");
        s.drain();
        for (int k = 0; k < 10; ++k) {
            const moa_req_info i = info_of(s, t[k]);
            CHECK(i.status == MOA_OK, "status %d", i.status);
            CHECK(i.t_submit_ns <= i.t_admit_ns && i.t_admit_ns <= i.t_start_ns && i.t_start_ns <= i.t_done_ns,
                  "timestamps ordered");
            const void *C = nullptr;
            int64_t bytes = 0;
            CHECK(s.result(t[k], &C, &bytes) == MOA_OK && C && bytes == 16 * 8 * 4, "result");
        }
        moa_serve_state st{};
        s.stats(&st);
        CHECK(st.held_bytes == 10 * a256(16 * 8 * 4), "results stay held until release: %lld", (long long)st.held_bytes);
        CHECK(st.peak_held_bytes <= (int64_t(1) << 20) && st.peak_pool_bytes <= (int64_t(1) << 20), "within budget");
        CHECK(st.completed == 10 && st.failed == 0, "counts");
        // two fills per request, A then B, with the request's seed
        CHECK(f.fills.size() == 20, "fills %zu", f.fills.size());
        std::map<uint64_t, int> tags;
        for (auto &x : f.fills) {
            tags[x.seed] |= 1 << x.tag;
            CHECK(x.count == (x.tag == 0 ? 16 * 24 : 24 * 8), "fill count");
        }
        for (int k = 0; k < 10; ++k) CHECK(tags[100 + k] == 3, "A and B drawn for seed %d", 100 + k);
        for (int k = 0; k < 10; ++k) CHECK(s.release(t[k]) == MOA_OK, "release");
        CHECK(s.release(t[0]) == MOA_ERR_INVALID, "double release");
        s.stats(&st);
        CHECK(st.held_bytes == 0, "nothing held after release");
        (void)r1;
    }
    CHECK(f.device_used == 0, "the pool returns its chunks when the server ends");
    CHECK(f.errors.empty(), "%s", f.errors.empty() ? "" : f.errors[0].c_str());
    std::printf("ok synthetic_lifecycle\n");
}

void test_device_error_on_completion() {
    Fake f(1);
    f.fail_query_at = 0;                  // the first group fails on the device
    Server s(cfg(int64_t(1) << 20, 1, 1), &f);
    uint64_t t[3];
    for (int k = 0; k < 3; ++k) s.submit_synthetic(synth(8, 8, 8, k), &t[k]);
    s.drain();
    CHECK(info_of(s, t[0]).status == MOA_ERR_DEVICE, "failed group reported");
    CHECK(info_of(s, t[1]).status == MOA_OK && info_of(s, t[2]).status == MOA_OK, "later requests still served");
    moa_serve_state st{};
    s.stats(&st);
    CHECK(st.failed == 1 && st.completed == 3, "counts %lld %lld", (long long)st.failed, (long long)st.completed);
    for (uint64_t x : t) s.release(x);
    s.stats(&st);
    CHECK(st.held_bytes == 0, "bytes of the failed request released");
    CHECK(f.errors.empty(), "%s", f.errors.empty() ? "" : f.errors[0].c_str());
    std::printf("ok device_error_on_completion\n");
}

void test_launch_and_marker_failures() {
    Fake f(1);
    f.fail_launch_at = 0;
    f.fail_mark_at = 1;
    Server s(cfg(int64_t(1) << 20, 1, 1), &f);
    uint64_t t[3];
    for (int k = 0; k < 3; ++k) s.submit_synthetic(synth(8, 8, 8, k), &t[k]);
    s.drain();
    CHECK(info_of(s, t[0]).status == MOA_ERR_DEVICE, "launch failure reported");
    CHECK(info_of(s, t[1]).status == MOA_ERR_DEVICE, "marker failure reported");
    CHECK(info_of(s, t[2]).status == MOA_OK, "then served again");
    CHECK(f.errors.empty(), "%s", f.errors.empty() ? "" : f.errors[0].c_str());
    std::printf("ok launch_and_marker_failures\n");
}

void test_device_out_of_memory() {
    Fake f(2);
    f.device_cap = 0;                     // the device has nothing to give
    Server s(cfg(int64_t(1) << 20, 2, 4), &f);
    uint64_t a, b;
    CHECK(s.submit_synthetic(synth(8, 8, 8, 1), &a) == MOA_OK, "submit");
    moa_gemm_desc d{};                    // caller-owned operands, scratch from the pool
    d.m = d.n = d.p = 8;
    d.dtype = MOA_F32;
    d.path = MOA_PATH_SPLIT_BF16;
    static float buf[3 * 64];
    d.A = buf;
    d.B = buf + 64;
    d.C = buf + 128;
    CHECK(s.submit(d, &b) == MOA_OK, "submit");
    s.drain();                            // must return: the requests fail instead of waiting
    CHECK(info_of(s, a).status == MOA_ERR_NOMEM, "synthetic request without device memory");
    CHECK(info_of(s, b).status == MOA_ERR_NOMEM, "scratch without device memory");
    CHECK(f.launches == 0, "nothing launched");
    CHECK(f.errors.empty(), "%s", f.errors.empty() ? "" : f.errors[0].c_str());
    std::printf("ok device_out_of_memory\n");
}

void test_budget_and_fcfs() {
    Fake f(4);
    f.polls_to_finish = 20;
    const int64_t small = reserve_of(f, 32, 32, 32), big = reserve_of(f, 64, 256, 64);
    const int64_t budget = big + small;   // the big request never runs beside more than one small one
    Server s(cfg(budget, 4, 2), &f);
    moa_synth_request too = synth(512, 512, 512, 9);
    uint64_t x;
    CHECK(s.submit_synthetic(too, &x) == MOA_ERR_NOMEM, "a request beyond the whole budget is refused at submit");
    std::vector<uint64_t> t;
    for (int k = 0; k < 24; ++k) {
        uint64_t q;
        s.submit_synthetic(k % 6 == 3 ? synth(64, 256, 64, k) : synth(32, 32, 32, k), &q);
        t.push_back(q);
    }
    // the client reads and releases each result as it completes: results
    // that stay unreleased keep counting against the budget
    std::vector<moa_req_info> infos(t.size());
    std::vector<bool> got(t.size(), false);
    for (size_t left = t.size(); left > 0;) {
        for (size_t k = 0; k < t.size(); ++k) {
            if (got[k] || s.poll(t[k], &infos[k]) != MOA_OK) continue;
            CHECK(s.release(t[k]) == MOA_OK, "release");
            got[k] = true;
            --left;
        }
        std::this_thread::sleep_for(std::chrono::microseconds(200));
    }
    moa_serve_state st{};
    s.stats(&st);
    CHECK(st.peak_held_bytes <= budget, "peak held %lld > budget %lld", (long long)st.peak_held_bytes, (long long)budget);
    CHECK(st.peak_pool_bytes <= budget, "pool %lld > budget %lld", (long long)st.peak_pool_bytes, (long long)budget);
    CHECK(st.held_bytes == 0, "nothing held after every release");
    int64_t last_admit = 0;
    for (size_t k = 0; k < t.size(); ++k) {
        CHECK(infos[k].status == MOA_OK, "status");
        CHECK(infos[k].t_admit_ns >= last_admit, "admission in arrival order (ticket %zu)", k);
        last_admit = infos[k].t_admit_ns;
    }
    CHECK(f.errors.empty(), "%s", f.errors.empty() ? "" : f.errors[0].c_str());
    std::printf("ok budget_and_fcfs\n");
}

void test_release_frees_budget_for_waiting_requests() {
    Fake f(1);
    const int64_t one = reserve_of(f, 16, 16, 16);
    Server s(cfg(one + a256(16 * 16 * 4), 1, 1), &f);   // room for one request and one held result
    uint64_t t[3];
    for (int k = 0; k < 3; ++k) s.submit_synthetic(synth(16, 16, 16, k), &t[k]);
    moa_req_info i{};
    while (s.poll(t[1], &i) == MOA_NOT_READY) {
        if (s.poll(t[0], &i) == MOA_OK && s.release(t[0]) == MOA_OK) {}
        std::this_thread::sleep_for(std::chrono::milliseconds(1));
    }
    CHECK(s.release(t[1]) == MOA_OK, "release");
    s.drain();
    CHECK(info_of(s, t[2]).status == MOA_OK, "third served once results were released");
    CHECK(f.errors.empty(), "%s", f.errors.empty() ? "" : f.errors[0].c_str());
    std::printf("ok release_frees_budget\n");
}

void test_batching_window() {
    Fake f(1);
    {
        Server s(cfg(int64_t(1) << 24, 1, 4, 200000), &f);   // 200 ms window
        uint64_t t[4];
        for (int k = 0; k < 4; ++k) s.submit_synthetic(synth(8, 8, 8, k), &t[k]);
        s.drain();
        for (uint64_t x : t) CHECK(info_of(s, x).group_size == 4, "a full group launches without waiting");
        uint64_t u[2];
        for (int k = 0; k < 2; ++k) s.submit_synthetic(synth(8, 8, 8, 10 + k), &u[k]);
        s.drain();
        const moa_req_info i = info_of(s, u[0]);
        CHECK(i.group_size == 2, "a partial group launches once the window has passed: %d", i.group_size);
        CHECK(i.t_admit_ns - i.t_submit_ns >= 190000000, "held open for the window: %lld ns",
              (long long)(i.t_admit_ns - i.t_submit_ns));
    }
    {
        Fake g(1);
        Server s(cfg(int64_t(1) << 24, 1, 4, 0), &g);
        g.hold = true;                    // first group stays on the device while three more arrive
        uint64_t t[4];
        s.submit_synthetic(synth(8, 8, 8, 0), &t[0]);
        std::this_thread::sleep_for(std::chrono::milliseconds(20));
        for (int k = 1; k < 4; ++k) s.submit_synthetic(synth(8, 8, 8, k), &t[k]);
        std::this_thread::sleep_for(std::chrono::milliseconds(20));
        g.hold = false;
        s.drain();
        CHECK(info_of(s, t[0]).group_size == 1, "no window: the first request launches alone");
        CHECK(info_of(s, t[1]).group_size == 3, "requests that arrived meanwhile form the next group");
    }
    std::printf("ok batching_window\n");
}

void test_pool_reserve() {
    {
        Fake f(2);
        moa_serve_cfg c = cfg(int64_t(64) << 20, 2, 4);
        c.pool_reserve_bytes = int64_t(8) << 20;
        Server s(c, &f);
        CHECK(s.reserved() && f.device_allocs == 1 && f.device_used == (int64_t(8) << 20), "reserve taken at creation");
        std::vector<uint64_t> t(12);
        for (int k = 0; k < 12; ++k) s.submit_synthetic(synth(32, 48, 40, k), &t[k]);
        s.drain();
        for (uint64_t x : t) {
            CHECK(info_of(s, x).status == MOA_OK, "served");
            s.release(x);
        }
        CHECK(f.device_allocs == 1, "no allocation while serving within the reserve: %d", f.device_allocs);
        CHECK(f.errors.empty(), "%s", f.errors.empty() ? "" : f.errors[0].c_str());
    }
    {
        Fake f(1);
        f.device_cap = int64_t(1) << 20;
        moa_serve_cfg c = cfg(int64_t(64) << 20, 1, 1);
        c.pool_reserve_bytes = int64_t(8) << 20;
        Server s(c, &f);
        CHECK(!s.reserved(), "a reserve the device cannot give is reported");
    }
    std::printf("ok pool_reserve\n");
}

void test_ticket_errors() {
    Fake f(1);
    f.hold = true;
    Server s(cfg(int64_t(1) << 20, 1, 1), &f);
    uint64_t t;
    s.submit_synthetic(synth(8, 8, 8, 1), &t);
    moa_req_info i{};
    const void *C = nullptr;
    int64_t bytes = 0;
    CHECK(s.poll(t, &i) == MOA_NOT_READY, "running");
    CHECK(s.result(t, &C, &bytes) == MOA_NOT_READY, "no result yet");
    CHECK(s.release(t) == MOA_NOT_READY, "cannot release a running request");
    CHECK(s.poll(t + 100, &i) == MOA_ERR_INVALID, "unknown ticket");
    f.hold = false;
    s.drain();
    CHECK(s.poll(t, &i) == MOA_OK, "done");
    CHECK(f.errors.empty(), "%s", f.errors.empty() ? "" : f.errors[0].c_str());
    std::printf("ok ticket_errors\n");
}

}  // namespace

int main() {
    test_pool_blocks();
    test_synthetic_lifecycle();
    test_device_error_on_completion();
    test_launch_and_marker_failures();
    test_device_out_of_memory();
    test_budget_and_fcfs();
    test_release_frees_budget_for_waiting_requests();
    test_batching_window();
    test_ticket_errors();
    test_pool_reserve();
    if (g_failures) {
        std::printf("%d failure(s)\n", g_failures);
        return 1;
    }
    std::printf("all ok\n");
    return 0;
}
