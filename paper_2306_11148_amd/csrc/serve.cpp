// Serving loop on HIP: the scheduler of serve_core.h driven through one
// stream and one completion event per slot. The pool's chunks are plain
// device allocations of the server; a group's scratch is carved from them
// (run_grouped with an arena), synthetic operands are drawn on the slot's
// stream right before the group's launch.
#include <memory>

#include "moa_internal.h"
#include "serve_core.h"

namespace {

class HipBackend final : public moa::serve::Backend {
  public:
    explicit HipBackend(int device) : device_(device) {}
    ~HipBackend() override {
        for (size_t k = 0; k < streams_.size(); ++k) {
            if (streams_[k]) {
                (void)hipStreamSynchronize(streams_[k]);
                (void)hipStreamDestroy(streams_[k]);
            }
            if (events_[k]) (void)hipEventDestroy(events_[k]);
        }
    }

    moa_status init(int slots) {
        int prev = 0;
        (void)hipGetDevice(&prev);
        (void)hipSetDevice(device_);
        streams_.assign((size_t)slots, nullptr);
        events_.assign((size_t)slots, nullptr);
        moa_status s = MOA_OK;
        for (int k = 0; k < slots && s == MOA_OK; ++k) {
            hipError_t e;
            if ((e = hipStreamCreateWithFlags(&streams_[k], hipStreamNonBlocking)) != hipSuccess ||
                (e = hipEventCreateWithFlags(&events_[k], hipEventDisableTiming)) != hipSuccess)
                s = moa::hip_fail(e, "slot stream/event");
        }
        (void)hipSetDevice(prev);
        return s;
    }

    void thread_start() override { (void)hipSetDevice(device_); }

    void *device_alloc(int64_t bytes) override {
        void *p = nullptr;
        if (hipMalloc(&p, (size_t)bytes) != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
        return p;
    }
    void device_free(void *p) override { (void)hipFree(p); }

    int64_t group_scratch_bytes(const moa_gemm_desc *d, int64_t count) override {
        return moa::grouped_scratch_bytes(d, count);
    }

    moa_status fill(int slot, float *x, int64_t count, uint64_t seed, uint32_t tag) override {
        const hipError_t e = moa::launch_synthetic(x, count, seed, tag, streams_[slot]);
        return e == hipSuccess ? MOA_OK : moa::hip_fail(e, "synthetic fill");
    }

    moa_status launch(int slot, const moa_gemm_desc *d, int64_t count, void *scratch, int64_t bytes) override {
        moa::ScratchArena arena;
        arena.base = scratch;
        arena.size = scratch ? bytes : 0;
        return moa::run_grouped(d, count, streams_[slot], &arena);
    }

    moa_status mark(int slot) override {
        const hipError_t e = hipEventRecord(events_[slot], streams_[slot]);
        return e == hipSuccess ? MOA_OK : moa::hip_fail(e, "completion event");
    }

    moa_status query(int slot) override {
        const hipError_t q = hipEventQuery(events_[slot]);
        if (q == hipSuccess) return MOA_OK;
        if (q == hipErrorNotReady) return MOA_NOT_READY;
        (void)hipGetLastError();
        return MOA_ERR_DEVICE;
    }

    void wait(int slot) override {
        if ((size_t)slot < streams_.size() && streams_[slot]) (void)hipStreamSynchronize(streams_[slot]);
    }

  private:
    int device_;
    std::vector<hipStream_t> streams_;
    std::vector<hipEvent_t> events_;
};

}  // namespace

// The backend outlives the scheduler: members are destroyed in reverse order.
struct moa_server {
    HipBackend backend;
    std::unique_ptr<moa::serve::Server> server;
    int64_t budget;
    explicit moa_server(int device, int64_t b) : backend(device), budget(b) {}
};

using namespace moa;

namespace {

moa_status status_of(moa_status s, moa_server *srv, uint64_t ticket) {
    switch (s) {
    case MOA_ERR_INVALID: return fail(s, "unknown ticket %llu", (unsigned long long)ticket);
    case MOA_ERR_NOMEM: return fail(s, "request needs more than the budget of %lld bytes", (long long)srv->budget);
    default: return s;
    }
}

}  // namespace

extern "C" {

moa_status moa_serve_create(const moa_serve_cfg *cfg, moa_server **out) {
    try {
        if (!cfg || !out) return fail(MOA_ERR_INVALID, "null argument");
        *out = nullptr;
        if (cfg->slots < 1 || cfg->max_group < 1 || cfg->hbm_budget_bytes <= 0 || cfg->batch_window_us < 0 ||
            cfg->pool_reserve_bytes < 0 || cfg->pool_reserve_bytes > cfg->hbm_budget_bytes)
            return fail(MOA_ERR_INVALID, "slots and max_group must be >= 1, the budget positive, the window not "
                                         "negative and the reserve within the budget");
        int ndev = 0, prev = 0;
        hipError_t e = hipGetDeviceCount(&ndev);
        if (e != hipSuccess) return hip_fail(e, "hipGetDeviceCount");
        if (cfg->device < 0 || cfg->device >= ndev) return fail(MOA_ERR_INVALID, "no device %d", cfg->device);
        auto *srv = new moa_server(cfg->device, cfg->hbm_budget_bytes);
        moa_status s = srv->backend.init(cfg->slots);
        if (s != MOA_OK) {
            delete srv;
            return s;
        }
        (void)hipGetDevice(&prev);
        (void)hipSetDevice(cfg->device);       // the reserve is allocated on the server's device
        srv->server.reset(new serve::Server(*cfg, &srv->backend));
        (void)hipSetDevice(prev);
        if (!srv->server->reserved()) {
            const long long want = (long long)cfg->pool_reserve_bytes;
            srv->server.reset();
            delete srv;
            return fail(MOA_ERR_NOMEM, "pool reserve of %lld bytes", want);
        }
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
        s = srv->server->submit(*desc, ticket);
        if (s == MOA_ERR_INVALID) return fail(s, "server is shutting down");
        return status_of(s, srv, 0);
    } catch (...) {
        return fail(MOA_ERR_DEVICE, "internal error");
    }
}

moa_status moa_serve_submit_synthetic(moa_server *srv, const moa_synth_request *req, uint64_t *ticket) {
    try {
        if (!srv || !req || !ticket) return fail(MOA_ERR_INVALID, "null argument");
        if (req->flags & MOA_FLAG_LAYOUT_MASK)
            return fail(MOA_ERR_INVALID, "synthetic operands are row-major: no layout flags");
        moa_gemm_desc d{};
        d.m = req->m;
        d.n = req->n;
        d.p = req->p;
        d.dtype = MOA_F32;
        d.path = (moa_path)req->path;
        d.flags = req->flags;
        moa_status s = validate(d, false);
        if (s != MOA_OK) return s;
        Plan pl;
        if (d.m > 0 && d.p > 0 && (s = make_plan(d, &pl)) != MOA_OK) return s;
        s = srv->server->submit_synthetic(*req, ticket);
        if (s == MOA_ERR_INVALID) return fail(s, "server is shutting down");
        return status_of(s, srv, 0);
    } catch (...) {
        return fail(MOA_ERR_DEVICE, "internal error");
    }
}

moa_status moa_serve_poll(moa_server *srv, uint64_t ticket, moa_req_info *out) {
    if (!srv || !out) return fail(MOA_ERR_INVALID, "null argument");
    return status_of(srv->server->poll(ticket, out), srv, ticket);
}

moa_status moa_serve_result(moa_server *srv, uint64_t ticket, const void **C) {
    if (!srv || !C) return fail(MOA_ERR_INVALID, "null argument");
    int64_t bytes = 0;
    return status_of(srv->server->result(ticket, C, &bytes), srv, ticket);
}

moa_status moa_serve_read(moa_server *srv, uint64_t ticket, void *dst, int64_t dst_bytes) {
    try {
        if (!srv || !dst) return fail(MOA_ERR_INVALID, "null argument");
        const void *C = nullptr;
        int64_t bytes = 0;
        moa_status s = srv->server->result(ticket, &C, &bytes);
        if (s != MOA_OK) return status_of(s, srv, ticket);
        if (dst_bytes < bytes) return fail(MOA_ERR_INVALID, "destination holds %lld bytes, C has %lld",
                                           (long long)dst_bytes, (long long)bytes);
        if (bytes == 0) return MOA_OK;
        const hipError_t e = hipMemcpy(dst, C, (size_t)bytes, hipMemcpyDefault);
        if (e != hipSuccess) return hip_fail(e, "copy of a result");
        return MOA_OK;
    } catch (...) {
        return fail(MOA_ERR_DEVICE, "internal error");
    }
}

moa_status moa_serve_release(moa_server *srv, uint64_t ticket) {
    if (!srv) return fail(MOA_ERR_INVALID, "null server");
    return status_of(srv->server->release(ticket), srv, ticket);
}

moa_status moa_serve_drain(moa_server *srv) {
    if (!srv) return fail(MOA_ERR_INVALID, "null server");
    srv->server->drain();
    return MOA_OK;
}

moa_status moa_serve_stats(moa_server *srv, moa_serve_state *out) {
    if (!srv || !out) return fail(MOA_ERR_INVALID, "null argument");
    srv->server->stats(out);
    return MOA_OK;
}

moa_status moa_serve_destroy(moa_server *srv) {
    if (!srv) return MOA_OK;
    srv->server.reset();
    delete srv;
    return MOA_OK;
}

}  // extern "C"
