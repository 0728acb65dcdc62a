// The serving scheduler, written against an abstract device so that its
// admission, batching, memory and failure handling build and run without a
// GPU. serve.cpp binds it to HIP streams, events and kernels.
//
// Clients submit requests (thread-safe) and receive tickets. One scheduler
// thread per server
//   1. retires finished groups (each slot's completion marker), releasing
//      their bytes and marking their requests done;
//   2. admits waiting requests in arrival order while the bytes they hold
//      stay within the budget (first-come first-served: a request that does
//      not fit yet blocks those behind it, so none starves), up to max_group
//      per group; with a batching window it holds a group open until the
//      window since its oldest request has passed or the group is full;
//   3. enqueues each admitted group on a free slot: the synthetic operands of
//      its members are drawn on the device, then one grouped launch runs,
//      then a completion marker.
// Requests that arrive while groups run are admitted as soon as a slot and
// budget are free, so their work overlaps the running groups on other slots.
//
// Memory. All device memory the server uses -- the operands and results of
// synthetic requests and the scratch of every group -- comes from its pool,
// whose chunks never total more than the budget. A request counts against
// the budget from admission: its operands and result (caller-owned ones
// included) and the scratch it would take as a one-member group; a synthetic
// request's result stays counted until the client releases it.
#pragma once

#include <condition_variable>
#include <cstdint>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "moa.h"

namespace moa {
namespace serve {

// What the scheduler needs from the device. Calls naming a slot are issued in
// order on that slot's queue; only query and wait look at the device's
// progress.
class Backend {
  public:
    virtual ~Backend() = default;
    virtual void thread_start() {}
    // device memory for the pool; nullptr when the device has none to give
    virtual void *device_alloc(int64_t bytes) = 0;
    virtual void device_free(void *p) = 0;
    // scratch bytes of one grouped launch over `descs` (pointers unused)
    virtual int64_t group_scratch_bytes(const moa_gemm_desc *descs, int64_t count) = 0;
    // enqueue on `slot`: the synthetic draw of `count` floats, the grouped
    // launch (scratch from the given block), the completion marker
    virtual moa_status fill(int slot, float *x, int64_t count, uint64_t seed, uint32_t tag) = 0;
    virtual moa_status launch(int slot, const moa_gemm_desc *descs, int64_t count, void *scratch,
                              int64_t scratch_bytes) = 0;
    virtual moa_status mark(int slot) = 0;
    // MOA_OK once the work before the marker has finished, MOA_NOT_READY
    // before, MOA_ERR_DEVICE if it failed
    virtual moa_status query(int slot) = 0;
    // blocks until everything enqueued on `slot` has finished
    virtual void wait(int slot) = 0;
};

// Device memory of one server: chunks taken from the backend while their
// total stays within `cap`, carved first-fit into 256-byte aligned blocks,
// neighbouring free blocks merged on release.
class Pool {
  public:
    static constexpr int64_t kChunk = int64_t(512) << 20;
    Pool(Backend *b, int64_t cap) : b_(b), cap_(cap) {}
    ~Pool();
    Pool(const Pool &) = delete;
    Pool &operator=(const Pool &) = delete;
    void *alloc(int64_t bytes);          // nullptr if no block can be found or added
    bool reserve(int64_t bytes);         // one chunk of `bytes` now (within the cap)
    void release(void *p);
    void trim();                         // with no live block: every chunk back to the backend
    int64_t live_bytes() const { return live_; }
    int64_t chunk_bytes() const { return total_; }

  private:
    struct Chunk {
        char *base = nullptr;
        int64_t size = 0;
        std::map<int64_t, int64_t> free;   // offset -> size
    };
    void *carve(size_t c, int64_t bytes);
    Backend *b_;
    int64_t cap_;
    std::vector<Chunk> chunks_;
    std::unordered_map<const void *, std::pair<size_t, int64_t>> blocks_;   // block -> (chunk, size)
    int64_t live_ = 0, total_ = 0;
};

class Server {
  public:
    // reserves cfg.pool_reserve_bytes (reserved() says whether that worked)
    Server(const moa_serve_cfg &cfg, Backend *b);
    ~Server();                           // waits for every submitted request, then stops
    bool reserved() const { return reserved_; }
    Server(const Server &) = delete;
    Server &operator=(const Server &) = delete;

    // `d` validated by the caller; its operands are caller-owned
    moa_status submit(const moa_gemm_desc &d, uint64_t *ticket);
    // `r` validated by the caller (FP32, row-major)
    moa_status submit_synthetic(const moa_synth_request &r, uint64_t *ticket);
    moa_status poll(uint64_t ticket, moa_req_info *out);
    // result of a finished request: device address and bytes of C
    moa_status result(uint64_t ticket, const void **C, int64_t *bytes);
    moa_status release(uint64_t ticket);
    void drain();
    void stats(moa_serve_state *out);

  private:
    struct Request {
        moa_gemm_desc d{};
        bool synthetic = false;
        uint64_t seed = 0;
        uint64_t ticket = 0;
        int64_t reserve = 0;       // counted against the budget from admission
        int64_t scratch = 0;       // the part of `reserve` that is one-member scratch
        int64_t keep = 0;          // still counted once done (a synthetic result)
        int64_t a_bytes = 0, b_bytes = 0, c_bytes = 0;
        void *ab = nullptr;        // synthetic A and B
        void *c = nullptr;         // synthetic C
        moa_req_info info{};
        bool done = false;
    };
    struct Slot {
        std::vector<Request *> members;
        void *scratch = nullptr;
        int64_t scratch_bytes = 0;
        int64_t bytes = 0;
        bool busy = false;
        bool mark_failed = false;
    };

    moa_status enqueue(Request *r, uint64_t *ticket);
    void run();
    bool retire_locked();
    bool admit_locked(size_t slot, int64_t now);
    bool materialise(Request *r);
    void unmaterialise(Request *r);
    void stuck_locked(int64_t now);
    void finish_locked(Request *r, moa_status st, int64_t now);
    bool any_busy() const;

    moa_serve_cfg cfg_;
    Backend *b_;
    Pool pool_;
    std::mutex mu_;
    std::condition_variable cv_work_, cv_done_;
    std::deque<Request *> waiting_;
    std::unordered_map<uint64_t, Request *> all_;
    std::vector<Slot> slots_;
    uint64_t next_ticket_ = 1;
    int64_t held_ = 0, peak_held_ = 0, peak_pool_ = 0;
    int64_t outstanding_ = 0, admitted_ = 0, completed_ = 0, failed_ = 0;
    bool trimmed_ = false;
    bool reserved_ = true;
    bool stop_ = false;
    std::thread sched_;
};

int64_t now_ns();

}  // namespace serve
}  // namespace moa
