// The serving scheduler (see serve_core.h). No device API is used here.
#include "serve_core.h"

#include <sys/prctl.h>

#include <algorithm>
#include <chrono>

namespace moa {
namespace serve {

int64_t now_ns() {
    return std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

namespace {
int64_t align256(int64_t x) { return (x + 255) & ~int64_t(255); }
int64_t round_up(int64_t x, int64_t to) { return (x + to - 1) / to * to; }
}  // namespace

// ------------------------------------------------------------------ pool --

Pool::~Pool() {
    for (Chunk &c : chunks_) b_->device_free(c.base);
}

void *Pool::carve(size_t c, int64_t bytes) {
    Chunk &ch = chunks_[c];
    for (auto it = ch.free.begin(); it != ch.free.end(); ++it) {
        if (it->second < bytes) continue;
        const int64_t off = it->first, size = it->second;
        ch.free.erase(it);
        if (size > bytes) ch.free.emplace(off + bytes, size - bytes);
        void *p = ch.base + off;
        blocks_[p] = {c, bytes};
        live_ += bytes;
        return p;
    }
    return nullptr;
}

void *Pool::alloc(int64_t bytes) {
    if (bytes <= 0) return nullptr;
    bytes = align256(bytes);
    for (size_t c = 0; c < chunks_.size(); ++c)
        if (void *p = carve(c, bytes)) return p;
    int64_t size = std::max(kChunk, round_up(bytes, int64_t(2) << 20));
    size = std::min(size, cap_ - total_);
    if (size < bytes) return nullptr;
    char *base = static_cast<char *>(b_->device_alloc(size));
    if (!base) return nullptr;
    Chunk ch;
    ch.base = base;
    ch.size = size;
    ch.free.emplace(0, size);
    chunks_.push_back(std::move(ch));
    total_ += size;
    return carve(chunks_.size() - 1, bytes);
}

bool Pool::reserve(int64_t bytes) {
    bytes = align256(bytes);
    if (bytes <= 0) return true;
    if (total_ + bytes > cap_) return false;
    char *base = static_cast<char *>(b_->device_alloc(bytes));
    if (!base) return false;
    Chunk ch;
    ch.base = base;
    ch.size = bytes;
    ch.free.emplace(0, bytes);
    chunks_.push_back(std::move(ch));
    total_ += bytes;
    return true;
}

void Pool::release(void *p) {
    if (!p) return;
    auto it = blocks_.find(p);
    if (it == blocks_.end()) return;
    Chunk &ch = chunks_[it->second.first];
    int64_t off = static_cast<char *>(p) - ch.base, size = it->second.second;
    live_ -= size;
    blocks_.erase(it);
    auto next = ch.free.lower_bound(off);
    if (next != ch.free.end() && next->first == off + size) {     // merge with the block after
        size += next->second;
        next = ch.free.erase(next);
    }
    if (next != ch.free.begin()) {                                 // and with the block before
        auto prev = std::prev(next);
        if (prev->first + prev->second == off) {
            prev->second += size;
            return;
        }
    }
    ch.free.emplace(off, size);
}

void Pool::trim() {
    if (!blocks_.empty()) return;
    for (Chunk &c : chunks_) b_->device_free(c.base);
    chunks_.clear();
    total_ = 0;
}

// ---------------------------------------------------------------- server --

Server::Server(const moa_serve_cfg &cfg, Backend *b)
    : cfg_(cfg), b_(b), pool_(b, cfg.hbm_budget_bytes), slots_((size_t)cfg.slots) {
    reserved_ = pool_.reserve(cfg.pool_reserve_bytes);
    peak_pool_ = pool_.chunk_bytes();
    sched_ = std::thread([this] { run(); });
}

Server::~Server() {
    {
        std::lock_guard<std::mutex> lk(mu_);
        stop_ = true;
    }
    cv_work_.notify_all();
    if (sched_.joinable()) sched_.join();
    for (size_t k = 0; k < slots_.size(); ++k) b_->wait((int)k);
    for (auto &kv : all_) {
        unmaterialise(kv.second);
        delete kv.second;
    }
}

moa_status Server::enqueue(Request *r, uint64_t *ticket) {
    r->info.t_submit_ns = now_ns();
    r->info.status = MOA_OK;
    if (r->reserve > cfg_.hbm_budget_bytes) {
        delete r;
        return MOA_ERR_NOMEM;
    }
    {
        std::lock_guard<std::mutex> lk(mu_);
        if (stop_) {
            delete r;
            return MOA_ERR_INVALID;
        }
        r->ticket = next_ticket_++;
        all_[r->ticket] = r;
        waiting_.push_back(r);
        ++outstanding_;
        *ticket = r->ticket;
    }
    cv_work_.notify_one();
    return MOA_OK;
}

moa_status Server::submit(const moa_gemm_desc &d, uint64_t *ticket) {
    auto *r = new Request();
    r->d = d;
    const int64_t es = d.dtype == MOA_F64 ? 8 : 4;
    r->scratch = d.m > 0 && d.p > 0 ? align256(b_->group_scratch_bytes(&d, 1)) : 0;
    r->reserve = (d.m * d.n + d.n * d.p + d.m * d.p) * es + r->scratch;
    return enqueue(r, ticket);
}

moa_status Server::submit_synthetic(const moa_synth_request &q, uint64_t *ticket) {
    auto *r = new Request();
    r->synthetic = true;
    r->seed = q.seed;
    r->d.m = q.m;
    r->d.n = q.n;
    r->d.p = q.p;
    r->d.dtype = MOA_F32;
    r->d.path = (moa_path)q.path;
    r->d.flags = q.flags;
    r->a_bytes = align256(q.m * q.n * 4);
    r->b_bytes = align256(q.n * q.p * 4);
    r->c_bytes = align256(q.m * q.p * 4);
    r->scratch = q.m > 0 && q.p > 0 ? align256(b_->group_scratch_bytes(&r->d, 1)) : 0;
    r->keep = r->c_bytes;
    r->reserve = r->a_bytes + r->b_bytes + r->c_bytes + r->scratch;
    return enqueue(r, ticket);
}

moa_status Server::poll(uint64_t ticket, moa_req_info *out) {
    std::lock_guard<std::mutex> lk(mu_);
    auto it = all_.find(ticket);
    if (it == all_.end()) return MOA_ERR_INVALID;
    if (!it->second->done) return MOA_NOT_READY;
    *out = it->second->info;
    return MOA_OK;
}

moa_status Server::result(uint64_t ticket, const void **C, int64_t *bytes) {
    std::lock_guard<std::mutex> lk(mu_);
    auto it = all_.find(ticket);
    if (it == all_.end()) return MOA_ERR_INVALID;
    const Request *r = it->second;
    if (!r->done) return MOA_NOT_READY;
    *C = r->synthetic ? r->c : r->d.C;
    *bytes = r->d.m * r->d.p * (r->d.dtype == MOA_F64 ? 8 : 4);
    return MOA_OK;
}

moa_status Server::release(uint64_t ticket) {
    {
        std::lock_guard<std::mutex> lk(mu_);
        auto it = all_.find(ticket);
        if (it == all_.end()) return MOA_ERR_INVALID;
        Request *r = it->second;
        if (!r->done) return MOA_NOT_READY;
        // a done request is referenced by no queue or slot any more
        held_ -= r->keep;
        unmaterialise(r);
        delete r;
        all_.erase(it);
    }
    cv_work_.notify_one();
    return MOA_OK;
}

void Server::drain() {
    std::unique_lock<std::mutex> lk(mu_);
    cv_done_.wait(lk, [&] { return outstanding_ == 0; });
}

void Server::stats(moa_serve_state *out) {
    std::lock_guard<std::mutex> lk(mu_);
    out->held_bytes = held_;
    out->peak_held_bytes = peak_held_;
    out->pool_bytes = pool_.chunk_bytes();
    out->peak_pool_bytes = peak_pool_;
    out->admitted = admitted_;
    out->completed = completed_;
    out->failed = failed_;
    out->waiting = (int64_t)waiting_.size();
}

bool Server::materialise(Request *r) {
    if (!r->synthetic) return true;
    if (r->a_bytes + r->b_bytes > 0 && !(r->ab = pool_.alloc(r->a_bytes + r->b_bytes))) return false;
    if (r->c_bytes > 0 && !(r->c = pool_.alloc(r->c_bytes))) {
        pool_.release(r->ab);
        r->ab = nullptr;
        return false;
    }
    char *ab = static_cast<char *>(r->ab);
    r->d.A = r->a_bytes ? ab : nullptr;
    r->d.B = r->b_bytes ? ab + r->a_bytes : nullptr;
    r->d.C = r->c;
    peak_pool_ = std::max(peak_pool_, pool_.chunk_bytes());
    return true;
}

void Server::unmaterialise(Request *r) {
    if (!r->synthetic) return;
    pool_.release(r->ab);
    pool_.release(r->c);
    r->ab = r->c = nullptr;
    r->d.A = r->d.B = nullptr;
    r->d.C = nullptr;
}

bool Server::any_busy() const {
    for (const Slot &s : slots_)
        if (s.busy) return true;
    return false;
}

void Server::finish_locked(Request *r, moa_status st, int64_t now) {
    r->info.status = st;
    r->info.t_done_ns = now;
    r->done = true;
    --outstanding_;
    ++failed_;
    cv_done_.notify_all();
}

// The head of the queue cannot be admitted. While work runs or results are
// held, memory will come back; with none, the pool's chunks are returned and
// admission tried once more; if that fails too the device cannot hold the
// request and it fails instead of waiting for ever.
void Server::stuck_locked(int64_t now) {
    if (any_busy() || held_ > 0 || waiting_.empty()) return;
    if (!trimmed_) {
        pool_.trim();
        trimmed_ = true;
        return;
    }
    Request *r = waiting_.front();
    waiting_.pop_front();
    finish_locked(r, MOA_ERR_NOMEM, now);
    trimmed_ = false;
}

bool Server::admit_locked(size_t k, int64_t now) {
    Slot &s = slots_[k];
    std::vector<Request *> members;
    int64_t add = 0;
    while (!waiting_.empty() && (int)members.size() < cfg_.max_group) {
        Request *r = waiting_.front();
        if (held_ + add + r->reserve > cfg_.hbm_budget_bytes) break;
        if (!materialise(r)) break;
        waiting_.pop_front();
        add += r->reserve;
        members.push_back(r);
    }
    if (members.empty()) {
        stuck_locked(now);
        return false;
    }
    // the group's scratch; members leave from the back if it does not fit
    std::vector<moa_gemm_desc> descs;
    void *scratch = nullptr;
    int64_t extra = 0, need = 0;
    for (;;) {
        descs.clear();
        int64_t reserved = 0;
        for (const Request *r : members) {
            descs.push_back(r->d);
            reserved += r->scratch;
        }
        need = align256(b_->group_scratch_bytes(descs.data(), (int64_t)descs.size()));
        extra = std::max<int64_t>(0, need - reserved);
        if (held_ + add + extra <= cfg_.hbm_budget_bytes && (need == 0 || (scratch = pool_.alloc(need)))) break;
        Request *last = members.back();
        members.pop_back();
        unmaterialise(last);
        add -= last->reserve;
        waiting_.push_front(last);
        if (members.empty()) {
            stuck_locked(now);
            return false;
        }
    }
    trimmed_ = false;
    peak_pool_ = std::max(peak_pool_, pool_.chunk_bytes());
    s.members = std::move(members);
    s.scratch = scratch;
    s.scratch_bytes = need;
    s.bytes = add + extra;
    s.busy = true;
    s.mark_failed = false;
    held_ += s.bytes;
    peak_held_ = std::max(peak_held_, held_);
    admitted_ += (int64_t)s.members.size();
    for (Request *r : s.members) {
        r->info.t_admit_ns = now;
        r->info.group_size = (int32_t)s.members.size();
    }
    return true;
}

bool Server::retire_locked() {
    bool any = false;
    for (size_t k = 0; k < slots_.size(); ++k) {
        Slot &s = slots_[k];
        if (!s.busy) continue;
        moa_status q;
        if (s.mark_failed) {
            b_->wait((int)k);
            q = MOA_ERR_DEVICE;
        } else {
            q = b_->query((int)k);
        }
        if (q == MOA_NOT_READY) continue;
        const int64_t t = now_ns();
        int64_t keep = 0;
        for (Request *r : s.members) {
            r->info.t_done_ns = t;
            if (q != MOA_OK && r->info.status == MOA_OK) r->info.status = MOA_ERR_DEVICE;
            if (r->info.status != MOA_OK) ++failed_;
            r->done = true;
            if (r->synthetic) {
                pool_.release(r->ab);
                r->ab = nullptr;
                r->d.A = r->d.B = nullptr;
            }
            keep += r->keep;
        }
        completed_ += (int64_t)s.members.size();
        outstanding_ -= (int64_t)s.members.size();
        pool_.release(s.scratch);
        held_ += keep - s.bytes;
        s.members.clear();
        s.scratch = nullptr;
        s.scratch_bytes = 0;
        s.bytes = 0;
        s.busy = false;
        any = true;
    }
    return any;
}

void Server::run() {
    b_->thread_start();
    // the completion polls below wait 20 us; the default timer slack of a
    // thread (50 us) would stretch each of them to about 70 us
    (void)prctl(PR_SET_TIMERSLACK, 1000UL, 0UL, 0UL, 0UL);
    const int64_t window_ns = (int64_t)std::max(0, cfg_.batch_window_us) * 1000;
    std::unique_lock<std::mutex> lk(mu_);
    std::vector<moa_gemm_desc> descs;
    for (;;) {
        if (retire_locked()) cv_done_.notify_all();
        bool launched = false;
        int64_t wake_at = 0;
        for (size_t k = 0; k < slots_.size(); ++k) {
            if (slots_[k].busy || waiting_.empty()) continue;
            const int64_t now = now_ns();
            if (window_ns > 0 && !stop_ && (int64_t)waiting_.size() < cfg_.max_group) {
                const int64_t ready = waiting_.front()->info.t_submit_ns + window_ns;
                if (now < ready) {
                    wake_at = ready;
                    break;
                }
            }
            if (!admit_locked(k, now)) {
                cv_done_.notify_all();     // a request may have failed for lack of memory
                break;
            }
            Slot &s = slots_[k];
            descs.clear();
            for (const Request *r : s.members) descs.push_back(r->d);
            const std::vector<Request *> members = s.members;
            void *scratch = s.scratch;
            const int64_t scratch_bytes = s.scratch_bytes;
            lk.unlock();   // enqueue without blocking submitters
            moa_status st = MOA_OK;
            for (const Request *r : members) {
                if (!r->synthetic || st != MOA_OK) continue;
                st = b_->fill((int)k, static_cast<float *>(const_cast<void *>(r->d.A)), r->d.m * r->d.n, r->seed, 0);
                if (st == MOA_OK)
                    st = b_->fill((int)k, static_cast<float *>(const_cast<void *>(r->d.B)), r->d.n * r->d.p, r->seed, 1);
            }
            const int64_t t_start = now_ns();
            if (st == MOA_OK) st = b_->launch((int)k, descs.data(), (int64_t)descs.size(), scratch, scratch_bytes);
            const moa_status mk = b_->mark((int)k);
            lk.lock();
            for (Request *r : members) {
                r->info.t_start_ns = t_start;
                if (st != MOA_OK) r->info.status = st;
            }
            if (mk != MOA_OK) slots_[k].mark_failed = true;
            launched = true;
        }
        if (stop_ && outstanding_ == 0) break;
        if (launched) continue;
        if (any_busy()) {
            // groups in flight: poll their markers at a fine interval
            cv_work_.wait_for(lk, std::chrono::microseconds(20));
        } else if (wake_at) {
            cv_work_.wait_for(lk, std::chrono::nanoseconds(std::max<int64_t>(0, wake_at - now_ns())));
        } else if (waiting_.empty()) {
            cv_work_.wait(lk, [&] { return stop_ || !waiting_.empty(); });
        } else {
            // blocked on memory that only a release can return
            cv_work_.wait_for(lk, std::chrono::milliseconds(1));
        }
    }
}

}  // namespace serve
}  // namespace moa
