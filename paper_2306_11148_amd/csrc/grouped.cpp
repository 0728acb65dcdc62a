// moa_gemm_grouped: independent products in one launch sequence.
//
// Members on the split-BF16 path (the path of the batching workload) are
// conditioned together and contracted by one persistent launch that walks a
// shared tile list; scaled-FP8 members likewise, one sequence per term count.
// Members on the ONF and FP32 matrix-core paths run as single launches, in
// order, on the same stream. The member tables of the persistent launches
// are written to pinned, coherent staging buffers, mapped into the device's
// address space, that are recycled once the stream has consumed them; each
// launch reads its table from there with a small kernel.
#include <algorithm>
#include <mutex>
#include <vector>

#include "moa_internal.h"

namespace moa {
namespace {

struct Staging {
    void *ptr = nullptr;
    void *dev = nullptr;                // ptr in the device's address space (null: not mapped)
    size_t bytes = 0;
    hipEvent_t done = nullptr;
};

std::mutex g_staging_mu;
std::vector<Staging> g_staging;

moa_status staging_acquire(size_t bytes, Staging *out) {
    {
        std::lock_guard<std::mutex> lk(g_staging_mu);
        for (size_t k = 0; k < g_staging.size(); ++k) {
            if (g_staging[k].bytes >= bytes && hipEventQuery(g_staging[k].done) == hipSuccess) {
                *out = g_staging[k];
                g_staging.erase(g_staging.begin() + (long)k);
                return MOA_OK;
            }
        }
    }
    Staging s;
    s.bytes = bytes < 4096 ? 4096 : (bytes + 255) / 256 * 256;   // whole 16-byte words for the table kernels
    hipError_t e = hipHostMalloc(&s.ptr, s.bytes, hipHostMallocMapped | hipHostMallocCoherent);
    if (e == hipSuccess) {
        if (hipHostGetDevicePointer(&s.dev, s.ptr, 0) != hipSuccess) {
            s.dev = nullptr;            // not mapped: the table goes up by a copy
            (void)hipGetLastError();
        }
    } else {                            // no coherent mapping: plain pinned memory and a copy
        (void)hipGetLastError();
        s.dev = nullptr;
        e = hipHostMalloc(&s.ptr, s.bytes, hipHostMallocDefault);
    }
    if (e != hipSuccess) return fail(MOA_ERR_NOMEM, "pinned staging of %zu bytes: %s", s.bytes, hipGetErrorString(e));
    e = hipEventCreateWithFlags(&s.done, hipEventDisableTiming);
    if (e != hipSuccess) {
        (void)hipHostFree(s.ptr);
        return hip_fail(e, "hipEventCreateWithFlags");
    }
    *out = s;
    return MOA_OK;
}

void staging_release(const Staging &s, hipStream_t stream) {
    (void)hipEventRecord(s.done, stream);
    std::lock_guard<std::mutex> lk(g_staging_mu);
    g_staging.push_back(s);
}

}  // namespace

moa_status check_group_overlap(const moa_gemm_desc *descs, int64_t count) {
    struct Span { uintptr_t lo, hi; int64_t owner; };
    std::vector<Span> outs;
    for (int64_t g = 0; g < count; ++g) {
        const moa_gemm_desc &d = descs[g];
        const int64_t es = d.dtype == MOA_F64 ? 8 : 4;
        if (d.m > 0 && d.p > 0)
            outs.push_back({(uintptr_t)d.C, (uintptr_t)d.C + (uintptr_t)(d.m * d.p * es), g});
    }
    std::sort(outs.begin(), outs.end(), [](const Span &a, const Span &b) { return a.lo < b.lo; });
    for (size_t k = 1; k < outs.size(); ++k)
        if (outs[k].lo < outs[k - 1].hi)
            return fail(MOA_ERR_INVALID, "C of members %lld and %lld overlap", (long long)outs[k - 1].owner,
                        (long long)outs[k].owner);
    auto hits = [&](uintptr_t lo, uintptr_t hi) {
        // first output span ending after lo
        size_t a = 0, b = outs.size();
        while (a < b) {
            const size_t mid = (a + b) / 2;
            if (outs[mid].hi <= lo) a = mid + 1; else b = mid;
        }
        return a < outs.size() && outs[a].lo < hi;
    };
    for (int64_t g = 0; g < count; ++g) {
        const moa_gemm_desc &d = descs[g];
        const int64_t es = d.dtype == MOA_F64 ? 8 : 4;
        if (d.m > 0 && d.n > 0 && hits((uintptr_t)d.A, (uintptr_t)d.A + (uintptr_t)(d.m * d.n * es)))
            return fail(MOA_ERR_INVALID, "A of member %lld overlaps a member's C", (long long)g);
        if (d.n > 0 && d.p > 0 && hits((uintptr_t)d.B, (uintptr_t)d.B + (uintptr_t)(d.n * d.p * es)))
            return fail(MOA_ERR_INVALID, "B of member %lld overlaps a member's C", (long long)g);
    }
    return MOA_OK;
}

namespace {

int64_t align256(int64_t x) { return (x + 255) & ~int64_t(255); }

// The next `bytes` of `arena` (256-byte aligned), or null when it is full.
void *arena_take(ScratchArena *a, int64_t bytes) {
    const int64_t off = align256(a->used);
    if (bytes <= 0) return nullptr;
    if (off + bytes > a->size) return nullptr;
    a->used = off + bytes;
    return static_cast<char *>(a->base) + off;
}

// One persistent launch sequence over `list`: workspace from `arena` when
// given, else from the scratch cache; member table through pinned staging.
template <class Bytes, class Launch>
moa_status run_list(const std::vector<const moa_gemm_desc *> &list, int64_t desc_bytes, Bytes ws_bytes,
                    Launch launch, hipStream_t stream, ScratchArena *arena) {
    if (list.empty()) return MOA_OK;
    if (list.size() > (size_t)INT32_MAX) return fail(MOA_ERR_INVALID, "too many members");
    const int cnt = (int)list.size();
    const int64_t need = ws_bytes(list.data(), cnt);
    void *ws = nullptr;
    moa_status s = MOA_OK;
    if (arena) {
        if (need > 0 && !(ws = arena_take(arena, need)))
            return fail(MOA_ERR_NOMEM, "grouped scratch of %lld bytes exceeds the arena", (long long)need);
    } else if ((s = scratch_alloc(&ws, need, stream)) != MOA_OK) {
        return s;
    }
    Staging st;
    s = staging_acquire((size_t)desc_bytes, &st);
    if (s != MOA_OK) {
        if (!arena) scratch_free(ws, stream);
        return s;
    }
    const hipError_t e = launch(list.data(), cnt, ws, st.ptr, st.dev);
    staging_release(st, stream);
    if (!arena) scratch_free(ws, stream);
    if (e != hipSuccess) return hip_fail(e, "grouped launch");
    return MOA_OK;
}

// The members that run as persistent launches (split-BF16; FP8 by term
// count) and those that run singly, as run_grouped splits them.
struct Partition {
    std::vector<const moa_gemm_desc *> single, split, fp8[2];
};

Partition partition(const moa_gemm_desc *descs, int64_t count, const char *split_k = nullptr) {
    Partition pt;
    for (int64_t g = 0; g < count; ++g) {
        const moa_gemm_desc &d = descs[g];
        if (d.m == 0 || d.p == 0) continue;
        const moa_path path = resolve_path(d);
        if (has_col_operand(d) || (split_k ? split_k[g] != 0 : plans_split_k(d)))   // the persistent launches take
            pt.single.push_back(&d);                  // row-major, unsplit members
        else if (path == MOA_PATH_SPLIT_BF16 && split_grouped_fits(d))
            pt.split.push_back(&d);
        else if (path == MOA_PATH_FP8_SCALED)
            pt.fp8[fp8_two_term(d) ? 1 : 0].push_back(&d);
        else
            pt.single.push_back(&d);
    }
    return pt;
}

}  // namespace

int64_t grouped_scratch_bytes(const moa_gemm_desc *descs, int64_t count) {
    const Partition pt = partition(descs, count);
    int64_t total = 0;
    for (const moa_gemm_desc *d : pt.single) total += align256(gemm_workspace_bytes(*d));
    if (!pt.split.empty())
        total += align256(split_grouped_workspace_bytes(pt.split.data(), (int)pt.split.size()));
    for (int two = 0; two < 2; ++two)
        if (!pt.fp8[two].empty())
            total += align256(fp8_grouped_workspace_bytes(pt.fp8[two].data(), (int)pt.fp8[two].size(), two != 0));
    return total;
}

moa_status run_grouped(const moa_gemm_desc *descs, int64_t count, hipStream_t stream, ScratchArena *arena,
                       int split_variant, const char *split_k) {
    const Partition pt = partition(descs, count, split_k);
    const int sv = pt.split.empty() ? 0 : split_grouped_choose(pt.split.data(), (int)pt.split.size(), split_variant,
                                                               nullptr);
    for (const moa_gemm_desc *d : pt.single) {
        moa_status s;
        if (arena) {
            const int64_t need = gemm_workspace_bytes(*d);
            void *ws = arena_take(arena, need);
            if (need > 0 && !ws)
                return fail(MOA_ERR_NOMEM, "scratch of %lld bytes exceeds the arena", (long long)need);
            s = run_gemm_in(*d, stream, ws ? ws : arena->base, need);
        } else {
            s = run_gemm(*d, stream);
        }
        if (s != MOA_OK) return s;
    }
    moa_status s = run_list(
        pt.split, split_grouped_desc_bytes(pt.split.data(), (int)pt.split.size()), split_grouped_workspace_bytes,
        [&](const moa_gemm_desc *const *m, int c, void *ws, void *host, void *host_dev) {
            return launch_split_grouped(m, c, sv, ws, host, host_dev, stream);
        },
        stream, arena);
    for (int two = 0; two < 2 && s == MOA_OK; ++two)
        s = run_list(
            pt.fp8[two], fp8_grouped_desc_bytes((int)pt.fp8[two].size()),
            [&](const moa_gemm_desc *const *m, int c) { return fp8_grouped_workspace_bytes(m, c, two != 0); },
            [&](const moa_gemm_desc *const *m, int c, void *ws, void *host, void *host_dev) {
                return launch_fp8_grouped(m, c, two != 0, ws, host, host_dev, stream);
            },
            stream, arena);
    return s;
}

}  // namespace moa

using namespace moa;

namespace {

// Validates every member and plans it once; `split_k` (optional) receives
// whether each member's plan splits k.
moa_status check_grouped_args(const moa_gemm_desc *descs, int64_t count, std::vector<char> *split_k = nullptr) {
    if (count < 0) return fail(MOA_ERR_INVALID, "negative count");
    if (count > 0 && !descs) return fail(MOA_ERR_INVALID, "null descriptor array");
    if (split_k) split_k->assign((size_t)count, 0);
    for (int64_t g = 0; g < count; ++g) {
        moa_status s = validate(descs[g], true);
        if (s != MOA_OK) return s;
        Plan pl;
        if (descs[g].m > 0 && descs[g].p > 0) {
            if ((s = make_plan(descs[g], &pl)) != MOA_OK) return s;
            if (split_k) (*split_k)[(size_t)g] = pl.split_k > 1 ? 1 : 0;
        }
    }
    return check_group_overlap(descs, count);
}

}  // namespace

extern "C" moa_status moa_gemm_grouped(const moa_gemm_desc *descs, int64_t count, void *stream) {
    return moa_gemm_grouped_variant(descs, count, -1, stream);
}

extern "C" moa_status moa_gemm_grouped_variant(const moa_gemm_desc *descs, int64_t count, int32_t variant,
                                               void *stream) {
    try {
        if (variant < -1 || variant >= split_grouped_variant_count())
            return fail(MOA_ERR_INVALID, "grouped variant %d out of range", (int)variant);
        std::vector<char> split_k;
        moa_status s = check_grouped_args(descs, count, &split_k);
        if (s != MOA_OK) return s;
        return run_grouped(descs, count, static_cast<hipStream_t>(stream), nullptr, variant, split_k.data());
    } catch (...) {
        return fail(MOA_ERR_DEVICE, "internal error");
    }
}

extern "C" moa_status moa_grouped_plan_query(const moa_gemm_desc *descs, int64_t count, int32_t *variant,
                                             int32_t *tuned, int64_t *persistent_members) {
    try {
        std::vector<char> split_k;
        moa_status s = check_grouped_args(descs, count, &split_k);
        if (s != MOA_OK) return s;
        const Partition pt = partition(descs, count, split_k.data());
        bool t = false;
        const int v = pt.split.empty() ? -1 : split_grouped_choose(pt.split.data(), (int)pt.split.size(), -1, &t);
        if (variant) *variant = v;
        if (tuned) *tuned = t ? 1 : 0;
        if (persistent_members) *persistent_members = (int64_t)pt.split.size();
        return MOA_OK;
    } catch (...) {
        return fail(MOA_ERR_DEVICE, "internal error");
    }
}

extern "C" moa_status moa_autotune_grouped(const moa_gemm_desc *descs, int64_t count, int32_t reps, void *stream,
                                           int32_t *chosen, double *best_ms) {
    try {
        if (reps < 1) return fail(MOA_ERR_INVALID, "reps must be >= 1");
        std::vector<char> split_k;
        moa_status s = check_grouped_args(descs, count, &split_k);
        if (s != MOA_OK) return s;
        const Partition pt = partition(descs, count, split_k.data());
        if (pt.split.empty()) return fail(MOA_ERR_UNSUPPORTED, "no member runs in the persistent split-BF16 launch");
        hipStream_t st = static_cast<hipStream_t>(stream);
        hipEvent_t e0 = nullptr, e1 = nullptr;
        hipError_t e = hipEventCreate(&e0);
        if (e == hipSuccess) e = hipEventCreate(&e1);
        if (e != hipSuccess) {
            if (e0) (void)hipEventDestroy(e0);
            return hip_fail(e, "hipEventCreate");
        }
        int best = -1;
        double best_t = 0;
        for (int v = 0; v < split_grouped_variant_count() && s == MOA_OK; ++v) {
            s = run_grouped(descs, count, st, nullptr, v, split_k.data());     // warm-up
            if (s == MOA_OK && (e = hipEventRecord(e0, st)) != hipSuccess) s = hip_fail(e, "autotune timing");
            for (int r = 0; r < reps && s == MOA_OK; ++r) s = run_grouped(descs, count, st, nullptr, v, split_k.data());
            if (s == MOA_OK && (e = hipEventRecord(e1, st)) != hipSuccess) s = hip_fail(e, "autotune timing");
            if (s == MOA_OK && (e = hipEventSynchronize(e1)) != hipSuccess) s = hip_fail(e, "autotune timing");
            float ms = 0;
            if (s == MOA_OK && (e = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) s = hip_fail(e, "autotune timing");
            if (s == MOA_OK && (best < 0 || ms / reps < best_t)) {
                best = v;
                best_t = ms / reps;
            }
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        if (s != MOA_OK) return s;
        record_tuned_group_variant(pt.split.data(), (int)pt.split.size(), best, best_t);
        if (chosen) *chosen = best;
        if (best_ms) *best_ms = best_t;
        return MOA_OK;
    } catch (...) {
        return fail(MOA_ERR_DEVICE, "internal error");
    }
}
