// Prepared groups: the grouped launch of a fixed set of products captured
// once in a HIP graph and replayed. The workspaces and the device member
// tables are owned by the group; the captured sequence (per persistent
// launch: counter reset, grouped conditioning, persistent contraction -- one
// for split-BF16 members and one per FP8 term count -- then single launches
// of ONF / FP32 matrix-core members, the latter with record workspaces of the
// group) allocates, copies and clears nothing outside kernels, so every
// replay repeats exactly the same work on the same buffers.
#include <vector>

#include "moa_internal.h"

struct moa_group {
    void *ws = nullptr;                 // split-BF16 members
    void *ws8[2] = {nullptr, nullptr};  // FP8 members, one and two terms
    void *wsf = nullptr;                // FP32 matrix-core members' records
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipEvent_t done = nullptr;          // recorded behind every replay
};

using namespace moa;

namespace {

void release(moa_group *g) {
    if (!g) return;
    // replays of one group never overlap, so the last one recorded covers all
    if (g->done) {
        (void)hipEventSynchronize(g->done);
        (void)hipEventDestroy(g->done);
    }
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    if (g->ws) (void)hipFree(g->ws);   // hipFree waits for work using it
    for (void *w : g->ws8)
        if (w) (void)hipFree(w);
    if (g->wsf) (void)hipFree(g->wsf);
    delete g;
}

}  // namespace

extern "C" {

moa_status moa_group_create(const moa_gemm_desc *descs, int64_t count, moa_group **out) {
    try {
        if (!out) return fail(MOA_ERR_INVALID, "null output");
        *out = nullptr;
        if (count < 0 || (count > 0 && !descs)) return fail(MOA_ERR_INVALID, "bad descriptor array");
        std::vector<const moa_gemm_desc *> split, fp8[2];
        std::vector<moa_gemm_desc> single, f32m;
        std::vector<Plan> f32p;
        int64_t f32_bytes = 0;
        for (int64_t k = 0; k < count; ++k) {
            const moa_gemm_desc &d = descs[k];
            moa_status s = validate(d, true);
            if (s != MOA_OK) return s;
            if (d.m == 0 || d.p == 0) continue;
            Plan pl;
            if ((s = make_plan(d, &pl)) != MOA_OK) return s;
            if (pl.split_k > 1 || has_col_operand(d))
                return fail(MOA_ERR_UNSUPPORTED, "member %lld runs split-k (MOA_FLAG_SPLIT_K(1) turns it off) or "
                            "has a column-major operand: not in a prepared group", (long long)k);
            if (pl.path == MOA_PATH_SPLIT_BF16 && !split_grouped_fits(d))
                return fail(MOA_ERR_UNSUPPORTED, "member %lld is too large for the persistent launch", (long long)k);
            if (pl.path == MOA_PATH_SPLIT_BF16) split.push_back(&d);
            else if (pl.path == MOA_PATH_FP8_SCALED) fp8[fp8_two_term(d) ? 1 : 0].push_back(&d);
            else if (pl.workspace_bytes == 0) single.push_back(d);
            else if (pl.path == MOA_PATH_MFMA_F32) {
                f32m.push_back(d);
                f32p.push_back(pl);
                f32_bytes += (pl.workspace_bytes + 255) & ~int64_t(255);
            } else {
                return fail(MOA_ERR_UNSUPPORTED, "member %lld needs per-call scratch", (long long)k);
            }
        }
        moa_status s = check_group_overlap(descs, count);
        if (s != MOA_OK) return s;
        auto *g = new moa_group();
        hipError_t e = hipEventCreateWithFlags(&g->done, hipEventDisableTiming);
        if (e != hipSuccess) {
            g->done = nullptr;
            release(g);
            return hip_fail(e, "hipEventCreateWithFlags");
        }
        GroupedWork work{0, 0, 0};
        const int cnt = (int)split.size();
        if (cnt > 0) {
            e = hipMalloc(&g->ws, (size_t)split_grouped_workspace_bytes(split.data(), cnt));
            if (e != hipSuccess) {
                release(g);
                return fail(MOA_ERR_NOMEM, "group workspace: %s", hipGetErrorString(e));
            }
            std::vector<char> host((size_t)split_grouped_desc_bytes(split.data(), cnt));
            work = split_grouped_layout(split.data(), cnt, g->ws, host.data(),
                                        split_grouped_choose(split.data(), cnt, -1, nullptr));
            e = hipMemcpy(static_cast<char *>(g->ws) + 256, host.data(), host.size(), hipMemcpyHostToDevice);
            if (e != hipSuccess) {
                release(g);
                return hip_fail(e, "group member upload");
            }
        }
        if (f32_bytes > 0 && (e = hipMalloc(&g->wsf, (size_t)f32_bytes)) != hipSuccess) {
            g->wsf = nullptr;
            release(g);
            return fail(MOA_ERR_NOMEM, "group workspace: %s", hipGetErrorString(e));
        }
        hipStream_t cs = nullptr;
        if ((e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking)) != hipSuccess) {
            release(g);
            return hip_fail(e, "capture stream");
        }
        Fp8GroupWork work8[2]{};
        for (int two = 0; two < 2; ++two) {
            const int c8 = (int)fp8[two].size();
            if (c8 == 0) continue;
            e = hipMalloc(&g->ws8[two], (size_t)fp8_grouped_workspace_bytes(fp8[two].data(), c8, two != 0));
            if (e != hipSuccess) {
                (void)hipStreamDestroy(cs);
                release(g);
                return fail(MOA_ERR_NOMEM, "group workspace: %s", hipGetErrorString(e));
            }
            std::vector<char> host((size_t)fp8_grouped_desc_bytes(c8));
            work8[two] = fp8_grouped_layout(fp8[two].data(), c8, two != 0, g->ws8[two], host.data());
            e = hipMemcpy(static_cast<char *>(g->ws8[two]) + work8[two].table_offset, host.data(), host.size(),
                          hipMemcpyHostToDevice);
            if (e != hipSuccess) {
                (void)hipStreamDestroy(cs);
                release(g);
                return hip_fail(e, "group member upload");
            }
        }
        e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess && cnt > 0) e = split_grouped_enqueue(g->ws, cnt, work, cs);
        for (int two = 0; two < 2 && e == hipSuccess; ++two)
            if (!fp8[two].empty()) e = fp8_grouped_enqueue(g->ws8[two], (int)fp8[two].size(), two != 0, work8[two], cs);
        moa_status rs = MOA_OK;
        for (size_t k = 0; e == hipSuccess && rs == MOA_OK && k < single.size(); ++k)
            rs = run_gemm(single[k], cs);
        for (size_t k = 0, off = 0; e == hipSuccess && rs == MOA_OK && k < f32m.size(); ++k) {
            e = launch_mfma_f32(f32m[k], f32p[k], static_cast<char *>(g->wsf) + off, cs);
            off += (size_t)((f32p[k].workspace_bytes + 255) & ~int64_t(255));
        }
        hipGraph_t graph = nullptr;
        const hipError_t ee = hipStreamEndCapture(cs, &graph);
        (void)hipStreamDestroy(cs);
        g->graph = graph;
        if (e != hipSuccess || ee != hipSuccess || rs != MOA_OK || !graph) {
            release(g);
            if (rs != MOA_OK) return rs;
            return hip_fail(e != hipSuccess ? e : ee, "group capture");
        }
        if ((e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0)) != hipSuccess) {
            release(g);
            return hip_fail(e, "hipGraphInstantiate");
        }
        *out = g;
        return MOA_OK;
    } catch (...) {
        return fail(MOA_ERR_DEVICE, "internal error");
    }
}

moa_status moa_group_launch(moa_group *g, void *stream) {
    if (!g) return fail(MOA_ERR_INVALID, "null group");
    hipError_t e = hipGraphLaunch(g->exec, static_cast<hipStream_t>(stream));
    if (e == hipSuccess) e = hipEventRecord(g->done, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
    return MOA_OK;
}

moa_status moa_group_destroy(moa_group *g) {
    release(g);
    return MOA_OK;
}

}  // extern "C"
