// Batches of images of uneven size (edt_batch_plan / edt_batch_submit): every
// phase of the transform runs as one persistent launch over a device table of
// the images, instead of one launch per phase per image, and a submission with
// the same buffers as the previous one replays a captured HIP graph of those
// launches.
#include "../../include/edt.h"
#include "edt_internal.h"

#include <cstdlib>
#include <cstring>
#include <new>
#include <vector>

namespace edt {

size_t table_bytes(int n) {
    return align_up(sizeof(BatchImage) * (size_t)n, 256) +
           kPhases * align_up(sizeof(int32_t) * ((size_t)n + 1), 256);
}

int32_t pack_table(const BatchImage* img, int n, uint8_t* dst, int* totals, int* max_w) {
    const size_t img_bytes = align_up(sizeof(BatchImage) * (size_t)n, 256);
    const size_t pre_bytes = align_up(sizeof(int32_t) * ((size_t)n + 1), 256);
    memcpy(dst, img, sizeof(BatchImage) * (size_t)n);
    int64_t acc[kPhases] = {};
    int mw = 0;
    for (int q = 0; q < n; ++q) {
        const int H = img[q].H, W = img[q].W;
        const bool lanes = takes_lanes(W);
        const int64_t items[kPhases] = {items_bits(H, W), items_carry(H, W), 1, items_near(H, W),
                                        lanes ? 0 : H, lanes ? items_lanes(H) : 0};
        for (int p = 0; p < kPhases; ++p) {
            int32_t* pre = reinterpret_cast<int32_t*>(dst + img_bytes + p * pre_bytes);
            pre[q] = (int32_t)acc[p];
            acc[p] += items[p];
            if (acc[p] > INT32_MAX) return EDT_ERR_TOO_LARGE;
        }
        if (!lanes && W > mw) mw = W;
    }
    for (int p = 0; p < kPhases; ++p) {
        reinterpret_cast<int32_t*>(dst + img_bytes + p * pre_bytes)[n] = (int32_t)acc[p];
        totals[p] = (int)acc[p];
    }
    *max_w = mw;
    return EDT_OK;
}

BatchTable table_view(const uint8_t* dev_table, int n) {
    const size_t img_bytes = align_up(sizeof(BatchImage) * (size_t)n, 256);
    const size_t pre_bytes = align_up(sizeof(int32_t) * ((size_t)n + 1), 256);
    BatchTable t;
    t.img = reinterpret_cast<const BatchImage*>(dev_table);
    for (int p = 0; p < kPhases; ++p)
        t.prefix[p] = reinterpret_cast<const int32_t*>(dev_table + img_bytes + p * pre_bytes);
    t.nimg = n;
    t.mask_base = t.dist_base = t.feat_base = t.ws_base = 0;
    return t;
}

hipError_t enqueue_batch(const BatchTable& t, const int* totals, int max_w, hipStream_t s) {
    hipError_t e = launch_column_pass_batch(t, totals, s);
    if (e == hipSuccess && totals[kPhRows] > 0) e = launch_row_pass_batch(t, totals, max_w, s);
    if (e == hipSuccess && totals[kPhLanes] > 0) e = launch_row_lanes_batch(t, totals[kPhLanes], s);
    return e;
}

}  // namespace edt

struct edt_plan {
    int nimg = 0;
    int want_dist = 1;
    int any_feat = 0;
    int max_w = 0;
    int totals[edt::kPhases] = {};
    size_t ws_bytes = 0;
    int device = 0;
    void* table = nullptr;  // device copy of the batch table
    // captured launches for one set of buffers
    hipStream_t cap_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    const void* key[4] = {nullptr, nullptr, nullptr, nullptr};
    hipEvent_t done = nullptr;
    bool use_graph = true;
};

namespace {

void drop_graph(edt_plan* p) {
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    p->exec = nullptr;
    p->graph = nullptr;
    for (auto& k : p->key) k = nullptr;
}

hipError_t enqueue(edt_plan* p, const edt::BatchTable& t, hipStream_t s) {
    return edt::enqueue_batch(t, p->totals, p->max_w, s);
}

}  // namespace

extern "C" {

edt_status edt_batch_plan(const edt_image_desc* images, int32_t n, int32_t want_dist,
                          edt_plan** plan, size_t* workspace_bytes) {
    if (!plan || !workspace_bytes || !images || n < 1) return EDT_ERR_INVALID_ARG;
    if (n > EDT_BATCH_MAX_IMAGES) return EDT_ERR_TOO_LARGE;
    *plan = nullptr;
    std::vector<edt::BatchImage> img(n);
    size_t ws = 0;
    int any_feat = 0;
    for (int q = 0; q < n; ++q) {
        const edt_image_desc& d = images[q];
        // the pointers are only checked for null later; a dummy non-null mask
        // lets the shared image check validate sizes, pitches and polarity
        const edt_status st = edt::check_image(reinterpret_cast<const uint8_t*>(1), d.H, d.W,
                                               d.mask_pitch, d.polarity,
                                               EDT_METRIC_EUCLIDEAN_SQ, d.out_pitch);
        if (st != EDT_OK) return st;
        if (d.W > EDT_BATCH_MAX_W) return EDT_ERR_TOO_LARGE;
        if (d.mask_offset < 0 || d.out_offset < 0) return EDT_ERR_INVALID_ARG;
        edt::BatchImage& b = img[q];
        b.mask_off = d.mask_offset;
        b.mpitch = d.mask_pitch;
        b.dist_off = d.out_offset;
        b.feat_off = d.out_offset;
        b.opitch = d.out_pitch;
        b.ws_off = (int64_t)ws;
        b.H = d.H;
        b.W = d.W;
        b.pol = d.polarity;
        b.outs = (want_dist ? edt::kOutDist : 0) | (d.want_feature ? edt::kOutFeat : 0);
        any_feat |= d.want_feature != 0;
        ws += edt::layout_for(d.H, d.W, false).total;
    }
    std::vector<uint8_t> host(edt::table_bytes(n));
    int totals[edt::kPhases], max_w = 0;
    const edt_status pst = edt::pack_table(img.data(), n, host.data(), totals, &max_w);
    if (pst != EDT_OK) return pst;

    edt_plan* pl = new (std::nothrow) edt_plan;
    if (!pl) return EDT_ERR_OUT_OF_MEMORY;
    pl->nimg = n;
    pl->want_dist = want_dist != 0;
    pl->any_feat = any_feat;
    pl->max_w = max_w;
    for (int p = 0; p < edt::kPhases; ++p) pl->totals[p] = totals[p];
    pl->ws_bytes = ws;
    pl->use_graph = std::getenv("EDT_NO_GRAPH") == nullptr;
    if (hipGetDevice(&pl->device) != hipSuccess || hipMalloc(&pl->table, host.size()) != hipSuccess) {
        delete pl;
        return EDT_ERR_OUT_OF_MEMORY;
    }
    bool ok = hipMemcpy(pl->table, host.data(), host.size(), hipMemcpyHostToDevice) == hipSuccess;
    if (ok) ok = hipEventCreateWithFlags(&pl->done, hipEventDisableTiming) == hipSuccess;
    if (ok && pl->use_graph)
        ok = hipStreamCreateWithFlags(&pl->cap_stream, hipStreamNonBlocking) == hipSuccess;
    if (!ok) {
        edt_plan_destroy(pl);
        return EDT_ERR_DEVICE;
    }
    *plan = pl;
    *workspace_bytes = ws;
    return EDT_OK;
}

edt_status edt_batch_submit(edt_plan* p, const uint8_t* mask_base, int32_t* dist_base,
                            int32_t* feat_base, void* workspace, size_t workspace_bytes,
                            void* stream) {
    if (!p || !mask_base || !workspace) return EDT_ERR_INVALID_ARG;
    if (p->want_dist && !dist_base) return EDT_ERR_INVALID_ARG;
    if (p->any_feat && !feat_base) return EDT_ERR_INVALID_ARG;
    if (!p->want_dist && !p->any_feat) return EDT_ERR_INVALID_ARG;
    if (workspace_bytes < p->ws_bytes || (reinterpret_cast<uintptr_t>(workspace) & 255) != 0)
        return EDT_ERR_INVALID_ARG;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    edt::BatchTable t = edt::table_view(static_cast<const uint8_t*>(p->table), p->nimg);
    t.mask_base = reinterpret_cast<uintptr_t>(mask_base);
    t.dist_base = p->want_dist ? reinterpret_cast<uintptr_t>(dist_base) : 0;
    t.feat_base = p->any_feat ? reinterpret_cast<uintptr_t>(feat_base) : 0;
    t.ws_base = reinterpret_cast<uintptr_t>(workspace);
    // Kernel timing needs the launches themselves, so it bypasses the graph.
    if (!p->use_graph || edt::prof_enabled()) {
        if (enqueue(p, t, s) != hipSuccess) return EDT_ERR_DEVICE;
        return hipEventRecord(p->done, s) == hipSuccess ? EDT_OK : EDT_ERR_DEVICE;
    }
    const void* key[4] = {mask_base, p->want_dist ? dist_base : nullptr,
                          p->any_feat ? feat_base : nullptr, workspace};
    bool same = p->exec != nullptr;
    for (int q = 0; q < 4 && same; ++q) same = key[q] == p->key[q];
    if (!same) {
        drop_graph(p);
        if (hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal) != hipSuccess)
            return EDT_ERR_DEVICE;
        const hipError_t le = enqueue(p, t, p->cap_stream);
        hipGraph_t g = nullptr;
        const hipError_t ce = hipStreamEndCapture(p->cap_stream, &g);
        if (le != hipSuccess || ce != hipSuccess || !g) {
            if (g) (void)hipGraphDestroy(g);
            return EDT_ERR_DEVICE;
        }
        p->graph = g;
        if (hipGraphInstantiate(&p->exec, g, nullptr, nullptr, 0) != hipSuccess) {
            drop_graph(p);
            return EDT_ERR_DEVICE;
        }
        for (int q = 0; q < 4; ++q) p->key[q] = key[q];
    }
    if (hipGraphLaunch(p->exec, s) != hipSuccess) return EDT_ERR_DEVICE;
    return hipEventRecord(p->done, s) == hipSuccess ? EDT_OK : EDT_ERR_DEVICE;
}

edt_status edt_plan_destroy(edt_plan* p) {
    if (!p) return EDT_ERR_INVALID_ARG;
    edt_status st = EDT_OK;
    if (p->done) {
        if (hipEventSynchronize(p->done) != hipSuccess) st = EDT_ERR_DEVICE;
        (void)hipEventDestroy(p->done);
    }
    drop_graph(p);
    if (p->cap_stream) (void)hipStreamDestroy(p->cap_stream);
    if (p->table && hipFree(p->table) != hipSuccess) st = EDT_ERR_DEVICE;
    delete p;
    return st;
}

}  // extern "C"
