// Batches of images of uneven size (edt_batch_plan / edt_batch_submit): every
// phase of the transform runs as one persistent launch over a device table of
// the images, instead of one launch per phase per image, and a submission with
// the same buffers as the previous one replays a captured HIP graph of those
// launches.  How the work is laid out is a schedule: which widths take the
// one-lane-per-row row pass, whether the images are listed largest first so
// that the longest work items start first, whether the images are split into
// two halves of about equal area whose launch sequences run side by side (two
// branches of the graph, so that one half's tail overlaps the other's work),
// and whether images wider than the lane pass run as single transforms (the
// segment path) instead of in the batch's row forms.  edt_batch_autotune
// times the candidate schedules on the caller's buffers and keeps the fastest.
#include "../../include/edt.h"
#include "edt_internal.h"

#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <new>
#include <vector>

namespace edt {

size_t table_bytes(int n) {
    return align_up(sizeof(BatchImage) * (size_t)n, 256) +
           2 * kPhases * align_up(sizeof(int32_t) * ((size_t)n + 1), 256);
}

int32_t pack_table(const BatchImage* img, int n, int lane_w, uint8_t* dst, int* totals,
                   int* max_w) {
    const size_t img_bytes = align_up(sizeof(BatchImage) * (size_t)n, 256);
    const size_t pre_bytes = align_up(sizeof(int32_t) * ((size_t)n + 1), 256);
    memcpy(dst, img, sizeof(BatchImage) * (size_t)n);
    int64_t acc[kPhases] = {};
    int mw = 0;
    for (int q = 0; q < n; ++q) {
        const int H = img[q].H, W = img[q].W;
        const bool lanes = W <= lane_w && H <= kLanePackMaxH;
        const int tiles = img[q].tr ? items_tiles(W, H) : 0;  // original sides W x H
        // images of the lane pass need no site-row lists (the pass works the
        // rows out from the band bits itself)
        const int64_t items[kPhases] = {items_bits(H, W), items_carry(H, W), 1,
                                        lanes ? 0 : items_near(H, W),
                                        lanes ? 0 : H, lanes ? items_lanes(H) : 0, tiles, tiles};
        for (int p = 0; p < kPhases; ++p) {
            int32_t* pre = reinterpret_cast<int32_t*>(dst + img_bytes + p * pre_bytes);
            pre[q] = (int32_t)acc[p];
            acc[p] += items[p];
            if (acc[p] > INT32_MAX) return EDT_ERR_TOO_LARGE;
        }
        if (!lanes && W > mw) mw = W;
    }
    for (int p = 0; p < kPhases; ++p) {
        const int32_t* pre = reinterpret_cast<const int32_t*>(dst + img_bytes + p * pre_bytes);
        reinterpret_cast<int32_t*>(dst + img_bytes + p * pre_bytes)[n] = (int32_t)acc[p];
        totals[p] = (int)acc[p];
        // coarse index: the image holding item k << s (the last image whose
        // prefix is at most that item)
        int32_t* first = reinterpret_cast<int32_t*>(dst + img_bytes + (kPhases + p) * pre_bytes);
        const int s = index_shift(totals[p], n);
        const int64_t entries = ((int64_t)totals[p] + (1ll << s) - 1) >> s;
        int im = 0;
        for (int64_t k = 0; k < entries; ++k) {
            const int64_t item = k << s;
            while (im + 1 < n && pre[im + 1] <= item) ++im;
            first[k] = im;
        }
    }
    *max_w = mw;
    return EDT_OK;
}

BatchTable table_view(const uint8_t* dev_table, int n, const int* totals) {
    const size_t img_bytes = align_up(sizeof(BatchImage) * (size_t)n, 256);
    const size_t pre_bytes = align_up(sizeof(int32_t) * ((size_t)n + 1), 256);
    BatchTable t;
    t.img = reinterpret_cast<const BatchImage*>(dev_table);
    for (int p = 0; p < kPhases; ++p) {
        t.prefix[p] = reinterpret_cast<const int32_t*>(dev_table + img_bytes + p * pre_bytes);
        t.first[p] =
            reinterpret_cast<const int32_t*>(dev_table + img_bytes + (kPhases + p) * pre_bytes);
        t.shift[p] = index_shift(totals[p], n);
    }
    t.nimg = n;
    t.mask_base = t.dist_base = t.feat_base = t.ws_base = 0;
    return t;
}

hipError_t enqueue_batch(const BatchTable& t, const int* totals, int max_w, hipStream_t s) {
    hipError_t e = hipSuccess;
    if (totals[kPhTrIn] > 0) e = launch_transpose_in(t, totals[kPhTrIn], s);
    if (e == hipSuccess) e = launch_column_pass_batch(t, totals, s);
    if (e == hipSuccess && totals[kPhRows] > 0) e = launch_row_pass_batch(t, totals, max_w, s);
    if (e == hipSuccess && totals[kPhLanes] > 0) e = launch_row_lanes_batch(t, totals[kPhLanes], s);
    if (e == hipSuccess && totals[kPhTrOut] > 0) e = launch_transpose_out(t, totals[kPhTrOut], s);
    return e;
}

}  // namespace edt

// One part of a batch under a schedule: a table over some of its images, its
// work totals and the widest image taking the several-lanes-per-row row pass.
struct Part {
    void* table = nullptr;  // device copy of the table
    int nimg = 0;
    int totals[edt::kPhases] = {};
    int max_w = 0;
};

// One way of laying out a batch: one or two parts (launched side by side),
// and the images run as single transforms.
struct Schedule {
    edt_schedule knobs = {edt::kLaneMaxW, 0, 1, 0, 0};
    std::vector<Part> parts;
    std::vector<int> singles;  // plan image indices run through the single-image path
};

struct edt_plan {
    int nimg = 0;
    int want_dist = 1;
    int any_feat = 0;
    int widest = 0;
    size_t ws_bytes = 0;
    int device = 0;
    std::vector<edt::BatchImage> img;  // host rows, in the order given
    std::vector<Schedule> sched;       // built so far
    int chosen = 0;
    // the second launch sequence of two-part schedules, joined by events
    hipStream_t aux = nullptr;
    hipEvent_t fork = nullptr, join = nullptr;
    // captured launches for one set of buffers
    hipStream_t cap_stream = nullptr, cap_aux = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    const void* key[4] = {nullptr, nullptr, nullptr, nullptr};
    hipEvent_t done = nullptr;
    bool use_graph = true;
};

namespace {

bool same_knobs(const edt_schedule& a, const edt_schedule& b) {
    return a.lane_w == b.lane_w && (a.largest_first != 0) == (b.largest_first != 0) &&
           a.branches == b.branches && (a.wide_single != 0) == (b.wide_single != 0) &&
           (a.transpose != 0) == (b.transpose != 0);
}

// An image the schedule processes as its transpose: wider than tall, and its
// transpose (W rows of H columns) takes the one-lane-per-row row pass.
bool transposes(const edt_schedule& k, const edt::BatchImage& b) {
    return k.transpose && b.W > b.H && b.H <= k.lane_w && b.W <= edt::kLanePackMaxH;
}

bool valid_knobs(const edt_schedule& k) {
    return k.lane_w >= 0 && k.lane_w <= edt::kLaneMaxW && (k.branches == 1 || k.branches == 2);
}

void drop_graph(edt_plan* p) {
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    p->exec = nullptr;
    p->graph = nullptr;
    for (auto& k : p->key) k = nullptr;
}

void free_schedule(Schedule& sc) {
    for (auto& pt : sc.parts)
        if (pt.table) (void)hipFree(pt.table);
    sc.parts.clear();
}

edt_status make_part(const std::vector<edt::BatchImage>& rows, int lane_w, Part* out) {
    const int n = (int)rows.size();
    std::vector<uint8_t> host(edt::table_bytes(n));
    Part pt;
    pt.nimg = n;
    const edt_status st = edt::pack_table(rows.data(), n, lane_w, host.data(), pt.totals, &pt.max_w);
    if (st != EDT_OK) return st;
    if (hipMalloc(&pt.table, host.size()) != hipSuccess) return EDT_ERR_OUT_OF_MEMORY;
    if (hipMemcpy(pt.table, host.data(), host.size(), hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipFree(pt.table);
        return EDT_ERR_DEVICE;
    }
    *out = pt;
    return EDT_OK;
}

// Build the schedule with these knobs (tables on the device).
edt_status make_schedule(edt_plan* p, const edt_schedule& knobs, Schedule* out) {
    Schedule sc;
    sc.knobs = knobs;
    std::vector<int> order;
    for (int q = 0; q < p->nimg; ++q) {
        if (knobs.wide_single && p->img[q].W > edt::kLaneMaxW)
            sc.singles.push_back(q);
        else
            order.push_back(q);
    }
    auto bigger = [&](int a, int b) {
        const edt::BatchImage &x = p->img[a], &y = p->img[b];
        return x.W != y.W ? x.W > y.W : x.H > y.H;
    };
    if (knobs.largest_first) std::stable_sort(order.begin(), order.end(), bigger);
    // two parts of about equal area: each image (largest area first) joins the
    // part with less so far; each part keeps the schedule's order
    std::vector<std::vector<int>> part_idx(knobs.branches == 2 ? 2 : 1);
    if (part_idx.size() == 1 || order.size() < 2) {
        part_idx.assign(1, order);
    } else {
        std::vector<int> by_area = order;
        std::stable_sort(by_area.begin(), by_area.end(), [&](int a, int b) {
            return (int64_t)p->img[a].H * p->img[a].W > (int64_t)p->img[b].H * p->img[b].W;
        });
        std::vector<char> side(p->nimg, 0);
        int64_t area[2] = {0, 0};
        for (int q : by_area) {
            const int k = area[1] < area[0] ? 1 : 0;
            side[q] = (char)k;
            area[k] += (int64_t)p->img[q].H * p->img[q].W;
        }
        for (int q : order) part_idx[side[q]].push_back(q);
    }
    for (const auto& idx : part_idx) {
        if (idx.empty()) continue;
        std::vector<edt::BatchImage> rows;
        rows.reserve(idx.size());
        for (int q : idx) {
            edt::BatchImage b = p->img[q];
            if (transposes(knobs, b)) {  // the table holds the transposed sides
                std::swap(b.H, b.W);
                b.tr = 1;
            }
            rows.push_back(b);
        }
        Part pt;
        const edt_status st = make_part(rows, knobs.lane_w, &pt);
        if (st != EDT_OK) {
            free_schedule(sc);
            return st;
        }
        sc.parts.push_back(pt);
    }
    *out = std::move(sc);
    return EDT_OK;
}

hipError_t enqueue_part(const edt_plan* p, const Part& pt, const uint8_t* mask_base,
                        int32_t* dist_base, int32_t* feat_base, void* workspace, hipStream_t s) {
    edt::BatchTable t = edt::table_view(static_cast<const uint8_t*>(pt.table), pt.nimg, pt.totals);
    t.mask_base = reinterpret_cast<uintptr_t>(mask_base);
    t.dist_base = p->want_dist ? reinterpret_cast<uintptr_t>(dist_base) : 0;
    t.feat_base = p->any_feat ? reinterpret_cast<uintptr_t>(feat_base) : 0;
    t.ws_base = reinterpret_cast<uintptr_t>(workspace);
    return edt::enqueue_batch(t, pt.totals, pt.max_w, s);
}

hipError_t enqueue_single_image(const edt_plan* p, int q, const uint8_t* mask_base,
                                int32_t* dist_base, int32_t* feat_base, void* workspace,
                                hipStream_t s) {
    const edt::BatchImage& b = p->img[q];
    edt::Img g;
    g.mask = mask_base + b.mask_off;
    g.mpitch = b.mpitch;
    g.dist = (b.outs & edt::kOutDist) ? dist_base + b.dist_off : nullptr;
    g.feat = (b.outs & edt::kOutFeat) ? feat_base + b.feat_off : nullptr;
    g.opitch = b.opitch;
    g.ws = static_cast<uint8_t*>(workspace) + b.ws_off;
    g.H = b.H;
    g.W = b.W;
    g.pol = b.pol;
    g.metric = EDT_METRIC_EUCLIDEAN_SQ;
    return edt::enqueue_single(g, s);
}

// The schedule's launches on s; a second part runs on aux, forked from and
// joined back into s with events (inside a capture, aux joins the capture).
hipError_t enqueue(edt_plan* p, const Schedule& sc, const uint8_t* mask_base, int32_t* dist_base,
                   int32_t* feat_base, void* workspace, hipStream_t s, hipStream_t aux) {
    const bool two = sc.parts.size() == 2;
    hipError_t e = hipSuccess;
    if (two) {
        e = hipEventRecord(p->fork, s);
        if (e == hipSuccess) e = hipStreamWaitEvent(aux, p->fork, 0);
    }
    for (size_t k = 0; k < sc.parts.size() && e == hipSuccess; ++k)
        e = enqueue_part(p, sc.parts[k], mask_base, dist_base, feat_base, workspace,
                         k == 1 ? aux : s);
    for (size_t k = 0; k < sc.singles.size() && e == hipSuccess; ++k)
        e = enqueue_single_image(p, sc.singles[k], mask_base, dist_base, feat_base, workspace,
                                 two && (k & 1) ? aux : s);
    if (two) {  // joined back even after a failure, so that no capture is left open on aux
        const hipError_t j = hipEventRecord(p->join, aux);
        const hipError_t w = j == hipSuccess ? hipStreamWaitEvent(s, p->join, 0) : j;
        if (e == hipSuccess) e = w;
    }
    return e;
}

edt_status check_buffers(edt_plan* p, const uint8_t* mask_base, int32_t* dist_base,
                         int32_t* feat_base, void* workspace, size_t workspace_bytes) {
    if (!p || !mask_base || !workspace) return EDT_ERR_INVALID_ARG;
    if (p->want_dist && !dist_base) return EDT_ERR_INVALID_ARG;
    if (p->any_feat && !feat_base) return EDT_ERR_INVALID_ARG;
    if (!p->want_dist && !p->any_feat) return EDT_ERR_INVALID_ARG;
    if (workspace_bytes < p->ws_bytes || (reinterpret_cast<uintptr_t>(workspace) & 255) != 0)
        return EDT_ERR_INVALID_ARG;
    return EDT_OK;
}

// Index of the schedule with these knobs, built if needed (-1 on error, *st set).
int find_or_make(edt_plan* p, const edt_schedule& knobs, edt_status* st) {
    for (size_t q = 0; q < p->sched.size(); ++q)
        if (same_knobs(p->sched[q].knobs, knobs)) return (int)q;
    Schedule sc;
    *st = make_schedule(p, knobs, &sc);
    if (*st != EDT_OK) return -1;
    p->sched.push_back(std::move(sc));
    return (int)p->sched.size() - 1;
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
        // every image asks for at least one output
        if (!want_dist && !d.want_feature) return EDT_ERR_INVALID_ARG;
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
        // images wider than the lane pass may run as single transforms, whose
        // workspace adds the segment buffers and row slots; images wider than
        // tall may run as their transposes, with transposed copies of the mask
        // and outputs
        size_t need =
            edt::layout_for(d.H, d.W, d.W > edt::kLaneMaxW, edt::lane_image(d.H, d.W)).total;
        if (d.W > d.H && d.H <= edt::kLaneMaxW && d.W <= edt::kLanePackMaxH)
            need = std::max(need, edt::tr_layout(d.W, d.H).total);
        b.tr = 0;
        b.pad_ = 0;
        ws += edt::align_up(need, 256);
    }
    {  // every candidate schedule must fit int32 totals: check the default
        std::vector<uint8_t> host(edt::table_bytes(n));
        int totals[edt::kPhases], max_w = 0;
        const edt_status pst =
            edt::pack_table(img.data(), n, edt::kLaneMaxW, host.data(), totals, &max_w);
        if (pst != EDT_OK) return pst;
    }
    edt_plan* pl = new (std::nothrow) edt_plan;
    if (!pl) return EDT_ERR_OUT_OF_MEMORY;
    pl->nimg = n;
    pl->want_dist = want_dist != 0;
    pl->any_feat = any_feat;
    pl->ws_bytes = ws;
    for (const auto& b : img) pl->widest = b.W > pl->widest ? b.W : pl->widest;
    pl->img = std::move(img);
    pl->use_graph = std::getenv("EDT_NO_GRAPH") == nullptr;
    Schedule sc;
    edt_status st = hipGetDevice(&pl->device) == hipSuccess ? EDT_OK : EDT_ERR_DEVICE;
    if (st == EDT_OK) st = make_schedule(pl, edt_schedule{edt::kLaneMaxW, 0, 1, 0, 0}, &sc);
    if (st == EDT_OK) pl->sched.push_back(std::move(sc));
    if (st == EDT_OK && (hipEventCreateWithFlags(&pl->done, hipEventDisableTiming) != hipSuccess ||
                         hipEventCreateWithFlags(&pl->fork, hipEventDisableTiming) != hipSuccess ||
                         hipEventCreateWithFlags(&pl->join, hipEventDisableTiming) != hipSuccess ||
                         hipStreamCreateWithFlags(&pl->aux, hipStreamNonBlocking) != hipSuccess))
        st = EDT_ERR_DEVICE;
    if (st == EDT_OK && pl->use_graph &&
        (hipStreamCreateWithFlags(&pl->cap_stream, hipStreamNonBlocking) != hipSuccess ||
         hipStreamCreateWithFlags(&pl->cap_aux, hipStreamNonBlocking) != hipSuccess))
        st = EDT_ERR_DEVICE;
    if (st != EDT_OK) {
        edt_plan_destroy(pl);
        return st;
    }
    *plan = pl;
    *workspace_bytes = ws;
    return EDT_OK;
}

edt_status edt_batch_submit(edt_plan* p, const uint8_t* mask_base, int32_t* dist_base,
                            int32_t* feat_base, void* workspace, size_t workspace_bytes,
                            void* stream) {
    const edt_status cs = check_buffers(p, mask_base, dist_base, feat_base, workspace,
                                        workspace_bytes);
    if (cs != EDT_OK) return cs;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const Schedule& sc = p->sched[p->chosen];
    // Kernel timing needs the launches themselves, so it bypasses the graph.
    if (!p->use_graph || edt::prof_enabled()) {
        if (enqueue(p, sc, mask_base, dist_base, feat_base, workspace, s, p->aux) != hipSuccess)
            return EDT_ERR_DEVICE;
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
        const hipError_t le = enqueue(p, sc, mask_base, dist_base, feat_base, workspace,
                                      p->cap_stream, p->cap_aux);
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

edt_status edt_batch_autotune(edt_plan* p, const uint8_t* mask_base, int32_t* dist_base,
                              int32_t* feat_base, void* workspace, size_t workspace_bytes,
                              void* stream, edt_tune_report* report) {
    const edt_status cs = check_buffers(p, mask_base, dist_base, feat_base, workspace,
                                        workspace_bytes);
    if (cs != EDT_OK) return cs;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    // candidate lane widths: none, then each width class up to kLaneMaxW that
    // changes which images take the lane pass
    std::vector<int> lane_ws = {0};
    for (int w : {256, edt::kLaneMaxW}) {
        const int eff = w < p->widest ? w : p->widest;
        if (eff > lane_ws.back()) lane_ws.push_back(w);
    }
    bool any_tr = false;  // some image is wider than tall and could run transposed
    for (const auto& b : p->img)
        any_tr |= transposes(edt_schedule{edt::kLaneMaxW, 0, 1, 0, 1}, b);
    std::vector<edt_schedule> cands;
    for (int tr : {0, 1}) {
        if (tr && !any_tr) continue;
        for (int ws_ : {0, 1}) {
            if (ws_ && p->widest <= edt::kLaneMaxW) continue;
            for (int br : {1, 2})
                for (int w : lane_ws)
                    for (int lf : {0, 1}) {
                        if (tr && w == 0) continue;  // no image takes the lane pass
                        cands.push_back(edt_schedule{w, lf, br, ws_, tr});
                    }
        }
    }
    if ((int)cands.size() > EDT_TUNE_MAX) cands.resize(EDT_TUNE_MAX);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        return EDT_ERR_DEVICE;
    }
    edt_status st = EDT_OK;
    float best = 0.f;
    int best_k = -1;
    edt_tune_report rep;
    memset(&rep, 0, sizeof(rep));
    for (size_t c = 0; c < cands.size() && st == EDT_OK; ++c) {
        const int k = find_or_make(p, cands[c], &st);
        if (k < 0) break;
        float t_min = 0.f;
        for (int rep_i = 0; rep_i < 4 && st == EDT_OK; ++rep_i) {  // one warm-up, three timed
            if (hipEventRecord(e0, s) != hipSuccess ||
                enqueue(p, p->sched[k], mask_base, dist_base, feat_base, workspace, s, p->aux) !=
                    hipSuccess ||
                hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
                st = EDT_ERR_DEVICE;
                break;
            }
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) st = EDT_ERR_DEVICE;
            if (rep_i > 0 && (rep_i == 1 || ms < t_min)) t_min = ms;
        }
        if (st != EDT_OK) break;
        rep.cand[c] = cands[c];
        rep.ms[c] = t_min;
        rep.tried = (int32_t)c + 1;
        if (best_k < 0 || t_min < best) {
            best = t_min;
            best_k = k;
            rep.chosen = (int32_t)c;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != EDT_OK) return st;
    if (p->chosen != best_k) drop_graph(p);
    p->chosen = best_k;
    if (report) *report = rep;
    return EDT_OK;
}

edt_status edt_batch_set_schedule(edt_plan* p, const edt_schedule* knobs) {
    if (!p || !knobs || !valid_knobs(*knobs)) return EDT_ERR_INVALID_ARG;
    edt_status st = EDT_OK;
    const int k = find_or_make(p, *knobs, &st);
    if (k < 0) return st;
    if (p->chosen != k) drop_graph(p);
    p->chosen = k;
    return EDT_OK;
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
    if (p->cap_aux) (void)hipStreamDestroy(p->cap_aux);
    if (p->aux) (void)hipStreamDestroy(p->aux);
    if (p->fork) (void)hipEventDestroy(p->fork);
    if (p->join) (void)hipEventDestroy(p->join);
    for (auto& sc : p->sched)
        for (auto& pt : sc.parts)
            if (pt.table && hipFree(pt.table) != hipSuccess) st = EDT_ERR_DEVICE;
    delete p;
    return st;
}

}  // extern "C"
