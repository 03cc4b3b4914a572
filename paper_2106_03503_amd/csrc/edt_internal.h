// Internal declarations shared by the libedt translation units (not part of
// the public ABI in include/edt.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace edt {

// Rows per band of the vertical pass: one 64-bit site mask per band column.
constexpr int kBand = 64;
// "No site below" marker of the band carries (larger than any row index).
constexpr int16_t kNoBelow = INT16_MAX;
// Columns per work item (one wavefront, four per lane) of the band-bit pass.
constexpr int kBitsCols = 256;
// Band carries: columns per workgroup and band slices (one wavefront each).
constexpr int kCarryCols = 64;
constexpr int kCarrySlices = 16;
// Listed columns per work item (one wavefront) of the nearest-row pass.
constexpr int kNearCols = 64;
// Wavefronts per workgroup of the band-bit and nearest-row passes; each
// wavefront takes work items of its own.
constexpr int kColWaves = 4;

// Row pass: candidate slots per lane.
constexpr int kRowS = 16;
// One-wavefront row pass for rows with at most kSparseMaxN candidates.
constexpr int kSparseLanes = 64;
constexpr int kSparseMaxN = kSparseLanes * kRowS;
// Widest row whose whole candidate list and envelope live in LDS.
constexpr int kLdsMaxW = 1024 * kRowS;
// Workgroups (and global-memory row slots) of the row pass for wider rows.
constexpr int kWideSlots = 512;
// Candidate capacity of one global row slot (1024 lanes x 2*kRowS slots).
constexpr int kWideCap = 1024 * 2 * kRowS;

__host__ __device__ inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Candidate-list capacity per row (multiple of 32 so every lane's chunk of
// 16 or 32 slots is whole).
__host__ __device__ inline int cand_pitch(int W) { return (int)align_up((size_t)W, 32); }
// Bytes of one global row slot (4-byte candidates, then 2-byte starts).
__host__ __device__ inline size_t wide_slot_bytes() { return align_up((size_t)kWideCap * 6, 256); }

// Byte offsets of the pieces of one image's workspace.
struct Layout {
    int nb;            // bands of kBand rows
    size_t bits;       // uint64 [nb][W]  site bits of each band column
    size_t up;         // int16  [nb][W]  last site row above the band (-1: none)
    size_t down;       // int16  [nb][W]  first site row below the band (kNoBelow: none)
    size_t flag;       // uint8  [cand_pitch(W)]  column holds a site (0 past W)
    size_t cols;       // int16  [cand_pitch(W)]  columns holding a site, increasing
    size_t meta;       // int32  [4]      {n = number of such columns, rc row pitch}
    size_t rc;         // int16  [H][cand_pitch(W)] nearest site row of each listed column
    size_t segm;       // int16  [H][seg_count(W)]  envelope size of each row segment
    size_t env;        // uint32 [H][cand_pitch(W)] segment envelopes (packed candidates)
    size_t rowfail;    // uint8  [H]      row left to the segment merge
    size_t slots;      // row slots for rows wider than kLdsMaxW (single images only)
    size_t stk;        // uint32 [H][cand_pitch(W)] envelopes of the one-lane-per-row pass
                       // (batch images it takes only), laid out per 64-row work item
    size_t total;
};

// Segments of the single-image row pass for dense rows: a row's candidate
// list is cut into segments of kSegL (or a multiple of it) candidates, whose
// envelopes are built one lane per (row, segment) and merged per row.
constexpr int kSegL = 64;
__host__ __device__ inline int seg_count(int W) { return (W + kSegL - 1) / kSegL; }
__host__ __device__ inline bool has_segments(int W) { return W > kSparseMaxN && W <= kLdsMaxW; }

// Workspace layout of one image; with_slots adds the global row slots and
// segment sizes that the single-image row pass uses for wide rows, with_stack
// the envelopes of the one-lane-per-row pass (last, so that no other offset
// depends on it).
__host__ __device__ inline Layout layout_for(int H, int W, bool with_slots = true,
                                             bool with_stack = false) {
    Layout L;
    L.nb = (H + kBand - 1) / kBand;
    const size_t cp = (size_t)cand_pitch(W);
    size_t off = 0;
    L.bits = off;
    off = align_up(off + (size_t)L.nb * W * 8, 256);
    L.up = off;
    off = align_up(off + (size_t)L.nb * W * 2, 256);
    L.down = off;
    off = align_up(off + (size_t)L.nb * W * 2, 256);
    L.flag = off;
    off = align_up(off + cp, 256);
    L.cols = off;
    off = align_up(off + cp * 2, 256);
    L.meta = off;
    off = align_up(off + 16, 256);
    L.rc = off;
    off = align_up(off + (size_t)H * cp * 2, 256);
    L.segm = off;
    if (with_slots && has_segments(W)) off = align_up(off + (size_t)H * seg_count(W) * 2, 256);
    L.env = off;
    if (with_slots && has_segments(W)) off = align_up(off + (size_t)H * cp * 4, 256);
    L.rowfail = off;
    if (with_slots && has_segments(W)) off = align_up(off + (size_t)H, 256);
    L.slots = off;
    if (with_slots && W > kLdsMaxW) off = align_up(off + (size_t)kWideSlots * wide_slot_bytes(), 256);
    L.stk = off;
    if (with_stack) off = align_up(off + (size_t)H * cp * 4, 256);
    L.total = off;
    return L;
}

// One image as the kernels see it.
struct Img {
    const uint8_t* mask;
    int64_t mpitch;    // bytes between mask rows
    int32_t* dist;     // may be null
    int32_t* feat;     // may be null
    int64_t opitch;    // elements between output rows
    uint8_t* ws;       // this image's workspace (layout_for(H, W))
    int H, W, pol;
    int metric;        // EDT_METRIC_*: 0 squared Euclidean, 1 city-block, 2 chessboard,
                       // 3 chamfer 4-3
    int fsq = 0;       // dist receives fp32 Euclidean distances (sqrt_bits of the squared
                       // ones) instead of int32 squared distances: single images,
                       // squared Euclidean metric, through kernels compiled for it
    int tr = 0;        // a batch image processed as its transpose: H, W, mask and
                       // outputs are the transposed ones (in its workspace), ties in
                       // the row pass go to the left column (the smaller original
                       // row), and features are original indices
};

// Pointers into an image's workspace.
struct Views {
    uint64_t* bits;
    int16_t* up;
    int16_t* down;
    uint8_t* flag;
    int16_t* cols;
    int32_t* meta;
    int16_t* rc;
};

__host__ __device__ inline Views views_of(const Img& g) {
    const Layout L = layout_for(g.H, g.W, false);
    Views v;
    v.bits = reinterpret_cast<uint64_t*>(g.ws + L.bits);
    v.up = reinterpret_cast<int16_t*>(g.ws + L.up);
    v.down = reinterpret_cast<int16_t*>(g.ws + L.down);
    v.flag = g.ws + L.flag;
    v.cols = reinterpret_cast<int16_t*>(g.ws + L.cols);
    v.meta = reinterpret_cast<int32_t*>(g.ws + L.meta);
    v.rc = reinterpret_cast<int16_t*>(g.ws + L.rc);
    return v;
}

// Work items of each phase for one image.
__host__ __device__ inline int items_bits(int H, int W) {
    return ((H + kBand - 1) / kBand) * ((W + kBitsCols - 1) / kBitsCols);
}
// Images of at most kCarrySmallBands bands take one thread per column over all
// of its bands (a work item is then kCarryCols * kCarrySlices columns); taller
// ones split each column into kCarrySlices slices of bands.
constexpr int kCarrySmallBands = 16;
__host__ __device__ inline int items_carry(int H, int W) {
    const int cols = (H + kBand - 1) / kBand <= kCarrySmallBands ? kCarryCols * kCarrySlices
                                                                 : kCarryCols;
    return (W + cols - 1) / cols;
}
__host__ __device__ inline int items_near(int H, int W) {
    return ((H + kBand - 1) / kBand) * ((W + kNearCols - 1) / kNearCols);
}

// Row pass with one lane per row: rows per work item (one wavefront), stack
// entries per lane kept in LDS, and the widest image of a batch that takes it.
constexpr int kLaneRows = 64;
constexpr int kLaneRing = 16;
constexpr int kLaneMaxW = 1024;
// Tallest image the one-lane-per-row pass takes (its stack entries pack the
// site row into 12 bits).
constexpr int kLanePackMaxH = 4096;
__host__ __device__ inline int items_lanes(int H) { return (H + kLaneRows - 1) / kLaneRows; }
// An image the one-lane-per-row pass can take (its workspace then holds the
// envelopes of that pass).
__host__ __device__ inline bool lane_image(int H, int W) {
    return W <= kLaneMaxW && H <= kLanePackMaxH;
}

// Phases of the transform, in launch order (a batch image's rows are work
// items of kPhRows, or row groups of kPhLanes when its width is at most the
// batch's lane width, itself at most kLaneMaxW).
enum Phase {
    kPhBits = 0,
    kPhCarry = 1,
    kPhCompact = 2,
    kPhNear = 3,
    kPhRows = 4,
    kPhLanes = 5,
    kPhTrIn = 6,   // 64 x 64 tiles of the masks of transposed images
    kPhTrOut = 7,  // 64 x 64 tiles of their outputs
    kPhases = 8
};

// Tiles of kTrTile x kTrTile pixels of an H x W image (transposition).
constexpr int kTrTile = 64;
__host__ __device__ inline int items_tiles(int H, int W) {
    return ((H + kTrTile - 1) / kTrTile) * ((W + kTrTile - 1) / kTrTile);
}

// One image of a batch, as offsets from the bases passed at submission (a
// base may be 0, and the offsets then absolute addresses).
struct BatchImage {
    int64_t mask_off;  // bytes from the mask base
    int64_t mpitch;    // bytes between mask rows
    int64_t dist_off;  // elements from the distance base
    int64_t feat_off;  // elements from the feature base
    int64_t opitch;    // elements between output rows
    int64_t ws_off;    // bytes from the workspace base
    int32_t H, W, pol;
    int32_t outs;      // kOutDist | kOutFeat: the outputs this image writes
    int32_t tr;        // processed as its transpose: H, W are the transposed sides,
                       // the offsets and pitches the caller's
    int32_t pad_;
};
constexpr int32_t kOutDist = 1;
constexpr int32_t kOutFeat = 2;

// Device table of a batch: images, then for each phase the exclusive prefix
// of work items over the images (nimg + 1 entries), and the bases.
struct BatchTable {
    const BatchImage* img;
    const int32_t* prefix[kPhases];
    // coarse index of each phase: first[p][k] is the image holding work item
    // k << shift[p] (at most nimg + 1 entries)
    const int32_t* first[kPhases];
    int shift[kPhases];
    int nimg;
    uintptr_t mask_base;
    uintptr_t dist_base;
    uintptr_t feat_base;
    uintptr_t ws_base;
};

// Integer products of pixel coordinates.  Every operand is a coordinate or
// the difference or sum of two (below 2^16 in magnitude) and every product
// stays below 2^31, so the 24-bit multiply gives it exactly -- at full issue
// rate, where a 32-bit multiply issues at a quarter of it.
__device__ __forceinline__ int mul_c(int a, int b) { return __mul24(a, b); }
__device__ __forceinline__ int sqr_c(int x) { return __mul24(x, x); }

// floor(num / den) + 1, clamped to [0, W], for 2 <= den < 2^16, num < 2^31
// and W < 2^15: a float estimate of the quotient (relative error below 2^-21,
// so within one of the floor wherever the result is below W), clamped to W
// (an estimate past W means a floor of at least W, which the correction then
// keeps; below by -1), corrected by one from the integer remainder, and 0 for
// a negative num; written without branches, so that the lanes of a wavefront
// taking it with different operands do not diverge, and defined for any
// operands.  It is the first pixel from which
// a parabola beats its left neighbour when num/den is their intersection
// (Eq. eq_intersection, with den = 2 (l - k)).  A host model of these steps, with the hardware
// reciprocal off by up to two ulp, gives the exact floor for every den in
// [2, 2^16) and W below 2^15 at each multiple of den and its neighbours.
__device__ __forceinline__ int first_after(int num, int den, int W) {
    const float qf = (float)num * __builtin_amdgcn_rcpf((float)den);
    // an estimate past W has a floor of at least W; clamping before the
    // conversion also keeps it defined for any operands
    const int q = (int)__builtin_amdgcn_fmed3f(qf, -1.0f, (float)W);
    const int r = num - mul_c(q, den);
    const int qc = q + (r >= den ? 1 : 0) - (r < 0 ? 1 : 0);
    return min(qc + 1, W) & ~(num >> 31);  // 0 for a negative num
}

// The fp32 Euclidean distance of a squared distance, as int32 bits for the
// output stores: the fp64 square root rounded to fp32 (the nearest fp32 to the
// true root for every d < 2^31), and +infinity for INT32_MAX (no site).
__device__ __forceinline__ int32_t sqrt_bits(int32_t d) {
    const float f = d == INT32_MAX ? __builtin_inff() : (float)sqrt((double)d);
    return __float_as_int(f);
}

// A device address as a pointer into global memory.  Going through the
// global address space lets the compiler emit global (not flat) loads and
// stores for everything derived from it; a flat access also counts as an
// LDS access, so every wait for LDS data would wait for memory as well.
template <typename T>
__device__ __forceinline__ T* global_ptr(uintptr_t a) {
    typedef __attribute__((address_space(1))) T GT;
    return (T*)(GT*)a;
}

// Values that every lane of the wavefront holds alike, moved to scalar
// registers: the batch kernels take one image per wavefront at a time, and the
// compiler cannot tell that what a wavefront reads from the batch table (in
// memory that the kernel also writes) is the same in every lane.
__device__ __forceinline__ int32_t wave_uniform(int32_t x) {
    return __builtin_amdgcn_readfirstlane(x);
}
__device__ __forceinline__ int64_t wave_uniform(int64_t x) {
    const uint64_t u = (uint64_t)x;
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)u);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(u >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

// Workspace of a batch image processed as its transpose (transposed sides
// H x W): the transform's own layout, then the transposed mask (rows
// align_up(W, 16) bytes apart) and the transposed outputs (rows align_up(W, 4)
// elements apart), written back to the caller's outputs at the end.
struct TrLayout {
    size_t mask, dist, feat, total;
    int64_t mpitch, opitch;
};
__host__ __device__ inline TrLayout tr_layout(int H, int W) {
    TrLayout T;
    T.mpitch = (int64_t)align_up((size_t)W, 16);
    T.opitch = (int64_t)align_up((size_t)W, 4);
    size_t off = align_up(layout_for(H, W, false, true).total, 256);
    T.mask = off;
    off = align_up(off + (size_t)H * T.mpitch, 256);
    T.dist = off;
    off = align_up(off + (size_t)H * T.opitch * 4, 256);
    T.feat = off;
    off = align_up(off + (size_t)H * T.opitch * 4, 256);
    T.total = off;
    return T;
}

// Image im of the batch; im is the same in every lane of the wavefront.
__device__ inline Img batch_img(const BatchTable& t, int im) {
    const BatchImage b = t.img[im];
    const int64_t mask_off = wave_uniform((int64_t)b.mask_off);
    const int64_t dist_off = wave_uniform((int64_t)b.dist_off);
    const int64_t feat_off = wave_uniform((int64_t)b.feat_off);
    const int64_t ws_off = wave_uniform((int64_t)b.ws_off);
    const int outs = wave_uniform((int32_t)b.outs);
    Img g;
    g.mask = global_ptr<const uint8_t>(t.mask_base + (uintptr_t)mask_off);
    g.mpitch = wave_uniform((int64_t)b.mpitch);
    g.dist = (outs & kOutDist) ? global_ptr<int32_t>(t.dist_base + 4 * (uintptr_t)dist_off)
                               : nullptr;
    g.feat = (outs & kOutFeat) ? global_ptr<int32_t>(t.feat_base + 4 * (uintptr_t)feat_off)
                               : nullptr;
    g.opitch = wave_uniform((int64_t)b.opitch);
    g.ws = global_ptr<uint8_t>(t.ws_base + (uintptr_t)ws_off);
    g.H = wave_uniform((int32_t)b.H);
    g.W = wave_uniform((int32_t)b.W);
    g.pol = wave_uniform((int32_t)b.pol);
    g.metric = 0;
    g.tr = wave_uniform((int32_t)b.tr);
    if (g.tr) {  // the transposed copies in the image's workspace
        const TrLayout T = tr_layout(g.H, g.W);
        const uintptr_t ws = t.ws_base + (uintptr_t)ws_off;
        g.mask = global_ptr<const uint8_t>(ws + T.mask);
        g.mpitch = T.mpitch;
        g.dist = (outs & kOutDist) ? global_ptr<int32_t>(ws + T.dist) : nullptr;
        g.feat = (outs & kOutFeat) ? global_ptr<int32_t>(ws + T.feat) : nullptr;
        g.opitch = T.opitch;
    }
    return g;
}

// Image of work item `item` of phase p: the last image whose prefix is <= item
// (item is the same in every lane of the wavefront).
// Work items per entry of a phase's coarse image index, as a power of two:
// the smallest 2^s with ceil(total / 2^s) <= n + 1 entries.
__host__ __device__ inline int index_shift(int total, int n) {
    int s = 0;
    while (((int64_t)(n + 1) << s) < (int64_t)total) ++s;
    return s;
}

// Image holding work item `item` of phase p: the last image whose prefix is at
// most the item.  The coarse index gives an image at or before it (the one
// holding the index entry's first item); a short forward walk over the prefix
// (one entry covers about one image's items) finds it, instead of a binary
// search of dependent loads over every image.
__device__ inline int batch_image_of(const BatchTable& t, int p, int item) {
    const int32_t* pre = t.prefix[p];
    int a = wave_uniform(t.first[p][item >> t.shift[p]]);
    while (a + 1 < t.nimg && wave_uniform(pre[a + 1]) <= item) ++a;
    return a;
}

// Batch tables (host side).  A table occupies table_bytes(n) bytes: the n
// BatchImage rows, then per phase the n + 1 prefix entries, then per phase the
// coarse image index (at most n + 1 entries), each part 256-byte aligned.  pack_table writes it to host memory `dst`: images no wider than
// lane_w (<= kLaneMaxW) take the one-lane-per-row pass; it returns the work
// totals per phase and the widest image that takes the pass with several
// lanes per row; EDT_ERR_TOO_LARGE if a total does not fit int32.  table_view
// points a BatchTable at a copy of it in device memory (totals: those
// pack_table returned, which fix the index shifts).
size_t table_bytes(int n);
int32_t pack_table(const BatchImage* img, int n, int lane_w, uint8_t* dst, int* totals,
                   int* max_w);
BatchTable table_view(const uint8_t* dev_table, int n, const int* totals);
// The whole transform of a batch, enqueued on stream.
hipError_t enqueue_batch(const BatchTable& t, const int* totals, int max_w, hipStream_t stream);
// Argument checks of one image (shared by the single, batch and serving calls).
int32_t check_image(const uint8_t* mask, int32_t H, int32_t W, int64_t mask_pitch,
                    int32_t polarity, int32_t metric, int64_t out_pitch);
// Enqueue the transform of one image (arguments already checked).
hipError_t enqueue_single(const Img& g, hipStream_t stream);
bool prof_enabled();

// Kernel timing (edt_profile_begin / edt_profile_end): a token from
// prof_begin (negative when timing is off) is closed by prof_end.
int prof_begin(const char* name, hipStream_t stream);
void prof_end(int token, hipStream_t stream);

// Launch-failure injection for tests of the error paths
// (edt_debug_fail_launch): skip_launch() is true for the armed launch and, on
// that thread, for every later launch until launch_status() reports the
// failure, so that no kernel runs on the state a skipped one should have
// written.  launch_status() is hipGetLastError(), or the injected failure.
bool skip_launch();
hipError_t launch_status();

// Launch a kernel on a stream, bracketed by timing events (recorded under
// `name`) when enabled.
#define EDT_LAUNCH_AS(name, kernel, grid, block, lds, stream, ...)           \
    do {                                                                     \
        if (::edt::skip_launch()) break;                                     \
        const int edt_tok_ = ::edt::prof_begin(name, stream);                \
        hipLaunchKernelGGL(kernel, grid, block, lds, stream, __VA_ARGS__);   \
        ::edt::prof_end(edt_tok_, stream);                                   \
    } while (0)
#define EDT_LAUNCH(kernel, grid, block, lds, stream, ...) \
    EDT_LAUNCH_AS(#kernel, kernel, grid, block, lds, stream, __VA_ARGS__)

// Number of compute units of the current device (cached per process).
int device_cus();

// Single image: the vertical pass and the row pass (enqueue on stream).
hipError_t launch_column_pass(const Img& g, hipStream_t stream);
hipError_t launch_row_pass(const Img& g, uint8_t* slots, hipStream_t stream);
// A batch described by a device table (totals[p] = work items of phase p;
// max_w = widest image, row forms are enqueued for the widths present).
hipError_t launch_column_pass_batch(const BatchTable& t, const int* totals, hipStream_t stream);
hipError_t launch_row_pass_batch(const BatchTable& t, const int* totals, int max_w,
                                 hipStream_t stream);
hipError_t launch_row_lanes_batch(const BatchTable& t, int total, hipStream_t stream);
// Masks of the transposed images of a batch into their workspaces, and their
// outputs back (totals: tiles of each phase).
hipError_t launch_transpose_in(const BatchTable& t, int total, hipStream_t stream);
hipError_t launch_transpose_out(const BatchTable& t, int total, hipStream_t stream);
// Workspace of the segment path for dense rows of one image: per row the
// envelope size of each segment, the envelopes themselves (entry e of segment
// c at slot c kSegL + e of the row, packed candidate; its start at the same
// slot of the row's list of site rows), and whether the row is left to the
// segment merge.
struct SegBufs {
    int16_t* segm;
    uint32_t* env;
    uint8_t* rowfail;
};
__host__ __device__ inline SegBufs seg_bufs(const Img& g) {
    const Layout L = layout_for(g.H, g.W);
    SegBufs b;
    b.segm = reinterpret_cast<int16_t*>(g.ws + L.segm);
    b.env = reinterpret_cast<uint32_t*>(g.ws + L.env);
    b.rowfail = g.ws + L.rowfail;
    return b;
}
// Dense rows of one image (has_segments(W), more than kSparseMaxN candidates,
// known only on the device): envelopes of row segments of L candidates (1, 2,
// 4 or 8 times kSegL), one lane per (row, segment), to `b`, segment c's entries at
// slots c L + e; every row is marked as not left to the merge.
hipError_t launch_row_segscan(const Img& g, int L, const SegBufs& b, hipStream_t stream);
hipError_t launch_sqrt(const int32_t* D, float* out, int64_t n, hipStream_t stream);

}  // namespace edt
