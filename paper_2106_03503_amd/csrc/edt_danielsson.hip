// Danielsson's approximate Euclidean distance transform (arXiv 2106.03503,
// Section 2.3, in the two-scan form the paper gives after Grevera): every
// pixel holds a relative position (dy, dx), the magnitudes of the offsets to
// the site it was reached from, and d^2 = dy^2 + dx^2.  A reached neighbour
// offers its position plus one in dy for a vertical step, in dx for a
// horizontal one and in both for a diagonal one; the pixel takes the offer
// when it is strictly nearer.  The first scan takes rows 1 .. H-1 downwards
// (upper neighbour for every pixel; left, upper-left from left to right;
// upper-right, right from right to left), the second rows H-2 .. 0 upwards
// (lower neighbour; left, lower-left; right, lower-right).
//
// The result depends on the order of the offers pixel by pixel, so a row's
// sweeps are one sequential chain: one workgroup of one wavefront takes the
// whole image, the vertical offers and the row transfers on all 64 lanes.  A
// sweep takes the row 64 pixels at a time into the lanes' registers and walks
// them in order, reading each pixel and its diagonal neighbour out of their
// lanes, taking the offers in scalar registers (a dependent step there costs
// a cycle or two, where the vector unit of a lone wavefront takes several)
// and writing the result back into the pixel's lane.  This is the approximate
// comparison, not a hot path.  Relative positions travel packed as
// (dy << 16) | dx, -1 = unreached.
#include "../../include/edt.h"
#include "edt_internal.h"

namespace edt {
namespace {

constexpr int kDanMaxW = 8192;  // two rows of packed positions in LDS
// The offers are one chain of about 4 H W steps: images are capped so that a
// call stays within seconds.
constexpr int64_t kDanMaxPixels = (int64_t)1 << 22;

__device__ __forceinline__ int d2_of(int32_t p) {
    const int dy = p >> 16, dx = p & 0xFFFF;
    return sqr_c(dy) + sqr_c(dx);
}

// The pixel holding `cur` takes `from` plus (ay, ax) when strictly nearer.
// Stored offsets stay within the image, so an offer is at most one past it;
// the field test only keeps a 16-bit field from overflowing.  One select and
// no branch:
// the sweeps run this as a chain of scalar instructions, where every branch
// would stall the lone wavefront.
__device__ __forceinline__ int32_t offer(int32_t cur, int32_t from, int ay, int ax) {
    const int32_t f = from < 0 ? 0 : from, c = cur < 0 ? 0 : cur;  // squares stay in range
    const int ny = (f >> 16) + ay, nx = (f & 0xFFFF) + ax;
    const int nd = sqr_c(ny) + sqr_c(nx);
    const bool take = (from >= 0) & (ny <= 0x7FFF) & (nx <= 0x7FFF) &
                      ((cur < 0) | (d2_of(c) > nd));
    return take ? (ny << 16) | nx : cur;
}

__device__ __forceinline__ int32_t initial(const uint8_t* mask, int64_t mpitch, int pol, int i,
                                           int j) {
    const bool obj = mask[(int64_t)i * mpitch + j] != 0;
    return (pol ? !obj : obj) ? 0 : -1;
}

// A sweep's chain carries the running position v packed, with its squared
// length vd.  Per chunk of 64 pixels the lanes first work out, for their own
// pixel, the squared length of its position (INT32_MAX when unreached) and the
// diagonal neighbour's offer: its position plus (1, 1) packed (-1 when the
// neighbour is unreached or a field would pass 0x7FFF) and its squared length.
// An offer of v plus (0, 1) is then v + 1 with length vd + 2 x + 1, so a step
// is a few scalar instructions.  Each offer is taken when strictly nearer,
// exactly as offer() decides.
struct Chunk {
    int32_t c, cd, dp, dd;  // this lane's pixel and its length; diagonal offer and its length
};

__device__ __forceinline__ Chunk chunk_of(int32_t c, int32_t diag) {
    Chunk k;
    k.c = c;
    k.cd = c < 0 ? INT32_MAX : d2_of(c);
    const int32_t f = diag < 0 ? 0 : diag;
    const int ny = (f >> 16) + 1, nx = (f & 0xFFFF) + 1;
    const bool ok = (diag >= 0) & (ny <= 0x7FFF) & (nx <= 0x7FFF);
    k.dp = ok ? (ny << 16) | nx : -1;
    k.dd = sqr_c(ny) + sqr_c(nx);
    return k;
}

// The pixel (p, pd) takes v plus (0, 1) when strictly nearer.
__device__ __forceinline__ void take_side(int32_t& p, int32_t& pd, int32_t v, int32_t vd) {
    const int vx = v & 0xFFFF;
    const int nd = vd + 2 * vx + 1;
    const bool t = (v >= 0) & (vx < 0x7FFF) & (pd > nd);
    p = t ? v + 1 : p;
    pd = t ? nd : pd;
}

// The pixel (p, pd) takes the diagonal offer (dp, dd) when strictly nearer.
__device__ __forceinline__ void take_diag(int32_t& p, int32_t& pd, int32_t dp, int32_t dd) {
    const bool t = (dp >= 0) & (pd > dd);
    p = t ? dp : p;
    pd = t ? dd : pd;
}

// Left-to-right sweep of row `cur` (both scans): pixel j takes its left
// neighbour's position plus (0, 1), then the upper (first scan) or lower
// (second scan) left neighbour's plus (1, 1), from `prev`.
__device__ void sweep_right(int32_t* cur, const int32_t* prev, int W, int lane) {
    int32_t v = -1, vd = INT32_MAX;
    for (int base = 0; base < W; base += 64) {
        const int j = base + lane;
        const Chunk ch = chunk_of(j < W ? cur[j] : -1, j < W && j > 0 ? prev[j - 1] : -1);
        int32_t out = ch.c;
        const int cnt = min(64, W - base);
        int k = 0;
        if (base == 0) {  // pixel 0 starts the chain as it is
            v = __builtin_amdgcn_readlane(ch.c, 0);
            vd = __builtin_amdgcn_readlane(ch.cd, 0);
            k = 1;
        }
        for (; k < cnt; ++k) {
            int32_t p = __builtin_amdgcn_readlane(ch.c, k);
            int32_t pd = __builtin_amdgcn_readlane(ch.cd, k);
            take_side(p, pd, v, vd);
            take_diag(p, pd, __builtin_amdgcn_readlane(ch.dp, k),
                      __builtin_amdgcn_readlane(ch.dd, k));
            v = p;
            vd = pd;
            out = lane == k ? v : out;
        }
        if (j < W) cur[j] = out;
    }
}

// Right-to-left sweep: pixel j takes the right neighbour's position plus
// (0, 1) and the upper or lower right neighbour's plus (1, 1), the diagonal
// first in the first scan (kDiagFirst) and second in the second.
template <bool kDiagFirst>
__device__ void sweep_left(int32_t* cur, const int32_t* prev, int W, int lane) {
    int32_t v = -1, vd = INT32_MAX;
    for (int base = (W - 1) & ~63; base >= 0; base -= 64) {
        const int j = base + lane;
        const Chunk ch = chunk_of(j < W ? cur[j] : -1, j + 1 < W ? prev[j + 1] : -1);
        int32_t out = ch.c;
        int k = min(64, W - base) - 1;
        if (base + k == W - 1) {  // pixel W - 1 starts the chain as it is
            v = __builtin_amdgcn_readlane(ch.c, k);
            vd = __builtin_amdgcn_readlane(ch.cd, k);
            --k;
        }
        for (; k >= 0; --k) {
            int32_t p = __builtin_amdgcn_readlane(ch.c, k);
            int32_t pd = __builtin_amdgcn_readlane(ch.cd, k);
            const int32_t dp = __builtin_amdgcn_readlane(ch.dp, k);
            const int32_t dd = __builtin_amdgcn_readlane(ch.dd, k);
            if (kDiagFirst) {
                take_diag(p, pd, dp, dd);
                take_side(p, pd, v, vd);
            } else {
                take_side(p, pd, v, vd);
                take_diag(p, pd, dp, dd);
            }
            v = p;
            vd = pd;
            out = lane == k ? v : out;
        }
        if (j < W) cur[j] = out;
    }
}

__global__ __launch_bounds__(64) void k_danielsson(const uint8_t* mask, int64_t mpitch, int H,
                                                   int W, int pol, int32_t* dist, int32_t* rel,
                                                   int64_t opitch) {
    __shared__ int32_t rowbuf[2][kDanMaxW];
    const int lane = threadIdx.x;
    int32_t* prev = rowbuf[0];
    int32_t* cur = rowbuf[1];
    auto swap_rows = [&]() {
        int32_t* t = prev;
        prev = cur;
        cur = t;
    };
    // row 0 as initialised (the first scan does not visit it)
    for (int j = lane; j < W; j += 64) {
        prev[j] = initial(mask, mpitch, pol, 0, j);
        rel[j] = prev[j];
    }
    __syncthreads();
    for (int i = 1; i < H; ++i) {  // first scan, downwards
        for (int j = lane; j < W; j += 64)
            cur[j] = offer(initial(mask, mpitch, pol, i, j), prev[j], 1, 0);
        __syncthreads();
        sweep_right(cur, prev, W, lane);
        sweep_left<true>(cur, prev, W, lane);
        __syncthreads();
        for (int j = lane; j < W; j += 64) rel[(int64_t)i * opitch + j] = cur[j];
        swap_rows();
        __syncthreads();
    }
    __threadfence();  // the second scan reads back what the first one wrote
    // prev holds row H-1 as the first scan left it
    for (int i = H - 2; i >= 0; --i) {  // second scan, upwards
        for (int j = lane; j < W; j += 64)
            cur[j] = offer(rel[(int64_t)i * opitch + j], prev[j], 1, 0);
        __syncthreads();
        sweep_right(cur, prev, W, lane);
        sweep_left<false>(cur, prev, W, lane);
        __syncthreads();
        for (int j = lane; j < W; j += 64) rel[(int64_t)i * opitch + j] = cur[j];
        swap_rows();
        __syncthreads();
    }
    __threadfence();
    for (int i = 0; i < H; ++i)
        for (int j = lane; j < W; j += 64) {
            const int32_t p = rel[(int64_t)i * opitch + j];
            dist[(int64_t)i * opitch + j] = p < 0 ? EDT_INF_SQ : d2_of(p);
        }
}

}  // namespace
}  // namespace edt

extern "C" {

edt_status edt_danielsson(const uint8_t* mask, int32_t H, int32_t W, int64_t mask_pitch,
                          int32_t polarity, int32_t* dist_sq, int32_t* rel, int64_t out_pitch,
                          void* stream) {
    if (H < 1 || W < 1 || H > EDT_MAX_SIDE || W > edt::kDanMaxW ||
        (int64_t)H * W > edt::kDanMaxPixels)
        return EDT_ERR_TOO_LARGE;
    if (!mask || !dist_sq || !rel || mask_pitch < W || out_pitch < W) return EDT_ERR_INVALID_ARG;
    if (polarity != EDT_TO_OBJECT && polarity != EDT_TO_BACKGROUND) return EDT_ERR_INVALID_ARG;
    const uintptr_t d0 = reinterpret_cast<uintptr_t>(dist_sq);
    const uintptr_t r0 = reinterpret_cast<uintptr_t>(rel);
    const uintptr_t span = 4 * (uintptr_t)((H - 1) * out_pitch + W);
    if (d0 < r0 + span && r0 < d0 + span) return EDT_ERR_INVALID_ARG;  // rel is read back
    EDT_LAUNCH_AS("k_danielsson", edt::k_danielsson, dim3(1), dim3(64), 0,
                  reinterpret_cast<hipStream_t>(stream), mask, mask_pitch, H, W, polarity,
                  dist_sq, rel, out_pitch);
    return edt::launch_status() == hipSuccess ? EDT_OK : EDT_ERR_DEVICE;
}

}  // extern "C"
