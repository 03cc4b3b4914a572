// Horizontal pass of the exact EDT (Section 3.3.1 of Strutz, arXiv
// 2106.03503): per row, the lower envelope of the parabolas
// D_k(j) = Dv(k) + (j - k)^2 (Eq. eq_parabola) over the columns k that hold a
// site, then a fill of every pixel from the parabola that owns it.
//
// Ties: the comparison between two parabolas at a pixel is lexicographic on
// (D, feature index), feature = r*W + k, so the owner of a pixel is the nearest
// site with the smallest row-major index.  For k < l, parabola l beats k at
// every j >= s where s is the first integer past the crossing of Eq.
// eq_intersection (or at it, when l wins the tie), computed with exact integer
// floor division and clamped to [0, W].
#include "edt_internal.h"

namespace edt {
namespace {

// First pixel j in [0, W] at which parabola l (site row rl) beats parabola k
// (site row rk), k < l, in row i.  W means "never inside the row".
__device__ __forceinline__ int first_win(int k, int rk, int l, int rl, int i, int W) {
    const int64_t dk = (int64_t)(i - rk) * (i - rk);
    const int64_t dl = (int64_t)(i - rl) * (i - rl);
    const int64_t num = dl - dk + (int64_t)(l - k) * (l + k);
    const int64_t den = 2 * (int64_t)(l - k);
    // l beats k at j iff j*den > num, or j*den == num and l has the smaller
    // index, i.e. a smaller site row (in the same row l's column is larger, so
    // its index is larger).  Hence s = floor((num - [l wins ties]) / den) + 1.
    const int64_t n2 = num - (rl < rk ? 1 : 0);
    if (n2 < 0) return 0;
    const int64_t q = n2 / den;
    return q + 1 < (int64_t)W ? (int)(q + 1) : W;
}

__global__ __launch_bounds__(kRowThreads) void k_row_envelope(
    const int16_t* __restrict__ rstar, int H, int W, int32_t* __restrict__ dist,
    int32_t* __restrict__ feat, int64_t out_pitch, uint8_t* __restrict__ scratch) {
    extern __shared__ uint32_t lds[];
    __shared__ int s_wave_count[kRowThreads / 64];
    __shared__ int s_m;
    uint32_t* cand;  // (column << 16) | site row, increasing column
    int16_t* start;  // first pixel owned by each stacked parabola
    if (scratch) {
        cand = reinterpret_cast<uint32_t*>(scratch + (size_t)blockIdx.x * row_slot_bytes(W));
    } else {
        cand = lds;
    }
    start = reinterpret_cast<int16_t*>(cand + W);
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;

    for (int i = blockIdx.x; i < H; i += gridDim.x) {
        const int16_t* row = rstar + (int64_t)i * W;
        // 1. Candidate columns (those with a site, Section 3.2.2), compacted in
        //    column order with a wavefront ballot and a workgroup prefix.
        int n = 0;
        for (int c0 = 0; c0 < W; c0 += kRowThreads) {
            const int c = c0 + threadIdx.x;
            const int r = (c < W) ? row[c] : -1;
            const bool is_cand = r >= 0;
            const uint64_t ballot = __ballot(is_cand);
            const int prefix = __popcll(ballot & ((1ull << lane) - 1));
            if (lane == 0) s_wave_count[wave] = __popcll(ballot);
            __syncthreads();
            int off = n, total = 0;
            for (int w = 0; w < kRowThreads / 64; ++w) {
                if (w < wave) off += s_wave_count[w];
                total += s_wave_count[w];
            }
            if (is_cand) cand[off + prefix] = ((uint32_t)c << 16) | (uint32_t)r;
            n += total;
            __syncthreads();
        }
        // 2. Lower envelope, one scan over the candidates with a stack kept in
        //    place at the front of the candidate list.
        if (threadIdx.x == 0) {
            int m = 0;
            for (int q = 0; q < n; ++q) {
                const uint32_t cq = cand[q];
                const int l = (int)(cq >> 16), rl = (int)(cq & 0xFFFF);
                int s = 0;
                while (m > 0) {
                    const uint32_t ct = cand[m - 1];
                    s = first_win((int)(ct >> 16), (int)(ct & 0xFFFF), l, rl, i, W);
                    if (s <= start[m - 1])
                        --m;  // the new parabola hides the one on top
                    else
                        break;
                }
                if (m == 0) {
                    cand[0] = cq;
                    start[0] = 0;
                    m = 1;
                } else if (s <= W - 1) {
                    cand[m] = cq;
                    start[m] = (int16_t)s;
                    ++m;
                }
            }
            s_m = m;
        }
        __syncthreads();
        const int m = s_m;
        // 3. Fill: each thread owns a contiguous run of pixels, finds the
        //    parabola owning its first pixel by binary search and walks on.
        const int seg = (W + kRowThreads - 1) / kRowThreads;
        const int j0 = threadIdx.x * seg;
        const int j1 = min(W, j0 + seg);
        int32_t* drow = dist ? dist + (int64_t)i * out_pitch : nullptr;
        int32_t* frow = feat ? feat + (int64_t)i * out_pitch : nullptr;
        if (m == 0) {
            for (int j = j0; j < j1; ++j) {
                if (drow) drow[j] = INT32_MAX;
                if (frow) frow[j] = -1;
            }
        } else if (j0 < j1) {
            int lo = 0, hi = m - 1;
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (start[mid] <= j0) lo = mid; else hi = mid - 1;
            }
            int e = lo;
            uint32_t ce = cand[e];
            int k = (int)(ce >> 16), r = (int)(ce & 0xFFFF);
            uint32_t dv = (uint32_t)((i - r) * (i - r));
            int next = (e + 1 < m) ? start[e + 1] : W;
            for (int j = j0; j < j1; ++j) {
                while (j >= next) {
                    ++e;
                    ce = cand[e];
                    k = (int)(ce >> 16);
                    r = (int)(ce & 0xFFFF);
                    dv = (uint32_t)((i - r) * (i - r));
                    next = (e + 1 < m) ? start[e + 1] : W;
                }
                if (drow) drow[j] = (int32_t)(dv + (uint32_t)((j - k) * (j - k)));
                if (frow) frow[j] = r * W + k;
            }
        }
        __syncthreads();  // the next row reuses the candidate list
    }
}

}  // namespace

hipError_t launch_row_pass(const int16_t* rstar, int H, int W, int32_t* dist,
                           int32_t* feat, int64_t out_pitch, uint8_t* ws,
                           const Layout& L, hipStream_t stream) {
    const bool wide = W > kRowLdsMaxW;
    const size_t lds = wide ? 0 : align_up((size_t)W * 6, 16);
    uint8_t* scratch = wide ? ws + L.rowscratch : nullptr;
    const int grid = H < kRowSlots ? H : kRowSlots;
    EDT_LAUNCH(k_row_envelope, dim3(grid), dim3(kRowThreads), lds, stream,
                       rstar, H, W, dist, feat, out_pitch, scratch);
    return hipGetLastError();
}

}  // namespace edt
