// Vertical pass of the exact EDT (Section 3.1 of Strutz, arXiv 2106.03503):
// for every pixel, the row of the nearest site in its own column, ties going to
// the upper site (the downward sweep keeps its value unless the upward sweep is
// strictly nearer).  The paper sweeps each column down and then up; here each
// column is cut into bands of kBand rows so that thousands of workgroups share
// the work:
//   k_band_bits    one 64-bit site mask per band column (reads the mask once);
//   k_band_carry   the state the two sweeps carry into each band: the last site
//                  row above it and the first site row below it;
//   k_col_compact  the list of columns holding any site -- the only columns
//                  whose parabolas can matter in any row (Section 3.2.2) --
//                  which is the same for every row;
//   k_nearest_row  per pixel of a listed column, the nearest site row from the
//                  band's bits and carries, stored compactly per row.
// Threads own adjacent columns, so the rows a wavefront touches are contiguous
// runs of bytes (mask) or int16s (outputs).
#include "edt_internal.h"

namespace edt {
namespace {

constexpr int kColThreads = 256;

// bit r of the result: pixel r of the band in this column is a site
template <bool kVec>
__device__ __forceinline__ void band_bits4(const uint8_t* __restrict__ p, int64_t pitch,
                                           int rows, uint32_t pol, int ncols,
                                           uint64_t out[4]) {
    uint64_t b0 = 0, b1 = 0, b2 = 0, b3 = 0;
    if (kVec) {
#pragma unroll 16
        for (int r = 0; r < rows; ++r) {
            const uint32_t v = *reinterpret_cast<const uint32_t*>(p + (int64_t)r * pitch);
            b0 |= (uint64_t)(((v & 0x000000ffu) != 0) ^ pol) << r;
            b1 |= (uint64_t)(((v & 0x0000ff00u) != 0) ^ pol) << r;
            b2 |= (uint64_t)(((v & 0x00ff0000u) != 0) ^ pol) << r;
            b3 |= (uint64_t)(((v & 0xff000000u) != 0) ^ pol) << r;
        }
    } else {
        for (int r = 0; r < rows; ++r) {
            const uint8_t* q = p + (int64_t)r * pitch;
            b0 |= (uint64_t)((q[0] != 0) ^ pol) << r;
            if (ncols > 1) b1 |= (uint64_t)((q[1] != 0) ^ pol) << r;
            if (ncols > 2) b2 |= (uint64_t)((q[2] != 0) ^ pol) << r;
            if (ncols > 3) b3 |= (uint64_t)((q[3] != 0) ^ pol) << r;
        }
    }
    out[0] = b0;
    out[1] = b1;
    out[2] = b2;
    out[3] = b3;
}

// Site bits of every band column, four columns per thread: bit r of
// bits[b][c] is set when pixel (b*kBand + r, c) is a site.
template <bool kVec>
__global__ __launch_bounds__(kColThreads) void k_band_bits(
    const uint8_t* __restrict__ mask, int H, int W, int64_t pitch, int polarity,
    uint64_t* __restrict__ bits) {
    const int c = (blockIdx.x * kColThreads + threadIdx.x) * 4;
    const int b = blockIdx.y;
    if (c >= W) return;
    const int row0 = b * kBand;
    const int rows = min(kBand, H - row0);
    const int ncols = min(4, W - c);
    uint64_t m[4];
    const uint8_t* p = mask + (int64_t)row0 * pitch + c;
    if (kVec && ncols == 4)
        band_bits4<true>(p, pitch, rows, (uint32_t)polarity, 4, m);
    else
        band_bits4<false>(p, pitch, rows, (uint32_t)polarity, ncols, m);
    uint64_t* o = bits + (int64_t)b * W + c;
    o[0] = m[0];
    if (ncols > 1) o[1] = m[1];
    if (ncols > 2) o[2] = m[2];
    if (ncols > 3) o[3] = m[3];
}

// Carries across band boundaries.  A workgroup owns kCarryCols columns; each
// of its kCarrySlices wavefronts owns a contiguous slice of bands.  up[b][c]
// is the last site row in the bands above b (the downward sweep's state
// entering band b) and down[b][c] the first site row in the bands below b (the
// upward sweep's state); flag[c] tells whether column c holds any site.
__global__ __launch_bounds__(kCarryCols* kCarrySlices) void k_band_carry(
    const uint64_t* __restrict__ bits, int nb, int W, int16_t* __restrict__ up,
    int16_t* __restrict__ down, int32_t* __restrict__ flag) {
    __shared__ int s_last[kCarrySlices][kCarryCols];
    __shared__ int s_first[kCarrySlices][kCarryCols];
    const int lane = threadIdx.x % kCarryCols;
    const int s = threadIdx.x / kCarryCols;
    const int c = blockIdx.x * kCarryCols + lane;
    const int b0 = (int)((int64_t)nb * s / kCarrySlices);
    const int b1 = (int)((int64_t)nb * (s + 1) / kCarrySlices);
    int last = -1, first = kNoBelow;
    if (c < W) {
        for (int b = b0; b < b1; ++b) {
            const uint64_t m = bits[(int64_t)b * W + c];
            if (m) {
                if (first == kNoBelow) first = b * kBand + __builtin_ctzll(m);
                last = b * kBand + 63 - __builtin_clzll(m);
            }
        }
    }
    s_last[s][lane] = last;
    s_first[s][lane] = first;
    __syncthreads();
    int run = -1;
    for (int q = 0; q < s; ++q) run = max(run, s_last[q][lane]);
    int run_dn = kNoBelow;
    for (int q = kCarrySlices - 1; q > s; --q) run_dn = min(run_dn, s_first[q][lane]);
    if (c >= W) return;
    for (int b = b0; b < b1; ++b) {
        up[(int64_t)b * W + c] = (int16_t)run;
        const uint64_t m = bits[(int64_t)b * W + c];
        if (m) run = b * kBand + 63 - __builtin_clzll(m);
    }
    if (s == kCarrySlices - 1) flag[c] = run >= 0;
    for (int b = b1 - 1; b >= b0; --b) {
        down[(int64_t)b * W + c] = (int16_t)run_dn;
        const uint64_t m = bits[(int64_t)b * W + c];
        if (m) run_dn = b * kBand + __builtin_ctzll(m);
    }
}

// List of the columns holding a site, in increasing order (one workgroup).
// meta[0] = their number n, meta[1] = the row pitch of the compact rows.
__global__ __launch_bounds__(1024) void k_col_compact(const int32_t* __restrict__ flag,
                                                      int W, int16_t* __restrict__ cols,
                                                      int32_t* __restrict__ meta) {
    __shared__ int s_wave[16];
    const int t = threadIdx.x;
    const int per = (W + 1023) / 1024;
    const int c0 = min(W, t * per), c1 = min(W, c0 + per);
    int cnt = 0;
    for (int c = c0; c < c1; ++c) cnt += flag[c] != 0;
    // workgroup exclusive prefix sum of cnt
    const int lane = t & 63, wave = t >> 6;
    int incl = cnt;
    for (int d = 1; d < 64; d <<= 1) {
        const int v = __shfl_up(incl, d, 64);
        if (lane >= d) incl += v;
    }
    if (lane == 63) s_wave[wave] = incl;
    __syncthreads();
    int pos = incl - cnt, total = 0;
    for (int w = 0; w < 16; ++w) {
        if (w < wave) pos += s_wave[w];
        total += s_wave[w];
    }
    for (int c = c0; c < c1; ++c)
        if (flag[c]) cols[pos++] = (int16_t)c;
    if (t == 0) {
        meta[0] = total;
        meta[1] = cand_pitch(total > 0 ? total : 1);
    }
}

// Nearest site row of every pixel of a listed column within one band: the
// last site at or above the pixel (inside the band, else the carry from above)
// against the first site at or below it (inside the band, else the carry from
// below); the upper one wins at equal distance.  Thread q handles the q-th
// listed column and writes rc[i][q].
__global__ __launch_bounds__(kColThreads) void k_nearest_row(
    const uint64_t* __restrict__ bits, const int16_t* __restrict__ up,
    const int16_t* __restrict__ down, const int16_t* __restrict__ cols,
    const int32_t* __restrict__ meta, int H, int W, int16_t* __restrict__ rc) {
    const int q = blockIdx.x * kColThreads + threadIdx.x;
    const int n = meta[0];
    if (q >= n) return;
    const int pitch = meta[1];
    const int b = blockIdx.y;
    const int c = cols[q];
    const int64_t bc = (int64_t)b * W + c;
    const uint64_t m = bits[bc];
    const int u = up[bc];
    const int d = down[bc];
    const int row0 = b * kBand;
    const int rows = min(kBand, H - row0);
    int16_t* out = rc + (int64_t)row0 * pitch + q;
    for (int r = 0; r < rows; ++r) {
        const int i = row0 + r;
        const uint64_t at_or_above = m & (r == 63 ? ~0ull : ((2ull << r) - 1));
        const uint64_t at_or_below = m & (~0ull << r);
        const int a = at_or_above ? row0 + 63 - __builtin_clzll(at_or_above) : u;
        const int bl = at_or_below ? row0 + __builtin_ctzll(at_or_below) : d;
        // the column holds a site, so at least one side exists
        const int best = (a >= 0 && (bl == kNoBelow || i - a <= bl - i)) ? a : bl;
        out[(int64_t)r * pitch] = (int16_t)best;
    }
}

}  // namespace

hipError_t launch_column_pass(const uint8_t* mask, int H, int W, int64_t pitch,
                              int polarity, uint8_t* ws, const Layout& L,
                              hipStream_t stream) {
    uint64_t* bits = reinterpret_cast<uint64_t*>(ws + L.bits);
    int16_t* up = reinterpret_cast<int16_t*>(ws + L.up);
    int16_t* down = reinterpret_cast<int16_t*>(ws + L.down);
    int32_t* flag = reinterpret_cast<int32_t*>(ws + L.flag);
    int16_t* cols = reinterpret_cast<int16_t*>(ws + L.cols);
    int32_t* meta = reinterpret_cast<int32_t*>(ws + L.meta);
    int16_t* rc = reinterpret_cast<int16_t*>(ws + L.rc);
    const bool vec = (reinterpret_cast<uintptr_t>(mask) % 4 == 0) && (pitch % 4 == 0);
    const dim3 gbits((W + 4 * kColThreads - 1) / (4 * kColThreads), L.nb);
    if (vec)
        EDT_LAUNCH_AS("k_band_bits", k_band_bits<true>, gbits, dim3(kColThreads), 0, stream, mask, H, W,
                   pitch, polarity, bits);
    else
        EDT_LAUNCH_AS("k_band_bits", k_band_bits<false>, gbits, dim3(kColThreads), 0, stream, mask, H, W,
                   pitch, polarity, bits);
    EDT_LAUNCH(k_band_carry, dim3((W + kCarryCols - 1) / kCarryCols),
               dim3(kCarryCols * kCarrySlices), 0, stream, bits, L.nb, W, up, down, flag);
    EDT_LAUNCH(k_col_compact, dim3(1), dim3(1024), 0, stream, flag, W, cols, meta);
    EDT_LAUNCH(k_nearest_row, dim3((W + kColThreads - 1) / kColThreads, L.nb),
               dim3(kColThreads), 0, stream, bits, up, down, cols, meta, H, W, rc);
    return hipGetLastError();
}

}  // namespace edt
