// Vertical pass of the exact EDT (Section 3.1 of Strutz, arXiv 2106.03503):
// for every pixel, the row of the nearest site in its own column, ties going to
// the upper site (the downward sweep keeps its value unless the upward sweep is
// strictly nearer).  The paper sweeps each column down and then up; here each
// column is cut into bands of kBand rows so that thousands of workgroups share
// the work:
//   bits     one 64-bit site mask per band column (reads the mask once);
//   carry    the state the two sweeps carry into each band: the last site row
//            above it and the first site row below it;
//   compact  the list of columns holding any site -- the only columns whose
//            parabolas can matter in any row (Section 3.2.2) -- the same list
//            for every row;
//   nearest  per pixel of a listed column, the nearest site row from the
//            band's bits and carries, stored compactly per row.
// Each phase is a device function over one image and one work item; the
// single-image kernels index work items by block, the batch kernels find the
// image of an item in the batch table.  Threads own adjacent columns, so the
// rows a wavefront touches are contiguous runs of bytes or int16s.
#include "edt_internal.h"

namespace edt {
namespace {

constexpr int kColThreads = 256;

// High bit of each byte of w set iff that byte is nonzero.
__device__ __forceinline__ uint32_t nonzero_bytes(uint32_t w) {
    return (((w & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | w) & 0x80808080u;
}

// ---------------------------------------------------------------- bits
// Work item (band b, column block bx) of 1024 columns: each of the four
// wavefronts loads 16 rows of the band (16 columns per lane and row: one
// 16-byte load when the mask allows, else four 4-byte or sixteen 1-byte
// loads) and builds 16-bit partial column masks, joined through LDS into the
// 64-bit band masks: bit r of bits[b][c] is set when pixel (b*kBand + r, c) is
// a site.
__device__ void bits_item(const Img& g, const Views& v, int item) {
    __shared__ uint16_t s_part[4][16][65];
    const int nbx = (g.W + kBitsCols - 1) / kBitsCols;
    const int b = item / nbx, bx = item - b * nbx;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int cbase = bx * kBitsCols;
    const int c = cbase + lane * 16;
    const int rw0 = b * kBand + wave * 16;
    const int rows = max(0, min(16, g.H - rw0));
    const int ncols = max(0, min(16, g.W - c));
    uint32_t part[16];
#pragma unroll
    for (int x = 0; x < 16; ++x) part[x] = 0u;
    const uint8_t* p = g.mask + (int64_t)rw0 * g.mpitch + c;
    const uint32_t flip = g.pol ? 0x80808080u : 0u;
    const uintptr_t pa = reinterpret_cast<uintptr_t>(p);
    if (ncols == 16 && rows == 16 && pa % 16 == 0 && g.mpitch % 16 == 0) {
        uint4 q[16];
#pragma unroll
        for (int k = 0; k < 16; ++k) q[k] = *reinterpret_cast<const uint4*>(p + (int64_t)k * g.mpitch);
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            const uint32_t w4[4] = {q[k].x, q[k].y, q[k].z, q[k].w};
#pragma unroll
            for (int h = 0; h < 4; ++h) {
                const uint32_t s = nonzero_bytes(w4[h]) ^ flip;
#pragma unroll
                for (int x = 0; x < 4; ++x) part[4 * h + x] |= ((s >> (8 * x + 7)) & 1u) << k;
            }
        }
    } else if (ncols == 16 && pa % 4 == 0 && g.mpitch % 4 == 0) {
        for (int k = 0; k < rows; ++k) {
            const uint32_t* q = reinterpret_cast<const uint32_t*>(p + (int64_t)k * g.mpitch);
#pragma unroll
            for (int h = 0; h < 4; ++h) {
                const uint32_t s = nonzero_bytes(q[h]) ^ flip;
#pragma unroll
                for (int x = 0; x < 4; ++x) part[4 * h + x] |= ((s >> (8 * x + 7)) & 1u) << k;
            }
        }
    } else if (ncols > 0) {
        const uint32_t pol = (uint32_t)g.pol;
        for (int k = 0; k < rows; ++k) {
            const uint8_t* q = p + (int64_t)k * g.mpitch;
            for (int x = 0; x < ncols; ++x) part[x] |= ((uint32_t)(q[x] != 0) ^ pol) << k;
        }
    }
#pragma unroll
    for (int x = 0; x < 16; ++x) s_part[wave][x][lane] = (uint16_t)part[x];
    __syncthreads();
#pragma unroll
    for (int y = 0; y < 4; ++y) {
        const int cl = threadIdx.x * 4 + y;
        const int cc = cbase + cl;
        if (cc < g.W) {
            const int ln = cl >> 4, x = cl & 15;
            v.bits[(int64_t)b * g.W + cc] = (uint64_t)s_part[0][x][ln] |
                                            ((uint64_t)s_part[1][x][ln] << 16) |
                                            ((uint64_t)s_part[2][x][ln] << 32) |
                                            ((uint64_t)s_part[3][x][ln] << 48);
        }
    }
    __syncthreads();  // s_part is reused by the next item of this workgroup
}

// --------------------------------------------------------------- carry
// Work item bx: kCarryCols columns; each of the kCarrySlices wavefronts owns a
// contiguous slice of bands.  up[b][c] is the last site row in the bands above
// b (the downward sweep's state entering band b), down[b][c] the first site
// row in the bands below b (the upward sweep's state); flag[c] tells whether
// column c holds any site (zero past W up to the list capacity).
__device__ void carry_item(const Img& g, const Views& v, int bx) {
    __shared__ int s_last[kCarrySlices][kCarryCols];
    __shared__ int s_first[kCarrySlices][kCarryCols];
    const int nb = (g.H + kBand - 1) / kBand;
    const int W = g.W;
    const int lane = threadIdx.x % kCarryCols;
    const int s = threadIdx.x / kCarryCols;
    const int c = bx * kCarryCols + lane;
    const int b0 = (int)((int64_t)nb * s / kCarrySlices);
    const int b1 = (int)((int64_t)nb * (s + 1) / kCarrySlices);
    int last = -1, first = kNoBelow;
    if (c < W) {
        for (int b = b0; b < b1; ++b) {
            const uint64_t m = v.bits[(int64_t)b * W + c];
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
    __syncthreads();  // s_last / s_first are reused by the next item
    if (c >= W) {
        if (s == 0 && c < cand_pitch(W)) v.flag[c] = 0;
        return;
    }
    for (int b = b0; b < b1; ++b) {
        v.up[(int64_t)b * W + c] = (int16_t)run;
        const uint64_t m = v.bits[(int64_t)b * W + c];
        if (m) run = b * kBand + 63 - __builtin_clzll(m);
    }
    if (s == kCarrySlices - 1) v.flag[c] = run >= 0;
    for (int b = b1 - 1; b >= b0; --b) {
        v.down[(int64_t)b * W + c] = (int16_t)run_dn;
        const uint64_t m = v.bits[(int64_t)b * W + c];
        if (m) run_dn = b * kBand + __builtin_ctzll(m);
    }
}

// ------------------------------------------------------------- compact
// The list of the columns holding a site, in increasing order (1024 threads,
// 32 column flags each).  meta[0] = their number n, meta[1] = the row pitch of
// the compact rows.
__device__ void compact_item(const Img& g, const Views& v) {
    __shared__ int s_wave[16];
    const int t = threadIdx.x;
    const int c0 = t * 32;
    uint32_t bitsv = 0;  // bit x: column c0 + x holds a site
    if (c0 < cand_pitch(g.W)) {
        const uint4* f = reinterpret_cast<const uint4*>(v.flag + c0);
        const uint4 a = f[0], b = f[1];
        const uint32_t wv[8] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
#pragma unroll
        for (int h = 0; h < 8; ++h) {
            const uint32_t s = nonzero_bytes(wv[h]);
#pragma unroll
            for (int x = 0; x < 4; ++x) bitsv |= ((s >> (8 * x + 7)) & 1u) << (4 * h + x);
        }
    }
    const int cnt = __popc(bitsv);
    const int lane = t & 63, wave = t >> 6;
    int incl = cnt;
    for (int d = 1; d < 64; d <<= 1) {
        const int x = __shfl_up(incl, d, 64);
        if (lane >= d) incl += x;
    }
    if (lane == 63) s_wave[wave] = incl;
    __syncthreads();
    int pos = incl - cnt, total = 0;
    for (int w = 0; w < 16; ++w) {
        if (w < wave) pos += s_wave[w];
        total += s_wave[w];
    }
    __syncthreads();  // s_wave is reused by the next item
    while (bitsv) {
        const int x = __ffs(bitsv) - 1;
        bitsv &= bitsv - 1;
        v.cols[pos++] = (int16_t)(c0 + x);
    }
    if (t == 0) {
        v.meta[0] = total;
        v.meta[1] = cand_pitch(total > 0 ? total : 1);
    }
}

// ------------------------------------------------------------- nearest
// Work item (band b, block qb of kNearCols listed columns): thread q handles
// listed column q and writes rc[i][q] for the band's rows.  The last site at or
// above the pixel (inside the band, else the carry from above) competes with
// the first site at or below it (inside the band, else the carry from below);
// the upper one wins at equal distance.  Items past the device-side count n
// do nothing.
__device__ void near_item(const Img& g, const Views& v, int item, int qblocks) {
    const int n = v.meta[0];
    const int pitch = v.meta[1];
    const int b = item / qblocks;
    const int q = (item - b * qblocks) * kNearCols + threadIdx.x;
    if (q >= n) return;
    const int c = v.cols[q];
    const int64_t bc = (int64_t)b * g.W + c;
    const uint64_t m = v.bits[bc];
    const int u = v.up[bc];
    const int d = v.down[bc];
    const int row0 = b * kBand;
    const int rows = min(kBand, g.H - row0);
    int16_t* out = v.rc + (int64_t)row0 * pitch + q;
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

// ------------------------------------------------------ single image
__global__ __launch_bounds__(kColThreads) void k_bits(Img g) {
    const Views v = views_of(g);
    bits_item(g, v, blockIdx.x);
}
__global__ __launch_bounds__(kCarryCols* kCarrySlices) void k_carry(Img g) {
    const Views v = views_of(g);
    carry_item(g, v, blockIdx.x);
}
__global__ __launch_bounds__(1024) void k_compact(Img g) {
    const Views v = views_of(g);
    compact_item(g, v);
}
// persistent grid over the items (their useful number depends on n)
__global__ __launch_bounds__(kNearCols) void k_near(Img g) {
    const Views v = views_of(g);
    // items per band from the device-side count of listed columns
    const int qblocks = (v.meta[0] + kNearCols - 1) / kNearCols;
    const int items = ((g.H + kBand - 1) / kBand) * qblocks;
    for (int item = blockIdx.x; item < items; item += gridDim.x) near_item(g, v, item, qblocks);
}

// --------------------------------------------------------------- batch
// Persistent grids over all work items of a phase in the batch; a workgroup
// looks up the image of each item in the table (one binary search per item,
// by thread 0, shared through LDS).
template <int kPh>
__device__ __forceinline__ int batch_lookup(const BatchTable& t, int item) {
    __shared__ int s_img;
    __syncthreads();
    if (threadIdx.x == 0) s_img = batch_image_of(t, kPh, item);
    __syncthreads();
    return s_img;
}

__global__ __launch_bounds__(kColThreads) void k_bits_batch(BatchTable t, int total) {
    for (int item = blockIdx.x; item < total; item += gridDim.x) {
        const int im = batch_lookup<kPhBits>(t, item);
        const Img g = batch_img(t, im);
        bits_item(g, views_of(g), item - t.prefix[kPhBits][im]);
    }
}
__global__ __launch_bounds__(kCarryCols* kCarrySlices) void k_carry_batch(BatchTable t, int total) {
    for (int item = blockIdx.x; item < total; item += gridDim.x) {
        const int im = batch_lookup<kPhCarry>(t, item);
        const Img g = batch_img(t, im);
        carry_item(g, views_of(g), item - t.prefix[kPhCarry][im]);
    }
}
__global__ __launch_bounds__(1024) void k_compact_batch(BatchTable t, int total) {
    for (int im = blockIdx.x; im < total; im += gridDim.x) {
        const Img g = batch_img(t, im);
        compact_item(g, views_of(g));
    }
}
__global__ __launch_bounds__(kNearCols) void k_near_batch(BatchTable t, int total) {
    for (int item = blockIdx.x; item < total; item += gridDim.x) {
        const int im = batch_lookup<kPhNear>(t, item);
        const Img g = batch_img(t, im);
        near_item(g, views_of(g), item - t.prefix[kPhNear][im], (g.W + kNearCols - 1) / kNearCols);
    }
}

}  // namespace

int device_cus() {
    static int cus = 0;
    if (cus == 0) {
        int dev = 0, v = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
            v > 0)
            cus = v;
        else
            cus = 256;
    }
    return cus;
}

hipError_t launch_column_pass(const Img& g, hipStream_t stream) {
    EDT_LAUNCH_AS("k_band_bits", k_bits, dim3(items_bits(g.H, g.W)), dim3(kColThreads), 0,
                  stream, g);
    EDT_LAUNCH_AS("k_band_carry", k_carry, dim3(items_carry(g.H, g.W)),
                  dim3(kCarryCols * kCarrySlices), 0, stream, g);
    EDT_LAUNCH_AS("k_col_compact", k_compact, dim3(1), dim3(1024), 0, stream, g);
    // enough workgroups for a dense image, few enough that idle ones are cheap
    const int items = items_near(g.H, g.W);
    EDT_LAUNCH_AS("k_nearest_row", k_near, dim3(items < 2048 ? items : 2048), dim3(kNearCols), 0,
                  stream, g);
    return hipGetLastError();
}

hipError_t launch_column_pass_batch(const BatchTable& t, const int* totals, hipStream_t stream) {
    const int cap = 16 * device_cus();
    auto grid = [&](int total) { return dim3((unsigned)(total < cap ? total : cap)); };
    EDT_LAUNCH_AS("k_band_bits", k_bits_batch, grid(totals[kPhBits]), dim3(kColThreads), 0,
                  stream, t, totals[kPhBits]);
    EDT_LAUNCH_AS("k_band_carry", k_carry_batch, grid(totals[kPhCarry]),
                  dim3(kCarryCols * kCarrySlices), 0, stream, t, totals[kPhCarry]);
    EDT_LAUNCH_AS("k_col_compact", k_compact_batch, grid(totals[kPhCompact]), dim3(1024), 0,
                  stream, t, totals[kPhCompact]);
    EDT_LAUNCH_AS("k_nearest_row", k_near_batch, grid(totals[kPhNear]), dim3(kNearCols), 0,
                  stream, t, totals[kPhNear]);
    return hipGetLastError();
}

}  // namespace edt
