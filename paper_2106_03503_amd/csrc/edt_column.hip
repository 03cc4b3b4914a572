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

// High bit of each byte of w set iff that byte is nonzero.
__device__ __forceinline__ uint32_t nonzero_bytes(uint32_t w) {
    return (((w & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | w) & 0x80808080u;
}

// ---------------------------------------------------------------- bits
// Work item (band b, block bx of kBitsCols columns) of one wavefront: lane l
// owns the four columns bx*kBitsCols + 4l .. 4l + 3 and reads them as one
// 4-byte word per row of the band.  Within a group of eight rows, the high
// bit of each nonzero byte, shifted down by (7 - row in the group), lands on
// bit (row in the group) of the same byte, so one word per group gathers
// eight rows of the lane's four columns; byte x of the eight group words,
// put side by side, is column x's 64-bit band mask: bit r of bits[b][c] is
// set when pixel (b*kBand + r, c) is a site.
//
// Loads are whole aligned 4-byte words.  When the mask's base and row pitch
// are multiples of 4 each lane reads one word per row; otherwise it reads the
// one or two aligned words that hold its four bytes.  A word that holds a
// pixel of the image may also hold bytes past column W - 1 (or before the
// row's first byte); those bytes are read and ignored.  An aligned word never
// straddles a page, so this reads no page the image does not touch.
__device__ __forceinline__ uint32_t gather_byte(const uint32_t (&acc)[8], int g0, int x) {
    uint32_t w = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) w |= ((acc[g0 + k] >> (8 * x)) & 0xFFu) << (8 * k);
    return w;
}

__device__ __forceinline__ void bits_item(const Img& g, const Views& v, int item, int lane) {
    const int nbx = (g.W + kBitsCols - 1) / kBitsCols;
    const int b = item / nbx, bx = item - b * nbx;
    const int c = bx * kBitsCols + lane * 4;
    const int row0 = b * kBand;
    const int rows = min(kBand, g.H - row0);
    const int ncols = min(4, g.W - c);
    if (ncols <= 0) return;
    const bool words = reinterpret_cast<uintptr_t>(g.mask) % 4 == 0 && g.mpitch % 4 == 0;
    // rows past H (last band) read row H - 1 again; their bits are dropped
    // below.  The row address is kept in scalar registers and the lane's
    // column added as a 32-bit offset, so a row costs one load instruction.
    const uint32_t cu = (uint32_t)c;
    auto row_ptr = [&](int k) {
        return global_ptr<const uint8_t>((uintptr_t)wave_uniform(reinterpret_cast<int64_t>(
                   g.mask + (int64_t)(row0 + min(k, rows - 1)) * g.mpitch))) + cu;
    };
    uint32_t acc[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) acc[k] = 0u;
    if (words) {
#pragma unroll
        for (int k = 0; k < kBand; ++k) {
            const uint32_t w = *reinterpret_cast<const uint32_t*>(row_ptr(k));
            acc[k >> 3] |= nonzero_bytes(w) >> (7 - (k & 7));
        }
    } else {
#pragma unroll
        for (int k = 0; k < kBand; ++k) {
            const uintptr_t a = reinterpret_cast<uintptr_t>(row_ptr(k));
            const uint32_t* wp = global_ptr<const uint32_t>(a & ~(uintptr_t)3);
            const int off = (int)(a & 3);
            // the second word only when the four bytes reach into it (else the
            // first again: its bytes then fall past the lane's columns)
            const uint32_t lo = wp[0];
            const uint32_t hi = wp[off + ncols > 4 ? 1 : 0];
            const uint32_t w = (uint32_t)((((uint64_t)hi << 32) | lo) >> (8 * off));
            acc[k >> 3] |= nonzero_bytes(w) >> (7 - (k & 7));
        }
    }
    // rows past H hold no site; with polarity 1 the sites are the zero bytes
    const uint64_t valid = rows == kBand ? ~0ull : (1ull << rows) - 1ull;
    uint64_t* out = v.bits + (int64_t)b * g.W + c;
#pragma unroll
    for (int x = 0; x < 4; ++x) {
        if (x < ncols) {
            uint64_t m = ((uint64_t)gather_byte(acc, 4, x) << 32) | gather_byte(acc, 0, x);
            out[x] = (g.pol ? ~m : m) & valid;
        }
    }
}

// --------------------------------------------------------------- carry
// Work item bx: kCarryCols columns; each of the kCarrySlices wavefronts owns a
// contiguous slice of bands (images of at most kCarrySmallBands bands: one
// thread per column and no slices, kCarryCols * kCarrySlices columns).  up[b][c] is the last site row in the bands above
// b (the downward sweep's state entering band b), down[b][c] the first site
// row in the bands below b (the upward sweep's state); flag[c] tells whether
// column c holds any site (zero past W up to the list capacity).
// With kCache (single images) a thread whose slice has at most kCarryPer bands
// reads their masks once, into registers, for the slice's summary and both
// sweeps; otherwise (batches, whose images are mostly one band per slice, and
// images taller than kCarryPer * kCarrySlices bands) it reads them again for
// each sweep, with fewer registers.
constexpr int kCarryPer = 16;

template <bool kCache>
__device__ void carry_item(const Img& g, const Views& v, int bx) {
    __shared__ int s_last[kCarrySlices][kCarryCols];
    __shared__ int s_first[kCarrySlices][kCarryCols];
    const int nb = (g.H + kBand - 1) / kBand;
    const int W = g.W;
    if (nb <= kCarrySmallBands) {  // uniform: one thread per column, all bands
        const int c = bx * (kCarryCols * kCarrySlices) + (int)threadIdx.x;
        if (c >= W) {
            if (c < cand_pitch(W)) v.flag[c] = 0;
            return;
        }
        uint64_t m[kCarrySmallBands];
#pragma unroll
        for (int b = 0; b < kCarrySmallBands; ++b)
            m[b] = b < nb ? v.bits[(int64_t)b * W + c] : 0ull;
        int run = -1;
#pragma unroll
        for (int b = 0; b < kCarrySmallBands; ++b) {
            if (b < nb) v.up[(int64_t)b * W + c] = (int16_t)run;
            if (m[b]) run = b * kBand + 63 - __builtin_clzll(m[b]);
        }
        v.flag[c] = run >= 0;
        int run_dn = kNoBelow;
#pragma unroll
        for (int b = kCarrySmallBands - 1; b >= 0; --b) {
            if (b < nb) v.down[(int64_t)b * W + c] = (int16_t)run_dn;
            if (m[b]) run_dn = b * kBand + __builtin_ctzll(m[b]);
        }
        return;
    }
    const int lane = threadIdx.x % kCarryCols;
    const int s = threadIdx.x / kCarryCols;
    const int c = bx * kCarryCols + lane;
    const int b0 = (int)((int64_t)nb * s / kCarrySlices);
    const int b1 = (int)((int64_t)nb * (s + 1) / kCarrySlices);
    if (kCache && nb <= kCarryPer * kCarrySlices) {  // uniform: every slice fits
        const int cnt = b1 - b0;
        uint64_t m[kCarryPer];
#pragma unroll
        for (int k = 0; k < kCarryPer; ++k) {
            m[k] = 0;
            if (k < cnt && c < W) m[k] = v.bits[(int64_t)(b0 + k) * W + c];
        }
        int last = -1, first = kNoBelow;
#pragma unroll
        for (int k = 0; k < kCarryPer; ++k) {
            if (m[k]) {  // zero past the slice
                if (first == kNoBelow) first = (b0 + k) * kBand + __builtin_ctzll(m[k]);
                last = (b0 + k) * kBand + 63 - __builtin_clzll(m[k]);
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
#pragma unroll
        for (int k = 0; k < kCarryPer; ++k) {
            if (k < cnt) v.up[(int64_t)(b0 + k) * W + c] = (int16_t)run;
            if (m[k]) run = (b0 + k) * kBand + 63 - __builtin_clzll(m[k]);
        }
        if (s == kCarrySlices - 1) v.flag[c] = run >= 0;
#pragma unroll
        for (int k = kCarryPer - 1; k >= 0; --k) {
            if (k < cnt) v.down[(int64_t)(b0 + k) * W + c] = (int16_t)run_dn;
            if (m[k]) run_dn = (b0 + k) * kBand + __builtin_ctzll(m[k]);
        }
        return;
    }
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
        v.meta[2] = 0;  // the segment search's count of claimed work items
    }
}

// ------------------------------------------------------------- nearest
// Work item (band b, block qb of kNearCols listed columns) of one wavefront:
// lane q handles listed column q and writes rc[i][q] for the band's rows.  A
// bottom-up walk of the band's site bits gives, per row, the nearest site at
// or below it (the carry from below past the band's last site); the top-down
// walk that writes the rows keeps the nearest site at or above (the carry from
// above before the band's first site).  Row i takes the upper site a rather
// than the lower one d when i - a <= d - i -- the upper site wins at equal
// distance -- i.e. when 2i <= a + d.  A missing side is a site kFar rows away,
// farther than any real one.  Items past the device-side count n do nothing,
// and so does every item of an image with at most kSparseMaxN listed columns:
// the one-wavefront row form that takes it works its site rows out itself.
constexpr int kFar = 1 << 20;

__device__ __forceinline__ void near_item(const Img& g, const Views& v, int item, int qblocks,
                                          int lane) {
    const int n = wave_uniform(v.meta[0]);
    if (n <= kSparseMaxN) return;  // the one-wavefront row form works its rows out itself
    const int pitch = wave_uniform(v.meta[1]);
    const int b = item / qblocks;
    const int q = (item - b * qblocks) * kNearCols + lane;
    if (q >= n) return;
    const int c = v.cols[q];
    const int64_t bc = (int64_t)b * g.W + c;
    const uint64_t m = v.bits[bc];
    const int up = v.up[bc];
    const int down = v.down[bc];
    const int row0 = b * kBand;
    const int rows = min(kBand, g.H - row0);
    int a = up < 0 ? -kFar : up;
    // quarters of 16 rows: the bottom-up walk of a quarter starts from the
    // nearest site below it (the next set bit, else the carry from below)
#pragma unroll
    for (int h = 0; h < kBand / 16; ++h) {
        if (16 * h < rows) {
            const uint64_t after = h == 3 ? 0ull : m >> (16 * h + 16);
            int d = after ? row0 + 16 * h + 16 + __builtin_ctzll(after)
                          : (down == kNoBelow ? kFar : down);
            const uint32_t mq = (uint32_t)(m >> (16 * h)) & 0xFFFFu;
            int dn[16];
#pragma unroll
            for (int r = 15; r >= 0; --r) {
                d = ((mq >> r) & 1u) ? row0 + 16 * h + r : d;
                dn[r] = d;
            }
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int i = row0 + 16 * h + r;
                if (16 * h + r < rows) {
                    a = ((mq >> r) & 1u) ? i : a;
                    int16_t* row = v.rc + (int64_t)i * pitch;
                    row[q] = (int16_t)(2 * i <= a + dn[r] ? a : dn[r]);
                }
            }
        }
    }
}

// ------------------------------------------------------ single image
__device__ __forceinline__ int wave_id() {
    return __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
}

__global__ __launch_bounds__(64 * kColWaves) void k_bits(Img g, int items) {
    const int item = blockIdx.x * kColWaves + wave_id();
    if (item < items) bits_item(g, views_of(g), item, threadIdx.x & 63);
}
__global__ __launch_bounds__(kCarryCols* kCarrySlices) void k_carry(Img g) {
    const Views v = views_of(g);
    carry_item<true>(g, v, blockIdx.x);
}
__global__ __launch_bounds__(1024) void k_compact(Img g) {
    const Views v = views_of(g);
    compact_item(g, v);
}
// persistent grid of wavefronts over the items (their useful number depends on n)
__global__ __launch_bounds__(64 * kColWaves) void k_near(Img g) {
    const Views v = views_of(g);
    // items per band from the device-side count of listed columns
    const int qblocks = (wave_uniform(v.meta[0]) + kNearCols - 1) / kNearCols;
    const int items = ((g.H + kBand - 1) / kBand) * qblocks;
    for (int item = blockIdx.x * kColWaves + wave_id(); item < items;
         item += gridDim.x * kColWaves)
        near_item(g, v, item, qblocks, threadIdx.x & 63);
}

// --------------------------------------------------------------- batch
// Persistent grids over all work items of a phase in the batch.  The band-bit
// and nearest-row passes take one item per wavefront and find its image by a
// binary search over the phase's prefix sums, uniform across the wavefront;
// the carry pass takes one item per workgroup, looked up by thread 0.
template <int kPh>
__device__ __forceinline__ int batch_lookup(const BatchTable& t, int item) {
    __shared__ int s_img;
    __syncthreads();
    if (threadIdx.x == 0) s_img = batch_image_of(t, kPh, item);
    __syncthreads();
    return s_img;
}

__global__ __launch_bounds__(64 * kColWaves) void k_bits_batch(BatchTable t, int total) {
    for (int item = blockIdx.x * kColWaves + wave_id(); item < total;
         item += gridDim.x * kColWaves) {
        const int im = batch_image_of(t, kPhBits, item);
        const Img g = batch_img(t, im);
        bits_item(g, views_of(g), item - wave_uniform(t.prefix[kPhBits][im]), threadIdx.x & 63);
    }
}
__global__ __launch_bounds__(kCarryCols* kCarrySlices) void k_carry_batch(BatchTable t, int total) {
    for (int item = blockIdx.x; item < total; item += gridDim.x) {
        const int im = batch_lookup<kPhCarry>(t, item);
        const Img g = batch_img(t, im);
        carry_item<false>(g, views_of(g), item - t.prefix[kPhCarry][im]);
    }
}
__global__ __launch_bounds__(1024) void k_compact_batch(BatchTable t, int total) {
    for (int im = blockIdx.x; im < total; im += gridDim.x) {
        const Img g = batch_img(t, im);
        compact_item(g, views_of(g));
    }
}
__global__ __launch_bounds__(64 * kColWaves) void k_near_batch(BatchTable t, int total) {
    for (int item = blockIdx.x * kColWaves + wave_id(); item < total;
         item += gridDim.x * kColWaves) {
        const int im = batch_image_of(t, kPhNear, item);
        const Img g = batch_img(t, im);
        near_item(g, views_of(g), item - wave_uniform(t.prefix[kPhNear][im]),
                  (g.W + kNearCols - 1) / kNearCols,
                  threadIdx.x & 63);
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
    const int bits = items_bits(g.H, g.W);
    EDT_LAUNCH_AS("k_band_bits", k_bits, dim3((bits + kColWaves - 1) / kColWaves),
                  dim3(64 * kColWaves), 0, stream, g, bits);
    EDT_LAUNCH_AS("k_band_carry", k_carry, dim3(items_carry(g.H, g.W)),
                  dim3(kCarryCols * kCarrySlices), 0, stream, g);
    EDT_LAUNCH_AS("k_col_compact", k_compact, dim3(1), dim3(1024), 0, stream, g);
    // enough workgroups for a dense image, few enough that idle ones are cheap
    const int near = (items_near(g.H, g.W) + kColWaves - 1) / kColWaves;
    EDT_LAUNCH_AS("k_nearest_row", k_near, dim3(near < 2048 ? near : 2048), dim3(64 * kColWaves),
                  0, stream, g);
    return launch_status();
}

hipError_t launch_column_pass_batch(const BatchTable& t, const int* totals, hipStream_t stream) {
    const int cap = 16 * device_cus();
    auto grid = [&](int total) { return dim3((unsigned)(total < cap ? total : cap)); };
    auto wave_grid = [&](int total) { return grid((total + kColWaves - 1) / kColWaves); };
    EDT_LAUNCH_AS("k_band_bits", k_bits_batch, wave_grid(totals[kPhBits]), dim3(64 * kColWaves),
                  0, stream, t, totals[kPhBits]);
    EDT_LAUNCH_AS("k_band_carry", k_carry_batch, grid(totals[kPhCarry]),
                  dim3(kCarryCols * kCarrySlices), 0, stream, t, totals[kPhCarry]);
    EDT_LAUNCH_AS("k_col_compact", k_compact_batch, grid(totals[kPhCompact]), dim3(1024), 0,
                  stream, t, totals[kPhCompact]);
    if (totals[kPhNear] > 0)  // none when every image takes the lane pass
        EDT_LAUNCH_AS("k_nearest_row", k_near_batch, wave_grid(totals[kPhNear]),
                      dim3(64 * kColWaves), 0, stream, t, totals[kPhNear]);
    return launch_status();
}

}  // namespace edt
