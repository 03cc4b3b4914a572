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

// High bit of each byte of w set iff that byte is nonzero.
__device__ __forceinline__ uint32_t nonzero_bytes(uint32_t w) {
    return (((w & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | w) & 0x80808080u;
}

// Site bits of every band column: bit r of bits[b][c] is set when pixel
// (b*kBand + r, c) is a site.  kMode 16: 16 columns per lane, 16-byte loads;
// kMode 4: 4 columns per lane, 4-byte loads; kMode 1: 4 columns, byte loads.
template <int kMode>
__global__ __launch_bounds__(kColThreads) void k_band_bits(
    const uint8_t* __restrict__ mask, int H, int W, int64_t pitch, int polarity,
    uint64_t* __restrict__ bits) {
    constexpr int CPL = kMode == 16 ? 16 : 4;
    const int c = (blockIdx.x * kColThreads + threadIdx.x) * CPL;
    if (c >= W) return;
    const int b = blockIdx.y;
    const int row0 = b * kBand;
    const int rows = min(kBand, H - row0);
    const int ncols = min(CPL, W - c);
    const uint8_t* p = mask + (int64_t)row0 * pitch + c;
    uint32_t lo[CPL], hi[CPL];
#pragma unroll
    for (int x = 0; x < CPL; ++x) lo[x] = hi[x] = 0u;
    if (kMode != 1 && ncols == CPL && rows == kBand) {
        // whole band, whole lane: no per-row guards, 16 rows of loads in flight
        const uint32_t flip = polarity ? 0x80808080u : 0u;
#pragma unroll
        for (int r0 = 0; r0 < kBand; r0 += 16) {
            uint32_t w[16][CPL / 4];
#pragma unroll
            for (int k = 0; k < 16; ++k) {
                const uint8_t* q = p + (int64_t)(r0 + k) * pitch;
                if constexpr (kMode == 16) {
                    const uint4 v = *reinterpret_cast<const uint4*>(q);
                    w[k][0] = v.x;
                    w[k][1] = v.y;
                    w[k][2] = v.z;
                    w[k][3] = v.w;
                } else {
                    w[k][0] = *reinterpret_cast<const uint32_t*>(q);
                }
            }
#pragma unroll
            for (int k = 0; k < 16; ++k) {
                const int r = r0 + k;
#pragma unroll
                for (int g = 0; g < CPL / 4; ++g) {
                    const uint32_t s = nonzero_bytes(w[k][g]) ^ flip;
#pragma unroll
                    for (int x = 0; x < 4; ++x) {
                        const uint32_t bit = (s >> (8 * x + 7)) & 1u;
                        if (r < 32)
                            lo[4 * g + x] |= bit << r;
                        else
                            hi[4 * g + x] |= bit << (r - 32);
                    }
                }
            }
        }
    } else {
        const uint32_t pol = (uint32_t)polarity;
        for (int r = 0; r < rows; ++r) {
            const uint8_t* q = p + (int64_t)r * pitch;
            for (int x = 0; x < ncols; ++x) {
                const uint32_t bit = (uint32_t)(q[x] != 0) ^ pol;
                if (r < 32)
                    lo[x] |= bit << r;
                else
                    hi[x] |= bit << (r - 32);
            }
        }
    }
    uint64_t* o = bits + (int64_t)b * W + c;
#pragma unroll
    for (int x = 0; x < CPL; ++x)
        if (x < ncols) o[x] = ((uint64_t)hi[x] << 32) | lo[x];
}

// Site bits, wide form for 16-byte aligned masks: a workgroup covers one band
// and 1024 columns; each of its four wavefronts loads 16 rows of the band at
// once (16 bytes = 16 columns per lane and row) and builds 16-bit partial
// column masks, which are joined through LDS into the 64-bit band masks.
__global__ __launch_bounds__(kColThreads) void k_band_bits_wide(
    const uint8_t* __restrict__ mask, int H, int W, int64_t pitch, int polarity,
    uint64_t* __restrict__ bits) {
    __shared__ uint16_t s_part[4][16][65];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int cbase = blockIdx.x * 1024;
    const int c = cbase + lane * 16;
    const int b = blockIdx.y;
    const int rw0 = b * kBand + wave * 16;  // first row of this wavefront
    const int rows = max(0, min(16, H - rw0));
    const int ncols = max(0, min(16, W - c));
    uint32_t part[16];
#pragma unroll
    for (int x = 0; x < 16; ++x) part[x] = 0u;
    const uint8_t* p = mask + (int64_t)rw0 * pitch + c;
    if (ncols == 16 && rows == 16) {
        const uint32_t flip = polarity ? 0x80808080u : 0u;
        uint4 v[16];
#pragma unroll
        for (int k = 0; k < 16; ++k) v[k] = *reinterpret_cast<const uint4*>(p + (int64_t)k * pitch);
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            const uint32_t w4[4] = {v[k].x, v[k].y, v[k].z, v[k].w};
#pragma unroll
            for (int g = 0; g < 4; ++g) {
                const uint32_t s = nonzero_bytes(w4[g]) ^ flip;
#pragma unroll
                for (int x = 0; x < 4; ++x) part[4 * g + x] |= ((s >> (8 * x + 7)) & 1u) << k;
            }
        }
    } else if (ncols > 0) {
        const uint32_t pol = (uint32_t)polarity;
        for (int k = 0; k < rows; ++k) {
            const uint8_t* q = p + (int64_t)k * pitch;
            for (int x = 0; x < ncols; ++x) part[x] |= ((uint32_t)(q[x] != 0) ^ pol) << k;
        }
    }
#pragma unroll
    for (int x = 0; x < 16; ++x) s_part[wave][x][lane] = (uint16_t)part[x];
    __syncthreads();
    // thread t joins the four partial masks of columns cbase + 4t .. 4t+3
#pragma unroll
    for (int y = 0; y < 4; ++y) {
        const int cl = threadIdx.x * 4 + y;
        const int cc = cbase + cl;
        if (cc < W) {
            const int ln = cl >> 4, x = cl & 15;
            bits[(int64_t)b * W + cc] = (uint64_t)s_part[0][x][ln] |
                                        ((uint64_t)s_part[1][x][ln] << 16) |
                                        ((uint64_t)s_part[2][x][ln] << 32) |
                                        ((uint64_t)s_part[3][x][ln] << 48);
        }
    }
}

// Carries across band boundaries.  A workgroup owns kCarryCols columns; each
// of its kCarrySlices wavefronts owns a contiguous slice of bands.  up[b][c]
// is the last site row in the bands above b (the downward sweep's state
// entering band b) and down[b][c] the first site row in the bands below b (the
// upward sweep's state); flag[c] (one byte, zero past W up to the list
// capacity) tells whether column c holds any site.
__global__ __launch_bounds__(kCarryCols* kCarrySlices) void k_band_carry(
    const uint64_t* __restrict__ bits, int nb, int W, int16_t* __restrict__ up,
    int16_t* __restrict__ down, uint8_t* __restrict__ flag) {
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
    if (c >= W) {
        if (s == 0 && c < cand_pitch(W)) flag[c] = 0;
        return;
    }
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

// List of the columns holding a site, in increasing order (one workgroup,
// 32 column flags per thread).  meta[0] = their number n, meta[1] = the row
// pitch of the compact rows.
__global__ __launch_bounds__(1024) void k_col_compact(const uint8_t* __restrict__ flag,
                                                      int W, int16_t* __restrict__ cols,
                                                      int32_t* __restrict__ meta) {
    __shared__ int s_wave[16];
    const int t = threadIdx.x;
    const int c0 = t * 32;
    uint32_t bitsv = 0;  // bit x: column c0 + x holds a site
    if (c0 < cand_pitch(W)) {
        const uint4* f = reinterpret_cast<const uint4*>(flag + c0);
        const uint4 a = f[0], b = f[1];
        const uint32_t wv[8] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
#pragma unroll
        for (int g = 0; g < 8; ++g) {
            const uint32_t s = nonzero_bytes(wv[g]);
#pragma unroll
            for (int x = 0; x < 4; ++x) bitsv |= ((s >> (8 * x + 7)) & 1u) << (4 * g + x);
        }
    }
    const int cnt = __popc(bitsv);
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
    while (bitsv) {
        const int x = __ffs(bitsv) - 1;
        bitsv &= bitsv - 1;
        cols[pos++] = (int16_t)(c0 + x);
    }
    if (t == 0) {
        meta[0] = total;
        meta[1] = cand_pitch(total > 0 ? total : 1);
    }
}

// Nearest site row of every pixel of the listed columns: work item (b, block)
// covers band b and 256 consecutive listed columns; thread q of the item
// handles listed column q and writes rc[i][q] for the band's rows.  The last
// site at or above the pixel (inside the band, else the carry from above)
// competes with the first site at or below it (inside the band, else the
// carry from below); the upper one wins at equal distance.  The grid is fixed
// and loops over the items, whose number depends on the device-side count n.
__global__ __launch_bounds__(kColThreads) void k_nearest_row(
    const uint64_t* __restrict__ bits, const int16_t* __restrict__ up,
    const int16_t* __restrict__ down, const int16_t* __restrict__ cols,
    const int32_t* __restrict__ meta, int H, int W, int nb, int16_t* __restrict__ rc) {
    const int n = meta[0];
    const int pitch = meta[1];
    const int qblocks = (n + kColThreads - 1) / kColThreads;
    const int items = qblocks * nb;
    for (int item = blockIdx.x; item < items; item += gridDim.x) {
        const int b = item / qblocks;
        const int q = (item - b * qblocks) * kColThreads + threadIdx.x;
        if (q >= n) continue;
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
}

}  // namespace

hipError_t launch_column_pass(const uint8_t* mask, int H, int W, int64_t pitch,
                              int polarity, uint8_t* ws, const Layout& L,
                              hipStream_t stream) {
    uint64_t* bits = reinterpret_cast<uint64_t*>(ws + L.bits);
    int16_t* up = reinterpret_cast<int16_t*>(ws + L.up);
    int16_t* down = reinterpret_cast<int16_t*>(ws + L.down);
    uint8_t* flag = ws + L.flag;
    int16_t* cols = reinterpret_cast<int16_t*>(ws + L.cols);
    int32_t* meta = reinterpret_cast<int32_t*>(ws + L.meta);
    int16_t* rc = reinterpret_cast<int16_t*>(ws + L.rc);
    const uintptr_t a = reinterpret_cast<uintptr_t>(mask);
    if (a % 16 == 0 && pitch % 16 == 0) {
        const dim3 g((W + 1023) / 1024, L.nb);
        EDT_LAUNCH_AS("k_band_bits", k_band_bits_wide, g, dim3(kColThreads), 0, stream, mask,
                      H, W, pitch, polarity, bits);
    } else if (a % 4 == 0 && pitch % 4 == 0) {
        const dim3 g((W + 4 * kColThreads - 1) / (4 * kColThreads), L.nb);
        EDT_LAUNCH_AS("k_band_bits", k_band_bits<4>, g, dim3(kColThreads), 0, stream, mask, H,
                      W, pitch, polarity, bits);
    } else {
        const dim3 g((W + 4 * kColThreads - 1) / (4 * kColThreads), L.nb);
        EDT_LAUNCH_AS("k_band_bits", k_band_bits<1>, g, dim3(kColThreads), 0, stream, mask, H,
                      W, pitch, polarity, bits);
    }
    EDT_LAUNCH(k_band_carry, dim3((W + kCarryCols - 1) / kCarryCols),
               dim3(kCarryCols * kCarrySlices), 0, stream, bits, L.nb, W, up, down, flag);
    EDT_LAUNCH(k_col_compact, dim3(1), dim3(1024), 0, stream, flag, W, cols, meta);
    // enough workgroups for a dense image, few enough that idle ones are cheap
    const int items_max = L.nb * ((W + kColThreads - 1) / kColThreads);
    const int grid = items_max < 2048 ? items_max : 2048;
    EDT_LAUNCH(k_nearest_row, dim3(grid), dim3(kColThreads), 0, stream, bits, up, down, cols,
               meta, H, W, L.nb, rc);
    return hipGetLastError();
}

}  // namespace edt
