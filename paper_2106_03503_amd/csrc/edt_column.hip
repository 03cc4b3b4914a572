// Vertical pass of the exact EDT (Section 3.1 of Strutz, arXiv 2106.03503):
// for every pixel, the row of the nearest site in its own column, ties going to
// the upper site (the downward sweep keeps its value unless the upward sweep is
// strictly nearer).  The paper sweeps each column down and then up; here the
// column is cut into bands of kBand rows so that thousands of workgroups share
// the work, each band's sites are held as one 64-bit mask per column, and the
// two sweeps become bit scans inside the band plus one carry per band
// boundary (the last site above the band, the first site below it).
//
// Threads own adjacent columns, so every row access of a wavefront is one
// contiguous run of bytes (mask) or int16s (nearest-row output).
#include "edt_internal.h"

namespace edt {
namespace {

constexpr int kColThreads = 256;

__device__ __forceinline__ uint64_t band_site_bits(const uint8_t* __restrict__ col,
                                                   int64_t pitch, int rows,
                                                   int polarity) {
    uint64_t bits = 0;
    for (int r = 0; r < rows; ++r) {
        const uint32_t object = col[(int64_t)r * pitch] != 0;
        bits |= (uint64_t)(object ^ (uint32_t)polarity) << r;
    }
    return bits;
}

// Site bits of every band column: bit r of bits[b][c] is set when pixel
// (b*kBand + r, c) is a site.
__global__ __launch_bounds__(kColThreads) void k_band_bits(
    const uint8_t* __restrict__ mask, int H, int W, int64_t pitch, int polarity,
    uint64_t* __restrict__ bits) {
    const int c = blockIdx.x * kColThreads + threadIdx.x;
    const int b = blockIdx.y;
    if (c >= W) return;
    const int row0 = b * kBand;
    const int rows = min(kBand, H - row0);
    bits[(int64_t)b * W + c] =
        band_site_bits(mask + (int64_t)row0 * pitch + c, pitch, rows, polarity);
}

// Carries across band boundaries, one thread per column: up[b][c] is the last
// site row in bands above b (the downward sweep's state entering the band),
// down[b][c] the first site row in bands below b (the upward sweep's state).
__global__ __launch_bounds__(kColThreads) void k_band_carry(
    const uint64_t* __restrict__ bits, int nb, int W, int16_t* __restrict__ up,
    int16_t* __restrict__ down) {
    const int c = blockIdx.x * kColThreads + threadIdx.x;
    if (c >= W) return;
    int last = -1;
    for (int b = 0; b < nb; ++b) {
        up[(int64_t)b * W + c] = (int16_t)last;
        const uint64_t m = bits[(int64_t)b * W + c];
        if (m) last = b * kBand + 63 - __builtin_clzll(m);
    }
    int first = kNoBelow;
    for (int b = nb - 1; b >= 0; --b) {
        down[(int64_t)b * W + c] = (int16_t)first;
        const uint64_t m = bits[(int64_t)b * W + c];
        if (m) first = b * kBand + __builtin_ctzll(m);
    }
}

// Nearest site row of every pixel of a band column: the last site at or above
// the pixel (inside the band, else the carry from above) against the first
// site at or below it (inside the band, else the carry from below); the upper
// one wins at equal distance.  -1 when the whole column has no site.
__global__ __launch_bounds__(kColThreads) void k_nearest_row(
    const uint64_t* __restrict__ bits, const int16_t* __restrict__ up,
    const int16_t* __restrict__ down, int H, int W, int16_t* __restrict__ rstar) {
    const int c = blockIdx.x * kColThreads + threadIdx.x;
    const int b = blockIdx.y;
    if (c >= W) return;
    const int64_t bc = (int64_t)b * W + c;
    const uint64_t m = bits[bc];
    const int u = up[bc];
    const int d = down[bc];
    const int row0 = b * kBand;
    const int rows = min(kBand, H - row0);
    int16_t* out = rstar + (int64_t)row0 * W + c;
    for (int r = 0; r < rows; ++r) {
        const int i = row0 + r;
        const uint64_t at_or_above = m & (r == 63 ? ~0ull : ((2ull << r) - 1));
        const uint64_t at_or_below = m & (~0ull << r);
        const int a = at_or_above ? row0 + 63 - __builtin_clzll(at_or_above) : u;
        const int bl = at_or_below ? row0 + __builtin_ctzll(at_or_below) : d;
        int best;
        if (a >= 0 && (bl == kNoBelow || i - a <= bl - i))
            best = a;
        else
            best = (bl == kNoBelow) ? -1 : bl;
        out[(int64_t)r * W] = (int16_t)best;
    }
}

}  // namespace

hipError_t launch_column_pass(const uint8_t* mask, int H, int W, int64_t pitch,
                              int polarity, uint8_t* ws, const Layout& L,
                              hipStream_t stream) {
    uint64_t* bits = reinterpret_cast<uint64_t*>(ws + L.bits);
    int16_t* up = reinterpret_cast<int16_t*>(ws + L.up);
    int16_t* down = reinterpret_cast<int16_t*>(ws + L.down);
    int16_t* rstar = reinterpret_cast<int16_t*>(ws + L.rstar);
    const dim3 block(kColThreads);
    const dim3 grid2((W + kColThreads - 1) / kColThreads, L.nb);
    const dim3 grid1((W + kColThreads - 1) / kColThreads);
    EDT_LAUNCH(k_band_bits, grid2, block, 0, stream, mask, H, W, pitch,
                       polarity, bits);
    EDT_LAUNCH(k_band_carry, grid1, block, 0, stream, bits, L.nb, W, up, down);
    EDT_LAUNCH(k_nearest_row, grid2, block, 0, stream, bits, up, down, H, W,
                       rstar);
    return hipGetLastError();
}

}  // namespace edt
