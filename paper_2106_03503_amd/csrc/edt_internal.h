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

// Threads per workgroup of the row pass.
constexpr int kRowThreads = 256;
// Widest row whose candidate list and envelope fit the row pass's LDS
// (4 B candidate + 2 B start per column, within 64 KiB per workgroup
// together with the kernel's few static LDS words).
constexpr int kRowLdsMaxW = 10880;
// Workgroups of the row pass (each loops over rows); also the number of
// global-memory row slots used when a row is wider than kRowLdsMaxW.
constexpr int kRowSlots = 1024;

__host__ __device__ inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Bytes of one global row slot (candidate list + envelope starts) for width W.
__host__ __device__ inline size_t row_slot_bytes(int W) { return align_up((size_t)W * 6, 256); }

// Byte offsets of the pieces of one image's workspace.
struct Layout {
    int nb;              // bands of kBand rows
    size_t bits;         // uint64 [nb][W]  site bits of each band column
    size_t up;           // int16  [nb][W]  last site row above the band (-1: none)
    size_t down;         // int16  [nb][W]  first site row below the band (kNoBelow: none)
    size_t rstar;        // int16  [H][W]   nearest site row in the pixel's column (-1: none)
    size_t rowscratch;   // per-slot candidate/start arrays for wide rows
    size_t total;
};

inline Layout layout_for(int H, int W) {
    Layout L;
    L.nb = (H + kBand - 1) / kBand;
    size_t off = 0;
    L.bits = off;
    off = align_up(off + (size_t)L.nb * W * 8, 256);
    L.up = off;
    off = align_up(off + (size_t)L.nb * W * 2, 256);
    L.down = off;
    off = align_up(off + (size_t)L.nb * W * 2, 256);
    L.rstar = off;
    off = align_up(off + (size_t)H * W * 2, 256);
    L.rowscratch = off;
    if (W > kRowLdsMaxW) off = align_up(off + (size_t)kRowSlots * row_slot_bytes(W), 256);
    L.total = off;
    return L;
}

// Kernel timing (edt_profile_begin / edt_profile_end): a token from
// prof_begin (negative when timing is off) is closed by prof_end.
int prof_begin(const char* name, hipStream_t stream);
void prof_end(int token, hipStream_t stream);

// Launch a kernel on a stream, bracketed by timing events when enabled.
#define EDT_LAUNCH(kernel, grid, block, lds, stream, ...)                    \
    do {                                                                     \
        const int edt_tok_ = ::edt::prof_begin(#kernel, stream);             \
        hipLaunchKernelGGL(kernel, grid, block, lds, stream, __VA_ARGS__);   \
        ::edt::prof_end(edt_tok_, stream);                                   \
    } while (0)

// Launchers (enqueue on stream; return the HIP error of the launch).
hipError_t launch_column_pass(const uint8_t* mask, int H, int W, int64_t pitch,
                              int polarity, uint8_t* ws, const Layout& L,
                              hipStream_t stream);
hipError_t launch_row_pass(const int16_t* rstar, int H, int W, int32_t* dist,
                           int32_t* feat, int64_t out_pitch, uint8_t* ws,
                           const Layout& L, hipStream_t stream);
hipError_t launch_sqrt(const int32_t* D, float* out, int64_t n, hipStream_t stream);

}  // namespace edt
