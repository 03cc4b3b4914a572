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
// Band carries: columns per workgroup and band slices (one wavefront each).
constexpr int kCarryCols = 64;
constexpr int kCarrySlices = 16;

// Row pass: candidate slots per lane (also pixels per lane in the dense fill).
constexpr int kRowS = 16;
// One-wavefront row pass for rows with at most kSparseMaxN candidates.
constexpr int kSparseLanes = 64;
constexpr int kSparseMaxN = kSparseLanes * kRowS;
// Widest row whose whole candidate list and envelope live in LDS.
constexpr int kLdsMaxW = 1024 * kRowS;
// Workgroups (and global-memory row slots) of the row pass for wider rows.
constexpr int kWideSlots = 512;

__host__ __device__ inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Candidate-list capacity per row (multiple of 32 so every lane's chunk of
// 16 or 32 slots is whole).
__host__ __device__ inline int cand_pitch(int W) { return (int)align_up((size_t)W, 32); }
// Candidate capacity of one global row slot (1024 lanes x 2*kRowS slots),
// used for rows wider than kLdsMaxW, and the slot's size in bytes
// (4-byte candidates, then 2-byte starts).
constexpr int kWideCap = 1024 * 2 * kRowS;
__host__ __device__ inline size_t wide_slot_bytes(int /*W*/) {
    return align_up((size_t)kWideCap * 6, 256);
}

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
    size_t slots;      // row slots for rows wider than kLdsMaxW
    size_t total;
};

inline Layout layout_for(int H, int W) {
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
    L.slots = off;
    if (W > kLdsMaxW) off = align_up(off + (size_t)kWideSlots * wide_slot_bytes(W), 256);
    L.total = off;
    return L;
}

// Kernel timing (edt_profile_begin / edt_profile_end): a token from
// prof_begin (negative when timing is off) is closed by prof_end.
int prof_begin(const char* name, hipStream_t stream);
void prof_end(int token, hipStream_t stream);

// Launch a kernel on a stream, bracketed by timing events (recorded under
// `name`) when enabled.
#define EDT_LAUNCH_AS(name, kernel, grid, block, lds, stream, ...)           \
    do {                                                                     \
        const int edt_tok_ = ::edt::prof_begin(name, stream);                \
        hipLaunchKernelGGL(kernel, grid, block, lds, stream, __VA_ARGS__);   \
        ::edt::prof_end(edt_tok_, stream);                                   \
    } while (0)
#define EDT_LAUNCH(kernel, grid, block, lds, stream, ...) \
    EDT_LAUNCH_AS(#kernel, kernel, grid, block, lds, stream, __VA_ARGS__)

// Launchers (enqueue on stream; return the HIP error of the launches).
hipError_t launch_column_pass(const uint8_t* mask, int H, int W, int64_t pitch,
                              int polarity, uint8_t* ws, const Layout& L,
                              hipStream_t stream);
hipError_t launch_row_pass(int H, int W, int32_t* dist, int32_t* feat,
                           int64_t out_pitch, uint8_t* ws, const Layout& L,
                           hipStream_t stream);
hipError_t launch_sqrt(const int32_t* D, float* out, int64_t n, hipStream_t stream);

}  // namespace edt
