// Batch images processed as their transposes.  Section 3.2.1 of Strutz
// (arXiv 2106.03503) notes that the column and row passes may run in either
// order and that the cheaper order depends on the image's aspect ratio.  Here
// the row pass is the one-lane-per-row scan, whose serial chain per lane is a
// row's number of candidate columns and whose parallel work is the number of
// rows: a wide image processed as its transpose puts its longer side on the
// parallel axis.  The transposed mask is written into the image's workspace
// before the transform and the transposed outputs are copied back after it,
// each through LDS tiles of kTrTile x kTrTile pixels so that both sides of a
// copy read and write row segments.  A pixel's feature is written as the
// original index by the row pass itself, so the copy back moves values only.
#include "edt_internal.h"

namespace edt {
namespace {

constexpr int TT = kTrTile;
constexpr int kTrThreads = 256;  // four threads per tile row, sixteen pixels each
static_assert(kTrThreads * 16 == TT * TT, "one tile per workgroup pass");

// Tile `k` of an image whose original sides are Ho x Wo: its first original
// row and column.
__device__ __forceinline__ void tile_at(int k, int Wo, int* r0, int* c0) {
    const int tcols = (Wo + TT - 1) / TT;
    *r0 = (k / tcols) * TT;
    *c0 = (k % tcols) * TT;
}

// Masks in: tile (r0, c0) of the caller's mask to the transposed mask in the
// workspace (transposed row = original column).  Sixteen threads take one
// 64-byte row of the tile, four bytes each, so a wavefront reads four rows'
// contiguous runs; writes go out as 16-byte pieces, sixteen threads per
// transposed row.
__global__ __launch_bounds__(kTrThreads) void k_tr_in(BatchTable tb, int total) {
    __shared__ uint8_t tile[TT][TT + 4];
    __shared__ int s_img;
    const int t = threadIdx.x;
    for (int item = blockIdx.x; item < total; item += gridDim.x) {
        __syncthreads();  // the previous tile's LDS reads are done
        if (t == 0) s_img = batch_image_of(tb, kPhTrIn, item);
        __syncthreads();
        const int im = s_img;
        const BatchImage b = tb.img[im];
        const int Ho = b.W, Wo = b.H;  // the table holds the transposed sides
        int r0, c0;
        tile_at(item - tb.prefix[kPhTrIn][im], Wo, &r0, &c0);
        const uint8_t* src = global_ptr<const uint8_t>(tb.mask_base + (uintptr_t)b.mask_off);
        const TrLayout L = tr_layout(b.H, b.W);
        uint8_t* dst = global_ptr<uint8_t>(tb.ws_base + (uintptr_t)b.ws_off + L.mask);
#pragma unroll
        for (int pass = 0; pass < 4; ++pass) {  // rows r, four bytes at column c
            const int r = pass * 16 + (t >> 4), c = (t & 15) * 4;
            const uint8_t* row = src + (int64_t)(r0 + r) * b.mpitch + c0 + c;
            uint32_t w = 0;
            if (r0 + r < Ho) {
                if (c0 + c + 4 <= Wo && (reinterpret_cast<uintptr_t>(row) & 3) == 0) {
                    w = *reinterpret_cast<const uint32_t*>(row);
                } else {
                    for (int q = 0; q < 4 && c0 + c + q < Wo; ++q) w |= (uint32_t)row[q] << (8 * q);
                }
            }
            *reinterpret_cast<uint32_t*>(&tile[r][c]) = w;
        }
        __syncthreads();
        {  // transposed row c0 + c, sixteen bytes: original rows r0 + r .. + 15
            const int c = t >> 2, r = (t & 3) * 16;
            if (c0 + c < Wo) {
                uint8_t* out = dst + (int64_t)(c0 + c) * L.mpitch + r0 + r;
                if (r0 + r + 16 <= Ho) {  // whole and 16-byte aligned
                    uint32_t w[4];
#pragma unroll
                    for (int k = 0; k < 4; ++k)
                        w[k] = (uint32_t)tile[r + 4 * k][c] | ((uint32_t)tile[r + 4 * k + 1][c] << 8) |
                               ((uint32_t)tile[r + 4 * k + 2][c] << 16) |
                               ((uint32_t)tile[r + 4 * k + 3][c] << 24);
                    *reinterpret_cast<uint4*>(out) = make_uint4(w[0], w[1], w[2], w[3]);
                } else {
                    for (int q = 0; r0 + r + q < Ho && q < 16; ++q) out[q] = tile[r + q][c];
                }
            }
        }
    }
}

// Outputs back: tile (r0, c0) of the caller's distance and feature outputs
// from the transposed outputs in the workspace.  Sixteen threads take one
// 256-byte row of the tile (four values each) on both sides, so a wavefront
// reads and writes four rows' contiguous runs.
__global__ __launch_bounds__(kTrThreads) void k_tr_out(BatchTable tb, int total) {
    __shared__ int32_t tile[TT][TT + 1];
    __shared__ int s_img;
    const int t = threadIdx.x;
    for (int item = blockIdx.x; item < total; item += gridDim.x) {
        __syncthreads();
        if (t == 0) s_img = batch_image_of(tb, kPhTrOut, item);
        __syncthreads();
        const int im = s_img;
        const BatchImage b = tb.img[im];
        const int Ho = b.W, Wo = b.H;
        int r0, c0;
        tile_at(item - tb.prefix[kPhTrOut][im], Wo, &r0, &c0);
        const TrLayout L = tr_layout(b.H, b.W);
        const uintptr_t ws = tb.ws_base + (uintptr_t)b.ws_off;
        for (int which = 0; which < 2; ++which) {
            const bool want = which == 0 ? (b.outs & kOutDist) : (b.outs & kOutFeat);
            if (!want) continue;  // the same in every thread
            const int32_t* src = global_ptr<const int32_t>(ws + (which == 0 ? L.dist : L.feat));
            int32_t* dst = which == 0
                               ? global_ptr<int32_t>(tb.dist_base + 4 * (uintptr_t)b.dist_off)
                               : global_ptr<int32_t>(tb.feat_base + 4 * (uintptr_t)b.feat_off);
            __syncthreads();  // the previous output's LDS reads are done
#pragma unroll
            for (int pass = 0; pass < 4; ++pass) {  // transposed row c, values r .. r + 3
                const int c = pass * 16 + (t >> 4), r = (t & 15) * 4;
                if (c0 + c < Wo) {
                    const int32_t* row = src + (int64_t)(c0 + c) * L.opitch + r0 + r;
                    if (r0 + r + 4 <= Ho) {  // 16-byte aligned: pitch and r0 + r multiples of 4
                        const int4 x = *reinterpret_cast<const int4*>(row);
                        tile[c][r] = x.x;
                        tile[c][r + 1] = x.y;
                        tile[c][r + 2] = x.z;
                        tile[c][r + 3] = x.w;
                    } else {
                        for (int q = 0; r0 + r + q < Ho && q < 4; ++q) tile[c][r + q] = row[q];
                    }
                }
            }
            __syncthreads();
#pragma unroll
            for (int pass = 0; pass < 4; ++pass) {  // original row r, values c .. c + 3
                const int r = pass * 16 + (t >> 4), c = (t & 15) * 4;
                if (r0 + r < Ho) {
                    int32_t* row = dst + (int64_t)(r0 + r) * b.opitch + c0 + c;
                    if (c0 + c + 4 <= Wo && (reinterpret_cast<uintptr_t>(row) & 15) == 0) {
                        typedef int v4i __attribute__((ext_vector_type(4)));
                        const v4i x = {tile[c][r], tile[c + 1][r], tile[c + 2][r], tile[c + 3][r]};
                        __builtin_nontemporal_store(x, reinterpret_cast<v4i*>(row));
                    } else {
                        for (int q = 0; q < 4 && c0 + c + q < Wo; ++q)
                            __builtin_nontemporal_store(tile[c + q][r], row + q);
                    }
                }
            }
        }
    }
}

template <typename K>
int blocks_per_cu(K kernel) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kernel, kTrThreads, 0) != hipSuccess ||
        nb < 1)
        nb = 1;
    return nb;
}

}  // namespace

hipError_t launch_transpose_in(const BatchTable& t, int total, hipStream_t stream) {
    static int per_cu = 0;
    if (total < 1) return hipSuccess;
    if (per_cu == 0) per_cu = blocks_per_cu(k_tr_in);
    const int grid = min(total, per_cu * device_cus());
    EDT_LAUNCH(k_tr_in, dim3(grid), dim3(kTrThreads), 0, stream, t, total);
    return launch_status();
}

hipError_t launch_transpose_out(const BatchTable& t, int total, hipStream_t stream) {
    static int per_cu = 0;
    if (total < 1) return hipSuccess;
    if (per_cu == 0) per_cu = blocks_per_cu(k_tr_out);
    const int grid = min(total, per_cu * device_cus());
    EDT_LAUNCH(k_tr_out, dim3(grid), dim3(kTrThreads), 0, stream, t, total);
    return launch_status();
}

}  // namespace edt
