// Horizontal pass with one lane per row, for batches (Section 3.3 of Strutz,
// arXiv 2106.03503: the lower envelope of the parabolas of Eq. eq_parabola,
// built with one left-to-right scan and a stack, then one more pass over the
// row to fill it).
//
// A wavefront takes 64 consecutive rows of one image and every lane runs the
// paper's scan on its own row, so no lane waits for another and there are no
// barriers: the candidate columns are the same for every row, only their site
// rows differ, so all lanes step through the candidates together and differ
// only in how many parabolas they pop.  The order of parabolas and the start
// of a new one are exactly those of the several-lanes-per-row pass: pixels
// compare lexicographically on (D, feature index), and parabola l takes over
// from k at floor((N - [l wins ties]) / (2 (l - k))) + 1 with N from Eq.
// eq_intersection.
//
// Where the stack lives: the top entries in registers and an LDS ring; older
// entries in memory, in blocks of RB entries.  In the batch kernel a work
// item's blocks sit in the image's workspace block-major: block k of the
// item's row r at 32-byte piece k * rows + r, so that a block is one whole
// 32-byte piece of memory and the lanes that move their k-th block together
// write one contiguous run (a piece per lane in each row's own output would
// be written as partial pieces wherever a row does not start on 32 bytes).
// Once every lane has finished, the wavefront fills the rows one by one from
// each row's envelope copied into LDS.  The segment scan of single images
// keeps the unpacked layout: entry e at slot e of its own row of envelopes
// and its start at slot e of the row's list of site rows, which the scan has
// already read there (e never exceeds the index of the candidate scanned).
#include "edt_internal.h"

namespace edt {
namespace {

constexpr int R = kLaneRing;
constexpr int RB = R / 2;  // stack entries per block moved between the ring and memory
static_assert((R & (R - 1)) == 0 && R % RB == 0, "ring slots are taken modulo R with a mask; blocks do not wrap");
static_assert(RB % 8 == 0, "blocks are whole 16-byte pieces of starts");
constexpr int kBlk = 32;  // candidates per load of site rows (64 bytes per lane)

// Stack entries.  Unpacked (the segment scan of single images, W up to
// 16384): the candidate (column << 16 | site row) in a 32-bit word and its
// start (first pixel it owns) in an int16 beside it.  Packed (batch images,
// W <= kLaneMaxW and H <= kLanePackMaxH): column, start and site row in one
// word, so that an entry moves as 4 bytes instead of 6 and the ring as one
// array.
__device__ __forceinline__ uint32_t pk_entry(int col, int start, int row) {
    return ((uint32_t)col << 22) | ((uint32_t)start << 12) | (uint32_t)row;
}
__device__ __forceinline__ int pk_col(uint32_t c) { return (int)(c >> 22); }
__device__ __forceinline__ int pk_start(uint32_t c) { return (int)((c >> 12) & 0x3FFu); }
__device__ __forceinline__ int pk_row(uint32_t c) { return (int)(c & 0xFFFu); }
static_assert(kLaneMaxW <= 1024 && kLanePackMaxH <= 4096,
              "ten bits of column, ten of start (below W), twelve of site row");

// LDS of one wavefront's scan: the top R stack entries of every lane.
template <bool kPk>
struct LaneRing {
    uint32_t c[R][kLaneRows];  // packed candidate (column << 16 | site row)
    int16_t s[R][kLaneRows];   // first pixel it owns
};
template <>
struct LaneRing<true> {
    uint32_t c[R][kLaneRows];  // packed entry
};

// LDS of the batch kernel: the ring while scanning, then one row's whole
// envelope (packed entries) while filling.
union LaneLds {
    LaneRing<true> ring;
    struct {
        uint32_t c[kLaneMaxW];
    } row;
};

typedef int v4i __attribute__((ext_vector_type(4)));

__device__ __forceinline__ void put4(int32_t* __restrict__ p, int j, int W, bool vec, int v0,
                                     int v1, int v2, int v3) {
    if (vec && j + 4 <= W) {
        const v4i v = {v0, v1, v2, v3};
        __builtin_nontemporal_store(v, reinterpret_cast<v4i*>(p + j));
    } else {
        __builtin_nontemporal_store(v0, p + j);
        if (j + 1 < W) __builtin_nontemporal_store(v1, p + j + 1);
        if (j + 2 < W) __builtin_nontemporal_store(v2, p + j + 2);
        if (j + 3 < W) __builtin_nontemporal_store(v3, p + j + 3);
    }
}

// Last index e in [lo, hi) whose packed entry starts at or before j, given
// that entry lo does.
__device__ __forceinline__ int last_at_or_before(const uint32_t* c, int lo, int hi, int j) {
    int a = lo, b = hi - 1;
    while (a < b) {
        const int mid = (a + b + 1) >> 1;
        if (pk_start(c[mid]) <= j)
            a = mid;
        else
            b = mid - 1;
    }
    return a;
}

// Move ring block [b, b + RB) of this lane to memory (the RB words at sc, and
// ranks b.. of rr for the unpacked starts); b is a multiple of RB.
template <bool kPk>
__device__ __forceinline__ void spill_block(int b, uint32_t* sc, int16_t* rr, bool vec,
                                            LaneRing<kPk>& ring, int lane) {
    const int s0 = b & (R - 1);  // a block never wraps round the ring
    uint32_t c[RB];
#pragma unroll
    for (int k = 0; k < RB; ++k) c[k] = ring.c[s0 + k][lane];
    if (vec) {
#pragma unroll
        for (int k = 0; k < RB / 4; ++k) {
            const v4i x = {(int)c[4 * k], (int)c[4 * k + 1], (int)c[4 * k + 2], (int)c[4 * k + 3]};
            *reinterpret_cast<v4i*>(sc + 4 * k) = x;
        }
    } else {
#pragma unroll
        for (int k = 0; k < RB; ++k) sc[k] = c[k];
    }
    if constexpr (!kPk) {
        uint32_t sp[RB / 2];
#pragma unroll
        for (int k = 0; k < RB / 2; ++k)
            sp[k] = (uint32_t)(uint16_t)ring.s[s0 + 2 * k][lane] |
                    ((uint32_t)(uint16_t)ring.s[s0 + 2 * k + 1][lane] << 16);
#pragma unroll
        for (int k = 0; k < RB / 8; ++k)
            *reinterpret_cast<int4*>(rr + b + 8 * k) =
                make_int4((int)sp[4 * k], (int)sp[4 * k + 1], (int)sp[4 * k + 2], (int)sp[4 * k + 3]);
    }
}

// Bring block [b, b + RB) of this lane back from memory (the RB words at sc)
// into the ring.
template <bool kPk>
__device__ __forceinline__ void fill_block(int b, const uint32_t* sc, const int16_t* rr, bool vec,
                                           LaneRing<kPk>& ring, int lane) {
    const int s0 = b & (R - 1);  // a block never wraps round the ring
    uint32_t c[RB];
    if (vec) {
#pragma unroll
        for (int k = 0; k < RB / 4; ++k) {
            const int4 x = *reinterpret_cast<const int4*>(sc + 4 * k);
            c[4 * k] = (uint32_t)x.x;
            c[4 * k + 1] = (uint32_t)x.y;
            c[4 * k + 2] = (uint32_t)x.z;
            c[4 * k + 3] = (uint32_t)x.w;
        }
    } else {
#pragma unroll
        for (int k = 0; k < RB; ++k) c[k] = sc[k];
    }
#pragma unroll
    for (int k = 0; k < RB; ++k) ring.c[s0 + k][lane] = c[k];
    if constexpr (!kPk) {
        uint32_t sp[RB / 2];
#pragma unroll
        for (int k = 0; k < RB / 8; ++k) {
            const int4 x = *reinterpret_cast<const int4*>(rr + b + 8 * k);
            sp[4 * k] = (uint32_t)x.x;
            sp[4 * k + 1] = (uint32_t)x.y;
            sp[4 * k + 2] = (uint32_t)x.z;
            sp[4 * k + 3] = (uint32_t)x.w;
        }
#pragma unroll
        for (int k = 0; k < RB; ++k)
            ring.s[s0 + k][lane] = (int16_t)(sp[k >> 1] >> (16 * (k & 1)));
    }
}

// Site row of a listed column for the lane's row in the batch kernel, worked
// out where it is needed instead of read from a list written by a kernel of
// its own: a work item's 64 rows are one band (kLaneRows == kBand), so the
// column's band bits and the carries above and below the band (the column
// pass's own state) give the nearest site at or above the row and the
// nearest at or below it, and the upper one wins at equal distance, as in the
// nearest-row pass.  The column is the same in every lane, so the three reads
// are scalar loads: through the constant address space, which these arrays
// are while the row pass runs (nothing writes them then).
struct BandRows {
    const uint64_t* bits;  // site bits [band][column] (one word each)
    const int16_t* up;     // [band][column] last site row above the band (-1: none)
    const int16_t* down;   // [band][column] first site row below it (kNoBelow: none)
    int64_t b0;            // the band's first element: band * W
    int row0, r;           // the band's first row and this lane's row in it
    uint64_t amask;        // bits 0..r

    __device__ __forceinline__ int row_of(int c, int i) const {
        constexpr int kFar = 1 << 20;  // a missing side: farther than any site
        typedef const uint64_t __attribute__((address_space(4))) CU64;
        typedef const uint32_t __attribute__((address_space(4))) CU32;
        // the int16 carries are read as the aligned 4-byte word holding them
        // (the arrays start 256-byte aligned; the band's offset may be odd)
        const int64_t k = b0 + __builtin_amdgcn_readfirstlane(c);
        const uint64_t m = *reinterpret_cast<CU64*>(reinterpret_cast<uintptr_t>(bits + k));
        const uint32_t uw = *reinterpret_cast<CU32*>(reinterpret_cast<uintptr_t>(up + (k & ~1ll)));
        const uint32_t dw =
            *reinterpret_cast<CU32*>(reinterpret_cast<uintptr_t>(down + (k & ~1ll)));
        const int u = (int16_t)(uw >> (16 * (k & 1))), dn = (int16_t)(dw >> (16 * (k & 1)));
        const int ua = u < 0 ? -kFar : u, db = dn == kNoBelow ? kFar : dn;
        if (m == 0) return 2 * i <= ua + db ? ua : db;  // no site in the band: the same test in every lane
        const uint64_t above = m & amask, below = m >> r;
        const int a = above ? row0 + 63 - __clzll(above) : ua;
        const int d = below ? i + __builtin_ctzll(below) : db;
        return 2 * i <= a + d ? a : d;
    }
};

// a + b, wrapping: the pop loop also unpacks stale ring slots, whose sums are
// never used but must not overflow
__device__ __forceinline__ int wrap_add(int a, int b) { return (int)((uint32_t)a + (uint32_t)b); }

// Scan of row i (this lane's row): builds the row's envelope as a stack and
// leaves it in memory, block e / RB at sc + (e / RB) ld (and the unpacked
// starts at rank e of rr); returns its size.  The
// top two entries stay in registers and the ranks [base, M) in an LDS ring of
// two blocks of R/2 entries; a full ring moves its older block to memory in one
// piece, and a pop below the ring brings a block back, so the loop touches
// memory in whole 64- and 32-byte pieces and waits for it only when it reads
// the next 32 site rows or, rarely, brings a block back.
// With kPf the site rows of the next 32 candidates are loaded while the
// current ones are scanned (16 more registers: the segment scan of single
// images, whose work items are short, takes it; the batch kernel keeps its
// registers for occupancy).  With kRows the site rows come from br instead of
// the list rr (the batch kernel).
template <bool kPk, bool kPf = false, bool kRows = false>
__device__ __forceinline__ int scan_row(const int i, const int n, const int W,
                                        const int16_t* __restrict__ cols, int16_t* rr,
                                        uint32_t* sc, const int ld, const bool vec,
                                        LaneRing<kPk>& ring, const int lane, const bool tl,
                                        const BandRows br = BandRows{}) {
    int4 pf0, pf1, pf2, pf3;
    if (kPf) {
        pf0 = *reinterpret_cast<const int4*>(rr);
        pf1 = *reinterpret_cast<const int4*>(rr + 8);
        pf2 = *reinterpret_cast<const int4*>(rr + 16);
        pf3 = *reinterpret_cast<const int4*>(rr + 24);
    }
    int M = 0, base = 0;
    int colA = 0, rowA = 0, gA = 0, sA = 0;  // top entry (M - 1)
    int dAs = 0, dAe = 0;  // the top's distances at its start sA and at pixel W - 1
    uint32_t cB = 0;       // entry below it (M - 2)
    int sB = 0;
    for (int q0 = 0; q0 < n; q0 += kBlk) {
        static_assert(kBlk == 32, "four 16-byte loads of site rows per block");
        int4 rv0, rv1, rv2, rv3;
        if (kPf) {
            rv0 = pf0;
            rv1 = pf1;
            rv2 = pf2;
            rv3 = pf3;
            // the next block lies inside the row's list whenever it starts
            // before n (the list's pitch is a multiple of 32), and the scan
            // writes starts only at ranks below the current candidate
            if (q0 + kBlk < n) {
                pf0 = *reinterpret_cast<const int4*>(rr + q0 + kBlk);
                pf1 = *reinterpret_cast<const int4*>(rr + q0 + kBlk + 8);
                pf2 = *reinterpret_cast<const int4*>(rr + q0 + kBlk + 16);
                pf3 = *reinterpret_cast<const int4*>(rr + q0 + kBlk + 24);
            }
        } else if (!kRows) {
            rv0 = *reinterpret_cast<const int4*>(rr + q0);
            rv1 = *reinterpret_cast<const int4*>(rr + q0 + 8);
            rv2 = *reinterpret_cast<const int4*>(rr + q0 + 16);
            rv3 = *reinterpret_cast<const int4*>(rr + q0 + 24);
        } else {
            rv0 = rv1 = rv2 = rv3 = make_int4(0, 0, 0, 0);  // not used
        }
        const int4 cv0 = *reinterpret_cast<const int4*>(cols + q0);
        const int4 cv1 = *reinterpret_cast<const int4*>(cols + q0 + 8);
        const int4 cv2 = *reinterpret_cast<const int4*>(cols + q0 + 16);
        const int4 cv3 = *reinterpret_cast<const int4*>(cols + q0 + 24);
        const int cnt = min(kBlk, n - q0);
        for (int k = 0; k < kBlk / 8; ++k) {
            if (8 * k >= cnt) break;
            const int4 r4 = k == 0 ? rv0 : k == 1 ? rv1 : k == 2 ? rv2 : rv3;
            const int4 c4 = k == 0 ? cv0 : k == 1 ? cv1 : k == 2 ? cv2 : cv3;
            const uint32_t rw[4] = {(uint32_t)r4.x, (uint32_t)r4.y, (uint32_t)r4.z, (uint32_t)r4.w};
            const uint32_t cw[4] = {(uint32_t)c4.x, (uint32_t)c4.y, (uint32_t)c4.z, (uint32_t)c4.w};
#pragma unroll
            for (int u8 = 0; u8 < 8; ++u8) {
                const int u = 8 * k + u8;
                if (u >= cnt) break;
                const int col = (int)((cw[u8 >> 1] >> (16 * (u8 & 1))) & 0xFFFFu);
                const int row = kRows ? br.row_of(col, i)
                                      : (int)((rw[u8 >> 1] >> (16 * (u8 & 1))) & 0xFFFFu);
                const int gC = sqr_c(i - row);
                const int dCe = gC + sqr_c(W - 1 - col);
                // pop every parabola that the new one beats where it starts
                // (the tests over lane values are bitwise, not && and ||:
                // short-circuit evaluation would cost the wavefront a
                // divergent branch per test; and the loop has one exit, the
                // stack size tested with the rest, so that a lane leaving it
                // costs one level of exec-mask bookkeeping, not two)
                for (;;) {
                    const int dC = wrap_add(gC, sqr_c(sA - col));
                    if (!((M > 0) & ((dC < dAs) | ((dC == dAs) & !tl & (row < rowA))))) break;
                    --M;
                    // the entry below becomes the top, and the ring's next
                    // entry the one below it; both are taken without testing
                    // M (the ring index stays in range, and what they give is
                    // read only while M holds them), which spares the
                    // wavefront two divergent branches per pop
                    if constexpr (kPk) {
                        colA = pk_col(cB);
                        rowA = pk_row(cB);
                        sA = pk_start(cB);
                    } else {
                        colA = (int)(cB >> 16);
                        rowA = (int)(cB & 0xFFFFu);
                        sA = sB;
                    }
                    gA = sqr_c(i - rowA);
                    dAs = wrap_add(gA, sqr_c(sA - colA));
                    dAe = wrap_add(gA, sqr_c(W - 1 - colA));
                    const int e = M - 2;
                    if ((M > 1) & (e < base)) {  // below the ring: bring its block back
                        base -= RB;
                        fill_block<kPk>(base, sc + (base / RB) * ld, rr, vec, ring, lane);
                    }
                    cB = ring.c[e & (R - 1)][lane];
                    if constexpr (!kPk) sB = ring.s[e & (R - 1)][lane];
                }
                // a parabola that does not beat the top at the row's last
                // pixel never wins in the row
                if ((M == 0) | (dCe < dAe) | ((dCe == dAe) & !tl & (row < rowA))) {
                    // the start is worked out by every lane that pushes and
                    // zeroed where the stack was empty (its operands are then
                    // stale: nothing in it can fault, and the numerator wraps
                    // rather than overflows)
                    const bool below = M > 0;
                    const uint32_t num = (uint32_t)gC - (uint32_t)gA +
                                         (uint32_t)mul_c(col - colA, col + colA) -
                                         ((!tl & (row < rowA)) ? 1u : 0u);
                    const int s = first_after((int)num, 2 * (col - colA), W) & -(int)below;
                    if constexpr (kPk) {
                        cB = below ? pk_entry(colA, sA, rowA) : cB;
                    } else {
                        cB = below ? ((uint32_t)colA << 16) | (uint32_t)rowA : cB;
                        sB = below ? sA : sB;
                    }
                    if (M - base == R) {  // ring full: its older block goes to memory
                        spill_block<kPk>(base, sc + (base / RB) * ld, rr, vec, ring, lane);
                        base += RB;
                    }
                    if constexpr (kPk) {
                        ring.c[M & (R - 1)][lane] = pk_entry(col, s, row);
                    } else {
                        ring.c[M & (R - 1)][lane] = ((uint32_t)col << 16) | (uint32_t)row;
                        ring.s[M & (R - 1)][lane] = (int16_t)s;
                    }
                    colA = col;
                    rowA = row;
                    gA = gC;
                    sA = s;
                    dAs = gC + sqr_c(s - col);
                    dAe = dCe;
                    ++M;
                }
            }
        }
    }
    // the rest of the stack to memory as whole blocks: the slots past M (up
    // to the next multiple of RB, within the row's list when n is) take
    // stale ring entries that nothing reads
    for (int b = base; b < M; b += RB) spill_block<kPk>(b, sc + (b / RB) * ld, rr, vec, ring, lane);
    return M;
}

// Work item = 64 consecutive rows of one image of the batch: every lane scans
// its own row, then the wavefront fills the rows one after another, each from
// its envelope copied into LDS, four adjacent pixels per lane and store.
__global__ __launch_bounds__(kLaneRows) void k_row_lanes_batch(BatchTable tb) {
    __shared__ LaneLds sh;
    __shared__ int s_m[kLaneRows];
    const int item = blockIdx.x;
    const int im = batch_image_of(tb, kPhLanes, item);
    const Img g = batch_img(tb, im);
    const int lane = threadIdx.x;
    const int i0 = (item - tb.prefix[kPhLanes][im]) * kLaneRows;
    const int rows = min(kLaneRows, g.H - i0);
    const Views v = views_of(g);
    const int n = v.meta[0];
    const int W = g.W;
    static_assert(kLaneRows == kBand, "a work item's rows are one band");
    // this item's envelopes: block k of row i0 + r at word (k rows + r) RB
    uint32_t* stk = reinterpret_cast<uint32_t*>(g.ws + layout_for(g.H, g.W, false).stk) +
                    (int64_t)i0 * cand_pitch(W);
    const bool vec = (!g.dist || reinterpret_cast<uintptr_t>(g.dist) % 16 == 0) &&
                     (!g.feat || reinterpret_cast<uintptr_t>(g.feat) % 16 == 0) &&
                     (g.opitch % 4 == 0);
    if (n > 0 && lane < rows) {
        const int i = i0 + lane;
        BandRows br;
        br.bits = v.bits;
        br.up = v.up;
        br.down = v.down;
        br.b0 = (int64_t)(i0 / kBand) * W;
        br.row0 = i0;
        br.r = lane;
        br.amask = lane == 63 ? ~0ull : (2ull << lane) - 1ull;
        s_m[lane] = scan_row<true, false, true>(i, n, W, v.cols, nullptr, stk + lane * RB,
                                                rows * RB, true, sh.ring, lane, g.tr != 0, br);
    }
    __syncthreads();  // stacks in memory are complete; the ring is free

    // the envelope of row r + 1 is in flight while row r is filled
    constexpr int kPer = kLaneMaxW / kLaneRows;  // entries per lane
    uint32_t pc[kPer];
    auto fetch = [&](int r) {
        const int Mr = n > 0 ? s_m[r] : 0;
        // entry e = lane + 64 k: block e / RB = lane / RB + 8 k
        const uint32_t* sc = stk + (r + (lane / RB) * rows) * RB + (lane & (RB - 1));
        const int step = (kLaneRows / RB) * rows * RB;
#pragma unroll
        for (int k = 0; k < kPer; ++k) {
            const int e = lane + k * kLaneRows;
            if (e < Mr) pc[k] = sc[k * step];
        }
    };
    if (rows > 0) fetch(0);
    for (int r = 0; r < rows; ++r) {
        const int i = i0 + r;
        int32_t* drow = g.dist ? g.dist + (int64_t)i * g.opitch : nullptr;
        int32_t* frow = g.feat ? g.feat + (int64_t)i * g.opitch : nullptr;
        const int M = n > 0 ? s_m[r] : 0;
#pragma unroll
        for (int k = 0; k < kPer; ++k) {
            const int e = lane + k * kLaneRows;
            if (e < M) sh.row.c[e] = pc[k];
        }
        __syncthreads();
        if (r + 1 < rows) fetch(r + 1);
        int e = 0;
        for (int j = 4 * lane; j < W; j += 4 * kLaneRows) {
            int d[4], f[4];
            if (M == 0) {
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    d[q] = INT32_MAX;
                    f[q] = -1;
                }
            } else {
                // owner of pixel j: the last entry starting at or before it,
                // searched from this lane's previous owner (reads past the
                // envelope are clamped to its last entry and their result
                // discarded, so that no read needs a branch of its own)
                int step = 1;
                for (;;) {
                    const int x = e + step;
                    if (!((x < M) & (pk_start(sh.row.c[min(x, M - 1)]) <= j))) break;
                    e = x;
                    step <<= 1;
                }
                e = last_at_or_before(sh.row.c, e, min(M, e + step), j);
                uint32_t c = sh.row.c[e];
                int nst = e + 1 < M ? pk_start(sh.row.c[min(e + 1, M - 1)]) : INT32_MAX;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int jj = j + q;
                    d[q] = 0;
                    f[q] = 0;
                    if (jj < W) {
                        while (jj >= nst) {
                            ++e;
                            c = sh.row.c[e];
                            nst = e + 1 < M ? pk_start(sh.row.c[min(e + 1, M - 1)]) : INT32_MAX;
                        }
                        const int col = pk_col(c), row = pk_row(c);
                        d[q] = sqr_c(i - row) + sqr_c(jj - col);
                        // a transposed image's site (row, col) is the
                        // original pixel (col, row) of an image g.H wide
                        f[q] = g.tr ? mul_c(col, g.H) + row : mul_c(row, W) + col;
                    }
                }
            }
            if (drow) put4(drow, j, W, vec, d[0], d[1], d[2], d[3]);
            if (frow) put4(frow, j, W, vec, f[0], f[1], f[2], f[3]);
        }
        __syncthreads();  // the next row reuses the LDS copy
    }
}

// Segment scan for dense rows of one image: work item (row group, segment y)
// scans the segment's candidates [y L, min(n, (y + 1) L)) of 64 rows, one lane
// per row, leaving each segment's envelope at slots y L + e of the row in
// b.env (starts in the row's list of site rows) and its size in
// b.segm[i][y].  The grid is persistent over the items, whose count depends
// on the device-side number n of listed columns; images with at most
// kSparseMaxN of them are left to the one-wavefront row pass.
template <int L>
__global__ __launch_bounds__(kLaneRows) void k_row_segscan(Img g, SegBufs b) {
    __shared__ LaneRing<false> ring;
    static_assert(L % kSegL == 0 && L % kBlk == 0, "segments of whole 32-candidate blocks");
    const Views v = views_of(g);
    const int n = v.meta[0];
    if (n <= kSparseMaxN) return;
    const int nseg = (n + L - 1) / L;
    const int total = items_lanes(g.H) * nseg;
    const int lane = threadIdx.x;
    const int pitch = v.meta[1];
    for (int item = blockIdx.x; item < total; item += gridDim.x) {
        const int grp = item / nseg, y = item - grp * nseg;
        const int q0 = y * L;
        const int i = grp * kLaneRows + lane;
        if (i < g.H) {
            uint32_t* sc = b.env + (int64_t)i * pitch + q0;
            const int M = scan_row<false, true>(i, min(L, n - q0), g.W, v.cols + q0,
                                                v.rc + (int64_t)i * pitch + q0, sc, RB, true,
                                                ring, lane, false);
            b.segm[(int64_t)i * seg_count(g.W) + y] = (int16_t)M;
            if (y == 0) b.rowfail[i] = 0;
        }
    }
}

template <typename K>
int lane_blocks_per_cu(K kernel) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kernel, kLaneRows, 0) != hipSuccess ||
        nb < 1)
        nb = 1;
    return nb;
}

template <int L>
hipError_t launch_segscan_l(const Img& g, const SegBufs& b, hipStream_t stream) {
    static int per_cu = 0;
    const int most = items_lanes(g.H) * ((g.W + L - 1) / L);  // items if every column is listed
    if (per_cu == 0) per_cu = lane_blocks_per_cu(k_row_segscan<L>);
    const int grid = min(most, per_cu * device_cus());
    EDT_LAUNCH_AS("k_row_segscan", k_row_segscan<L>, dim3(grid), dim3(kLaneRows), 0, stream, g, b);
    return launch_status();
}

}  // namespace

hipError_t launch_row_segscan(const Img& g, int L, const SegBufs& b, hipStream_t stream) {
    if (L == 8 * kSegL) return launch_segscan_l<8 * kSegL>(g, b, stream);
    if (L == 4 * kSegL) return launch_segscan_l<4 * kSegL>(g, b, stream);
    if (L == 2 * kSegL) return launch_segscan_l<2 * kSegL>(g, b, stream);
    return launch_segscan_l<kSegL>(g, b, stream);
}

hipError_t launch_row_lanes_batch(const BatchTable& tb, int total, hipStream_t stream) {
    if (total < 1) return hipSuccess;
    EDT_LAUNCH_AS("k_row_lanes", k_row_lanes_batch, dim3(total), dim3(kLaneRows), 0, stream, tb);
    return launch_status();
}

}  // namespace edt
