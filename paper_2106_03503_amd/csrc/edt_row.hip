// Horizontal pass of the exact EDT (Section 3.3 of Strutz, arXiv 2106.03503):
// per row, the lower envelope of the parabolas D_k(j) = Dv(k) + (j - k)^2
// (Eq. eq_parabola) over the columns k that hold a site (the same list for
// every row), then every pixel is filled from the parabola that owns it.
//
// The same pass serves the city-block and chessboard metrics: the parabola of
// column k is replaced by |i - r_k| + |j - k| or max(|i - r_k|, |j - k|), for
// which, as for parabolas, a column right of another beats it on a suffix of
// the row (their difference never falls as j grows), so the envelope, the
// merges and the fill are unchanged and only the cost and the first winning
// pixel differ.
//
// Order and ties: parabolas are compared at a pixel lexicographically on
// (D, feature index), feature = r*W + k, so every pixel is owned by its nearest
// site with the smallest row-major index.  For columns k < l, parabola l beats
// k on a suffix j >= s of the row; s is the first integer past the crossing of
// Eq. eq_intersection, or the crossing itself when l has the smaller index.
//
// The paper builds the envelope with one left-to-right scan and a stack.  Here
// the candidate list of a row is cut into chunks of S candidates, one per lane:
//   1. every lane builds the envelope of its chunk with that scan, the stack
//      kept in place over the chunk's slots;
//   2. neighbouring envelopes are merged pairwise up a binary tree.  Two
//      envelopes whose columns do not interleave cross only once (every
//      parabola of the right one gains on every parabola of the left one as j
//      grows), so the merge keeps a prefix of the left envelope and a suffix of
//      the right one; it walks inwards from the seam, dropping a parabola of
//      the left side when the right side's first parabola already wins where it
//      starts, and one of the right side when the left side's last parabola
//      still wins where it ends.  Each step removes one parabola, so the tree
//      costs O(candidates) in total;
//   3. the survivors are compacted in order and the row is filled, four
//      adjacent pixels per lane and store, so that a wavefront writes 1 KiB of
//      contiguous output per instruction.
// All position tests compare parabola values directly; an exact integer
// division is needed only when a parabola is stored with a new start.
#include "edt_internal.h"

namespace edt {
namespace {

// A candidate is packed as (column << 16) | site row.
__device__ __forceinline__ int ccol(uint32_t c) { return (int)(c >> 16); }
__device__ __forceinline__ int crow(uint32_t c) { return (int)(c & 0xFFFFu); }

// Distance from pixel (i, j) to the site of candidate C under metric kM: the
// squared Euclidean distance (kM = 0, below 2^31 for sides up to 32767), the
// city-block distance (1), the chessboard distance (2) or the chamfer 4-3
// distance (3: min(|di|, |dj|) diagonal steps of 4 and the rest straight
// steps of 3).
template <int kM>
__device__ __forceinline__ int dist_to(uint32_t C, int i, int j) {
    const int dr = i - crow(C), dc = j - ccol(C);
    if (kM == 0) return sqr_c(dr) + sqr_c(dc);
    const int ar = dr < 0 ? -dr : dr, ac = dc < 0 ? -dc : dc;
    if (kM == 1) return ar + ac;
    if (kM == 2) return max(ar, ac);
    return 3 * max(ar, ac) + min(ar, ac);
}

// Ties under the chessboard metric.  At chessboard distance D from pixel
// (i, j) every site of the square [i - D, i + D] x [j - D, j + D] lies at
// exactly D (D being the smallest distance), so the nearest site with the
// smallest index is the square's topmost one, leftmost among those.  A column
// k with max(|i - r_k|, |j - k|) = D offers its topmost site at or below row
// i - D, which may lie above its nearest site r_k; two columns that tie are
// therefore compared on that row, then on the column.  The row is read from
// the column pass: the band's site bits from row i - D on, else the first
// site row below the band.  Where two columns tie over several pixels D is
// constant there (both costs are flat), so the comparison is the same at each
// of them and a column right of another still beats it on a suffix of the
// row.
struct TieCtx {
    const uint64_t* bits;  // [nb][W] site bits of each band column
    const int16_t* down;   // [nb][W] first site row below each band
    int W;
};

// First site row at or after row x (x < 0 counts as 0) in column c, which
// holds a site at or after x.
__device__ __forceinline__ int next_site(const TieCtx& tc, int c, int x) {
    x = max(x, 0);
    const int64_t at = (int64_t)(x >> 6) * tc.W + c;
    const uint64_t m = tc.bits[at] >> (x & 63);
    return m ? x + __builtin_ctzll(m) : tc.down[at];
}

// Does B (a column right of A's) beat A at pixel j of row i?
template <int kM>
__device__ __forceinline__ bool beats(uint32_t B, uint32_t A, int i, int j, const TieCtx& tc) {
    const int fb = dist_to<kM>(B, i, j), fa = dist_to<kM>(A, i, j);
    if (fb != fa) return fb < fa;
    if (kM == 2) return next_site(tc, ccol(B), i - fb) < next_site(tc, ccol(A), i - fa);
    return crow(B) < crow(A);
}

// Feature of pixel (i, j) owned by candidate C at distance d: the site's
// linear index (under the chessboard metric, the topmost site of C's column
// at distance d).
template <int kM>
__device__ __forceinline__ int feature_of(uint32_t C, int i, int d, int W, const TieCtx& tc) {
    const int r = kM == 2 ? next_site(tc, ccol(C), i - d) : crow(C);
    return mul_c(r, W) + ccol(C);
}

// First pixel j in [0, W] from which B beats A (W: never inside the row); B
// beats A on a suffix of the row under each metric.
//   Euclidean: B beats A at j iff j*den > num, or j*den == num and B has the
//   smaller index (a smaller site row: B's column is larger), with num and den
//   from Eq. eq_intersection; so j >= floor((num - [B wins ties]) / den) + 1.
//   City-block: with vertical offsets fa, fb, B wins left of both columns iff
//   fb + l < fa + k (ties by index), right of both iff fb - l < fa - k, and in
//   between from the first j with 2j > fb - fa + l + k.
//   Chessboard and chamfer 4-3: the suffix is found by bisection.
template <int kM>
__device__ __forceinline__ int first_win(uint32_t A, uint32_t B, int i, int W,
                                         const TieCtx& tc) {
    const int k = ccol(A), l = ccol(B), rk = crow(A), rl = crow(B);
    const int t = rl < rk ? 1 : 0;  // B wins ties
    if (kM == 0) {
        const int num = sqr_c(i - rl) - sqr_c(i - rk) + mul_c(l - k, l + k);
        return first_after(num - t, 2 * (l - k), W);
    } else if (kM == 1) {
        const int fk = i > rk ? i - rk : rk - i, fl = i > rl ? i - rl : rl - i;
        const int a = fk + k, b = fl + l;
        if (b < a || (b == a && t)) return 0;
        const int ra = fk - k, rb = fl - l;
        if (!(rb < ra || (rb == ra && t))) return W;
        const int j = ((fl - fk + l + k - t) >> 1) + 1;  // floor division by 2
        return min(max(j, 0), W);
    } else {
        int lo = 0, hi = W;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (beats<kM>(B, A, i, mid, tc))
                hi = mid;
            else
                lo = mid + 1;
        }
        return lo;
    }
}

// Chunk slots: logical slot l = t*S + u (slot u of lane t's chunk) is stored
// at u*T + t, so that lanes working on their own chunks touch consecutive LDS
// banks.
template <int T, int S>
struct Slots {
    uint32_t* cand;
    int16_t* st;
    __device__ __forceinline__ int at(int l) const { return (l % S) * T + l / S; }
    __device__ __forceinline__ uint32_t& c(int l) const { return cand[at(l)]; }
    __device__ __forceinline__ int16_t& s(int l) const { return st[at(l)]; }
};

// Slots stored in logical order (logical slot l at l).
struct PlainSlots {
    uint32_t* cand;
    int16_t* st;
    __device__ __forceinline__ uint32_t& c(int l) const { return cand[l]; }
    __device__ __forceinline__ int16_t& s(int l) const { return st[l]; }
};

// Merge the envelope of chunk group R (first chunk g_r) into the group to its
// left, L (first chunk g_l).  Per chunk c: survivors occupy logical slots
// [lo, hi), nxt/prv link the non-empty chunks of a group, gf/gl hold the first
// and last non-empty chunk of the group starting at c.  The first survivor of
// a group always starts at pixel 0.
template <int kM, typename SL>
__device__ void merge_groups(int g_l, int g_r, const SL& sl,
                             int16_t* __restrict__ lo, int16_t* __restrict__ hi,
                             int16_t* __restrict__ nxt, int16_t* __restrict__ prv,
                             int16_t* __restrict__ gf, int16_t* __restrict__ gl, int i,
                             int W, const TieCtx& tc) {
    const int Ll = gl[g_l], Rf = gf[g_r], Rl = gl[g_r];
    if (Rf < 0) return;
    if (Ll < 0) {
        gf[g_l] = (int16_t)Rf;
        gl[g_l] = (int16_t)Rl;
        return;
    }
    int ca = Ll, ia = hi[ca] - 1;
    int cb = Rf, ib = lo[cb];
    bool left_alive = true, right_alive = true;
    for (;;) {
        const uint32_t A = sl.c(ia), B = sl.c(ib);
        if (beats<kM>(B, A, i, sl.s(ia), tc)) {  // A is hidden wherever it owned pixels
            if (ia > lo[ca]) {
                --ia;
                continue;
            }
            hi[ca] = lo[ca];
            ca = prv[ca];
            if (ca < 0) {
                left_alive = false;
                break;
            }
            ia = hi[ca] - 1;
            continue;
        }
        int bend;  // first pixel after B's range in the right envelope
        if (ib + 1 < hi[cb]) {
            bend = sl.s(ib + 1);
        } else {
            const int cn = nxt[cb];
            bend = cn >= 0 ? sl.s(lo[cn]) : W;
        }
        if (!beats<kM>(B, A, i, bend - 1, tc)) {  // B is hidden wherever it owned pixels
            if (ib + 1 < hi[cb]) {
                ++ib;
                continue;
            }
            lo[cb] = hi[cb];
            cb = nxt[cb];
            if (cb < 0) {
                right_alive = false;
                break;
            }
            ib = lo[cb];
            continue;
        }
        sl.s(ib) = (int16_t)first_win<kM>(A, B, i, W, tc);  // the seam
        break;
    }
    if (left_alive && right_alive) {
        hi[ca] = (int16_t)(ia + 1);
        lo[cb] = (int16_t)ib;
        nxt[ca] = (int16_t)cb;
        prv[cb] = (int16_t)ca;
        gl[g_l] = (int16_t)Rl;
    } else if (!left_alive) {  // the right envelope alone remains
        lo[cb] = (int16_t)ib;
        prv[cb] = -1;
        sl.s(ib) = 0;
        gf[g_l] = (int16_t)cb;
        gl[g_l] = (int16_t)Rl;
    } else {  // the left envelope alone remains
        hi[ca] = (int16_t)(ia + 1);
        nxt[ca] = -1;
        gl[g_l] = (int16_t)ca;
    }
}

// Last index e in [lo, hi) with st[e] <= j, given st[lo] <= j.
__device__ __forceinline__ int last_le(const int16_t* __restrict__ st, int lo, int hi, int j) {
    int a = lo, b = hi - 1;
    while (a < b) {
        const int mid = (a + b + 1) >> 1;
        if (st[mid] <= j)
            a = mid;
        else
            b = mid - 1;
    }
    return a;
}

// Last index in [e, M) with st[idx] <= j, given st[e] <= j: gallop forward
// from e, then bisect the last stride (O(1) when the owner is unchanged).
__device__ __forceinline__ int advance(const int16_t* __restrict__ st, int e, int M, int j) {
    int step = 1;
    while (e + step < M && st[e + step] <= j) {
        e += step;
        step <<= 1;
    }
    return last_le(st, e, min(M, e + step), j);
}

typedef int v4i __attribute__((ext_vector_type(4)));

// Four output pixels; the outputs are written once and not read back by this
// library, so they are stored non-temporally (streamed past the caches).
__device__ __forceinline__ void store4(int32_t* __restrict__ p, int j, int W, bool vec,
                                       int v0, int v1, int v2, int v3) {
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

// Fill row i from its envelope (M survivors in column order: candidates in
// cand, first owned pixels in st), four adjacent pixels per lane and store, so
// that a wavefront writes 1 KiB of contiguous output per instruction.
template <int kM, int T, bool kF = false>
__device__ __forceinline__ void fill_row(const Img& g, int i, const uint32_t* cand,
                                         const int16_t* st, int M, bool vec, const TieCtx& tc) {
    const int W = g.W;
    const int t = threadIdx.x;
    int32_t* drow = g.dist ? g.dist + (int64_t)i * g.opitch : nullptr;
    int32_t* frow = g.feat ? g.feat + (int64_t)i * g.opitch : nullptr;
    int e = 0;
    for (int j = 4 * t; j < W; j += 4 * T) {
        int d[4], f[4];
        if (M == 0) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                d[q] = INT32_MAX;
                f[q] = -1;
            }
        } else {
            // owner of pixel j: the last survivor starting at or before j,
            // searched forward from this lane's previous owner
            e = advance(st, e, M, j);
            uint32_t C = cand[e];
            int nst = e + 1 < M ? st[e + 1] : INT32_MAX;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int jj = j + q;
                if (jj < W) {
                    while (jj >= nst) {
                        ++e;
                        C = cand[e];
                        nst = e + 1 < M ? st[e + 1] : INT32_MAX;
                    }
                    d[q] = dist_to<kM>(C, i, jj);
                    f[q] = frow ? feature_of<kM>(C, i, d[q], W, tc) : 0;
                } else {
                    d[q] = 0;
                    f[q] = 0;
                }
            }
        }
        if (drow) {
            if constexpr (kF) {
#pragma unroll
                for (int q = 0; q < 4; ++q) d[q] = sqrt_bits(d[q]);
            }
            store4(drow, j, W, vec, d[0], d[1], d[2], d[3]);
        }
        if (frow) store4(frow, j, W, vec, f[0], f[1], f[2], f[3]);
    }
}

// Row pass over the rows [i0, i1) (step di) of one image.  T lanes per row, S
// candidate slots per lane.  A form takes an image only if the image's
// device-side count n of candidate columns is in its range: the sparse form
// (one wavefront, kSparse) takes n <= T*S, each dense form the images with
// n > kSparseMaxN whose width is in (T*S/2, T*S].  With kGlobal the candidate
// list lives in the global-memory slot `gslot` instead of LDS.
template <int T, int S, bool kSparse, bool kGlobal>
struct RowLds {
    static constexpr int CAP = kGlobal ? 1 : T * S;
    uint32_t cand[CAP];
    int16_t st[CAP];
    int16_t lo[T], hi[T], nxt[T], prv[T], gf[T], gl[T];
    int wsum[T / 64];
};

template <int T, int S, bool kSparse, bool kGlobal>
__device__ __forceinline__ bool form_takes(int n, int W) {
    if (kSparse) return n <= T * S;
    return n > kSparseMaxN && W > T * S / 2 && W <= T * S;
}

template <int kM, int T, int S, bool kSparse, bool kGlobal, bool kF>
__device__ void process_rows(const Img& g, int i0, int i1, int di,
                             RowLds<T, S, kSparse, kGlobal>& sh, uint8_t* gslot) {
    constexpr int NW = T / 64;
    static_assert(!kGlobal || T * S <= kWideCap, "global row slot too small");
    static_assert((S & (S - 1)) == 0 && (T & (T - 1)) == 0, "T and S must be powers of two");
    const Views v = views_of(g);
    const int n = v.meta[0];
    const int W = g.W;
    if (!form_takes<T, S, kSparse, kGlobal>(n, W)) return;  // another form's image
    const TieCtx tc{v.bits, v.down, W};
    const int pitch = v.meta[1];
    uint32_t* cand;
    int16_t* st;
    if (kGlobal) {
        cand = reinterpret_cast<uint32_t*>(gslot);
        st = reinterpret_cast<int16_t*>(gslot + (size_t)kWideCap * 4);
    } else {
        cand = sh.cand;
        st = sh.st;
    }
    const Slots<T, S> sl{cand, st};
    const int t = threadIdx.x;
    const int lane = t & 63, wave = t >> 6;
    const int nchunks = (n + S - 1) / S;
    const int base = t * S;
    const int cnt = min(max(n - base, 0), S);
    const bool vec = (!g.dist || reinterpret_cast<uintptr_t>(g.dist) % 16 == 0) &&
                     (!g.feat || reinterpret_cast<uintptr_t>(g.feat) % 16 == 0) &&
                     (g.opitch % 4 == 0);

    // The candidate columns of this lane's chunk are the same in every row.
    uint32_t colhi[S];
#pragma unroll
    for (int u = 0; u < S; ++u) colhi[u] = u < cnt ? ((uint32_t)(uint16_t)v.cols[base + u] << 16) : 0u;

    for (int i = i0; i < i1; i += di) {
        // 1. this row's candidates of the chunk: (column, nearest site row).
        // The one-wavefront form works the site rows out from the column's
        // band bits and the carries above and below the band (the nearest
        // site at or above the row and at or below it, the upper one at equal
        // distance, as the nearest-row pass does), so that pass has nothing
        // to do for the images this form takes; the other forms read the
        // list of site rows it writes.
        const int16_t* rrow = v.rc + (int64_t)i * pitch + base;
        if (kSparse) {
            constexpr int kFar = 1 << 20;  // a missing side: farther than any site
            const int bb = i / kBand, r = i - bb * kBand;
            const uint64_t amask = r == 63 ? ~0ull : (2ull << r) - 1ull;  // rows 0..r
            const int64_t b0 = (int64_t)bb * W;
#pragma unroll 2
            for (int u = 0; u < S; ++u) {
                if (u < cnt) {
                    const int64_t k = b0 + (int)(colhi[u] >> 16);
                    const uint64_t m = v.bits[k];
                    const int up = v.up[k], dn = v.down[k];
                    const uint64_t above = m & amask, below = m >> r;
                    const int a =
                        above ? bb * kBand + 63 - __clzll(above) : (up < 0 ? -kFar : up);
                    const int d = below ? i + __builtin_ctzll(below) : (dn == kNoBelow ? kFar : dn);
                    sl.c(base + u) = colhi[u] | (uint32_t)(2 * i <= a + d ? a : d);
                }
            }
        } else if (cnt == S) {
            uint32_t w[S / 2];
#pragma unroll
            for (int q = 0; q < S / 8; ++q) {
                const int4 x = reinterpret_cast<const int4*>(rrow)[q];
                w[4 * q + 0] = (uint32_t)x.x;
                w[4 * q + 1] = (uint32_t)x.y;
                w[4 * q + 2] = (uint32_t)x.z;
                w[4 * q + 3] = (uint32_t)x.w;
            }
#pragma unroll
            for (int u = 0; u < S; ++u)
                sl.c(base + u) = colhi[u] | ((w[u >> 1] >> (16 * (u & 1))) & 0xFFFFu);
        } else {
#pragma unroll
            for (int u = 0; u < S; ++u)
                if (u < cnt) sl.c(base + u) = colhi[u] | (uint32_t)(uint16_t)rrow[u];
        }
        // 2. envelope of the chunk: left-to-right scan, stack in place
        int m = 0;
        for (int u = 0; u < cnt; ++u) {
            const uint32_t C = sl.c(base + u);
            bool keep = true;
            while (m > 0) {
                const uint32_t A = sl.c(base + m - 1);
                if (beats<kM>(C, A, i, sl.s(base + m - 1), tc)) {  // C hides the stack top
                    --m;
                    continue;
                }
                keep = beats<kM>(C, A, i, W - 1, tc);  // C wins somewhere inside the row
                if (keep) sl.s(base + m) = (int16_t)first_win<kM>(A, C, i, W, tc);
                break;
            }
            if (m == 0) {
                sl.s(base) = 0;
                sl.c(base) = C;
                m = 1;
            } else if (keep) {
                sl.c(base + m) = C;
                ++m;
            }
        }
        sh.lo[t] = (int16_t)base;
        sh.hi[t] = (int16_t)(base + m);
        sh.nxt[t] = -1;
        sh.prv[t] = -1;
        sh.gf[t] = (int16_t)(m > 0 ? t : -1);
        sh.gl[t] = (int16_t)(m > 0 ? t : -1);
        __syncthreads();
        // 3. merge up the tree
        for (int w = 1; w < nchunks; w <<= 1) {
            if ((t & (2 * w - 1)) == 0 && t + w < nchunks)
                merge_groups<kM>(t, t + w, sl, sh.lo, sh.hi, sh.nxt, sh.prv, sh.gf, sh.gl, i, W,
                                 tc);
            __syncthreads();
        }
        // 4. survivors to the front of the list, in column order (plain layout)
        const int lo = sh.lo[t];
        const int c = sh.hi[t] - lo;
        uint32_t kc[S];
        int16_t ks[S];
#pragma unroll
        for (int u = 0; u < S; ++u) {
            if (u < c) {
                kc[u] = sl.c(lo + u);
                ks[u] = sl.s(lo + u);
            }
        }
        int incl = c;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const int x = __shfl_up(incl, d, 64);
            if (lane >= d) incl += x;
        }
        if (lane == 63) sh.wsum[wave] = incl;
        __syncthreads();
        int pos = incl - c, M = 0;
#pragma unroll
        for (int q = 0; q < NW; ++q) {
            if (q < wave) pos += sh.wsum[q];
            M += sh.wsum[q];
        }
#pragma unroll
        for (int u = 0; u < S; ++u) {
            if (u < c) {
                cand[pos + u] = kc[u];
                st[pos + u] = ks[u];
            }
        }
        __syncthreads();
        // 5. fill, four adjacent pixels per lane and step
        fill_row<kM, T, kF>(g, i, cand, st, M, vec, tc);
        __syncthreads();  // the next row reuses the list and the chunk tables
    }
}

// One image: rows blockIdx.x, blockIdx.x + gridDim.x, ...  With kF the
// distances are written as fp32 Euclidean distances (sqrt_bits); the sparse
// form then asks for 5 waves per SIMD, as it reaches without the conversion
// (its fp64 square root would otherwise take it to 102 VGPRs and 4 waves).
template <int kM, int T, int S, bool kSparse, bool kGlobal, bool kF = false>
__global__ __launch_bounds__(T, (kF && kSparse) ? 5 : 1) void k_row_single(Img g, uint8_t* __restrict__ slots) {
    __shared__ RowLds<T, S, kSparse, kGlobal> sh;
    uint8_t* gslot = kGlobal ? slots + (size_t)blockIdx.x * wide_slot_bytes() : nullptr;
    process_rows<kM, T, S, kSparse, kGlobal, kF>(g, blockIdx.x, g.H, gridDim.x, sh, gslot);
}

// Dense rows of one image after the segment scan: the envelope of segment c
// (candidates [c L, (c + 1) L), built one lane per row and segment) holds
// segm[i][c] entries at slots c L + e of the row in env (packed candidate)
// and in its list of site rows (start).
//
// k_row_segwin fills every pixel from the best of the segment envelopes near
// it, with the bounded search of Section 3.2.2 at the level of segments:
// starting from the segment under the pixel, a walk goes left and right and
// stops on each side at the first segment whose nearest column is
// horizontally farther than the best distance found (strictly farther, so
// that an equally near site with a smaller index is still seen); every
// candidate beyond it is farther still.  A work item is one tile of kWinTile
// pixels of a row; it copies into LDS the segments under the tile and
// win_halo<L>() more on each side, and reads a segment beyond those from
// memory (4096-pixel tiles with two more segments a side were the fastest of
// the tile widths 1024..8192, halos 1..4 and 256..1024 lanes measured with
// 64- and 128-candidate segments; 512-candidate segments span at least 512
// columns, and one more a side is faster there).
// A row where some pixel would need more than kWinCap segments besides its
// own is marked in rowfail and done by k_row_segfill instead: its segments
// are merged up a binary tree (log2(n / L) levels), the survivors compacted,
// and the row filled from them.
constexpr int kWinTile = 4096;
constexpr int kWinLanes = 256;
template <int L>
constexpr int win_halo() {
    return L >= 512 ? 1 : 2;
}
constexpr int kWinCap = 24;
// Segments of L candidates: those a tile's columns can touch (each spans at
// least L columns), plus the halo, and the most a row can have.
template <int L>
struct WinShape {
    static constexpr int kSegs = kWinTile / L + 1 + 2 * win_halo<L>();
    static constexpr int kMax = kLdsMaxW / L;
    static constexpr int kPer = (kSegs * L + kWinLanes - 1) / kWinLanes;  // slots per lane
};

template <int L>
struct WinLds {
    static constexpr int S = WinShape<L>::kSegs, G = WinShape<L>::kMax;
    uint32_t cand[S * L];
    int16_t st[S * L];
    int eleft[S], eright[S];   // envelope of each loaded segment at its first and last column
    int16_t cnt[S];            // entries of each loaded segment
    int16_t segof[kWinTile / 16];  // segment under every 16th pixel of the tile
    int16_t first[G], last[G];     // columns of each segment's first and last candidate
};

// Last index e in [lo, hi) with st[e] <= j, given st[lo] <= j (LDS or memory).
template <typename SP>
__device__ __forceinline__ int last_le_any(SP st, int lo, int hi, int j) {
    int a = lo, b = hi - 1;
    while (a < b) {
        const int mid = (a + b + 1) >> 1;
        if (st[mid] <= j)
            a = mid;
        else
            b = mid - 1;
    }
    return a;
}

// Best entry of one segment envelope (entries [lo, hi) of cand / st, the first
// starting at pixel 0) at the four pixels j..j+3 of row i, folded into (bd, bf)
// lexicographically.
template <typename CP, typename SP>
__device__ __forceinline__ void seg_best4(CP cand, SP st, int lo, int hi, int i, int j, int W,
                                          int* bd, int* bf) {
    int e = last_le_any(st, lo, hi, j);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int jj = j + q;
        while (e + 1 < hi && st[e + 1] <= jj) ++e;
        const uint32_t C = cand[e];
        const int d = sqr_c(i - crow(C)) + sqr_c(jj - ccol(C));
        const int f = mul_c(crow(C), W) + ccol(C);
        if (d < bd[q] || (d == bd[q] && f < bf[q])) {
            bd[q] = d;
            bf[q] = f;
        }
    }
}

// The last segment whose first column is at or before x (0 if none).
__device__ __forceinline__ int seg_at(const int16_t* first, int nseg, int x) {
    int a = 0, b = nseg - 1;
    while (a < b) {
        const int mid = (a + b + 1) >> 1;
        if (first[mid] <= x)
            a = mid;
        else
            b = mid - 1;
    }
    return a;
}

// Up to 128-candidate segments the LDS copy leaves room for 5 workgroups per
// CU, and the kernel is held to the registers of 5 waves per SIMD (96, with no
// spills); the longer segments' copy allows 4.
template <int L, bool kF = false>
__global__ __launch_bounds__(kWinLanes, L <= 128 ? 5 : 1) void k_row_segwin(Img g, SegBufs sb) {
    __shared__ WinLds<L> sh;
    constexpr int kPer = WinShape<L>::kPer;
    static_assert(L >= 16, "a 16-pixel step crosses at most one segment start");
    __shared__ int s_lo, s_hi, s_next;
    const Views v = views_of(g);
    const int n = v.meta[0];
    if (n <= kSparseMaxN) return;  // the one-wavefront row pass took the image
    const int W = g.W;
    const int pitch = v.meta[1];
    const int nseg = (n + L - 1) / L;
    const int ntiles = (W + kWinTile - 1) / kWinTile;
    const int total = g.H * ntiles;
    const int t = threadIdx.x;
    const int sstride = seg_count(W);
    const bool vec = (!g.dist || reinterpret_cast<uintptr_t>(g.dist) % 16 == 0) &&
                     (!g.feat || reinterpret_cast<uintptr_t>(g.feat) % 16 == 0) &&
                     (g.opitch % 4 == 0);
    for (int c = t; c < nseg; c += kWinLanes) {
        sh.first[c] = v.cols[c * L];
        sh.last[c] = v.cols[min((c + 1) * L, n) - 1];
    }
    // With many items per workgroup they are taken in the order workgroups
    // claim them: each workgroup's first is its own index, and while working
    // on one it claims the next from a counter (zeroed by the column-list
    // pass), so that rows of uneven cost spread over the workgroups as they
    // free up.  With few, the claim's latency (its first load waits for it:
    // loads and atomics share one counter) costs more than the balance gains,
    // and a workgroup takes every gridDim.x-th item.
    const bool claimed = total >= 16 * (int)gridDim.x;
    for (int item = blockIdx.x; item < total;) {
        const int i = item / ntiles;
        const int x0 = (item - i * ntiles) * kWinTile, x1 = min(W, x0 + kWinTile);
        __syncthreads();  // the previous item is done with the LDS copy
        int claim = 0;
        if (t == 0) {
            if (claimed) claim = atomicAdd(&v.meta[2], 1);
            s_lo = max(0, seg_at(sh.first, nseg, x0) - win_halo<L>());
            s_hi = min(nseg - 1, seg_at(sh.first, nseg, x1 - 1) + win_halo<L>());
        }
        __syncthreads();
        const int lo = s_lo, hi = s_hi;  // loaded segments [lo, hi], at most WinShape<L>::kSegs
        const uint32_t* erow = sb.env + (int64_t)i * pitch;
        const int16_t* srow = v.rc + (int64_t)i * pitch;
        const int16_t* mrow = sb.segm + (int64_t)i * sstride;
        // every load in flight before the LDS writes: slots of candidates
        // past a segment's envelope are copied too and never read
        const int q0 = lo * L, qn = min(n, (hi + 1) * L);
        uint32_t vc[kPer];
        int vs[kPer];
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
            const int q = q0 + t + u * kWinLanes;
            if (q < qn) {
                vc[u] = erow[q];
                vs[u] = srow[q];
            }
        }
        const int mt = t <= hi - lo ? mrow[lo + t] : 0;
        if (t <= hi - lo) sh.cnt[t] = (int16_t)mt;
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
            const int q = q0 + t + u * kWinLanes;
            if (q < qn) {
                sh.cand[q - q0] = vc[u];
                sh.st[q - q0] = (int16_t)vs[u];
            }
        }
        __syncthreads();
        // A candidate k of segment c and a pixel x left of c's first column f
        // have (k - x)^2 >= (k - f)^2 + (f - x)^2, so c's envelope at x is at
        // least its value at f plus (f - x)^2; likewise right of its last
        // column.  These two values bound a segment before it is searched.
        if (t < kWinTile / 16) sh.segof[t] = (int16_t)seg_at(sh.first, nseg, x0 + 16 * t);
        if (t <= hi - lo) {
            const int b0 = t * L, f = sh.first[lo + t], l = sh.last[lo + t];
            const uint32_t Cf = sh.cand[last_le_any(sh.st, b0, b0 + mt, f)];
            const uint32_t Cl = sh.cand[last_le_any(sh.st, b0, b0 + mt, l)];
            sh.eleft[t] = sqr_c(i - crow(Cf)) + sqr_c(f - ccol(Cf));
            sh.eright[t] = sqr_c(i - crow(Cl)) + sqr_c(l - ccol(Cl));
        }
        __syncthreads();
        int32_t* drow = g.dist ? g.dist + (int64_t)i * g.opitch : nullptr;
        int32_t* frow = g.feat ? g.feat + (int64_t)i * g.opitch : nullptr;
        bool ok = true;
        for (int j = x0 + 4 * t; j < x1 && ok; j += 4 * kWinLanes) {
            int bd[4], bf[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                bd[q] = INT32_MAX;
                bf[q] = INT32_MAX;
            }
            // best of segment c at j..j+3, from LDS when it is loaded
            auto visit = [&](int c) {
                if (c >= lo && c <= hi) {
                    const int b0 = (c - lo) * L;
                    seg_best4(sh.cand, sh.st, b0, b0 + sh.cnt[c - lo], i, j, W, bd, bf);
                } else {
                    seg_best4(erow, srow, c * L, c * L + mrow[c], i, j, W, bd, bf);
                }
            };
            // a segment spans at least L >= 16 columns: at most one more
            // starts within the 16 pixels
            int s0 = sh.segof[(j - x0) >> 4];
            if (s0 + 1 < nseg && sh.first[s0 + 1] <= j) ++s0;
            visit(s0);
            const int jl = min(j + 3, W - 1);  // pixels past the row end do not widen the search
            auto farthest = [&]() {
                int f = 0;
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    if (j + q < W) f = max(f, bd[q]);
                return f;
            };
            int far = farthest(), evals = 0;
            for (int c = s0 - 1; c >= 0; --c) {
                const int l = sh.last[c];
                const int gap = j - l;  // >= 1: every column of c lies left of j
                if (sqr_c(gap) > far) break;
                if (c >= lo && c <= hi) {
                    // skip c if its bound beats no pixel of the group
                    const int e = sh.eright[c - lo];
                    bool need = false;
#pragma unroll
                    for (int q = 0; q < 4; ++q)
                        need |= j + q < W && e + sqr_c(j + q - l) <= bd[q];
                    if (!need) continue;
                }
                if (++evals > kWinCap) {
                    ok = false;
                    break;
                }
                visit(c);
                far = farthest();
            }
            for (int c = s0 + 1; c < nseg && ok; ++c) {
                const int f = sh.first[c];
                const int gap = f - jl;  // may be <= 0: c starts inside the group
                if (gap > 0 && sqr_c(gap) > far) break;
                if (gap > 0 && c >= lo && c <= hi) {
                    const int e = sh.eleft[c - lo];
                    bool need = false;
#pragma unroll
                    for (int q = 0; q < 4; ++q)
                        need |= j + q < W && e + sqr_c(f - j - q) <= bd[q];
                    if (!need) continue;
                }
                if (++evals > kWinCap) {
                    ok = false;
                    break;
                }
                visit(c);
                far = farthest();
            }
            if (!ok) break;
            if (drow) {
                if constexpr (kF) {
#pragma unroll
                    for (int q = 0; q < 4; ++q) bd[q] = sqrt_bits(bd[q]);
                }
                store4(drow, j, W, vec, bd[0], bd[1], bd[2], bd[3]);
            }
            if (frow) store4(frow, j, W, vec, bf[0], bf[1], bf[2], bf[3]);
        }
        if (!ok) sb.rowfail[i] = 1;
        if (t == 0) s_next = claimed ? (int)gridDim.x + claim : item + (int)gridDim.x;
        __syncthreads();
        item = s_next;
    }
}

// The rows that k_row_segwin left to the merge: per row, copy the segment
// envelopes into LDS, merge them up a binary tree, compact the survivors and
// fill.  The form with T lanes takes widths in (8 T, 16 T].
template <int T, int L>
struct SegLds {
    static constexpr int CAP = 16 * T;
    static constexpr int G = CAP / L;
    uint32_t cand[CAP];
    int16_t st[CAP];
    int16_t lo[G], hi[G], nxt[G], prv[G], gf[G], gl[G];
    int pos[G];
    int wsum[T / 64];
};

template <int T, int L, bool kF = false>
__global__ __launch_bounds__(T, T <= 512 ? 6 : 1) void k_row_segfill(Img g, SegBufs sb) {
    __shared__ SegLds<T, L> sh;
    constexpr int CAP = SegLds<T, L>::CAP, NW = T / 64, PER = CAP / T;
    static_assert(SegLds<T, L>::G <= T, "one lane per segment");
    static_assert(L % kSegL == 0, "segment envelopes are laid out L slots apart");
    const Views v = views_of(g);
    const int n = v.meta[0];
    const int W = g.W;
    if (n <= kSparseMaxN || W <= CAP / 2 || W > CAP) return;  // another form's image
    const TieCtx tc{v.bits, v.down, W};
    const int pitch = v.meta[1];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int nchunks = (n + L - 1) / L;
    const int sstride = seg_count(W);
    const bool vec = (!g.dist || reinterpret_cast<uintptr_t>(g.dist) % 16 == 0) &&
                     (!g.feat || reinterpret_cast<uintptr_t>(g.feat) % 16 == 0) &&
                     (g.opitch % 4 == 0);
    const PlainSlots sl{sh.cand, sh.st};
    for (int i = blockIdx.x; i < g.H; i += gridDim.x) {
        if (!sb.rowfail[i]) continue;  // the same in every lane
        const uint32_t* sc = sb.env + (int64_t)i * pitch;
        const int16_t* rr = v.rc + (int64_t)i * pitch;
        if (t < nchunks) {
            const int m = sb.segm[(int64_t)i * sstride + t];
            sh.lo[t] = (int16_t)(t * L);
            sh.hi[t] = (int16_t)(t * L + m);
            sh.nxt[t] = -1;
            sh.prv[t] = -1;
            sh.gf[t] = (int16_t)(m > 0 ? t : -1);
            sh.gl[t] = (int16_t)(m > 0 ? t : -1);
        }
        __syncthreads();
        // four loads in flight per lane before their LDS writes wait
#pragma unroll
        for (int k0 = 0; k0 < PER; k0 += 4) {
            uint32_t vc[4];
            int16_t vs[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int q = t + (k0 + k) * T;
                if (q < n) {
                    vc[k] = sc[q];
                    vs[k] = rr[q];
                }
            }
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int q = t + (k0 + k) * T;
                if (q < n && q < sh.hi[q / L]) {
                    sh.cand[q] = vc[k];
                    sh.st[q] = vs[k];
                }
            }
        }
        __syncthreads();
        for (int w = 1; w < nchunks; w <<= 1) {
            if (t < nchunks && (t & (2 * w - 1)) == 0 && t + w < nchunks)
                merge_groups<0>(t, t + w, sl, sh.lo, sh.hi, sh.nxt, sh.prv, sh.gf, sh.gl, i, W,
                                tc);
            __syncthreads();
        }
        // survivors to the front, in column order
        const int c = t < nchunks ? sh.hi[t] - sh.lo[t] : 0;
        int incl = c;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const int x = __shfl_up(incl, d, 64);
            if (lane >= d) incl += x;
        }
        if (lane == 63) sh.wsum[wave] = incl;
        __syncthreads();
        int pos = incl - c, M = 0;
#pragma unroll
        for (int q = 0; q < NW; ++q) {
            if (q < wave) pos += sh.wsum[q];
            M += sh.wsum[q];
        }
        if (t < nchunks) sh.pos[t] = pos;
        __syncthreads();
        // in two rounds of slots: a survivor only moves down, so the first
        // round's writes land below every slot the second round reads
        constexpr int HALF = PER / 2;
#pragma unroll
        for (int r = 0; r < 2; ++r) {
            uint32_t kc[HALF];
            int16_t ks[HALF];
            int kd[HALF];
#pragma unroll
            for (int k = 0; k < HALF; ++k) {
                const int q = t + (r * HALF + k) * T;
                kd[k] = -1;
                if (q < n) {
                    const int cq = q / L;
                    if (q >= sh.lo[cq] && q < sh.hi[cq]) {
                        kc[k] = sh.cand[q];
                        ks[k] = sh.st[q];
                        kd[k] = sh.pos[cq] + q - sh.lo[cq];
                    }
                }
            }
            __syncthreads();
#pragma unroll
            for (int k = 0; k < HALF; ++k) {
                if (kd[k] >= 0) {
                    sh.cand[kd[k]] = kc[k];
                    sh.st[kd[k]] = ks[k];
                }
            }
        }
        __syncthreads();
        fill_row<0, T, kF>(g, i, sh.cand, sh.st, M, vec, tc);
        __syncthreads();  // the next row reuses the tables
    }
}

// A batch: workgroup g takes the contiguous run of row items
// [g*chunk, (g+1)*chunk) across the images of the table, so that it stays on
// one image for many rows.
template <int T, int S, bool kSparse>
__global__ __launch_bounds__(T) void k_row_batch(BatchTable tb, int total) {
    __shared__ RowLds<T, S, kSparse, false> sh;
    __shared__ int s_img;
    const int chunk = (total + gridDim.x - 1) / gridDim.x;
    int item = blockIdx.x * chunk;
    const int end = min(total, item + chunk);
    while (item < end) {
        __syncthreads();
        if (threadIdx.x == 0) s_img = batch_image_of(tb, kPhRows, item);
        __syncthreads();
        const int im = s_img;
        const Img g = batch_img(tb, im);
        const int r0 = item - tb.prefix[kPhRows][im];
        const int r1 = min(g.H, end - tb.prefix[kPhRows][im]);
        process_rows<0, T, S, kSparse, false, false>(g, r0, r1, 1, sh, nullptr);
        item += r1 - r0;
    }
}

template <typename K>
int blocks_per_cu(K kernel, int threads) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kernel, threads, 0) != hipSuccess ||
        nb < 1)
        nb = 1;
    return nb;
}

template <int kM, int T, int S, bool kSparse, bool kGlobal, bool kF = false>
hipError_t launch_single(const Img& g, uint8_t* slots, hipStream_t stream) {
    static int per_cu = 0;
    if (per_cu == 0) per_cu = blocks_per_cu(k_row_single<kM, T, S, kSparse, kGlobal, kF>, T);
    int grid = per_cu * device_cus();
    if (kGlobal && grid > kWideSlots) grid = kWideSlots;
    if (grid > g.H) grid = g.H;
    const char* name = kSparse ? "k_row_sparse" : (kGlobal ? "k_row_dense_global" : "k_row_dense");
    EDT_LAUNCH_AS(name, (k_row_single<kM, T, S, kSparse, kGlobal, kF>), dim3(grid), dim3(T), 0,
                  stream, g, slots);
    return launch_status();
}

template <int T, int S, bool kSparse>
hipError_t launch_batch(const BatchTable& tb, int total, hipStream_t stream) {
    static int per_cu = 0;
    if (per_cu == 0) per_cu = blocks_per_cu(k_row_batch<T, S, kSparse>, T);
    int grid = per_cu * device_cus();
    if (grid > total) grid = total;
    if (grid < 1) return hipSuccess;
    const char* name = kSparse ? "k_row_sparse" : "k_row_dense";
    EDT_LAUNCH_AS(name, (k_row_batch<T, S, kSparse>), dim3(grid), dim3(T), 0, stream, tb, total);
    return launch_status();
}

template <int T, int L, bool kF>
hipError_t launch_segfill(const Img& g, const SegBufs& sb, hipStream_t stream) {
    static int per_cu = 0;
    if (per_cu == 0) per_cu = blocks_per_cu(k_row_segfill<T, L, kF>, T);
    int grid = per_cu * device_cus();
    if (grid > g.H) grid = g.H;
    EDT_LAUNCH_AS("k_row_segfill", (k_row_segfill<T, L, kF>), dim3(grid), dim3(T), 0, stream, g,
                  sb);
    return launch_status();
}

template <int L, bool kF>
hipError_t launch_segwin(const Img& g, const SegBufs& sb, hipStream_t stream) {
    static int per_cu = 0;
    if (per_cu == 0) per_cu = blocks_per_cu(k_row_segwin<L, kF>, kWinLanes);
    const int total = g.H * ((g.W + kWinTile - 1) / kWinTile);
    const int grid = min(total, per_cu * device_cus());
    EDT_LAUNCH_AS("k_row_segwin", (k_row_segwin<L, kF>), dim3(grid), dim3(kWinLanes), 0, stream,
                  g, sb);
    return launch_status();
}

template <int L, bool kF>
hipError_t launch_segments_l(const Img& g, const SegBufs& sb, hipStream_t stream) {
    hipError_t e = launch_row_segscan(g, L, sb, stream);
    if (e == hipSuccess) e = launch_segwin<L, kF>(g, sb, stream);
    if (e != hipSuccess) return e;
    const int W = g.W;
    if (W <= 2048) return launch_segfill<128, L, kF>(g, sb, stream);
    if (W <= 4096) return launch_segfill<256, L, kF>(g, sb, stream);
    if (W <= 8192) return launch_segfill<512, L, kF>(g, sb, stream);
    return launch_segfill<1024, L, kF>(g, sb, stream);
}

// Dense rows of one image, squared Euclidean: segment scan, the bounded
// search over segments, then the merge for the rows it left.  Longer
// segments cut the segments a pixel visits and the scan's work items; the
// longest of 512, 256 and 128 candidates that still gives the scan at least
// 4096 work items is taken, else 64 (measured on 16384^2 disks, scan and
// search: 2.47 ms with 128, 2.33 with 256, 2.19 with 512 and 2.71 with 1024,
// 128 having beaten 64 there by 0.3 ms; on 4096^2 disks the longer ones are
// slower: too few scan items).
template <bool kF>
hipError_t launch_rows_segments(const Img& g, hipStream_t stream) {
    const SegBufs sb = seg_bufs(g);
    auto items = [&](int L) { return (int64_t)items_lanes(g.H) * ((g.W + L - 1) / L); };
    if (items(8 * kSegL) >= 4096) return launch_segments_l<8 * kSegL, kF>(g, sb, stream);
    if (items(4 * kSegL) >= 4096) return launch_segments_l<4 * kSegL, kF>(g, sb, stream);
    if (items(2 * kSegL) >= 4096) return launch_segments_l<2 * kSegL, kF>(g, sb, stream);
    return launch_segments_l<kSegL, kF>(g, sb, stream);
}

// kF (squared Euclidean only): distances written as fp32 Euclidean ones; the
// kernels without it compile exactly as if the option did not exist.
template <int kM, bool kF = false>
hipError_t launch_rows_metric(const Img& g, uint8_t* slots, hipStream_t stream) {
    static_assert(!kF || kM == 0, "fp32 distances are Euclidean only");
    // Both forms are enqueued; each returns at once unless the image's number
    // of candidate columns (known only on the device) is in its range.
    hipError_t e = launch_single<kM, kSparseLanes, kRowS, true, false, kF>(g, slots, stream);
    const int W = g.W;
    if (e != hipSuccess || W <= kSparseMaxN) return e;
    if (kM == 0 && has_segments(W)) return launch_rows_segments<kF>(g, stream);
    if (W <= 2048) return launch_single<kM, 128, kRowS, false, false, kF>(g, slots, stream);
    if (W <= 4096) return launch_single<kM, 256, kRowS, false, false, kF>(g, slots, stream);
    if (W <= 8192) return launch_single<kM, 512, kRowS, false, false, kF>(g, slots, stream);
    if (W <= kLdsMaxW) return launch_single<kM, 1024, kRowS, false, false, kF>(g, slots, stream);
    return launch_single<kM, 1024, 2 * kRowS, false, true, kF>(g, slots, stream);
}

}  // namespace

hipError_t launch_row_pass(const Img& g, uint8_t* slots, hipStream_t stream) {
    if (g.fsq) return g.metric == 0 ? launch_rows_metric<0, true>(g, slots, stream)
                                    : hipErrorInvalidValue;
    if (g.metric == 1) return launch_rows_metric<1>(g, slots, stream);
    if (g.metric == 2) return launch_rows_metric<2>(g, slots, stream);
    if (g.metric == 3) return launch_rows_metric<3>(g, slots, stream);
    return launch_rows_metric<0>(g, slots, stream);
}

hipError_t launch_row_pass_batch(const BatchTable& tb, const int* totals, int max_w,
                                 hipStream_t stream) {
    const int total = totals[kPhRows];
    hipError_t e = launch_batch<kSparseLanes, kRowS, true>(tb, total, stream);
    if (e == hipSuccess && max_w > 1024) e = launch_batch<128, kRowS, false>(tb, total, stream);
    if (e == hipSuccess && max_w > 2048) e = launch_batch<256, kRowS, false>(tb, total, stream);
    if (e == hipSuccess && max_w > 4096) e = launch_batch<512, kRowS, false>(tb, total, stream);
    if (e == hipSuccess && max_w > 8192) e = launch_batch<1024, kRowS, false>(tb, total, stream);
    return e;
}

}  // namespace edt
