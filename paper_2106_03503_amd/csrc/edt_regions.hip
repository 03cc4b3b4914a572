// Region labels (arXiv 2106.03503, Section 1.1: after the transform each region
// stands for one object point or one cluster of connected points, Figures
// fig_voronoi and fig_blobs; Section 1.2: 4- and 8-neighbourhood).  The sites
// are joined into connected components by a union-find forest kept in the
// labels buffer itself; every pixel then takes the label of the component
// that holds its nearest site (the feature transform).
//
// A site (r, c) is the node (r << 15) | c: it orders like the linear index
// r*W + c and finds its slot r*out_pitch + c without a division.  Links only
// ever point to a smaller node, so a root is the smallest node of its tree and
// the label of a finished component is its smallest linear index.  Joining two
// trees takes the known lock-free form: find both roots, write the smaller
// into the larger root with an atomic minimum, and start over from the value
// the minimum returns when that root had been linked meanwhile.
//   k_reg_init     every site linked to the first site of its run in its
//                  wavefront's 64 columns, the run's root
//   k_reg_union    the runs joined with their site neighbours to the left
//                  (across wavefronts) and above (and above-left, above-right
//                  under 8-neighbourhood), each join made once per run overlap
//   k_reg_flatten  every site points at its root
//   k_reg_others   every non-site pixel: its nearest site's root, as a linear
//                  index (it reads only site slots, writes only its own)
//   k_reg_sites    every site: its root as a linear index (its own slot only)
#include "../../include/edt.h"
#include "edt_internal.h"

namespace edt {
namespace {

constexpr int kRegThreads = 256;

struct RegImg {
    const uint8_t* mask;
    int64_t mpitch;
    const int32_t* feat;
    int32_t* lab;
    int64_t opitch;
    int H, W, pol, conn;
    uint64_t wmagic;  // floor(2^33 / W) + 1, for the row of a linear index below 2^30
};

__device__ __forceinline__ int node(int r, int c) { return (r << 15) | c; }

__device__ __forceinline__ int32_t* slot(const RegImg& g, int x) {
    return g.lab + (int64_t)(x >> 15) * g.opitch + (x & 0x7FFF);
}

__device__ __forceinline__ bool site_at(const RegImg& g, int r, int c) {
    const bool obj = g.mask[(int64_t)r * g.mpitch + c] != 0;
    return g.pol ? !obj : obj;
}

// Root of node x.  The forest changes under concurrent joins, so parents are
// read as device-coherent atomics; any value read is an ancestor of x.
__device__ int find_root(const RegImg& g, int x) {
    int p = __hip_atomic_load(slot(g, x), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    while (p != x) {
        x = p;
        p = __hip_atomic_load(slot(g, x), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    return x;
}

__device__ void unite(const RegImg& g, int a, int b) {
    for (;;) {
        a = find_root(g, a);
        b = find_root(g, b);
        if (a == b) return;
        if (a < b) {
            const int t = a;
            a = b;
            b = t;
        }
        const int old = atomicMin(slot(g, a), b);  // link the larger root under the smaller
        if (old == a) return;
        a = old;  // a had been linked elsewhere: join that tree with b instead
    }
}

// Pixel of this thread: row blockIdx.y, column blockIdx.x * kRegThreads + threadIdx.x;
// a wavefront covers 64 adjacent columns of one row.
//
// Every site starts linked to the first site of its run of adjacent sites
// within its wavefront's 64 columns (found with a ballot), which is its own
// root: no atomics, and the unions only have to join runs.
__global__ __launch_bounds__(kRegThreads) void k_reg_init(RegImg g) {
    const int r = blockIdx.y, c = blockIdx.x * kRegThreads + threadIdx.x;
    const int lane = threadIdx.x & 63;
    const bool site = c < g.W && site_at(g, r, c);
    const uint64_t sites = __ballot(site);
    if (!site) return;
    // the run starts after the last non-site lane at or before this one
    const uint64_t gaps = ~sites & (lane == 63 ? ~0ull : ((2ull << lane) - 1));
    const int start = gaps ? 64 - __builtin_clzll(gaps) : 0;
    *slot(g, node(r, c)) = node(r, c - lane + start);
}

// Joins of a site x = (r, c) with the sites around it.  Skipped joins are
// those another site of x's run makes: (a) across a wavefront boundary to the
// left neighbour (inside a wavefront the run is linked already); (b) upward to
// u = (r-1, c) unless the left neighbour and ul = (r-1, c-1) are both sites,
// in which case the left neighbour's own join (or one further left along the
// run, by induction) reaches u's run; (c) under 8-neighbourhood, when u is no
// site: to ul unless the left neighbour is a site (its join with its own up
// neighbour, ul, covers it), and to ur = (r-1, c+1) unless the right
// neighbour is a site (its own up neighbour is ur, and its join is not
// skipped because u is no site).
__global__ __launch_bounds__(kRegThreads) void k_reg_union(RegImg g) {
    const int r = blockIdx.y, c = blockIdx.x * kRegThreads + threadIdx.x;
    if (c >= g.W || !site_at(g, r, c)) return;
    const int x = node(r, c);
    const bool left = c > 0 && site_at(g, r, c - 1);
    if (left && (c & 63) == 0) unite(g, x, node(r, c - 1));
    if (r == 0) return;
    const bool up = site_at(g, r - 1, c);
    const bool ul = c > 0 && site_at(g, r - 1, c - 1);
    if (up) {
        if (!(left && ul)) unite(g, x, node(r - 1, c));
    } else if (g.conn == 8) {
        if (ul && !left) unite(g, x, node(r - 1, c - 1));
        if (c + 1 < g.W && site_at(g, r - 1, c + 1) && !site_at(g, r, c + 1))
            unite(g, x, node(r - 1, c + 1));
    }
}

__global__ __launch_bounds__(kRegThreads) void k_reg_flatten(RegImg g) {
    const int r = blockIdx.y, c = blockIdx.x * kRegThreads + threadIdx.x;
    if (c >= g.W || !site_at(g, r, c)) return;
    const int x = node(r, c);
    __hip_atomic_store(slot(g, x), find_root(g, x), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ int32_t linear_of(const RegImg& g, int x) {
    return (x >> 15) * g.W + (x & 0x7FFF);
}

__global__ __launch_bounds__(kRegThreads) void k_reg_others(RegImg g) {
    const int r = blockIdx.y, c = blockIdx.x * kRegThreads + threadIdx.x;
    if (c >= g.W || site_at(g, r, c)) return;
    const int32_t f = g.feat[(int64_t)r * g.opitch + c];
    int32_t out = -1;
    if (f >= 0 && f < g.H * g.W) {
        // row of the nearest site: f * wmagic / 2^33 exceeds f / W by less
        // than f / 2^33 < 1/8, so the estimate is the quotient or one more,
        // and the remainder settles it
        int q = (int)(((uint64_t)(uint32_t)f * g.wmagic) >> 33);
        const int rem = f - q * g.W;
        if (rem < 0)
            --q;
        else if (rem >= g.W)
            ++q;
        out = linear_of(g, *slot(g, node(q, f - q * g.W)));
    }
    g.lab[(int64_t)r * g.opitch + c] = out;
}

__global__ __launch_bounds__(kRegThreads) void k_reg_sites(RegImg g) {
    const int r = blockIdx.y, c = blockIdx.x * kRegThreads + threadIdx.x;
    if (c >= g.W || !site_at(g, r, c)) return;
    int32_t* s = slot(g, node(r, c));
    *s = linear_of(g, *s);
}

}  // namespace
}  // namespace edt

extern "C" {

edt_status edt_regions(const uint8_t* mask, int32_t H, int32_t W, int64_t mask_pitch,
                       int32_t polarity, int32_t connectivity, const int32_t* feature,
                       int32_t* labels, int64_t out_pitch, void* stream) {
    if (H < 1 || W < 1 || H > EDT_MAX_SIDE || W > EDT_MAX_SIDE) return EDT_ERR_TOO_LARGE;
    if (!mask || !feature || !labels || mask_pitch < W || out_pitch < W)
        return EDT_ERR_INVALID_ARG;
    if (polarity != EDT_TO_OBJECT && polarity != EDT_TO_BACKGROUND) return EDT_ERR_INVALID_ARG;
    if (connectivity != 4 && connectivity != 8) return EDT_ERR_INVALID_ARG;
    if ((int64_t)H * out_pitch >= ((int64_t)1 << 31)) return EDT_ERR_TOO_LARGE;
    // labels holds the forest: it must not share memory with the inputs
    const uintptr_t l0 = reinterpret_cast<uintptr_t>(labels);
    const uintptr_t l1 = l0 + 4 * (uintptr_t)((H - 1) * out_pitch + W);
    const uintptr_t f0 = reinterpret_cast<uintptr_t>(feature);
    const uintptr_t f1 = f0 + 4 * (uintptr_t)((H - 1) * out_pitch + W);
    const uintptr_t m0 = reinterpret_cast<uintptr_t>(mask);
    const uintptr_t m1 = m0 + (uintptr_t)((H - 1) * mask_pitch + W);
    if ((l0 < f1 && f0 < l1) || (l0 < m1 && m0 < l1)) return EDT_ERR_INVALID_ARG;

    edt::RegImg g;
    g.mask = mask;
    g.mpitch = mask_pitch;
    g.feat = feature;
    g.lab = labels;
    g.opitch = out_pitch;
    g.H = H;
    g.W = W;
    g.pol = polarity;
    g.conn = connectivity;
    g.wmagic = ((uint64_t)1 << 33) / (uint64_t)W + 1;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const dim3 grid((unsigned)((W + edt::kRegThreads - 1) / edt::kRegThreads), (unsigned)H);
    const dim3 block(edt::kRegThreads);
    EDT_LAUNCH_AS("k_reg_init", edt::k_reg_init, grid, block, 0, s, g);
    EDT_LAUNCH_AS("k_reg_union", edt::k_reg_union, grid, block, 0, s, g);
    EDT_LAUNCH_AS("k_reg_flatten", edt::k_reg_flatten, grid, block, 0, s, g);
    EDT_LAUNCH_AS("k_reg_others", edt::k_reg_others, grid, block, 0, s, g);
    EDT_LAUNCH_AS("k_reg_sites", edt::k_reg_sites, grid, block, 0, s, g);
    return edt::launch_status() == hipSuccess ? EDT_OK : EDT_ERR_DEVICE;
}

}  // extern "C"
