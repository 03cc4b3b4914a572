/*
 * edt.h -- C ABI of libedt, an MI355X (gfx950) implementation of the exact
 * Euclidean distance transform and feature transform of binary images
 * (T. Strutz, "The Distance Transform and its Computation -- An
 * Introduction", arXiv 2106.03503).
 *
 * The operation (Section 1.1 and Section 3 of the paper): given a binary image
 * and a choice of direction, every pixel receives the squared Euclidean
 * distance to the nearest "site" (Eq. eq_squaredEuclid), and optionally the
 * index of that site (the feature transform; the assignment k* of Section 3.3,
 * which partitions the image into the Voronoi regions of Figures fig_voronoi
 * and fig_blobs).  The square root may be drawn afterwards (Section 3.1).
 *
 * Conventions shared by every entry point:
 *   - Image layout: row-major; H rows (the paper's M), W columns (its L);
 *     1 <= H, W <= EDT_MAX_SIDE.  Row i, column j are 0-based.
 *   - Mask: uint8, byte 0 = background, any other value = object pixel
 *     (Section 1.1: a binary image holds one of two values per pixel).
 *     mask_pitch is the distance in BYTES between row starts (>= W).  Mask
 *     rows are read in whole aligned 4-byte words: the bytes of such a word
 *     that lie before a row's first or after its last pixel (at most 3 on
 *     either side, never on another page) are read and ignored.
 *   - polarity EDT_TO_OBJECT: sites are the object pixels, i.e. every pixel
 *     gets its distance to the nearest object pixel (Figure fig_examples(c));
 *     EDT_TO_BACKGROUND: sites are the background pixels (Figure
 *     fig_examples(b)).  There is no implicit site outside the image.
 *   - Outputs: int32, row-major, out_pitch in ELEMENTS between row starts
 *     (>= W).  dist_sq = d^2 (0 exactly at sites); feature = r*W + c, the
 *     0-based row-major index of the nearest site, with ties between equally
 *     near sites broken towards the SMALLEST index.  Where the image holds no
 *     site at all, dist_sq = EDT_INF_SQ and feature = EDT_NO_SITE (the paper's
 *     "sufficiently large" initial value, Section 3.1).
 *   - Pointers are DEVICE pointers unless marked "host".  The caller allocates
 *     and owns all device memory (masks, outputs, workspaces); the library
 *     never allocates or frees it.  Handles (plans) are owned by the library
 *     and released by the caller through the matching destroy call.
 *   - stream is a hipStream_t passed as void* (NULL = the default stream).
 *     Work is enqueued on it asynchronously; arguments are validated
 *     synchronously before anything is enqueued, and an error leaves the
 *     outputs untouched.  A launch failure returns EDT_ERR_DEVICE.
 *   - No entry point aborts, throws or prints.
 */
#ifndef EDT_H
#define EDT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define EDT_ABI_VERSION 2

typedef int32_t edt_status;
#define EDT_OK 0
#define EDT_ERR_INVALID_ARG (-1)   /* null pointer, bad pitch, bad enum, short workspace */
#define EDT_ERR_UNSUPPORTED (-2)   /* reserved: a metric or output not provided */
#define EDT_ERR_TOO_LARGE (-3)     /* H or W outside [1, EDT_MAX_SIDE] */
#define EDT_ERR_OUT_OF_MEMORY (-4) /* a host or library-owned allocation failed */
#define EDT_ERR_BUSY (-5)          /* a server's memory budget or queue is full */
#define EDT_ERR_NOT_READY (-6)     /* a wait timed out; the work is still in flight */
#define EDT_ERR_DEVICE (-7)        /* a HIP call or kernel launch failed */

#define EDT_TO_OBJECT 0
#define EDT_TO_BACKGROUND 1

/* Metrics of the Minkowski family (Eq. eq_Minkowski, Section 1.3.1).  For the
 * squared Euclidean metric dist_sq holds d^2; for city-block (e = 1, d = |di| +
 * |dj|) and chessboard (e = infinity, d = max(|di|, |dj|)) it holds d itself.
 * Chamfer 4-3 (Section 1.3.2, Eq. eq_rel; its transform in Section 2.2): the
 * shortest path with steps of 3 horizontally and vertically and 4 diagonally,
 * d = 3 max(|di|, |dj|) + min(|di|, |dj|) -- three times the approximate
 * Euclidean distance, in integers. */
#define EDT_METRIC_EUCLIDEAN_SQ 0
#define EDT_METRIC_CITYBLOCK 1
#define EDT_METRIC_CHESSBOARD 2
#define EDT_METRIC_CHAMFER34 3

#define EDT_INF_SQ INT32_MAX /* dist_sq where the image has no site */
#define EDT_NO_SITE (-1)     /* feature where the image has no site */
#define EDT_MAX_SIDE 32767   /* row indices travel as int16 between passes */

/* Version of this ABI (EDT_ABI_VERSION of the build). */
int32_t edt_abi_version(void);

/* Static, human-readable name of a status code; never NULL. */
const char *edt_status_string(edt_status s);

/* Bytes of device workspace that edt_sq / edt_feature need for an H x W image
 * (the size does not depend on want_feature at present).  Returns 0 when H or
 * W is outside [1, EDT_MAX_SIDE]. */
size_t edt_workspace_bytes(int32_t H, int32_t W, int32_t want_feature);

/* Exact distance transform: squared Euclidean (Section 3: the vertical pass
 * of Section 3.1, then per row the lower envelope of parabolas of Section
 * 3.3.1, Eq. eq_parabola and Eq. eq_intersection), or city-block / chessboard
 * / chamfer 4-3 (the same two passes with the row costs |j - k| + |i - r|,
 * max(|j - k|, |i - r|) and 3 max + min of the two in place of the parabolas;
 * equal to the propagation scans of Section 2.1 for city-block and to the two
 * raster scans of Section 2.2 for chamfer 4-3).
 *   mask        device, uint8, H x W with row pitch mask_pitch bytes
 *   polarity    EDT_TO_OBJECT or EDT_TO_BACKGROUND
 *   metric      EDT_METRIC_EUCLIDEAN_SQ, _CITYBLOCK, _CHESSBOARD or _CHAMFER34
 *               (other values: EDT_ERR_INVALID_ARG)
 *   dist_sq     device, int32, H x W with row pitch out_pitch elements; written
 *   workspace   device, at least edt_workspace_bytes(H, W, 0) bytes, 256-byte
 *               aligned; contents on entry are ignored and on exit undefined
 * The workspace must not be shared by calls that may overlap in time. */
edt_status edt_sq(const uint8_t *mask, int32_t H, int32_t W, int64_t mask_pitch,
                  int32_t polarity, int32_t metric, int32_t *dist_sq,
                  int64_t out_pitch, void *workspace, size_t workspace_bytes,
                  void *stream);

/* Exact distance plus feature transform (the nearest site's index, Section
 * 3.3: the column that gives the minimum, extended with the site's row from
 * the vertical pass), for every metric.  Under the chessboard metric the
 * sites at the smallest distance D from a pixel are those of the square of
 * half-side D around it, and the feature is its topmost site, leftmost among
 * those (the smallest index).  Same arguments as edt_sq, plus
 *   dist_sq     may be NULL when only the features are wanted
 *   feature     device, int32, H x W with row pitch out_pitch elements; written */
edt_status edt_feature(const uint8_t *mask, int32_t H, int32_t W,
                       int64_t mask_pitch, int32_t polarity, int32_t metric,
                       int32_t *dist_sq, int32_t *feature, int64_t out_pitch,
                       void *workspace, size_t workspace_bytes, void *stream);

/* edt_feature without a workspace argument, for callers that cannot allocate
 * device memory (work under HIP graph capture, tight serving loops, harnesses
 * that forbid allocation).  The workspace is a static device array of
 * EDT_NOALLOC_SCRATCH_BYTES inside the library, one per device, held until the
 * process ends; its address is looked up on the first call on each device.
 * The call allocates nothing.  Same arguments, results and errors as
 * edt_feature, without workspace and workspace_bytes, plus
 * EDT_ERR_TOO_LARGE when edt_workspace_bytes(H, W, 1) exceeds
 * EDT_NOALLOC_SCRATCH_BYTES (a 4096 x 4096 image fits).  Every call on a device shares that device's array: calls
 * that may overlap in time on one device (two streams, two threads) race
 * and give undefined results.  As for edt_feature's workspace, the results do
 * not depend on the array's contents on entry, so what the previous call left
 * in it does not matter. */
#define EDT_NOALLOC_SCRATCH_BYTES (128u << 20)
edt_status edt_feature_noalloc(const uint8_t *mask, int32_t H, int32_t W,
                               int64_t mask_pitch, int32_t polarity, int32_t metric,
                               int32_t *dist_sq, int32_t *feature, int64_t out_pitch,
                               void *stream);

/* Voronoi regions of the objects (Section 1.1: after the transform each region
 * stands for one object point or one cluster of connected points, Figures
 * fig_voronoi and fig_blobs).  The sites are grouped into connected components
 * under the 4- or 8-neighbourhood of Section 1.2; every pixel gets the label of
 * the component holding its nearest site, a component's label being the
 * smallest linear index r*W + c of its sites.
 *   mask, H, W, mask_pitch, polarity   the image and its sites, as for
 *               edt_feature
 *   connectivity 4 or 8
 *   feature     device, int32, H x W with row pitch out_pitch elements: the
 *               feature transform of this mask and polarity (edt_feature's
 *               output, any metric); read only.  Other contents give
 *               unspecified labels but no access outside the buffers.
 *   labels      device, int32, H x W with row pitch out_pitch elements;
 *               written, EDT_NO_SITE where the image holds no site.  It holds
 *               the union-find forest of the sites during the call, so it may
 *               not overlap mask or feature (EDT_ERR_INVALID_ARG).
 * No workspace.  EDT_ERR_TOO_LARGE for sides outside [1, EDT_MAX_SIDE] or
 * H * out_pitch >= 2^31; EDT_ERR_INVALID_ARG for null pointers, pitches below
 * W, or a connectivity other than 4 or 8. */
edt_status edt_regions(const uint8_t *mask, int32_t H, int32_t W, int64_t mask_pitch,
                       int32_t polarity, int32_t connectivity, const int32_t *feature,
                       int32_t *labels, int64_t out_pitch, void *stream);

/* Danielsson's APPROXIMATE Euclidean transform (Section 2.3, the two-scan form
 * given after Grevera), for comparison with the exact one: every pixel holds
 * the relative position (dy, dx) propagated to it -- the magnitudes of the
 * offsets to the site it was reached from -- and dist_sq = dy^2 + dx^2, which
 * is never below the exact value and can exceed it where a site's Voronoi
 * region is disconnected.  The first scan visits rows 1 .. H-1 and the second
 * rows H-2 .. 0, so a one-row image propagates nothing.
 *   mask, H, W, mask_pitch, polarity   as for edt_sq; W <= 8192
 *   dist_sq     device, int32, H x W, row pitch out_pitch; written
 *               (EDT_INF_SQ where no position arrived)
 *   rel         device, int32, H x W, row pitch out_pitch; written:
 *               (dy << 16) | dx, or -1 where no position arrived; it holds
 *               the propagation state during the call and may not overlap
 *               dist_sq (EDT_ERR_INVALID_ARG)
 * One workgroup runs the two scans in order (the offers are a sequential
 * chain along each row): this is a comparison kernel, not a fast path.
 * EDT_ERR_TOO_LARGE for H outside [1, EDT_MAX_SIDE], W outside [1, 8192] or
 * more than 2^22 pixels (the sequential chain takes about 0.8 s per million
 * pixels). */
edt_status edt_danielsson(const uint8_t *mask, int32_t H, int32_t W, int64_t mask_pitch,
                          int32_t polarity, int32_t *dist_sq, int32_t *rel,
                          int64_t out_pitch, void *stream);

/* Euclidean distances in fp32 written by the row pass itself, with no second
 * pass over the output (Section 3.1 takes the square root once the squared
 * distances are known): dist holds the square root of the squared Euclidean
 * distance edt_sq computes, rounded exactly as edt_sqrt_f32 rounds it, and
 * +infinity where the image has no site.  Same arguments as edt_feature
 * without metric, with
 *   dist        device, fp32, H x W with row pitch out_pitch elements; written
 *   feature     device or NULL: int32 nearest-site indices, as edt_feature
 * Errors as edt_feature; EDT_ERR_INVALID_ARG when dist is NULL. */
edt_status edt_dist_f32(const uint8_t *mask, int32_t H, int32_t W, int64_t mask_pitch,
                        int32_t polarity, float *dist, int32_t *feature, int64_t out_pitch,
                        void *workspace, size_t workspace_bytes, void *stream);

/* d = sqrt(D) drawn after all squared distances are known (Section 3.1):
 * computed in fp64 and rounded to fp32 (the nearest fp32 to the true root for
 * every D < 2^31); EDT_INF_SQ maps to +infinity.  dist_sq and dist are device
 * arrays of n elements (they may not overlap). */
edt_status edt_sqrt_f32(const int32_t *dist_sq, float *dist, int64_t n,
                        void *stream);

/* ---- batches of images of uneven size ----------------------------------- */

/* One image of a batch.  Its mask starts mask_offset bytes after the batch's
 * mask base (rows mask_pitch bytes apart); its outputs start out_offset
 * elements after the batch's dist/feature bases (rows out_pitch elements
 * apart).  Images may have different sizes and polarities; the feature index
 * is local to the image (r*W + c). */
typedef struct {
    int64_t mask_offset;
    int64_t mask_pitch;
    int64_t out_offset;
    int64_t out_pitch;
    int32_t H, W;          /* 1 <= H <= EDT_MAX_SIDE, 1 <= W <= EDT_BATCH_MAX_W */
    int32_t polarity;      /* EDT_TO_OBJECT or EDT_TO_BACKGROUND */
    int32_t want_feature;  /* 0: this image's features are not written */
} edt_image_desc;

#define EDT_BATCH_MAX_W 16384  /* widest image of a batch */
#define EDT_BATCH_MAX_IMAGES (1 << 20)

typedef struct edt_plan edt_plan;

/* Plan a batch of n images (host array `images`).  The same transform as
 * edt_feature / edt_sq runs on every image; all images' phases run in one
 * persistent launch per phase over a table of the images (owned by the plan,
 * in device memory of the current device), and repeated submissions with the
 * same buffers replay a captured HIP graph.  want_dist = 0: no distances are
 * written (dist_base may then be NULL at submission); every image must then
 * have want_feature != 0, else EDT_ERR_INVALID_ARG (an image writes at least
 * one output).  *workspace_bytes (host)
 * receives the device workspace the submissions need.  The plan is not safe
 * for concurrent submissions from several threads.  Errors: EDT_ERR_TOO_LARGE
 * (a side, or the total of rows or work items, out of range),
 * EDT_ERR_INVALID_ARG, EDT_ERR_OUT_OF_MEMORY, EDT_ERR_DEVICE. */
edt_status edt_batch_plan(const edt_image_desc *images, int32_t n, int32_t want_dist,
                          edt_plan **plan, size_t *workspace_bytes);

/* Enqueue the batch on stream.  mask_base, dist_base, feat_base and workspace
 * are device pointers (feat_base may be NULL when no image wants features,
 * dist_base when the plan has want_dist = 0); the workspace is 256-byte
 * aligned, at least the planned size, and must not be shared with work that
 * may overlap.  Results are bit-identical to edt_feature / edt_sq on each
 * image alone. */
edt_status edt_batch_submit(edt_plan *plan, const uint8_t *mask_base, int32_t *dist_base,
                            int32_t *feat_base, void *workspace, size_t workspace_bytes,
                            void *stream);

/* How a batch is laid out on the GPU (host struct).  Results never depend on
 * it. */
typedef struct {
    int32_t lane_w;        /* widest image given the one-lane-per-row row pass,
                              0..1024 (that pass also takes only images of at
                              most 4096 rows) */
    int32_t largest_first; /* != 0: images listed by decreasing width, then
                              height, so that the longest work items start first */
    int32_t branches;      /* 1, or 2: the images split into two halves of about
                              equal area, each with its own table and launches,
                              the two launch sequences running side by side
                              (two branches of the captured graph) */
    int32_t wide_single;   /* != 0: images wider than 1024 columns run as single
                              transforms (the segment path of edt_feature) instead
                              of in the batch's row forms */
    int32_t transpose;     /* != 0: images wider than tall whose transpose takes
                              the one-lane-per-row pass (H <= lane_w, W <= 4096)
                              run as their transposes, the order of the two passes
                              exchanged (Section 3.2.1): the mask is copied
                              transposed into the workspace and the outputs
                              copied back */
} edt_schedule;

/* Result of edt_batch_autotune (host struct). */
#define EDT_TUNE_MAX 48
typedef struct {
    int32_t tried;                   /* candidate schedules timed */
    int32_t chosen;                  /* index of the one kept */
    edt_schedule cand[EDT_TUNE_MAX]; /* the candidates, in the order timed */
    float ms[EDT_TUNE_MAX];          /* best of three timed submissions */
} edt_tune_report;

/* Autotune the plan's schedule on these buffers (same arguments as
 * edt_batch_submit; the outputs are written, with the same values, by every
 * candidate).  Candidates: every combination of lane_w (0, 256, 1024, as the
 * batch's widths make them differ), largest_first (0, 1), branches (1, 2),
 * wide_single (0, 1) if some image is wider than 1024 columns, and
 * transpose (0, 1) if some image could run transposed.  Each is
 * run once untimed and three times timed with HIP events on `stream` (this
 * call waits for them); the fastest is kept for later submissions.  report
 * (host) may be NULL. */
edt_status edt_batch_autotune(edt_plan *plan, const uint8_t *mask_base, int32_t *dist_base,
                              int32_t *feat_base, void *workspace, size_t workspace_bytes,
                              void *stream, edt_tune_report *report);

/* Use the schedule *s (host) for later submissions, e.g. one that
 * edt_batch_autotune picked for batches of the same shapes.  Errors:
 * EDT_ERR_INVALID_ARG (a field out of range), EDT_ERR_OUT_OF_MEMORY,
 * EDT_ERR_DEVICE. */
edt_status edt_batch_set_schedule(edt_plan *plan, const edt_schedule *s);

/* Release a plan (its device tables and graphs).  Work already enqueued with
 * it must have completed. */
edt_status edt_plan_destroy(edt_plan *plan);

/* ---- serving: continuous batching of independent requests -------------- */

/* A server owns a scheduler thread and n_streams HIP streams of the current
 * device.  Requests (one image each, with caller-owned device mask and
 * outputs) queue in arrival order; whenever launch slots are free, the
 * scheduler admits the longest prefix of the queue whose workspaces fit in
 * the memory budget and launches it at once, as one batch (the persistent
 * launches of edt_batch_submit) or, for a lone request, as a single
 * transform; a request wider than 1024 columns is always launched alone (it
 * fills the GPU by itself).  Requests arriving meanwhile join the next
 * launch.  Workspaces are carved from a caller-owned device arena: a
 * request takes edt_workspace_bytes(H, W, 1) bytes, and, when max_group > 1
 * and the image is at most 1024 wide and 4096 tall, 4 more bytes per pixel
 * of its rows rounded up to 32 columns (the envelopes of the batch row pass),
 * each rounded up to 256 bytes.
 * Results are bit-identical to edt_feature / edt_sq on the request alone. */
typedef struct {
    size_t hbm_budget_bytes; /* arena bytes the server may hold at once for
                                admitted work (<= arena_bytes; 0: the whole arena) */
    int32_t max_inflight;    /* requests queued or running at once, >= 1;
                                one more is refused with EDT_ERR_BUSY */
    int32_t n_streams;       /* streams launched on, 1..EDT_SERVE_MAX_STREAMS */
    int32_t max_group;       /* most requests per launch, 1..EDT_SERVE_MAX_GROUP
                                (0: EDT_SERVE_MAX_GROUP) */
} edt_serve_config;

#define EDT_SERVE_MAX_STREAMS 16
#define EDT_SERVE_MAX_GROUP 1024

/* One request. */
typedef struct {
    const uint8_t *mask; /* device, H x W, rows mask_pitch bytes apart */
    int64_t mask_pitch;
    int32_t H, W;        /* 1 <= H, W <= EDT_MAX_SIDE */
    int32_t polarity;    /* EDT_TO_OBJECT or EDT_TO_BACKGROUND */
    int32_t reserved;    /* must be 0 */
    int32_t *dist_sq;    /* device or NULL: squared distances, out_pitch elements */
    int32_t *feature;    /* device or NULL (not both NULL): nearest-site indices */
    int64_t out_pitch;
    void *stream;        /* the mask is read only after the work enqueued on
                            this stream (NULL: the default stream) before the
                            submission; outputs are complete when the ticket
                            is done */
} edt_request;

typedef struct {
    uint64_t submitted;          /* accepted by edt_serve_submit */
    uint64_t rejected_busy;      /* refused with EDT_ERR_BUSY */
    uint64_t rejected_too_large; /* refused with EDT_ERR_TOO_LARGE */
    uint64_t done;               /* completed, successfully or not */
    uint64_t failed;             /* completed with an error */
    uint64_t launches;           /* groups launched */
    uint64_t pixels_done;        /* sum of H*W over the successful requests */
    double p50_ns, p99_ns, mean_ns, max_ns; /* latency, submission to observed
                                               completion: mean and max over
                                               every done request, p50 and p99
                                               over the last 65536 of them */
    double gpix_per_s;           /* pixels_done / (last completion - first submission) */
    size_t hbm_in_use;           /* arena bytes held by admitted requests now */
    size_t hbm_high_water;       /* most such bytes ever held at once */
} edt_serve_counters;

typedef struct edt_server edt_server;

/* Create a server on the current device.  cfg is host memory; arena is a
 * device buffer of arena_bytes (256-byte aligned) that the server uses as
 * workspace until edt_serve_destroy returns.  Errors: EDT_ERR_INVALID_ARG,
 * EDT_ERR_OUT_OF_MEMORY, EDT_ERR_DEVICE. */
edt_status edt_serve_create(const edt_serve_config *cfg, void *arena, size_t arena_bytes,
                            edt_server **out);

/* Bytes at the start of the arena that a server with this configuration keeps
 * for its launch tables (2 * n_streams tables of max_group images); they come
 * out of the memory budget.  0 for an invalid configuration. */
size_t edt_serve_reserved_bytes(const edt_serve_config *cfg);

/* Queue one request (host struct; its device buffers must stay valid until
 * the ticket is done).  *ticket (host) receives its ticket.  Errors:
 * EDT_ERR_INVALID_ARG or EDT_ERR_TOO_LARGE (also when the request alone needs
 * more than the memory budget), EDT_ERR_BUSY (max_inflight requests are
 * queued or running; retry later). */
edt_status edt_serve_submit(edt_server *s, const edt_request *r, uint64_t *ticket);

/* *done (host) = 1 once the ticket has completed, else 0.  Returns the
 * request's own status once done (EDT_OK, or EDT_ERR_DEVICE if its launch
 * failed), EDT_OK while it is pending, EDT_ERR_INVALID_ARG for an unknown
 * ticket.  Every ticket the server issued can be asked about for its whole
 * life; it keeps an entry per ticket only from the oldest one still in flight
 * on, plus one per failed ticket. */
edt_status edt_serve_poll(edt_server *s, uint64_t ticket, int32_t *done);

/* Block until the ticket completes (timeout_ns < 0: no limit) and return its
 * status; EDT_ERR_NOT_READY if the time ran out first. */
edt_status edt_serve_wait(edt_server *s, uint64_t ticket, int64_t timeout_ns);

/* Counters and latency percentiles so far (host struct). */
edt_status edt_serve_stats(edt_server *s, edt_serve_counters *out);

/* Finish all queued and running requests, then release the server's
 * threads, streams and host memory (not the arena).  Returns EDT_ERR_DEVICE
 * if any request failed. */
edt_status edt_serve_destroy(edt_server *s);

/* ---- kernel timing (observability) ------------------------------------ */

/* Total device time of one kernel of the library between edt_profile_begin
 * and edt_profile_end. */
typedef struct {
    char name[48];    /* kernel name, NUL-terminated */
    int64_t launches; /* launches timed */
    double total_ms;  /* summed event-to-event time on the launch streams */
} edt_kernel_time;

/* Start timing: from now on every kernel the library launches (from any
 * thread, on any stream) is bracketed by two HIP events recorded on its own
 * stream.  Clears earlier records. */
edt_status edt_profile_begin(void);

/* Stop timing, wait for the recorded events and write up to capacity per-kernel
 * totals to out (host); *count (host) receives the number of distinct kernels
 * timed.  Returns EDT_ERR_DEVICE if an event could not be read. */
edt_status edt_profile_end(edt_kernel_time *out, int32_t capacity, int32_t *count);

/* ---- testing ---------------------------------------------------------- */

/* Arm a launch failure, for tests of the error paths: the k-th kernel launch
 * of the library from now on (k >= 1, counted over all threads and entry
 * points) is not enqueued, nor is any later launch of the same call, and the
 * call reports the failure as a failed launch would (EDT_ERR_DEVICE; for a
 * served request, its ticket's status).  The failed call's outputs are
 * undefined; no kernel runs on state a skipped one should have written.  A
 * batch submission that replays a captured graph launches no kernel through
 * this path.  k = 0 disarms.  Errors: EDT_ERR_INVALID_ARG for k < 0. */
edt_status edt_debug_fail_launch(int32_t k);

#ifdef __cplusplus
}
#endif

#endif /* EDT_H */
