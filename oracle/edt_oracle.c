/*
 * edt_oracle.c -- plain, slow CPU oracle for the exact squared Euclidean
 * distance transform (EEDT) and its feature transform, written from
 * T. Strutz, "The Distance Transform and its Computation -- An Introduction"
 * (arXiv 2106.03503).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check of the graft
 * entry point and the cpu_baseline leg of bench.py may load this library.  It
 * shares no code, header, table or helper with the HIP library under
 * paper_2106_03503_amd/, and the product path never calls it.
 *
 * Conventions (0-based row i and column j; the paper's L columns are W here and
 * its M rows are H, see the notation table of Section 3):
 *   - A mask byte != 0 is an object pixel, 0 is background (Section 1.1: a
 *     binary image holds one of two values per pixel).
 *   - polarity 0: distances of every pixel to the nearest OBJECT pixel
 *     (Figure fig_examples(c)); polarity 1: distances to the nearest BACKGROUND
 *     pixel (Figure fig_examples(b)).  The pixels distances are measured to are
 *     called "sites" below; a site has distance 0 by definition (Section 2.1).
 *   - D is the squared distance d^2 (Eq. eq_squaredEuclid, Section 3.1).
 *   - F is the row-major linear index r*W + c of the nearest site (the
 *     assignment k* of Section 3.3 extended by the site row).  Where several
 *     sites are nearest, F is the smallest such index.
 *   - Where no site exists, D = INT32_MAX and F = -1: the paper only asks for a
 *     value larger than (M-1)^2 + (L-1)^2 (Section 3.1).
 *
 * Functions:
 *   oracle_brute         O1, the definition itself: every pixel against every
 *                        site (the naive approach opening Section 3).
 *   oracle_brute_at      O1 at a list of pixels, against the contour sites only.
 *   oracle_column_pass   the vertical pass of Section 3.1 (downward sweep, then
 *                        upward sweep), returning the nearest site row per pixel.
 *   oracle_row_envelope  the lower envelope of parabolas of Section 3.3.1 for
 *                        one row (Eq. eq_parabola and Eq. eq_intersection).
 *   oracle_separable     O2: column pass + envelope + fill (Section 3.3.1).
 *   oracle_basic_rows    O3: column pass + the basic O(M L^2) row pass of
 *                        Section 3.1 (every pixel against every column).
 *   oracle_sqrt_f32      d = sqrt(D) drawn after all squared distances are known
 *                        (Section 3.1), in fp64 then rounded to fp32.
 *   oracle_brute_metric  O1 for the city-block (e=1) and chessboard (e=inf)
 *                        members of the Minkowski family (Eq. eq_Minkowski),
 *                        and for the chamfer 4-3 metric (Section 1.3.2).
 *   oracle_brute_metric_at  the same at a list of pixels.
 *   oracle_cityblock_scans  the city-block transform by the four propagation
 *                        scans of Section 2.1 (columns down and up, then rows
 *                        forward and backward, one comparison per pixel each).
 *   oracle_chamfer_scans the chamfer 4-3 transform by the two raster scans of
 *                        Section 2.2 (four comparisons per pixel and scan).
 *   oracle_regions       Voronoi regions of the connected objects (Section
 *                        1.1 with the neighbourhoods of Section 1.2): the
 *                        component of each pixel's nearest site.
 *   oracle_danielsson    Danielsson's approximate transform by propagation of
 *                        relative positions, two scans (Section 2.3).
 *
 * Integer arithmetic is done in int64 throughout; nothing here is tuned.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#include <pthread.h>

#define ORACLE_INF_SQ INT32_MAX
#define ORACLE_NO_SITE (-1)

/* ------------------------------------------------------------------ sites */

/* Site predicate: object pixels for polarity 0, background pixels for
 * polarity 1 (Section 1.1, Figure fig_examples). */
static int is_site(uint8_t v, int32_t polarity)
{
    int object = (v != 0);
    return polarity ? !object : object;
}

typedef struct {
    int32_t r, c;
} site_t;

/* All sites in row-major order.  With contour_only, keep only sites that have
 * at least one 4-neighbour inside the image that is not a site (the "inner
 * contour" of Section 3).  Returns the count; *out is malloc'ed. */
static int64_t collect_sites(const uint8_t *mask, int32_t H, int32_t W,
                             int64_t pitch, int32_t polarity,
                             int32_t contour_only, site_t **out)
{
    int64_t n = 0;
    site_t *s = (site_t *)malloc(sizeof(site_t) * ((size_t)H * (size_t)W + 1));
    for (int32_t r = 0; r < H; ++r) {
        for (int32_t c = 0; c < W; ++c) {
            if (!is_site(mask[(int64_t)r * pitch + c], polarity))
                continue;
            if (contour_only) {
                int keep = 0;
                if (r > 0 && !is_site(mask[(int64_t)(r - 1) * pitch + c], polarity)) keep = 1;
                if (r + 1 < H && !is_site(mask[(int64_t)(r + 1) * pitch + c], polarity)) keep = 1;
                if (c > 0 && !is_site(mask[(int64_t)r * pitch + c - 1], polarity)) keep = 1;
                if (c + 1 < W && !is_site(mask[(int64_t)r * pitch + c + 1], polarity)) keep = 1;
                if (!keep)
                    continue;
            }
            s[n].r = r;
            s[n].c = c;
            ++n;
        }
    }
    *out = s;
    return n;
}

/* Nearest site of pixel (i, j): minimum of D, then of the linear index.  The
 * site list is in row-major order, so keeping the first strict minimum keeps
 * the smallest index among equal distances. */
static void nearest_of(const site_t *s, int64_t n, int32_t W, int32_t i,
                       int32_t j, int32_t *D, int32_t *F)
{
    int64_t best = -1;
    int64_t bestf = ORACLE_NO_SITE;
    for (int64_t q = 0; q < n; ++q) {
        int64_t di = (int64_t)i - s[q].r;
        int64_t dj = (int64_t)j - s[q].c;
        int64_t d = di * di + dj * dj;
        if (best < 0 || d < best) {
            best = d;
            bestf = (int64_t)s[q].r * W + s[q].c;
        }
    }
    *D = best < 0 ? ORACLE_INF_SQ : (int32_t)best;
    *F = (int32_t)bestf;
}

/* ------------------------------------------------------------ threading */

typedef void (*range_fn)(void *ctx, int64_t lo, int64_t hi);
typedef struct {
    range_fn fn;
    void *ctx;
    int64_t lo, hi;
} range_job;

static void *range_thread(void *p)
{
    range_job *j = (range_job *)p;
    j->fn(j->ctx, j->lo, j->hi);
    return NULL;
}

/* Split [0, n) into nthreads contiguous ranges and run fn on each. */
static void parallel_for(int64_t n, int32_t nthreads, range_fn fn, void *ctx)
{
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    if ((int64_t)nthreads > n) nthreads = (int32_t)(n > 0 ? n : 1);
    if (nthreads == 1) {
        fn(ctx, 0, n);
        return;
    }
    pthread_t th[256];
    range_job jobs[256];
    for (int32_t t = 0; t < nthreads; ++t) {
        jobs[t].fn = fn;
        jobs[t].ctx = ctx;
        jobs[t].lo = n * t / nthreads;
        jobs[t].hi = n * (t + 1) / nthreads;
        pthread_create(&th[t], NULL, range_thread, &jobs[t]);
    }
    for (int32_t t = 0; t < nthreads; ++t)
        pthread_join(th[t], NULL);
}

/* ------------------------------------------------------------------- O1 */

typedef struct {
    const uint8_t *mask;
    int64_t pitch;
    int32_t H, W, polarity, contour_only;
    const site_t *s;
    int64_t n;
    const int64_t *lin;
    int32_t *D, *F;
} brute_ctx;

static void brute_rows(void *p, int64_t lo, int64_t hi)
{
    brute_ctx *b = (brute_ctx *)p;
    for (int64_t i = lo; i < hi; ++i) {
        for (int32_t j = 0; j < b->W; ++j) {
            int64_t o = i * b->W + j;
            if (b->contour_only && is_site(b->mask[i * b->pitch + j], b->polarity)) {
                b->D[o] = 0; /* a site is its own nearest site */
                b->F[o] = (int32_t)o;
                continue;
            }
            nearest_of(b->s, b->n, b->W, (int32_t)i, j, &b->D[o], &b->F[o]);
        }
    }
}

/* O1: for every pixel, the minimum over ALL sites of (D, F).  With
 * contour_only, sites whose in-image 4-neighbours are all sites are skipped:
 * from such a site q, the neighbour one step towards any other pixel p along
 * an axis where p and q differ is also a site and strictly closer to p, so q
 * is never nearest to a pixel other than itself.  D and F are H x W, row-major,
 * contiguous.  Returns the number of sites used. */
int64_t oracle_brute(const uint8_t *mask, int32_t H, int32_t W, int64_t pitch,
                     int32_t polarity, int32_t contour_only, int32_t nthreads,
                     int32_t *D, int32_t *F)
{
    site_t *s = NULL;
    int64_t n = collect_sites(mask, H, W, pitch, polarity, contour_only, &s);
    brute_ctx b = {mask, pitch, H, W, polarity, contour_only, s, n, NULL, D, F};
    parallel_for(H, nthreads, brute_rows, &b);
    free(s);
    return n;
}

static void brute_points(void *p, int64_t lo, int64_t hi)
{
    brute_ctx *b = (brute_ctx *)p;
    for (int64_t q = lo; q < hi; ++q) {
        int64_t o = b->lin[q];
        int32_t i = (int32_t)(o / b->W), j = (int32_t)(o % b->W);
        if (is_site(b->mask[(int64_t)i * b->pitch + j], b->polarity)) {
            b->D[q] = 0;
            b->F[q] = (int32_t)o;
            continue;
        }
        nearest_of(b->s, b->n, b->W, i, j, &b->D[q], &b->F[q]);
    }
}

/* O1 at n selected pixels given by their linear indices lin[q] = i*W + j,
 * against the contour sites (exact, see oracle_brute).  Returns the number of
 * contour sites. */
int64_t oracle_brute_at(const uint8_t *mask, int32_t H, int32_t W, int64_t pitch,
                        int32_t polarity, const int64_t *lin, int64_t n,
                        int32_t nthreads, int32_t *D, int32_t *F)
{
    site_t *s = NULL;
    int64_t ns = collect_sites(mask, H, W, pitch, polarity, 1, &s);
    brute_ctx b = {mask, pitch, H, W, polarity, 1, s, ns, lin, D, F};
    parallel_for(n, nthreads, brute_points, &b);
    free(s);
    return ns;
}

/* ------------------------------------------------------- column pass (3.1) */

typedef struct {
    const uint8_t *mask;
    int64_t pitch;
    int32_t H, W, polarity, sweeps;
    int32_t *R;  /* nearest site row per pixel, -1 = none */
    int64_t *Dv; /* squared vertical distance, -1 = "infinity" */
} col_ctx;

static void column_range(void *p, int64_t lo, int64_t hi)
{
    col_ctx *c = (col_ctx *)p;
    const int32_t H = c->H, W = c->W;
    for (int64_t j = lo; j < hi; ++j) {
        /* Downward sweep: a site resets the distance to 0; otherwise the value
         * of the pixel above grows by the odd step 2x+1, x being the distance
         * reached so far ((x+1)^2 - x^2 = 2x+1), and the source row is carried
         * along. */
        for (int32_t i = 0; i < H; ++i) {
            int64_t o = (int64_t)i * W + j;
            if (is_site(c->mask[(int64_t)i * c->pitch + j], c->polarity)) {
                c->R[o] = i;
                c->Dv[o] = 0;
            } else if (i > 0 && c->R[o - W] >= 0) {
                int64_t x = (int64_t)(i - 1) - c->R[o - W];
                c->R[o] = c->R[o - W];
                c->Dv[o] = c->Dv[o - W] + 2 * x + 1;
            } else {
                c->R[o] = -1;
                c->Dv[o] = -1;
            }
        }
        if (c->sweeps < 2)
            continue;
        /* Upward sweep: the nearest site at or below each pixel replaces the
         * downward value only when it is strictly nearer, so an upper site
         * keeps equal distances. */
        int32_t below = -1;
        for (int32_t i = H - 1; i >= 0; --i) {
            int64_t o = (int64_t)i * W + j;
            if (is_site(c->mask[(int64_t)i * c->pitch + j], c->polarity))
                below = i;
            if (below < 0)
                continue;
            int64_t db = (int64_t)below - i;
            if (c->Dv[o] < 0 || c->Dv[o] > db * db) {
                c->R[o] = below;
                c->Dv[o] = db * db;
            }
        }
    }
}

/* Vertical pass of Section 3.1 on an H x W mask: for every pixel, the row of
 * the nearest site in its own column (R, -1 if the column has none) and the
 * squared vertical distance Dv (-1 for "infinity").  sweeps = 1 stops after the
 * downward sweep (Figure fig_EEDT2); sweeps = 2 adds the upward sweep (Figure
 * fig_EEDT(b)).  R and Dv are H x W, row-major, contiguous. */
void oracle_column_pass(const uint8_t *mask, int32_t H, int32_t W, int64_t pitch,
                        int32_t polarity, int32_t sweeps, int32_t nthreads,
                        int32_t *R, int64_t *Dv)
{
    col_ctx c = {mask, pitch, H, W, polarity, sweeps, R, Dv};
    parallel_for(W, nthreads, column_range, &c);
}

/* ------------------------------------------------- row envelope (3.3.1) */

/* floor(a / b) for b > 0, rounding towards minus infinity. */
static int64_t floor_div(int64_t a, int64_t b)
{
    int64_t q = a / b;
    if ((a % b != 0) && (a < 0))
        --q;
    return q;
}

/* First pixel position j at which parabola l (vertex column l > k) beats
 * parabola k in a row, for the tie rule:
 *   rule 0: at equal D the smaller linear index R*W + column wins;
 *   rule 1: at equal D the parabola further right wins (what rounding the
 *           intersection up gives in the paper's fast algorithm).
 * The two parabolas cross at j_s = (Dv_l - Dv_k - k^2 + l^2) / (2 (l - k))
 * (Eq. eq_intersection); l is strictly better for j > j_s and equal at j_s. */
static int64_t first_win(const int64_t *Dv, const int32_t *R, int32_t W,
                         int32_t rule, int32_t k, int32_t l)
{
    int64_t num = Dv[l] - Dv[k] - (int64_t)k * k + (int64_t)l * l;
    int64_t den = 2 * (int64_t)(l - k);
    int l_wins_tie;
    if (rule == 1) {
        l_wins_tie = 1;
    } else {
        int64_t fk = (int64_t)R[k] * W + k, fl = (int64_t)R[l] * W + l;
        l_wins_tie = fl < fk;
    }
    /* l wins at integer j iff j*den > num, or j*den == num and l wins ties. */
    if (l_wins_tie)
        return -floor_div(-num, den); /* ceil(num / den) */
    return floor_div(num, den) + 1;
}

/* Lower envelope of the parabolas Dv[k] + (j - k)^2 (Eq. eq_parabola) over
 * the columns k with finite Dv[k], for one row of width W (Section 3.3.1).
 * The columns are visited from left to right; a new parabola hides the
 * parabola on top of the stack when it already wins at the first pixel that
 * parabola owns, and is stored only if it wins somewhere inside the row.
 * Writes the contributing columns ks[0..n) and the first pixel each owns
 * js[0..n) (js[0] = 0; contributor e owns [js[e], js[e+1]) and the last owns
 * up to W - 1).  Returns n (0 when no column has a finite Dv). */
int32_t oracle_row_envelope(const int64_t *Dv, const int32_t *R, int32_t W,
                            int32_t rule, int32_t *ks, int32_t *js)
{
    int32_t n = 0;
    for (int32_t m = 0; m < W; ++m) {
        if (Dv[m] < 0)
            continue; /* columns without any site cannot contribute (3.2.2) */
        int64_t s = 0;
        while (n > 0) {
            s = first_win(Dv, R, W, rule, ks[n - 1], m);
            if (s <= js[n - 1])
                --n; /* the new parabola hides the previous one */
            else
                break;
        }
        if (n == 0) {
            ks[0] = m;
            js[0] = 0;
            n = 1;
        } else if (s <= W - 1) {
            ks[n] = m;
            js[n] = (int32_t)s;
            ++n;
        }
    }
    return n;
}

/* ------------------------------------------------------------------- O2 */

typedef struct {
    int32_t H, W;
    const int32_t *R;
    const int64_t *Dv;
    int32_t *D, *F;
    int32_t basic; /* 1: O3 basic row pass instead of the envelope */
} row_ctx;

static void row_range(void *p, int64_t lo, int64_t hi)
{
    row_ctx *c = (row_ctx *)p;
    const int32_t W = c->W;
    int32_t *ks = (int32_t *)malloc(sizeof(int32_t) * (size_t)W);
    int32_t *js = (int32_t *)malloc(sizeof(int32_t) * (size_t)W);
    for (int64_t i = lo; i < hi; ++i) {
        const int64_t *dv = c->Dv + i * W;
        const int32_t *r = c->R + i * W;
        int32_t *D = c->D + i * W, *F = c->F + i * W;
        if (c->basic) {
            /* Section 3.1: every pixel j against every column k. */
            for (int32_t j = 0; j < W; ++j) {
                int64_t best = -1, bestf = -1;
                for (int32_t k = 0; k < W; ++k) {
                    if (dv[k] < 0)
                        continue;
                    int64_t d = dv[k] + (int64_t)(k - j) * (k - j);
                    int64_t f = (int64_t)r[k] * W + k;
                    if (best < 0 || d < best || (d == best && f < bestf)) {
                        best = d;
                        bestf = f;
                    }
                }
                D[j] = best < 0 ? ORACLE_INF_SQ : (int32_t)best;
                F[j] = (int32_t)bestf;
            }
            continue;
        }
        int32_t n = oracle_row_envelope(dv, r, W, 0, ks, js);
        if (n == 0) {
            for (int32_t j = 0; j < W; ++j) {
                D[j] = ORACLE_INF_SQ;
                F[j] = ORACLE_NO_SITE;
            }
            continue;
        }
        /* Second scan: each contributor fills the pixels it owns (Eq.
         * eq_parabola). */
        for (int32_t e = 0; e < n; ++e) {
            int32_t k = ks[e];
            int32_t end = (e + 1 < n) ? js[e + 1] : W;
            for (int32_t j = js[e]; j < end; ++j) {
                D[j] = (int32_t)(dv[k] + (int64_t)(j - k) * (j - k));
                F[j] = r[k] * W + k;
            }
        }
    }
    free(ks);
    free(js);
}

static void separable_common(const uint8_t *mask, int32_t H, int32_t W,
                             int64_t pitch, int32_t polarity, int32_t nthreads,
                             int32_t basic, int32_t *D, int32_t *F)
{
    int32_t *R = (int32_t *)malloc(sizeof(int32_t) * (size_t)H * (size_t)W);
    int64_t *Dv = (int64_t *)malloc(sizeof(int64_t) * (size_t)H * (size_t)W);
    oracle_column_pass(mask, H, W, pitch, polarity, 2, nthreads, R, Dv);
    row_ctx c = {H, W, R, Dv, D, F, basic};
    parallel_for(H, nthreads, row_range, &c);
    free(R);
    free(Dv);
}

/* O2: the separable exact EDT of Section 3: vertical pass, then per row the
 * lower envelope of parabolas and the fill from it (Section 3.3.1), with ties
 * going to the smallest linear index.  Columns, then rows, are split over
 * nthreads POSIX threads.  D and F are H x W, row-major, contiguous. */
void oracle_separable(const uint8_t *mask, int32_t H, int32_t W, int64_t pitch,
                      int32_t polarity, int32_t nthreads, int32_t *D, int32_t *F)
{
    separable_common(mask, H, W, pitch, polarity, nthreads, 0, D, F);
}

/* O3: vertical pass, then the basic row pass of Section 3.1 in which every
 * pixel is compared with every column (O(M L^2)). */
void oracle_basic_rows(const uint8_t *mask, int32_t H, int32_t W, int64_t pitch,
                       int32_t polarity, int32_t nthreads, int32_t *D, int32_t *F)
{
    separable_common(mask, H, W, pitch, polarity, nthreads, 1, D, F);
}

/* ------------------------------------------------------------- sqrt (3.1) */

/* d = sqrt(D) once all squared distances are known (Section 3.1): computed in
 * fp64 and rounded to fp32; the "no site" value maps to +infinity. */
void oracle_sqrt_f32(const int32_t *D, int64_t n, float *out)
{
    for (int64_t q = 0; q < n; ++q)
        out[q] = (D[q] == ORACLE_INF_SQ) ? (float)INFINITY : (float)sqrt((double)D[q]);
}

/* ------------------------------------------------- other Minkowski metrics */

/* O1 for the other exact members of the Minkowski family (Eq. eq_Minkowski):
 * metric 1 = city-block (e = 1), metric 2 = chessboard (e = infinity); and
 * metric 3 = the chamfer 4-3 distance of Section 1.3.2, the length of the
 * shortest 8-connected path when a horizontal or vertical step costs 3 and a
 * diagonal step 4 (Eq. eq_rel scaled by 3): min(di, dj) diagonal steps and
 * max - min straight ones.  D is the distance itself (not squared); F the
 * smallest linear index among the nearest sites.  Returns the number of
 * sites. */
static void metric_nearest(const site_t *s, int64_t n, int32_t W, int32_t metric,
                           int32_t i, int32_t j, int32_t *D, int32_t *F)
{
    int64_t best = -1, bestf = -1;
    for (int64_t q = 0; q < n; ++q) {
        int64_t di = llabs((int64_t)i - s[q].r);
        int64_t dj = llabs((int64_t)j - s[q].c);
        int64_t lo = di < dj ? di : dj, hi = di < dj ? dj : di;
        int64_t d = (metric == 1) ? di + dj
                  : (metric == 2) ? hi
                                  : 4 * lo + 3 * (hi - lo);
        if (best >= 0 && d >= best)
            continue; /* sites come in row-major order: the first of equals stays */
        best = d;
        bestf = (int64_t)s[q].r * W + s[q].c;
    }
    *D = best < 0 ? ORACLE_INF_SQ : (int32_t)best;
    *F = (int32_t)bestf;
}

int64_t oracle_brute_metric(const uint8_t *mask, int32_t H, int32_t W,
                            int64_t pitch, int32_t polarity, int32_t metric,
                            int32_t *D, int32_t *F)
{
    site_t *s = NULL;
    int64_t n = collect_sites(mask, H, W, pitch, polarity, 0, &s);
    for (int32_t i = 0; i < H; ++i)
        for (int32_t j = 0; j < W; ++j) {
            const int64_t o = (int64_t)i * W + j;
            metric_nearest(s, n, W, metric, i, j, &D[o], &F[o]);
        }
    free(s);
    return n;
}

typedef struct {
    const site_t *s;
    int64_t n;
    int32_t W, metric;
    const int64_t *lin;
    int32_t *D, *F;
} metric_at_ctx;

static void metric_points(void *p, int64_t lo, int64_t hi)
{
    metric_at_ctx *b = (metric_at_ctx *)p;
    for (int64_t q = lo; q < hi; ++q) {
        const int64_t o = b->lin[q];
        metric_nearest(b->s, b->n, b->W, b->metric, (int32_t)(o / b->W), (int32_t)(o % b->W),
                       &b->D[q], &b->F[q]);
    }
}

/* The same definition at n selected pixels with linear indices lin[q] = i*W + j
 * (every site compared, as in oracle_brute_metric).  Returns the number of
 * sites. */
int64_t oracle_brute_metric_at(const uint8_t *mask, int32_t H, int32_t W, int64_t pitch,
                               int32_t polarity, int32_t metric, const int64_t *lin,
                               int64_t n, int32_t nthreads, int32_t *D, int32_t *F)
{
    site_t *s = NULL;
    int64_t ns = collect_sites(mask, H, W, pitch, polarity, 0, &s);
    metric_at_ctx b = {s, ns, W, metric, lin, D, F};
    parallel_for(n, nthreads, metric_points, &b);
    free(s);
    return ns;
}

/* City-block distance transform by the four one-comparison scans of Section
 * 2.1: initialise sites with 0 and every other pixel with a value above any
 * possible distance; then in every column a downward scan (d(i,j) > d(i-1,j)+1
 * lowers d(i,j)) and an upward scan (same with d(i+1,j)); then in every row a
 * forward scan (with d(i,j-1)) and a backward scan (with d(i,j+1)).  stages = 2
 * stops after the two column scans (the vertical distances of Figure
 * fig_cityblockDTparallel(b)), stages = 4 runs all four.  Cells that keep the
 * initial value (no site reachable) come out as INT32_MAX. */
void oracle_cityblock_scans(const uint8_t *mask, int32_t H, int32_t W, int64_t pitch,
                            int32_t polarity, int32_t stages, int32_t *D)
{
    const int64_t big = (int64_t)H + W; /* above (H-1) + (W-1) */
    int64_t *d = (int64_t *)malloc(sizeof(int64_t) * (size_t)H * (size_t)W);
    for (int32_t i = 0; i < H; ++i)
        for (int32_t j = 0; j < W; ++j)
            d[(int64_t)i * W + j] = is_site(mask[(int64_t)i * pitch + j], polarity) ? 0 : big;
    for (int32_t j = 0; j < W; ++j) {
        for (int32_t i = 1; i < H; ++i) { /* downward */
            int64_t *c = &d[(int64_t)i * W + j], up = d[(int64_t)(i - 1) * W + j];
            if (*c > up + 1) *c = up + 1;
        }
        for (int32_t i = H - 2; i >= 0; --i) { /* upward */
            int64_t *c = &d[(int64_t)i * W + j], dn = d[(int64_t)(i + 1) * W + j];
            if (*c > dn + 1) *c = dn + 1;
        }
    }
    if (stages >= 4) {
        for (int32_t i = 0; i < H; ++i) {
            int64_t *row = &d[(int64_t)i * W];
            for (int32_t j = 1; j < W; ++j) /* forward */
                if (row[j] > row[j - 1] + 1) row[j] = row[j - 1] + 1;
            for (int32_t j = W - 2; j >= 0; --j) /* backward */
                if (row[j] > row[j + 1] + 1) row[j] = row[j + 1] + 1;
        }
    }
    for (int64_t q = 0; q < (int64_t)H * W; ++q)
        D[q] = d[q] >= big ? ORACLE_INF_SQ : (int32_t)d[q];
    free(d);
}

/* Chamfer 4-3 distance transform by the two raster scans of Section 2.2, all
 * distances scaled by 3 (Eq. eq_rel: steps of 3 horizontally and vertically,
 * 4 diagonally).  Sites start at 0 and every other pixel above any reachable
 * distance.  The forward scan takes the rows top-down and each row left to
 * right, and lowers d(i,j) to d(i,j-1)+3, d(i-1,j)+3, d(i-1,j-1)+4 and
 * d(i-1,j+1)+4 in turn where that is smaller; the backward scan takes the rows
 * bottom-up and each row right to left with d(i,j+1)+3, d(i+1,j)+3,
 * d(i+1,j-1)+4 and d(i+1,j+1)+4.  passes = 1 stops after the forward scan
 * (Figure fig_chamfer43DT(a)), passes = 2 gives the transform (Figure
 * fig_chamfer43DT(b)).  Pixels no site reaches come out as INT32_MAX. */
void oracle_chamfer_scans(const uint8_t *mask, int32_t H, int32_t W, int64_t pitch,
                          int32_t polarity, int32_t passes, int32_t *D)
{
    const int64_t big = 4 * ((int64_t)H + W); /* above 4 (H-1) + 3 (W-1) and the mirror */
    int64_t *d = (int64_t *)malloc(sizeof(int64_t) * (size_t)H * (size_t)W);
#define AT(i, j) d[(int64_t)(i) * W + (j)]
#define LOWER(i, j, v) do { if (AT(i, j) > (v)) AT(i, j) = (v); } while (0)
    for (int32_t i = 0; i < H; ++i)
        for (int32_t j = 0; j < W; ++j)
            AT(i, j) = is_site(mask[(int64_t)i * pitch + j], polarity) ? 0 : big;
    for (int32_t i = 0; i < H; ++i) { /* forward: top-left to bottom-right */
        for (int32_t j = 0; j < W; ++j) {
            if (j > 0) LOWER(i, j, AT(i, j - 1) + 3);
            if (i > 0) LOWER(i, j, AT(i - 1, j) + 3);
            if (i > 0 && j > 0) LOWER(i, j, AT(i - 1, j - 1) + 4);
            if (i > 0 && j + 1 < W) LOWER(i, j, AT(i - 1, j + 1) + 4);
        }
    }
    if (passes >= 2) {
        for (int32_t i = H - 1; i >= 0; --i) { /* backward: bottom-right to top-left */
            for (int32_t j = W - 1; j >= 0; --j) {
                if (j + 1 < W) LOWER(i, j, AT(i, j + 1) + 3);
                if (i + 1 < H) LOWER(i, j, AT(i + 1, j) + 3);
                if (i + 1 < H && j > 0) LOWER(i, j, AT(i + 1, j - 1) + 4);
                if (i + 1 < H && j + 1 < W) LOWER(i, j, AT(i + 1, j + 1) + 4);
            }
        }
    }
#undef LOWER
#undef AT
    for (int64_t q = 0; q < (int64_t)H * W; ++q)
        D[q] = d[q] >= big ? ORACLE_INF_SQ : (int32_t)d[q];
    free(d);
}

/* ------------------------------------------------------- region labels */

/* Voronoi regions of the objects (Section 1.1: after the transform each region
 * stands for one object point or one cluster of connected points, Figures
 * fig_voronoi and fig_blobs).  The sites are grouped into connected components
 * under the 4- or the 8-neighbourhood of Section 1.2 by a breadth-first flood
 * fill started from each unlabelled site in raster order, so that a
 * component's label is the linear index r*W + c of its first site in raster
 * order, the smallest.  Every pixel then takes the label of the component
 * that holds its nearest site F (the feature transform); pixels of an image
 * without sites (F = -1) get -1.  F is row-major with row pitch W. */
void oracle_regions(const uint8_t *mask, int32_t H, int32_t W, int64_t pitch,
                    int32_t polarity, int32_t connectivity, const int32_t *F,
                    int32_t *labels)
{
    const int64_t n = (int64_t)H * W;
    int32_t *comp = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int64_t *queue = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    for (int64_t q = 0; q < n; ++q) comp[q] = -1;
    for (int32_t i0 = 0; i0 < H; ++i0) {
        for (int32_t j0 = 0; j0 < W; ++j0) {
            const int64_t start = (int64_t)i0 * W + j0;
            if (comp[start] >= 0 || !is_site(mask[(int64_t)i0 * pitch + j0], polarity)) continue;
            int64_t head = 0, tail = 0;
            comp[start] = (int32_t)start;
            queue[tail++] = start;
            while (head < tail) {
                const int64_t cur = queue[head++];
                const int32_t i = (int32_t)(cur / W), j = (int32_t)(cur % W);
                for (int32_t di = -1; di <= 1; ++di) {
                    for (int32_t dj = -1; dj <= 1; ++dj) {
                        if (di == 0 && dj == 0) continue;
                        if (connectivity == 4 && di != 0 && dj != 0) continue;
                        const int32_t a = i + di, b = j + dj;
                        if (a < 0 || a >= H || b < 0 || b >= W) continue;
                        const int64_t nb = (int64_t)a * W + b;
                        if (comp[nb] >= 0 || !is_site(mask[(int64_t)a * pitch + b], polarity)) continue;
                        comp[nb] = (int32_t)start;
                        queue[tail++] = nb;
                    }
                }
            }
        }
    }
    for (int64_t q = 0; q < n; ++q) labels[q] = F[q] < 0 ? -1 : comp[F[q]];
    free(queue);
    free(comp);
}

/* ------------------------------------------------------------ Danielsson */

/* Danielsson's approximate transform in the two-scan form of Section 2.3 (after
 * Grevera): every pixel keeps a relative position (dy, dx) -- magnitudes of
 * the vertical and horizontal offset to the site it was reached from -- and
 * d^2 = dy^2 + dx^2.  Sites start at (0, 0), every other pixel unreached.  A
 * neighbour that has been reached offers its position with one added to dy
 * for a vertical step, to dx for a horizontal step and to both for a diagonal
 * one; the pixel takes the offer when it is strictly nearer than what it
 * holds.  The first scan takes the rows from the second one down: per row,
 * first every pixel's upper neighbour, then left to right the left and the
 * upper-left neighbour, then right to left the upper-right and the right
 * neighbour.  The second scan takes the rows from the second-last one up,
 * mirrored: every pixel's lower neighbour, then left to right the left and
 * the lower-left neighbour, then right to left the right and the lower-right
 * neighbour.  passes = 1 stops after the first scan (Figure
 * fig_DanielssonDT(b)), passes = 2 gives the result (Figure
 * fig_DanielssonDT(c)).  Outputs: D = d^2 (INT32_MAX where unreached) and
 * R = (dy << 16) | dx (-1 where unreached), row-major with pitch W. */
static void dan_offer(int64_t *d, int32_t *y, int32_t *x, int64_t to, int64_t from,
                      int32_t ay, int32_t ax)
{
    if (y[from] < 0) return; /* nothing to propagate */
    const int32_t ny = y[from] + ay, nx = x[from] + ax;
    const int64_t nd = (int64_t)ny * ny + (int64_t)nx * nx;
    if (d[to] > nd) {
        d[to] = nd;
        y[to] = ny;
        x[to] = nx;
    }
}

void oracle_danielsson(const uint8_t *mask, int32_t H, int32_t W, int64_t pitch,
                       int32_t polarity, int32_t passes, int32_t *D, int32_t *R)
{
    const int64_t n = (int64_t)H * W;
    const int64_t unreached = INT64_MAX;
    int64_t *d = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    int32_t *y = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int32_t *x = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    for (int32_t i = 0; i < H; ++i)
        for (int32_t j = 0; j < W; ++j) {
            const int64_t o = (int64_t)i * W + j;
            const int s = is_site(mask[(int64_t)i * pitch + j], polarity);
            d[o] = s ? 0 : unreached;
            y[o] = s ? 0 : -1;
            x[o] = s ? 0 : -1;
        }
#define P(i, j) ((int64_t)(i) * W + (j))
    for (int32_t i = 1; i < H; ++i) { /* first scan, downwards */
        for (int32_t j = 0; j < W; ++j) dan_offer(d, y, x, P(i, j), P(i - 1, j), 1, 0);
        for (int32_t j = 1; j < W; ++j) {
            dan_offer(d, y, x, P(i, j), P(i, j - 1), 0, 1);
            dan_offer(d, y, x, P(i, j), P(i - 1, j - 1), 1, 1);
        }
        for (int32_t j = W - 2; j >= 0; --j) {
            dan_offer(d, y, x, P(i, j), P(i - 1, j + 1), 1, 1);
            dan_offer(d, y, x, P(i, j), P(i, j + 1), 0, 1);
        }
    }
    if (passes >= 2) {
        for (int32_t i = H - 2; i >= 0; --i) { /* second scan, upwards */
            for (int32_t j = 0; j < W; ++j) dan_offer(d, y, x, P(i, j), P(i + 1, j), 1, 0);
            for (int32_t j = 1; j < W; ++j) {
                dan_offer(d, y, x, P(i, j), P(i, j - 1), 0, 1);
                dan_offer(d, y, x, P(i, j), P(i + 1, j - 1), 1, 1);
            }
            for (int32_t j = W - 2; j >= 0; --j) {
                dan_offer(d, y, x, P(i, j), P(i, j + 1), 0, 1);
                dan_offer(d, y, x, P(i, j), P(i + 1, j + 1), 1, 1);
            }
        }
    }
#undef P
    for (int64_t o = 0; o < n; ++o) {
        D[o] = y[o] < 0 ? ORACLE_INF_SQ : (int32_t)d[o];
        R[o] = y[o] < 0 ? -1 : (int32_t)(((uint32_t)y[o] << 16) | (uint32_t)x[o]);
    }
    free(x);
    free(y);
    free(d);
}
