/*
 * isoclust.h -- C ABI of the MI355X (gfx950) library for the data-parallel hot
 * path of "An Efficient Parallel Data Clustering Algorithm Using Isoperimetric
 * Number of Trees" (Javadi & Ashkboos, arXiv 1702.04739):
 *
 *   iso_mst           Euclidean minimum spanning tree of n points in R^d
 *                     (Sec. 2.2 step 2, Sec. 3.5), returned as the paper's
 *                     "parent list" (Sec. 3.3): parent[] and edge lengths.
 *   iso_subpartition  the tree's optimal k-subpartition and the k-th
 *                     isoperimetric number MISO_k(T) (eqs. 2.4 and 2.6), by the
 *                     decision procedure of Algorithm 1 inside the bisection of
 *                     Algorithm 2, labelled as in Algorithm 4.
 *   iso_backward      gradient of the total tree length and of the optimal
 *                     subpartition's cost with respect to the points and sigma,
 *                     with the tree and the subpartition held fixed.
 *
 * Conventions for every entry point:
 *   - Pointers are DEVICE pointers unless marked (host).  Device buffers are
 *     owned by the caller; the library never frees them and keeps no state
 *     between calls.
 *   - Work is enqueued on `stream` (a hipStream_t; NULL = the null stream).
 *     An entry point that writes a (host) result synchronises `stream` before
 *     it returns; the others return once their work is enqueued.
 *   - Vertex ids are int32 (n < 2^31).  Points are FP32, row-major, row stride
 *     `ld` elements (ld >= d).
 *   - Every argument is validated before any device work is enqueued.  On
 *     error the return value is negative, device outputs are unspecified, and
 *     iso_last_error() describes the failure.
 *   - Workspace: pass ws = NULL to let the library allocate (hipMallocAsync on
 *     `stream`, freed before return), or a device buffer of at least the size
 *     the matching *_workspace_size call reports (else ISO_ERR_WORKSPACE).
 */
#ifndef ISOCLUST_H
#define ISOCLUST_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t iso_status;
#define ISO_OK 0
#define ISO_ERR_INVALID_ARG (-1)  /* argument outside its documented domain        */
#define ISO_ERR_NONFINITE (-2)    /* a point coordinate is NaN or infinite          */
#define ISO_ERR_NO_DEVICE (-3)    /* no usable gfx950 device                        */
#define ISO_ERR_HIP (-4)          /* a HIP runtime call failed                      */
#define ISO_ERR_OOM (-5)          /* device allocation failed                       */
#define ISO_ERR_WORKSPACE (-6)    /* caller workspace smaller than required         */
#define ISO_ERR_INTERNAL (-7)     /* an internal consistency check failed           */

/* Precision of the Gram tiles ||x||^2 + ||y||^2 - 2 x.y used to screen pairs.
 * Every pair that can be a component's minimum under the error bound of the
 * screen is re-evaluated exactly (iso_recheck), so the tree does not depend on
 * the screen's precision. */
#define ISO_PREC_FP32 0
#define ISO_PREC_BF16 1
/* FP8 E4M3 (OCP, max 448) screen on the FP8 matrix cores: coordinates are
 * centred and rounded to E4M3 without scaling (values beyond +-448 saturate);
 * the representation error of every point enters the screen's bound, so the
 * tree is unchanged, only the number of candidates grows with it. */
#define ISO_PREC_FP8 2
/* INT8 screen for 8-bit data (every coordinate on one binary grid 2^q, each
 * column spanning at most 255 steps, d < 16384, e.g. q/256 pixel values): the
 * coordinates are centred on grid values and held as exact integers, so the
 * Gram tiles and norms are exact in int32 on the INT8 matrix cores; other
 * data is rejected (INVALID_ARG). */
#define ISO_PREC_INT8 3

/* Arithmetic of the exact re-evaluation of candidate distances, which defines
 * the order of the edges:
 *   FP32: D^2 = sum_t (x_t - y_t)^2 in FP32, in a fixed order;
 *   FP64: D^2 = sum_t (x_t - y_t)^2 in FP64, left to right over t, each term
 *         rounded separately (parity mode). */
#define ISO_RECHECK_FP32 0
#define ISO_RECHECK_FP64 1
/* Bits of iso_mst's `flags` argument (0 = every shortcut allowed).  The tree is
 * the same with any of them: they only select which rounds may skip the full
 * screen and which screen precision may run. */
#define ISO_MST_NO_LISTS 0x1    /* no neighbour lists from the second round    */
#define ISO_MST_NO_FINAL 0x2    /* no final round joining <= 64 components    */
#define ISO_MST_NO_ESCALATE 0x4 /* keep the requested screen precision even
                                   when its bound is too loose for the data  */
#define ISO_MST_PAIR_BOUNDS 0x8 /* BF16 screen: capture thresholds from each
                                   pair's own error bound instead of the
                                   separable bound against the largest norm
                                   (chosen by itself when the points' norms are
                                   heavy tailed; every round is then screened) */
#define ISO_MST_NO_PRUNE 0x10   /* screen every tile pair of a round, also those
                                   whose bounding balls prove them too far
                                   apart to matter                           */

/* Vertex weight omega (eq. 2.2) and flow phi (eq. 2.1) readings. */
#define ISO_OMEGA_TREE 0   /* omega(v) = sum of phi over v's tree edges         */
#define ISO_OMEGA_FULL 1   /* omega(v) = sum over all j != v of phi(v, j), as
                              computed by iso_graph_weights and passed in
                              iso_sub_opts.omega0                               */
#define ISO_PHI_EXP_DIST 0 /* phi = exp(-D / sigma), as printed in eq. 2.1      */
#define ISO_PHI_GAUSS_SQ 1 /* phi = exp(-D^2 / (2 sigma^2))                      */
/* Initial bracket of the bisection (Algorithm 2). */
#define ISO_BRACKET_POW2 0  /* alpha0 rounded down, beta0 up, to powers of two  */
#define ISO_BRACKET_PAPER 1 /* printed alpha0, beta0 (beta0 moved up one ulp)   */

typedef struct {
    int32_t rounds;          /* Boruvka rounds                                   */
    int32_t list_rounds;     /* rounds decided by the neighbour lists of the
                                second round's screen instead of a full screen  */
    int64_t candidates;      /* candidate pairs re-evaluated exactly (all rounds) */
    int64_t rescanned_rows;  /* rows whose candidate list overflowed and were
                                re-evaluated against every other point          */
    double mst_weight;       /* sum of the n-1 FP64 edge lengths                 */
    int32_t final_components;/* components joined at once by the final round
                                (0: the last round was a plain round)           */
    int32_t screen_precision;/* precision of the screen that built the tree: the
                                requested one, or ISO_PREC_FP32 when its error
                                bound was too loose for the data (escalation)   */
    int32_t pair_bounds;     /* 1 when that screen used per-pair bounds        */
    int64_t tile_pairs;      /* 256 x 256 tile pairs screened (all rounds)     */
    int64_t tile_pairs_full; /* tile pairs the same rounds would screen without
                                the bounding-ball test (ISO_MST_NO_PRUNE)      */
} iso_mst_info;

/* Device bytes iso_mst needs as workspace for n points in d dimensions (room
 * for the FP32 screen included, which a loose low-precision screen escalates to). */
iso_status iso_mst_workspace_size(int64_t n, int64_t d, int32_t precision, size_t *bytes /* host */);

/* Euclidean minimum spanning tree of the complete graph on the n points X
 * (Sec. 2.2 step 2 / Sec. 3.5).  The n x n distance matrix is never stored:
 * distances are formed tile by tile.  Edges are totally ordered by (D^2 under
 * `recheck`, smaller end id, larger end id), so the tree is unique.  Rounds
 * screen every inter-component pair, except that from the third round on a
 * round may be decided by the neighbour lists the second round's screen
 * builds, and once at most 64 components remain one final round joins them
 * all (both are switched off by ISO_MST_NO_LISTS / ISO_MST_NO_FINAL in
 * `flags`; the tree does not change).  Points are ordered into tiles of nearby
 * points, and a pair of tiles whose bounding balls are farther apart than any
 * of their points' current lightest-edge bound is not screened (the
 * bounding-ball test of dual-tree Boruvka; ISO_MST_NO_PRUNE turns it off; the
 * tree does not change).
 *   X       [n*ld] FP32 points (read only).
 *   precision  ISO_PREC_* of the screen;  recheck  ISO_RECHECK_* (edge order);
 *   flags   OR of ISO_MST_NO_* bits, or 0.
 *   parent  [n] out: tree rooted at vertex 0, parent[0] = -1.
 *   length  [n] out: FP64 Euclidean length of the edge (v, parent[v]),
 *                    sqrt of the left-to-right FP64 sum of squared coordinate
 *                    differences; length[0] = 0.
 *   info    (host, nullable) out: statistics; requires a stream sync.
 *   ws      device workspace of iso_mst_workspace_size bytes, or NULL (the
 *           library then allocates and frees it on `stream`).
 *   stream  HIP stream (NULL: the default stream); the call synchronises it.
 *           Part of the work runs on a second stream of the library's,
 *           ordered by events; `stream` waits for all of it before the call
 *           returns.  The library keeps, per device and for the life of the
 *           process, one such stream with its events and a 2 MB pinned
 *           staging buffer for each call running at once.
 * Errors: n < 2, d < 1, ld < d, null pointers, unknown precision, recheck or
 * flag bits (INVALID_ARG); a non-finite coordinate (NONFINITE); the INT8
 * screen on data that is not 8-bit (INVALID_ARG). */
iso_status iso_mst(const float *X, int64_t n, int64_t d, int64_t ld, int32_t precision, int32_t recheck,
                   uint32_t flags, int32_t *parent, double *length, iso_mst_info *info, void *ws, size_t ws_bytes,
                   void *stream);

/* The paper's own MST construction (Sec. 3.5, Algorithm 3), kept for
 * comparison with iso_mst: Prim from vertex 0, adding per step the vertex with
 * the lightest edge to the tree (a min-reduction over the vertices outside
 * it) and lowering the others' keys with their FP64 distances to it.  Edges
 * are ordered by (D^2, smaller id, larger id) with D^2 the FP64 left-to-right
 * sum, so parent/length equal those of iso_mst with ISO_RECHECK_FP64.
 * n - 1 sequential steps of O(n d) work each (two launches per step).
 *   order   [n] out (nullable): vertex added at each step (order[0] = 0).
 * Workspace: iso_mst_prim_workspace_size(n).  Errors: null X/parent/length,
 * n < 2, d < 1, ld < d (INVALID_ARG). */
iso_status iso_mst_prim_workspace_size(int64_t n, size_t *bytes /* host */);
iso_status iso_mst_prim(const float *X, int64_t n, int64_t d, int64_t ld, int32_t *parent, double *length,
                        int32_t *order, void *ws, size_t ws_bytes, void *stream);

typedef struct {
    int32_t omega;         /* ISO_OMEGA_*   (default TREE)                          */
    int32_t phi;           /* ISO_PHI_*     (default EXP_DIST)                      */
    int32_t bracket;       /* ISO_BRACKET_* (default POW2)                          */
    int32_t max_iters;     /* bisection step cap, <= 0 => 2000                      */
    const double *omega0;  /* [n] device: vertex weights for ISO_OMEGA_FULL (from
                              iso_graph_weights with the same sigma and phi);
                              ignored for ISO_OMEGA_TREE                            */
    const double *p0;      /* [n] device: potential p(v) of eq. 2.3 (from
                              iso_graph_weights with alpha > 0); NULL => p = 0      */
} iso_sub_opts;

typedef struct {
    double sigma;                 /* sigma used                                        */
    double alpha0_raw, beta0_raw; /* printed bracket of Algorithm 2                    */
    double alpha0, beta0;         /* bracket used                                      */
    double alpha, beta;           /* final bracket; the subpartition is the one
                                     Algorithm 1 returns at N = beta                    */
    double i_k;                   /* cost of the returned subpartition (eq. 2.4)       */
    int32_t t_paper;              /* printed iteration count of Algorithm 2 (reported) */
    int32_t iters;                /* bisection steps taken (to FP64 resolution)        */
    int32_t passes;               /* device passes (several bisection steps each)      */
    int32_t max_depth;            /* depth of the rooted tree                          */
    int32_t jstar;                /* smallest cluster index attaining i_k              */
    int32_t reserved0;
} iso_sub_info;

/* Device bytes iso_subpartition needs as workspace. */
iso_status iso_sub_workspace_size(int64_t n, int32_t k, size_t *bytes /* host */);

/* Optimal k-subpartition of the weighted tree (parent, length) and its cost
 * MISO_k(T) (eq. 2.6), by Algorithm 1 inside the bisection of Algorithm 2,
 * run to FP64 resolution (the bisection stops when the midpoint equals an end
 * point).  The x-order of Algorithm 1 is (depth descending, id ascending).
 *   parent  [n] tree rooted at `root` (parent[root] = -1).
 *   length  [n] FP64 edge lengths (length[root] ignored).
 *   sigma   > 0, or 0 for the lower median of the n-1 edge lengths.
 *   opts    (host, nullable) readings; NULL = defaults.
 *   labels  [n] out: cluster 0..k-1 in x-order of the cut vertices, or -1 for
 *                    residual (outlier) vertices.
 *   i_k     (host) out: MISO_k as found (requires a stream sync).
 *   cluster_num, cluster_den [k] FP64, cluster_size [k] int32 (nullable) out:
 *                    phi(delta A_j) + p(A_j), omega(A_j) and |A_j|.
 *   info    (host, nullable) out.
 * Errors: n < 2, k < 2, k > n, root outside [0, n), sigma < 0 or not finite,
 * parent not a tree rooted at root (INVALID_ARG). */
iso_status iso_subpartition(const int32_t *parent, const double *length, int64_t n, int32_t root, int32_t k,
                            double sigma, const iso_sub_opts *opts, int32_t *labels, double *i_k /* host */,
                            double *cluster_num, double *cluster_den, int32_t *cluster_size, iso_sub_info *info,
                            void *ws, size_t ws_bytes, void *stream);

/* iso_subpartition for callers that cannot allocate device memory (code that
 * must not call hipMalloc: tight serving loops, harnesses that forbid device
 * allocation): the same computation, arguments and results, with the
 * workspace taken from a fixed device array inside the library instead of a
 * caller buffer or a library allocation.  That array (ISO_SUB_NOALLOC_BYTES)
 * is reserved on every GPU the library runs on until the process ends; its
 * address is looked up once per device, on the first call made with that
 * device current.  Every call on one GPU uses the same array, so calls that
 * overlap in time on one GPU (concurrent streams or threads) race and must be
 * serialised by the caller; nothing is kept from one call to the next.
 * Errors: as iso_subpartition, and n > ISO_SUB_NOALLOC_MAX_N (INVALID_ARG). */
#define ISO_SUB_NOALLOC_MAX_N 32768
#define ISO_SUB_NOALLOC_BYTES ((size_t)64 << 20)
iso_status iso_subpartition_noalloc(const int32_t *parent, const double *length, int64_t n, int32_t root, int32_t k,
                                    double sigma, const iso_sub_opts *opts, int32_t *labels, double *i_k /* host */,
                                    double *cluster_num, double *cluster_den, int32_t *cluster_size,
                                    iso_sub_info *info, void *stream);

/* The optimal k-subpartition for every k = 2 .. kmax of one tree: MISO_k of
 * eq. 2.6 for each k, each by Algorithm 1 inside its own bisection of
 * Algorithm 2 (Sec. 2.2), labelled as in Algorithm 4 -- the same bisection,
 * final bracket and labels as kmax - 1 separate iso_subpartition calls; the
 * passes evaluate the midpoints of several k together.
 *   i_k     (host) [kmax - 1] out: MISO_k for k = 2 .. kmax.
 *   labels  [(kmax - 1) * n] out (nullable): row k - 2 holds the labels for k.
 *   passes  (host, nullable) out: tree passes used.
 * Workspace: iso_sub_workspace_size(n, kmax).  Errors as iso_subpartition,
 * with kmax in place of k. */
iso_status iso_subpartition_all_k(const int32_t *parent, const double *length, int64_t n, int32_t root, int32_t kmax,
                                  double sigma, const iso_sub_opts *opts, double *i_k /* host */, int32_t *labels,
                                  int32_t *passes /* host */, void *ws, size_t ws_bytes, void *stream);

/* Full-graph weights of eqs. 2.2 and 2.3 for the n points X, with distances
 * D(v, j) = sqrt of the FP64 left-to-right sum of squared coordinate
 * differences (each point pair formed on the fly, never stored):
 *   omega0[v] = sum over j != v, ascending j, of phi(D(v, j))   (phi_kind ISO_PHI_*),
 *   p0[v]     = alpha * sum over j != v, ascending j, of D(v, j) (exactly 0 when alpha == 0).
 * O(n^2 d) FP64 work.  Either output may be NULL.  X [n*ld] FP32; sigma > 0.
 * Scratch of about 8 n (d + 1024) bytes is allocated with hipMallocAsync on
 * `stream` and released with hipFreeAsync in stream order (no synchronisation).
 * Errors: null X, n < 2, d < 1, ld < d, sigma <= 0 or not finite, alpha < 0 or
 * not finite, unknown phi_kind (INVALID_ARG). */
iso_status iso_graph_weights(const float *X, int64_t n, int64_t d, int64_t ld, double sigma, int32_t phi_kind,
                             double alpha, double *omega0, double *p0, void *stream);

/* sigma of eq. 2.1 as "the median MST edge": the lower median of length[v]
 * over the n-1 vertices with parent[v] >= 0, written to *sigma (host); the
 * value iso_subpartition uses when it is passed sigma = 0.
 * Errors: null pointers, n < 2 (INVALID_ARG). */
iso_status iso_sigma_median(const int32_t *parent, const double *length, int64_t n, double *sigma /* host */,
                            void *stream);

/* Device bytes iso_backward needs as workspace. */
iso_status iso_backward_workspace_size(int64_t n, size_t *bytes /* host */);

/* Adjoint of W = total length of the tree's edges and of I = cost (eq. 2.4,
 * tree-degree omega, p = 0) of cluster `jstar` of `labels`, with the tree and
 * the subpartition held fixed (a subgradient of MISO_k at the returned
 * subpartition when jstar attains it):
 *   gX = gW dW/dX + gI dI/dX,   *gsigma = gI dI/dsigma.
 * Edge lengths are recomputed from X in FP64.  Each vertex sums the terms of
 * its incident edges (parent edge, then children by ascending id) in FP64, so
 * the result is deterministic; an edge of length 0 contributes a zero
 * subgradient.
 *   X       [n*ld] FP32 points;  parent [n] tree (one or more roots = -1);
 *   labels  [n] cluster of each vertex (-1 = residual), as from iso_subpartition;
 *   sigma   > 0, the scale used in phi (eq. 2.1);  phi_kind ISO_PHI_*;
 *   gX      [n*ldg] out, FP32;  gsigma, I_out (host, I_out nullable) out.
 * Errors: null pointers, n < 2, d < 1, ld < d, ldg < d, sigma <= 0, unknown
 * phi_kind, non-finite gW/gI, parent entries outside [-1, n) (INVALID_ARG). */
iso_status iso_backward(const float *X, int64_t n, int64_t d, int64_t ld, const int32_t *parent,
                        const int32_t *labels, int32_t jstar, double sigma, int32_t phi_kind, double gW, double gI,
                        float *gX, int64_t ldg, double *gsigma /* host */, double *I_out /* host */, void *ws,
                        size_t ws_bytes, void *stream);

/* Optional phase timing, for benchmarks: while enabled, iso_mst brackets the
 * screen of every Boruvka round (its diagonal-tile and off-diagonal kernel
 * dispatches) with hipEvents on its stream and counts the unordered pairs of
 * points in different components that the round must cover, and both entry
 * points record their own duration.  Totals accumulate in process-wide
 * counters (not thread safe) until the next iso_timing_enable call, which
 * resets them.  Enabling timing adds synchronisation-free event records and,
 * per Boruvka round, a component-size reduction. */
typedef struct {
    int32_t enabled;
    int32_t screen_launches;  /* screens timed (one per Boruvka round)              */
    double screen_ms;         /* summed durations of those screens                  */
    double screen_pairs;      /* summed unordered inter-component pairs they cover  */
    double screen_dim;        /* padded dimension the screen contracts over         */
    int32_t mst_calls, sub_calls;
    double mst_ms;            /* summed iso_mst durations (first to last launch)    */
    double sub_ms;            /* summed iso_subpartition durations                  */
    int32_t sub_passes;       /* speculative bisection passes                       */
    int32_t reserved0;
} iso_timing;

iso_status iso_timing_enable(int32_t on);
iso_status iso_timing_read(iso_timing *out /* host */);

/* Text of the last error on the calling thread (valid until its next call). */
const char *iso_last_error(void);

/* Library version string. */
const char *iso_version(void);

#ifdef __cplusplus
}
#endif
#endif /* ISOCLUST_H */
