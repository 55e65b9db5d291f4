/*
 * oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow FP64 CPU reference of the clustering method of
 * Javadi & Ashkboos, "An Efficient Parallel Data Clustering Algorithm Using
 * Isoperimetric Number of Trees" (arXiv 1702.04739):
 *
 *   1. the Euclidean minimum spanning tree of the points, by dense Prim from
 *      vertex 0 (Sec. 3.5, Algorithm 3, run sequentially here), never storing
 *      an n x n matrix (one thread, or an explicit number of threads for each
 *      step's key update, with the same result);
 *   2. the weight functions of the tree: flow phi (Sec. 2.1, eq. 2.1), vertex
 *      weight omega (eq. 2.2) and potential p (eq. 2.3);
 *   3. the decision procedure that tells whether some k-subpartition costs at
 *      most N (Sec. 2.2, Algorithm 1) and the bisection around it (Algorithm 2),
 *      with the labelling of Algorithm 4 (Sec. 3.6);
 *   4. the adjoint of the total MST weight and of the optimal subpartition's
 *      cost with respect to the points and sigma, holding the tree and the
 *      subpartition fixed.
 *
 * Only the test-suite, the smoke check and the benchmark's CPU-baseline leg may
 * load this library. It shares no code with the GPU library and includes none
 * of its headers.  Build: gcc -O2 -ffp-contract=off -fPIC -shared (no -ffast-math):
 * every floating-point operation below is a separately rounded IEEE FP64
 * operation, in the order written.
 *
 * Readings taken where the paper is silent or ambiguous (each is also listed
 * in the design notes):
 *   R1  omega: default is the weighted degree in the tree (Sec. 2.2 step 2
 *       computes phi, omega and p on the tree T; Algorithm 1 takes a weighted
 *       tree).  The literal full-graph sum of eq. 2.2 is available as
 *       omega_mode = 1.  The self term j = i is excluded (phi is only defined
 *       for i != j, eq. 2.1).
 *   R2  phi: eq. 2.1 as printed, exp(-||xi-xj||_2 / sigma); phi_kind = 1 gives
 *       exp(-||xi-xj||^2 / (2 sigma^2)) as an option.
 *   R3  MST ties: edges are totally ordered by (D^2, min id, max id), D^2 the
 *       FP64 left-to-right sum of squared coordinate differences.  The MST is
 *       therefore unique.
 *   R4  root = vertex 0; "BFS order" x_1..x_n = vertices sorted by (depth
 *       descending, id ascending), so x_n is the root.
 *   R5  root: no parent edge, phi(e) = 0, join impossible.
 *   R6  the else branch "p(u) <- p(u) + phi(x_i)" uses phi of x_i's parent
 *       edge (parent-list notation of Sec. 3.3).
 *   R7  bisection runs to FP64 resolution (stop when the midpoint equals an
 *       end point) instead of the printed iteration count t, which is
 *       reported only; t = ceil(log2(2 omega*^2 (beta0-alpha0)) -
 *       log2(phi_* + p_*)).
 *   R8  bracket: default rounds alpha0 down to a power of two and beta0 up to
 *       the next power of two strictly above; bracket = 1 keeps the printed
 *       values and only moves beta0 up by one ulp.
 *   R9  clusters = the first k cut vertices in x-order; a vertex v belongs to
 *       cluster j if the first non-joined vertex on its path to the root is
 *       the j-th cut vertex; every other vertex is residual (label -1).
 *   R10 sigma = 0 requests the lower median of the n-1 tree edge lengths.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_EINVAL -1
#define ORC_ENOMEM -2
#define ORC_ENOTTREE -3
#define ORC_EBRACKET -4

/* ------------------------------------------------------------------ */
/* Distances (Sec. 2.2 step 1: d(xi,xj) = ||xi - xj||_2)               */
/* ------------------------------------------------------------------ */

/* Squared Euclidean distance, FP64, left to right over coordinates, each term
 * rounded separately (no fused multiply-add). */
double orc_sqdist(const float *X, int64_t ld, int64_t d, int64_t i, int64_t j) {
    const float *a = X + i * ld;
    const float *b = X + j * ld;
    double s = 0.0;
    for (int64_t t = 0; t < d; ++t) {
        double diff = (double)a[t] - (double)b[t];
        double sq = diff * diff;
        s = s + sq;
    }
    return s;
}

/* Strict total order on edges (R3): returns 1 if (d2a, {ua,va}) < (d2b, {ub,vb}). */
static int edge_less(double d2a, int64_t ua, int64_t va, double d2b, int64_t ub, int64_t vb) {
    if (d2a < d2b) return 1;
    if (d2a > d2b) return 0;
    int64_t a0 = ua < va ? ua : va, a1 = ua < va ? va : ua;
    int64_t b0 = ub < vb ? ub : vb, b1 = ub < vb ? vb : ub;
    if (a0 != b0) return a0 < b0;
    return a1 < b1;
}

/* ------------------------------------------------------------------ */
/* Minimum spanning tree: Prim from vertex 0 (Sec. 3.5, Algorithm 3)   */
/* ------------------------------------------------------------------ */

/* Outputs parent[n] (parent[0] = -1), len[n] (len[0] = 0, len[v] = sqrt of the
 * FP64 squared distance to the parent), depth[n] (nullable) and order_added[n]
 * (nullable; the order in which Prim added the vertices).  Memory is O(n):
 * each step recomputes the distances from the newly added vertex only. */
int orc_prim_mst_threads(const float *X, int64_t n, int64_t d, int64_t ld, int32_t *parent, double *len,
                         int32_t *depth, int32_t *order_added, int32_t threads);

int orc_prim_mst(const float *X, int64_t n, int64_t d, int64_t ld, int32_t *parent, double *len,
                 int32_t *depth, int32_t *order_added) {
    return orc_prim_mst_threads(X, n, d, ld, parent, len, depth, order_added, 1);
}

/* The same with the per-step update of the remaining vertices' keys split over
 * `threads` OpenMP threads.  Each vertex's update reads only its own key and
 * the new tree vertex, and the choice of the next vertex stays one sequential
 * scan, so the result does not depend on the thread count. */
int orc_prim_mst_threads(const float *X, int64_t n, int64_t d, int64_t ld, int32_t *parent, double *len,
                         int32_t *depth, int32_t *order_added, int32_t threads) {
    if (!X || n < 1 || d < 1 || ld < d || !parent || !len || threads < 1) return ORC_EINVAL;
    double *key = (double *)malloc(sizeof(double) * n);
    int64_t *keyu = (int64_t *)malloc(sizeof(int64_t) * n);
    char *in_tree = (char *)calloc(n, 1);
    int32_t *dep = (int32_t *)malloc(sizeof(int32_t) * n);
    if (!key || !keyu || !in_tree || !dep) {
        free(key); free(keyu); free(in_tree); free(dep);
        return ORC_ENOMEM;
    }
    /* Step: add the root and record its distance to every other vertex. */
    in_tree[0] = 1;
    parent[0] = -1;
    len[0] = 0.0;
    dep[0] = 0;
    if (order_added) order_added[0] = 0;
    for (int64_t v = 1; v < n; ++v) {
        key[v] = orc_sqdist(X, ld, d, 0, v);
        keyu[v] = 0;
    }
    for (int64_t step = 1; step < n; ++step) {
        /* Vertex outside the tree whose connecting edge is smallest. */
        int64_t best = -1;
        for (int64_t v = 1; v < n; ++v) {
            if (in_tree[v]) continue;
            if (best < 0 || edge_less(key[v], keyu[v], v, key[best], keyu[best], best)) best = v;
        }
        /* Add it, with its parent and depth. */
        in_tree[best] = 1;
        parent[best] = (int32_t)keyu[best];
        len[best] = sqrt(key[best]);
        dep[best] = dep[keyu[best]] + 1;
        if (order_added) order_added[step] = (int32_t)best;
        /* Update every remaining vertex's distance to the tree. */
#pragma omp parallel for schedule(static) num_threads(threads) if (threads > 1)
        for (int64_t v = 1; v < n; ++v) {
            if (in_tree[v]) continue;
            double d2 = orc_sqdist(X, ld, d, best, v);
            if (edge_less(d2, best, v, key[v], keyu[v], v)) {
                key[v] = d2;
                keyu[v] = best;
            }
        }
    }
    if (depth) memcpy(depth, dep, sizeof(int32_t) * n);
    free(key); free(keyu); free(in_tree); free(dep);
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* Rooted-tree bookkeeping (Sec. 2.2 step 3; R4)                       */
/* ------------------------------------------------------------------ */

/* Depth of every vertex from the parent array; fails unless parent describes a
 * tree rooted at `root` (parent[root] = -1, every other parent in range, no
 * cycle). */
int orc_tree_depth(const int32_t *parent, int64_t n, int32_t root, int32_t *depth) {
    if (!parent || !depth || n < 1 || root < 0 || root >= n) return ORC_EINVAL;
    if (parent[root] != -1) return ORC_ENOTTREE;
    for (int64_t v = 0; v < n; ++v) {
        if (v != root && (parent[v] < 0 || parent[v] >= n)) return ORC_ENOTTREE;
        depth[v] = -1;
    }
    depth[root] = 0;
    int32_t *stack = (int32_t *)malloc(sizeof(int32_t) * n);
    if (!stack) return ORC_ENOMEM;
    for (int64_t v = 0; v < n; ++v) {
        int64_t top = 0, u = v;
        while (depth[u] < 0) {
            if (top >= n) { free(stack); return ORC_ENOTTREE; }
            stack[top++] = (int32_t)u;
            u = parent[u];
        }
        int32_t dd = depth[u];
        while (top > 0) depth[stack[--top]] = ++dd;
    }
    free(stack);
    return ORC_OK;
}

/* x-order of Algorithm 1: vertices sorted by (depth descending, id ascending). */
int orc_tree_order(const int32_t *depth, int64_t n, int32_t *order) {
    int32_t maxd = 0;
    for (int64_t v = 0; v < n; ++v) if (depth[v] > maxd) maxd = depth[v];
    int64_t *cnt = (int64_t *)calloc((size_t)maxd + 2, sizeof(int64_t));
    if (!cnt) return ORC_ENOMEM;
    for (int64_t v = 0; v < n; ++v) cnt[maxd - depth[v] + 1]++;
    for (int32_t b = 1; b <= maxd + 1; ++b) cnt[b] += cnt[b - 1];
    for (int64_t v = 0; v < n; ++v) order[cnt[maxd - depth[v]]++] = (int32_t)v;
    free(cnt);
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* Weight functions on the tree (Sec. 2.1, eqs. 2.1-2.3)               */
/* ------------------------------------------------------------------ */

static double flow_of(double dist, double sigma, int phi_kind) {
    if (phi_kind == 1) return exp(-(dist * dist) / (2.0 * sigma * sigma));
    return exp(-dist / sigma);
}

/* Lower median of len[v], v != root (R10). */
static int cmp_double(const void *a, const void *b) {
    double x = *(const double *)a, y = *(const double *)b;
    return (x > y) - (x < y);
}

double orc_lower_median(const int32_t *parent, const double *len, int64_t n) {
    if (n < 2) return 0.0;
    double *v = (double *)malloc(sizeof(double) * (n - 1));
    if (!v) return -1.0;
    int64_t m = 0;
    for (int64_t i = 0; i < n; ++i) if (parent[i] >= 0) v[m++] = len[i];
    qsort(v, (size_t)m, sizeof(double), cmp_double);
    double med = v[(m - 1) / 2];
    free(v);
    return med;
}

/* phi[v] = flow of v's parent edge (0 at the root); omega0[v] and p0[v] per R1:
 *   omega_mode 0: sum over tree neighbours w of v, ascending w, of phi(vw);
 *   omega_mode 1: sum over all j != v, ascending j, of flow(D(v,j)) (eq. 2.2);
 *   p0[v] = alpha_pot * sum over all j != v, ascending j, of D(v,j) (eq. 2.3),
 *           and exactly 0 when alpha_pot == 0. */
int orc_tree_weights(const int32_t *parent, const double *len, int64_t n, int32_t root, double sigma,
                     int omega_mode, int phi_kind, double alpha_pot, const float *X, int64_t d, int64_t ld,
                     double *phi, double *omega0, double *p0) {
    if (!parent || !len || !phi || !omega0 || !p0 || n < 1 || !(sigma > 0.0)) return ORC_EINVAL;
    if ((omega_mode == 1 || alpha_pot != 0.0) && (!X || d < 1 || ld < d)) return ORC_EINVAL;
    for (int64_t v = 0; v < n; ++v) phi[v] = (v == root) ? 0.0 : flow_of(len[v], sigma, phi_kind);
    if (omega_mode == 0) {
        /* children lists in ascending id: counting sort by parent, filled in v order */
        int64_t *off = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
        int32_t *kids = (int32_t *)malloc(sizeof(int32_t) * (n > 1 ? n : 1));
        if (!off || !kids) { free(off); free(kids); return ORC_ENOMEM; }
        for (int64_t v = 0; v < n; ++v) if (v != root) off[parent[v] + 1]++;
        for (int64_t u = 0; u < n; ++u) off[u + 1] += off[u];
        int64_t *cur = (int64_t *)malloc(sizeof(int64_t) * n);
        if (!cur) { free(off); free(kids); return ORC_ENOMEM; }
        for (int64_t u = 0; u < n; ++u) cur[u] = off[u];
        for (int64_t v = 0; v < n; ++v) if (v != root) kids[cur[parent[v]]++] = (int32_t)v;
        for (int64_t v = 0; v < n; ++v) {
            double s = 0.0;
            int parent_done = (v == root);
            for (int64_t c = off[v]; c < off[v + 1]; ++c) {
                int32_t w = kids[c];
                if (!parent_done && parent[v] < w) { s = s + phi[v]; parent_done = 1; }
                s = s + phi[w];
            }
            if (!parent_done) s = s + phi[v];
            omega0[v] = s;
        }
        free(off); free(kids); free(cur);
    } else {
        for (int64_t v = 0; v < n; ++v) {
            double s = 0.0;
            for (int64_t j = 0; j < n; ++j) {
                if (j == v) continue;
                s = s + flow_of(sqrt(orc_sqdist(X, ld, d, v, j)), sigma, phi_kind);
            }
            omega0[v] = s;
        }
    }
    for (int64_t v = 0; v < n; ++v) {
        if (alpha_pot == 0.0) { p0[v] = 0.0; continue; }
        double s = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            if (j == v) continue;
            s = s + sqrt(orc_sqdist(X, ld, d, v, j));
        }
        p0[v] = alpha_pot * s;
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* Algorithm 1: decision "exists A in D_k(X) with cost(A) <= N"         */
/* ------------------------------------------------------------------ */

/* Decision "is there a k-subpartition of cost at most N" (Sec. 2.2,
 * Algorithm 1), written as a fold over the rooted tree.
 *
 * Each vertex x owns a pending set eta(x): x itself plus the descendants that
 * were merged into it.  Two numbers describe eta(x) once all of x's children
 * are settled: its weight w(x) = omega(eta(x)) and its charge p(x) = the
 * potential of eta(x) plus the flow of the tree edges that leave eta(x)
 * downwards (to children that were not merged).  The only edge of eta(x) not
 * yet accounted for is x's parent edge e, of flow fe (0 at the root).
 *
 * By eq. 2.4, eta(x) is a valid cluster at level N when its cost, parent edge
 * included, is at most N:   fe + p(x) <= N w(x)   ->  x is CUT (a cluster).
 * Otherwise eta(x) is either merged into the parent's set, or left behind as
 * residual vertices.  Either way the parent's own test N w - p changes:
 *   merged:  w += w(x), p += p(x)     (e becomes an inner edge),
 *   left:    p += fe                  (e becomes a boundary edge of the parent).
 * Merging is taken when it leaves the parent more room, i.e. when
 * N w(x) - p(x) > -fe, evaluated as   p(x) - fe < N w(x)   ->  x is JOINED;
 * else x is DROPPED.  A cut child also puts its edge on the parent's boundary
 * (p += fe).  The root has no parent edge and can only be cut or dropped.
 *
 * Vertices are settled in x-order (children before parents); a vertex folds its
 * children's outcomes in ascending child id.  The sweep stops at the k-th cut.
 * Returns the number of cuts reached (<= k); the answer is YES iff it equals k.
 * wbuf/pbuf [n] receive w and p of the settled vertices.  With rec_cut the
 * first cuts (in x-order) are stored with fe + p(x) in rec_num and w(x) in
 * rec_den, and joined[v] = 1 marks the merged vertices.  Returns -1 when its
 * scratch memory cannot be allocated. */
enum { ORC_OPEN = 0, ORC_CUT = 1, ORC_JOINED = 2, ORC_DROPPED = 3 };

int64_t orc_decide(const int32_t *parent, const int32_t *order, const double *phi, const double *omega0,
                   const double *p0, int64_t n, int64_t k, double N, double *wbuf, double *pbuf,
                   int32_t *rec_cut, double *rec_num, double *rec_den, uint8_t *joined) {
    /* children of every vertex in ascending id (counting sort on the parent) */
    int64_t *first = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    int32_t *kids = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    uint8_t *state = (uint8_t *)calloc((size_t)n, 1);
    if (!first || !kids || !state) { free(first); free(kids); free(state); return -1; }
    for (int64_t v = 0; v < n; ++v) if (parent[v] >= 0) first[parent[v] + 1]++;
    for (int64_t u = 0; u < n; ++u) first[u + 1] += first[u];
    {
        int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
        if (!fill) { free(first); free(kids); free(state); return -1; }
        memcpy(fill, first, sizeof(int64_t) * (size_t)n);
        for (int64_t v = 0; v < n; ++v) if (parent[v] >= 0) kids[fill[parent[v]]++] = (int32_t)v;
        free(fill);
    }
    if (joined) memset(joined, 0, (size_t)n);

    int64_t cuts = 0;
    for (int64_t i = 0; i < n && cuts < k; ++i) {
        const int32_t x = order[i];
        double w = omega0[x], p = p0[x];
        for (int64_t c = first[x]; c < first[x + 1]; ++c) {
            const int32_t y = kids[c];
            if (state[y] == ORC_JOINED) {
                w = w + wbuf[y];
                p = p + pbuf[y];
            } else {
                p = p + phi[y];   /* cut or dropped child: its edge bounds eta(x) */
            }
        }
        wbuf[x] = w;
        pbuf[x] = p;
        const int has_parent = parent[x] >= 0;
        const double fe = has_parent ? phi[x] : 0.0;
        const double room = N * w;
        if (fe + p <= room) {
            state[x] = ORC_CUT;
            if (rec_cut) { rec_cut[cuts] = x; rec_num[cuts] = fe + p; rec_den[cuts] = w; }
            cuts = cuts + 1;
        } else if (has_parent && p - fe < room) {
            state[x] = ORC_JOINED;
            if (joined) joined[x] = 1;
        } else {
            state[x] = ORC_DROPPED;
        }
    }
    free(first); free(kids); free(state);
    return cuts;
}

/* ------------------------------------------------------------------ */
/* Algorithm 2 (bisection) + Algorithm 4 labelling                     */
/* ------------------------------------------------------------------ */

typedef struct {
    double sigma;       /* sigma used (after the median rule) */
    double phi_sum, phi_min, omega_sum, omega_min, p_sum, p_min;
    double alpha0_raw, beta0_raw;   /* printed bracket of Algorithm 2 */
    double alpha0, beta0;           /* bracket actually used (R8) */
    double alpha, beta;             /* final bracket */
    double i_k;                     /* cost of the returned subpartition */
    int32_t t_paper;                /* printed iteration count (R7), reported only */
    int32_t iters;                  /* bisection steps taken */
    int32_t jstar;                  /* smallest index of a cluster attaining i_k */
    int32_t max_depth;
} orc_sub_info;

static double pow2_floor(double x) {
    if (!(x > 0.0)) return 0.0;
    int e;
    frexp(x, &e);                  /* x = m 2^e, m in [0.5, 1) */
    return ldexp(1.0, e - 1);
}

static double pow2_above(double x) {
    int e;
    frexp(x, &e);
    return ldexp(1.0, e);          /* strictly greater than x */
}

/* Full tree stage: weights, bounds, bisection to FP64 resolution, labels.
 *   sigma <= 0 selects the lower median of the tree edge lengths.
 *   labels[n]: cluster index 0..k-1 or -1 (residual).
 *   cl_num, cl_den, cl_size [k] (nullable).
 * X/d/ld are needed only for omega_mode 1 or alpha_pot != 0. */
int orc_subpartition(const int32_t *parent, const double *len, int64_t n, int32_t root, int64_t k, double sigma,
                     int omega_mode, int phi_kind, int bracket, double alpha_pot, int32_t max_iters,
                     const float *X, int64_t d, int64_t ld, int32_t *labels, double *cl_num, double *cl_den,
                     int32_t *cl_size, orc_sub_info *info) {
    if (!parent || !len || !labels || !info || n < 2 || k < 2 || k > n || root < 0 || root >= n) return ORC_EINVAL;
    if (!(sigma >= 0.0) || isinf(sigma)) return ORC_EINVAL;
    if (max_iters <= 0) max_iters = 2000;
    int rc = ORC_OK;
    int32_t *depth = (int32_t *)malloc(sizeof(int32_t) * n);
    int32_t *order = (int32_t *)malloc(sizeof(int32_t) * n);
    double *phi = (double *)malloc(sizeof(double) * n);
    double *om = (double *)malloc(sizeof(double) * n);
    double *p0 = (double *)malloc(sizeof(double) * n);
    double *wb = (double *)malloc(sizeof(double) * n);
    double *pb = (double *)malloc(sizeof(double) * n);
    int32_t *cutv = (int32_t *)malloc(sizeof(int32_t) * k);
    double *num = (double *)malloc(sizeof(double) * k);
    double *den = (double *)malloc(sizeof(double) * k);
    uint8_t *joined = (uint8_t *)malloc((size_t)n);
    int32_t *rep = (int32_t *)malloc(sizeof(int32_t) * n);
    int32_t *cidx = (int32_t *)malloc(sizeof(int32_t) * n);
    if (!depth || !order || !phi || !om || !p0 || !wb || !pb || !cutv || !num || !den || !joined || !rep || !cidx) {
        rc = ORC_ENOMEM;
        goto done;
    }
    rc = orc_tree_depth(parent, n, root, depth);
    if (rc) goto done;
    rc = orc_tree_order(depth, n, order);
    if (rc) goto done;
    memset(info, 0, sizeof(*info));
    for (int64_t v = 0; v < n; ++v) if (depth[v] > info->max_depth) info->max_depth = depth[v];

    if (sigma == 0.0) sigma = orc_lower_median(parent, len, n);
    if (!(sigma > 0.0)) { rc = ORC_EINVAL; goto done; }
    info->sigma = sigma;
    rc = orc_tree_weights(parent, len, n, root, sigma, omega_mode, phi_kind, alpha_pot, X, d, ld, phi, om, p0);
    if (rc) goto done;

    /* Bounds phi^*, phi_*, omega^*, omega_*, p^*, p_* (Sec. 2.2), sums in
     * ascending vertex order; phi over the n-1 tree edges only. */
    {
        double ps = 0.0, pm = INFINITY, os = 0.0, omn = INFINITY, qs = 0.0, qm = INFINITY;
        for (int64_t v = 0; v < n; ++v) {
            if (v != root) { ps = ps + phi[v]; if (phi[v] < pm) pm = phi[v]; }
            os = os + om[v]; if (om[v] < omn) omn = om[v];
            qs = qs + p0[v]; if (p0[v] < qm) qm = p0[v];
        }
        info->phi_sum = ps; info->phi_min = pm; info->omega_sum = os; info->omega_min = omn;
        info->p_sum = qs; info->p_min = qm;
    }
    info->alpha0_raw = (info->phi_min + info->p_min) / info->omega_sum;
    info->beta0_raw = (info->phi_sum + info->p_sum) / info->omega_min;
    {
        double tt = log2(2.0 * info->omega_sum * info->omega_sum * (info->beta0_raw - info->alpha0_raw)) -
                    log2(info->phi_min + info->p_min);
        info->t_paper = isfinite(tt) ? (int32_t)ceil(tt) : -1;
    }
    if (bracket == 1) {
        info->alpha0 = info->alpha0_raw;
        info->beta0 = nextafter(info->beta0_raw, INFINITY);
    } else {
        info->alpha0 = pow2_floor(info->alpha0_raw);
        info->beta0 = pow2_above(info->beta0_raw);
    }
    if (orc_decide(parent, order, phi, om, p0, n, k, info->beta0, wb, pb, NULL, NULL, NULL, NULL) != k) {
        rc = ORC_EBRACKET;
        goto done;
    }

    /* Algorithm 2: MISO_k lies in (lo, hi] with decide(hi) = YES.  Each step
     * asks decide at the FP64 midpoint and keeps the half that still holds the
     * threshold; it ends when no double lies strictly between the two ends
     * (FP64 resolution, R7) or after max_iters steps. */
    {
        double lo = info->alpha0, hi = info->beta0;
        int32_t steps = 0;
        for (; steps < max_iters; ++steps) {
            const double mid = (lo + hi) / 2.0;
            if (!(lo < mid && mid < hi)) break;
            const int64_t cuts = orc_decide(parent, order, phi, om, p0, n, k, mid, wb, pb, NULL, NULL, NULL, NULL);
            if (cuts < 0) { rc = ORC_ENOMEM; goto done; }
            if (cuts == k) hi = mid; else lo = mid;
        }
        info->alpha = lo; info->beta = hi; info->iters = steps;
    }

    /* Final decision at beta, recording Cut and eta (Algorithm 4). */
    if (orc_decide(parent, order, phi, om, p0, n, k, info->beta, wb, pb, cutv, num, den, joined) != k) {
        rc = ORC_EBRACKET;
        goto done;
    }
    /* Cluster index of each cut vertex: its rank among the first k cuts in
     * x-order (exclusive scan of Cut). */
    for (int64_t v = 0; v < n; ++v) cidx[v] = -1;
    for (int64_t j = 0; j < k; ++j) cidx[cutv[j]] = (int32_t)j;
    /* rep(v): first non-joined vertex on the path from v to the root,
     * resolved in root-first order (reverse x-order). */
    for (int64_t i = n - 1; i >= 0; --i) {
        int32_t v = order[i];
        rep[v] = joined[v] ? rep[parent[v]] : v;
    }
    for (int64_t v = 0; v < n; ++v) labels[v] = cidx[rep[v]];
    {
        double best = -1.0;
        int32_t js = 0;
        for (int64_t j = 0; j < k; ++j) {
            double c = num[j] / den[j];
            if (c > best) { best = c; js = (int32_t)j; }
        }
        info->i_k = best;
        info->jstar = js;
    }
    if (cl_num) for (int64_t j = 0; j < k; ++j) cl_num[j] = num[j];
    if (cl_den) for (int64_t j = 0; j < k; ++j) cl_den[j] = den[j];
    if (cl_size) {
        for (int64_t j = 0; j < k; ++j) cl_size[j] = 0;
        for (int64_t v = 0; v < n; ++v) if (labels[v] >= 0) cl_size[labels[v]]++;
    }
done:
    free(depth); free(order); free(phi); free(om); free(p0); free(wb); free(pb);
    free(cutv); free(num); free(den); free(joined); free(rep); free(cidx);
    return rc;
}

/* ------------------------------------------------------------------ */
/* Adjoint with the tree and the subpartition held fixed               */
/* ------------------------------------------------------------------ */

/* W = sum of tree edge lengths D_e; I = cost of cluster jstar of `labels`
 *   = phi(delta A) / omega(A) with omega the tree degree (R1), alpha = 0:
 *   num = sum of phi_e over tree edges with exactly one end in A,
 *   den = sum over v in A of omega0(v) = 2 * (phi over edges inside A) + num.
 * dI/dphi_e = (den - num)/den^2 on boundary edges, -2 num/den^2 on inner
 * edges; dphi_e/dD_e = -phi_e/sigma and dphi_e/dsigma = phi_e D_e/sigma^2
 * (eq. 2.1; phi_kind 1: -phi_e D_e/sigma^2 and phi_e D_e^2/sigma^3);
 * dD_e/dx_v = (x_v - x_w)/D_e.  Zero-length edges contribute a zero
 * subgradient and are counted in *n_degenerate.
 * gX[n*d] (row-major, FP64) = gW * dW/dX + gI * dI/dX; *gsigma = gI * dI/dsigma.
 * Edge lengths D_e are recomputed from X (FP64, left to right). */
int orc_backward(const float *X, int64_t n, int64_t d, int64_t ld, const int32_t *parent, int32_t root,
                 const int32_t *labels, int32_t jstar, double sigma, int phi_kind, double gW, double gI,
                 double *gX, double *gsigma, double *W_out, double *I_out, int64_t *n_degenerate) {
    if (!X || !parent || !labels || !gX || !gsigma || n < 2 || d < 1 || ld < d || !(sigma > 0.0)) return ORC_EINVAL;
    double *De = (double *)malloc(sizeof(double) * n);
    double *ph = (double *)malloc(sizeof(double) * n);
    if (!De || !ph) { free(De); free(ph); return ORC_ENOMEM; }
    double W = 0.0, num = 0.0, inner = 0.0;
    for (int64_t v = 0; v < n; ++v) {
        if (v == root) { De[v] = 0.0; ph[v] = 0.0; continue; }
        De[v] = sqrt(orc_sqdist(X, ld, d, v, parent[v]));
        ph[v] = flow_of(De[v], sigma, phi_kind);
        W = W + De[v];
        int inv = labels[v] == jstar, inu = labels[parent[v]] == jstar;
        if (inv != inu) num = num + ph[v];
        else if (inv && inu) inner = inner + ph[v];
    }
    double den = 2.0 * inner + num;
    double I = (den > 0.0) ? num / den : 0.0;
    memset(gX, 0, sizeof(double) * n * d);
    double gs = 0.0;
    int64_t ndeg = 0;
    for (int64_t v = 0; v < n; ++v) {
        if (v == root) continue;
        int64_t u = parent[v];
        int inv = labels[v] == jstar, inu = labels[u] == jstar;
        double dIdphi = 0.0;
        if (den > 0.0) {
            if (inv != inu) dIdphi = (den - num) / (den * den);
            else if (inv && inu) dIdphi = -2.0 * num / (den * den);
        }
        double dphidD, dphids;
        if (phi_kind == 1) {
            dphidD = -ph[v] * De[v] / (sigma * sigma);
            dphids = ph[v] * De[v] * De[v] / (sigma * sigma * sigma);
        } else {
            dphidD = -ph[v] / sigma;
            dphids = ph[v] * De[v] / (sigma * sigma);
        }
        gs = gs + gI * dIdphi * dphids;
        if (!(De[v] > 0.0)) { ndeg++; continue; }
        double coef = (gW + gI * dIdphi * dphidD) / De[v];
        const float *xv = X + v * ld, *xu = X + u * ld;
        for (int64_t t = 0; t < d; ++t) {
            double diff = (double)xv[t] - (double)xu[t];
            gX[v * d + t] = gX[v * d + t] + coef * diff;
            gX[u * d + t] = gX[u * d + t] - coef * diff;
        }
    }
    *gsigma = gs;
    if (W_out) *W_out = W;
    if (I_out) *I_out = I;
    if (n_degenerate) *n_degenerate = ndeg;
    free(De); free(ph);
    return ORC_OK;
}
