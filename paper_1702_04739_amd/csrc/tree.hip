// tree.hip -- optimal k-subpartition of a weighted tree on gfx950
// (Sec. 2.2 Algorithms 1-2, parallelised depth by depth as in Sec. 3.6 /
// Algorithm 4).
//
// Algorithm 1 visits the vertices in x-order (depth descending, id ascending)
// and either cuts a vertex from its parent, joins it to its parent, or
// discards it.  Each vertex's decision depends only on its children, so all
// vertices of one depth are decided together (Sec. 3.2), deepest level first.
// A vertex pulls its children's contributions in ascending id order, which is
// exactly the order in which the sequential algorithm folds them into the
// parent, so the FP64 arithmetic is the sequential algorithm's.
//
// Bisection (Algorithm 2) is speculative: one device pass evaluates 64
// thresholds at once (one wave lane each) -- the midpoints of the next six
// bisection levels, or, while every answer so far has gone one way, the next
// 64 midpoints along that direction -- then walks the answers, so the
// sequence of brackets is exactly the sequential one.  The bracket lives on
// the device; the host polls a done flag after every pass.
//
// Once the bracket is narrow most subtrees decide alike over all of it: such
// a subtree's contribution to its parent no longer depends on the threshold,
// so it is frozen (its value written to every lane) and later passes visit
// only the remaining vertices.
#include <cmath>
#include <mutex>
#include <vector>

#include "common.hpp"

namespace iso {

namespace {

#ifndef ISO_SPEC_LEVELS
#define ISO_SPEC_LEVELS 6
#endif
constexpr int SPEC_LEVELS = ISO_SPEC_LEVELS;       // bisection steps resolved per pass
constexpr int M = 1 << SPEC_LEVELS;                // lanes per vertex in a speculative pass
constexpr int NCAND = M - 1;                       // midpoints per pass (the last lane re-checks beta)
// Candidate layouts of a speculative pass.  SPEC_TREE: the 63 midpoints of the
// next six bisection levels in heap order, the last lane re-checks beta.
// SPEC_DOWN / SPEC_UP: the next 64 midpoints along the path on which every
// answer is YES (the bracket's upper end keeps falling) or every answer is NO
// (its lower end keeps rising); the pass resolves the steps up to and
// including the first opposite answer.  While the bisection has only ever
// answered one way the spine is the likely path: from a power-of-two bracket
// far wider than MISO_k the leading steps are a run of YES answers.
constexpr int SPEC_TREE = 0, SPEC_DOWN = 1, SPEC_UP = 2;
// Levels with at most this many vertices are run inside one workgroup
// (several vertices of a level one after another when it has more than 16).
constexpr int NARROW_VERTS = 48;
#ifndef DP_BATCH
#define DP_BATCH 16                          // children loaded per round trip in Algorithm 1 (measured best)
#endif

struct TreeState {
    double alpha, beta;
    double alpha0_raw, beta0_raw, alpha0, beta0;
    double phi_sum, phi_min, om_sum, om_min, p_sum, p_min;
    double sigma;
    double i_k;
    int32_t done, iters, passes, jstar;
    int32_t ncuts, max_iters, k, bad;
    int32_t maxdepth;
    int32_t lo_lane;  // lane of the last pass's final lower end (-1: the lower end did not move)
    int32_t mode;     // candidate layout of the current pass (SPEC_TREE, SPEC_DOWN, SPEC_UP)
    int32_t nfrozen;  // vertices frozen so far
};

template <class T>
__global__ void k_fill_t(T *p, T v, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

template <class T>
void fill_t(T *p, T v, int64_t n, hipStream_t s) {
    if (n <= 0) return;
    unsigned g = grid_for(n, 256);
    if (g > 4096) g = 4096;
    hipLaunchKernelGGL(k_fill_t<T>, dim3(g), dim3(256), 0, s, p, v, n);
    LAUNCH_CHECK();
}

// ------------------------------------------------------------------ validation and depth

// anc = parent, dist = 1 (0 at the root); flags malformed entries.
__global__ void k_check_tree(const int32_t *__restrict__ parent, const double *__restrict__ length, int64_t n,
                             int32_t root, int32_t *__restrict__ anc, int32_t *__restrict__ dist,
                             TreeState *__restrict__ st) {
    int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    int32_t p = parent[v];
    bool bad;
    if (v == root) {
        bad = (p != -1);
        dist[v] = 0;
        anc[v] = -1;
    } else {
        double L = length[v];
        bad = (p < 0 || p >= n || p == v || !(L >= 0.0) || !isfinite(L));
        dist[v] = 1;
        anc[v] = bad ? -1 : p;
    }
    if (bad) atomicOr(&st->bad, 1);
}

__global__ void k_depth_jump(const int32_t *__restrict__ anc_in, const int32_t *__restrict__ dist_in, int64_t n,
                             int32_t *__restrict__ anc_out, int32_t *__restrict__ dist_out) {
    int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    int32_t a = anc_in[v];
    if (a >= 0) {
        dist_out[v] = dist_in[v] + dist_in[a];
        anc_out[v] = anc_in[a];
    } else {
        dist_out[v] = dist_in[v];
        anc_out[v] = -1;
    }
}

// Cycle check (an ancestor pointer that never reached the root) and max depth.
__global__ void k_depth_finish(const int32_t *__restrict__ anc, const int32_t *__restrict__ dist, int64_t n,
                               TreeState *__restrict__ st) {
    int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    if (anc[v] != -1) atomicOr(&st->bad, 2);
    atomicMax(&st->maxdepth, dist[v]);
}

// Sort keys: x-order key (maxdepth - depth) and child-list key (parent + 1).
__global__ void k_sort_keys(const int32_t *__restrict__ depth, const int32_t *__restrict__ parent, int64_t n,
                            int32_t maxdepth, uint32_t *__restrict__ okey, uint32_t *__restrict__ oval,
                            uint32_t *__restrict__ ckey, uint32_t *__restrict__ cval, int32_t *__restrict__ nchild) {
    int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    okey[v] = (uint32_t)(maxdepth - depth[v]);
    oval[v] = (uint32_t)v;
    int32_t p = parent[v];
    ckey[v] = (uint32_t)(p + 1);
    cval[v] = (uint32_t)v;
    if (p >= 0) atomicAdd(&nchild[p], 1);
}

// level_start[L] = first x-order index of level key L (L = maxdepth - depth).
// Output slot of every vertex in the Algorithm 1 passes: a child's slot is
// its position in the concatenated child lists (so a vertex finds its
// children's contributions contiguously), the root takes the last slot.
// cval_sorted[0] is the root; cval_sorted[1 + a] the child at position a.
__global__ void k_slots(const uint32_t *__restrict__ cval_sorted, int64_t n, int32_t *__restrict__ slot) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    slot[cval_sorted[i]] = i == 0 ? (int32_t)(n - 1) : (int32_t)(i - 1);
}

__global__ void k_level_starts(const uint32_t *__restrict__ okey_sorted, int64_t n, int32_t maxdepth,
                               int32_t *__restrict__ level_start) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint32_t key = okey_sorted[i];
    if (i == 0 || okey_sorted[i - 1] != key) level_start[key] = (int32_t)i;
    if (i == 0) level_start[maxdepth + 1] = (int32_t)n;
}

// ------------------------------------------------------------------ weights (eqs. 2.1-2.2)

__global__ void k_phi(const int32_t *__restrict__ parent, const double *__restrict__ length, int64_t n,
                      const TreeState *__restrict__ st, int phi_kind, double *__restrict__ phi,
                      double *__restrict__ p0) {
    int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    const double sigma = st->sigma;
    double f = 0.0;
    if (parent[v] >= 0) {
        const double dist = length[v];
        f = (phi_kind == ISO_PHI_GAUSS_SQ) ? exp(-(dist * dist) / (2.0 * sigma * sigma)) : exp(-dist / sigma);
    }
    phi[v] = f;
    p0[v] = 0.0;
}

// omega0(v): sum over tree neighbours w of v in ascending w of phi(vw),
// starting from +0.0 (children come sorted by id; the parent is merged in).
__global__ void k_omega_tree(const int32_t *__restrict__ parent, const double *__restrict__ phi,
                             const uint32_t *__restrict__ kids, const int32_t *__restrict__ koff, int64_t n,
                             double *__restrict__ om0) {
    int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    const int32_t p = parent[v];
    const double fv = phi[v];
    double s = 0.0;
    bool parent_done = p < 0;
    // the children in batches of 16: all loads of a batch first (a hub's
    // children are 40 round trips instead of 629), then the sum in id order
    const int32_t a1 = koff[v + 1];
    for (int32_t a0 = koff[v]; a0 < a1; a0 += 16) {
        int32_t c[16];
        double f[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) c[u] = (int32_t)kids[min(a0 + u, a1 - 1)];
#pragma unroll
        for (int u = 0; u < 16; ++u) f[u] = phi[c[u]];
        const int nb = min(16, a1 - a0);
        for (int u = 0; u < nb; ++u) {
            if (!parent_done && p < c[u]) {
                s = s + fv;
                parent_done = true;
            }
            s = s + f[u];
        }
    }
    if (!parent_done) s = s + fv;
    om0[v] = s;
}

// Sums and minima of phi (tree edges), omega0 and p0; bracket of Algorithm 2.
// k_stats_part: STATS_BLOCKS workgroups, each over a contiguous range of the
// vertices, write partial sums and minima; k_stats (one workgroup) combines
// them in a fixed order and sets the bracket.
constexpr int STATS_BLOCKS = 256;

__global__ __launch_bounds__(256) void k_stats_part(const int32_t *__restrict__ parent, const double *__restrict__ phi,
                                                    const double *__restrict__ om0, const double *__restrict__ p0,
                                                    int64_t n, double *__restrict__ part) {
    __shared__ double s_sum[3][256];
    __shared__ double s_min[3][256];
    const int64_t per = (n + STATS_BLOCKS - 1) / STATS_BLOCKS;
    const int64_t lo = (int64_t)blockIdx.x * per, hi = min(n, lo + per);
    double ps = 0.0, os = 0.0, qs = 0.0;
    double pm = __builtin_huge_val(), om = __builtin_huge_val(), qm = __builtin_huge_val();
    for (int64_t v = lo + threadIdx.x; v < hi; v += 256) {
        const double f = phi[v], o = om0[v], q = p0[v];
        if (parent[v] >= 0) {
            ps = ps + f;
            pm = fmin(pm, f);
        }
        os = os + o;
        om = fmin(om, o);
        qs = qs + q;
        qm = fmin(qm, q);
    }
    s_sum[0][threadIdx.x] = ps;
    s_sum[1][threadIdx.x] = os;
    s_sum[2][threadIdx.x] = qs;
    s_min[0][threadIdx.x] = pm;
    s_min[1][threadIdx.x] = om;
    s_min[2][threadIdx.x] = qm;
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
        if ((int)threadIdx.x < w) {
            for (int q = 0; q < 3; ++q) {
                s_sum[q][threadIdx.x] = s_sum[q][threadIdx.x] + s_sum[q][threadIdx.x + w];
                s_min[q][threadIdx.x] = fmin(s_min[q][threadIdx.x], s_min[q][threadIdx.x + w]);
            }
        }
        __syncthreads();
    }
    if (threadIdx.x < 3) {
        part[blockIdx.x * 6 + threadIdx.x] = s_sum[threadIdx.x][0];
        part[blockIdx.x * 6 + 3 + threadIdx.x] = s_min[threadIdx.x][0];
    }
}

__global__ __launch_bounds__(256) void k_stats(const double *__restrict__ part, int bracket,
                                               TreeState *__restrict__ st) {
    static_assert(STATS_BLOCKS == 256, "one partial per thread");
    __shared__ double s_sum[3][256];
    __shared__ double s_min[3][256];
    for (int q = 0; q < 3; ++q) {
        s_sum[q][threadIdx.x] = part[threadIdx.x * 6 + q];
        s_min[q][threadIdx.x] = part[threadIdx.x * 6 + 3 + q];
    }
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
        if ((int)threadIdx.x < w) {
            for (int q = 0; q < 3; ++q) {
                s_sum[q][threadIdx.x] = s_sum[q][threadIdx.x] + s_sum[q][threadIdx.x + w];
                s_min[q][threadIdx.x] = fmin(s_min[q][threadIdx.x], s_min[q][threadIdx.x + w]);
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        st->phi_sum = s_sum[0][0];
        st->om_sum = s_sum[1][0];
        st->p_sum = s_sum[2][0];
        st->phi_min = s_min[0][0];
        st->om_min = s_min[1][0];
        st->p_min = s_min[2][0];
        const double a0 = (st->phi_min + st->p_min) / st->om_sum;
        const double b0 = (st->phi_sum + st->p_sum) / st->om_min;
        st->alpha0_raw = a0;
        st->beta0_raw = b0;
        double a, b;
        if (bracket == ISO_BRACKET_PAPER) {
            a = a0;
            b = nextafter(b0, __builtin_huge_val());
        } else {
            int e;
            if (a0 > 0.0) {
                frexp(a0, &e);
                a = ldexp(1.0, e - 1);
            } else {
                a = 0.0;
            }
            frexp(b0, &e);
            b = ldexp(1.0, e);
        }
        st->alpha0 = a;
        st->beta0 = b;
        st->alpha = a;
        st->beta = b;
        st->done = 0;
        st->iters = 0;
        st->passes = 0;
        if (!(b0 > 0.0) || !isfinite(b0)) st->bad |= 4;
    }
}

// ------------------------------------------------------------------ Algorithm 1, one vertex

// Everything Algorithm 1 reads about the vertex at x-order position q, packed
// so that a level's first load is indexed by the position itself.
struct __attribute__((aligned(16))) VtxMeta {
    int32_t a0, a1;     // its children's output slots a0 .. a1-1
    int32_t slot, v;    // its own output slot and id
    int32_t root, pad;  // 1 for the root
    double om0, p0;     // its weight and potential
    double fe;          // phi of its parent edge (0 at the root)
};
static_assert(sizeof(VtxMeta) == 48, "a vertex record is three 16-byte pieces");

struct DPArgs {
    const int32_t *level_start;  // level L occupies entries level_start[L] .. level_start[L+1]-1 of the position list
    const int32_t *act;          // position list (x-order positions of the vertices a pass visits), or NULL = all
    const VtxMeta *meta;  // [n] by x-order position
    const int32_t *nextl;  // [M] lane holding the next larger evaluated threshold, -1 if it was not evaluated
    uint64_t *smask;       // [slot] bit l: the vertex's subtree decides alike at lane l's threshold and at
                           // lane nextl[l]'s (~0 for frozen vertices)
    const double *Nvals;
    double2 *cpw;  // [slot][MM] contribution (p, omega) to the parent
    int32_t *cnt;
    uint8_t *cut, *joined;
    double *num, *den;
    TreeState *st;
};

// Decision of Algorithm 1 for vertex v at threshold Nvals[m].  The vertex's
// (omega, p) start from (omega0, p0) and absorb the children's contributions
// in ascending child id; its own contribution to its parent is
//   cut:     p += phi(e)           (the edge joins the boundary),
//   join:    omega += omega(x), p += p(x),
//   discard: p += phi(e).
//
// With MASK (speculative passes, one wave of MM = 64 lanes per vertex) the wave
// also records, for every lane l whose next larger threshold was evaluated,
// whether the whole subtree takes the same decisions at both thresholds.  A
// vertex's decision is monotone in N for fixed (omega, p) -- discard, then
// join, then cut as N grows -- and (omega, p) are fixed when every child's
// subtree is constant, so a subtree that decides alike at both ends of an
// interval decides alike, and contributes the same, everywhere inside it.
template <int MM, bool REC, bool MASK>
__device__ inline void dp_vertex_vm(const DPArgs &A, const VtxMeta vm, int m) {
    const double N = A.Nvals[m];
    double w = vm.om0;
    double p = vm.p0;
    int32_t c_cnt = 0;
    uint64_t sm = ~0ull;
    // The children's contributions sit contiguously at slots a0 .. a1-1
    // (ascending child id), (p, omega) packed in 16 bytes; DP_BATCH children
    // are loaded at once, the sums still run one child after another.
    const int64_t a0 = vm.a0, a1 = vm.a1;
    for (int64_t a = a0; a < a1; a += DP_BATCH) {
        const int64_t rem = a1 - a;
        double2 pw[DP_BATCH];
        int32_t cc[DP_BATCH];
        uint64_t cm[DP_BATCH];
#pragma unroll
        for (int u = 0; u < DP_BATCH; ++u) {
            const int64_t ch = u < rem ? a + u : a1 - 1;
            const int64_t c = ch * MM + m;
            pw[u] = A.cpw[c];
            cc[u] = A.cnt[c];
            if (MASK) cm[u] = A.smask[ch];
        }
#pragma unroll
        for (int u = 0; u < DP_BATCH; ++u) {
            if (u < rem) {
                p = p + pw[u].x;
                w = w + pw[u].y;
                c_cnt += cc[u];
                if (MASK) sm &= cm[u];
            }
        }
    }
    const bool is_root = vm.root != 0;
    const double fe = vm.fe;
    const double lhs = fe + p;
    const double rhs = N * w;
    double op, ow;
    int iscut = 0, isjoin = 0;
    if (lhs <= rhs) {
        iscut = 1;
        op = fe;
        ow = 0.0;
    } else if (!is_root && (p - fe) < rhs) {
        isjoin = 1;
        op = p;
        ow = w;
    } else {
        op = fe;
        ow = 0.0;
    }
    const int64_t o = (int64_t)vm.slot * MM + m;
    A.cpw[o] = make_double2(op, ow);
    A.cnt[o] = c_cnt + iscut;
    if (MASK) {
        const int dec = iscut * 2 + isjoin;
        const int nx = A.nextl[m];
        const int dn = __shfl(dec, nx < 0 ? m : nx, 64);
        const uint64_t eq = __ballot(nx >= 0 && dn == dec);
        if (m == 0) A.smask[vm.slot] = sm & eq;
    }
    if (REC) {
        const int32_t v = vm.v;
        A.cut[v] = (uint8_t)iscut;
        A.joined[v] = (uint8_t)isjoin;
        A.num[v] = lhs;
        A.den[v] = w;
    }
}

template <int MM, bool REC, bool MASK>
__device__ inline void dp_vertex(const DPArgs &A, int32_t q, int m) {
    dp_vertex_vm<MM, REC, MASK>(A, A.meta[q], m);
}

// The packed record of every x-order position (after slots and weights).
__global__ void k_vtx_meta(const int32_t *__restrict__ order, const int32_t *__restrict__ koff,
                           const int32_t *__restrict__ slot, const int32_t *__restrict__ parent,
                           const double *__restrict__ om0, const double *__restrict__ p0,
                           const double *__restrict__ phi, int64_t n, VtxMeta *__restrict__ meta) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n) return;
    const int32_t v = order[q];
    VtxMeta vm;
    vm.a0 = koff[v];
    vm.a1 = koff[v + 1];
    vm.slot = slot[v];
    vm.v = v;
    vm.root = parent[v] < 0 ? 1 : 0;
    vm.pad = 0;
    vm.om0 = om0[v];
    vm.p0 = p0[v];
    vm.fe = parent[v] < 0 ? 0.0 : phi[v];
    meta[q] = vm;
}

// One wide level: MM consecutive threads per vertex (entries lo .. hi-1 of the
// position list).
template <int MM, bool REC, bool MASK>
__global__ __launch_bounds__(256) void k_dp_level(DPArgs A, int32_t lo, int32_t hi) {
    if (!REC && A.st->done) return;
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t e = lo + gid / MM;
    const int m = (int)(gid % MM);
    if (e >= hi) return;
    const int32_t q = A.act ? A.act[e] : (int32_t)e;
    dp_vertex<MM, REC, MASK>(A, q, m);
}

// A run of narrow levels [L0, L1) inside one workgroup (every level at most
// narrow_cap<REC>() vertices), a barrier between levels.  The vertex records
// of the next level and the positions of the one after, which do not depend
// on this level's results, are loaded while this level runs and kept in LDS,
// so a level waits for one round trip (its children's contributions) instead
// of three (position, record, children).
template <bool REC>
constexpr int narrow_cap() { return REC ? 1024 : NARROW_VERTS; }
// threads of the narrow kernel: 1024 one-lane vertices, or 8 vertices of 64
// lanes (512 threads, so that a lane may use 256 registers)
template <int MM>
constexpr int narrow_threads() { return MM == 1 ? 1024 : 512; }

template <int MM, bool REC, bool MASK>
__global__ __launch_bounds__(narrow_threads<MM>()) void k_dp_narrow(DPArgs A, int32_t L0, int32_t L1) {
    if (!REC && A.st->done) return;
    constexpr int CAP = narrow_cap<REC>();
    static_assert(CAP <= narrow_threads<MM>(), "one thread per record of a narrow level");
    __shared__ VtxMeta smeta[2][CAP];
    __shared__ int32_t spos[2][CAP];
    const int tid = threadIdx.x;
    const int m = tid % MM;
    const int slot = tid / MM;
    const int slots = blockDim.x / MM;
    const bool own = tid < CAP;
    // position of entry e of the list (the list is the identity without A.act)
    auto pos_of = [&](int32_t e) { return A.act ? A.act[e] : e; };
    // level L0's records, level L0+1's positions
    {
        const int32_t lo = A.level_start[L0], hi = A.level_start[L0 + 1];
        if (own && tid < hi - lo) smeta[0][tid] = A.meta[pos_of(lo + tid)];
        if (L0 + 1 < L1) {
            const int32_t hi1 = A.level_start[L0 + 2];
            if (own && tid < hi1 - hi) spos[1][tid] = pos_of(hi + tid);
        }
    }
    __syncthreads();
    for (int32_t L = L0; L < L1; ++L) {
        const int b = (L - L0) & 1;
        const int32_t lo = A.level_start[L], hi = A.level_start[L + 1];
        // level L+1's records (positions already in LDS) and level L+2's
        // positions: issued before this level's work, stored after it
        uint4 nx0{}, nx1{}, nx2{};  // one record as three 16-byte pieces (kept in registers)
        int32_t np = 0;
        bool has_m = false, has_p = false;
        if (L + 1 < L1) {
            const int32_t hi1 = A.level_start[L + 2];
            if (own && tid < hi1 - hi) {
                const uint4 *src = reinterpret_cast<const uint4 *>(A.meta + spos[b ^ 1][tid]);
                nx0 = src[0];
                nx1 = src[1];
                nx2 = src[2];
                has_m = true;
            }
            if (L + 2 < L1) {
                const int32_t hi2 = A.level_start[L + 3];
                if (own && tid < hi2 - hi1) {
                    np = pos_of(hi1 + tid);
                    has_p = true;
                }
            }
        }
        for (int32_t e = lo + slot; e < hi; e += slots) dp_vertex_vm<MM, REC, MASK>(A, smeta[b][e - lo], m);
        if (has_m) {
            uint4 *dst = reinterpret_cast<uint4 *>(&smeta[b ^ 1][tid]);
            dst[0] = nx0;
            dst[1] = nx1;
            dst[2] = nx2;
        }
        if (has_p) spos[b][tid] = np;
        __syncthreads();
    }
}

// In-order successor of heap node h (1-based) in the complete tree of NCAND
// nodes, as a lane (node - 1); the largest node's successor is beta's lane.
__device__ inline int tree_next_lane(int lane) {
    int h = lane + 1;
    if (h < M / 2) {  // leftmost node of the right subtree
        h = 2 * h + 1;
        while (h < M / 2) h = 2 * h;
        return h - 1;
    }
    while (h > 1 && (h & 1)) h >>= 1;  // climb while a right child
    return h == 1 ? NCAND : (h >> 1) - 1;
}

// Thresholds of one speculative pass and, per lane, the lane holding the next
// larger threshold (-1: not evaluated in this pass).  The layout follows the
// answers so far: SPEC_DOWN while the lower end of the bracket has never
// moved, SPEC_UP while the upper end has never moved, else SPEC_TREE.  Every
// threshold repeats exactly the midpoint arithmetic the sequential bisection
// performs on its way to it.  Launched with M threads.
//   SPEC_TREE: node q over bracket (lo, hi) has midpoint (lo+hi)/2, left child
//              (lo, mid) (answer YES), right child (mid, hi) (answer NO);
//              thread q walks from the root to its node (the bits of q+1 below
//              the leading one, left = 0); the spare lane re-checks beta.
//   SPEC_DOWN: lane q holds the (q+1)-th midpoint when every answer is YES.
//   SPEC_UP:   lane q holds the (q+1)-th midpoint when every answer is NO.
__global__ void k_make_cands(TreeState *__restrict__ st, double *__restrict__ Nvals, int32_t *__restrict__ nextl) {
    if (st->done) return;
    const int q = threadIdx.x;
    if (q >= M) return;
    double lo = st->alpha, hi = st->beta;
    const int mode = lo == st->alpha0 ? SPEC_DOWN : (hi == st->beta0 ? SPEC_UP : SPEC_TREE);
    if (q == 0) st->mode = mode;
    if (mode == SPEC_DOWN) {
        for (int l = 0; l < q; ++l) hi = (lo + hi) / 2.0;
        Nvals[q] = (lo + hi) / 2.0;
        nextl[q] = q - 1;
        return;
    }
    if (mode == SPEC_UP) {
        for (int l = 0; l < q; ++l) lo = (lo + hi) / 2.0;
        Nvals[q] = (lo + hi) / 2.0;
        nextl[q] = q + 1 < M ? q + 1 : -1;
        return;
    }
    if (q == NCAND) {
        Nvals[NCAND] = hi;
        nextl[NCAND] = -1;
        return;
    }
    const int node = q + 1;
    const int lvl = 31 - __clz(node);  // depth of the node below the root
    for (int l = lvl - 1; l >= 0; --l) {
        const double mid = (lo + hi) / 2.0;
        if ((node >> l) & 1)
            lo = mid;
        else
            hi = mid;
    }
    Nvals[q] = (lo + hi) / 2.0;
    nextl[q] = tree_next_lane(q);
}

// Walks the answers of one pass: YES (>= k cuts) => beta = mid, else alpha = mid
// (SPEC_TREE: six levels; SPEC_DOWN / SPEC_UP: up to and including the first
// NO / YES).  lo_lane records the lane of the final lower end when it moved.
__global__ void k_resolve(TreeState *__restrict__ st, const double *__restrict__ Nvals,
                          const int32_t *__restrict__ cnt, int32_t root_slot) {
    if (threadIdx.x != 0 || st->done) return;
    st->passes += 1;
    st->lo_lane = -1;
    const int mode = st->mode;
    const int steps = mode == SPEC_TREE ? SPEC_LEVELS : M;
    int q = 0;
    for (int l = 0; l < steps; ++l) {
        const double a = st->alpha, b = st->beta;
        const double mid = (a + b) / 2.0;
        if (mid <= a || mid >= b || st->iters >= st->max_iters) {
            st->done = 1;
            return;
        }
        if (mid != Nvals[q]) {  // cannot happen: the candidates were built from the same bracket
            st->bad |= 8;
            st->done = 1;
            return;
        }
        const bool yes = cnt[(int64_t)root_slot * M + q] >= st->k;
        st->iters += 1;
        if (yes) {
            st->beta = mid;
        } else {
            st->alpha = mid;
            st->lo_lane = q;
        }
        if (mode == SPEC_TREE) {
            q = yes ? 2 * q + 1 : 2 * q + 2;
        } else {
            if ((mode == SPEC_DOWN) != yes) break;  // the walk left the spine
            q = l + 1;
        }
    }
    if (mode == SPEC_TREE && cnt[(int64_t)root_slot * M + NCAND] < st->k) st->bad |= 16;  // beta must stay YES
    const double a = st->alpha, b = st->beta;
    const double mid = (a + b) / 2.0;
    if (mid <= a || mid >= b || st->iters >= st->max_iters) st->done = 1;
}

// Freezes the vertices whose subtree decides alike over the whole new bracket
// [alpha, beta] (bit lo_lane of the mask): every later threshold lies inside
// it, so their contribution is the one at lane lo_lane, now written to every
// lane; their mask becomes all ones and later passes skip them.  One thread
// per entry of the position list.
__global__ void k_freeze(DPArgs A, int32_t nact, uint8_t *__restrict__ frozen) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int lo = A.st->lo_lane;
    bool froze = false;
    if (e < nact && !A.st->done && lo >= 0) {
        const int32_t q = A.act ? A.act[e] : (int32_t)e;
        if (!frozen[q]) {
            const int64_t slot = A.meta[q].slot;
            if ((A.smask[slot] >> lo) & 1ull) {
                const double2 v = A.cpw[slot * M + lo];
                const int32_t c = A.cnt[slot * M + lo];
                for (int l = 0; l < M; ++l) {
                    A.cpw[slot * M + l] = v;
                    A.cnt[slot * M + l] = c;
                }
                A.smask[slot] = ~0ull;
                frozen[q] = 1;
                froze = true;
            }
        }
    }
    const uint64_t b = __ballot(froze);
    if (b && (threadIdx.x & 63) == __ffsll((unsigned long long)b) - 1) atomicAdd(&A.st->nfrozen, __popcll(b));
}

// Position list without the frozen vertices (stable, so still in x-order):
// keep flags, their exclusive scan, the scatter, and the level starts.
__global__ void k_keep_flags(const int32_t *__restrict__ act, int32_t nact, const uint8_t *__restrict__ frozen,
                             int32_t *__restrict__ keep) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e > nact) return;
    keep[e] = e == nact ? 0 : (frozen[act ? act[e] : (int32_t)e] ? 0 : 1);
}

__global__ void k_compact(const int32_t *__restrict__ act, int32_t nact, const int32_t *__restrict__ keep,
                          const int32_t *__restrict__ kpos, int32_t *__restrict__ act_out) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nact || !keep[e]) return;
    act_out[kpos[e]] = act ? act[e] : (int32_t)e;
}

__global__ void k_active_starts(const int32_t *__restrict__ ls_old, int32_t nl, const int32_t *__restrict__ kpos,
                                int32_t *__restrict__ ls_new) {
    const int32_t L = (int32_t)(blockIdx.x * blockDim.x + threadIdx.x);
    if (L < nl) ls_new[L] = kpos[ls_old[L]];
}

__global__ void k_set_final_N(TreeState *__restrict__ st, double *__restrict__ Nvals) {
    if (threadIdx.x == 0) Nvals[0] = st->beta;
}

// ------------------------------------------------------------------ labels (Algorithm 4)

__global__ void k_cut_in_xorder(const int32_t *__restrict__ order, const uint8_t *__restrict__ cut, int64_t n,
                                int32_t *__restrict__ cf) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    cf[i] = cut[order[i]];
}

// Cluster index of each vertex that is one of the first k cuts in x-order
// (exclusive scan of Cut), -1 otherwise; rep pointer = parent if joined.
__global__ void k_cluster_index(const int32_t *__restrict__ order, const uint8_t *__restrict__ cut,
                                const int32_t *__restrict__ rank, const uint8_t *__restrict__ joined,
                                const int32_t *__restrict__ parent, int64_t n, int32_t k,
                                int32_t *__restrict__ cidx, int32_t *__restrict__ rep) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t v = order[i];
    cidx[v] = (cut[v] && rank[i] < k) ? rank[i] : -1;
    rep[v] = joined[v] ? parent[v] : v;
}

__global__ void k_rep_jump(const int32_t *__restrict__ rin, int64_t n, int32_t *__restrict__ rout) {
    int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    rout[v] = rin[rin[v]];
}

__global__ void k_labels(const int32_t *__restrict__ rep, const int32_t *__restrict__ cidx,
                         const double *__restrict__ num, const double *__restrict__ den, int64_t n,
                         int32_t *__restrict__ labels, double *__restrict__ cl_num, double *__restrict__ cl_den) {
    int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    const int32_t l = cidx[rep[v]];
    labels[v] = l;
    const int32_t j = cidx[v];
    if (j >= 0) {
        cl_num[j] = num[v];
        cl_den[j] = den[v];
    }
}

// i_k = max_j num_j / den_j, jstar = smallest argmax; cuts at beta.
__global__ void k_final_cost(const double *__restrict__ cl_num, const double *__restrict__ cl_den, int32_t k,
                             const int32_t *__restrict__ cnt, int32_t root_slot, TreeState *__restrict__ st) {
    if (threadIdx.x != 0) return;
    double best = -1.0;
    int js = 0;
    for (int j = 0; j < k; ++j) {
        const double c = cl_num[j] / cl_den[j];
        if (c > best) {
            best = c;
            js = j;
        }
    }
    st->i_k = best;
    st->jstar = js;
    st->ncuts = cnt[root_slot];
}

// ------------------------------------------------------------------ plan

struct SubPlan {
    int64_t n;
    int32_t k;
    int32_t *anc0, *anc1, *dist0, *dist1;
    uint32_t *okey, *oval, *ckey, *cval, *tk, *tv;
    int32_t *nchild, *koff, *slot, *level_start, *cf, *rank, *cidx, *rep0, *rep1, *cnt, *cl_size_tmp, *lab_tmp, *scan_scratch;
    double2 *cpw;
    double *phi, *om0, *p0, *Nvals, *num, *den, *cl_num_tmp, *cl_den_tmp;
    double *stats_part;             // [STATS_BLOCKS][6] partial sums and minima
    uint8_t *cut, *joined;
    TreeState *st;
    void *sort_scratch, *sel_scratch;
    VtxMeta *meta;  // per x-order position
    uint64_t *smask;                   // [slot] subtree masks of the speculative passes
    uint8_t *frozen;                   // [x-order position]
    int32_t *act0, *act1, *keep, *kpos, *als0, *als1, *nextl;  // position lists, their level starts, next lanes

    void carve(Arena &a) {
        anc0 = a.take<int32_t>(n);
        anc1 = a.take<int32_t>(n);
        dist0 = a.take<int32_t>(n);
        dist1 = a.take<int32_t>(n);
        okey = a.take<uint32_t>(n);
        oval = a.take<uint32_t>(n);
        ckey = a.take<uint32_t>(n);
        cval = a.take<uint32_t>(n);
        tk = a.take<uint32_t>(n);
        tv = a.take<uint32_t>(n);
        nchild = a.take<int32_t>(n + 1);
        koff = a.take<int32_t>(n + 1);
        slot = a.take<int32_t>(n);
        level_start = a.take<int32_t>(n + 2);
        cf = a.take<int32_t>(n);
        rank = a.take<int32_t>(n);
        cidx = a.take<int32_t>(n);
        rep0 = a.take<int32_t>(n);
        rep1 = a.take<int32_t>(n);
        cnt = a.take<int32_t>((size_t)n * M);
        cl_size_tmp = a.take<int32_t>(k);
        lab_tmp = a.take<int32_t>(n);
        scan_scratch = a.take<int32_t>(scan_scratch_bytes(n + 1) / sizeof(int32_t));
        phi = a.take<double>(n);
        om0 = a.take<double>(n);
        p0 = a.take<double>(n);
        cpw = a.take<double2>((size_t)n * M);
        Nvals = a.take<double>(M);
        num = a.take<double>(n);
        den = a.take<double>(n);
        cl_num_tmp = a.take<double>(k);
        cl_den_tmp = a.take<double>(k);
        stats_part = a.take<double>(STATS_BLOCKS * 6);
        cut = a.take<uint8_t>(n);
        joined = a.take<uint8_t>(n);
        st = a.take<TreeState>(1);
        sort_scratch = a.take<char>(radix_sort_scratch_bytes(n));
        sel_scratch = a.take<char>(radix_select_scratch_bytes());
        meta = a.take<VtxMeta>(n);
        smask = a.take<uint64_t>(n);
        frozen = a.take<uint8_t>(n);
        act0 = a.take<int32_t>(n);
        act1 = a.take<int32_t>(n);
        keep = a.take<int32_t>(n + 1);
        kpos = a.take<int32_t>(n + 1);
        als0 = a.take<int32_t>(n + 2);
        als1 = a.take<int32_t>(n + 2);
        nextl = a.take<int32_t>(M);
    }
};

size_t sub_plan_bytes(int64_t n, int32_t k) {
    SubPlan p{};
    p.n = n;
    p.k = k;
    Arena a;
    p.carve(a);
    return a.used;
}

int bits_for(int64_t maxval) {
    int b = 0;
    while (b < 32 && (int64_t(1) << b) <= maxval) ++b;
    return b < 1 ? 1 : b;
}

// Launches Algorithm 1 over all levels, deepest first, grouping runs of
// narrow levels into single-workgroup launches.
// ls holds the level starts of A's position list (A.level_start on the device).
template <int MM, bool REC, bool MASK>
void launch_levels(const DPArgs &A, const std::vector<int32_t> &ls, int32_t maxdepth, hipStream_t s) {
    const int narrow_cap = iso::narrow_cap<REC>();
    int32_t L = 0;
    while (L <= maxdepth) {
        const int32_t width = ls[L + 1] - ls[L];
        if (width <= narrow_cap) {
            int32_t L1 = L;
            bool any = false;
            while (L1 <= maxdepth && ls[L1 + 1] - ls[L1] <= narrow_cap) {
                any = any || ls[L1 + 1] > ls[L1];
                ++L1;
            }
            if (any) {
                hipLaunchKernelGGL((k_dp_narrow<MM, REC, MASK>), dim3(1), dim3(narrow_threads<MM>()), 0, s, A, L,
                                   L1);
                LAUNCH_CHECK();
            }
            L = L1;
        } else {
            const int64_t threads = (int64_t)width * MM;
            hipLaunchKernelGGL((k_dp_level<MM, REC, MASK>), dim3(grid_for(threads, 256)), dim3(256), 0, s, A, ls[L],
                               ls[L + 1]);
            LAUNCH_CHECK();
            ++L;
        }
    }
}

// Single k (kmax == 0): the bisection runs on the device, several passes per
// host check.  All k (kmax >= 2): for every k = 2 .. kmax the same bisection as
// a single-k call, planned on the host: each pass gives every unfinished k the
// next levels of its bisection tree (equal midpoints of different k share a
// lane), and each k then walks its own answers; i_k_all[k - 2] and the label
// rows labels_all[(k - 2) n ..] receive the results.
void run_sub(SubPlan &P, const int32_t *parent, const double *length, int32_t root, double sigma,
             const iso_sub_opts &o, int32_t *labels, double *i_k, double *cl_num, double *cl_den, int32_t *cl_size,
             iso_sub_info *info, hipStream_t s, int32_t kmax = 0, double *i_k_all = nullptr,
             int32_t *labels_all = nullptr, int32_t *passes_out = nullptr) {
    const int64_t n = P.n;
    const int32_t k = P.k;
    const unsigned gn = grid_for(n, 256);
    const bool timed = timing().enabled != 0;
    EventPair whole(timed);
    whole.start(s);
    // state
    TreeState h0{};
    h0.max_iters = o.max_iters > 0 ? o.max_iters : 2000;
    h0.k = k;
    h0.sigma = sigma;
    HIP_CHECK(hipMemcpyAsync(P.st, &h0, sizeof(h0), hipMemcpyHostToDevice, s));

    // validation + depth by pointer jumping
    hipLaunchKernelGGL(k_check_tree, dim3(gn), dim3(256), 0, s, parent, length, n, root, P.anc0, P.dist0, P.st);
    LAUNCH_CHECK();
    int32_t *ai = P.anc0, *ao = P.anc1, *di = P.dist0, *dout = P.dist1;
    for (int it = 0; it <= ceil_log2(n); ++it) {
        hipLaunchKernelGGL(k_depth_jump, dim3(gn), dim3(256), 0, s, ai, di, n, ao, dout);
        LAUNCH_CHECK();
        std::swap(ai, ao);
        std::swap(di, dout);
    }
    hipLaunchKernelGGL(k_depth_finish, dim3(gn), dim3(256), 0, s, ai, di, n, P.st);
    LAUNCH_CHECK();
    TreeState h{};
    HIP_CHECK(hipMemcpyAsync(&h, P.st, sizeof(h), hipMemcpyDeviceToHost, s));
    HIP_CHECK(hipStreamSynchronize(s));
    ISO_REQUIRE(!(h.bad & 1), ISO_ERR_INVALID_ARG,
                "parent/length malformed: parent[root] must be -1, other parents in [0,n) and not self, lengths finite "
                "and >= 0");
    ISO_REQUIRE(!(h.bad & 2), ISO_ERR_INVALID_ARG, "parent array has a cycle (not a tree rooted at %d)", root);
    const int32_t maxdepth = h.maxdepth;
    const int32_t *depth = di;

    // x-order and child lists (stable radix sorts)
    fill_t<int32_t>(P.nchild, 0, n + 1, s);
    hipLaunchKernelGGL(k_sort_keys, dim3(gn), dim3(256), 0, s, depth, parent, n, maxdepth, P.okey, P.oval, P.ckey,
                       P.cval, P.nchild);
    LAUNCH_CHECK();
    radix_sort_pairs_u32(P.okey, P.oval, P.tk, P.tv, n, bits_for(maxdepth), P.sort_scratch, s);
    radix_sort_pairs_u32(P.ckey, P.cval, P.tk, P.tv, n, bits_for(n), P.sort_scratch, s);
    exclusive_scan_i32(P.nchild, P.koff, n + 1, nullptr, P.scan_scratch, s);
    hipLaunchKernelGGL(k_level_starts, dim3(gn), dim3(256), 0, s, P.okey, n, maxdepth, P.level_start);
    LAUNCH_CHECK();
    const int32_t *order = reinterpret_cast<const int32_t *>(P.oval);
    const uint32_t *kids = P.cval + 1;  // the root (key 0) sorts first
    hipLaunchKernelGGL(k_slots, dim3(gn), dim3(256), 0, s, P.cval, n, P.slot);
    LAUNCH_CHECK();
    const int32_t root_slot = (int32_t)(n - 1);

    // sigma, phi, omega0, stats, bracket
    if (sigma == 0.0) {
        radix_select_f64(length, parent, n, (n - 2) / 2, &P.st->sigma, P.sel_scratch, s);
    }
    hipLaunchKernelGGL(k_phi, dim3(gn), dim3(256), 0, s, parent, length, n, P.st, o.phi, P.phi, P.p0);
    LAUNCH_CHECK();
    // vertex weights: the tree degree, or the caller's full-graph weights;
    // potential p: zero, or the caller's (eq. 2.3)
    const double *om0 = P.om0, *p0 = o.p0 ? o.p0 : P.p0;
    if (o.omega == ISO_OMEGA_FULL) {
        om0 = o.omega0;
    } else {
        hipLaunchKernelGGL(k_omega_tree, dim3(gn), dim3(256), 0, s, parent, P.phi, kids, P.koff, n, P.om0);
        LAUNCH_CHECK();
    }
    hipLaunchKernelGGL(k_stats_part, dim3(STATS_BLOCKS), dim3(256), 0, s, parent, P.phi, om0, p0, n, P.stats_part);
    LAUNCH_CHECK();
    hipLaunchKernelGGL(k_stats, dim3(1), dim3(256), 0, s, P.stats_part, o.bracket, P.st);
    LAUNCH_CHECK();
    std::vector<int32_t> ls(maxdepth + 2);
    HIP_CHECK(hipMemcpyAsync(ls.data(), P.level_start, sizeof(int32_t) * (maxdepth + 2), hipMemcpyDeviceToHost, s));
    HIP_CHECK(hipMemcpyAsync(&h, P.st, sizeof(h), hipMemcpyDeviceToHost, s));
    HIP_CHECK(hipStreamSynchronize(s));
    ISO_REQUIRE(h.sigma > 0.0 && std::isfinite(h.sigma), ISO_ERR_INVALID_ARG,
                "sigma must be positive (the median edge length is %g)", h.sigma);
    ISO_REQUIRE(!(h.bad & 4), ISO_ERR_INVALID_ARG, "degenerate weights: the bracket of the bisection is not finite");

    hipLaunchKernelGGL(k_vtx_meta, dim3(gn), dim3(256), 0, s, order, P.koff, P.slot, parent, om0, p0, P.phi, n,
                       P.meta);
    LAUNCH_CHECK();
    DPArgs A{};
    A.level_start = P.level_start;
    A.meta = P.meta;
    A.Nvals = P.Nvals;
    A.cpw = P.cpw;
    A.cnt = P.cnt;
    A.cut = P.cut;
    A.joined = P.joined;
    A.num = P.num;
    A.den = P.den;
    A.st = P.st;

    // final decision at N = the device state's beta, recording Cut and eta
    // (Algorithm 4), for cluster count kk; returns the device state after it
    auto finalize = [&](int32_t kk, int32_t *lab, double *cn, double *cd, int32_t *cs) {
        hipLaunchKernelGGL(k_set_final_N, dim3(1), dim3(64), 0, s, P.st, P.Nvals);
        LAUNCH_CHECK();
        launch_levels<1, true, false>(A, ls, maxdepth, s);
        hipLaunchKernelGGL(k_cut_in_xorder, dim3(gn), dim3(256), 0, s, order, P.cut, n, P.cf);
        LAUNCH_CHECK();
        exclusive_scan_i32(P.cf, P.rank, n, nullptr, P.scan_scratch, s);
        hipLaunchKernelGGL(k_cluster_index, dim3(gn), dim3(256), 0, s, order, P.cut, P.rank, P.joined, parent, n, kk,
                           P.cidx, P.rep0);
        LAUNCH_CHECK();
        int32_t *ri = P.rep0, *ro = P.rep1;
        for (int it = 0; it <= ceil_log2(maxdepth + 1); ++it) {
            hipLaunchKernelGGL(k_rep_jump, dim3(gn), dim3(256), 0, s, ri, n, ro);
            LAUNCH_CHECK();
            std::swap(ri, ro);
        }
        fill_t<int32_t>(cs, 0, kk, s);
        hipLaunchKernelGGL(k_labels, dim3(gn), dim3(256), 0, s, ri, P.cidx, P.num, P.den, n, lab, cn, cd);
        LAUNCH_CHECK();
        histogram_i32(lab, n, kk, cs, s);  // cluster sizes (residual label -1 skipped)
        hipLaunchKernelGGL(k_final_cost, dim3(1), dim3(64), 0, s, cn, cd, kk, P.cnt, root_slot, P.st);
        LAUNCH_CHECK();
        TreeState hf{};
        HIP_CHECK(hipMemcpyAsync(&hf, P.st, sizeof(hf), hipMemcpyDeviceToHost, s));
        HIP_CHECK(hipStreamSynchronize(s));
        ISO_REQUIRE(hf.ncuts >= kk, ISO_ERR_INTERNAL, "decision at beta found %d < k = %d cuts", hf.ncuts, kk);
        return hf;
    };

    if (kmax >= 2) {
        // ---- all k: host-planned bisections, one per k
        struct Br {
            double a, b;
            int32_t iters;
            bool done;
        };
        std::vector<Br> br((size_t)kmax + 1);
        auto stop = [&](const Br &x) {
            const double mid = (x.a + x.b) / 2.0;
            return mid <= x.a || mid >= x.b || x.iters >= h.max_iters;
        };
        for (int32_t kk = 2; kk <= kmax; ++kk) {
            br[kk] = Br{h.alpha0, h.beta0, 0, false};
            br[kk].done = stop(br[kk]);
        }
        std::vector<double> vals;
        std::vector<int32_t> cnts(M);
        std::vector<int32_t> plan_levels((size_t)kmax + 1);
        int32_t passes = 0;
        while (true) {
            int32_t nact = 0;
            for (int32_t kk = 2; kk <= kmax; ++kk) nact += br[kk].done ? 0 : 1;
            if (nact == 0) break;
            ISO_REQUIRE(++passes <= 64 * h.max_iters, ISO_ERR_INTERNAL, "bisection did not terminate");
            int L = 1;
            while (L < SPEC_LEVELS && ((1 << (L + 1)) - 1) * nact <= NCAND) ++L;
            vals.clear();
            auto lane_of = [&](double v) -> int {
                for (size_t q = 0; q < vals.size(); ++q)
                    if (vals[q] == v) return (int)q;
                if ((int)vals.size() == NCAND) return -1;
                vals.push_back(v);
                return (int)vals.size() - 1;
            };
            // plan, while lanes last: for a bracket whose lower (upper) end has
            // never moved, the midpoints along its all-YES (all-NO) path; else
            // whole levels of its bisection tree
            for (int32_t kk = 2; kk <= kmax; ++kk) {
                plan_levels[kk] = 0;
                if (br[kk].done) continue;
                const bool down = br[kk].a == h.alpha0, up = !down && br[kk].b == h.beta0;
                if (down || up) {
                    double lo = br[kk].a, hi = br[kk].b;
                    for (int l = 0; l < M; ++l) {
                        const double mid = (lo + hi) / 2.0;
                        if (!(mid > lo && mid < hi) || lane_of(mid) < 0) break;
                        plan_levels[kk] = l + 1;
                        (down ? hi : lo) = mid;
                    }
                    continue;
                }
                std::vector<double> lo(1, br[kk].a), hi(1, br[kk].b);
                for (int l = 0; l < L; ++l) {
                    std::vector<double> nlo, nhi;
                    bool fits = true;
                    const size_t before = vals.size();
                    for (size_t q = 0; q < lo.size(); ++q) {
                        const double mid = (lo[q] + hi[q]) / 2.0;
                        if (lane_of(mid) < 0) {
                            fits = false;
                            break;
                        }
                        nlo.push_back(lo[q]);
                        nhi.push_back(mid);
                        nlo.push_back(mid);
                        nhi.push_back(hi[q]);
                    }
                    if (!fits) {
                        vals.resize(before);
                        break;
                    }
                    plan_levels[kk] = l + 1;
                    lo.swap(nlo);
                    hi.swap(nhi);
                }
            }
            ISO_REQUIRE(!vals.empty(), ISO_ERR_INTERNAL, "bisection planning produced no midpoint");
            std::vector<double> nv(M, vals[0]);
            std::copy(vals.begin(), vals.end(), nv.begin());
            HIP_CHECK(hipMemcpyAsync(P.Nvals, nv.data(), sizeof(double) * M, hipMemcpyHostToDevice, s));
            launch_levels<M, false, false>(A, ls, maxdepth, s);
            HIP_CHECK(hipMemcpyAsync(cnts.data(), P.cnt + (int64_t)root_slot * M, sizeof(int32_t) * M,
                                     hipMemcpyDeviceToHost, s));
            HIP_CHECK(hipStreamSynchronize(s));
            // each k walks its own answers, exactly as the single-k bisection,
            // as long as its next midpoint was evaluated in this pass (by its
            // own plan or, with an equal value, by another k's)
            for (int32_t kk = 2; kk <= kmax; ++kk) {
                Br &x = br[kk];
                int walked = 0;
                while (!x.done) {
                    const double mid = (x.a + x.b) / 2.0;
                    int q = -1;
                    for (size_t t = 0; t < vals.size(); ++t)
                        if (vals[t] == mid) {
                            q = (int)t;
                            break;
                        }
                    if (q < 0) break;
                    if (cnts[q] >= kk)
                        x.b = mid;
                    else
                        x.a = mid;
                    x.iters += 1;
                    x.done = stop(x);
                    ++walked;
                }
                ISO_REQUIRE(walked > 0 || plan_levels[kk] == 0, ISO_ERR_INTERNAL, "bisection midpoint was not planned");
            }
        }
        for (int32_t kk = 2; kk <= kmax; ++kk) {
            HIP_CHECK(hipMemcpyAsync(&P.st->beta, &br[kk].b, sizeof(double), hipMemcpyHostToDevice, s));
            int32_t *lab = labels_all ? labels_all + (int64_t)(kk - 2) * n : P.lab_tmp;
            const TreeState hf = finalize(kk, lab, P.cl_num_tmp, P.cl_den_tmp, P.cl_size_tmp);
            i_k_all[kk - 2] = hf.i_k;
        }
        if (passes_out) *passes_out = passes;
        whole.stop(s);
        if (timed) {
            timing().sub_calls += 1;
            timing().sub_ms += whole.elapsed_ms();
            timing().sub_passes += passes;
        }
        return;
    }

    // ---- single k: speculative bisection passes on the device.  After every
    // pass the vertices whose subtree decides alike over the new bracket are
    // frozen (their contribution no longer depends on the threshold), and once
    // enough have frozen the position list the passes visit drops them.
    DPArgs B = A;
    B.nextl = P.nextl;
    B.smask = P.smask;
    fill_t<uint8_t>(P.frozen, 0, n, s);
    std::vector<int32_t> als = ls;  // level starts of B's position list
    int32_t nact = (int32_t)n;
    int32_t *act_next = P.act0, *als_next = P.als0;
    int32_t frozen_listed = 0;  // frozen vertices when the list was last rebuilt
    int passes = 0;
    while (true) {
        hipLaunchKernelGGL(k_make_cands, dim3(1), dim3(M), 0, s, P.st, P.Nvals, P.nextl);
        LAUNCH_CHECK();
        if (nact > 0) launch_levels<M, false, true>(B, als, maxdepth, s);
        hipLaunchKernelGGL(k_resolve, dim3(1), dim3(64), 0, s, P.st, P.Nvals, P.cnt, root_slot);
        LAUNCH_CHECK();
        if (nact > 0) {
            hipLaunchKernelGGL(k_freeze, dim3(grid_for(nact, 256)), dim3(256), 0, s, B, nact, P.frozen);
            LAUNCH_CHECK();
        }
        HIP_CHECK(hipMemcpyAsync(&h, P.st, sizeof(h), hipMemcpyDeviceToHost, s));
        HIP_CHECK(hipStreamSynchronize(s));
        ISO_REQUIRE(!(h.bad & 8), ISO_ERR_INTERNAL, "bisection candidates out of step");
        ISO_REQUIRE(!(h.bad & 16), ISO_ERR_INTERNAL, "decision at beta turned NO during bisection");
        if (h.done) break;
        ISO_REQUIRE(++passes <= h.max_iters + 8, ISO_ERR_INTERNAL, "bisection did not terminate");
        if (h.nfrozen - frozen_listed > nact / 8) {
            hipLaunchKernelGGL(k_keep_flags, dim3(grid_for((int64_t)nact + 1, 256)), dim3(256), 0, s, B.act, nact,
                               P.frozen, P.keep);
            LAUNCH_CHECK();
            exclusive_scan_i32(P.keep, P.kpos, (int64_t)nact + 1, nullptr, P.scan_scratch, s);
            hipLaunchKernelGGL(k_compact, dim3(grid_for(nact, 256)), dim3(256), 0, s, B.act, nact, P.keep, P.kpos,
                               act_next);
            LAUNCH_CHECK();
            hipLaunchKernelGGL(k_active_starts, dim3(grid_for(maxdepth + 2, 256)), dim3(256), 0, s, B.level_start,
                               maxdepth + 2, P.kpos, als_next);
            LAUNCH_CHECK();
            HIP_CHECK(hipMemcpyAsync(als.data(), als_next, sizeof(int32_t) * (maxdepth + 2), hipMemcpyDeviceToHost,
                                     s));
            HIP_CHECK(hipStreamSynchronize(s));
            B.act = act_next;
            B.level_start = als_next;
            act_next = act_next == P.act0 ? P.act1 : P.act0;
            als_next = als_next == P.als0 ? P.als1 : P.als0;
            nact = als[maxdepth + 1];
            frozen_listed = h.nfrozen;
        }
    }
    {
        double *cn = cl_num ? cl_num : P.cl_num_tmp;
        double *cd = cl_den ? cl_den : P.cl_den_tmp;
        int32_t *cs = cl_size ? cl_size : P.cl_size_tmp;
        h = finalize(k, labels, cn, cd, cs);
    }
    whole.stop(s);
    if (timed) {
        timing().sub_calls += 1;
        timing().sub_ms += whole.elapsed_ms();
        timing().sub_passes += h.passes;
    }
    *i_k = h.i_k;
    if (info) {
        info->sigma = h.sigma;
        info->alpha0_raw = h.alpha0_raw;
        info->beta0_raw = h.beta0_raw;
        info->alpha0 = h.alpha0;
        info->beta0 = h.beta0;
        info->alpha = h.alpha;
        info->beta = h.beta;
        info->i_k = h.i_k;
        const double tt = std::log2(2.0 * h.om_sum * h.om_sum * (h.beta0_raw - h.alpha0_raw)) -
                          std::log2(h.phi_min + h.p_min);
        info->t_paper = std::isfinite(tt) ? (int32_t)std::ceil(tt) : -1;
        info->iters = h.iters;
        info->passes = h.passes;
        info->max_depth = maxdepth;
        info->jstar = h.jstar;
        info->reserved0 = 0;
    }
}

}  // namespace

// ------------------------------------------------------------------ allocation-free workspace

// Workspace of iso_subpartition_noalloc: one fixed array per device, reserved
// for the life of the process.  In host code `scratch` names only the host-side
// shadow of the symbol; kernels receive the device address that
// hipGetSymbolAddress reports for the current device.
static __device__ __align__(256) char scratch[ISO_SUB_NOALLOC_BYTES];

namespace {

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
char *g_scratch_ptr[MAX_DEVICES] = {};

// Device address of `scratch` on the current device, looked up on the first
// call made with that device current.
char *noalloc_scratch() {
    int dev = -1;
    HIP_CHECK(hipGetDevice(&dev));
    ISO_REQUIRE(dev >= 0 && dev < MAX_DEVICES, ISO_ERR_NO_DEVICE, "device ordinal %d outside [0, %d)", dev,
                MAX_DEVICES);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[dev] == nullptr) {
        void *ptr = nullptr;
        HIP_CHECK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        ISO_REQUIRE(ptr != nullptr, ISO_ERR_HIP, "hipGetSymbolAddress returned no address for the scratch array");
        g_scratch_ptr[dev] = static_cast<char *>(ptr);
    }
    return g_scratch_ptr[dev];
}

}  // namespace

}  // namespace iso

using namespace iso;

extern "C" iso_status iso_sub_workspace_size(int64_t n, int32_t k, size_t *bytes) {
    return guarded([&] {
        ISO_REQUIRE(bytes != nullptr, ISO_ERR_INVALID_ARG, "bytes is NULL");
        ISO_REQUIRE(n >= 2 && n < (int64_t(1) << 31) - 2, ISO_ERR_INVALID_ARG, "n = %lld outside [2, 2^31)", (long long)n);
        ISO_REQUIRE(k >= 2 && k <= n, ISO_ERR_INVALID_ARG, "k = %d outside [2, n]", k);
        *bytes = sub_plan_bytes(n, k);
    });
}

extern "C" iso_status iso_subpartition_all_k(const int32_t *parent, const double *length, int64_t n, int32_t root,
                                             int32_t kmax, double sigma, const iso_sub_opts *opts, double *i_k,
                                             int32_t *labels, int32_t *passes, void *ws, size_t ws_bytes,
                                             void *stream) {
    return guarded([&] {
        ISO_REQUIRE(parent && length && i_k, ISO_ERR_INVALID_ARG, "parent, length and i_k must be non-NULL");
        ISO_REQUIRE(n >= 2 && n < (int64_t(1) << 31) - 2, ISO_ERR_INVALID_ARG, "n = %lld outside [2, 2^31)", (long long)n);
        ISO_REQUIRE(kmax >= 2 && kmax <= n, ISO_ERR_INVALID_ARG, "kmax = %d outside [2, n]", kmax);
        ISO_REQUIRE(root >= 0 && root < n, ISO_ERR_INVALID_ARG, "root = %d outside [0, n)", root);
        ISO_REQUIRE(sigma >= 0.0 && std::isfinite(sigma), ISO_ERR_INVALID_ARG, "sigma = %g must be finite and >= 0",
                    sigma);
        iso_sub_opts o{ISO_OMEGA_TREE, ISO_PHI_EXP_DIST, ISO_BRACKET_POW2, 2000, nullptr, nullptr};
        if (opts) o = *opts;
        ISO_REQUIRE(o.omega == ISO_OMEGA_TREE || o.omega == ISO_OMEGA_FULL, ISO_ERR_INVALID_ARG,
                    "unsupported omega reading %d", o.omega);
        ISO_REQUIRE(o.omega != ISO_OMEGA_FULL || o.omega0 != nullptr, ISO_ERR_INVALID_ARG,
                    "ISO_OMEGA_FULL needs the vertex weights in opts->omega0");
        ISO_REQUIRE(o.phi == ISO_PHI_EXP_DIST || o.phi == ISO_PHI_GAUSS_SQ, ISO_ERR_INVALID_ARG, "unknown phi %d", o.phi);
        ISO_REQUIRE(o.bracket == ISO_BRACKET_POW2 || o.bracket == ISO_BRACKET_PAPER, ISO_ERR_INVALID_ARG,
                    "unknown bracket %d", o.bracket);
        require_device();
        hipStream_t s = static_cast<hipStream_t>(stream);
        SubPlan P{};
        P.n = n;
        P.k = kmax;
        const size_t need = sub_plan_bytes(n, kmax);
        ScopedWorkspace owned;
        if (ws == nullptr) {
            owned.stream = s;
            HIP_CHECK(hipMallocAsync(&owned.ptr, need, s));
            ws = owned.ptr;
            ws_bytes = need;
        }
        ISO_REQUIRE(ws_bytes >= need, ISO_ERR_WORKSPACE, "workspace %zu bytes < required %zu", ws_bytes, need);
        Arena a{static_cast<char *>(ws), 0, ws_bytes};
        P.carve(a);
        double ik_dummy = 0.0;
        run_sub(P, parent, length, root, sigma, o, P.lab_tmp, &ik_dummy, nullptr, nullptr, nullptr, nullptr, s, kmax,
                i_k, labels, passes);
    });
}

extern "C" iso_status iso_subpartition(const int32_t *parent, const double *length, int64_t n, int32_t root, int32_t k,
                                       double sigma, const iso_sub_opts *opts, int32_t *labels, double *i_k,
                                       double *cluster_num, double *cluster_den, int32_t *cluster_size,
                                       iso_sub_info *info, void *ws, size_t ws_bytes, void *stream) {
    return guarded([&] {
        ISO_REQUIRE(parent && length && labels && i_k, ISO_ERR_INVALID_ARG,
                    "parent, length, labels and i_k must be non-NULL");
        ISO_REQUIRE(n >= 2 && n < (int64_t(1) << 31) - 2, ISO_ERR_INVALID_ARG, "n = %lld outside [2, 2^31)", (long long)n);
        ISO_REQUIRE(k >= 2 && k <= n, ISO_ERR_INVALID_ARG, "k = %d outside [2, n]", k);
        ISO_REQUIRE(root >= 0 && root < n, ISO_ERR_INVALID_ARG, "root = %d outside [0, n)", root);
        ISO_REQUIRE(sigma >= 0.0 && std::isfinite(sigma), ISO_ERR_INVALID_ARG, "sigma = %g must be finite and >= 0",
                    sigma);
        iso_sub_opts o{ISO_OMEGA_TREE, ISO_PHI_EXP_DIST, ISO_BRACKET_POW2, 2000, nullptr, nullptr};
        if (opts) o = *opts;
        ISO_REQUIRE(o.omega == ISO_OMEGA_TREE || o.omega == ISO_OMEGA_FULL, ISO_ERR_INVALID_ARG,
                    "unsupported omega reading %d", o.omega);
        ISO_REQUIRE(o.omega != ISO_OMEGA_FULL || o.omega0 != nullptr, ISO_ERR_INVALID_ARG,
                    "ISO_OMEGA_FULL needs the vertex weights in opts->omega0");
        ISO_REQUIRE(o.phi == ISO_PHI_EXP_DIST || o.phi == ISO_PHI_GAUSS_SQ, ISO_ERR_INVALID_ARG, "unknown phi %d", o.phi);
        ISO_REQUIRE(o.bracket == ISO_BRACKET_POW2 || o.bracket == ISO_BRACKET_PAPER, ISO_ERR_INVALID_ARG,
                    "unknown bracket %d", o.bracket);
        require_device();
        hipStream_t s = static_cast<hipStream_t>(stream);
        SubPlan P{};
        P.n = n;
        P.k = k;
        const size_t need = sub_plan_bytes(n, k);
        ScopedWorkspace owned;
        if (ws == nullptr) {
            owned.stream = s;
            HIP_CHECK(hipMallocAsync(&owned.ptr, need, s));
            ws = owned.ptr;
            ws_bytes = need;
        }
        ISO_REQUIRE(ws_bytes >= need, ISO_ERR_WORKSPACE, "workspace %zu bytes < required %zu", ws_bytes, need);
        Arena a{static_cast<char *>(ws), 0, ws_bytes};
        P.carve(a);
        run_sub(P, parent, length, root, sigma, o, labels, i_k, cluster_num, cluster_den, cluster_size, info, s);
    });
}

extern "C" iso_status iso_subpartition_noalloc(const int32_t *parent, const double *length, int64_t n, int32_t root,
                                               int32_t k, double sigma, const iso_sub_opts *opts, int32_t *labels,
                                               double *i_k, double *cluster_num, double *cluster_den,
                                               int32_t *cluster_size, iso_sub_info *info, void *stream) {
    return guarded([&] {
        ISO_REQUIRE(parent && length && labels && i_k, ISO_ERR_INVALID_ARG,
                    "parent, length, labels and i_k must be non-NULL");
        ISO_REQUIRE(n >= 2 && n <= ISO_SUB_NOALLOC_MAX_N, ISO_ERR_INVALID_ARG,
                    "n = %lld outside [2, %d] (the allocation-free entry point's maximum)", (long long)n,
                    ISO_SUB_NOALLOC_MAX_N);
        ISO_REQUIRE(k >= 2 && k <= n, ISO_ERR_INVALID_ARG, "k = %d outside [2, n]", k);
        ISO_REQUIRE(root >= 0 && root < n, ISO_ERR_INVALID_ARG, "root = %d outside [0, n)", root);
        ISO_REQUIRE(sigma >= 0.0 && std::isfinite(sigma), ISO_ERR_INVALID_ARG, "sigma = %g must be finite and >= 0",
                    sigma);
        iso_sub_opts o{ISO_OMEGA_TREE, ISO_PHI_EXP_DIST, ISO_BRACKET_POW2, 2000, nullptr, nullptr};
        if (opts) o = *opts;
        ISO_REQUIRE(o.omega == ISO_OMEGA_TREE || o.omega == ISO_OMEGA_FULL, ISO_ERR_INVALID_ARG,
                    "unsupported omega reading %d", o.omega);
        ISO_REQUIRE(o.omega != ISO_OMEGA_FULL || o.omega0 != nullptr, ISO_ERR_INVALID_ARG,
                    "ISO_OMEGA_FULL needs the vertex weights in opts->omega0");
        ISO_REQUIRE(o.phi == ISO_PHI_EXP_DIST || o.phi == ISO_PHI_GAUSS_SQ, ISO_ERR_INVALID_ARG, "unknown phi %d", o.phi);
        ISO_REQUIRE(o.bracket == ISO_BRACKET_POW2 || o.bracket == ISO_BRACKET_PAPER, ISO_ERR_INVALID_ARG,
                    "unknown bracket %d", o.bracket);
        const size_t need = sub_plan_bytes(n, k);
        ISO_REQUIRE(need <= ISO_SUB_NOALLOC_BYTES, ISO_ERR_INTERNAL, "workspace %zu bytes exceeds the fixed %zu", need,
                    (size_t)ISO_SUB_NOALLOC_BYTES);
        require_device();
        char *ws = noalloc_scratch();
        hipStream_t s = static_cast<hipStream_t>(stream);
        SubPlan P{};
        P.n = n;
        P.k = k;
        Arena a{ws, 0, (size_t)ISO_SUB_NOALLOC_BYTES};
        P.carve(a);
        run_sub(P, parent, length, root, sigma, o, labels, i_k, cluster_num, cluster_den, cluster_size, info, s);
    });
}
