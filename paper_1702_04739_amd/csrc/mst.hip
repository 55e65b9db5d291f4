// mst.hip -- Euclidean minimum spanning tree on gfx950 by Boruvka rounds over
// on-the-fly distance tiles (the paper builds the MST with Prim over a stored
// n x n affinity matrix, Secs. 3.4-3.5; here the matrix is never stored).
//
// One Boruvka round:
//   screen    : every unordered pair of points is formed once, tile pair by
//               tile pair (screen_pairs.hip): Dhat^2 = ||x_i||^2 + ||x_j||^2
//               - 2 x_i.x_j on the matrix cores; over pairs in different
//               components every point keeps its running minimum b_i and the
//               partners whose lower bound Dhat^2 - E_ij can still reach
//               b_i + E_i, where E bounds |Dhat^2 - D^2| (candidates); points
//               whose list overflows are screened again from their final
//               minimum (gathered pass, screen_mfma.hip);
//   comp_ub   : U_c = min over rows of component c of b_i + E_i, an upper
//               bound on c's lightest outgoing edge;
//   recheck   : exact D^2 of the candidates that can still reach U_c, giving
//               each row its lightest outgoing edge under the total order
//               (D^2, smaller id, larger id); rows whose list overflowed again
//               are re-evaluated against every point (rescan);
//   comp_min  : lightest outgoing edge per component (two 64-bit atomic mins);
//   hook/jump : each component hooks onto the component across its edge;
//               mutual pairs keep the smaller id as root; pointer jumping;
//   relabel   : compact component ids by an exclusive scan.
// After the last round: FP64 edge lengths, and an Euler tour of the tree whose
// first-taken arcs give the parent list (Sec. 3.3) rooted at vertex 0.
#include <algorithm>
#include <cfloat>
#include <cmath>
#include <cstring>
#include <exception>
#include <mutex>
#include <tuple>
#include <utility>
#include <vector>

#include "screen.hpp"

namespace iso {

namespace {

constexpr int GT = 256;        // row padding granule (the tile-pair screen's tile)
constexpr uint32_t U32_MAX = 0xFFFFFFFFu;
constexpr uint64_t U64_MAX = ~0ull;

enum Counter : int {
    C_EDGES = 0,        // edges appended so far
    C_NCOMP = 1,        // components after relabel
    C_NONFINITE = 2,    // nonfinite coordinate seen
    C_OVF = 3,          // overflow rows this round
    C_NOEDGE = 4,       // a component without an outgoing edge (internal error)
    // 5 unused
    C_GATHER = 6,       // rows queued for the gathered pass this round
    C_FORCE = 7,        // rows the neighbour lists leave undecided this round
    C_CAND = 8,         // candidates re-evaluated (int64 at [8..9])
    C_RESCAN = 10,      // rows rescanned (int64 at [10..11])
    C_SUMSQ = 12,       // sum over components of size^2 (int64 at [12..13], timing only)
    C_I8BAD = 14,       // the points are not 8-bit integers on a common grid (INT8 screen)
    C_FRWORK = 16,      // final round: candidates its recheck would evaluate (int64 at [16..17])
    C_PAIRS = 18,       // point pairs of the screened tile pairs (int64 at [18..19], pruned rounds)
    C_TPFULL = 20,      // tile pairs a full screen would run (pruned rounds)
    C_COUNT = 21
};

// ------------------------------------------------------------------ small kernels

template <class T>
__global__ void k_fill(T *p, T v, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// Workgroups (four waves, one row per wave per step) for a grid-stride walk
// over n rows: enough to fill the chip, few enough to dispatch quickly.
unsigned row_grid(int64_t n) { return std::min<unsigned>(grid_for(n, 4), 16u * (unsigned)device_cus()); }

template <class T>
void fill(T *p, T v, int64_t n, hipStream_t s) {
    if (n <= 0) return;
    unsigned g = grid_for(n, 256);
    if (g > 4096) g = 4096;
    hipLaunchKernelGGL(k_fill<T>, dim3(g), dim3(256), 0, s, p, v, n);
    LAUNCH_CHECK();
}

// ------------------------------------------------------------------ screen representation

constexpr int COL_RB = 256;    // rows per partial column sum
constexpr int GRID_NONE = 1 << 20;

// Exponent q of the coarsest binary grid 2^q holding the finite float x
// (x = odd integer * 2^q); GRID_NONE for 0.
__device__ __forceinline__ int grid_exponent(float x) {
    const uint32_t u = __float_as_uint(x) & 0x7FFFFFFFu;
    if (u == 0u) return GRID_NONE;
    const int ef = (int)(u >> 23);
    const uint32_t mant = u & 0x7FFFFFu;
    if (ef == 0) return -149 + __builtin_ctz(mant);  // subnormal
    return ef - 150 + __builtin_ctz(mant | 0x800000u);
}

// Partial per-coordinate sums (FP64) and maxima of |x| over row blocks;
// non-finite check.
__global__ __launch_bounds__(256) void k_colstats_partial(const float *__restrict__ X, int64_t n, int64_t d,
                                                          int64_t ld, double *__restrict__ psum,
                                                          int32_t *__restrict__ pgrid, float *__restrict__ pmin,
                                                          float *__restrict__ pmax, int32_t *__restrict__ counters) {
    const int64_t t = (int64_t)blockIdx.y * 256 + threadIdx.x;
    const int64_t rb = blockIdx.x;
    if (t >= d) return;
    const int64_t lo = rb * COL_RB, hi = lo + COL_RB < n ? lo + COL_RB : n;
    double s = 0.0;
    int q = GRID_NONE;
    bool bad = false;
    float mn = __builtin_huge_valf(), mx = -__builtin_huge_valf();
#pragma unroll 8
    for (int64_t i = lo; i < hi; ++i) {
        const float x = X[i * ld + t];
        bad |= !isfinite(x);
        s = s + (double)x;
        q = min(q, grid_exponent(x));
        mn = fminf(mn, x);
        mx = fmaxf(mx, x);
    }
    psum[rb * d + t] = s;
    pgrid[rb * d + t] = q;
    pmin[rb * d + t] = mn;
    pmax[rb * d + t] = mx;
    if (bad) atomicExch(&counters[C_NONFINITE], 1);
}

// Centre mu_t: the coordinate mean rounded to the coarsest binary grid 2^q_t
// that holds every value of the column, so that centring keeps values that
// sit on a grid (e.g. q/256) on it; 0 for empty columns and beyond d.
// One wave per coordinate: lane l sums the partials l, l + 64, ... (a fixed
// order), then the wave combines them.
__global__ __launch_bounds__(256) void k_colstats_final(const double *__restrict__ psum,
                                                        const int32_t *__restrict__ pgrid, int64_t nrb, int64_t n,
                                                        int64_t d, int64_t d_pad, float *__restrict__ mu) {
    const int64_t t = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (t >= d_pad) return;
    if (t >= d) {
        if (lane == 0) mu[t] = 0.0f;
        return;
    }
    double s = 0.0;
    int q = GRID_NONE;
    for (int64_t rb = lane; rb < nrb; rb += 64) {
        s = s + psum[rb * d + t];
        q = min(q, pgrid[rb * d + t]);
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        s += __shfl_xor(s, o, 64);
        q = min(q, __shfl_xor(q, o, 64));
    }
    if (lane != 0) return;
    if (q == GRID_NONE) {
        mu[t] = 0.0f;
        return;
    }
    const double grid = ldexp(1.0, q);
    mu[t] = (float)(rint((s / (double)n) / grid) * grid);
}

// INT8 representation, first step: every column's grid, minimum and maximum;
// the common grid 2^qg (the finest column grid) into *qg.
__global__ void k_colrange_i8(const int32_t *__restrict__ pgrid, const float *__restrict__ pmin,
                              const float *__restrict__ pmax, int64_t nrb, int64_t d, float *__restrict__ cmin,
                              float *__restrict__ cmax, int32_t *__restrict__ qg) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= d) return;
    int q = GRID_NONE;
    float mn = __builtin_huge_valf(), mx = -__builtin_huge_valf();
    for (int64_t rb = 0; rb < nrb; ++rb) {
        q = min(q, pgrid[rb * d + t]);
        mn = fminf(mn, pmin[rb * d + t]);
        mx = fmaxf(mx, pmax[rb * d + t]);
    }
    cmin[t] = mn;
    cmax[t] = mx;
    if (q != GRID_NONE) atomicMin(qg, q);
}

// INT8 representation, second step: centre mu_t = min_t + 128 * 2^qg, so that
// every (x - mu_t) / 2^qg is an integer in [-128, 127] exactly when the
// column's range is at most 255 grid steps; a column that does not fit (or a
// centre that does not round exactly) flags counters[C_I8BAD].
__global__ void k_center_i8(const float *__restrict__ cmin, const float *__restrict__ cmax, int64_t d, int64_t d_pad,
                            const int32_t *__restrict__ qg, float *__restrict__ mu, int32_t *__restrict__ counters) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= d_pad) return;
    if (t >= d) {
        mu[t] = 0.0f;
        return;
    }
    const int q = *qg;
    if (q == GRID_NONE) {  // every coordinate is zero
        mu[t] = 0.0f;
        return;
    }
    const double step = ldexp(1.0, q);
    const double m = (double)cmin[t] + 128.0 * step;
    const bool fits = (double)cmax[t] - (double)cmin[t] <= 255.0 * step && (double)(float)m == m && q > -120 &&
                      q < 100;
    mu[t] = (float)m;
    if (!fits) atomicExch(&counters[C_I8BAD], 1);
}

__device__ __forceinline__ uint16_t bf16_rne(float x) {
    uint32_t u = __float_as_uint(x);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float bf16_to_f32(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

// E4M3 (OCP) rounding of x with saturation at +-448 (the hardware conversion
// rounds to nearest even; the clamp keeps it away from the NaN code).
__device__ __forceinline__ uint8_t fp8_rne(float x) {
    const float c = fminf(fmaxf(x, -448.0f), 448.0f);
    return (uint8_t)(__builtin_amdgcn_cvt_pk_fp8_f32(c, 0.0f, 0, false) & 0xFF);
}

__device__ __forceinline__ float fp8_to_f32(uint8_t b) { return __builtin_amdgcn_cvt_f32_fp8((int)b, 0); }

// One wave per (padded) row: x' = rep(x - mu) written row-major, s = fl(||x'||^2)
// (fixed order), and upper bounds r >= ||x'||, e >= ||x' - (x - mu)|| computed
// from the stored values.
template <int REP>
__global__ __launch_bounds__(256) void k_repr_rows(const float *__restrict__ X, int64_t n, int64_t d, int64_t ld,
                                                   int64_t n_pad, int64_t d_pad, const float *__restrict__ mu,
                                                   void *__restrict__ Xr, float *__restrict__ sq,
                                                   float *__restrict__ rn, float *__restrict__ re,
                                                   uint32_t *__restrict__ rmax_bits, uint32_t *__restrict__ emax_bits,
                                                   int32_t *__restrict__ grid_min, int32_t *__restrict__ sqi,
                                                   float inv_step) {
    const int lane = threadIdx.x & 63;
    // rows are walked with the stride of all waves; the maxima of r and e and
    // the grid exponent are merged into the globals once per wave
    uint32_t wr = 0u, we = 0u;
    int wq = GRID_NONE;
    const int64_t nwaves = (int64_t)gridDim.x * 4;
    for (int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); i < n_pad; i += nwaves) {
    float s = 0.0f;
    double m2 = 0.0, e2 = 0.0;
    int q = GRID_NONE;
    int32_t si = 0;  // INT8: exact squared norm in grid units
    for (int64_t t = lane; t < d_pad; t += 64) {
        float xv = 0.0f, y = 0.0f;
        if (i < n && t < d) {
            xv = X[i * ld + t];
            y = xv - mu[t];
        }
        float yr;
        if (REP == ISO_PREC_BF16) {
            const uint16_t b = bf16_rne(y);
            static_cast<uint16_t *>(Xr)[i * d_pad + t] = b;
            yr = bf16_to_f32(b);
        } else if (REP == ISO_PREC_FP8) {
            const uint8_t b = fp8_rne(y);
            static_cast<uint8_t *>(Xr)[i * d_pad + t] = b;
            yr = fp8_to_f32(b);
        } else if (REP == ISO_PREC_INT8) {
            // (x - mu) / 2^qg is an integer in [-128, 127] (checked by the
            // centre); y = x - mu is exact
            const int v = (int)rintf(y * inv_step);
            static_cast<int8_t *>(Xr)[i * d_pad + t] = (int8_t)v;
            si = si + v * v;
            yr = y;
        } else {
            static_cast<float *>(Xr)[i * d_pad + t] = y;
            yr = y;
        }
        s = fmaf(yr, yr, s);
        q = min(q, grid_exponent(yr));
        const double yd = (double)yr;
        m2 = m2 + yd * yd;
        if (i < n && t < d) {
            const double df = yd - ((double)xv - (double)mu[t]);
            e2 = e2 + df * df;
        }
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        s += __shfl_xor(s, off, 64);
        si += __shfl_xor(si, off, 64);
        m2 += __shfl_xor(m2, off, 64);
        e2 += __shfl_xor(e2, off, 64);
        q = min(q, __shfl_xor(q, off, 64));
    }
    const float r = __double2float_ru(sqrt(m2) * (1.0 + 0x1p-40));
    const float e = __double2float_ru(sqrt(e2) * (1.0 + 0x1p-40));
    if (lane == 0) {
        sq[i] = i < n ? s : __builtin_huge_valf();  // padding: every Dhat^2 with it is +inf
        rn[i] = r;
        re[i] = e;
        if (REP == ISO_PREC_INT8) sqi[i] = i < n ? si : (1 << 30);  // padding: a distance at or beyond 2^30 means none
    }
    wq = min(wq, q);
    wr = max(wr, __float_as_uint(r));
    we = max(we, __float_as_uint(e));
    }
    if (lane == 0) {
        if (wq != GRID_NONE) atomicMin(grid_min, wq);
        if (wr) atomicMax(rmax_bits, wr);
        if (we) atomicMax(emax_bits, we);
    }
}

__global__ void k_row_bound(const float *__restrict__ rn, const float *__restrict__ re, int64_t n, ScreenBound B,
                            const uint32_t *__restrict__ rmax_bits, const uint32_t *__restrict__ emax_bits,
                            float *__restrict__ Emax) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    Emax[i] = pair_bound(B, rn[i], __uint_as_float(*rmax_bits), re[i], __uint_as_float(*emax_bits)) + 1e-30f;
}

// Sums of r_i and e_i over the points (one atomic per workgroup each).
__global__ __launch_bounds__(256) void k_norm_sums(const float *__restrict__ rn, const float *__restrict__ re,
                                                  int64_t n, double *__restrict__ out) {
    __shared__ double sr[256], se[256];
    double a = 0.0, b = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        a += rn[i];
        b += re[i];
    }
    sr[threadIdx.x] = a;
    se[threadIdx.x] = b;
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
        if ((int)threadIdx.x < w) {
            sr[threadIdx.x] += sr[threadIdx.x + w];
            se[threadIdx.x] += se[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        atomicAdd(&out[0], sr[0]);
        atomicAdd(&out[1], se[0]);
    }
}

__global__ void k_iota_comp(int32_t *comp, int64_t n, int64_t n_pad) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_pad; i += (int64_t)gridDim.x * blockDim.x)
        comp[i] = i < n ? (int32_t)i : -1;
}

// ------------------------------------------------------------------ exact distances

// FP32 exact-recheck distance: lane l sums (x_t - y_t)^2 for t = l, l+64, ...
// with fused multiply-adds, then an xor butterfly over the 64 lanes.  Every
// lane returns the same value, which depends only on the unordered pair.
__device__ inline float d2_f32_wave(const float *__restrict__ x, const float *__restrict__ y, int64_t d) {
    const int lane = threadIdx.x & 63;
    float acc = 0.0f;
    int64_t t = lane;
    // eight strides loaded ahead, then folded in the same order as one at a time
    for (; t + 7 * 64 < d; t += 8 * 64) {
        float a[8], b[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            a[u] = x[t + 64 * u];
            b[u] = y[t + 64 * u];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const float df = a[u] - b[u];
            acc = fmaf(df, df, acc);
        }
    }
    for (; t < d; t += 64) {
        float df = x[t] - y[t];
        acc = fmaf(df, df, acc);
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) acc += __shfl_xor(acc, off, 64);
    return acc;
}

// FP64 exact-recheck distance: left to right over t, each product and sum
// rounded separately (the library is compiled without FP contraction).
__device__ inline double d2_f64_lane(const float *__restrict__ x, const float *__restrict__ y, int64_t d) {
    double s = 0.0;
    for (int64_t t = 0; t < d; ++t) {
        double df = (double)x[t] - (double)y[t];
        double p = df * df;
        s = s + p;
    }
    return s;
}

__device__ inline bool key_less(double d2a, int ja, double d2b, int jb) {
    return d2a < d2b || (d2a == d2b && ja < jb);
}

// U_c = min over rows i of c of (b_i + Emax_i) (1 + rho), rounded up: an upper
// bound on the recheck value of c's lightest outgoing edge.  With pair bounds
// (ub != nullptr) ub_i, the least Dhat^2 + E_ij screened, replaces b_i + Emax_i.
// Thread t takes the point at position t of the tile order `order` (npos
// positions, ids >= n are padding): the order keeps the points of a component
// together (components only merge), so a wave's points mostly share one
// component and the grouped atomic issues one or two atomics per wave.
__global__ void k_comp_ub(const int32_t *__restrict__ order, int64_t npos, const float *__restrict__ best,
                          const float *__restrict__ Emax, const float *__restrict__ ub,
                          const int32_t *__restrict__ comp, int64_t n, float up, uint32_t *__restrict__ comp_ub) {
    const int64_t pos = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t i = pos < npos ? order[pos] : n;
    const float b = i < n ? best[i] : SCR_INF;
    const bool active = b < SCR_INF;
    const float u = active ? (ub ? ub[i] : b + Emax[i]) * up : 0.0f;
    grouped_atomic_min(comp_ub, active ? comp[i] : 0, __float_as_uint(u), active);
}

// Exact lightest candidate of row i among the cnt entries (js, ls) whose lower
// bound is <= thr, by (D^2, j).  One wave; every lane returns the result.
template <bool F64>
__device__ inline void eval_candidates(const float *__restrict__ X, int64_t ld, int64_t d, int64_t i,
                                       const int32_t *__restrict__ js, const float *__restrict__ ls, int cnt, float thr,
                                       double &out_d2, int &out_j, int &evaluated) {
    const int lane = threadIdx.x & 63;
    const float *xi = X + i * ld;
    out_d2 = __builtin_huge_val();
    out_j = -1;
    evaluated = 0;
    if (!F64) {
        for (int q = 0; q < cnt; ++q) {
            if (!(ls[q] <= thr)) continue;
            const int j = js[q];
            const double d2 = (double)d2_f32_wave(xi, X + (int64_t)j * ld, d);
            ++evaluated;
            if (key_less(d2, j, out_d2, out_j)) {
                out_d2 = d2;
                out_j = j;
            }
        }
    } else {
        double my = __builtin_huge_val();
        int myj = -1;
        for (int q0 = 0; q0 < cnt; q0 += 64) {
            const int q = q0 + lane;
            if (q < cnt && ls[q] <= thr) {
                const int j = js[q];
                const double d2 = d2_f64_lane(xi, X + (int64_t)j * ld, d);
                ++evaluated;
                if (key_less(d2, j, my, myj)) {
                    my = d2;
                    myj = j;
                }
            }
        }
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) {
            const double od = __shfl_xor(my, off, 64);
            const int oj = __shfl_xor(myj, off, 64);
            evaluated += __shfl_xor(evaluated, off, 64);
            if (oj >= 0 && (myj < 0 || key_less(od, oj, my, myj))) {
                my = od;
                myj = oj;
            }
        }
        out_d2 = my;
        out_j = myj;
    }
}

// Threshold for a row's candidates (on the real-D^2 scale of the lower
// bounds): they must be able to beat both the row's own minimum and the
// component's bound U (a recheck value, so divided by 1 - rho).
// With pair bounds (ub != nullptr) the row's own upper bound ub_i replaces
// b_i + Emax_i; the lower bound b_i - Emax_i stays (it must hold for every j).
__device__ inline bool row_threshold(const float *__restrict__ best, const float *__restrict__ Emax,
                                     const float *__restrict__ ub, const int32_t *__restrict__ comp,
                                     const uint32_t *__restrict__ comp_ub, int64_t i, float kappa, float dn,
                                     float &thr) {
    const float b = best[i];
    const uint32_t ubits = comp_ub[comp[i]];
    if (!(b < SCR_INF) || ubits == 0xFFFFFFFFu) return false;
    const float U = __uint_as_float(ubits) * dn;
    const float E = Emax[i];
    if (lower_of(b, E) > U) return false;  // the row cannot hold its component's lightest edge
    thr = fminf((ub ? ub[i] : b + E) * kappa, U);
    return true;
}

// One wave per row: exact recheck of the sweep's candidates.  Rows whose
// list overflowed, and rows marked SCR_FORCE, are queued for the gathered pass.
template <bool F64>
__global__ __launch_bounds__(256) void k_recheck_rows(const float *__restrict__ X, int64_t n, int64_t d, int64_t ld,
                                                      const float *__restrict__ best, const float *__restrict__ Emax,
                                                      const float *__restrict__ ub, const int32_t *__restrict__ comp,
                                                      const uint32_t *__restrict__ comp_ub,
                                                      const int32_t *__restrict__ ccnt, const int32_t *__restrict__ cj,
                                                      const float *__restrict__ cl, float kappa, float dn,
                                                      double *__restrict__ rb_d2, int32_t *__restrict__ rb_j,
                                                      int32_t *__restrict__ glist, int32_t *__restrict__ counters) {
    const int lane = threadIdx.x & 63;
    int evaluated = 0;
    // rows are walked with the stride of all waves (a few thousand workgroups
    // instead of one per four rows: the dispatch of 50k small workgroups costs
    // more than their work)
    for (int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); i < n; i += (int64_t)gridDim.x * 4) {
        double out_d2 = __builtin_huge_val();
        int out_j = -1, ev = 0;
        float thr;
        const int cnt = ccnt[i];
        if (cnt == SCR_FORCE) {
            if (lane == 0) glist[atomicAdd(&counters[C_GATHER], 1)] = (int32_t)i;
        } else if (row_threshold(best, Emax, ub, comp, comp_ub, i, kappa, dn, thr)) {
            if (cnt > SCR_CAP) {
                if (lane == 0) glist[atomicAdd(&counters[C_GATHER], 1)] = (int32_t)i;
            } else {
                eval_candidates<F64>(X, ld, d, i, cj + i * SCR_CAP, cl + i * SCR_CAP, cnt, thr, out_d2, out_j, ev);
            }
        }
        if (lane == 0) {
            rb_d2[i] = out_d2;
            rb_j[i] = out_j;
        }
        evaluated += ev;
    }
    if (lane == 0 && evaluated) atomicAdd((unsigned long long *)&counters[C_CAND], (unsigned long long)evaluated);
}

// One wave per gathered row: exact recheck of the gathered pass's candidates;
// rows that overflowed again are queued for the exact rescan.
template <bool F64>
__global__ __launch_bounds__(256) void k_recheck_gather(const float *__restrict__ X, int64_t d, int64_t ld,
                                                        const float *__restrict__ best, const float *__restrict__ Emax,
                                                        const float *__restrict__ ub, const int32_t *__restrict__ comp,
                                                        const uint32_t *__restrict__ comp_ub,
                                                        const int32_t *__restrict__ glist, int32_t ng,
                                                        const int32_t *__restrict__ gcnt,
                                                        const int32_t *__restrict__ gcj,
                                                        const float *__restrict__ gcl, float kappa, float dn,
                                                        double *__restrict__ rb_d2, int32_t *__restrict__ rb_j,
                                                        int32_t *__restrict__ rlist, int32_t *__restrict__ counters) {
    const int lane = threadIdx.x & 63;
    const int64_t q = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (q >= ng) return;
    const int64_t i = glist[q];
    double out_d2 = __builtin_huge_val();
    int out_j = -1, evaluated = 0;
    float thr;
    if (row_threshold(best, Emax, ub, comp, comp_ub, i, kappa, dn, thr)) {
        const int cnt = gcnt[q];
        if (cnt > SCR_CAP2) {
            if (lane == 0) rlist[atomicAdd(&counters[C_OVF], 1)] = (int32_t)i;
        } else {
            eval_candidates<F64>(X, ld, d, i, gcj + q * SCR_CAP2, gcl + q * SCR_CAP2, cnt, thr, out_d2, out_j,
                                 evaluated);
        }
    }
    if (lane == 0) {
        rb_d2[i] = out_d2;
        rb_j[i] = out_j;
        if (evaluated) atomicAdd((unsigned long long *)&counters[C_CAND], (unsigned long long)evaluated);
    }
}

// Exact re-evaluation of a row against every point of another component: one
// workgroup per queued row, four waves over the columns.
template <bool F64>
__global__ __launch_bounds__(256) void k_rescan(const float *__restrict__ X, int64_t n, int64_t d, int64_t ld,
                                                const int32_t *__restrict__ comp, const int32_t *__restrict__ rlist,
                                                int32_t *__restrict__ counters, double *__restrict__ rb_d2,
                                                int32_t *__restrict__ rb_j) {
    __shared__ double s_d2[256];
    __shared__ int s_j[256];
    const int nr = counters[C_OVF];
    const int w = threadIdx.x >> 6;
    for (int r = blockIdx.x; r < nr; r += gridDim.x) {
        const int64_t i = rlist[r];
        const int ci = comp[i];
        const float *xi = X + i * ld;
        double bd = __builtin_huge_val();
        int bj = -1;
        if (!F64) {
            for (int64_t j = w; j < n; j += 4) {
                if (comp[j] == ci) continue;
                double d2 = (double)d2_f32_wave(xi, X + j * ld, d);
                if (key_less(d2, (int)j, bd, bj)) {
                    bd = d2;
                    bj = (int)j;
                }
            }
        } else {
            for (int64_t j = threadIdx.x; j < n; j += 256) {
                if (comp[j] == ci) continue;
                double d2 = d2_f64_lane(xi, X + j * ld, d);
                if (key_less(d2, (int)j, bd, bj)) {
                    bd = d2;
                    bj = (int)j;
                }
            }
        }
        s_d2[threadIdx.x] = bd;
        s_j[threadIdx.x] = bj;
        __syncthreads();
        if (threadIdx.x == 0) {
            for (int q = 1; q < 256; ++q)
                if (s_j[q] >= 0 && (bj < 0 || key_less(s_d2[q], s_j[q], bd, bj))) {
                    bd = s_d2[q];
                    bj = s_j[q];
                }
            rb_d2[i] = bd;
            rb_j[i] = bj;
            atomicAdd((unsigned long long *)&counters[C_RESCAN], 1ull);
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------------ neighbour lists
//
// The tile-pair screen of the second round appends to each point i every
// point j of another component with Dhat^2_ij <= tau_i = LIST_LAMBDA b_i, b_i
// the point's first-round minimum (its nearest neighbour's Dhat^2).  Points
// left out have Dhat^2_ij > tau_i, or >= the smallest dropped value once the
// list was full, so t_i = min(tau_i, dropped) bounds every absent j from below:
// D^2_ij >= t_i - E_ij >= t_i - Emax_i.  Components only merge, so a pair that
// is absent because its points shared a component then stays irrelevant.  In a
// later round a row is decided by its list when that lower bound exceeds the
// recheck threshold the row's candidates are filtered with (min of
// kappa (b + Emax) and the component bound U): every column that can still be
// the row's or its component's lightest edge is then in the list, and the
// row's list entries replace its screen.  Undecided rows are screened in the
// gathered pass; when there are many, the round runs the full screen instead.

constexpr float LIST_LAMBDA = 1.1f;
constexpr double FR_EVAL_PER_POINT = 16.0;  // final round: most exact evaluations per point on average

__global__ void k_list_init(const float *__restrict__ best, int64_t n, float *__restrict__ ltau,
                            int32_t *__restrict__ lcnt, uint32_t *__restrict__ ldrop) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float b = best[i];
    ltau[i] = b < SCR_INF ? b * LIST_LAMBDA : -1.0f;  // a point without a first-round minimum keeps no list
    lcnt[i] = 0;
    ldrop[i] = 0x7F800000u;
}

// One wave per row: b_i = min over the list's entries in other components of
// their Dhat^2 (an upper bound of the row's minimum; +inf without such entries).
__global__ __launch_bounds__(256) void k_list_best(int64_t n, const int32_t *__restrict__ comp,
                                                   const int32_t *__restrict__ lcnt, const int32_t *__restrict__ lj,
                                                   const float *__restrict__ lv, float *__restrict__ best) {
    const int lane = threadIdx.x & 63;
    for (int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); i < n; i += (int64_t)gridDim.x * 4) {
        const int ci = comp[i];
        const int cnt = min(lcnt[i], LIST_CAP);
        uint32_t m = 0x7F800000u;
        for (int q = lane; q < cnt; q += 64) {
            const int32_t j = lj[i * LIST_CAP + q];
            if (comp[j] != ci) m = min(m, __float_as_uint(lv[i * LIST_CAP + q]));
        }
        m = wave_min_u32(m);
        if (lane == 0) best[i] = __uint_as_float(m);
    }
}

// One wave per row: decide the row from its list (candidates into cj/cl as
// the screen would leave them, ccnt > SCR_CAP on overflow) or mark it
// SCR_FORCE for the gathered pass.
__global__ __launch_bounds__(256) void k_list_capture(
    int64_t n, const int32_t *__restrict__ comp, const uint32_t *__restrict__ comp_ub, const float *__restrict__ best,
    const float *__restrict__ Emax, const float *__restrict__ rn, const float *__restrict__ re, ScreenBound bound,
    const float *__restrict__ ltau, const int32_t *__restrict__ lcnt, const uint32_t *__restrict__ ldrop,
    const int32_t *__restrict__ lj, const float *__restrict__ lv, float kappa, float dn, int32_t *__restrict__ ccnt,
    int32_t *__restrict__ cj, float *__restrict__ cl, int32_t *__restrict__ counters) {
    const int lane = threadIdx.x & 63;
    for (int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); i < n; i += (int64_t)gridDim.x * 4) {
        const int ci = comp[i];
        const float b = best[i], E = Emax[i];
        const uint32_t ubits = comp_ub[ci];
        const float U = ubits == U32_MAX ? SCR_INF : __uint_as_float(ubits) * dn;
        const float thr = fminf(b < SCR_INF ? (b + E) * kappa : SCR_INF, U);
        const float t = fminf(ltau[i], __uint_as_float(ldrop[i]));
        if (!(thr < SCR_INF) || !(lower_of(t, E) > thr)) {
            if (lane == 0) {
                ccnt[i] = SCR_FORCE;
                atomicAdd(&counters[C_FORCE], 1);
            }
            continue;
        }
        const int cnt = min(lcnt[i], LIST_CAP);
        const float ri = rn[i], ei = re[i];
        int taken = 0;
        for (int q0 = 0; q0 < cnt; q0 += 64) {
            const int q = q0 + lane;
            bool keep = false;
            int32_t j = 0;
            float L = 0.0f;
            if (q < cnt) {
                j = lj[i * LIST_CAP + q];
                if (comp[j] != ci) {
                    L = lower_of(lv[i * LIST_CAP + q], pair_bound(bound, ri, rn[j], ei, re[j]));
                    keep = L <= thr;
                }
            }
            const unsigned long long bal = __ballot(keep);
            const int pos = taken + __popcll(bal & ((1ull << lane) - 1ull));
            if (keep && pos < SCR_CAP) {
                cj[i * SCR_CAP + pos] = j;
                cl[i * SCR_CAP + pos] = L;
            }
            taken += __popcll(bal);
        }
        if (lane == 0) ccnt[i] = taken > SCR_CAP ? SCR_CAP + 1 : taken;
    }
}

// ------------------------------------------------------------------ final round
//
// Once at most FR_KC components remain, one screen gives every point its
// minimum into every other component (tiles hold single components, the
// order padding each component to whole tiles), and the exact recheck of its
// candidates gives, for every pair of components, their lightest edge under
// the total order (D^2, smaller id, larger id).  The tree of the components
// under these edges (Kruskal on at most FR_KC nodes) completes the MST: with
// a total order the MST of the whole graph is the forest found so far plus
// the MST of the graph contracted along it, where parallel edges between two
// components reduce to the lightest.

// Points of the component-sorted order into their padded positions: the
// component c occupies [pstart[c], pstart[c] + |c|) of the tile order, its
// points in sorted[sstart[c] ..).
__global__ void k_fr_perm(const int32_t *__restrict__ sorted, const int32_t *__restrict__ comp, int64_t n,
                          const int32_t *__restrict__ pstart, const int32_t *__restrict__ sstart,
                          int32_t *__restrict__ permF, int32_t *__restrict__ posF) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n) return;
    const int32_t id = sorted[q];
    const int c = comp[id];
    const int32_t pos = pstart[c] + (int32_t)(q - sstart[c]);
    permF[pos] = id;
    posF[id] = pos;
}

// One wave per row: exact values of the row's candidates that can still be
// its lightest edge into their component and their pair of components' (the
// screen's bound U), the row's lightest (D^2, j) per
// other component (with i fixed the total order is (D^2, j)), and W1 = the
// smallest D^2 per pair of components.
template <bool F64>
__global__ __launch_bounds__(256) void k_fr_recheck(const float *__restrict__ X, int64_t n, int64_t d, int64_t ld,
                                                    const int32_t *__restrict__ comp, const float *__restrict__ Emax,
                                                    const float *__restrict__ bestc, const int32_t *__restrict__ posF,
                                                    int64_t bstride, const uint32_t *__restrict__ upair,
                                                    const int32_t *__restrict__ ccnt, const int32_t *__restrict__ gcj,
                                                    const float *__restrict__ gcl, float kappa, float dn,
                                                    double *__restrict__ rowd, int32_t *__restrict__ rowj,
                                                    unsigned long long *__restrict__ W1,
                                                    int32_t *__restrict__ counters) {
    __shared__ unsigned long long td[4][FR_KC];
    __shared__ int32_t tj[4][FR_KC];
    __shared__ double dv[4][SCR_CAP2];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int evaluated = 0;
    // rows in a grid-stride walk; the trip count is the same for the four
    // waves of a workgroup (the barriers below are workgroup-wide)
    for (int64_t base = (int64_t)blockIdx.x * 4; base < n; base += (int64_t)gridDim.x * 4) {
        const int64_t i = base + w;
        const bool valid = i < n;
        const int cnt0 = valid ? ccnt[i] : 0;
        const int cnt = cnt0 <= SCR_CAP2 ? cnt0 : 0;  // (runs only when no list overflowed)
        const int ci = valid ? comp[i] : 0;
        const float E = valid ? Emax[i] : 0.0f;
        const float *xi = X + (valid ? i : 0) * ld;
        const float *bci = bestc + (valid ? posF[i] : 0);  // the row's minima per component, stride bstride
        const int32_t *js = gcj + (valid ? i : 0) * SCR_CAP2;
        const float *ls = gcl + (valid ? i : 0) * SCR_CAP2;
        for (int c = lane; c < FR_KC; c += 64) {
            td[w][c] = U64_MAX;
            tj[w][c] = 0x7FFFFFFF;
        }
        __syncthreads();
        if (F64) {
            for (int q = lane; q < cnt; q += 64) {
                const int32_t j = js[q];
                const int c2 = comp[j];
                double v = __builtin_huge_val();
                if (ls[q] <= fminf((bci[c2 * bstride] + E) * kappa, __uint_as_float(upair[fr_pair(ci, c2)]) * dn)) {
                    v = d2_f64_lane(xi, X + (int64_t)j * ld, d);
                    ++evaluated;
                    atomicMin(&td[w][c2], (unsigned long long)__double_as_longlong(v));
                }
                dv[w][q] = v;
            }
        } else {
            for (int q = 0; q < cnt; ++q) {
                const int32_t j = js[q];
                const int c2 = comp[j];
                double v = __builtin_huge_val();
                if (ls[q] <= fminf((bci[c2 * bstride] + E) * kappa, __uint_as_float(upair[fr_pair(ci, c2)]) * dn)) {
                    v = (double)d2_f32_wave(xi, X + (int64_t)j * ld, d);
                    if (lane == 0) {
                        ++evaluated;
                        atomicMin(&td[w][c2], (unsigned long long)__double_as_longlong(v));
                    }
                }
                if (lane == 0) dv[w][q] = v;
            }
        }
        __syncthreads();
        for (int q = lane; q < cnt; q += 64) {
            const double v = dv[w][q];
            if (!(v < __builtin_huge_val())) continue;
            const int32_t j = js[q];
            const int c2 = comp[j];
            if ((unsigned long long)__double_as_longlong(v) == td[w][c2]) atomicMin(&tj[w][c2], j);
        }
        __syncthreads();
        if (valid) {
            for (int c = lane; c < FR_KC; c += 64) {
                const unsigned long long b = td[w][c];
                rowd[i * FR_KC + c] = b == U64_MAX ? __builtin_huge_val() : __longlong_as_double((long long)b);
                rowj[i * FR_KC + c] = b == U64_MAX ? -1 : tj[w][c];
                if (b != U64_MAX) atomicMin(&W1[fr_pair(ci, c)], b);
            }
        }
        __syncthreads();  // the next row reinitialises this wave's tables
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) evaluated += __shfl_xor(evaluated, off, 64);
    if (lane == 0 && evaluated)
        atomicAdd((unsigned long long *)&counters[C_CAND], (unsigned long long)evaluated);
}

// The work the recheck would do: candidates that pass its filter (C_FRWORK)
// and rows whose list overflowed (C_OVF).  One wave per row.
__global__ __launch_bounds__(256) void k_fr_count(int64_t n, const int32_t *__restrict__ comp,
                                                  const float *__restrict__ Emax, const float *__restrict__ bestc,
                                                  const int32_t *__restrict__ posF, int64_t bstride,
                                                  const uint32_t *__restrict__ upair,
                                                  const int32_t *__restrict__ ccnt, const int32_t *__restrict__ gcj,
                                                  const float *__restrict__ gcl, float kappa, float dn,
                                                  int32_t *__restrict__ counters) {
    const int lane = threadIdx.x & 63;
    int pass = 0;
    for (int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); i < n; i += (int64_t)gridDim.x * 4) {
        const int cnt0 = ccnt[i];
        if (cnt0 > SCR_CAP2) {
            if (lane == 0) atomicAdd(&counters[C_OVF], 1);
            continue;
        }
        const int ci = comp[i];
        const float E = Emax[i];
        const float *bci = bestc + posF[i];
        for (int q = lane; q < cnt0; q += 64) {
            const int c2 = comp[gcj[i * SCR_CAP2 + q]];
            pass += gcl[i * SCR_CAP2 + q] <=
                    fminf((bci[c2 * bstride] + E) * kappa, __uint_as_float(upair[fr_pair(ci, c2)]) * dn);
        }
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) pass += __shfl_xor(pass, off, 64);
    if (lane == 0 && pass) atomicAdd((unsigned long long *)&counters[C_FRWORK], (unsigned long long)pass);
}

// W2 = the smallest (smaller id, larger id) among the rows' records that reach
// W1 of their pair of components.
__global__ void k_fr_pick(const double *__restrict__ rowd, const int32_t *__restrict__ rowj,
                          const int32_t *__restrict__ comp, int64_t n, const unsigned long long *__restrict__ W1,
                          unsigned long long *__restrict__ W2) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= n * FR_KC) return;
    const int32_t j = rowj[g];
    if (j < 0) return;
    const int64_t i = g / FR_KC;
    const int c = (int)(g % FR_KC);
    const int pr = fr_pair(comp[i], c);
    if ((unsigned long long)__double_as_longlong(rowd[g]) != W1[pr]) return;
    const uint32_t lo = (uint32_t)min((int64_t)j, i), hi = (uint32_t)max((int64_t)j, i);
    atomicMin(&W2[pr], ((unsigned long long)lo << 32) | hi);
}

// ------------------------------------------------------------------ contraction

__global__ void k_comp_min1(const double *__restrict__ rb_d2, const int32_t *__restrict__ rb_j,
                            const int32_t *__restrict__ comp, int64_t n, unsigned long long *__restrict__ ck1) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || rb_j[i] < 0) return;
    atomicMin(&ck1[comp[i]], (unsigned long long)__double_as_longlong(rb_d2[i]));
}

__global__ void k_comp_min2(const double *__restrict__ rb_d2, const int32_t *__restrict__ rb_j,
                            const int32_t *__restrict__ comp, int64_t n, const unsigned long long *__restrict__ ck1,
                            unsigned long long *__restrict__ ck2) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || rb_j[i] < 0) return;
    const int c = comp[i];
    if ((unsigned long long)__double_as_longlong(rb_d2[i]) != ck1[c]) return;
    const uint32_t j = (uint32_t)rb_j[i];
    const uint32_t lo = (uint32_t)i < j ? (uint32_t)i : j;
    const uint32_t hi = (uint32_t)i < j ? j : (uint32_t)i;
    atomicMin(&ck2[c], ((unsigned long long)lo << 32) | hi);
}

__global__ void k_hook1(const unsigned long long *__restrict__ ck2, const int32_t *__restrict__ comp, int64_t ncomp,
                        int32_t *__restrict__ cpar, int32_t *__restrict__ counters) {
    int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncomp) return;
    unsigned long long key = ck2[c];
    if (key == U64_MAX) {
        atomicExch(&counters[C_NOEDGE], 1);
        cpar[c] = (int32_t)c;
        return;
    }
    int a = (int)(key >> 32), b = (int)(key & 0xFFFFFFFFu);
    int ca = comp[a], cb = comp[b];
    cpar[c] = (ca == (int)c) ? cb : ca;
}

__global__ void k_hook2(const unsigned long long *__restrict__ ck2, const int32_t *__restrict__ cpar, int64_t ncomp,
                        int32_t *__restrict__ npar, int32_t *__restrict__ eu, int32_t *__restrict__ ev,
                        int64_t edge_cap, int32_t *__restrict__ counters) {
    int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncomp) return;
    int o = cpar[c];
    if (o == (int)c) {
        npar[c] = (int32_t)c;
        return;
    }
    if (cpar[o] == (int)c && (int)c < o) {  // mutual pair: the smaller id is the root
        npar[c] = (int32_t)c;
        return;
    }
    npar[c] = o;
    unsigned long long key = ck2[c];
    int p = atomicAdd(&counters[C_EDGES], 1);
    if (p < edge_cap) {  // more than n-1 edges would be an internal error, reported by the host
        eu[p] = (int32_t)(key >> 32);
        ev[p] = (int32_t)(key & 0xFFFFFFFFu);
    }
}

__global__ void k_jump(int32_t *__restrict__ npar, int64_t ncomp) {
    int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncomp) return;
    npar[c] = npar[npar[c]];
}

__global__ void k_isroot(const int32_t *__restrict__ npar, int64_t ncomp, int32_t *__restrict__ flag) {
    int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncomp) return;
    flag[c] = npar[c] == (int32_t)c ? 1 : 0;
}

__global__ void k_relabel(int32_t *__restrict__ comp, int64_t n, const int32_t *__restrict__ npar,
                          const int32_t *__restrict__ newid) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    comp[i] = newid[npar[comp[i]]];
}

// Sum of the squared component sizes (timing only: the screen of a round must
// cover (n^2 - sum |c|^2) / 2 unordered pairs).
__global__ __launch_bounds__(1024) void k_sum_squares(const int32_t *__restrict__ size, int64_t m,
                                                      int32_t *__restrict__ counters) {
    __shared__ unsigned long long s[1024];
    unsigned long long acc = 0;
    for (int64_t c = threadIdx.x; c < m; c += 1024) acc += (unsigned long long)size[c] * (unsigned long long)size[c];
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 512; w >= 1; w >>= 1) {
        if ((int)threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *(unsigned long long *)&counters[C_SUMSQ] = s[0];
}

// ------------------------------------------------------------------ FP64 lengths and rooting

// Length of each tree edge: sqrt of the FP64 left-to-right sum of squared
// coordinate differences.
// FP64 edge lengths: one lane per edge sums its squared coordinate differences
// left to right (as d2_f64_lane); the two rows of the wave's 64 edges are
// staged through LDS 16 coordinates at a time with coalesced loads.
constexpr int REF_T = 16;
__global__ __launch_bounds__(256) void k_refine(const float *__restrict__ X, int64_t d, int64_t ld,
                                                const int32_t *__restrict__ eu, const int32_t *__restrict__ ev,
                                                int64_t m, double *__restrict__ elen) {
    __shared__ float st[4][2][64][REF_T + 1];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t e0 = ((int64_t)blockIdx.x * 4 + w) * 64;
    // loader roles: slot k of this lane stages 4 coordinates of row (r) of edge
    // e0 + ed, ed = idx / 8, r = (idx / 4) mod 2, part = idx mod 4, idx = lane + 64 k
    const float *src[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const int idx = lane + 64 * k;
        const int64_t ee = e0 + (idx >> 3);
        const int r = (idx >> 2) & 1;
        src[k] = ee < m ? X + (int64_t)(r ? ev[ee] : eu[ee]) * ld + 4 * (idx & 3) : nullptr;
    }
    double s = 0.0;
    for (int64_t t0 = 0; t0 < d; t0 += REF_T) {
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int idx = lane + 64 * k;
            float v[4] = {0.0f, 0.0f, 0.0f, 0.0f};
            if (src[k]) {
#pragma unroll
                for (int c = 0; c < 4; ++c)
                    if (t0 + 4 * (idx & 3) + c < d) v[c] = src[k][t0 + c];
            }
#pragma unroll
            for (int c = 0; c < 4; ++c) st[w][(idx >> 2) & 1][idx >> 3][4 * (idx & 3) + c] = v[c];
        }
        __syncthreads();
        const int tn = d - t0 < REF_T ? (int)(d - t0) : REF_T;
        for (int c = 0; c < tn; ++c) {
            const double df = (double)st[w][0][lane][c] - (double)st[w][1][lane][c];
            const double p = df * df;
            s = s + p;
        }
        __syncthreads();
    }
    if (e0 + lane < m) elen[e0 + lane] = sqrt(s);
}

__global__ void k_degree(const int32_t *__restrict__ eu, const int32_t *__restrict__ ev, int64_t m,
                         int32_t *__restrict__ deg) {
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= m) return;
    atomicAdd(&deg[eu[e]], 1);
    atomicAdd(&deg[ev[e]], 1);
}

// Adjacency lists of the tree: arc a -> b of edge e sits in a's list, and
// earc[2 e], earc[2 e + 1] record the positions of its two arcs (eu -> ev, ev -> eu).
__global__ void k_fill_adj(const int32_t *__restrict__ eu, const int32_t *__restrict__ ev, int64_t m,
                           const int32_t *__restrict__ off, int32_t *__restrict__ cursor, int32_t *__restrict__ adj,
                           int32_t *__restrict__ adje, int32_t *__restrict__ earc) {
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= m) return;
    int a = eu[e], b = ev[e];
    int pa = off[a] + atomicAdd(&cursor[a], 1);
    adj[pa] = b;
    adje[pa] = (int32_t)e;
    int pb = off[b] + atomicAdd(&cursor[b], 1);
    adj[pb] = a;
    adje[pb] = (int32_t)e;
    earc[2 * e] = pa;
    earc[2 * e + 1] = pb;
}

// Rooting at vertex 0 by an Euler tour: the tour walks every arc once, and
// after arc u -> v it takes the arc that follows v -> u in v's list
// (cyclically); the arc that would lead back to the root's first arc (arc 0)
// ends it.  Each arc's distance to the end of the tour comes from pointer
// jumping (log2 of the arc count rounds); of an edge's two arcs the one taken
// first, the farther from the end, goes from parent to child.  Whatever order
// the adjacency lists have, the parents are the tree's unique ones.
__global__ void k_tour_succ(const int32_t *__restrict__ off, const int32_t *__restrict__ adj,
                            const int32_t *__restrict__ adje, const int32_t *__restrict__ earc, int64_t narcs,
                            int32_t *__restrict__ nxt, int32_t *__restrict__ rk) {
    const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= narcs) return;
    const int32_t e = adje[x];
    const int32_t r = earc[2 * e] == (int32_t)x ? earc[2 * e + 1] : earc[2 * e];  // the reverse arc, in v's list
    const int32_t v = adj[x];
    int32_t nx = r + 1 < off[v + 1] ? r + 1 : off[v];
    if (nx == 0) nx = -1;  // back at the root's first arc: the tour ends
    nxt[x] = nx;
    rk[x] = 1;
}

__global__ void k_tour_jump(const int32_t *__restrict__ nxt_in, const int32_t *__restrict__ rk_in, int64_t narcs,
                            int32_t *__restrict__ nxt_out, int32_t *__restrict__ rk_out) {
    const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= narcs) return;
    int32_t nx = nxt_in[x], r = rk_in[x];
    if (nx >= 0) {
        r += rk_in[nx];
        nx = nxt_in[nx];
    }
    nxt_out[x] = nx;
    rk_out[x] = r;
}

__global__ void k_tour_orient(const int32_t *__restrict__ eu, const int32_t *__restrict__ ev,
                              const int32_t *__restrict__ earc, const int32_t *__restrict__ rk,
                              const double *__restrict__ elen, int64_t m, int32_t *__restrict__ parent,
                              double *__restrict__ length) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e == 0) {
        parent[0] = -1;
        length[0] = 0.0;
    }
    if (e >= m) return;
    const int32_t a = eu[e], b = ev[e];
    const bool a_first = rk[earc[2 * e]] > rk[earc[2 * e + 1]];  // arc a -> b taken before b -> a
    const int32_t child = a_first ? b : a;
    parent[child] = a_first ? a : b;
    length[child] = elen[e];
}

// Deterministic FP64 sum of length[1..n) (one workgroup, fixed tree).
__global__ __launch_bounds__(1024) void k_sum_lengths(const double *__restrict__ length, int64_t n,
                                                      double *__restrict__ out) {
    __shared__ double s[1024];
    double acc = 0.0;
    for (int64_t v = 1 + threadIdx.x; v < n; v += 1024) acc = acc + length[v];
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 512; w >= 1; w >>= 1) {
        if ((int)threadIdx.x < w) s[threadIdx.x] = s[threadIdx.x] + s[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = s[0];
}

// ------------------------------------------------------------------ tile order

// Identity tile order (positions = point ids), padding included.
__global__ void k_perm_identity(int32_t *__restrict__ perm, int64_t n_pad) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_pad; i += (int64_t)gridDim.x * blockDim.x)
        perm[i] = (int32_t)i;
}

// Sort keys for the tile order: (component, id), stable sort by component.
__global__ void k_perm_keys(const int32_t *__restrict__ comp, int64_t n, uint32_t *__restrict__ keys,
                            int32_t *__restrict__ vals) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    keys[i] = (uint32_t)comp[i];
    vals[i] = (int32_t)i;
}

// Component range of every tile of the order (points sorted by component, so
// the first and last valid point bound it).
__global__ void k_tile_ranges(const int32_t *__restrict__ perm, const int32_t *__restrict__ comp, int64_t n,
                              int64_t nt, int64_t tile, int32_t *__restrict__ tlo, int32_t *__restrict__ thi) {
    const int64_t T = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (T >= nt) return;
    const int64_t first = T * tile;
    const int64_t last = std::min<int64_t>(first + tile, n) - 1;
    tlo[T] = first < n ? comp[perm[first]] : -1;
    thi[T] = first < n ? comp[perm[last]] : -2;
}

// A tile pair is skipped when all of its points lie in one component (no pair
// of it can be an outgoing edge); a kept pair is screened with the component
// mask (keep_m) when it is diagonal or its tiles share a component, else
// without it (keep_u).  The order is sorted by component and pr.x <= pr.y, so
// the tiles share a component exactly when the greatest of the first reaches
// the least of the second.  Pruned rounds (phase 1 and 2, see the tile-pair
// pruning above) keep in phase 1 the pairs whose balls meet (plb = 0) and in
// phase 2 those with 0 < plb <= the larger reach of their tiles; they count
// the tile pairs a full screen would run (phase 1, C_TPFULL) and the point
// pairs of the kept ones (C_PAIRS: cnt_I cnt_J off the diagonal; on it
// cnt (cnt - 1) / 2 when diag_all, i.e. every point its own component, else 0,
// since a diagonal tile's pairs within one component are not counted).
__global__ void k_pair_keep(const int2 *__restrict__ pairs, int64_t npairs, const int32_t *__restrict__ tlo,
                            const int32_t *__restrict__ thi, const float *__restrict__ plb,
                            const float *__restrict__ tthr, const int32_t *__restrict__ tcnt, int phase,
                            int diag_all, int32_t *__restrict__ keep_m, int32_t *__restrict__ keep_u,
                            int32_t *__restrict__ counters) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    bool full = false;
    unsigned long long np = 0;
    if (k < npairs) {
        const int2 pr = pairs[k];
        const bool one = tlo[pr.x] == thi[pr.x] && tlo[pr.y] == thi[pr.y] && tlo[pr.x] == tlo[pr.y];
        const bool masked = pr.x == pr.y || thi[pr.x] >= tlo[pr.y];
        bool sel = !one;
        full = sel;
        if (phase == 1) {
            sel = sel && plb[k] <= 0.0f;
        } else if (phase == 2) {
            const float l = plb[k];
            sel = sel && l > 0.0f && l <= fmaxf(tthr[pr.x], tthr[pr.y]);
        }
        keep_m[k] = sel && masked ? 1 : 0;
        keep_u[k] = sel && !masked ? 1 : 0;
        if (phase > 0 && sel) {
            const unsigned long long a = (unsigned long long)tcnt[pr.x], b = (unsigned long long)tcnt[pr.y];
            np = pr.x != pr.y ? (masked ? 0ull : a * b) : (diag_all && a > 0 ? a * (a - 1) / 2 : 0ull);
        }
    }
    if (phase == 0) return;
    const unsigned long long nfull = __popcll(__ballot(phase == 1 && full));
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) np += __shfl_xor(np, o, 64);
    if ((threadIdx.x & 63) == 0) {
        if (np) atomicAdd(reinterpret_cast<unsigned long long *>(&counters[C_PAIRS]), np);
        if (nfull) atomicAdd(&counters[C_TPFULL], (int32_t)nfull);
    }
}

// Rows of the representation in the tile order, stored tile by tile and,
// within a tile, K chunk by K chunk: the 64-byte pieces of chunk c of the
// tile's GT rows are contiguous (position q, 16-byte piece t of its row at
// uint4 index (q / GT) GT row_u4 + (t / 4) 4 GT + (q mod GT) 4 + t mod 4), so
// the tile-pair screen stages each chunk from whole, consecutive cache lines.
// One workgroup per (tile, chunk); npos is a multiple of GT.
__global__ __launch_bounds__(256) void k_permute_rows(const uint4 *__restrict__ Xr, const int32_t *__restrict__ perm,
                                                      int64_t nchunks, int64_t row_u4, uint4 *__restrict__ Xq) {
    static_assert(GT == 256, "four pieces per thread cover a chunk of the tile");
    const int64_t tile = blockIdx.x / nchunks, c = blockIdx.x - tile * nchunks;
    uint4 *dst = Xq + (tile * nchunks + c) * (4 * GT);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int e = k * 256 + (int)threadIdx.x;  // row e / 4 of the tile, piece e mod 4 of the chunk
        dst[e] = Xr[(int64_t)perm[tile * GT + (e >> 2)] * row_u4 + c * 4 + (e & 3)];
    }
}

// The same copy in the BF16 screen's fragment order: within the 16 KB of
// chunk c of a tile, 32-row block b at uint4 128 b, 16-wide K step t at +64 t,
// then lane l = 32 h + (row mod 32) at +l, holding elements 16 t + 8 h .. +7
// of the chunk (the row's 16-byte piece 2 t + h): the operand one lane feeds to
// a 32 x 32 x 16 MFMA, so a wave reads a block's K step as one contiguous 1 KB.
__global__ __launch_bounds__(256) void k_permute_rows_frag(const uint4 *__restrict__ Xr,
                                                           const int32_t *__restrict__ perm, int64_t nchunks,
                                                           int64_t row_u4, uint4 *__restrict__ Xq) {
    static_assert(GT == 256, "four pieces per thread cover a chunk of the tile");
    const int64_t tile = blockIdx.x / nchunks, c = blockIdx.x - tile * nchunks;
    uint4 *dst = Xq + (tile * nchunks + c) * (4 * GT);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int u = k * 256 + (int)threadIdx.x;  // destination slot
        const int row = 32 * (u >> 7) + (u & 31), piece = 2 * ((u >> 6) & 1) + ((u >> 5) & 1);
        dst[u] = Xr[(int64_t)perm[tile * GT + row] * row_u4 + c * 4 + piece];
    }
}

// Per-position copies of the per-point values the tile-pair screen reads, in
// the tile order `order` (npos positions; ids >= n are padding: Emax 0).
// Optional inputs (nullptr) are skipped.
__global__ void k_pos_gather(const int32_t *__restrict__ order, int64_t npos, int64_t n, const float *__restrict__ sq,
                             const int32_t *__restrict__ comp, const float *__restrict__ Emax,
                             const float *__restrict__ rn, const float *__restrict__ re, const int32_t *__restrict__ sqi,
                             const float *__restrict__ ltau, float *__restrict__ psq, int32_t *__restrict__ pcomp,
                             float *__restrict__ pEmax, float *__restrict__ prn, float *__restrict__ pre,
                             int32_t *__restrict__ psqi, float *__restrict__ pltau) {
    const int64_t pos = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (pos >= npos) return;
    const int32_t id = order[pos];
    const bool real = id < n;
    psq[pos] = sq[id];
    pcomp[pos] = comp[id];
    pEmax[pos] = real ? Emax[id] : 0.0f;
    if (rn) {
        prn[pos] = rn[id];
        pre[pos] = re[id];
    }
    if (sqi) psqi[pos] = sqi[id];
    if (ltau) pltau[pos] = real ? ltau[id] : -1.0f;
}

// Largest r and e over each tile's positions (padding has r = e = 0).
__global__ void k_tile_max(const float *__restrict__ prn, const float *__restrict__ pre, int64_t ntiles, int tile,
                           float *__restrict__ trmax, float *__restrict__ temax) {
    const int64_t T = (int64_t)blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64;
    const int lane = threadIdx.x & 63;
    if (T >= ntiles) return;
    float r = 0.0f, e = 0.0f;
    for (int q = lane; q < tile; q += 64) {
        r = fmaxf(r, prn[T * tile + q]);
        e = fmaxf(e, pre[T * tile + q]);
    }
    for (int o = 32; o > 0; o >>= 1) {
        r = fmaxf(r, __shfl_xor(r, o));
        e = fmaxf(e, __shfl_xor(e, o));
    }
    if (lane == 0) {
        trmax[T] = r;
        temax[T] = e;
    }
}

// Folds running minima kept by position back into the per-point array.
// The projection's reference tiles q ntiles / nref (q < nref): their centroids
// (rows of out) and point counts (out_cnt), gathered for one copy to the host.
__global__ void k_ref_gather(const float *__restrict__ cen, const int32_t *__restrict__ tcnt, int64_t ntiles,
                             int64_t d, int nref, float *__restrict__ out, int32_t *__restrict__ out_cnt) {
    const int q = blockIdx.x;
    const int64_t t = (int64_t)q * ntiles / nref;
    for (int64_t k = threadIdx.x; k < d; k += blockDim.x) out[(int64_t)q * d + k] = cen[t * d + k];
    if (threadIdx.x == 0) out_cnt[q] = tcnt[t];
}

__global__ void k_pos_scatter(const int32_t *__restrict__ order, int64_t npos, int64_t n,
                              const float *__restrict__ pv, float *__restrict__ v) {
    const int64_t pos = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (pos >= npos) return;
    const int32_t id = order[pos];
    if (id < n) v[id] = pv[pos];
}

// Stable partition of the kept pairs: the masked ones first (positions pos_m),
// then the others (pos_u after the masked total pos_m[npairs]).
__global__ void k_pair_scatter(const int2 *__restrict__ pairs, int64_t npairs, const int32_t *__restrict__ keep_m,
                               const int32_t *__restrict__ pos_m, const int32_t *__restrict__ keep_u,
                               const int32_t *__restrict__ pos_u, int2 *__restrict__ out) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= npairs) return;
    if (keep_m[k]) out[pos_m[k]] = pairs[k];
    if (keep_u[k]) out[pos_m[npairs] + pos_u[k]] = pairs[k];
}

// ------------------------------------------------------------------ tile-pair pruning
//
// A tile pair whose two point sets are provably farther apart than the reach of
// every one of their points is not screened (the bounding-ball test of
// dual-tree Boruvka, March, Ram and Gray, KDD 2010, on the screen's tiles).
// With c_T the centroid of tile T's rows and rad_T >= max ||x - c_T|| over
// them (exact FP32 inputs), the triangle inequality gives, for every i in I and
// j in J, D(i, j) >= LB = ||c_I - c_J|| - rad_I - rad_J.  The reach of a point
// bounds every value the round can still need from it:
//   R_i = kappa (b_i + Emax_i) once its running minimum b_i is known: its
//   lightest edge has a recheck value of at most (1 + rho) (b_i + Emax_i),
//   while a pair with real distance >= LB has one of at least (1 - rho) LB^2;
//   (with pair bounds R_i = kappa ub_i, ub_i the running upper bound);
//   R_i may be lowered to U_c dn, c = comp(i), U_c the component's upper
//   bound of its lightest outgoing edge (recheck scale): the round needs only
//   that edge of every component (the pair, within its own row's reach, keeps
//   the row's capture);
//   in the round that builds neighbour lists R_i >= tau_i + Emax_i as well
//   (a list takes the partners with Dhat^2 <= tau_i, and Dhat^2 >= D^2 - Emax_i).
// A tile pair with LB^2 > max R over both tiles then holds no edge the round
// selects and no list entry, so every component's lightest edge, the lists
// and the tree are those of the full screen (a row whose own lightest edge
// lies beyond its component's U may keep a larger running minimum, which only
// bounds its own candidates).
// Each round screens first the tile pairs whose balls meet (LB = 0), then,
// with the reach known, the other pairs that the bound cannot exclude.  Tiles
// group nearby points: the first round orders the points by their nearest of
// PIV pivot rows (the pivots in a nearest-neighbour chain), and the component
// labels follow that order, so every later round's component order stays
// spatial.  The final round applies the same bound per pair of components
// (see run_mst).

constexpr int PIV = 32;              // pivot rows of the first round's order
constexpr int PRUNE_MIN_TILES = 32;  // fewer tiles (n < 8,192): every pair is screened, which costs less
constexpr int64_t PRUNE_MAX_D = 8192;  // the tile centroid is held in LDS
constexpr int64_t PRUNE_MAX_TILES = 8192;  // the final round's supports: ntF^2 floats

// Nearest pivot of each of `count` rows (row rows[r], or r when rows is null),
// by FP32 sums of squared differences; 128 rows x PIV pivots per workgroup
// (thread t: rows 4 (t / 8) .. +3, pivots 4 (t mod 8) .. +3), 64 coordinates
// at a time through LDS; ties go to the smaller pivot index.  dist (nullable)
// receives the PIV squared distances of every row.
__global__ __launch_bounds__(256) void k_pivot_near(const float *__restrict__ X, int64_t d, int64_t ld,
                                                    const int32_t *__restrict__ rows, int64_t count,
                                                    const int32_t *__restrict__ piv, uint32_t *__restrict__ key,
                                                    float *__restrict__ dist) {
    static_assert(PIV == 32, "eight groups of four pivots");
    __shared__ float sx[128][65];
    __shared__ float sp[PIV][65];
    __shared__ int64_t roff[128 + PIV];  // element offsets of the rows, then of the pivots; -1: no row
    const int tid = threadIdx.x, tr = tid >> 3, tp = tid & 7, w = tid >> 6, c = tid & 63;
    const int64_t r0 = (int64_t)blockIdx.x * 128;
    if (tid < 128) {
        const int64_t g = r0 + tid;
        roff[tid] = g < count ? (rows ? (int64_t)rows[g] : g) * ld : -1;
    } else if (tid < 128 + PIV) {
        roff[tid] = (int64_t)piv[tid - 128] * ld;
    }
    __syncthreads();
    float acc[4][4] = {};
    for (int64_t k0 = 0; k0 < d; k0 += 64) {
        // every load first (no branch between them), then the LDS writes; a
        // missing row or a coordinate beyond d reads X[0] and stores 0
        const int64_t k = k0 + c;
        float vx[32], vp[8];
#pragma unroll
        for (int e = 0; e < 32; ++e) {
            const int64_t o = roff[w + 4 * e];
            const bool ok = o >= 0 && k < d;
            vx[e] = X[ok ? o + k : 0];
            vx[e] = ok ? vx[e] : 0.0f;
        }
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const bool ok = k < d;
            vp[e] = X[ok ? roff[128 + w + 4 * e] + k : 0];
            vp[e] = ok ? vp[e] : 0.0f;
        }
#pragma unroll
        for (int e = 0; e < 32; ++e) sx[w + 4 * e][c] = vx[e];
#pragma unroll
        for (int e = 0; e < 8; ++e) sp[w + 4 * e][c] = vp[e];
        __syncthreads();
#pragma unroll 4
        for (int c = 0; c < 64; ++c) {
            float xa[4], pb[4];
#pragma unroll
            for (int a = 0; a < 4; ++a) xa[a] = sx[4 * tr + a][c];
#pragma unroll
            for (int b = 0; b < 4; ++b) pb[b] = sp[4 * tp + b][c];
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b = 0; b < 4; ++b) {
                    const float t = xa[a] - pb[b];
                    acc[a][b] = fmaf(t, t, acc[a][b]);
                }
        }
        __syncthreads();
    }
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        const int64_t g = r0 + 4 * tr + a;
        float best = acc[a][0];
        int bi = 4 * tp;
#pragma unroll
        for (int b = 1; b < 4; ++b)
            if (acc[a][b] < best) {
                best = acc[a][b];
                bi = 4 * tp + b;
            }
        // the 8 lanes of one row group differ in their low three bits
#pragma unroll
        for (int o = 1; o < 8; o <<= 1) {
            const float ob = __shfl_xor(best, o, 64);
            const int oi = __shfl_xor(bi, o, 64);
            if (ob < best || (ob == best && oi < bi)) {
                best = ob;
                bi = oi;
            }
        }
        if (g < count) {
            if (tp == 0) key[g] = (uint32_t)bi;
            if (dist)
#pragma unroll
                for (int b = 0; b < 4; ++b) dist[g * PIV + 4 * tp + b] = acc[a][b];
        }
    }
}

// Sort keys of the first round's order: the rank of the point's pivot in the chain.
__global__ void k_pivot_keys(uint32_t *__restrict__ keys, const int32_t *__restrict__ rank, int64_t n,
                             int32_t *__restrict__ vals) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    keys[v] = (uint32_t)rank[keys[v]];
    vals[v] = (int32_t)v;
}

// Component labels of the first round in the order's sequence: comp[order[p]] = p.
__global__ void k_comp_from_order(const int32_t *__restrict__ order, int64_t n, int32_t *__restrict__ comp) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    comp[order[p]] = (int32_t)p;
}

// Ball of every tile of the order (GT positions each; ids >= n are padding),
// in two kernels: cen = the centroid of its rows (FP64 sums rounded to FP32)
// and cnt = its rows, then rad >= the largest distance of a row from that
// stored centroid (FP64 sums widened by their rounding bound, rounded up).
// k_tile_centroid: grid (tiles, ceil(d / 256)), one coordinate per thread.
__global__ __launch_bounds__(256) void k_tile_centroid(const float *__restrict__ X, int64_t n, int64_t d, int64_t ld,
                                                       const int32_t *__restrict__ order, float *__restrict__ cen,
                                                       int32_t *__restrict__ cnt) {
    static_assert(GT == 256, "one position per thread");
    __shared__ int32_t rid[GT];
    __shared__ int32_t first;
    const int tid = threadIdx.x;
    const int64_t T = blockIdx.x;
    if (tid == 0) first = GT;
    const int32_t id = order[T * GT + tid];
    const bool valid = id < n;
    rid[tid] = valid ? id : -1;
    __syncthreads();
    if (valid) atomicMin(&first, tid);
    const int nv = __syncthreads_count(valid);
    if (blockIdx.y == 0 && tid == 0) cnt[T] = nv;
    if (nv == 0) return;
    const int64_t k = (int64_t)blockIdx.y * 256 + tid;
    if (k >= d) return;
    // (a padding position reads the tile's first row with weight 0)
    const int64_t f = rid[first];
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    for (int r = 0; r < GT; r += 16) {
        float x[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int32_t v = rid[r + u];
            x[u] = X[(v >= 0 ? (int64_t)v : f) * ld + k];
        }
#pragma unroll
        for (int u = 0; u < 16; u += 4) {
            s0 += rid[r + u] >= 0 ? (double)x[u] : 0.0;
            s1 += rid[r + u + 1] >= 0 ? (double)x[u + 1] : 0.0;
            s2 += rid[r + u + 2] >= 0 ? (double)x[u + 2] : 0.0;
            s3 += rid[r + u + 3] >= 0 ? (double)x[u + 3] : 0.0;
        }
    }
    cen[T * d + k] = (float)(((s0 + s1) + (s2 + s3)) / (double)nv);
}

// k_tile_radius: grid (tiles, 4), 64 positions per workgroup, each wave eight
// rows at a time; the centroid in dynamic LDS (d floats).  rad must hold 0
// (or a smaller bound) before: blocks combine by an atomic max of the bits
// (nonnegative floats order like their bits).
__global__ __launch_bounds__(256) void k_tile_radius(const float *__restrict__ X, int64_t n, int64_t d, int64_t ld,
                                                     const int32_t *__restrict__ order, const float *__restrict__ cen,
                                                     const int32_t *__restrict__ cnt, float *__restrict__ rad) {
    extern __shared__ float cs[];
    __shared__ double wmax[4];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int64_t T = blockIdx.x;
    if (cnt[T] == 0) return;
    for (int64_t k = tid; k < d; k += 256) cs[k] = cen[T * d + k];
    __syncthreads();
    double m = 0.0;
    const int64_t p0 = T * GT + (int64_t)blockIdx.y * 64 + w * 16;
    for (int r0 = 0; r0 < 16; r0 += 8) {
        // eight rows at a time, loads without branches (a padding position
        // reads row 0 and is left out of the maximum)
        int64_t off[8];
        bool ok[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int32_t id = order[p0 + r0 + j];
            ok[j] = id < n;
            off[j] = ok[j] ? (int64_t)id * ld : 0;
        }
        double a[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        for (int64_t k = lane; k < d; k += 64) {
            const double c = (double)cs[k];
            float x[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) x[j] = X[off[j] + k];
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const double t = (double)x[j] - c;
                a[j] = fma(t, t, a[j]);
            }
        }
#pragma unroll
        for (int j = 0; j < 8; ++j) {
#pragma unroll
            for (int o = 32; o >= 1; o >>= 1) a[j] += __shfl_xor(a[j], o, 64);
            if (ok[j]) m = fmax(m, a[j]);
        }
    }
    if (lane == 0) wmax[w] = m;
    __syncthreads();
    if (tid == 0) {
        const double mm = fmax(fmax(wmax[0], wmax[1]), fmax(wmax[2], wmax[3]));
        // recursive FP64 sums of d + 64 nonnegative terms: relative error below (d + 64) 2^-53
        const double r = sqrt(mm) * (1.0 + (double)(d + 68) * 0x1p-52);
        float f = (float)r;
        if ((double)f < r) f = nextafterf(f, SCR_INF);
        atomicMax(reinterpret_cast<unsigned int *>(rad) + T, __float_as_uint(f));
    }
}

// The support bound of the final round.  In high dimension the ball bound
// is loose: a row's deviation from its tile's centroid is nearly orthogonal
// to the direction of another tile, so the rows reach far less toward it than
// the radius.  With u = x - c_I, v = y - c_J and Delta = c_I - c_J,
//   D^2 = |Delta + u - v|^2 >= |Delta|^2 + 2 Delta.u - 2 Delta.v,
// and for any KQ x d matrix Q, Delta.u = (Q Delta).(Q u) + ((I - Q'Q) Delta).u,
// where |(I - Q'Q) Delta|^2 = |Delta|^2 - |Q Delta|^2 + (Q Delta)'(Q Q' - I)(Q Delta)
// <= |Delta|^2 - (1 - eta) |Q Delta|^2, eta >= ||Q Q' - I||.  Hence
//   D^2 >= |Delta|^2 - 2 (S_I(J) + S_J(I)) - 2 |Delta_perp| (rad_I + rad_J),
//   S_I(J) = max over x in I of (Q x - Q c_I).(Q c_J - Q c_I),
// with Q orthonormal rows spanning the differences of a few tile centroids
// (the directions that separate clusters).  Q, z = Q x and zc = Q c are FP64
// (rounding errors below 1e-11 of the magnitudes involved, mag^2 =
// (|c_I| + |c_J| + rad_I + rad_J + 1)^2, for d <= PRUNE_MAX_D), the supports
// FP32 (below 3e-6 mag^2 each); the bound keeps a margin of 4e-5 mag^2.
constexpr int KQ = 32;  // rows of Q

// z = Q x of every point (FP64): 256 points x KQ rows per workgroup, thread t
// owns points 4 (t / 4) .. +3 and rows 8 (t mod 4) .. +7; 32 coordinates at a
// time through LDS.
__global__ __launch_bounds__(256) void k_project(const float *__restrict__ X, int64_t n, int64_t d, int64_t ld,
                                                 const double *__restrict__ Q, double *__restrict__ z) {
    static_assert(KQ == 32, "four groups of eight rows");
    __shared__ float sx[256][33];
    __shared__ double sq[KQ][33];
    const int tid = threadIdx.x, tr = tid >> 2, tg = tid & 3, h = tid >> 5, c = tid & 31;
    const int64_t r0 = (int64_t)blockIdx.x * 256;
    double acc[4][8] = {};
    for (int64_t k0 = 0; k0 < d; k0 += 32) {
        // every load first, then the LDS writes (rows beyond n and
        // coordinates beyond d read X[0] or Q[0] and store 0)
        const int64_t k = k0 + c;
        float vx[32];
        double vq[4];
#pragma unroll
        for (int e = 0; e < 32; ++e) {
            const int64_t g = r0 + h + 8 * e;
            const bool ok = g < n && k < d;
            vx[e] = X[ok ? g * ld + k : 0];
            vx[e] = ok ? vx[e] : 0.0f;
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const bool ok = k < d;
            vq[e] = Q[ok ? (int64_t)(h + 8 * e) * d + k : 0];
            vq[e] = ok ? vq[e] : 0.0;
        }
#pragma unroll
        for (int e = 0; e < 32; ++e) sx[h + 8 * e][c] = vx[e];
#pragma unroll
        for (int e = 0; e < 4; ++e) sq[h + 8 * e][c] = vq[e];
        __syncthreads();
#pragma unroll 4
        for (int c = 0; c < 32; ++c) {
            double xa[4], qb[8];
#pragma unroll
            for (int a = 0; a < 4; ++a) xa[a] = (double)sx[4 * tr + a][c];
#pragma unroll
            for (int b = 0; b < 8; ++b) qb[b] = sq[8 * tg + b][c];
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b = 0; b < 8; ++b) acc[a][b] = fma(qb[b], xa[a], acc[a][b]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        const int64_t g = r0 + 4 * tr + a;
        if (g < n)
#pragma unroll
            for (int b = 0; b < 8; ++b) z[g * KQ + 8 * tg + b] = acc[a][b];
    }
}

// zc = Q c of every tile's stored centroid and cn >= |c| (FP64).  One
// workgroup per tile: thread t sums row t mod 32 of Q over its eighth of d.
__global__ __launch_bounds__(256) void k_tile_project(const float *__restrict__ cen, const int32_t *__restrict__ cnt,
                                                      int64_t d, const double *__restrict__ Q,
                                                      double *__restrict__ zc, double *__restrict__ cn) {
    __shared__ double part[8][KQ + 1];
    __shared__ double nrm[8];
    const int tid = threadIdx.x, q = tid & 31, h = tid >> 5;
    const int64_t T = blockIdx.x;
    const float *c = cen + T * d;
    const bool live = cnt[T] > 0;
    double s = 0.0, s2 = 0.0;
    if (live)
        for (int64_t k = h; k < d; k += 8) {
            const double v = (double)c[k];
            s = fma(Q[(int64_t)q * d + k], v, s);
            if (q == 0) s2 = fma(v, v, s2);
        }
    part[h][q] = s;
    if (q == 0) nrm[h] = s2;
    __syncthreads();
    if (tid < KQ) {
        double t = 0.0;
#pragma unroll
        for (int j = 0; j < 8; ++j) t += part[j][tid];
        zc[T * KQ + tid] = t;
    }
    if (tid == 0) {
        double t = 0.0;
#pragma unroll
        for (int j = 0; j < 8; ++j) t += nrm[j];
        cn[T] = sqrt(t) * (1.0 + 1e-12);
    }
}

// S[I][J] = max over the rows x of tile I of (z_x - zc_I).(zc_J - zc_I) in
// FP32 (both factors rounded to FP32, FP32 sums: an error below 3e-6 |u| |g|,
// which the pair bound's margin covers); -inf for a tile without rows.  One
// workgroup per tile I: its rows' u = z_x - zc_I in LDS, one tile J per thread.
__global__ __launch_bounds__(256) void k_tile_support(const int32_t *__restrict__ order, int64_t n,
                                                      const double *__restrict__ z, const double *__restrict__ zc,
                                                      const int32_t *__restrict__ cnt, int64_t nt,
                                                      float *__restrict__ S) {
    __shared__ __align__(16) float us[GT][KQ + 4];  // (rows 16-byte aligned: vector LDS reads)
    __shared__ int32_t ok[GT];
    const int tid = threadIdx.x;
    const int64_t T = blockIdx.x;
    if (cnt[T] == 0) {
        for (int64_t j = tid; j < nt; j += 256) S[T * nt + j] = -SCR_INF;
        return;
    }
    __shared__ double zt[KQ];
    if (tid < KQ) zt[tid] = zc[T * KQ + tid];
    {
        // (loads without branches: a padding row reads point 0 and is left out)
        const int32_t id = order[T * GT + tid];
        const bool valid = id < n;
        ok[tid] = valid ? 1 : 0;
        const double *zi = z + (valid ? (int64_t)id : 0) * KQ;
        double v[KQ];
#pragma unroll
        for (int q = 0; q < KQ; ++q) v[q] = zi[q];
        __syncthreads();
#pragma unroll
        for (int q = 0; q < KQ; ++q) us[tid][q] = valid ? (float)(v[q] - zt[q]) : 0.0f;
    }
    __syncthreads();
    for (int64_t J = tid; J - tid < nt; J += 256) {
        const bool live = J < nt;
        const double *zj = zc + (live ? J : T) * KQ;
        float g[KQ];
#pragma unroll
        for (int q = 0; q < KQ; ++q) g[q] = (float)(zj[q] - zt[q]);
        float m = -SCR_INF;
        for (int r = 0; r < GT; ++r) {
            float t = 0.0f;
#pragma unroll
            for (int q = 0; q < KQ; ++q) t = fmaf(us[r][q], g[q], t);
            m = ok[r] ? fmaxf(m, t) : m;
        }
        if (live) S[T * nt + J] = m;
    }
}

// Squared distances between the stored tile centroids, FP64 sums of the
// (exact) FP64 differences, rounded down to FP32: Dm[I][J] for I, J < nt (both
// halves).  Grid (ceil(nt / 32), ceil(nt / 32)); 32 x 32 tile pairs per
// workgroup, thread t: row 32 t / 256, columns 4 (t mod 8) .. +3; 32
// coordinates at a time through LDS.
__global__ __launch_bounds__(256) void k_tile_dist(const float *__restrict__ cen, int64_t nt, int64_t d,
                                                   float *__restrict__ Dm) {
    __shared__ float sa[32][33];
    __shared__ float sb[32][33];
    const int tid = threadIdx.x, i = tid >> 3, jg = tid & 7;
    const int64_t I0 = (int64_t)blockIdx.x * 32, J0 = (int64_t)blockIdx.y * 32;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int64_t k0 = 0; k0 < d; k0 += 32) {
        float va[4], vb[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int idx = tid + 256 * e, r = idx >> 5, c = idx & 31;
            const int64_t k = k0 + c;
            const bool oka = I0 + r < nt && k < d, okb = J0 + r < nt && k < d;
            va[e] = cen[oka ? (I0 + r) * d + k : 0];
            vb[e] = cen[okb ? (J0 + r) * d + k : 0];
            va[e] = oka ? va[e] : 0.0f;
            vb[e] = okb ? vb[e] : 0.0f;
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int idx = tid + 256 * e, r = idx >> 5, c = idx & 31;
            sa[r][c] = va[e];
            sb[r][c] = vb[e];
        }
        __syncthreads();
#pragma unroll 8
        for (int c = 0; c < 32; ++c) {
            const double x = (double)sa[i][c];
#pragma unroll
            for (int jj = 0; jj < 4; ++jj) {
                const double t = x - (double)sb[4 * jg + jj][c];
                acc[jj] = fma(t, t, acc[jj]);
            }
        }
        __syncthreads();
    }
    const int64_t I = I0 + i;
#pragma unroll
    for (int jj = 0; jj < 4; ++jj) {
        const int64_t J = J0 + 4 * jg + jj;
        if (I < nt && J < nt) {
            float f = (float)acc[jj];
            if ((double)f > acc[jj]) f = nextafterf(f, 0.0f);
            Dm[I * nt + J] = f;
        }
    }
}

// LB^2 of every tile pair, rounded down to FP32: the larger of the ball bound
// (LB = ||c_I - c_J|| - rad_I - rad_J, the distance from Dm narrowed by the
// rounding of its FP64 sum and of its FP32 storage, the radii widened) and,
// when S is given, the support bound above; 0 when neither excludes anything;
// NaN when a tile has no row (such a pair holds no pair of points and is never
// screened).  One thread per pair; nt is the row stride of Dm and S.
__global__ __launch_bounds__(256) void k_pair_lb(const int2 *__restrict__ pairs, int64_t npairs,
                                                 const float *__restrict__ Dm, const float *__restrict__ rad,
                                                 const int32_t *__restrict__ cnt, int64_t d,
                                                 const float *__restrict__ S, const double *__restrict__ zc,
                                                 const double *__restrict__ cn, int64_t nt, double eta,
                                                 float *__restrict__ plb) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= npairs) return;
    const int2 pr = pairs[k];
    const bool empty = cnt[pr.x] == 0 || cnt[pr.y] == 0;
    if (empty || pr.x == pr.y) {
        plb[k] = empty ? __builtin_nanf("") : 0.0f;
        return;
    }
    const double s = (double)Dm[(int64_t)pr.x * nt + pr.y];  // <= |c_I - c_J|^2 (1 + (d + 4) 2^-53)
    const float rI = rad[pr.x], rJ = rad[pr.y];
    const double dist = sqrt(s) * (1.0 - (double)(d + 68) * 0x1p-52);
    const double rs = ((double)rI + (double)rJ) * (1.0 + 0x1p-52);
    const double lb = dist - rs;
    double l2 = lb > 0.0 ? lb * lb * (1.0 - 0x1p-50) : 0.0;
    if (S) {
        // (the absolute slack 1e-10 mag^2 under the root covers the rounding
        // of g2 = |Q Delta|^2, below 1e-11 mag^2; s is at most 2^-24 + (d + 4)
        // 2^-53 below |Delta|^2 and enters the root with a margin of 1e-6)
        double g2 = 0.0;
        const double *za = zc + (int64_t)pr.x * KQ, *zb = zc + (int64_t)pr.y * KQ;
#pragma unroll 8
        for (int q = 0; q < KQ; ++q) {
            const double t = za[q] - zb[q];
            g2 = fma(t, t, g2);
        }
        const double sIJ = (double)S[(int64_t)pr.x * nt + pr.y], sJI = (double)S[(int64_t)pr.y * nt + pr.x];
        const double mag = cn[pr.x] + cn[pr.y] + rs + 1.0;
        const double perp =
            sqrt(fmax(0.0, s * (1.0 + 1e-6) - g2 * (1.0 - eta) + 1e-10 * mag * mag)) * (1.0 + 1e-12);
        const double sup = s * (1.0 - 1e-11) - 2.0 * (sIJ + sJI) - 2.0 * perp * rs -
                           1e-9 * (s + 2.0 * (fabs(sIJ) + fabs(sJI))) - 4e-5 * mag * mag;
        l2 = fmax(l2, sup);
    }
    float f = 0.0f;
    if (l2 > 0.0) {
        f = (float)l2;
        if ((double)f > l2) f = nextafterf(f, 0.0f);
    }
    plb[k] = f;
}

// Reach of every tile: the largest R over its points (padding, comp < 0,
// excluded); -inf for a tile without points.  A point's reach is also capped
// by its component's U (comp_ub, recheck scale; an unset U is NaN and caps
// nothing): Boruvka needs only each component's lightest outgoing edge, whose
// recheck value is at most U, and a pair with real distance >= LB has a
// recheck value of at least (1 - rho) LB^2.  pub (pair bounds) and pltau (the
// round that builds lists) are nullable.  One wave per tile.
__global__ __launch_bounds__(256) void k_tile_reach(const float *__restrict__ pbest, const float *__restrict__ pEmax,
                                                    const float *__restrict__ pub, const float *__restrict__ pltau,
                                                    const int32_t *__restrict__ pcomp,
                                                    const uint32_t *__restrict__ comp_ub, int64_t ntiles, float kappa,
                                                    float dn, float *__restrict__ tthr) {
    const int64_t T = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (T >= ntiles) return;
    float m = -SCR_INF;
    for (int q = lane; q < GT; q += 64) {
        const int64_t pos = T * GT + q;
        const int32_t c = pcomp[pos];
        if (c < 0) continue;
        float r = pub ? pub[pos] * kappa : (pbest[pos] + pEmax[pos]) * kappa;
        r = fminf(r, __uint_as_float(comp_ub[c]) * dn);
        if (pltau) {
            const float tau = pltau[pos];
            if (tau >= 0.0f) r = fmaxf(r, (tau + pEmax[pos]) * THR_UP);
        }
        m = fmaxf(m, r);
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) m = fmaxf(m, __shfl_xor(m, o, 64));
    if (lane == 0) tthr[T] = m;
}

// Final round, tile pairs on the device.  k_fr_keep flags the pairs of two
// different components (I < J; tiles hold single components).
__global__ void k_fr_keep(const int2 *__restrict__ pairs, int64_t np, const int32_t *__restrict__ tco,
                          int32_t *__restrict__ flag) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= np) return;
    const int2 pr = pairs[k];
    flag[k] = pr.x < pr.y && tco[pr.x] != tco[pr.y] ? 1 : 0;
}

// Per pair of components, its tile pair of least LB^2 (NaN as +inf; ties to
// the first): the low word of best holds its index.
__global__ void k_fr_best(const int2 *__restrict__ pairs, int64_t np, const int32_t *__restrict__ tco,
                          const float *__restrict__ plb, unsigned long long *__restrict__ best) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool live = k < np;
    int pc = -1;
    unsigned long long key = ~0ull;
    if (live) {
        const int2 pr = pairs[k];
        const float l = plb[k];
        key = ((unsigned long long)__float_as_uint(l == l ? l : SCR_INF) << 32) | (unsigned long long)(uint32_t)k;
        pc = fr_pair(tco[pr.x], tco[pr.y]);
    }
    // consecutive pairs mostly join the same two components: a wave whose
    // live lanes agree takes its minimum first and issues one atomic
    const int pc0 = __shfl(pc, 0, 64);
    if (__all(!live || pc == pc0)) {
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) {
            const unsigned long long ok = __shfl_xor(key, o, 64);
            key = ok < key ? ok : key;
        }
        if ((threadIdx.x & 63) == 0 && pc0 >= 0) atomicMin(&best[pc0], key);
    } else if (live) {
        atomicMin(&best[pc], key);
    }
}

// Phase 1 (B == nullptr): the pairs whose balls meet and each pair of
// components' pair of least LB; phase 2: the others with LB^2 <= B dn, B the
// bottleneck bound of their pair of components.  Counts the point pairs of
// the selected ones (C_PAIRS).
__global__ void k_fr_select(const int2 *__restrict__ pairs, int64_t np, const int32_t *__restrict__ tco,
                            const float *__restrict__ plb, const unsigned long long *__restrict__ best,
                            const float *__restrict__ B, float dn, const int32_t *__restrict__ tcnt,
                            int32_t *__restrict__ flag, int32_t *__restrict__ counters) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    unsigned long long npp = 0;
    if (k < np) {
        const int2 pr = pairs[k];
        const int pc = fr_pair(tco[pr.x], tco[pr.y]);
        const float l = plb[k];
        const bool first = l <= 0.0f || (uint32_t)(best[pc] & 0xFFFFFFFFull) == (uint32_t)k;
        const bool sel = B ? (!first && l <= B[pc] * dn) : first;
        flag[k] = sel ? 1 : 0;
        if (sel) npp = (unsigned long long)tcnt[pr.x] * (unsigned long long)tcnt[pr.y];
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) npp += __shfl_xor(npp, o, 64);
    if ((threadIdx.x & 63) == 0 && npp) atomicAdd(reinterpret_cast<unsigned long long *>(&counters[C_PAIRS]), npp);
}

// Stable compaction of the flagged pairs (pos: exclusive scan of flag).
__global__ void k_flag_scatter(const int2 *__restrict__ pairs, int64_t np, const int32_t *__restrict__ flag,
                               const int32_t *__restrict__ pos, int2 *__restrict__ out) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < np && flag[k]) out[pos[k]] = pairs[k];
}

// ------------------------------------------------------------------ plan

size_t rep_bytes(int32_t precision) {
    return precision == ISO_PREC_BF16 ? 2 : (precision == ISO_PREC_FP8 || precision == ISO_PREC_INT8) ? 1 : 4;
}


struct MstPlan {
    int64_t n, d, ld, n_pad, d_pad, nrb;
    int32_t precision;
    void *Xr;                       // screen representation (FP32, BF16 or FP8), [n_pad][d_pad]
    void *Xq;                       // the tile-pair screen's copy: rows in the tile order, chunk-major per tile
    float *mu, *sq, *rn, *re, *Emax, *best, *ub, *cl, *gcl;
    double *nsum;                   // sums of the norm and representation-error bounds (pair-bound decision)
    int32_t *pgrid, *grid_min, *sqi, *qg;
    float *pmin, *pmax, *cmin, *cmax;
    int2 *pairs, *pairs_r;          // all tile pairs (diagonal first); the pairs kept this round
    int64_t npairs, nt;
    int32_t *perm, *pvals, *tlo, *thi, *keep, *kpos, *keepu, *kposu, *scan_scratch;  // pvals: the final round's sorted ids
    float *psq, *pEmax, *prn, *pre, *pltau, *pbest, *pub;  // the tile-pair screen's per-position copies
    float *trmax, *temax;                                   // and its per-tile largest r and e
    int32_t *pcomp, *psqi;
    uint32_t *pkeys, *ptk, *ptv;
    void *psort;
    double *psum;
    uint32_t *rmax, *emax, *comp_ub;
    int32_t *comp, *ccnt, *cj, *glist, *gcnt, *gcj, *rlist, *rb_j, *cpar, *npar, *flag, *newid, *eu, *ev;
    int32_t *deg, *aoff, *cursor, *adj, *adje, *earc, *tnxt0, *tnxt1, *trk0, *trk1;
    float *ltau, *lv;               // neighbour lists: thresholds, [n][LIST_CAP] values
    int32_t *lscnt, *lj;            // entries offered, [n][LIST_CAP] partners
    uint32_t *ldrop;                // smallest dropped value
    // final round: padded tile order, per (point, component) minima and records
    int32_t *permF, *posF, *tcompF, *fr_pstart, *fr_sstart, *rowj;
    int2 *pairsF, *pairsFA;         // the final round's tile pairs of two components; every tile pair
    int32_t *frk, *frpos;           // its selection flags and their exclusive scan
    unsigned long long *frbest;     // per pair of components: (least LB^2, its tile pair)
    float *frB;                     // per pair of components: the bottleneck bound
    int64_t ntF_cap;
    int32_t options;                // ISO_MST_NO_LISTS / ISO_MST_NO_FINAL / ISO_MST_NO_ESCALATE
    float *bestc;                   // final round: [component][position] minima, ntF_cap * GT positions per row
    double *rowd;
    unsigned long long *W1, *W2;
    uint32_t *upair;
    // tile-pair pruning: tile balls and reach, LB^2 per tile pair, pivots
    bool prune_ok;                  // sizes allow the tile-pair test (see make_plan)
    float *cen, *rad, *tthr, *plb, *pivd;
    int32_t *tcnt, *piv, *piv_rank;
    int2 *pairsF2;                  // the final round's tile pairs of one phase
    double *Q, *z, *zc, *cn;        // final round's support bound: projection, points, tiles
    float *refbuf;                  // the projection's reference centroids and counts, for one copy
    float *S;                       // [ntF_cap][ntF_cap] supports
    float *Dm;                      // [ntb][ntb] squared distances between tile centroids
    double *rb_d2, *elen, *wsum;
    unsigned long long *ck1, *ck2;
    int32_t *counters;

    void carve(Arena &a) {
        const size_t esz = rep_bytes(precision);
        Xr = a.take<char>((size_t)n_pad * d_pad * esz);
        Xq = a.take<char>((size_t)(n_pad + FR_KC * GT) * d_pad * esz);  // room for the final round's padding
        mu = a.take<float>(d_pad);
        psum = a.take<double>((size_t)nrb * d);
        pgrid = a.take<int32_t>((size_t)nrb * d);
        pmin = a.take<float>((size_t)nrb * d);
        pmax = a.take<float>((size_t)nrb * d);
        cmin = a.take<float>(d);
        cmax = a.take<float>(d);
        qg = a.take<int32_t>(1);
        sqi = a.take<int32_t>(n_pad);
        grid_min = a.take<int32_t>(1);
        sq = a.take<float>(n_pad);
        rn = a.take<float>(n_pad);
        re = a.take<float>(n_pad);
        Emax = a.take<float>(n);
        ub = a.take<float>(n);
        nsum = a.take<double>(2);
        best = a.take<float>(n);
        cl = a.take<float>((size_t)n * SCR_CAP);
        rmax = a.take<uint32_t>(1);
        emax = a.take<uint32_t>(1);
        comp_ub = a.take<uint32_t>(n);
        comp = a.take<int32_t>(n_pad);
        ccnt = a.take<int32_t>(n);
        cj = a.take<int32_t>((size_t)n * SCR_CAP);
        glist = a.take<int32_t>(n);
        gcnt = a.take<int32_t>(n);
        rlist = a.take<int32_t>(n);
        rb_j = a.take<int32_t>(n);
        cpar = a.take<int32_t>(n);
        npar = a.take<int32_t>(n);
        flag = a.take<int32_t>(n);
        newid = a.take<int32_t>(n);
        eu = a.take<int32_t>(n);
        ev = a.take<int32_t>(n);
        deg = a.take<int32_t>(n + 1);
        aoff = a.take<int32_t>(n + 1);
        cursor = a.take<int32_t>(n);
        adj = a.take<int32_t>(2 * n);
        adje = a.take<int32_t>(2 * n);
        earc = a.take<int32_t>(2 * n);   // the two arcs of each tree edge
        tnxt0 = a.take<int32_t>(2 * n);  // Euler tour: successor and distance to the end, double-buffered
        tnxt1 = a.take<int32_t>(2 * n);
        trk0 = a.take<int32_t>(2 * n);
        trk1 = a.take<int32_t>(2 * n);
        rb_d2 = a.take<double>(n);
        elen = a.take<double>(n);
        wsum = a.take<double>(1);
        ck1 = a.take<unsigned long long>(n);
        ck2 = a.take<unsigned long long>(n);
        counters = a.take<int32_t>(C_COUNT);
        pairs = a.take<int2>(npairs);
        pairs_r = a.take<int2>(npairs);
        perm = a.take<int32_t>(n_pad);
        pvals = a.take<int32_t>(n);
        pkeys = a.take<uint32_t>(n);
        ptk = a.take<uint32_t>(n);
        ptv = a.take<uint32_t>(n);
        psort = a.take<char>(radix_sort_scratch_bytes(n));
        tlo = a.take<int32_t>(nt);
        thi = a.take<int32_t>(nt);
        keep = a.take<int32_t>(npairs);
        kpos = a.take<int32_t>(npairs + 1);
        keepu = a.take<int32_t>(npairs);
        kposu = a.take<int32_t>(npairs + 1);
        {
            const int64_t npos = std::max<int64_t>(n_pad, ntF_cap * GT);
            psq = a.take<float>(npos);
            pcomp = a.take<int32_t>(npos);
            pEmax = a.take<float>(npos);
            prn = a.take<float>(npos);
            pre = a.take<float>(npos);
            psqi = a.take<int32_t>(npos);
            pltau = a.take<float>(npos);
            pbest = a.take<float>(n_pad);
            pub = a.take<float>(n_pad);
            trmax = a.take<float>(npos / GT);
            temax = a.take<float>(npos / GT);
        }
        scan_scratch = a.take<int32_t>(
            scan_scratch_bytes(std::max<int64_t>(std::max<int64_t>(npairs, n + 1), ntF_cap * (ntF_cap + 1) / 2)) /
            sizeof(int32_t));
        ltau = a.take<float>(n);
        lscnt = a.take<int32_t>(n);
        ldrop = a.take<uint32_t>(n);
        lj = a.take<int32_t>((size_t)n * LIST_CAP);
        lv = a.take<float>((size_t)n * LIST_CAP);
        permF = a.take<int32_t>(n_pad + FR_KC * GT);
        posF = a.take<int32_t>(n);
        tcompF = a.take<int32_t>(ntF_cap);
        fr_pstart = a.take<int32_t>(FR_KC);
        fr_sstart = a.take<int32_t>(FR_KC);
        pairsF = a.take<int2>(ntF_cap * (ntF_cap - 1) / 2);
        pairsFA = a.take<int2>(ntF_cap * (ntF_cap + 1) / 2);
        frk = a.take<int32_t>(ntF_cap * (ntF_cap + 1) / 2);
        frpos = a.take<int32_t>(ntF_cap * (ntF_cap + 1) / 2 + 1);
        frbest = a.take<unsigned long long>(FR_KC * FR_KC);
        frB = a.take<float>(FR_KC * FR_KC);
        bestc = a.take<float>((size_t)FR_KC * ntF_cap * GT);
        rowd = a.take<double>((size_t)n * FR_KC);
        rowj = a.take<int32_t>((size_t)n * FR_KC);
        W1 = a.take<unsigned long long>(FR_KC * FR_KC);
        W2 = a.take<unsigned long long>(FR_KC * FR_KC);
        upair = a.take<uint32_t>(FR_KC * FR_KC);
        if (prune_ok) {
            const int64_t ntb = std::max<int64_t>(nt, ntF_cap);
            const int64_t nfp = ntF_cap * (ntF_cap - 1) / 2;
            cen = a.take<float>((size_t)ntb * (size_t)d);
            rad = a.take<float>(ntb);
            tcnt = a.take<int32_t>(ntb);
            tthr = a.take<float>(ntb);
            plb = a.take<float>(std::max<int64_t>(npairs, nfp));
            pairsF2 = a.take<int2>(nfp);
            piv = a.take<int32_t>(PIV);
            piv_rank = a.take<int32_t>(PIV);
            pivd = a.take<float>(PIV * PIV);
            Q = a.take<double>((size_t)KQ * (size_t)d);
            refbuf = a.take<float>((size_t)(KQ + 1) * (size_t)(d + 1));
            z = a.take<double>((size_t)n * KQ);
            zc = a.take<double>((size_t)ntb * KQ);
            cn = a.take<double>(ntb);
            S = a.take<float>((size_t)ntF_cap * (size_t)ntF_cap);
            Dm = a.take<float>((size_t)ntb * (size_t)ntb);
        }
    }
    // The gathered pass's candidate lists reuse the memory of nothing else:
    // they are sized for all rows (rows are gathered at most once per round).
    size_t gather_bytes() const { return (size_t)n * SCR_CAP2 * (sizeof(int32_t) + sizeof(float)); }
};

MstPlan make_plan(int64_t n, int64_t d, int64_t ld, int32_t precision) {
    MstPlan p{};
    p.n = n;
    p.d = d;
    p.ld = ld;
    p.precision = precision;
    p.n_pad = (n / GT + 1) * GT;  // at least one padding row (the final round pads with it)
    const int64_t kc = 64 / (int64_t)rep_bytes(precision);  // 64-byte K chunks
    p.d_pad = (d + kc - 1) / kc * kc;
    p.nrb = (n + COL_RB - 1) / COL_RB;
    p.nt = p.n_pad / pair_tile();
    p.npairs = p.nt * (p.nt + 1) / 2;
    p.ntF_cap = (n + pair_tile() - 1) / pair_tile() + FR_KC;
    p.prune_ok = p.nt >= PRUNE_MIN_TILES && d <= PRUNE_MAX_D && p.ntF_cap <= PRUNE_MAX_TILES;
    return p;
}

size_t plan_bytes(MstPlan p) {
    Arena a;
    p.carve(a);
    a.take<char>(p.gather_bytes());
    return a.used;
}

// A screen whose error bound is too loose for the data (every row's candidates
// overflow, and rows fall through to the exact O(n d) rescan) is abandoned:
// run_mst sets *escalate and returns, and the caller starts again with the
// FP32 screen, whose representation is exact.  Thresholds: more than a
// quarter of the points in the gathered pass, or more than 64 + n/64 rescans.
constexpr double ESCALATE_GATHER = 0.25, ESCALATE_RESCAN = 1.0 / 64.0;
constexpr double PB_RATIO = 4.0;  // separable / typical bound above which BF16 uses pair bounds

// A second stream for the pruning's work that reads only X (the points'
// nearest pivots, their projection z = Q x, the FP64 edge lengths), so that it
// overlaps the main stream's work; events order it after its inputs and before
// its consumers.  Non-blocking, default priority.  Creating and destroying a
// stream per call costs more than the work it overlaps, so the streams (with
// their events) are kept per device for the life of the process: a call takes
// one from its device's pool (a new one when the pool is empty) and gives it
// back at the end, after making the main stream wait for everything queued on
// it (the workspace it writes may be reused once the main stream moves on).
// On an error the stream is synchronised and destroyed instead.
constexpr size_t PIN_BYTES = size_t(2) << 20;  // pinned staging of small device-to-host reads

struct AuxSet {
    hipStream_t s = nullptr;
    hipEvent_t ev0 = nullptr, ev_key = nullptr, ev_z = nullptr, ev_len = nullptr, ev_end = nullptr;
    char *pin = nullptr;
};

struct AuxPool {
    std::mutex mu;
    std::vector<std::pair<int, AuxSet>> free;  // (device, set)
};
AuxPool &aux_pool() {
    static AuxPool *p = new AuxPool();  // never destroyed: the streams live until the process ends
    return *p;
}

struct AuxStream {
    hipStream_t s = nullptr;
    hipEvent_t ev0 = nullptr, ev_key = nullptr, ev_z = nullptr, ev_len = nullptr, ev_end = nullptr;
    char *pin = nullptr;
    hipStream_t main = nullptr;
    int dev = -1;
    int uncaught = 0;
    void start(hipStream_t main_stream) {
        main = main_stream;
        uncaught = std::uncaught_exceptions();
        HIP_CHECK(hipGetDevice(&dev));
        AuxSet a;
        {
            std::lock_guard<std::mutex> lock(aux_pool().mu);
            auto &fl = aux_pool().free;
            for (size_t i = 0; i < fl.size(); ++i)
                if (fl[i].first == dev) {
                    a = fl[i].second;
                    fl.erase(fl.begin() + (std::ptrdiff_t)i);
                    break;
                }
        }
        if (!a.s) {
            HIP_CHECK(hipStreamCreateWithFlags(&a.s, hipStreamNonBlocking));
            s = a.s;  // (released by the destructor if what follows fails)
            for (hipEvent_t *e : {&a.ev0, &a.ev_key, &a.ev_z, &a.ev_len, &a.ev_end})
                HIP_CHECK(hipEventCreateWithFlags(e, hipEventDisableTiming));
            HIP_CHECK(hipHostMalloc(reinterpret_cast<void **>(&a.pin), PIN_BYTES, hipHostMallocDefault));
        }
        s = a.s;
        pin = a.pin;
        ev0 = a.ev0;
        ev_key = a.ev_key;
        ev_z = a.ev_z;
        ev_len = a.ev_len;
        ev_end = a.ev_end;
    }
    // work queued on s from now on runs after the main stream's work so far
    void after(hipStream_t m) {
        HIP_CHECK(hipEventRecord(ev0, m));
        HIP_CHECK(hipStreamWaitEvent(s, ev0, 0));
    }
    ~AuxStream() {
        if (!s) return;
        const bool ok = std::uncaught_exceptions() == uncaught && hipEventRecord(ev_end, s) == hipSuccess &&
                        hipStreamWaitEvent(main, ev_end, 0) == hipSuccess;
        if (ok) {
            std::lock_guard<std::mutex> lock(aux_pool().mu);
            aux_pool().free.push_back({dev, AuxSet{s, ev0, ev_key, ev_z, ev_len, ev_end, pin}});
            return;
        }
        (void)hipStreamSynchronize(s);
        (void)hipStreamSynchronize(main);
        (void)hipStreamDestroy(s);
        for (hipEvent_t e : {ev0, ev_key, ev_z, ev_len, ev_end})
            if (e) (void)hipEventDestroy(e);
        if (pin) (void)hipHostFree(pin);
    }
};

// Small device-to-host reads staged through the pinned buffer: a copy to
// pageable memory waits for the stream by itself, so several of them cost
// several waits; staged, they queue behind the kernels and share the one
// synchronisation, after which sync() moves them to their destinations.
// A read too large for the buffer is a direct copy.
struct HostReads {
    char *pin = nullptr;
    size_t used = 0;
    struct Pending {
        void *dst;
        size_t off, bytes;
    };
    std::vector<Pending> pend;
    void get(void *dst, const void *src, size_t bytes, hipStream_t s) {
        if (!pin || used + bytes > PIN_BYTES) {
            HIP_CHECK(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, s));
            return;
        }
        HIP_CHECK(hipMemcpyAsync(pin + used, src, bytes, hipMemcpyDeviceToHost, s));
        pend.push_back({dst, used, bytes});
        used += (bytes + 15) & ~size_t(15);
    }
    void sync(hipStream_t s) {
        HIP_CHECK(hipStreamSynchronize(s));
        for (const Pending &q : pend) std::memcpy(q.dst, pin + q.off, q.bytes);
        pend.clear();
        used = 0;
    }
};

void run_mst(MstPlan &P, Arena &arena, const float *X, int32_t recheck, int32_t *parent, double *length,
             iso_mst_info *info, hipStream_t s, bool *escalate) {
    const int64_t n = P.n, d = P.d, ld = P.ld;
    const bool timed = timing().enabled != 0;
    const int32_t rep = P.precision;
    const bool f64 = recheck == ISO_RECHECK_FP64;
    EventPair whole(timed), scr(timed);
    whole.start(s);
    *escalate = false;
    const bool may_escalate = rep != ISO_PREC_FP32 && !(P.options & ISO_MST_NO_ESCALATE);
    const bool prune = !(P.options & ISO_MST_NO_PRUNE) && P.prune_ok;
    int64_t tp_run = 0, tp_full = 0;  // tile pairs screened, and those full screens would have run
    auto give_up = [&]() {
        whole.stop(s);
        if (timed) timing().mst_ms += whole.elapsed_ms();
        *escalate = true;
    };
    // gathered-pass lists: [n][SCR_CAP2] of j and of lower bounds
    char *gbuf = arena.take<char>(P.gather_bytes());
    P.gcj = reinterpret_cast<int32_t *>(gbuf);
    P.gcl = reinterpret_cast<float *>(gbuf + (size_t)n * SCR_CAP2 * sizeof(int32_t));

    fill<int32_t>(P.counters, 0, C_COUNT, s);
    // The pruned first round orders the points by their nearest pivot (rows
    // q n / PIV); that assignment reads only X and runs on the second stream
    // while the main stream computes the representation.
    AuxStream aux;
    aux.start(s);
    HostReads R;
    R.pin = aux.pin;
    std::vector<int32_t> h_piv(PIV), h_rank(PIV, -1);
    if (prune) {
        for (int q = 0; q < PIV; ++q) h_piv[q] = (int32_t)((int64_t)q * n / PIV);
        HIP_CHECK(hipMemcpyAsync(P.piv, h_piv.data(), sizeof(int32_t) * PIV, hipMemcpyHostToDevice, s));
        aux.after(s);
        hipLaunchKernelGGL(k_pivot_near, dim3((unsigned)((n + 127) / 128)), dim3(256), 0, aux.s, X, d, ld,
                           static_cast<const int32_t *>(nullptr), n, P.piv, P.pkeys, static_cast<float *>(nullptr));
        LAUNCH_CHECK();
        HIP_CHECK(hipEventRecord(aux.ev_key, aux.s));
    }
    fill<uint32_t>(P.rmax, 0u, 1, s);
    fill<uint32_t>(P.emax, 0u, 1, s);
    fill<int32_t>(P.grid_min, GRID_NONE, 1, s);
    hipLaunchKernelGGL(k_colstats_partial, dim3((unsigned)P.nrb, (unsigned)((d + 255) / 256)), dim3(256), 0, s, X, n, d,
                       ld, P.psum, P.pgrid, P.pmin, P.pmax, P.counters);
    LAUNCH_CHECK();
    int32_t h_nonfinite = 0;
    R.get(&h_nonfinite, P.counters + C_NONFINITE, sizeof(int32_t), s);
    R.sync(s);
    ISO_REQUIRE(h_nonfinite == 0, ISO_ERR_NONFINITE, "points contain a NaN or infinite coordinate");
    float inv_step = 1.0f;  // INT8: 2^-qg
    int32_t h_qg = GRID_NONE;
    if (rep == ISO_PREC_INT8) {
        ISO_REQUIRE(d < 16384, ISO_ERR_INVALID_ARG, "the INT8 screen needs d < 16384 (d = %lld)", (long long)d);
        fill<int32_t>(P.qg, GRID_NONE, 1, s);
        hipLaunchKernelGGL(k_colrange_i8, dim3(grid_for(d, 256)), dim3(256), 0, s, P.pgrid, P.pmin, P.pmax, P.nrb, d,
                           P.cmin, P.cmax, P.qg);
        LAUNCH_CHECK();
        hipLaunchKernelGGL(k_center_i8, dim3(grid_for(P.d_pad, 256)), dim3(256), 0, s, P.cmin, P.cmax, d, P.d_pad, P.qg,
                           P.mu, P.counters);
        LAUNCH_CHECK();
        int32_t hb[2] = {0, 0};
        R.get(&hb[0], P.counters + C_I8BAD, sizeof(int32_t), s);
        R.get(&h_qg, P.qg, sizeof(int32_t), s);
        R.sync(s);
        ISO_REQUIRE(hb[0] == 0, ISO_ERR_INVALID_ARG,
                    "the INT8 screen needs 8-bit data: every coordinate on one binary grid 2^q with each column "
                    "spanning at most 255 steps");
        if (h_qg != GRID_NONE) inv_step = (float)std::ldexp(1.0, -h_qg);
    } else {
        hipLaunchKernelGGL(k_colstats_final, dim3(grid_for(P.d_pad, 4)), dim3(256), 0, s, P.psum, P.pgrid, P.nrb, n,
                           d, P.d_pad, P.mu);
        LAUNCH_CHECK();
    }
    {
        auto kern = rep == ISO_PREC_BF16   ? k_repr_rows<ISO_PREC_BF16>
                    : rep == ISO_PREC_FP8  ? k_repr_rows<ISO_PREC_FP8>
                    : rep == ISO_PREC_INT8 ? k_repr_rows<ISO_PREC_INT8>
                                           : k_repr_rows<ISO_PREC_FP32>;
        const unsigned g = std::min<unsigned>(grid_for(P.n_pad, 4), 8u * (unsigned)device_cus());
        hipLaunchKernelGGL(kern, dim3(g), dim3(256), 0, s, X, n, d, ld, P.n_pad, P.d_pad, P.mu, P.Xr, P.sq, P.rn, P.re,
                           P.rmax, P.emax, P.grid_min, P.sqi, inv_step);
    }
    LAUNCH_CHECK();
    const double u = 1.0 / 8388608.0;  // 2^-23
    const double du = (double)(d + 4) * u;
    ScreenBound bound{};
    bound.g = (float)(du / (1.0 - du) * (1.0 + 1.0 / 1024.0));
    // Exact-accumulation certificate: when every screen value is a multiple of
    // 2^q, products are multiples of 2^2q, and a pair whose norms are at most
    // R = 2^(11.5 + q) has every partial sum of its dot product and of both
    // squared norms below 2^(23 + 2q) in magnitude, so all of them are exact in
    // FP32; only fl(s_i + s_j) and the final fused multiply-add round, which
    // costs at most 3.01 u (r_i + r_j)^2.
    int32_t h_grid = GRID_NONE;
    R.get(&h_grid, P.grid_min, sizeof(int32_t), s);
    R.sync(s);
    bound.g_exact = (float)(4.0 * u);
    bound.rlim = (h_grid != GRID_NONE && h_grid > -120)
                     ? (float)(std::sqrt(2.0) * std::ldexp(1.0, h_grid + 11) * (1.0 - 0x1p-20))
                     : 0.0f;
    // recheck order vs real D^2: relative error <= rho = gamma_{d+2} at the
    // recheck's unit roundoff (2^-24 FP32, 2^-53 FP64)
    const double ur = f64 ? 0x1p-53 : 0x1p-24;
    const double rho = (double)(d + 2) * ur / (1.0 - (double)(d + 2) * ur);
    if (rep == ISO_PREC_INT8) {
        // exact integer Gram and norms: the only rounding is the conversion of
        // the exact integer Dhat^2 to FP32 (the power-of-two scale is exact)
        bound.g = bound.g_exact = (float)(2.0 * u * (1.0 + 1.0 / 1024.0));
        bound.rlim = 0.0f;
    }
    const float kappa = (float)((1.0 + rho) / (1.0 - rho) * (1.0 + 0x1p-20));
    const float up = (float)((1.0 + rho) * (1.0 + 0x1p-20));
    const float dn = (float)(1.0 / (1.0 - rho) * (1.0 + 0x1p-20));
    hipLaunchKernelGGL(k_row_bound, dim3(grid_for(n, 256)), dim3(256), 0, s, P.rn, P.re, n, bound, P.rmax, P.emax,
                       P.Emax);
    LAUNCH_CHECK();
    // Pair bounds (BF16): when the separable bound of a typical row against
    // the largest norm and representation error, pair_bound(r_mean, r_max,
    // e_mean, e_max), exceeds PB_RATIO times the bound of two typical rows, the
    // thresholds use each pair's own bound (heavy-tailed norms); the flag
    // ISO_MST_PAIR_BOUNDS forces them.
    bool pb = false;
    if (rep == ISO_PREC_BF16) {
        fill<double>(P.nsum, 0.0, 2, s);
        hipLaunchKernelGGL(k_norm_sums, dim3(std::min<unsigned>(grid_for(n, 256), 1024u)), dim3(256), 0, s, P.rn,
                           P.re, n, P.nsum);
        LAUNCH_CHECK();
        double hs[2] = {0.0, 0.0};
        uint32_t hm[2] = {0u, 0u};
        R.get(hs, P.nsum, sizeof(hs), s);
        R.get(&hm[0], P.rmax, sizeof(uint32_t), s);
        R.get(&hm[1], P.emax, sizeof(uint32_t), s);
        R.sync(s);
        float rmx, emx;
        std::memcpy(&rmx, &hm[0], sizeof(float));
        std::memcpy(&emx, &hm[1], sizeof(float));
        const double rm = hs[0] / (double)n, em = hs[1] / (double)n, g = bound.g;
        auto pbound = [&](double ri, double rj, double ei, double ej) {
            return g * (ri + rj) * (ri + rj) + (ei + ej) * (2.0 * (ri + rj) + ei + ej);
        };
        const double typ = pbound(rm, rm, em, em), sep = pbound(rm, rmx, em, emx);
        pb = (P.options & ISO_MST_PAIR_BOUNDS) != 0 || (typ > 0.0 && sep > PB_RATIO * typ);
    }
    float *const ubp = pb ? P.ub : nullptr;
    hipLaunchKernelGGL(k_iota_comp, dim3(grid_for(P.n_pad, 256)), dim3(256), 0, s, P.comp, n, P.n_pad);
    LAUNCH_CHECK();

    ScreenArgs SA{};
    SA.rep = rep;
    SA.XT = rep == ISO_PREC_FP32 ? static_cast<const float *>(P.Xr) : nullptr;
    SA.XB = rep == ISO_PREC_BF16 ? static_cast<const uint16_t *>(P.Xr) : nullptr;
    SA.XF8 = rep == ISO_PREC_FP8 ? static_cast<const uint8_t *>(P.Xr) : nullptr;
    SA.XI8 = rep == ISO_PREC_INT8 ? static_cast<const int8_t *>(P.Xr) : nullptr;
    SA.sqi = P.sqi;
    SA.scale2 = (rep == ISO_PREC_INT8 && h_qg != GRID_NONE) ? (float)std::ldexp(1.0, 2 * h_qg) : 1.0f;
    SA.n = n;
    SA.n_pad = P.n_pad;
    SA.d_pad = P.d_pad;
    SA.d = d;
    SA.sq = P.sq;
    SA.rn = P.rn;
    SA.re = P.re;
    SA.Emax = P.Emax;
    SA.comp = P.comp;
    SA.bound = bound;
    SA.kappa = kappa;
    SA.best = P.best;
    SA.ccnt = P.ccnt;
    SA.cj = P.cj;
    SA.cl = P.cl;
    SA.best_in = P.best;
    SA.rows = P.glist;
    SA.gcnt = P.gcnt;
    SA.gcj = P.gcj;
    SA.gcl = P.gcl;
    auto screen = [&](bool gather) { launch_screen_rows(SA, gather, s); };
    ISO_REQUIRE(P.n_pad / pair_tile() == P.nt && P.npairs == P.nt * (P.nt + 1) / 2, ISO_ERR_INTERNAL,
                "tile-pair order of %lld tiles", (long long)P.nt);
    launch_pair_order(P.nt, P.pairs, s, prune);
    hipLaunchKernelGGL(k_perm_identity, dim3(grid_for(P.n_pad, 256)), dim3(256), 0, s, P.perm, P.n_pad);
    LAUNCH_CHECK();
    if (prune) {
        // The first round's order: the points by their nearest pivot, the
        // pivots in a nearest-neighbour chain from the first; component labels
        // follow the order.  (The pivots' own distances: keys into the sort's
        // spare keys, which the assignment on the second stream does not touch.)
        hipLaunchKernelGGL(k_pivot_near, dim3(1), dim3(256), 0, s, X, d, ld, P.piv, (int64_t)PIV, P.piv, P.ptk,
                           P.pivd);
        LAUNCH_CHECK();
        std::vector<float> pd((size_t)PIV * PIV);
        R.get(pd.data(), P.pivd, sizeof(float) * pd.size(), s);
        R.sync(s);
        int cur = 0;
        h_rank[0] = 0;
        for (int q = 1; q < PIV; ++q) {
            int nx = -1;
            for (int c = 0; c < PIV; ++c)
                if (h_rank[c] < 0 && (nx < 0 || pd[(size_t)cur * PIV + c] < pd[(size_t)cur * PIV + nx])) nx = c;
            h_rank[nx] = q;
            cur = nx;
        }
        HIP_CHECK(hipMemcpyAsync(P.piv_rank, h_rank.data(), sizeof(int32_t) * PIV, hipMemcpyHostToDevice, s));
        HIP_CHECK(hipStreamWaitEvent(s, aux.ev_key, 0));  // every point's nearest pivot
        hipLaunchKernelGGL(k_pivot_keys, dim3(grid_for(n, 256)), dim3(256), 0, s, P.pkeys, P.piv_rank, n, P.perm);
        LAUNCH_CHECK();
        radix_sort_pairs_u32(P.pkeys, reinterpret_cast<uint32_t *>(P.perm), P.ptk, P.ptv, n, 5, P.psort, s);
        hipLaunchKernelGGL(k_comp_from_order, dim3(grid_for(n, 256)), dim3(256), 0, s, P.perm, n, P.comp);
        LAUNCH_CHECK();
    }
    // The tile-pair screen reads its own copy of the representation (Xq), in
    // the tile order and chunk-major within each tile (the final round
    // overwrites it with its own order; every later plain round copies it again).
    const int64_t row_u4 = (int64_t)(P.d_pad * rep_bytes(rep) / 16);
    auto tile_copy = [&](const int32_t *order, int64_t npos) {
        const int64_t nchunks = row_u4 / 4;
        ISO_REQUIRE(npos % GT == 0 && row_u4 % 4 == 0 && npos / GT * nchunks <= (int64_t)UINT32_MAX, ISO_ERR_INTERNAL,
                    "tile copy of %lld rows", (long long)npos);
        hipLaunchKernelGGL(rep == ISO_PREC_BF16 ? k_permute_rows_frag : k_permute_rows,
                           dim3((unsigned)(npos / GT * nchunks)), dim3(256), 0, s, static_cast<const uint4 *>(P.Xr),
                           order, nchunks, row_u4, static_cast<uint4 *>(P.Xq));
        LAUNCH_CHECK();
    };
    tile_copy(P.perm, P.n_pad);
    SA.perm = P.perm;
    SA.Xtile = P.Xq;

    int64_t ncomp = n;
    int rounds = 0, list_rounds = 0, final_components = 0;
    // (the neighbour lists and the final round decide with the separable
    // bound, which pair-bound data makes useless: every round is screened)
    enum { LISTS_NONE, LISTS_BUILDING, LISTS_READY, LISTS_OFF } lists =
        ((P.options & ISO_MST_NO_LISTS) || pb) ? LISTS_OFF : LISTS_NONE;
    bool final_off = (P.options & ISO_MST_NO_FINAL) != 0 || pb;
    SA.ub = ubp;
    SA.psq = P.psq;
    SA.pcomp = P.pcomp;
    SA.pEmax = P.pEmax;
    SA.prn = P.prn;
    SA.pre = P.pre;
    SA.psqi = P.psqi;
    SA.pltau = P.pltau;
    SA.pbest = P.pbest;
    SA.pub = ubp ? P.pub : nullptr;
    SA.trmax = P.trmax;
    SA.temax = P.temax;
    // the tile-pair screen's per-position copies and per-tile maxima for the
    // tile order `order` (npos positions, a whole number of tiles)
    auto pos_gather = [&](const int32_t *order, int64_t npos, bool with_ltau) {
        hipLaunchKernelGGL(k_pos_gather, dim3(grid_for(npos, 256)), dim3(256), 0, s, order, npos, n, P.sq, P.comp,
                           P.Emax, P.rn, P.re, rep == ISO_PREC_INT8 ? P.sqi : nullptr, with_ltau ? P.ltau : nullptr,
                           P.psq, P.pcomp, P.pEmax, P.prn, P.pre, P.psqi, P.pltau);
        LAUNCH_CHECK();
        const int64_t ntiles = npos / GT;
        hipLaunchKernelGGL(k_tile_max, dim3(grid_for(ntiles * 64, 256)), dim3(256), 0, s, P.prn, P.pre, ntiles, (int)GT,
                           P.trmax, P.temax);
        LAUNCH_CHECK();
    };

    // Tile balls of the order (ntiles tiles) and LB^2 of the tile pairs `pairs`.
    // Tile balls of the order (ntiles tiles) and LB^2 of the tile pairs
    // `pairs`; with `support` the support bound as well (the projection Q and
    // the points' z = Q x are made at its first use, from the centroids of
    // KQ + 1 tiles spread over the order).
    bool have_q = false;
    double h_eta = 0.0;
    std::vector<float> h_ref;    // reference centroids, KQ + 1 rows of d
    std::vector<int32_t> h_refc;  // and their tiles' row counts
    // the centroids of KQ + 1 tiles spread over the current order (P.cen)
    auto fetch_ref = [&](int64_t ntiles) {
        // gathered on the device first: one copy instead of two per reference
        // (each copy to pageable memory waits for the stream)
        const int nref = KQ + 1;
        int32_t *cnt_dev = reinterpret_cast<int32_t *>(P.refbuf + (size_t)nref * d);
        hipLaunchKernelGGL(k_ref_gather, dim3(nref), dim3(256), 0, s, P.cen, P.tcnt, ntiles, d, nref, P.refbuf,
                           cnt_dev);
        LAUNCH_CHECK();
        std::vector<float> hb((size_t)nref * (d + 1));
        R.get(hb.data(), P.refbuf, sizeof(float) * hb.size(), s);
        R.sync(s);
        h_ref.assign(hb.begin(), hb.begin() + (size_t)nref * d);
        h_refc.assign(nref, 0);
        std::memcpy(h_refc.data(), hb.data() + (size_t)nref * d, sizeof(int32_t) * nref);
    };
    // Q by Gram-Schmidt (twice) in FP64 of the differences of the reference
    // centroids to the first (directions that vanish stay zero rows), eta, and
    // z = Q x of every point (queued on the stream)
    std::vector<double> hq;  // (the source of Q's copy: lives as long as the call)
    auto build_q = [&]() {
        const int nref = KQ + 1;
        hq.assign((size_t)KQ * d, 0.0);
        std::vector<double> v(d);
        std::vector<int> live;
        for (int q = 1; q < nref && h_refc[0] > 0; ++q) {
            if (h_refc[q] == 0) continue;
            double n0 = 0.0;
            for (int64_t k = 0; k < d; ++k) {
                v[k] = (double)h_ref[(size_t)q * d + k] - (double)h_ref[k];
                n0 += v[k] * v[k];
            }
            for (int pass = 0; pass < 2; ++pass)
                for (int j : live) {
                    const double *qj = hq.data() + (size_t)j * d;
                    double t = 0.0;
                    for (int64_t k = 0; k < d; ++k) t += qj[k] * v[k];
                    for (int64_t k = 0; k < d; ++k) v[k] -= t * qj[k];
                }
            double nv = 0.0;
            for (int64_t k = 0; k < d; ++k) nv += v[k] * v[k];
            if (!(nv > 1e-16 * n0) || !(nv > 0.0)) continue;
            const int row = (int)live.size();
            const double inv = 1.0 / std::sqrt(nv);
            for (int64_t k = 0; k < d; ++k) hq[(size_t)row * d + k] = v[k] * inv;
            live.push_back(row);
        }
        // eta >= ||Q Q' - I|| over the nonzero rows (bounded by KQ times the largest entry)
        double emax = 0.0;
        for (int i : live)
            for (int j : live) {
                if (j < i) continue;
                double t = 0.0;
                for (int64_t k = 0; k < d; ++k) t += hq[(size_t)i * d + k] * hq[(size_t)j * d + k];
                emax = std::max(emax, std::fabs(t - (i == j ? 1.0 : 0.0)));
            }
        h_eta = (double)KQ * emax * 2.0 + 1e-13;
        HIP_CHECK(hipMemcpyAsync(P.Q, hq.data(), sizeof(double) * hq.size(), hipMemcpyHostToDevice, s));
        // z on the second stream (it reads X and Q only); the supports wait for it
        aux.after(s);
        hipLaunchKernelGGL(k_project, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, aux.s, X, n, d, ld, P.Q, P.z);
        LAUNCH_CHECK();
        HIP_CHECK(hipEventRecord(aux.ev_z, aux.s));
        have_q = true;
    };
    auto tile_bounds = [&](const int32_t *order, int64_t ntiles, const int2 *pairs, int64_t npr, bool support) {
        hipLaunchKernelGGL(k_tile_centroid, dim3((unsigned)ntiles, (unsigned)((d + 255) / 256)), dim3(256), 0, s, X, n,
                           d, ld, order, P.cen, P.tcnt);
        LAUNCH_CHECK();
        fill<float>(P.rad, 0.0f, ntiles, s);
        hipLaunchKernelGGL(k_tile_radius, dim3((unsigned)ntiles, 4), dim3(256), (size_t)d * sizeof(float), s, X, n, d,
                           ld, order, P.cen, P.tcnt, P.rad);
        LAUNCH_CHECK();
        support = support && ntiles <= P.ntF_cap;
        if (support && !have_q) {
            fetch_ref(ntiles);
            build_q();
        }
        if (support) {
            hipLaunchKernelGGL(k_tile_project, dim3((unsigned)ntiles), dim3(256), 0, s, P.cen, P.tcnt, d, P.Q, P.zc,
                               P.cn);
            LAUNCH_CHECK();
            HIP_CHECK(hipStreamWaitEvent(s, aux.ev_z, 0));
            hipLaunchKernelGGL(k_tile_support, dim3((unsigned)ntiles), dim3(256), 0, s, order, n, P.z, P.zc, P.tcnt,
                               ntiles, P.S);
            LAUNCH_CHECK();
        }
        if (npr > 0) {
            const unsigned tb = (unsigned)((ntiles + 31) / 32);
            hipLaunchKernelGGL(k_tile_dist, dim3(tb, tb), dim3(256), 0, s, P.cen, ntiles, d, P.Dm);
            LAUNCH_CHECK();
            hipLaunchKernelGGL(k_pair_lb, dim3(grid_for(npr, 256)), dim3(256), 0, s, pairs, npr, P.Dm, P.rad, P.tcnt,
                               d, support ? P.S : nullptr, P.zc, P.cn, ntiles, h_eta, P.plb);
            LAUNCH_CHECK();
        }
    };
    // The plain rounds' tile pairs of one phase (0: every pair that is not
    // inside one component; 1, 2: the pruned phases) into pairs_r, masked ones
    // first: returns (masked, unmasked) counts.
    auto compact = [&](int phase, bool diag_all) -> std::pair<int64_t, int64_t> {
        hipLaunchKernelGGL(k_pair_keep, dim3(grid_for(P.npairs, 256)), dim3(256), 0, s, P.pairs, P.npairs, P.tlo,
                           P.thi, P.plb, P.tthr, P.tcnt, phase, diag_all ? 1 : 0, P.keep, P.keepu, P.counters);
        LAUNCH_CHECK();
        exclusive_scan_i32(P.keep, P.kpos, P.npairs, P.kpos + P.npairs, P.scan_scratch, s);
        exclusive_scan_i32(P.keepu, P.kposu, P.npairs, P.kposu + P.npairs, P.scan_scratch, s);
        hipLaunchKernelGGL(k_pair_scatter, dim3(grid_for(P.npairs, 256)), dim3(256), 0, s, P.pairs, P.npairs, P.keep,
                           P.kpos, P.keepu, P.kposu, P.pairs_r);
        LAUNCH_CHECK();
        int32_t hk[2] = {0, 0};
        R.get(&hk[0], P.kpos + P.npairs, sizeof(int32_t), s);
        R.get(&hk[1], P.kposu + P.npairs, sizeof(int32_t), s);
        R.sync(s);
        ISO_REQUIRE(hk[0] >= 0 && hk[1] >= 0 && hk[0] + hk[1] <= P.npairs, ISO_ERR_INTERNAL, "tile-pair compaction");
        return {(int64_t)hk[0], (int64_t)hk[1]};
    };
    EventPair scr2(timed);

    // The final round (at most FR_KC components left): true when it joined
    // them all, false when a point's candidate list overflowed (the round is
    // then screened the plain way).
    auto final_round = [&]() -> bool {
        const int K = (int)ncomp;
        const int64_t bstride = P.ntF_cap * GT;  // positions per component row of bestc
        // component sizes -> padded tile order (host: at most FR_KC components)
        fill<int32_t>(P.flag, 0, K, s);
        histogram_i32(P.comp, n, K, P.flag, s);
        std::vector<int32_t> hs(K), pst(K), sst(K), tco;
        R.get(hs.data(), P.flag, sizeof(int32_t) * K, s);
        R.sync(s);
        int64_t pos = 0, srt = 0;
        for (int c = 0; c < K; ++c) {
            sst[c] = (int32_t)srt;
            pst[c] = (int32_t)pos;
            srt += hs[c];
            const int64_t tiles = (hs[c] + GT - 1) / GT;
            for (int64_t t = 0; t < tiles; ++t) tco.push_back(c);
            pos += tiles * GT;
        }
        const int64_t ntF = (int64_t)tco.size();
        ISO_REQUIRE(srt == n && ntF <= P.ntF_cap, ISO_ERR_INTERNAL, "final-round tile order (%lld points, %lld tiles)",
                    (long long)srt, (long long)ntF);
        HIP_CHECK(hipMemcpyAsync(P.fr_pstart, pst.data(), sizeof(int32_t) * K, hipMemcpyHostToDevice, s));
        HIP_CHECK(hipMemcpyAsync(P.fr_sstart, sst.data(), sizeof(int32_t) * K, hipMemcpyHostToDevice, s));
        HIP_CHECK(hipMemcpyAsync(P.tcompF, tco.data(), sizeof(int32_t) * ntF, hipMemcpyHostToDevice, s));
        // flagged tile pairs of `pairs` (np) into out, in order; returns their count
        auto fr_compact = [&](const int2 *pairs, int64_t np, int2 *out) -> int64_t {
            exclusive_scan_i32(P.frk, P.frpos, np, P.frpos + np, P.scan_scratch, s);
            hipLaunchKernelGGL(k_flag_scatter, dim3(grid_for(np, 256)), dim3(256), 0, s, pairs, np, P.frk, P.frpos,
                               out);
            LAUNCH_CHECK();
            int32_t c = 0;
            R.get(&c, P.frpos + np, sizeof(int32_t), s);
            R.sync(s);
            ISO_REQUIRE(c >= 0 && c <= np, ISO_ERR_INTERNAL, "final-round tile-pair compaction");
            return c;
        };
        // the tile pairs of two different components, in the tile-pair order
        const int64_t nall = ntF * (ntF + 1) / 2;
        launch_pair_order(ntF, P.pairsFA, s, prune);
        hipLaunchKernelGGL(k_fr_keep, dim3(grid_for(nall, 256)), dim3(256), 0, s, P.pairsFA, nall, P.tcompF, P.frk);
        LAUNCH_CHECK();
        const int64_t nF = fr_compact(P.pairsFA, nall, P.pairsF);
        // points sorted by component, then placed at their padded positions
        // (padding positions hold the padding row n_pad - 1: +inf distances)
        int kb = 1;
        while ((int64_t(1) << kb) < K) ++kb;
        // (sorted into pvals: perm keeps the plain rounds' order in case this round falls back)
        hipLaunchKernelGGL(k_perm_keys, dim3(grid_for(n, 256)), dim3(256), 0, s, P.comp, n, P.pkeys, P.pvals);
        LAUNCH_CHECK();
        radix_sort_pairs_u32(P.pkeys, reinterpret_cast<uint32_t *>(P.pvals), P.ptk, P.ptv, n, kb, P.psort, s);
        fill<int32_t>(P.permF, (int32_t)(P.n_pad - 1), ntF * GT, s);
        hipLaunchKernelGGL(k_fr_perm, dim3(grid_for(n, 256)), dim3(256), 0, s, P.pvals, P.comp, n, P.fr_pstart,
                           P.fr_sstart, P.permF, P.posF);
        LAUNCH_CHECK();
        tile_copy(P.permF, ntF * GT);
        pos_gather(P.permF, ntF * GT, false);
        ScreenArgs FA = SA;
        FA.perm = P.permF;
        FA.Xtile = P.Xq;
        FA.bestc = P.bestc;
        FA.bestc_stride = bstride;
        FA.tcomp = P.tcompF;
        FA.upair = P.upair;
        FA.up = up;
        FA.dn = dn;
        FA.lcnt = nullptr;
        FA.rows = nullptr;
        FA.nrows = 0;
        fill<uint32_t>(reinterpret_cast<uint32_t *>(P.bestc), 0x7F800000u, (int64_t)K * bstride, s);
        fill<uint32_t>(P.upair, 0x7F800000u, FR_KC * FR_KC, s);
        fill<int32_t>(P.ccnt, 0, n, s);
        const bool fr_pruned = prune && nF > 0;
        if (fr_pruned) {
            // Pruned per pair of components (a, b): the first phase screens the
            // tile pairs whose balls meet and, for every pair of components,
            // its tile pair of least LB, which gives every U(a, b); B(a, b) =
            // the least over paths from a to b of the largest U on the path
            // (U closed under the bottleneck path).  An edge of the contracted
            // MST between a and b weighs at most B(a, b) (it is the lightest
            // bottleneck link), so a tile pair with (1 - rho) LB^2 > B(a, b)
            // holds none; the second phase screens the others.  The recheck
            // then gives every MST edge exactly, and every other pair of
            // components at most a heavier edge, which Kruskal leaves out.
            tile_bounds(P.permF, ntF, P.pairsF, nF, true);
            fill<unsigned long long>(P.frbest, U64_MAX, FR_KC * FR_KC, s);
            hipLaunchKernelGGL(k_fr_best, dim3(grid_for(nF, 256)), dim3(256), 0, s, P.pairsF, nF, P.tcompF, P.plb,
                               P.frbest);
            LAUNCH_CHECK();
            hipLaunchKernelGGL(k_fr_select, dim3(grid_for(nF, 256)), dim3(256), 0, s, P.pairsF, nF, P.tcompF, P.plb,
                               P.frbest, static_cast<const float *>(nullptr), dn, P.tcnt, P.frk, P.counters);
            LAUNCH_CHECK();
            const int64_t n1 = fr_compact(P.pairsF, nF, P.pairsF2);
            scr.start(s);
            launch_screen_pairs(FA, P.pairsF2, 0, n1, s);
            scr.stop(s);
            std::vector<uint32_t> hu(FR_KC * FR_KC);
            R.get(hu.data(), P.upair, sizeof(uint32_t) * hu.size(), s);
            R.sync(s);
            std::vector<float> B((size_t)K * K), hb(FR_KC * FR_KC, 0.0f);
            for (int a = 0; a < K; ++a)
                for (int b = 0; b < K; ++b) {
                    float u = 0.0f;
                    if (a != b) std::memcpy(&u, &hu[fr_pair(a, b)], sizeof(float));
                    B[(size_t)a * K + b] = u;
                }
            for (int m = 0; m < K; ++m)
                for (int a = 0; a < K; ++a) {
                    const float bam = B[(size_t)a * K + m];
                    float *row = B.data() + (size_t)a * K;
                    const float *rm = B.data() + (size_t)m * K;
                    for (int b = 0; b < K; ++b) row[b] = std::min(row[b], std::max(bam, rm[b]));
                }
            for (int a = 0; a < K; ++a)
                for (int b = a + 1; b < K; ++b) hb[fr_pair(a, b)] = B[(size_t)a * K + b];
            HIP_CHECK(hipMemcpyAsync(P.frB, hb.data(), sizeof(float) * hb.size(), hipMemcpyHostToDevice, s));
            hipLaunchKernelGGL(k_fr_select, dim3(grid_for(nF, 256)), dim3(256), 0, s, P.pairsF, nF, P.tcompF, P.plb,
                               P.frbest, P.frB, dn, P.tcnt, P.frk, P.counters);
            LAUNCH_CHECK();
            const int64_t n2 = fr_compact(P.pairsF, nF, P.pairsF2);  // (synchronises: hb has been read)
            scr2.start(s);
            launch_screen_pairs(FA, P.pairsF2, 0, n2, s);
            scr2.stop(s);
            tp_run += n1 + n2;
            tp_full += nF;
        } else {
            scr.start(s);
            launch_screen_pairs(FA, P.pairsF, 0, nF, s);
            scr.stop(s);
            tp_run += nF;
            tp_full += nF;
        }
        // the recheck runs only when its work is modest: no overflowed list
        // and at most FR_EVAL_PER_POINT candidates per point on average (with
        // a loose screen bound, e.g. FP8 at large d, the plain rounds are cheaper)
        {
            int32_t hc[C_COUNT];
            fill<int32_t>(P.counters + C_OVF, 0, 1, s);
            fill<int32_t>(P.counters + C_FRWORK, 0, 2, s);
            hipLaunchKernelGGL(k_fr_count, dim3(row_grid(n)), dim3(256), 0, s, n, P.comp, P.Emax, P.bestc, P.posF,
                               bstride, P.upair, P.ccnt, P.gcj, P.gcl, kappa, dn, P.counters);
            LAUNCH_CHECK();
            R.get(hc, P.counters, sizeof(hc), s);
            R.sync(s);
            unsigned long long work = 0;
            memcpy(&work, &hc[C_FRWORK], sizeof(work));
            if (timed) {
                unsigned long long sumsq = 0;
                memcpy(&sumsq, &hc[C_SUMSQ], sizeof(sumsq));
                iso_timing &T = timing();
                T.screen_launches += 1;
                T.screen_ms += scr.elapsed_ms() + (fr_pruned ? scr2.elapsed_ms() : 0.0);
                if (!prune) T.screen_pairs += 0.5 * ((double)n * (double)n - (double)sumsq);
                T.screen_dim = (double)P.d_pad;
            }
            if (hc[C_OVF] > 0 || (double)work > FR_EVAL_PER_POINT * (double)n) return false;
        }
        fill<unsigned long long>(P.W1, U64_MAX, FR_KC * FR_KC, s);
        fill<unsigned long long>(P.W2, U64_MAX, FR_KC * FR_KC, s);
        if (f64)
            hipLaunchKernelGGL(k_fr_recheck<true>, dim3(row_grid(n)), dim3(256), 0, s, X, n, d, ld, P.comp, P.Emax,
                               P.bestc, P.posF, bstride, P.upair, P.ccnt, P.gcj, P.gcl, kappa, dn, P.rowd, P.rowj,
                               P.W1, P.counters);
        else
            hipLaunchKernelGGL(k_fr_recheck<false>, dim3(row_grid(n)), dim3(256), 0, s, X, n, d, ld, P.comp,
                               P.Emax, P.bestc, P.posF, bstride, P.upair, P.ccnt, P.gcj, P.gcl, kappa, dn, P.rowd,
                               P.rowj, P.W1, P.counters);
        LAUNCH_CHECK();
        hipLaunchKernelGGL(k_fr_pick, dim3(grid_for(n * FR_KC, 256)), dim3(256), 0, s, P.rowd, P.rowj, P.comp, n,
                           P.W1, P.W2);
        LAUNCH_CHECK();
        std::vector<unsigned long long> w1(FR_KC * FR_KC), w2(FR_KC * FR_KC);
        int32_t h[C_COUNT];
        R.get(w1.data(), P.W1, sizeof(unsigned long long) * w1.size(), s);
        R.get(w2.data(), P.W2, sizeof(unsigned long long) * w2.size(), s);
        R.get(h, P.counters, sizeof(h), s);
        R.sync(s);
        // Kruskal over the components' lightest edges, ordered by (D^2, ids)
        struct CE {
            unsigned long long d2, ids;
            int a, b;
        };
        std::vector<CE> ce;
        for (int a = 0; a < K; ++a)
            for (int b = a + 1; b < K; ++b)
                if (w2[a * FR_KC + b] != U64_MAX) ce.push_back({w1[a * FR_KC + b], w2[a * FR_KC + b], a, b});
        std::sort(ce.begin(), ce.end(),
                  [](const CE &x, const CE &y) { return x.d2 != y.d2 ? x.d2 < y.d2 : x.ids < y.ids; });
        std::vector<int> uf(K);
        for (int c = 0; c < K; ++c) uf[c] = c;
        auto root = [&](int c) {
            while (uf[c] != c) c = uf[c] = uf[uf[c]];
            return c;
        };
        std::vector<int32_t> nu, nv;
        for (const CE &e : ce) {
            const int ra = root(e.a), rb = root(e.b);
            if (ra == rb) continue;
            uf[ra] = rb;
            nu.push_back((int32_t)(e.ids >> 32));
            nv.push_back((int32_t)(e.ids & 0xFFFFFFFFu));
        }
        ISO_REQUIRE((int)nu.size() == K - 1, ISO_ERR_INTERNAL, "final round joined %zu of %d components", nu.size() + 1,
                    K);
        const int32_t off = h[C_EDGES];
        ISO_REQUIRE(off >= 0 && (int64_t)off + K - 1 <= n - 1, ISO_ERR_INTERNAL, "final round edge count");
        HIP_CHECK(hipMemcpyAsync(P.eu + off, nu.data(), sizeof(int32_t) * nu.size(), hipMemcpyHostToDevice, s));
        HIP_CHECK(hipMemcpyAsync(P.ev + off, nv.data(), sizeof(int32_t) * nv.size(), hipMemcpyHostToDevice, s));
        const int32_t total = off + K - 1;
        HIP_CHECK(hipMemcpyAsync(P.counters + C_EDGES, &total, sizeof(int32_t), hipMemcpyHostToDevice, s));
        R.sync(s);
        final_components = K;
        return true;
    };

    while (ncomp > 1) {
        ++rounds;
        ISO_REQUIRE(rounds <= 64, ISO_ERR_INTERNAL, "Boruvka did not converge");
        if (timed) {
            fill<int32_t>(P.flag, 0, ncomp, s);
            histogram_i32(P.comp, n, ncomp, P.flag, s);
            hipLaunchKernelGGL(k_sum_squares, dim3(1), dim3(1024), 0, s, P.flag, ncomp, P.counters);
            LAUNCH_CHECK();
        }
        if (!final_off && ncomp <= FR_KC && rounds >= 2) {
            if (final_round()) {
                ncomp = 1;
                break;
            }
            final_off = true;  // a candidate list overflowed: this and later rounds screen the plain way
        }
        // From the third round on, rows are first decided by their neighbour
        // lists; the round screens only when too many rows stay undecided.
        bool list_round = false;
        if (lists == LISTS_READY) {
            hipLaunchKernelGGL(k_list_best, dim3(row_grid(n)), dim3(256), 0, s, n, P.comp, P.lscnt, P.lj, P.lv,
                               P.best);
            LAUNCH_CHECK();
            fill<uint32_t>(P.comp_ub, U32_MAX, ncomp, s);
            hipLaunchKernelGGL(k_comp_ub, dim3(grid_for(P.n_pad, 256)), dim3(256), 0, s, P.perm, P.n_pad, P.best,
                               P.Emax, ubp, P.comp, n, up, P.comp_ub);
            LAUNCH_CHECK();
            fill<int32_t>(P.counters + C_FORCE, 0, 1, s);
            hipLaunchKernelGGL(k_list_capture, dim3(row_grid(n)), dim3(256), 0, s, n, P.comp, P.comp_ub, P.best,
                               P.Emax, P.rn, P.re, bound, P.ltau, P.lscnt, P.ldrop, P.lj, P.lv, kappa, dn, P.ccnt, P.cj,
                               P.cl, P.counters);
            LAUNCH_CHECK();
            int32_t h_force = 0;
            R.get(&h_force, P.counters + C_FORCE, sizeof(int32_t), s);
            R.sync(s);
            // an undecided row costs a row sweep over all points, a screen
            // round about half of one per row: lists pay below ~1/6 undecided
            if ((double)h_force <= 0.15 * (double)n) {
                list_round = true;
                ++list_rounds;
            } else {
                lists = LISTS_OFF;  // components only grow: later rounds would fare worse
            }
        }
        if (!list_round) {
            // Tile order and tile pairs of this round.  The screen masks pairs
            // of one component only in its first nmask tile pairs: in the first
            // round (identity order, every point its own component) those are
            // the diagonal pairs; from the second round on the points are
            // ordered by component, tile pairs lying inside one component are
            // dropped, and the diagonal pairs and those whose tiles share a
            // component go first.
            const int2 *pairs_use = P.pairs;
            int64_t nmask = P.nt, noff = P.npairs - P.nt;
            if (rounds > 1) {
                int kb = 1;
                while ((int64_t(1) << kb) < ncomp) ++kb;
                hipLaunchKernelGGL(k_perm_keys, dim3(grid_for(n, 256)), dim3(256), 0, s, P.comp, n, P.pkeys, P.perm);
                LAUNCH_CHECK();
                radix_sort_pairs_u32(P.pkeys, reinterpret_cast<uint32_t *>(P.perm), P.ptk, P.ptv, n, kb, P.psort, s);
                tile_copy(P.perm, P.n_pad);
            }
            if (rounds > 1 || prune) {
                hipLaunchKernelGGL(k_tile_ranges, dim3(grid_for(P.nt, 256)), dim3(256), 0, s, P.perm, P.comp, n, P.nt,
                                   pair_tile(), P.tlo, P.thi);
                LAUNCH_CHECK();
                if (prune) {
                    tile_bounds(P.perm, P.nt, P.pairs, P.npairs, false);
                    fill<int32_t>(P.counters + C_TPFULL, 0, 1, s);
                }
                std::tie(nmask, noff) = compact(prune ? 1 : 0, rounds == 1);
                pairs_use = P.pairs_r;
            }
            // the final round's projection is built from this order's tiles
            // while the first phase of this round's screen runs
            const bool want_q = prune && !have_q && !final_off;
            if (want_q) fetch_ref(P.nt);
            tp_run += nmask + noff;
            if (!prune) tp_full += nmask + noff;  // (pruned rounds: C_TPFULL, read with the round's counters)
            if (lists == LISTS_NONE && rounds == 2) {
                // the second round's screen builds the lists from the first
                // round's minima (still in best)
                hipLaunchKernelGGL(k_list_init, dim3(grid_for(n, 256)), dim3(256), 0, s, P.best, n, P.ltau, P.lscnt,
                                   P.ldrop);
                LAUNCH_CHECK();
                SA.ltau = P.ltau;
                SA.lcnt = P.lscnt;
                SA.ldrop = P.ldrop;
                SA.lj = P.lj;
                SA.lv = P.lv;
                lists = LISTS_BUILDING;
            }
            pos_gather(P.perm, P.n_pad, SA.lcnt != nullptr);
            fill<uint32_t>(reinterpret_cast<uint32_t *>(P.pbest), 0x7F800000u, P.n_pad, s);  // +inf
            if (ubp) fill<uint32_t>(reinterpret_cast<uint32_t *>(P.pub), 0x7F800000u, P.n_pad, s);
            fill<int32_t>(P.ccnt, 0, n, s);
            SA.rows = nullptr;
            SA.nrows = 0;
            scr.start(s);
            launch_screen_pairs(SA, pairs_use, nmask, noff, s);
            scr.stop(s);
            if (want_q) build_q();
            if (prune) {
                // the second phase: the reach of every tile from the minima so
                // far, then the pairs whose bound does not exclude them
                hipLaunchKernelGGL(k_pos_scatter, dim3(grid_for(P.n_pad, 256)), dim3(256), 0, s, P.perm, P.n_pad, n,
                                   P.pbest, P.best);
                LAUNCH_CHECK();
                if (ubp) {
                    hipLaunchKernelGGL(k_pos_scatter, dim3(grid_for(P.n_pad, 256)), dim3(256), 0, s, P.perm, P.n_pad,
                                       n, P.pub, ubp);
                    LAUNCH_CHECK();
                }
                fill<uint32_t>(P.comp_ub, U32_MAX, ncomp, s);
                hipLaunchKernelGGL(k_comp_ub, dim3(grid_for(P.n_pad, 256)), dim3(256), 0, s, P.perm, P.n_pad, P.best,
                                   P.Emax, ubp, P.comp, n, up, P.comp_ub);
                LAUNCH_CHECK();
                hipLaunchKernelGGL(k_tile_reach, dim3(grid_for(P.nt, 4)), dim3(256), 0, s, P.pbest, P.pEmax,
                                   ubp ? P.pub : nullptr, SA.lcnt ? P.pltau : nullptr, P.pcomp, P.comp_ub, P.nt,
                                   kappa, dn, P.tthr);
                LAUNCH_CHECK();
                const std::pair<int64_t, int64_t> c2 = compact(2, rounds == 1);
                tp_run += c2.first + c2.second;
                scr2.start(s);
                launch_screen_pairs(SA, P.pairs_r, c2.first, c2.second, s);
                scr2.stop(s);
            }
            hipLaunchKernelGGL(k_pos_scatter, dim3(grid_for(P.n_pad, 256)), dim3(256), 0, s, P.perm, P.n_pad, n, P.pbest,
                               P.best);
            LAUNCH_CHECK();
            if (ubp) {
                hipLaunchKernelGGL(k_pos_scatter, dim3(grid_for(P.n_pad, 256)), dim3(256), 0, s, P.perm, P.n_pad, n,
                                   P.pub, ubp);
                LAUNCH_CHECK();
            }
            if (lists == LISTS_BUILDING) {
                SA.lcnt = nullptr;
                lists = LISTS_READY;
            }
            fill<uint32_t>(P.comp_ub, U32_MAX, ncomp, s);
            hipLaunchKernelGGL(k_comp_ub, dim3(grid_for(P.n_pad, 256)), dim3(256), 0, s, P.perm, P.n_pad, P.best,
                               P.Emax, ubp, P.comp, n, up, P.comp_ub);
            LAUNCH_CHECK();
        }
        fill<int32_t>(P.counters + C_OVF, 0, 1, s);
        fill<int32_t>(P.counters + C_GATHER, 0, 1, s);
        if (f64)
            hipLaunchKernelGGL(k_recheck_rows<true>, dim3(row_grid(n)), dim3(256), 0, s, X, n, d, ld, P.best, P.Emax,
                               ubp, P.comp, P.comp_ub, P.ccnt, P.cj, P.cl, kappa, dn, P.rb_d2, P.rb_j, P.glist,
                               P.counters);
        else
            hipLaunchKernelGGL(k_recheck_rows<false>, dim3(row_grid(n)), dim3(256), 0, s, X, n, d, ld, P.best,
                               P.Emax, ubp, P.comp, P.comp_ub, P.ccnt, P.cj, P.cl, kappa, dn, P.rb_d2, P.rb_j, P.glist,
                               P.counters);
        LAUNCH_CHECK();
        int32_t h_gather = 0;
        R.get(&h_gather, P.counters + C_GATHER, sizeof(int32_t), s);
        R.sync(s);
        if (timed && !list_round) {
            iso_timing &T = timing();
            T.screen_launches += 1;
            T.screen_ms += scr.elapsed_ms() + (prune ? scr2.elapsed_ms() : 0.0);
        }
        // (with pair bounds an overflowing list reflects the loose early
        // thresholds of the screen, not a loose bound: the gathered pass settles
        // such rows, and only rows that overflow it again count)
        if (may_escalate && !pb && (double)h_gather > ESCALATE_GATHER * (double)n) {
            give_up();
            return;
        }
        if (h_gather > 0) {
            SA.rows = P.glist;
            SA.nrows = h_gather;
            fill<int32_t>(P.gcnt, 0, h_gather, s);
            screen(true);
            if (list_round) {
                // the gathered rows' minima are now exact: a tighter U
                fill<uint32_t>(P.comp_ub, U32_MAX, ncomp, s);
                hipLaunchKernelGGL(k_comp_ub, dim3(grid_for(P.n_pad, 256)), dim3(256), 0, s, P.perm, P.n_pad, P.best,
                                   P.Emax, ubp, P.comp, n, up, P.comp_ub);
                LAUNCH_CHECK();
            }
            if (f64)
                hipLaunchKernelGGL(k_recheck_gather<true>, dim3(grid_for(h_gather, 4)), dim3(256), 0, s, X, d, ld,
                                   P.best, P.Emax, ubp, P.comp, P.comp_ub, P.glist, h_gather, P.gcnt, P.gcj, P.gcl, kappa,
                                   dn, P.rb_d2, P.rb_j, P.rlist, P.counters);
            else
                hipLaunchKernelGGL(k_recheck_gather<false>, dim3(grid_for(h_gather, 4)), dim3(256), 0, s, X, d, ld,
                                   P.best, P.Emax, ubp, P.comp, P.comp_ub, P.glist, h_gather, P.gcnt, P.gcj, P.gcl, kappa,
                                   dn, P.rb_d2, P.rb_j, P.rlist, P.counters);
            LAUNCH_CHECK();
            if (may_escalate) {
                int32_t h_ovf = 0;
                R.get(&h_ovf, P.counters + C_OVF, sizeof(int32_t), s);
                R.sync(s);
                if ((double)h_ovf > 64.0 + ESCALATE_RESCAN * (double)n) {
                    give_up();
                    return;
                }
            }
            if (f64)
                hipLaunchKernelGGL(k_rescan<true>, dim3(1024), dim3(256), 0, s, X, n, d, ld, P.comp, P.rlist, P.counters,
                                   P.rb_d2, P.rb_j);
            else
                hipLaunchKernelGGL(k_rescan<false>, dim3(1024), dim3(256), 0, s, X, n, d, ld, P.comp, P.rlist,
                                   P.counters, P.rb_d2, P.rb_j);
            LAUNCH_CHECK();
        }
        fill<unsigned long long>(P.ck1, U64_MAX, ncomp, s);
        fill<unsigned long long>(P.ck2, U64_MAX, ncomp, s);
        hipLaunchKernelGGL(k_comp_min1, dim3(grid_for(n, 256)), dim3(256), 0, s, P.rb_d2, P.rb_j, P.comp, n, P.ck1);
        LAUNCH_CHECK();
        hipLaunchKernelGGL(k_comp_min2, dim3(grid_for(n, 256)), dim3(256), 0, s, P.rb_d2, P.rb_j, P.comp, n, P.ck1,
                           P.ck2);
        LAUNCH_CHECK();
        hipLaunchKernelGGL(k_hook1, dim3(grid_for(ncomp, 256)), dim3(256), 0, s, P.ck2, P.comp, ncomp, P.cpar,
                           P.counters);
        LAUNCH_CHECK();
        hipLaunchKernelGGL(k_hook2, dim3(grid_for(ncomp, 256)), dim3(256), 0, s, P.ck2, P.cpar, ncomp, P.npar, P.eu,
                           P.ev, n - 1, P.counters);
        LAUNCH_CHECK();
        for (int it = 0; it <= ceil_log2(ncomp); ++it) {
            hipLaunchKernelGGL(k_jump, dim3(grid_for(ncomp, 256)), dim3(256), 0, s, P.npar, ncomp);
            LAUNCH_CHECK();
        }
        hipLaunchKernelGGL(k_isroot, dim3(grid_for(ncomp, 256)), dim3(256), 0, s, P.npar, ncomp, P.flag);
        LAUNCH_CHECK();
        exclusive_scan_i32(P.flag, P.newid, ncomp, P.counters + C_NCOMP, P.scan_scratch, s);
        hipLaunchKernelGGL(k_relabel, dim3(grid_for(n, 256)), dim3(256), 0, s, P.comp, n, P.npar, P.newid);
        LAUNCH_CHECK();
        int32_t h[C_COUNT];
        R.get(h, P.counters, sizeof(h), s);
        R.sync(s);
        ISO_REQUIRE(h[C_NOEDGE] == 0, ISO_ERR_INTERNAL, "a component found no outgoing edge in round %d", rounds);
        if (prune && !list_round) tp_full += h[C_TPFULL];
        ISO_REQUIRE(h[C_NCOMP] >= 1 && h[C_NCOMP] < ncomp, ISO_ERR_INTERNAL,
                    "Boruvka round %d did not contract (%lld -> %d components)", rounds, (long long)ncomp, h[C_NCOMP]);
        if (timed && !list_round && !prune) {
            unsigned long long sumsq = 0;
            memcpy(&sumsq, &h[C_SUMSQ], sizeof(sumsq));
            iso_timing &T = timing();
            T.screen_pairs += 0.5 * ((double)n * (double)n - (double)sumsq);
            T.screen_dim = (double)P.d_pad;
        }
        ncomp = h[C_NCOMP];
    }

    if (timed && prune) {
        unsigned long long pp = 0;
        R.get(&pp, P.counters + C_PAIRS, sizeof(pp), s);
        R.sync(s);
        timing().screen_pairs += (double)pp;
        timing().screen_dim = (double)P.d_pad;
    }
    const int64_t m = n - 1;
    int32_t h_edges = 0;
    R.get(&h_edges, P.counters + C_EDGES, sizeof(int32_t), s);
    R.sync(s);
    ISO_REQUIRE(h_edges == m, ISO_ERR_INTERNAL, "MST has %d edges, expected %lld", h_edges, (long long)m);

    // The FP64 lengths read only X and the edge list, and the rooting needs
    // them only for its last step: with the second stream started they run
    // there, beside the rooting's small latency-bound launches.
    if (aux.s) aux.after(s);
    hipLaunchKernelGGL(k_refine, dim3(grid_for(m, 256)), dim3(256), 0, aux.s ? aux.s : s, X, d, ld, P.eu, P.ev, m,
                       P.elen);
    LAUNCH_CHECK();
    if (aux.s) HIP_CHECK(hipEventRecord(aux.ev_len, aux.s));
    fill<int32_t>(P.deg, 0, n + 1, s);
    hipLaunchKernelGGL(k_degree, dim3(grid_for(m, 256)), dim3(256), 0, s, P.eu, P.ev, m, P.deg);
    LAUNCH_CHECK();
    exclusive_scan_i32(P.deg, P.aoff, n + 1, nullptr, P.scan_scratch, s);
    fill<int32_t>(P.cursor, 0, n, s);
    hipLaunchKernelGGL(k_fill_adj, dim3(grid_for(m, 256)), dim3(256), 0, s, P.eu, P.ev, m, P.aoff, P.cursor, P.adj,
                       P.adje, P.earc);
    LAUNCH_CHECK();
    // rooting: Euler tour, pointer jumping, orientation
    const int64_t narcs = 2 * m;
    hipLaunchKernelGGL(k_tour_succ, dim3(grid_for(narcs, 256)), dim3(256), 0, s, P.aoff, P.adj, P.adje, P.earc, narcs,
                       P.tnxt0, P.trk0);
    LAUNCH_CHECK();
    int32_t *tn = P.tnxt0, *tr = P.trk0, *tn2 = P.tnxt1, *tr2 = P.trk1;
    for (int64_t span = 1; span < narcs; span *= 2) {
        hipLaunchKernelGGL(k_tour_jump, dim3(grid_for(narcs, 256)), dim3(256), 0, s, tn, tr, narcs, tn2, tr2);
        LAUNCH_CHECK();
        std::swap(tn, tn2);
        std::swap(tr, tr2);
    }
    if (aux.s) HIP_CHECK(hipStreamWaitEvent(s, aux.ev_len, 0));  // the lengths
    hipLaunchKernelGGL(k_tour_orient, dim3(grid_for(m, 256)), dim3(256), 0, s, P.eu, P.ev, P.earc, tr, P.elen, m,
                       parent, length);
    LAUNCH_CHECK();
    // the tour from the root covers every arc exactly when the edges form one tree
    int32_t h_tour[2] = {0, 0};
    R.get(&h_tour[0], tr, sizeof(int32_t), s);
    R.get(&h_tour[1], P.aoff + 1, sizeof(int32_t), s);
    hipLaunchKernelGGL(k_sum_lengths, dim3(1), dim3(1024), 0, s, length, n, P.wsum);
    LAUNCH_CHECK();
    R.sync(s);
    ISO_REQUIRE(h_tour[1] > 0 && (int64_t)h_tour[0] == narcs, ISO_ERR_INTERNAL,
                "the rooting tour covers %d of %lld arcs (root degree %d)", h_tour[0], (long long)narcs, h_tour[1]);
    whole.stop(s);
    if (timed) {
        timing().mst_calls += 1;
        timing().mst_ms += whole.elapsed_ms();
    }
    if (info) {
        long long cand = 0, resc = 0;
        R.get(&cand, P.counters + C_CAND, sizeof(cand), s);
        R.get(&resc, P.counters + C_RESCAN, sizeof(resc), s);
        R.get(&info->mst_weight, P.wsum, sizeof(double), s);
        R.sync(s);
        info->rounds = rounds;
        info->list_rounds = list_rounds;
        info->final_components = final_components;
        info->screen_precision = rep;
        info->pair_bounds = pb ? 1 : 0;
        info->candidates = cand;
        info->rescanned_rows = resc;
        info->tile_pairs = tp_run;
        info->tile_pairs_full = tp_full;
    }
}

}  // namespace

}  // namespace iso

using namespace iso;

extern "C" iso_status iso_mst_workspace_size(int64_t n, int64_t d, int32_t precision, size_t *bytes) {
    return guarded([&] {
        ISO_REQUIRE(bytes != nullptr, ISO_ERR_INVALID_ARG, "bytes is NULL");
        ISO_REQUIRE(n >= 2 && n < (int64_t(1) << 31) - GT, ISO_ERR_INVALID_ARG, "n = %lld outside [2, 2^31)", (long long)n);
        ISO_REQUIRE(d >= 1, ISO_ERR_INVALID_ARG, "d = %lld < 1", (long long)d);
        ISO_REQUIRE(precision == ISO_PREC_FP32 || precision == ISO_PREC_BF16 || precision == ISO_PREC_FP8 ||
                        precision == ISO_PREC_INT8,
                    ISO_ERR_INVALID_ARG, "unknown precision %d", precision);
        // room for the FP32 screen too (a screen whose bound is too loose escalates to it)
        *bytes = std::max(plan_bytes(make_plan(n, d, d, precision)), plan_bytes(make_plan(n, d, d, ISO_PREC_FP32)));
    });
}

extern "C" iso_status iso_mst(const float *X, int64_t n, int64_t d, int64_t ld, int32_t precision, int32_t recheck,
                              uint32_t flags, int32_t *parent, double *length, iso_mst_info *info, void *ws,
                              size_t ws_bytes, void *stream) {
    return guarded([&] {
        ISO_REQUIRE(X && parent && length, ISO_ERR_INVALID_ARG, "X, parent and length must be non-NULL");
        ISO_REQUIRE(n >= 2 && n < (int64_t(1) << 31) - GT, ISO_ERR_INVALID_ARG, "n = %lld outside [2, 2^31)", (long long)n);
        ISO_REQUIRE(d >= 1, ISO_ERR_INVALID_ARG, "d = %lld < 1", (long long)d);
        ISO_REQUIRE(ld >= d, ISO_ERR_INVALID_ARG, "ld = %lld < d = %lld", (long long)ld, (long long)d);
        ISO_REQUIRE(precision == ISO_PREC_FP32 || precision == ISO_PREC_BF16 || precision == ISO_PREC_FP8 ||
                        precision == ISO_PREC_INT8,
                    ISO_ERR_INVALID_ARG, "unknown precision %d", precision);
        ISO_REQUIRE(recheck == ISO_RECHECK_FP32 || recheck == ISO_RECHECK_FP64, ISO_ERR_INVALID_ARG,
                    "unknown recheck %d", recheck);
        ISO_REQUIRE((flags & ~(uint32_t)(ISO_MST_NO_LISTS | ISO_MST_NO_FINAL | ISO_MST_NO_ESCALATE |
                                          ISO_MST_PAIR_BOUNDS | ISO_MST_NO_PRUNE)) == 0,
                    ISO_ERR_INVALID_ARG, "unknown flag bits 0x%x", flags);
        const int32_t options = (int32_t)flags;
        require_device();
        hipStream_t s = static_cast<hipStream_t>(stream);
        MstPlan P = make_plan(n, d, ld, precision);
        P.options = options;
        const size_t need = std::max(plan_bytes(P), plan_bytes(make_plan(n, d, ld, ISO_PREC_FP32)));
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
        bool escalate = false;
        run_mst(P, a, X, recheck, parent, length, info, s, &escalate);
        if (escalate) {
            MstPlan P32 = make_plan(n, d, ld, ISO_PREC_FP32);
            P32.options = options;
            Arena a32{static_cast<char *>(ws), 0, ws_bytes};
            P32.carve(a32);
            run_mst(P32, a32, X, recheck, parent, length, info, s, &escalate);
            ISO_REQUIRE(!escalate, ISO_ERR_INTERNAL, "the FP32 screen cannot escalate");
        }
    });
}

extern "C" const char *iso_last_error(void) { return iso::get_error(); }

extern "C" const char *iso_version(void) { return "isoclust 0.1 (gfx950)"; }
