// screen.hpp -- shared pieces of the Boruvka screen kernels (FP32, BF16 and
// FP8 MFMA): the error bound of the Gram-form distance, and the epilogue that
// keeps a running minimum per row and captures every column that can still be
// the row's lightest outgoing edge.
//
// Representation: x'_i = rep(x_i - mu) with mu a per-coordinate centre (exact
// translation invariance of distances), rep = FP32, BF16 or FP8 E4M3 rounding.
// The screen forms Dhat^2_ij = fl(s_i + s_j - 2 G_ij), s_i = fl(||x'_i||^2),
// G_ij the FP32-accumulated dot product, clamped at 0.  With r_i >= ||x'_i||,
// e_i >= ||x'_i - (x_i - mu)|| and g = gamma_{d+4} (unit roundoff 2^-23, so the
// bound holds for any faithful rounding and any accumulation order):
//   |Dhat^2_ij - D^2_ij| <= E_ij = g (r_i + r_j)^2 + (e_i + e_j)(2 (r_i + r_j) + e_i + e_j).
// (The first term bounds the norms' and the dot product's rounding, using
//  s_i + s_j + 2 r_i r_j = (r_i + r_j)^2; the second the representation error
//  through |D - D'| <= e_i + e_j and D' <= r_i + r_j.)
// Emax_i = E with j's terms replaced by their maxima bounds E_ij for all j.
//
// A column j of row i is a candidate when its lower bound
//   L_ij = Dhat^2_ij - E_ij  <=  kappa (b_i + Emax_i),
// b_i the running minimum of Dhat^2 over the row; b_i only decreases, so a
// column that is never captured can never be the row's lightest edge.  The
// edges are ordered by the exact recheck value O(i,j), which differs from the
// real D^2 by at most rho D^2 (rho = gamma_{d+2} at the recheck's unit
// roundoff); kappa = (1 + rho) / (1 - rho) (1 + 2^-20) makes the capture hold
// every column whose O can reach the row's minimum O.
#pragma once

#include <vector>

#include "common.hpp"

namespace iso {

constexpr int SCR_ROWS = 128;    // rows per workgroup
constexpr int SCR_COLS = 128;    // columns per tile
constexpr int SCR_CAP = 32;      // candidate slots per row in the sweep (LDS)
constexpr int SCR_CAP2 = 512;    // candidate slots per row in the gathered pass (global)
constexpr int SCR_FORCE = SCR_CAP + 2;  // ccnt marker: the row must be screened in the gathered pass
constexpr int LIST_CAP = 128;    // neighbour-list slots per point
constexpr int FR_KC = 64;        // final round: most components it joins at once
constexpr float SCR_INF = __builtin_huge_valf();
constexpr float THR_UP = 1.0f + 1.0f / 1048576.0f;  // covers the rounding of a sum of two nonnegative terms

// Constants of the error bound: g = gamma_{d+4}; pairs whose norm bounds are
// both <= rlim are certified exactly accumulated (see the exact-accumulation
// certificate in mst.hip) and use g_exact instead.
struct ScreenBound {
    float g;
    float g_exact;
    float rlim;
};

struct ScreenArgs {
    int32_t rep;             // ISO_PREC_FP32 / ISO_PREC_BF16 / ISO_PREC_FP8 / ISO_PREC_INT8
    const float *XT;         // FP32 screen: [n_pad][d_pad] centred, row-major
    const uint16_t *XB;      // BF16 screen: [n_pad][d_pad] centred, row-major (bf16 bits)
    const uint8_t *XF8;      // FP8 screen: [n_pad][d_pad] centred, row-major (E4M3 bytes)
    const int8_t *XI8;       // INT8 screen: [n_pad][d_pad] (x - mu) / 2^q as integers, row-major
    const int32_t *sqi;      // INT8 screen: [n_pad] exact ||(x - mu) / 2^q||^2, 2^30 on padding
    float scale2;            // INT8 screen: 2^2q, the unit of the integer distances
    int64_t n, n_pad, d_pad;
    int64_t d;               // coordinates that may be nonzero (the rest of d_pad is zero padding)
    const float *sq;         // [n_pad] fl(||x'||^2) as used in Dhat^2 (0 on padding)
    const float *rn;         // [n_pad] r_i
    const float *re;         // [n_pad] e_i
    const float *Emax;       // [n]
    const int32_t *comp;     // [n_pad] component of each point, -1 on padding
    const int32_t *perm;     // tile-pair screen: [n_pad] point at each position of the tile order
                             // (points sorted by component, padding last)
    const void *Xtile;       // tile-pair screen: the representation, rows in the tile order, stored tile by
                             // tile and chunk-major within a tile (the PT rows' bytes 64 c .. 64 c + 63 contiguous)
    // tile-pair screen: per-position copies, in the tile order A.perm, of the
    // per-point values it reads (gathered once per order, so that a work item's
    // loads are coalesced and none waits for a point id): s, component, Emax
    // (0 on padding), r and e (pair bounds), the exact integer squared norms
    // (INT8) and the list thresholds (lists); and the running minima by
    // position (plain and list rounds: +inf on entry, folded into best[] by the
    // caller afterwards; the pair bounds' ub likewise)
    const float *psq;
    const int32_t *pcomp;
    const float *pEmax, *prn, *pre;
    const int32_t *psqi;
    const float *pltau;
    float *pbest, *pub;
    const float *trmax, *temax;  // tile-pair screen: per tile of the order, the largest r and e of its points
    ScreenBound bound;       // error bound constants
    float kappa;             // capture threshold scale (recheck order slack and rounding)
    // gathered pass (rows == nullptr for the full sweep)
    const int32_t *rows;     // [nrows] row of each gathered slot
    int32_t nrows;
    const float *best_in;    // [n] running minimum from the sweep
    int32_t *gcnt;           // [nrows] candidates per slot (> SCR_CAP2 = overflow); zero on entry
    int64_t col_split;       // gathered pass: columns per workgroup (multiple of SCR_COLS)
    int32_t *gcj;            // [nrows * SCR_CAP2]
    float *gcl;              // [nrows * SCR_CAP2]
    // pair bounds (ub != nullptr, BF16 only): the capture thresholds use
    // ub[i] = min over the partners screened so far of Dhat^2_ij + E_ij (an
    // upper bound of the row's lightest D^2, +inf on entry) instead of
    // b_i + Emax_i, and a partner is captured when Dhat^2_ij - E_ij <= kappa ub_i;
    // for data whose norms are heavy tailed, where Emax_i (taken over the
    // largest norm of any point) is far above the pairs' own bounds
    float *ub;               // [n]
    // sweep outputs
    float *best;             // [n]
    int32_t *ccnt;           // [n] candidates (> SCR_CAP = overflow)
    int32_t *cj;             // [n * SCR_CAP]
    float *cl;               // [n * SCR_CAP]
    // neighbour lists (tile-pair screen; lcnt == nullptr: none are built):
    // every pair with Dhat^2 <= ltau of one of its points is appended to that
    // point's list; past LIST_CAP entries the smallest dropped value is kept
    const float *ltau;       // [n] capture threshold
    int32_t *lcnt;           // [n] entries offered (zero on entry)
    uint32_t *ldrop;         // [n] smallest dropped Dhat^2 as bits (+inf on entry)
    int32_t *lj;             // [n * LIST_CAP]
    float *lv;               // [n * LIST_CAP] Dhat^2 of the entry
    // final round (bestc != nullptr): every tile holds points of one
    // component (tcomp), the minima are kept per (other component, position
    // in the tile order) in bestc[c * bestc_stride + pos] (so that an item's
    // rows and columns read and lower consecutive entries), and candidates go
    // to gcj/gcl (SCR_CAP2 per point, counted in ccnt)
    float *bestc;
    int64_t bestc_stride;
    const int32_t *tcomp;    // [tiles] component of each tile of the order
    uint32_t *upair;         // [FR_KC * FR_KC] (fr_pair) running bound of each pair of components' lightest
                             // edge on the recheck scale, as float bits (+inf on entry)
    float up, dn;            // recheck-scale factors: bound = (Dhat^2 + Emax) up; real-scale threshold = bound dn
};

// Slot of the unordered pair of components (a, b) in the final round's tables.
__host__ __device__ inline int fr_pair(int a, int b) { return a < b ? a * FR_KC + b : b * FR_KC + a; }

struct ScreenLDS {
    uint32_t rowbest[SCR_ROWS];
    uint32_t rowub[SCR_ROWS];  // pair bounds: the row's running upper bound ub
    int32_t rowcnt[SCR_ROWS];
    int32_t rowovf[SCR_ROWS];
    float rowE[SCR_ROWS];
    int32_t lj[SCR_ROWS][SCR_CAP];
    float ll[SCR_ROWS][SCR_CAP];
    float csq[SCR_COLS], crn[SCR_COLS], cre[SCR_COLS];
    int32_t ccomp[SCR_COLS];
    int32_t csqi[SCR_COLS];  // INT8: exact integer squared norms
};

// Minimum over the 64 lanes of a wave (every lane receives it), unsigned.
__device__ __forceinline__ uint32_t wave_min_u32(uint32_t v) {
    v = min(v, (uint32_t)__builtin_amdgcn_update_dpp((int)~0u, (int)v, 0xB1, 0xF, 0xF, false));   // quad xor 1
    v = min(v, (uint32_t)__builtin_amdgcn_update_dpp((int)~0u, (int)v, 0x4E, 0xF, 0xF, false));   // quad xor 2
    v = min(v, (uint32_t)__builtin_amdgcn_update_dpp((int)~0u, (int)v, 0x141, 0xF, 0xF, false));  // half-row mirror
    v = min(v, (uint32_t)__builtin_amdgcn_update_dpp((int)~0u, (int)v, 0x140, 0xF, 0xF, false));  // row mirror
    const auto r16 = __builtin_amdgcn_permlane16_swap(v, v, false, false);
    v = min(v, min((uint32_t)r16[0], (uint32_t)r16[1]));
    const auto r32 = __builtin_amdgcn_permlane32_swap(v, v, false, false);
    return min(v, min((uint32_t)r32[0], (uint32_t)r32[1]));
}

// atomicMin(&base[key], val) for the active lanes of a wave, with lanes that
// share a key combined first (up to four keys per wave; the rest go straight
// to the atomic).  Every lane of the wave must call it.
__device__ __forceinline__ void grouped_atomic_min(uint32_t *base, int key, uint32_t val, bool active) {
    const int lane = threadIdx.x & 63;
#pragma unroll 1
    for (int it = 0; it < 4; ++it) {
        const unsigned long long act = __ballot(active);
        if (act == 0ull) return;
        const int leader = __ffsll((long long)act) - 1;
        const int lk = __shfl(key, leader, 64);
        const bool mine = active && key == lk;
        const uint32_t m = wave_min_u32(mine ? val : 0xFFFFFFFFu);
        if (lane == leader) atomicMin(&base[lk], m);
        active = active && !mine;
    }
    if (active) atomicMin(&base[key], val);
}

__device__ __forceinline__ float pair_bound(const ScreenBound &B, float ri, float rj, float ei, float ej) {
    const float t = ri + rj, f = ei + ej;
    const float g = fmaxf(ri, rj) <= B.rlim ? B.g_exact : B.g;
    return (g * t * t + f * (2.0f * t + f)) * (1.0f + 1.0f / 1024.0f);
}

// Lower bound of D^2 from Dhat^2 = v and the bound E (both >= 0): the 2^-21
// slack covers the two roundings of this evaluation.
__device__ __forceinline__ float lower_of(float v, float E) { return fmaf(-0x1p-21f, v + E, v - E); }

// Workgroup-wide initialisation of the per-row state; `row_of(q)` gives the
// global row of local slot q (or -1).
template <bool GATHER>
__device__ __forceinline__ void screen_init_rows(ScreenLDS &S, const ScreenArgs &A, int64_t i0) {
    for (int q = threadIdx.x; q < SCR_ROWS; q += blockDim.x) {
        int64_t i;
        if (GATHER) {
            const int64_t slot = i0 + q;
            i = slot < A.nrows ? A.rows[slot] : -1;
        } else {
            i = i0 + q < A.n ? i0 + q : -1;
        }
        S.rowbest[q] = (GATHER && i >= 0) ? __float_as_uint(A.best_in[i]) : __float_as_uint(SCR_INF);
        S.rowub[q] = (GATHER && i >= 0 && A.ub) ? __float_as_uint(A.ub[i]) : __float_as_uint(SCR_INF);
        S.rowcnt[q] = 0;
        S.rowovf[q] = 0;
        S.rowE[q] = i >= 0 ? A.Emax[i] : 0.0f;
    }
}

// Column constants of the tile starting at j0.
__device__ __forceinline__ void screen_load_cols(ScreenLDS &S, const ScreenArgs &A, int64_t j0) {
    for (int q = threadIdx.x; q < SCR_COLS; q += blockDim.x) {
        const int64_t j = j0 + q;
        S.csq[q] = A.sq[j];
        S.crn[q] = A.rn[j];
        S.cre[q] = A.re[j];
        S.ccomp[q] = A.comp[j];
        S.csqi[q] = A.sqi ? A.sqi[j] : 0;
    }
}

// Masked Dhat^2 of one element.
__device__ __forceinline__ float screen_value(float G, float si, float sj, int ci, int cj) {
    const float t = fmaxf(fmaf(-2.0f, G, si + sj), 0.0f);
    return (ci >= 0 && cj >= 0 && cj != ci) ? t : SCR_INF;
}

__device__ __forceinline__ void screen_row_min(ScreenLDS &S, int rl, float m) {
    if (m < SCR_INF) atomicMin(&S.rowbest[rl], __float_as_uint(m));
}

// Capture test and store of one element (v = masked Dhat^2).
template <bool GATHER>
__device__ __forceinline__ void screen_capture(ScreenLDS &S, const ScreenArgs &A, int rl, int64_t slot, float v,
                                               float thr_cheap, float thr, float ri, float ei, int cl,
                                               int64_t j) {
    if (!(v <= thr_cheap)) return;
    const float E = pair_bound(A.bound, ri, S.crn[cl], ei, S.cre[cl]);
    const float L = lower_of(v, E);
    if (!(L <= thr)) return;
    if (GATHER) {
        const int pos = atomicAdd(&A.gcnt[slot], 1);  // several workgroups share a slot
        if (pos < SCR_CAP2) {
            A.gcj[slot * SCR_CAP2 + pos] = (int32_t)j;
            A.gcl[slot * SCR_CAP2 + pos] = L;
        }
    } else {
        const int pos = atomicAdd(&S.rowcnt[rl], 1);
        if (pos < SCR_CAP) {
            S.lj[rl][pos] = (int32_t)j;
            S.ll[rl][pos] = L;
        } else {
            S.rowovf[rl] = 1;
        }
    }
}

// Pair bounds: capture of one element whose lower bound L is already known.
template <bool GATHER>
__device__ __forceinline__ void screen_capture_lb(ScreenLDS &S, const ScreenArgs &A, int rl, int64_t slot, float L,
                                                  float thr, int64_t j) {
    if (!(L <= thr)) return;
    if (GATHER) {
        const int pos = atomicAdd(&A.gcnt[slot], 1);
        if (pos < SCR_CAP2) {
            A.gcj[slot * SCR_CAP2 + pos] = (int32_t)j;
            A.gcl[slot * SCR_CAP2 + pos] = L;
        }
    } else {
        const int pos = atomicAdd(&S.rowcnt[rl], 1);
        if (pos < SCR_CAP) {
            S.lj[rl][pos] = (int32_t)j;
            S.ll[rl][pos] = L;
        } else {
            S.rowovf[rl] = 1;
        }
    }
}

// Per-row thresholds from the current running minimum.
__device__ __forceinline__ void screen_thresholds(const ScreenLDS &S, int rl, float kappa, float &thr_cheap,
                                                  float &thr) {
    const float b = __uint_as_float(S.rowbest[rl]);
    const float E = S.rowE[rl];
    thr_cheap = (b + 2.0f * E) * kappa;
    thr = (b + E) * kappa;
}

// Drops captured entries that the current minimum has ruled out, for rows
// whose list is more than half full.  One thread per row.
__device__ __forceinline__ void screen_compact(ScreenLDS &S, float kappa) {
    for (int rl = threadIdx.x; rl < SCR_ROWS; rl += blockDim.x) {
        const int cnt = S.rowcnt[rl];
        if (S.rowovf[rl] || cnt <= SCR_CAP / 2) continue;
        float tc, thr;
        screen_thresholds(S, rl, kappa, tc, thr);
        int keep = 0;
        for (int q = 0; q < cnt && q < SCR_CAP; ++q) {
            const float L = S.ll[rl][q];
            if (L <= thr) {
                S.lj[rl][keep] = S.lj[rl][q];
                S.ll[rl][keep] = L;
                ++keep;
            }
        }
        S.rowcnt[rl] = keep;
    }
}

// Writes the per-row results of the workgroup.
template <bool GATHER>
__device__ __forceinline__ void screen_finish(ScreenLDS &S, const ScreenArgs &A, int64_t i0) {
    for (int rl = threadIdx.x; rl < SCR_ROWS; rl += blockDim.x) {
        if (GATHER) {
            // counts were accumulated in gcnt directly
        } else {
            const int64_t i = i0 + rl;
            if (i >= A.n) continue;
            A.best[i] = __uint_as_float(S.rowbest[rl]);
            if (A.ub) A.ub[i] = __uint_as_float(S.rowub[rl]);
            const int cnt = S.rowovf[rl] ? SCR_CAP + 1 : S.rowcnt[rl];
            A.ccnt[i] = cnt;
            for (int q = 0; q < cnt && q < SCR_CAP; ++q) {
                A.cj[i * SCR_CAP + q] = S.lj[rl][q];
                A.cl[i * SCR_CAP + q] = S.ll[rl][q];
            }
        }
    }
}

// Row-sweep screen (screen_mfma.hip): every workgroup owns SCR_ROWS rows and
// sweeps a range of columns; used for the gathered second pass, where the
// columns are split over workgroups (gcnt must be zero on entry).  best[] of a
// gathered row enters as an upper bound of its minimum (the exact minimum
// after a full screen) and leaves as the minimum: the column blocks merge
// their running minima into it after every tile and continue from it.
void launch_screen_rows(const ScreenArgs &A, bool gather, hipStream_t s);

// Symmetric tile-pair screen (screen_pairs.hip): best[] must hold +inf and
// ccnt[] zero on entry; both are updated with atomics, indexed by point id.
int64_t pair_tile();
// The order of the ntiles (ntiles + 1) / 2 tile pairs (I <= J), written to out
// on the stream: the diagonal pairs first, then the others in small blocks,
// block row by block row, or with `band` by distance from the diagonal.
void launch_pair_order(int64_t ntiles, int2 *out, hipStream_t s, bool band);
// pairs: nmask tile pairs screened with the component mask (every diagonal
// pair, and any pair whose tiles may share a component), then noff pairs whose
// two tiles share no component, which are screened without it (positions in
// the tile order A.perm).
void launch_screen_pairs(const ScreenArgs &A, const int2 *pairs, int64_t nmask, int64_t noff, hipStream_t s);

}  // namespace iso
