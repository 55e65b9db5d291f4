// screen_pairs.hip -- symmetric Boruvka screen over tile pairs (gfx950 MFMA).
//
// The points are cut into tiles of PT = 256.  Every tile pair (I, J) with
// I <= J is screened once, so every unordered pair of points is formed once:
// the Gram block G = X'_J X'_I^T is accumulated on MFMA (FP32 accumulate), then
//   Dhat^2 = s_i + s_j - 2 G  (masked: valid points, different components,
//                              and i < j on the diagonal tile pairs)
// updates both sides: the running minimum of every row i of I (over the
// block's columns) and of every column j of J (over the block's rows) is
// merged into a global per-point minimum with atomic min, and every element
// whose lower bound can still beat that point's minimum is appended to the
// point's global candidate list (screen.hpp gives the bound).  Lists are
// append-only: an entry stays even when a later minimum rules it out (the
// recheck filters it), and a point whose list overflows is re-screened by the
// row-sweep kernel starting from its final minimum.  With neighbour lists
// requested (A.lcnt set), every element at or below a point's list threshold
// is also appended to that point's neighbour list.  In the final round
// (A.bestc set) every tile holds one component and the minima and candidate
// lists are kept per (point, other component).
//
// One workgroup (4 waves) screens one half of a tile pair: all PT rows of I
// against PH = 128 columns of J.  Its LDS footprint (three 24 KB stages of the
// K pipeline plus 5 KB of tile constants) lets two workgroups share a CU, so
// one workgroup's epilogue, barriers and load latency overlap the other's
// MFMA work.  Wave (wi, wj) computes rows [128 wi, +128) x columns
// [64 wj, +64) as 4 x 2 blocks of the transposed 32 x 32 MFMA (MFMA rows =
// columns j, MFMA columns = rows i; result register q of lane l is MFMA row
// 8 (q div 4) + 4 (l div 32) + (q mod 4), MFMA column l mod 32): BF16
// 32x32x16, FP8 E4M3 32x32x64 (unit block scales), INT8 32x32x32 (int32
// accumulate) or FP32 32x32x2.  The operands come from a copy of the
// representation stored chunk-major within each tile (the 64-byte K chunk c
// of a tile's PT rows is contiguous), so each wave's 1 KB DMA run of a chunk
// reads eight consecutive whole cache lines.
//
// Tiles are runs of 256 positions of a tile order (A.perm maps positions to
// points); after the first round the order groups points by component and the
// caller drops tile pairs inside one component.  Work items (tile pair, half)
// are enumerated with the pairs that need the component mask (the diagonal
// pairs, and pairs whose tiles share a component) in a launch of their own,
// and the others, whose epilogue has no mask, in blocks of PAIR_SB x PAIR_SB
// tiles;
// each XCD receives a contiguous run of that order (workgroup ids are dealt
// to the eight XCDs in turn), so the workgroups resident on one XCD share
// their I and J tiles in its L2.
#include <algorithm>
#include <vector>

#include "screen.hpp"

namespace iso {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef int intx8 __attribute__((ext_vector_type(8)));
typedef int intx4 __attribute__((ext_vector_type(4)));
typedef int intx16 __attribute__((ext_vector_type(16)));
typedef float floatx16 __attribute__((ext_vector_type(16)));

constexpr int PT = 256;                // points per tile (rows of a work item)
constexpr int PH = 128;                // columns of a work item (half of tile J)
constexpr int SROWS = PH + PT;         // staged rows per K chunk: the columns, then the rows
constexpr int NW = 4;                  // waves per workgroup
constexpr int RUNS = SROWS * 4 / 64 / NW;  // 1 KB DMA runs per wave and chunk (both operands staged)
constexpr int CRUNS = PH * 4 / 64 / NW;    // 1 KB DMA runs per wave and chunk (columns only)
constexpr int NPRE = (PT + PH + 64 * NW - 1) / (64 * NW);
#ifndef PAIR_SB
#define PAIR_SB 4                      // tile pairs are ordered in blocks of PAIR_SB x PAIR_SB tiles
#endif
static_assert(RUNS * NW * 64 == SROWS * 4, "runs cover the staged slots");
static_assert(PH % 16 == 0, "a run never straddles the column and row parts");

// s_waitcnt immediate waiting for vmcnt <= n (expcnt and lgkmcnt left at their maxima)
#define VMCNT(n) (((n) & 0xF) | (((n) >> 4) << 14) | (0x7 << 4) | (0xF << 8))

template <int REP>
struct PPrec;

template <>
struct PPrec<ISO_PREC_BF16> {
    using T = uint16_t;
    static constexpr int KC = 32;      // K elements per chunk (64 bytes per row)
    static constexpr int KSTEP = 16;
    static constexpr int VEC = 8;
};

template <>
struct PPrec<ISO_PREC_FP8> {
    using T = uint8_t;
    static constexpr int KC = 64;
    static constexpr int KSTEP = 64;
    static constexpr int VEC = 32;
};

template <>
struct PPrec<ISO_PREC_INT8> {
    using T = int8_t;
    static constexpr int KC = 64;
    static constexpr int KSTEP = 32;
    static constexpr int VEC = 16;
};

template <>
struct PPrec<ISO_PREC_FP32> {
    using T = float;
    static constexpr int KC = 16;
    static constexpr int KSTEP = 2;
    static constexpr int VEC = 1;
};

struct PairLDS {
    uint32_t rmin[PT];     // tile minima of the rows; after the merge, the current global minima
    uint32_t cmin[PH];     // same for the columns
    float rE[PT], cE[PH];  // Emax
    float csq[PH];         // s of the columns
    int32_t ccomp[PH];     // component of the columns
    int32_t rhot[PT];      // bit 0: row's tile minimum is within its capture margin; bit 1: within its list threshold
    uint32_t chot[PH / 32];
    uint32_t clst[PH / 32];  // column's tile minimum is within its list threshold
    int32_t rid[PT], cid[PH];  // point ids of the rows and columns
    int32_t csqi[PH];          // INT8: exact integer squared norms of the columns
    int32_t nlist;             // neighbour-list entries staged by this work item
    int32_t ncap;              // candidates staged by this work item
    uint32_t umin;             // final round: the item's bound of its pair of components' lightest edge
};

// Pair bounds (BF16 plain rounds with A.ub set): per element its own bound
// E_ij, the tile minima of Dhat^2 + E_ij (upper bounds) and of the lower bound
// Dhat^2 - E_ij, and the columns' norm and representation-error bounds; kept in
// the list-staging half of the epilogue buffer, which plain rounds leave idle.
struct PBLDS {
    uint32_t rminU[PT], rminL[PT];
    uint32_t cminU[PH], cminL[PH];
    float rrn[PT], rre[PT];
    float crn[PH], cre[PH];
};

// After the K loop the first staging buffer holds up to LIST_STAGE
// neighbour-list entries (point, partner, Dhat^2) and the second up to
// CAP_STAGE candidates (point, partner, lower bound of D^2).
constexpr int LIST_STAGE = SROWS * 4 * 16 / 12;
constexpr int CAP_STAGE = SROWS * 4 * 16 / 12;

constexpr uint32_t INF_BITS = 0x7F800000u;  // +inf; every screen value is a nonnegative float or +inf

// Minimum over the 32 lanes of each half wave of nonnegative floats compared
// as unsigned bit patterns (every lane receives it): DPP min within quads,
// 8-lane and 16-lane rows, then a swap of neighbouring 16-lane rows.
__device__ __forceinline__ uint32_t min32(uint32_t v) {
    v = min(v, (uint32_t)__builtin_amdgcn_update_dpp((int)~0u, (int)v, 0xB1, 0xF, 0xF, false));   // quad xor 1
    v = min(v, (uint32_t)__builtin_amdgcn_update_dpp((int)~0u, (int)v, 0x4E, 0xF, 0xF, false));   // quad xor 2
    v = min(v, (uint32_t)__builtin_amdgcn_update_dpp((int)~0u, (int)v, 0x141, 0xF, 0xF, false));  // half-row mirror
    v = min(v, (uint32_t)__builtin_amdgcn_update_dpp((int)~0u, (int)v, 0x140, 0xF, 0xF, false));  // row mirror
    const auto r = __builtin_amdgcn_permlane16_swap(v, v, false, false);  // rows 2k and 2k+1 exchange
    return min(v, min((uint32_t)r[0], (uint32_t)r[1]));
}

// Minimum of lanes l and l xor 32.
__device__ __forceinline__ uint32_t min_halves(uint32_t v) {
    const auto r = __builtin_amdgcn_permlane32_swap(v, v, false, false);
    return min(v, min((uint32_t)r[0], (uint32_t)r[1]));
}

// The same for signed values.
__device__ __forceinline__ int32_t min_halves_i32(int32_t v) {
    const auto r = __builtin_amdgcn_permlane32_swap((uint32_t)v, (uint32_t)v, false, false);
    return min(v, min((int32_t)r[0], (int32_t)r[1]));
}

template <int CTRL>
__device__ __forceinline__ int32_t dpp_i32(int32_t v) {
    return __builtin_amdgcn_update_dpp(0x7FFFFFFF, v, CTRL, 0xF, 0xF, false);
}

// Column minima of a 32 x 16 block held one row per lane (lane l mod 32 of
// each half wave holds row l mod 32 of its half's sixteen columns c[0..15]):
// a reduce-scatter over the five lane bits of the half.  Each step pairs every
// lane with a partner that differs in one more bit and keeps half of the
// columns (the lower half where that bit is 0): bit 4 by swapping the rows of
// 16 lanes between the registers of columns q and q + 8, bit 3 by a rotation
// of 16-lane rows by 8, bit 2 by the mirror of 8-lane half rows (lane l with
// l xor 7), bits 1 and 0 by quad permutations.  Lanes 2 m and 2 m + 1 of each
// half end with the minimum of column m over all 32 rows.  38 instructions for
// 16 columns, against 16 separate 32-lane reductions.
__device__ __forceinline__ int32_t col_min16(const int32_t (&c)[16], int lane) {
    int32_t d[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        // rows 1 and 3 of column q trade places with rows 0 and 2 of column q + 8
        const auto r = __builtin_amdgcn_permlane16_swap((uint32_t)c[q], (uint32_t)c[q + 8], false, false);
        d[q] = min((int32_t)r[0], (int32_t)r[1]);  // column q + 8 (l >> 4 & 1)
    }
    const bool b3 = (lane >> 3) & 1, b2 = (lane >> 2) & 1, b1 = (lane >> 1) & 1;
    int32_t e[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int32_t lo = min(d[q], dpp_i32<0x128>(d[q]));          // row_ror:8 = lane xor 8
        const int32_t hi = min(d[q + 4], dpp_i32<0x128>(d[q + 4]));
        e[q] = b3 ? hi : lo;
    }
    int32_t f[2];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const int32_t lo = min(e[q], dpp_i32<0x141>(e[q]));          // half-row mirror = lane xor 7
        const int32_t hi = min(e[q + 2], dpp_i32<0x141>(e[q + 2]));
        f[q] = b2 ? hi : lo;
    }
    const int32_t lo = min(f[0], dpp_i32<0x4E>(f[0]));                // quad lane xor 2
    const int32_t hi = min(f[1], dpp_i32<0x4E>(f[1]));
    const int32_t g = b1 ? hi : lo;
    return min(g, dpp_i32<0xB1>(g));                                  // quad lane xor 1
}

// Appends (other, v) to point p's neighbour list, or lowers its smallest
// dropped value once the list is full.
__device__ __forceinline__ void list_push_global(const ScreenArgs &A, int64_t p, int32_t other, float v) {
    const int pos = atomicAdd(&A.lcnt[p], 1);
    if (pos < LIST_CAP) {
        A.lj[p * LIST_CAP + pos] = other;
        A.lv[p * LIST_CAP + pos] = v;
    } else {
        atomicMin(&A.ldrop[p], __float_as_uint(v));
    }
}

// MODE: MODE_PLAIN, MODE_LIST (neighbour lists as well) or MODE_FINAL (minima
// and candidates per (point, other component); no diagonal pairs).
constexpr int MODE_PLAIN = 0, MODE_LIST = 1, MODE_FINAL = 2;

// BF16 (register rows): wave w computes rows [64 w, +64) x all PH columns as
// 2 x 4 blocks; the rows' operand is loaded straight into registers (each
// wave's rows are its own), only the columns, which all four waves read, are
// staged in LDS.  The other precisions: wave (wi, wj) computes rows
// [128 wi, +128) x columns [64 wj, +64) as 4 x 2 blocks, both operands staged.
template <int REP>
struct PWave {
    static constexpr bool RR = REP == ISO_PREC_BF16;  // rows in registers
    static constexpr int RW = RR ? 64 : 128, CW = RR ? PH : 64;
    static constexpr int NIB = RW / 32, NJB = CW / 32;
    static constexpr int STAGE_U4 = (RR ? PH : SROWS) * 4;  // uint4 slots of one LDS stage
};

template <int REP, bool MASKED, int MODE, bool PB = false>
__global__ __launch_bounds__(64 * NW, 2) void k_screen_pairs(ScreenArgs A, const int2 *__restrict__ pairs,
                                                            int64_t per_xcd, int64_t nitems) {
    constexpr bool LIST = MODE == MODE_LIST, FINAL = MODE == MODE_FINAL;
    static_assert(!(FINAL && MASKED), "the final round pairs tiles of different components only");
    static_assert(!PB || (MODE == MODE_PLAIN && REP == ISO_PREC_BF16), "pair bounds: BF16 plain rounds only");
    using P = PPrec<REP>;
    using T = typename P::T;
    using WL = PWave<REP>;
    constexpr bool RR = WL::RR;
    constexpr int RW = WL::RW, CW = WL::CW, NIB = WL::NIB, NJB = WL::NJB;
    __shared__ PairLDS S;
    // NSTAGE = 3 staging buffers of one K chunk.  Both operands staged: rows
    // 0..PH-1 = the columns j, rows PH.. = the rows i; 64 bytes per row in four
    // 16-byte slots, slot (row, part) at row * 4 + (part xor ((row >> 2) & 3)),
    // which makes the MFMA fragment reads (16 consecutive rows, one part)
    // bank-conflict free.  Register rows (BF16): the PH columns in the
    // fragment order of the screen copy (1 KB per 32-column block and 16-wide
    // K step, lane l's 16 bytes at 16 l), so every fragment read is one
    // contiguous 1 KB.
    __shared__ __attribute__((aligned(16))) uint4 stage0[WL::STAGE_U4];
    __shared__ __attribute__((aligned(16))) uint4 stage1[WL::STAGE_U4];
    __shared__ __attribute__((aligned(16))) uint4 stage2[WL::STAGE_U4];
    // register rows: the epilogue's list and candidate staging, which the
    // other layout keeps in the idle K stages
    __shared__ __attribute__((aligned(16))) uint4 xstage[RR ? 2 * SROWS * 4 : 1];
    static_assert(sizeof(PBLDS) <= SROWS * 4 * sizeof(uint4), "pair-bound tables fit the list-staging half");
    PBLDS &PS = *reinterpret_cast<PBLDS *>(xstage);

    const int tid = threadIdx.x;
    const int lane = tid & 63, w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wi = RR ? w : w >> 1, wj = RR ? 0 : w & 1;
    const T *X = reinterpret_cast<const T *>(A.Xtile);  // rows in the tile order
    const int64_t d_pad = A.d_pad;

    // XCD-aware placement: workgroup b runs on XCD b mod 8, and each XCD takes
    // a contiguous run of the item order
    const int64_t b = blockIdx.x;
    const int64_t idx = (b & 7) * per_xcd + (b >> 3);
    if (idx >= nitems) return;
    const int2 pr = pairs[idx >> 1];
    const int half = (int)(idx & 1);
    // positions in the tile order; A.perm maps them to point ids
    const int64_t I0 = (int64_t)pr.x * PT, J0 = (int64_t)pr.y * PT + half * PH;
    const int32_t *__restrict__ perm = A.perm;
    // final round: rows' minima go to the column tile's component and back
    const int32_t compI = FINAL ? A.tcomp[pr.x] : 0, compJ = FINAL ? A.tcomp[pr.y] : 0;
    // the diagonal tile pairs form each pair of points once (i < j)
    const bool diag = MASKED && pr.x == pr.y;

    // asynchronous staging: each wave moves RUNS 1 KB runs of slots per chunk
    // with global_load_lds_dwordx4 (lane L of a run fills slot base + L); a run
    // covers 16 rows, all columns (runs < PH / 16) or all rows
    static_assert(P::KC * sizeof(T) == 64, "one K chunk is 64 bytes per row");
    // Xtile is chunk-major within each tile: chunk C of the tile's PT rows is
    // PT x 64 contiguous bytes, row t of the tile at byte 64 t
    const char *XJb = reinterpret_cast<const char *>(X + (int64_t)pr.y * PT * d_pad);
    const char *XIb = reinterpret_cast<const char *>(X + I0 * d_pad);
    uint32_t soff[RUNS];  // byte offset of this lane's slot source within chunk 0 of its tile
#pragma unroll
    for (int r = 0; r < RUNS; ++r) {
        const int slot = (w * RUNS + r) * 64 + lane;
        const int row = slot >> 2;
        const int part = (slot & 3) ^ ((row >> 2) & 3);
        const int trow = row < PH ? half * PH + row : row - PH;  // row within its tile
        soff[r] = (uint32_t)(trow * 64 + part * 16);
    }
    const int nchunks = (int)(d_pad / P::KC);
    // Register rows (BF16): the first two chunks are requested right after the
    // tile constants' DMA.  Both prologue issues are unconditional (with one chunk
    // the second re-reads chunk 0 and is never used), so that the loop's first
    // step sees the same loads in flight from either predecessor.
    static_assert(!RR || (NIB == 2 && NJB * 32 == PH && CRUNS == 2), "register-row layout");
    const char *colb = XJb + half * (PH * 64) + (int64_t)lane * 16;
    const char *rowb = XIb + (int64_t)(2 * w) * 2048 + (int64_t)lane * 16;
    uint4 rg0[2][2], rg1[2][2], rg2[2][2];  // [block][K step] of chunks c, c+1, c+2 (mod 3)
#define ISO_RISSUE(STG, RG, C)                                                                                \
    {                                                                                                        \
        _Pragma("unroll") for (int r = 0; r < CRUNS; ++r) __builtin_amdgcn_global_load_lds(                 \
            (const void *)(colb + (int64_t)(C) * (PT * 64) + (w * CRUNS + r) * 1024),                         \
            (__attribute__((address_space(3))) void *)&STG[(w * CRUNS + r) * 64], 16, 0, 0);                \
        _Pragma("unroll") for (int ib = 0; ib < 2; ++ib) _Pragma("unroll") for (int t = 0; t < 2; ++t) RG[ib][t] = \
            *reinterpret_cast<const uint4 *>(rowb + (int64_t)(C) * (PT * 64) + ib * 2048 + t * 1024);        \
    }

    // Tile constants, from the per-position copies: the running tile minima
    // start at +inf (written before any DMA is in flight, so no LDS write waits
    // for one); the point ids, Emax, and the columns' s and components go to
    // LDS by DMA (one dword per lane, ahead of the first chunks, so the first
    // pipeline step's wait covers them); the rows' s and components, which stay
    // in registers, are plain loads.
    static_assert(64 * NW == PT && PH % 64 == 0, "one thread per row, whole waves per column set");
    S.rmin[tid] = INF_BITS;
    if (tid < PH) S.cmin[tid] = INF_BITS;
    if constexpr (PB) {
        PS.rminU[tid] = INF_BITS;
        PS.rminL[tid] = INF_BITS;
        if (tid < PH) {
            PS.cminU[tid] = INF_BITS;
            PS.cminL[tid] = INF_BITS;
        }
    }
    auto dma4 = [&](const void *src, void *lds_wave_base) {
        __builtin_amdgcn_global_load_lds(src, (__attribute__((address_space(3))) void *)lds_wave_base, 4, 0, 0);
    };
    dma4(perm + I0 + tid, &S.rid[64 * w]);
    dma4(A.pEmax + I0 + tid, &S.rE[64 * w]);
    if constexpr (PB) {
        dma4(A.prn + I0 + tid, &PS.rrn[64 * w]);
        dma4(A.pre + I0 + tid, &PS.rre[64 * w]);
    }
    if (w < PH / 64) {
        dma4(perm + J0 + tid, &S.cid[64 * w]);
        dma4(A.pEmax + J0 + tid, &S.cE[64 * w]);
        dma4(A.psq + J0 + tid, &S.csq[64 * w]);
        dma4(A.pcomp + J0 + tid, &S.ccomp[64 * w]);
        if constexpr (REP == ISO_PREC_INT8) dma4(A.psqi + J0 + tid, &S.csqi[64 * w]);
        if constexpr (PB) {
            dma4(A.prn + J0 + tid, &PS.crn[64 * w]);
            dma4(A.pre + J0 + tid, &PS.cre[64 * w]);
        }
    }
    float si[NIB];
    int ci[NIB];
    int32_t sii[NIB];  // INT8: exact integer squared norms of the rows
#pragma unroll
    for (int ib = 0; ib < NIB; ++ib) {
        const int64_t pos = I0 + RW * wi + 32 * ib + (lane & 31);
        si[ib] = A.psq[pos];
        ci[ib] = A.pcomp[pos];
        sii[ib] = REP == ISO_PREC_INT8 ? A.psqi[pos] : 0;
    }
    if constexpr (RR) {
        ISO_RISSUE(stage0, rg0, 0)
        ISO_RISSUE(stage1, rg1, nchunks > 1 ? 1 : 0)
    }

#define ISO_ISSUE(STG, C)                                                                                     \
    {                                                                                                        \
        _Pragma("unroll") for (int r = 0; r < RUNS; ++r) __builtin_amdgcn_global_load_lds(                  \
            (const void *)((w * RUNS + r < PH / 16 ? XJb : XIb) + (int64_t)(C) * (PT * 64) + soff[r]),              \
            (__attribute__((address_space(3))) void *)&STG[(w * RUNS + r) * 64], 16, 0, 0);                \
    }

    floatx16 acc[NIB][NJB];
#pragma unroll
    for (int ib = 0; ib < NIB; ++ib)
#pragma unroll
        for (int jb = 0; jb < NJB; ++jb)
#pragma unroll
            for (int q = 0; q < 16; ++q) acc[ib][jb][q] = 0.0f;

    // fragment slot of (staged row, k offset in elements) in a stage
    auto frag_slot = [](int row, int kel) {
        const int part = (kel * (int)sizeof(T)) >> 4;
        return row * 4 + (part ^ ((row >> 2) & 3));
    };

    // One pipeline step on chunk C held in stage SB: wait for it (chunk C+1 may
    // stay in flight), barrier (no fence: the DMA data is in LDS once the
    // issuing wave's vmcnt has dropped; every wave has finished reading stage
    // SN, consumed in the previous step), refill stage SN with chunk C+2, compute.
#define ISO_STEP(SB, SN, C)                                                                                   \
    if ((C) < nchunks) {                                                                                     \
        if ((C) + 1 < nchunks)                                                                               \
            __builtin_amdgcn_s_waitcnt(VMCNT(RUNS));                                                         \
        else                                                                                                 \
            __builtin_amdgcn_s_waitcnt(VMCNT(0));                                                            \
        __builtin_amdgcn_s_barrier();                                                                        \
        if ((C) + 2 < nchunks) ISO_ISSUE(SN, (C) + 2)                                                        \
        ISO_COMPUTE(SB)                                                                                      \
    }

#define ISO_PIPELINE                                                                                          \
    if (0 < nchunks) ISO_ISSUE(stage0, 0)                                                                    \
    if (1 < nchunks) ISO_ISSUE(stage1, 1)                                                                    \
    for (int c = 0; c < nchunks; c += 3) {                                                                   \
        ISO_STEP(stage0, stage2, c)                                                                          \
        ISO_STEP(stage1, stage0, c + 1)                                                                      \
        ISO_STEP(stage2, stage1, c + 2)                                                                      \
    }
    if constexpr (RR) {
        // Register rows (BF16 only).  The screen copy is in fragment order:
        // chunk C of a tile is 16 KB, 32-row block b at 2 KB b, 16-wide K step
        // t at +1 KB t, lane l's 16 bytes at +16 l (row 32 b + l mod 32, K
        // elements 32 C + 16 t + 8 (l div 32) .. +7).  The PH columns of the
        // item are blocks 4 half .. 4 half + 3 of tile J (8 KB, staged by
        // CRUNS 1 KB DMA runs per wave); wave w's rows are blocks 2 w, 2 w + 1
        // of tile I (four 16-byte loads per lane and chunk, straight into
        // registers, issued two chunks ahead).
#define ISO_RCOMPUTE(SB, RG, NT)                                                                              \
    _Pragma("unroll") for (int t = 0; t < 2; ++t) if (t < (NT)) {                                            \
        bf16x8 a[NJB];                                                                                        \
        _Pragma("unroll") for (int jb = 0; jb < NJB; ++jb) {                                                  \
            const uint4 v = SB[(jb * 2 + t) * 64 + lane];                                                     \
            a[jb] = *reinterpret_cast<const bf16x8 *>(&v);                                                    \
        }                                                                                                     \
        _Pragma("unroll") for (int ib = 0; ib < 2; ++ib) {                                                    \
            const bf16x8 bb = *reinterpret_cast<const bf16x8 *>(&RG[ib][t]);                                  \
            _Pragma("unroll") for (int jb = 0; jb < NJB; ++jb) acc[ib][jb] =                                  \
                __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[jb], bb, acc[ib][jb], 0, 0, 0);                     \
        }                                                                                                     \
    }
#define ISO_RSTEP(SB, RG, SN, RN, C)                                                                          \
    if ((C) < nchunks) {                                                                                     \
        if ((C) + 1 < nchunks)                                                                               \
            __builtin_amdgcn_s_waitcnt(VMCNT(CRUNS + 4));                                                    \
        else                                                                                                 \
            __builtin_amdgcn_s_waitcnt(VMCNT(0));                                                            \
        __builtin_amdgcn_s_barrier();                                                                        \
        if ((C) + 2 < nchunks) ISO_RISSUE(SN, RN, (C) + 2)                                                   \
        ISO_RCOMPUTE(SB, RG, (C) + 1 == nchunks && d_last_half ? 1 : 2)                                      \
    }
        // Steps inside the loop issue unconditionally, so every step finds
        // exactly two chunks (12 loads) in flight and the register loads need
        // no wait beyond the one before the barrier; the last one to four
        // chunks run in the guarded steps after it.
#define ISO_RSTEP_FULL(SB, RG, SN, RN, C)                                                                     \
    {                                                                                                        \
        __builtin_amdgcn_s_waitcnt(VMCNT(CRUNS + 4));                                                        \
        __builtin_amdgcn_s_barrier();                                                                        \
        ISO_RISSUE(SN, RN, (C) + 2)                                                                          \
        ISO_RCOMPUTE(SB, RG, 2)                                                                              \
    }
        // the last chunk's second 16-wide K step holds only zero padding when
        // d ends in the chunk's first half: its MFMAs are skipped
        const bool d_last_half = A.d <= (int64_t)(nchunks - 1) * P::KC + P::KC / 2;
        int c = 0;
        for (; c + 4 < nchunks; c += 3) {
            ISO_RSTEP_FULL(stage0, rg0, stage2, rg2, c)
            ISO_RSTEP_FULL(stage1, rg1, stage0, rg0, c + 1)
            ISO_RSTEP_FULL(stage2, rg2, stage1, rg1, c + 2)
        }
        ISO_RSTEP(stage0, rg0, stage2, rg2, c)
        ISO_RSTEP(stage1, rg1, stage0, rg0, c + 1)
        ISO_RSTEP(stage2, rg2, stage1, rg1, c + 2)
        ISO_RSTEP(stage0, rg0, stage2, rg2, c + 3)
#undef ISO_RSTEP_FULL
#undef ISO_RSTEP
#undef ISO_RCOMPUTE
#undef ISO_RISSUE
    } else if constexpr (REP == ISO_PREC_FP8) {
        // one 32 x 32 x 64 FP8 MFMA per block and chunk: lane l supplies row
        // l mod 32 and k = 32 (l div 32) .. +31, i.e. slots 2 (l div 32) and
        // 2 (l div 32) + 1 of the row; unit block scales (E8M0 code 127)
#define ISO_FRAG8(SB, ROW, OUT)                                                                               \
    {                                                                                                        \
        const uint4 v0 = SB[frag_slot((ROW), 32 * (lane >> 5))];                                             \
        const uint4 v1 = SB[frag_slot((ROW), 32 * (lane >> 5) + 16)];                                        \
        OUT = intx8{(int)v0.x, (int)v0.y, (int)v0.z, (int)v0.w, (int)v1.x, (int)v1.y, (int)v1.z, (int)v1.w};  \
    }
#define ISO_COMPUTE(SB)                                                                                       \
    {                                                                                                        \
        intx8 a[NJB], bb[NIB];                                                                                \
        _Pragma("unroll") for (int jb = 0; jb < NJB; ++jb) ISO_FRAG8(SB, CW * wj + 32 * jb + (lane & 31), a[jb]) \
        _Pragma("unroll") for (int ib = 0; ib < NIB; ++ib)                                                    \
            ISO_FRAG8(SB, PH + RW * wi + 32 * ib + (lane & 31), bb[ib])                                       \
        _Pragma("unroll") for (int ib = 0; ib < NIB; ++ib) _Pragma("unroll") for (int jb = 0; jb < NJB; ++jb) \
            acc[ib][jb] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a[jb], bb[ib], acc[ib][jb], 0, 0, 0,   \
                                                                          0x7F7F7F7F, 0, 0x7F7F7F7F);         \
    }
        ISO_PIPELINE
#undef ISO_COMPUTE
#undef ISO_FRAG8
    } else if constexpr (REP == ISO_PREC_INT8) {
        // two 32 x 32 x 32 INT8 MFMAs per block and chunk (int32 accumulators
        // held in the FP32 accumulator registers, bit for bit)
#define ISO_COMPUTE(SB)                                                                                       \
    _Pragma("unroll") for (int ks = 0; ks < P::KC; ks += P::KSTEP) {                                          \
        const int kel = ks + (lane >> 5) * P::VEC;                                                             \
        intx4 a[NJB], bb[NIB];                                                                                \
        _Pragma("unroll") for (int jb = 0; jb < NJB; ++jb) {                                                  \
            const uint4 v = SB[frag_slot(CW * wj + 32 * jb + (lane & 31), kel)];                               \
            a[jb] = intx4{(int)v.x, (int)v.y, (int)v.z, (int)v.w};                                             \
        }                                                                                                     \
        _Pragma("unroll") for (int ib = 0; ib < NIB; ++ib) {                                                  \
            const uint4 v = SB[frag_slot(PH + RW * wi + 32 * ib + (lane & 31), kel)];                          \
            bb[ib] = intx4{(int)v.x, (int)v.y, (int)v.z, (int)v.w};                                            \
        }                                                                                                     \
        _Pragma("unroll") for (int ib = 0; ib < NIB; ++ib) _Pragma("unroll") for (int jb = 0; jb < NJB; ++jb) \
            acc[ib][jb] = __builtin_bit_cast(floatx16, __builtin_amdgcn_mfma_i32_32x32x32_i8(                  \
                a[jb], bb[ib], __builtin_bit_cast(intx16, acc[ib][jb]), 0, 0, 0));                            \
    }
        ISO_PIPELINE
#undef ISO_COMPUTE
    } else {
#define ISO_COMPUTE(SB)                                                                                       \
    _Pragma("unroll") for (int ks = 0; ks < P::KC; ks += P::KSTEP) {                                          \
        const int kel = ks + (lane >> 5) * P::VEC;                                                             \
        const float *sf = reinterpret_cast<const float *>(SB);                                                \
        const int within = kel & 3;                                                                           \
        float a[NJB], bb[NIB];                                                                                \
        _Pragma("unroll") for (int jb = 0; jb < NJB; ++jb) a[jb] =                                            \
            sf[frag_slot(CW * wj + 32 * jb + (lane & 31), kel) * 4 + within];                                  \
        _Pragma("unroll") for (int ib = 0; ib < NIB; ++ib) bb[ib] =                                           \
            sf[frag_slot(PH + RW * wi + 32 * ib + (lane & 31), kel) * 4 + within];                             \
        _Pragma("unroll") for (int ib = 0; ib < NIB; ++ib) _Pragma("unroll") for (int jb = 0; jb < NJB; ++jb) \
            acc[ib][jb] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[jb], bb[ib], acc[ib][jb], 0, 0, 0);           \
    }
        ISO_PIPELINE
#undef ISO_COMPUTE
    }
#undef ISO_PIPELINE
#undef ISO_STEP
#undef ISO_ISSUE
    // (the epilogue uses only PairLDS, so no barrier is needed before it)

    // The items' points' running minima (list thresholds, pair bounds) are
    // read now, so that their latency overlaps the epilogue's arithmetic.  A
    // value read early can only be larger than the current one (minima only
    // fall), and it is the value of a real pair, so every threshold built
    // from it remains a valid upper bound: an early read only captures more.
    uint32_t pre_old[NPRE], pre_oldu[NPRE];
    float pre_tau[NPRE], pre_r[NPRE], pre_e[NPRE];
#pragma unroll
    for (int e = 0; e < NPRE; ++e) {
        const int u = tid + e * 64 * NW;
        pre_old[e] = pre_oldu[e] = INF_BITS;
        pre_tau[e] = pre_r[e] = pre_e[e] = 0.0f;
        if (u >= PT + PH) continue;
        const bool is_row = u < PT;
        const int t = is_row ? u : u - PT;
        const int64_t p = is_row ? S.rid[t] : S.cid[t];
        if (p >= A.n) continue;
        const int64_t pos = is_row ? I0 + t : J0 + t;
        if constexpr (!PB) {
            pre_r[e] = A.prn[pos];
            pre_e[e] = A.pre[pos];
        }
        const uint32_t *const bp = FINAL ? reinterpret_cast<const uint32_t *>(A.bestc) +
                                               (is_row ? compJ : compI) * A.bestc_stride + pos
                                         : reinterpret_cast<const uint32_t *>(A.pbest) + pos;
        pre_old[e] = *reinterpret_cast<const volatile uint32_t *>(bp);
        if constexpr (LIST) pre_tau[e] = A.pltau[pos];
        if constexpr (PB) pre_oldu[e] = reinterpret_cast<const volatile uint32_t *>(A.pub)[pos];
    }

    // ---- epilogue 1, items whose tiles share no component (the caller's
    // guarantee for the unmasked launch; BF16, FP8 and FP32 without pair
    // bounds): no mask.  Dhat^2 as signed 32-bit patterns (a negative rounding
    // result, sign bit set, orders below every nonnegative value; the reduced
    // minima are clamped at +0, and the accumulators keep the raw value, which
    // the staging below clamps; padding has s = +inf), tile minima of rows
    // (in-lane over the lane's columns, then lanes l, l+32) and of columns
    // (in-lane over the lane's rows, then a reduce-scatter over the half wave:
    // lanes 2 m, 2 m + 1 hold column m of a 32-column block; lane parity picks
    // which of two blocks a lane merges into LDS)
    constexpr bool UNMASKED = !MASKED && !PB && REP != ISO_PREC_INT8;
    if constexpr (UNMASKED) {
        {
            int32_t m[NIB];
#pragma unroll
            for (int ib = 0; ib < NIB; ++ib) m[ib] = (int32_t)INF_BITS;
            int32_t own[(NJB + 1) / 2];
#pragma unroll
            for (int jb = 0; jb < NJB; ++jb) {
                int32_t c[16];
#pragma unroll
                for (int q = 0; q < 16; ++q) {
                    const int jl = CW * wj + 32 * jb + 8 * (q >> 2) + 4 * (lane >> 5) + (q & 3);
                    const float sj = S.csq[jl];
                    int32_t cq = (int32_t)INF_BITS;
#pragma unroll
                    for (int ib = 0; ib < NIB; ++ib) {
                        const int32_t v = __float_as_int(fmaf(-2.0f, acc[ib][jb][q], si[ib] + sj));
                        acc[ib][jb][q] = __int_as_float(v);
                        m[ib] = min(m[ib], v);
                        cq = min(cq, v);
                    }
                    c[q] = cq;
                }
                const int32_t cm = col_min16(c, lane);
                if (jb & 1)
                    own[jb >> 1] = (lane & 1) ? cm : own[jb >> 1];
                else
                    own[jb >> 1] = cm;
            }
#pragma unroll
            for (int o = 0; o < (NJB + 1) / 2; ++o) {
                const int jo = 2 * o + (lane & 1), qo = (lane & 31) >> 1;
                const int jl = CW * wj + 32 * jo + 8 * (qo >> 2) + 4 * (lane >> 5) + (qo & 3);
                const uint32_t v = (uint32_t)max(own[o], 0);
                if (jo < NJB && v < INF_BITS) atomicMin(&S.cmin[jl], v);
            }
#pragma unroll
            for (int ib = 0; ib < NIB; ++ib) {
                const uint32_t mm = (uint32_t)max(min_halves_i32(m[ib]), 0);  // lanes l and l+32 hold the same rows
                if ((lane >> 5) == 0 && mm < INF_BITS) atomicMin(&S.rmin[RW * wi + 32 * ib + (lane & 31)], mm);
            }
        }
    }
    // ---- epilogue 1, the other items: masked Dhat^2 as bit patterns (padding has
    // s = +inf; a negative rounding result becomes +0), tile minima of rows
    // (in-lane over the lane's 32 columns, then lanes l, l+32) and of columns
    // (in-lane over the lane's 4 rows, then the 32 lanes of the half wave; lane
    // 16 jb + q of each half keeps column (jb, q) and merges it into LDS once at
    // the end)
    if constexpr (!UNMASKED) {
        uint32_t m[NIB];
#pragma unroll
        for (int ib = 0; ib < NIB; ++ib) m[ib] = INF_BITS;
        uint32_t cown[NJB / 2];  // lane 16 (jb mod 2) + q of each half keeps column (jb, q) in slot jb / 2
#pragma unroll
        for (int o = 0; o < NJB / 2; ++o) cown[o] = INF_BITS;
#pragma unroll
        for (int jb = 0; jb < NJB; ++jb)
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                const int jl = CW * wj + 32 * jb + 8 * (q >> 2) + 4 * (lane >> 5) + (q & 3);
                const float sj = S.csq[jl];
                const int cjj = S.ccomp[jl];
                const uint32_t sjq = REP == ISO_PREC_INT8 ? (uint32_t)S.csqi[jl] : 0u;
                uint32_t cmin = INF_BITS;
#pragma unroll
                for (int ib = 0; ib < NIB; ++ib) {
                    int32_t tb;
                    if constexpr (REP == ISO_PREC_INT8) {
                        // exact integer squared distance; 2^30 and beyond only with padding
                        const uint32_t d2 = (uint32_t)sii[ib] + sjq - 2u * (uint32_t)__float_as_int(acc[ib][jb][q]);
                        tb = d2 >= (1u << 30) ? (int32_t)INF_BITS : __float_as_int((float)d2 * A.scale2);
                    } else {
                        tb = __float_as_int(fmaf(-2.0f, acc[ib][jb][q], si[ib] + sj));
                    }
                    uint32_t v = (cjj == ci[ib]) ? INF_BITS : (uint32_t)max(tb, 0);
                    if (diag && half * PH + jl <= RW * wi + 32 * ib + (lane & 31)) v = INF_BITS;  // each pair once
                    acc[ib][jb][q] = __uint_as_float(v);
                    m[ib] = min(m[ib], v);
                    cmin = min(cmin, v);
                }
                const uint32_t cm = min32(cmin);
                if ((lane & 31) == 16 * (jb & 1) + q) cown[jb >> 1] = cm;
                if ((q & 3) == 3) __builtin_amdgcn_sched_barrier(0);  // bound the columns in flight
            }
#pragma unroll
        for (int o = 0; o < NJB / 2; ++o) {
            const int qo = lane & 15, jo = 2 * o + ((lane >> 4) & 1);
            const int jl = CW * wj + 32 * jo + 8 * (qo >> 2) + 4 * (lane >> 5) + (qo & 3);
            if (cown[o] < INF_BITS) atomicMin(&S.cmin[jl], cown[o]);
        }
#pragma unroll
        for (int ib = 0; ib < NIB; ++ib) {
            const uint32_t mm = min_halves(m[ib]);  // lanes l and l+32 hold the same rows
            if ((lane >> 5) == 0 && mm < INF_BITS) atomicMin(&S.rmin[RW * wi + 32 * ib + (lane & 31)], mm);
        }
    }
    // ---- pair bounds: each element's own bound E_ij; the tile minima of the
    // upper bounds Dhat^2 + E_ij and of the lower bounds max(Dhat^2 - E_ij, 0),
    // which replace Dhat^2 in the accumulators for the captures (rolled over
    // the columns, indexed register access, to keep the registers of the
    // unrolled epilogue)
    if constexpr (PB) {
        float rr[NIB], re_[NIB];
        uint32_t mu[NIB], ml[NIB];
#pragma unroll
        for (int ib = 0; ib < NIB; ++ib) {
            const int il = RW * wi + 32 * ib + (lane & 31);
            rr[ib] = PS.rrn[il];
            re_[ib] = PS.rre[il];
            mu[ib] = ml[ib] = INF_BITS;
        }
#pragma unroll
        for (int jb = 0; jb < NJB; ++jb) {
            uint32_t ownU = INF_BITS, ownL = INF_BITS;
#pragma unroll 1
            for (int q = 0; q < 16; ++q) {
                const int jl = CW * wj + 32 * jb + 8 * (q >> 2) + 4 * (lane >> 5) + (q & 3);
                const float rj = PS.crn[jl], ej = PS.cre[jl];
                uint32_t cU = INF_BITS, cL = INF_BITS;
#pragma unroll
                for (int ib = 0; ib < NIB; ++ib) {
                    const uint32_t v = __float_as_uint(acc[ib][jb][q]);
                    const float vf = __uint_as_float(v);
                    const float E = pair_bound(A.bound, rr[ib], rj, re_[ib], ej);
                    const uint32_t uU = __float_as_uint(vf + E);
                    const uint32_t uL = v < INF_BITS ? __float_as_uint(fmaxf(lower_of(vf, E), 0.0f)) : INF_BITS;
                    mu[ib] = min(mu[ib], uU);
                    ml[ib] = min(ml[ib], uL);
                    cU = min(cU, uU);
                    cL = min(cL, uL);
                    acc[ib][jb][q] = __uint_as_float(uL);
                }
                const uint32_t cu = min32(cU), cl = min32(cL);
                if ((lane & 31) == q) {
                    ownU = cu;
                    ownL = cl;
                }
            }
            // lane q (< 16) of each half owns column (jb, q) of its half
            if ((lane & 31) < 16) {
                const int qo = lane & 15;
                const int jl = CW * wj + 32 * jb + 8 * (qo >> 2) + 4 * (lane >> 5) + (qo & 3);
                if (ownU < INF_BITS) atomicMin(&PS.cminU[jl], ownU);
                if (ownL < INF_BITS) atomicMin(&PS.cminL[jl], ownL);
            }
        }
#pragma unroll
        for (int ib = 0; ib < NIB; ++ib) {
            const int il = RW * wi + 32 * ib + (lane & 31);
            const uint32_t mmu = min_halves(mu[ib]), mml = min_halves(ml[ib]);
            if ((lane >> 5) == 0 && mmu < INF_BITS) atomicMin(&PS.rminU[il], mmu);
            if ((lane >> 5) == 0 && mml < INF_BITS) atomicMin(&PS.rminL[il], mml);
        }
    }
    if (tid < PH / 32) {
        S.chot[tid] = 0u;
        S.clst[tid] = 0u;
    }
    if (tid == 0) {
        S.nlist = 0;
        S.ncap = 0;
        S.umin = INF_BITS;
    }
    __syncthreads();

    // ---- epilogue 2: merge into the global minima (no-return atomics, only
    // where the item lowers the current value); the merged value
    // replaces the tile minimum in LDS as the threshold base; flag the rows and
    // columns whose tile minimum can still be captured.  In the final round
    // every row and column of the item belongs to the same pair of components
    // (compI, compJ): their merged minima also lower that pair's bound U (one
    // atomic per item), and a row or column is hot only while its tile minimum
    // can still reach U.
    // (the capture thresholds: E_tile, the pair bound of the point against the
    // largest r and e of the other tile, bounds every element's own E_ij, so
    // an element is captured when its lower bound Dhat^2 - E_tile is at most
    // the threshold thr = (b + E) kappa (and, in the final round, U); a row or
    // column is flagged when its tile minimum passes that test.  After this
    // epilogue the LDS holds thr and E_tile in place of b and E.)
    float upair = SCR_INF;  // final round: U on the real-D^2 scale
    uint32_t tmin[NPRE];
    float etile[NPRE];
    const float rmxI = A.trmax[pr.x], emxI = A.temax[pr.x], rmxJ = A.trmax[pr.y], emxJ = A.temax[pr.y];
#pragma unroll
    for (int e = 0; e < NPRE; ++e) {
        const int u = tid + e * 64 * NW;
        if (u >= PT + PH) break;
        const bool is_row = u < PT;
        const int t = is_row ? u : u - PT;
        const int64_t p = is_row ? S.rid[t] : S.cid[t];
        const uint32_t m = is_row ? S.rmin[t] : S.cmin[t];
        const int64_t pos = is_row ? I0 + t : J0 + t;
        uint32_t *const bp = FINAL ? reinterpret_cast<uint32_t *>(A.bestc) + (is_row ? compJ : compI) * A.bestc_stride + pos
                                   : reinterpret_cast<uint32_t *>(A.pbest) + pos;
        const uint32_t old = pre_old[e];
        if (p < A.n && m < old) atomicMin(bp, m);
        const float cur = p < A.n ? __uint_as_float(min(old, m)) : SCR_INF;
        const float E = is_row ? S.rE[t] : S.cE[t];
        etile[e] = fminf(pair_bound(A.bound, pre_r[e], is_row ? rmxJ : rmxI, pre_e[e], is_row ? emxJ : emxI), E);
        if constexpr (PB) {
            // the running upper bound ub; the row is hot when its least lower
            // bound can reach kappa ub; the threshold base becomes ub
            const uint32_t mU = is_row ? PS.rminU[t] : PS.cminU[t];
            const uint32_t mL = is_row ? PS.rminL[t] : PS.cminL[t];
            uint32_t *const up = reinterpret_cast<uint32_t *>(A.pub) + pos;
            const uint32_t oldu = pre_oldu[e];
            if (p < A.n && mU < oldu) atomicMin(up, mU);
            const float curu = p < A.n ? __uint_as_float(min(oldu, mU)) : SCR_INF;
            const float thr = curu * A.kappa;  // (the staged values are already lower bounds)
            const bool hotu = p < A.n && mL < INF_BITS && __uint_as_float(mL) <= thr;
            if (is_row) {
                S.rmin[t] = __float_as_uint(thr);
                S.rE[t] = 0.0f;
                S.rhot[t] = hotu ? 1 : 0;
            } else {
                S.cmin[t] = __float_as_uint(thr);
                S.cE[t] = 0.0f;
                if (hotu) atomicOr(&S.chot[t >> 5], 1u << (t & 31));
            }
            continue;
        }
        if constexpr (FINAL) {
            tmin[e] = m;
            if (cur < SCR_INF) atomicMin(&S.umin, __float_as_uint((cur + E) * A.up));
            if (is_row)
                S.rmin[t] = __float_as_uint(cur);
            else
                S.cmin[t] = __float_as_uint(cur);
            continue;
        }
        // (a row or column with no valid element in the item, m = +inf, is never hot)
        const float thr = (cur + E) * A.kappa, cheap = (cur + E + etile[e]) * A.kappa;
        const bool hot = p < A.n && m < INF_BITS && __uint_as_float(m) <= cheap;
        const bool lst = LIST && p < A.n && __uint_as_float(m) <= pre_tau[e];
        if (is_row) {
            S.rmin[t] = __float_as_uint(thr);
            S.rE[t] = etile[e];
            S.rhot[t] = (hot ? 1 : 0) | (lst ? 2 : 0);
        } else {
            S.cmin[t] = __float_as_uint(thr);
            S.cE[t] = etile[e];
            if (hot) atomicOr(&S.chot[t >> 5], 1u << (t & 31));
            if (lst) atomicOr(&S.clst[t >> 5], 1u << (t & 31));
            // (the columns' s are no longer read: their slots take the
            // columns' list thresholds for the list scan, -inf where the
            // column's tile minimum is above its threshold)
            if constexpr (LIST) S.csq[t] = lst ? pre_tau[e] : -SCR_INF;
        }
    }
    if constexpr (FINAL) {
        __syncthreads();
        if (tid == 0) {
            uint32_t *const gp = A.upair + fr_pair(compI, compJ);
            const uint32_t g = *reinterpret_cast<const volatile uint32_t *>(gp);
            const uint32_t mine = S.umin;
            if (mine < g) atomicMin(gp, mine);
            S.umin = min(g, mine);
        }
        __syncthreads();
        upair = __uint_as_float(S.umin) * A.dn;
#pragma unroll
        for (int e = 0; e < NPRE; ++e) {
            const int u = tid + e * 64 * NW;
            if (u >= PT + PH) break;
            const bool is_row = u < PT;
            const int t = is_row ? u : u - PT;
            const int64_t p = is_row ? S.rid[t] : S.cid[t];
            const float cur = __uint_as_float(is_row ? S.rmin[t] : S.cmin[t]);
            const float E = is_row ? S.rE[t] : S.cE[t];
            // (also within reach of the pair's bound U: an element above the
            // cheap bound has L > U; the 2^-18 covers lower_of's slack and the roundings)
            const float thr = fminf((cur + E) * A.kappa, upair);
            const float cheap =
                fminf((cur + E + etile[e]) * A.kappa, (upair + E + etile[e]) * (1.0f + 0x1p-18f));
            const bool hot = p < A.n && tmin[e] < INF_BITS && __uint_as_float(tmin[e]) <= cheap;
            if (is_row) {
                S.rmin[t] = __float_as_uint(thr);
                S.rE[t] = etile[e];
                S.rhot[t] = hot ? 1 : 0;
            } else {
                S.cmin[t] = __float_as_uint(thr);
                S.cE[t] = etile[e];
                if (hot) atomicOr(&S.chot[t >> 5], 1u << (t & 31));
            }
        }
    }
    __syncthreads();

    // ---- epilogue 3: capture candidates (rows of hot rows, columns of hot
    // columns).  An element whose lower bound passes its row's or column's
    // threshold is staged in LDS (the second staging buffer, idle since the
    // barrier before epilogue 2) with that bound; after the barrier below all
    // threads append them at once, so the latency of the returning atomics is
    // paid once per work item rather than once per candidate.
    constexpr int CAP = FINAL ? SCR_CAP2 : SCR_CAP;
    int32_t *const cjs = FINAL ? A.gcj : A.cj;
    float *const cls = FINAL ? A.gcl : A.cl;
    int32_t *const ccnt = A.ccnt;
    int32_t *const cp = reinterpret_cast<int32_t *>(RR ? xstage + SROWS * 4 : stage1);
    int32_t *const co = cp + CAP_STAGE;
    float *const cv = reinterpret_cast<float *>(co + CAP_STAGE);
    auto commit = [&](int64_t p, int64_t o, float L) {
        const int pos = atomicAdd(&ccnt[p], 1);
        if (pos < CAP) {
            cjs[p * CAP + pos] = (int32_t)o;
            cls[p * CAP + pos] = L;
        }
    };
    // (p, o): the element's point and partner; v its Dhat^2 (pair bounds: its
    // lower bound); thr and et the point's threshold and tile bound
    auto stage_cap = [&](int64_t p, int64_t o, float v, float thr, float et) {
        v = __int_as_float(max(__float_as_int(v), 0));  // an unmasked item's negative value becomes +0
        const float L = PB ? v : lower_of(v, et);
        if (!(L <= thr)) return;
        const int pos = atomicAdd(&S.ncap, 1);
        if (pos < CAP_STAGE) {
            cp[pos] = (int32_t)p;
            co[pos] = (int32_t)o;
            cv[pos] = L;
        } else {
            commit(p, o, L);
        }
    };
    // (the emit closures are taken by value, and the candidate counts through
    // a local pointer: a closure or kernel argument reached through a
    // reference here has made the compiler keep it in scratch memory)
    // The scans below visit few elements: a row's flagged elements are found
    // by one compare per element, whose wave mask (any lane at or below its
    // threshold) marks a column position; only marked positions are then
    // read again (uniform position: indexed register read) and staged.  A
    // flagged column is one register position of one half wave.
    auto scan_row = [&](int ib, float thr, auto emit) {
#pragma unroll
        for (int jb = 0; jb < NJB; ++jb) {  // (jb static: only q indexes a register dynamically)
            uint32_t any = 0;
#pragma unroll
            for (int q = 0; q < 16; ++q)
                if (__ballot(acc[ib][jb][q] <= thr)) any |= 1u << q;
            while (any) {
                const int q = __builtin_ctz(any);
                any &= any - 1;
                const float v = acc[ib][jb][q];
                if (v <= thr) emit(CW * wj + 32 * jb + 8 * (q >> 2) + 4 * (lane >> 5) + (q & 3), v);
            }
        }
    };
    auto scan_col = [&](int jb, uint32_t bits, auto emit) {
        bits = __builtin_amdgcn_readfirstlane(bits);
        while (bits) {
            const int jc = __builtin_ctz(bits);  // column within the 32-block
            bits &= bits - 1;
            const int q = ((jc >> 3) << 2) | (jc & 3);
            const bool mine = (lane >> 5) == ((jc >> 2) & 1);
            float v[NIB];
#pragma unroll
            for (int ib = 0; ib < NIB; ++ib) v[ib] = acc[ib][jb][q];
            emit(CW * wj + 32 * jb + jc, v, mine);
        }
    };
#pragma unroll
    for (int ib = 0; ib < NIB; ++ib) {
        const int il = RW * wi + 32 * ib + (lane & 31);
        const bool hot = S.rhot[il] & 1;
        if (!__ballot(hot)) continue;
        const int64_t i = S.rid[il];
        const float r_thr = __uint_as_float(S.rmin[il]), r_et = S.rE[il];
        // (an element above this bound has lower_of(v, E_tile) > thr)
        const float r_cheap = hot ? (r_thr + r_et) * (1.0f + 0x1p-18f) : -SCR_INF;
        scan_row(ib, r_cheap, [&](int jl, float v) { stage_cap(i, S.cid[jl], v, r_thr, r_et); });
    }
    // columns: this wave's CW columns are bits [CW wj, +CW) of the hot set
#pragma unroll
    for (int jb = 0; jb < NJB; ++jb)
        scan_col(jb, S.chot[(CW * wj) / 32 + jb], [&](int jl, const float (&v)[NIB], bool mine) {
            const int64_t j = S.cid[jl];
            const float c_thr = __uint_as_float(S.cmin[jl]), c_et = S.cE[jl];
            const float c_cheap = (c_thr + c_et) * (1.0f + 0x1p-18f);
#pragma unroll
            for (int ib = 0; ib < NIB; ++ib)
                if (mine && v[ib] <= c_cheap)
                    stage_cap(j, S.rid[RW * wi + 32 * ib + (lane & 31)], v[ib], c_thr, c_et);
        });

    // ---- epilogue 4: neighbour lists (rows, then columns, whose tile minimum
    // reaches their list threshold), staged in the first staging buffer and
    // appended after the barrier like the candidates.
    if constexpr (LIST) {
        int32_t *lp = reinterpret_cast<int32_t *>(RR ? xstage : stage0);
        int32_t *lo = lp + LIST_STAGE;
        float *lvv = reinterpret_cast<float *>(lo + LIST_STAGE);
        auto stage = [&](int64_t p, int32_t other, float v) {
            v = __int_as_float(max(__float_as_int(v), 0));
            const int pos = atomicAdd(&S.nlist, 1);
            if (pos < LIST_STAGE) {
                lp[pos] = (int32_t)p;
                lo[pos] = other;
                lvv[pos] = v;
            } else {
                list_push_global(A, p, other, v);
            }
        };
#pragma unroll
        for (int ib = 0; ib < NIB; ++ib) {
            const int il = RW * wi + 32 * ib + (lane & 31);
            const bool lst = S.rhot[il] & 2;
            if (!__ballot(lst)) continue;
            const int64_t i = S.rid[il];
            const float tau = lst ? A.pltau[I0 + il] : -SCR_INF;
            scan_row(ib, tau, [&](int jl, float v) { stage(i, S.cid[jl], v); });
        }
        // columns: every element against its own column's threshold (from
        // LDS), one compare per element as for the rows, instead of a walk
        // over the flagged columns
#pragma unroll
        for (int jb = 0; jb < NJB; ++jb) {
            if (!S.clst[(CW * wj) / 32 + jb]) continue;
            const int cb = CW * wj + 32 * jb + 4 * (lane >> 5);  // + 8 (q / 4) + q mod 4: the lane's column q
#pragma unroll
            for (int ib = 0; ib < NIB; ++ib) {
                uint32_t any = 0;
#pragma unroll
                for (int q = 0; q < 16; ++q)
                    if (__ballot(acc[ib][jb][q] <= S.csq[cb + 8 * (q >> 2) + (q & 3)])) any |= 1u << q;
                if (!any) continue;
                const int64_t irow = S.rid[RW * wi + 32 * ib + (lane & 31)];
                while (any) {
                    const int q = __builtin_ctz(any);
                    any &= any - 1;
                    const int jl = cb + 8 * (q >> 2) + (q & 3);
                    const float v = acc[ib][jb][q];
                    if (v <= S.csq[jl]) stage(S.cid[jl], irow, v);
                }
            }
        }
    }
    __syncthreads();
    {
        const int cnt = min(S.ncap, CAP_STAGE);
#pragma unroll 1
        for (int e = tid; e < cnt; e += 64 * NW) commit(cp[e], co[e], cv[e]);
    }
    if constexpr (LIST) {
        const int32_t *lp = reinterpret_cast<const int32_t *>(RR ? xstage : stage0);
        const int32_t *lo = lp + LIST_STAGE;
        const float *lvv = reinterpret_cast<const float *>(lo + LIST_STAGE);
        const int cnt = min(S.nlist, LIST_STAGE);
#pragma unroll 1
        for (int e = tid; e < cnt; e += 64 * NW) list_push_global(A, lp[e], lo[e], lvv[e]);
    }
}

}  // namespace

int64_t pair_tile() { return PT; }

// Tile pairs (I <= J) of nt tiles: the nt diagonal pairs first, then the
// others in blocks of PAIR_SB x PAIR_SB tiles, within a block row-major.  The
// blocks go block row by block row (each by block column), or, with `band`,
// band by band (bj - bi = 0, 1, ...; each by block row): with tiles of nearby
// points the pairs of near tiles, which set most running minima, come first.
// Written on the device: one thread per diagonal pair, and one per block pair
// (bi, bj), bi <= bj, which finds its offset from the counts before it.
__global__ void k_pair_order(int64_t nt, int band, int2 *__restrict__ out) {
    constexpr int64_t SB = PAIR_SB;
    const int64_t nb = (nt + SB - 1) / SB;
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < nt) out[q] = make_int2((int)q, (int)q);
    const int64_t bi = q / nb, bj = q - bi * nb;
    if (bi >= nb || bj < bi) return;
    auto sz = [&](int64_t b) { return std::min<int64_t>(SB, nt - b * SB); };
    auto end = [&](int64_t b) { return std::min<int64_t>(nt, (b + 1) * SB); };
    int64_t off = nt;
    if (band) {
        // band 0 holds nb - 1 full diagonal blocks and the last one; band x > 0
        // holds nb - 1 - x full blocks and one against the last block row
        const int64_t sl = sz(nb - 1), dl = bj - bi;
        for (int64_t x = 0; x < dl; ++x)
            off += x == 0 ? (nb - 1) * (SB * (SB - 1) / 2) + sl * (sl - 1) / 2 : (nb - 1 - x) * SB * SB + SB * sl;
        off += bi * (dl == 0 ? SB * (SB - 1) / 2 : SB * SB);
    } else {
        for (int64_t b = 0; b < bi; ++b) off += sz(b) * (sz(b) - 1) / 2 + sz(b) * (nt - end(b));
        if (bj > bi) off += sz(bi) * (sz(bi) - 1) / 2 + sz(bi) * (std::min<int64_t>(nt, bj * SB) - end(bi));
    }
    for (int64_t I = bi * SB; I < end(bi); ++I)
        for (int64_t J = bj * SB; J < end(bj); ++J)
            if (I < J) out[off++] = make_int2((int)I, (int)J);
}

void launch_pair_order(int64_t nt, int2 *out, hipStream_t s, bool band) {
    const int64_t nb = (nt + PAIR_SB - 1) / PAIR_SB;
    const int64_t threads = std::max<int64_t>(nt, nb * nb);
    hipLaunchKernelGGL(k_pair_order, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, s, nt, band ? 1 : 0, out);
    LAUNCH_CHECK();
}

namespace {

template <int REP>
void launch_pairs(const ScreenArgs &A, const int2 *pairs, int64_t nmask, int64_t noff, hipStream_t s) {
    ISO_REQUIRE(A.d_pad % PPrec<REP>::KC == 0, ISO_ERR_INTERNAL, "padded dimension is not a whole number of chunks");
    ISO_REQUIRE(A.d > A.d_pad - PPrec<REP>::KC && A.d <= A.d_pad, ISO_ERR_INTERNAL, "dimension %lld outside the last chunk of %lld",
                (long long)A.d, (long long)A.d_pad);
    ISO_REQUIRE(A.perm != nullptr, ISO_ERR_INTERNAL, "tile-pair screen without a tile order");
    ISO_REQUIRE(A.psq && A.pcomp && A.pEmax && A.prn && A.pre && A.trmax && A.temax && A.ccnt && A.rn && A.re,
                ISO_ERR_INTERNAL, "tile-pair screen without its per-position inputs");
    ISO_REQUIRE(A.bestc != nullptr || A.pbest != nullptr, ISO_ERR_INTERNAL, "tile-pair screen without its minima");
    ISO_REQUIRE(A.ub == nullptr || A.pub != nullptr, ISO_ERR_INTERNAL, "pair bounds without their minima");
    ISO_REQUIRE(A.lcnt == nullptr || (A.pltau && A.ldrop && A.lj && A.lv), ISO_ERR_INTERNAL,
                "neighbour lists without their arrays");
    ISO_REQUIRE(A.bestc == nullptr || (A.tcomp && A.upair && A.gcj && A.gcl), ISO_ERR_INTERNAL,
                "final round without its arrays");
    ISO_REQUIRE(A.bestc != nullptr || (A.cj && A.cl), ISO_ERR_INTERNAL, "tile-pair screen without candidate lists");
    ISO_REQUIRE(A.rep != ISO_PREC_INT8 || A.psqi != nullptr, ISO_ERR_INTERNAL, "INT8 screen without integer norms");
    const dim3 block(64 * NW);
    auto grid = [](int64_t per_xcd) { return dim3((unsigned)(8 * per_xcd)); };
    const bool list = A.lcnt != nullptr, final_round = A.bestc != nullptr, pb = A.ub != nullptr;
    ISO_REQUIRE(!(final_round && (list || nmask > 0)), ISO_ERR_INTERNAL, "final round with lists or masked pairs");
    ISO_REQUIRE(!pb || (REP == ISO_PREC_BF16 && !list && !final_round), ISO_ERR_INTERNAL,
                "pair bounds only in plain BF16 rounds");
    // the unmasked tile pairs, two halves each ...
    if (noff > 0) {
        const int64_t items = 2 * noff, per_xcd = (items + 7) / 8;
        if (final_round)
            hipLaunchKernelGGL((k_screen_pairs<REP, false, MODE_FINAL>), grid(per_xcd), block, 0, s, A, pairs + nmask,
                               per_xcd, items);
        else if (list)
            hipLaunchKernelGGL((k_screen_pairs<REP, false, MODE_LIST>), grid(per_xcd), block, 0, s, A, pairs + nmask,
                               per_xcd, items);
        else if (pb)
            hipLaunchKernelGGL((k_screen_pairs<REP, false, MODE_PLAIN, REP == ISO_PREC_BF16>), grid(per_xcd), block, 0,
                               s, A, pairs + nmask, per_xcd, items);
        else
            hipLaunchKernelGGL((k_screen_pairs<REP, false, MODE_PLAIN>), grid(per_xcd), block, 0, s, A, pairs + nmask,
                               per_xcd, items);
        LAUNCH_CHECK();
    }
    // ... then the masked tile pairs (on the diagonal only i < j counted), two
    // halves each: a small launch, run after the large one, when most points'
    // running minima are already low, so that few of its rows are flagged
    if (nmask > 0) {
        const int64_t items = 2 * nmask, per_xcd = (items + 7) / 8;
        if (list)
            hipLaunchKernelGGL((k_screen_pairs<REP, true, MODE_LIST>), grid(per_xcd), block, 0, s, A, pairs, per_xcd,
                               items);
        else if (pb)
            hipLaunchKernelGGL((k_screen_pairs<REP, true, MODE_PLAIN, REP == ISO_PREC_BF16>), grid(per_xcd), block, 0,
                               s, A, pairs, per_xcd, items);
        else
            hipLaunchKernelGGL((k_screen_pairs<REP, true, MODE_PLAIN>), grid(per_xcd), block, 0, s, A, pairs, per_xcd,
                               items);
        LAUNCH_CHECK();
    }
}

}  // namespace

void launch_screen_pairs(const ScreenArgs &A, const int2 *pairs, int64_t nmask, int64_t noff, hipStream_t s) {
    if (A.rep == ISO_PREC_BF16)
        launch_pairs<ISO_PREC_BF16>(A, pairs, nmask, noff, s);
    else if (A.rep == ISO_PREC_FP8)
        launch_pairs<ISO_PREC_FP8>(A, pairs, nmask, noff, s);
    else if (A.rep == ISO_PREC_INT8)
        launch_pairs<ISO_PREC_INT8>(A, pairs, nmask, noff, s);
    else
        launch_pairs<ISO_PREC_FP32>(A, pairs, nmask, noff, s);
}

}  // namespace iso
