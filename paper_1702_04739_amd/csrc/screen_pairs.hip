// screen_pairs.hip -- symmetric Boruvka screen over tile pairs (gfx950 MFMA).
//
// The points are cut into tiles of PT = 256.  One workgroup handles one tile
// pair (I, J) with I <= J, so every unordered pair of points is formed once:
// the Gram tile G = X'_J X'_I^T is accumulated on MFMA (FP32 accumulate), then
//   Dhat^2 = s_i + s_j - 2 G  (masked: valid points, different components,
//                              and i < j on the diagonal tile pairs)
// updates both sides: the running minimum of every row i of I (over the
// tile's columns) and of every column j of J (over the tile's rows) is merged
// into a global per-point minimum with one atomic min per point and tile, and
// every element whose lower bound can still beat that point's minimum is
// appended to the point's global candidate list (screen.hpp gives the bound).
// Lists are append-only: an entry stays even when a later minimum rules it
// out (the recheck filters it), and a point whose list overflows is re-screened
// by the row-sweep kernel starting from its final minimum.
//
// Tile pairs are enumerated in blocks of SB x SB tiles, and each XCD receives a
// contiguous run of that order (workgroup ids are dealt to the eight XCDs in
// turn), so the workgroups resident on one XCD share their I and J tiles in
// its L2.
//
// Workgroup: 8 waves; wave (wi, wj) computes rows i in [128 wi, +128) x
// columns j in [64 wj, +64) as 4 x 2 blocks of the transposed 32 x 32 MFMA
// (MFMA rows = columns j, MFMA columns = rows i; result register q of lane l
// is MFMA row 8 (q div 4) + 4 (l div 32) + (q mod 4), MFMA column l mod 32).
#include <vector>

#include "screen.hpp"

namespace iso {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx16 __attribute__((ext_vector_type(16)));

constexpr int PT = 256;     // points per tile
constexpr int NSTAGE = 4;   // LDS stages of the K pipeline (loads run NSTAGE-1 chunks ahead)

// s_waitcnt immediate waiting for vmcnt <= n (expcnt and lgkmcnt left at their maxima)
#define VMCNT(n) (((n) & 0xF) | (((n) >> 4) << 14) | (0x7 << 4) | (0xF << 8))

template <bool BF16>
struct PPrec;

template <>
struct PPrec<true> {
    using T = uint16_t;
    static constexpr int KC = 32;
    static constexpr int LDK = KC + 8;
    static constexpr int KSTEP = 16;
    static constexpr int VEC = 8;
};

template <>
struct PPrec<false> {
    using T = float;
    static constexpr int KC = 16;
    static constexpr int LDK = KC + 4;
    static constexpr int KSTEP = 2;
    static constexpr int VEC = 1;
};

struct PairLDS {
    uint32_t rmin[PT], cmin[PT];   // tile minima of rows (I) and columns (J)
    float rthr[PT], cthr[PT];      // current global minima after the merge
    float rE[PT], cE[PT];          // Emax of the tile's rows and columns
    float csq[PT], crn[PT], cre[PT];
    int32_t ccomp[PT];
    float rrn[PT], rre[PT];
    uint32_t chot[PT / 32];        // bit set: column's tile minimum is within its capture margin
    int32_t rhot[PT];              // row's tile minimum is within its capture margin
};

// Minimum over the 32 lanes of each half wave (every lane receives it): DPP
// min within quads, 8-lane and 16-lane rows, then one swap across the rows.
__device__ __forceinline__ float min32(float v) {
    v = fminf(v, __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0xB1, 0xF, 0xF, false)));   // quad xor 1
    v = fminf(v, __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x4E, 0xF, 0xF, false)));   // quad xor 2
    v = fminf(v, __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x141, 0xF, 0xF, false)));  // half-row mirror
    v = fminf(v, __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x140, 0xF, 0xF, false)));  // row mirror
    return fminf(v, __shfl_xor(v, 16, 64));
}

template <bool BF16>
__global__ __launch_bounds__(512, 1) void k_screen_pairs(ScreenArgs A, const int2 *__restrict__ pairs,
                                                         int64_t per_xcd, int64_t npairs) {
    using P = PPrec<BF16>;
    using T = typename P::T;
    __shared__ PairLDS S;
    // NSTAGE staging buffers of one K chunk: rows 0..255 = tile J (columns j),
    // rows 256..511 = tile I (rows i); 64 bytes per row in four 16-byte slots,
    // slot (row, part) at row * 4 + (part xor ((row >> 2) & 3)), which makes
    // the MFMA fragment reads (16 consecutive rows, one part) bank-conflict free.
    __shared__ __attribute__((aligned(16))) uint4 stage0[2 * PT * 4];
    __shared__ __attribute__((aligned(16))) uint4 stage1[2 * PT * 4];
    __shared__ __attribute__((aligned(16))) uint4 stage2[2 * PT * 4];
    __shared__ __attribute__((aligned(16))) uint4 stage3[2 * PT * 4];

    // XCD-aware placement: workgroup b runs on XCD b mod 8
    const int64_t b = blockIdx.x;
    const int64_t idx = (b & 7) * per_xcd + (b >> 3);
    if (idx >= npairs) return;
    const int2 pr = pairs[idx];
    const int64_t I0 = (int64_t)pr.x * PT, J0 = (int64_t)pr.y * PT;
    const bool diag = pr.x == pr.y;

    const int tid = threadIdx.x;
    const int lane = tid & 63, w = tid >> 6;
    const int wi = w >> 2, wj = w & 3;  // wi in 0..1 (128 rows), wj in 0..3 (64 columns)
    const T *X = BF16 ? reinterpret_cast<const T *>(A.XB) : reinterpret_cast<const T *>(A.XT);
    const int64_t d_pad = A.d_pad;

    // tile constants
    if (tid < PT) {
        const int64_t i = I0 + tid, j = J0 + tid;
        S.rmin[tid] = __float_as_uint(SCR_INF);
        S.cmin[tid] = __float_as_uint(SCR_INF);
        S.rE[tid] = i < A.n ? A.Emax[i] : 0.0f;
        S.cE[tid] = j < A.n ? A.Emax[j] : 0.0f;
        S.rrn[tid] = A.rn[i];
        S.rre[tid] = A.re[i];
        S.csq[tid] = A.sq[j];
        S.crn[tid] = A.rn[j];
        S.cre[tid] = A.re[j];
        S.ccomp[tid] = A.comp[j];
    }
    float si[4];
    int ci[4];
#pragma unroll
    for (int ib = 0; ib < 4; ++ib) {
        const int64_t i = I0 + 128 * wi + 32 * ib + (lane & 31);
        si[ib] = A.sq[i];
        ci[ib] = A.comp[i];
    }

    // asynchronous staging: each wave moves four 1 KB runs of slots per chunk
    // with global_load_lds_dwordx4 (lane L of a run fills slot base + L)
    constexpr int CHUNK = 16 / sizeof(T);  // elements per slot
    static_assert(P::KC * sizeof(T) == 64, "one K chunk is 64 bytes per row");
    const T *srcp[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int slot = (w * 4 + r) * 64 + lane;
        const int row = slot >> 2;
        const int part = (slot & 3) ^ ((row >> 2) & 3);
        const int64_t g = row < PT ? J0 + row : I0 + (row - PT);
        srcp[r] = X + g * d_pad + part * CHUNK;
    }
    const int nchunks = (int)(d_pad / P::KC);
#define ISO_ISSUE(STG, C)                                                                                     \
    {                                                                                                        \
        _Pragma("unroll") for (int r = 0; r < 4; ++r) __builtin_amdgcn_global_load_lds(                     \
            (const void *)(srcp[r] + (int64_t)(C) * P::KC),                                                  \
            (__attribute__((address_space(3))) void *)&STG[(w * 4 + r) * 64], 16, 0, 0);                   \
    }

    floatx16 acc[4][2];
#pragma unroll
    for (int ib = 0; ib < 4; ++ib)
#pragma unroll
        for (int jb = 0; jb < 2; ++jb)
#pragma unroll
            for (int q = 0; q < 16; ++q) acc[ib][jb][q] = 0.0f;

    // fragment slot of (operand row, k offset in elements) in a stage
    auto frag_slot = [](int row, int kel) {
        const int part = (kel * (int)sizeof(T)) >> 4;
        return row * 4 + (part ^ ((row >> 2) & 3));
    };

    // One pipeline step on chunk C held in stage SB: wait for it (chunks C+1, C+2
    // may stay in flight), barrier (no fence: the DMA data is in LDS once the
    // issuing wave's vmcnt has dropped), refill stage SN with chunk C+3, compute.
#define ISO_STEP(SB, SN, C)                                                                                   \
    if ((C) < nchunks) {                                                                                     \
        if ((C) + 2 < nchunks)                                                                               \
            __builtin_amdgcn_s_waitcnt(VMCNT(8));                                                            \
        else if ((C) + 1 < nchunks)                                                                          \
            __builtin_amdgcn_s_waitcnt(VMCNT(4));                                                            \
        else                                                                                                 \
            __builtin_amdgcn_s_waitcnt(VMCNT(0));                                                            \
        __builtin_amdgcn_s_barrier();                                                                        \
        if ((C) + 3 < nchunks) ISO_ISSUE(SN, (C) + 3)                                                        \
        ISO_COMPUTE(SB)                                                                                      \
    }

    if constexpr (BF16) {
#define ISO_COMPUTE(SB)                                                                                       \
    _Pragma("unroll") for (int ks = 0; ks < P::KC; ks += P::KSTEP) {                                          \
        const int kel = ks + (lane >> 5) * P::VEC;                                                             \
        bf16x8 a[2], bb[4];                                                                                   \
        _Pragma("unroll") for (int jb = 0; jb < 2; ++jb) {                                                    \
            const uint4 v = SB[frag_slot(64 * wj + 32 * jb + (lane & 31), kel)];                               \
            a[jb] = *reinterpret_cast<const bf16x8 *>(&v);                                                    \
        }                                                                                                     \
        _Pragma("unroll") for (int ib = 0; ib < 4; ++ib) {                                                    \
            const uint4 v = SB[frag_slot(PT + 128 * wi + 32 * ib + (lane & 31), kel)];                         \
            bb[ib] = *reinterpret_cast<const bf16x8 *>(&v);                                                   \
        }                                                                                                     \
        _Pragma("unroll") for (int ib = 0; ib < 4; ++ib) _Pragma("unroll") for (int jb = 0; jb < 2; ++jb)     \
            acc[ib][jb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[jb], bb[ib], acc[ib][jb], 0, 0, 0);        \
    }
        if (0 < nchunks) ISO_ISSUE(stage0, 0)
        if (1 < nchunks) ISO_ISSUE(stage1, 1)
        if (2 < nchunks) ISO_ISSUE(stage2, 2)
        for (int c = 0; c < nchunks; c += 4) {
            ISO_STEP(stage0, stage3, c)
            ISO_STEP(stage1, stage0, c + 1)
            ISO_STEP(stage2, stage1, c + 2)
            ISO_STEP(stage3, stage2, c + 3)
        }
#undef ISO_COMPUTE
    } else {
#define ISO_COMPUTE(SB)                                                                                       \
    _Pragma("unroll") for (int ks = 0; ks < P::KC; ks += P::KSTEP) {                                          \
        const int kel = ks + (lane >> 5) * P::VEC;                                                             \
        const float *sf = reinterpret_cast<const float *>(SB);                                                \
        const int within = kel & 3;                                                                           \
        float a[2], bb[4];                                                                                    \
        _Pragma("unroll") for (int jb = 0; jb < 2; ++jb) a[jb] =                                              \
            sf[frag_slot(64 * wj + 32 * jb + (lane & 31), kel) * 4 + within];                                  \
        _Pragma("unroll") for (int ib = 0; ib < 4; ++ib) bb[ib] =                                             \
            sf[frag_slot(PT + 128 * wi + 32 * ib + (lane & 31), kel) * 4 + within];                            \
        _Pragma("unroll") for (int ib = 0; ib < 4; ++ib) _Pragma("unroll") for (int jb = 0; jb < 2; ++jb)     \
            acc[ib][jb] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[jb], bb[ib], acc[ib][jb], 0, 0, 0);           \
    }
        if (0 < nchunks) ISO_ISSUE(stage0, 0)
        if (1 < nchunks) ISO_ISSUE(stage1, 1)
        if (2 < nchunks) ISO_ISSUE(stage2, 2)
        for (int c = 0; c < nchunks; c += 4) {
            ISO_STEP(stage0, stage3, c)
            ISO_STEP(stage1, stage0, c + 1)
            ISO_STEP(stage2, stage1, c + 2)
            ISO_STEP(stage3, stage2, c + 3)
        }
#undef ISO_COMPUTE
    }
#undef ISO_STEP
#undef ISO_ISSUE
    __syncthreads();  // all DMA traffic retired before LDS is reused by the epilogue

    // ---- epilogue 1: masked Dhat^2 (padding has s = +inf), tile minima of rows
    // (in-lane over the lane's 32 columns, then lanes l, l+32) and of columns
    // (in-lane over the lane's 4 rows, then the 32 lanes of the half wave)
    {
        float m[4] = {SCR_INF, SCR_INF, SCR_INF, SCR_INF};
#pragma unroll
        for (int jb = 0; jb < 2; ++jb)
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                const int jl = 64 * wj + 32 * jb + 8 * (q >> 2) + 4 * (lane >> 5) + (q & 3);
                const float sj = S.csq[jl];
                const int cjj = S.ccomp[jl];
                float cmin = SCR_INF;
#pragma unroll
                for (int ib = 0; ib < 4; ++ib) {
                    const float t = fmaxf(fmaf(-2.0f, acc[ib][jb][q], si[ib] + sj), 0.0f);
                    float v = (cjj == ci[ib]) ? SCR_INF : t;
                    if (diag && jl <= 128 * wi + 32 * ib + (lane & 31)) v = SCR_INF;  // each pair once
                    acc[ib][jb][q] = v;
                    m[ib] = fminf(m[ib], v);
                    cmin = fminf(cmin, v);
                }
                const float v = min32(cmin);
                if (((16 * jb + q) & 31) == (lane & 31) && v < SCR_INF) atomicMin(&S.cmin[jl], __float_as_uint(v));
                if ((q & 3) == 3) __builtin_amdgcn_sched_barrier(0);  // bound the columns in flight
            }
#pragma unroll
        for (int ib = 0; ib < 4; ++ib) {
            const float mm = fminf(m[ib], __shfl_xor(m[ib], 32, 64));  // lanes l and l+32 hold the same rows
            if ((lane >> 5) == 0 && mm < SCR_INF)
                atomicMin(&S.rmin[128 * wi + 32 * ib + (lane & 31)], __float_as_uint(mm));
        }
    }
    __syncthreads();

    // ---- epilogue 2: merge into the global minima; thresholds from the merged
    // values; flag the rows and columns whose tile minimum can still be captured
    if (tid < PT / 32) S.chot[tid] = 0u;
    __syncthreads();
    {
        const int t = tid & (PT - 1);
        const bool is_row = tid < PT;
        const int64_t p = (is_row ? I0 : J0) + t;
        float cur = SCR_INF;
        const uint32_t m = is_row ? S.rmin[t] : S.cmin[t];
        if (p < A.n) {
            uint32_t old = reinterpret_cast<const volatile uint32_t *>(A.best)[p];
            if (m < old) old = atomicMin(reinterpret_cast<uint32_t *>(A.best) + p, m);  // only when it can lower it
            cur = __uint_as_float(old < m ? old : m);
        }
        const float E = is_row ? S.rE[t] : S.cE[t];
        const bool hot = p < A.n && __uint_as_float(m) <= (cur + 2.0f * E) * A.kappa;
        if (is_row) {
            S.rthr[t] = cur;
            S.rhot[t] = hot ? 1 : 0;
        } else {
            S.cthr[t] = cur;
            if (hot) atomicOr(&S.chot[t >> 5], 1u << (t & 31));
        }
    }
    __syncthreads();

    // ---- epilogue 3: capture candidates (rows of hot rows, columns of hot columns)
#pragma unroll
    for (int ib = 0; ib < 4; ++ib) {
        const int il = 128 * wi + 32 * ib + (lane & 31);
        if (!S.rhot[il]) continue;
        const int64_t i = I0 + il;
        const float Ei = S.rE[il];
        const float rb_ = S.rthr[il];
        const float r_cheap = (rb_ + 2.0f * Ei) * A.kappa;
        const float r_thr = (rb_ + Ei) * A.kappa;
        const float ri = S.rrn[il], ei = S.rre[il];
#pragma unroll
        for (int jb = 0; jb < 2; ++jb)
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                const float v = acc[ib][jb][q];
                if (!(v <= r_cheap)) continue;
                const int jl = 64 * wj + 32 * jb + 8 * (q >> 2) + 4 * (lane >> 5) + (q & 3);
                const float L = lower_of(v, pair_bound(A.bound, ri, S.crn[jl], ei, S.cre[jl]));
                if (!(L <= r_thr)) continue;
                const int pos = atomicAdd(&A.ccnt[i], 1);
                if (pos < SCR_CAP) {
                    A.cj[i * SCR_CAP + pos] = (int32_t)(J0 + jl);
                    A.cl[i * SCR_CAP + pos] = L;
                }
                __builtin_amdgcn_sched_barrier(0);
            }
    }
    // columns: this wave's 64 columns are bits [64 wj, +64) of the hot set
    const uint32_t h0 = S.chot[2 * wj + 0], h1 = S.chot[2 * wj + 1];
    if (h0 | h1) {
#pragma unroll
        for (int jb = 0; jb < 2; ++jb) {
            const uint32_t hw = jb == 0 ? h0 : h1;
            if (!hw) continue;
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                const int jc = 8 * (q >> 2) + 4 * (lane >> 5) + (q & 3);  // column within the 32-block
                if (!((hw >> jc) & 1u)) continue;
                const int jl = 64 * wj + 32 * jb + jc;
                const int64_t j = J0 + jl;
                const float Ej = S.cE[jl];
                const float cb = S.cthr[jl];
                const float c_cheap = (cb + 2.0f * Ej) * A.kappa;
                const float c_thr = (cb + Ej) * A.kappa;
#pragma unroll
                for (int ib = 0; ib < 4; ++ib) {
                    const float v = acc[ib][jb][q];
                    if (!(v <= c_cheap)) continue;
                    const int il = 128 * wi + 32 * ib + (lane & 31);
                    const float L = lower_of(v, pair_bound(A.bound, S.rrn[il], S.crn[jl], S.rre[il], S.cre[jl]));
                    if (!(L <= c_thr)) continue;
                    const int pos = atomicAdd(&A.ccnt[j], 1);
                    if (pos < SCR_CAP) {
                        A.cj[j * SCR_CAP + pos] = (int32_t)(I0 + il);
                        A.cl[j * SCR_CAP + pos] = L;
                    }
                    __builtin_amdgcn_sched_barrier(0);
                }
            }
        }
    }
}

}  // namespace

int64_t pair_tile() { return PT; }

// Tile pairs (I <= J) of nt tiles in blocks of SB x SB tiles.
std::vector<int2> make_pair_order(int64_t nt) {
    constexpr int64_t SB = 4;
    std::vector<int2> out;
    out.reserve((size_t)(nt * (nt + 1) / 2));
    const int64_t nb = (nt + SB - 1) / SB;
    for (int64_t bi = 0; bi < nb; ++bi)
        for (int64_t bj = bi; bj < nb; ++bj)
            for (int64_t I = bi * SB; I < (bi + 1) * SB && I < nt; ++I)
                for (int64_t J = bj * SB; J < (bj + 1) * SB && J < nt; ++J)
                    if (I <= J) out.push_back(make_int2((int)I, (int)J));
    return out;
}

void launch_screen_pairs(const ScreenArgs &A, const int2 *pairs, int64_t npairs, bool bf16, hipStream_t s) {
    const int64_t per_xcd = (npairs + 7) / 8;
    const unsigned blocks = (unsigned)(per_xcd * 8);
    if (bf16)
        hipLaunchKernelGGL(k_screen_pairs<true>, dim3(blocks), dim3(512), 0, s, A, pairs, per_xcd, npairs);
    else
        hipLaunchKernelGGL(k_screen_pairs<false>, dim3(blocks), dim3(512), 0, s, A, pairs, per_xcd, npairs);
    LAUNCH_CHECK();
}

}  // namespace iso
