// screen_mfma.hip -- Boruvka screen on the matrix cores (gfx950).
//
// Each workgroup owns SCR_ROWS rows (points i) and sweeps a range of column
// tiles (points j), forming the Gram tile G = X'_I X'_J^T on MFMA with FP32
// accumulation, then the masked Dhat^2 = s_i + s_j - 2 G, a running minimum per
// row and the capture of near-minimal columns (screen.hpp).  The n x n
// distance matrix is never stored: each tile lives in accumulators only.
//
// The MFMA is issued transposed (MFMA rows = columns j, MFMA columns = rows
// i), so that each lane of the 32 x 32 result holds one row i and sixteen
// columns j: the row state stays in registers and the column constants are
// broadcast from LDS.
//   BF16: v_mfma_f32_32x32x16_bf16, lane l supplies row (l mod 32), k = 8 (l div 32) .. +7
//   FP32: v_mfma_f32_32x32x2_f32,    lane l supplies row (l mod 32), k = l div 32
//   result register q of lane l: MFMA row 8 (q div 4) + 4 (l div 32) + (q mod 4), MFMA column l mod 32.
//   FP8:  v_mfma_scale_f32_32x32x64_f8f6f4 (E4M3, unit block scales), lane l supplies row (l mod 32),
//         k = 32 (l div 32) .. +31
//   INT8: v_mfma_i32_32x32x32_i8, lane l supplies row (l mod 32), k = 16 (l div 32) .. +15 (int32
//         accumulators kept bit for bit in the FP32 accumulator registers)
// Workgroup: 4 waves in a 2 x 2 grid, each wave a 64 x 64 sub-tile (2 x 2 MFMA blocks).
#include "screen.hpp"

namespace iso {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef int intx8 __attribute__((ext_vector_type(8)));
typedef int intx4 __attribute__((ext_vector_type(4)));
typedef int intx16 __attribute__((ext_vector_type(16)));
typedef float floatx16 __attribute__((ext_vector_type(16)));

template <int REP>
struct Prec;

template <>
struct Prec<ISO_PREC_BF16> {
    using T = uint16_t;                       // bf16 bits
    static constexpr int KC = 32;             // K elements per LDS stage
    static constexpr int LDK = KC + 8;        // padded LDS row (elements)
    static constexpr int KSTEP = 16;          // K per MFMA
    static constexpr int VEC = 8;             // elements per lane per operand
};

template <>
struct Prec<ISO_PREC_FP8> {
    using T = uint8_t;                        // E4M3 bytes
    static constexpr int KC = 64;
    static constexpr int LDK = KC + 16;
    static constexpr int KSTEP = 64;
    static constexpr int VEC = 32;
};

template <>
struct Prec<ISO_PREC_INT8> {
    using T = int8_t;                         // integer coordinates
    static constexpr int KC = 64;
    static constexpr int LDK = KC + 16;
    static constexpr int KSTEP = 32;
    static constexpr int VEC = 16;
};

template <>
struct Prec<ISO_PREC_FP32> {
    using T = float;
    static constexpr int KC = 16;
    static constexpr int LDK = KC + 4;
    static constexpr int KSTEP = 2;
    static constexpr int VEC = 1;
};

template <int REP, bool GATHER>
__global__ __launch_bounds__(256, 2) void k_screen_mfma(ScreenArgs A) {
    using P = Prec<REP>;
    using T = typename P::T;
    __shared__ ScreenLDS S;
    __shared__ __attribute__((aligned(16))) T As[2][SCR_COLS * P::LDK];  // column points j (double buffer)
    __shared__ __attribute__((aligned(16))) T Bs[2][SCR_ROWS * P::LDK];  // row points i

    const int tid = threadIdx.x;
    const int lane = tid & 63, w = tid >> 6;
    const int wi = w >> 1, wj = w & 1;
    const int64_t i0 = (int64_t)blockIdx.x * SCR_ROWS;
    const T *X = REP == ISO_PREC_BF16   ? reinterpret_cast<const T *>(A.XB)
                 : REP == ISO_PREC_FP8  ? reinterpret_cast<const T *>(A.XF8)
                 : REP == ISO_PREC_INT8 ? reinterpret_cast<const T *>(A.XI8)
                                        : reinterpret_cast<const T *>(A.XT);
    const int64_t d_pad = A.d_pad;
    const bool pb = REP == ISO_PREC_BF16 && A.ub != nullptr;  // pair bounds

    screen_init_rows<GATHER>(S, A, i0);

    // this lane's two rows (local index, global index, constants)
    int rl[2];
    int64_t gi[2];
    float si[2], ri[2], ei[2];
    int ci[2];
    int32_t sii[2];  // INT8: exact integer squared norms
#pragma unroll
    for (int ib = 0; ib < 2; ++ib) {
        rl[ib] = 64 * wi + 32 * ib + (lane & 31);
        int64_t i;
        if (GATHER) {
            const int64_t slot = i0 + rl[ib];
            i = slot < A.nrows ? A.rows[slot] : -1;
        } else {
            i = i0 + rl[ib] < A.n ? i0 + rl[ib] : -1;
        }
        gi[ib] = i;
        si[ib] = i >= 0 ? A.sq[i] : 0.0f;
        ri[ib] = i >= 0 ? A.rn[i] : 0.0f;
        ei[ib] = i >= 0 ? A.re[i] : 0.0f;
        ci[ib] = i >= 0 ? A.comp[i] : -1;
        sii[ib] = (REP == ISO_PREC_INT8 && i >= 0) ? A.sqi[i] : 0;
    }
    // staging: each thread moves LOADS 16-byte pieces of each operand per chunk
    constexpr int CHUNK = 16 / sizeof(T);               // elements per 16-byte load
    constexpr int PARTS = P::KC / CHUNK;                // 16-byte loads per staged row
    constexpr int LOADS = SCR_ROWS * PARTS / 256;       // per thread per operand
    static_assert(LOADS == 2, "staging assumes two pieces per thread and operand");
    const int srow0 = tid / PARTS, spart0 = tid % PARTS;
    const int srow1 = (tid + 256) / PARTS, spart1 = (tid + 256) % PARTS;
    int64_t brow0, brow1;
    if (GATHER) {
        brow0 = i0 + srow0 < A.nrows ? A.rows[i0 + srow0] : -1;
        brow1 = i0 + srow1 < A.nrows ? A.rows[i0 + srow1] : -1;
    } else {
        brow0 = i0 + srow0;
        brow1 = i0 + srow1;
    }
    uint4 ra0, ra1, rb0, rb1;
#define ISO_GLOAD(J0, K0)                                                                                   \
    {                                                                                                      \
        ra0 = *reinterpret_cast<const uint4 *>(X + ((J0) + srow0) * d_pad + (K0) + spart0 * CHUNK);          \
        ra1 = *reinterpret_cast<const uint4 *>(X + ((J0) + srow1) * d_pad + (K0) + spart1 * CHUNK);          \
        rb0 = brow0 >= 0 ? *reinterpret_cast<const uint4 *>(X + brow0 * d_pad + (K0) + spart0 * CHUNK)      \
                         : make_uint4(0, 0, 0, 0);                                                         \
        rb1 = brow1 >= 0 ? *reinterpret_cast<const uint4 *>(X + brow1 * d_pad + (K0) + spart1 * CHUNK)      \
                         : make_uint4(0, 0, 0, 0);                                                         \
    }
#define ISO_SSTORE(BUF)                                                                                     \
    {                                                                                                      \
        *reinterpret_cast<uint4 *>(&As[(BUF)][srow0 * P::LDK + spart0 * CHUNK]) = ra0;                       \
        *reinterpret_cast<uint4 *>(&As[(BUF)][srow1 * P::LDK + spart1 * CHUNK]) = ra1;                       \
        *reinterpret_cast<uint4 *>(&Bs[(BUF)][srow0 * P::LDK + spart0 * CHUNK]) = rb0;                       \
        *reinterpret_cast<uint4 *>(&Bs[(BUF)][srow1 * P::LDK + spart1 * CHUNK]) = rb1;                       \
    }
    // this workgroup's columns
    const int64_t jbeg = (int64_t)blockIdx.y * A.col_split;
    const int64_t jend = jbeg + A.col_split < A.n_pad ? jbeg + A.col_split : A.n_pad;
    ISO_GLOAD(jbeg, 0)
    ISO_SSTORE(0)
    __syncthreads();
    int buf = 0;

    for (int64_t j0 = jbeg; j0 < jend; j0 += SCR_COLS) {
        screen_load_cols(S, A, j0);
        floatx16 acc[2][2];
#pragma unroll
        for (int ib = 0; ib < 2; ++ib)
#pragma unroll
            for (int jb = 0; jb < 2; ++jb)
#pragma unroll
                for (int q = 0; q < 16; ++q) acc[ib][jb][q] = 0.0f;

        for (int64_t k0 = 0; k0 < d_pad; k0 += P::KC) {
            // prefetch the next chunk (of this tile, or the first of the next tile)
            int64_t nj0 = j0, nk0 = k0 + P::KC;
            if (nk0 >= d_pad) {
                nk0 = 0;
                nj0 = j0 + SCR_COLS;
            }
            const bool has_next = nj0 < jend;
            if (has_next) {
                ISO_GLOAD(nj0, nk0)
            }
            const T *Ab = As[buf];
            const T *Bb = Bs[buf];
#pragma unroll
            for (int ks = 0; ks < P::KC; ks += P::KSTEP) {
                const int kofs = ks + (lane >> 5) * P::VEC;
                if constexpr (REP == ISO_PREC_INT8) {
                    intx4 a[2], b[2];
#pragma unroll
                    for (int jb = 0; jb < 2; ++jb)
                        a[jb] = *reinterpret_cast<const intx4 *>(&Ab[(64 * wj + 32 * jb + (lane & 31)) * P::LDK + kofs]);
#pragma unroll
                    for (int ib = 0; ib < 2; ++ib)
                        b[ib] = *reinterpret_cast<const intx4 *>(&Bb[(64 * wi + 32 * ib + (lane & 31)) * P::LDK + kofs]);
#pragma unroll
                    for (int ib = 0; ib < 2; ++ib)
#pragma unroll
                        for (int jb = 0; jb < 2; ++jb)
                            acc[ib][jb] = __builtin_bit_cast(
                                floatx16, __builtin_amdgcn_mfma_i32_32x32x32_i8(
                                              a[jb], b[ib], __builtin_bit_cast(intx16, acc[ib][jb]), 0, 0, 0));
                } else if constexpr (REP == ISO_PREC_FP8) {
                    intx8 a[2], b[2];
#pragma unroll
                    for (int jb = 0; jb < 2; ++jb)
                        a[jb] = *reinterpret_cast<const intx8 *>(&Ab[(64 * wj + 32 * jb + (lane & 31)) * P::LDK + kofs]);
#pragma unroll
                    for (int ib = 0; ib < 2; ++ib)
                        b[ib] = *reinterpret_cast<const intx8 *>(&Bb[(64 * wi + 32 * ib + (lane & 31)) * P::LDK + kofs]);
#pragma unroll
                    for (int ib = 0; ib < 2; ++ib)
#pragma unroll
                        for (int jb = 0; jb < 2; ++jb)
                            acc[ib][jb] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a[jb], b[ib], acc[ib][jb], 0, 0,
                                                                                          0, 0x7F7F7F7F, 0, 0x7F7F7F7F);
                } else if constexpr (REP == ISO_PREC_BF16) {
                    bf16x8 a[2], b[2];
#pragma unroll
                    for (int jb = 0; jb < 2; ++jb)
                        a[jb] = *reinterpret_cast<const bf16x8 *>(&Ab[(64 * wj + 32 * jb + (lane & 31)) * P::LDK + kofs]);
#pragma unroll
                    for (int ib = 0; ib < 2; ++ib)
                        b[ib] = *reinterpret_cast<const bf16x8 *>(&Bb[(64 * wi + 32 * ib + (lane & 31)) * P::LDK + kofs]);
#pragma unroll
                    for (int ib = 0; ib < 2; ++ib)
#pragma unroll
                        for (int jb = 0; jb < 2; ++jb)
                            acc[ib][jb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[jb], b[ib], acc[ib][jb], 0, 0, 0);
                } else {
                    float a[2], b[2];
#pragma unroll
                    for (int jb = 0; jb < 2; ++jb) a[jb] = Ab[(64 * wj + 32 * jb + (lane & 31)) * P::LDK + kofs];
#pragma unroll
                    for (int ib = 0; ib < 2; ++ib) b[ib] = Bb[(64 * wi + 32 * ib + (lane & 31)) * P::LDK + kofs];
#pragma unroll
                    for (int ib = 0; ib < 2; ++ib)
#pragma unroll
                        for (int jb = 0; jb < 2; ++jb)
                            acc[ib][jb] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[jb], b[ib], acc[ib][jb], 0, 0, 0);
                }
            }
            if (has_next) {
                ISO_SSTORE(buf ^ 1)
            }
            __syncthreads();
            buf ^= 1;
        }

        // phase A: masked Dhat^2 and the row minima (pair bounds: also each
        // element's own bound E_ij, the row's least Dhat^2 + E_ij, and the
        // element's lower bound kept in place of Dhat^2 for phase B)
#pragma unroll
        for (int ib = 0; ib < 2; ++ib) {
            float m = SCR_INF, mu = SCR_INF;
#pragma unroll
            for (int jb = 0; jb < 2; ++jb)
#pragma unroll
                for (int q = 0; q < 16; ++q) {
                    const int jl = 64 * wj + 32 * jb + 8 * (q >> 2) + 4 * (lane >> 5) + (q & 3);
                    float v;
                    if constexpr (REP == ISO_PREC_INT8) {
                        const uint32_t d2 = (uint32_t)sii[ib] + (uint32_t)S.csqi[jl] -
                                            2u * (uint32_t)__float_as_int(acc[ib][jb][q]);
                        v = (ci[ib] >= 0 && S.ccomp[jl] >= 0 && S.ccomp[jl] != ci[ib] && d2 < (1u << 30))
                                ? (float)d2 * A.scale2
                                : SCR_INF;
                    } else {
                        v = screen_value(acc[ib][jb][q], si[ib], S.csq[jl], ci[ib], S.ccomp[jl]);
                    }
                    m = fminf(m, v);
                    if (pb) {
                        const float E = pair_bound(A.bound, ri[ib], S.crn[jl], ei[ib], S.cre[jl]);
                        mu = fminf(mu, v + E);
                        v = v < SCR_INF ? fmaxf(lower_of(v, E), 0.0f) : SCR_INF;
                    }
                    acc[ib][jb][q] = v;
                }
            screen_row_min(S, rl[ib], m);
            if (pb && mu < SCR_INF) atomicMin(&S.rowub[rl[ib]], __float_as_uint(mu));
        }
        __syncthreads();
        if (GATHER) {
            // the column blocks of a row share its running minimum through
            // best[] (a row may enter with only an upper bound of it)
            for (int q = tid; q < SCR_ROWS; q += 256) {
                const int64_t slot = i0 + q;
                if (slot >= A.nrows) continue;
                const int64_t i = A.rows[slot];
                const uint32_t g = reinterpret_cast<const volatile uint32_t *>(A.best)[i];
                const uint32_t m = S.rowbest[q];
                if (m < g)
                    atomicMin(reinterpret_cast<uint32_t *>(A.best) + i, m);
                else
                    S.rowbest[q] = g;
                if (pb) {
                    const uint32_t gu = reinterpret_cast<const volatile uint32_t *>(A.ub)[i];
                    const uint32_t mu = S.rowub[q];
                    if (mu < gu)
                        atomicMin(reinterpret_cast<uint32_t *>(A.ub) + i, mu);
                    else
                        S.rowub[q] = gu;
                }
            }
            __syncthreads();
        }
        // phase B: capture
#pragma unroll
        for (int ib = 0; ib < 2; ++ib) {
            if (gi[ib] < 0) continue;
            float tc, thr;
            screen_thresholds(S, rl[ib], A.kappa, tc, thr);
            const int64_t slot = GATHER ? i0 + rl[ib] : gi[ib];
            if (pb) {
                const float thr_pb = __uint_as_float(S.rowub[rl[ib]]) * A.kappa;
#pragma unroll
                for (int jb = 0; jb < 2; ++jb)
#pragma unroll
                    for (int q = 0; q < 16; ++q) {
                        const int jl = 64 * wj + 32 * jb + 8 * (q >> 2) + 4 * (lane >> 5) + (q & 3);
                        screen_capture_lb<GATHER>(S, A, rl[ib], slot, acc[ib][jb][q], thr_pb, j0 + jl);
                    }
                continue;
            }
#pragma unroll
            for (int jb = 0; jb < 2; ++jb)
#pragma unroll
                for (int q = 0; q < 16; ++q) {
                    const int jl = 64 * wj + 32 * jb + 8 * (q >> 2) + 4 * (lane >> 5) + (q & 3);
                    screen_capture<GATHER>(S, A, rl[ib], slot, acc[ib][jb][q], tc, thr, ri[ib], ei[ib], jl, j0 + jl);
                }
        }
        __syncthreads();
        if (!GATHER && !pb) screen_compact(S, A.kappa);
    }
    __syncthreads();
    screen_finish<GATHER>(S, A, i0);
#undef ISO_GLOAD
#undef ISO_SSTORE
}

template <int REP>
void launch(const ScreenArgs &A0, bool gather, hipStream_t s) {
    ScreenArgs A = A0;
    if (gather) {
        if (A.nrows <= 0) return;
        // enough workgroups to fill the chip: split the columns so that row
        // blocks x column blocks >= 4 per CU (column blocks of whole tiles)
        const int64_t rblocks = (A.nrows + SCR_ROWS - 1) / SCR_ROWS;
        const int64_t tiles = A.n_pad / SCR_COLS;
        int64_t splits = (4 * (int64_t)device_cus() + rblocks - 1) / rblocks;
        splits = splits < 1 ? 1 : (splits > tiles ? tiles : splits);
        A.col_split = (tiles + splits - 1) / splits * SCR_COLS;
        splits = (A.n_pad + A.col_split - 1) / A.col_split;
        hipLaunchKernelGGL((k_screen_mfma<REP, true>), dim3((unsigned)rblocks, (unsigned)splits), dim3(256), 0, s, A);
    } else {
        A.col_split = A.n_pad;
        const unsigned blocks = (unsigned)(A.n_pad / SCR_ROWS);
        hipLaunchKernelGGL((k_screen_mfma<REP, false>), dim3(blocks), dim3(256), 0, s, A);
    }
    LAUNCH_CHECK();
}

}  // namespace

void launch_screen_rows(const ScreenArgs &A, bool gather, hipStream_t s) {
    if (A.rep == ISO_PREC_BF16)
        launch<ISO_PREC_BF16>(A, gather, s);
    else if (A.rep == ISO_PREC_FP8)
        launch<ISO_PREC_FP8>(A, gather, s);
    else if (A.rep == ISO_PREC_INT8)
        launch<ISO_PREC_INT8>(A, gather, s);
    else
        launch<ISO_PREC_FP32>(A, gather, s);
}

}  // namespace iso
