// graph.hip -- full-graph vertex weights of eqs. 2.2 and 2.3 on gfx950, and the
// "median MST edge" sigma.
//
//   omega0[v] = sum over j != v, ascending j, of phi(D(v, j))          (eq. 2.2)
//   p0[v]     = alpha * sum over j != v, ascending j, of D(v, j)       (eq. 2.3)
//
// D(v, j) is the square root of the FP64 left-to-right sum over coordinates of
// the squared differences (each difference and square rounded separately, as
// everywhere on the exact path), so every distance is the same double the
// FP64 definition gives.  One workgroup owns 64 rows and sweeps the column
// blocks in ascending order; a block's 64 x 64 distances are formed in
// registers (4 x 4 per thread) from coordinates staged in LDS, their phi and D
// values pass through LDS, and one thread per row adds them in ascending j, so
// the row sums follow the definition's order too.
#include <cmath>

#include "common.hpp"

namespace iso {

namespace {

constexpr int GW_T = 64;  // rows (and columns) per block
constexpr int GW_K = 32;  // coordinates per LDS stage

template <int PHI>
__global__ __launch_bounds__(256) void k_graph_weights(const float *__restrict__ X, int64_t n, int64_t d, int64_t ld,
                                                       double sigma, double alpha, double *__restrict__ omega0,
                                                       double *__restrict__ p0) {
    __shared__ float xr[GW_T][GW_K + 1], xc[GW_T][GW_K + 1];
    __shared__ double fv[GW_T][GW_T + 1], dv[GW_T][GW_T + 1];
    const int tid = threadIdx.x;
    const int tr = tid >> 4, tc = tid & 15;  // rows 4 tr .. +3, columns 4 tc .. +3 of the block
    const int64_t i0 = (int64_t)blockIdx.x * GW_T;
    double so = 0.0, sp = 0.0;  // running sums of row i0 + tid (threads < 64)
    for (int64_t j0 = 0; j0 < n; j0 += GW_T) {
        double acc[4][4];
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b) acc[a][b] = 0.0;
        for (int64_t t0 = 0; t0 < d; t0 += GW_K) {
            for (int q = tid; q < GW_T * GW_K; q += 256) {
                const int r = q / GW_K, c = q % GW_K;
                const int64_t t = t0 + c;
                xr[r][c] = (i0 + r < n && t < d) ? X[(i0 + r) * ld + t] : 0.0f;
                xc[r][c] = (j0 + r < n && t < d) ? X[(j0 + r) * ld + t] : 0.0f;
            }
            __syncthreads();
            const int tn = d - t0 < GW_K ? (int)(d - t0) : GW_K;
            for (int c = 0; c < tn; ++c) {
#pragma unroll
                for (int a = 0; a < 4; ++a)
#pragma unroll
                    for (int b = 0; b < 4; ++b) {
                        const double df = (double)xr[4 * tr + a][c] - (double)xc[4 * tc + b][c];
                        const double sq = df * df;
                        acc[a][b] = acc[a][b] + sq;
                    }
            }
            __syncthreads();
        }
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const double dist = sqrt(acc[a][b]);
                fv[4 * tr + a][4 * tc + b] =
                    PHI == ISO_PHI_GAUSS_SQ ? exp(-(dist * dist) / (2.0 * sigma * sigma)) : exp(-dist / sigma);
                dv[4 * tr + a][4 * tc + b] = dist;
            }
        __syncthreads();
        if (tid < GW_T) {
            const int64_t i = i0 + tid;
            for (int c = 0; c < GW_T; ++c) {
                const int64_t j = j0 + c;
                if (j >= n) break;
                if (j == i) continue;
                so = so + fv[tid][c];
                sp = sp + dv[tid][c];
            }
        }
        __syncthreads();
    }
    if (tid < GW_T && i0 + tid < n) {
        const int64_t i = i0 + tid;
        if (omega0) omega0[i] = so;
        if (p0) p0[i] = alpha == 0.0 ? 0.0 : alpha * sp;
    }
}

}  // namespace

}  // namespace iso

using namespace iso;

extern "C" iso_status iso_graph_weights(const float *X, int64_t n, int64_t d, int64_t ld, double sigma,
                                        int32_t phi_kind, double alpha, double *omega0, double *p0, void *stream) {
    return guarded([&] {
        ISO_REQUIRE(X != nullptr, ISO_ERR_INVALID_ARG, "X must be non-NULL");
        ISO_REQUIRE(n >= 2 && n < (int64_t(1) << 31), ISO_ERR_INVALID_ARG, "n = %lld outside [2, 2^31)", (long long)n);
        ISO_REQUIRE(d >= 1, ISO_ERR_INVALID_ARG, "d = %lld < 1", (long long)d);
        ISO_REQUIRE(ld >= d, ISO_ERR_INVALID_ARG, "ld = %lld < d = %lld", (long long)ld, (long long)d);
        ISO_REQUIRE(sigma > 0.0 && std::isfinite(sigma), ISO_ERR_INVALID_ARG, "sigma = %g must be finite and > 0", sigma);
        ISO_REQUIRE(alpha >= 0.0 && std::isfinite(alpha), ISO_ERR_INVALID_ARG, "alpha = %g must be finite and >= 0",
                    alpha);
        ISO_REQUIRE(phi_kind == ISO_PHI_EXP_DIST || phi_kind == ISO_PHI_GAUSS_SQ, ISO_ERR_INVALID_ARG, "unknown phi %d",
                    phi_kind);
        require_device();
        if (omega0 == nullptr && p0 == nullptr) return;
        hipStream_t s = static_cast<hipStream_t>(stream);
        const unsigned blocks = (unsigned)((n + GW_T - 1) / GW_T);
        if (phi_kind == ISO_PHI_GAUSS_SQ)
            hipLaunchKernelGGL(k_graph_weights<ISO_PHI_GAUSS_SQ>, dim3(blocks), dim3(256), 0, s, X, n, d, ld, sigma,
                               alpha, omega0, p0);
        else
            hipLaunchKernelGGL(k_graph_weights<ISO_PHI_EXP_DIST>, dim3(blocks), dim3(256), 0, s, X, n, d, ld, sigma,
                               alpha, omega0, p0);
        LAUNCH_CHECK();
    });
}

extern "C" iso_status iso_sigma_median(const int32_t *parent, const double *length, int64_t n, double *sigma,
                                       void *stream) {
    return guarded([&] {
        ISO_REQUIRE(parent && length && sigma, ISO_ERR_INVALID_ARG, "parent, length and sigma must be non-NULL");
        ISO_REQUIRE(n >= 2 && n < (int64_t(1) << 31), ISO_ERR_INVALID_ARG, "n = %lld outside [2, 2^31)", (long long)n);
        require_device();
        hipStream_t s = static_cast<hipStream_t>(stream);
        ScopedWorkspace owned;
        owned.stream = s;
        const size_t need = radix_select_scratch_bytes() + 256;
        HIP_CHECK(hipMallocAsync(&owned.ptr, need, s));
        double *out = static_cast<double *>(owned.ptr);
        void *scratch = static_cast<char *>(owned.ptr) + 256;
        // lower median of the n - 1 edge lengths: rank (n - 2) / 2, the root skipped
        radix_select_f64(length, parent, n, (n - 2) / 2, out, scratch, s);
        HIP_CHECK(hipMemcpyAsync(sigma, out, sizeof(double), hipMemcpyDeviceToHost, s));
        HIP_CHECK(hipStreamSynchronize(s));
    });
}
