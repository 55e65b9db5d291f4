// graph.hip -- full-graph vertex weights of eqs. 2.2 and 2.3 on gfx950, and the
// "median MST edge" sigma.
//
//   omega0[v] = sum over j != v, ascending j, of phi(D(v, j))          (eq. 2.2)
//   p0[v]     = alpha * sum over j != v, ascending j, of D(v, j)       (eq. 2.3)
//
// D(v, j) is the square root of the FP64 left-to-right sum over coordinates of
// the squared differences (each difference and square rounded separately, as
// everywhere on the exact path), so every distance is the same double the
// FP64 definition gives.  The rows' sums must follow the definition's order,
// so the work is split by column slabs of up to GW_SLAB columns: for each slab
// in ascending order, k_gw_dist forms every distance D(i, j) of the slab in
// parallel (64 x 64 tiles, 4 x 4 per thread, coordinates staged in LDS as
// FP64) and stores it transposed (slab column major, so that the next pass
// reads consecutive rows), then k_gw_sum adds the slab's phi(D) and D to the
// rows' running sums in ascending j: a workgroup of 64 rows forms phi of 32
// columns at a time with all its threads (loads and exp in parallel) and one
// thread per row adds them in order.
#include <cmath>

#include "common.hpp"

namespace iso {

namespace {

constexpr int GW_T = 64;       // rows and columns per distance tile
constexpr int GW_K = 16;       // coordinates per LDS stage
constexpr int64_t GW_SLAB = 1024;  // columns per slab

// The points as FP64 (exact), row-major n x d.
__global__ void k_gw_widen(const float *__restrict__ X, int64_t n, int64_t d, int64_t ld, double *__restrict__ Xd) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n * d; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = e / d, t = e - i * d;
        Xd[e] = (double)X[i * ld + t];
    }
}

// Dt[jj * n + i] = D(i, j0 + jj) for the slab's columns jj < w: the square
// root of sum over t (left to right) of (x_it - x_jt)^2, each difference and
// square rounded separately.
__global__ __launch_bounds__(256) void k_gw_dist(const double *__restrict__ Xd, int64_t n, int64_t d, int64_t j0,
                                                 int64_t w, double *__restrict__ Dt) {
    __shared__ double xr[GW_T][GW_K + 1], xc[GW_T][GW_K + 1];
    const int tid = threadIdx.x;
    // rows ti + 16 a and slab columns tj + 16 b (a, b < 4) of the tile: the 16
    // rows a wave's lanes read at once are consecutive, so their FP64 LDS reads
    // fall in distinct banks, and the stores cover 16 consecutive rows
    const int ti = tid & 15, tj = tid >> 4;
    const int64_t i0 = (int64_t)blockIdx.x * GW_T, c0 = (int64_t)blockIdx.y * GW_T;
    double acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = 0.0;
    for (int64_t t0 = 0; t0 < d; t0 += GW_K) {
        for (int q = tid; q < GW_T * GW_K; q += 256) {
            const int r = q / GW_K, c = q % GW_K;
            const int64_t t = t0 + c;
            xr[r][c] = (i0 + r < n && t < d) ? Xd[(i0 + r) * d + t] : 0.0;
            xc[r][c] = (c0 + r < w && t < d) ? Xd[(j0 + c0 + r) * d + t] : 0.0;
        }
        __syncthreads();
        const int tn = d - t0 < GW_K ? (int)(d - t0) : GW_K;
        for (int c = 0; c < tn; ++c) {
            double xa[4], xb[4];
#pragma unroll
            for (int a = 0; a < 4; ++a) xa[a] = xr[ti + 16 * a][c];
#pragma unroll
            for (int b = 0; b < 4; ++b) xb[b] = xc[tj + 16 * b][c];
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b = 0; b < 4; ++b) {
                    const double df = xa[a] - xb[b];
                    const double sq = df * df;
                    acc[a][b] = acc[a][b] + sq;
                }
        }
        __syncthreads();
    }
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        const int64_t jj = c0 + tj + 16 * b;
        if (jj >= w) continue;
#pragma unroll
        for (int a = 0; a < 4; ++a) {
            const int64_t i = i0 + ti + 16 * a;
            if (i < n) Dt[jj * n + i] = sqrt(acc[a][b]);
        }
    }
}

// Rows i0 .. i0+63 add phi(D(i, j)) and D(i, j) of the slab's columns,
// ascending j, j != i.  Per step of GW_SC columns every thread loads and maps
// GW_SC / 4 elements (coalesced over the rows) into LDS, then the first wave
// adds them, one lane per row, in column order.
constexpr int GW_SR = 64, GW_SC = 32;
template <int PHI>
__global__ __launch_bounds__(256) void k_gw_sum(const double *__restrict__ Dt, int64_t n, int64_t j0, int64_t w,
                                                double sigma, double *__restrict__ so, double *__restrict__ sp) {
    __shared__ double dd[GW_SC][GW_SR + 1], pp[GW_SC][GW_SR + 1];
    const int tid = threadIdx.x;
    const int64_t i0 = (int64_t)blockIdx.x * GW_SR;
    const int64_t iown = i0 + tid;  // the row lane tid < GW_SR adds
    double a = 0.0, b = 0.0;
    if (tid < GW_SR && iown < n) {
        a = so[iown];
        b = sp[iown];
    }
    for (int64_t c0 = 0; c0 < w; c0 += GW_SC) {
#pragma unroll
        for (int q = 0; q < GW_SC * GW_SR / 256; ++q) {
            const int idx = tid + 256 * q;
            const int cl = idx / GW_SR, rl = idx % GW_SR;
            const int64_t jj = c0 + cl, i = i0 + rl;
            const double dist = (jj < w && i < n) ? Dt[jj * n + i] : 0.0;
            dd[cl][rl] = dist;
            pp[cl][rl] = PHI == ISO_PHI_GAUSS_SQ ? exp(-(dist * dist) / (2.0 * sigma * sigma)) : exp(-dist / sigma);
        }
        __syncthreads();
        if (tid < GW_SR) {
            const int cn = w - c0 < GW_SC ? (int)(w - c0) : GW_SC;
            for (int cl = 0; cl < cn; ++cl) {
                if (j0 + c0 + cl == iown) continue;
                a = a + pp[cl][tid];
                b = b + dd[cl][tid];
            }
        }
        __syncthreads();
    }
    if (tid < GW_SR && iown < n) {
        so[iown] = a;
        sp[iown] = b;
    }
}

__global__ void k_gw_zero(double *__restrict__ so, double *__restrict__ sp, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    so[i] = 0.0;
    sp[i] = 0.0;
}

__global__ void k_gw_finish(const double *__restrict__ so, const double *__restrict__ sp, int64_t n, double alpha,
                            double *__restrict__ omega0, double *__restrict__ p0) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (omega0) omega0[i] = so[i];
    if (p0) p0[i] = alpha == 0.0 ? 0.0 : alpha * sp[i];
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
        // workspace: allocated and released in stream order (no synchronisation)
        const int64_t slab = n < GW_SLAB ? n : GW_SLAB;
        struct StreamBuffer {
            void *p = nullptr;
            hipStream_t s = nullptr;
            ~StreamBuffer() {
                if (p) (void)hipFreeAsync(p, s);
            }
        } buf;
        buf.s = s;
        Arena a;
        auto carve = [&](double *&Xd, double *&Dt, double *&so, double *&sp) {
            Xd = a.take<double>((size_t)(n * d));
            Dt = a.take<double>((size_t)(slab * n));
            so = a.take<double>((size_t)n);
            sp = a.take<double>((size_t)n);
        };
        double *Xd, *Dt, *so, *sp;
        carve(Xd, Dt, so, sp);
        HIP_CHECK(hipMallocAsync(&buf.p, a.used, s));
        a = Arena{static_cast<char *>(buf.p), 0, a.used};
        carve(Xd, Dt, so, sp);
        const unsigned gn = grid_for(n, 256);
        const unsigned gw = grid_for(n * d, 256) < 65536 ? grid_for(n * d, 256) : 65536;
        hipLaunchKernelGGL(k_gw_widen, dim3(gw), dim3(256), 0, s, X, n, d, ld, Xd);
        LAUNCH_CHECK();
        hipLaunchKernelGGL(k_gw_zero, dim3(gn), dim3(256), 0, s, so, sp, n);
        LAUNCH_CHECK();
        for (int64_t j0 = 0; j0 < n; j0 += slab) {
            const int64_t w = n - j0 < slab ? n - j0 : slab;
            hipLaunchKernelGGL(k_gw_dist, dim3((unsigned)((n + GW_T - 1) / GW_T), (unsigned)((w + GW_T - 1) / GW_T)),
                               dim3(256), 0, s, Xd, n, d, j0, w, Dt);
            LAUNCH_CHECK();
            const unsigned gs = (unsigned)((n + GW_SR - 1) / GW_SR);
            if (phi_kind == ISO_PHI_GAUSS_SQ)
                hipLaunchKernelGGL(k_gw_sum<ISO_PHI_GAUSS_SQ>, dim3(gs), dim3(256), 0, s, Dt, n, j0, w, sigma, so, sp);
            else
                hipLaunchKernelGGL(k_gw_sum<ISO_PHI_EXP_DIST>, dim3(gs), dim3(256), 0, s, Dt, n, j0, w, sigma, so, sp);
            LAUNCH_CHECK();
        }
        hipLaunchKernelGGL(k_gw_finish, dim3(gn), dim3(256), 0, s, so, sp, n, alpha, omega0, p0);
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
