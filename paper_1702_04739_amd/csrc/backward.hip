// backward.hip -- adjoint of the total tree length W and of the cost of one
// cluster of the subpartition, with the tree and the subpartition held fixed.
//
//   W = sum over tree edges e = (v, parent(v)) of D_e,  D_e = ||x_v - x_p||
//   I = phi(delta A) / omega(A),  A = {v : labels[v] == jstar}, omega the tree
//       degree (eq. 2.2 reading), so omega(A) = 2 phi(E[A]) + phi(delta A)
//   dI/dphi_e = (den - num)/den^2 on boundary edges, -2 num/den^2 on edges
//   inside A, 0 elsewhere; dphi/dD and dphi/dsigma from eq. 2.1 (or the
//   squared-exponential option); dD_e/dx_v = (x_v - x_p)/D_e.
// grad_x = gW dW/dx + gI dI/dx,  grad_sigma = gI dI/dsigma.
//
// Every edge's coefficient c_e = (gW + gI dI/dphi_e dphi_e/dD_e) / D_e is
// computed once; each vertex then sums its incident edges (its parent edge,
// then its children in ascending id) in FP64, so the result is deterministic
// without atomics.  Edge lengths are recomputed in FP64, left to right.
#include <cmath>

#include "common.hpp"

namespace iso {

namespace {

struct BwState {
    double num, inner, gs;
    int32_t ndeg, bad;
};

__device__ inline double d2_f64_row(const float *__restrict__ x, const float *__restrict__ y, int64_t d) {
    double s = 0.0;
    for (int64_t t = 0; t < d; ++t) {
        const double df = (double)x[t] - (double)y[t];
        const double p = df * df;
        s = s + p;
    }
    return s;
}

__global__ void k_bw_edges(const float *__restrict__ X, int64_t n, int64_t d, int64_t ld,
                           const int32_t *__restrict__ parent, const int32_t *__restrict__ labels, int32_t jstar,
                           double sigma, int phi_kind, double *__restrict__ De, double *__restrict__ phi,
                           int8_t *__restrict__ kind, int32_t *__restrict__ nchild, BwState *__restrict__ st) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    const int32_t p = parent[v];
    if (p < 0) {
        De[v] = 0.0;
        phi[v] = 0.0;
        kind[v] = 0;
        return;
    }
    if (p >= n) {
        atomicOr(&st->bad, 1);
        kind[v] = 0;
        return;
    }
    atomicAdd(&nchild[p], 1);
    const double D = sqrt(d2_f64_row(X + v * ld, X + (int64_t)p * ld, d));
    De[v] = D;
    phi[v] = (phi_kind == ISO_PHI_GAUSS_SQ) ? exp(-(D * D) / (2.0 * sigma * sigma)) : exp(-D / sigma);
    const bool iv = labels[v] == jstar, ip = labels[p] == jstar;
    kind[v] = (iv != ip) ? 1 : ((iv && ip) ? 2 : 0);  // 1 boundary, 2 inside A
}

// Deterministic sums of phi over boundary and inner edges (one workgroup).
__global__ __launch_bounds__(1024) void k_bw_sums(const double *__restrict__ phi, const int8_t *__restrict__ kind,
                                                  int64_t n, BwState *__restrict__ st) {
    __shared__ double sb[1024], si[1024];
    double b = 0.0, in = 0.0;
    for (int64_t v = threadIdx.x; v < n; v += 1024) {
        if (kind[v] == 1) b = b + phi[v];
        else if (kind[v] == 2) in = in + phi[v];
    }
    sb[threadIdx.x] = b;
    si[threadIdx.x] = in;
    __syncthreads();
    for (int w = 512; w >= 1; w >>= 1) {
        if ((int)threadIdx.x < w) {
            sb[threadIdx.x] = sb[threadIdx.x] + sb[threadIdx.x + w];
            si[threadIdx.x] = si[threadIdx.x] + si[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        st->num = sb[0];
        st->inner = si[0];
    }
}

// Per-edge coefficient c_e and per-edge sigma term.
__global__ void k_bw_coef(const double *__restrict__ De, const double *__restrict__ phi,
                          const int8_t *__restrict__ kind, const int32_t *__restrict__ parent, int64_t n, double sigma,
                          int phi_kind, double gW, double gI, const BwState *__restrict__ st, double *__restrict__ coef,
                          double *__restrict__ sterm, int32_t *__restrict__ ndeg) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    if (parent[v] < 0) {
        coef[v] = 0.0;
        sterm[v] = 0.0;
        return;
    }
    const double num = st->num, den = 2.0 * st->inner + st->num;
    double dIdphi = 0.0;
    if (den > 0.0) {
        if (kind[v] == 1) dIdphi = (den - num) / (den * den);
        else if (kind[v] == 2) dIdphi = -2.0 * num / (den * den);
    }
    const double D = De[v], f = phi[v];
    double dphidD, dphids;
    if (phi_kind == ISO_PHI_GAUSS_SQ) {
        dphidD = -f * D / (sigma * sigma);
        dphids = f * D * D / (sigma * sigma * sigma);
    } else {
        dphidD = -f / sigma;
        dphids = f * D / (sigma * sigma);
    }
    sterm[v] = gI * dIdphi * dphids;
    if (!(D > 0.0)) {
        coef[v] = 0.0;
        atomicAdd(ndeg, 1);
        return;
    }
    coef[v] = (gW + gI * dIdphi * dphidD) / D;
}

__global__ __launch_bounds__(1024) void k_bw_sigma(const double *__restrict__ sterm, int64_t n,
                                                   BwState *__restrict__ st) {
    __shared__ double s[1024];
    double a = 0.0;
    for (int64_t v = threadIdx.x; v < n; v += 1024) a = a + sterm[v];
    s[threadIdx.x] = a;
    __syncthreads();
    for (int w = 512; w >= 1; w >>= 1) {
        if ((int)threadIdx.x < w) s[threadIdx.x] = s[threadIdx.x] + s[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) st->gs = s[0];
}

__global__ void k_bw_keys(const int32_t *__restrict__ parent, int64_t n, uint32_t *__restrict__ key,
                          uint32_t *__restrict__ val) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    key[v] = (uint32_t)(parent[v] + 1);
    val[v] = (uint32_t)v;
}

// One wave per vertex, lanes over coordinates:
//   g_v = c_v (x_v - x_p) + sum over children c (ascending) of c_c (x_v - x_c).
__global__ __launch_bounds__(256) void k_bw_scatter(const float *__restrict__ X, int64_t n, int64_t d, int64_t ld,
                                                    const int32_t *__restrict__ parent,
                                                    const double *__restrict__ coef, const uint32_t *__restrict__ kids,
                                                    const int32_t *__restrict__ koff, float *__restrict__ gX,
                                                    int64_t ldg) {
    const int lane = threadIdx.x & 63;
    const int64_t v = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (v >= n) return;
    const int32_t p = parent[v];
    const float *xv = X + v * ld;
    for (int64_t t = lane; t < d; t += 64) {
        const double xt = (double)xv[t];
        double acc = 0.0;
        if (p >= 0) acc = acc + coef[v] * (xt - (double)X[(int64_t)p * ld + t]);
        for (int32_t a = koff[v]; a < koff[v + 1]; ++a) {
            const int64_t c = kids[a];
            acc = acc + coef[c] * (xt - (double)X[c * ld + t]);
        }
        gX[v * ldg + t] = (float)acc;
    }
}

struct BwPlan {
    int64_t n;
    double *De, *phi, *coef, *sterm;
    int8_t *kind;
    int32_t *nchild, *koff, *ndeg;
    uint32_t *key, *val, *tk, *tv;
    BwState *st;
    void *sort_scratch;
    void carve(Arena &a) {
        De = a.take<double>(n);
        phi = a.take<double>(n);
        coef = a.take<double>(n);
        sterm = a.take<double>(n);
        kind = a.take<int8_t>(n);
        nchild = a.take<int32_t>(n + 1);
        koff = a.take<int32_t>(n + 1);
        ndeg = a.take<int32_t>(1);
        key = a.take<uint32_t>(n);
        val = a.take<uint32_t>(n);
        tk = a.take<uint32_t>(n);
        tv = a.take<uint32_t>(n);
        st = a.take<BwState>(1);
        sort_scratch = a.take<char>(radix_sort_scratch_bytes(n));
    }
};

size_t bw_bytes(int64_t n) {
    BwPlan p{};
    p.n = n;
    Arena a;
    p.carve(a);
    return a.used;
}

template <class T>
__global__ void k_fill_b(T *p, T v, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

int bits_of(int64_t maxval) {
    int b = 0;
    while (b < 32 && (int64_t(1) << b) <= maxval) ++b;
    return b < 1 ? 1 : b;
}

}  // namespace

}  // namespace iso

using namespace iso;

extern "C" iso_status iso_backward_workspace_size(int64_t n, size_t *bytes) {
    return guarded([&] {
        ISO_REQUIRE(bytes != nullptr, ISO_ERR_INVALID_ARG, "bytes is NULL");
        ISO_REQUIRE(n >= 2 && n < (int64_t(1) << 31) - 2, ISO_ERR_INVALID_ARG, "n = %lld outside [2, 2^31)", (long long)n);
        *bytes = bw_bytes(n);
    });
}

namespace iso {
namespace {

void check_backward_args(const float *X, int64_t n, int64_t d, int64_t ld, const int32_t *parent,
                         const int32_t *labels, double sigma, int32_t phi_kind, double gW, double gI, const float *gX,
                         int64_t ldg, const double *gsigma) {
    ISO_REQUIRE(X && parent && labels && gX && gsigma, ISO_ERR_INVALID_ARG,
                "X, parent, labels, gX and gsigma must be non-NULL");
    ISO_REQUIRE(n >= 2 && n < (int64_t(1) << 31) - 2, ISO_ERR_INVALID_ARG, "n = %lld outside [2, 2^31)", (long long)n);
    ISO_REQUIRE(d >= 1 && ld >= d && ldg >= d, ISO_ERR_INVALID_ARG, "need d >= 1, ld >= d, ldg >= d");
    ISO_REQUIRE(sigma > 0.0 && std::isfinite(sigma), ISO_ERR_INVALID_ARG, "sigma = %g must be positive", sigma);
    ISO_REQUIRE(phi_kind == ISO_PHI_EXP_DIST || phi_kind == ISO_PHI_GAUSS_SQ, ISO_ERR_INVALID_ARG,
                "unknown phi %d", phi_kind);
    ISO_REQUIRE(std::isfinite(gW) && std::isfinite(gI), ISO_ERR_INVALID_ARG, "gW and gI must be finite");
}

// The adjoint proper, on a workspace of at least bw_bytes(n) bytes.  Every
// buffer that must start at a known value is set by a kernel or a copy here,
// so the workspace may hold anything (e.g. a previous call's state).
void run_backward(const float *X, int64_t n, int64_t d, int64_t ld, const int32_t *parent, const int32_t *labels,
                  int32_t jstar, double sigma, int32_t phi_kind, double gW, double gI, float *gX, int64_t ldg,
                  double *gsigma, double *I_out, void *ws, size_t ws_bytes, hipStream_t s) {
    BwPlan P{};
    P.n = n;
    Arena a{static_cast<char *>(ws), 0, ws_bytes};
    P.carve(a);
    const unsigned gn = grid_for(n, 256);
    hipLaunchKernelGGL(k_fill_b<int32_t>, dim3(gn), dim3(256), 0, s, P.nchild, 0, n + 1);
    LAUNCH_CHECK();
    hipLaunchKernelGGL(k_fill_b<int32_t>, dim3(1), dim3(64), 0, s, P.ndeg, 0, (int64_t)1);
    LAUNCH_CHECK();
    BwState h0{};
    HIP_CHECK(hipMemcpyAsync(P.st, &h0, sizeof(h0), hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_bw_edges, dim3(gn), dim3(256), 0, s, X, n, d, ld, parent, labels, jstar, sigma, phi_kind,
                       P.De, P.phi, P.kind, P.nchild, P.st);
    LAUNCH_CHECK();
    BwState h{};
    HIP_CHECK(hipMemcpyAsync(&h, P.st, sizeof(h), hipMemcpyDeviceToHost, s));
    HIP_CHECK(hipStreamSynchronize(s));
    ISO_REQUIRE(h.bad == 0, ISO_ERR_INVALID_ARG, "parent entries must be -1 or in [0, n)");
    hipLaunchKernelGGL(k_bw_sums, dim3(1), dim3(1024), 0, s, P.phi, P.kind, n, P.st);
    LAUNCH_CHECK();
    hipLaunchKernelGGL(k_bw_coef, dim3(gn), dim3(256), 0, s, P.De, P.phi, P.kind, parent, n, sigma, phi_kind, gW, gI,
                       P.st, P.coef, P.sterm, P.ndeg);
    LAUNCH_CHECK();
    hipLaunchKernelGGL(k_bw_sigma, dim3(1), dim3(1024), 0, s, P.sterm, n, P.st);
    LAUNCH_CHECK();
    hipLaunchKernelGGL(k_bw_keys, dim3(gn), dim3(256), 0, s, parent, n, P.key, P.val);
    LAUNCH_CHECK();
    radix_sort_pairs_u32(P.key, P.val, P.tk, P.tv, n, bits_of(n), P.sort_scratch, s);
    exclusive_scan_i32(P.nchild, P.koff, n + 1, nullptr, nullptr, s);
    // vertices without a parent sort first (key 0); the child lists follow
    int32_t total_children = 0;
    HIP_CHECK(hipMemcpyAsync(&total_children, P.koff + n, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIP_CHECK(hipStreamSynchronize(s));
    const int64_t nroots = n - total_children;
    hipLaunchKernelGGL(k_bw_scatter, dim3(grid_for(n, 4)), dim3(256), 0, s, X, n, d, ld, parent, P.coef,
                       P.val + nroots, P.koff, gX, ldg);
    LAUNCH_CHECK();
    HIP_CHECK(hipMemcpyAsync(&h, P.st, sizeof(h), hipMemcpyDeviceToHost, s));
    HIP_CHECK(hipStreamSynchronize(s));
    *gsigma = h.gs;
    if (I_out) {
        const double den = 2.0 * h.inner + h.num;
        *I_out = den > 0.0 ? h.num / den : 0.0;
    }
}

}  // namespace
}  // namespace iso

extern "C" iso_status iso_backward(const float *X, int64_t n, int64_t d, int64_t ld, const int32_t *parent,
                                   const int32_t *labels, int32_t jstar, double sigma, int32_t phi_kind, double gW,
                                   double gI, float *gX, int64_t ldg, double *gsigma, double *I_out, void *ws,
                                   size_t ws_bytes, void *stream) {
    return guarded([&] {
        check_backward_args(X, n, d, ld, parent, labels, sigma, phi_kind, gW, gI, gX, ldg, gsigma);
        require_device();
        hipStream_t s = static_cast<hipStream_t>(stream);
        const size_t need = bw_bytes(n);
        ScopedWorkspace owned;
        if (ws == nullptr) {
            owned.stream = s;
            HIP_CHECK(hipMallocAsync(&owned.ptr, need, s));
            ws = owned.ptr;
            ws_bytes = need;
        }
        ISO_REQUIRE(ws_bytes >= need, ISO_ERR_WORKSPACE, "workspace %zu bytes < required %zu", ws_bytes, need);
        run_backward(X, n, d, ld, parent, labels, jstar, sigma, phi_kind, gW, gI, gX, ldg, gsigma, I_out, ws, ws_bytes,
                     s);
    });
}
