// prim.hip -- the paper's own MST construction (Algorithm 3, Sec. 3.5) on the
// GPU, kept as a comparison path for the Boruvka screen: Prim from vertex 0,
// one vertex per step chosen by a min-reduction over the keys of the vertices
// outside the tree, the keys then lowered with the distances from the vertex
// just added.  Distances are the FP64 left-to-right sums of squared coordinate
// differences and edges are ordered by (D^2, smaller id, larger id), so the
// tree, the lengths and the order in which vertices join are those of the FP64
// definition.  Each step is two launches (key update + block minima, then the
// final minimum and the insertion); n - 1 steps run back to back with no host
// synchronisation.
#include <cmath>

#include "common.hpp"

namespace iso {

namespace {

constexpr int PRIM_BLOCK = 256;

__device__ __forceinline__ bool edge_lt(double da, int32_t ua, int32_t va, double db, int32_t ub, int32_t vb) {
    if (da != db) return da < db;
    const int32_t a0 = min(ua, va), a1 = max(ua, va), b0 = min(ub, vb), b1 = max(ub, vb);
    return a0 != b0 ? a0 < b0 : a1 < b1;
}

__device__ __forceinline__ double sqdist_f64(const float *__restrict__ x, const float *__restrict__ y, int64_t d) {
    double s = 0.0;
    for (int64_t t = 0; t < d; ++t) {
        const double df = (double)x[t] - (double)y[t];
        const double sq = df * df;
        s = s + sq;
    }
    return s;
}

__global__ void k_prim_init(const float *__restrict__ X, int64_t n, int64_t d, int64_t ld, double *__restrict__ key,
                            int32_t *__restrict__ keyu, uint8_t *__restrict__ in_tree, int32_t *__restrict__ parent,
                            double *__restrict__ length, int32_t *__restrict__ last, int32_t *__restrict__ order) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    if (v == 0) {
        in_tree[0] = 1;
        parent[0] = -1;
        length[0] = 0.0;
        *last = -1;  // keys below already hold the distances from vertex 0
        if (order) order[0] = 0;
        return;
    }
    in_tree[v] = 0;
    key[v] = sqdist_f64(X, X + v * ld, d);
    keyu[v] = 0;
}

// Lower the keys with the distances from the vertex added last, then the
// block's lightest outside edge (d2 +inf when the block has none).
__global__ __launch_bounds__(PRIM_BLOCK) void k_prim_update(const float *__restrict__ X, int64_t n, int64_t d,
                                                            int64_t ld, const int32_t *__restrict__ last,
                                                            double *__restrict__ key, int32_t *__restrict__ keyu,
                                                            const uint8_t *__restrict__ in_tree,
                                                            double *__restrict__ part_d2,
                                                            int32_t *__restrict__ part_u, int32_t *__restrict__ part_v) {
    __shared__ double sd[PRIM_BLOCK];
    __shared__ int32_t su[PRIM_BLOCK], sv[PRIM_BLOCK];
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int32_t u = *last;
    double kd = __builtin_huge_val();
    int32_t ku = -1, kv = -1;
    if (v < n && !in_tree[v]) {
        kd = key[v];
        ku = keyu[v];
        if (u >= 0) {
            const double d2 = sqdist_f64(X + (int64_t)u * ld, X + v * ld, d);
            if (edge_lt(d2, u, (int32_t)v, kd, ku, (int32_t)v)) {
                kd = d2;
                ku = u;
                key[v] = d2;
                keyu[v] = u;
            }
        }
        kv = (int32_t)v;
    }
    sd[threadIdx.x] = kd;
    su[threadIdx.x] = ku;
    sv[threadIdx.x] = kv;
    __syncthreads();
    for (int w = PRIM_BLOCK / 2; w >= 1; w >>= 1) {
        if ((int)threadIdx.x < w) {
            const int o = threadIdx.x + w;
            if (sv[o] >= 0 && (sv[threadIdx.x] < 0 || edge_lt(sd[o], su[o], sv[o], sd[threadIdx.x], su[threadIdx.x],
                                                               sv[threadIdx.x]))) {
                sd[threadIdx.x] = sd[o];
                su[threadIdx.x] = su[o];
                sv[threadIdx.x] = sv[o];
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part_d2[blockIdx.x] = sd[0];
        part_u[blockIdx.x] = su[0];
        part_v[blockIdx.x] = sv[0];
    }
}

// The lightest edge over the block minima joins the tree.
__global__ __launch_bounds__(PRIM_BLOCK) void k_prim_pick(int64_t nblocks, int64_t step,
                                                          const double *__restrict__ part_d2,
                                                          const int32_t *__restrict__ part_u,
                                                          const int32_t *__restrict__ part_v,
                                                          uint8_t *__restrict__ in_tree, int32_t *__restrict__ parent,
                                                          double *__restrict__ length, int32_t *__restrict__ last,
                                                          int32_t *__restrict__ order) {
    __shared__ double sd[PRIM_BLOCK];
    __shared__ int32_t su[PRIM_BLOCK], sv[PRIM_BLOCK];
    double bd = __builtin_huge_val();
    int32_t bu = -1, bv = -1;
    for (int64_t b = threadIdx.x; b < nblocks; b += PRIM_BLOCK) {
        const int32_t v = part_v[b];
        if (v >= 0 && (bv < 0 || edge_lt(part_d2[b], part_u[b], v, bd, bu, bv))) {
            bd = part_d2[b];
            bu = part_u[b];
            bv = v;
        }
    }
    sd[threadIdx.x] = bd;
    su[threadIdx.x] = bu;
    sv[threadIdx.x] = bv;
    __syncthreads();
    for (int w = PRIM_BLOCK / 2; w >= 1; w >>= 1) {
        if ((int)threadIdx.x < w) {
            const int o = threadIdx.x + w;
            if (sv[o] >= 0 && (sv[threadIdx.x] < 0 || edge_lt(sd[o], su[o], sv[o], sd[threadIdx.x], su[threadIdx.x],
                                                               sv[threadIdx.x]))) {
                sd[threadIdx.x] = sd[o];
                su[threadIdx.x] = su[o];
                sv[threadIdx.x] = sv[o];
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const int32_t v = sv[0];
        if (v >= 0) {
            in_tree[v] = 1;
            parent[v] = su[0];
            length[v] = sqrt(sd[0]);
            if (order) order[step] = v;
        }
        *last = v;
    }
}

struct PrimPlan {
    int64_t n, nblocks;
    double *key, *part_d2;
    int32_t *keyu, *part_u, *part_v, *last;
    uint8_t *in_tree;
    void carve(Arena &a) {
        key = a.take<double>(n);
        keyu = a.take<int32_t>(n);
        in_tree = a.take<uint8_t>(n);
        part_d2 = a.take<double>(nblocks);
        part_u = a.take<int32_t>(nblocks);
        part_v = a.take<int32_t>(nblocks);
        last = a.take<int32_t>(1);
    }
};

size_t prim_bytes(int64_t n) {
    PrimPlan p{};
    p.n = n;
    p.nblocks = (n + PRIM_BLOCK - 1) / PRIM_BLOCK;
    Arena a;
    p.carve(a);
    return a.used;
}

}  // namespace

}  // namespace iso

using namespace iso;

extern "C" iso_status iso_mst_prim_workspace_size(int64_t n, size_t *bytes) {
    return guarded([&] {
        ISO_REQUIRE(bytes != nullptr, ISO_ERR_INVALID_ARG, "bytes is NULL");
        ISO_REQUIRE(n >= 2 && n < (int64_t(1) << 31), ISO_ERR_INVALID_ARG, "n = %lld outside [2, 2^31)", (long long)n);
        *bytes = prim_bytes(n);
    });
}

extern "C" iso_status iso_mst_prim(const float *X, int64_t n, int64_t d, int64_t ld, int32_t *parent, double *length,
                                   int32_t *order, void *ws, size_t ws_bytes, void *stream) {
    return guarded([&] {
        ISO_REQUIRE(X && parent && length, ISO_ERR_INVALID_ARG, "X, parent and length must be non-NULL");
        ISO_REQUIRE(n >= 2 && n < (int64_t(1) << 31), ISO_ERR_INVALID_ARG, "n = %lld outside [2, 2^31)", (long long)n);
        ISO_REQUIRE(d >= 1, ISO_ERR_INVALID_ARG, "d = %lld < 1", (long long)d);
        ISO_REQUIRE(ld >= d, ISO_ERR_INVALID_ARG, "ld = %lld < d = %lld", (long long)ld, (long long)d);
        require_device();
        hipStream_t s = static_cast<hipStream_t>(stream);
        PrimPlan P{};
        P.n = n;
        P.nblocks = (n + PRIM_BLOCK - 1) / PRIM_BLOCK;
        const size_t need = prim_bytes(n);
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
        const unsigned g = (unsigned)P.nblocks;
        hipLaunchKernelGGL(k_prim_init, dim3(g), dim3(PRIM_BLOCK), 0, s, X, n, d, ld, P.key, P.keyu, P.in_tree, parent,
                           length, P.last, order);
        LAUNCH_CHECK();
        for (int64_t step = 1; step < n; ++step) {
            hipLaunchKernelGGL(k_prim_update, dim3(g), dim3(PRIM_BLOCK), 0, s, X, n, d, ld, P.last, P.key, P.keyu,
                               P.in_tree, P.part_d2, P.part_u, P.part_v);
            LAUNCH_CHECK();
            hipLaunchKernelGGL(k_prim_pick, dim3(1), dim3(PRIM_BLOCK), 0, s, P.nblocks, step, P.part_d2, P.part_u,
                               P.part_v, P.in_tree, parent, length, P.last, order);
            LAUNCH_CHECK();
        }
        HIP_CHECK(hipStreamSynchronize(s));
    });
}
