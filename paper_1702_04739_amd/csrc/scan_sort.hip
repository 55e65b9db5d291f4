// scan_sort.hip -- error state, device check, and the generic primitives the
// pipeline needs: exclusive scan, stable radix sort, radix select.
#include <algorithm>
#include <cstring>

#include "common.hpp"

namespace iso {

// ------------------------------------------------------------------ errors

static thread_local char g_err[512] = "no error";

void set_error(const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}

const char *get_error() { return g_err; }

void require_device() {
    int count = 0;
    hipError_t e = hipGetDeviceCount(&count);
    ISO_REQUIRE(e == hipSuccess && count > 0, ISO_ERR_NO_DEVICE, "no HIP device available (%s)",
                e == hipSuccess ? "device count is 0" : hipGetErrorString(e));
    int dev = 0;
    HIP_CHECK(hipGetDevice(&dev));
    hipDeviceProp_t prop;
    HIP_CHECK(hipGetDeviceProperties(&prop, dev));
    ISO_REQUIRE(std::strncmp(prop.gcnArchName, "gfx950", 6) == 0, ISO_ERR_NO_DEVICE,
                "device %d is %s; this library is built for gfx950 only", dev, prop.gcnArchName);
}

int device_cus() {
    static int cached[64] = {0};
    int dev = 0;
    HIP_CHECK(hipGetDevice(&dev));
    if (dev >= 0 && dev < 64 && cached[dev] > 0) return cached[dev];
    int cus = 0;
    HIP_CHECK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    ISO_REQUIRE(cus > 0, ISO_ERR_HIP, "device %d reports %d compute units", dev, cus);
    if (dev >= 0 && dev < 64) cached[dev] = cus;
    return cus;
}

// ------------------------------------------------------------------ timing

static iso_timing g_timing{};

iso_timing &timing() { return g_timing; }

// ------------------------------------------------------------------ exclusive scan (one workgroup)

constexpr int SCAN_BLOCK = 1024;

__device__ inline int32_t wave_inclusive_scan(int32_t v) {
    const int lane = threadIdx.x & (WAVE - 1);
#pragma unroll
    for (int off = 1; off < WAVE; off <<= 1) {
        int32_t o = __shfl_up(v, off, WAVE);
        if (lane >= off) v += o;
    }
    return v;
}

// Block-wide exclusive scan of one value per thread; returns the prefix and
// writes the block total to *block_total.
__device__ inline int32_t block_exclusive_scan(int32_t v, int32_t *block_total) {
    __shared__ int32_t wave_sums[SCAN_BLOCK / WAVE];
    const int lane = threadIdx.x & (WAVE - 1);
    const int w = threadIdx.x / WAVE;
    int32_t inc = wave_inclusive_scan(v);
    if (lane == WAVE - 1) wave_sums[w] = inc;
    __syncthreads();
    if (w == 0) {
        int32_t s = lane < (int)(blockDim.x / WAVE) ? wave_sums[lane] : 0;
        int32_t si = wave_inclusive_scan(s);
        if (lane < (int)(blockDim.x / WAVE)) wave_sums[lane] = si - s;
        if (lane == (int)(blockDim.x / WAVE) - 1) *block_total = si;
    }
    __syncthreads();
    int32_t r = inc - v + wave_sums[w];
    __syncthreads();
    return r;
}

__global__ __launch_bounds__(SCAN_BLOCK) void k_exclusive_scan(const int32_t *in, int32_t *out, int64_t n,
                                                               int32_t *total) {
    __shared__ int32_t s_total;
    const int64_t chunk = (n + SCAN_BLOCK - 1) / SCAN_BLOCK;
    const int64_t lo = threadIdx.x * chunk;
    const int64_t hi = lo + chunk < n ? lo + chunk : n;
    int32_t s = 0;
#pragma unroll 8
    for (int64_t i = lo; i < hi; ++i) s += in[i];
    int32_t run = block_exclusive_scan(s, &s_total);
    for (int64_t i = lo; i < hi; ++i) {
        int32_t x = in[i];
        out[i] = run;
        run += x;
    }
    if (threadIdx.x == 0 && total) *total = s_total;
}

// Multi-block scan for long inputs: tiles of SCAN_TILE elements, each thread
// holding elements base + r * SCAN_BLOCK + tid (r = 0 .. SCAN_ROUNDS-1, so the
// loads are coalesced); tile sums, their exclusive scan, then each tile rescans
// round by round in index order from its offset.
constexpr int SCAN_ROUNDS = 8;
constexpr int64_t SCAN_TILE = (int64_t)SCAN_BLOCK * SCAN_ROUNDS;

__global__ __launch_bounds__(SCAN_BLOCK) void k_scan_tile_sums(const int32_t *in, int64_t n, int32_t *sums) {
    __shared__ int32_t s_total;
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
    int32_t v = 0;
#pragma unroll
    for (int r = 0; r < SCAN_ROUNDS; ++r) {
        const int64_t i = base + (int64_t)r * SCAN_BLOCK + threadIdx.x;
        v += i < n ? in[i] : 0;
    }
    (void)block_exclusive_scan(v, &s_total);
    if (threadIdx.x == 0) sums[blockIdx.x] = s_total;
}

__global__ __launch_bounds__(SCAN_BLOCK) void k_scan_tile_apply(const int32_t *in, int32_t *out, int64_t n,
                                                                const int32_t *offsets) {
    __shared__ int32_t s_total;
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
    int32_t run = offsets[blockIdx.x];
    for (int r = 0; r < SCAN_ROUNDS; ++r) {
        const int64_t i = base + (int64_t)r * SCAN_BLOCK + threadIdx.x;
        const int32_t v = i < n ? in[i] : 0;
        const int32_t pre = block_exclusive_scan(v, &s_total);
        if (i < n) out[i] = run + pre;
        run += s_total;
    }
}

size_t scan_scratch_bytes(int64_t n) { return sizeof(int32_t) * 2 * (size_t)((n + SCAN_TILE - 1) / SCAN_TILE); }

void exclusive_scan_i32(const int32_t *in, int32_t *out, int64_t n, int32_t *total, int32_t *scratch,
                        hipStream_t s) {
    if (n <= 0) {
        if (total) HIP_CHECK(hipMemsetAsync(total, 0, sizeof(int32_t), s));
        return;
    }
    const int64_t tiles = (n + SCAN_TILE - 1) / SCAN_TILE;
    if (tiles <= 8 || scratch == nullptr) {
        hipLaunchKernelGGL(k_exclusive_scan, dim3(1), dim3(SCAN_BLOCK), 0, s, in, out, n, total);
        LAUNCH_CHECK();
        return;
    }
    int32_t *sums = scratch, *offs = scratch + tiles;
    hipLaunchKernelGGL(k_scan_tile_sums, dim3((unsigned)tiles), dim3(SCAN_BLOCK), 0, s, in, n, sums);
    LAUNCH_CHECK();
    hipLaunchKernelGGL(k_exclusive_scan, dim3(1), dim3(SCAN_BLOCK), 0, s, sums, offs, tiles, total);
    LAUNCH_CHECK();
    hipLaunchKernelGGL(k_scan_tile_apply, dim3((unsigned)tiles), dim3(SCAN_BLOCK), 0, s, in, out, n, offs);
    LAUNCH_CHECK();
}

// ------------------------------------------------------------------ stable radix sort

constexpr int RS_BLOCK = 256;
constexpr int RS_ROUNDS = 16;
constexpr int RS_TILE = RS_BLOCK * RS_ROUNDS;
constexpr int RS_WAVES = RS_BLOCK / WAVE;

__global__ __launch_bounds__(RS_BLOCK) void k_rs_hist(const uint32_t *keys, int64_t n, int shift,
                                                      int32_t *hist, int nblocks) {
    __shared__ int32_t cnt[256];
    cnt[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * RS_TILE;
    for (int r = 0; r < RS_ROUNDS; ++r) {
        int64_t e = base + r * RS_BLOCK + threadIdx.x;
        if (e < n) atomicAdd(&cnt[(keys[e] >> shift) & 0xFF], 1);
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * nblocks + blockIdx.x] = cnt[threadIdx.x];
}

__global__ __launch_bounds__(RS_BLOCK) void k_rs_scatter(const uint32_t *keys, const uint32_t *vals,
                                                         uint32_t *okeys, uint32_t *ovals, int64_t n, int shift,
                                                         const int32_t *offsets, int nblocks) {
    __shared__ int32_t run[256];
    __shared__ int32_t wcnt[RS_WAVES][256];
    const int lane = threadIdx.x & (WAVE - 1);
    const int w = threadIdx.x / WAVE;
    run[threadIdx.x] = 0;
    for (int q = 0; q < RS_WAVES; ++q) wcnt[q][threadIdx.x] = 0;
    __syncthreads();
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (WAVE - lane));
    const int64_t base = (int64_t)blockIdx.x * RS_TILE;
    for (int r = 0; r < RS_ROUNDS; ++r) {
        const int64_t e = base + r * RS_BLOCK + threadIdx.x;
        const bool valid = e < n;
        uint32_t key = valid ? keys[e] : 0u;
        uint32_t val = valid ? vals[e] : 0u;
        const int g = (key >> shift) & 0xFF;
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            uint64_t bb = __ballot(valid && ((g >> b) & 1));
            peers &= ((g >> b) & 1) ? bb : ~bb;
        }
        const int rank = __popcll(peers & lt_mask);
        if (valid && rank == 0) wcnt[w][g] = __popcll(peers);
        __syncthreads();
        if (valid) {
            int32_t pos = run[g] + rank;
            for (int q = 0; q < w; ++q) pos += wcnt[q][g];
            int64_t dst = (int64_t)offsets[(int64_t)g * nblocks + blockIdx.x] + pos;
            okeys[dst] = key;
            ovals[dst] = val;
        }
        __syncthreads();
        int32_t add = 0;
        for (int q = 0; q < RS_WAVES; ++q) {
            add += wcnt[q][threadIdx.x];
            wcnt[q][threadIdx.x] = 0;
        }
        run[threadIdx.x] += add;
        __syncthreads();
    }
}

size_t radix_sort_scratch_bytes(int64_t n) {
    int64_t nblocks = (n + RS_TILE - 1) / RS_TILE;
    if (nblocks < 1) nblocks = 1;
    return align_up(sizeof(int32_t) * 256 * nblocks, 256);
}

void radix_sort_pairs_u32(uint32_t *keys, uint32_t *vals, uint32_t *tmp_keys, uint32_t *tmp_vals, int64_t n,
                          int key_bits, void *scratch, hipStream_t s) {
    if (n <= 1) return;
    const int nblocks = (int)((n + RS_TILE - 1) / RS_TILE);
    int32_t *hist = static_cast<int32_t *>(scratch);
    uint32_t *ka = keys, *va = vals, *kb = tmp_keys, *vb = tmp_vals;
    int passes = 0;
    for (int shift = 0; shift < key_bits; shift += 8) {
        hipLaunchKernelGGL(k_rs_hist, dim3(nblocks), dim3(RS_BLOCK), 0, s, ka, n, shift, hist, nblocks);
        LAUNCH_CHECK();
        exclusive_scan_i32(hist, hist, (int64_t)256 * nblocks, nullptr, nullptr, s);
        hipLaunchKernelGGL(k_rs_scatter, dim3(nblocks), dim3(RS_BLOCK), 0, s, ka, va, kb, vb, n, shift, hist,
                           nblocks);
        LAUNCH_CHECK();
        std::swap(ka, kb);
        std::swap(va, vb);
        ++passes;
    }
    if (passes & 1) {
        HIP_CHECK(hipMemcpyAsync(keys, ka, sizeof(uint32_t) * n, hipMemcpyDeviceToDevice, s));
        HIP_CHECK(hipMemcpyAsync(vals, va, sizeof(uint32_t) * n, hipMemcpyDeviceToDevice, s));
    }
}

// ------------------------------------------------------------------ radix select (FP64 >= 0)

struct SelState {
    uint64_t prefix;
    uint64_t mask;
    int64_t rank;
    int32_t hist[256];
};

__global__ __launch_bounds__(256) void k_sel_init(SelState *st, int64_t rank) {
    st->hist[threadIdx.x] = 0;
    if (threadIdx.x == 0) {
        st->prefix = 0;
        st->mask = 0;
        st->rank = rank;
    }
}

__global__ __launch_bounds__(256) void k_sel_hist(const double *vals, const int32_t *skip_if_neg, int64_t n,
                                                  int shift, SelState *st) {
    __shared__ int32_t cnt[256];
    cnt[threadIdx.x] = 0;
    __syncthreads();
    const uint64_t prefix = st->prefix, mask = st->mask;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        if (skip_if_neg && skip_if_neg[i] < 0) continue;
        uint64_t b = (uint64_t)__double_as_longlong(vals[i]);
        if ((b & mask) == prefix) atomicAdd(&cnt[(b >> shift) & 0xFF], 1);
    }
    __syncthreads();
    if (cnt[threadIdx.x]) atomicAdd(&st->hist[threadIdx.x], cnt[threadIdx.x]);
}

__global__ __launch_bounds__(256) void k_sel_pick(SelState *st, int shift, double *out, int last) {
    if (threadIdx.x == 0) {
        int64_t r = st->rank;
        int digit = 255;
        for (int g = 0; g < 256; ++g) {
            if (r < st->hist[g]) { digit = g; break; }
            r -= st->hist[g];
        }
        st->rank = r;
        st->prefix |= (uint64_t)digit << shift;
        st->mask |= (uint64_t)0xFF << shift;
        if (last) *out = __longlong_as_double((long long)st->prefix);
    }
    __syncthreads();
    st->hist[threadIdx.x] = 0;
}

size_t radix_select_scratch_bytes() { return align_up(sizeof(SelState), 256); }

void radix_select_f64(const double *vals, const int32_t *skip_if_neg, int64_t n, int64_t rank, double *out,
                      void *scratch, hipStream_t s) {
    SelState *st = static_cast<SelState *>(scratch);
    hipLaunchKernelGGL(k_sel_init, dim3(1), dim3(256), 0, s, st, rank);
    LAUNCH_CHECK();
    const unsigned g = grid_for(n, 256) < 1024 ? grid_for(n, 256) : 1024;
    for (int shift = 56; shift >= 0; shift -= 8) {
        hipLaunchKernelGGL(k_sel_hist, dim3(g), dim3(256), 0, s, vals, skip_if_neg, n, shift, st);
        LAUNCH_CHECK();
        hipLaunchKernelGGL(k_sel_pick, dim3(1), dim3(256), 0, s, st, shift, out, shift == 0);
        LAUNCH_CHECK();
    }
}

// ------------------------------------------------------------------ histogram

namespace {

__global__ __launch_bounds__(256) void k_hist_lds(const int32_t *__restrict__ key, int64_t n, int32_t nbins,
                                                  int32_t *__restrict__ count) {
    __shared__ int32_t h[HIST_LDS_BINS];
    for (int b = threadIdx.x; b < nbins; b += blockDim.x) h[b] = 0;
    __syncthreads();
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t k = key[i];
        if (k >= 0 && k < nbins) atomicAdd(&h[k], 1);
    }
    __syncthreads();
    for (int b = threadIdx.x; b < nbins; b += blockDim.x)
        if (h[b]) atomicAdd(&count[b], h[b]);
}

__global__ void k_hist_global(const int32_t *__restrict__ key, int64_t n, int64_t nbins, int32_t *__restrict__ count) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t k = key[i];
    if (k >= 0 && k < nbins) atomicAdd(&count[k], 1);
}

}  // namespace

void histogram_i32(const int32_t *key, int64_t n, int64_t nbins, int32_t *count, hipStream_t s) {
    if (n <= 0 || nbins <= 0) return;
    if (nbins <= HIST_LDS_BINS) {
        const unsigned g = std::min<unsigned>(grid_for(n, 256), 4u * (unsigned)device_cus());
        hipLaunchKernelGGL(k_hist_lds, dim3(g), dim3(256), 0, s, key, n, (int32_t)nbins, count);
    } else {
        hipLaunchKernelGGL(k_hist_global, dim3(grid_for(n, 256)), dim3(256), 0, s, key, n, nbins, count);
    }
    LAUNCH_CHECK();
}

}  // namespace iso

extern "C" iso_status iso_timing_enable(int32_t on) {
    iso::g_timing = iso_timing{};
    iso::g_timing.enabled = on ? 1 : 0;
    return ISO_OK;
}

extern "C" iso_status iso_timing_read(iso_timing *out) {
    if (!out) {
        iso::set_error("out is NULL");
        return ISO_ERR_INVALID_ARG;
    }
    *out = iso::g_timing;
    return ISO_OK;
}
