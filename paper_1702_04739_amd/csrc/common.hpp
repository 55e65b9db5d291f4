// common.hpp -- shared host/device helpers of the isoclust HIP library (gfx950).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstddef>
#include <cstdint>
#include <cstdio>
#include <string>

#include "isoclust.h"

namespace iso {

// ------------------------------------------------------------------ errors

void set_error(const char *fmt, ...);
const char *get_error();

struct Fail {
    iso_status code;
};

#define ISO_REQUIRE(cond, code, ...)              \
    do {                                          \
        if (!(cond)) {                            \
            ::iso::set_error(__VA_ARGS__);        \
            throw ::iso::Fail{code};              \
        }                                         \
    } while (0)

#define HIP_CHECK(expr)                                                                             \
    do {                                                                                            \
        hipError_t e_ = (expr);                                                                     \
        if (e_ != hipSuccess) {                                                                     \
            ::iso::set_error("%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_), __FILE__, __LINE__); \
            throw ::iso::Fail{e_ == hipErrorOutOfMemory ? ISO_ERR_OOM : ISO_ERR_HIP};               \
        }                                                                                           \
    } while (0)

#define LAUNCH_CHECK() HIP_CHECK(hipGetLastError())

// Runs `body`, translating Fail into its status code.
template <class F>
iso_status guarded(F &&body) {
    try {
        body();
        return ISO_OK;
    } catch (const Fail &f) {
        return f.code;
    } catch (...) {
        set_error("unexpected C++ exception");
        return ISO_ERR_INTERNAL;
    }
}

// Ensures a usable device is current; throws NO_DEVICE otherwise.
void require_device();
// Compute units of the current device (cached per device).
int device_cus();

// ------------------------------------------------------------------ workspace

inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Bump allocator over a caller (or library) owned device buffer.  The same
// plan is run twice: once with base = nullptr to measure, once to carve.
struct Arena {
    char *base = nullptr;
    size_t used = 0;
    size_t cap = 0;
    template <class T>
    T *take(size_t count) {
        size_t off = align_up(used, 256);
        used = off + align_up(count * sizeof(T), 256);
        if (base == nullptr) return nullptr;
        ISO_REQUIRE(used <= cap, ISO_ERR_WORKSPACE, "workspace too small: need at least %zu bytes, have %zu", used, cap);
        return reinterpret_cast<T *>(base + off);
    }
};

// Owns library-allocated workspace when the caller passes ws = NULL.
struct ScopedWorkspace {
    void *ptr = nullptr;
    hipStream_t stream = nullptr;
    ~ScopedWorkspace() {
        if (ptr) {
            (void)hipFreeAsync(ptr, stream);
            (void)hipStreamSynchronize(stream);
        }
    }
};

// ------------------------------------------------------------------ timing

iso_timing &timing();

// Records a hipEvent pair around a region of work on one stream (no-op when
// timing is disabled); elapsed() requires the stream to have passed `stop`.
struct EventPair {
    hipEvent_t a = nullptr, b = nullptr;
    bool on = false;
    explicit EventPair(bool enable) : on(enable) {
        if (on) {
            HIP_CHECK(hipEventCreate(&a));
            HIP_CHECK(hipEventCreate(&b));
        }
    }
    ~EventPair() {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
    }
    void start(hipStream_t s) {
        if (on) HIP_CHECK(hipEventRecord(a, s));
    }
    void stop(hipStream_t s) {
        if (on) HIP_CHECK(hipEventRecord(b, s));
    }
    double elapsed_ms() {
        if (!on) return 0.0;
        float ms = 0.0f;
        HIP_CHECK(hipEventSynchronize(b));
        HIP_CHECK(hipEventElapsedTime(&ms, a, b));
        return ms;
    }
};

// ------------------------------------------------------------------ launch helpers

constexpr int WAVE = 64;

inline unsigned grid_for(int64_t work, int block) {
    int64_t g = (work + block - 1) / block;
    if (g < 1) g = 1;
    return static_cast<unsigned>(g);
}

inline int ceil_log2(int64_t x) {
    int r = 0;
    while ((int64_t(1) << r) < x) ++r;
    return r;
}

// ------------------------------------------------------------------ histogram

constexpr int HIST_LDS_BINS = 4096;  // bins a workgroup counts in LDS before one global add per bin

// count[key[i]] += 1 for i < n with key[i] in [0, nbins) (other keys are
// skipped).  With at most HIST_LDS_BINS bins each workgroup counts in LDS and
// adds its nonzero bins once; otherwise every element adds to global memory.
// count must be zero (or hold the counts to add to) on entry.
void histogram_i32(const int32_t *key, int64_t n, int64_t nbins, int32_t *count, hipStream_t s);

// ------------------------------------------------------------------ primitives (scan_sort.hip)

// Exclusive scan of int32 in[0..n) into out[0..n) (in-place allowed); writes
// the total to *total (device) when total != nullptr.  With scratch (device,
// scan_scratch_bytes(n)) long inputs are scanned by many workgroups; without
// it, by one.
size_t scan_scratch_bytes(int64_t n);
void exclusive_scan_i32(const int32_t *in, int32_t *out, int64_t n, int32_t *total, int32_t *scratch,
                        hipStream_t s);

// Stable LSD radix sort of (key, value) pairs by the low `key_bits` bits of
// key.  tmp_* are scratch of n entries each; results land in keys/vals.
size_t radix_sort_scratch_bytes(int64_t n);
void radix_sort_pairs_u32(uint32_t *keys, uint32_t *vals, uint32_t *tmp_keys, uint32_t *tmp_vals, int64_t n,
                          int key_bits, void *scratch, hipStream_t s);

// Value of rank `rank` (0-based, ascending) among n nonnegative doubles
// (ordered by their bit patterns), written to *out (device).
size_t radix_select_scratch_bytes();
void radix_select_f64(const double *vals, const int32_t *skip_if_neg, int64_t n, int64_t rank, double *out,
                      void *scratch, hipStream_t s);

}  // namespace iso
