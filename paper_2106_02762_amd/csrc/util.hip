// Errors, budgeted device memory, timing and the library sort / scan primitives.
#include <chrono>
#include <cstdarg>

#include <cstring>

#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/device/device_scan.hpp>

#include "internal.h"

namespace dt {

static thread_local std::string g_last_error;

int fail(int code, const char *fmt, ...) {
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

void clear_error() { g_last_error.clear(); }

const char *last_error() { return g_last_error.c_str(); }

namespace {

// most bytes the cache may hold: half the budget, or 32 GiB without one
uint64_t pool_cap(const dt_ctx *ctx) { return ctx->budget ? ctx->budget / 2 : (32ull << 30); }

void pool_put(dt_ctx *ctx, void *p, size_t bytes) {
    std::lock_guard<std::mutex> lk(ctx->pool_mu);
    ctx->pool.emplace(bytes, p);
    ctx->pool_bytes += bytes;
    while (ctx->pool_bytes > pool_cap(ctx) && !ctx->pool.empty()) {   // largest first
        auto it = std::prev(ctx->pool.end());
        (void)hipFree(it->second);
        ctx->used -= it->first;
        ctx->pool_bytes -= it->first;
        ctx->pool.erase(it);
    }
}

}  // namespace

void pool_trim(dt_ctx *ctx, uint64_t keep_bytes) {
    std::lock_guard<std::mutex> lk(ctx->pool_mu);
    while (ctx->pool_bytes > keep_bytes && !ctx->pool.empty()) {
        auto it = std::prev(ctx->pool.end());
        (void)hipFree(it->second);
        ctx->used -= it->first;
        ctx->pool_bytes -= it->first;
        ctx->pool.erase(it);
    }
}

void DevMem::reset() {
    if (ptr) {
        if (pooled && ctx) {
            pool_put(ctx, ptr, bytes);
        } else {
            (void)hipFree(ptr);
            if (ctx) ctx->used -= bytes;
        }
    }
    ctx = nullptr;
    ptr = nullptr;
    bytes = 0;
    pooled = false;
}

DevMem &DevMem::operator=(DevMem &&o) noexcept {
    if (this != &o) {
        reset();
        ctx = o.ctx;
        ptr = o.ptr;
        bytes = o.bytes;
        pooled = o.pooled;
        o.ctx = nullptr;
        o.ptr = nullptr;
        o.bytes = 0;
        o.pooled = false;
    }
    return *this;
}

int dev_alloc(dt_ctx *ctx, DevMem &m, size_t bytes, bool pooled) {
    m.reset();
    if (bytes == 0) bytes = 256;   // a valid pointer even for empty arrays
    bytes = (bytes + 255) & ~size_t(255);
    if (pooled) {
        // best fit among cached blocks, wasting at most an eighth plus 2 MiB
        std::lock_guard<std::mutex> lk(ctx->pool_mu);
        auto it = ctx->pool.lower_bound(bytes);
        if (it != ctx->pool.end() && it->first <= bytes + bytes / 8 + (2u << 20)) {
            m.ctx = ctx;
            m.ptr = it->second;
            m.bytes = it->first;
            m.pooled = true;
            ctx->pool_bytes -= it->first;
            ctx->pool.erase(it);
            return DT_OK;
        }
    }
    if (ctx->budget && ctx->used.load() + bytes > ctx->budget) {
        const uint64_t over = ctx->used.load() + bytes - ctx->budget;
        pool_trim(ctx, ctx->pool_bytes > over ? ctx->pool_bytes - over : 0);
    }
    if (ctx->budget && ctx->used.load() + bytes > ctx->budget)
        return fail(DT_ENOMEM, "device allocation of %zu bytes exceeds the budget (%llu used of %llu)",
                    bytes, (unsigned long long)ctx->used.load(), (unsigned long long)ctx->budget);
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) {   // cached blocks may be what is missing
        (void)hipGetLastError();
        pool_trim(ctx, 0);
        e = hipMalloc(&p, bytes);
    }
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(DT_ENOMEM, "hipMalloc(%zu) failed: %s", bytes, hipGetErrorString(e));
    }
    m.ctx = ctx;
    m.ptr = p;
    m.bytes = bytes;
    m.pooled = pooled;
    ctx->used += bytes;
    return DT_OK;
}

int ensure(dt_ctx *ctx, DevMem &m, size_t bytes) {
    if (m.ptr && m.bytes >= bytes) return DT_OK;
    return dev_alloc(ctx, m, bytes + bytes / 4, false);
}

double now_ms() {
    using namespace std::chrono;
    return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

int sort_pairs_u64_u32(dt_ctx *ctx, const uint64_t *kin, uint64_t *kout, const uint32_t *vin,
                       uint32_t *vout, size_t n, int end_bit, hipStream_t s) {
    if (n == 0) return DT_OK;
    size_t bytes = 0;
    DT_HIP(rocprim::radix_sort_pairs(nullptr, bytes, kin, kout, vin, vout, n, 0u,
                                     (unsigned)end_bit, s));
    DevMem tmp;
    DT_TRY(dev_alloc(ctx, tmp, bytes));
    DT_HIP(rocprim::radix_sort_pairs(tmp.ptr, bytes, kin, kout, vin, vout, n, 0u,
                                     (unsigned)end_bit, s));
    // the temporary goes back to the context's cache, whose blocks are reused in stream order on
    // the context's stream only: another stream must finish with it first
    if (s != ctx->stream) DT_HIP(hipStreamSynchronize(s));
    return DT_OK;
}

int sort_pairs_u64_u64(dt_ctx *ctx, const uint64_t *kin, uint64_t *kout, const uint64_t *vin,
                       uint64_t *vout, size_t n, int end_bit, hipStream_t s) {
    if (n == 0) return DT_OK;
    size_t bytes = 0;
    DT_HIP(rocprim::radix_sort_pairs(nullptr, bytes, kin, kout, vin, vout, n, 0u,
                                     (unsigned)end_bit, s));
    DevMem tmp;
    DT_TRY(dev_alloc(ctx, tmp, bytes));
    DT_HIP(rocprim::radix_sort_pairs(tmp.ptr, bytes, kin, kout, vin, vout, n, 0u,
                                     (unsigned)end_bit, s));
    // the temporary goes back to the context's cache, whose blocks are reused in stream order on
    // the context's stream only: another stream must finish with it first
    if (s != ctx->stream) DT_HIP(hipStreamSynchronize(s));
    return DT_OK;
}

int sort_pairs_u16_u4(dt_ctx *ctx, const uint16_t *kin, uint16_t *kout, const uint4 *vin, uint4 *vout,
                      size_t n, int end_bit, hipStream_t s, DevMem *keep) {
    if (n == 0) return DT_OK;
    size_t bytes = 0;
    DT_HIP(rocprim::radix_sort_pairs(nullptr, bytes, kin, kout, vin, vout, n, 0u, (unsigned)end_bit, s));
    DevMem tmp;
    DT_TRY(dev_alloc(ctx, tmp, bytes));
    DT_HIP(rocprim::radix_sort_pairs(tmp.ptr, bytes, kin, kout, vin, vout, n, 0u, (unsigned)end_bit, s));
    if (keep) *keep = std::move(tmp);   // the caller releases it after joining stream s
    else if (s != ctx->stream) DT_HIP(hipStreamSynchronize(s));
    return DT_OK;
}

int exclusive_scan_u32(dt_ctx *ctx, const uint32_t *in, uint32_t *out, size_t n, hipStream_t s, DevMem *keep) {
    if (n == 0) return DT_OK;
    size_t bytes = 0;
    DT_HIP(rocprim::exclusive_scan(nullptr, bytes, in, out, 0u, n, rocprim::plus<uint32_t>(), s));
    DevMem tmp;
    DT_TRY(dev_alloc(ctx, tmp, bytes));
    DT_HIP(rocprim::exclusive_scan(tmp.ptr, bytes, in, out, 0u, n, rocprim::plus<uint32_t>(), s));
    // the temporary goes back to the context's cache, whose blocks are reused in stream order on
    // the context's stream only: another stream must finish with it first (or the caller keeps it)
    if (s != ctx->stream) {
        if (keep) *keep = std::move(tmp);
        else DT_HIP(hipStreamSynchronize(s));
    }
    return DT_OK;
}

int exclusive_scan_u64(dt_ctx *ctx, const uint64_t *in, uint64_t *out, size_t n, hipStream_t s) {
    if (n == 0) return DT_OK;
    size_t bytes = 0;
    DT_HIP(rocprim::exclusive_scan(nullptr, bytes, in, out, (uint64_t)0, n,
                                   rocprim::plus<uint64_t>(), s));
    DevMem tmp;
    DT_TRY(dev_alloc(ctx, tmp, bytes));
    DT_HIP(rocprim::exclusive_scan(tmp.ptr, bytes, in, out, (uint64_t)0, n,
                                   rocprim::plus<uint64_t>(), s));
    // the temporary goes back to the context's cache, whose blocks are reused in stream order on
    // the context's stream only: another stream must finish with it first
    if (s != ctx->stream) DT_HIP(hipStreamSynchronize(s));
    return DT_OK;
}

}  // namespace dt
