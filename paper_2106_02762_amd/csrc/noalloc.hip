// A count that allocates nothing: dt_count_async's work with its scratch (the per-block partial
// sums and the prefix arrays of the heavy path) in a fixed device array instead of memory the
// context allocates, for callers that cannot allocate (HIP graph capture, tight serving loops).
//
// The array is one per device, for the whole process.  Host code never passes its name to a
// kernel or a copy (on the host that name is only a stand-in for the symbol): the context's setup
// takes each device's own address of the array once, with that device current, and the count uses
// that address.  Every call on a device shares the array: calls that overlap on one device race,
// and each call leaves its contents behind.  Nothing in it needs to start at zero: every kernel
// writes its partial slots and prefix values before the reduction reads them.
#include "internal.h"

namespace dt {

namespace {

constexpr size_t kNoAllocScratchBytes = 64ull << 20;   // 64 MiB per device
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

std::mutex g_mu;
void *g_ptr[kMaxDevices] = {};

}  // namespace

// Takes the calling device's address of the scratch array (once per device); the device must be
// current.
int noalloc_init(int device) {
    if (device < 0 || device >= kMaxDevices) return fail(DT_EINVAL, "device %d out of range", device);
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_ptr[device]) return DT_OK;
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
        return fail(DT_EDEVICE, "hipGetSymbolAddress of the count scratch failed on device %d: %s", device,
                    hipGetErrorString(e));
    g_ptr[device] = p;
    return DT_OK;
}

size_t noalloc_capacity() { return kNoAllocScratchBytes; }

static void *noalloc_ptr(int device) {
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_mu);
    return g_ptr[device];
}

}  // namespace dt

using namespace dt;

extern "C" int dt_count_noalloc(dt_graph *g, const dt_query *q, int64_t *out8, void *hip_stream) {
    clear_error();
    if (!g) return fail(DT_EINVAL, "null graph");
    if (!g->built) return fail(DT_ENOTBUILT, "graph not built (call dt_graph_build)");
    if (!out8) return fail(DT_EINVAL, "null output");
    if (g->held_by || g->swapped)   // (bringing it back would allocate)
        return fail(DT_EBUSY, "the graph's arrays are in host memory or held by a swapping server");
    DQuery dq;
    bool empty = false;
    DT_TRY(normalise_query(g, q, &dq, &empty));
    if ((g->sum_sigma3 >> 63) != 0)
        return fail(DT_EOVERFLOW, "the sum of multiplicity products exceeds 2^63; counts may not fit int64");
    dt_ctx *ctx = g->ctx;
    int prev = -1;
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != ctx->device) DT_HIP(hipSetDevice(ctx->device));
    struct Restore {
        int prev, dev;
        ~Restore() {
            if (prev >= 0 && prev != dev) (void)hipSetDevice(prev);
        }
    } restore{prev, ctx->device};
    hipStream_t s = hip_stream ? (hipStream_t)hip_stream : ctx->stream;
    uint8_t *base = static_cast<uint8_t *>(noalloc_ptr(ctx->device));
    if (!base) return fail(DT_EDEVICE, "the count scratch of device %d was not set up", ctx->device);
    if (empty || g->n_tri == 0) {
        // the reduction of no partials: a kernel that fills the output with zeros on the stream
        count_reduce(0, reinterpret_cast<int64_t *>(base), out8, s);
        DT_HIP(hipGetLastError());
        return DT_OK;
    }
    CountPlan p;
    count_plan(g, dq, 15, p);
    const size_t part_bytes = (p.part_bytes + 255) & ~size_t(255);
    if (part_bytes + p.heavy_bytes > kNoAllocScratchBytes)
        return fail(DT_ENOMEM, "this count needs %zu bytes of scratch; the no-allocation count holds %zu",
                    part_bytes + p.heavy_bytes, kNoAllocScratchBytes);
    ScratchView sv;
    sv.part = reinterpret_cast<int64_t *>(base);
    sv.part_bytes = part_bytes;
    sv.heavy = base + part_bytes;
    sv.heavy_bytes = kNoAllocScratchBytes - part_bytes;
    // the context's side streams carry part of the count: they wait for the caller's stream and
    // are joined back into it (as in dt_count_async)
    if (s != ctx->stream) {
        DT_HIP(hipEventRecord(ctx->ev_a, ctx->stream));
        DT_HIP(hipStreamWaitEvent(s, ctx->ev_a, 0));
    }
    DT_TRY(count_launch(g, dq, p, out8, s, false, nullptr, sv));
    if (s != ctx->stream) {
        DT_HIP(hipEventRecord(ctx->ev_b, s));
        DT_HIP(hipStreamWaitEvent(ctx->stream, ctx->ev_b, 0));
    }
    return DT_OK;
}
