// Stream mode (bi_stream_*): a queue of ragged multiplication bursts.
//
// With a graph, every burst runs the ragged path with device-side binning
// into size classes and one persistent list kernel per class, each reading
// its instance count on the device, so the launch sequence does not depend on
// the burst: it is captured into a HIP graph and each submission is one
// descriptor copy plus one graph launch.  Without a graph the host, which
// validates every descriptor anyway, also bins them: the copy carries the
// class lists and counts too, and only the classes present are launched, each
// with a grid sized to its count.  Descriptors pass through staging slots, each a
// pinned host buffer and a device buffer of its own; a slot is reused only
// after the event of its previous burst has completed.  The copies run on a
// side stream, so the copy of a burst overlaps the bursts queued before it.
//
// Bursts run on kLanes lanes, each a stream of the queue's own with its own
// binning and transform scratch: burst t on lane t mod kLanes, after its
// descriptor copy, so consecutive bursts overlap on the GPU (a burst's class
// kernels are sized to its instances and rarely fill the GPU alone).  The
// lanes start after the work queued on the caller's stream at open; the
// caller's stream waits for every burst in submission order, so work queued
// there after a submission sees its results.
#include <hip/hip_runtime.h>

#include <cstring>
#include <new>

#include "bi_internal.hpp"

namespace {

constexpr int kSlots = 4;
constexpr int kLanes = 2;  // kSlots is a multiple of it: a slot always runs on the same lane
// Staging layout: count (u64) at 0, per-class counts (u32, host binning) at
// kCountsAt, descriptors from kHeader, then (host binning) the class lists.
constexpr size_t kHeader = 256;
constexpr size_t kCountsAt = 64;
static_assert(kCountsAt + 4 * bi::kNumClasses <= kHeader, "class counts fit the header");

struct Slot {
    void *host = nullptr;  // pinned: header + descriptors
    void *dev = nullptr;   // device copy of the same
    hipEvent_t copied = nullptr;  // on the copy stream
    hipEvent_t done = nullptr;    // on the queue's stream, after the burst
    hipGraphExec_t exec = nullptr;  // the captured burst that reads this slot's device copy
    uint64_t ticket = ~0ull;
};

}  // namespace

struct bi_stream {
    bi_ctx *ctx = nullptr;
    const void *a = nullptr, *b = nullptr;
    void *out = nullptr;
    uint64_t a_limbs = 0, b_limbs = 0, out_limbs = 0;
    uint32_t limb_bits = 32;
    uint64_t max_descs = 0;
    int algo = BI_MUL_AUTO;
    bi::Tune tune{};
    hipStream_t st = nullptr;
    hipStream_t copy_st = nullptr;  // descriptor copies
    hipStream_t lane_st[kLanes] = {};
    void *scratch[kLanes] = {};  // per lane: binning lists and transform scratch
    Slot slots[kSlots];
    uint64_t next = 0;
    bool graphs = false;
};

namespace {

void release(bi_stream *q) {
    for (Slot &s : q->slots) {
        if (s.exec) (void)hipGraphExecDestroy(s.exec);
        if (s.done) (void)hipEventDestroy(s.done);
        if (s.copied) (void)hipEventDestroy(s.copied);
        if (s.host) (void)hipHostFree(s.host);
        if (s.dev) (void)hipFree(s.dev);
    }
    if (q->copy_st) (void)hipStreamDestroy(q->copy_st);
    for (int l = 0; l < kLanes; ++l) {
        if (q->lane_st[l]) (void)hipStreamDestroy(q->lane_st[l]);
        if (q->scratch[l]) (void)hipFree(q->scratch[l]);
    }
    delete q;
}

// One burst over the descriptors in the device copy of slot `s`, with the
// scratch of the slot's lane.
hipError_t launch_burst(bi_stream *q, int s, hipStream_t st) {
    const Slot &slot = q->slots[s];
    const bi_desc *d = reinterpret_cast<const bi_desc *>(static_cast<char *>(slot.dev) + kHeader);
    const uint64_t *cnt = static_cast<const uint64_t *>(slot.dev);
    return bi::launch_bigmul_v_core(q->ctx->impl, q->tune, q->a, q->b, q->out, d, q->max_descs, cnt, q->limb_bits,
                                    q->algo, q->scratch[s % kLanes], st);
}

}  // namespace

extern "C" {

bi_status bi_stream_open(bi_ctx *ctx, const void *a, uint64_t a_limbs, const void *b, uint64_t b_limbs, void *out,
                         uint64_t out_limbs, uint32_t limb_bits, uint64_t max_descs, int algo, int use_graph,
                         void *stream, bi_stream **qout) {
    using bi::set_error;
    if (!qout) return set_error(BI_EINVAL, "q is NULL");
    *qout = nullptr;
    if (!ctx) return set_error(BI_EINVAL, "ctx is NULL");
    if (limb_bits != 32 && limb_bits != 64) return set_error(BI_ELIMB, "limb_bits must be 32 or 64 (got %u)", limb_bits);
    if (!a || !b || !out) return set_error(BI_EINVAL, "operand or output buffer is NULL");
    const uintptr_t al = limb_bits / 8;
    if (reinterpret_cast<uintptr_t>(a) % al || reinterpret_cast<uintptr_t>(b) % al ||
        reinterpret_cast<uintptr_t>(out) % al)
        return set_error(BI_ELIMB, "buffers must be aligned to %u-bit limbs", limb_bits);
    if (max_descs == 0 || max_descs > (uint64_t(1) << 24))
        return set_error(BI_ESIZE, "max_descs must be in [1, 2^24] (got %llu)", (unsigned long long)max_descs);
    if (algo < BI_MUL_AUTO || algo > BI_MUL_KARATSUBA) return set_error(BI_EINVAL, "unknown algorithm %d", algo);
    bi::DeviceGuard g(ctx->device);
    if (g.err != hipSuccess) return set_error(BI_EHIP, "hipSetDevice: %s", hipGetErrorString(g.err));

    bi_stream *q = new (std::nothrow) bi_stream;
    if (!q) return set_error(BI_ENOMEM, "queue allocation failed");
    q->ctx = ctx;
    q->a = a; q->b = b; q->out = out;
    q->a_limbs = a_limbs; q->b_limbs = b_limbs; q->out_limbs = out_limbs;
    q->limb_bits = limb_bits;
    q->max_descs = max_descs;
    q->algo = algo;
    q->tune = ctx->impl.tune;
    q->st = static_cast<hipStream_t>(stream);
    const size_t dbytes = kHeader + max_descs * (sizeof(bi_desc) + sizeof(uint32_t));
    for (int l = 0; l < kLanes; ++l) {
        if (hipMalloc(&q->scratch[l], bi::batch_scratch_bytes(max_descs, ctx->impl.num_cus)) != hipSuccess) {
            release(q);
            return set_error(BI_ENOMEM, "queue device buffers");
        }
        if (hipStreamCreateWithFlags(&q->lane_st[l], hipStreamNonBlocking) != hipSuccess) {
            release(q);
            return set_error(BI_EHIP, "lane stream creation");
        }
    }
    if (hipStreamCreateWithFlags(&q->copy_st, hipStreamNonBlocking) != hipSuccess) {
        release(q);
        return set_error(BI_EHIP, "copy stream creation");
    }
    for (Slot &s : q->slots) {
        if (hipMalloc(&s.dev, dbytes) != hipSuccess || hipHostMalloc(&s.host, dbytes, hipHostMallocDefault) != hipSuccess) {
            release(q);
            return set_error(BI_ENOMEM, "staging slot buffers");
        }
        if (hipEventCreateWithFlags(&s.done, hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&s.copied, hipEventDisableTiming) != hipSuccess) {
            release(q);
            return set_error(BI_EHIP, "event creation");
        }
    }
    // Every slot's device count starts at 0; one empty burst outside capture
    // sets up the launchers' per-kernel attributes.
    hipError_t e = hipSuccess;
    for (Slot &s : q->slots)
        if (e == hipSuccess) e = hipMemsetAsync(s.dev, 0, kHeader, q->st);
    if (e == hipSuccess) e = launch_burst(q, 0, q->st);
    // the lanes start after everything queued on the caller's stream so far
    if (e == hipSuccess) e = hipStreamSynchronize(q->st);
    if (e != hipSuccess) {
        release(q);
        return set_error(BI_EHIP, "queue set-up: %s", hipGetErrorString(e));
    }
    if (use_graph) {
        hipStream_t cap = nullptr;
        e = hipStreamCreateWithFlags(&cap, hipStreamNonBlocking);
        for (int si = 0; si < kSlots; ++si) {
            Slot &s = q->slots[si];
            hipGraph_t graph = nullptr;
            if (e == hipSuccess) e = hipStreamBeginCapture(cap, hipStreamCaptureModeRelaxed);
            if (e != hipSuccess) break;
            const hipError_t le = launch_burst(q, si, cap);
            e = hipStreamEndCapture(cap, &graph);
            if (le != hipSuccess) e = le;
            if (e == hipSuccess) e = hipGraphInstantiate(&s.exec, graph, nullptr, nullptr, 0);
            if (graph) (void)hipGraphDestroy(graph);
        }
        q->graphs = e == hipSuccess;
        if (cap) (void)hipStreamDestroy(cap);
        if (e != hipSuccess) {
            release(q);
            return set_error(BI_EHIP, "graph capture: %s", hipGetErrorString(e));
        }
    }
    *qout = q;
    return BI_OK;
}

bi_status bi_stream_submit(bi_stream *q, const bi_desc *descs, uint64_t count, uint64_t *ticket) {
    using bi::set_error;
    if (!q || !descs || !ticket) return set_error(BI_EINVAL, "NULL argument");
    if (count == 0 || count > q->max_descs)
        return set_error(BI_ESIZE, "count must be in [1, %llu] (got %llu)", (unsigned long long)q->max_descs,
                         (unsigned long long)count);
    const uint64_t maxn = BI_MAX_BITS / q->limb_bits;
    for (uint64_t i = 0; i < count; ++i) {
        const bi_desc &d = descs[i];
        if (d.reserved != 0) return set_error(BI_EINVAL, "descriptor %llu: reserved is not 0", (unsigned long long)i);
        if (d.n_limbs == 0 || d.n_limbs > maxn)
            return set_error(BI_ESIZE, "descriptor %llu: n_limbs %u outside [1, %llu]", (unsigned long long)i,
                             d.n_limbs, (unsigned long long)maxn);
        const uint64_t n = d.n_limbs;
        if (d.a_off > q->a_limbs || q->a_limbs - d.a_off < n || d.b_off > q->b_limbs || q->b_limbs - d.b_off < n ||
            d.out_off > q->out_limbs || q->out_limbs - d.out_off < 2 * n)
            return set_error(BI_EINVAL, "descriptor %llu: range outside its buffer", (unsigned long long)i);
    }
    bi::DeviceGuard g(q->ctx->device);
    if (g.err != hipSuccess) return set_error(BI_EHIP, "hipSetDevice: %s", hipGetErrorString(g.err));
    const uint64_t t = q->next;
    Slot &s = q->slots[t % kSlots];
    const int lane = int(t % kSlots) % kLanes;
    const hipStream_t ls = q->lane_st[lane];
    if (s.ticket != ~0ull) {
        const hipError_t e = hipEventSynchronize(s.done);
        if (e != hipSuccess) return set_error(BI_EHIP, "staging slot wait: %s", hipGetErrorString(e));
    }
    char *h = static_cast<char *>(s.host);
    std::memset(h, 0, kHeader);
    std::memcpy(h, &count, sizeof count);
    std::memcpy(h + kHeader, descs, count * sizeof(bi_desc));
    size_t bytes = kHeader + count * sizeof(bi_desc);
    uint32_t counts[bi::kNumClasses] = {};
    if (!q->graphs) {  // bin on the host: counts, then the lists in class order
        const uint32_t wpl = q->limb_bits / 32;
        uint32_t next[bi::kNumClasses];
        for (uint64_t i = 0; i < count; ++i) ++counts[bi::size_class_host(descs[i].n_limbs * wpl)];
        for (uint32_t k = 0, o = 0; k < bi::kNumClasses; ++k) {
            next[k] = o;
            o += counts[k];
        }
        uint32_t *lists = reinterpret_cast<uint32_t *>(h + bytes);
        for (uint64_t i = 0; i < count; ++i) lists[next[bi::size_class_host(descs[i].n_limbs * wpl)]++] = uint32_t(i);
        std::memcpy(h + kCountsAt, counts, sizeof counts);
        bytes += count * sizeof(uint32_t);
    }
    hipError_t e = hipMemcpyAsync(s.dev, s.host, bytes, hipMemcpyHostToDevice, q->copy_st);
    if (e == hipSuccess) e = hipEventRecord(s.copied, q->copy_st);
    if (e == hipSuccess) e = hipStreamWaitEvent(ls, s.copied, 0);
    if (e == hipSuccess) {
        if (q->graphs) {
            e = hipGraphLaunch(s.exec, ls);
        } else {
            char *d = static_cast<char *>(s.dev);
            e = bi::launch_bigmul_v_binned(q->ctx->impl, q->tune, q->a, q->b, q->out,
                                           reinterpret_cast<const bi_desc *>(d + kHeader),
                                           reinterpret_cast<const uint32_t *>(d + kHeader + count * sizeof(bi_desc)),
                                           reinterpret_cast<const uint32_t *>(d + kCountsAt), counts, q->limb_bits,
                                           q->algo, q->scratch[lane], ls);
        }
    }
    if (e == hipSuccess) e = hipEventRecord(s.done, ls);
    // the caller's stream sees the bursts complete in submission order
    if (e == hipSuccess) e = hipStreamWaitEvent(q->st, s.done, 0);
    if (e != hipSuccess) return set_error(BI_EHIP, "burst launch: %s", hipGetErrorString(e));
    s.ticket = t;
    q->next = t + 1;
    *ticket = t;
    return BI_OK;
}

bi_status bi_stream_poll(bi_stream *q, uint64_t ticket, int *done) {
    using bi::set_error;
    if (!q || !done) return set_error(BI_EINVAL, "NULL argument");
    if (ticket >= q->next) return set_error(BI_EINVAL, "ticket %llu was not issued", (unsigned long long)ticket);
    const Slot &s = q->slots[ticket % kSlots];
    if (s.ticket != ticket) {  // the slot was reused, which waited for this burst
        *done = 1;
        return BI_OK;
    }
    const hipError_t e = hipEventQuery(s.done);
    if (e == hipSuccess) { *done = 1; return BI_OK; }
    if (e == hipErrorNotReady) { *done = 0; return BI_OK; }
    return set_error(BI_EHIP, "poll: %s", hipGetErrorString(e));
}

bi_status bi_stream_wait(bi_stream *q, uint64_t ticket) {
    using bi::set_error;
    if (!q) return set_error(BI_EINVAL, "q is NULL");
    if (ticket >= q->next) return set_error(BI_EINVAL, "ticket %llu was not issued", (unsigned long long)ticket);
    const Slot &s = q->slots[ticket % kSlots];
    if (s.ticket != ticket) return BI_OK;
    const hipError_t e = hipEventSynchronize(s.done);
    if (e != hipSuccess) return set_error(BI_EHIP, "wait: %s", hipGetErrorString(e));
    return BI_OK;
}

bi_status bi_stream_close(bi_stream *q) {
    if (!q) return BI_OK;
    bi::DeviceGuard g(q->ctx->device);
    hipError_t first = g.err;
    for (Slot &s : q->slots) {
        if (s.ticket != ~0ull) {
            const hipError_t e = hipEventSynchronize(s.done);
            if (first == hipSuccess) first = e;
        }
    }
    release(q);
    if (first != hipSuccess) return bi::set_error(BI_EHIP, "close: %s", hipGetErrorString(first));
    return BI_OK;
}

}  // extern "C"
