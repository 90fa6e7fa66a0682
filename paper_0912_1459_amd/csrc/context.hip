// Context, error text, workspace and event-timer plumbing of the cdsigma library.
#include "cds_internal.h"

#include <cstdlib>
#include <cstring>

int cds_fail(cds_ctx *ctx, int code, const char *fmt, ...)
{
    if (ctx) {
        char buf[1024];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        ctx->err = buf;
        if (code == CDS_EDEVICE) ctx->broken = true;
    }
    return code;
}

int cds_enter(cds_ctx *ctx)
{
    if (!ctx) return CDS_EINVAL;
    ctx->err.clear();
    if (ctx->broken)
        return cds_fail(ctx, CDS_ESTATE, "context unusable after an earlier device error");
    CDS_HIP(ctx, hipSetDevice(ctx->device));
    return CDS_OK;
}

int cds_ws(cds_ctx *ctx, int slot, size_t bytes, void **out)
{
    if (bytes == 0) bytes = 256;
    if (ctx->ws_bytes[slot] < bytes) {
        if (ctx->ws[slot]) {
            CDS_HIP(ctx, hipStreamSynchronize(ctx->stream));
            if (ctx->stream2) CDS_HIP(ctx, hipStreamSynchronize(ctx->stream2));
            CDS_HIP(ctx, hipFree(ctx->ws[slot]));
            ctx->ws[slot] = nullptr;
            ctx->ws_bytes[slot] = 0;
        }
        size_t want = bytes + bytes / 8;          // grow with headroom
        want = (want + 255) & ~(size_t)255;
        hipError_t e = hipMalloc(&ctx->ws[slot], want);
        if (e != hipSuccess) {
            ctx->ws[slot] = nullptr;
            return cds_fail(ctx, CDS_ENOMEM, "workspace slot %d: hipMalloc(%zu) failed: %s", slot,
                            want, hipGetErrorString(e));
        }
        ctx->ws_bytes[slot] = want;
    }
    *out = ctx->ws[slot];
    return CDS_OK;
}

int cds_pinned(cds_ctx *ctx, size_t bytes, void **out)
{
    if (ctx->pinned_bytes < bytes) {
        if (ctx->pinned) {
            CDS_HIP(ctx, hipStreamSynchronize(ctx->stream));
            CDS_HIP(ctx, hipHostFree(ctx->pinned));
            ctx->pinned = nullptr;
        }
        size_t want = bytes < 4096 ? 4096 : bytes;
        CDS_HIP(ctx, hipHostMalloc(&ctx->pinned, want, hipHostMallocDefault));
        ctx->pinned_bytes = want;
    }
    *out = ctx->pinned;
    return CDS_OK;
}

static int get_event(cds_ctx *ctx, hipEvent_t *e)
{
    if (!ctx->free_events.empty()) {
        *e = ctx->free_events.back();
        ctx->free_events.pop_back();
        return CDS_OK;
    }
    CDS_HIP(ctx, hipEventCreate(e));
    return CDS_OK;
}

int cds_timer_start(cds_ctx *ctx, CdsTimer *t)
{
    CDS_CALL(get_event(ctx, &t->a));
    CDS_HIP(ctx, hipEventRecord(t->a, ctx->stream));
    return CDS_OK;
}

int cds_timer_stop(cds_ctx *ctx, CdsTimer *t, double *acc)
{
    CDS_CALL(get_event(ctx, &t->b));
    CDS_HIP(ctx, hipEventRecord(t->b, ctx->stream));
    t->acc = acc;
    ctx->pending.push_back(*t);
    return CDS_OK;
}

int cds_timers_flush(cds_ctx *ctx)
{
    if (ctx->pending.empty()) return CDS_OK;
    CDS_HIP(ctx, hipStreamSynchronize(ctx->stream));
    for (auto &t : ctx->pending) {
        float ms = 0.f;
        CDS_HIP(ctx, hipEventElapsedTime(&ms, t.a, t.b));
        *t.acc += ms;
        ctx->free_events.push_back(t.a);
        ctx->free_events.push_back(t.b);
    }
    ctx->pending.clear();
    return CDS_OK;
}

extern "C" {

const char *cds_version(void) { return "cdsigma 0.1 (gfx950)"; }

int cds_create(int device, void *hip_stream, cds_ctx **out)
{
    if (!out) return CDS_EINVAL;
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return CDS_EINVAL;
    if (hipSetDevice(device) != hipSuccess) return CDS_EDEVICE;
    cds_ctx *c = new (std::nothrow) cds_ctx();
    if (!c) return CDS_ENOMEM;
    c->device = device;
    c->stream = (hipStream_t)hip_stream;
    // the allocation-free path's array on this device (its name is no device address)
    if (cds_noalloc_scratch_address(&c->scratch) != CDS_OK) c->scratch = nullptr;
    *out = c;
    return CDS_OK;
}

void cds_destroy(cds_ctx *ctx)
{
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    if (ctx->stream2) {
        (void)hipStreamSynchronize(ctx->stream2);
        (void)hipStreamDestroy(ctx->stream2);
    }
    if (ctx->join) (void)hipEventDestroy(ctx->join);
    if (ctx->gate) (void)hipEventDestroy(ctx->gate);
    if (ctx->trset) (void)hipEventDestroy(ctx->trset);
    for (auto &t : ctx->pending) {
        (void)hipEventDestroy(t.a);
        (void)hipEventDestroy(t.b);
    }
    for (auto e : ctx->free_events) (void)hipEventDestroy(e);
    for (int s = 0; s < WS_SLOTS; ++s)
        if (ctx->ws[s]) (void)hipFree(ctx->ws[s]);
    if (ctx->pinned) (void)hipHostFree(ctx->pinned);
    if (ctx->mail) (void)hipHostFree(ctx->mail);
    delete ctx;
}

const char *cds_last_error(const cds_ctx *ctx) { return ctx ? ctx->err.c_str() : "null context"; }

int cds_workspace_bytes(const cds_ctx *ctx, size_t *out)
{
    if (!ctx || !out) return CDS_EINVAL;
    size_t n = 0;
    for (int i = 0; i < WS_SLOTS; ++i) n += ctx->ws_bytes[i];
    *out = n;
    return CDS_OK;
}

int cds_get_stats(const cds_ctx *ctx, cds_stats *out)
{
    if (!ctx || !out) return CDS_EINVAL;
    cds_ctx *c = const_cast<cds_ctx *>(ctx);
    CDS_CALL(cds_timers_flush(c));
    *out = c->stats;
    return CDS_OK;
}

int cds_reset_stats(cds_ctx *ctx)
{
    if (!ctx) return CDS_EINVAL;
    CDS_CALL(cds_timers_flush(ctx));
    ctx->stats = cds_stats{};
    return CDS_OK;
}

}  // extern "C"
