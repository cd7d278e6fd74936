// Serving: a request loop for many clients, each owning persistent device
// state (current regions and their shadows).  Requests (snapshot or restore)
// are queued per client and run first-in first-out per client, so a client's
// results never depend on the other clients.  Worker slots take the oldest
// ready request of any idle client and run it on their own context, streams
// and device staging buffer, so requests of different clients overlap on the
// device: one slot's diff and pack run on the compute units while other
// slots' drains run on the copy engines.
//
// A snapshot is admitted against the pinned-memory budget in one of two ways.
// When the arena can hold the client's worst-case image at once, that much is
// reserved, the snapshot drains into it while it runs (its pipelined order),
// and the reservation is then trimmed to the image.  Otherwise the image is
// first built in the slot's device staging (its exact size is then known),
// exactly that many pinned bytes are reserved -- waiting while the budget is
// exhausted -- and the image is drained into them.  A client's latest image
// stays reserved until its next snapshot completes; a restore request
// re-applies it (verified) into the client's regions.
#include "crum.h"
#include "crum_internal.h"
#include "crum_serve_core.h"

#include <hip/hip_runtime.h>

#include <vector>

using crum::check_ranges;
using crum::DeviceGuard;
using crum::page_size_ok;

namespace {

// Device work of the serving loop on libcrum: each slot owns a context, a
// stream, a device staging buffer sized for the largest client's worst-case
// image and a pinned status.  Every call waits for its stream.
struct HipBackend {
    int device = 0;
    struct Slot {
        crum_ctx* ctx = nullptr;
        hipStream_t stream = nullptr;
        uint8_t* staging = nullptr;
        uint64_t staging_bytes = 0;
        crum_status* st = nullptr;
    };

    bool open(Slot& s, uint64_t staging_bytes)
    {
        DeviceGuard g(device);
        if (crum_ctx_create(device, nullptr, &s.ctx) != CRUM_OK ||
            hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking) != hipSuccess ||
            hipMalloc(reinterpret_cast<void**>(&s.staging), staging_bytes) != hipSuccess ||
            hipHostMalloc(reinterpret_cast<void**>(&s.st), sizeof(crum_status), 0) != hipSuccess)
            return false;
        s.staging_bytes = staging_bytes;
        return true;
    }
    void close(Slot& s)
    {
        DeviceGuard g(device);
        if (s.stream)
            (void)hipStreamSynchronize(s.stream);
        if (s.st)
            (void)hipHostFree(s.st);
        if (s.staging)
            (void)hipFree(s.staging);
        if (s.stream)
            (void)hipStreamDestroy(s.stream);
        crum_ctx_destroy(s.ctx);
        s = Slot{};
    }
    void* stream(Slot& s) { return s.stream; }

    int wait(Slot& s, int rc)
    {
        if (rc == CRUM_OK && hipStreamSynchronize(s.stream) != hipSuccess)
            rc = CRUM_EHIP;
        return rc;
    }
    static void take(const crum_status* st, crum::serve::SnapOut* o)
    {
        o->code = st->code;
        o->n_dirty = st->n_dirty;
        o->image_bytes = st->image_bytes;
    }
    int snapshot(Slot& s, const crum::serve::Client& cl, uint64_t seq, uint8_t* dst,
                 uint64_t dst_cap, crum::serve::SnapOut* o)
    {
        DeviceGuard g(device);
        const int rc = wait(s, crum_snapshot(s.ctx, cl.regions.data(), (uint32_t)cl.regions.size(),
                                             cl.page_size, CRUM_UPDATE_SHADOW, seq, s.staging,
                                             cl.worst, dst, dst ? dst_cap : 0, s.stream, s.st));
        if (rc == CRUM_OK)
            take(s.st, o);
        return rc;
    }
    int drain(Slot& s, uint8_t* dst, uint64_t n)
    {
        DeviceGuard g(device);
        if (hipMemcpyAsync(dst, s.staging, n, hipMemcpyDeviceToHost, s.stream) != hipSuccess)
            return CRUM_EHIP;
        return wait(s, CRUM_OK);
    }
    int restore(Slot& s, const crum::serve::Client& cl, const uint8_t* img, uint64_t n,
                crum::serve::SnapOut* o)
    {
        DeviceGuard g(device);
        const int rc = wait(s, crum_restore(s.ctx, cl.regions.data(), (uint32_t)cl.regions.size(),
                                            img, n, CRUM_VERIFY | CRUM_UPDATE_SHADOW, s.staging,
                                            cl.worst, s.stream, s.st));
        if (rc == CRUM_OK)
            take(s.st, o);
        return rc;
    }
};

}  // namespace

struct crum_server {
    int device = 0;
    uint8_t* arena = nullptr;  // pinned
    crum::serve::Core<HipBackend>* core = nullptr;
};

extern "C" {

int crum_server_create(int device, const crum_client* clients, uint32_t n_clients,
                       uint32_t n_slots, uint64_t pinned_budget, crum_server** out)
{
    if (!out || (n_clients && !clients) || n_slots == 0 || n_slots > 64 || pinned_budget < 4096)
        return CRUM_EINVAL;
    *out = nullptr;
    std::vector<crum_region> all;
    std::vector<crum::serve::Client> cls(n_clients);
    for (uint32_t c = 0; c < n_clients; ++c) {
        const crum_client& d = clients[c];
        if ((d.n_regions && !d.regions) || !page_size_ok(d.page_size))
            return CRUM_EINVAL;
        crum::serve::Client& cl = cls[c];
        cl.regions.assign(d.regions, d.regions + d.n_regions);
        cl.page_size = d.page_size;
        uint64_t G = 0;
        for (const crum_region& r : cl.regions) {
            if (r.len % d.page_size || !r.shadow)
                return CRUM_EINVAL;  // served clients keep a resident shadow
            G += r.len / d.page_size;
            all.push_back(r);
        }
        if (crum_image_bytes(d.n_regions, G, G, d.page_size, &cl.worst) != CRUM_OK)
            return CRUM_EINVAL;
    }
    if (check_ranges(all.data(), (uint32_t)all.size()) != CRUM_OK)
        return CRUM_EINVAL;
    int n_dev = 0;
    if (hipGetDeviceCount(&n_dev) != hipSuccess)
        return CRUM_EHIP;
    if (device < 0 || device >= n_dev)
        return CRUM_EINVAL;
    crum_server* s = new crum_server();
    s->device = device;
    {
        DeviceGuard g(device);
        if (hipHostMalloc(reinterpret_cast<void**>(&s->arena), pinned_budget, 0) != hipSuccess) {
            delete s;
            return CRUM_EHIP;
        }
    }
    HipBackend be;
    be.device = device;
    s->core = new crum::serve::Core<HipBackend>(be);
    s->core->init(std::move(cls), s->arena, pinned_budget);
    s->core->start(n_slots);
    *out = s;
    return CRUM_OK;
}

int crum_server_set_policy(crum_server* s, int policy)
{
    if (!s)
        return CRUM_EINVAL;
    return s->core->set_policy(policy);
}

int crum_server_set_prepare(crum_server* s, crum_server_prepare_fn fn, void* user)
{
    if (!s)
        return CRUM_EINVAL;
    s->core->set_prepare(fn, user);
    return CRUM_OK;
}

double crum_server_time(crum_server* s) { return s ? s->core->now() : 0.0; }

int crum_server_submit(crum_server* s, uint32_t client, uint32_t kind, uint64_t tag,
                       uint64_t* id)
{
    if (!s)
        return CRUM_EINVAL;
    return s->core->submit(client, kind, tag, id);
}

int crum_server_poll(crum_server* s, crum_server_completion* out, uint32_t max, uint32_t* n,
                     int wait_all)
{
    if (!s || !n || (max && !out))
        return CRUM_EINVAL;
    return s->core->poll(out, max, n, wait_all);
}

int crum_server_pinned_used(crum_server* s, uint64_t* bytes)
{
    if (!s || !bytes)
        return CRUM_EINVAL;
    *bytes = s->core->pinned_used();
    return CRUM_OK;
}

int crum_server_latest_image(crum_server* s, uint32_t client, const void** ptr, uint64_t* bytes)
{
    if (!s || !ptr || !bytes)
        return CRUM_EINVAL;
    return s->core->latest_image(client, ptr, bytes);
}

void crum_server_destroy(crum_server* s)
{
    if (!s)
        return;
    s->core->stop_workers();
    delete s->core;
    {
        DeviceGuard g(s->device);
        (void)hipHostFree(s->arena);
    }
    delete s;
}

}  // extern "C"
