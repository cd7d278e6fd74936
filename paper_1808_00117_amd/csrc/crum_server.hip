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

#include <hip/hip_runtime.h>

#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

using crum::check_ranges;
using crum::DeviceGuard;
using crum::page_size_ok;

namespace {

using Clock = std::chrono::steady_clock;

// First-fit allocator over one pinned arena (4 KiB granules).
class Arena {
public:
    bool init(uint64_t bytes)
    {
        if (hipHostMalloc(reinterpret_cast<void**>(&base_), bytes, 0) != hipSuccess)
            return false;
        size_ = bytes;
        free_[0] = bytes;
        return true;
    }
    ~Arena()
    {
        if (base_)
            (void)hipHostFree(base_);
    }
    // returns offset or UINT64_MAX when no block is large enough
    uint64_t alloc(uint64_t n)
    {
        n = (n + 4095) & ~4095ull;
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= n) {
                const uint64_t off = it->first, rest = it->second - n;
                free_.erase(it);
                if (rest)
                    free_[off + n] = rest;
                used_ += n;
                return off;
            }
        }
        return UINT64_MAX;
    }
    void release(uint64_t off, uint64_t n)
    {
        n = (n + 4095) & ~4095ull;
        used_ -= n;
        auto it = free_.emplace(off, n).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    uint8_t* ptr(uint64_t off) const { return base_ + off; }
    uint64_t size() const { return size_; }
    uint64_t used() const { return used_; }

private:
    uint8_t* base_ = nullptr;
    uint64_t size_ = 0, used_ = 0;
    std::map<uint64_t, uint64_t> free_;
};

struct Request {
    uint64_t id;
    uint32_t client;
    uint32_t kind;
    uint64_t tag;
    double arrival;
};

struct Client {
    std::vector<crum_region> regions;
    uint32_t page_size = 0;
    uint64_t worst = 0;
    std::deque<Request> queue;
    bool busy = false;
    uint64_t seq = 0;
    bool has_image = false;
    uint64_t img_off = 0, img_bytes = 0;
};

}  // namespace

struct crum_server {
    int device = 0;
    std::vector<Client> clients;
    Arena arena;
    std::mutex mu;
    std::condition_variable cv_work, cv_budget, cv_done;
    std::deque<uint32_t> ready;  // clients with a queued head request, in arrival order
    std::vector<crum_server_completion> done;
    uint64_t next_id = 0, in_flight = 0, queued = 0;
    bool stop = false;
    std::vector<std::thread> workers;
    crum_server_prepare_fn prepare = nullptr;
    void* prepare_user = nullptr;
    Clock::time_point t0;
    std::atomic<int> fatal{0};
    uint64_t max_worst = 0;
    int policy = CRUM_SERVE_ADAPTIVE;
};

namespace {

double now_s(const crum_server* s)
{
    return std::chrono::duration<double>(Clock::now() - s->t0).count();
}

// Reserve pinned bytes, waiting while the budget is exhausted (at most
// kReserveWaitS seconds). Called with the lock held; returns UINT64_MAX if
// the bytes never become free.
constexpr double kReserveWaitS = 30.0;

uint64_t reserve(crum_server* s, std::unique_lock<std::mutex>& lk, uint64_t n)
{
    if (((n + 4095) & ~4095ull) > s->arena.size())
        return UINT64_MAX;
    const auto deadline = Clock::now() + std::chrono::duration<double>(kReserveWaitS);
    for (;;) {
        const uint64_t off = s->arena.alloc(n);
        if (off != UINT64_MAX || s->stop)
            return off;
        if (s->cv_budget.wait_until(lk, deadline) == std::cv_status::timeout)
            return s->arena.alloc(n);
    }
}

void worker(crum_server* s, int slot)
{
    DeviceGuard g(s->device);
    crum_ctx* ctx = nullptr;
    hipStream_t stream = nullptr;
    uint8_t* staging = nullptr;
    crum_status* st = nullptr;
    if (crum_ctx_create(s->device, &ctx) != CRUM_OK ||
        hipStreamCreateWithFlags(&stream, hipStreamNonBlocking) != hipSuccess ||
        hipMalloc(reinterpret_cast<void**>(&staging), std::max<uint64_t>(s->max_worst, 4096)) !=
            hipSuccess ||
        hipHostMalloc(reinterpret_cast<void**>(&st), sizeof(crum_status), 0) != hipSuccess) {
        // release what was created; the server reports CRUM_EHIP from now on
        if (st)
            (void)hipHostFree(st);
        if (staging)
            (void)hipFree(staging);
        if (stream)
            (void)hipStreamDestroy(stream);
        crum_ctx_destroy(ctx);
        s->fatal = 1;
        std::lock_guard<std::mutex> lk(s->mu);
        s->cv_done.notify_all();
        return;
    }
    (void)slot;
    for (;;) {
        Request rq;
        {
            std::unique_lock<std::mutex> lk(s->mu);
            s->cv_work.wait(lk, [&] { return s->stop || !s->ready.empty(); });
            if (s->stop && s->ready.empty())
                break;
            const uint32_t c = s->ready.front();
            s->ready.pop_front();
            Client& cl = s->clients[c];
            rq = cl.queue.front();
            cl.queue.pop_front();
            cl.busy = true;
            s->queued -= 1;
            s->in_flight += 1;
        }
        Client& cl = s->clients[rq.client];
        crum_server_completion out{};
        out.id = rq.id;
        out.tag = rq.tag;
        out.client = rq.client;
        out.kind = rq.kind;
        out.arrival_s = rq.arrival;
        out.start_s = now_s(s);
        if (s->prepare)
            s->prepare(s->prepare_user, rq.client, rq.kind, rq.tag, stream);
        int code = CRUM_OK;
        if (rq.kind == CRUM_REQ_SNAPSHOT) {
            // Fast path: when the arena can hold the client's worst-case image
            // right now, reserve it, let the snapshot drain into it while it
            // runs (pipelined order), then trim the reservation to the image.
            const uint64_t worst_r = (cl.worst + 4095) & ~4095ull;
            uint64_t off = UINT64_MAX;
            {
                std::lock_guard<std::mutex> lk(s->mu);
                const bool fast = s->policy == CRUM_SERVE_PIPELINED ||
                                  (s->policy == CRUM_SERVE_ADAPTIVE && s->queued == 0);
                if (fast)
                    off = s->arena.alloc(cl.worst);
            }
            if (off != UINT64_MAX) {
                uint8_t* dst = s->arena.ptr(off);
                int rc = crum_snapshot(ctx, cl.regions.data(), (uint32_t)cl.regions.size(),
                                       cl.page_size, CRUM_UPDATE_SHADOW, ++cl.seq, staging,
                                       cl.worst, dst, worst_r, stream, st);
                if (rc == CRUM_OK && hipStreamSynchronize(stream) != hipSuccess)
                    rc = CRUM_EHIP;
                code = rc != CRUM_OK ? rc : st->code;
                std::lock_guard<std::mutex> lk(s->mu);
                if (code == CRUM_OK) {
                    out.n_dirty = st->n_dirty;
                    out.image_bytes = st->image_bytes;
                    std::memcpy(&out.meta_crc, dst + 56, 4);
                    std::memcpy(&out.crcs_crc, dst + 60, 4);
                    const uint64_t keep = (st->image_bytes + 4095) & ~4095ull;
                    if (keep < worst_r)
                        s->arena.release(off + keep, worst_r - keep);
                    if (cl.has_image)
                        s->arena.release(cl.img_off, cl.img_bytes);
                    cl.has_image = true;
                    cl.img_off = off;
                    cl.img_bytes = st->image_bytes;
                } else {
                    s->arena.release(off, worst_r);
                }
                s->cv_budget.notify_all();
            } else {
            // stage 1: build the image on the device, learn its exact size
            int rc = crum_snapshot(ctx, cl.regions.data(), (uint32_t)cl.regions.size(),
                                   cl.page_size, CRUM_UPDATE_SHADOW, ++cl.seq, staging,
                                   cl.worst, nullptr, 0, stream, st);
            if (rc == CRUM_OK && hipStreamSynchronize(stream) != hipSuccess)
                rc = CRUM_EHIP;
            code = rc != CRUM_OK ? rc : st->code;
            if (code == CRUM_OK) {
                out.n_dirty = st->n_dirty;
                out.image_bytes = st->image_bytes;
                // stage 2: the shadow now holds this snapshot, so the previous
                // delta image is obsolete; reserve exactly the new image's
                // bytes and drain into them
                uint64_t off2;
                {
                    std::unique_lock<std::mutex> lk(s->mu);
                    if (cl.has_image) {
                        s->arena.release(cl.img_off, cl.img_bytes);
                        cl.has_image = false;
                        s->cv_budget.notify_all();
                    }
                    off2 = reserve(s, lk, st->image_bytes);
                }
                if (off2 == UINT64_MAX) {
                    code = CRUM_ENOSPC;
                } else {
                    uint8_t* dst = s->arena.ptr(off2);
                    if (hipMemcpyAsync(dst, staging, st->image_bytes, hipMemcpyDeviceToHost,
                                       stream) != hipSuccess ||
                        hipStreamSynchronize(stream) != hipSuccess) {
                        code = CRUM_EHIP;
                        std::lock_guard<std::mutex> lk(s->mu);
                        s->arena.release(off2, st->image_bytes);
                        s->cv_budget.notify_all();
                    } else {
                        std::memcpy(&out.meta_crc, dst + 56, 4);
                        std::memcpy(&out.crcs_crc, dst + 60, 4);
                        std::lock_guard<std::mutex> lk(s->mu);
                        cl.has_image = true;
                        cl.img_off = off2;
                        cl.img_bytes = st->image_bytes;
                        s->cv_budget.notify_all();
                    }
                }
            }
            }
        } else {
            if (!cl.has_image) {
                code = CRUM_EINVAL;
            } else {
                int rc = crum_restore(ctx, cl.regions.data(), (uint32_t)cl.regions.size(),
                                      s->arena.ptr(cl.img_off), cl.img_bytes,
                                      CRUM_VERIFY | CRUM_UPDATE_SHADOW, staging, cl.worst,
                                      stream, st);
                if (rc == CRUM_OK && hipStreamSynchronize(stream) != hipSuccess)
                    rc = CRUM_EHIP;
                code = rc != CRUM_OK ? rc : st->code;
                out.n_dirty = st->n_dirty;
                out.image_bytes = cl.img_bytes;
                std::memcpy(&out.meta_crc, s->arena.ptr(cl.img_off) + 56, 4);
                std::memcpy(&out.crcs_crc, s->arena.ptr(cl.img_off) + 60, 4);
            }
        }
        out.code = code;
        out.done_s = now_s(s);
        {
            std::lock_guard<std::mutex> lk(s->mu);
            s->done.push_back(out);
            s->in_flight -= 1;
            cl.busy = false;
            if (!cl.queue.empty())
                s->ready.push_back(rq.client);
            s->cv_work.notify_all();
            s->cv_done.notify_all();
        }
    }
    (void)hipStreamSynchronize(stream);
    (void)hipFree(staging);
    (void)hipHostFree(st);
    (void)hipStreamDestroy(stream);
    crum_ctx_destroy(ctx);
}

}  // namespace

extern "C" {

int crum_server_create(int device, const crum_client* clients, uint32_t n_clients,
                       uint32_t n_slots, uint64_t pinned_budget, crum_server** out)
{
    if (!out || (n_clients && !clients) || n_slots == 0 || n_slots > 64 || pinned_budget < 4096)
        return CRUM_EINVAL;
    *out = nullptr;
    std::vector<crum_region> all;
    crum_server* s = new crum_server();
    s->device = device;
    s->clients.resize(n_clients);
    for (uint32_t c = 0; c < n_clients; ++c) {
        const crum_client& d = clients[c];
        if ((d.n_regions && !d.regions) || !page_size_ok(d.page_size)) {
            delete s;
            return CRUM_EINVAL;
        }
        Client& cl = s->clients[c];
        cl.regions.assign(d.regions, d.regions + d.n_regions);
        cl.page_size = d.page_size;
        uint64_t G = 0;
        for (const crum_region& r : cl.regions) {
            if (r.len % d.page_size || !r.shadow) {
                delete s;
                return CRUM_EINVAL;  // served clients keep a resident shadow
            }
            G += r.len / d.page_size;
            all.push_back(r);
        }
        if (crum_image_bytes(d.n_regions, G, G, d.page_size, &cl.worst) != CRUM_OK) {
            delete s;
            return CRUM_EINVAL;
        }
        s->max_worst = std::max(s->max_worst, cl.worst);
    }
    if (check_ranges(all.data(), (uint32_t)all.size()) != CRUM_OK) {
        delete s;
        return CRUM_EINVAL;
    }
    {
        DeviceGuard g(device);
        if (!s->arena.init(pinned_budget)) {
            delete s;
            return CRUM_EHIP;
        }
    }
    s->t0 = Clock::now();
    for (uint32_t i = 0; i < n_slots; ++i)
        s->workers.emplace_back(worker, s, (int)i);
    *out = s;
    return CRUM_OK;
}

int crum_server_set_policy(crum_server* s, int policy)
{
    if (!s || policy < CRUM_SERVE_ADAPTIVE || policy > CRUM_SERVE_PIPELINED)
        return CRUM_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    s->policy = policy;
    return CRUM_OK;
}

int crum_server_set_prepare(crum_server* s, crum_server_prepare_fn fn, void* user)
{
    if (!s)
        return CRUM_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    s->prepare = fn;
    s->prepare_user = user;
    return CRUM_OK;
}

double crum_server_time(crum_server* s) { return s ? now_s(s) : 0.0; }

int crum_server_submit(crum_server* s, uint32_t client, uint32_t kind, uint64_t tag,
                       uint64_t* id)
{
    if (!s || client >= s->clients.size() ||
        (kind != CRUM_REQ_SNAPSHOT && kind != CRUM_REQ_RESTORE))
        return CRUM_EINVAL;
    if (s->fatal)
        return CRUM_EHIP;
    std::lock_guard<std::mutex> lk(s->mu);
    Request r{s->next_id++, client, kind, tag, now_s(s)};
    Client& cl = s->clients[client];
    const bool was_idle = cl.queue.empty() && !cl.busy;
    cl.queue.push_back(r);
    s->queued += 1;
    if (was_idle)
        s->ready.push_back(client);
    if (id)
        *id = r.id;
    s->cv_work.notify_one();
    return CRUM_OK;
}

int crum_server_poll(crum_server* s, crum_server_completion* out, uint32_t max, uint32_t* n,
                     int wait_all)
{
    if (!s || !n || (max && !out))
        return CRUM_EINVAL;
    std::unique_lock<std::mutex> lk(s->mu);
    if (wait_all)
        s->cv_done.wait(lk, [&] { return s->fatal || (s->queued == 0 && s->in_flight == 0); });
    const uint32_t k = (uint32_t)std::min<size_t>(max, s->done.size());
    for (uint32_t i = 0; i < k; ++i)
        out[i] = s->done[i];
    s->done.erase(s->done.begin(), s->done.begin() + k);
    *n = k;
    return s->fatal ? CRUM_EHIP : CRUM_OK;
}

int crum_server_pinned_used(crum_server* s, uint64_t* bytes)
{
    if (!s || !bytes)
        return CRUM_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    *bytes = s->arena.used();
    return CRUM_OK;
}

int crum_server_latest_image(crum_server* s, uint32_t client, const void** ptr, uint64_t* bytes)
{
    if (!s || client >= s->clients.size() || !ptr || !bytes)
        return CRUM_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    const Client& cl = s->clients[client];
    if (!cl.has_image)
        return CRUM_EINVAL;
    *ptr = s->arena.ptr(cl.img_off);
    *bytes = cl.img_bytes;
    return CRUM_OK;
}

void crum_server_destroy(crum_server* s)
{
    if (!s)
        return;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
        s->cv_work.notify_all();
        s->cv_budget.notify_all();
    }
    for (auto& t : s->workers)
        t.join();
    delete s;
}

}  // extern "C"
