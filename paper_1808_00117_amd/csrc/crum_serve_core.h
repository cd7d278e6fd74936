// Scheduling core of the serving loop, host-only (no HIP types): per-client
// FIFO queues, worker slots, pinned-arena admission and completion records.
// The device work of a request -- snapshot, drain, restore -- is done by a
// backend, so the same scheduling code runs on the GPU (libcrum's backend,
// crum_server.hip) and on the CPU under sanitizers with a stub backend.
//
// Backend B provides (each call synchronous; calls on distinct slots may run
// concurrently from different threads):
//   struct Slot;                                  per-worker state
//   bool open(Slot&, uint64_t staging_bytes)      false: the worker cannot run
//   void close(Slot&)                             after a failed open too
//   void* stream(Slot&)                           handed to the prepare hook
//   int snapshot(Slot&, const Client&, uint64_t seq, uint8_t* dst,
//                uint64_t dst_cap, SnapOut*)      dst == nullptr: build the
//                                                 image in the slot's staging
//   int drain(Slot&, uint8_t* dst, uint64_t n)    staging -> dst
//   int restore(Slot&, const Client&, const uint8_t* img, uint64_t n,
//               SnapOut*)
// Each returns a CRUM_* code; SnapOut carries the device-reported status.
#pragma once
#include "crum.h"

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstdint>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

namespace crum {
namespace serve {

using Clock = std::chrono::steady_clock;

// First-fit allocator over one arena (4 KiB granules); the memory itself is
// the caller's.  Not thread-safe: the core calls it under its lock.
class Arena {
public:
    void init(uint8_t* base, uint64_t bytes)
    {
        base_ = base;
        size_ = bytes & ~4095ull;
        free_.clear();
        if (size_)
            free_[0] = size_;
        used_ = 0;
    }
    // offset of a block of at least n bytes, or UINT64_MAX
    uint64_t alloc(uint64_t n)
    {
        n = (n + 4095) & ~4095ull;
        if (n == 0)
            n = 4096;
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
    // give back a block returned by alloc(n) (same n), or its tail
    // [off + keep, off + n) as release(off + keep, n - keep) with keep a
    // multiple of 4 KiB
    void release(uint64_t off, uint64_t n)
    {
        n = (n + 4095) & ~4095ull;
        if (n == 0)
            n = 4096;
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
    size_t free_blocks() const { return free_.size(); }

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
    uint64_t worst = 0;  // image bytes with every page dirty
    std::deque<Request> queue;
    bool busy = false;
    uint64_t seq = 0;
    bool has_image = false;
    uint64_t img_off = 0, img_bytes = 0;
};

struct SnapOut {
    int32_t code = 0;
    uint64_t n_dirty = 0;
    uint64_t image_bytes = 0;
};

template <class B>
class Core {
public:
    using Slot = typename B::Slot;

    explicit Core(B backend) : be_(std::move(backend)) {}
    ~Core() { stop_workers(); }
    Core(const Core&) = delete;
    Core& operator=(const Core&) = delete;

    // clients: validated, every region with a shadow; worst[c]: client c's
    // image bytes with every page dirty.  The arena memory is the caller's.
    void init(std::vector<Client> clients, uint8_t* arena, uint64_t arena_bytes)
    {
        clients_ = std::move(clients);
        for (const Client& c : clients_)
            max_worst_ = std::max(max_worst_, c.worst);
        arena_.init(arena, arena_bytes);
        t0_ = Clock::now();
    }

    void start(uint32_t n_slots)
    {
        for (uint32_t i = 0; i < n_slots; ++i)
            workers_.emplace_back([this, i] { worker((int)i); });
    }

    // Finish queued requests, then join the workers.
    void stop_workers()
    {
        {
            std::lock_guard<std::mutex> lk(mu_);
            stop_ = true;
            cv_work_.notify_all();
            cv_budget_.notify_all();
        }
        for (auto& t : workers_)
            if (t.joinable())
                t.join();
        workers_.clear();
    }

    double now() const { return std::chrono::duration<double>(Clock::now() - t0_).count(); }

    int set_policy(int policy)
    {
        if (policy < CRUM_SERVE_ADAPTIVE || policy > CRUM_SERVE_PIPELINED)
            return CRUM_EINVAL;
        std::lock_guard<std::mutex> lk(mu_);
        policy_ = policy;
        return CRUM_OK;
    }

    void set_prepare(crum_server_prepare_fn fn, void* user)
    {
        std::lock_guard<std::mutex> lk(mu_);
        prepare_ = fn;
        prepare_user_ = user;
    }

    void set_reserve_wait(double seconds)
    {
        std::lock_guard<std::mutex> lk(mu_);
        reserve_wait_s_ = seconds;
    }

    int submit(uint32_t client, uint32_t kind, uint64_t tag, uint64_t* id)
    {
        if (client >= clients_.size() || (kind != CRUM_REQ_SNAPSHOT && kind != CRUM_REQ_RESTORE))
            return CRUM_EINVAL;
        std::lock_guard<std::mutex> lk(mu_);
        if (fatal_ || stop_)
            return CRUM_EHIP;
        Request r{next_id_++, client, kind, tag, now()};
        Client& cl = clients_[client];
        const bool was_idle = cl.queue.empty() && !cl.busy;
        cl.queue.push_back(r);
        queued_ += 1;
        if (was_idle)
            ready_.push_back(client);
        if (id)
            *id = r.id;
        cv_work_.notify_one();
        return CRUM_OK;
    }

    int poll(crum_server_completion* out, uint32_t max, uint32_t* n, int wait_all)
    {
        std::unique_lock<std::mutex> lk(mu_);
        if (wait_all)
            cv_done_.wait(lk, [&] { return fatal_ || (queued_ == 0 && in_flight_ == 0); });
        const uint32_t k = (uint32_t)std::min<size_t>(max, done_.size());
        for (uint32_t i = 0; i < k; ++i)
            out[i] = done_[i];
        done_.erase(done_.begin(), done_.begin() + k);
        *n = k;
        return fatal_ ? CRUM_EHIP : CRUM_OK;
    }

    uint64_t pinned_used()
    {
        std::lock_guard<std::mutex> lk(mu_);
        return arena_.used();
    }

    int latest_image(uint32_t client, const void** ptr, uint64_t* bytes)
    {
        if (client >= clients_.size())
            return CRUM_EINVAL;
        std::lock_guard<std::mutex> lk(mu_);
        const Client& cl = clients_[client];
        if (!cl.has_image)
            return CRUM_EINVAL;
        *ptr = arena_.ptr(cl.img_off);
        *bytes = cl.img_bytes;
        return CRUM_OK;
    }

    bool failed() const { return fatal_ != 0; }
    uint64_t max_worst() const { return max_worst_; }
    const std::vector<Client>& clients() const { return clients_; }
    B& backend() { return be_; }

    // Every live reservation (the latest image of each client): for checks.
    uint64_t reserved_by_images()
    {
        std::lock_guard<std::mutex> lk(mu_);
        uint64_t n = 0;
        for (const Client& c : clients_)
            if (c.has_image)
                n += (c.img_bytes + 4095) & ~4095ull;
        return n;
    }

private:
    // Reserve n pinned bytes, waiting while the arena is full (at most
    // reserve_wait_s_).  Called with the lock held; UINT64_MAX when the bytes
    // never become free.
    uint64_t reserve(std::unique_lock<std::mutex>& lk, uint64_t n)
    {
        if (((n + 4095) & ~4095ull) > arena_.size())
            return UINT64_MAX;
        const auto deadline = Clock::now() + std::chrono::duration_cast<Clock::duration>(
                                                 std::chrono::duration<double>(reserve_wait_s_));
        for (;;) {
            const uint64_t off = arena_.alloc(n);
            if (off != UINT64_MAX || stop_)
                return off;
            if (cv_budget_.wait_until(lk, deadline) == std::cv_status::timeout)
                return arena_.alloc(n);
        }
    }

    // Record a finished request, free its client for its next request.
    void finish(const Request& rq, crum_server_completion& out)
    {
        out.done_s = now();
        std::lock_guard<std::mutex> lk(mu_);
        done_.push_back(out);
        in_flight_ -= 1;
        Client& cl = clients_[rq.client];
        cl.busy = false;
        if (!cl.queue.empty())
            ready_.push_back(rq.client);
        cv_work_.notify_all();
        cv_done_.notify_all();
    }

    void run_snapshot(Slot& slot, Client& cl, crum_server_completion& out)
    {
        // Fast path: when the arena can hold the client's worst-case image
        // right now, reserve it, let the snapshot drain into it while it runs
        // (pipelined order), then trim the reservation to the image.
        const uint64_t worst_r = (cl.worst + 4095) & ~4095ull;
        uint64_t off = UINT64_MAX;
        {
            std::lock_guard<std::mutex> lk(mu_);
            const bool fast = policy_ == CRUM_SERVE_PIPELINED ||
                              (policy_ == CRUM_SERVE_ADAPTIVE && queued_ == 0);
            if (fast)
                off = arena_.alloc(cl.worst);
        }
        SnapOut so;
        const uint64_t seq = ++cl.seq;
        if (off != UINT64_MAX) {
            uint8_t* dst = arena_.ptr(off);
            int code = be_.snapshot(slot, cl, seq, dst, worst_r, &so);
            if (code == CRUM_OK)
                code = so.code;
            std::lock_guard<std::mutex> lk(mu_);
            if (code == CRUM_OK) {
                out.n_dirty = so.n_dirty;
                out.image_bytes = so.image_bytes;
                std::memcpy(&out.meta_crc, dst + 56, 4);
                std::memcpy(&out.crcs_crc, dst + 60, 4);
                const uint64_t keep = (so.image_bytes + 4095) & ~4095ull;
                if (keep < worst_r)
                    arena_.release(off + keep, worst_r - keep);
                if (cl.has_image)
                    arena_.release(cl.img_off, cl.img_bytes);
                cl.has_image = true;
                cl.img_off = off;
                cl.img_bytes = so.image_bytes;
            } else {
                arena_.release(off, worst_r);
            }
            out.code = code;
            cv_budget_.notify_all();
            return;
        }
        // stage 1: build the image on the device, learn its exact size
        int code = be_.snapshot(slot, cl, seq, nullptr, 0, &so);
        if (code == CRUM_OK)
            code = so.code;
        if (code != CRUM_OK) {
            out.code = code;
            return;
        }
        out.n_dirty = so.n_dirty;
        out.image_bytes = so.image_bytes;
        // stage 2: the shadow now holds this snapshot, so the previous delta
        // image is obsolete; reserve exactly the new image's bytes and drain
        // into them
        uint64_t off2;
        {
            std::unique_lock<std::mutex> lk(mu_);
            if (cl.has_image) {
                arena_.release(cl.img_off, cl.img_bytes);
                cl.has_image = false;
                cv_budget_.notify_all();
            }
            off2 = reserve(lk, so.image_bytes);
        }
        if (off2 == UINT64_MAX) {
            out.code = CRUM_ENOSPC;
            return;
        }
        uint8_t* dst = arena_.ptr(off2);
        code = be_.drain(slot, dst, so.image_bytes);
        std::lock_guard<std::mutex> lk(mu_);
        if (code != CRUM_OK) {
            arena_.release(off2, so.image_bytes);
        } else {
            std::memcpy(&out.meta_crc, dst + 56, 4);
            std::memcpy(&out.crcs_crc, dst + 60, 4);
            cl.has_image = true;
            cl.img_off = off2;
            cl.img_bytes = so.image_bytes;
        }
        out.code = code;
        cv_budget_.notify_all();
    }

    void run_restore(Slot& slot, Client& cl, crum_server_completion& out)
    {
        // the client's image is changed only by its own requests, which run
        // one at a time: reading it here needs no lock
        if (!cl.has_image) {
            out.code = CRUM_EINVAL;
            return;
        }
        const uint8_t* img = arena_.ptr(cl.img_off);
        SnapOut so;
        int code = be_.restore(slot, cl, img, cl.img_bytes, &so);
        if (code == CRUM_OK)
            code = so.code;
        out.code = code;
        out.n_dirty = so.n_dirty;
        out.image_bytes = cl.img_bytes;
        std::memcpy(&out.meta_crc, img + 56, 4);
        std::memcpy(&out.crcs_crc, img + 60, 4);
    }

    void worker(int index)
    {
        Slot slot{};
        if (!be_.open(slot, std::max<uint64_t>(max_worst_, 4096))) {
            be_.close(slot);
            // the server reports CRUM_EHIP from now on; queued requests stay
            // queued and waiters are woken
            std::lock_guard<std::mutex> lk(mu_);
            fatal_ = 1;
            cv_done_.notify_all();
            return;
        }
        (void)index;
        for (;;) {
            Request rq;
            crum_server_prepare_fn prep;
            void* prep_user;
            {
                std::unique_lock<std::mutex> lk(mu_);
                cv_work_.wait(lk, [&] { return stop_ || !ready_.empty(); });
                if (ready_.empty())
                    break;  // stop_ with nothing left to run
                const uint32_t c = ready_.front();
                ready_.pop_front();
                Client& cl = clients_[c];
                rq = cl.queue.front();
                cl.queue.pop_front();
                cl.busy = true;
                queued_ -= 1;
                in_flight_ += 1;
                prep = prepare_;
                prep_user = prepare_user_;
            }
            Client& cl = clients_[rq.client];
            crum_server_completion out{};
            out.id = rq.id;
            out.tag = rq.tag;
            out.client = rq.client;
            out.kind = rq.kind;
            out.arrival_s = rq.arrival;
            out.start_s = now();
            if (prep)
                prep(prep_user, rq.client, rq.kind, rq.tag, be_.stream(slot));
            if (rq.kind == CRUM_REQ_SNAPSHOT)
                run_snapshot(slot, cl, out);
            else
                run_restore(slot, cl, out);
            finish(rq, out);
        }
        be_.close(slot);
    }

    B be_;
    std::vector<Client> clients_;
    Arena arena_;
    std::mutex mu_;
    std::condition_variable cv_work_, cv_budget_, cv_done_;
    std::deque<uint32_t> ready_;  // clients with a queued head request, in arrival order
    std::vector<crum_server_completion> done_;
    uint64_t next_id_ = 0, in_flight_ = 0, queued_ = 0;
    bool stop_ = false;
    std::vector<std::thread> workers_;
    crum_server_prepare_fn prepare_ = nullptr;
    void* prepare_user_ = nullptr;
    Clock::time_point t0_;
    std::atomic<int> fatal_{0};
    uint64_t max_worst_ = 0;
    int policy_ = CRUM_SERVE_ADAPTIVE;
    double reserve_wait_s_ = 30.0;
};

}  // namespace serve
}  // namespace crum
