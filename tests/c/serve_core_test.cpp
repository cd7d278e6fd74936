// CPU test of the serving loop's scheduling core (crum_serve_core.h) with a
// stub backend whose "device memory" is host memory, built with gcc under
// AddressSanitizer + UndefinedBehaviorSanitizer and, separately,
// ThreadSanitizer.  It drives many clients through several worker slots
// with random request mixes, policies and arena budgets, plus the failure
// paths (a slot that cannot open, an exhausted budget, destroy with queued
// work), and checks:
//   * every request completes, in submit order per client;
//   * after each client's last request its shadow equals its current bytes
//     (snapshots update the shadow, restores write both);
//   * the arena's reservations are what the clients' latest images need, and
//     no two live images overlap (each latest image still verifies at the end);
//   * a failed slot makes submit and poll report CRUM_EHIP without a hang.
// Exit status 0 on success; the first failed check is printed.
#include "crum_serve_core.h"

#include <atomic>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <random>
#include <thread>
#include <vector>

using crum::serve::Client;
using crum::serve::Core;
using crum::serve::SnapOut;

#define CHECK(cond)                                                                  \
    do {                                                                             \
        if (!(cond)) {                                                               \
            std::fprintf(stderr, "%s:%d: check failed: %s\n", __FILE__, __LINE__, #cond); \
            std::exit(1);                                                            \
        }                                                                            \
    } while (0)

namespace {

// Stub image: 64-byte header ("STUBIMG1", u64 D, u64 seq, u64 page size,
// u64 G, ..., u32 meta at 56 = checksum of the rest, u32 at 60 = D), then D
// records of {u64 page index, page bytes}.
uint32_t fnv(const uint8_t* p, uint64_t n, uint32_t h = 2166136261u)
{
    for (uint64_t i = 0; i < n; ++i)
        h = (h ^ p[i]) * 16777619u;
    return h;
}

uint64_t image_bytes(uint64_t D, uint64_t P) { return 64 + D * (8 + P); }

struct StubBackend {
    std::shared_ptr<std::atomic<int>> opens = std::make_shared<std::atomic<int>>(0);
    int fail_open_at = -1;
    int max_sleep_us = 200;
    struct Slot {
        std::vector<uint8_t> staging;
        std::mt19937 rng;
        bool opened = false;
    };
    bool open(Slot& s, uint64_t staging_bytes)
    {
        const int k = opens->fetch_add(1);
        if (k == fail_open_at)
            return false;
        s.staging.assign(staging_bytes, 0);
        s.rng.seed((unsigned)k * 7919u + 1);
        s.opened = true;
        return true;
    }
    void close(Slot& s)
    {
        s.staging.clear();
        s.staging.shrink_to_fit();
        s.opened = false;
    }
    void* stream(Slot&) { return nullptr; }
    void nap(Slot& s)
    {
        if (max_sleep_us > 0)
            std::this_thread::sleep_for(std::chrono::microseconds(s.rng() % max_sleep_us));
    }
    int snapshot(Slot& s, const Client& cl, uint64_t seq, uint8_t* dst, uint64_t dst_cap,
                 SnapOut* o)
    {
        CHECK(s.opened);
        const uint64_t P = cl.page_size;
        std::vector<uint64_t> dirty;
        uint64_t G = 0;
        for (const crum_region& r : cl.regions) {
            const uint8_t* a = static_cast<const uint8_t*>(r.base);
            const uint8_t* b = static_cast<const uint8_t*>(r.shadow);
            for (uint64_t p = 0; p < r.len / P; ++p, ++G)
                if (std::memcmp(a + p * P, b + p * P, P) != 0)
                    dirty.push_back(G);
        }
        const uint64_t n = image_bytes(dirty.size(), P);
        nap(s);
        o->n_dirty = dirty.size();
        o->image_bytes = n;
        if (n > s.staging.size() || (dst && n > dst_cap) || n > cl.worst) {
            o->code = CRUM_ENOSPC;
            return CRUM_OK;
        }
        uint8_t* img = dst ? dst : s.staging.data();
        std::memset(img, 0, 64);
        std::memcpy(img, "STUBIMG1", 8);
        const uint64_t D = dirty.size();
        std::memcpy(img + 8, &D, 8);
        std::memcpy(img + 16, &seq, 8);
        std::memcpy(img + 24, &P, 8);
        std::memcpy(img + 32, &G, 8);
        uint8_t* rec = img + 64;
        uint64_t g0 = 0;
        size_t k = 0;
        for (const crum_region& r : cl.regions) {
            const uint64_t np = r.len / P;
            for (; k < dirty.size() && dirty[k] < g0 + np; ++k) {
                const uint64_t p = dirty[k] - g0;
                std::memcpy(rec, &dirty[k], 8);
                std::memcpy(rec + 8, static_cast<const uint8_t*>(r.base) + p * P, P);
                // shadow update: the snapshot is the new baseline
                std::memcpy(static_cast<uint8_t*>(r.shadow) + p * P,
                            static_cast<const uint8_t*>(r.base) + p * P, P);
                rec += 8 + P;
            }
            g0 += np;
        }
        const uint32_t meta = fnv(img + 64, n - 64, fnv(img, 56));
        const uint32_t d32 = (uint32_t)D;
        std::memcpy(img + 56, &meta, 4);
        std::memcpy(img + 60, &d32, 4);
        o->code = CRUM_OK;
        return CRUM_OK;
    }
    int drain(Slot& s, uint8_t* dst, uint64_t n)
    {
        CHECK(n <= s.staging.size());
        nap(s);
        std::memcpy(dst, s.staging.data(), n);
        return CRUM_OK;
    }
    int restore(Slot& s, const Client& cl, const uint8_t* img, uint64_t n, SnapOut* o)
    {
        CHECK(s.opened && n >= 64 && std::memcmp(img, "STUBIMG1", 8) == 0);
        uint32_t meta;
        std::memcpy(&meta, img + 56, 4);
        CHECK(meta == fnv(img + 64, n - 64, fnv(img, 56)));
        uint64_t D, P;
        std::memcpy(&D, img + 8, 8);
        std::memcpy(&P, img + 24, 8);
        CHECK(P == cl.page_size && n == image_bytes(D, P));
        nap(s);
        const uint8_t* rec = img + 64;
        for (uint64_t k = 0; k < D; ++k, rec += 8 + P) {
            uint64_t g;
            std::memcpy(&g, rec, 8);
            uint64_t g0 = 0;
            for (const crum_region& r : cl.regions) {
                const uint64_t np = r.len / P;
                if (g < g0 + np) {
                    std::memcpy(static_cast<uint8_t*>(r.base) + (g - g0) * P, rec + 8, P);
                    std::memcpy(static_cast<uint8_t*>(r.shadow) + (g - g0) * P, rec + 8, P);
                    break;
                }
                g0 += np;
            }
        }
        o->code = CRUM_OK;
        o->n_dirty = D;
        o->image_bytes = n;
        return CRUM_OK;
    }
};

struct Harness {
    uint32_t n_clients, P;
    std::vector<std::vector<uint8_t>> cur, sh;
    std::vector<Client> clients;
    std::vector<uint8_t> arena;
    std::vector<std::vector<uint64_t>> last_dirty;  // pages changed before each client's snapshot
    std::atomic<uint64_t> prepares{0};

    Harness(uint32_t n, uint32_t page, uint32_t seed, uint64_t arena_bytes)
        : n_clients(n), P(page), cur(n), sh(n), clients(n), arena(arena_bytes), last_dirty(n)
    {
        std::mt19937 rng(seed);
        for (uint32_t c = 0; c < n; ++c) {
            const uint32_t pages = 1 + rng() % 24;
            cur[c].resize((uint64_t)pages * P);
            for (auto& b : cur[c])
                b = (uint8_t)rng();
            sh[c] = cur[c];
            // one or two regions per client
            const uint32_t cut = pages > 1 ? 1 + rng() % (pages - 1) : pages;
            Client& cl = clients[c];
            cl.page_size = P;
            cl.regions.push_back({cur[c].data(), sh[c].data(), (uint64_t)cut * P, 1000 + 2ull * c});
            if (cut < pages)
                cl.regions.push_back({cur[c].data() + (uint64_t)cut * P,
                                      sh[c].data() + (uint64_t)cut * P,
                                      (uint64_t)(pages - cut) * P, 1001 + 2ull * c});
            cl.worst = image_bytes(pages, P);
        }
    }

    // prepare hook: before a snapshot, change a few random pages of the
    // client (on the worker's thread; the client runs one request at a time)
    static void prepare(void* user, uint32_t client, uint32_t kind, uint64_t tag, void*)
    {
        Harness* h = static_cast<Harness*>(user);
        h->prepares.fetch_add(1);
        if (kind != CRUM_REQ_SNAPSHOT)
            return;
        std::mt19937 rng((uint32_t)(tag * 2654435761u + client));
        auto& v = h->cur[client];
        const uint64_t pages = v.size() / h->P;
        const uint32_t n = rng() % 4;
        h->last_dirty[client].clear();
        for (uint32_t i = 0; i < n; ++i) {
            const uint64_t p = rng() % pages;
            v[p * h->P + rng() % h->P] ^= (uint8_t)(1 + rng() % 255);
            h->last_dirty[client].push_back(p);
        }
    }
};

void run_mix(uint32_t n_clients, uint32_t slots, int policy, uint64_t arena_bytes, uint32_t seed,
             int n_requests)
{
    Harness h(n_clients, 4096, seed, arena_bytes);
    StubBackend be;
    Core<StubBackend> core(be);
    core.init(h.clients, h.arena.data(), h.arena.size());
    core.set_prepare(&Harness::prepare, &h);
    CHECK(core.set_policy(policy) == CRUM_OK);
    core.set_reserve_wait(5.0);
    core.start(slots);
    // a base image for every client first, then a random mix (4:1)
    std::vector<std::vector<uint64_t>> ids(n_clients);
    uint64_t id;
    for (uint32_t c = 0; c < n_clients; ++c) {
        CHECK(core.submit(c, CRUM_REQ_SNAPSHOT, 1u << 30, &id) == CRUM_OK);
        ids[c].push_back(id);
    }
    std::mt19937 rng(seed + 1);
    for (int i = 0; i < n_requests; ++i) {
        const uint32_t c = rng() % n_clients;
        const uint32_t kind = rng() % 5 ? CRUM_REQ_SNAPSHOT : CRUM_REQ_RESTORE;
        CHECK(core.submit(c, kind, (uint64_t)i, &id) == CRUM_OK);
        ids[c].push_back(id);
        if (i % 17 == 0)
            std::this_thread::sleep_for(std::chrono::microseconds(rng() % 300));
    }
    std::vector<crum_server_completion> out(64);
    std::vector<std::vector<uint64_t>> got(n_clients);
    uint64_t total = 0;
    for (;;) {
        uint32_t n = 0;
        CHECK(core.poll(out.data(), (uint32_t)out.size(), &n, 0) == CRUM_OK);
        for (uint32_t i = 0; i < n; ++i) {
            const auto& d = out[i];
            CHECK(d.code == CRUM_OK);
            CHECK(d.done_s >= d.start_s && d.start_s >= d.arrival_s);
            got[d.client].push_back(d.id);
            total += 1;
        }
        if (total == (uint64_t)(n_requests + n_clients))
            break;
        if (n == 0) {
            CHECK(core.poll(out.data(), 0, &n, 1) == CRUM_OK);  // wait for the rest
        }
    }
    for (uint32_t c = 0; c < n_clients; ++c)
        CHECK(got[c] == ids[c]);  // first in, first out per client
    CHECK(core.pinned_used() == core.reserved_by_images());
    // every latest image verifies, and restoring it onto a copy of the state
    // that preceded it is what the client holds now; here: the shadow equals
    // the current bytes after the last request (a snapshot or a restore)
    for (uint32_t c = 0; c < n_clients; ++c) {
        const void* p;
        uint64_t nb;
        CHECK(core.latest_image(c, &p, &nb) == CRUM_OK);
        const uint8_t* img = static_cast<const uint8_t*>(p);
        uint32_t meta;
        std::memcpy(&meta, img + 56, 4);
        CHECK(std::memcmp(img, "STUBIMG1", 8) == 0 && meta == fnv(img + 64, nb - 64, fnv(img, 56)));
        CHECK(h.cur[c] == h.sh[c]);
    }
    core.stop_workers();
    CHECK(h.prepares.load() == (uint64_t)(n_requests + n_clients));
}

void run_budget_exhausted()
{
    // the arena cannot hold one image: two-stage admission waits, then ENOSPC
    Harness h(2, 4096, 5, 2 * 4096);
    StubBackend be;
    be.max_sleep_us = 0;
    Core<StubBackend> core(be);
    core.init(h.clients, h.arena.data(), h.arena.size());
    core.set_reserve_wait(0.05);
    CHECK(core.set_policy(CRUM_SERVE_TWO_STAGE) == CRUM_OK);
    core.start(2);
    uint64_t id;
    // client 0's first snapshot has every page dirty (the shadow is the
    // initial copy, so D = 0): force changes through the prepare hook
    core.set_prepare(&Harness::prepare, &h);
    CHECK(core.submit(0, CRUM_REQ_SNAPSHOT, 3, &id) == CRUM_OK);
    CHECK(core.submit(1, CRUM_REQ_SNAPSHOT, 4, &id) == CRUM_OK);
    std::vector<crum_server_completion> out(8);
    uint32_t n = 0;
    CHECK(core.poll(out.data(), 8, &n, 1) == CRUM_OK);
    CHECK(n == 2);
    for (uint32_t i = 0; i < n; ++i) {
        const uint64_t need = image_bytes(out[i].n_dirty, 4096);
        if (need > 2 * 4096)
            CHECK(out[i].code == CRUM_ENOSPC);  // larger than the whole arena
        else
            CHECK(out[i].code == CRUM_OK || out[i].code == CRUM_ENOSPC);  // may wait out
    }
    CHECK(core.pinned_used() == core.reserved_by_images());
    // a client without an image: its restore is an argument error
    for (uint32_t i = 0; i < n; ++i) {
        if (out[i].code != CRUM_ENOSPC)
            continue;
        CHECK(core.submit(out[i].client, CRUM_REQ_RESTORE, 9, &id) == CRUM_OK);
        CHECK(core.poll(out.data(), 8, &n, 1) == CRUM_OK && n == 1);
        CHECK(out[0].code == CRUM_EINVAL);
        break;
    }
    core.stop_workers();
}

void run_failed_slot()
{
    Harness h(4, 4096, 9, 1 << 20);
    StubBackend be;
    be.fail_open_at = 1;
    Core<StubBackend> core(be);
    core.init(h.clients, h.arena.data(), h.arena.size());
    core.start(3);
    // wait for the failed open to be seen
    for (int i = 0; i < 2000 && !core.failed(); ++i)
        std::this_thread::sleep_for(std::chrono::milliseconds(1));
    CHECK(core.failed());
    uint64_t id;
    CHECK(core.submit(0, CRUM_REQ_SNAPSHOT, 1, &id) == CRUM_EHIP);
    uint32_t n = 0;
    crum_server_completion out[4];
    CHECK(core.poll(out, 4, &n, 1) == CRUM_EHIP);  // returns at once
    core.stop_workers();
}

void run_destroy_with_queue()
{
    Harness h(8, 4096, 13, 8 << 20);
    StubBackend be;
    Core<StubBackend>* core = new Core<StubBackend>(be);
    core->init(h.clients, h.arena.data(), h.arena.size());
    core->set_prepare(&Harness::prepare, &h);
    core->start(4);
    uint64_t id;
    for (int i = 0; i < 200; ++i)
        CHECK(core->submit(i % 8, i % 7 ? CRUM_REQ_SNAPSHOT : CRUM_REQ_RESTORE, i, &id) == CRUM_OK);
    delete core;  // finishes the queue, joins the workers
    CHECK(h.prepares.load() == 200);
}

}  // namespace

int main(int argc, char** argv)
{
    const int rounds = argc > 1 ? std::atoi(argv[1]) : 3;
    for (int r = 0; r < rounds; ++r) {
        run_mix(32, 6, CRUM_SERVE_ADAPTIVE, 2 << 20, 100 + r, 400);
        run_mix(32, 6, CRUM_SERVE_TWO_STAGE, 1 << 20, 200 + r, 300);
        run_mix(16, 3, CRUM_SERVE_PIPELINED, 8 << 20, 300 + r, 300);
        run_mix(5, 1, CRUM_SERVE_ADAPTIVE, 1 << 20, 400 + r, 100);
    }
    run_budget_exhausted();
    run_failed_slot();
    run_destroy_with_queue();
    std::printf("serve core: ok\n");
    return 0;
}
