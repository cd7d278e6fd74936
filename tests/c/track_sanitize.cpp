// The host write tracker (crum_track.hip, host code only) built with gcc as
// C++ under AddressSanitizer + UndefinedBehaviorSanitizer (with the
// sanitizer's own SIGSEGV handling off, since the tracker owns that signal):
// writer threads store into random pages of two
// views while the main thread flushes them again and again; after the writers
// stop and a last flush, each real region equals its view, every page
// written since the first flush is in the pending set, and a new tracker's
// pages are all dirty.  A flush may copy a page while its writer stores into
// it (the copy is then torn, and the page is dirty again for the next
// flush).  Exit status 0 on success.  Usage: track_sanitize ROUNDS
#include "crum.h"

#include <atomic>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <random>
#include <thread>
#include <vector>

#define CHECK(c)                                                             \
    do {                                                                     \
        if (!(c)) {                                                          \
            std::fprintf(stderr, "%s:%d: check failed: %s\n", __FILE__, __LINE__, #c); \
            std::exit(1);                                                    \
        }                                                                    \
    } while (0)

int main(int argc, char** argv)
{
    const int rounds = argc > 1 ? std::atoi(argv[1]) : 20;
    const uint32_t P[2] = {4096, 65536};
    const uint64_t pages[2] = {300, 40};
    crum_track* t[2];
    std::vector<std::vector<uint8_t>> real(2);
    for (int k = 0; k < 2; ++k) {
        CHECK(crum_track_create(pages[k] * P[k], P[k], &t[k]) == CRUM_OK);
        crum_track_info info;
        CHECK(crum_track_stats(t[k], &info) == CRUM_OK);
        CHECK(info.pages == pages[k] && info.dirty_pages == pages[k] && info.faults == 0);
        real[k].assign(pages[k] * P[k], 0);
        uint64_t n = 0;
        CHECK(crum_track_flush(t[k], real[k].data(), 3, &n) == CRUM_OK && n == pages[k]);
        std::vector<uint64_t> w((pages[k] + 63) / 64);
        CHECK(crum_track_pending(t[k], w.data(), w.size(), 1) == CRUM_OK);
    }
    // which pages each writer touched (written only by that writer)
    std::vector<std::vector<uint8_t>> touched(4, std::vector<uint8_t>(pages[0] + pages[1], 0));
    std::atomic<bool> stop{false};
    std::vector<std::thread> writers;
    for (int id = 0; id < 4; ++id) {
        writers.emplace_back([&, id]() {
            std::mt19937_64 rng(1234 + id);
            while (!stop.load(std::memory_order_relaxed)) {
                const int k = (int)(rng() & 1);
                // each writer owns the pages p with p % 4 == id
                const uint64_t p = (rng() % (pages[k] / 4)) * 4 + (uint64_t)id;
                const uint64_t o = rng() % (P[k] - 32);
                uint8_t* v = static_cast<uint8_t*>(crum_track_view(t[k]));
                uint8_t buf[32];
                for (auto& b : buf)
                    b = (uint8_t)rng();
                std::memcpy(v + p * P[k] + o, buf, sizeof buf);
                touched[id][k ? pages[0] + p : p] = 1;
            }
        });
    }
    for (int r = 0; r < rounds; ++r)
        for (int k = 0; k < 2; ++k)
            CHECK(crum_track_flush(t[k], real[k].data(), 2, nullptr) == CRUM_OK);
    stop.store(true);
    for (auto& w : writers)
        w.join();
    for (int k = 0; k < 2; ++k) {
        CHECK(crum_track_flush(t[k], real[k].data(), 2, nullptr) == CRUM_OK);
        const uint8_t* v = static_cast<const uint8_t*>(crum_track_view(t[k]));
        CHECK(std::memcmp(real[k].data(), v, real[k].size()) == 0);
        std::vector<uint64_t> w((pages[k] + 63) / 64);
        CHECK(crum_track_pending(t[k], w.data(), w.size(), 0) == CRUM_OK);
        for (uint64_t p = 0; p < pages[k]; ++p) {
            bool any = false;
            for (int id = 0; id < 4; ++id)
                any |= touched[id][k ? pages[0] + p : p] != 0;
            if (any)
                CHECK((w[p / 64] >> (p % 64)) & 1u);
        }
        crum_track_info info;
        CHECK(crum_track_stats(t[k], &info) == CRUM_OK && info.dirty_pages == 0);
        crum_track_destroy(t[k]);
    }
    std::printf("track sanitize: ok\n");
    return 0;
}
