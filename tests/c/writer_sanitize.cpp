// The image writer (crum_writer.hip, host code only) built with gcc as C++
// under ThreadSanitizer and, separately, AddressSanitizer +
// UndefinedBehaviorSanitizer: several threads submit writes of random sizes
// (chunked over the writer's pool, with and without O_DIRECT and fdatasync,
// overwriting earlier files), poll them, and every file must equal its
// buffer; a write into a missing directory must fail cleanly.  Exit status 0
// on success.  Usage: writer_sanitize DIR
#include "crum.h"

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <random>
#include <string>
#include <thread>
#include <vector>

#define CHECK(c)                                                             \
    do {                                                                     \
        if (!(c)) {                                                          \
            std::fprintf(stderr, "%s:%d: check failed: %s\n", __FILE__, __LINE__, #c); \
            std::exit(1);                                                    \
        }                                                                    \
    } while (0)

static std::vector<uint8_t> read_file(const std::string& path)
{
    std::vector<uint8_t> v;
    FILE* f = std::fopen(path.c_str(), "rb");
    if (!f)
        return v;
    uint8_t buf[65536];
    size_t n;
    while ((n = std::fread(buf, 1, sizeof buf, f)) > 0)
        v.insert(v.end(), buf, buf + n);
    std::fclose(f);
    return v;
}

int main(int argc, char** argv)
{
    CHECK(argc > 1);
    const std::string dir = argv[1];
    for (uint32_t flags : {0u, (uint32_t)CRUM_WRITE_SYNC, (uint32_t)CRUM_WRITE_DIRECT,
                           (uint32_t)(CRUM_WRITE_DIRECT | CRUM_WRITE_SYNC)}) {
        crum_writer* w = nullptr;
        CHECK(crum_writer_create(4, 64 << 10, flags, &w) == CRUM_OK);
        const int submitters = 3, per = 6;
        std::vector<std::vector<uint8_t>> bufs(submitters * per);
        std::vector<std::thread> th;
        for (int t = 0; t < submitters; ++t) {
            th.emplace_back([&, t] {
                std::mt19937 rng(100 * flags + t);
                for (int i = 0; i < per; ++i) {
                    const int k = t * per + i;
                    const size_t n = (rng() % 3 == 0) ? (rng() % 5000)
                                                      : 4096 * (1 + rng() % 80) + (rng() % 2) * 17;
                    std::vector<uint8_t>& b = bufs[k];
                    b.resize(n);
                    for (auto& x : b)
                        x = (uint8_t)rng();
                    // files overwrite each other's names on purpose (by k % 5)
                    const std::string path = dir + "/f" + std::to_string(t) + "_" +
                                             std::to_string(i % 2) + ".bin";
                    uint64_t ticket = 0;
                    CHECK(crum_writer_submit(w, path.c_str(), b.data(), n, &ticket) == CRUM_OK);
                    crum_write_status st{};
                    CHECK(crum_writer_poll(w, ticket, 1, &st) == CRUM_OK);
                    CHECK(st.code == CRUM_OK && st.bytes == n);
                    CHECK(read_file(path) == b);
                    CHECK(crum_writer_poll(w, ticket, 1, &st) == CRUM_EINVAL);
                }
            });
        }
        for (auto& x : th)
            x.join();
        uint64_t ticket = 0;
        uint8_t one = 1;
        CHECK(crum_writer_submit(w, (dir + "/missing/x.bin").c_str(), &one, 1, &ticket) ==
              CRUM_EIO);
        crum_writer_destroy(w);
    }
    std::printf("writer sanitize: ok\n");
    return 0;
}
