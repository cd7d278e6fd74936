// Host write tracking for host-written managed memory (paper section 3.2,
// Algorithm 1, and section 3.2.1).
//
// The application writes a host-side view of a region: ordinary anonymous
// memory that the GPU never maps.  A clean page of the view is read-only, so
// the first write to it faults; the fault handler makes the page writable
// and marks it dirty, and the write goes through.  A flush (the paper does one
// at every call into the GPU runtime) copies each dirty page into the real
// region (the managed allocation the GPU reads), makes the page read-only
// again and clears its dirty bit; the flushed page is also recorded as
// written since the last snapshot.  A new view starts with every page dirty,
// as a new region is all-dirty in Algorithm 1.
//
// The pages recorded since the last snapshot are the candidate set of
// crum_snapshot_tracked: a host-written page outside it has not been written
// since the shadow was last updated, so the snapshot need not read it.
//
// Protection changes only ever touch the view, never memory the GPU maps.
// Host code only: no HIP call is made.
#include "crum.h"

#include <signal.h>
#include <sys/mman.h>
#include <unistd.h>

#include <algorithm>
#include <atomic>
#include <cerrno>
#include <cstring>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

struct crum_track {
    uint8_t* view = nullptr;
    uint64_t bytes = 0;
    uint64_t page_size = 0;
    uint64_t n_pages = 0;
    uint64_t n_words = 0;
    std::atomic<uint64_t>* dirty = nullptr;    // written since the last flush
    std::atomic<uint64_t>* pending = nullptr;  // flushed since the last take
    std::atomic<uint64_t> faults{0};
    std::atomic<uint64_t> flushed_pages{0};
    std::mutex flush_mu;  // one flush or take at a time
    int slot = -1;
};

namespace {

constexpr int kMaxTrackers = 64;
std::atomic<crum_track*> g_slots[kMaxTrackers];
std::mutex g_reg_mu;
struct sigaction g_prev;
bool g_installed = false;

static_assert(std::atomic<uint64_t>::is_always_lock_free, "signal-safe bit updates");
static_assert(std::atomic<crum_track*>::is_always_lock_free, "signal-safe registry");

// Runs the handler that was installed before ours (or the default action).
void chain(int sig, siginfo_t* si, void* uc)
{
    if (g_prev.sa_flags & SA_SIGINFO) {
        if (g_prev.sa_sigaction) {
            g_prev.sa_sigaction(sig, si, uc);
            return;
        }
    } else if (g_prev.sa_handler != SIG_DFL && g_prev.sa_handler != SIG_IGN) {
        g_prev.sa_handler(sig);
        return;
    }
    // default action: returning re-executes the access, which now takes it
    struct sigaction dfl;
    std::memset(&dfl, 0, sizeof(dfl));
    dfl.sa_handler = SIG_DFL;
    sigemptyset(&dfl.sa_mask);
    sigaction(sig, &dfl, nullptr);
}

// A write to a read-only (clean) page of a view: make it writable, then mark
// it dirty; the faulting write is retried on return.  In this order a flush
// running at the same time either takes the new dirty bit (and protects and
// copies the page again later) or leaves it for the next flush; marking
// first could let a flush take the bit and protect the page just before it
// is made writable, so that the write would go unrecorded.  Only lock-free
// atomics and mprotect are used (async-signal-safe).
void on_fault(int sig, siginfo_t* si, void* uc)
{
    const uintptr_t a = reinterpret_cast<uintptr_t>(si->si_addr);
    for (int i = 0; i < kMaxTrackers; ++i) {
        crum_track* t = g_slots[i].load(std::memory_order_acquire);
        if (!t)
            continue;
        const uintptr_t b = reinterpret_cast<uintptr_t>(t->view);
        if (a < b || a >= b + t->bytes)
            continue;
        const uint64_t p = (a - b) / t->page_size;
        if (mprotect(t->view + p * t->page_size, t->page_size, PROT_READ | PROT_WRITE) != 0)
            break;
        t->dirty[p >> 6].fetch_or(1ull << (p & 63), std::memory_order_acq_rel);
        t->faults.fetch_add(1, std::memory_order_relaxed);
        return;
    }
    chain(sig, si, uc);
}

int install_handler()
{
    if (g_installed)
        return CRUM_OK;
    struct sigaction sa;
    std::memset(&sa, 0, sizeof(sa));
    sa.sa_sigaction = on_fault;
    sa.sa_flags = SA_SIGINFO | SA_NODEFER;
    sigemptyset(&sa.sa_mask);
    if (sigaction(SIGSEGV, &sa, &g_prev) != 0)
        return CRUM_EINVAL;
    g_installed = true;
    return CRUM_OK;
}

// Runs of set bits of `bits` (words [w0, w1) of a page bitmap) as
// [first, end) page ranges.
template <typename F>
void for_runs(const std::vector<uint64_t>& bits, uint64_t n_pages, F f)
{
    uint64_t p = 0;
    while (p < n_pages) {
        const uint64_t w = bits[p >> 6] >> (p & 63);
        if (!w) {
            p = (p | 63) + 1;
            continue;
        }
        p += (uint64_t)__builtin_ctzll(w);
        if (p >= n_pages)
            break;
        uint64_t e = p + 1;
        while (e < n_pages && ((bits[e >> 6] >> (e & 63)) & 1ull))
            ++e;
        f(p, e);
        p = e;
    }
}

}  // namespace

extern "C" {

int crum_track_create(uint64_t bytes, uint32_t page_size, crum_track** out)
{
    if (!out)
        return CRUM_EINVAL;
    *out = nullptr;
    const long os_page = sysconf(_SC_PAGESIZE);
    if (page_size < 4096 || (page_size & (page_size - 1)) || page_size > (1u << 30) ||
        (os_page > 0 && page_size % (uint64_t)os_page) || bytes == 0 || bytes % page_size)
        return CRUM_EINVAL;
    crum_track* t = new (std::nothrow) crum_track();
    if (!t)
        return CRUM_EINVAL;
    t->bytes = bytes;
    t->page_size = page_size;
    t->n_pages = bytes / page_size;
    t->n_words = (t->n_pages + 63) / 64;
    void* v = mmap(nullptr, bytes, PROT_READ | PROT_WRITE, MAP_PRIVATE | MAP_ANONYMOUS | MAP_NORESERVE,
                   -1, 0);
    t->dirty = new (std::nothrow) std::atomic<uint64_t>[t->n_words];
    t->pending = new (std::nothrow) std::atomic<uint64_t>[t->n_words];
    if (v == MAP_FAILED || !t->dirty || !t->pending) {
        if (v != MAP_FAILED)
            munmap(v, bytes);
        delete[] t->dirty;
        delete[] t->pending;
        delete t;
        return CRUM_EINVAL;
    }
    t->view = static_cast<uint8_t*>(v);
    // a new region: every page dirty (and writable), nothing flushed yet
    for (uint64_t w = 0; w < t->n_words; ++w) {
        const uint64_t valid = (w + 1) * 64 <= t->n_pages ? ~0ull
                                                          : (1ull << (t->n_pages - w * 64)) - 1;
        t->dirty[w].store(valid, std::memory_order_relaxed);
        t->pending[w].store(0, std::memory_order_relaxed);
    }
    std::lock_guard<std::mutex> g(g_reg_mu);
    int rc = install_handler();
    if (rc == CRUM_OK) {
        rc = CRUM_EINVAL;
        for (int i = 0; i < kMaxTrackers; ++i) {
            if (!g_slots[i].load(std::memory_order_relaxed)) {
                t->slot = i;
                g_slots[i].store(t, std::memory_order_release);
                rc = CRUM_OK;
                break;
            }
        }
    }
    if (rc != CRUM_OK) {
        munmap(t->view, bytes);
        delete[] t->dirty;
        delete[] t->pending;
        delete t;
        return rc;
    }
    *out = t;
    return CRUM_OK;
}

void* crum_track_view(crum_track* t)
{
    return t ? t->view : nullptr;
}

int crum_track_flush(crum_track* t, void* dst, uint32_t n_threads, uint64_t* n_flushed)
{
    if (!t || !dst || n_threads == 0 || n_threads > 256)
        return CRUM_EINVAL;
    std::lock_guard<std::mutex> g(t->flush_mu);
    // take the dirty set: clear each bit first, then write-protect, then copy,
    // so a write racing with the flush either lands before the protection
    // (and is copied) or faults and marks the page dirty again
    std::vector<uint64_t> take(t->n_words);
    for (uint64_t w = 0; w < t->n_words; ++w)
        take[w] = t->dirty[w].exchange(0, std::memory_order_acq_rel);
    std::vector<std::pair<uint64_t, uint64_t>> runs;
    for_runs(take, t->n_pages, [&](uint64_t a, uint64_t b) { runs.emplace_back(a, b); });
    const uint64_t P = t->page_size;
    int rc = CRUM_OK;
    for (auto& r : runs)
        if (mprotect(t->view + r.first * P, (r.second - r.first) * P, PROT_READ) != 0)
            rc = CRUM_EINVAL;
    if (rc != CRUM_OK) {
        // leave the pages dirty (and writable) so nothing is lost
        for (auto& r : runs)
            (void)mprotect(t->view + r.first * P, (r.second - r.first) * P,
                           PROT_READ | PROT_WRITE);
        for (uint64_t w = 0; w < t->n_words; ++w)
            t->dirty[w].fetch_or(take[w], std::memory_order_acq_rel);
        return rc;
    }
    // copy the runs, cut into pieces of at most 64 MiB spread over threads
    std::vector<std::pair<uint64_t, uint64_t>> pieces;  // byte offset, length
    const uint64_t cut = std::max<uint64_t>(P, 64ull << 20);
    uint64_t total = 0;
    for (auto& r : runs) {
        for (uint64_t o = r.first * P; o < r.second * P; o += cut)
            pieces.emplace_back(o, std::min(cut, r.second * P - o));
        total += r.second - r.first;
    }
    uint8_t* d = static_cast<uint8_t*>(dst);
    std::atomic<size_t> next{0};
    auto worker = [&]() {
        for (size_t i = next.fetch_add(1); i < pieces.size(); i = next.fetch_add(1))
            std::memcpy(d + pieces[i].first, t->view + pieces[i].first, pieces[i].second);
    };
    const uint32_t nt = (uint32_t)std::min<size_t>(n_threads, pieces.size());
    std::vector<std::thread> th;
    for (uint32_t i = 1; i < nt; ++i)
        th.emplace_back(worker);
    worker();
    for (auto& x : th)
        x.join();
    for (uint64_t w = 0; w < t->n_words; ++w)
        if (take[w])
            t->pending[w].fetch_or(take[w], std::memory_order_acq_rel);
    t->flushed_pages.fetch_add(total, std::memory_order_relaxed);
    if (n_flushed)
        *n_flushed = total;
    return CRUM_OK;
}

int crum_track_pending(crum_track* t, uint64_t* words, uint64_t n_words, int clear)
{
    if (!t || (n_words && !words))
        return CRUM_EINVAL;
    std::lock_guard<std::mutex> g(t->flush_mu);
    for (uint64_t w = 0; w < t->n_words; ++w) {
        const uint64_t v = clear ? t->pending[w].exchange(0, std::memory_order_acq_rel)
                                 : t->pending[w].load(std::memory_order_acquire);
        if (w < n_words)
            words[w] = v;
    }
    for (uint64_t w = t->n_words; w < n_words; ++w)
        words[w] = 0;
    return CRUM_OK;
}

int crum_track_dirty(crum_track* t, uint64_t* words, uint64_t n_words)
{
    if (!t || (n_words && !words))
        return CRUM_EINVAL;
    for (uint64_t w = 0; w < n_words; ++w)
        words[w] = w < t->n_words ? t->dirty[w].load(std::memory_order_acquire) : 0;
    return CRUM_OK;
}

int crum_track_stats(crum_track* t, crum_track_info* out)
{
    if (!t || !out)
        return CRUM_EINVAL;
    uint64_t d = 0, p = 0;
    for (uint64_t w = 0; w < t->n_words; ++w) {
        d += (uint64_t)__builtin_popcountll(t->dirty[w].load(std::memory_order_acquire));
        p += (uint64_t)__builtin_popcountll(t->pending[w].load(std::memory_order_acquire));
    }
    out->pages = t->n_pages;
    out->dirty_pages = d;
    out->pending_pages = p;
    out->faults = t->faults.load(std::memory_order_relaxed);
    out->flushed_pages = t->flushed_pages.load(std::memory_order_relaxed);
    return CRUM_OK;
}

void crum_track_destroy(crum_track* t)
{
    if (!t)
        return;
    {
        std::lock_guard<std::mutex> g(g_reg_mu);
        if (t->slot >= 0)
            g_slots[t->slot].store(nullptr, std::memory_order_release);
    }
    munmap(t->view, t->bytes);
    delete[] t->dirty;
    delete[] t->pending;
    delete t;
}

}  // extern "C"
