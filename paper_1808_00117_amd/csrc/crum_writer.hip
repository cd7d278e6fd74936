// Persisting images to storage while the caller continues.
//
// The paper's phase two writes the checkpoint image to disk from a forked
// child while the application resumes (section 3.3).  Here the image is
// already in pinned host memory when the snapshot returns, so a pool of
// writer threads in the same process persists it: the file is cut into
// chunks, each written with pwrite at its own offset (in parallel across the
// pool), through an O_DIRECT descriptor where the chunk, its offset and the
// buffer are 4 KiB aligned and the file system allows it, otherwise through
// a buffered descriptor.  Host code only; no device work.
#include "crum.h"

#include <atomic>
#include <cerrno>
#include <chrono>
#include <condition_variable>
#include <cstdint>
#include <cstring>
#include <deque>
#include <fcntl.h>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unistd.h>
#include <vector>

namespace {

using Clock = std::chrono::steady_clock;
constexpr uint64_t kAlign = 4096;

struct Job {
    uint64_t ticket = 0;
    const uint8_t* img = nullptr;
    uint64_t bytes = 0;
    int fd_buf = -1;
    int fd_direct = -1;
    uint64_t n_chunks = 0;
    std::atomic<uint64_t> next{0};
    uint64_t chunks_done = 0;  // under the writer's lock
    int err = 0;               // under the writer's lock
    // Direct I/O can be refused per buffer (pinned memory that the kernel
    // cannot map for it gives EFAULT): the chunk then goes through the page
    // cache and the job stops trying.
    std::atomic<bool> direct_ok{true};
    std::atomic<bool> direct_used{false};
    bool done = false;
    Clock::time_point t0;
    crum_write_status st{};
};

// pwrite all of [p, p+n) at offset off; returns 0 or errno
int write_all(int fd, const uint8_t* p, uint64_t n, uint64_t off)
{
    while (n) {
        const ssize_t w = pwrite(fd, p, n, (off_t)off);
        if (w < 0) {
            if (errno == EINTR)
                continue;
            return errno;
        }
        if (w == 0)
            return EIO;
        p += w;
        n -= (uint64_t)w;
        off += (uint64_t)w;
    }
    return 0;
}

}  // namespace

struct crum_writer {
    uint64_t chunk_bytes = 0;
    uint32_t flags = 0;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<std::shared_ptr<Job>> active;  // jobs with chunks left to claim
    std::map<uint64_t, std::shared_ptr<Job>> jobs;
    uint64_t next_ticket = 1;
    bool stop = false;
    std::vector<std::thread> threads;
};

namespace {

void finish(crum_writer* w, Job& j)
{
    // called once, without the lock, by the thread that wrote the last chunk
    int err = 0;
    {
        std::lock_guard<std::mutex> lk(w->mu);
        err = j.err;
    }
    // the file was opened without O_TRUNC (truncating a large cached file
    // frees its pages, which would stall the caller in submit); set its
    // length here, on a writer thread
    if (!err && ftruncate(j.fd_buf, (off_t)j.bytes) != 0)
        err = errno;
    if (!err && (w->flags & CRUM_WRITE_SYNC) && fdatasync(j.fd_buf) != 0)
        err = errno;
    if (j.fd_direct >= 0)
        close(j.fd_direct);
    if (close(j.fd_buf) != 0 && !err)
        err = errno;
    std::lock_guard<std::mutex> lk(w->mu);
    j.st.code = err ? (int32_t)CRUM_EIO : (int32_t)CRUM_OK;
    j.st.err = err;
    j.st.bytes = err ? 0 : j.bytes;
    j.st.direct = j.direct_used.load() ? 1u : 0u;
    j.st.seconds = std::chrono::duration<double>(Clock::now() - j.t0).count();
    j.done = true;
    w->cv_done.notify_all();
}

void run(crum_writer* w)
{
    for (;;) {
        std::shared_ptr<Job> job;
        uint64_t k = 0;
        {
            std::unique_lock<std::mutex> lk(w->mu);
            for (;;) {
                while (!w->active.empty() &&
                       w->active.front()->next.load() >= w->active.front()->n_chunks)
                    w->active.pop_front();
                if (!w->active.empty()) {
                    job = w->active.front();
                    k = job->next.fetch_add(1);
                    if (k < job->n_chunks)
                        break;
                    continue;
                }
                if (w->stop)
                    return;
                w->cv_work.wait(lk);
            }
        }
        const uint64_t off = k * w->chunk_bytes;
        const uint64_t len = std::min<uint64_t>(w->chunk_bytes, job->bytes - off);
        const bool direct = job->fd_direct >= 0 && job->direct_ok.load() && len % kAlign == 0;
        int err = write_all(direct ? job->fd_direct : job->fd_buf, job->img + off, len, off);
        if (direct && !err)
            job->direct_used = true;
        if (direct && (err == EFAULT || err == EINVAL || err == EOPNOTSUPP)) {
            job->direct_ok = false;
            err = write_all(job->fd_buf, job->img + off, len, off);
        }
        bool last = false;
        {
            std::lock_guard<std::mutex> lk(w->mu);
            if (err && !job->err)
                job->err = err;
            last = ++job->chunks_done == job->n_chunks;
        }
        if (last)
            finish(w, *job);
    }
}

}  // namespace

extern "C" {

int crum_writer_create(uint32_t n_threads, uint64_t chunk_bytes, uint32_t flags,
                       crum_writer** out)
{
    if (!out || n_threads == 0 || n_threads > 256 || chunk_bytes == 0 ||
        chunk_bytes % kAlign || (flags & ~(uint32_t)(CRUM_WRITE_DIRECT | CRUM_WRITE_SYNC)))
        return CRUM_EINVAL;
    crum_writer* w = new crum_writer();
    w->chunk_bytes = chunk_bytes;
    w->flags = flags;
    for (uint32_t i = 0; i < n_threads; ++i)
        w->threads.emplace_back(run, w);
    *out = w;
    return CRUM_OK;
}

int crum_writer_submit(crum_writer* w, const char* path, const void* image, uint64_t bytes,
                       uint64_t* ticket)
{
    if (!w || !path || !ticket || (bytes && !image))
        return CRUM_EINVAL;
    auto job = std::make_shared<Job>();
    job->t0 = Clock::now();
    job->img = static_cast<const uint8_t*>(image);
    job->bytes = bytes;
    job->fd_buf = open(path, O_WRONLY | O_CREAT | O_CLOEXEC, 0644);
    if (job->fd_buf < 0)
        return CRUM_EIO;
    if ((w->flags & CRUM_WRITE_DIRECT) && bytes >= kAlign &&
        reinterpret_cast<uintptr_t>(image) % kAlign == 0)
        job->fd_direct = open(path, O_WRONLY | O_DIRECT | O_CLOEXEC);  // -1: not supported here
    job->n_chunks = (bytes + w->chunk_bytes - 1) / w->chunk_bytes;
    std::unique_lock<std::mutex> lk(w->mu);
    job->ticket = w->next_ticket++;
    *ticket = job->ticket;
    w->jobs[job->ticket] = job;
    if (job->n_chunks == 0) {
        lk.unlock();
        finish(w, *job);
        return CRUM_OK;
    }
    w->active.push_back(job);
    w->cv_work.notify_all();
    return CRUM_OK;
}

int crum_writer_poll(crum_writer* w, uint64_t ticket, int wait, crum_write_status* out)
{
    if (!w || !out)
        return CRUM_EINVAL;
    std::unique_lock<std::mutex> lk(w->mu);
    auto it = w->jobs.find(ticket);
    if (it == w->jobs.end())
        return CRUM_EINVAL;
    std::shared_ptr<Job> job = it->second;
    if (!job->done) {
        if (!wait)
            return CRUM_EAGAIN;
        w->cv_done.wait(lk, [&] { return job->done; });
    }
    *out = job->st;
    w->jobs.erase(ticket);
    return CRUM_OK;
}

void crum_writer_destroy(crum_writer* w)
{
    if (!w)
        return;
    {
        std::unique_lock<std::mutex> lk(w->mu);
        // finish what was submitted
        w->cv_done.wait(lk, [&] {
            for (auto& kv : w->jobs)
                if (!kv.second->done)
                    return false;
            return true;
        });
        w->stop = true;
        w->cv_work.notify_all();
    }
    for (auto& t : w->threads)
        t.join();
    delete w;
}

}  // extern "C"
