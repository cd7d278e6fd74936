/* A C99 client of the library's C ABI: no Python, no torch.  Two regions
 * (one with a shadow, one without), a snapshot with the image in pinned
 * memory, a verified restore into fresh buffers holding the shadow's bytes,
 * an on-demand restore of the same image (one touch, then finish), then a
 * snapshot with shadow update and one more that must find nothing dirty,
 * then host write tracking over a managed region with a tracked snapshot and
 * the allocation-free snapshot of the same region.  In between, a plan of
 * the two regions as two requests is launched twice and each request's
 * image compared with the plain snapshot's, and one of them is persisted
 * to a file by the writer and read back; at the end a serving loop with one
 * client snapshots, repairs a clobbered page by a restore request and finds
 * nothing changed after it.  Prints one line and exits 0 when every check
 * holds. */
#define _POSIX_C_SOURCE 200809L
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <unistd.h>

#include <hip/hip_runtime_api.h>

#include "crum.h"

#define PAGE 4096u
#define N0 40u /* pages of region 0 (has a shadow) */
#define N1 9u  /* pages of region 1 (no shadow: all dirty) */

static int fail(const char* what, long v)
{
    printf("abi_roundtrip: FAIL %s (%ld)\n", what, v);
    return 1;
}

#define HIPOK(x)                                    \
    do {                                            \
        if ((x) != hipSuccess)                      \
            return fail(#x, (long)hipGetLastError()); \
    } while (0)

int main(void)
{
    const size_t b0 = (size_t)N0 * PAGE, b1 = (size_t)N1 * PAGE;
    uint8_t* h_cur0 = malloc(b0);
    uint8_t* h_sh0 = malloc(b0);
    uint8_t* h_cur1 = malloc(b1);
    uint8_t* h_back = malloc(b0 > b1 ? b0 : b1);
    if (!h_cur0 || !h_sh0 || !h_cur1 || !h_back)
        return fail("malloc", 0);
    uint32_t x = 12345u;
    for (size_t i = 0; i < b0; ++i) {
        x = x * 1664525u + 1013904223u;
        h_cur0[i] = (uint8_t)(x >> 24);
    }
    for (size_t i = 0; i < b1; ++i) {
        x = x * 1664525u + 1013904223u;
        h_cur1[i] = (uint8_t)(x >> 24);
    }
    memcpy(h_sh0, h_cur0, b0);
    unsigned n_changed = 0;
    for (unsigned p = 0; p < N0; p += 3) { /* pages 0, 3, 6, ... differ */
        h_sh0[(size_t)p * PAGE + (p * 97u) % PAGE] ^= 0x5a;
        ++n_changed;
    }

    void *cur0, *sh0, *cur1, *t0, *t1, *staging;
    HIPOK(hipMalloc(&cur0, b0));
    HIPOK(hipMalloc(&sh0, b0));
    HIPOK(hipMalloc(&cur1, b1));
    HIPOK(hipMalloc(&t0, b0));
    HIPOK(hipMalloc(&t1, b1));
    HIPOK(hipMemcpy(cur0, h_cur0, b0, hipMemcpyHostToDevice));
    HIPOK(hipMemcpy(sh0, h_sh0, b0, hipMemcpyHostToDevice));
    HIPOK(hipMemcpy(cur1, h_cur1, b1, hipMemcpyHostToDevice));

    uint64_t cap = 0;
    if (crum_image_bytes(2, N0 + N1, N0 + N1, PAGE, &cap) != CRUM_OK)
        return fail("crum_image_bytes", 0);
    HIPOK(hipMalloc(&staging, cap));
    void* h_image = NULL;
    crum_status* st = NULL;
    HIPOK(hipHostMalloc(&h_image, cap, 0));
    HIPOK(hipHostMalloc((void**)&st, sizeof(*st), 0));
    hipStream_t s;
    HIPOK(hipStreamCreate(&s));

    crum_ctx* ctx = NULL;
    int rc = crum_ctx_create(0, NULL, &ctx);
    if (rc != CRUM_OK)
        return fail("crum_ctx_create", rc);
    crum_region regs[2] = {{cur0, sh0, b0, 71}, {cur1, NULL, b1, 72}};
    rc = crum_snapshot(ctx, regs, 2, PAGE, 0, 9, staging, cap, h_image, cap, s, st);
    if (rc != CRUM_OK)
        return fail("crum_snapshot", rc);
    HIPOK(hipStreamSynchronize(s));
    if (st->code != CRUM_OK || st->n_dirty != n_changed + N1 || st->total_pages != N0 + N1)
        return fail("snapshot status", (long)st->n_dirty);
    const uint64_t image_bytes = st->image_bytes;

    /* restore into buffers that hold the shadow's bytes (and garbage) */
    HIPOK(hipMemcpy(t0, h_sh0, b0, hipMemcpyHostToDevice));
    HIPOK(hipMemset(t1, 0xee, b1));
    crum_region targets[2] = {{t0, NULL, b0, 71}, {t1, NULL, b1, 72}};
    rc = crum_restore(ctx, targets, 2, h_image, image_bytes, CRUM_VERIFY, staging, cap, s, st);
    if (rc != CRUM_OK)
        return fail("crum_restore", rc);
    HIPOK(hipStreamSynchronize(s));
    if (st->code != CRUM_OK)
        return fail("restore status", st->code);
    HIPOK(hipMemcpy(h_back, t0, b0, hipMemcpyDeviceToHost));
    if (memcmp(h_back, h_cur0, b0) != 0)
        return fail("region 0 restored bytes", 0);
    HIPOK(hipMemcpy(h_back, t1, b1, hipMemcpyDeviceToHost));
    if (memcmp(h_back, h_cur1, b1) != 0)
        return fail("region 1 restored bytes", 0);

    /* a wrong id is refused before anything is enqueued */
    targets[1].id = 99;
    rc = crum_restore(ctx, targets, 2, h_image, image_bytes, CRUM_VERIFY, staging, cap, s, st);
    if (rc != CRUM_EMISMATCH || st->code != CRUM_EMISMATCH)
        return fail("restore with a wrong id", rc);

    /* a plan: region 0 and region 1 as two requests (caller's order), two
     * launches; each image equals the plain snapshot of that region alone */
    {
        uint64_t cap0 = 0, cap1 = 0;
        if (crum_image_bytes(1, N0, N0, PAGE, &cap0) != CRUM_OK ||
            crum_image_bytes(1, N1, N1, PAGE, &cap1) != CRUM_OK)
            return fail("crum_image_bytes (plan)", 0);
        const uint64_t pcap = (cap0 + 4095) / 4096 * 4096 + (cap1 + 4095) / 4096 * 4096;
        void *pstage = NULL, *h_plan = NULL, *h_one = NULL;
        crum_request_status* pst = NULL;
        HIPOK(hipMalloc(&pstage, pcap));
        HIPOK(hipHostMalloc(&h_plan, pcap, 0));
        HIPOK(hipHostMalloc(&h_one, cap0 > cap1 ? cap0 : cap1, 0));
        HIPOK(hipHostMalloc((void**)&pst, 2 * sizeof(*pst), 0));
        crum_request reqs[2] = {{&regs[0], 1, PAGE, 0, 0, 31}, {&regs[1], 1, PAGE, 0, 0, 32}};
        crum_plan* plan = NULL;
        rc = crum_plan_create(ctx, reqs, 2, pstage, pcap, h_plan, pcap, &plan);
        if (rc != CRUM_OK)
            return fail("crum_plan_create", rc);
        for (int launch = 0; launch < 2; ++launch) {
            memset(pst, 0, 2 * sizeof(*pst));
            rc = crum_plan_launch(plan, s, pst);
            HIPOK(hipStreamSynchronize(s));
            if (rc != CRUM_OK || pst[0].status.code != CRUM_OK ||
                pst[1].status.code != CRUM_OK || pst[0].status.n_dirty != n_changed ||
                pst[1].status.n_dirty != N1 || pst[1].image_offset % 4096 != 0)
                return fail("crum_plan_launch", rc);
        }
        uint32_t n_groups = 0;
        if (crum_plan_groups(plan, &n_groups, NULL, 0) != CRUM_OK || n_groups < 1)
            return fail("crum_plan_groups", (long)n_groups);
        for (unsigned q = 0; q < 2; ++q) {
            rc = crum_snapshot(ctx, &regs[q], 1, PAGE, 0, 31 + q, staging, cap, h_one,
                               q ? cap1 : cap0, s, st);
            HIPOK(hipStreamSynchronize(s));
            if (rc != CRUM_OK || st->code != CRUM_OK ||
                st->image_bytes != pst[q].status.image_bytes ||
                memcmp((const uint8_t*)h_plan + pst[q].image_offset, h_one, st->image_bytes))
                return fail("plan image vs plain snapshot", (long)q);
        }
        crum_plan_destroy(plan);

        /* the writer persists request 0's image; the file reads back equal */
        char path[] = "/tmp/crum_abi_XXXXXX";
        const int fd = mkstemp(path);
        if (fd < 0)
            return fail("mkstemp", 0);
        close(fd);
        crum_writer* wr = NULL;
        uint64_t ticket = 0;
        crum_write_status ws;
        const uint64_t ib0 = pst[0].status.image_bytes;
        if (crum_writer_create(2, 1u << 20, 0, &wr) != CRUM_OK ||
            crum_writer_submit(wr, path, (const uint8_t*)h_plan + pst[0].image_offset, ib0,
                               &ticket) != CRUM_OK ||
            crum_writer_poll(wr, ticket, 1, &ws) != CRUM_OK || ws.code != CRUM_OK ||
            ws.bytes != ib0)
            return fail("crum_writer", 0);
        crum_writer_destroy(wr);
        FILE* f = fopen(path, "rb");
        uint8_t* back = malloc(ib0 + 1);
        if (!f || !back)
            return fail("read back the file", 0);
        const size_t got = fread(back, 1, ib0 + 1, f);
        fclose(f);
        unlink(path);
        if (got != ib0 || memcmp(back, (const uint8_t*)h_plan + pst[0].image_offset, ib0))
            return fail("file equals the image", (long)got);
        free(back);
        HIPOK(hipFree(pstage));
        HIPOK(hipHostFree(h_plan));
        HIPOK(hipHostFree(h_one));
        HIPOK(hipHostFree(pst));
    }

    /* on-demand restore of the same image into buffers holding old bytes:
     * one touch of region 0's page 3 (dirty) fetches exactly that page, then
     * finish fetches the rest */
    targets[1].id = 72;
    HIPOK(hipMemcpy(t0, h_sh0, b0, hipMemcpyHostToDevice));
    HIPOK(hipMemset(t1, 0xee, b1));
    crum_lazy* lz = NULL;
    rc = crum_lazy_open(ctx, targets, 2, h_image, image_bytes, CRUM_VERIFY, 0, staging, cap, s,
                        st, &lz);
    if (rc != CRUM_OK)
        return fail("crum_lazy_open", rc);
    uint64_t fetched = 0;
    rc = crum_lazy_touch(lz, 0, 3u * PAGE + 5u, 1, s, st, &fetched);
    HIPOK(hipStreamSynchronize(s));
    if (rc != CRUM_OK || st->code != CRUM_OK || fetched != 1)
        return fail("crum_lazy_touch", (long)fetched);
    HIPOK(hipMemcpy(h_back, t0, b0, hipMemcpyDeviceToHost));
    if (memcmp(h_back + 3u * PAGE, h_cur0 + 3u * PAGE, PAGE) != 0 ||
        memcmp(h_back + 6u * PAGE, h_sh0 + 6u * PAGE, PAGE) != 0)
        return fail("page 3 fetched alone", 0);
    rc = crum_lazy_finish(lz, s, st);
    HIPOK(hipStreamSynchronize(s));
    crum_lazy_info info;
    if (rc != CRUM_OK || st->code != CRUM_OK || crum_lazy_stats(lz, &info) != CRUM_OK ||
        info.pages_fetched != n_changed + N1 || info.faults != 1)
        return fail("crum_lazy_finish", rc);
    crum_lazy_close(lz);
    HIPOK(hipMemcpy(h_back, t0, b0, hipMemcpyDeviceToHost));
    if (memcmp(h_back, h_cur0, b0) != 0)
        return fail("region 0 after the on-demand restore", 0);
    HIPOK(hipMemcpy(h_back, t1, b1, hipMemcpyDeviceToHost));
    if (memcmp(h_back, h_cur1, b1) != 0)
        return fail("region 1 after the on-demand restore", 0);

    /* shadow update, then nothing is dirty */
    rc = crum_snapshot(ctx, regs, 1, PAGE, CRUM_UPDATE_SHADOW, 10, staging, cap, h_image, cap, s,
                       st);
    HIPOK(hipStreamSynchronize(s));
    if (rc != CRUM_OK || st->code != CRUM_OK || st->n_dirty != n_changed)
        return fail("snapshot with shadow update", rc);
    rc = crum_snapshot(ctx, regs, 1, PAGE, 0, 11, staging, cap, h_image, cap, s, st);
    HIPOK(hipStreamSynchronize(s));
    if (rc != CRUM_OK || st->code != CRUM_OK || st->n_dirty != 0)
        return fail("snapshot after shadow update", (long)st->n_dirty);

    /* host write tracking: a tracker's view over a managed region of N0
     * pages; the first flush (every page of a new view is dirty) fills the
     * region with region 0's bytes, which sh0 now holds too (shadow updated
     * above); then writes to pages 5 and 17 through the view fault once each
     * and are the only candidates of the tracked snapshot, which finds
     * exactly them; the allocation-free entry point gives the same image */
    void* man = NULL;
    HIPOK(hipMallocManaged(&man, b0, hipMemAttachGlobal));
    crum_track* tr = NULL;
    rc = crum_track_create(b0, PAGE, &tr);
    if (rc != CRUM_OK)
        return fail("crum_track_create", rc);
    uint8_t* view = (uint8_t*)crum_track_view(tr);
    memcpy(view, h_cur0, b0);
    uint64_t n_flushed = 0;
    rc = crum_track_flush(tr, man, 2, &n_flushed);
    if (rc != CRUM_OK || n_flushed != N0)
        return fail("first flush", (long)n_flushed);
    uint64_t cand[1];
    if (crum_track_pending(tr, cand, 1, 1) != CRUM_OK || cand[0] != (1ull << N0) - 1)
        return fail("pending after the first flush", 0);
    view[5u * PAGE + 7u] ^= 0x01;
    view[17u * PAGE] ^= 0x02;
    view[17u * PAGE + 1u] ^= 0x04;
    crum_track_info ti;
    if (crum_track_stats(tr, &ti) != CRUM_OK || ti.faults != 2 || ti.dirty_pages != 2)
        return fail("write faults", (long)ti.faults);
    rc = crum_track_flush(tr, man, 1, &n_flushed);
    if (rc != CRUM_OK || n_flushed != 2 || crum_track_pending(tr, cand, 1, 1) != CRUM_OK ||
        cand[0] != ((1ull << 5) | (1ull << 17)))
        return fail("flush of the written pages", (long)n_flushed);
    crum_region mreg[1] = {{man, sh0, b0, 73}};
    rc = crum_snapshot_tracked(ctx, mreg, 1, PAGE, 0, 12, cand, 1, staging, cap, h_image, cap, s,
                               st);
    HIPOK(hipStreamSynchronize(s));
    if (rc != CRUM_OK || st->code != CRUM_OK || st->n_dirty != 2)
        return fail("tracked snapshot", (long)st->n_dirty);
    const uint64_t tracked_bytes = st->image_bytes;
    memcpy(h_back, h_image, tracked_bytes < b0 ? tracked_bytes : b0);
    rc = crum_snapshot_noalloc(ctx, mreg, 1, PAGE, 0, 12, staging, cap, h_image, cap, s, st);
    HIPOK(hipStreamSynchronize(s));
    if (rc != CRUM_OK || st->code != CRUM_OK || st->n_dirty != 2 ||
        st->image_bytes != tracked_bytes || tracked_bytes > b0 ||
        memcmp(h_back, h_image, tracked_bytes) != 0)
        return fail("allocation-free snapshot of the managed region", rc);
    crum_track_destroy(tr);
    HIPOK(hipFree(man));

    /* the serving loop: one client (fresh copies of region 0's bytes and old
     * shadow), two slots; a snapshot finds the changed pages, a restore
     * after clobbering a changed page repairs it, and a second snapshot then
     * finds nothing */
    {
        void *scur = NULL, *ssh = NULL;
        HIPOK(hipMalloc(&scur, b0));
        HIPOK(hipMalloc(&ssh, b0));
        HIPOK(hipMemcpy(scur, h_cur0, b0, hipMemcpyHostToDevice));
        HIPOK(hipMemcpy(ssh, h_sh0, b0, hipMemcpyHostToDevice));
        crum_region sreg[1] = {{scur, ssh, b0, 74}};
        crum_client cl[1] = {{sreg, 1, PAGE}};
        crum_server* srv = NULL;
        rc = crum_server_create(0, cl, 1, 2, 16u << 20, &srv);
        if (rc != CRUM_OK)
            return fail("crum_server_create", rc);
        crum_server_completion done[2];
        uint32_t n_done = 0;
        uint64_t id = 0;
        uint64_t want = 0;
        if (crum_image_bytes(1, N0, n_changed, PAGE, &want) != CRUM_OK)
            return fail("crum_image_bytes (server)", 0);
        if (crum_server_submit(srv, 0, CRUM_REQ_SNAPSHOT, 1, &id) != CRUM_OK ||
            crum_server_poll(srv, done, 2, &n_done, 1) != CRUM_OK || n_done != 1 ||
            done[0].code != CRUM_OK || done[0].n_dirty != n_changed ||
            done[0].image_bytes != want)
            return fail("served snapshot", (long)done[0].n_dirty);
        const void* img_ptr = NULL;
        uint64_t img_len = 0;
        if (crum_server_latest_image(srv, 0, &img_ptr, &img_len) != CRUM_OK || img_len != want)
            return fail("crum_server_latest_image", (long)img_len);
        HIPOK(hipMemset((uint8_t*)scur + 3u * PAGE, 0xee, PAGE)); /* page 3 changed */
        HIPOK(hipDeviceSynchronize()); /* the workers' streams do not wait for it */
        if (crum_server_submit(srv, 0, CRUM_REQ_RESTORE, 2, &id) != CRUM_OK ||
            crum_server_submit(srv, 0, CRUM_REQ_SNAPSHOT, 3, &id) != CRUM_OK ||
            crum_server_poll(srv, done, 2, &n_done, 1) != CRUM_OK || n_done != 2 ||
            done[0].tag != 2 || done[0].code != CRUM_OK || done[1].tag != 3 ||
            done[1].code != CRUM_OK || done[1].n_dirty != 0)
            return fail("served restore, then snapshot", (long)done[1].n_dirty);
        crum_server_destroy(srv);
        HIPOK(hipMemcpy(h_back, scur, b0, hipMemcpyDeviceToHost));
        if (memcmp(h_back, h_cur0, b0) != 0)
            return fail("served restore repaired the page", 0);
        HIPOK(hipFree(scur));
        HIPOK(hipFree(ssh));
    }

    crum_ctx_destroy(ctx);
    HIPOK(hipStreamDestroy(s));
    hipFree(cur0);
    hipFree(sh0);
    hipFree(cur1);
    hipFree(t0);
    hipFree(t1);
    hipFree(staging);
    hipHostFree(h_image);
    hipHostFree(st);
    free(h_cur0);
    free(h_sh0);
    free(h_cur1);
    free(h_back);
    printf("abi_roundtrip: ok (%u + %u dirty pages, image %llu bytes)\n", n_changed, N1,
           (unsigned long long)image_bytes);
    return 0;
}
