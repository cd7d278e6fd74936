/*
 * The CPU oracle (oracle/crum_oracle.c) under AddressSanitizer and
 * UndefinedBehaviorSanitizer: snapshots of random tables (page sizes, NULL
 * shadows, zero-length regions, capacity limits), the streamed-input
 * snapshot with a page source, and the parser and restore fed every
 * truncation of an image prefix plus random bit flips anywhere in it.  The
 * sanitizers catch any out-of-bounds access, use of freed memory or
 * undefined arithmetic on these inputs; the results are checked too.
 * Exit status 0 on success.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    uint8_t* cur;
    uint8_t* shadow;
    uint64_t len;
    uint64_t id;
} orc_region;

typedef struct {
    int32_t code;
    uint32_t first_bad;
    uint64_t n_dirty;
    uint64_t total_pages;
    uint64_t image_bytes;
} orc_status;

typedef struct {
    uint32_t version, page_size, n_regions, flags;
    uint64_t total_pages, n_dirty, seq, data_off;
    uint32_t meta_crc, crcs_crc;
} orc_header;

typedef struct {
    uint64_t len;
    uint64_t id;
    uint32_t has_shadow;
    uint32_t reserved;
} orc_stream_region;

typedef int (*orc_page_fn)(void*, uint32_t, uint64_t, uint8_t*, uint8_t*);

uint32_t orc_crc32c(const uint8_t* p, uint64_t n);
int orc_snapshot(const orc_region* r, uint32_t nr, uint32_t page_size, uint32_t flags,
                 uint64_t seq, uint64_t staging_cap, uint8_t* image, uint64_t image_cap,
                 uint64_t* bitmap_out, uint64_t bitmap_out_words, orc_status* st);
int orc_snapshot_stream(const orc_stream_region* r, uint32_t nr, uint32_t page_size,
                        uint64_t seq, orc_page_fn src, void* user, uint8_t* image,
                        uint64_t image_cap, uint64_t* bitmap_out, uint64_t bitmap_out_words,
                        orc_status* st);
int orc_parse(const uint8_t* img, uint64_t n, orc_header* h);
int orc_restore(const orc_region* r, uint32_t nr, const uint8_t* img, uint64_t n,
                uint32_t flags, orc_status* st);

#define CHECK(c)                                                             \
    do {                                                                     \
        if (!(c)) {                                                          \
            fprintf(stderr, "%s:%d: check failed: %s\n", __FILE__, __LINE__, #c); \
            exit(1);                                                         \
        }                                                                    \
    } while (0)

static uint64_t rs = 88172645463325252ull;
static uint64_t rnd(void)
{
    rs ^= rs << 13;
    rs ^= rs >> 7;
    rs ^= rs << 17;
    return rs;
}

typedef struct {
    uint32_t nr;
    orc_region* r;
    uint32_t P;
} table_src;

/* page source over in-memory regions */
static int src_fn(void* user, uint32_t region, uint64_t page, uint8_t* cur, uint8_t* shadow)
{
    table_src* t = (table_src*)user;
    if (region >= t->nr || (page + 1) * t->P > t->r[region].len)
        return -1;
    memcpy(cur, t->r[region].cur + page * t->P, t->P);
    if (shadow)
        memcpy(shadow, t->r[region].shadow + page * t->P, t->P);
    return 0;
}

static void one_case(int it)
{
    const uint32_t P = 4096u << (rnd() % 3);
    const uint32_t nr = (uint32_t)(rnd() % 5);
    orc_region r[4];
    orc_stream_region sr[4];
    uint64_t G = 0;
    for (uint32_t i = 0; i < nr; ++i) {
        const uint64_t pages = rnd() % 70;
        r[i].len = pages * P;
        r[i].id = 100 + i;
        r[i].cur = (uint8_t*)aligned_alloc(16, r[i].len ? r[i].len : 16);
        r[i].shadow = NULL;
        for (uint64_t b = 0; b < r[i].len; ++b)
            r[i].cur[b] = (uint8_t)rnd();
        const int with_shadow = (rnd() % 4) != 0;
        if (with_shadow) {
            r[i].shadow = (uint8_t*)aligned_alloc(16, r[i].len ? r[i].len : 16);
            memcpy(r[i].shadow, r[i].cur, r[i].len);
            for (uint64_t p = 0; p < pages; ++p)
                if (rnd() % 3 == 0)
                    r[i].shadow[p * P + rnd() % P] ^= (uint8_t)(1 + rnd() % 255);
        }
        sr[i].len = r[i].len;
        sr[i].id = r[i].id;
        sr[i].has_shadow = with_shadow;
        sr[i].reserved = 0;
        G += pages;
    }
    const uint64_t W = (G + 63) / 64;
    const uint64_t cap = 4096 * 2 + 32 * 4 + 8 * W + G * P + 4 * G + 8;
    uint8_t* img = (uint8_t*)malloc(cap);
    uint8_t* img2 = (uint8_t*)malloc(cap);
    uint64_t* bm = (uint64_t*)calloc(W + 1, 8);
    orc_status st, st2;
    CHECK(orc_snapshot(nr ? r : NULL, nr, P, 0, (uint64_t)it, G * P, img, cap, bm, W, &st) ==
          0);
    table_src ts = {nr, r, P};
    CHECK(orc_snapshot_stream(nr ? sr : NULL, nr, P, (uint64_t)it, src_fn, &ts, img2, cap, bm,
                              W, &st2) == 0);
    CHECK(st.image_bytes == st2.image_bytes && memcmp(img, img2, st.image_bytes) == 0);
    const uint64_t n = st.image_bytes;
    orc_header h;
    CHECK(orc_parse(img, n, &h) == 0);
    /* a capacity one byte short: ENOSPC, or EINVAL below the prefix */
    CHECK(orc_snapshot(nr ? r : NULL, nr, P, 0, 0, G * P, img2, n - 1, bm, W, &st2) ==
          (n - 1 < h.data_off ? -1 : -2));
    /* every truncation of the first 4 KiB + 64 bytes, and of the end */
    for (uint64_t k = 0; k < n && k < 4096 + 64; ++k) {
        uint8_t* t = (uint8_t*)malloc(k ? k : 1);
        memcpy(t, img, k);
        CHECK(orc_parse(t, k, &h) != 0);
        free(t);
    }
    /* random bit flips anywhere: parse never reads out of bounds; restore
       either succeeds or fails cleanly */
    for (int f = 0; f < 64; ++f) {
        memcpy(img2, img, n);
        const uint64_t pos = rnd() % n;
        img2[pos] ^= (uint8_t)(1u << (rnd() % 8));
        (void)orc_parse(img2, n, &h);
        (void)orc_restore(nr ? r : NULL, nr, img2, n, 2, &st2);
    }
    /* restore of the intact image with verification */
    CHECK(orc_restore(nr ? r : NULL, nr, img, n, 3, &st2) == 0);
    for (uint32_t i = 0; i < nr; ++i) {
        if (r[i].shadow)
            CHECK(memcmp(r[i].shadow, r[i].cur, r[i].len) == 0);
        free(r[i].cur);
        free(r[i].shadow);
    }
    free(img);
    free(img2);
    free(bm);
}

int main(int argc, char** argv)
{
    const int n = argc > 1 ? atoi(argv[1]) : 60;
    for (int i = 0; i < n; ++i)
        one_case(i);
    /* known value: CRC-32C of "123456789" */
    CHECK(orc_crc32c((const uint8_t*)"123456789", 9) == 0xE3069283u);
    printf("oracle sanitize: ok\n");
    return 0;
}
