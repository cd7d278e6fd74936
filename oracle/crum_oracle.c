/*
 * crum_oracle.c -- plain CPU oracle for the incremental GPU snapshot.
 *
 * TEST INFRASTRUCTURE.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may call this code.  The product library never
 * links, loads or calls it, and the two share no code, header, table or
 * constant generator.  It is written for obviousness, not speed: one thread,
 * byte-wise CRC, memcmp per page, loops in the order the definitions give.
 *
 * What it computes (every step exact; there is no floating point):
 *
 *  1. Region table (paper section 3.4, checkpoint: every active device and
 *     managed region is read back to the host).  Page boundaries are relative
 *     to each region's base; pages are numbered globally in table order.
 *  2. Dirty set.  A page is dirty when its current bytes differ from its
 *     shadow bytes (memcmp).  A region without a shadow has every page dirty,
 *     as a freshly created shadow region has all pages dirty in the paper's
 *     shadow-page scheme (section 3.2, Algorithm 1 and the text after it).
 *  3. Compaction: dirty pages are appended in ascending global page order.
 *  4. CRC-32C (iSCSI polynomial 0x1EDC6F41, reflected, init and final XOR
 *     0xFFFFFFFF) of every packed page, computed byte at a time with a
 *     256-entry table that is itself built from the bitwise rule (Sarwate's
 *     table method).
 *  5. Optional shadow update after a successful snapshot: the analogue of the
 *     paper's flush-then-clear-dirty step (Algorithm 1, CUDA-call event).
 *  6. The checkpoint image, layout v1 (see orc_snapshot below).
 *  7. Restore (paper section 3.4, restart: data copied back into re-created
 *     regions): parse and check the image, check the destination table,
 *     optionally verify every page CRC before writing anything, then copy
 *     packed page k to the k-th set bit's page.
 *  8. The snapshot of steps 1-4 and 6 again with the region bytes handed in
 *     one page at a time by a caller's source (orc_snapshot_stream), for
 *     workloads of tens of GB that cannot be held twice in host memory.
 *
 * Status codes: 0 OK, -1 EINVAL, -2 ENOSPC, -3 ECRC, -4 EFORMAT, -6 EMISMATCH.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_EINVAL (-1)
#define ORC_ENOSPC (-2)
#define ORC_ECRC (-3)
#define ORC_EFORMAT (-4)
#define ORC_EMISMATCH (-6)

#define ORC_UPDATE_SHADOW 1u
#define ORC_VERIFY 2u

typedef struct {
    uint8_t* cur;     /* region bytes (read by snapshot, written by restore) */
    uint8_t* shadow;  /* NULL: no baseline */
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
    uint32_t version;
    uint32_t page_size;
    uint32_t n_regions;
    uint32_t flags;
    uint64_t total_pages;
    uint64_t n_dirty;
    uint64_t seq;
    uint64_t data_off;
    uint32_t meta_crc;
    uint32_t crcs_crc;
} orc_header;

/* ------------------------------------------------------------------ CRC-32C */

static uint32_t crc_table[256];
static int crc_table_ready = 0;

/* One table entry per byte value: the register after shifting that byte
 * through eight steps of the bitwise rule (reflected polynomial 0x82F63B78). */
static void build_crc_table(void)
{
    for (uint32_t b = 0; b < 256; ++b) {
        uint32_t c = b;
        for (int k = 0; k < 8; ++k)
            c = (c & 1u) ? (c >> 1) ^ 0x82F63B78u : (c >> 1);
        crc_table[b] = c;
    }
    crc_table_ready = 1;
}

uint32_t orc_crc32c(const uint8_t* p, uint64_t n)
{
    if (!crc_table_ready)
        build_crc_table();
    uint32_t c = 0xFFFFFFFFu;
    for (uint64_t i = 0; i < n; ++i)
        c = (c >> 8) ^ crc_table[(c ^ p[i]) & 0xFFu];
    return c ^ 0xFFFFFFFFu;
}

/* ------------------------------------------------------------ little endian */

static void put_u32(uint8_t* p, uint32_t v)
{
    for (int i = 0; i < 4; ++i)
        p[i] = (uint8_t)(v >> (8 * i));
}

static void put_u64(uint8_t* p, uint64_t v)
{
    for (int i = 0; i < 8; ++i)
        p[i] = (uint8_t)(v >> (8 * i));
}

static uint32_t get_u32(const uint8_t* p)
{
    uint32_t v = 0;
    for (int i = 0; i < 4; ++i)
        v |= (uint32_t)p[i] << (8 * i);
    return v;
}

static uint64_t get_u64(const uint8_t* p)
{
    uint64_t v = 0;
    for (int i = 0; i < 8; ++i)
        v |= (uint64_t)p[i] << (8 * i);
    return v;
}

static uint64_t round_up(uint64_t x, uint64_t a) { return (x + a - 1) / a * a; }

/* -------------------------------------------------------------- validation */

static int page_size_ok(uint64_t p)
{
    if (p < 4096u || p > (1u << 30))
        return 0;
    return (p & (p - 1)) == 0;
}

static int ranges_overlap(uintptr_t a, uint64_t alen, uintptr_t b, uint64_t blen)
{
    if (alen == 0 || blen == 0)
        return 0;
    return a < b + blen && b < a + alen;
}

/* Pointer rules: non-empty regions have a current pointer; every pointer is
 * 16-byte aligned; no current or shadow range overlaps another. */
static int orc_validate_ranges(const orc_region* r, uint32_t nr)
{
    if (nr > 0 && r == NULL)
        return ORC_EINVAL;
    for (uint32_t i = 0; i < nr; ++i) {
        if (r[i].len > 0 && r[i].cur == NULL)
            return ORC_EINVAL;
        if (((uintptr_t)r[i].cur & 15u) || ((uintptr_t)r[i].shadow & 15u))
            return ORC_EINVAL;
    }
    /* every pair of ranges among {cur_i, shadow_i}: pairwise disjoint */
    for (uint32_t i = 0; i < nr; ++i) {
        if (r[i].shadow && ranges_overlap((uintptr_t)r[i].cur, r[i].len,
                                          (uintptr_t)r[i].shadow, r[i].len))
            return ORC_EINVAL;
        for (uint32_t j = i + 1; j < nr; ++j) {
            if (ranges_overlap((uintptr_t)r[i].cur, r[i].len, (uintptr_t)r[j].cur, r[j].len))
                return ORC_EINVAL;
            if (r[j].shadow &&
                ranges_overlap((uintptr_t)r[i].cur, r[i].len, (uintptr_t)r[j].shadow, r[j].len))
                return ORC_EINVAL;
            if (r[i].shadow &&
                ranges_overlap((uintptr_t)r[i].shadow, r[i].len, (uintptr_t)r[j].cur, r[j].len))
                return ORC_EINVAL;
            if (r[i].shadow && r[j].shadow &&
                ranges_overlap((uintptr_t)r[i].shadow, r[i].len, (uintptr_t)r[j].shadow,
                               r[j].len))
                return ORC_EINVAL;
        }
    }
    return ORC_OK;
}

/* Snapshot argument rules: page size a power of two in [4 KiB, 1 GiB], every
 * length a multiple of the page size, and the pointer rules above. */
int orc_validate(const orc_region* r, uint32_t nr, uint32_t page_size)
{
    if (!page_size_ok(page_size))
        return ORC_EINVAL;
    if (nr > 0 && r == NULL)
        return ORC_EINVAL;
    for (uint32_t i = 0; i < nr; ++i)
        if (r[i].len % page_size != 0)
            return ORC_EINVAL;
    return orc_validate_ranges(r, nr);
}

/* Bytes before the first packed page: header (64) + region table (32 per
 * region) + bitmap (8 per 64 pages), rounded up to 4096. */
uint64_t orc_prefix_bytes(uint32_t nr, uint64_t total_pages)
{
    const uint64_t words = (total_pages + 63) / 64;
    return round_up(64 + 32 * (uint64_t)nr + 8 * words, 4096);
}

/* ---------------------------------------------------------------- snapshot */

/*
 * Image layout v1 (little-endian, every pad byte zero):
 *    0  magic "CRUMIMG1"         8  u32 version = 1      12  u32 page_size
 *   16  u32 n_regions           20  u32 flags (bit 0: no region had a shadow)
 *   24  u64 total_pages G       32  u64 n_dirty D       40  u64 seq
 *   48  u64 data_off            56  u32 meta_crc        60  u32 crcs_crc
 *   64  region table: per region u64 id, u64 len, u64 first_page, u64 0
 *   64+32R  bitmap: ceil(G/64) u64 words, bit (g mod 64) of word g/64
 *   zero pad up to data_off = roundup(64 + 32R + 8W, 4096)
 *   data_off       D packed pages, ascending global page index
 *   data_off+D*P   D u32 page CRCs, then zero pad to a multiple of 8
 * crcs_crc = CRC-32C of the D*4 CRC bytes; meta_crc = CRC-32C of bytes
 * [0, 64 + 32R + 8W) with bytes 56..59 read as zero (computed last).
 *
 * ENOSPC when D*P > staging_cap or the image exceeds image_cap: then nothing
 * is written to the image or the shadows, but n_dirty, total_pages,
 * image_bytes (the size that would be needed) and the bitmap are reported.
 */
int orc_snapshot(const orc_region* r, uint32_t nr, uint32_t page_size, uint32_t flags,
                 uint64_t seq, uint64_t staging_cap, uint8_t* image, uint64_t image_cap,
                 uint64_t* bitmap_out, uint64_t bitmap_out_words, orc_status* st)
{
    memset(st, 0, sizeof(*st));
    if (orc_validate(r, nr, page_size) != ORC_OK || image == NULL) {
        st->code = ORC_EINVAL;
        return ORC_EINVAL;
    }
    const uint64_t P = page_size;

    /* flatten: first page of each region, total G */
    uint64_t G = 0;
    uint64_t* first = (uint64_t*)calloc(nr ? nr : 1, sizeof(uint64_t));
    for (uint32_t i = 0; i < nr; ++i) {
        first[i] = G;
        G += r[i].len / P;
    }
    const uint64_t W = (G + 63) / 64;
    const uint64_t prefix_end = 64 + 32 * (uint64_t)nr + 8 * W;
    const uint64_t data_off = round_up(prefix_end, 4096);
    if (image_cap < data_off) {
        free(first);
        st->code = ORC_EINVAL;
        return ORC_EINVAL;
    }

    /* diff: one bit per page */
    uint64_t* bitmap = (uint64_t*)calloc(W ? W : 1, sizeof(uint64_t));
    uint64_t D = 0;
    for (uint32_t i = 0; i < nr; ++i) {
        for (uint64_t p = 0; p < r[i].len / P; ++p) {
            const uint64_t g = first[i] + p;
            int dirty;
            if (r[i].shadow == NULL)
                dirty = 1;
            else
                dirty = memcmp(r[i].cur + p * P, r[i].shadow + p * P, P) != 0;
            if (dirty) {
                bitmap[g / 64] |= (uint64_t)1 << (g % 64);
                D += 1;
            }
        }
    }
    const uint64_t total = data_off + D * P + round_up(4 * D, 8);
    st->n_dirty = D;
    st->total_pages = G;
    st->image_bytes = total;
    if (bitmap_out) {
        for (uint64_t w = 0; w < W && w < bitmap_out_words; ++w)
            bitmap_out[w] = bitmap[w];
    }
    if (D * P > staging_cap || total > image_cap) {
        free(first);
        free(bitmap);
        st->code = ORC_ENOSPC;
        return ORC_ENOSPC;
    }

    /* header, region table, bitmap, zero pad */
    memset(image, 0, data_off);
    memcpy(image, "CRUMIMG1", 8);
    put_u32(image + 8, 1);
    put_u32(image + 12, page_size);
    put_u32(image + 16, nr);
    uint32_t img_flags = 1;
    for (uint32_t i = 0; i < nr; ++i)
        if (r[i].shadow != NULL)
            img_flags = 0;
    put_u32(image + 20, img_flags);
    put_u64(image + 24, G);
    put_u64(image + 32, D);
    put_u64(image + 40, seq);
    put_u64(image + 48, data_off);
    for (uint32_t i = 0; i < nr; ++i) {
        uint8_t* e = image + 64 + 32 * (uint64_t)i;
        put_u64(e, r[i].id);
        put_u64(e + 8, r[i].len);
        put_u64(e + 16, first[i]);
        put_u64(e + 24, 0);
    }
    for (uint64_t w = 0; w < W; ++w)
        put_u64(image + 64 + 32 * (uint64_t)nr + 8 * w, bitmap[w]);

    /* pages in ascending g, and their CRCs */
    uint8_t* pages = image + data_off;
    uint8_t* crcs = pages + D * P;
    uint64_t k = 0;
    for (uint32_t i = 0; i < nr; ++i) {
        for (uint64_t p = 0; p < r[i].len / P; ++p) {
            const uint64_t g = first[i] + p;
            if ((bitmap[g / 64] >> (g % 64)) & 1u) {
                memcpy(pages + k * P, r[i].cur + p * P, P);
                put_u32(crcs + 4 * k, orc_crc32c(r[i].cur + p * P, P));
                k += 1;
            }
        }
    }
    memset(crcs + 4 * D, 0, round_up(4 * D, 8) - 4 * D);

    put_u32(image + 60, orc_crc32c(crcs, 4 * D));
    put_u32(image + 56, 0);
    put_u32(image + 56, orc_crc32c(image, prefix_end));

    /* shadow update only after success */
    if (flags & ORC_UPDATE_SHADOW) {
        for (uint32_t i = 0; i < nr; ++i) {
            if (r[i].shadow == NULL)
                continue;
            for (uint64_t p = 0; p < r[i].len / P; ++p) {
                const uint64_t g = first[i] + p;
                if ((bitmap[g / 64] >> (g % 64)) & 1u)
                    memcpy(r[i].shadow + p * P, r[i].cur + p * P, P);
            }
        }
    }
    free(first);
    free(bitmap);
    st->code = ORC_OK;
    return ORC_OK;
}

/* -------------------------------------------------------- streamed input */

/*
 * The same snapshot with the region bytes supplied one page at a time by the
 * caller instead of as whole buffers, for workloads too large to hold twice
 * in host memory (tens of GB).  Nothing else changes: the same definition,
 * in the same order.  The source fills `cur` with page `page` of region
 * `region` and, when `shadow` is not NULL, the shadow's copy of that page;
 * it returns 0, or nonzero to abort (status EINVAL).  A region without a
 * shadow has every page dirty and is never asked for shadow bytes.  There is
 * no shadow update: the source owns the bytes.
 *
 * Two passes over the pages, as the definition reads: first the diff of
 * every page (building the bitmap), then the dirty pages again in ascending
 * order, each copied into the image with its CRC.
 */
typedef int (*orc_page_fn)(void* user, uint32_t region, uint64_t page, uint8_t* cur,
                           uint8_t* shadow);

typedef struct {
    uint64_t len;
    uint64_t id;
    uint32_t has_shadow;
    uint32_t reserved;
} orc_stream_region;

int orc_snapshot_stream(const orc_stream_region* r, uint32_t nr, uint32_t page_size,
                        uint64_t seq, orc_page_fn src, void* user, uint8_t* image,
                        uint64_t image_cap, uint64_t* bitmap_out, uint64_t bitmap_out_words,
                        orc_status* st)
{
    memset(st, 0, sizeof(*st));
    if (!page_size_ok(page_size) || (nr > 0 && r == NULL) || src == NULL || image == NULL) {
        st->code = ORC_EINVAL;
        return ORC_EINVAL;
    }
    for (uint32_t i = 0; i < nr; ++i) {
        if (r[i].len % page_size != 0) {
            st->code = ORC_EINVAL;
            return ORC_EINVAL;
        }
    }
    const uint64_t P = page_size;

    /* flatten: first page of each region, total G */
    uint64_t G = 0;
    uint64_t* first = (uint64_t*)calloc(nr ? nr : 1, sizeof(uint64_t));
    for (uint32_t i = 0; i < nr; ++i) {
        first[i] = G;
        G += r[i].len / P;
    }
    const uint64_t W = (G + 63) / 64;
    const uint64_t prefix_end = 64 + 32 * (uint64_t)nr + 8 * W;
    const uint64_t data_off = round_up(prefix_end, 4096);
    uint8_t* cur = (uint8_t*)malloc(P);
    uint8_t* sh = (uint8_t*)malloc(P);
    uint64_t* bitmap = (uint64_t*)calloc(W ? W : 1, sizeof(uint64_t));
    int rc = ORC_OK;
    if (image_cap < data_off)
        rc = ORC_EINVAL;

    /* diff: one bit per page */
    uint64_t D = 0;
    for (uint32_t i = 0; i < nr && rc == ORC_OK; ++i) {
        for (uint64_t p = 0; p < r[i].len / P; ++p) {
            const uint64_t g = first[i] + p;
            if (src(user, i, p, cur, r[i].has_shadow ? sh : NULL) != 0) {
                rc = ORC_EINVAL;
                break;
            }
            const int dirty = !r[i].has_shadow || memcmp(cur, sh, P) != 0;
            if (dirty) {
                bitmap[g / 64] |= (uint64_t)1 << (g % 64);
                D += 1;
            }
        }
    }
    const uint64_t total = data_off + D * P + round_up(4 * D, 8);
    if (rc == ORC_OK) {
        st->n_dirty = D;
        st->total_pages = G;
        st->image_bytes = total;
        if (bitmap_out) {
            for (uint64_t w = 0; w < W && w < bitmap_out_words; ++w)
                bitmap_out[w] = bitmap[w];
        }
        if (total > image_cap)
            rc = ORC_ENOSPC;
    }

    if (rc == ORC_OK) {
        /* header, region table, bitmap, zero pad */
        memset(image, 0, data_off);
        memcpy(image, "CRUMIMG1", 8);
        put_u32(image + 8, 1);
        put_u32(image + 12, page_size);
        put_u32(image + 16, nr);
        uint32_t img_flags = 1;
        for (uint32_t i = 0; i < nr; ++i)
            if (r[i].has_shadow)
                img_flags = 0;
        put_u32(image + 20, img_flags);
        put_u64(image + 24, G);
        put_u64(image + 32, D);
        put_u64(image + 40, seq);
        put_u64(image + 48, data_off);
        for (uint32_t i = 0; i < nr; ++i) {
            uint8_t* e = image + 64 + 32 * (uint64_t)i;
            put_u64(e, r[i].id);
            put_u64(e + 8, r[i].len);
            put_u64(e + 16, first[i]);
            put_u64(e + 24, 0);
        }
        for (uint64_t w = 0; w < W; ++w)
            put_u64(image + 64 + 32 * (uint64_t)nr + 8 * w, bitmap[w]);

        /* pages in ascending g, and their CRCs */
        uint8_t* pages = image + data_off;
        uint8_t* crcs = pages + D * P;
        uint64_t k = 0;
        for (uint32_t i = 0; i < nr && rc == ORC_OK; ++i) {
            for (uint64_t p = 0; p < r[i].len / P; ++p) {
                const uint64_t g = first[i] + p;
                if (!((bitmap[g / 64] >> (g % 64)) & 1u))
                    continue;
                if (src(user, i, p, pages + k * P, NULL) != 0) {
                    rc = ORC_EINVAL;
                    break;
                }
                put_u32(crcs + 4 * k, orc_crc32c(pages + k * P, P));
                k += 1;
            }
        }
        if (rc == ORC_OK) {
            memset(crcs + 4 * D, 0, round_up(4 * D, 8) - 4 * D);
            put_u32(image + 60, orc_crc32c(crcs, 4 * D));
            put_u32(image + 56, 0);
            put_u32(image + 56, orc_crc32c(image, prefix_end));
        }
    }
    free(first);
    free(cur);
    free(sh);
    free(bitmap);
    if (rc == ORC_EINVAL) {
        memset(st, 0, sizeof(*st));
    }
    st->code = rc;
    return rc;
}

/* ------------------------------------------------------------------- parse */

int orc_parse(const uint8_t* img, uint64_t n, orc_header* h)
{
    memset(h, 0, sizeof(*h));
    if (img == NULL || n < 64)
        return ORC_EFORMAT;
    if (memcmp(img, "CRUMIMG1", 8) != 0)
        return ORC_EFORMAT;
    h->version = get_u32(img + 8);
    h->page_size = get_u32(img + 12);
    h->n_regions = get_u32(img + 16);
    h->flags = get_u32(img + 20);
    h->total_pages = get_u64(img + 24);
    h->n_dirty = get_u64(img + 32);
    h->seq = get_u64(img + 40);
    h->data_off = get_u64(img + 48);
    h->meta_crc = get_u32(img + 56);
    h->crcs_crc = get_u32(img + 60);
    if (h->version != 1 || !page_size_ok(h->page_size) || (h->flags & ~1u) != 0)
        return ORC_EFORMAT;
    const uint64_t P = h->page_size, G = h->total_pages, D = h->n_dirty, R = h->n_regions;
    if (G > ((uint64_t)1 << 40) || D > G)
        return ORC_EFORMAT;
    const uint64_t W = (G + 63) / 64;
    const uint64_t prefix_end = 64 + 32 * R + 8 * W;
    if (h->data_off != round_up(prefix_end, 4096) || h->data_off > n)
        return ORC_EFORMAT;
    if (D > (n - h->data_off) / P)
        return ORC_EFORMAT;
    const uint64_t total = h->data_off + D * P + round_up(4 * D, 8);
    if (total != n)
        return ORC_EFORMAT;

    /* region table: zero reserved word, lengths multiple of P, first_page chain */
    uint64_t chain = 0;
    for (uint64_t i = 0; i < R; ++i) {
        const uint8_t* e = img + 64 + 32 * i;
        const uint64_t len = get_u64(e + 8), fp = get_u64(e + 16), rsv = get_u64(e + 24);
        if (rsv != 0 || len % P != 0 || fp != chain)
            return ORC_EFORMAT;
        chain += len / P;
        if (chain > G)
            return ORC_EFORMAT;
    }
    if (chain != G)
        return ORC_EFORMAT;

    /* bitmap: popcount equals D, no bit at or beyond G */
    uint64_t ones = 0;
    for (uint64_t w = 0; w < W; ++w) {
        const uint64_t word = get_u64(img + 64 + 32 * R + 8 * w);
        for (int b = 0; b < 64; ++b) {
            if ((word >> b) & 1u) {
                if (w * 64 + (uint64_t)b >= G)
                    return ORC_EFORMAT;
                ones += 1;
            }
        }
    }
    if (ones != D)
        return ORC_EFORMAT;

    /* both pads are zero */
    for (uint64_t i = prefix_end; i < h->data_off; ++i)
        if (img[i] != 0)
            return ORC_EFORMAT;
    for (uint64_t i = h->data_off + D * P + 4 * D; i < total; ++i)
        if (img[i] != 0)
            return ORC_EFORMAT;

    /* checksums */
    if (orc_crc32c(img + h->data_off + D * P, 4 * D) != h->crcs_crc)
        return ORC_EFORMAT;
    uint8_t* meta = (uint8_t*)malloc(prefix_end);
    memcpy(meta, img, prefix_end);
    put_u32(meta + 56, 0);
    const uint32_t mc = orc_crc32c(meta, prefix_end);
    free(meta);
    if (mc != h->meta_crc)
        return ORC_EFORMAT;
    return ORC_OK;
}

/* ----------------------------------------------------------------- restore */

int orc_restore(const orc_region* r, uint32_t nr, const uint8_t* img, uint64_t n,
                uint32_t flags, orc_status* st)
{
    memset(st, 0, sizeof(*st));
    /* order of checks: pointer rules, then the image, then the table */
    orc_header h;
    int rc = orc_validate_ranges(r, nr);
    if (rc == ORC_OK)
        rc = orc_parse(img, n, &h);
    if (rc != ORC_OK) {
        st->code = rc;
        return rc;
    }
    const uint64_t P = h.page_size, D = h.n_dirty, G = h.total_pages;
    st->n_dirty = D;
    st->total_pages = G;
    st->image_bytes = n;
    if (nr != h.n_regions) {
        st->code = ORC_EMISMATCH;
        return ORC_EMISMATCH;
    }
    for (uint32_t i = 0; i < nr; ++i) {
        const uint8_t* e = img + 64 + 32 * (uint64_t)i;
        if (get_u64(e) != r[i].id || get_u64(e + 8) != r[i].len) {
            st->code = ORC_EMISMATCH;
            return ORC_EMISMATCH;
        }
    }
    const uint8_t* pages = img + h.data_off;
    const uint8_t* crcs = pages + D * P;
    if (flags & ORC_VERIFY) {
        for (uint64_t k = 0; k < D; ++k) {
            if (orc_crc32c(pages + k * P, P) != get_u32(crcs + 4 * k)) {
                st->code = ORC_ECRC;
                st->first_bad = (uint32_t)k;
                return ORC_ECRC;
            }
        }
    }
    const uint8_t* bm = img + 64 + 32 * (uint64_t)nr;
    uint64_t k = 0, g = 0;
    for (uint32_t i = 0; i < nr; ++i) {
        for (uint64_t p = 0; p < r[i].len / P; ++p, ++g) {
            const uint64_t word = get_u64(bm + 8 * (g / 64));
            if ((word >> (g % 64)) & 1u) {
                memcpy(r[i].cur + p * P, pages + k * P, P);
                if ((flags & ORC_UPDATE_SHADOW) && r[i].shadow != NULL)
                    memcpy(r[i].shadow + p * P, pages + k * P, P);
                k += 1;
            }
        }
    }
    st->code = ORC_OK;
    return ORC_OK;
}
