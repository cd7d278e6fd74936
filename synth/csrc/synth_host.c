/*
 * Seeded synthetic memory images: host fill.
 *
 * Word j (8 bytes, little-endian) of region r under seed s is the SplitMix64
 * output function (Steele, Lea & Flood, "Fast splittable pseudorandom number
 * generators", OOPSLA 2014) applied to the counter
 *     s * 0x9E3779B97F4A7C15 + r * 0xD1B54A32D192ED03 + j      (mod 2^64).
 * The bytes stand in for the paper's incompressible random-fp32 synthetic
 * benchmark (section 4.4). This file holds no checkpoint arithmetic; the same
 * generator is written again as a HIP kernel (synth_dev.hip) and in numpy
 * (synth/splitmix.py), and the three are cross-checked by tests.
 */
#include <stdint.h>
#include <string.h>

static inline uint64_t sm64_mix(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

uint64_t synth_word(uint64_t seed, uint64_t region, uint64_t j)
{
    return sm64_mix(seed * 0x9E3779B97F4A7C15ULL + region * 0xD1B54A32D192ED03ULL + j);
}

/* Fill `nbytes` bytes (any count) starting at byte offset `byte_off` of the
 * region's infinite generator stream. */
void synth_fill_host(uint8_t* dst, uint64_t nbytes, uint64_t seed, uint64_t region,
                     uint64_t byte_off)
{
    const uint64_t base = seed * 0x9E3779B97F4A7C15ULL + region * 0xD1B54A32D192ED03ULL;
    uint64_t pos = byte_off;
    uint64_t end = byte_off + nbytes;
    /* leading partial word */
    while (pos < end && (pos & 7)) {
        uint64_t w = sm64_mix(base + (pos >> 3));
        *dst++ = (uint8_t)(w >> (8 * (pos & 7)));
        ++pos;
    }
    while (pos + 8 <= end) {
        uint64_t w = sm64_mix(base + (pos >> 3));
        memcpy(dst, &w, 8); /* x86-64 is little-endian */
        dst += 8;
        pos += 8;
    }
    while (pos < end) {
        uint64_t w = sm64_mix(base + (pos >> 3));
        *dst++ = (uint8_t)(w >> (8 * (pos & 7)));
        ++pos;
    }
}

/*
 * Page mutations (applied to a shadow copy so that the page differs from the
 * generator's bytes).  For page i of region r under mutation seed ms, the
 * hash stream is h_t = mix(ms*0x9E3779B97F4A7C15 + r*0xD1B54A32D192ED03 +
 * i*0x8CB92BA72F3D8DD7 + t).
 *
 * kind 0 ("words"): k = 1 + (h_0 & 15) distinct 4-byte words of the page,
 *   at positions (start + t*step) mod W for t < k, where W = P/4 (a power of
 *   two), start = (h_0 >> 8) mod W and step = ((h_0 >> 40) | 1) mod W (odd, so
 *   the k positions are distinct); word t is XORed with m_t = 1 + (h_{t+1} mod
 *   (2^32 - 1)), which is never 0, so every chosen word changes.
 * kind 1 ("span"): one 256-byte span at byte offset o = h_0 mod (P - 255);
 *   byte b of the span is XORed with byte (b & 7) of h_{1 + b/8}, except that
 *   byte 0 uses 1 + (h_1 mod 255) so the span always changes.
 */
static inline uint64_t mut_hash(uint64_t ms, uint64_t region, uint64_t page, uint64_t t)
{
    return sm64_mix(ms * 0x9E3779B97F4A7C15ULL + region * 0xD1B54A32D192ED03ULL +
                    page * 0x8CB92BA72F3D8DD7ULL + t);
}

void synth_mutate_page_host(uint8_t* page_bytes, uint64_t page_size, int kind, uint64_t ms,
                            uint64_t region, uint64_t page)
{
    const uint64_t h0 = mut_hash(ms, region, page, 0);
    if (kind == 0) {
        const uint64_t W = page_size / 4;
        const uint64_t k = 1 + (h0 & 15);
        const uint64_t start = (h0 >> 8) % W;
        const uint64_t step = ((h0 >> 40) | 1) % W;
        for (uint64_t t = 0; t < k; ++t) {
            const uint64_t pos = (start + t * step) % W;
            const uint32_t m = (uint32_t)(1 + mut_hash(ms, region, page, t + 1) % 0xFFFFFFFFULL);
            uint32_t w;
            memcpy(&w, page_bytes + 4 * pos, 4);
            w ^= m;
            memcpy(page_bytes + 4 * pos, &w, 4);
        }
    } else {
        const uint64_t o = h0 % (page_size - 255);
        for (uint64_t b = 0; b < 256; ++b) {
            const uint64_t h = mut_hash(ms, region, page, 1 + b / 8);
            uint8_t m = (uint8_t)(h >> (8 * (b & 7)));
            if (b == 0)
                m = (uint8_t)(1 + h % 255);
            page_bytes[o + b] ^= m;
        }
    }
}

/* Mutate the listed pages of a region buffer held in host memory. */
void synth_mutate_host(uint8_t* region_bytes, uint64_t page_size, const int64_t* pages,
                       uint64_t n_pages, int kind, uint64_t ms, uint64_t region)
{
    for (uint64_t i = 0; i < n_pages; ++i)
        synth_mutate_page_host(region_bytes + (uint64_t)pages[i] * page_size, page_size, kind, ms,
                               region, (uint64_t)pages[i]);
}

/*
 * Page source for a streamed-input snapshot: page `page` of region `region`
 * of a scenario, regenerated on the host.  The current bytes are generator
 * output; the shadow's copy equals them, with the mutation rule above applied
 * when the page is in the region's (sorted) list of mutated pages.  Returns 0,
 * or -1 for a page or region out of range.  Generation only: nothing here
 * compares, packs or checksums.
 */
typedef struct {
    uint64_t nbytes;
    uint64_t fill_seed;
    uint64_t fill_region;
    const int64_t* mutated; /* sorted page indices whose shadow differs */
    uint64_t n_mutated;
    int32_t mut_kind;
    int32_t has_shadow;
} synth_src_region;

typedef struct {
    uint64_t page_size;
    uint64_t mut_seed;
    uint64_t n_regions;
    const synth_src_region* regions;
} synth_src;

static int sorted_contains(const int64_t* a, uint64_t n, int64_t v)
{
    uint64_t lo = 0, hi = n;
    while (lo < hi) {
        const uint64_t mid = lo + (hi - lo) / 2;
        if (a[mid] < v)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo < n && a[lo] == v;
}

int synth_page_source(void* user, uint32_t region, uint64_t page, uint8_t* cur, uint8_t* shadow)
{
    const synth_src* s = (const synth_src*)user;
    if (region >= s->n_regions)
        return -1;
    const synth_src_region* r = &s->regions[region];
    const uint64_t P = s->page_size;
    if ((page + 1) * P > r->nbytes)
        return -1;
    synth_fill_host(cur, P, r->fill_seed, r->fill_region, page * P);
    if (shadow) {
        memcpy(shadow, cur, P);
        if (r->has_shadow && sorted_contains(r->mutated, r->n_mutated, (int64_t)page))
            synth_mutate_page_host(shadow, P, r->mut_kind, s->mut_seed, r->fill_region, page);
    }
    return 0;
}
