/* Independent CRC-32C for pinning the oracle: the x86 SSE4.2 crc32
 * instruction computes the raw CRC-32C register update in hardware; the
 * standard init and final XOR (0xFFFFFFFF) are applied around it. */
#include <nmmintrin.h>
#include <stdint.h>
#include <string.h>

uint32_t hw_crc32c(const uint8_t* p, uint64_t n)
{
    uint64_t c = 0xFFFFFFFFu;
    while (n >= 8) {
        uint64_t v;
        memcpy(&v, p, 8);
        c = _mm_crc32_u64(c, v);
        p += 8;
        n -= 8;
    }
    uint32_t c32 = (uint32_t)c;
    while (n--)
        c32 = _mm_crc32_u8(c32, *p++);
    return c32 ^ 0xFFFFFFFFu;
}
