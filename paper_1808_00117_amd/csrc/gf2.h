// GF(2) arithmetic for CRC-32C in the reflected bit order.
//
// A 32-bit value v stands for the polynomial whose x^i coefficient is bit
// (31 - i) of v: this is the bit order of a reflected CRC register, in which
// the register after a message M is (I * x^(8|M|) + M(x) * x^32) mod P(x) for
// the CRC-32C polynomial P (0x1EDC6F41, reflected 0x82F63B78).  With this:
//
//  * multiplying by x is a right shift, folding the x^32 overflow back with
//    the reflected polynomial;
//  * shifting a CRC state through n zero bytes multiplies it by x^(8n);
//  * the CRC of A||B is crc(A) * x^(8|B|) + crc(B) (zero initial value),
//    which lets independent pieces of a page be combined (the "CRC combine"
//    identity; see e.g. the zlib manual's crc32_combine).
#pragma once
#include <stdint.h>

#ifndef CRUM_HD
#define CRUM_HD __host__ __device__ constexpr inline
#endif

namespace crum {

constexpr uint32_t kPolyReflected = 0x82F63B78u;

// a * b mod P
CRUM_HD uint32_t gf2_mulmod(uint32_t a, uint32_t b)
{
    uint32_t p = 0;
    for (int i = 0; i < 32; ++i) {
        if (a & (0x80000000u >> i))  // coefficient of x^i in a
            p ^= b;                  // b currently holds b * x^i
        b = (b & 1u) ? (b >> 1) ^ kPolyReflected : (b >> 1);
    }
    return p;
}

// x^(8n) mod P, by square-and-multiply
CRUM_HD uint32_t gf2_xpow8n(uint64_t n)
{
    uint32_t r = 0x80000000u;     // x^0
    uint32_t base = 0x00800000u;  // x^8
    while (n) {
        if (n & 1u)
            r = gf2_mulmod(r, base);
        base = gf2_mulmod(base, base);
        n >>= 1;
    }
    return r;
}

// CRC state s carried through n zero bytes
CRUM_HD uint32_t gf2_shift(uint32_t s, uint64_t n) { return gf2_mulmod(s, gf2_xpow8n(n)); }

// Constant that turns the zero-initialised CRC of an n-byte message into the
// standard CRC-32C: crc = raw ^ init_fix(n), since the register with initial
// value 0xFFFFFFFF differs from the zero-initialised one by 0xFFFFFFFF*x^(8n),
// and the final XOR adds 0xFFFFFFFF.
CRUM_HD uint32_t crc_init_fix(uint64_t n) { return gf2_shift(0xFFFFFFFFu, n) ^ 0xFFFFFFFFu; }

}  // namespace crum
