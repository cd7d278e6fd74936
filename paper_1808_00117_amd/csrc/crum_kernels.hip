// HIP kernels of the incremental snapshot (gfx950, wave64).
//
// Snapshot pipeline (one launch of each per chunk of the page space, or per
// group of requests of a plan):
//   k_diff    per diff unit (min(page, 4-16 KiB)): OR over 16-byte words of
//             (cur ^ shadow) != 0, read with coalesced 128-bit loads and
//             reduced across the wave by ballot; one flag byte per unit.
//   k_bitmap  per 64 pages: OR of each page's unit flags, then one ballot
//             gives the u64 bitmap word.
//   k_scan    one workgroup: exclusive prefix sum of popcount(word) -> slot of
//             each word's first dirty page, continuing a running total so the
//             page space can be processed in chunks; at the end, per-request
//             dirty counts, image offsets and the capacity check.  A short
//             range also gets the k_list step here.
//   k_list    per word: ballot compaction, lane with bit set writes its page
//             index at prefix + popcount(bits below the lane).
//   k_pack    per dirty page (or piece of up to 64 KiB): copy into the
//             image's page area, optionally into the shadow, and CRC-32C on
//             the way; k_finalize combines the piece CRCs of larger pages.
//   k_header  per request, over one or more workgroups: header, region
//             table, bitmap, CRC array, pads, crcs_crc, meta_crc.
// Restore: k_restore_check (the image's own checks, also over one or more
// workgroups), k_scan, k_list, k_pack (verify), k_scatter.
//
// CRC-32C on the device.  The polynomial arithmetic is in gf2.h.  A wave
// processes a piece of n = 64*T 16-byte words; lane l takes words l, l+64,
// ..., so every load is coalesced.  Lane l keeps a Horner accumulator
//   C_l = sum_t raw(w_{l+64t}) * x^(8*1024*(T-1-t)),
// stepping with "shift by 1024 bytes" (4 table lookups) plus slicing-by-16 of
// the new word (16 lookups).  The piece's raw CRC is
//   sum_l C_l * x^(8*16*(63-l)),
// formed by a 6-level butterfly over lanes (level k shifts the lower half by
// 16*2^k bytes).  Pieces of one page combine the same way with a shift by the
// piece length; the standard CRC adds crc_init_fix(page bytes).  Each table
// lookup may also be done as two lookups into 16-entry nibble tables, which
// never conflict in LDS banks (CrcVariant).
#include "crum_dev.h"
#include "gf2.h"

namespace crum {

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// Pointers into global memory.  Region and staging pointers reach the kernels
// inside structs or after arithmetic the compiler cannot follow, so it would
// use flat instructions; a flat access counts against the LDS/scalar counter
// as well, so every wait for an LDS table lookup would also wait for each
// load and store in flight.  Casting keeps them global.
typedef const u32x4 __attribute__((address_space(1)))* gcv4;
typedef u32x4 __attribute__((address_space(1)))* gv4;
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
typedef const u32x2 __attribute__((address_space(1)))* gcv2;
typedef u32x2 __attribute__((address_space(1)))* gv2;
typedef const uint32_t __attribute__((address_space(1)))* gcu32;
typedef uint32_t __attribute__((address_space(1)))* gu32;

// ------------------------------------------------------------ CRC tables

void build_crc_tables(CrcTables* h)
{
    for (int k = 0; k < 16; ++k) {
        const uint32_t xk = gf2_xpow8n((uint64_t)k + 1);
        for (int b = 0; b < 256; ++b)
            h->t[k][b] = gf2_mulmod((uint32_t)b, xk);
    }
    const uint64_t L[7] = {32, 64, 128, 256, 512, 1024, 4096};
    for (int j = 0; j < 7; ++j) {
        const uint32_t xl = gf2_xpow8n(L[j]);
        for (int i = 0; i < 4; ++i)
            for (int b = 0; b < 256; ++b)
                h->z[j][i][b] = gf2_mulmod((uint32_t)b << (8 * i), xl);
    }
    for (int i = 0; i < 64; ++i)
        h->xp[i] = gf2_xpow8n(1ull << i);
    for (int k = 0; k < 20; ++k) {
        const uint32_t* T = k < 16 ? h->t[k] : h->z[5][k - 16];
        for (int n = 0; n < 16; ++n) {
            h->nib[k][0][n] = T[n];
            h->nib[k][1][n] = T[n << 4];
        }
    }
}

// LDS layout of the header and restore-check kernels (words): the slicing
// tables, then all seven shift levels z[0..6] (44 KiB), as in CrcTables.
constexpr int kSliceWords = 16 * 256;                      // 16 KiB
constexpr int kAllTabWords = kSliceWords + 7 * 4 * 256;    // 44 KiB

// LDS layout of the pack and verify kernels (words): slicing tables, nibble
// tables, shift-by-1-KiB tables; 22.5 KiB.  The butterfly's shift tables
// (used once per piece) are read from global memory: holding nibble versions
// of them in LDS as well (25 KiB) measured no faster.
constexpr int kNibOff = kSliceWords;
constexpr int kZ5Off = kNibOff + 20 * 2 * 16;
constexpr int kPackLdsWords = kZ5Off + 4 * 256;

// Every kernel of this file runs 256-thread workgroups.
constexpr int kBlock = 256;

// Copy WORDS 4-byte words (16-byte aligned at both ends) from global memory
// into LDS: each thread issues all of its 16-byte loads before its first LDS
// store.  A word-per-iteration loop waits for every load in turn, which cost
// each workgroup tens of memory round trips before its first useful step.
template <int WORDS>
__device__ __forceinline__ void stage_words(uint32_t* __restrict__ dst,
                                            const uint32_t* __restrict__ src)
{
    static_assert(WORDS % 4 == 0, "whole 16-byte vectors");
    constexpr int V = WORDS / 4;
    constexpr int N = (V + kBlock - 1) / kBlock;
    const uint4* s = reinterpret_cast<const uint4*>(src);
    uint4* d = reinterpret_cast<uint4*>(dst);
    uint4 v[N];
#pragma unroll
    for (int k = 0; k < N; ++k) {
        const int i = (int)threadIdx.x + kBlock * k;
        if (V % kBlock == 0 || i < V)
            v[k] = s[i];
    }
#pragma unroll
    for (int k = 0; k < N; ++k) {
        const int i = (int)threadIdx.x + kBlock * k;
        if (V % kBlock == 0 || i < V)
            d[i] = v[k];
    }
}

__device__ __forceinline__ void load_pack_tables(uint32_t* lds, const CrcTables* tabs)
{
    stage_words<kSliceWords>(lds, &tabs->t[0][0]);
    stage_words<20 * 2 * 16>(lds + kNibOff, &tabs->nib[0][0][0]);
    stage_words<4 * 256>(lds + kZ5Off, &tabs->z[5][0][0]);
    __syncthreads();
}

// Variants of the per-word CRC step that trade LDS bank conflicts (a byte
// lookup into a 256-entry table) against VALU work (two conflict-free nibble
// lookups): the first NB of the 16 data bytes use byte tables, the rest
// nibble tables; SB selects byte tables for the 4-byte shift by 1 KiB.
template <int V> struct CrcVariant;
template <> struct CrcVariant<0> { static constexpr int NB = 16, SB = 1; };
template <> struct CrcVariant<1> { static constexpr int NB = 8, SB = 0; };
template <> struct CrcVariant<2> { static constexpr int NB = 6, SB = 0; };
template <> struct CrcVariant<3> { static constexpr int NB = 4, SB = 0; };
template <> struct CrcVariant<4> { static constexpr int NB = 0, SB = 0; };
template <> struct CrcVariant<5> { static constexpr int NB = 6, SB = 1; };
constexpr int kCrcVariants = 6;

// raw CRC of one 16-byte word (bytes b0..b15, b0 = low byte of w.x)
__device__ __forceinline__ uint32_t word_crc(const uint32_t* __restrict__ T, uint4 w)
{
    return T[15 * 256 + (w.x & 255u)] ^ T[14 * 256 + ((w.x >> 8) & 255u)] ^
           T[13 * 256 + ((w.x >> 16) & 255u)] ^ T[12 * 256 + (w.x >> 24)] ^
           T[11 * 256 + (w.y & 255u)] ^ T[10 * 256 + ((w.y >> 8) & 255u)] ^
           T[9 * 256 + ((w.y >> 16) & 255u)] ^ T[8 * 256 + (w.y >> 24)] ^
           T[7 * 256 + (w.z & 255u)] ^ T[6 * 256 + ((w.z >> 8) & 255u)] ^
           T[5 * 256 + ((w.z >> 16) & 255u)] ^ T[4 * 256 + (w.z >> 24)] ^
           T[3 * 256 + (w.w & 255u)] ^ T[2 * 256 + ((w.w >> 8) & 255u)] ^
           T[1 * 256 + ((w.w >> 16) & 255u)] ^ T[0 * 256 + (w.w >> 24)];
}

// state carried through 16 zero bytes: the first four slicing tables
__device__ __forceinline__ uint32_t shift16(const uint32_t* __restrict__ T, uint32_t s)
{
    return T[15 * 256 + (s & 255u)] ^ T[14 * 256 + ((s >> 8) & 255u)] ^
           T[13 * 256 + ((s >> 16) & 255u)] ^ T[12 * 256 + (s >> 24)];
}

// state carried through L_j zero bytes (Z points at z[j])
__device__ __forceinline__ uint32_t shiftz(const uint32_t* __restrict__ Z, uint32_t s)
{
    return Z[s & 255u] ^ Z[256 + ((s >> 8) & 255u)] ^ Z[512 + ((s >> 16) & 255u)] ^
           Z[768 + (s >> 24)];
}

// The slicing tables and all shift tables (t and z are contiguous in CrcTables).
__device__ __forceinline__ void load_all_tables(uint32_t* lds, const CrcTables* tabs)
{
    static_assert(offsetof(CrcTables, z) == sizeof(uint32_t) * kSliceWords, "t then z");
    stage_words<kAllTabWords>(lds, &tabs->t[0][0]);
    __syncthreads();
}

// LDS word at byte offset `off` (a multiple of 4)
__device__ __forceinline__ uint32_t lds_at(const uint32_t* __restrict__ L, uint32_t off)
{
    return *reinterpret_cast<const uint32_t*>(reinterpret_cast<const char*>(L) + off);
}

// byte jj of q in the low byte, zeros above (one v_perm_b32)
__device__ __forceinline__ uint32_t byte_of(uint32_t q, int jj)
{
    return __builtin_amdgcn_perm(0u, q, 0x0c0c0c00u | (uint32_t)jj);
}

// a ^ b ^ c in one instruction
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c)
{
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

// XOR of the table entries of the 4 bytes of q, byte jj at table position
// k0 - jj (k0 = 15 - 4*word for data words).  Nibble lookups take their
// addresses from two masked copies of q that hold 4*nibble in every byte, so
// each lookup costs one byte extract; byte lookups shift the extracted byte.
// `nb` (constant after unrolling) is how many of the 4 bytes use byte tables.
__device__ __forceinline__ uint32_t word4_crc(const uint32_t* __restrict__ L, uint32_t q,
                                              int nb, int byte_base0, int byte_step,
                                              int nib_k0, uint32_t r)
{
    const uint32_t lo4 = (q << 2) & 0x3C3C3C3Cu;
    const uint32_t hi4 = (q >> 2) & 0x3C3C3C3Cu;
    uint32_t pend = 0;  // a byte-table value waiting for a partner in xor3
    bool have = false;
#pragma unroll
    for (int jj = 0; jj < 4; ++jj) {
        if (jj < nb) {
            const uint32_t a = byte_of(q, jj) << 2;
            const uint32_t v = lds_at(L, 4u * (uint32_t)(byte_base0 + jj * byte_step) + a);
            if (have) {
                r = xor3(r, pend, v);
                have = false;
            } else {
                pend = v;
                have = true;
            }
        } else {
            const uint32_t base = 4u * (uint32_t)(kNibOff + (nib_k0 - jj) * 32);
            r = xor3(r, lds_at(L, base + byte_of(lo4, jj)), lds_at(L, base + 64u + byte_of(hi4, jj)));
        }
    }
    return have ? r ^ pend : r;
}

// raw CRC of one 16-byte word with the pack layout (as word_crc): byte j of
// the word uses table position 15 - j; the first NB bytes use byte tables
template <int V>
__device__ __forceinline__ uint32_t word_crc_v(const uint32_t* __restrict__ L, uint4 w)
{
    constexpr int NB = CrcVariant<V>::NB;
    const uint32_t v[4] = {w.x, w.y, w.z, w.w};
    uint32_t r = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int nb = NB - 4 * q < 0 ? 0 : (NB - 4 * q > 4 ? 4 : NB - 4 * q);
        r = word4_crc(L, v[q], nb, (15 - 4 * q) * 256, -256, 15 - 4 * q, r);
    }
    return r;
}

// state carried through 1024 zero bytes with the pack layout: byte i of the
// state uses z[5][i], i.e. nibble position 16 + i
template <int V>
__device__ __forceinline__ uint32_t shift1k_v(const uint32_t* __restrict__ L, uint32_t s)
{
    constexpr int SB = CrcVariant<V>::SB;
    if (SB) {
        return lds_at(L, 4u * kZ5Off + ((s << 2) & 0x3FCu)) ^
               lds_at(L, 4u * (kZ5Off + 256) + ((s >> 6) & 0x3FCu)) ^
               lds_at(L, 4u * (kZ5Off + 512) + ((s >> 14) & 0x3FCu)) ^
               lds_at(L, 4u * (kZ5Off + 768) + ((s >> 22) & 0x3FCu));
    }
    // nibble positions 16..19 ascend with the byte index
    const uint32_t lo4 = (s << 2) & 0x3C3C3C3Cu;
    const uint32_t hi4 = (s >> 2) & 0x3C3C3C3Cu;
    uint32_t r = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const uint32_t base = 4u * (uint32_t)(kNibOff + (16 + i) * 32);
        r = xor3(r, lds_at(L, base + byte_of(lo4, i)), lds_at(L, base + 64u + byte_of(hi4, i)));
    }
    return r;
}

// Butterfly over the 64 lanes: afterwards every lane holds sum_l C_l*x^(128(63-l)).
// T: the slicing tables; Z: z[0] of the shift tables (LDS or global memory).
__device__ __forceinline__ uint32_t lane_combine_z(const uint32_t* __restrict__ T,
                                                   const uint32_t* __restrict__ Z, uint32_t s,
                                                   uint32_t lane)
{
#pragma unroll
    for (int lvl = 0; lvl < 6; ++lvl) {
        const uint32_t other = (uint32_t)__shfl_xor((int)s, 1 << lvl);
        const bool upper = (lane >> lvl) & 1u;
        const uint32_t left = upper ? other : s;
        const uint32_t right = upper ? s : other;
        const uint32_t sh = lvl == 0 ? shift16(T, left) : shiftz(Z + (lvl - 1) * 1024, left);
        s = sh ^ right;
    }
    return s;
}

// The butterfly with all tables in LDS in the header layout.
__device__ __forceinline__ uint32_t lane_combine(const uint32_t* __restrict__ lds, uint32_t s,
                                                 uint32_t lane)
{
    return lane_combine_z(lds, lds + kSliceWords, s, lane);
}

// Source of a piece, 1 KiB step by step.  Bit j of `dirty` tells whether
// diff unit j of the piece (units of 2^(ush+10) bytes) differed from the
// shadow; a clean unit's bytes equal the shadow's, so they may be read from
// `alt` (the shadow) instead of `cur`.  That keeps re-reads off the host link
// when the current bytes live in host memory.  alt == nullptr: always cur.
struct PieceSrc {
    gcv4 cur;
    gcv4 alt;
    uint32_t dirty;
    uint32_t ush;
    __device__ __forceinline__ bool is_dirty(uint32_t t) const { return (dirty >> (t >> ush)) & 1u; }
    __device__ __forceinline__ gcv4 at(uint32_t t) const
    {
        return (alt && !is_dirty(t)) ? alt : cur;
    }
};

// lds: the pack layout (kPackLdsWords); V: the CRC step variant.  STORE: 0
// reads only (verify), 1 copies into dst, 2 copies with non-temporal stores
// (the image is streamed out and not read again by the kernels).
template <int LD>
__device__ __forceinline__ u32x4 piece_load(gcv4 p)
{
    if (LD)
        return __builtin_nontemporal_load(p);
    return *p;
}

template <int STORE, int U, int V, int LD = 0>
__device__ __forceinline__ uint32_t piece_steps(const PieceSrc& src, gv4 __restrict__ dst,
                                                gv4 __restrict__ sh, uint32_t* t_io,
                                                uint32_t steps, uint32_t lane,
                                                const uint32_t* __restrict__ lds, uint32_t s)
{
    uint32_t t = *t_io;
    for (; t + U <= steps; t += U) {
        u32x4 w[U];
#pragma unroll
        for (int u = 0; u < U; ++u)
            w[u] = piece_load<LD>(src.at(t + u) + (t + u) * 64 + lane);
        if (STORE) {
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if (STORE == 2)
                    __builtin_nontemporal_store(w[u], dst + (t + u) * 64 + lane);
                else
                    dst[(t + u) * 64 + lane] = w[u];
            }
            if (sh) {
                // clean units already hold these bytes in the shadow
#pragma unroll
                for (int u = 0; u < U; ++u)
                    if (src.is_dirty(t + u))
                        sh[(t + u) * 64 + lane] = w[u];
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
            s = shift1k_v<V>(lds, s) ^
                word_crc_v<V>(lds, make_uint4(w[u].x, w[u].y, w[u].z, w[u].w));
    }
    *t_io = t;
    return s;
}

// As piece_steps, with the loads of the next U steps issued before the
// stores and CRC of the current ones, so a wave keeps page loads in flight
// while it works through its LDS table lookups.
template <int STORE, int U, int V, int LD = 0>
__device__ __forceinline__ uint32_t piece_steps_pf(const PieceSrc& src, gv4 __restrict__ dst,
                                                   gv4 __restrict__ sh, uint32_t* t_io,
                                                   uint32_t steps, uint32_t lane,
                                                   const uint32_t* __restrict__ lds, uint32_t s)
{
    uint32_t t = *t_io;
    if (t + U > steps)
        return s;
    u32x4 w[U];
#pragma unroll
    for (int u = 0; u < U; ++u)
        w[u] = piece_load<LD>(src.at(t + u) + (t + u) * 64 + lane);
    for (;;) {
        const bool more = t + 2 * U <= steps;
        u32x4 nx[U];
        if (more) {
#pragma unroll
            for (int u = 0; u < U; ++u)
                nx[u] = piece_load<LD>(src.at(t + U + u) + (t + U + u) * 64 + lane);
        }
        if (STORE) {
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if (STORE == 2)
                    __builtin_nontemporal_store(w[u], dst + (t + u) * 64 + lane);
                else
                    dst[(t + u) * 64 + lane] = w[u];
            }
            if (sh) {
#pragma unroll
                for (int u = 0; u < U; ++u)
                    if (src.is_dirty(t + u))
                        sh[(t + u) * 64 + lane] = w[u];
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
            s = shift1k_v<V>(lds, s) ^
                word_crc_v<V>(lds, make_uint4(w[u].x, w[u].y, w[u].z, w[u].w));
        t += U;
        if (!more)
            break;
#pragma unroll
        for (int u = 0; u < U; ++u)
            w[u] = nx[u];
    }
    *t_io = t;
    return s;
}

// Raw (zero-initialised) CRC of `steps` KiB, copied to dst (and to the shadow
// sh, dirty units only) when STORE.  DEPTH: 16-byte loads each lane issues
// before it folds them into its CRC; PF: the next DEPTH loads are issued
// before the current ones are folded.  All lanes return the same value.
// gz: z[0] of the shift tables in global memory (the butterfly's shifts).
template <int STORE, int DEPTH, int V, bool PF, int LD = 0>
__device__ __forceinline__ uint32_t wave_piece_crc(const PieceSrc& src, gv4 __restrict__ dst,
                                                   gv4 __restrict__ sh, uint32_t steps,
                                                   uint32_t lane,
                                                   const uint32_t* __restrict__ lds,
                                                   const uint32_t* __restrict__ gz)
{
    uint32_t s = 0;
    uint32_t t = 0;
    if (PF)
        s = piece_steps_pf<STORE, DEPTH, V, LD>(src, dst, sh, &t, steps, lane, lds, s);
    else
        s = piece_steps<STORE, DEPTH, V, LD>(src, dst, sh, &t, steps, lane, lds, s);
    if (DEPTH > 4)
        s = piece_steps<STORE, 4, V, LD>(src, dst, sh, &t, steps, lane, lds, s);
    s = piece_steps<STORE, 1, V, LD>(src, dst, sh, &t, steps, lane, lds, s);
    return lane_combine_z(lds, gz, s, lane);
}

// ------------------------------------------------------------ region lookup

// Last region whose field (3 first_page, 4 first_unit) is <= key.
template <int FIELD>
__device__ __forceinline__ uint32_t find_region(const DevRegion* __restrict__ regs, uint32_t n,
                                                uint64_t key)
{
    uint32_t lo = 0, hi = n;
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        const uint64_t v = FIELD == 3 ? regs[mid].first_page : regs[mid].first_unit;
        if (v <= key)
            lo = mid;
        else
            hi = mid;
    }
    return lo;
}

// ------------------------------------------------------------ k_diff

// OR over the lane's LOADS 16-byte words of (a ^ b), a and b already offset
// by the lane; loads are 1 KiB apart so each one is coalesced across the wave.
// NT marks the loads non-temporal: the streamed bytes are not kept in the
// caches, which stay available to co-running work.
template <int LOADS, bool NT>
__device__ __forceinline__ uint32_t xor_or(gcv4 __restrict__ a, gcv4 __restrict__ b)
{
    u32x4 va[LOADS], vb[LOADS];
#pragma unroll
    for (int j = 0; j < LOADS; ++j) {
        if (NT) {
            va[j] = __builtin_nontemporal_load(a + j * 64);
            vb[j] = __builtin_nontemporal_load(b + j * 64);
        } else {
            va[j] = a[j * 64];
            vb[j] = b[j * 64];
        }
    }
    u32x4 x = va[0] ^ vb[0];
#pragma unroll
    for (int j = 1; j < LOADS; ++j)
        x |= va[j] ^ vb[j];
    return x.x | x.y | x.z | x.w;
}

// G consecutive 4 KiB units read as one span of G * 4 KiB: 4G loads per
// array in flight per lane, x[k] = OR of (a ^ b) over unit k's four loads.
template <int G, bool NT>
__device__ __forceinline__ void xor_or_group(gcv4 __restrict__ a, gcv4 __restrict__ b,
                                             uint32_t* x)
{
    u32x4 va[4 * G], vb[4 * G];
#pragma unroll
    for (int j = 0; j < 4 * G; ++j) {
        if (NT) {
            va[j] = __builtin_nontemporal_load(a + j * 64);
            vb[j] = __builtin_nontemporal_load(b + j * 64);
        } else {
            va[j] = a[j * 64];
            vb[j] = b[j * 64];
        }
    }
#pragma unroll
    for (int k = 0; k < G; ++k) {
        u32x4 o = va[4 * k] ^ vb[4 * k];
#pragma unroll
        for (int j = 1; j < 4; ++j)
            o |= va[4 * k + j] ^ vb[4 * k + j];
        x[k] = o.x | o.y | o.z | o.w;
    }
}

// The flag of unit u (one wave); the region lookup is cached in r, r_lo, r_hi.
template <bool NT>
__device__ __forceinline__ void diff_unit(const DevRegion* __restrict__ regs, uint32_t n_regs,
                                          uint64_t u, uint8_t* __restrict__ unit_flags,
                                          const uint64_t* __restrict__ cand, uint32_t lane,
                                          uint32_t& r, uint64_t& r_lo, uint64_t& r_hi)
{
    if (u < r_lo || u >= r_hi) {
        r = find_region<4>(regs, n_regs, u);
        r_lo = regs[r].first_unit;
        r_hi = r_lo + (regs[r].len >> regs[r].unit_shift);
    }
    const DevRegion& R = regs[r];
    const uint32_t us = R.unit_shift;
    if (cand && R.shadow != nullptr) {
        const uint64_t g = R.first_page + ((u - R.first_unit) >> (R.page_shift - us));
        if (!((cand[g >> 6] >> (g & 63)) & 1ull)) {
            if (lane == 0)
                unit_flags[u] = 0;
            return;
        }
    }
    uint32_t x = 1;
    if (R.shadow != nullptr) {
        const uint64_t off = (u - R.first_unit) << us;
        const gcv4 a = (gcv4)(R.cur + off) + lane;
        const gcv4 b = (gcv4)(R.shadow + off) + lane;
        x = us == 12 ? xor_or<4, NT>(a, b) : us == 13 ? xor_or<8, NT>(a, b)
                                                      : xor_or<16, NT>(a, b);
    }
    const uint64_t m = __ballot(x != 0);
    if (lane == 0)
        unit_flags[u] = m != 0;
}

// Diff of global units [u0, u1); unit_flags[u] = 1 when any byte of the unit
// differs from the shadow (or the region has none).  G = 1: one wave per
// unit.  G = 2 or 4: one wave per G consecutive units (from u0); G 4 KiB
// units of one region with a shadow, all candidates when a candidate set is
// given, are read as one span of G * 4 KiB, so a wave keeps 4G loads per
// array in flight; other groups are done one unit at a time.
// prio 1..3 raises the waves' issue priority on their compute unit above
// that of co-running kernels' waves (0 leaves it at the default).
// cand (may be null): a bitmap over global pages from host write tracking;
// a page whose bit is clear is known to equal its shadow, so its units are
// flagged clean without reading either copy.
// stamp (may be null): stamp[0] gets the constant-rate wall clock when
// workgroup 0 starts (the first one dispatched), stamp[1] the largest clock
// at which a workgroup ends.  stamp[1] needs no reset between launches: a
// later launch's clocks exceed every earlier one's.
template <bool NT, int G>
__global__ __launch_bounds__(256) void k_diff(const DevRegion* __restrict__ regs,
                                              uint32_t n_regs, uint64_t u0, uint64_t u1,
                                              uint8_t* __restrict__ unit_flags, uint32_t prio,
                                              const uint64_t* __restrict__ cand,
                                              uint64_t* __restrict__ stamp)
{
    if (stamp && blockIdx.x == 0 && threadIdx.x == 0)
        stamp[0] = wall_clock64();
    if (prio == 1)
        __builtin_amdgcn_s_setprio(1);
    else if (prio == 2)
        __builtin_amdgcn_s_setprio(2);
    else if (prio >= 3)
        __builtin_amdgcn_s_setprio(3);
    const uint32_t lane = threadIdx.x & 63u;
    const uint64_t wave =
        (uint64_t)blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint64_t n_waves = (uint64_t)gridDim.x * 4;
    uint32_t r = 0;
    uint64_t r_lo = 1, r_hi = 0;
    if (G == 1) {
        for (uint64_t u = u0 + wave; u < u1; u += n_waves)
            diff_unit<NT>(regs, n_regs, u, unit_flags, cand, lane, r, r_lo, r_hi);
    } else {
        for (uint64_t base = u0 + G * wave; base < u1; base += G * n_waves) {
            const uint64_t end = base + G < u1 ? base + G : u1;
            if (base < r_lo || base >= r_hi) {
                r = find_region<4>(regs, n_regs, base);
                r_lo = regs[r].first_unit;
                r_hi = r_lo + (regs[r].len >> regs[r].unit_shift);
            }
            const DevRegion& R = regs[r];
            bool fused = end == base + G && base + G <= r_hi && R.unit_shift == 12 &&
                         R.shadow != nullptr;
            if (fused && cand) {
                const uint32_t sh = R.page_shift - 12;
                for (uint64_t u = base; u < end; ++u) {
                    const uint64_t g = R.first_page + ((u - R.first_unit) >> sh);
                    fused = fused && ((cand[g >> 6] >> (g & 63)) & 1ull);
                }
            }
            if (fused) {
                const uint64_t off = (base - R.first_unit) << 12;
                uint32_t x[G];
                xor_or_group<G, NT>((gcv4)(R.cur + off) + lane, (gcv4)(R.shadow + off) + lane,
                                    x);
#pragma unroll
                for (int k = 0; k < G; ++k) {
                    const uint64_t m = __ballot(x[k] != 0);
                    if (lane == 0)
                        unit_flags[base + k] = m != 0;
                }
            } else {
                for (uint64_t u = base; u < end; ++u)
                    diff_unit<NT>(regs, n_regs, u, unit_flags, cand, lane, r, r_lo, r_hi);
            }
        }
    }
    if (stamp) {
        __syncthreads();
        if (threadIdx.x == 0)
            atomicMax(reinterpret_cast<unsigned long long*>(stamp + 1),
                      (unsigned long long)wall_clock64());
    }
}

hipError_t launch_diff(const DevRegion* regs, uint32_t n_regs, uint64_t u0, uint64_t u1,
                       uint8_t* unit_flags, int blocks, int nontemporal, int prio,
                       hipStream_t s, const uint64_t* cand, uint64_t* stamp, int group)
{
    if (u1 <= u0)
        return hipSuccess;
    if (group != 2 && group != 4)
        group = 1;
    const uint64_t need = ((u1 - u0 + group - 1) / group + 3) / 4;
    const uint64_t nb = need < (uint64_t)blocks ? need : (uint64_t)blocks;
#define CRUM_DIFF(NTV, GV)                                                                   \
    hipLaunchKernelGGL((k_diff<NTV, GV>), dim3((unsigned)nb), dim3(256), 0, s, regs, n_regs, \
                       u0, u1, unit_flags, (uint32_t)prio, cand, stamp)
    if (nontemporal) {
        if (group == 4)
            CRUM_DIFF(true, 4);
        else if (group == 2)
            CRUM_DIFF(true, 2);
        else
            CRUM_DIFF(true, 1);
    } else {
        if (group == 4)
            CRUM_DIFF(false, 4);
        else if (group == 2)
            CRUM_DIFF(false, 2);
        else
            CRUM_DIFF(false, 1);
    }
#undef CRUM_DIFF
    return hipGetLastError();
}

// ------------------------------------------------------------ k_bitmap

// One wave per bitmap word in [w0, w1): lane l owns global page 64w + l, ORs
// its unit flags, and a ballot forms the word.
__global__ __launch_bounds__(256) void k_bitmap(const DevRegion* __restrict__ regs,
                                                uint32_t n_regs, uint64_t w0, uint64_t w1,
                                                const uint8_t* __restrict__ unit_flags,
                                                uint64_t* __restrict__ bitmap)
{
    const uint32_t lane = threadIdx.x & 63u;
    const uint64_t w =
        w0 + (uint64_t)blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (w >= w1)
        return;
    const uint64_t g = w * 64 + lane;
    const uint32_t r = find_region<3>(regs, n_regs, g);
    const DevRegion& R = regs[r];
    bool dirty = false;
    const uint64_t np = R.len >> R.page_shift;
    if (g >= R.first_page && g - R.first_page < np) {
        const uint64_t pi = g - R.first_page;
        const uint32_t upp_shift = R.page_shift - R.unit_shift;
        const uint8_t* f = unit_flags + R.first_unit + (pi << upp_shift);
        uint32_t acc = 0;
        for (uint32_t i = 0; i < (1u << upp_shift); ++i)
            acc |= f[i];
        dirty = acc != 0;
    }
    const uint64_t m = __ballot(dirty);
    if (lane == 0)
        bitmap[w] = m;
}

hipError_t launch_bitmap(const DevRegion* regs, uint32_t n_regs, uint64_t w0, uint64_t w1,
                         const uint8_t* unit_flags, uint64_t* bitmap, hipStream_t s)
{
    if (w1 <= w0)
        return hipSuccess;
    hipLaunchKernelGGL(k_bitmap, dim3((unsigned)((w1 - w0 + 3) / 4)), dim3(256), 0, s, regs,
                       n_regs, w0, w1, unit_flags, bitmap);
    return hipGetLastError();
}

// ------------------------------------------------------------ k_scan

// A range of at most this many bitmap words gets its slot list from k_scan
// itself (the k_list work, from LDS, with no second launch).  One workgroup
// writes the list at about 5 ns a word, so past this a separate k_list (about
// 5 us plus a launch gap) is faster.
constexpr uint64_t kScanListWords = 512;

__global__ __launch_bounds__(1024) void k_scan(const uint64_t* __restrict__ bitmap, uint64_t w0,
                                               uint64_t w1, uint64_t n_words_total,
                                               uint32_t* __restrict__ prefix,
                                               uint64_t* __restrict__ bounds_out, int final,
                                               const DevRequest* __restrict__ reqs, uint32_t q0,
                                               uint32_t q1, DevReqOut* __restrict__ out,
                                               DevGlobal* __restrict__ glob, uint64_t capacity,
                                               int restore_mode, uint32_t* __restrict__ list)
{
    constexpr int V = 4;  // words per thread per pass
    static_assert(kScanListWords <= 1024 * V, "a fused list range takes one pass");
    __shared__ uint32_t wave_tot[16];
    __shared__ uint64_t s_words[kScanListWords];  // with `list`: the words and their
    __shared__ uint32_t s_pre[kScanListWords];    // prefixes, for the list below
    const uint32_t tid = threadIdx.x, lane = tid & 63u, wv = tid >> 6;
    uint32_t carry = (uint32_t)glob->running;
    for (uint64_t base = w0; base < w1; base += 1024 * V) {
        uint32_t c[V];
        uint32_t local = 0;
#pragma unroll
        for (int v = 0; v < V; ++v) {
            const uint64_t w = base + (uint64_t)tid * V + v;
            const uint64_t word = w < w1 ? bitmap[w] : 0ull;
            if (list && w < w1)
                s_words[w - w0] = word;
            c[v] = (uint32_t)__popcll(word);
            local += c[v];
        }
        uint32_t incl = local;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const uint32_t y = (uint32_t)__shfl_up((int)incl, d);
            if (lane >= (uint32_t)d)
                incl += y;
        }
        if (lane == 63)
            wave_tot[wv] = incl;
        __syncthreads();
        uint32_t woff = 0, blk = 0;
        for (uint32_t i = 0; i < 16; ++i) {
            if (i < wv)
                woff += wave_tot[i];
            blk += wave_tot[i];
        }
        uint32_t excl = carry + woff + incl - local;
#pragma unroll
        for (int v = 0; v < V; ++v) {
            const uint64_t w = base + (uint64_t)tid * V + v;
            if (w < w1) {
                prefix[w] = excl;
                if (list)
                    s_pre[w - w0] = excl;
            }
            excl += c[v];
        }
        carry += blk;
        __syncthreads();
    }
    if (list) {
        // the k_list step: wave wv takes words 4wv .. 4wv + 3, then 64 further
        // on, ... (four LDS reads in flight); the lane of each set bit writes
        // its page at the word's prefix plus the set bits below it
        const uint64_t n = w1 - w0;
        for (uint64_t i0 = 4 * wv; i0 < n; i0 += 64) {
            uint64_t m[4];
            uint32_t pre[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                m[u] = i0 + u < n ? s_words[i0 + u] : 0ull;
                pre[u] = i0 + u < n ? s_pre[i0 + u] : 0u;
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const uint32_t below = __builtin_amdgcn_mbcnt_hi(
                    (uint32_t)(m[u] >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m[u], 0u));
                if ((m[u] >> lane) & 1u)
                    list[pre[u] + below] = (uint32_t)((w0 + i0 + u) * 64 + lane);
            }
        }
    }
    __threadfence_block();
    __syncthreads();
    if (tid != 0)
        return;
    glob->running = carry;
    if (bounds_out)
        *bounds_out = carry;
    if (!final)
        return;
    // results of requests [q0, q1); their images follow glob->img_next (4 KiB aligned)
    uint64_t img = glob->img_next, used = glob->staging_used;
    const bool full = glob->code != 0;
    for (uint32_t q = q0; q < q1; ++q) {
        const DevRequest& Q = reqs[q];
        // every word of these requests lies in [.., w1): a prefix at or past
        // w1 is the running total, not a (not yet scanned) later word
        const uint64_t a = Q.first_word, b = Q.first_word + Q.n_words;
        const uint64_t p0 = a < w1 ? prefix[a] : carry;
        const uint64_t p1 = b < w1 ? prefix[b] : carry;
        const uint64_t D = p1 - p0;
        DevReqOut& O = out[q];
        O.n_dirty = D;
        O.total_pages = Q.n_pages;
        O.slot_base = p0;
        O.acc[0] = O.acc[1] = O.acc[2] = O.acc[3] = 0;
        if (!restore_mode) {
            const uint64_t ib = Q.data_off + (D << Q.page_shift) + ((4 * D + 7) & ~7ull);
            O.code = 0;
            O.first_bad = 0;
            O.image_bytes = ib;
            O.img_base = img;
            used = img + ib;
            img = (used + 4095) & ~4095ull;
        }
    }
    glob->total_dirty = carry;
    if (!restore_mode) {
        if (full || used > capacity) {
            // the group does not fit: no request of it (or of a later group) is packed
            glob->code = -2;  // CRUM_ENOSPC
            for (uint32_t q = q0; q < q1; ++q)
                out[q].code = -2;
        } else {
            glob->staging_used = used;
            glob->img_next = img;
        }
    }
}

hipError_t launch_scan(const uint64_t* bitmap, uint64_t w0, uint64_t w1, uint64_t n_words_total,
                       uint32_t* prefix, uint64_t* bounds_out, int final, const DevRequest* reqs,
                       uint32_t q0, uint32_t q1, DevReqOut* out, DevGlobal* glob,
                       uint64_t capacity, int restore_mode, uint32_t* list, hipStream_t s)
{
    const bool fused = list && w1 - w0 <= kScanListWords;
    hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, s, bitmap, w0, w1, n_words_total, prefix,
                       bounds_out, final, reqs, q0, q1, out, glob, capacity, restore_mode,
                       fused ? list : nullptr);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess && list && !fused)
        e = launch_list(bitmap, prefix, w0, w1, list, s);
    return e;
}

// ------------------------------------------------------------ k_list

// Ballot compaction: the lane of each set bit writes its page index at the
// word's prefix plus the number of set bits below the lane.
__global__ __launch_bounds__(256) void k_list(const uint64_t* __restrict__ bitmap,
                                              const uint32_t* __restrict__ prefix, uint64_t w0,
                                              uint64_t w1, uint32_t* __restrict__ list)
{
    const uint32_t lane = threadIdx.x & 63u;
    const uint64_t w =
        w0 + (uint64_t)blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (w >= w1)
        return;
    const uint64_t m = bitmap[w];
    if (m == 0)
        return;
    const uint32_t below = __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                                     __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
    if ((m >> lane) & 1u)
        list[prefix[w] + below] = (uint32_t)(w * 64 + lane);
}

hipError_t launch_list(const uint64_t* bitmap, const uint32_t* prefix, uint64_t w0, uint64_t w1,
                       uint32_t* list, hipStream_t s)
{
    if (w1 <= w0)
        return hipSuccess;
    hipLaunchKernelGGL(k_list, dim3((unsigned)((w1 - w0 + 3) / 4)), dim3(256), 0, s, bitmap,
                       prefix, w0, w1, list);
    return hipGetLastError();
}

// ------------------------------------------------------------ k_pack / verify

__device__ __forceinline__ void slot_range(const SlotRange& sr, uint64_t* lo, uint64_t* hi)
{
    if (sr.bounds) {
        *lo = sr.chunk ? sr.bounds[sr.chunk - 1] : 0;
        *hi = sr.bounds[sr.chunk];
    } else {
        *lo = sr.lo;
        *hi = sr.hi;
    }
}

// Work item = (slot, piece); pieces per slot = 2^np_shift for the launch.
// Pack: copy the dirty page into the image's page area (and the shadow) and
// write its CRC to crc_out[slot].  Verify: recompute the CRC of a packed page
// of the image and compare with the image's CRC array.
template <int MODE, int DEPTH, int V>
__global__ __launch_bounds__(256) void k_pack(const DevRegion* __restrict__ regs, uint32_t n_regs,
                                              const DevRequest* __restrict__ reqs,
                                              const DevReqOut* __restrict__ out,
                                              const uint32_t* __restrict__ list, SlotRange sr,
                                              uint32_t np_shift, uint32_t piece_shift,
                                              const uint8_t* __restrict__ unit_flags,
                                              uint8_t* __restrict__ staging,
                                              uint32_t* __restrict__ crc_out,
                                              uint32_t* __restrict__ partials,
                                              const CrcTables* __restrict__ tabs,
                                              DevGlobal* __restrict__ glob, uint32_t nt_store)
{
    __shared__ __attribute__((aligned(16))) uint32_t lds[kPackLdsWords];
    if (MODE == kModeVerify && glob->fmt_bad)
        return;
    uint64_t slot0, slot1;
    slot_range(sr, &slot0, &slot1);
    const uint64_t n_items = (slot1 - slot0) << np_shift;
    // a grid sized for the most slots the launch could get: workgroups past
    // the items leave before staging their tables
    if ((uint64_t)blockIdx.x * 4 >= n_items)
        return;
    load_pack_tables(lds, tabs);
    const uint32_t* gz = &tabs->z[0][0][0];
    const uint32_t lane = threadIdx.x & 63u;
    const uint64_t wave =
        (uint64_t)blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint64_t n_waves = (uint64_t)gridDim.x * 4;
    uint32_t r = 0;
    uint64_t r_lo = 1, r_hi = 0;
    for (uint64_t item = wave; item < n_items; item += n_waves) {
        const uint64_t k = slot0 + (item >> np_shift);
        const uint32_t piece = (uint32_t)(item & ((1ull << np_shift) - 1));
        const uint64_t g = list[k];
        if (g < r_lo || g >= r_hi) {
            r = find_region<3>(regs, n_regs, g);
            r_lo = regs[r].first_page;
            r_hi = r_lo + (regs[r].len >> regs[r].page_shift);
        }
        const DevRegion& R = regs[r];
        if (g < r_lo || g >= r_hi)
            continue;  // only reachable for a corrupt restore bitmap (gated above)
        const DevRequest& Q = reqs[R.req];
        const DevReqOut& O = out[R.req];
        if (MODE == kModePack && O.code != 0)
            continue;  // the request's image did not fit: nothing is written
        const uint32_t ps = R.page_shift;
        const uint32_t pb_shift = ps < piece_shift ? ps : piece_shift;
        if (piece >= (1u << (ps - pb_shift)))
            continue;
        const uint64_t local = k - O.slot_base;
        const uint64_t page_off = (g - R.first_page) << ps;
        const uint64_t piece_off = (uint64_t)piece << pb_shift;
        uint8_t* img = staging + O.img_base;
        uint8_t* slot_ptr = img + Q.data_off + (local << ps) + piece_off;
        const uint32_t steps = 1u << (pb_shift - 10);
        uint32_t raw;
        if (MODE == kModePack) {
            PieceSrc src{(gcv4)(R.cur + page_off + piece_off), nullptr,
                         ~0u, 0};
            if (unit_flags && R.shadow) {
                // the piece's diff units: clean ones are read from the shadow
                const uint32_t us = R.unit_shift;
                const uint64_t u0 = R.first_unit + ((page_off + piece_off) >> us);
                const uint32_t n_u = pb_shift > us ? 1u << (pb_shift - us) : 1u;
                uint32_t m = 0;
                for (uint32_t j = 0; j < n_u; ++j)
                    m |= (unit_flags[u0 + j] ? 1u : 0u) << j;
                src.alt = (gcv4)(R.shadow + page_off + piece_off);
                src.dirty = m;
                src.ush = us - 10;
            }
            gv4 sh = ((R.flags & 1u) && R.shadow)
                            ? (gv4)(R.shadow + page_off + piece_off)
                            : nullptr;
            if (nt_store & 4u)
                raw = (nt_store & 1u) ? wave_piece_crc<2, DEPTH, V, false, 1>(
                                            src, (gv4)slot_ptr, sh, steps, lane, lds, gz)
                                      : wave_piece_crc<1, DEPTH, V, false, 1>(
                                            src, (gv4)slot_ptr, sh, steps, lane, lds, gz);
            else if (nt_store & 2u)
                raw = (nt_store & 1u) ? wave_piece_crc<2, DEPTH, V, true>(
                                            src, (gv4)slot_ptr, sh, steps, lane, lds, gz)
                                      : wave_piece_crc<1, DEPTH, V, true>(
                                            src, (gv4)slot_ptr, sh, steps, lane, lds, gz);
            else
                raw = (nt_store & 1u) ? wave_piece_crc<2, DEPTH, V, false>(
                                            src, (gv4)slot_ptr, sh, steps, lane, lds, gz)
                                      : wave_piece_crc<1, DEPTH, V, false>(
                                            src, (gv4)slot_ptr, sh, steps, lane, lds, gz);
        } else {
            const PieceSrc src{(gcv4)slot_ptr, nullptr, ~0u, 0};
            raw = (nt_store & 4u)
                      ? wave_piece_crc<0, DEPTH, V, false, 1>(src, nullptr, nullptr, steps, lane,
                                                              lds, gz)
                  : (nt_store & 2u)
                      ? wave_piece_crc<0, DEPTH, V, true>(src, nullptr, nullptr, steps, lane, lds,
                                                          gz)
                      : wave_piece_crc<0, DEPTH, V, false>(src, nullptr, nullptr, steps, lane,
                                                           lds, gz);
        }
        if (lane != 0)
            continue;
        if (ps > pb_shift) {
            partials[item] = raw;
            continue;
        }
        const uint32_t crc = raw ^ Q.init_fix;
        if (MODE == kModePack) {
            crc_out[k] = crc;
        } else {
            const uint32_t* img_crc =
                reinterpret_cast<const uint32_t*>(img + Q.data_off + (O.n_dirty << ps));
            if (crc != img_crc[local])
                atomicMin(&glob->crc_bad, (uint32_t)local);
        }
    }
}

template <int MODE, int DEPTH, int V>
static void launch_pack_one(dim3 grid, hipStream_t s, const DevRegion* regs, uint32_t n_regs,
                            const DevRequest* reqs, const DevReqOut* out, const uint32_t* list,
                            SlotRange range, uint32_t np_shift, uint32_t piece_shift,
                            const uint8_t* unit_flags, uint8_t* staging, uint32_t* crc_out,
                            uint32_t* partials, const CrcTables* tabs, DevGlobal* glob,
                            uint32_t nt_store)
{
    hipLaunchKernelGGL((k_pack<MODE, DEPTH, V>), grid, dim3(256), 0, s, regs, n_regs, reqs, out,
                       list, range, np_shift, piece_shift, unit_flags, staging, crc_out,
                       partials, tabs, glob, nt_store);
}

template <int MODE, int DEPTH>
static void launch_pack_depth(int variant, dim3 grid, hipStream_t s, const DevRegion* regs,
                              uint32_t n_regs, const DevRequest* reqs, const DevReqOut* out,
                              const uint32_t* list, SlotRange range, uint32_t np_shift,
                              uint32_t piece_shift, const uint8_t* unit_flags, uint8_t* staging,
                              uint32_t* crc_out, uint32_t* partials, const CrcTables* tabs,
                              DevGlobal* glob, uint32_t nt_store)
{
#define CRUM_PACK_V(v)                                                                        \
    launch_pack_one<MODE, DEPTH, v>(grid, s, regs, n_regs, reqs, out, list, range, np_shift, \
                                    piece_shift, unit_flags, staging, crc_out, partials, tabs, \
                                    glob, nt_store)
    switch (variant) {
    case 0: CRUM_PACK_V(0); break;
    case 1: CRUM_PACK_V(1); break;
    case 2: CRUM_PACK_V(2); break;
    case 3: CRUM_PACK_V(3); break;
    case 4: CRUM_PACK_V(4); break;
    default: CRUM_PACK_V(5); break;
    }
#undef CRUM_PACK_V
}

template <int MODE>
static void launch_pack_mode(dim3 grid, int depth, int variant, hipStream_t s,
                             const DevRegion* regs, uint32_t n_regs, const DevRequest* reqs,
                             const DevReqOut* out, const uint32_t* list, SlotRange range,
                             uint32_t np_shift, uint32_t piece_shift, const uint8_t* unit_flags,
                             uint8_t* staging, uint32_t* crc_out, uint32_t* partials,
                             const CrcTables* tabs, DevGlobal* glob, uint32_t nt_store)
{
    if (depth == 16)
        launch_pack_depth<MODE, 16>(variant, grid, s, regs, n_regs, reqs, out, list, range,
                                    np_shift, piece_shift, unit_flags, staging, crc_out,
                                    partials, tabs, glob, nt_store);
    else if (depth == 8)
        launch_pack_depth<MODE, 8>(variant, grid, s, regs, n_regs, reqs, out, list, range,
                                   np_shift, piece_shift, unit_flags, staging, crc_out, partials,
                                   tabs, glob, nt_store);
    else
        launch_pack_depth<MODE, 4>(variant, grid, s, regs, n_regs, reqs, out, list, range,
                                   np_shift, piece_shift, unit_flags, staging, crc_out, partials,
                                   tabs, glob, nt_store);
}

hipError_t launch_pack(int mode, const DevRegion* regs, uint32_t n_regs, const DevRequest* reqs,
                       const DevReqOut* out, const uint32_t* list, SlotRange range,
                       uint32_t np_shift, uint32_t piece_shift, const uint8_t* unit_flags,
                       uint8_t* staging, uint32_t* crc_out, uint32_t* partials,
                       const CrcTables* tabs, DevGlobal* glob, int blocks, int depth,
                       int variant, hipStream_t s, int nt_store)
{
    const uint64_t max_items = range.max_slots << np_shift;
    if (max_items == 0)
        return hipSuccess;
    if (piece_shift < kPieceShiftMin || piece_shift > kPieceShift)
        return hipErrorInvalidValue;
    const uint64_t need = (max_items + 3) / 4;
    const uint64_t nb = need < (uint64_t)blocks ? need : (uint64_t)blocks;
    const dim3 grid((unsigned)nb);
    if (variant == kCrcVariantAuto)
        variant = mode == kModePack ? 0 : 3;
    if (mode == kModePack)
        launch_pack_mode<kModePack>(grid, depth, variant, s, regs, n_regs, reqs, out, list,
                                    range, np_shift, piece_shift, unit_flags, staging, crc_out,
                                    partials, tabs, glob, (uint32_t)nt_store);
    else
        launch_pack_mode<kModeVerify>(grid, depth, variant, s, regs, n_regs, reqs, out, list,
                                      range, np_shift, piece_shift, nullptr, staging, crc_out,
                                      partials, tabs, glob, (uint32_t)nt_store & 6u);
    return hipGetLastError();
}

// One thread per slot: combine the slot's piece CRCs (pages above 64 KiB).
// partials are indexed by the item of the matching pack launch.
template <int MODE>
__global__ __launch_bounds__(256) void k_finalize(const DevRegion* __restrict__ regs,
                                                  uint32_t n_regs,
                                                  const DevRequest* __restrict__ reqs,
                                                  const DevReqOut* __restrict__ out,
                                                  const uint32_t* __restrict__ list,
                                                  SlotRange sr, uint32_t np_shift,
                                                  uint32_t piece_shift,
                                                  const uint32_t* __restrict__ partials,
                                                  uint32_t* __restrict__ crc_out,
                                                  uint8_t* __restrict__ staging,
                                                  DevGlobal* __restrict__ glob,
                                                  const CrcTables* __restrict__ tabs)
{
    if (MODE == kModeVerify && glob->fmt_bad)
        return;
    uint64_t slot0, slot1;
    slot_range(sr, &slot0, &slot1);
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= slot1 - slot0)
        return;
    const uint64_t k = slot0 + i;
    const uint64_t g = list[k];
    const DevRegion& R = regs[find_region<3>(regs, n_regs, g)];
    if (g < R.first_page || g - R.first_page >= (R.len >> R.page_shift))
        return;
    const uint32_t ps = R.page_shift;
    if (ps <= piece_shift)
        return;
    const DevRequest& Q = reqs[R.req];
    const DevReqOut& O = out[R.req];
    if (MODE == kModePack && O.code != 0)
        return;
    const uint32_t np = 1u << (ps - piece_shift);
    const uint32_t K = tabs->xp[piece_shift];  // x^(8 * piece bytes)
    uint32_t s = 0;
    for (uint32_t j = 0; j < np; ++j)
        s = gf2_mulmod(s, K) ^ partials[(i << np_shift) + j];
    const uint32_t crc = s ^ Q.init_fix;
    if (MODE == kModePack) {
        crc_out[k] = crc;
    } else {
        const uint64_t local = k - O.slot_base;
        const uint32_t* img_crc = reinterpret_cast<const uint32_t*>(
            staging + O.img_base + Q.data_off + (O.n_dirty << ps));
        if (crc != img_crc[local])
            atomicMin(&glob->crc_bad, (uint32_t)local);
    }
}

hipError_t launch_finalize(int mode, const DevRegion* regs, uint32_t n_regs,
                           const DevRequest* reqs, const DevReqOut* out, const uint32_t* list,
                           SlotRange range, uint32_t np_shift, uint32_t piece_shift,
                           const uint32_t* partials, uint32_t* crc_out, uint8_t* staging,
                           DevGlobal* glob, const CrcTables* tabs, hipStream_t s)
{
    if (range.max_slots == 0 || np_shift == 0)
        return hipSuccess;
    const unsigned nb = (unsigned)((range.max_slots + 255) / 256);
    if (mode == kModePack)
        hipLaunchKernelGGL(k_finalize<kModePack>, dim3(nb), dim3(256), 0, s, regs, n_regs, reqs,
                           out, list, range, np_shift, piece_shift, partials, crc_out, staging,
                           glob, tabs);
    else
        hipLaunchKernelGGL(k_finalize<kModeVerify>, dim3(nb), dim3(256), 0, s, regs, n_regs,
                           reqs, out, list, range, np_shift, piece_shift, partials, crc_out,
                           staging, glob, tabs);
    return hipGetLastError();
}

// ------------------------------------------------------------ block CRC

// x^(8n) mod P from the table xp[i] = x^(8 * 2^i): the product of the
// entries for the set bits of n, reduced across the wave.  Every lane returns
// it; all lanes of the wave must call.
__device__ __forceinline__ uint32_t xpow8n_wave(uint64_t n, const uint32_t* __restrict__ xp,
                                               uint32_t lane)
{
    uint32_t v = ((n >> lane) & 1u) ? xp[lane] : 0x80000000u;  // x^0 when the bit is clear
#pragma unroll
    for (int d = 1; d < 64; d <<= 1)
        v = gf2_mulmod(v, (uint32_t)__shfl_xor((int)v, d));
    return v;
}

// x^(8 n_w) for one n per wave of a 256-thread workgroup, the four computed
// in parallel, into pw[w]; the caller synchronises before reading them.
__device__ __forceinline__ void wave_powers(uint64_t n0, uint64_t n1, uint64_t n2, uint64_t n3,
                                            const uint32_t* __restrict__ xp, uint32_t* pw)
{
    const uint32_t wave = threadIdx.x >> 6, lane = threadIdx.x & 63u;
    const uint64_t n = wave == 0 ? n0 : wave == 1 ? n1 : wave == 2 ? n2 : n3;
    const uint32_t v = xpow8n_wave(n, xp, lane);
    if (lane == 0)
        pw[wave] = v;
}

// Standard CRC-32C of an n-byte message from its raw CRC (zero initial
// value, no final inversion) and x^(8n): the all-ones initial value carried
// through the n bytes, plus the final inversion.
__device__ __forceinline__ uint32_t crc_from_raw(uint32_t raw, uint32_t x8n)
{
    return raw ^ gf2_mulmod(0xFFFFFFFFu, x8n) ^ 0xFFFFFFFFu;
}

// Raw CRC of the 4 KiB steps [j0, j1) of a message by one 256-thread
// workgroup.  load(j) gives thread t's 16-byte word t of step j (the caller
// left-pads the message with zero bytes to whole steps, which leaves a raw
// CRC unchanged); use(j, w) is called on it in step order (a store of the
// word, or nothing).  Thread t keeps a Horner accumulator with a "shift by
// 4 KiB" step over its words, the wave butterfly combines lanes and each wave
// is shifted by the 1 KiB stripes that follow it.  Eight steps' loads are in
// flight before they are folded.  lds: slicing tables and all seven shift
// levels.  Uniform over the workgroup; all threads return the value.
template <typename Load, typename Use>
__device__ __forceinline__ uint32_t wg_crc_steps(Load load, Use use, uint64_t j0, uint64_t j1,
                                                 const uint32_t* __restrict__ lds, uint32_t* red)
{
    const uint32_t tid = threadIdx.x;
    const uint32_t lane = tid & 63u;
    const uint32_t wave = tid >> 6;
    const uint32_t* Z1024 = lds + kSliceWords + 5 * 1024;
    const uint32_t* Z4096 = lds + kSliceWords + 6 * 1024;
    constexpr int U = 8;
    uint32_t s = 0;
    uint64_t j = j0;
    for (; j + U <= j1; j += U) {
        uint4 w[U];
#pragma unroll
        for (int u = 0; u < U; ++u)
            w[u] = load(j + u);
#pragma unroll
        for (int u = 0; u < U; ++u) {
            use(j + u, w[u]);
            s = shiftz(Z4096, s) ^ word_crc(lds, w[u]);
        }
    }
    for (; j < j1; ++j) {
        const uint4 w = load(j);
        use(j, w);
        s = shiftz(Z4096, s) ^ word_crc(lds, w);
    }
    s = lane_combine(lds, s, lane);
    for (uint32_t k = wave; k < 3; ++k)
        s = shiftz(Z1024, s);
    if (lane == 0)
        red[wave] = s;
    __syncthreads();
    const uint32_t raw = red[0] ^ red[1] ^ red[2] ^ red[3];
    __syncthreads();
    return raw;
}

// A message of n bytes cut into S = ceil(n / 4096) steps of 4 KiB after
// left-padding with zeros; workgroup b of nb takes steps [S b / nb,
// S (b + 1) / nb).  Its raw CRC times x^(8 * bytes after its steps) is its
// share of the message's raw CRC, and the shares XOR to the whole.
struct StepSplit {
    uint64_t steps, j0, j1;
    int64_t pad;  // zero bytes in front of the message
    __device__ StepSplit(uint64_t n, uint32_t b, uint32_t nb)
    {
        steps = (n + 4095) >> 12;
        pad = (int64_t)(steps * 4096 - n);
        j0 = steps * b / nb;
        j1 = steps * (b + 1) / nb;
    }
    // message offset of thread t's first byte of step j (negative: padding)
    __device__ int64_t at(uint64_t j) const
    {
        return (int64_t)((j * 256 + threadIdx.x) * 16) - pad;
    }
};

// This workgroup's share of the raw CRC of the message split by sp: the raw
// CRC of its steps times x_after = x^(8 * bytes after them), zero when it
// has no steps.  load and use as for wg_crc_steps.  Uniform over the
// workgroup.
template <typename Load, typename Use>
__device__ __forceinline__ uint32_t wg_crc_share(const StepSplit& sp, Load load, Use use,
                                                 uint32_t x_after,
                                                 const uint32_t* __restrict__ lds, uint32_t* red)
{
    if (sp.j0 >= sp.j1)
        return 0;
    return gf2_mulmod(wg_crc_steps(load, use, sp.j0, sp.j1, lds, red), x_after);
}

// Workgroups a request's header or image check uses: about two 4 KiB steps
// each over the longer of its two CRC messages, at most the nb launched.
__device__ __forceinline__ uint32_t active_blocks(uint64_t bytes_a, uint64_t bytes_b, uint32_t nb)
{
    const uint64_t steps = ((bytes_a > bytes_b ? bytes_a : bytes_b) + 4095) >> 12;
    const uint64_t want = (steps + 1) / 2;
    return want < 1 ? 1u : want < nb ? (uint32_t)want : nb;
}

// Called once by every workgroup of a request after its atomics: true in
// exactly one of them, the last to arrive, which then sees every other
// workgroup's atomics.  Not called when a request has one workgroup.
__device__ __forceinline__ bool last_arrival(uint32_t* count, uint32_t nb, uint32_t* s_flag)
{
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0)
        *s_flag = atomicAdd(count, 1u) == nb - 1 ? 1u : 0u;
    __syncthreads();
    const bool last = *s_flag != 0;
    __syncthreads();
    if (last)
        __threadfence();
    return last;
}

// acc[0..3] read at L2 (device-scope atomics) by threads 0-3 at once, into
// LDS for the workgroup.
__device__ __forceinline__ void read_accs(uint32_t* acc, uint32_t* s_vals)
{
    if (threadIdx.x < 4)
        s_vals[threadIdx.x] = atomicAdd(&acc[threadIdx.x], 0u);
    __syncthreads();
}

// 0xFFFFFFFF * x^(8 * 60): the all-ones initial value carried to the end of
// the header's first 60 bytes.
constexpr uint32_t kInitOver60 = gf2_shift(0xFFFFFFFFu, 60);

// ------------------------------------------------------------ k_header

// nb workgroups launched per request of [q0, q0 + gridDim.x / nb), of which
// the first active_blocks() work.  Each writes its share of the prefix
// (header, region table, bitmap) and of the CRC array into the image while
// folding the same words into its shares of the raw meta_crc and crcs_crc
// (read from the sources, never back from the image, which may sit in host
// memory).  In the meta message the header's last two words (meta_crc,
// crcs_crc) count as zero; crcs_crc is added at the end by linearity.  With
// several workgroups O.acc collects the shares and the arrivals (zero on
// entry: the final scan clears it) and the last to arrive writes the two CRC
// words; a single workgroup keeps its shares in registers.
__global__ __launch_bounds__(256) void k_header(const DevRegion* __restrict__ regs,
                                                const DevRequest* __restrict__ reqs,
                                                DevReqOut* __restrict__ out,
                                                const uint64_t* __restrict__ bitmap,
                                                const uint32_t* __restrict__ crcs,
                                                uint8_t* __restrict__ staging, uint32_t q0,
                                                uint32_t nb, uint64_t capacity,
                                                const CrcTables* __restrict__ tabs)
{
    __shared__ __attribute__((aligned(16))) uint32_t lds[kAllTabWords];
    __shared__ uint32_t red[4];
    __shared__ uint32_t s_word;
    __shared__ uint32_t s_hdr[16];
    __shared__ uint32_t s_pw[4];
    __shared__ uint32_t s_acc[4];
    const uint32_t q = q0 + blockIdx.x / nb, b = blockIdx.x % nb;
    const DevRequest& Q = reqs[q];
    DevReqOut& O = out[q];
    if (O.code != 0 && O.img_base + Q.data_off > capacity)
        return;  // no room even for the prefix
    const uint32_t tid = threadIdx.x;
    uint8_t* img = staging + O.img_base;
    const uint64_t R = Q.n_regions;
    const uint64_t table_end = 64 + 32 * R;
    const uint64_t prefix_end = table_end + 8 * Q.n_words;
    const uint64_t D = O.n_dirty;
    const uint64_t first_page0 = Q.first_word * 64;
    const bool ok = O.code == 0;
    const uint32_t ne = active_blocks(prefix_end, ok ? 4 * D : 0, nb);
    if (b >= ne)
        return;
    const StepSplit m(prefix_end, b, ne);
    const StepSplit c(ok ? 4 * D : 0, b, ne);
    // the shares' shifts, and for the last workgroup x^(8 * 4D) and
    // x^(8 * (prefix_end - 60)) (crcs_crc's place in the meta message)
    wave_powers((c.steps - c.j1) * 4096, (m.steps - m.j1) * 4096, 4 * D, prefix_end - 60,
                tabs->xp, s_pw);
    load_all_tables(lds, tabs);

    // header words (the two CRC words zero), in the workgroups whose steps
    // hold some of its bytes: padded positions [m.pad, m.pad + 64)
    const bool has_hdr = m.j0 < m.j1 && m.j0 * 4096 < (uint64_t)m.pad + 64 &&
                         m.j1 * 4096 > (uint64_t)m.pad;
    uint32_t shadowed = 0;
    if (has_hdr)
        for (uint64_t i = tid; i < R; i += blockDim.x)
            shadowed |= regs[Q.first_region + i].shadow ? 1u : 0u;
    const int any_shadow = __syncthreads_or((int)shadowed);
    if (tid == 0) {
        s_hdr[0] = 0x4D555243u;  // "CRUM"
        s_hdr[1] = 0x31474D49u;  // "IMG1"
        s_hdr[2] = 1;
        s_hdr[3] = 1u << Q.page_shift;
        s_hdr[4] = (uint32_t)R;
        s_hdr[5] = any_shadow ? 0u : 1u;
        s_hdr[6] = (uint32_t)Q.n_pages;
        s_hdr[7] = (uint32_t)(Q.n_pages >> 32);
        s_hdr[8] = (uint32_t)D;
        s_hdr[9] = (uint32_t)(D >> 32);
        s_hdr[10] = (uint32_t)Q.seq;
        s_hdr[11] = (uint32_t)(Q.seq >> 32);
        s_hdr[12] = (uint32_t)Q.data_off;
        s_hdr[13] = (uint32_t)(Q.data_off >> 32);
        s_hdr[14] = 0;
        s_hdr[15] = 0;
    }
    __syncthreads();
    const uint64_t gt = (uint64_t)b * blockDim.x + tid, gstride = (uint64_t)ne * blockDim.x;
    for (uint64_t o = prefix_end + 8 * gt; o < Q.data_off; o += 8 * gstride)
        *reinterpret_cast<uint64_t*>(img + o) = 0;

    // prefix word at byte r: header, region table entries {id, len, first
    // page within the request, 0}, then the bitmap
    const gcu32 bm32 = (gcu32)(bitmap + Q.first_word);
    auto prefix_word = [&](uint64_t r) -> uint32_t {
        if (r < 64)
            return s_hdr[r >> 2];
        if (r < table_end) {
            const uint64_t t = r - 64;
            const DevRegion& G = regs[Q.first_region + (t >> 5)];
            const uint32_t k = (uint32_t)(t >> 2) & 7u;
            const uint64_t v = k < 2 ? G.id : k < 4 ? G.len : k < 6 ? G.first_page - first_page0 : 0;
            return (uint32_t)(v >> (32 * (k & 1)));
        }
        return bm32[(r - table_end) >> 2];
    };
    // m.pad is a multiple of 8, so each thread's 16 bytes are two aligned
    // 8-byte pairs; the pair at 56 is the two CRC words, written last
    auto m_load = [&](uint64_t j) {
        const int64_t v = m.at(j);
        uint32_t w[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int64_t r = v + 4 * i;
            w[i] = r >= 0 ? prefix_word((uint64_t)r) : 0u;
        }
        return make_uint4(w[0], w[1], w[2], w[3]);
    };
    auto m_use = [&](uint64_t j, uint4 w) {
        const int64_t v = m.at(j);
        if (v >= 0 && v != 56)
            *(gv2)(img + v) = u32x2{w.x, w.y};
        if (v + 8 >= 0 && v + 8 != 56)
            *(gv2)(img + v + 8) = u32x2{w.z, w.w};
    };
    const uint32_t m_share = wg_crc_share(m, m_load, m_use, s_pw[1], lds, red);
    uint32_t c_share = 0;
    if (ok) {
        const uint64_t crcs_off = Q.data_off + (D << Q.page_shift);
        const gcu32 src = (gcu32)(crcs + O.slot_base);
        uint8_t* dst = img + crcs_off;
        const bool even = (D & 1) == 0;  // then c.pad, and every v, is a multiple of 8
        auto c_load = [&](uint64_t j) {
            const int64_t v = c.at(j);
            uint32_t w[4];
#pragma unroll
            for (int i = 0; i < 4; ++i)
                w[i] = v + 4 * i >= 0 ? src[(v >> 2) + i] : 0u;
            return make_uint4(w[0], w[1], w[2], w[3]);
        };
        auto c_use = [&](uint64_t j, uint4 w) {
            const int64_t v = c.at(j);
            if (even) {
                if (v >= 0)
                    *(gv2)(dst + v) = u32x2{w.x, w.y};
                if (v + 8 >= 0)
                    *(gv2)(dst + v + 8) = u32x2{w.z, w.w};
            } else {
                const uint32_t ws[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    if (v + 4 * i >= 0)
                        ((gu32)dst)[(v >> 2) + i] = ws[i];
            }
        };
        c_share = wg_crc_share(c, c_load, c_use, s_pw[0], lds, red);
        if (b == 0 && tid == 0 && !even)
            ((gu32)dst)[D] = 0;
    }

    uint32_t c_raw = c_share, m_raw = m_share;
    if (ne > 1) {
        if (tid == 0) {
            if (c_share)
                atomicXor(&O.acc[0], c_share);
            if (m_share)
                atomicXor(&O.acc[1], m_share);
        }
        if (!last_arrival(&O.acc[2], ne, &s_word))
            return;
        read_accs(O.acc, s_acc);
        c_raw = s_acc[0];
        m_raw = s_acc[1];
    }
    if (tid == 0) {
        const uint32_t crcs_crc = ok ? crc_from_raw(c_raw, s_pw[2]) : 0u;
        // raw meta with crcs_crc in place, then the initial value and inversion
        const uint32_t meta = m_raw ^ gf2_mulmod(crcs_crc ^ kInitOver60, s_pw[3]) ^ 0xFFFFFFFFu;
        *(gv2)(img + 56) = u32x2{meta, crcs_crc};
    }
}

// Workgroups per request for the header and image-check kernels: about two
// 4 KiB CRC steps each over the larger of the prefix and the CRC array, at
// most 128.
uint32_t header_blocks(uint64_t n_regions, uint64_t n_words, uint64_t n_crcs)
{
    const uint64_t prefix = 64 + 32 * n_regions + 8 * n_words;
    const uint64_t bytes = prefix > 4 * n_crcs ? prefix : 4 * n_crcs;
    const uint64_t steps = (bytes + 4095) >> 12;
    const uint64_t nb = (steps + 1) / 2;
    return (uint32_t)(nb < 1 ? 1 : nb > 128 ? 128 : nb);
}

hipError_t launch_header(const DevRegion* regs, const DevRequest* reqs, uint32_t q0, uint32_t q1,
                         uint32_t blocks, DevReqOut* out, const uint64_t* bitmap,
                         const uint32_t* crcs, uint8_t* staging, uint64_t capacity,
                         const CrcTables* tabs, hipStream_t s)
{
    if (q1 <= q0)
        return hipSuccess;
    if (blocks == 0 || (uint64_t)(q1 - q0) * blocks > 0x7FFFFFFFull)
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_header, dim3((q1 - q0) * blocks), dim3(256), 0, s, regs, reqs, out,
                       bitmap, crcs, staging, q0, blocks, capacity, tabs);
    return hipGetLastError();
}

__global__ void k_plan_init(DevGlobal* __restrict__ glob)
{
    glob->total_dirty = 0;
    glob->staging_used = 0;
    glob->code = 0;
    glob->fmt_bad = 0;
    glob->crc_bad = kNoBad;
    glob->running = 0;
    glob->img_next = 0;
}

hipError_t launch_plan_init(DevGlobal* glob, hipStream_t s)
{
    hipLaunchKernelGGL(k_plan_init, dim3(1), dim3(1), 0, s, glob);
    return hipGetLastError();
}

__global__ void k_plan_status(const DevReqOut* __restrict__ out, uint32_t n,
                              uint8_t* __restrict__ dst)
{
    const uint32_t q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n)
        return;
    const DevReqOut& O = out[q];
    uint8_t* d = dst + 40ull * q;
    *reinterpret_cast<int32_t*>(d) = O.code;
    *reinterpret_cast<uint32_t*>(d + 4) = O.first_bad;
    *reinterpret_cast<uint64_t*>(d + 8) = O.n_dirty;
    *reinterpret_cast<uint64_t*>(d + 16) = O.total_pages;
    *reinterpret_cast<uint64_t*>(d + 24) = O.image_bytes;
    *reinterpret_cast<uint64_t*>(d + 32) = O.img_base;
}

hipError_t launch_plan_status(const DevReqOut* out, uint32_t n, uint8_t* dst, hipStream_t s)
{
    if (n == 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_plan_status, dim3((n + 255) / 256), dim3(256), 0, s, out, n, dst);
    return hipGetLastError();
}

// ------------------------------------------------------------ restore

// Device-side image checks that need the bytes: meta_crc, crcs_crc, bitmap
// population and unused bits, zero pads.  The host has already checked the
// header fields, lengths and the region table.  nb workgroups launched per
// request, of which the first active_blocks() work; each takes a share of the
// bitmap, the pad and the two CRC messages.  With several, O.acc (zero on
// entry: the host uploads it cleared) collects the CRC shares, the arrivals
// and the population, and the last workgroup to arrive compares.
__global__ __launch_bounds__(256) void k_restore_check(const DevRequest* __restrict__ reqs,
                                                       DevReqOut* __restrict__ out,
                                                       const uint8_t* __restrict__ staging,
                                                       uint32_t nb,
                                                       const CrcTables* __restrict__ tabs,
                                                       DevGlobal* __restrict__ glob)
{
    __shared__ __attribute__((aligned(16))) uint32_t lds[kAllTabWords];
    __shared__ uint32_t red[4];
    __shared__ uint32_t s_pop;
    __shared__ uint32_t s_word;
    __shared__ uint32_t s_pw[4];
    __shared__ uint32_t s_acc[4];
    const uint32_t tid = threadIdx.x;
    const uint32_t q = blockIdx.x / nb, b = blockIdx.x % nb;
    const DevRequest& Q = reqs[q];
    DevReqOut& O = out[q];
    const uint8_t* img = staging + O.img_base;
    const gcu32 img32 = (gcu32)img;
    const uint64_t R = Q.n_regions;
    const uint64_t prefix_end = 64 + 32 * R + 8 * Q.n_words;
    const uint64_t D = reinterpret_cast<const uint64_t*>(img)[4];
    const uint64_t crcs_off = Q.data_off + (D << Q.page_shift);
    const uint32_t ne = active_blocks(prefix_end, 4 * D, nb);
    if (b >= ne)
        return;
    const StepSplit c(4 * D, b, ne);
    const StepSplit m(prefix_end, b, ne);
    wave_powers((c.steps - c.j1) * 4096, (m.steps - m.j1) * 4096, 4 * D, prefix_end, tabs->xp,
                s_pw);
    if (tid == 0)
        s_pop = 0;
    load_all_tables(lds, tabs);

    const uint64_t gt = (uint64_t)b * blockDim.x + tid, gstride = (uint64_t)ne * blockDim.x;
    const uint64_t* bm = reinterpret_cast<const uint64_t*>(img + 64 + 32 * R);
    uint32_t pop = 0, bad = 0;
    for (uint64_t w = gt; w < Q.n_words; w += gstride) {
        const uint64_t word = bm[w];
        pop += (uint32_t)__popcll(word);
        if (w == Q.n_words - 1 && (Q.n_pages & 63)) {
            if (word >> (Q.n_pages & 63))
                bad = 1;
        }
    }
    for (uint64_t o = prefix_end + 8 * gt; o < Q.data_off; o += 8 * gstride)
        if (*reinterpret_cast<const uint64_t*>(img + o))
            bad = 1;
    if (gt == 0) {
        for (uint64_t o = crcs_off + 4 * D; o < O.image_bytes; ++o)
            if (img[o])
                bad = 1;
    }
    if (bad)
        atomicOr(&glob->fmt_bad, 1u);
    if (pop)
        atomicAdd(&s_pop, pop);

    auto no_use = [](uint64_t, uint4) {};
    const gcu32 c32 = (gcu32)(img + crcs_off);
    auto c_load = [&](uint64_t j) {
        const int64_t v = c.at(j);
        uint32_t w[4];
#pragma unroll
        for (int i = 0; i < 4; ++i)
            w[i] = v + 4 * i >= 0 ? c32[(v >> 2) + i] : 0u;
        return make_uint4(w[0], w[1], w[2], w[3]);
    };
    const uint32_t c_share = wg_crc_share(c, c_load, no_use, s_pw[0], lds, red);
    auto m_load = [&](uint64_t j) {
        const int64_t v = m.at(j);
        uint32_t w[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int64_t r = v + 4 * i;
            w[i] = r >= 0 && r != 56 ? img32[r >> 2] : 0u;  // meta_crc itself reads as zero
        }
        return make_uint4(w[0], w[1], w[2], w[3]);
    };
    const uint32_t m_share = wg_crc_share(m, m_load, no_use, s_pw[1], lds, red);
    __syncthreads();
    uint32_t c_raw = c_share, m_raw = m_share, total_pop = s_pop;
    if (ne > 1) {
        if (tid == 0) {
            if (c_share)
                atomicXor(&O.acc[0], c_share);
            if (m_share)
                atomicXor(&O.acc[1], m_share);
            if (s_pop)
                atomicAdd(&O.acc[3], s_pop);
        }
        if (!last_arrival(&O.acc[2], ne, &s_word))
            return;
        read_accs(O.acc, s_acc);
        c_raw = s_acc[0];
        m_raw = s_acc[1];
        total_pop = s_acc[3];
    }
    if (tid == 0) {
        const uint32_t crcs = crc_from_raw(c_raw, s_pw[2]);
        const uint32_t meta = crc_from_raw(m_raw, s_pw[3]);
        if ((uint64_t)total_pop != D || crcs != img32[15] || meta != img32[14])
            atomicOr(&glob->fmt_bad, 1u);
    }
}

hipError_t launch_restore_check(const DevRequest* reqs, uint32_t n_reqs, uint32_t blocks,
                                DevReqOut* out, const uint8_t* staging, const CrcTables* tabs,
                                DevGlobal* glob, hipStream_t s)
{
    if (n_reqs == 0)
        return hipSuccess;
    if (blocks == 0 || (uint64_t)n_reqs * blocks > 0x7FFFFFFFull)
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_restore_check, dim3(n_reqs * blocks), dim3(256), 0, s, reqs, out,
                       staging, blocks, tabs, glob);
    return hipGetLastError();
}

// Wave per (slot, piece): packed page -> its page (and shadow).
__global__ __launch_bounds__(256) void k_scatter(const DevRegion* __restrict__ regs,
                                                 uint32_t n_regs,
                                                 const DevRequest* __restrict__ reqs,
                                                 const DevReqOut* __restrict__ out,
                                                 const uint32_t* __restrict__ list,
                                                 uint64_t n_items, uint32_t np_shift,
                                                 uint32_t piece_shift,
                                                 const uint8_t* __restrict__ staging,
                                                 int update_shadow,
                                                 const DevGlobal* __restrict__ glob)
{
    if (glob->fmt_bad || glob->crc_bad != kNoBad)
        return;
    const uint32_t lane = threadIdx.x & 63u;
    const uint64_t wave = (uint64_t)blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint64_t n_waves = (uint64_t)gridDim.x * 4;
    uint32_t r = 0;
    uint64_t r_lo = 1, r_hi = 0;
    for (uint64_t item = wave; item < n_items; item += n_waves) {
        const uint64_t k = item >> np_shift;
        const uint32_t piece = (uint32_t)(item & ((1ull << np_shift) - 1));
        const uint64_t g = list[k];
        if (g < r_lo || g >= r_hi) {
            r = find_region<3>(regs, n_regs, g);
            r_lo = regs[r].first_page;
            r_hi = r_lo + (regs[r].len >> regs[r].page_shift);
        }
        const DevRegion& R = regs[r];
        if (g < r_lo || g >= r_hi)
            continue;
        const DevRequest& Q = reqs[R.req];
        const DevReqOut& O = out[R.req];
        const uint32_t ps = R.page_shift;
        const uint32_t pb_shift = ps < piece_shift ? ps : piece_shift;
        if (piece >= (1u << (ps - pb_shift)))
            continue;
        const uint64_t page_off = (g - R.first_page) << ps;
        const uint64_t piece_off = (uint64_t)piece << pb_shift;
        const gcv4 src =
            (gcv4)(staging + O.img_base + Q.data_off + ((k - O.slot_base) << ps) + piece_off);
        const gv4 dst = (gv4)(R.cur + page_off + piece_off);
        const gv4 sh = (update_shadow && R.shadow) ? (gv4)(R.shadow + page_off + piece_off)
                                                   : nullptr;
        const uint32_t n16 = 1u << (pb_shift - 4);
        for (uint32_t i = lane; i < n16; i += 64 * 4) {
            u32x4 w[4];
#pragma unroll
            for (int u = 0; u < 4; ++u)
                if (i + 64 * u < n16)
                    w[u] = src[i + 64 * u];
#pragma unroll
            for (int u = 0; u < 4; ++u)
                if (i + 64 * u < n16) {
                    dst[i + 64 * u] = w[u];
                    if (sh)
                        sh[i + 64 * u] = w[u];
                }
        }
    }
}

hipError_t launch_scatter(const DevRegion* regs, uint32_t n_regs, const DevRequest* reqs,
                             const DevReqOut* out, const uint32_t* list, uint64_t n_slots,
                             uint32_t np_shift, uint32_t piece_shift, const uint8_t* staging,
                             int update_shadow, const DevGlobal* glob, int blocks, hipStream_t s)
{
    if (n_slots == 0)
        return hipSuccess;
    if (piece_shift < kPieceShiftMin || piece_shift > kPieceShift)
        return hipErrorInvalidValue;
    const uint64_t n_items = n_slots << np_shift;
    const uint64_t need = (n_items + 3) / 4;
    const uint64_t nb = need < (uint64_t)blocks ? need : (uint64_t)blocks;
    hipLaunchKernelGGL(k_scatter, dim3((unsigned)nb), dim3(256), 0, s, regs, n_regs, reqs, out,
                       list, n_items, np_shift, piece_shift, staging, update_shadow, glob);
    return hipGetLastError();
}

__global__ void k_restore_finish(DevReqOut* __restrict__ out, DevGlobal* __restrict__ glob)
{
    DevReqOut& O = out[0];
    if (glob->fmt_bad) {
        O.code = -4;  // CRUM_EFORMAT
        O.first_bad = 0;
    } else if (glob->crc_bad != kNoBad) {
        O.code = -3;  // CRUM_ECRC
        O.first_bad = glob->crc_bad;
    } else {
        O.code = 0;
        O.first_bad = 0;
    }
}

hipError_t launch_restore_finish(DevReqOut* out, uint32_t, DevGlobal* glob, hipStream_t s)
{
    hipLaunchKernelGGL(k_restore_finish, dim3(1), dim3(1), 0, s, out, glob);
    return hipGetLastError();
}

}  // namespace crum
