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
//             dirty counts, image offsets and the capacity check.
//   k_list    per word: ballot compaction, lane with bit set writes its page
//             index at prefix + popcount(bits below the lane).
//   k_pack    per dirty page (or piece of up to 64 KiB): copy into the
//             image's page area, optionally into the shadow, and CRC-32C on
//             the way; k_finalize combines the piece CRCs of larger pages.
//   k_header  per request: header, region table, bitmap, CRC array, pads,
//             crcs_crc, meta_crc.
// Restore: k_restore_check, k_scan, k_list, k_pack (verify), k_scatter.
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
// (used once per piece) are read from global memory.
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

// lds: the pack layout (kPackLdsWords); V: the CRC step variant.
template <bool STORE, int U, int V>
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
            w[u] = src.at(t + u)[(t + u) * 64 + lane];
        if (STORE) {
#pragma unroll
            for (int u = 0; u < U; ++u)
                dst[(t + u) * 64 + lane] = w[u];
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

// Raw (zero-initialised) CRC of `steps` KiB, copied to dst (and to the shadow
// sh, dirty units only) when STORE.  DEPTH: 16-byte loads each lane issues
// before it folds them into its CRC.  All lanes return the same value.
// gz: z[0] of the shift tables in global memory (the butterfly's shifts).
template <bool STORE, int DEPTH, int V>
__device__ __forceinline__ uint32_t wave_piece_crc(const PieceSrc& src, gv4 __restrict__ dst,
                                                   gv4 __restrict__ sh, uint32_t steps,
                                                   uint32_t lane,
                                                   const uint32_t* __restrict__ lds,
                                                   const uint32_t* __restrict__ gz)
{
    uint32_t s = 0;
    uint32_t t = 0;
    s = piece_steps<STORE, DEPTH, V>(src, dst, sh, &t, steps, lane, lds, s);
    if (DEPTH > 4)
        s = piece_steps<STORE, 4, V>(src, dst, sh, &t, steps, lane, lds, s);
    s = piece_steps<STORE, 1, V>(src, dst, sh, &t, steps, lane, lds, s);
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

// One wave per diff unit of global units [u0, u1); unit_flags[u] = 1 when
// any byte of the unit differs from the shadow (or the region has none).
// prio 1..3 raises the waves' issue priority on their compute unit above
// that of co-running kernels' waves (0 leaves it at the default).
template <bool NT>
__global__ __launch_bounds__(256) void k_diff(const DevRegion* __restrict__ regs,
                                              uint32_t n_regs, uint64_t u0, uint64_t u1,
                                              uint8_t* __restrict__ unit_flags, uint32_t prio)
{
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
    for (uint64_t u = u0 + wave; u < u1; u += n_waves) {
        if (u < r_lo || u >= r_hi) {
            r = find_region<4>(regs, n_regs, u);
            r_lo = regs[r].first_unit;
            r_hi = r_lo + (regs[r].len >> regs[r].unit_shift);
        }
        const DevRegion& R = regs[r];
        const uint32_t us = R.unit_shift;
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
}

hipError_t launch_diff(const DevRegion* regs, uint32_t n_regs, uint64_t u0, uint64_t u1,
                       uint8_t* unit_flags, int blocks, int nontemporal, int prio,
                       hipStream_t s)
{
    if (u1 <= u0)
        return hipSuccess;
    const uint64_t need = (u1 - u0 + 3) / 4;
    const uint64_t nb = need < (uint64_t)blocks ? need : (uint64_t)blocks;
    if (nontemporal)
        hipLaunchKernelGGL(k_diff<true>, dim3((unsigned)nb), dim3(256), 0, s, regs, n_regs, u0,
                           u1, unit_flags, (uint32_t)prio);
    else
        hipLaunchKernelGGL(k_diff<false>, dim3((unsigned)nb), dim3(256), 0, s, regs, n_regs, u0,
                           u1, unit_flags, (uint32_t)prio);
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

__global__ __launch_bounds__(1024) void k_scan(const uint64_t* __restrict__ bitmap, uint64_t w0,
                                               uint64_t w1, uint64_t n_words_total,
                                               uint32_t* __restrict__ prefix,
                                               uint64_t* __restrict__ bounds_out, int final,
                                               const DevRequest* __restrict__ reqs, uint32_t q0,
                                               uint32_t q1, DevReqOut* __restrict__ out,
                                               DevGlobal* __restrict__ glob, uint64_t capacity,
                                               int restore_mode)
{
    constexpr int V = 4;  // words per thread per pass
    __shared__ uint32_t wave_tot[16];
    const uint32_t tid = threadIdx.x, lane = tid & 63u, wv = tid >> 6;
    uint32_t carry = (uint32_t)glob->running;
    for (uint64_t base = w0; base < w1; base += 1024 * V) {
        uint32_t c[V];
        uint32_t local = 0;
#pragma unroll
        for (int v = 0; v < V; ++v) {
            const uint64_t w = base + (uint64_t)tid * V + v;
            c[v] = w < w1 ? (uint32_t)__popcll(bitmap[w]) : 0u;
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
            if (w < w1)
                prefix[w] = excl;
            excl += c[v];
        }
        carry += blk;
        __syncthreads();
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
                       uint64_t capacity, int restore_mode, hipStream_t s)
{
    hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, s, bitmap, w0, w1, n_words_total, prefix,
                       bounds_out, final, reqs, q0, q1, out, glob, capacity, restore_mode);
    return hipGetLastError();
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
                                              DevGlobal* __restrict__ glob)
{
    __shared__ __attribute__((aligned(16))) uint32_t lds[kPackLdsWords];
    if (MODE == kModeVerify && glob->fmt_bad)
        return;
    uint64_t slot0, slot1;
    slot_range(sr, &slot0, &slot1);
    const uint64_t n_items = (slot1 - slot0) << np_shift;
    if (n_items == 0)
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
            raw = wave_piece_crc<true, DEPTH, V>(src, (gv4)slot_ptr, sh,
                                                 steps, lane, lds, gz);
        } else {
            const PieceSrc src{(gcv4)slot_ptr, nullptr, ~0u, 0};
            raw = wave_piece_crc<false, DEPTH, V>(src, nullptr, nullptr, steps, lane, lds, gz);
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
                            uint32_t* partials, const CrcTables* tabs, DevGlobal* glob)
{
    hipLaunchKernelGGL((k_pack<MODE, DEPTH, V>), grid, dim3(256), 0, s, regs, n_regs, reqs, out,
                       list, range, np_shift, piece_shift, unit_flags, staging, crc_out,
                       partials, tabs, glob);
}

template <int MODE, int DEPTH>
static void launch_pack_depth(int variant, dim3 grid, hipStream_t s, const DevRegion* regs,
                              uint32_t n_regs, const DevRequest* reqs, const DevReqOut* out,
                              const uint32_t* list, SlotRange range, uint32_t np_shift,
                              uint32_t piece_shift, const uint8_t* unit_flags, uint8_t* staging,
                              uint32_t* crc_out, uint32_t* partials, const CrcTables* tabs,
                              DevGlobal* glob)
{
#define CRUM_PACK_V(v)                                                                        \
    launch_pack_one<MODE, DEPTH, v>(grid, s, regs, n_regs, reqs, out, list, range, np_shift, \
                                    piece_shift, unit_flags, staging, crc_out, partials, tabs, \
                                    glob)
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
                             const CrcTables* tabs, DevGlobal* glob)
{
    if (depth == 16)
        launch_pack_depth<MODE, 16>(variant, grid, s, regs, n_regs, reqs, out, list, range,
                                    np_shift, piece_shift, unit_flags, staging, crc_out,
                                    partials, tabs, glob);
    else if (depth == 8)
        launch_pack_depth<MODE, 8>(variant, grid, s, regs, n_regs, reqs, out, list, range,
                                   np_shift, piece_shift, unit_flags, staging, crc_out, partials,
                                   tabs, glob);
    else
        launch_pack_depth<MODE, 4>(variant, grid, s, regs, n_regs, reqs, out, list, range,
                                   np_shift, piece_shift, unit_flags, staging, crc_out, partials,
                                   tabs, glob);
}

hipError_t launch_pack(int mode, const DevRegion* regs, uint32_t n_regs, const DevRequest* reqs,
                       const DevReqOut* out, const uint32_t* list, SlotRange range,
                       uint32_t np_shift, uint32_t piece_shift, const uint8_t* unit_flags,
                       uint8_t* staging, uint32_t* crc_out, uint32_t* partials,
                       const CrcTables* tabs, DevGlobal* glob, int blocks, int depth,
                       int variant, hipStream_t s)
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
                                    partials, tabs, glob);
    else
        launch_pack_mode<kModeVerify>(grid, depth, variant, s, regs, n_regs, reqs, out, list,
                                      range, np_shift, piece_shift, nullptr, staging, crc_out,
                                      partials, tabs, glob);
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

// Standard CRC-32C of n bytes at p (p 16-byte aligned) computed by one
// 256-thread workgroup; the 4 bytes at zero_off (a multiple of 4, or ~0) are
// read as zero.  T is the slicing table in LDS.  All threads return it.
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

// Standard CRC-32C of n bytes at p (p and n multiples of 4) by one
// 256-thread workgroup; the 4 bytes at zero_off (a multiple of 4, or ~0) are
// read as zero.  The message is taken as left-padded with zero bytes to a
// multiple of 4096 (which leaves a zero-initialised CRC unchanged); thread t
// reads 16-byte words t, t+256, ... and keeps a Horner accumulator with a
// "shift by 4096 bytes" step, the wave butterfly combines lanes and each wave
// is shifted by the 1 KiB stripes that follow it.  lds: slicing tables and
// all seven shift levels.  All threads return the value.
__device__ __forceinline__ uint32_t wg_crc(const uint8_t* __restrict__ p, uint64_t n,
                                          uint64_t zero_off, const uint32_t* __restrict__ lds,
                                          const uint32_t* __restrict__ xp, uint32_t* red)
{
    const uint32_t tid = threadIdx.x;
    const uint32_t lane = tid & 63u;
    const uint32_t wave = tid >> 6;
    const uint32_t* Z1024 = lds + kSliceWords + 5 * 1024;
    const uint32_t* Z4096 = lds + kSliceWords + 6 * 1024;
    const uint64_t steps = (n + 4095) / 4096;
    const int64_t pad = (int64_t)(steps * 4096 - n);
    typedef const uint32_t __attribute__((address_space(1)))* gcu32;
    const gcu32 g = (gcu32)p;
    // thread tid's 16 bytes of 4 KiB step j, the step's zero padding (and
    // the word at zero_off) read as zero
    auto load_step = [&](uint64_t j) {
        const int64_t v = (int64_t)((j * 256 + tid) * 16) - pad;
        uint32_t w[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int64_t r = v + 4 * i;
            w[i] = (r >= 0 && (uint64_t)r != zero_off) ? g[r >> 2] : 0u;
        }
        return make_uint4(w[0], w[1], w[2], w[3]);
    };
    // eight steps' loads in flight before they are folded, in step order
    constexpr int U = 8;
    uint32_t s = 0;
    uint64_t j = 0;
    for (; j + U <= steps; j += U) {
        uint4 w[U];
#pragma unroll
        for (int u = 0; u < U; ++u)
            w[u] = load_step(j + u);
#pragma unroll
        for (int u = 0; u < U; ++u)
            s = shiftz(Z4096, s) ^ word_crc(lds, w[u]);
    }
    for (; j < steps; ++j)
        s = shiftz(Z4096, s) ^ word_crc(lds, load_step(j));
    s = lane_combine(lds, s, lane);
    for (uint32_t k = wave; k < 3; ++k)
        s = shiftz(Z1024, s);
    if (lane == 0)
        red[wave] = s;
    const uint32_t fix = gf2_mulmod(0xFFFFFFFFu, xpow8n_wave(n, xp, lane)) ^ 0xFFFFFFFFu;
    __syncthreads();
    const uint32_t raw = red[0] ^ red[1] ^ red[2] ^ red[3];
    __syncthreads();
    return raw ^ fix;
}

// ------------------------------------------------------------ k_header

// dst[i] = src[i] for i < n by one workgroup, 16 loads in flight per thread.
template <typename T>
__device__ __forceinline__ void copy_words(T* __restrict__ dst, const T* __restrict__ src,
                                           uint64_t n)
{
    constexpr uint32_t U = 16;
    const uint64_t stride = (uint64_t)blockDim.x * U;
    uint64_t i = threadIdx.x;
    for (; i + (U - 1) * blockDim.x < n; i += stride) {
        T v[U];
#pragma unroll
        for (uint32_t u = 0; u < U; ++u)
            v[u] = src[i + u * blockDim.x];
#pragma unroll
        for (uint32_t u = 0; u < U; ++u)
            dst[i + u * blockDim.x] = v[u];
    }
    for (; i < n; i += blockDim.x)
        dst[i] = src[i];
}

__global__ __launch_bounds__(256) void k_header(const DevRegion* __restrict__ regs,
                                                const DevRequest* __restrict__ reqs,
                                                const DevReqOut* __restrict__ out,
                                                const uint64_t* __restrict__ bitmap,
                                                const uint32_t* __restrict__ crcs,
                                                uint8_t* __restrict__ staging, uint32_t q0,
                                                uint64_t capacity,
                                                const CrcTables* __restrict__ tabs)
{
    __shared__ __attribute__((aligned(16))) uint32_t lds[kAllTabWords];
    __shared__ uint32_t red[4];
    __shared__ uint32_t s_shadowed;
    const DevRequest& Q = reqs[q0 + blockIdx.x];
    const DevReqOut& O = out[q0 + blockIdx.x];
    if (O.code != 0 && O.img_base + Q.data_off > capacity)
        return;  // no room even for the prefix
    load_all_tables(lds, tabs);
    const uint32_t tid = threadIdx.x;
    uint8_t* img = staging + O.img_base;
    const uint64_t R = Q.n_regions;
    const uint64_t prefix_end = 64 + 32 * R + 8 * Q.n_words;
    const uint64_t D = O.n_dirty;
    const uint64_t first_page0 = Q.first_word * 64;
    if (tid == 0)
        s_shadowed = 0;
    __syncthreads();
    for (uint64_t i = tid; i < R; i += blockDim.x) {
        const DevRegion& G = regs[Q.first_region + i];
        uint64_t* e = reinterpret_cast<uint64_t*>(img + 64 + 32 * i);
        e[0] = G.id;
        e[1] = G.len;
        e[2] = G.first_page - first_page0;
        e[3] = 0;
        if (G.shadow)
            atomicOr(&s_shadowed, 1u);
    }
    copy_words(reinterpret_cast<uint64_t*>(img + 64 + 32 * R), bitmap + Q.first_word,
               Q.n_words);
    for (uint64_t o = prefix_end + 8 * tid; o < Q.data_off; o += 8 * blockDim.x)
        *reinterpret_cast<uint64_t*>(img + o) = 0;
    const bool ok = O.code == 0;
    if (ok) {
        uint32_t* dst = reinterpret_cast<uint32_t*>(img + Q.data_off + (D << Q.page_shift));
        copy_words(dst, crcs + O.slot_base, D);
        if (tid == 0 && (D & 1))
            dst[D] = 0;
    }
    __syncthreads();
    uint32_t* h32 = reinterpret_cast<uint32_t*>(img);
    uint64_t* h64 = reinterpret_cast<uint64_t*>(img);
    if (tid == 0) {
        h64[0] = 0x31474D494D555243ull;  // "CRUMIMG1"
        h32[2] = 1;
        h32[3] = 1u << Q.page_shift;
        h32[4] = (uint32_t)R;
        h32[5] = s_shadowed ? 0u : 1u;
        h64[3] = Q.n_pages;
        h64[4] = D;
        h64[5] = Q.seq;
        h64[6] = Q.data_off;
        h32[14] = 0;
        h32[15] = 0;
    }
    uint32_t crcs_crc = 0;
    if (ok)
        crcs_crc = wg_crc(img + Q.data_off + (D << Q.page_shift), 4 * D, ~0ull, lds, tabs->xp,
                          red);
    if (tid == 0)
        h32[15] = crcs_crc;
    __threadfence_block();
    __syncthreads();
    const uint32_t meta = wg_crc(img, prefix_end, ~0ull, lds, tabs->xp, red);
    if (tid == 0)
        h32[14] = meta;
}

hipError_t launch_header(const DevRegion* regs, const DevRequest* reqs, uint32_t q0, uint32_t q1,
                         const DevReqOut* out, const uint64_t* bitmap, const uint32_t* crcs,
                         uint8_t* staging, uint64_t capacity, const CrcTables* tabs,
                         hipStream_t s)
{
    if (q1 <= q0)
        return hipSuccess;
    hipLaunchKernelGGL(k_header, dim3(q1 - q0), dim3(256), 0, s, regs, reqs, out, bitmap, crcs,
                       staging, q0, capacity, tabs);
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
// header fields, lengths and the region table.
__global__ __launch_bounds__(256) void k_restore_check(const DevRequest* __restrict__ reqs,
                                                       const DevReqOut* __restrict__ out,
                                                       const uint8_t* __restrict__ staging,
                                                       const CrcTables* __restrict__ tabs,
                                                       DevGlobal* __restrict__ glob)
{
    __shared__ __attribute__((aligned(16))) uint32_t lds[kAllTabWords];
    __shared__ uint32_t red[4];
    __shared__ unsigned long long s_pop;
    __shared__ uint32_t s_bad;
    load_all_tables(lds, tabs);
    const uint32_t tid = threadIdx.x;
    const DevRequest& Q = reqs[blockIdx.x];
    const DevReqOut& O = out[blockIdx.x];
    const uint8_t* img = staging + O.img_base;
    const uint64_t R = Q.n_regions;
    const uint64_t prefix_end = 64 + 32 * R + 8 * Q.n_words;
    const uint32_t* h32 = reinterpret_cast<const uint32_t*>(img);
    const uint64_t D = reinterpret_cast<const uint64_t*>(img)[4];
    if (tid == 0) {
        s_pop = 0;
        s_bad = 0;
    }
    __syncthreads();
    const uint64_t* bm = reinterpret_cast<const uint64_t*>(img + 64 + 32 * R);
    unsigned long long pop = 0;
    uint32_t bad = 0;
    for (uint64_t w = tid; w < Q.n_words; w += blockDim.x) {
        const uint64_t word = bm[w];
        pop += __popcll(word);
        if (w == Q.n_words - 1 && (Q.n_pages & 63)) {
            if (word >> (Q.n_pages & 63))
                bad = 1;
        }
    }
    for (uint64_t o = prefix_end + 8 * tid; o < Q.data_off; o += 8 * blockDim.x)
        if (*reinterpret_cast<const uint64_t*>(img + o))
            bad = 1;
    if (tid == 0) {
        const uint64_t tail = Q.data_off + (D << Q.page_shift) + 4 * D;
        for (uint64_t o = tail; o < O.image_bytes; ++o)
            if (img[o])
                bad = 1;
    }
    atomicAdd(&s_pop, pop);
    if (bad)
        atomicOr(&s_bad, 1u);
    const uint32_t crcs =
        wg_crc(img + Q.data_off + (D << Q.page_shift), 4 * D, ~0ull, lds, tabs->xp, red);
    const uint32_t meta = wg_crc(img, prefix_end, 56, lds, tabs->xp, red);
    __syncthreads();
    if (tid == 0) {
        if (s_bad || s_pop != D || crcs != h32[15] || meta != h32[14])
            atomicOr(&glob->fmt_bad, 1u);
    }
}

hipError_t launch_restore_check(const DevRequest* reqs, uint32_t n_reqs, const DevReqOut* out,
                                const uint8_t* staging, const CrcTables* tabs, DevGlobal* glob,
                                hipStream_t s)
{
    hipLaunchKernelGGL(k_restore_check, dim3(n_reqs), dim3(256), 0, s, reqs, out, staging, tabs,
                       glob);
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
