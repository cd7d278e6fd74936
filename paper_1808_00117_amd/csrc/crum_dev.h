// Internal device-side structures and kernel launch interface of libcrum.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace crum {

// Diff unit: min(page, 2^unit_shift_max) bytes, unit_shift_max in 12..14
// (default 14).  A wave compares one unit per step with 64 lanes x 16-byte
// loads, i.e. unit/1 KiB loads per array per lane.
constexpr uint32_t kUnitShiftDefault = 14;
// CRC piece: pages larger than this are split across waves and combined.
constexpr uint32_t kPieceShift = 16;  // largest pack piece: 64 KiB
constexpr uint32_t kPieceShiftMin = 12;
// Default piece: 16 KiB.  Four times the waves of whole 64 KiB pages per
// launch; on the 16 GiB workload's 23 117 dirty 64 KiB pages the pack ran at
// 4.15-4.43 TB/s pipelined and 5.27-5.32 TB/s in one launch with 16 KiB
// pieces, against 3.87-3.92 and 5.13-5.26 TB/s with 64 KiB ones.
constexpr uint32_t kPieceShiftDefault = 14;
// CRC step variants 0..5 (see launch_pack); kCrcVariantAuto picks the one
// measured fastest per kernel: byte tables for pack, variant 3 for verify.
constexpr int kCrcVariantAuto = 6;
constexpr uint32_t kNoBad = 0xFFFFFFFFu;

// One region of the flattened page space (host-built, uploaded per call).
// Page indices are global across all requests of a launch; each request
// starts at a multiple of 64 pages so that bitmap words never straddle
// requests.
struct DevRegion {
    const uint8_t* cur;
    uint8_t* shadow;     // NULL: no baseline
    uint64_t len;
    uint64_t first_page; // global page index of page 0
    uint64_t first_unit; // global diff-unit index of unit 0
    uint64_t id;
    uint32_t page_shift; // log2 page size
    uint32_t req;        // request index
    uint32_t unit_shift; // log2 diff unit = min(page_shift, unit_shift_max)
    uint32_t flags;      // bit 0: copy dirty pages into the shadow
};
static_assert(sizeof(DevRegion) == 64, "DevRegion layout");

// One request (one image) of a launch.
struct DevRequest {
    uint64_t first_word;   // first bitmap word (global)
    uint64_t n_words;
    uint64_t n_pages;      // pages of the request (unpadded G)
    uint64_t first_region; // index into the region table
    uint64_t n_regions;
    uint64_t data_off;     // image prefix bytes
    uint64_t seq;
    uint32_t page_shift;
    uint32_t init_fix;     // CRC constant for one page (see gf2.h)
};
static_assert(sizeof(DevRequest) == 64, "DevRequest layout");

// Per-request results written on the device.
struct DevReqOut {
    int32_t code;
    uint32_t first_bad;
    uint64_t n_dirty;
    uint64_t total_pages;
    uint64_t image_bytes;
    uint64_t slot_base;  // global slot of the request's first packed page
    uint64_t img_base;   // byte offset of the request's image in staging
    // header / image-check kernels: CRC shares of crcs_crc and meta_crc,
    // arrivals, and a flag or count; zero before those kernels run (the final
    // scan clears them for a snapshot, the host for a restore)
    uint32_t acc[4];
};
static_assert(sizeof(DevReqOut) == 64, "DevReqOut layout");

// Launch-wide counters written on the device.
struct DevGlobal {
    uint64_t total_dirty;    // sum of D over requests
    uint64_t staging_used;   // bytes of staging the images occupy
    int32_t code;            // CRUM_OK or CRUM_ENOSPC (any request) / CRUM_EFORMAT
    uint32_t fmt_bad;        // restore: image check failed
    uint32_t crc_bad;        // restore: lowest failing slot, kNoBad if none
    uint32_t pad0;
    uint64_t running;        // dirty pages counted by the scans so far
    uint64_t img_next;       // 4 KiB-aligned staging offset for the next image
    uint64_t pad[2];
};
static_assert(sizeof(DevGlobal) == 64, "DevGlobal layout");

// CRC lookup tables held in device memory and staged into LDS:
//   t[k][b]    = b * x^(8(k+1))        (slicing-by-16 for one 16-byte word)
//   z[j][i][b] = (b << 8i) * x^(8 L_j)  (shift of a 32-bit state by L_j bytes)
// with L_j = 32, 64, 128, 256, 512, 1024 for j = 0..5.
// t[k][b] = b * x^(8(k+1)) (slicing by 16); z[j][i][b] = (b << 8i) * x^(8 L_j)
// for L = 32, 64, 128, 256, 512, 1024, 4096 bytes; xp[i] = x^(8 * 2^i).
// nib[k] splits a byte table by nibbles (a table is linear in its index):
// nib[k][0][n] = T[n] and nib[k][1][n] = T[n << 4] for T = t[k] (k < 16) or
// T = z[5][k - 16] (the shift by 1 KiB), so T[b] = nib[k][0][b & 15] ^
// nib[k][1][b >> 4] with two 16-entry lookups that never conflict in LDS banks.
struct CrcTables {
    uint32_t t[16][256];
    uint32_t z[7][4][256];
    uint32_t xp[64];
    uint32_t nib[20][2][16];
};

enum PackMode { kModePack = 0, kModeVerify = 1 };

struct LaunchShape {
    int diff_blocks;   // persistent grid of the diff kernel (256-thread blocks)
    int pack_blocks;   // persistent grid of the pack/verify/scatter kernels
};

// Slot range of a pack launch: [lo, hi) given on the host, or, when `bounds`
// is non-null, read on the device as [chunk ? bounds[chunk-1] : 0, bounds[chunk]).
struct SlotRange {
    uint64_t lo, hi;
    const uint64_t* bounds;
    uint32_t chunk;
    uint64_t max_slots;  // upper bound on hi - lo (grid sizing)
};

// Kernel launchers (crum_kernels.hip).  All enqueue on `s`.
void build_crc_tables(CrcTables* host);
// cand (may be null): bitmap over global pages; pages whose bit is clear are
// flagged clean without being read (they are known to equal their shadow).
// stamp (may be null): two words, the wall clock at the launch's start and
// the latest end of its workgroups (stamp[1] must start below any clock
// value, e.g. zeroed once).
// group 2 or 4: each wave takes that many consecutive units (as many 4 KiB
// units of a region read as one span); other values: one unit per wave.
hipError_t launch_diff(const DevRegion* regs, uint32_t n_regs, uint64_t u0, uint64_t u1,
                       uint8_t* unit_flags, int blocks, int nontemporal, int prio,
                       hipStream_t s, const uint64_t* cand = nullptr,
                       uint64_t* stamp = nullptr, int group = 1);
hipError_t launch_bitmap(const DevRegion* regs, uint32_t n_regs, uint64_t w0, uint64_t w1,
                         const uint8_t* unit_flags, uint64_t* bitmap, hipStream_t s);
// Scans words [w0, w1) continuing glob->running; writes the new running total
// to *bounds_out when non-null.  With `final`, also fills the results of
// requests [q0, q1) (whose words must all have been scanned), lays their
// images out from glob->img_next and applies the capacity check: a group that
// does not fit, and every later group, gets CRUM_ENOSPC.  With `list`, also
// writes the slot list of the words (as launch_list): inside the scan kernel
// when the range takes one pass, else by a launch_list behind it.
hipError_t launch_scan(const uint64_t* bitmap, uint64_t w0, uint64_t w1, uint64_t n_words_total,
                       uint32_t* prefix, uint64_t* bounds_out, int final, const DevRequest* reqs,
                       uint32_t q0, uint32_t q1, DevReqOut* out, DevGlobal* glob,
                       uint64_t capacity, int restore_mode, uint32_t* list, hipStream_t s);
hipError_t launch_list(const uint64_t* bitmap, const uint32_t* prefix, uint64_t w0, uint64_t w1,
                       uint32_t* list, hipStream_t s);
// Pack, verify and scatter work on (slot, piece) items: a page of 2^ps bytes
// is cut into pieces of 2^min(ps, piece_shift) bytes, np_shift is log2 of the
// largest piece count per slot in the launch, and finalize combines the piece
// CRCs of pages larger than one piece.  depth: 16-byte loads in flight per
// lane (4, 8 or 16).  variant (0..5): how the CRC step splits its table
// lookups between byte and nibble tables.  Pack updates the shadows of regions whose flags bit 0
// is set.  unit_flags (pack only, may be null): the diff's per-unit flags of
// the same page space; units flagged clean are then read from the shadow.
// nt_store: bit 0 (pack only) writes the image with non-temporal stores;
// bit 1 issues each lane's next loads before folding the current ones.
hipError_t launch_pack(int mode, const DevRegion* regs, uint32_t n_regs, const DevRequest* reqs,
                       const DevReqOut* out, const uint32_t* list, SlotRange range,
                       uint32_t np_shift, uint32_t piece_shift, const uint8_t* unit_flags,
                       uint8_t* staging, uint32_t* crc_out, uint32_t* partials,
                       const CrcTables* tabs, DevGlobal* glob, int blocks, int depth,
                       int variant, hipStream_t s, int nt_store = 0);
hipError_t launch_finalize(int mode, const DevRegion* regs, uint32_t n_regs,
                           const DevRequest* reqs, const DevReqOut* out, const uint32_t* list,
                           SlotRange range, uint32_t np_shift, uint32_t piece_shift,
                           const uint32_t* partials, uint32_t* crc_out, uint8_t* staging,
                           DevGlobal* glob, const CrcTables* tabs, hipStream_t s);
// Workgroups per request for launch_header and launch_restore_check, from
// the request's region count, bitmap words and (a bound on) its CRC count.
uint32_t header_blocks(uint64_t n_regions, uint64_t n_words, uint64_t n_crcs);
// `blocks` workgroups per request of [q0, q1).  Requests with ENOSPC get only
// their prefix (header, table, bitmap), and only when it fits within
// `capacity`.
hipError_t launch_header(const DevRegion* regs, const DevRequest* reqs, uint32_t q0, uint32_t q1,
                         uint32_t blocks, DevReqOut* out, const uint64_t* bitmap,
                         const uint32_t* crcs, uint8_t* staging, uint64_t capacity,
                         const CrcTables* tabs, hipStream_t s);
// Resets the launch-wide counters (graph-safe: a kernel, not a memset).
hipError_t launch_plan_init(DevGlobal* glob, hipStream_t s);
// Compact per-request results: {code, first_bad, n_dirty, total_pages,
// image_bytes, image_offset} (40 bytes each) for requests [0, n).
hipError_t launch_plan_status(const DevReqOut* out, uint32_t n, uint8_t* dst, hipStream_t s);
// The image checks that need its bytes (bitmap population and unused bits,
// zero pads, crcs_crc, meta_crc), `blocks` workgroups per request; a failure
// sets glob->fmt_bad.  out[q].acc must be zero.
hipError_t launch_restore_check(const DevRequest* reqs, uint32_t n_reqs, uint32_t blocks,
                                DevReqOut* out, const uint8_t* staging, const CrcTables* tabs,
                                DevGlobal* glob, hipStream_t s);
hipError_t launch_scatter(const DevRegion* regs, uint32_t n_regs, const DevRequest* reqs,
                          const DevReqOut* out, const uint32_t* list, uint64_t n_slots,
                          uint32_t np_shift, uint32_t piece_shift, const uint8_t* staging,
                          int update_shadow,
                          const DevGlobal* glob, int blocks, hipStream_t s);
hipError_t launch_restore_finish(DevReqOut* out, uint32_t n_reqs, DevGlobal* glob,
                                 hipStream_t s);

}  // namespace crum
