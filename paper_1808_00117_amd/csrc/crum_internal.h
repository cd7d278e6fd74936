// Internal host-side definitions shared by the C-ABI sources of libcrum.
#pragma once
#include "crum.h"
#include "crum_dev.h"

#include <algorithm>
#include <string>
#include <utility>
#include <vector>

namespace crum {

constexpr int kTimingClasses = 7;
// Pinned buffer of crum_snapshot_noalloc, allocated with the context: the
// upload (region table, request, counters) and read-back below
// kNoAllocSortOff, the argument check's interval sort above it.
constexpr uint64_t kNoAllocSortOff = 160ull << 10;
constexpr uint64_t kNoAllocPinnedBytes = 256ull << 10;
// Address of crum_snapshot_noalloc's device scratch on `device` (current).
int noalloc_scratch(int device, uint8_t** out);

// Tuned shapes of one workload class from the shape tuner's cache: kind 0 =
// single snapshots of page_size bytes, kind 1 = plans; the class holds calls
// whose scanned bytes N satisfy 2^log2_bytes <= N < 2^(log2_bytes+1).
struct TunedClass {
    int kind = 0;
    uint32_t page_size = 0;
    uint32_t log2_bytes = 0;
    std::vector<std::pair<int, uint64_t>> params;  // CRUM_PARAM_* id, value
};
// Reads the classes of `device_key` from the cache file (crum_tune.hip).
int tune_load(const char* path, const std::string& device_key, std::vector<TunedClass>* out);
const TunedClass* tune_find(const std::vector<TunedClass>& v, int kind, uint32_t page_size,
                            uint64_t bytes);
// crum_ctx_set_param without marking the parameter as set by the caller.
int set_param_raw(crum_ctx* c, int param, uint64_t v);
// The tuner's device key of `device` (crum_capi.hip).
int device_key(int device, std::string* out);
enum { kTDiff = 0, kTPack = 1, kTDrain = 2, kTScan = 3, kTHeader = 4, kTVerify = 5, kTScatter = 6 };

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev)
    {
        if (hipGetDevice(&prev) != hipSuccess)
            prev = -1;
        if (prev != dev)
            (void)hipSetDevice(dev);
    }
    ~DeviceGuard()
    {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev)
            (void)hipSetDevice(prev);
    }
};

inline uint64_t round_up(uint64_t x, uint64_t a) { return (x + a - 1) / a * a; }

inline int log2_exact(uint64_t p)
{
    int s = 0;
    while ((1ull << s) < p)
        ++s;
    return s;
}

inline bool page_size_ok(uint64_t p) { return p >= 4096 && p <= (1ull << 30) && (p & (p - 1)) == 0; }


// Pointer rules shared by snapshot and restore: non-empty regions have a
// base, every pointer is 16-byte aligned, and no current or shadow range
// overlaps another.
inline int check_ranges(const crum_region* regs, uint32_t n)
{
    std::vector<std::pair<uintptr_t, uintptr_t>> iv;
    iv.reserve(2 * (size_t)n);
    for (uint32_t i = 0; i < n; ++i) {
        const crum_region& r = regs[i];
        if ((reinterpret_cast<uintptr_t>(r.base) & 15u) ||
            (reinterpret_cast<uintptr_t>(r.shadow) & 15u))
            return CRUM_EINVAL;
        if (r.len == 0)
            continue;
        if (!r.base)
            return CRUM_EINVAL;
        const uintptr_t b = reinterpret_cast<uintptr_t>(r.base);
        if (b + r.len < b)
            return CRUM_EINVAL;
        iv.emplace_back(b, b + r.len);
        if (r.shadow) {
            const uintptr_t s = reinterpret_cast<uintptr_t>(r.shadow);
            if (s + r.len < s)
                return CRUM_EINVAL;
            iv.emplace_back(s, s + r.len);
        }
    }
    std::sort(iv.begin(), iv.end());
    for (size_t i = 1; i < iv.size(); ++i)
        if (iv[i].first < iv[i - 1].second)
            return CRUM_EINVAL;
    return CRUM_OK;
}


// One region table as DevRegion entries of request 0: global first page and
// first diff unit of each region (table order), diff unit
// 2^min(ps, us_max), region_flags in every entry.
void flatten_regions(const crum_region* regs, uint32_t n, uint32_t ps, uint32_t us_max,
                     uint32_t region_flags, DevRegion* out, uint64_t* n_pages, uint64_t* n_units);

// Fields of an image header that passed the host-side checks.
struct ImageInfo {
    uint32_t page_size = 0, ps = 0;
    uint64_t R = 0, G = 0, D = 0, seq = 0, data_off = 0, W = 0;
};

// Host-side checks of an image's header and region table against the
// caller's table: magic, version, page size, flags, sizes and offsets, the
// chaining of first_page, then count, lengths and ids.  `avail` bytes are
// readable at h.  Returns CRUM_OK, CRUM_EFORMAT or CRUM_EMISMATCH; G and D
// are filled once the header fields are read.
int parse_image_prefix(const uint8_t* h, uint64_t avail, uint64_t image_bytes,
                       const crum_region* regions, uint32_t n_regions, ImageInfo* out);

}  // namespace crum

struct crum_ctx {
    using CrcTables = crum::CrcTables;
    using LaunchShape = crum::LaunchShape;
    int device = 0;
    int cus = 256;
    hipStream_t side = nullptr;
    CrcTables* d_tabs = nullptr;
    uint8_t* d_scratch = nullptr;
    size_t scratch_cap = 0;
    uint8_t* h_pin = nullptr;  // uploads, then readback area
    size_t pin_cap = 0;
    hipEvent_t ev_upload = nullptr, ev_count = nullptr, ev_done = nullptr, ev_hdr = nullptr;
    std::vector<hipEvent_t> ev_chunk;  // pack of chunk i done
    std::vector<hipEvent_t> ev_cnt;    // dirty count of chunk i read back
    LaunchShape shape{};
    uint64_t chunk_bytes = 128ull << 20;
    uint64_t chunk_max_bytes = 4ull << 30;
    uint32_t unit_shift_max = crum::kUnitShiftDefault;
    bool diff_nt = true;
    uint64_t drain_chunk_bytes = 8ull << 20;
    uint32_t piece_shift = crum::kPieceShiftDefault;
    int pack_depth = 4;
    int diff_prio = 0;
    int crc_variant = crum::kCrcVariantAuto;
    int plan_order = 0;
    uint64_t direct_bytes = 0;  // opt-in: worst-case images up to this size go straight to the host
    uint32_t chunk_growth = 4;  // growth factor of pipelined chunks and plan groups
    bool pack_nt = false;       // non-temporal image stores in the pack
    bool pack_ntl = true;       // pack/verify: non-temporal page loads
    uint8_t diff_group = 2;     // diff: 4 KiB units per wave (1, 2 or 4)
    bool pack_pf = false;       // pack/verify: next loads issued before folding the current
    // tuned shapes per workload class (crum_ctx_create's tuning cache), applied
    // to a call's parameters that crum_ctx_set_param has not set
    std::vector<crum::TunedClass> tuned;
    uint64_t explicit_params = 0;  // bit p: parameter p set by crum_ctx_set_param
    bool eager = true;
    uint32_t timing_mask = 0;  // bit c: time launches of class c
    bool partial_call = false;  // a call stopped part-way through its enqueue
    std::vector<hipEvent_t> pool;
    size_t pool_used = 0;
    // scratch of on-demand restore sessions, lent to one open session at a
    // time (allocating per session costs more than the rest of opening one)
    uint8_t* lazy_d = nullptr;
    size_t lazy_d_cap = 0;
    uint8_t* lazy_h = nullptr;  // pinned
    size_t lazy_h_cap = 0;
    bool lazy_busy = false;
    // crum_snapshot_noalloc: the device's static scratch and a pinned buffer
    uint8_t* na_scratch = nullptr;
    uint8_t* na_pin = nullptr;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> spans[crum::kTimingClasses];
    // launches timed elsewhere (inside a plan's graphs), already summed
    uint64_t extra_n[crum::kTimingClasses] = {};
    double extra_ms[crum::kTimingClasses] = {};
};


namespace crum {

// Accessors used by the batched-plan code.
using DeviceGuardC = DeviceGuard;
inline bool ctx_page_size_ok(uint64_t p) { return page_size_ok(p); }
inline int ctx_log2(uint64_t p) { return log2_exact(p); }
inline int ctx_check_ranges(const crum_region* r, uint32_t n) { return check_ranges(r, n); }
inline uint32_t ctx_unit_shift_max(const crum_ctx* c) { return c->unit_shift_max; }
inline uint64_t ctx_chunk_bytes(const crum_ctx* c) { return c->chunk_bytes; }
inline uint64_t ctx_chunk_max_bytes(const crum_ctx* c) { return c->chunk_max_bytes; }
inline int ctx_device(const crum_ctx* c) { return c->device; }
inline LaunchShape ctx_shape(const crum_ctx* c) { return c->shape; }
inline const CrcTables* ctx_tables(const crum_ctx* c) { return c->d_tabs; }
inline int ctx_diff_nt(const crum_ctx* c) { return c->diff_nt ? 1 : 0; }
inline hipStream_t ctx_side_stream(const crum_ctx* c) { return c->side; }
inline uint32_t ctx_piece_shift(const crum_ctx* c) { return c->piece_shift; }
inline int ctx_pack_depth(const crum_ctx* c) { return c->pack_depth; }
inline int ctx_diff_prio(const crum_ctx* c) { return c->diff_prio; }
inline int ctx_crc_variant(const crum_ctx* c) { return c->crc_variant; }
inline int ctx_plan_order(const crum_ctx* c) { return c->plan_order; }
inline bool ctx_times(const crum_ctx* c, int cls) { return (c->timing_mask >> cls) & 1u; }
inline void ctx_add_timing(crum_ctx* c, int cls, double ms)
{
    c->extra_n[cls] += 1;
    c->extra_ms[cls] += ms;
}
inline uint32_t ctx_chunk_growth(const crum_ctx* c) { return c->chunk_growth; }
inline int ctx_pack_nt(const crum_ctx* c) { return c->pack_nt ? 1 : 0; }
// launch_pack's flag bits: 1 non-temporal image stores, 2 prefetching loop
// bit 0: non-temporal image stores; bit 1: next loads issued early (cached
// loads only); bit 2: non-temporal page loads
// Units per wave of a diff launch whose smallest unit is 1 << min_us bytes:
// the context's group for 4 KiB units, else one.
inline int ctx_diff_group(const crum_ctx* c, uint32_t min_us)
{
    return min_us == 12 ? c->diff_group : 1;
}
inline int ctx_pack_flags(const crum_ctx* c)
{
    return (c->pack_nt ? 1 : 0) | (c->pack_pf ? 2 : 0) | (c->pack_ntl ? 4 : 0);
}

// Applies the context's tuned shapes for one call's workload class, for the
// duration of the call (a context is used by one thread at a time), to the
// parameters the caller has not set explicitly; restores them afterwards.
// No allocation.
class TunedScope {
public:
    TunedScope(crum_ctx* c, int kind, uint32_t page_size, uint64_t bytes);
    ~TunedScope();
    TunedScope(const TunedScope&) = delete;
    TunedScope& operator=(const TunedScope&) = delete;

private:
    crum_ctx* c_;
    int n_ = 0;
    int id_[32];
    uint64_t old_[32];
};

}  // namespace crum

#define CRUM_TRY_C(expr)                        \
    do {                                        \
        hipError_t e_ = (expr);                 \
        if (e_ != hipSuccess)                   \
            return CRUM_EHIP;                   \
    } while (0)
