// Snapshot without allocation, for callers that cannot allocate (code under
// HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).
//
// It computes what crum_snapshot computes (same kernels, same image), in the
// diff-first order: the whole diff, the scan with the capacity check, one
// read-back of the dirty count, the compaction list, one pack launch over all
// dirty pages, the header, and one copy of the whole image to h_image.  Its
// device scratch (region table, unit flags, bitmap, prefix sums, slot list,
// CRC array, piece CRCs, counters) is the file-scope array below, of
// CRUM_NOALLOC_SCRATCH_BYTES bytes: one copy per device, held until the
// process ends, its address taken once per device when a context is created
// there.  Uploads and the count read-back go through a small pinned buffer
// that the context allocates when it is created.  Nothing is allocated per
// call: no hipMalloc, hipHostMalloc, event or stream creation.
//
// Every call on a device uses that device's one array: calls that overlap on
// one device (through different contexts, or one context from several
// threads) race.  Consecutive calls through one context are ordered by the
// context's completion event.
#include "crum.h"
#include "crum_dev.h"
#include "crum_internal.h"
#include "gf2.h"

#include <algorithm>
#include <cstring>
#include <mutex>
#include <utility>

using namespace crum;

namespace {

static __device__ __align__(256) uint8_t scratch[CRUM_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
uint8_t* g_ptr[kMaxDevices] = {};

// Offsets of one call's data in the scratch array (256-byte aligned pieces).
struct NaLayout {
    uint64_t regs = 0, reqs = 0, out = 0, glob = 0, upload_end = 0;
    uint64_t flags = 0, bitmap = 0, prefix = 0, list = 0, crcs = 0, partials = 0, bounds = 0;
    uint64_t total = 0;
};

NaLayout na_layout(uint64_t n_regs, uint64_t n_units, uint64_t n_words, uint64_t partial_cap)
{
    NaLayout L;
    uint64_t off = 0;
    auto take = [&](uint64_t bytes) {
        const uint64_t o = off;
        off = round_up(off + bytes, 256);
        return o;
    };
    L.regs = take(64 * std::max<uint64_t>(1, n_regs));
    L.reqs = take(64);
    L.out = take(128);
    L.glob = L.out + 64;
    L.upload_end = off;
    L.flags = take(std::max<uint64_t>(n_units, 1));
    L.bitmap = take(8 * std::max<uint64_t>(n_words, 1));
    L.prefix = take(4 * std::max<uint64_t>(n_words, 1));
    L.list = take(4 * 64 * std::max<uint64_t>(n_words, 1));
    L.crcs = take(4 * 64 * std::max<uint64_t>(n_words, 1));
    L.partials = take(4 * std::max<uint64_t>(partial_cap, 1));
    L.bounds = take(8);
    L.total = off;
    return L;
}

// The pointer rules of crum_snapshot (16-byte alignment, no current or
// shadow range overlapping another) without allocating: the intervals are
// sorted in `buf`, room for 2 * n of them.
int check_ranges_in(const crum_region* regs, uint32_t n, std::pair<uintptr_t, uintptr_t>* buf)
{
    size_t k = 0;
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
        buf[k++] = {b, b + r.len};
        if (r.shadow) {
            const uintptr_t s = reinterpret_cast<uintptr_t>(r.shadow);
            if (s + r.len < s)
                return CRUM_EINVAL;
            buf[k++] = {s, s + r.len};
        }
    }
    std::sort(buf, buf + k);
    for (size_t i = 1; i < k; ++i)
        if (buf[i].first < buf[i - 1].second)
            return CRUM_EINVAL;
    return CRUM_OK;
}

}  // namespace

namespace crum {

// The scratch array's address on `device`, which must be the current device
// (each device holds its own copy of the array at its own address).  Taken
// once per device; called when a context is created.
int noalloc_scratch(int device, uint8_t** out)
{
    *out = nullptr;
    if (device < 0 || device >= kMaxDevices)
        return CRUM_EINVAL;
    std::lock_guard<std::mutex> g(g_mu);
    if (!g_ptr[device]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p)
            return CRUM_EHIP;
        g_ptr[device] = static_cast<uint8_t*>(p);
    }
    *out = g_ptr[device];
    return CRUM_OK;
}

}  // namespace crum

extern "C" {

int crum_snapshot_noalloc(crum_ctx* c, const crum_region* regions, uint32_t n_regions,
                          uint32_t page_size, uint32_t flags, uint64_t seq, void* d_staging,
                          uint64_t staging_bytes, void* h_image, uint64_t h_image_bytes,
                          void* stream_, crum_status* h_status)
{
    // ---- synchronous argument checks, as crum_snapshot's
    if (!c || !h_status || (n_regions && !regions) || !d_staging ||
        (reinterpret_cast<uintptr_t>(d_staging) & 15u) || !page_size_ok(page_size) ||
        (flags & ~(uint32_t)CRUM_UPDATE_SHADOW))
        return CRUM_EINVAL;
    if (n_regions > CRUM_NOALLOC_MAX_REGIONS)
        return CRUM_ELIMIT;
    if (!c->na_scratch || !c->na_pin)
        return CRUM_EHIP;
    const uint32_t ps = (uint32_t)log2_exact(page_size);
    for (uint32_t i = 0; i < n_regions; ++i)
        if (regions[i].len % page_size)
            return CRUM_EINVAL;
    // the sort's room: the top of the pinned buffer, which no copy touches
    auto* iv = reinterpret_cast<std::pair<uintptr_t, uintptr_t>*>(c->na_pin + kNoAllocSortOff);
    if (check_ranges_in(regions, n_regions, iv) != CRUM_OK)
        return CRUM_EINVAL;
    uint64_t G = 0;
    for (uint32_t i = 0; i < n_regions; ++i)
        G += regions[i].len >> ps;
    if (G > 0xFFFFFF00ull)
        return CRUM_EINVAL;
    const uint64_t W = (G + 63) / 64;
    const uint64_t data_off = round_up(64 + 32ull * n_regions + 8 * W, 4096);
    if (staging_bytes < data_off || (h_image && h_image_bytes < data_off))
        return CRUM_EINVAL;
    const uint64_t capacity = h_image ? std::min(staging_bytes, h_image_bytes) : staging_bytes;

    // ---- the fixed limits
    const uint32_t pc_shift = c->piece_shift;
    const uint32_t np_shift = ps > pc_shift ? ps - pc_shift : 0;
    const uint32_t us = std::min<uint32_t>(ps, c->unit_shift_max);
    uint64_t n_units = 0;
    for (uint32_t i = 0; i < n_regions; ++i)
        n_units += regions[i].len >> us;
    const NaLayout L = na_layout(n_regions, n_units, W, np_shift ? (W * 64) << np_shift : 0);
    if (L.total > CRUM_NOALLOC_SCRATCH_BYTES)
        return CRUM_ELIMIT;
    const uint64_t rb_off = round_up(L.upload_end, 256);
    static_assert(64 * CRUM_NOALLOC_MAX_REGIONS + 1024 <= kNoAllocSortOff,
                  "upload and read-back below the sort's room");
    static_assert(kNoAllocSortOff + 2 * CRUM_NOALLOC_MAX_REGIONS * 16 <= kNoAllocPinnedBytes,
                  "sort room inside the pinned buffer");

    hipStream_t stream = static_cast<hipStream_t>(stream_);
    DeviceGuard g(c->device);
    // the previous upload from the pinned buffer must have left it
    CRUM_TRY_C(hipEventSynchronize(c->ev_upload));
    uint8_t* P = c->na_pin;
    std::memset(P, 0, L.upload_end);
    uint64_t n_pages = 0, n_units2 = 0;
    flatten_regions(regions, n_regions, ps, c->unit_shift_max,
                    (flags & CRUM_UPDATE_SHADOW) ? 1u : 0u,
                    reinterpret_cast<DevRegion*>(P + L.regs), &n_pages, &n_units2);
    DevRequest rq{};
    rq.first_word = 0;
    rq.n_words = W;
    rq.n_pages = G;
    rq.first_region = 0;
    rq.n_regions = n_regions;
    rq.data_off = data_off;
    rq.seq = seq;
    rq.page_shift = ps;
    rq.init_fix = crc_init_fix(page_size);
    std::memcpy(P + L.reqs, &rq, sizeof(rq));
    DevGlobal gl{};
    gl.crc_bad = kNoBad;
    std::memcpy(P + L.glob, &gl, sizeof(gl));

    uint8_t* S = c->na_scratch;
    const DevRegion* d_regs = reinterpret_cast<const DevRegion*>(S + L.regs);
    const DevRequest* d_reqs = reinterpret_cast<const DevRequest*>(S + L.reqs);
    DevReqOut* d_out = reinterpret_cast<DevReqOut*>(S + L.out);
    DevGlobal* d_glob = reinterpret_cast<DevGlobal*>(S + L.glob);
    uint8_t* d_flags = S + L.flags;
    uint64_t* d_bitmap = reinterpret_cast<uint64_t*>(S + L.bitmap);
    uint32_t* d_prefix = reinterpret_cast<uint32_t*>(S + L.prefix);
    uint32_t* d_list = reinterpret_cast<uint32_t*>(S + L.list);
    uint32_t* d_crcs = reinterpret_cast<uint32_t*>(S + L.crcs);
    uint32_t* d_partials = reinterpret_cast<uint32_t*>(S + L.partials);
    uint64_t* d_bounds = reinterpret_cast<uint64_t*>(S + L.bounds);
    uint8_t* staging = static_cast<uint8_t*>(d_staging);
    uint8_t* rb = P + rb_off;
    const uint32_t hdr_blocks = header_blocks(n_regions, W, G);

    // after this context's previous call (whose kernels may still use the array)
    c->partial_call = true;
    CRUM_TRY_C(hipStreamWaitEvent(stream, c->ev_done, 0));
    CRUM_TRY_C(hipMemcpyAsync(S, P, L.upload_end, hipMemcpyHostToDevice, stream));
    CRUM_TRY_C(hipEventRecord(c->ev_upload, stream));
    CRUM_TRY_C(launch_diff(d_regs, n_regions, 0, n_units, d_flags, c->shape.diff_blocks,
                           c->diff_nt, c->diff_prio, stream, nullptr, nullptr,
                           ctx_diff_group(c, us)));
    CRUM_TRY_C(launch_bitmap(d_regs, n_regions, 0, W, d_flags, d_bitmap, stream));
    CRUM_TRY_C(launch_scan(d_bitmap, 0, W, W, d_prefix, d_bounds, 1, d_reqs, 0, 1, d_out, d_glob,
                           capacity, 0, nullptr, stream));
    CRUM_TRY_C(hipMemcpyAsync(rb, d_out, 128, hipMemcpyDeviceToHost, stream));
    CRUM_TRY_C(hipEventRecord(c->ev_count, stream));
    CRUM_TRY_C(hipEventSynchronize(c->ev_count));
    DevReqOut o;
    std::memcpy(&o, rb, sizeof(o));
    uint64_t copy_bytes = 0;  // ENOSPC: the prefix stays in staging, as crum_snapshot's
    if (o.code == CRUM_OK) {
        const uint64_t D = o.n_dirty;
        if (D) {
            CRUM_TRY_C(launch_list(d_bitmap, d_prefix, 0, W, d_list, stream));
            const SlotRange sr{0, D, nullptr, 0, D};
            CRUM_TRY_C(launch_pack(kModePack, d_regs, n_regions, d_reqs, d_out, d_list, sr,
                                   np_shift, pc_shift, d_flags, staging, d_crcs, d_partials,
                                   c->d_tabs, d_glob, c->shape.pack_blocks, c->pack_depth,
                                   c->crc_variant, stream, ctx_pack_flags(c)));
            CRUM_TRY_C(launch_finalize(kModePack, d_regs, n_regions, d_reqs, d_out, d_list, sr,
                                       np_shift, pc_shift, d_partials, d_crcs, staging, d_glob,
                                       c->d_tabs, stream));
        }
        copy_bytes = o.image_bytes;
    }
    CRUM_TRY_C(launch_header(d_regs, d_reqs, 0, 1, hdr_blocks, d_out, d_bitmap, d_crcs, staging,
                             capacity, c->d_tabs, stream));
    if (h_image && copy_bytes)
        CRUM_TRY_C(hipMemcpyAsync(h_image, staging, copy_bytes, hipMemcpyDeviceToHost, stream));
    CRUM_TRY_C(hipMemcpyAsync(h_status, d_out, sizeof(crum_status), hipMemcpyDeviceToHost,
                              stream));
    CRUM_TRY_C(hipEventRecord(c->ev_done, stream));
    c->partial_call = false;
    return CRUM_OK;
}

}  // extern "C"
