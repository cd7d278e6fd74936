// On-demand (lazy) restore of an image.
//
// Section 4.2 fills the application's copy of a unified-memory region on read
// faults: a small region is read whole at its first fault; in a large region
// the first fault reads the page holding the faulting address and each later
// fault of that region reads twice as many pages as the one before.  Here the
// device takes no page faults (XNACK is off), so the caller announces each
// access with crum_lazy_touch.  The packed pages of the image are "absent"
// until fetched; a touch that reaches an absent page is a fault, whose window
// starts at the first absent page it reaches, spans max(2^f, pages to the end
// of the access) pages (f: the region's earlier faults), clipped at the
// region's end, or the whole region when the region is small.  The absent
// image pages of the window are fetched in runs of consecutive slots: one
// host-to-device copy of the run's packed pages into the staging buffer (at
// their offsets in the image layout), the CRC check of the run (with
// CRUM_VERIFY) and the scatter of the run into the regions.  Runs of up to
// 2 MiB skip the copy: when the host image is device-mapped pinned memory,
// their check and scatter read the packed pages from it in place.
//
// Open uploads only the image prefix (header, table, bitmap) and the CRC
// array, checks them on the device as a full restore does and builds the
// slot -> page list; the host keeps the bitmap with per-word slot prefixes to
// map a page range to its slots, and one bit per page for "fetched".
//
// The host-to-device copies run on the context's side stream (creating a
// stream per session costs more than the rest of open), and the caller's
// stream waits for each touch's copies before its checks and scatters: the copies of the next fault then overlap the kernels of this
// one.  Every run has its own slots of the staging buffer, so a copy never
// overwrites bytes a kernel still reads.  The checks and scatter of a short
// run cut its pages into smaller pieces, so that it still spreads over many
// waves (the piece CRCs are combined as for large pages).
#include "crum.h"
#include "crum_dev.h"
#include "crum_internal.h"
#include "gf2.h"

#include <cstring>
#include <vector>

using namespace crum;

struct crum_lazy {
    crum_ctx* ctx = nullptr;
    int device = 0;
    std::vector<crum_region> regions;
    std::vector<uint64_t> first_page;  // per region, global page of its page 0
    std::vector<uint32_t> faults;      // per region
    ImageInfo info;
    const uint8_t* h_image = nullptr;
    uint64_t image_bytes = 0;
    uint8_t* staging = nullptr;
    uint32_t flags = 0;
    uint64_t small_bytes = 0;
    uint32_t pc_shift = 0, np_shift = 0;
    int pack_blocks = 0, depth = 4, variant = kCrcVariantAuto, pack_flags = 0;
    std::vector<uint64_t> bitmap;   // image bitmap, W words
    std::vector<uint64_t> prefix;   // slots before word w
    std::vector<uint64_t> fetched;  // bit per page: its fetch has been enqueued
    crum_lazy_info st{};
    // device scratch: regs | req | out (+ glob) | prefix | list | partials | crcs
    uint8_t* d_mem = nullptr;
    size_t o_regs = 0, o_req = 0, o_out = 0, o_glob = 0, o_prefix = 0, o_list = 0,
           o_partials = 0, o_crcs = 0, upload_end = 0;
    uint8_t* h_up = nullptr;  // pinned upload of the tables
    bool borrowed = false;    // d_mem and h_up are the context's lazy scratch
    bool host_mapped = false; // the device maps h_image at the same address
    hipStream_t copy = nullptr;  // the context's side stream
    hipEvent_t ev_done = nullptr;    // the last call's work on the caller's stream
    hipStream_t done_stream = nullptr;  // the stream ev_done was last recorded on
    hipEvent_t ev_copied = nullptr;  // the last touch's copies
};

namespace {

size_t take(size_t* off, size_t bytes)
{
    const size_t o = *off;
    *off = round_up(*off + bytes, 256);
    return o;
}

void lazy_free(crum_lazy* z)
{
    if (z->borrowed) {
        z->ctx->lazy_busy = false;
    } else {
        if (z->d_mem)
            (void)hipFree(z->d_mem);
        if (z->h_up)
            (void)hipHostFree(z->h_up);
    }
    if (z->ev_done)
        (void)hipEventDestroy(z->ev_done);
    if (z->ev_copied)
        (void)hipEventDestroy(z->ev_copied);
    delete z;
}

int open_fail(crum_status* st, int code, const ImageInfo& I, uint64_t n)
{
    st->code = code;
    st->first_bad = 0;
    st->n_dirty = I.D;
    st->total_pages = I.G;
    st->image_bytes = n;
    return code;
}

// Slot of image page g (g's bit set in the bitmap).
uint64_t slot_of(const crum_lazy* z, uint64_t g)
{
    const uint64_t w = g >> 6;
    const uint64_t below = z->bitmap[w] & ((1ull << (g & 63)) - 1);
    return z->prefix[w] + (uint64_t)__builtin_popcountll(below);
}

// Waves a run's checks and scatter should spread over: a wave works through
// its piece one 1 KiB step after another, so a run of a few 64 KiB pages in
// whole-page pieces takes tens of microseconds; pieces are made smaller (down
// to 4 KiB) until the run has about this many.
constexpr uint64_t kRunWaves = 1024;

// Log2 of the piece size for a run of n slots: the context's piece size (at
// most a page), halved while the run has fewer than kRunWaves pieces.  A
// halved run has fewer than 2 * kRunWaves pieces.
uint32_t run_piece_shift(const crum_lazy* z, uint64_t n)
{
    const uint32_t ps = z->info.ps;
    uint32_t pcs = std::min(z->pc_shift, ps);
    while (pcs > kPieceShiftMin && (n << (ps - pcs)) < kRunWaves)
        --pcs;
    return pcs;
}

// Runs of at most this many packed bytes are checked and scattered straight
// from the pinned host image (the kernels read it over the host link): a
// copy to staging and the wait for it cost more than the transfer itself.
constexpr uint64_t kInPlaceRunBytes = 2ull << 20;

// Checks and scatter of slots [k0, k1), whose packed pages are at their
// image offsets from `src` (the staging buffer, or the host image itself).
hipError_t run_kernels(crum_lazy* z, uint64_t k0, uint64_t k1, uint8_t* src, hipStream_t s)
{
    const uint32_t ps = z->info.ps;
    const uint64_t n = k1 - k0;
    const uint32_t pcs = run_piece_shift(z, n);
    const uint32_t nps = ps > pcs ? ps - pcs : 0;
    uint8_t* M = z->d_mem;
    const DevRegion* regs = reinterpret_cast<const DevRegion*>(M + z->o_regs);
    const DevRequest* req = reinterpret_cast<const DevRequest*>(M + z->o_req);
    DevReqOut* out = reinterpret_cast<DevReqOut*>(M + z->o_out);
    DevGlobal* glob = reinterpret_cast<DevGlobal*>(M + z->o_glob);
    const uint32_t* list = reinterpret_cast<const uint32_t*>(M + z->o_list);
    uint32_t* partials = reinterpret_cast<uint32_t*>(M + z->o_partials);
    uint32_t* crcs = reinterpret_cast<uint32_t*>(M + z->o_crcs);
    const uint32_t nr = (uint32_t)z->regions.size();
    hipError_t e;
    if (z->flags & CRUM_VERIFY) {
        const SlotRange sr{k0, k1, nullptr, 0, n};
        e = launch_pack(kModeVerify, regs, nr, req, out, list, sr, nps, pcs,
                        nullptr, src, crcs, partials, ctx_tables(z->ctx), glob,
                        z->pack_blocks, z->depth, z->variant, s, z->pack_flags & 2);
        if (e != hipSuccess)
            return e;
        e = launch_finalize(kModeVerify, regs, nr, req, out, list, sr, nps, pcs,
                            partials, crcs, src, glob, ctx_tables(z->ctx), s);
        if (e != hipSuccess)
            return e;
    }
    // the scatter numbers slots from the list pointer and finds a slot's
    // packed page from the source pointer, so both start at slot k0
    return launch_scatter(regs, nr, req, out, list + k0, n, nps, pcs, src + (k0 << ps),
                          (z->flags & CRUM_UPDATE_SHADOW) ? 1 : 0, glob, z->pack_blocks, s);
}

// Fetch every absent image page of global pages [g0, g1): the copies of the
// runs that are not read in place on the copy stream, then on `s` a wait for
// them and each run's kernels.  Returns the pages enqueued in *pages and the
// runs in *runs.
hipError_t fetch_window(crum_lazy* z, uint64_t g0, uint64_t g1, hipStream_t s, uint64_t* pages,
                        uint64_t* runs)
{
    *pages = 0;
    *runs = 0;
    if (g1 <= g0)
        return hipSuccess;
    std::vector<std::pair<uint64_t, uint64_t>> rs;  // runs of slots [first, second)
    for (uint64_t w = g0 >> 6; w <= (g1 - 1) >> 6; ++w) {
        uint64_t m = z->bitmap[w] & ~z->fetched[w];
        if (w == g0 >> 6)
            m &= ~0ull << (g0 & 63);
        if (w == (g1 - 1) >> 6 && (g1 & 63))
            m &= (1ull << (g1 & 63)) - 1;
        while (m) {
            const uint32_t b = (uint32_t)__builtin_ctzll(m);
            m &= m - 1;
            const uint64_t g = (w << 6) | b;
            const uint64_t k = slot_of(z, g);
            if (!rs.empty() && rs.back().second == k)
                ++rs.back().second;
            else
                rs.emplace_back(k, k + 1);
            z->fetched[w] |= 1ull << b;
            ++*pages;
        }
    }
    if (rs.empty())
        return hipSuccess;
    const ImageInfo& I = z->info;
    uint8_t* host = const_cast<uint8_t*>(z->h_image);  // read only
    auto in_place = [&](const std::pair<uint64_t, uint64_t>& r) {
        return z->host_mapped && ((r.second - r.first) << I.ps) <= kInPlaceRunBytes;
    };
    bool copied = false;
    hipError_t e = hipSuccess;
    for (const auto& r : rs) {
        if (in_place(r))
            continue;
        const uint64_t off = I.data_off + (r.first << I.ps);
        e = hipMemcpyAsync(z->staging + off, z->h_image + off, (r.second - r.first) << I.ps,
                           hipMemcpyHostToDevice, z->copy);
        if (e != hipSuccess)
            return e;
        copied = true;
    }
    if (copied) {
        e = hipEventRecord(z->ev_copied, z->copy);
        if (e == hipSuccess)
            e = hipStreamWaitEvent(s, z->ev_copied, 0);
        if (e != hipSuccess)
            return e;
    }
    for (const auto& r : rs) {
        e = run_kernels(z, r.first, r.second, in_place(r) ? host : z->staging, s);
        if (e != hipSuccess)
            return e;
    }
    *runs = rs.size();
    return hipSuccess;
}

// Status of the session after the work enqueued so far, into h_status (the
// status is cumulative, so nothing is enqueued without a destination).
hipError_t enqueue_status(crum_lazy* z, crum_status* h_status, hipStream_t s)
{
    if (!h_status)
        return hipSuccess;
    DevReqOut* out = reinterpret_cast<DevReqOut*>(z->d_mem + z->o_out);
    DevGlobal* glob = reinterpret_cast<DevGlobal*>(z->d_mem + z->o_glob);
    hipError_t e = launch_restore_finish(out, 1, glob, s);
    if (e != hipSuccess)
        return e;
    return hipMemcpyAsync(h_status, out, sizeof(crum_status), hipMemcpyDeviceToHost, s);
}

// Order `s` after the session's earlier work: nothing to do on the stream
// that work was enqueued on.
hipError_t wait_done(crum_lazy* z, hipStream_t s)
{
    return s == z->done_stream ? hipSuccess : hipStreamWaitEvent(s, z->ev_done, 0);
}

hipError_t record_done(crum_lazy* z, hipStream_t s)
{
    hipError_t e = hipEventRecord(z->ev_done, s);
    if (e == hipSuccess)
        z->done_stream = s;
    return e;
}

}  // namespace

extern "C" {

int crum_lazy_open(crum_ctx* c, const crum_region* regions, uint32_t n_regions,
                   const void* h_image, uint64_t image_bytes, uint32_t flags,
                   uint64_t small_bytes, void* d_staging, uint64_t staging_bytes, void* stream_,
                   crum_status* h_status, crum_lazy** out)
{
    if (!out)
        return CRUM_EINVAL;
    *out = nullptr;
    if (!c || !h_status || !h_image || (n_regions && !regions) || !d_staging ||
        (reinterpret_cast<uintptr_t>(d_staging) & 15u) ||
        (flags & ~(uint32_t)(CRUM_UPDATE_SHADOW | CRUM_VERIFY)))
        return CRUM_EINVAL;
    if (check_ranges(regions, n_regions) != CRUM_OK)
        return CRUM_EINVAL;
    hipStream_t stream = static_cast<hipStream_t>(stream_);
    DeviceGuard g(ctx_device(c));

    // ---- host-side checks: the full restore's, then the bitmap itself (the
    // host maps pages to slots with it)
    const uint8_t* h = static_cast<const uint8_t*>(h_image);
    ImageInfo I;
    const int rc = parse_image_prefix(h, image_bytes, image_bytes, regions, n_regions, &I);
    if (rc != CRUM_OK)
        return open_fail(h_status, rc, I, image_bytes);
    if (staging_bytes < image_bytes)
        return open_fail(h_status, CRUM_ENOSPC, I, image_bytes);
    const uint64_t W = I.W, G = I.G, D = I.D;
    std::vector<uint64_t> bm(std::max<uint64_t>(W, 1), 0);
    if (W)
        std::memcpy(bm.data(), h + 64 + 32 * I.R, 8 * W);
    std::vector<uint64_t> prefix(std::max<uint64_t>(W, 1), 0);
    uint64_t pop = 0;
    for (uint64_t w = 0; w < W; ++w) {
        prefix[w] = pop;
        pop += (uint64_t)__builtin_popcountll(bm[w]);
    }
    if (pop != D || ((G & 63) && W && (bm[W - 1] >> (G & 63))))
        return open_fail(h_status, CRUM_EFORMAT, I, image_bytes);

    crum_lazy* z = new crum_lazy();
    z->ctx = c;
    z->device = ctx_device(c);
    z->copy = ctx_side_stream(c);
    z->regions.assign(regions, regions + n_regions);
    z->faults.assign(n_regions, 0);
    uint64_t page = 0;
    for (uint32_t i = 0; i < n_regions; ++i) {
        z->first_page.push_back(page);
        page += regions[i].len >> I.ps;
    }
    z->info = I;
    z->h_image = h;
    z->image_bytes = image_bytes;
    {
        hipPointerAttribute_t a{};
        z->host_mapped = hipPointerGetAttributes(&a, h_image) == hipSuccess &&
                         a.type == hipMemoryTypeHost && a.devicePointer == h_image;
        (void)hipGetLastError();
    }
    z->staging = static_cast<uint8_t*>(d_staging);
    z->flags = flags;
    z->small_bytes = small_bytes;
    z->pc_shift = ctx_piece_shift(c);
    z->np_shift = I.ps > z->pc_shift ? I.ps - z->pc_shift : 0;
    z->pack_blocks = ctx_shape(c).pack_blocks;
    z->depth = ctx_pack_depth(c);
    z->pack_flags = ctx_pack_flags(c);
    z->variant = ctx_crc_variant(c);
    z->bitmap = std::move(bm);
    z->prefix = std::move(prefix);
    z->fetched.assign(std::max<uint64_t>(W, 1), 0);
    z->st.pages_total = D;

    size_t off = 0;
    z->o_regs = take(&off, 64ull * std::max<uint32_t>(1, n_regions));
    z->o_req = take(&off, 64);
    z->o_out = take(&off, 128);
    z->o_glob = z->o_out + 64;
    z->upload_end = off;
    z->o_prefix = take(&off, 4 * std::max<uint64_t>(W, 1));
    z->o_list = take(&off, 4 * std::max<uint64_t>(W * 64, 1));
    z->o_partials = take(&off, 4 * std::max<uint64_t>(D << z->np_shift, 2 * kRunWaves));
    z->o_crcs = take(&off, 4 * std::max<uint64_t>(D, 1));
    if (!c->lazy_busy) {
        // the context's scratch: free while no session holds it, so a
        // session that closed has finished with it (close waits)
        z->borrowed = true;
        c->lazy_busy = true;
        if (c->lazy_d_cap < off) {
            if (c->lazy_d)
                (void)hipFree(c->lazy_d);
            c->lazy_d = nullptr;
            c->lazy_d_cap = 0;
            const size_t cap = round_up(off + off / 4, 1 << 20);
            if (hipMalloc(reinterpret_cast<void**>(&c->lazy_d), cap) == hipSuccess)
                c->lazy_d_cap = cap;
        }
        if (c->lazy_h_cap < z->upload_end) {
            if (c->lazy_h)
                (void)hipHostFree(c->lazy_h);
            c->lazy_h = nullptr;
            c->lazy_h_cap = 0;
            const size_t cap = round_up(z->upload_end + z->upload_end / 4, 1 << 16);
            if (hipHostMalloc(reinterpret_cast<void**>(&c->lazy_h), cap, 0) == hipSuccess)
                c->lazy_h_cap = cap;
        }
        z->d_mem = c->lazy_d_cap >= off ? c->lazy_d : nullptr;
        z->h_up = c->lazy_h_cap >= z->upload_end ? c->lazy_h : nullptr;
        if (!z->d_mem || !z->h_up) {
            lazy_free(z);
            return CRUM_EHIP;
        }
    } else if (hipMalloc(reinterpret_cast<void**>(&z->d_mem), off) != hipSuccess ||
               hipHostMalloc(reinterpret_cast<void**>(&z->h_up), z->upload_end, 0) !=
                   hipSuccess) {
        lazy_free(z);
        return CRUM_EHIP;
    }
    if (hipEventCreateWithFlags(&z->ev_done, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&z->ev_copied, hipEventDisableTiming) != hipSuccess) {
        lazy_free(z);
        return CRUM_EHIP;
    }

    uint8_t* P = z->h_up;
    std::memset(P, 0, z->upload_end);
    std::vector<DevRegion> dregs(std::max<uint32_t>(1, n_regions));
    uint64_t n_pages = 0, n_units = 0;
    flatten_regions(regions, n_regions, I.ps, ctx_unit_shift_max(c), 0, dregs.data(), &n_pages,
                    &n_units);
    std::memcpy(P + z->o_regs, dregs.data(), sizeof(DevRegion) * n_regions);
    DevRequest rq{};
    rq.n_words = W;
    rq.n_pages = G;
    rq.n_regions = n_regions;
    rq.data_off = I.data_off;
    rq.seq = I.seq;
    rq.page_shift = I.ps;
    rq.init_fix = crc_init_fix(I.page_size);
    std::memcpy(P + z->o_req, &rq, sizeof(rq));
    DevReqOut o{};
    o.n_dirty = D;
    o.total_pages = G;
    o.image_bytes = image_bytes;
    std::memcpy(P + z->o_out, &o, sizeof(o));
    DevGlobal gl{};
    gl.crc_bad = kNoBad;
    std::memcpy(P + z->o_glob, &gl, sizeof(gl));

    uint8_t* M = z->d_mem;
    const DevRequest* d_req = reinterpret_cast<const DevRequest*>(M + z->o_req);
    DevReqOut* d_out = reinterpret_cast<DevReqOut*>(M + z->o_out);
    DevGlobal* d_glob = reinterpret_cast<DevGlobal*>(M + z->o_glob);
    uint32_t* d_prefix = reinterpret_cast<uint32_t*>(M + z->o_prefix);
    uint32_t* d_list = reinterpret_cast<uint32_t*>(M + z->o_list);
    const uint64_t* img_bitmap =
        reinterpret_cast<const uint64_t*>(z->staging + 64 + 32 * I.R);
    const uint64_t pages_end = I.data_off + (D << I.ps);
    auto fail = [&]() {
        (void)hipStreamSynchronize(stream);
        lazy_free(z);
        return CRUM_EHIP;
    };
    if (hipMemcpyAsync(M, P, z->upload_end, hipMemcpyHostToDevice, stream) != hipSuccess ||
        hipMemcpyAsync(z->staging, h, I.data_off, hipMemcpyHostToDevice, stream) != hipSuccess ||
        hipMemcpyAsync(z->staging + pages_end, h + pages_end, image_bytes - pages_end,
                       hipMemcpyHostToDevice, stream) != hipSuccess ||
        launch_restore_check(d_req, 1, header_blocks(n_regions, W, D), d_out, z->staging,
                             ctx_tables(c), d_glob, stream) !=
            hipSuccess ||
        launch_scan(img_bitmap, 0, W, W, d_prefix, nullptr, 1, d_req, 0, 1, d_out, d_glob, 0, 1,
                    d_list, stream) != hipSuccess ||
        enqueue_status(z, h_status, stream) != hipSuccess ||
        record_done(z, stream) != hipSuccess ||
        // page copies start after everything the caller enqueued before
        // open (the image may have been drained on `stream`)
        hipStreamWaitEvent(z->copy, z->ev_done, 0) != hipSuccess)
        return fail();
    *out = z;
    return CRUM_OK;
}

int crum_lazy_touch(crum_lazy* z, uint32_t region, uint64_t offset, uint64_t len, void* stream_,
                    crum_status* h_status, uint64_t* n_fetched)
{
    if (n_fetched)
        *n_fetched = 0;
    if (!z || region >= z->regions.size() || len == 0)
        return CRUM_EINVAL;
    const uint64_t rlen = z->regions[region].len;
    if (offset > rlen || len > rlen - offset)
        return CRUM_EINVAL;
    hipStream_t stream = static_cast<hipStream_t>(stream_);
    DeviceGuard g(z->device);
    // the caller's work after this call sees every fetch enqueued before it
    CRUM_TRY_C(wait_done(z, stream));

    const uint32_t ps = z->info.ps;
    const uint64_t base = z->first_page[region];
    const uint64_t lo = base + (offset >> ps);
    const uint64_t hi = base + ((offset + len - 1) >> ps) + 1;
    // first absent image page the access reaches
    uint64_t first_absent = hi;
    for (uint64_t w = lo >> 6; w <= (hi - 1) >> 6 && first_absent == hi; ++w) {
        uint64_t m = z->bitmap[w] & ~z->fetched[w];
        if (w == lo >> 6)
            m &= ~0ull << (lo & 63);
        if (w == (hi - 1) >> 6 && (hi & 63))
            m &= (1ull << (hi & 63)) - 1;
        if (m)
            first_absent = (w << 6) | (uint64_t)__builtin_ctzll(m);
    }
    if (first_absent == hi)
        return CRUM_OK;  // not a fault: nothing enqueued, *h_status untouched

    const uint64_t region_end = base + (rlen >> ps);
    uint64_t w0, w1;
    if (rlen <= z->small_bytes) {
        w0 = base;
        w1 = region_end;
    } else {
        const uint32_t f = z->faults[region];
        const uint64_t span = f >= 63 ? ~0ull : (1ull << f);
        w0 = first_absent;
        w1 = std::max(span > region_end - w0 ? region_end : w0 + span, hi);
        w1 = std::min(w1, region_end);
    }
    uint64_t pages = 0, runs = 0;
    CRUM_TRY_C(fetch_window(z, w0, w1, stream, &pages, &runs));
    CRUM_TRY_C(enqueue_status(z, h_status, stream));
    CRUM_TRY_C(record_done(z, stream));
    ++z->faults[region];
    z->st.faults += 1;
    z->st.pages_fetched += pages;
    z->st.copies += runs;
    z->st.bytes_fetched += pages << ps;
    if (n_fetched)
        *n_fetched = pages;
    return CRUM_OK;
}

int crum_lazy_finish(crum_lazy* z, void* stream_, crum_status* h_status)
{
    if (!z || !h_status)
        return CRUM_EINVAL;
    hipStream_t stream = static_cast<hipStream_t>(stream_);
    DeviceGuard g(z->device);
    CRUM_TRY_C(wait_done(z, stream));
    uint64_t pages = 0, runs = 0;
    CRUM_TRY_C(fetch_window(z, 0, z->info.G, stream, &pages, &runs));
    CRUM_TRY_C(enqueue_status(z, h_status, stream));
    CRUM_TRY_C(record_done(z, stream));
    z->st.pages_fetched += pages;
    z->st.copies += runs;
    z->st.bytes_fetched += pages << z->info.ps;
    return CRUM_OK;
}

int crum_lazy_stats(crum_lazy* z, crum_lazy_info* out)
{
    if (!z || !out)
        return CRUM_EINVAL;
    *out = z->st;
    return CRUM_OK;
}

int crum_lazy_fetched(crum_lazy* z, uint64_t* words, uint64_t n_words)
{
    if (!z || (n_words && !words))
        return CRUM_EINVAL;
    const uint64_t n = std::min<uint64_t>(n_words, z->info.W);
    if (n)
        std::memcpy(words, z->fetched.data(), 8 * n);
    for (uint64_t w = n; w < n_words; ++w)
        words[w] = 0;
    return CRUM_OK;
}

void crum_lazy_close(crum_lazy* z)
{
    if (!z)
        return;
    DeviceGuard g(z->device);
    (void)hipEventSynchronize(z->ev_done);
    (void)hipStreamSynchronize(z->copy);
    lazy_free(z);
}

}  // extern "C"
