// Host runtime and C ABI of libcrum: argument validation, flattening of the
// region table, scratch management, stream/event orchestration of the
// snapshot and restore pipelines, and the chunked drain.
#include "crum.h"
#include "crum_dev.h"
#include "crum_internal.h"
#include "gf2.h"

#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <utility>
#include <vector>

using namespace crum;

namespace {


// Scratch layout of one launch (offsets into ctx->d_scratch).
struct Layout {
    size_t regs = 0, reqs = 0, out = 0, glob = 0, cand = 0, upload_end = 0;
    size_t flags = 0, bitmap = 0, prefix = 0, list = 0, crcs = 0, partials = 0, bounds = 0,
           total = 0;
};

Layout make_layout(uint32_t n_regs, uint32_t n_reqs, uint64_t n_units, uint64_t n_words,
                   uint64_t list_cap, uint64_t partial_cap, uint64_t n_chunks,
                   uint64_t cand_words = 0)
{
    Layout L;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = round_up(off + bytes, 256);
        return o;
    };
    L.regs = take(64ull * std::max<uint32_t>(1, n_regs));
    L.reqs = take(64ull * n_reqs);
    L.out = take(64ull * n_reqs + 64);
    L.glob = L.out + 64ull * n_reqs;
    L.cand = take(8 * cand_words);
    L.upload_end = off;
    L.flags = take(std::max<uint64_t>(n_units, 1));
    L.bitmap = take(8 * std::max<uint64_t>(n_words, 1));
    L.prefix = take(4 * std::max<uint64_t>(n_words, 1));
    L.list = take(4 * std::max<uint64_t>(list_cap, 1));
    L.crcs = take(4 * std::max<uint64_t>(list_cap, 1));
    L.partials = take(4 * std::max<uint64_t>(partial_cap, 1));
    L.bounds = take(8 * std::max<uint64_t>(n_chunks, 1));
    L.total = off;
    return L;
}

}  // namespace

namespace {

hipEvent_t timing_event(crum_ctx* c)
{
    if (c->pool_used == c->pool.size()) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess)
            return nullptr;
        c->pool.push_back(e);
    }
    return c->pool[c->pool_used++];
}

// Brackets launches with timing events when the context measures.
struct Span {
    crum_ctx* c;
    int cls;
    hipStream_t s;
    hipEvent_t a = nullptr;
    Span(crum_ctx* c_, int cls_, hipStream_t s_) : c(c_), cls(cls_), s(s_)
    {
        if (((c->timing_mask >> cls) & 1u) && (a = timing_event(c)))
            (void)hipEventRecord(a, s);
    }
    void end()
    {
        if (!a)
            return;
        hipEvent_t b = timing_event(c);
        if (b && hipEventRecord(b, s) == hipSuccess)
            c->spans[cls].emplace_back(a, b);
        a = nullptr;
    }
    ~Span() { end(); }
};

// Grows the context's device scratch.  A call that enqueued all its work
// recorded ev_done after its last use of the scratch (kernels, read-backs and
// the status copy), so waiting for that is enough and other contexts on the
// device keep running; after a call that stopped part-way (a HIP error while
// enqueueing), the whole device is waited for.
hipError_t ensure_scratch(crum_ctx* c, size_t bytes)
{
    if (bytes <= c->scratch_cap)
        return hipSuccess;
    hipError_t e = c->partial_call ? hipDeviceSynchronize() : hipEventSynchronize(c->ev_done);
    if (e != hipSuccess)
        return e;
    if (c->d_scratch)
        (void)hipFree(c->d_scratch);
    c->d_scratch = nullptr;
    c->scratch_cap = 0;
    const size_t cap = round_up(bytes + bytes / 4, 1 << 20);
    e = hipMalloc(reinterpret_cast<void**>(&c->d_scratch), cap);
    if (e == hipSuccess)
        c->scratch_cap = cap;
    return e;
}

hipError_t ensure_pinned(crum_ctx* c, size_t bytes)
{
    if (bytes <= c->pin_cap)
        return hipSuccess;
    hipError_t e = c->partial_call ? hipDeviceSynchronize() : hipEventSynchronize(c->ev_upload);
    if (e != hipSuccess)
        return e;
    e = hipEventSynchronize(c->ev_done);
    if (e != hipSuccess)
        return e;
    if (c->h_pin)
        (void)hipHostFree(c->h_pin);
    c->h_pin = nullptr;
    c->pin_cap = 0;
    const size_t cap = round_up(bytes + bytes / 4, 1 << 16);
    e = hipHostMalloc(reinterpret_cast<void**>(&c->h_pin), cap, 0);
    if (e == hipSuccess)
        c->pin_cap = cap;
    return e;
}

hipError_t ensure_events(std::vector<hipEvent_t>& v, size_t n)
{
    while (v.size() < n) {
        hipEvent_t e;
        hipError_t err = hipEventCreateWithFlags(&e, hipEventDisableTiming);
        if (err != hipSuccess)
            return err;
        v.push_back(e);
    }
    return hipSuccess;
}

#define CRUM_TRY(expr)                          \
    do {                                        \
        hipError_t e_ = (expr);                 \
        if (e_ != hipSuccess)                   \
            return CRUM_EHIP;                   \
    } while (0)

}  // namespace

namespace crum {

static uint32_t rd32(const uint8_t* p)
{
    uint32_t v;
    std::memcpy(&v, p, 4);
    return v;
}

static uint64_t rd64(const uint8_t* p)
{
    uint64_t v;
    std::memcpy(&v, p, 8);
    return v;
}

// Flatten one table into DevRegion entries (single request, request 0).
void flatten_regions(const crum_region* regs, uint32_t n, uint32_t ps, uint32_t us_max,
                     uint32_t region_flags, DevRegion* out, uint64_t* n_pages, uint64_t* n_units)
{
    uint64_t page = 0, unit = 0;
    const uint32_t us = std::min<uint32_t>(ps, us_max);
    for (uint32_t i = 0; i < n; ++i) {
        DevRegion& d = out[i];
        d.cur = static_cast<const uint8_t*>(regs[i].base);
        d.shadow = static_cast<uint8_t*>(regs[i].shadow);
        d.len = regs[i].len;
        d.first_page = page;
        d.first_unit = unit;
        d.id = regs[i].id;
        d.page_shift = ps;
        d.req = 0;
        d.unit_shift = us;
        d.flags = region_flags;
        page += regs[i].len >> ps;
        unit += regs[i].len >> us;
    }
    *n_pages = page;
    *n_units = unit;
}

int parse_image_prefix(const uint8_t* h, uint64_t avail, uint64_t image_bytes,
                       const crum_region* regions, uint32_t n_regions, ImageInfo* out)
{
    *out = ImageInfo{};
    if (image_bytes < 64 || avail < 64)
        return CRUM_EFORMAT;
    if (std::memcmp(h, "CRUMIMG1", 8) != 0 || rd32(h + 8) != 1 || !page_size_ok(rd32(h + 12)) ||
        (rd32(h + 20) & ~1u))
        return CRUM_EFORMAT;
    ImageInfo& I = *out;
    I.page_size = rd32(h + 12);
    I.ps = (uint32_t)log2_exact(I.page_size);
    I.R = rd32(h + 16);
    I.G = rd64(h + 24);
    I.D = rd64(h + 32);
    I.seq = rd64(h + 40);
    I.data_off = rd64(h + 48);
    if (I.G > 0xFFFFFF00ull || I.D > I.G)
        return CRUM_EFORMAT;
    I.W = (I.G + 63) / 64;
    const uint64_t prefix_end = 64 + 32 * I.R + 8 * I.W;
    if (I.data_off != round_up(prefix_end, 4096) ||
        I.data_off + (I.D << I.ps) + round_up(4 * I.D, 8) != image_bytes)
        return CRUM_EFORMAT;
    if (I.R != n_regions)
        return CRUM_EMISMATCH;
    if (avail < 64 + 32 * I.R)
        return CRUM_EFORMAT;
    uint64_t chain = 0;
    bool mismatch = false;
    for (uint64_t i = 0; i < I.R; ++i) {
        const uint8_t* e = h + 64 + 32 * i;
        const uint64_t len = rd64(e + 8);
        if (rd64(e + 24) != 0 || len % I.page_size || rd64(e + 16) != chain)
            return CRUM_EFORMAT;
        chain += len >> I.ps;
        if (rd64(e) != regions[i].id || len != regions[i].len)
            mismatch = true;
    }
    if (chain != I.G)
        return CRUM_EFORMAT;
    return mismatch ? CRUM_EMISMATCH : CRUM_OK;
}

}  // namespace crum

extern "C" {

int crum_image_prefix_bytes(uint32_t n_regions, uint64_t total_pages, uint64_t* out)
{
    if (!out || total_pages > (1ull << 40))
        return CRUM_EINVAL;
    *out = round_up(64 + 32ull * n_regions + 8 * ((total_pages + 63) / 64), 4096);
    return CRUM_OK;
}

int crum_image_bytes(uint32_t n_regions, uint64_t total_pages, uint64_t n_dirty,
                     uint32_t page_size, uint64_t* out)
{
    uint64_t pre = 0;
    if (!out || !page_size_ok(page_size) || n_dirty > total_pages ||
        crum_image_prefix_bytes(n_regions, total_pages, &pre) != CRUM_OK)
        return CRUM_EINVAL;
    *out = pre + n_dirty * page_size + round_up(4 * n_dirty, 8);
    return CRUM_OK;
}

int crum_ctx_create(int device, const char* tuning_cache, crum_ctx** out)
{
    if (!out)
        return CRUM_EINVAL;
    *out = nullptr;
    int n_dev = 0;
    if (hipGetDeviceCount(&n_dev) != hipSuccess)
        return CRUM_EHIP;
    if (device < 0 || device >= n_dev)
        return CRUM_EINVAL;
    std::vector<TunedClass> tuned;
    if (tuning_cache) {
        std::string key;
        if (device_key(device, &key) != CRUM_OK)
            return CRUM_EHIP;
        if (tune_load(tuning_cache, key, &tuned) != CRUM_OK)
            return CRUM_EINVAL;
    }
    DeviceGuard g(device);
    crum_ctx* c = new crum_ctx();
    c->device = device;
    c->tuned = std::move(tuned);
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess &&
        cus > 0)
        c->cus = cus;
    c->shape.diff_blocks = c->cus * 8;
    c->shape.pack_blocks = c->cus * 4;
    CrcTables host;
    build_crc_tables(&host);
    bool ok = hipMalloc(reinterpret_cast<void**>(&c->d_tabs), sizeof(CrcTables)) == hipSuccess &&
              hipMemcpy(c->d_tabs, &host, sizeof(CrcTables), hipMemcpyHostToDevice) ==
                  hipSuccess &&
              hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking) == hipSuccess &&
              hipEventCreateWithFlags(&c->ev_upload, hipEventDisableTiming) == hipSuccess &&
              hipEventCreateWithFlags(&c->ev_count, hipEventDisableTiming) == hipSuccess &&
              hipEventCreateWithFlags(&c->ev_done, hipEventDisableTiming) == hipSuccess &&
              hipEventCreateWithFlags(&c->ev_hdr, hipEventDisableTiming) == hipSuccess &&
              hipHostMalloc(reinterpret_cast<void**>(&c->na_pin), kNoAllocPinnedBytes, 0) ==
                  hipSuccess &&
              noalloc_scratch(device, &c->na_scratch) == CRUM_OK;
    if (!ok) {
        crum_ctx_destroy(c);
        return CRUM_EHIP;
    }
    *out = c;
    return CRUM_OK;
}

void crum_ctx_destroy(crum_ctx* c)
{
    if (!c)
        return;
    DeviceGuard g(c->device);
    (void)hipDeviceSynchronize();
    for (hipEvent_t e : c->pool)
        (void)hipEventDestroy(e);
    for (hipEvent_t e : c->ev_chunk)
        (void)hipEventDestroy(e);
    for (hipEvent_t e : c->ev_cnt)
        (void)hipEventDestroy(e);
    for (hipEvent_t e : {c->ev_upload, c->ev_count, c->ev_done, c->ev_hdr})
        if (e)
            (void)hipEventDestroy(e);
    if (c->side)
        (void)hipStreamDestroy(c->side);
    if (c->d_tabs)
        (void)hipFree(c->d_tabs);
    if (c->d_scratch)
        (void)hipFree(c->d_scratch);
    if (c->h_pin)
        (void)hipHostFree(c->h_pin);
    if (c->na_pin)
        (void)hipHostFree(c->na_pin);
    if (c->lazy_d)
        (void)hipFree(c->lazy_d);
    if (c->lazy_h)
        (void)hipHostFree(c->lazy_h);
    delete c;
}

int crum_ctx_set_param(crum_ctx* c, int param, uint64_t v)
{
    const int rc = crum::set_param_raw(c, param, v);
    if (rc == CRUM_OK && param > 0 && param < 64)
        c->explicit_params |= 1ull << param;
    return rc;
}

int crum_ctx_tuned_classes(crum_ctx* c, uint32_t* n)
{
    if (!c || !n)
        return CRUM_EINVAL;
    *n = (uint32_t)c->tuned.size();
    return CRUM_OK;
}

int crum_tuning_check(const char* path, const char* device_key, uint32_t* n_classes)
{
    if (!path || !device_key)
        return CRUM_EINVAL;
    std::vector<TunedClass> v;
    const int rc = tune_load(path, device_key, &v);
    if (rc == CRUM_OK && n_classes)
        *n_classes = (uint32_t)v.size();
    return rc;
}

}  // extern "C"

namespace crum {

int set_param_raw(crum_ctx* c, int param, uint64_t v)
{
    if (!c)
        return CRUM_EINVAL;
    if (param == CRUM_PARAM_EAGER || param == CRUM_PARAM_DIFF_NONTEMPORAL ||
        param == CRUM_PARAM_PACK_NT_STORE || param == CRUM_PARAM_PACK_PREFETCH ||
        param == CRUM_PARAM_PACK_NT_LOAD) {
        if (v > 1)
            return CRUM_EINVAL;
        (param == CRUM_PARAM_EAGER                ? c->eager
         : param == CRUM_PARAM_DIFF_NONTEMPORAL ? c->diff_nt
         : param == CRUM_PARAM_PACK_NT_STORE    ? c->pack_nt
         : param == CRUM_PARAM_PACK_NT_LOAD     ? c->pack_ntl
                                                : c->pack_pf) = v != 0;
        return CRUM_OK;
    }
    if (param == CRUM_PARAM_DIFF_GROUP) {
        if (v != 1 && v != 2 && v != 4)
            return CRUM_EINVAL;
        c->diff_group = (uint8_t)v;
        return CRUM_OK;
    }
    if (param == CRUM_PARAM_CHUNK_GROWTH) {
        if (v < 2 || v > 16)
            return CRUM_EINVAL;
        c->chunk_growth = (uint32_t)v;
        return CRUM_OK;
    }
    if (param == CRUM_PARAM_DIFF_UNIT_SHIFT) {
        if (v < 12 || v > 14)
            return CRUM_EINVAL;
        c->unit_shift_max = (uint32_t)v;
        return CRUM_OK;
    }
    if (param == CRUM_PARAM_PIECE_SHIFT) {
        if (v < kPieceShiftMin || v > kPieceShift)
            return CRUM_EINVAL;
        c->piece_shift = (uint32_t)v;
        return CRUM_OK;
    }
    if (param == CRUM_PARAM_DIRECT_BYTES) {
        c->direct_bytes = v;
        return CRUM_OK;
    }
    if (param == CRUM_PARAM_PLAN_ORDER) {
        if (v > 1)
            return CRUM_EINVAL;
        c->plan_order = (int)v;
        return CRUM_OK;
    }
    if (param == CRUM_PARAM_CRC_VARIANT) {
        if (v > (uint64_t)kCrcVariantAuto)
            return CRUM_EINVAL;
        c->crc_variant = (int)v;
        return CRUM_OK;
    }
    if (param == CRUM_PARAM_DIFF_PRIORITY) {
        if (v > 3)
            return CRUM_EINVAL;
        c->diff_prio = (int)v;
        return CRUM_OK;
    }
    if (param == CRUM_PARAM_PACK_DEPTH) {
        if (v != 4 && v != 8 && v != 16)
            return CRUM_EINVAL;
        c->pack_depth = (int)v;
        return CRUM_OK;
    }
    if (v == 0)
        return CRUM_EINVAL;
    switch (param) {
    case CRUM_PARAM_DIFF_BLOCKS:
        if (v > (1u << 20))
            return CRUM_EINVAL;
        c->shape.diff_blocks = (int)v;
        return CRUM_OK;
    case CRUM_PARAM_PACK_BLOCKS:
        if (v > (1u << 20))
            return CRUM_EINVAL;
        c->shape.pack_blocks = (int)v;
        return CRUM_OK;
    case CRUM_PARAM_CHUNK_BYTES:
        c->chunk_bytes = v;
        return CRUM_OK;
    case CRUM_PARAM_CHUNK_MAX_BYTES:
        c->chunk_max_bytes = v;
        return CRUM_OK;
    case CRUM_PARAM_DRAIN_CHUNK_BYTES:
        c->drain_chunk_bytes = v;
        return CRUM_OK;
    default:
        return CRUM_EINVAL;
    }
}

TunedScope::TunedScope(crum_ctx* c, int kind, uint32_t page_size, uint64_t bytes) : c_(c)
{
    const TunedClass* t = tune_find(c->tuned, kind, page_size, bytes);
    if (!t)
        return;
    for (const auto& kv : t->params) {
        if (n_ == 32)
            break;
        if (kv.first > 0 && kv.first < 64 && ((c->explicit_params >> kv.first) & 1u))
            continue;
        uint64_t old = 0;
        if (crum_ctx_get_param(c, kv.first, &old) != CRUM_OK)
            continue;
        if (set_param_raw(c, kv.first, kv.second) == CRUM_OK) {
            id_[n_] = kv.first;
            old_[n_] = old;
            ++n_;
        }
    }
}

TunedScope::~TunedScope()
{
    for (int i = n_ - 1; i >= 0; --i)
        (void)set_param_raw(c_, id_[i], old_[i]);
}

// "cc<major>.<minor>-<CUs>cu|hip<runtime version>", as the shape tuner keys
// its cache.
int device_key(int device, std::string* out)
{
    int major = 0, minor = 0, cus = 0, ver = 0;
    if (hipDeviceGetAttribute(&major, hipDeviceAttributeComputeCapabilityMajor, device) !=
            hipSuccess ||
        hipDeviceGetAttribute(&minor, hipDeviceAttributeComputeCapabilityMinor, device) !=
            hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) !=
            hipSuccess ||
        hipRuntimeGetVersion(&ver) != hipSuccess)
        return CRUM_EHIP;
    *out = "cc" + std::to_string(major) + "." + std::to_string(minor) + "-" +
           std::to_string(cus) + "cu|hip" + std::to_string(ver);
    return CRUM_OK;
}

}  // namespace crum

extern "C" {

int crum_ctx_get_param(crum_ctx* c, int param, uint64_t* v)
{
    if (!c || !v)
        return CRUM_EINVAL;
    switch (param) {
    case CRUM_PARAM_DIFF_BLOCKS: *v = (uint64_t)c->shape.diff_blocks; return CRUM_OK;
    case CRUM_PARAM_PACK_BLOCKS: *v = (uint64_t)c->shape.pack_blocks; return CRUM_OK;
    case CRUM_PARAM_CHUNK_BYTES: *v = c->chunk_bytes; return CRUM_OK;
    case CRUM_PARAM_CHUNK_MAX_BYTES: *v = c->chunk_max_bytes; return CRUM_OK;
    case CRUM_PARAM_EAGER: *v = c->eager ? 1 : 0; return CRUM_OK;
    case CRUM_PARAM_DRAIN_CHUNK_BYTES: *v = c->drain_chunk_bytes; return CRUM_OK;
    case CRUM_PARAM_DIFF_UNIT_SHIFT: *v = c->unit_shift_max; return CRUM_OK;
    case CRUM_PARAM_DIFF_NONTEMPORAL: *v = c->diff_nt ? 1 : 0; return CRUM_OK;
    case CRUM_PARAM_PIECE_SHIFT: *v = c->piece_shift; return CRUM_OK;
    case CRUM_PARAM_PACK_DEPTH: *v = (uint64_t)c->pack_depth; return CRUM_OK;
    case CRUM_PARAM_DIFF_PRIORITY: *v = (uint64_t)c->diff_prio; return CRUM_OK;
    case CRUM_PARAM_CRC_VARIANT: *v = (uint64_t)c->crc_variant; return CRUM_OK;
    case CRUM_PARAM_PLAN_ORDER: *v = (uint64_t)c->plan_order; return CRUM_OK;
    case CRUM_PARAM_DIRECT_BYTES: *v = c->direct_bytes; return CRUM_OK;
    case CRUM_PARAM_CHUNK_GROWTH: *v = c->chunk_growth; return CRUM_OK;
    case CRUM_PARAM_PACK_NT_STORE: *v = c->pack_nt ? 1 : 0; return CRUM_OK;
    case CRUM_PARAM_PACK_PREFETCH: *v = c->pack_pf ? 1 : 0; return CRUM_OK;
    case CRUM_PARAM_PACK_NT_LOAD: *v = c->pack_ntl ? 1 : 0; return CRUM_OK;
    case CRUM_PARAM_DIFF_GROUP: *v = c->diff_group; return CRUM_OK;
    default: return CRUM_EINVAL;
    }
}

int crum_ctx_set_timing(crum_ctx* c, int classes)
{
    if (!c)
        return CRUM_EINVAL;
    c->timing_mask = classes < 0 ? (1u << kTimingClasses) - 1 : (uint32_t)classes;
    return CRUM_OK;
}

int crum_ctx_timing_reset(crum_ctx* c)
{
    if (!c)
        return CRUM_EINVAL;
    DeviceGuard g(c->device);
    for (auto& v : c->spans) {
        for (auto& p : v)
            if (hipEventSynchronize(p.second) != hipSuccess)
                return CRUM_EHIP;
        v.clear();
    }
    c->pool_used = 0;
    for (int k = 0; k < kTimingClasses; ++k) {
        c->extra_n[k] = 0;
        c->extra_ms[k] = 0;
    }
    return CRUM_OK;
}

int crum_ctx_timing(crum_ctx* c, int which, uint64_t* launches, double* total_ms)
{
    if (!c || which < 0 || which >= kTimingClasses || !launches || !total_ms)
        return CRUM_EINVAL;
    DeviceGuard g(c->device);
    double tot = 0;
    for (auto& p : c->spans[which]) {
        float ms = 0;
        if (hipEventSynchronize(p.second) != hipSuccess ||
            hipEventElapsedTime(&ms, p.first, p.second) != hipSuccess)
            return CRUM_EHIP;
        tot += ms;
    }
    *launches = c->spans[which].size() + c->extra_n[which];
    *total_ms = tot + c->extra_ms[which];
    return CRUM_OK;
}

static bool himg_ok_for_direct(const crum_ctx* c, const void* h_image, uint64_t worst)
{
    return h_image && c->direct_bytes && worst <= c->direct_bytes;
}

// The snapshot of crum_snapshot; h_cand (may be null) is the candidate
// bitmap of crum_snapshot_tracked, cand_words long.
static int snapshot_impl(crum_ctx* c, const crum_region* regions, uint32_t n_regions,
                         uint32_t page_size, uint32_t flags, uint64_t seq,
                         const uint64_t* h_cand, uint64_t cand_words, void* d_staging,
                         uint64_t staging_bytes, void* h_image, uint64_t h_image_bytes,
                         void* stream_, crum_status* h_status)
{
    // ---- synchronous argument checks (nothing enqueued on failure)
    if (!c || !h_status || (n_regions && !regions) || !d_staging ||
        (reinterpret_cast<uintptr_t>(d_staging) & 15u) || !page_size_ok(page_size) ||
        (flags & ~(uint32_t)CRUM_UPDATE_SHADOW))
        return CRUM_EINVAL;
    const uint32_t ps = (uint32_t)log2_exact(page_size);
    for (uint32_t i = 0; i < n_regions; ++i)
        if (regions[i].len % page_size)
            return CRUM_EINVAL;
    if (check_ranges(regions, n_regions) != CRUM_OK)
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
    if (h_cand && cand_words < W)
        return CRUM_EINVAL;
    const uint64_t capacity = h_image ? std::min(staging_bytes, h_image_bytes) : staging_bytes;
    // When every page fits, ENOSPC cannot happen and the page space is
    // processed in chunks whose drain overlaps the diff of later chunks.
    // Otherwise, or when the pages make a single chunk (nothing to overlap),
    // the whole diff and the capacity check come before any write.
    const uint64_t worst = data_off + (G << ps) + round_up(4 * G, 8);
    hipStream_t stream = static_cast<hipStream_t>(stream_);
    DeviceGuard g(c->device);
    const TunedScope tuned(c, 0, page_size, G << ps);
    // Small images may be built straight in the pinned host image (the pack
    // and header kernels write it over the host link): no staging, no drain
    // copy, and the host never waits on a dirty count.  Only for host memory
    // that the device maps at the same address.
    bool direct = false;
    if (himg_ok_for_direct(c, h_image, worst)) {
        hipPointerAttribute_t a{};
        direct = hipPointerGetAttributes(&a, h_image) == hipSuccess &&
                 a.type == hipMemoryTypeHost && a.devicePointer == h_image;
        (void)hipGetLastError();
    }
    bool eager = !direct && c->eager && capacity >= worst && G > 0;

    // ---- chunk plan (page ranges aligned to bitmap words)
    std::vector<uint64_t> cuts{0};
    if (eager) {
        uint64_t chunk_bytes = c->chunk_bytes;
        uint64_t gp = 0;
        while (gp < G) {
            const uint64_t pages = std::max<uint64_t>(64, (chunk_bytes >> ps) & ~63ull);
            gp = std::min(G, gp + pages);
            cuts.push_back(gp);
            chunk_bytes = std::min<uint64_t>(chunk_bytes * c->chunk_growth,
                                             std::max(c->chunk_max_bytes, c->chunk_bytes));
        }
    } else {
        cuts.push_back(G);
    }
    const size_t n_chunks = cuts.size() - 1;

    // ---- flatten, scratch, upload
    const uint32_t pc_shift = c->piece_shift;
    const uint32_t np_shift = ps > pc_shift ? ps - pc_shift : 0;
    const uint32_t us = std::min<uint32_t>(ps, c->unit_shift_max);
    std::vector<DevRegion> dregs(std::max<uint32_t>(1, n_regions));
    uint64_t n_pages = 0, n_units = 0;
    flatten_regions(regions, n_regions, ps, c->unit_shift_max,
                    (flags & CRUM_UPDATE_SHADOW) ? 1u : 0u, dregs.data(), &n_pages, &n_units);
    const Layout L = make_layout(n_regions, 1, n_units, W, W * 64, np_shift ? G << np_shift : 0,
                                 n_chunks, h_cand ? W : 0);
    CRUM_TRY(ensure_scratch(c, L.total));
    const size_t rb_off = round_up(L.upload_end, 256);
    CRUM_TRY(ensure_pinned(c, rb_off + 128 + 8 * n_chunks));
    CRUM_TRY(ensure_events(c->ev_chunk, n_chunks));
    CRUM_TRY(ensure_events(c->ev_cnt, n_chunks));
    CRUM_TRY(hipEventSynchronize(c->ev_upload));
    uint8_t* P = c->h_pin;
    std::memset(P, 0, L.upload_end);
    std::memcpy(P + L.regs, dregs.data(), sizeof(DevRegion) * n_regions);
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
    if (h_cand && W)
        std::memcpy(P + L.cand, h_cand, 8 * W);

    uint8_t* S = c->d_scratch;
    const uint64_t* d_cand = h_cand ? reinterpret_cast<const uint64_t*>(S + L.cand) : nullptr;
    const DevRegion* d_regs = reinterpret_cast<const DevRegion*>(S + L.regs);
    const DevRequest* d_reqs = reinterpret_cast<const DevRequest*>(S + L.reqs);
    DevReqOut* d_out = reinterpret_cast<DevReqOut*>(S + L.out);
    DevGlobal* d_glob = reinterpret_cast<DevGlobal*>(S + L.glob);
    const uint32_t hdr_blocks = header_blocks(n_regions, W, G);
    uint8_t* d_flags = S + L.flags;
    uint64_t* d_bitmap = reinterpret_cast<uint64_t*>(S + L.bitmap);
    uint32_t* d_prefix = reinterpret_cast<uint32_t*>(S + L.prefix);
    uint32_t* d_list = reinterpret_cast<uint32_t*>(S + L.list);
    uint32_t* d_crcs = reinterpret_cast<uint32_t*>(S + L.crcs);
    uint32_t* d_partials = reinterpret_cast<uint32_t*>(S + L.partials);
    uint64_t* d_bounds = reinterpret_cast<uint64_t*>(S + L.bounds);
    uint8_t* staging = static_cast<uint8_t*>(d_staging);
    uint8_t* himg = static_cast<uint8_t*>(h_image);
    uint8_t* rb = P + rb_off;

    // the previous call on this context may still be draining from scratch
    c->partial_call = true;  // cleared once ev_done is recorded
    CRUM_TRY(hipStreamWaitEvent(stream, c->ev_done, 0));
    CRUM_TRY(hipMemcpyAsync(S, P, L.upload_end, hipMemcpyHostToDevice, stream));
    CRUM_TRY(hipEventRecord(c->ev_upload, stream));

    if (direct) {
        // ---- direct order: diff, scan (with the capacity check), list, then
        // pack and header into the host image; slot counts stay on the device
        {
            Span sp(c, kTDiff, stream);
            CRUM_TRY(launch_diff(d_regs, n_regions, 0, n_units, d_flags, c->shape.diff_blocks,
                                 c->diff_nt, c->diff_prio, stream, d_cand, nullptr,
                                 ctx_diff_group(c, us)));
        }
        {
            Span sp(c, kTScan, stream);
            CRUM_TRY(launch_bitmap(d_regs, n_regions, 0, W, d_flags, d_bitmap, stream));
            CRUM_TRY(launch_scan(d_bitmap, 0, W, W, d_prefix, d_bounds, 1, d_reqs, 0, 1, d_out,
                                 d_glob, capacity, 0, d_list, stream));
        }
        {
            Span sp(c, kTPack, stream);
            SlotRange sr{0, 0, d_bounds, 0, G};
            CRUM_TRY(launch_pack(kModePack, d_regs, n_regions, d_reqs, d_out, d_list, sr,
                                 np_shift, pc_shift, d_flags, himg, d_crcs, d_partials,
                                 c->d_tabs, d_glob, c->shape.pack_blocks, c->pack_depth,
                                 c->crc_variant, stream, ctx_pack_flags(c)));
            sp.end();  // k_finalize is not part of the pack's timing
            CRUM_TRY(launch_finalize(kModePack, d_regs, n_regions, d_reqs, d_out, d_list, sr,
                                     np_shift, pc_shift, d_partials, d_crcs, himg, d_glob,
                                     c->d_tabs, stream));
        }
        {
            Span sp(c, kTHeader, stream);
            CRUM_TRY(launch_header(d_regs, d_reqs, 0, 1, hdr_blocks, d_out, d_bitmap, d_crcs,
                                   himg, capacity, c->d_tabs, stream));
        }
        CRUM_TRY(hipMemcpyAsync(h_status, d_out, sizeof(crum_status), hipMemcpyDeviceToHost,
                                stream));
        CRUM_TRY(hipEventRecord(c->ev_done, stream));
        c->partial_call = false;
        return CRUM_OK;
    }

    uint64_t D = 0, image_bytes = 0;
    if (eager) {
        // ---- enqueue every chunk: diff, bitmap, scan, count readback, list, pack
        for (size_t ci = 0; ci < n_chunks; ++ci) {
            const uint64_t g0 = cuts[ci], g1 = cuts[ci + 1];
            const uint64_t w0 = g0 / 64, w1 = (g1 + 63) / 64;
            {
                Span sp(c, kTDiff, stream);
                CRUM_TRY(launch_diff(d_regs, n_regions, g0 << (ps - us), g1 << (ps - us), d_flags,
                                     c->shape.diff_blocks, c->diff_nt, c->diff_prio, stream,
                                     d_cand, nullptr,
                                     ctx_diff_group(c, us)));
            }
            {
                Span sp(c, kTScan, stream);
                CRUM_TRY(launch_bitmap(d_regs, n_regions, w0, w1, d_flags, d_bitmap, stream));
                CRUM_TRY(launch_scan(d_bitmap, w0, w1, W, d_prefix, d_bounds + ci,
                                     ci + 1 == n_chunks, d_reqs, 0, 1, d_out, d_glob, capacity,
                                     0, d_list, stream));
            }
            CRUM_TRY(hipMemcpyAsync(rb + 128 + 8 * ci, d_bounds + ci, 8, hipMemcpyDeviceToHost,
                                    stream));
            CRUM_TRY(hipEventRecord(c->ev_cnt[ci], stream));
            {
                Span sp(c, kTPack, stream);
                SlotRange sr{0, 0, d_bounds, (uint32_t)ci, g1 - g0};
                CRUM_TRY(launch_pack(kModePack, d_regs, n_regions, d_reqs, d_out, d_list, sr,
                                     np_shift, pc_shift, d_flags, staging, d_crcs,
                                     d_partials, c->d_tabs, d_glob, c->shape.pack_blocks,
                                     c->pack_depth, c->crc_variant, stream, ctx_pack_flags(c)));
                sp.end();  // k_finalize is not part of the pack's timing
                CRUM_TRY(launch_finalize(kModePack, d_regs, n_regions, d_reqs, d_out, d_list, sr,
                                         np_shift, pc_shift, d_partials, d_crcs, staging, d_glob,
                                         c->d_tabs, stream));
            }
            CRUM_TRY(hipEventRecord(c->ev_chunk[ci], stream));
        }
        // the header takes its sizes from the device, so it follows the last
        // pack without waiting for the host
        {
            Span sp(c, kTHeader, stream);
            CRUM_TRY(launch_header(d_regs, d_reqs, 0, 1, hdr_blocks, d_out, d_bitmap, d_crcs,
                                   staging, capacity, c->d_tabs, stream));
        }
        // ---- drain each chunk as soon as its count is known (one chunk: the
        // whole image in one copy behind the header, below)
        uint64_t prev = 0;
        for (size_t ci = 0; ci < n_chunks; ++ci) {
            CRUM_TRY(hipEventSynchronize(c->ev_cnt[ci]));
            uint64_t cnt;
            std::memcpy(&cnt, rb + 128 + 8 * ci, 8);
            if (himg && cnt > prev && n_chunks > 1) {
                CRUM_TRY(hipStreamWaitEvent(c->side, c->ev_chunk[ci], 0));
                const uint64_t off = data_off + (prev << ps);
                Span sp(c, kTDrain, c->side);
                CRUM_TRY(hipMemcpyAsync(himg + off, staging + off, (cnt - prev) << ps,
                                        hipMemcpyDeviceToHost, c->side));
            }
            prev = cnt;
        }
        D = prev;
        image_bytes = data_off + (D << ps) + round_up(4 * D, 8);
    } else {
        // ---- checked order: whole diff, scan with the capacity check, readback
        {
            Span sp(c, kTDiff, stream);
            CRUM_TRY(launch_diff(d_regs, n_regions, 0, n_units, d_flags, c->shape.diff_blocks,
                                 c->diff_nt, c->diff_prio, stream, d_cand, nullptr,
                                 ctx_diff_group(c, us)));
        }
        {
            Span sp(c, kTScan, stream);
            CRUM_TRY(launch_bitmap(d_regs, n_regions, 0, W, d_flags, d_bitmap, stream));
            CRUM_TRY(launch_scan(d_bitmap, 0, W, W, d_prefix, d_bounds, 1, d_reqs, 0, 1, d_out,
                                 d_glob, capacity, 0, nullptr, stream));
        }
        CRUM_TRY(hipMemcpyAsync(rb, d_out, 128, hipMemcpyDeviceToHost, stream));
        CRUM_TRY(hipEventRecord(c->ev_count, stream));
        CRUM_TRY(hipEventSynchronize(c->ev_count));
        DevReqOut o;
        std::memcpy(&o, rb, sizeof(o));
        if (o.code != CRUM_OK) {
            // ENOSPC: header, table and bitmap only; nothing packed or drained
            Span sp(c, kTHeader, stream);
            CRUM_TRY(launch_header(d_regs, d_reqs, 0, 1, hdr_blocks, d_out, d_bitmap, d_crcs,
                                   staging, capacity, c->d_tabs, stream));
            sp.end();
            CRUM_TRY(hipMemcpyAsync(h_status, d_out, sizeof(crum_status), hipMemcpyDeviceToHost,
                                    stream));
            CRUM_TRY(hipEventRecord(c->ev_done, stream));
            c->partial_call = false;
            return CRUM_OK;
        }
        D = o.n_dirty;
        image_bytes = o.image_bytes;
        if (D) {
            Span sp(c, kTScan, stream);
            CRUM_TRY(launch_list(d_bitmap, d_prefix, 0, W, d_list, stream));
        }
        // pack in slot chunks with the drain of each behind it
        uint64_t k0 = 0;
        uint64_t chunk_bytes = c->drain_chunk_bytes;
        size_t ci = 0;
        while (k0 < D) {
            const uint64_t n_slots = std::max<uint64_t>(1, chunk_bytes >> ps);
            const uint64_t k1 = std::min(D, k0 + n_slots);
            {
                Span sp(c, kTPack, stream);
                SlotRange sr{k0, k1, nullptr, 0, k1 - k0};
                CRUM_TRY(launch_pack(kModePack, d_regs, n_regions, d_reqs, d_out, d_list, sr,
                                     np_shift, pc_shift, d_flags, staging, d_crcs,
                                     d_partials, c->d_tabs, d_glob, c->shape.pack_blocks,
                                     c->pack_depth, c->crc_variant, stream, ctx_pack_flags(c)));
                sp.end();  // k_finalize is not part of the pack's timing
                CRUM_TRY(launch_finalize(kModePack, d_regs, n_regions, d_reqs, d_out, d_list, sr,
                                         np_shift, pc_shift, d_partials, d_crcs, staging, d_glob,
                                         c->d_tabs, stream));
            }
            if (himg) {
                CRUM_TRY(ensure_events(c->ev_chunk, ci + 1));
                CRUM_TRY(hipEventRecord(c->ev_chunk[ci], stream));
                CRUM_TRY(hipStreamWaitEvent(c->side, c->ev_chunk[ci], 0));
                const uint64_t off = data_off + (k0 << ps);
                Span sp(c, kTDrain, c->side);
                CRUM_TRY(hipMemcpyAsync(himg + off, staging + off, (k1 - k0) << ps,
                                        hipMemcpyDeviceToHost, c->side));
            }
            ++ci;
            k0 = k1;
            chunk_bytes = std::min<uint64_t>(chunk_bytes * 2,
                                             std::max<uint64_t>(256ull << 20, chunk_bytes));
        }
    }

    // ---- header (with the CRC array; already enqueued in the chunked order),
    // then the prefix and tail of the drain
    if (!eager) {
        Span sp(c, kTHeader, stream);
        CRUM_TRY(launch_header(d_regs, d_reqs, 0, 1, hdr_blocks, d_out, d_bitmap, d_crcs,
                               staging, capacity, c->d_tabs, stream));
    }
    if (himg) {
        CRUM_TRY(hipEventRecord(c->ev_hdr, stream));
        CRUM_TRY(hipStreamWaitEvent(c->side, c->ev_hdr, 0));
        const uint64_t tail = data_off + (D << ps);
        Span sp(c, kTDrain, c->side);
        if (eager && n_chunks == 1) {
            CRUM_TRY(hipMemcpyAsync(himg, staging, image_bytes, hipMemcpyDeviceToHost, c->side));
        } else {
            CRUM_TRY(hipMemcpyAsync(himg, staging, data_off, hipMemcpyDeviceToHost, c->side));
            if (image_bytes > tail)
                CRUM_TRY(hipMemcpyAsync(himg + tail, staging + tail, image_bytes - tail,
                                        hipMemcpyDeviceToHost, c->side));
        }
        sp.end();
        CRUM_TRY(hipMemcpyAsync(h_status, d_out, sizeof(crum_status), hipMemcpyDeviceToHost,
                                c->side));
        CRUM_TRY(hipEventRecord(c->ev_done, c->side));
        c->partial_call = false;
        CRUM_TRY(hipStreamWaitEvent(stream, c->ev_done, 0));
    } else {
        CRUM_TRY(hipMemcpyAsync(h_status, d_out, sizeof(crum_status), hipMemcpyDeviceToHost,
                                stream));
        CRUM_TRY(hipEventRecord(c->ev_done, stream));
        c->partial_call = false;
    }
    return CRUM_OK;
}

int crum_snapshot(crum_ctx* c, const crum_region* regions, uint32_t n_regions,
                  uint32_t page_size, uint32_t flags, uint64_t seq, void* d_staging,
                  uint64_t staging_bytes, void* h_image, uint64_t h_image_bytes, void* stream_,
                  crum_status* h_status)
{
    return snapshot_impl(c, regions, n_regions, page_size, flags, seq, nullptr, 0, d_staging,
                         staging_bytes, h_image, h_image_bytes, stream_, h_status);
}

int crum_snapshot_tracked(crum_ctx* c, const crum_region* regions, uint32_t n_regions,
                          uint32_t page_size, uint32_t flags, uint64_t seq,
                          const uint64_t* h_candidates, uint64_t n_words, void* d_staging,
                          uint64_t staging_bytes, void* h_image, uint64_t h_image_bytes,
                          void* stream_, crum_status* h_status)
{
    if (!h_candidates)
        return CRUM_EINVAL;
    return snapshot_impl(c, regions, n_regions, page_size, flags, seq, h_candidates, n_words,
                         d_staging, staging_bytes, h_image, h_image_bytes, stream_, h_status);
}

static int restore_fail(crum_status* st, int code, uint64_t D, uint64_t G, uint64_t n)
{
    st->code = code;
    st->first_bad = 0;
    st->n_dirty = D;
    st->total_pages = G;
    st->image_bytes = n;
    return code;
}


int crum_restore(crum_ctx* c, const crum_region* regions, uint32_t n_regions,
                 const void* h_image, uint64_t image_bytes, uint32_t flags, void* d_staging,
                 uint64_t staging_bytes, void* stream_, crum_status* h_status)
{
    if (!c || !h_status || (n_regions && !regions) || !d_staging ||
        (reinterpret_cast<uintptr_t>(d_staging) & 15u) ||
        (flags & ~(uint32_t)(CRUM_UPDATE_SHADOW | CRUM_VERIFY)))
        return CRUM_EINVAL;
    if (check_ranges(regions, n_regions) != CRUM_OK)
        return CRUM_EINVAL;
    hipStream_t stream = static_cast<hipStream_t>(stream_);
    DeviceGuard g(c->device);

    // ---- host-side header and table checks
    std::vector<uint8_t> hdr_copy;
    const uint8_t* h = static_cast<const uint8_t*>(h_image);
    if (image_bytes < 64)
        return restore_fail(h_status, CRUM_EFORMAT, 0, 0, image_bytes);
    if (!h) {
        const uint64_t want = std::min<uint64_t>(image_bytes, 64 + 32ull * n_regions);
        hdr_copy.resize(want);
        CRUM_TRY(hipStreamSynchronize(stream));
        CRUM_TRY(hipMemcpy(hdr_copy.data(), d_staging, want, hipMemcpyDeviceToHost));
        h = hdr_copy.data();
    }
    ImageInfo info;
    const int rc = parse_image_prefix(h, hdr_copy.size() ? hdr_copy.size() : image_bytes,
                                      image_bytes, regions, n_regions, &info);
    const uint64_t G = info.G, D = info.D;
    if (rc != CRUM_OK)
        return restore_fail(h_status, rc, D, G, image_bytes);
    const uint32_t ps = info.ps;
    const uint64_t R = info.R, W = info.W, seq = info.seq, data_off = info.data_off;
    const uint32_t page_size = info.page_size;
    if (staging_bytes < image_bytes)
        return restore_fail(h_status, CRUM_ENOSPC, D, G, image_bytes);

    // ---- device tables
    const uint32_t pc_shift = c->piece_shift;
    const uint32_t np_shift = ps > pc_shift ? ps - pc_shift : 0;
    std::vector<DevRegion> dregs(std::max<uint32_t>(1, n_regions));
    uint64_t n_pages = 0, n_units = 0;
    flatten_regions(regions, n_regions, ps, c->unit_shift_max, 0, dregs.data(), &n_pages,
                    &n_units);
    const Layout L = make_layout(n_regions, 1, 0, W, W * 64, np_shift ? D << np_shift : 0, 1);
    CRUM_TRY(ensure_scratch(c, L.total));
    CRUM_TRY(ensure_pinned(c, L.upload_end));
    CRUM_TRY(hipEventSynchronize(c->ev_upload));
    uint8_t* P = c->h_pin;
    std::memset(P, 0, L.upload_end);
    std::memcpy(P + L.regs, dregs.data(), sizeof(DevRegion) * n_regions);
    DevRequest rq{};
    rq.n_words = W;
    rq.n_pages = G;
    rq.n_regions = n_regions;
    rq.data_off = data_off;
    rq.seq = seq;
    rq.page_shift = ps;
    rq.init_fix = crc_init_fix(page_size);
    std::memcpy(P + L.reqs, &rq, sizeof(rq));
    DevReqOut o{};
    o.n_dirty = D;
    o.total_pages = G;
    o.image_bytes = image_bytes;
    std::memcpy(P + L.out, &o, sizeof(o));
    DevGlobal gl{};
    gl.crc_bad = kNoBad;
    std::memcpy(P + L.glob, &gl, sizeof(gl));

    uint8_t* S = c->d_scratch;
    const DevRegion* d_regs = reinterpret_cast<const DevRegion*>(S + L.regs);
    const DevRequest* d_reqs = reinterpret_cast<const DevRequest*>(S + L.reqs);
    DevReqOut* d_out = reinterpret_cast<DevReqOut*>(S + L.out);
    DevGlobal* d_glob = reinterpret_cast<DevGlobal*>(S + L.glob);
    uint32_t* d_prefix = reinterpret_cast<uint32_t*>(S + L.prefix);
    uint32_t* d_list = reinterpret_cast<uint32_t*>(S + L.list);
    uint32_t* d_partials = reinterpret_cast<uint32_t*>(S + L.partials);
    uint32_t* d_crcs = reinterpret_cast<uint32_t*>(S + L.crcs);
    uint8_t* staging = static_cast<uint8_t*>(d_staging);
    const uint64_t* img_bitmap = reinterpret_cast<const uint64_t*>(staging + 64 + 32 * R);

    c->partial_call = true;
    CRUM_TRY(hipStreamWaitEvent(stream, c->ev_done, 0));
    CRUM_TRY(hipMemcpyAsync(S, P, L.upload_end, hipMemcpyHostToDevice, stream));
    CRUM_TRY(hipEventRecord(c->ev_upload, stream));
    if (h_image)
        CRUM_TRY(hipMemcpyAsync(staging, h_image, image_bytes, hipMemcpyHostToDevice, stream));
    {
        Span sp(c, kTScan, stream);
        CRUM_TRY(launch_restore_check(d_reqs, 1, header_blocks(n_regions, W, D), d_out, staging,
                                      c->d_tabs, d_glob, stream));
        CRUM_TRY(launch_scan(img_bitmap, 0, W, W, d_prefix, nullptr, 1, d_reqs, 0, 1, d_out,
                             d_glob, 0, 1, d_list, stream));
    }
    if (flags & CRUM_VERIFY) {
        Span sp(c, kTVerify, stream);
        SlotRange sr{0, D, nullptr, 0, D};
        CRUM_TRY(launch_pack(kModeVerify, d_regs, n_regions, d_reqs, d_out, d_list, sr, np_shift,
                             pc_shift, nullptr, staging, d_crcs, d_partials, c->d_tabs,
                             d_glob, c->shape.pack_blocks, c->pack_depth, c->crc_variant,
                             stream, ctx_pack_flags(c)));
        sp.end();  // k_finalize is not part of the verify's timing
        CRUM_TRY(launch_finalize(kModeVerify, d_regs, n_regions, d_reqs, d_out, d_list, sr,
                                 np_shift, pc_shift, d_partials, d_crcs, staging, d_glob,
                                 c->d_tabs, stream));
    }
    {
        Span sp(c, kTScatter, stream);
        CRUM_TRY(launch_scatter(d_regs, n_regions, d_reqs, d_out, d_list, D, np_shift, pc_shift,
                                staging,
                                (flags & CRUM_UPDATE_SHADOW) ? 1 : 0, d_glob,
                                c->shape.pack_blocks, stream));
    }
    CRUM_TRY(launch_restore_finish(d_out, 1, d_glob, stream));
    CRUM_TRY(hipMemcpyAsync(h_status, d_out, sizeof(crum_status), hipMemcpyDeviceToHost, stream));
    CRUM_TRY(hipEventRecord(c->ev_done, stream));
    c->partial_call = false;
    return CRUM_OK;
}

}  // extern "C"
