// Batched snapshots: many requests (each its own region table, page size and
// image) flattened into one page space and run as a sequence of captured HIP
// graphs, one per group of whole requests.  Each group's graph runs one
// persistent diff over all units of its requests, the bitmap, the scan (which
// lays the group's images out back to back in staging and checks capacity),
// the compaction list, the pack with CRCs, and the headers.  The host drains
// each group's images with one contiguous copy as soon as the group is done,
// so copies of early groups overlap the compute of later ones.
#include "crum.h"
#include "crum_dev.h"
#include "crum_internal.h"
#include "gf2.h"

#include <algorithm>
#include <cstring>
#include <vector>

using namespace crum;

struct crum_plan {
    crum_ctx* ctx = nullptr;
    uint32_t n_reqs = 0;
    std::vector<uint32_t> order;  // position -> index of the request in the caller's list
    uint32_t n_regs = 0;
    std::vector<uint32_t> group_q;  // group g holds requests [group_q[g], group_q[g+1])
    uint8_t* d_mem = nullptr;
    uint8_t* h_rb = nullptr;  // pinned: per-group staging end, read by the host
    uint8_t* staging = nullptr;
    uint64_t staging_bytes = 0;
    uint8_t* h_images = nullptr;
    uint64_t h_images_bytes = 0;
    DevReqOut* d_out = nullptr;
    uint8_t* d_status = nullptr;
    hipStream_t cap_stream = nullptr;
    std::vector<hipGraph_t> graphs;
    std::vector<hipGraphExec_t> execs;
    std::vector<hipEvent_t> ev_group;
    hipEvent_t ev_done = nullptr;
    // timing of the last launch: start, and the end of each group's drain
    hipEvent_t t_start = nullptr;
    std::vector<hipEvent_t> t_group;
    bool timed = false;
    // with the context timing its diff class at plan creation: each group's
    // diff launch writes its start and end wall clock to d_stamp (2 words per
    // group); a launch copies them after h_rb and adds the durations to the
    // context's diff timing
    uint64_t* d_stamp = nullptr;
    std::vector<uint64_t> diff_units;  // diff units of each group (0: no diff launch)
    bool diff_timed = false;
    double clock_khz = 0;
};

namespace {

void plan_free(crum_plan* p)
{
    for (auto e : p->execs)
        (void)hipGraphExecDestroy(e);
    for (auto g : p->graphs)
        (void)hipGraphDestroy(g);
    for (auto e : p->ev_group)
        (void)hipEventDestroy(e);
    for (auto e : p->t_group)
        (void)hipEventDestroy(e);
    if (p->t_start)
        (void)hipEventDestroy(p->t_start);
    if (p->ev_done)
        (void)hipEventDestroy(p->ev_done);
    if (p->cap_stream)
        (void)hipStreamDestroy(p->cap_stream);
    if (p->d_mem)
        (void)hipFree(p->d_mem);
    if (p->h_rb)
        (void)hipHostFree(p->h_rb);
    delete p;
}

// Status records of requests in processing order q, written at the caller's
// index order[q] (40 bytes each, as k_plan_status writes them).
__global__ void k_plan_status_ordered(const DevReqOut* __restrict__ out, uint32_t n,
                                      const uint32_t* __restrict__ order,
                                      uint8_t* __restrict__ dst)
{
    const uint32_t q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n)
        return;
    const DevReqOut& O = out[q];
    uint8_t* d = dst + 40ull * order[q];
    *reinterpret_cast<int32_t*>(d) = O.code;
    *reinterpret_cast<uint32_t*>(d + 4) = O.first_bad;
    *reinterpret_cast<uint64_t*>(d + 8) = O.n_dirty;
    *reinterpret_cast<uint64_t*>(d + 16) = O.total_pages;
    *reinterpret_cast<uint64_t*>(d + 24) = O.image_bytes;
    *reinterpret_cast<uint64_t*>(d + 32) = O.img_base;
}

}  // namespace

extern "C" {

int crum_plan_create(crum_ctx* c, const crum_request* reqs, uint32_t n_reqs, void* d_staging,
                     uint64_t staging_bytes, void* h_images, uint64_t h_images_bytes,
                     crum_plan** out)
{
    if (!c || !out || (n_reqs && !reqs) || !d_staging ||
        (reinterpret_cast<uintptr_t>(d_staging) & 15u))
        return CRUM_EINVAL;
    *out = nullptr;
    // ---- validate every request and the union of all ranges
    std::vector<crum_region> all;
    uint64_t total_regs = 0;
    for (uint32_t q = 0; q < n_reqs; ++q) {
        const crum_request& r = reqs[q];
        if ((r.n_regions && !r.regions) || !ctx_page_size_ok(r.page_size) ||
            (r.flags & ~(uint32_t)CRUM_UPDATE_SHADOW))
            return CRUM_EINVAL;
        for (uint32_t i = 0; i < r.n_regions; ++i) {
            if (r.regions[i].len % r.page_size)
                return CRUM_EINVAL;
            all.push_back(r.regions[i]);
        }
        total_regs += r.n_regions;
    }
    if (total_regs > 0xFFFFFFFFull || ctx_check_ranges(all.data(), (uint32_t)all.size()) != CRUM_OK)
        return CRUM_EINVAL;
    uint64_t all_bytes = 0;
    for (const crum_region& r : all)
        all_bytes += r.len;
    // the plan's shapes: the caller's parameters, or the tuned ones of its class
    const TunedScope tuned(c, 1, 0, all_bytes);

    // ---- processing order: the caller's, or smallest scanned bytes first
    std::vector<uint32_t> order(n_reqs);
    for (uint32_t q = 0; q < n_reqs; ++q)
        order[q] = q;
    if (ctx_plan_order(c) == 1) {
        std::vector<uint64_t> bytes(n_reqs, 0);
        for (uint32_t q = 0; q < n_reqs; ++q)
            for (uint32_t i = 0; i < reqs[q].n_regions; ++i)
                bytes[q] += reqs[q].regions[i].len;
        std::stable_sort(order.begin(), order.end(),
                         [&](uint32_t a, uint32_t b) { return bytes[a] < bytes[b]; });
    }
    bool reordered = false;
    for (uint32_t q = 0; q < n_reqs; ++q)
        reordered |= order[q] != q;

    // ---- flatten (in processing order): requests padded to 64-page
    // boundaries in one page space
    std::vector<DevRegion> dregs(std::max<uint64_t>(1, total_regs));
    std::vector<DevRequest> dreq(std::max<uint32_t>(1, n_reqs));
    std::vector<uint64_t> req_unit0(n_reqs + 1, 0), req_bytes(n_reqs, 0);
    uint64_t page = 0, unit = 0, ri = 0, max_np_shift = 0;
    const uint32_t pc_shift = ctx_piece_shift(c);
    for (uint32_t q = 0; q < n_reqs; ++q) {
        const crum_request& r = reqs[order[q]];
        const uint32_t ps = (uint32_t)ctx_log2(r.page_size);
        const uint32_t us = std::min<uint32_t>(ps, ctx_unit_shift_max(c));
        DevRequest& Q = dreq[q];
        Q.first_word = page / 64;
        Q.first_region = ri;
        Q.n_regions = r.n_regions;
        Q.seq = r.seq;
        Q.page_shift = ps;
        Q.init_fix = crc_init_fix(r.page_size);
        req_unit0[q] = unit;
        uint64_t g = 0;
        for (uint32_t i = 0; i < r.n_regions; ++i, ++ri) {
            DevRegion& d = dregs[ri];
            d.cur = static_cast<const uint8_t*>(r.regions[i].base);
            d.shadow = static_cast<uint8_t*>(r.regions[i].shadow);
            d.len = r.regions[i].len;
            d.first_page = page + g;
            d.first_unit = unit;
            d.id = r.regions[i].id;
            d.page_shift = ps;
            d.req = q;
            d.unit_shift = us;
            d.flags = (r.flags & CRUM_UPDATE_SHADOW) ? 1u : 0u;
            g += d.len >> ps;
            unit += d.len >> us;
            req_bytes[q] += d.len;
        }
        if (g > 0xFFFFFF00ull)
            return CRUM_EINVAL;
        Q.n_pages = g;
        Q.n_words = (g + 63) / 64;
        Q.data_off = (64 + 32ull * r.n_regions + 8 * Q.n_words + 4095) / 4096 * 4096;
        page += Q.n_words * 64;
        if (ps > pc_shift)
            max_np_shift = std::max<uint64_t>(max_np_shift, ps - pc_shift);
    }
    req_unit0[n_reqs] = unit;
    const uint64_t G = page, W = page / 64;
    if (G > 0xFFFFFF00ull)
        return CRUM_EINVAL;
    const uint32_t np_shift = (uint32_t)max_np_shift;

    crum_plan* p = new crum_plan();
    p->ctx = c;
    p->n_reqs = n_reqs;
    p->order = order;
    p->n_regs = (uint32_t)total_regs;
    p->staging = static_cast<uint8_t*>(d_staging);
    p->staging_bytes = staging_bytes;
    p->h_images = static_cast<uint8_t*>(h_images);
    p->h_images_bytes = h_images_bytes;
    const uint64_t capacity = h_images ? std::min(staging_bytes, h_images_bytes) : staging_bytes;

    // ---- groups of whole requests: scanned bytes start at CHUNK_BYTES and
    // grow by CHUNK_GROWTH per group up to CHUNK_MAX_BYTES
    p->group_q.push_back(0);
    {
        uint64_t target = ctx_chunk_bytes(c), acc = 0;
        for (uint32_t q = 0; q < n_reqs; ++q) {
            acc += req_bytes[q];
            if (acc >= target || q + 1 == n_reqs) {
                p->group_q.push_back(q + 1);
                acc = 0;
                target = std::min<uint64_t>(target * ctx_chunk_growth(c),
                                            std::max(ctx_chunk_max_bytes(c), ctx_chunk_bytes(c)));
            }
        }
        if (n_reqs == 0)
            p->group_q.push_back(0);
    }
    const size_t n_groups = p->group_q.size() - 1;

    // ---- plan-owned device memory
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = (off + bytes + 255) / 256 * 256;
        return o;
    };
    const size_t o_regs = take(sizeof(DevRegion) * dregs.size());
    const size_t o_reqs = take(sizeof(DevRequest) * dreq.size());
    const size_t o_out = take(sizeof(DevReqOut) * (n_reqs + 1));
    const size_t o_flags = take(std::max<uint64_t>(unit, 1));
    const size_t o_bitmap = take(8 * std::max<uint64_t>(W, 1));
    const size_t o_prefix = take(4 * std::max<uint64_t>(W, 1));
    const size_t o_list = take(4 * std::max<uint64_t>(G, 1));
    const size_t o_crcs = take(4 * std::max<uint64_t>(G, 1));
    const size_t o_part = take(4 * std::max<uint64_t>(np_shift ? G << np_shift : 0, 1));
    const size_t o_bounds = take(8 * std::max<size_t>(n_groups, 1));
    const size_t o_status = take(40ull * std::max<uint32_t>(n_reqs, 1));
    const size_t o_order = take(4ull * std::max<uint32_t>(n_reqs, 1));
    const size_t o_stamp = take(16 * std::max<size_t>(n_groups, 1));
    const size_t rb_bytes = 24 * std::max<size_t>(n_groups, 1);  // ends, then stamps
    DeviceGuardC g(ctx_device(c));
    auto fail = [&](int code) {
        plan_free(p);
        return code;
    };
    if (hipMalloc(reinterpret_cast<void**>(&p->d_mem), off) != hipSuccess ||
        hipHostMalloc(reinterpret_cast<void**>(&p->h_rb), rb_bytes, 0) != hipSuccess ||
        hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&p->ev_done, hipEventDisableTiming) != hipSuccess ||
        hipEventCreate(&p->t_start) != hipSuccess)
        return fail(CRUM_EHIP);
    std::memset(p->h_rb, 0, rb_bytes);
    uint8_t* M = p->d_mem;
    if (hipMemcpy(M + o_regs, dregs.data(), sizeof(DevRegion) * dregs.size(),
                  hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(M + o_reqs, dreq.data(), sizeof(DevRequest) * dreq.size(),
                  hipMemcpyHostToDevice) != hipSuccess ||
        (n_reqs && hipMemcpy(M + o_order, order.data(), 4ull * n_reqs,
                             hipMemcpyHostToDevice) != hipSuccess))
        return fail(CRUM_EHIP);
    const uint32_t* d_order = reinterpret_cast<const uint32_t*>(M + o_order);
    const DevRegion* d_regs = reinterpret_cast<const DevRegion*>(M + o_regs);
    const DevRequest* d_reqs = reinterpret_cast<const DevRequest*>(M + o_reqs);
    DevReqOut* d_out = reinterpret_cast<DevReqOut*>(M + o_out);
    DevGlobal* d_glob = reinterpret_cast<DevGlobal*>(M + o_out + sizeof(DevReqOut) * n_reqs);
    uint8_t* d_flags = M + o_flags;
    uint64_t* d_bitmap = reinterpret_cast<uint64_t*>(M + o_bitmap);
    uint32_t* d_prefix = reinterpret_cast<uint32_t*>(M + o_prefix);
    uint32_t* d_list = reinterpret_cast<uint32_t*>(M + o_list);
    uint32_t* d_crcs = reinterpret_cast<uint32_t*>(M + o_crcs);
    uint32_t* d_part = reinterpret_cast<uint32_t*>(M + o_part);
    uint64_t* d_bounds = reinterpret_cast<uint64_t*>(M + o_bounds);
    p->d_out = d_out;
    p->d_status = M + o_status;
    const LaunchShape shape = ctx_shape(c);
    const CrcTables* tabs = ctx_tables(c);
    p->diff_timed = ctx_times(c, kTDiff);
    if (p->diff_timed) {
        int khz = 0;
        if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, ctx_device(c)) !=
                hipSuccess ||
            khz <= 0 || hipMemset(M + o_stamp, 0, 16 * std::max<size_t>(n_groups, 1)) != hipSuccess)
            return fail(CRUM_EHIP);
        p->clock_khz = khz;
        p->d_stamp = reinterpret_cast<uint64_t*>(M + o_stamp);
    }

    // ---- capture one graph per group
    for (size_t gi = 0; gi < n_groups; ++gi) {
        const uint32_t q0 = p->group_q[gi], q1 = p->group_q[gi + 1];
        const uint64_t w0 = q0 < n_reqs ? dreq[q0].first_word : W;
        const uint64_t w1 = q1 < n_reqs ? dreq[q1].first_word : W;
        const uint64_t u0 = req_unit0[q0], u1 = req_unit0[q1];
        p->diff_units.push_back(u1 - u0);
        uint32_t hdr_blocks = 1, min_us = 64;
        for (uint32_t q = q0; q < q1; ++q) {
            hdr_blocks = std::max(hdr_blocks, header_blocks(dreq[q].n_regions, dreq[q].n_words,
                                                            dreq[q].n_pages));
            if (dreq[q].n_regions)
                min_us = std::min(min_us, dregs[dreq[q].first_region].unit_shift);
        }
        hipStream_t s = p->cap_stream;
        if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess)
            return fail(CRUM_EHIP);
        hipError_t e = hipSuccess;
        if (gi == 0)
            e = launch_plan_init(d_glob, s);
        if (e == hipSuccess)
            e = launch_diff(d_regs, p->n_regs, u0, u1, d_flags, shape.diff_blocks,
                            ctx_diff_nt(c), ctx_diff_prio(c), s, nullptr,
                            p->d_stamp ? p->d_stamp + 2 * gi : nullptr,
                            ctx_diff_group(c, min_us));
        if (e == hipSuccess)
            e = launch_bitmap(d_regs, p->n_regs, w0, w1, d_flags, d_bitmap, s);
        if (e == hipSuccess)
            e = launch_scan(d_bitmap, w0, w1, W, d_prefix, d_bounds + gi, 1, d_reqs, q0, q1,
                            d_out, d_glob, capacity, 0, d_list, s);
        if (e == hipSuccess)
            e = hipMemcpyAsync(p->h_rb + 8 * gi, &d_glob->staging_used, 8,
                               hipMemcpyDeviceToHost, s);
        SlotRange sr{0, 0, d_bounds, (uint32_t)gi, (w1 - w0) * 64};
        if (e == hipSuccess)
            e = launch_pack(kModePack, d_regs, p->n_regs, d_reqs, d_out, d_list, sr, np_shift,
                            pc_shift, d_flags, p->staging, d_crcs, d_part, tabs, d_glob,
                            shape.pack_blocks, ctx_pack_depth(c), ctx_crc_variant(c), s,
                            ctx_pack_flags(c));
        if (e == hipSuccess)
            e = launch_finalize(kModePack, d_regs, p->n_regs, d_reqs, d_out, d_list, sr, np_shift,
                                pc_shift, d_part, d_crcs, p->staging, d_glob, tabs, s);
        if (e == hipSuccess)
            e = launch_header(d_regs, d_reqs, q0, q1, hdr_blocks, d_out, d_bitmap, d_crcs,
                              p->staging, capacity, tabs, s);
        if (e == hipSuccess && gi + 1 == n_groups) {
            if (!reordered) {
                e = launch_plan_status(d_out, n_reqs, p->d_status, s);
            } else {
                hipLaunchKernelGGL(k_plan_status_ordered, dim3((n_reqs + 255) / 256), dim3(256),
                                   0, s, d_out, n_reqs, d_order, p->d_status);
                e = hipGetLastError();
            }
        }
        hipGraph_t graph = nullptr;
        const hipError_t e2 = hipStreamEndCapture(s, &graph);
        if (e != hipSuccess || e2 != hipSuccess || !graph) {
            if (graph)
                (void)hipGraphDestroy(graph);
            return fail(CRUM_EHIP);
        }
        p->graphs.push_back(graph);
        hipGraphExec_t ex = nullptr;
        if (hipGraphInstantiate(&ex, graph, nullptr, nullptr, 0) != hipSuccess)
            return fail(CRUM_EHIP);
        p->execs.push_back(ex);
        hipEvent_t ev, te;
        if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess)
            return fail(CRUM_EHIP);
        p->ev_group.push_back(ev);
        if (hipEventCreate(&te) != hipSuccess)
            return fail(CRUM_EHIP);
        p->t_group.push_back(te);
    }
    *out = p;
    return CRUM_OK;
}

int crum_plan_launch(crum_plan* p, void* stream_, crum_request_status* h_status)
{
    if (!p || !h_status)
        return CRUM_EINVAL;
    crum_ctx* c = p->ctx;
    DeviceGuardC g(ctx_device(c));
    hipStream_t stream = static_cast<hipStream_t>(stream_);
    hipStream_t side = ctx_side_stream(c);
    const size_t n_groups = p->execs.size();
    CRUM_TRY_C(hipStreamWaitEvent(stream, p->ev_done, 0));
    CRUM_TRY_C(hipEventRecord(p->t_start, stream));
    for (size_t gi = 0; gi < n_groups; ++gi) {
        CRUM_TRY_C(hipGraphLaunch(p->execs[gi], stream));
        CRUM_TRY_C(hipEventRecord(p->ev_group[gi], stream));
    }
    uint64_t prev = 0;
    for (size_t gi = 0; gi < n_groups; ++gi) {
        CRUM_TRY_C(hipEventSynchronize(p->ev_group[gi]));
        uint64_t used;
        std::memcpy(&used, p->h_rb + 8 * gi, 8);
        CRUM_TRY_C(hipStreamWaitEvent(side, p->ev_group[gi], 0));
        if (p->h_images && used > prev) {
            CRUM_TRY_C(hipMemcpyAsync(p->h_images + prev, p->staging + prev, used - prev,
                                      hipMemcpyDeviceToHost, side));
            prev = used;
        }
        CRUM_TRY_C(hipEventRecord(p->t_group[gi], side));
    }
    if (p->n_reqs)
        CRUM_TRY_C(hipMemcpyAsync(h_status, p->d_status, 40ull * p->n_reqs,
                                  hipMemcpyDeviceToHost, side));
    uint64_t* h_stamp = reinterpret_cast<uint64_t*>(p->h_rb + 8 * n_groups);
    if (p->diff_timed)
        CRUM_TRY_C(hipMemcpyAsync(h_stamp, p->d_stamp, 16 * n_groups, hipMemcpyDeviceToHost,
                                  side));
    CRUM_TRY_C(hipEventRecord(p->ev_done, side));
    CRUM_TRY_C(hipStreamWaitEvent(stream, p->ev_done, 0));
    p->timed = true;
    if (p->diff_timed) {
        // a plan that times its diff launches returns after its drains end
        CRUM_TRY_C(hipEventSynchronize(p->ev_done));
        for (size_t gi = 0; gi < n_groups; ++gi)
            if (p->diff_units[gi] && h_stamp[2 * gi + 1] > h_stamp[2 * gi])
                ctx_add_timing(c, kTDiff,
                               (double)(h_stamp[2 * gi + 1] - h_stamp[2 * gi]) / p->clock_khz);
    }
    return CRUM_OK;
}

int crum_plan_groups(crum_plan* p, uint32_t* n_groups, uint32_t* first_request, uint32_t cap)
{
    if (!p || !n_groups)
        return CRUM_EINVAL;
    const uint32_t n = (uint32_t)(p->group_q.size() - 1);
    *n_groups = n;
    if (first_request)
        for (uint32_t i = 0; i <= n && i < cap; ++i)
            first_request[i] = p->group_q[i];
    return CRUM_OK;
}

int crum_plan_order(crum_plan* p, uint32_t* order, uint32_t cap)
{
    if (!p || (cap && !order))
        return CRUM_EINVAL;
    for (uint32_t i = 0; i < p->n_reqs && i < cap; ++i)
        order[i] = p->order[i];
    return CRUM_OK;
}

int crum_plan_group_times(crum_plan* p, double* ms, uint32_t cap)
{
    if (!p || !ms || !p->timed)
        return CRUM_EINVAL;
    DeviceGuardC g(ctx_device(p->ctx));
    for (size_t gi = 0; gi < p->t_group.size() && gi < cap; ++gi) {
        float v = 0;
        if (hipEventSynchronize(p->t_group[gi]) != hipSuccess ||
            hipEventElapsedTime(&v, p->t_start, p->t_group[gi]) != hipSuccess)
            return CRUM_EHIP;
        ms[gi] = v;
    }
    return CRUM_OK;
}

void crum_plan_destroy(crum_plan* p)
{
    if (!p)
        return;
    DeviceGuardC g(ctx_device(p->ctx));
    (void)hipEventSynchronize(p->ev_done);
    (void)hipStreamSynchronize(p->cap_stream);
    plan_free(p);
}

}  // extern "C"
