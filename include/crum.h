/*
 * crum.h -- C ABI of the incremental GPU snapshot library (gfx950 / MI355X).
 *
 * The library implements phase one of a GPU checkpoint: after the application
 * has quiesced its work (paper section 3.4: synchronise the device, then read
 * back every active device and managed region), the device memory named by a
 * region table is drained to host memory.  It is incremental: each region may
 * come with a shadow copy of its last snapshot in device memory, and only
 * pages whose bytes differ from the shadow are packed and copied.  A region
 * without a shadow has every page dirty, as a freshly created shadow region
 * is all-dirty in the paper's shadow-page scheme (section 3.2, Algorithm 1).
 * Restore is the inverse (section 3.4, restart: data copied back into the
 * re-created regions).
 *
 * Every buffer argument is caller-owned: regions, shadows, the device staging
 * buffer, the pinned host image, the status.  The context owns only internal
 * scratch, CRC tables, one side stream and events.  Device pointers may come
 * from hipMalloc, hipMallocManaged or a framework allocator; host image and
 * status pointers must be pinned host memory (hipHostMalloc or equivalent).
 *
 * Image layout v1 (little-endian, pad bytes zero):
 *    0 "CRUMIMG1" | 8 u32 version=1 | 12 u32 page_size | 16 u32 n_regions
 *   20 u32 flags (bit 0: no region had a shadow) | 24 u64 total_pages G
 *   32 u64 n_dirty D | 40 u64 seq | 48 u64 data_off | 56 u32 meta_crc
 *   60 u32 crcs_crc | 64 region table: n_regions x {u64 id, u64 len,
 *   u64 first_page, u64 0} | 64+32R bitmap: ceil(G/64) u64 words (bit g%64 of
 *   word g/64 set when global page g is dirty) | zero pad to
 *   data_off = roundup(64+32R+8W, 4096) | D packed pages in ascending page
 *   order | D u32 CRC-32C values, one per packed page | zero pad to 8 bytes.
 *   crcs_crc is the CRC-32C of the CRC array; meta_crc is the CRC-32C of
 *   bytes [0, 64+32R+8W) with bytes 56..59 read as zero.  Pages are numbered
 *   globally in table order; page boundaries are relative to each region base.
 *   CRC-32C: polynomial 0x1EDC6F41 reflected, init and final XOR 0xFFFFFFFF.
 *
 * Error conventions.  Argument errors are returned synchronously and nothing
 * is enqueued (CRUM_EINVAL).  A failing HIP call returns CRUM_EHIP.  Errors
 * found on the device (ENOSPC, ECRC, EFORMAT) are reported in *h_status, which
 * is valid once `stream` has passed the call.  A context is not thread-safe;
 * distinct contexts may be used from distinct threads.  Regions must not be
 * written while a snapshot of them is in flight.
 */
#ifndef CRUM_H
#define CRUM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct crum_ctx crum_ctx;
typedef struct crum_plan crum_plan;
typedef struct crum_server crum_server;

/* One snapshotted allocation.  base: device or managed address of the
 * current bytes; shadow: device address of the baseline copy, or NULL (all
 * pages dirty); len: bytes, a multiple of the page size (0 allowed); id:
 * caller tag stored in the image and checked at restore.  base and shadow are
 * 16-byte aligned; no current or shadow range may overlap another. */
typedef struct {
    void* base;
    void* shadow;
    uint64_t len;
    uint64_t id;
} crum_region;

/* Result of one call, written asynchronously on the call's stream.
 * code: CRUM_OK or a device-detected error; first_bad: lowest packed-page
 * slot whose CRC failed (ECRC only); n_dirty: D; total_pages: G;
 * image_bytes: size of the image (for ENOSPC, the size that was needed). */
typedef struct {
    int32_t code;
    uint32_t first_bad;
    uint64_t n_dirty;
    uint64_t total_pages;
    uint64_t image_bytes;
} crum_status;

enum {
    CRUM_OK = 0,
    CRUM_EINVAL = -1,    /* bad argument; nothing enqueued */
    CRUM_ENOSPC = -2,    /* image larger than the staging or host capacity */
    CRUM_ECRC = -3,      /* a packed page failed CRC verification */
    CRUM_EFORMAT = -4,   /* image header, table, bitmap, pads or checksums invalid */
    CRUM_EHIP = -5,      /* a HIP runtime call failed (kernel launches are checked with
                            hipGetLastError, so a failure of the caller's own that is
                            still pending in the calling thread shows here too) */
    CRUM_EMISMATCH = -6  /* restore table differs from the image (count, len, id) */
};

enum {
    CRUM_UPDATE_SHADOW = 1u, /* snapshot: copy each dirty page into its shadow on success;
                                restore: also write restored pages into the shadows */
    CRUM_VERIFY = 2u         /* restore: check every page CRC before writing any byte */
};

/* Create a context on HIP device `device`; builds the CRC tables, the side
 * stream and events.  tuning_cache: path of the shape tuner's JSON cache, or
 * NULL for the default shapes.  The entries for this device (its key is
 * "cc<major>.<minor>-<CUs>cu|hip<runtime version>") and for the classes
 * "snapshot|p<page size>|b<k>" (single snapshots of that page size scanning
 * 2^k..2^(k+1) bytes) and "plan|b<k>" (plans whose requests scan that much)
 * are loaded; a snapshot or plan of a loaded class then runs with that class's
 * shapes, except for parameters set with crum_ctx_set_param, which always
 * win.  Shapes change speed only, never an image.  Returns CRUM_OK,
 * CRUM_EINVAL (bad device, out==NULL, a cache file that cannot be read or
 * parsed) or CRUM_EHIP. */
int crum_ctx_create(int device, const char* tuning_cache, crum_ctx** out);

/* Number of tuned classes the context loaded for its device. */
int crum_ctx_tuned_classes(crum_ctx* ctx, uint32_t* n_classes);

/* Parse a tuning cache file as crum_ctx_create does, for the given device
 * key: CRUM_OK and the number of classes found, or CRUM_EINVAL.  Host only. */
int crum_tuning_check(const char* path, const char* device_key, uint32_t* n_classes);

/* Destroy a context (waits for its outstanding work). NULL is ignored. */
void crum_ctx_destroy(crum_ctx* ctx);

/* Bytes of the image before the first packed page (data_off) for a table of
 * n_regions regions holding total_pages pages.  Pure host computation. */
int crum_image_prefix_bytes(uint32_t n_regions, uint64_t total_pages, uint64_t* out);

/* Bytes of an image with the given shape and dirty count. Pure host computation. */
int crum_image_bytes(uint32_t n_regions, uint64_t total_pages, uint64_t n_dirty,
                     uint32_t page_size, uint64_t* out);

/* Incremental snapshot (paper section 3.4, checkpoint: quiesce, then read back
 * every active region; section 3.2: per-page dirty state, all-dirty without a
 * baseline, dirty cleared after a flush).
 *
 * Enqueues on `stream` (a hipStream_t; NULL = the null stream): diff of every
 * page against its shadow -> dirty bitmap -> prefix sum -> pack of dirty pages
 * with their CRC-32C -> image header, all built in d_staging in the image
 * layout above, and the drain of the image to h_image on the context's side
 * stream; `stream` is made to wait for the drain.  The calling thread blocks
 * only on small device-to-host reads of dirty counts.  Two orders give the
 * same image: when both capacities hold an image with every page dirty and
 * CRUM_PARAM_EAGER is 1, the page space is processed in chunks and each chunk
 * is drained while later chunks are diffed (an image of one chunk is drained
 * in one copy behind the header); otherwise the whole diff and the capacity
 * check run first, then pack chunks with their drain behind them.  A third order applies when an image with every page dirty is at most
 * CRUM_PARAM_DIRECT_BYTES and h_image is host memory the device maps at the
 * same address (hipHostMalloc): the pack and header kernels write the image
 * straight into h_image, d_staging is not written, and the calling thread
 * does not wait at all.  With CRUM_UPDATE_SHADOW, every dirty page is also
 * copied into its shadow, but only when the status is CRUM_OK.
 *
 * d_staging: device buffer of staging_bytes, at least data_off bytes, 16-byte
 * aligned; receives the image (except in the direct order).  h_image: pinned host buffer of h_image_bytes,
 * or NULL to keep the image on the device only.  If the image does not fit
 * either capacity, status CRUM_ENOSPC: nothing is packed, no shadow changes,
 * n_dirty/image_bytes and the bitmap (at d_staging + 64 + 32R) are valid.
 * h_status: pinned host memory, valid after `stream` passes the call.
 * Returns CRUM_OK (enqueued), CRUM_EINVAL or CRUM_EHIP. */
int crum_snapshot(crum_ctx* ctx, const crum_region* regions, uint32_t n_regions,
                  uint32_t page_size, uint32_t flags, uint64_t seq, void* d_staging,
                  uint64_t staging_bytes, void* h_image, uint64_t h_image_bytes, void* stream,
                  crum_status* h_status);

/* Restore (paper section 3.4, restart: the re-created regions receive the
 * saved data).  The image is read from h_image (pinned host, image_bytes
 * long) into d_staging, or, when h_image is NULL, is taken to be already in
 * d_staging.  The host checks the header and region table synchronously:
 * CRUM_EFORMAT or CRUM_EMISMATCH are returned (and written to *h_status) with
 * nothing enqueued.  On the device: meta_crc, crcs_crc, bitmap and pads are
 * checked (CRUM_EFORMAT); with CRUM_VERIFY every page CRC is checked
 * (CRUM_ECRC, first_bad = lowest failing slot); only then is each packed page
 * scattered to its page (and its shadow with CRUM_UPDATE_SHADOW).  On any
 * device-detected error no region byte is written.  staging_bytes below
 * image_bytes returns CRUM_ENOSPC synchronously. */
int crum_restore(crum_ctx* ctx, const crum_region* regions, uint32_t n_regions,
                 const void* h_image, uint64_t image_bytes, uint32_t flags, void* d_staging,
                 uint64_t staging_bytes, void* stream, crum_status* h_status);

/* ---------------------------------------------------------------------------
 * Host write tracking (section 3.2, Algorithm 1, and section 3.2.1: the
 * application writes a shadow of each unified-memory region on the host; a
 * write to a write-protected page faults and marks the page dirty, and at
 * each call into the GPU runtime the dirty pages are flushed to the real
 * region, write-protected again and marked clean; a new region starts with
 * every page dirty).
 *
 * crum_track_create maps a host view of `bytes` bytes (anonymous memory that
 * the GPU never maps) cut into pages of page_size bytes (a power of two in
 * [4 KiB, 1 GiB], a multiple of the OS page size, dividing bytes).  The
 * application writes its data through crum_track_view.  Every page starts
 * dirty and writable.  A write to a clean (read-only) page is caught by a
 * SIGSEGV handler that the first tracker installs (once per process, before
 * any handler installed later; faults outside every view go to the handler
 * that was installed before it, or take the default action): the page is made
 * writable and marked dirty, and the write completes.
 *
 * crum_track_flush copies every dirty page to the same offset of dst (the real
 * region: for example a hipMallocManaged allocation, read and written by the
 * host here), on up to n_threads host threads, after making it read-only and
 * clearing its dirty bit; each flushed page is added to the pending set.
 * *n_flushed (may be NULL) receives the pages flushed.
 *
 * The pending set holds the pages flushed since it was last cleared:
 * crum_track_pending copies it as a bitmap (bit p % 64 of words[p / 64] for
 * page p; n_words words are written, words past the view's pages as zero)
 * and, with clear, empties it.  A caller that updates the shadows at each
 * snapshot (CRUM_UPDATE_SHADOW) clears the pending set at the same time; the
 * pages outside it are then equal to their shadows unless something other
 * than the view (the GPU) wrote them, and those go into the candidate set of
 * crum_snapshot_tracked as well.
 *
 * Flushes of one tracker are serialised; writes to the view may run on any
 * thread, also during a flush (a page written while it is copied stays
 * dirty).  No write to the view may run during crum_track_destroy.  Returns
 * CRUM_OK or CRUM_EINVAL (bad argument, mmap or mprotect failure, more than
 * 64 trackers at once).  Host code only: no HIP call is made.
 * -------------------------------------------------------------------------*/
typedef struct crum_track crum_track;

typedef struct {
    uint64_t pages;          /* pages of the view */
    uint64_t dirty_pages;    /* written since the last flush */
    uint64_t pending_pages;  /* flushed since the pending set was last cleared */
    uint64_t faults;         /* write faults taken so far */
    uint64_t flushed_pages;  /* pages copied by all flushes so far */
} crum_track_info;

int crum_track_create(uint64_t bytes, uint32_t page_size, crum_track** out);
void* crum_track_view(crum_track* track);
int crum_track_flush(crum_track* track, void* dst, uint32_t n_threads, uint64_t* n_flushed);
int crum_track_pending(crum_track* track, uint64_t* words, uint64_t n_words, int clear);
/* The dirty set (written since the last flush), as crum_track_pending. */
int crum_track_dirty(crum_track* track, uint64_t* words, uint64_t n_words);
int crum_track_stats(crum_track* track, crum_track_info* out);
void crum_track_destroy(crum_track* track);

/* Snapshot with a candidate set (section 3.2: only pages written since the
 * last flush can differ from it).  As crum_snapshot, except that a page whose
 * bit in h_candidates (host memory, bit g % 64 of word g / 64 for global page
 * g, at least ceil(G/64) words in n_words) is clear is taken to equal its
 * shadow: neither copy of it is read, and it is not dirty.  The image equals
 * crum_snapshot's whenever every page that differs from its shadow has its
 * bit set; regions without a shadow ignore the set (all their pages are
 * dirty).  The bitmap is read before the call returns.  Returns as
 * crum_snapshot; CRUM_EINVAL also for h_candidates NULL or n_words too small. */
int crum_snapshot_tracked(crum_ctx* ctx, const crum_region* regions, uint32_t n_regions,
                          uint32_t page_size, uint32_t flags, uint64_t seq,
                          const uint64_t* h_candidates, uint64_t n_words, void* d_staging,
                          uint64_t staging_bytes, void* h_image, uint64_t h_image_bytes,
                          void* stream, crum_status* h_status);

/* Snapshot without allocation, for callers that cannot allocate: code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * Arguments, result and image as crum_snapshot's, always in its diff-first
 * order (whole diff, capacity check, one pack launch, header), the image
 * copied to h_image with one hipMemcpyAsync on `stream`; the calling thread
 * waits for the dirty count.  The device scratch is a fixed array of
 * CRUM_NOALLOC_SCRATCH_BYTES per device (held until the process ends), the
 * host side a pinned buffer allocated by crum_ctx_create: no call allocates.
 * Inputs whose scratch would not fit (more than CRUM_NOALLOC_MAX_REGIONS
 * regions, or roughly 7 million pages of 4 KiB, 5 million of 64 KiB) return
 * CRUM_ELIMIT with nothing enqueued.  Every call on one device shares that
 * device's array: calls that overlap on one device (different contexts, or
 * different threads) race; consecutive calls through one context are
 * ordered.  Timing classes are not recorded by this call. */
#define CRUM_NOALLOC_SCRATCH_BYTES (64ull << 20)
#define CRUM_NOALLOC_MAX_REGIONS 2048u
enum { CRUM_ELIMIT = -9 /* input larger than the fixed scratch of crum_snapshot_noalloc */ };
int crum_snapshot_noalloc(crum_ctx* ctx, const crum_region* regions, uint32_t n_regions,
                          uint32_t page_size, uint32_t flags, uint64_t seq, void* d_staging,
                          uint64_t staging_bytes, void* h_image, uint64_t h_image_bytes,
                          void* stream, crum_status* h_status);

/* ---------------------------------------------------------------- batched
 * Many snapshot requests in one plan (the batched pattern).  Each request is a
 * region table with its own page size, flags (CRUM_UPDATE_SHADOW) and seq,
 * and produces exactly the image that crum_snapshot would produce for it.
 * Requests are processed in the caller's order, or smallest scanned bytes
 * first when CRUM_PARAM_PLAN_ORDER is 1 (a request then waits only for
 * smaller ones), and grouped in that order (groups of whole requests,
 * scanned bytes per group starting at CRUM_PARAM_CHUNK_BYTES and growing by
 * CRUM_PARAM_CHUNK_GROWTH up
 * to CRUM_PARAM_CHUNK_MAX_BYTES); each group's device work -- one persistent diff
 * over all units of its requests, bitmap, scan, compaction, pack with CRCs and
 * headers -- is captured once as a HIP graph at plan creation.  Request images
 * are laid out back to back in processing order in d_staging (each at a 4
 * KiB-aligned offset) and
 * copied to the same offsets of h_images, one contiguous copy per group on the
 * context's side stream as soon as the group is done. */
typedef struct {
    const crum_region* regions; /* caller-owned, read at plan creation */
    uint32_t n_regions;
    uint32_t page_size;
    uint32_t flags;             /* CRUM_UPDATE_SHADOW or 0 */
    uint32_t reserved;          /* 0 */
    uint64_t seq;
} crum_request;

/* Per-request result of a plan launch; image_offset is the byte offset of
 * the request's image in d_staging and h_images. */
typedef struct {
    crum_status status;
    uint64_t image_offset;
} crum_request_status;

/* Validate the requests (as crum_snapshot does, and all current and shadow
 * ranges of all requests pairwise disjoint), flatten them, upload the tables
 * and capture the group graphs, using the context's current parameters.  The
 * plan keeps the region pointers, d_staging and h_images (pinned host memory
 * or NULL).  If the images of a group do not fit the capacity
 * (min(staging_bytes, h_images_bytes)), that group and every later group (in
 * processing order) report CRUM_ENOSPC and write no page, CRC or shadow.
 * Returns CRUM_OK, CRUM_EINVAL or CRUM_EHIP. */
int crum_plan_create(crum_ctx* ctx, const crum_request* reqs, uint32_t n_reqs, void* d_staging,
                     uint64_t staging_bytes, void* h_images, uint64_t h_images_bytes,
                     crum_plan** out);

/* Snapshot every request of the plan: launch the group graphs on `stream`,
 * and drain each group behind it (the calling thread waits for each group's
 * end to size its copy).  h_status: pinned array of n_reqs entries, valid
 * once `stream` passes the launch, indexed in the caller's order of the
 * requests.  Calls on one plan must not overlap. */
int crum_plan_launch(crum_plan* plan, void* stream, crum_request_status* h_status);

/* Group layout: n_groups, and first_request[0..n_groups] (group g holds the
 * requests at processing positions [first_request[g], first_request[g+1])),
 * up to cap entries. */
int crum_plan_groups(crum_plan* plan, uint32_t* n_groups, uint32_t* first_request, uint32_t cap);

/* Processing order: order[k] is the caller's index of the request at
 * position k, for k < min(n_reqs, cap). */
int crum_plan_order(crum_plan* plan, uint32_t* order, uint32_t cap);

/* For the last launch: milliseconds from its start to the end of each
 * group's drain (waits for them), up to cap entries. */
int crum_plan_group_times(crum_plan* plan, double* ms, uint32_t cap);

/* Destroy a plan (waits for its outstanding work). NULL is ignored. */
void crum_plan_destroy(crum_plan* plan);

/* ---------------------------------------------------------------- serving
 * A request loop for many clients, each owning persistent device state
 * (regions with resident shadows).  Requests run first-in first-out per
 * client, so a client's results do not depend on the other clients; up to
 * n_slots requests of different clients run at once, each slot with its own
 * context, streams and device staging buffer (sized for the largest client's
 * worst-case image), so their device work overlaps.  Snapshots use
 * CRUM_UPDATE_SHADOW and land in a pinned arena of pinned_budget bytes: on the
 * pipelined path (see crum_server_set_policy) the client's worst-case image is
 * reserved when it fits at once, the snapshot drains into it while it runs,
 * and the reservation is trimmed to the image; otherwise the image is built on the device first, the
 * client's previous image is released (the shadow now holds the new
 * snapshot), exactly the new image's bytes are reserved -- waiting while the
 * arena is full, CRUM_ENOSPC after 30 s -- and the image is drained into them.
 * A restore re-applies the client's latest image with CRUM_VERIFY |
 * CRUM_UPDATE_SHADOW. */
enum { CRUM_REQ_SNAPSHOT = 1, CRUM_REQ_RESTORE = 2 };

typedef struct {
    const crum_region* regions; /* every region needs a shadow; copied at creation */
    uint32_t n_regions;
    uint32_t page_size;
} crum_client;

typedef struct {
    uint64_t id;          /* as returned by crum_server_submit */
    uint64_t tag;         /* caller value given at submit */
    uint32_t client;
    uint32_t kind;        /* CRUM_REQ_SNAPSHOT or CRUM_REQ_RESTORE */
    int32_t code;         /* CRUM_OK or an error */
    uint32_t meta_crc;    /* bytes 56..59 of the image (with crcs_crc, a digest of it) */
    uint32_t crcs_crc;
    uint32_t reserved;
    uint64_t n_dirty;
    uint64_t image_bytes;
    double arrival_s;     /* seconds since server creation: submit, start, completion */
    double start_s;
    double done_s;
} crum_server_completion;

/* Called on a worker thread before a request runs, with the stream the
 * request will use; a harness enqueues its own work (for example changes to
 * the client's memory) on that stream. */
typedef void (*crum_server_prepare_fn)(void* user, uint32_t client, uint32_t kind, uint64_t tag,
                                       void* stream);

/* Returns CRUM_OK, CRUM_EINVAL (bad client table, overlapping ranges, a
 * region without shadow, n_slots outside 1..64) or CRUM_EHIP. */
int crum_server_create(int device, const crum_client* clients, uint32_t n_clients,
                       uint32_t n_slots, uint64_t pinned_budget, crum_server** out);
int crum_server_set_prepare(crum_server* server, crum_server_prepare_fn fn, void* user);
/* Which snapshot path to use: CRUM_SERVE_TWO_STAGE always builds the image on
 * the device before reserving; CRUM_SERVE_PIPELINED reserves the worst case
 * whenever it fits; CRUM_SERVE_ADAPTIVE (default) pipelines only when no other
 * request is waiting (latency), and builds first under a backlog (throughput:
 * one long copy per request keeps the link busier than many short ones). */
enum { CRUM_SERVE_ADAPTIVE = 0, CRUM_SERVE_TWO_STAGE = 1, CRUM_SERVE_PIPELINED = 2 };
int crum_server_set_policy(crum_server* server, int policy);
/* Enqueue a request (non-blocking); *id receives its id. */
int crum_server_submit(crum_server* server, uint32_t client, uint32_t kind, uint64_t tag,
                       uint64_t* id);
/* Move up to max completions into out (*n of them); with wait_all, first wait
 * until no request is queued or running. */
int crum_server_poll(crum_server* server, crum_server_completion* out, uint32_t max, uint32_t* n,
                     int wait_all);
/* Seconds since the server was created (the clock of the completion times). */
double crum_server_time(crum_server* server);
/* Pinned bytes currently reserved by images. */
int crum_server_pinned_used(crum_server* server, uint64_t* bytes);
/* The client's latest image (pinned host memory owned by the server); valid
 * while no request of that client is queued or running. */
int crum_server_latest_image(crum_server* server, uint32_t client, const void** ptr,
                             uint64_t* bytes);
/* Finish queued requests, stop the workers and free everything. */
void crum_server_destroy(crum_server* server);

/* Launch and pipeline parameters of a context (defaults in parentheses).
 * They change speed only: every image is the same whatever their values.
 * CRUM_PARAM_DIFF_BLOCKS: persistent grid of the diff kernel, in 256-thread
 *   workgroups (8 per compute unit).  CRUM_PARAM_PACK_BLOCKS: grid of the
 *   pack, verify and scatter kernels (4 per compute unit).
 * CRUM_PARAM_CHUNK_BYTES / CRUM_PARAM_CHUNK_MAX_BYTES: scanned bytes of the
 *   first and of the largest chunk when the snapshot is pipelined by chunks
 *   (128 MiB / 4 GiB); chunks grow by CRUM_PARAM_CHUNK_GROWTH up to the maximum.
 * CRUM_PARAM_EAGER: 1 pipelines the snapshot by chunks whenever the staging
 *   and host capacities hold an image with every page dirty (so ENOSPC is
 *   impossible); 0 always runs the whole diff first (1).
 * CRUM_PARAM_DRAIN_CHUNK_BYTES: first pack/drain chunk of the non-pipelined
 *   order (8 MiB, doubling up to 256 MiB).
 * CRUM_PARAM_DIFF_UNIT_SHIFT: log2 of the largest diff unit, 12..14 (14):
 *   each wave compares min(page, 2^value) bytes per step.
 * CRUM_PARAM_DIFF_NONTEMPORAL: 1 marks the diff kernel's loads non-temporal (1).
 * CRUM_PARAM_PIECE_SHIFT: log2 of the largest piece of a page one wave packs,
 *   verifies or scatters, 12..16 (14); larger pages are split into pieces
 *   whose CRCs are combined afterwards.
 * CRUM_PARAM_PACK_DEPTH: 16-byte loads each lane keeps in flight in the pack
 *   and verify kernels, 4, 8 or 16 (4).
 * CRUM_PARAM_DIFF_PRIORITY: issue priority of the diff kernel's waves on
 *   their compute units relative to co-running kernels, 0..3 (0).
 * CRUM_PARAM_PLAN_ORDER: processing order of a plan's requests, 0 = the
 *   caller's, 1 = smallest scanned bytes first (0).
 * CRUM_PARAM_DIRECT_BYTES: snapshots whose image with every page dirty is at
 *   most this many bytes are built straight in the pinned host image (see
 *   crum_snapshot), an opt-in alternative to the staged drain; 0 turns the
 *   direct order off (0: every image is drained by hipMemcpyAsync).
 * CRUM_PARAM_CRC_VARIANT: how the pack and verify kernels' CRC step splits
 *   its table lookups between 256-entry byte tables (bank conflicts) and
 *   16-entry nibble tables (conflict-free, more ALU work): 0 = byte tables
 *   only, 1..5 = mixes, 6 = byte tables for pack and mix 3 for verify, the
 *   fastest of each on MI355X (6).
 * CRUM_PARAM_CHUNK_GROWTH: factor, 2..16, by which successive pipelined
 *   chunks and plan groups grow, up to their maximum (4).
 * CRUM_PARAM_PACK_NT_STORE: 1 writes the image with non-temporal stores in
 *   the pack kernel (0).
 * CRUM_PARAM_PACK_PREFETCH: 1 makes each lane of the pack and verify kernels
 *   issue its next loads before folding the current ones into its CRC (0);
 *   it applies with cached loads only (CRUM_PARAM_PACK_NT_LOAD 0).
 * CRUM_PARAM_PACK_NT_LOAD: 1 reads the pages in the pack and verify kernels
 *   with non-temporal loads, which are not kept in the caches (1).
 * CRUM_PARAM_DIFF_GROUP: 4 KiB diff units per wave of the diff kernel, 1, 2
 *   or 4, for launches whose smallest unit is 4 KiB: 2 or 4 units of one
 *   region are read as one span with 8 or 16 loads per array in flight per
 *   lane (16 KiB units always have 16); other values are rejected (2).
 * Values of 0 are rejected (CRUM_EINVAL) except for the on/off switches,
 * the priority and the direct-order size. */
enum {
    CRUM_PARAM_DIFF_BLOCKS = 1,
    CRUM_PARAM_PACK_BLOCKS = 2,
    CRUM_PARAM_CHUNK_BYTES = 3,
    CRUM_PARAM_CHUNK_MAX_BYTES = 4,
    CRUM_PARAM_EAGER = 5,
    CRUM_PARAM_DRAIN_CHUNK_BYTES = 6,
    CRUM_PARAM_DIFF_UNIT_SHIFT = 7,
    CRUM_PARAM_DIFF_NONTEMPORAL = 8,
    CRUM_PARAM_PIECE_SHIFT = 9,
    CRUM_PARAM_PACK_DEPTH = 10,
    CRUM_PARAM_DIFF_PRIORITY = 11,
    CRUM_PARAM_CRC_VARIANT = 12,
    CRUM_PARAM_PLAN_ORDER = 13,
    CRUM_PARAM_DIRECT_BYTES = 14,
    CRUM_PARAM_CHUNK_GROWTH = 15,
    CRUM_PARAM_PACK_NT_STORE = 16,
    CRUM_PARAM_PACK_PREFETCH = 17,
    CRUM_PARAM_PACK_NT_LOAD = 18,
    CRUM_PARAM_DIFF_GROUP = 19
};
int crum_ctx_set_param(crum_ctx* ctx, int param, uint64_t value);
int crum_ctx_get_param(crum_ctx* ctx, int param, uint64_t* value);

/* Per-kernel timing, for measurement.  The context brackets each launch of
 * the selected kernel classes (0 diff, 1 pack, 2 drain copies,
 * 3 scan/bitmap/list, 4 header, 5 verify, 6 scatter; the pack and verify
 * classes time their k_pack launches only, not the k_finalize that combines
 * the CRCs of pages larger than one piece) with timing events:
 * `classes` is a bit mask (bit c selects class c), 0 turns timing off and a
 * negative value selects every class.  Each event record costs host time, so
 * short snapshots are timed with few classes.  crum_ctx_timing returns, for
 * class `which`, the number of launches and the summed duration in
 * milliseconds since the last reset; it waits for the recorded events.
 * A plan created while the diff class is timed has each group's diff kernel
 * write the device's constant-rate wall clock at its start and end; each
 * launch of that plan adds those durations to the diff class and returns
 * only after the plan's drains have ended. */
int crum_ctx_set_timing(crum_ctx* ctx, int classes);
int crum_ctx_timing(crum_ctx* ctx, int which, uint64_t* launches, double* total_ms);
int crum_ctx_timing_reset(crum_ctx* ctx);

/* ---------------------------------------------------------------------------
 * On-demand restore (section 4.2: unified-memory data is brought into the
 * application's copy on read faults; a small region is read whole at its
 * first fault, a large one one page at the first fault and twice as many
 * pages at each later fault of the same region).  The device takes no page
 * faults here, so the caller announces each access with crum_lazy_touch
 * before work that reads or writes the range.
 *
 * The packed pages of the image are absent until fetched; every other page
 * of the regions is taken to hold its bytes already (as in crum_restore).  A
 * touch is a fault when its range covers an absent page.  The fault's window
 * starts at the first absent page the range covers and spans
 * max(2^f, pages to the end of the range) pages, f being the number of
 * earlier faults of the region, clipped at the region's end; a region of at
 * most small_bytes bytes has the whole region as its window.  Every absent
 * image page of the window is fetched: its packed bytes are copied from
 * h_image into d_staging (at their image offsets), CRC-checked with
 * CRUM_VERIFY, and written to the page (and its shadow with
 * CRUM_UPDATE_SHADOW), in runs of consecutive packed pages, one copy per run
 * (runs of up to 2 MiB are read in place from h_image when the device maps
 * it at the same address, as hipHostMalloc memory is).
 *
 * Verification is per fetched run: a run that fails is not written, and
 * neither is anything fetched after it; pages written before stay written.
 * The session then reports CRUM_ECRC (first_bad: lowest failing slot) for
 * every later call.  A session whose image failed the device-side checks of
 * open reports CRUM_EFORMAT for every call and writes nothing.  After a call
 * returns CRUM_EHIP the session is unusable; close it.  Like a context, a
 * session is not thread-safe: calls on one session must not overlap.
 * -------------------------------------------------------------------------*/
typedef struct crum_lazy crum_lazy;

typedef struct {
    uint64_t pages_total;   /* D: packed pages in the image */
    uint64_t pages_fetched; /* pages whose fetch has been enqueued */
    uint64_t faults;        /* touches that found an absent page */
    uint64_t copies;        /* runs of packed pages fetched (copied, or read in place) */
    uint64_t bytes_fetched; /* packed-page bytes copied */
} crum_lazy_info;

/* Start an on-demand restore.  The host checks the header and region table
 * as crum_restore does (returning CRUM_EFORMAT, CRUM_EMISMATCH or, for
 * staging_bytes below image_bytes, CRUM_ENOSPC, written to *h_status, with
 * nothing enqueued and *out NULL), and that the bitmap holds n_dirty bits
 * below total_pages.  Then enqueues on `stream` the upload of the image
 * prefix and CRC array into d_staging, their device-side checks (meta_crc,
 * crcs_crc, bitmap, pads: CRUM_EFORMAT in *h_status) and the slot list; no
 * page is fetched.  h_image (pinned host memory) and d_staging must stay
 * valid and unchanged until crum_lazy_close.  The session keeps the ctx's CRC
 * tables and the launch shapes in force at open; the ctx must outlive it.
 * Returns CRUM_OK, CRUM_EINVAL (bad argument, h_image NULL), an image error
 * above, or CRUM_EHIP. */
int crum_lazy_open(crum_ctx* ctx, const crum_region* regions, uint32_t n_regions,
                   const void* h_image, uint64_t image_bytes, uint32_t flags,
                   uint64_t small_bytes, void* d_staging, uint64_t staging_bytes, void* stream,
                   crum_status* h_status, crum_lazy** out);

/* Announce an access to bytes [offset, offset + len) of region `region`
 * (len > 0, within the region).  Makes `stream` wait for every fetch
 * enqueued before, so work after the call on `stream` sees the pages.  On a
 * fault, enqueues the fetch of its window on `stream` and, when h_status
 * (pinned) is not NULL, the session's status into it; *n_fetched (may be
 * NULL) receives the pages fetched.  A touch that is not a fault enqueues
 * at most the wait (none on the stream of the session's last fetch) and
 * leaves *h_status as it is.  Streams given to a session must stay alive
 * until it is closed.  Returns CRUM_OK, CRUM_EINVAL or CRUM_EHIP. */
int crum_lazy_touch(crum_lazy* lazy, uint32_t region, uint64_t offset, uint64_t len,
                    void* stream, crum_status* h_status, uint64_t* n_fetched);

/* Fetch every page still absent (the rest of a full restore) on `stream`
 * after the earlier fetches; the session's status into *h_status (pinned). */
int crum_lazy_finish(crum_lazy* lazy, void* stream, crum_status* h_status);

/* Counters of the session so far (host values, no wait). */
int crum_lazy_stats(crum_lazy* lazy, crum_lazy_info* out);

/* Which pages have been fetched: bit g % 64 of words[g / 64] is set once the
 * fetch of global page g has been enqueued (pages numbered across regions in
 * table order); n_words words are written. */
int crum_lazy_fetched(crum_lazy* lazy, uint64_t* words, uint64_t n_words);

/* Wait for the session's enqueued work and free it. NULL is ignored. */
void crum_lazy_close(crum_lazy* lazy);

/* ---------------------------------------------------------------------------
 * Persisting images: phase two of the paper's checkpoint (section 3.3), where
 * a forked child writes the image to storage while the application resumes.
 * Here the image is already in pinned host memory when the snapshot ends, so
 * a pool of writer threads persists it to a file while the caller goes on
 * (for example with its next snapshot into another buffer).  The file is cut
 * into chunks of chunk_bytes written in parallel with pwrite at their
 * offsets; with CRUM_WRITE_DIRECT, chunks whose length, offset and buffer
 * are 4 KiB aligned go through an O_DIRECT descriptor when the file system
 * supports one and the kernel accepts the buffer for direct I/O (HIP pinned
 * memory is refused on some systems), the rest through the page cache.  With CRUM_WRITE_SYNC the
 * file's data is flushed (fdatasync) before the write counts as done.
 * Host code only: no HIP call is made.
 * -------------------------------------------------------------------------*/
typedef struct crum_writer crum_writer;

typedef struct {
    int32_t code;      /* CRUM_OK or CRUM_EIO */
    int32_t err;       /* errno of the first failing call, else 0 */
    uint64_t bytes;    /* bytes written (0 on error) */
    uint32_t direct;   /* 1 when some chunk was written with O_DIRECT */
    uint32_t reserved;
    double seconds;    /* from submit until the last byte is written (and synced) */
} crum_write_status;

enum {
    CRUM_EIO = -7,     /* a file could not be opened or written */
    CRUM_EAGAIN = -8   /* crum_writer_poll without wait: not done yet */
};
enum { CRUM_WRITE_DIRECT = 1u, CRUM_WRITE_SYNC = 2u };

/* n_threads 1..256; chunk_bytes a positive multiple of 4096.  Returns
 * CRUM_OK or CRUM_EINVAL. */
int crum_writer_create(uint32_t n_threads, uint64_t chunk_bytes, uint32_t flags,
                       crum_writer** out);
/* Creates or overwrites `path` (its length becomes `bytes` when the write
 * completes) and queues the write of image[0, bytes).  The
 * caller keeps the buffer valid and unchanged until crum_writer_poll reports
 * the ticket done.  Returns CRUM_OK (queued), CRUM_EINVAL, or CRUM_EIO when
 * the file cannot be opened (nothing queued). */
int crum_writer_submit(crum_writer* writer, const char* path, const void* image,
                       uint64_t bytes, uint64_t* ticket);
/* With wait != 0 blocks until the ticket's write is done; fills *out and
 * forgets the ticket.  Without wait returns CRUM_EAGAIN while it runs.
 * CRUM_EINVAL for an unknown (or already collected) ticket. */
int crum_writer_poll(crum_writer* writer, uint64_t ticket, int wait, crum_write_status* out);
/* Waits for every submitted write, then stops the threads. */
void crum_writer_destroy(crum_writer* writer);

#ifdef __cplusplus
}
#endif

#endif /* CRUM_H */
