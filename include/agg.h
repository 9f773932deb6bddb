/*
 * agg.h -- C ABI of libagg.so, the MI355X (gfx950) in-memory aggregation scan.
 *
 * The operation (paper Section 2.1 with the kernel of Figure 4; Section 3.2
 * for the specialised GPU form): read every item x[0..n) of one column and
 * fold it with an aggregation function into one summary value,
 * r = aggregate(r, x[i]) for all i.  Functions: SUM, MIN, MAX, COUNT, AVG.
 * Columns are dense, non-nullable arrays of int32, int64 or float32.
 *
 * Results:
 *   integer SUM     two's-complement sum mod 2^64 of the items widened to
 *                   int64 (exact, bit-identical to any evaluation order);
 *   integer MIN/MAX the extreme item, widened to int64;
 *   COUNT           n;
 *   integer AVG     RN(RN(SUM) / RN(n)) in IEEE double;
 *   float SUM/AVG   an approximation of the exact sum (see agg_prec) held in
 *                   a double; AVG divides it by RN(n);
 *   float MIN/MAX   the extreme item (NaN items skipped), widened to double.
 * Empty column: SUM = 0 and COUNT = 0; MIN, MAX and AVG report is_null = 1.
 *
 * Determinism: for a given (dtype, op, prec, n) the library always uses one
 * canonical reduction shape (agg_canonical_shape).  The result bits depend
 * only on the column's contents and that shape -- not on the tuning
 * parameters, the grid, the source (device / pinned host / zero-copy), or
 * whether the column runs alone (agg_run) or inside a batch (agg_batch_run).
 *
 * Conventions:
 *   - Every function returns AGG_OK (0) or a negative AGG_E_* code and never
 *     aborts; after AGG_E_HIP, agg_last_hip_error() gives the hipError_t.
 *   - Pointers are plain addresses.  The caller owns columns and result
 *     buffers; plans and batches own their workspaces (allocated at creation,
 *     freed by the destroy call), so agg_run and agg_batch_run allocate
 *     nothing.
 *   - Work is asynchronous on the caller's HIP stream (`stream` is a
 *     hipStream_t; NULL = the legacy default stream).  A result is valid once
 *     that stream has been synchronised.
 *   - A plan, batch, group-by plan or server is not re-entrant: two calls that
 *     overlap in time (for instance on two streams) must use two of them.
 */
#ifndef AGG_H
#define AGG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---- */
#define AGG_OK 0
#define AGG_E_INVALID (-1)     /* bad argument: null pointer, n < 0, n > max_n,
                                  bad enum, misaligned or non-device pointer */
#define AGG_E_NOMEM (-2)       /* a workspace allocation failed */
#define AGG_E_NODEVICE (-3)    /* no HIP device, or not a gfx950 device */
#define AGG_E_HIP (-4)         /* a HIP runtime call failed */

/* ---- enums (passed as int32_t) ---- */
enum { AGG_I32 = 0, AGG_I64 = 1, AGG_F32 = 2 };
enum { AGG_SUM = 0, AGG_MIN = 1, AGG_MAX = 2, AGG_COUNT = 3, AGG_AVG = 4 };
/* Float SUM / AVG precision modes (ignored for other dtype/op pairs):
 *   NEUMAIER     per-lane Neumaier-compensated float32 (sum, correction)
 *                pairs, renormalised by an exact two-sum after every 8 rounds
 *                of loads and after the last, combined across lanes by exact
 *                two-sum (then renormalised); each segment partial is
 *                sum + correction in double; double combine.  A-priori bound:
 *                |error| <= 1.01 ((44 ceil(m/8) + 24) u^2 + (k + 8) v) sum|x|
 *                with u = 2^-24, v = 2^-53, m = seg_bytes / 1024 items per
 *                lane accumulator and k = ceil(nseg / 256); for 2^30 items
 *                that is 1.0e-11 sum|x|.
 *   F32          plain float32 everywhere, including the final combine.
 *   F64_COMBINE  plain float32 lanes and wave reduction, segment partials
 *                widened to double, double combine. */
enum { AGG_PREC_NEUMAIER = 0, AGG_PREC_F32 = 1, AGG_PREC_F64_COMBINE = 2 };
/* Where the column lives:
 *   DEVICE       device memory (HBM), the on-device scan;
 *   PINNED_HOST  page-locked host memory, staged to HBM in chunks on a copy
 *                stream that overlaps the scan (end to end, Section 5.3);
 *   ZEROCOPY     page-locked host memory read directly by the kernel over
 *                PCIe. */
enum { AGG_SRC_DEVICE = 0, AGG_SRC_PINNED_HOST = 1, AGG_SRC_ZEROCOPY = 2 };

/* ---- records ---- */
typedef struct agg_result {   /* 32 bytes */
    int64_t i64;      /* integer SUM / MIN / MAX, COUNT; integer AVG: the SUM */
    double f64;       /* float results, AVG; integer results converted */
    int64_t count;    /* n */
    int32_t is_null;  /* 1: MIN / MAX / AVG of an empty column;
                         -1: agg_run_packed met a corrupt block header (its
                         payload would lie outside the buffer, or bits > 32):
                         that block was not read and no other field is valid */
    int32_t prec_used;/* agg_prec for float SUM / AVG, else -1 */
} agg_result;

/* Launch parameters.  None of them changes a result bit. */
typedef struct agg_tune {
    int32_t waves_per_block;  /* 1, 2, 4, 8 or 16 (block = 64 * waves_per_block threads) */
    int32_t blocks_per_cu;    /* 1..32; grid = blocks_per_cu * CU count,
                                 capped by the work available */
    int32_t unroll;           /* 4, 8, 16 or 32 outstanding 16-byte loads per lane */
    int32_t nontemporal;      /* 1: streaming (non-temporal) loads */
    int64_t chunk_bytes;      /* PINNED_HOST: bytes per staged chunk */
    int32_t staging_depth;    /* PINNED_HOST: chunks in flight, 2..4 */
    int32_t reserved;
} agg_tune;

/* The canonical reduction shape of a column.  The column's bytes are cut
 * into nseg contiguous segments of seg_bytes (the last one may be short).
 * Segment j is folded by one wave: lane l reads the 16-byte vectors at
 * byte offsets j*seg_bytes + r*1024 + 16*l for r = 0, 1, ..., each vector
 * component into its own accumulator in order of r; the components are
 * merged as (c0 + c1) + (c2 + c3) (int64 / f32 with 4 per vector) or c0 + c1;
 * the 64 lanes are merged by a fixed butterfly (xor 1, 2; mirrors in 8 and
 * 16 lanes; row pairs; halves).  The nseg segment partials are folded by 256
 * lanes, lane L taking partials L, L + 256, ... in order, then the same
 * butterfly, then the four wave totals as (w0 + w1) + (w2 + w3). */
typedef struct agg_shape {
    int64_t seg_bytes;     /* power of two, >= 16 KiB */
    int64_t nseg;          /* ceil(n * width / seg_bytes), <= 8192 */
    int64_t elems_per_seg; /* seg_bytes / width */
    int32_t width;         /* bytes per item: 4 or 8 */
    int32_t reserved;
} agg_shape;

/* One column of a batch. */
typedef struct agg_col {
    const void* ptr;   /* device address of item 0, aligned to the item width */
    int64_t n;         /* items, >= 0 */
    int32_t dtype;     /* AGG_I32 / AGG_I64 / AGG_F32 */
    int32_t op;        /* AGG_SUM .. AGG_AVG */
    int32_t prec;      /* agg_prec (float SUM / AVG) */
    int32_t reserved;
} agg_col;

typedef struct agg_plan_s* agg_plan_t;
typedef struct agg_batch_s* agg_batch_t;

/* ---- library ---- */

/* Select and check the HIP device (must be gfx950); idempotent per device.
 * Every other call on a device performs it implicitly. */
int agg_init(int32_t device);

/* Device facts used by the tuner: compute-unit count and gfx arch name
 * (written NUL-terminated into arch[arch_len]). */
int agg_device_info(int32_t device, int32_t* cu_count, char* arch, int32_t arch_len);

/* The canonical reduction shape for a column of n items of dtype (pure host
 * computation, no device needed). */
int agg_canonical_shape(int32_t dtype, int64_t n, agg_shape* out);

/* Default launch parameters for (dtype, op, prec, n, src): the tuning-cache
 * entry of the nearest size bucket for that fold kind and source (filled by
 * agg_autotune or agg_tune_load), else the built-in table measured on
 * MI355X. */
int agg_default_tune(int32_t dtype, int32_t op, int32_t prec, int64_t n, int32_t src,
                     agg_tune* out);

/* ---- single column (agg_plan / agg_run) ---- */

/* Create a plan for columns of up to max_n items.  Allocates the device
 * workspace (segment partials, filtered-run counts and two zeroed words,
 * 128 KiB + 256 B; plus
 * staging_depth * chunk_bytes of device staging, a copy stream and events
 * for PINNED_HOST).  tune == NULL: agg_default_tune for max_n. */
int agg_plan(agg_plan_t* out, int32_t dtype, int32_t op, int32_t prec, int64_t max_n,
             int32_t src, const agg_tune* tune);

/* Aggregate col[0..n) into *out on `stream`.  col: an address in the memory
 * the plan's src names, aligned to the item width, with n items readable.
 * out: device memory or page-locked host memory, written by the GPU.
 * Enqueues the scan kernel and the one-workgroup combine kernel (DEVICE,
 * ZEROCOPY; a column of at most 1024 segment partials whose scan runs on at
 * most one workgroup per CU takes the scan launch alone, its last workgroup
 * merging the partials in the same canonical order, so the result bits are
 * the same), or one copy + scan kernel per chunk and then the combine
 * (PINNED_HOST); never allocates and never synchronises the stream, so it
 * may be captured into a HIP graph (DEVICE, ZEROCOPY).  Calls with one plan
 * must not overlap (they share its workspace). */
int agg_run(agg_plan_t plan, const void* col, int64_t n, agg_result* out, void* stream);

/* agg_run without a plan, for callers that cannot allocate (code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation):
 * it allocates nothing, on the device or the host.  The segment partials (and
 * the single-launch scan's finished-workgroup counter) live in a
 * 64 KiB + 256 B array in the library's device code, one per device (held until
 * the process ends; agg_init sets it up, else the first call on a device).
 * Same kernels, canonical shape and result bits as agg_run with a plan of the
 * same (dtype, op, prec); launch parameters from agg_default_tune.
 *   src: AGG_SRC_DEVICE or AGG_SRC_ZEROCOPY (PINNED_HOST would need a staging
 *        ring, so it is AGG_E_INVALID);
 *   col, n, out: as for agg_run; n <= 2^40 (any such column fits the array).
 * All calls on one device share its array: two calls that overlap in time on
 * that device (two streams, two threads) race and give wrong results;
 * serialise them (for instance on one stream).  Returns AGG_E_INVALID for bad
 * arguments, AGG_E_NODEVICE without a gfx950 device, AGG_E_HIP if the array's
 * address cannot be obtained. */
int agg_run_noalloc(int32_t dtype, int32_t op, int32_t prec, int32_t src, const void* col, int64_t n,
                    agg_result* out, void* stream);

/* The canonical shape and launch parameters the plan uses for n items. */
int agg_plan_info(agg_plan_t plan, int64_t n, agg_shape* shape, agg_tune* tune);

int agg_plan_destroy(agg_plan_t plan);

/* ---- many columns in one launch (agg_batch) ---- */

/* Build a batch over cols[0..ncols): the work table (runs of whole segments
 * of each column), partial and result buffers, and a HIP graph holding the
 * persistent scan kernel and the per-column combine kernel.  Column memory
 * must stay valid and unchanged in address while the batch is used; its
 * contents may change between runs. */
int agg_batch_plan(agg_batch_t* out, const agg_col* cols, int32_t ncols, const agg_tune* tune);

/* Launch the batch graph on `stream` and copy the ncols results into
 * out[0..ncols) (device or page-locked host memory). */
int agg_batch_run(agg_batch_t batch, agg_result* out, void* stream);

int agg_batch_destroy(agg_batch_t batch);

/* Work items, total segments and the launch parameters the batch graph uses. */
int agg_batch_info(agg_batch_t batch, int64_t* nitems, int64_t* nseg_total, agg_tune* tune);

/* Re-capture the batch graph with other launch parameters (results
 * unchanged).  Waits for the batch's previous runs to finish. */
int agg_batch_retune(agg_batch_t batch, const agg_tune* tune);

/* Time the batch graph under a fixed set of launch parameters on `stream`
 * (waves per block x blocks per CU x loads in flight), keep the fastest and
 * return it with its time per run in milliseconds.  Synchronises `stream`. */
int agg_batch_autotune(agg_batch_t batch, void* stream, agg_tune* best, double* best_ms);

/* ---- autotuner and tuning cache ---- */

/* Time a fixed set of candidate launch parameters for (dtype, op, prec) on
 * the caller's column col[0..n) in memory of kind `src` (device: waves per
 * block x blocks per CU x loads in flight, then temporal vs non-temporal
 * loads; pinned host: staging chunk x depth), on `stream`.  The fastest goes
 * into the process-wide tuning cache under (fold kind, src, size bucket
 * ceil(log2(n * width))) and is returned with its GB/s.  Creates and destroys
 * temporary plans (so it allocates) and synchronises `stream`. */
int agg_autotune(int32_t dtype, int32_t op, int32_t prec, const void* col, int64_t n, int32_t src,
                 void* stream, agg_tune* best, double* best_gbs);

/* Persist / restore the tuning cache as JSON.  A file written for another
 * gfx arch or CU count, or one that does not parse, is rejected with
 * AGG_E_INVALID and leaves the cache unchanged. */
int agg_tune_save(const char* path);
int agg_tune_load(const char* path);
int agg_tune_clear(void);

/* ---- fused filter + aggregate ---- */

/* A range predicate on a second column of the same length: item i of the
 * value column is aggregated when lo <= y[i] <= hi (each bound inclusive or
 * exclusive) for the filter column y.  Integer filter columns compare as
 * int64 against ilo / ihi, float32 ones as double against flo / fhi (NaN
 * items are never selected; use +-infinity for an open side).  Operator
 * fusion is the paper's stated next step (Section 8): both columns are read
 * once in the same scan instead of materialising a selection. */
typedef struct agg_filter {
    const void* col;        /* filter column, device memory, aligned to its item width */
    int32_t dtype;          /* AGG_I32 / AGG_I64 / AGG_F32 */
    int32_t lo_inclusive;   /* 1: y >= lo; 0: y > lo */
    int32_t hi_inclusive;   /* 1: y <= hi; 0: y < hi */
    int32_t reserved;
    int64_t ilo, ihi;       /* bounds for integer filter columns */
    double flo, fhi;        /* bounds for float32 filter columns */
} agg_filter;

/* Aggregate the selected items of col[0..n) (plan src must be AGG_SRC_DEVICE).
 * The reduction shape is the value column's canonical shape with every
 * unselected item replaced by the function's identity, so an always-true
 * predicate gives agg_run's bits.  COUNT = number of selected items; AVG
 * divides by it; MIN / MAX / AVG are null when nothing is selected; the
 * result's count field is the selected count.  (A float SUM whose selected
 * items sum to -0.0 may come out as +0.0.) */
int agg_run_filtered(agg_plan_t plan, const void* col, int64_t n, const agg_filter* filter,
                     agg_result* out, void* stream);

/* ---- group-by aggregation ---- */

/* For every distinct key k of keys[0..n), the aggregate of the values whose
 * key is k (the group-by aggregation of the prior GPU work the paper cites,
 * Section 7).  Per group: integer SUM mod 2^64, MIN, MAX, COUNT and AVG as for
 * whole columns; float SUM is the exact sum of the group's items rounded
 * once to double (accumulated in fixed-point digits, so every result is
 * deterministic and independent of thread order), float AVG divides it by
 * the count, float MIN / MAX skip NaN.  Groups come out in an unspecified
 * order. */
typedef struct agg_group {   /* 32 bytes */
    int64_t key;
    int64_t i64;     /* integer SUM / MIN / MAX, COUNT; integer AVG: the SUM */
    double f64;      /* float results, AVG; integer results converted */
    int64_t count;   /* items in the group */
} agg_group;

typedef struct agg_groupby_s* agg_groupby_t;

/* Plan a group-by for int32 / int64 keys and int32 / int64 / float32 values
 * with up to max_n items and max_groups distinct keys: allocates the device
 * hash table (2 x max_groups slots rounded up to a power of two; float SUM /
 * AVG tables carry 9 fixed-point digits per slot); with more groups than a
 * workgroup's LDS table holds, also a staging copy of min(max_n, 2^28) rows
 * and a partition histogram.  max_n <= 2^36; float SUM / AVG plans take at most
 * 2^31 items per run. */
int agg_groupby_plan(agg_groupby_t* out, int32_t key_dtype, int32_t val_dtype, int32_t op, int64_t max_n,
                     int64_t max_groups);

/* Group keys[0..n) / vals[0..n) (device memory) on `stream`: writes up to
 * max_groups groups to groups[] (device memory) and the number of groups to
 * *ngroups (device or page-locked host memory), or -1 if the input has more
 * distinct keys than the plan's max_groups.  Never allocates. */
int agg_groupby_run(agg_groupby_t plan, const void* keys, const void* vals, int64_t n, agg_group* groups,
                    int64_t* ngroups, void* stream);

int agg_groupby_destroy(agg_groupby_t plan);

/* ---- compressed int32 columns (frame of reference + bit packing) ---- */

/* The paper finds host-to-device transfer to dominate end-to-end time and
 * names compression as the way to cut it (Sections 5.3 and 8).  A packed
 * column stores int32 items in blocks of AGG_PACK_BLOCK items: block b holds
 * items [b*2048, b*2048 + 2048) as base = their minimum and, for each item,
 * d = item - base (< 2^32) in `bits` bits, bits = bit width of (max - base).
 * Payload of a block: 64 * bits 32-bit words at payload[word_off ...]; word
 * j * 64 + l is word j of lane l, and lane l's `bits` words hold the d of
 * items b*2048 + 32*l + i, i = 0..31, item i in bits [i*bits, (i+1)*bits) of
 * the lane's words taken as one little-endian bit string.  Items past n in
 * the last block are encoded as d = 0.  Every item is recovered exactly, so
 * SUM / MIN / MAX / COUNT / AVG of a packed column equal those of the raw
 * column bit for bit. */
#define AGG_PACK_BLOCK 2048

typedef struct agg_packed_block {  /* 16 bytes */
    int32_t base;
    uint32_t bits;      /* 0..32 */
    int64_t word_off;   /* first payload word of the block */
} agg_packed_block;

typedef struct agg_packed {
    const agg_packed_block* blocks;  /* nblocks = ceil(n / 2048) entries */
    const uint32_t* payload;
    int64_t n;                       /* items */
    int64_t payload_words;
    int32_t dtype;                   /* AGG_I32 */
    int32_t reserved;
} agg_packed;

/* Upper bound of payload words for n items (every block at 32 bits). */
int agg_pack_bound(int64_t n, int64_t* max_payload_words);

/* Encode x[0..n) (host memory) into blocks[ceil(n/2048)] and payload
 * (host memory of payload_cap words) with `threads` host threads (<= 0: one
 * per core, at most 64); *payload_words receives the words used.  Pure host
 * code, no device needed. */
int agg_pack_i32(const int32_t* x, int64_t n, agg_packed_block* blocks, uint32_t* payload,
                 int64_t payload_cap, int64_t* payload_words, int32_t threads);

/* Aggregate a packed column with a plan for dtype AGG_I32 (any op) whose
 * src is AGG_SRC_DEVICE (blocks and payload in device memory) or
 * AGG_SRC_ZEROCOPY (in page-locked host memory, read by the kernel over PCIe
 * as it decodes).  n <= the plan's max_n.  Enqueues the decoding scan and the
 * combine on `stream`; results equal agg_run on the raw column.  The headers
 * live in memory the host does not read here, so a corrupt one is found by
 * the kernel: it reads nothing through it and the result comes back with
 * is_null = -1 (COUNT reads no block and always gives n). */
int agg_run_packed(agg_plan_t plan, const agg_packed* col, agg_result* out, void* stream);

/* ---- serving: continuous admission of requests (agg_serve) ---- */

typedef struct agg_server_s* agg_server_t;

/* One aggregation request.  Requests passed to agg_serve_run are sorted by
 * arrival_s.  A resident request reads device memory; a shipped one reads
 * page-locked host memory, which the server copies over PCIe into its HBM
 * arena.  Requests with the same column_id must name the same bytes. */
typedef struct agg_request {
    const void* ptr;     /* item 0: device address (resident) or pinned host address (shipped) */
    int64_t n;           /* items */
    int64_t column_id;   /* identity of the column's contents (for the resident cache) */
    double arrival_s;    /* seconds after agg_serve_run starts */
    int32_t dtype, op, prec;
    int32_t resident;    /* 1: ptr is device memory; 0: ship from pinned host memory */
} agg_request;

typedef struct agg_serve_config {
    int64_t hbm_budget_bytes;  /* device arena for shipped (and cached) columns */
    int32_t max_slots;         /* requests in flight on the GPU, 1..64; each slot owns
                                  a compute stream and a copy stream */
    int32_t cache_shipped;     /* 1: a shipped column stays in the arena after its request
                                  (LRU eviction by need), serving later requests with the
                                  same column_id without PCIe traffic */
    int64_t chunk_bytes;       /* copy / scan pipelining chunk for shipped columns */
    int32_t max_shipping;      /* shipped requests in flight at once, 1..max_slots: they
                                  share one PCIe link, so more only stretches each of them
                                  and holds slots that resident requests could use */
    int32_t progress_every;    /* > 0: agg_serve_run writes a line to stderr each time this
                                  many more requests have completed (long runs); 0: silent */
} agg_serve_config;

typedef struct agg_request_stats {
    double arrival_s;      /* as requested */
    double admit_s;        /* when the scheduler gave it a slot (and memory) */
    double done_s;         /* when the host saw its result */
    int64_t bytes_shipped; /* bytes copied over PCIe for it */
    int32_t slot;          /* slot it ran in, -1 if never admitted */
    int32_t status;        /* AGG_OK; AGG_E_NOMEM if the column exceeds the whole budget */
    int32_t cache_hit;     /* 1: served from a cached copy */
    int32_t reserved;
} agg_request_stats;

typedef struct agg_serve_summary {
    double makespan_s;            /* first arrival to last completion */
    int64_t bytes_scanned;
    int64_t bytes_shipped;
    int64_t peak_reserved_bytes;  /* high-water mark of the arena (<= the budget) */
    int32_t peak_busy_slots;      /* most requests in flight at once */
    int32_t completed, failed, cache_hits;
} agg_serve_summary;

/* Create a server: allocates the hbm_budget_bytes arena, per-slot streams,
 * events and partial workspaces, and page-locked result slots. */
int agg_serve_create(agg_server_t* out, const agg_serve_config* cfg);

/* Serve reqs[0..n) in real time on the current device.  The scheduler
 * releases each request at its arrival time, admits waiting requests in
 * arrival order whenever a slot is free and, for a shipped request, fewer
 * than max_shipping shipped requests are in flight and the arena has room
 * (evicting idle cached columns in LRU order); a shipped request that cannot
 * start holds back later shipped requests but not resident or cached ones.  Each admitted request runs the agg_run kernels
 * (same canonical shape, hence the same bits as alone) on its slot's
 * streams, copies of shipped chunks overlapping the scan of earlier chunks.
 * Fills results[i] (host memory) and stats[i]; returns when all are done.
 * Pointers are validated up front (AGG_E_INVALID before any work). */
int agg_serve_run(agg_server_t server, const agg_request* reqs, int32_t n, agg_result* results,
                  agg_request_stats* stats, agg_serve_summary* summary);

int agg_serve_destroy(agg_server_t server);

/* The same scheduler on the CPU with a simulated clock: copies share one
 * link of pcie_gbs GB/s, scans run at hbm_gbs GB/s, each request adds
 * launch_s seconds.  No device is touched; for testing the admission,
 * budget and cache logic. */
int agg_serve_simulate(const agg_serve_config* cfg, const agg_request* reqs, int32_t n, double pcie_gbs,
                       double hbm_gbs, double launch_s, agg_request_stats* stats,
                       agg_serve_summary* summary);

/* ---- errors ---- */
const char* agg_strerror(int32_t code);
int32_t agg_last_hip_error(void);  /* hipError_t of the last AGG_E_HIP on this thread */

/* ---- fault injection (tests of the error paths) ----
 * Not part of the paper's method: it forces, from the host, failures the
 * hardware rarely produces, so that tests can check that every call reports
 * them with a status code and that plans, batches, group-by plans and
 * servers stay usable afterwards.  A countdown per site: the countdown-th
 * next event at the site fails (1 = the next one), 0 disarms it.
 *   AGG_FAULT_ALLOC  a device or page-locked host allocation made by the
 *                    library (agg_plan, agg_batch_plan, agg_groupby_plan,
 *                    agg_serve_create, agg_autotune): the call returns
 *                    AGG_E_NOMEM and allocates nothing.
 *   AGG_FAULT_SHIP   the host-to-device copy of a chunk of a shipped serving
 *                    request (agg_serve_run; in agg_serve_simulate, the
 *                    simulated copy): that request ends with status AGG_E_HIP
 *                    (agg_last_hip_error() = hipErrorUnknown), its arena
 *                    region is freed and never cached, and later requests run
 *                    normally.
 * The failing runtime call is never issued, so nothing reaches the device.
 * The environment variable AGG_FAULT_INJECT="alloc:n,ship:n" arms the
 * countdowns at the library's first call; agg_fault_inject overrides it.
 * Counters are process-wide; concurrent calls share them. */
enum { AGG_FAULT_NONE = 0, AGG_FAULT_ALLOC = 1, AGG_FAULT_SHIP = 2, AGG_FAULT_SITES = 3 };
int agg_fault_inject(int32_t site, int32_t countdown);

#ifdef __cplusplus
}
#endif

#endif /* AGG_H */
