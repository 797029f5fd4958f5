/*
 * dfr.h -- C ABI of a GPU implementation of the Diverting Fast Radix (DFR) sort
 * (Thiel et al., "ThielSort: Implementing the Diverting Fast Radix Algorithm",
 * arXiv 2207.14334) for AMD Instinct MI355X (gfx950).
 *
 * The problem (Sec. 2.2, diverting-MSD paragraph; Sec. 3): records held in an input
 * area, an extra buffer of the same size, and the key's digits; the result ends in
 * the original area (Sec. 2.1: the last deal lands back in the original space).
 * Every sort here is a *stable* ascending sort of unsigned integer keys, with an
 * optional payload that travels with its key.  The output is the unique
 * arrangement in which record i sits at
 *     rank(i) = #{ j : k_j < k_i } + #{ j < i : k_j == k_i }.
 *
 * Memory.  keys, vals and temp are DEVICE pointers owned by the caller; they must
 * stay allocated and untouched until the work enqueued on `stream` has finished.
 * Arrays are contiguous structure-of-arrays: keys[n] and, when given, vals[n] of
 * the stated widths.  Pointers must be aligned to their element size.  keys, vals
 * and temp must not overlap.  The context owns a small amount of scratch device
 * memory (histograms, look-back words, bucket lists) that it grows on demand and
 * frees in dfr_destroy.
 *
 * Streams.  `stream` is a hipStream_t passed as void*; NULL is the null stream.
 * Work is enqueued on that stream in order.  A sort call blocks the calling host
 * thread while it reads small planning results back from the device (digit
 * histograms, bucket lists); when it returns DFR_OK the sorted result may still be
 * in flight on `stream`.
 *
 * Errors.  Every call returns a dfr_status.  Argument errors are detected before any
 * device work is enqueued and leave the buffers untouched.  A HIP runtime failure
 * returns DFR_E_HIP, marks the context failed (later calls return DFR_E_HIP) and
 * records text for dfr_last_error.  Contexts are not thread-safe.
 */
#ifndef DFR_H
#define DFR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t dfr_status;

#define DFR_OK 0
#define DFR_E_INVALID_ARG (-1) /* NULL with n > 0, misaligned, overlapping, bad width,  */
                               /* temp too small, malformed segment offsets           */
#define DFR_E_TOO_LARGE (-2)   /* a segment of 2^32 records or more                    */
#define DFR_E_NO_MEMORY (-3)   /* device scratch could not be allocated               */
#define DFR_E_HIP (-4)         /* HIP runtime error; detail in dfr_last_error          */
#define DFR_E_PENDING (-5)     /* request not finished yet                             */
#define DFR_E_NOT_FOUND (-6)   /* unknown ticket                                       */
#define DFR_E_BUDGET (-7)      /* request can never fit the context's memory budget    */
#define DFR_E_UNSUPPORTED (-8) /* entry point or option not available                  */
#define DFR_E_INTERNAL (-9)    /* a kernel's bounded wait expired; results invalid     */

/* Largest number of records in one sort, or in one segment of a segmented sort,
 * 2^32 - 1: digit counts, bucket positions inside a segment and the deal's scatter
 * offsets are 32-bit. */
#define DFR_MAX_SEGMENT_RECORDS ((size_t)0xffffffffu)

typedef struct dfr_ctx dfr_ctx;

/* Create a context bound to HIP device `hip_device`.  `hbm_budget_bytes` bounds the
 * device memory that queued requests (dfr_submit) may hold at once; 0 means a
 * quarter of the device's memory.  On success *out receives the context. */
dfr_status dfr_create(int hip_device, size_t hbm_budget_bytes, dfr_ctx** out);

/* Wait for the context's own work, then free its scratch memory and the context. */
void dfr_destroy(dfr_ctx* ctx);

/* Static text for a status code. */
const char* dfr_status_string(dfr_status s);

/* Text of the last error recorded on `ctx` ("" if none); valid until the next call. */
const char* dfr_last_error(const dfr_ctx* ctx);

/* Bytes of caller-provided temp storage a sort of n records needs: the extra buffer
 * of the paper's statement of the problem (Sec. 2.2), n * (key_bytes + val_bytes),
 * rounded up to 256 bytes.  key_bytes is 4 or 8; val_bytes 0, 4 or 8. */
size_t dfr_temp_bytes(size_t n, int key_bytes, int val_bytes);

/* ---------------------------------------------------------------------------------
 * Plain sort (Sec. 3, DFR; Alg. 4 in the paper).
 *
 * Stable ascending sort of keys[0..n) in place; vals[0..n) (may be NULL) moves with
 * its key.  temp: device buffer of at least dfr_temp_bytes(n, kb, vb) bytes, or NULL
 * to use storage the context allocates once and caches.  n <= 1 returns DFR_OK with
 * nothing enqueued.  n > DFR_MAX_SEGMENT_RECORDS returns DFR_E_TOO_LARGE.
 * ------------------------------------------------------------------------------- */
dfr_status dfr_sort_u32(dfr_ctx* ctx, uint32_t* keys, uint32_t* vals, size_t n, void* temp,
                        size_t temp_bytes, void* stream);
dfr_status dfr_sort_u64(dfr_ctx* ctx, uint64_t* keys, uint64_t* vals, size_t n, void* temp,
                        size_t temp_bytes, void* stream);

/* ---------------------------------------------------------------------------------
 * Allocation-free plain sort, for callers that cannot allocate device memory: code
 * under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
 *
 * The same stable ascending sort as dfr_sort_u32/u64 (unsigned keys of key_bytes 4 or
 * 8; vals NULL with val_bytes 0, else val_bytes 4 or 8), on at most
 * DFR_NOALLOC_MAX_RECORDS records, at the default launch settings (the context's
 * options and tunings do not apply; "timing" is ignored).  It allocates nothing:
 * the temp buffer, the per-level lists and the status block live in a fixed device
 * array of DFR_NOALLOC_SCRATCH_BYTES that the library holds on every GPU it runs on
 * until the process ends (its address is looked up once per device by dfr_create),
 * and the host staging is the pinned buffer dfr_create reserves.  Every such call on
 * one GPU, from any context, shares that GPU's array and leaves its contents behind;
 * calls that overlap in time on one GPU (different streams or threads) race on it and
 * must be serialised by the caller.  Like the plain sort it blocks the host for its
 * planning read-backs.  DFR_E_TOO_LARGE for n > DFR_NOALLOC_MAX_RECORDS; other errors
 * as for the plain sort.
 * ------------------------------------------------------------------------------- */
#define DFR_NOALLOC_MAX_RECORDS ((size_t)1 << 22)
#define DFR_NOALLOC_SCRATCH_BYTES ((size_t)192 << 20)

dfr_status dfr_sort_noalloc(dfr_ctx* ctx, void* keys, void* vals, size_t n, int key_bytes,
                            int val_bytes, void* stream);

/* ---------------------------------------------------------------------------------
 * Segmented sort: many independent arrays laid end to end, each sorted on its own
 * exactly as the plain sort would sort it (Sec. 3; large buckets are themselves
 * sorted by the same procedure).
 *
 * seg_offsets: num_segments + 1 entries, seg_offsets[0] == 0, non-decreasing,
 * seg_offsets[num_segments] == n (total records), in host memory or in device memory
 * (then read back after the work already queued on `stream`, which blocks the host
 * until that work is done).  Empty segments are allowed.  keys/vals/temp as for the
 * plain sort, covering all n records.
 * ------------------------------------------------------------------------------- */
dfr_status dfr_sort_segmented_u32(dfr_ctx* ctx, uint32_t* keys, uint32_t* vals,
                                  const uint64_t* seg_offsets, size_t num_segments,
                                  void* temp, size_t temp_bytes, void* stream);
dfr_status dfr_sort_segmented_u64(dfr_ctx* ctx, uint64_t* keys, uint64_t* vals,
                                  const uint64_t* seg_offsets, size_t num_segments,
                                  void* temp, size_t temp_bytes, void* stream);

/* ---------------------------------------------------------------------------------
 * Signed and floating-point keys.  The paper sorts unsigned integer keys; these
 * entry points map the keys in place to unsigned integers of the same order, sort
 * those, and map them back, so the caller's keys end sorted in their own encoding:
 *   DFR_KEY_I32/I64  two's-complement value order (sign bit flipped for the sort);
 *   DFR_KEY_F32/F64  IEEE 754 totalOrder: -NaN < -inf < ... < -0 < +0 < ... < +inf
 *                    < +NaN, NaNs by payload (negative encodings fully inverted,
 *                    positive ones with the sign bit flipped, for the sort).
 * DFR_KEY_U32/U64 sort as dfr_sort_u32/u64.  val_bytes is 0 (vals NULL), 4 or 8,
 * independent of the key width.  Arguments, errors and temp as for the plain and
 * segmented sorts; after an error past argument checking the keys are still mapped
 * back.  Two extra passes over the keys (read and write) per call.
 * ------------------------------------------------------------------------------- */
#define DFR_KEY_U32 0
#define DFR_KEY_U64 1
#define DFR_KEY_I32 2
#define DFR_KEY_I64 3
#define DFR_KEY_F32 4
#define DFR_KEY_F64 5

dfr_status dfr_sort_keys(dfr_ctx* ctx, int32_t key_type, void* keys, void* vals, int val_bytes,
                         size_t n, void* temp, size_t temp_bytes, void* stream);
dfr_status dfr_sort_segmented_keys(dfr_ctx* ctx, int32_t key_type, void* keys, void* vals,
                                   int val_bytes, const uint64_t* seg_offsets,
                                   size_t num_segments, void* temp, size_t temp_bytes,
                                   void* stream);

/* ---------------------------------------------------------------------------------
 * Stages, in the paper's vocabulary (Sec. 2): a count and a deal on one digit.
 * ------------------------------------------------------------------------------- */

/* count: for every digit j < num_digits, hist[j * 2^bits + v] = number of keys whose
 * digit j, (key >> (j * bits)) mod 2^bits, equals v.  hist is a DEVICE array of
 * num_digits * 2^bits uint32 entries, overwritten.  bits in [1, 8];
 * num_digits * bits <= 8 * key_bytes. */
dfr_status dfr_count(dfr_ctx* ctx, const void* keys, int key_bytes, size_t n, int bits,
                     int num_digits, uint32_t* hist, void* stream);

/* deal: one stable counting-sort pass on the digit (key >> shift) mod 2^bits, from
 * (keys_in, vals_in) to (keys_out, vals_out): records with a smaller digit come
 * first and records with equal digits keep their input order.  vals_in/vals_out may
 * be NULL together (val_bytes then 0).  bits in [1, 8]; shift + bits <= 8*key_bytes.
 * Output arrays must not overlap the inputs. */
dfr_status dfr_deal(dfr_ctx* ctx, const void* keys_in, const void* vals_in, void* keys_out,
                    void* vals_out, int key_bytes, int val_bytes, size_t n, int shift,
                    int bits, void* stream);

/* Bandwidth reference: copy `bytes` (a multiple of 16; both pointers 16-byte aligned,
 * not overlapping) from src to dst on the device with a plain streaming kernel of this
 * library, enqueued on `stream`.  Every pass of the sort reads and writes each record
 * once, as this copy does, so its rate is the ceiling those passes are measured
 * against beside the HBM peak.  DFR_E_INVALID_ARG for bad pointers or sizes. */
dfr_status dfr_stream_copy(dfr_ctx* ctx, const void* src, void* dst, size_t bytes, void* stream);

/* Bandwidth reference of the counts: read `bytes` (a multiple of 16, possibly 0; src
 * 16-byte aligned) on the device with a plain streaming kernel of this library,
 * enqueued on `stream`, and write the XOR of every 32-bit word read to *xor_out (one
 * device word, 4-byte aligned, outside the source; 0 for no bytes).  A count reads each
 * key once and writes little, so this rate is its ceiling beside the HBM peak.
 * DFR_E_INVALID_ARG for bad pointers or sizes. */
dfr_status dfr_stream_read(dfr_ctx* ctx, const void* src, size_t bytes, uint32_t* xor_out,
                           void* stream);

/* ---------------------------------------------------------------------------------
 * Serving: submit sort requests of any size and width, poll for completion.
 *
 * Requests are sorted by worker threads of the context (3 by default), each with its
 * own HIP stream and scratch.  A worker takes the oldest queued request and every
 * later queued request with the same widths and at most "serve_gather_records"
 * records, up to "serve_batch_records" records in all (a larger request is sorted
 * alone), and sorts them as one segmented sort (each request is one segment, so the
 * result is the one a plain sort of that request alone gives): the records are
 * gathered into a staging buffer, sorted, and scattered back into the requests' own
 * buffers (a batch of one request is sorted in place).  Requests that arrive while
 * batches run join the next batch; the workers' batches overlap on the device.
 * Device memory the workers hold (staging, temp, scratch) stays within the
 * context's HBM budget (dfr_create): batches shrink, or wait, to fit.
 * ------------------------------------------------------------------------------- */
typedef struct {
    int key_bytes; /* 4 or 8 */
    int val_bytes; /* 0, or equal to key_bytes */
    void* keys;    /* device, sorted in place */
    void* vals;    /* device, or NULL with val_bytes 0 */
    size_t n;      /* at most DFR_MAX_SEGMENT_RECORDS */
} dfr_request;

/* Queue a request; *ticket identifies it.  The request's device memory must hold its
 * data when this is called (all writes to it complete) and must stay alive and
 * untouched until dfr_poll returns a status other than DFR_E_PENDING for it.
 * DFR_E_INVALID_ARG for bad widths, pointers or overlapping keys/vals;
 * DFR_E_TOO_LARGE beyond DFR_MAX_SEGMENT_RECORDS; DFR_E_BUDGET if the request alone
 * needs more device memory than the budget.  Thread-safe with dfr_poll. */
dfr_status dfr_submit(dfr_ctx* ctx, const dfr_request* req, uint64_t* ticket);

/* DFR_OK once the request's result is in place (the ticket is then consumed and
 * *latency_s, if not NULL, receives the seconds from its submit to the end of its
 * batch on the device); DFR_E_PENDING while it is queued or running; DFR_E_NOT_FOUND
 * for an unknown or consumed ticket; another status (consuming the ticket) if its
 * batch failed, with detail in dfr_last_error.  Thread-safe with dfr_submit. */
dfr_status dfr_poll(dfr_ctx* ctx, uint64_t ticket, double* latency_s);

typedef struct {
    uint64_t batches;            /* batches sorted                                */
    uint64_t requests;           /* requests completed                            */
    uint64_t records;            /* records sorted                                */
    uint64_t max_batch_requests; /* most requests in one batch                    */
    uint64_t peak_held_bytes;    /* most device memory held by the workers        */
    uint64_t budget_bytes;       /* the context's HBM budget                      */
    uint64_t held_bytes;         /* device memory the workers hold now            */
    uint64_t queued;             /* requests waiting for a batch now              */
    uint64_t allocs;             /* device allocations the workers made           */
    double ms_alloc;             /* host time in those allocations (and frees)    */
    double ms_batch_wall;        /* host time from batch start to its completion  */
    double ms_gather;            /* device time gathering requests into batches   */
    double ms_sort;              /* device time sorting batches                   */
    double ms_scatter;           /* device time scattering results back           */
    int32_t workers;             /* worker threads (0 before the first submit)    */
} dfr_serve_stats;

/* Counters of the serving workers (all zero before the first submit). */
dfr_status dfr_get_serve_stats(dfr_ctx* ctx, dfr_serve_stats* out);

/* ---------------------------------------------------------------------------------
 * Options, plan inspection and timing.
 * ------------------------------------------------------------------------------- */

/* Set a tuning option on the context.  Names:
 *   "divert_records"  N_d, the bucket size below which buckets are diverted to the
 *                     in-LDS local sort (Sec. 3.1); clamped to the local sort's
 *                     capacity.  0 restores the default.
 *   "force_top_digits" d, the number of top digits dealt before diversion at the
 *                     first level (0 = estimate it, Sec. 3).  A value >= the number
 *                     of varying digits deals all of them (plain LSD, Sec. 2.1).
 *   "timing"          1 to record per-stage kernel durations with HIP events, 2 to
 *                     record only the deal launches (fewer events in the stream), 0
 *                     to stop.
 *   "force_lookback"  1 to deal every level with decoupled look-back between tiles
 *                     instead of scanning the tiles' bucket bases ahead of the deal
 *                     (same result; for testing and measurement), 0 to restore.
 *   "force_key_heads" 1 to find every level's bucket heads by reading the keys, also
 *                     where a level could take them from its digit counts (one segment
 *                     dealt on two digits) or histograms (dealt on one digit); same
 *                     result, for testing.  0 to restore.
 *   "estimated_buckets" 1 to deal the first level of a plain sort the Fast Radix way
 *                     (Sec. 3): no count, two top digits when n alone predicts two for
 *                     uniform keys, the lower one dealt into buckets of estimated size
 *                     n / 2^b with overflow slots (Sec. 3.1), the upper one counted in
 *                     that pass and dealt exactly; a level whose buckets outgrow their
 *                     slots is dealt with counted buckets instead.  Same result.  0 to
 *                     restore.
 *   "plan_lengths_records" first levels whose segments all hold at most this many
 *                     records choose their top digits from the lengths alone, as for
 *                     uniform keys (Sec. 3.1), instead of from their digit histograms,
 *                     so that nothing is read back before their deals (a one-level sort
 *                     then waits on the device only at its end); skewed keys may then
 *                     leave large buckets to a second level.  0 (the default) always
 *                     plans from the histograms.  Same result.
 *   "radix_bits"      digit width b of the deal passes, 4..8 with at most 8 digits
 *                     per key (so 8 for 64-bit keys); the paper's digits are 8 bits
 *                     (Sec. 4).  0 = tuned or default.
 *   "tile_records"    records per deal tile: dfr_deal_tile_records(kb, vb) or half
 *                     of it.  0 = tuned or default.
 *   "serve_workers"   worker threads of the serving queue, 1..8 (default 3),
 *   "serve_batch_records" most records in one serving batch (default 2^25), and
 *   "serve_gather_records" largest request gathered into a batch with others (larger
 *                     ones are sorted alone, in place; default 2^20, 0 = no limit); all
 *                     three only before the first dfr_submit (DFR_E_UNSUPPORTED after).
 *   "serve_fail_batches" test hook: the next this-many serving batches are reported
 *                     failed (DFR_E_HIP from dfr_poll for each of their requests) once
 *                     their device work is queued; the worker still waits for that work
 *                     before the requests are done.  0 (the default) injects nothing.
 *   "window_records"  width of the windows that pack runs of small buckets into
 *                     local-sort chunks (Sec. 3: runs of small buckets), 16 ..
 *                     capacity / 2.  0 = tuned or default.
 * "radix_bits", "tile_records", "window_records" and "divert_records" override a
 * tuned setting (dfr_autotune);
 * a combination that no kernel supports falls back to the defaults.  None of them
 * changes the result.  Unknown names return DFR_E_UNSUPPORTED. */
dfr_status dfr_set_option(dfr_ctx* ctx, const char* name, int64_t value);

/* What the last sort call did.  Kernel times are in milliseconds and are filled
 * only while the "timing" option is on (they force a stream synchronisation). */
typedef struct {
    int32_t levels;           /* recursion levels run (1 = no recursion)          */
    int32_t top_digits;       /* digits dealt at the first level                  */
    int32_t deal_passes;      /* deal launches over all levels                    */
    int32_t used_diversion;   /* 1 if the local sort finished buckets             */
    uint64_t large_buckets;   /* buckets recursed on, over all levels             */
    uint64_t chunks;          /* local-sort work items, over all levels           */
    double ms_count;          /* summed kernel time per stage (timing option)     */
    double ms_deal;
    double ms_buckets;
    double ms_local_sort;
    double ms_other;
    int32_t deal_launches_timed; /* number of deal launches summed in ms_deal     */
    double estimated_overflow; /* fraction of the records that Fast Radix's
                                  estimated buckets (ceil(n / 2^b) slots each, Sec.
                                  3.1) would have overflowed when dealing the first
                                  level's top varying digit; measured from the counts */
    /* Which kernel forms ran, over all levels (for tests and profiling). */
    uint64_t chunks_form0;       /* local-sort chunks sorted on 32-bit words holding
                                    their position                                   */
    uint64_t chunks_form1;       /* ... on 32-bit words with the position beside them */
    uint64_t chunks_form2;       /* ... on 64-bit words                               */
    uint64_t chunks_general;     /* ... by the general stable radix kernel in LDS     */
    int32_t deal_passes_scanned;  /* deal launches whose bucket bases were scanned    */
    int32_t deal_passes_lookback; /* deal launches with decoupled look-back          */
    int32_t levels_heads_keys;    /* levels whose bucket heads came from the keys    */
    int32_t levels_heads_counts;  /* ... from the two dealt digits' counts           */
    int32_t levels_heads_hist;    /* ... from the dealt digit's histograms           */
    int32_t deal_passes_estimated; /* deal launches into estimated buckets (Sec. 3) */
    int32_t plan_from_lengths;    /* 1 if the first level was planned from the segment
                                     lengths alone (no read-back before its deals)  */
} dfr_stats;

dfr_status dfr_get_stats(const dfr_ctx* ctx, dfr_stats* out);

/* Host-only planning helper, usable without a GPU: given the digit histograms of n
 * keys (hist[j * 256 + v] for 8-bit digits j = 0 .. 8*key_bytes/8 - 1), return the
 * number of top varying digits the first level deals before diversion, as the
 * sort itself would choose it (Sec. 3: estimate the number of most significant
 * digits; Sec. 3.1: diversion threshold N_d).  *varying_digits receives how many
 * digits are not constant.  divert_records 0 = default. */
dfr_status dfr_plan_top_digits(const uint32_t* hist, size_t n, int key_bytes, int val_bytes,
                               size_t divert_records, int32_t* top_digits,
                               int32_t* varying_digits);

/* Records one local-sort work item may hold (its LDS capacity) for these widths. */
size_t dfr_local_sort_capacity(int key_bytes, int val_bytes);

/* Records per deal tile by default for these widths (half of it is also built). */
size_t dfr_deal_tile_records(int key_bytes, int val_bytes);

/* ---------------------------------------------------------------------------------
 * Autotuning of the launch settings.  None of these settings changes the result;
 * they trade deal passes against local-sort work (Sec. 3, Sec. 3.1) and pick tile
 * shapes.  Settings are kept per (key bytes, value bytes, size class), where the size
 * class of a call is floor(log2) of the size-biased mean length, sum(len^2)/sum(len),
 * of its segments longer than one record (a plain sort is one segment).
 * ------------------------------------------------------------------------------- */
#define DFR_TUNE_CLASSES 32

typedef struct {
    int32_t radix_bits;       /* digit width b of the deal passes                 */
    uint32_t tile_records;    /* records per deal tile                            */
    uint64_t divert_records;  /* N_d                                              */
    uint64_t window_records;  /* small-bucket window width                        */
    double ms;                /* measured time of one sort (dfr_autotune), else 0 */
    double ms_default;        /* same input with the default settings, else 0     */
} dfr_tune;

/* Size class of a segmented call (seg_offsets as for dfr_sort_segmented_*). */
int32_t dfr_size_class(const uint64_t* seg_offsets, size_t num_segments);

/* Time sorts of copies of the given data (keys/vals: device, vals NULL for key-only;
 * seg_offsets: host, num_segments + 1 entries, {0, n} for a plain sort) under
 * candidate settings, by coordinate descent from the defaults, `reps` timed sorts per
 * candidate (minimum taken; <= 0 means 2).  The caller's buffers are only read.  The
 * best setting is stored in the context for this (widths, size class) and returned in
 * *out.  Allocates and frees two device buffers the size of the data, and uses the
 * context's cached temp buffer.  Blocks the host until done. */
dfr_status dfr_autotune(dfr_ctx* ctx, int key_bytes, int val_bytes, const void* keys,
                        const void* vals, const uint64_t* seg_offsets, size_t num_segments,
                        int reps, void* stream, dfr_tune* out);

/* Read the stored setting for (widths, size class); DFR_E_NOT_FOUND if none. */
dfr_status dfr_get_tune(const dfr_ctx* ctx, int key_bytes, int val_bytes, int32_t size_class,
                        dfr_tune* out);

/* Store a setting (e.g. one saved from an earlier process on the same GPU model);
 * DFR_E_INVALID_ARG if no kernel supports it.  tune == NULL removes the entry. */
dfr_status dfr_set_tune(dfr_ctx* ctx, int key_bytes, int val_bytes, int32_t size_class,
                        const dfr_tune* tune);

#ifdef __cplusplus
}
#endif

#endif /* DFR_H */
