/*
 * rtsort.h -- C ABI of the MI355X (gfx950) stable LSD radix sort.
 *
 * The library sorts 32-bit unsigned keys, optionally carrying 32-bit values,
 * in ascending unsigned order; equal keys keep their input order (stable).
 * This is the problem of Wassenberg & Sanders, "Faster Radix Sort via Virtual
 * Memory and Write-Combining" (arXiv:1008.2849): abstract and Section 1 fix
 * the item (32-bit key, optional 32-bit value), Section 3 the counting-sort
 * pass (digit histogram, exclusive prefix sum, scatter with increment) and
 * Section 4 the LSD order of passes and their stability.
 *
 * Conventions shared by every call below
 *  - Arrays are device pointers into HBM (hipMalloc'd or torch tensors) owned
 *    by the caller; the library never frees them.  Any 4-byte alignment works.
 *  - Every sort call is stream-ordered: it enqueues kernels on `stream` and
 *    returns; results are valid once the stream has synchronised.  No call
 *    synchronises the host, except a call with RT_FLAG_VALIDATE (which waits
 *    for its own work and reports device-side errors) and, with the
 *    environment variable RT_DEBUG_SYNC=1, every call.  The library's own
 *    workspace grows in stream order (hipMallocAsync / hipFreeAsync on the
 *    call's stream), so growing it does not wait either.
 *  - Argument errors are reported synchronously, before any device work.
 *    n = 0 and n = 1 are valid and do nothing.  n >= 2^32 is RT_ERR_TOO_LARGE.
 *  - The result is in place from the caller's view.  The library keeps a
 *    workspace per (device, stream) (temporary ping-pong buffers, digit
 *    histograms, lookback state); calls on different streams may run
 *    concurrently.  Calls that pass their own workspace (the _ex forms) may
 *    be captured into a HIP graph: they then issue kernel launches only.
 *  - rt_last_error() returns a thread-local text for the last failure.
 */
#ifndef RTSORT_H
#define RTSORT_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum rt_status {
    RT_OK = 0,
    RT_ERR_INVALID_ARG = 1,   /* null pointer with n > 0, aliasing, bad config */
    RT_ERR_TOO_LARGE = 2,     /* n or a segment offset >= 2^32 */
    RT_ERR_OUT_OF_MEMORY = 3, /* device or host allocation failed */
    RT_ERR_HIP = 4,           /* a HIP call or kernel launch failed */
    RT_ERR_BUDGET = 5,        /* serving: request larger than the HBM budget */
    RT_ERR_UNSUPPORTED = 6,   /* a configuration the library does not provide */
    RT_ERR_CANCELLED = 7,     /* serving: request cancelled, or dropped at shutdown */
    RT_ERR_TIMEOUT = 8,       /* serving: wait timed out, request still live */
    RT_ERR_NOT_FOUND = 9      /* serving: unknown or already collected ticket */
} rt_status;

#define RT_MAX_PASSES 8
#define RT_MAX_DIGIT_BITS 11

/* rt_config.flags */
#define RT_FLAG_NO_SKIP 0x1u   /* run every pass, even when its digit is constant */
#define RT_FLAG_NT_STORES 0x2u /* scatter with non-temporal stores */
/* Wait for the sort and report device-side errors as RT_ERR_HIP: a
 * lookback wait that gave up (the bounded wait of the onesweep pass; the
 * output is then wrong) and, for batched sorts, malformed segment offsets.
 * Without it these errors leave a flag in the workspace that no call reads
 * (RT_DEBUG_SYNC=1 reads it too).  Accepted by every sort call with flags or
 * a config. */
#define RT_FLAG_VALIDATE 0x4u
/* Write every item straight from registers to its output slot instead of
 * staging the tile by digit in LDS first: the counting-sort pass without
 * write-combining (Section 2's technique switched off, the paper's "VM
 * only" row of Table 1), for measuring what the staging buys.  Same result;
 * not combinable with RT_FLAG_NT_STORES. */
#define RT_FLAG_DIRECT_SCATTER 0x8u
/* XCD chunks.  A sort whose digits are all at most 8 bits wide may split
 * every pass's input into 8 chunks, one per XCD: the tiles of a chunk run on
 * that XCD, and each chunk has its own lookback chain and output start per
 * digit (from per-chunk counts taken by the upfront histogram read), so the
 * ends of neighbouring digit runs, which share cache lines, are written
 * through one L2.  By default a sort of at least 2^25 items samples its keys
 * first and uses chunks unless they would be badly unbalanced or the
 * per-chunk counting would contend on a few frequent digits (skewed keys).
 * RT_FLAG_ONE_CHAIN: never use chunks (one lookback chain per pass).
 * RT_FLAG_CHUNKS: always use chunks, at any size, without sampling (ignored
 * if a digit is wider than 8 bits).  The result is the same in every case;
 * the flags are for measuring and testing.  They exclude each other. */
#define RT_FLAG_ONE_CHAIN 0x10u
#define RT_FLAG_CHUNKS 0x20u
/* Fused next-digit histogram (Section 4, Algorithm 2's histogram2, counted
 * while the data passes anyway): the upfront read counts only the first
 * pass's digit, and each pass counts the next pass's digit of the items it
 * writes; a small planning launch between passes turns those counts into
 * the next pass's digit starts.  For measuring that trade against the
 * upfront read of every digit.  Same result.  Implies RT_FLAG_ONE_CHAIN and
 * RT_FLAG_NO_SKIP (the later histograms do not exist when the buffers are
 * planned); digits of at most 8 bits; not combinable with RT_FLAG_CHUNKS,
 * RT_FLAG_DIRECT_SCATTER or RT_FLAG_NT_STORES (RT_ERR_UNSUPPORTED).
 * Single-array 32-bit sorts only. */
#define RT_FLAG_FUSED_HISTOGRAM 0x40u
/* rt_sort_msd_first only: the number of MSD levels (see there).  By default
 * the call picks by n; these force one or two.  They exclude each other. */
#define RT_FLAG_MSD_ONE_LEVEL 0x80u
#define RT_FLAG_MSD_TWO_LEVELS 0x100u

/*
 * Sort configuration.  Zero-initialised fields mean "tuned default".
 * digit_bits[p] is the width of pass p's digit, least significant first
 * (Section 4: digits are processed from the least significant one upward);
 * the widths must sum to 32 and each lies in 1..RT_MAX_DIGIT_BITS.
 * Every decomposition gives the same result; they differ in speed.
 * Tile shapes built (block_threads x items_per_thread): 256x16, 512x16,
 * 1024x8, 1024x12, 1024x16 and 512x32 for digits of up to 8 bits, and
 * 256x16, 512x8 and 512x16 for wider ones.  512x32 stages the keys, then the
 * values, through one LDS stage so that two blocks share a CU; with
 * RT_FLAG_NT_STORES, RT_FLAG_DIRECT_SCATTER or RT_FLAG_FUSED_HISTOGRAM it is
 * RT_ERR_UNSUPPORTED.
 */
typedef struct rt_config {
    uint32_t num_passes;                 /* 0 = tuned default */
    uint32_t digit_bits[RT_MAX_PASSES];  /* used when num_passes > 0 */
    uint32_t block_threads;              /* 0 = tuned */
    uint32_t items_per_thread;           /* 0 = tuned */
    uint32_t flags;                      /* RT_FLAG_* */
} rt_config;

/* ------------------------------------------------------------------------
 * Single-array sorts
 * --------------------------------------------------------------------- */

/*
 * Sort n keys in place (stable LSD radix sort, Section 4; each pass the
 * counting sort of Section 3).  keys: device u32[n].
 */
rt_status rt_sort_keys(uint32_t *keys, size_t n, hipStream_t stream);

/*
 * Sort n key/value pairs in place by key; each value moves with its key and
 * equal keys keep their input order.  keys, vals: device u32[n], distinct
 * and not overlapping.  vals == NULL is RT_ERR_INVALID_ARG (use
 * rt_sort_keys).
 */
rt_status rt_sort_pairs(uint32_t *keys, uint32_t *vals, size_t n, hipStream_t stream);

/*
 * Bytes of workspace rt_sort_pairs_ex needs for n items (with_values 0 or 1)
 * under cfg (NULL = tuned default).  Returns 0 for n < 2.
 */
size_t rt_workspace_bytes(size_t n, int with_values, const rt_config *cfg);

/*
 * Explicit form: cfg (NULL = tuned default) and a caller-owned device
 * workspace of at least rt_workspace_bytes() bytes, 256-byte aligned (NULL =
 * library cache).  vals may be NULL (keys only).  With a caller workspace and
 * no RT_FLAG_VALIDATE the call issues kernel launches only, so it may be
 * captured into a HIP graph; concurrent calls must not share a workspace.
 * With RT_FLAG_VALIDATE in cfg->flags the call waits for the sort and
 * returns RT_ERR_HIP if a pass's lookback gave up.
 */
rt_status rt_sort_pairs_ex(uint32_t *keys, uint32_t *vals, size_t n, const rt_config *cfg,
                           void *workspace, size_t workspace_bytes, hipStream_t stream);

/*
 * rt_sort_pairs_ex for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same sort, with the library's static per-device scratch
 * array (64 MiB, held until the process ends) as its workspace.  It calls
 * no hipMalloc, hipFree or other allocating routine.  n items must fit that
 * scratch (rt_workspace_bytes(n, vals != NULL, cfg) <= 64 MiB: about 3.9M
 * pairs or 7.8M keys with the tuned configuration); larger n is
 * RT_ERR_TOO_LARGE, before any device work.  Arguments, cfg, flags and
 * errors as for rt_sort_pairs_ex.  Every call on one GPU uses that GPU's
 * one scratch array: calls that overlap on a GPU (other streams, other
 * threads) race and corrupt each other's results; calls ordered on one
 * stream are fine.  Each call clears, with its own kernels, whatever part
 * of the scratch must start at zero.
 */
rt_status rt_sort_pairs_noalloc(uint32_t *keys, uint32_t *vals, size_t n, const rt_config *cfg,
                                hipStream_t stream);

/* ------------------------------------------------------------------------
 * 64-bit keys
 * --------------------------------------------------------------------- */

/*
 * Sort n 64-bit unsigned keys in place, ascending and stable, by the same
 * LSD radix sort on K = 64-bit keys (Section 4; each pass Section 3's
 * counting sort).  The paper sorts 32-bit keys and notes that its items may
 * be wider than one 64-bit key-value word; this is that variant.
 * keys: device u64[n], 8-byte aligned.
 */
rt_status rt_sort_keys64(uint64_t *keys, size_t n, hipStream_t stream);

/*
 * As rt_sort_keys64, moving a 32-bit value with each key.  keys: device
 * u64[n], 8-byte aligned; vals: device u32[n], 4-byte aligned, not
 * overlapping the keys.  vals == NULL is RT_ERR_INVALID_ARG.
 */
rt_status rt_sort_pairs64(uint64_t *keys, uint32_t *vals, size_t n, hipStream_t stream);

/*
 * Explicit form.  value_bytes: 0 (keys only, vals ignored), 4 or 8 bytes per
 * item; vals is then a device array of n such values, aligned to
 * value_bytes.  cfg (NULL = built-in default: eight 8-bit digits, in
 * 16K-item tiles from 2^24 items (12K with 8-byte values) and 8K-item tiles
 * below): digit_bits must sum to 64, each 1..RT_MAX_DIGIT_BITS; tile shapes
 * built are 1024x16, 1024x12, 1024x8 and 512x16 for digits of up to 8 bits
 * and 512x8 for wider ones (correct, but several times slower than 8-bit
 * digits); flags: RT_FLAG_NO_SKIP, RT_FLAG_ONE_CHAIN, RT_FLAG_CHUNKS (XCD
 * chunks as for 32-bit keys), RT_FLAG_VALIDATE (anything else is
 * RT_ERR_UNSUPPORTED).  workspace: at least rt_workspace_bytes64() bytes,
 * 256-byte aligned, or NULL for the library's per-stream cache; with a
 * caller workspace the call only enqueues kernels.  Errors and stream
 * behaviour as for rt_sort_pairs_ex.
 */
rt_status rt_sort64_ex(uint64_t *keys, void *vals, uint32_t value_bytes, size_t n, const rt_config *cfg,
                       void *workspace, size_t workspace_bytes, hipStream_t stream);

/* Workspace bytes of rt_sort64_ex (0 for n < 2, n >= 2^32, a value_bytes
 * other than 0, 4 or 8, or an invalid cfg). */
size_t rt_workspace_bytes64(size_t n, uint32_t value_bytes, const rt_config *cfg);

/* ------------------------------------------------------------------------
 * Batched segmented sort
 * --------------------------------------------------------------------- */

/*
 * Sort every segment s = [seg_offsets[s], seg_offsets[s+1]) of keys/vals
 * independently and stably (Section 4's LSD sort applied to each segment
 * as to an array of its own; segments are not described by the paper, which
 * sorts one array).  seg_offsets: device u32[num_segments + 1],
 * nondecreasing, read only on the device.  Items outside
 * [seg_offsets[0], seg_offsets[num_segments]) are not touched; empty and
 * one-item segments are fine.  vals may be NULL (keys only); keys and vals
 * must not overlap.  max_total bounds seg_offsets[num_segments] -
 * seg_offsets[0] and sizes the workspace (pass the total when known).
 * Segments of up to 16384 items are sorted whole in LDS, larger ones by
 * four 8-bit onesweep passes over 16K-item tiles.
 *
 * Errors: argument errors are returned before any device work.  A segment
 * whose offsets decrease or reach past seg_offsets[0] + max_total is left
 * unsorted and flagged on the device; the plain call does not wait for the
 * device, so only RT_FLAG_VALIDATE (or RT_DEBUG_SYNC=1) reports it, as
 * RT_ERR_INVALID_ARG.  The call is stream-ordered and never writes outside
 * the segments and the library's workspace.
 */
rt_status rt_sort_pairs_batched(uint32_t *keys, uint32_t *vals, const uint32_t *seg_offsets,
                                uint32_t num_segments, size_t max_total, hipStream_t stream);

/* Workspace bytes of a batched sort of num_segments segments totalling at
 * most max_total items (0 when there is nothing to sort). */
size_t rt_batched_workspace_bytes(uint32_t num_segments, size_t max_total, int with_values);

/*
 * Explicit form of rt_sort_pairs_batched: flags (RT_FLAG_VALIDATE or 0) and
 * a caller-owned device workspace of at least rt_batched_workspace_bytes()
 * bytes, 256-byte aligned (NULL = library cache).  With a caller workspace
 * and no RT_FLAG_VALIDATE the call only enqueues kernels, so it may be
 * captured into a HIP graph; concurrent calls must not share a workspace.
 */
rt_status rt_sort_batched_ex(uint32_t *keys, uint32_t *vals, const uint32_t *seg_offsets,
                             uint32_t num_segments, size_t max_total, uint32_t flags, void *workspace,
                             size_t workspace_bytes, hipStream_t stream);

/* ------------------------------------------------------------------------
 * MSD-first sort ("reverse sorting")
 * --------------------------------------------------------------------- */

/*
 * Workspace bytes of rt_sort_msd_first for n items (with_values 0 or 1);
 * 0 when n < 2 or n >= 2^32.
 */
size_t rt_msd_first_workspace_bytes(size_t n, int with_values);

/*
 * Sorts n keys (and values) in place like rt_sort_pairs_ex, by Section 4's
 * "reverse sorting" as Algorithm 2 arranges it on one processing element:
 * one counting-sort pass on the most significant 8-bit digit moves the
 * items into a temporary array of the workspace, partitioned into 256 MSD
 * buckets whose starts are the exclusive prefix sum of the MSD histogram;
 * then each bucket is sorted on its own.  With one MSD level, by LSD passes
 * over digits 0, 1 and 2, the last of which writes the caller's arrays.
 * With two, a second partition pass on digit 2 inside every bucket writes
 * the caller's arrays, cut into 65536 sub-buckets (the buckets' digit-2
 * counts give their bounds), and each sub-bucket is then sorted on digits 0
 * and 1: whole in LDS when it holds at most 16384 items (the LDS is the
 * fast memory the buckets are sized for, as the paper sizes them for the
 * cache), else by two tiled passes.  The result equals rt_sort_pairs_ex's
 * bit for bit (a stable sort has one result); passes are never skipped, so
 * keys whose top byte is constant still pay the partition pass.  Buckets
 * and sub-buckets of at most 16384 items are sorted whole in LDS.
 *
 * keys, vals: device u32[n], not overlapping; vals may be NULL (keys only).
 * flags: 0 or any of RT_FLAG_VALIDATE (wait, and report a device error
 * word as RT_ERR_HIP), RT_FLAG_MSD_ONE_LEVEL, RT_FLAG_MSD_TWO_LEVELS (by
 * default two levels from 2^26 items).  workspace: device memory of at least
 * rt_msd_first_workspace_bytes(n, vals != NULL) bytes, 256-byte aligned,
 * or NULL for the library's per-stream cache; with a caller workspace and
 * no RT_FLAG_VALIDATE the call only enqueues kernels.  Argument errors are
 * returned before any device work; n = 0 and n = 1 do nothing.
 */
rt_status rt_sort_msd_first(uint32_t *keys, uint32_t *vals, size_t n, uint32_t flags, void *workspace,
                            size_t workspace_bytes, hipStream_t stream);

/* ------------------------------------------------------------------------
 * Pieces of the path, exported for parity tests and measurement
 * --------------------------------------------------------------------- */

/*
 * Digit histograms of all passes in one read of the keys (Section 3's
 * counting step for every digit at once).  hist: device
 * u32[num_passes * 2^RT_MAX_DIGIT_BITS]; pass p's 2^digit_bits[p] counters
 * start at offset p * 2^RT_MAX_DIGIT_BITS; the whole array is overwritten.
 * cfg as for rt_sort_pairs_ex (NULL = tuned default).
 */
rt_status rt_digit_histograms(const uint32_t *keys, size_t n, const rt_config *cfg,
                              uint32_t *hist, hipStream_t stream);

/*
 * The XCD-chunk decision that rt_sort_pairs_ex (with_values != 0) or
 * rt_sort_keys-style calls (with_values == 0) make for these n keys under
 * cfg (NULL = tuned default), written to *mode (device u32): 1 = the passes
 * run in XCD chunks, 0 = one lookback chain per pass.  Where the sort
 * samples its keys (see RT_FLAG_CHUNKS) this runs the same sample kernel on
 * the same keys; otherwise it writes what the size, the digit widths and the
 * flags fix.  n < 2 writes 0.  A measurement and test hook: the sort's
 * result does not depend on the decision.  Errors as for rt_digit_histograms
 * (mode NULL: RT_ERR_INVALID_ARG).
 */
rt_status rt_chunk_decision(const uint32_t *keys, size_t n, int with_values, const rt_config *cfg,
                            uint32_t *mode, hipStream_t stream);

/* The same for a sort of 64-bit keys with value_bytes of 0, 4 or 8
 * (rt_sort64_ex's decision). */
rt_status rt_chunk_decision64(const uint64_t *keys, size_t n, uint32_t value_bytes, const rt_config *cfg,
                              uint32_t *mode, hipStream_t stream);

/*
 * One stable counting-sort pass, out of place (Section 3, naive algorithm:
 * histogram, exclusive prefix sum, scatter with increment) on digit
 * [shift, shift + width).  kin/vin are read, kout/vout written (vin and vout
 * both NULL for keys only); inputs and outputs must not overlap.
 * width 1..RT_MAX_DIGIT_BITS, shift + width <= 32.
 */
rt_status rt_counting_pass(const uint32_t *kin, const uint32_t *vin, uint32_t *kout,
                           uint32_t *vout, size_t n, uint32_t shift, uint32_t width,
                           hipStream_t stream);

/*
 * Streaming copy of `bytes` bytes (a multiple of 4) from src to dst: the
 * achievable read+write bandwidth probe the per-pass figures are set
 * against.
 */
rt_status rt_copy(const void *src, void *dst, size_t bytes, hipStream_t stream);

/*
 * Bandwidth probes: the ceilings a pass's HBM rate is set against, for
 * measurement.  kind RT_PROBE_COPY: the copy of rt_copy (one 16-byte word
 * per thread); RT_PROBE_COPY_NT: copy with four 16-byte words in flight per
 * thread and non-temporal loads and stores, 16 blocks per CU in a
 * grid-stride loop; RT_PROBE_READ: reads src only (an XOR of every word,
 * written to the device word *sink only if it hits a fixed value, so the
 * loads stay); RT_PROBE_WRITE: writes dst only (a fixed pattern).  src and
 * dst: device memory of `bytes` bytes, 16-byte aligned, bytes a multiple of
 * 16 (src unused by RT_PROBE_WRITE, dst by RT_PROBE_READ).
 */
#define RT_PROBE_COPY 0u
#define RT_PROBE_COPY_NT 1u
#define RT_PROBE_READ 2u
#define RT_PROBE_WRITE 3u
rt_status rt_bandwidth_probe(const void *src, void *dst, size_t bytes, uint32_t kind, uint32_t *sink,
                             hipStream_t stream);

/* ------------------------------------------------------------------------
 * Device input generator (counter-based SplitMix64)
 * --------------------------------------------------------------------- */

#define RT_DIST_UNIFORM 0u /* low 32 bits of word i */
#define RT_DIST_AND4 1u    /* AND of the four 32-bit halves of words 2i, 2i+1 */
#define RT_DIST_ZIPF16 2u  /* dictionary[first r with hi32(word i) < thresholds[r]] */

typedef struct rt_gen_params {
    uint32_t dist;            /* RT_DIST_* */
    uint64_t state;           /* SplitMix64 state of the stream */
    uint32_t dictionary[16];  /* RT_DIST_ZIPF16 only */
    uint64_t thresholds[16];  /* RT_DIST_ZIPF16 only; increasing, last = 2^32 */
} rt_gen_params;

/*
 * Fill keys[0..n) from the counter-based generator: word i of the stream is
 * mix64(state + (i + 1) * 0x9E3779B97F4A7C15) (SplitMix64, Steele, Lea &
 * Flood, OOPSLA 2014).  vals (may be NULL) receives vals[i] = value_base + i.
 * params is a host pointer, read during the call.
 */
rt_status rt_generate(uint32_t *keys, uint32_t *vals, size_t n, const rt_gen_params *params,
                      uint32_t value_base, hipStream_t stream);

/* ------------------------------------------------------------------------
 * Serving loop
 * --------------------------------------------------------------------- */

typedef struct rt_server rt_server;

/*
 * Start a server on the current device.  hbm_budget_bytes bounds the device
 * memory its admitted requests hold (inputs it generates, ping-pong buffers,
 * metadata); max_active bounds how many requests are in flight.  The server
 * owns a scheduler thread and a stream of its own.
 */
rt_status rt_server_create(size_t hbm_budget_bytes, uint32_t max_active, rt_server **out);

/*
 * Submit a request whose key/value arrays already live on the device.
 * keys, vals: the input, device u32[n] (vals may be NULL: keys only).
 * out_keys, out_vals: where the sorted result goes, device u32[n]; NULL
 * (or the input arrays themselves) sorts in place.  An out-of-place request
 * copies its input into its outputs on the device when it is admitted and
 * never writes the input; inputs and outputs must then not overlap, and
 * out_vals must be given when vals is.  Every array is caller-owned and must
 * stay untouched by the caller until rt_server_wait (or rt_server_wait_any)
 * has reported the request.  A request whose footprint exceeds the whole
 * budget is RT_ERR_BUDGET.
 */
rt_status rt_server_submit(rt_server *s, const uint32_t *keys, const uint32_t *vals, uint32_t *out_keys,
                           uint32_t *out_vals, size_t n, uint64_t *ticket);

/*
 * Submit a request whose input the server generates on the device at
 * admission from params (rt_generate's definition) with vals[i] = i; the
 * result stays in server memory until rt_server_fetch or rt_server_release.
 */
rt_status rt_server_submit_generated(rt_server *s, const rt_gen_params *params, size_t n,
                                     uint64_t *ticket);

/*
 * Wait for a request.  timeout_us < 0 waits forever; on expiry returns
 * RT_ERR_TIMEOUT and the request stays live.  latency_us (may be NULL)
 * receives completion time minus submit time.  The request's own status is
 * returned (RT_OK, RT_ERR_HIP, RT_ERR_CANCELLED, ...).
 */
rt_status rt_server_wait(rt_server *s, uint64_t ticket, int64_t timeout_us, double *latency_us);

/*
 * Wait for whichever request finishes next (completion order) that no wait
 * has reported yet; *ticket receives it.  Same timeout, latency and status
 * rules as rt_server_wait; RT_ERR_NOT_FOUND when no request is outstanding.
 * A generated request stays fetchable until rt_server_fetch or
 * rt_server_release.
 */
rt_status rt_server_wait_any(rt_server *s, int64_t timeout_us, uint64_t *ticket, double *latency_us);

/*
 * Copy a finished generated request's sorted arrays into caller device
 * buffers (out_vals may be NULL) and release its memory.
 */
rt_status rt_server_fetch(rt_server *s, uint64_t ticket, uint32_t *out_keys, uint32_t *out_vals);

/* Release a finished request's server memory without copying it. */
rt_status rt_server_release(rt_server *s, uint64_t ticket);

/*
 * Cancel a request.  A queued request ends at once; an admitted one takes no
 * further pass, gives its memory back to the budget and ends when the step
 * now being planned has run.  Either way rt_server_wait (or
 * rt_server_wait_any) then reports it as RT_ERR_CANCELLED.  What a cancelled
 * request leaves behind: an in-place request's arrays hold its input or the
 * state after an even number of passes (a permutation of the input, not
 * sorted); an out-of-place request's outputs are unspecified and its input
 * untouched; a generated request keeps its memory until rt_server_release.
 * Returns RT_OK if the request will take no further pass (it then ends as
 * RT_ERR_CANCELLED, or with the error of a step that had already failed
 * it), RT_ERR_INVALID_ARG if it has finished or its last pass is already
 * under way (its result stands), RT_ERR_NOT_FOUND for an unknown or
 * collected ticket.  A wait already in
 * progress on the request returns RT_ERR_CANCELLED when it ends.
 */
rt_status rt_server_cancel(rt_server *s, uint64_t ticket);

/*
 * Latency percentiles (us) over completed requests and throughput
 * (completed items / (last completion - first admission), Gkeys/s).
 * Any output pointer may be NULL.
 */
rt_status rt_server_stats(rt_server *s, double *p50_us, double *p99_us, double *gkeys_per_s);

/* As rt_server_stats, plus the number of completed requests and the
 * high-water mark of budgeted device memory (peak_bytes). */
rt_status rt_server_stats_ex(rt_server *s, double *p50_us, double *p99_us, double *gkeys_per_s,
                             uint64_t *completed, size_t *peak_bytes);

/* One request of an arrival trace for rt_server_replay: a generated input
 * of n key/value pairs (as rt_server_submit_generated), arriving
 * arrival_us microseconds after the replay starts. */
typedef struct rt_replay_request {
    double arrival_us;
    uint64_t n;
    rt_gen_params params;
} rt_replay_request;

/*
 * Open-loop replay of an arrival trace, for measuring the server under a
 * given offered load without the client's own submission cost in the way.
 * A native thread submits reqs[i] (arrival_us nondecreasing) at its arrival
 * time, never earlier; the calling thread collects completions in
 * completion order and releases each result.  latency_us[i] receives the
 * completion time of request i minus its scheduled arrival (so a late
 * submission counts against the server, not for it); *span_us (may be
 * NULL) the last completion minus the start.  The server must have no
 * other requests outstanding and no other client while it runs.  Returns
 * when every submitted request has finished: RT_OK, or the first failure
 * (a submission refused, e.g. RT_ERR_BUDGET, or a request's own error), in
 * which case latencies of requests not completed are negative.
 */
rt_status rt_server_replay(rt_server *s, const rt_replay_request *reqs, size_t count, double *latency_us,
                           double *span_us);

/* Stop the scheduler; requests not yet finished end as RT_ERR_CANCELLED. */
rt_status rt_server_destroy(rt_server *s);

/* ------------------------------------------------------------------------
 * Tuning and diagnostics
 * --------------------------------------------------------------------- */

/*
 * Load a tuning table (JSON written by the autotuner).  Its "keys" and
 * "pairs" entries map single-array sorts of n in [min_n, max_n] to digit
 * widths, block size, items per thread and flags; its "segments" entries
 * (increasing max_n, at most 4, each at most 16384 and within its shape,
 * digits 8,8,8,8 or 11,11,10) are the whole-in-LDS size classes of the
 * segmented sort (see rt_segment_classes), and a "segments_tiled" entry
 * (block x ipt of 1024x16 or 512x16, digits 8,8,8,8) its tiled passes' tile
 * (see rt_segment_config).  A malformed table is RT_ERR_INVALID_ARG and
 * leaves the loaded one in force.  NULL restores the built-in defaults.
 */
rt_status rt_load_tuning(const char *json_path);

/* Tuned configuration the library would use for n items. */
rt_status rt_tuned_config(size_t n, int with_values, rt_config *out);

/*
 * Kernel timing, for measurement.  Between rt_profile_start and
 * rt_profile_stop every kernel the library launches is followed by a HIP
 * event recorded on the launch's stream (one more event precedes each
 * call's first kernel), so a kernel's duration is the time between the
 * event before it and the one after it on that stream.  At most max_marks
 * events are recorded; later launches go unrecorded.  rt_profile_stop waits
 * for the events, writes up to `capacity` (kind, milliseconds) pairs into the
 * host arrays kinds/ms in launch order, stores their number in *count and
 * frees the events.  Kinds: RT_KIND_* below; kind 0 opens each call and
 * carries the idle time since the previous mark on its stream (0 for the
 * first).
 */
#define RT_KIND_FILL 1u
#define RT_KIND_HISTOGRAM 2u
#define RT_KIND_PLAN 3u
#define RT_KIND_COPY_BACK 4u
#define RT_KIND_COPY 5u
#define RT_KIND_GENERATE 6u
#define RT_KIND_SEGMENTED 7u /* segmented sort: tile lists of the tiled segments */
#define RT_KIND_SEG_SMALL 8u /* segmented sort: segments sorted whole in LDS */
#define RT_KIND_MSD_PASS 9u  /* MSD-first sort: the partition pass on the top digit */
#define RT_KIND_PROBE 10u    /* sample of the keys that chooses XCD chunks or one chain */
#define RT_KIND_PASS 16u     /* + pass index: one counting-sort pass (onesweep) */
rt_status rt_profile_start(uint32_t max_marks);
rt_status rt_profile_stop(uint32_t *kinds, float *ms, uint32_t capacity, uint32_t *count);

/*
 * The whole-in-LDS size classes of the segmented sort in force (built in,
 * or the tuning table's "segments" entries): *count classes, class c sorting
 * the segments of up to max_n[c] items (more than max_n[c - 1]) with one
 * block of block[c] threads x ipt[c] items; larger segments are tiled.  The
 * host arrays hold at least 4 entries; any of them may be NULL.  Batched
 * calls and the MSD-first sort use the classes in force when their layout
 * is computed (rt_batched_workspace_bytes sizes the workspace for them), a
 * server those in force when it was created.
 */
rt_status rt_segment_classes(uint32_t *count, uint32_t *max_n, uint32_t *block, uint32_t *ipt);

/*
 * The rest of the segmented sort's tuning in force: bits[c] (host array of
 * at least 4 entries, may be NULL) the digit width of class c's passes (8:
 * four 8-bit passes; 11: passes of 11, 11 and 10 bits), and the tile of the
 * tiled segments' passes in batched calls and MSD-first sorts, tile_block x
 * tile_ipt items (1024 x 16 or 512 x 16; the server keeps 1024 x 16).  Any
 * pointer may be NULL.
 */
rt_status rt_segment_config(uint32_t *bits, uint32_t *tile_block, uint32_t *tile_ipt);

const char *rt_status_string(rt_status s);
const char *rt_last_error(void);
const char *rt_version(void);

#ifdef __cplusplus
}
#endif

#endif /* RTSORT_H */
