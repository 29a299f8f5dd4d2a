/*
 * lbsort — load-balanced sample sort on one AMD MI355X (gfx950).
 *
 * C ABI of the library.  The operation is the distributed sort of Khatami et
 * al., "A Load-Balanced Parallel and Distributed Sorting Algorithm Implemented
 * with PGX.D" (arXiv 1611.00463), Section IV, run on one GPU: the P processors
 * of the paper become P virtual processors, each owning one contiguous block
 * of the input, and the six steps are
 *
 *   1. each block is sorted locally (stable LSD radix sort, Section IV.A);
 *   2. regular samples are taken from each sorted block (Section IV.B);
 *   3. P-1 splitters are chosen from the pooled samples (step 3);
 *   4. every splitter is searched in every sorted block, and the investigator
 *      divides runs of keys equal to a duplicated splitter (Section IV.B,
 *      Fig. 3);
 *   5. the ranges are exchanged: block i's slice for partition k lands at the
 *      receive offset known from the broadcast range table (Section IV.C);
 *   6. each partition merges what it received with the handler (Section IV.A,
 *      Fig. 2), yielding the globally sorted data; smaller keys sit in
 *      partitions with smaller ids (Section IV.C).
 *
 * Keys are 32- or 64-bit unsigned integers, signed integers or IEEE floats
 * (the interface is generic over the data type, Section IV.C), sorted
 * ascending in their type's order; floats in IEEE 754-2008 totalOrder:
 * -NaN < -inf < negative numbers < -0 < +0 < positive numbers < +inf < +NaN.
 * Values are opaque 32-bit payloads carried with their keys, or generated:
 * with LBSORT_VAL_INDEX each key carries its input position (inside its
 * instance), which gives the provenance of every sorted entry (step 6 and
 * Section IV.C).  In the default investigator mode (COUNT) the output equals
 * a stable sort of the input.
 *
 * Conventions shared by every entry point
 *   - All data pointers are DEVICE pointers unless marked "host".
 *   - The caller owns every buffer.  The library allocates no device memory
 *     in the sort calls; scratch space comes from the caller's workspace.
 *   - Two-phase workspace: call once with ws == NULL to receive the needed
 *     size in *ws_bytes (host), allocate it, and call again.  A workspace
 *     smaller than needed returns LBSORT_ERR_WORKSPACE_TOO_SMALL.
 *   - Work is enqueued on `stream` (a hipStream_t passed as void*, NULL for
 *     the default stream) and is asynchronous: results are valid once the
 *     stream has been synchronised.  Inputs are read-only and must not
 *     overlap outputs or the workspace.  Calls that share a workspace must
 *     not run concurrently.
 *   - Every function returns a status code (0 = success, negative = error)
 *     and never aborts; lbsort_last_error() returns this thread's last error
 *     text.  Errors found on the device (a bounded wait that gave up, a
 *     malformed segment table) are latched in the workspace and returned by
 *     lbsort_check().
 */
#ifndef LBSORT_H
#define LBSORT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define LBSORT_OK 0
#define LBSORT_ERR_INVALID_ARG (-1)
#define LBSORT_ERR_WORKSPACE_TOO_SMALL (-2)
#define LBSORT_ERR_UNSUPPORTED (-3)
#define LBSORT_ERR_HIP (-4)
#define LBSORT_ERR_OOM (-5)
#define LBSORT_ERR_DEVICE (-6)

/* key types */
#define LBSORT_U32 1 /* uint32_t                                       */
#define LBSORT_U64 2 /* uint64_t                                       */
#define LBSORT_I32 3 /* int32_t, two's complement                      */
#define LBSORT_I64 4 /* int64_t                                        */
#define LBSORT_F32 5 /* IEEE binary32, totalOrder                      */
#define LBSORT_F64 6 /* IEEE binary64, totalOrder                      */
/* value types */
#define LBSORT_NOVAL 0     /* keys only                                               */
#define LBSORT_VAL_U32 1   /* one uint32_t payload per key from vals_in                */
#define LBSORT_VAL_INDEX 2 /* vals_in ignored; vals_out receives each key's input
                              position inside its instance (uint32_t; instances of
                              at most 2^32 keys, else LBSORT_ERR_UNSUPPORTED for one
                              instance, the device error E_RANGE for a batch)       */

/* investigator modes (step 4, Section IV.B) */
#define LBSORT_INV_COUNT 0 /* default: equal-key runs split at global ranks floor(kN/P) */
#define LBSORT_INV_NONE 1  /* plain regular sampling, no investigator (Fig. 3b)       */
#define LBSORT_INV_PAPER 2 /* each block's equal-key range cut into d+1 equal pieces  */

/* limits */
#define LBSORT_MAX_P 1024
#define LBSORT_MAX_SAMPLES (1u << 20)

typedef struct lbsort_params {
  uint32_t P;            /* virtual processors = output partitions, 1..LBSORT_MAX_P      */
  uint32_t s;            /* regular samples per block; 0 = the paper's budget: one 256 KB
                            read buffer over all processors, b = 262144 / (P * key bytes),
                            taken as the largest multiple of P not above b (b if b < P,
                            at least 1)                                                     */
  uint32_t investigator; /* LBSORT_INV_*                                                     */
  uint32_t fanin;        /* handler merge fan-in F per pass: 0 = tuned, else 2, 4, 8 or 16
                            (LBSORT_HANDLER_PASSES); with LBSORT_HANDLER_ONE_PASS 0 or the
                            power of two reaching P (up to 64)                              */
  uint32_t merge_tile;   /* elements per merge tile: 0 = tuned, else 1024, 2048 or 4096
                            (LBSORT_HANDLER_ONE_PASS: 2048 or 4096, the tile's capacity)    */
  uint32_t radix_tile;   /* keys per radix tile of the local sort: 0 = tuned, else 4096,
                            8192 or, for 32-bit keys, 16384 (digits are 8 bits wide in
                            every case)                                                     */
  uint32_t handler;      /* step 6: 0 = tuned, LBSORT_HANDLER_PASSES or
                            LBSORT_HANDLER_ONE_PASS                                         */
  uint32_t presorted;    /* step 1: 0 = tuned, LBSORT_PRESORTED_DETECT (blocks already in
                            order or in reverse order skip the radix passes; the default)
                            or LBSORT_PRESORTED_IGNORE                                      */
  uint32_t reserved;     /* must be 0                                                        */
} lbsort_params;

#define LBSORT_PRESORTED_DETECT 1
#define LBSORT_PRESORTED_IGNORE 2

/* Handler (step 6, Section IV.A, Fig. 2) schedules.  Both merge each
 * partition's P runs stably (ties to the lower block) and give the same bytes.
 *   PASSES:   ceil(log_F P) passes of F-way merges; every tile of a pass holds
 *             exactly merge_tile outputs, its boundary found by an exact
 *             multi-sequence selection.
 *   ONE_PASS: one pass of a P-way merge (P <= 64, total_n <= 2^32); tile
 *             boundaries are regular samples of the runs (every 16th element
 *             of each run, merged by the PASSES schedule at 1/16 of the size),
 *             which bounds every tile by merge_tile without selection rounds. */
#define LBSORT_HANDLER_PASSES 1
#define LBSORT_HANDLER_ONE_PASS 2

/* Partition outputs (device arrays).  For a batch every array is stacked per
 * instance: instance b's part_offsets are at part_offsets[b*(P+1)], etc. */
typedef struct lbsort_parts {
  uint64_t *part_offsets; /* [P+1] required: G_0 = 0 <= G_1 <= ... <= G_P = n; partition k
                             is output positions [G_k, G_{k+1}) (relative to the segment) */
  uint64_t *part_counts;  /* [P]   optional (NULL): G_{k+1} - G_k                            */
  void *splitters;        /* [P-1] optional: v_1..v_{P-1}, key type                          */
  uint64_t *send_counts;  /* [P*P] optional: C[i][k] = keys block i sends to partition k     */
  uint64_t *cuts;         /* [P*(P+1)] optional: c[i][k], block i sends sorted positions
                             [c[i][k], c[i][k+1]) to partition k                             */
} lbsort_parts;

/*
 * Sort n keys (steps 1-6).  keys_in/keys_out: n keys of `key_type`.
 * Block i of the input is positions [floor(i n / P), floor((i+1) n / P)).
 * n may be 0.  params may be NULL (P = 1, all defaults).
 */
int lbsort_sort_keys(int key_type, const void *keys_in, void *keys_out, uint64_t n,
                     const lbsort_params *params, const lbsort_parts *parts, void *ws,
                     size_t *ws_bytes, void *stream);

/* Same, carrying one 32-bit value per key: from vals_in (LBSORT_VAL_U32) or
 * the key's input position (LBSORT_VAL_INDEX, vals_in ignored). */
int lbsort_sort_pairs(int key_type, int val_type, const void *keys_in, const void *vals_in,
                      void *keys_out, void *vals_out, uint64_t n, const lbsort_params *params,
                      const lbsort_parts *parts, void *ws, size_t *ws_bytes, void *stream);

/*
 * Allocation-free form of lbsort_sort_pairs, for callers that cannot
 * allocate device memory at all (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc).  Same arguments and results as
 * lbsort_sort_pairs (val_type may also be LBSORT_NOVAL: keys only), but no
 * workspace: the scratch space is one static device array of
 * LBSORT_NOALLOC_SCRATCH_BYTES inside the library, of which every device the
 * library runs on holds its own copy until the process ends.  Nothing is
 * allocated by this call (no hipMalloc, no hipFree, no allocating library
 * routine); the first call made with a device current looks up the array's
 * address on that device.  The call runs on the current device and `stream`
 * must belong to it.
 *
 * Limit: a problem whose workspace (as lbsort_sort_pairs would size it)
 * exceeds LBSORT_NOALLOC_SCRATCH_BYTES returns LBSORT_ERR_UNSUPPORTED before
 * anything is enqueued; that is about 5.3 million 64-bit keys with values
 * (4.4 million with LBSORT_HANDLER_ONE_PASS at P = 64), or 7.9 million
 * 32-bit keys with values.
 *
 * All calls on one device share that device's array and each call starts
 * by clearing what must start at zero: calls that overlap on one device
 * (different streams, or host threads) race and give undefined results;
 * serialise them.  dev_err (device, may be NULL) receives the device error
 * bits this call latched (0 = none; see lbsort_check), written on `stream`
 * after the sort.
 */
#define LBSORT_NOALLOC_SCRATCH_BYTES (64ull << 20)
int lbsort_sort_pairs_noalloc(int key_type, int val_type, const void *keys_in, const void *vals_in,
                              void *keys_out, void *vals_out, uint64_t n, const lbsort_params *params,
                              const lbsort_parts *parts, uint32_t *dev_err, void *stream);

/*
 * Sort B independent instances at once ("sort multiple different data
 * simultaneously", Section IV.C).  Instance b is input positions
 * [seg_offsets[b], seg_offsets[b+1]) of keys_in/vals_in and is sorted into the
 * same positions of keys_out/vals_out.  seg_offsets is a DEVICE array of B+1
 * non-decreasing values with seg_offsets[0] = 0 and seg_offsets[B] = total_n.
 * Every instance uses the same params; parts arrays are stacked per instance
 * and offsets are relative to the instance's segment.  vals_in may be NULL
 * with val_type = LBSORT_NOVAL.  Nothing is read back to the host, so the
 * whole call can be captured into a HIP graph.
 */
int lbsort_sort_batch(int key_type, int val_type, const void *keys_in, const void *vals_in,
                      void *keys_out, void *vals_out, const uint64_t *seg_offsets, uint32_t B,
                      uint64_t total_n, const lbsort_params *params, const lbsort_parts *parts,
                      void *ws, size_t *ws_bytes, void *stream);

/*
 * Step 1 alone: every block of every instance sorted on its own (stable),
 * written to the same positions of keys_out/vals_out.  Same arguments as
 * lbsort_sort_batch without the partition outputs.
 */
int lbsort_local_sort(int key_type, int val_type, const void *keys_in, const void *vals_in,
                      void *keys_out, void *vals_out, const uint64_t *seg_offsets, uint32_t B,
                      uint64_t total_n, const lbsort_params *params, void *ws, size_t *ws_bytes,
                      void *stream);

/*
 * Binary search over sorted data (Section III, Section IV.C: the sorted
 * result can be searched).  sorted_keys: n keys of key_type in ascending
 * order of that type, e.g. the keys_out of a sort; queries: nq keys of the
 * same type.  For every query j:
 *   pos_out[j]  = number of sorted keys < queries[j] (upper = 0) or
 *                 <= queries[j] (upper = 1), compared in the key type's order
 *                 (floats: totalOrder, so -0 < +0 and NaNs are ordered too);
 *   part_out[j] = the partition k with part_offsets[k] <= pos_out[j] <
 *                 part_offsets[k+1] (the processor that holds that position),
 *                 or P when pos_out[j] = n.  part_out may be NULL; if not,
 *                 part_offsets ([P+1] device, as written by a sort) is required.
 * All arrays are device memory owned by the caller; nothing is allocated.
 * Unsorted input gives unspecified positions but never reads out of range.
 */
int lbsort_search(int key_type, const void *sorted_keys, uint64_t n, const void *queries, uint64_t nq,
                  int upper, const uint64_t *part_offsets, uint32_t P, uint64_t *pos_out,
                  uint32_t *part_out, void *stream);

/*
 * Search index over sorted data (Section III, Section IV.C: the sorted result
 * can be searched; the same queries as lbsort_search, with
 * fewer memory lines per query).  Level l >= 1 of the index holds the keys
 * at positions i * 16^l of sorted_keys, n_l = ceil(n_{l-1} / 16) keys, up to
 * the first level of at most 16 keys; each level starts on a 128-byte
 * boundary.  A query reads one group of 16 keys per level (about
 * log16(n) + 1 cache lines) instead of one line per halving of the range.
 *
 * lbsort_search_index_bytes: bytes of the index of n keys of key_type (0 when
 * n <= 16, where no index is needed; 0 for an invalid key_type).
 *
 * lbsort_search_build_index: writes the index of sorted_keys (n keys, device)
 * into index (device, caller-owned, lbsort_search_index_bytes(key_type, n)
 * bytes, 128-byte aligned), asynchronously on `stream`.  The index stays valid
 * while sorted_keys is unchanged.  Nothing is allocated.
 *
 * lbsort_search_indexed: lbsort_search with the index built for the same
 * sorted_keys and n (index may be NULL when n <= 16); same arguments
 * otherwise, bit-identical outputs.
 */
uint64_t lbsort_search_index_bytes(int key_type, uint64_t n);
int lbsort_search_build_index(int key_type, const void *sorted_keys, uint64_t n, void *index, void *stream);
int lbsort_search_indexed(int key_type, const void *sorted_keys, uint64_t n, const void *index,
                          const void *queries, uint64_t nq, int upper, const uint64_t *part_offsets,
                          uint32_t P, uint64_t *pos_out, uint32_t *part_out, void *stream);

/*
 * Provenance of sorted entries (step 6 of Section IV keeps, for every entry,
 * the processor and the index it came from; Section IV.C exposes them).
 * src_index: count input positions (the vals_out of an LBSORT_VAL_INDEX sort
 * of n keys over P processors).  For each g = src_index[j] < n:
 *   src_block[j]  = the block (processor) i whose input range
 *                   [floor(i n / P), floor((i+1) n / P)) holds g;
 *   src_offset[j] = g - floor(i n / P), the index inside that block.
 * Positions >= n give 0xFFFFFFFF in both.  Either output may be NULL (not
 * both).  n <= 2^32.  Device arrays owned by the caller; nothing allocated.
 */
int lbsort_provenance(const uint32_t *src_index, uint64_t count, uint64_t n, uint32_t P,
                      uint32_t *src_block, uint32_t *src_offset, void *stream);

/*
 * Synchronise `stream` and return the device error latched in `ws` by the
 * last call that used it (LBSORT_OK if none), then clear it.
 */
int lbsort_check(void *ws, void *stream);

/* Static text for a status code, and this thread's last error message. */
const char *lbsort_status_string(int status);
const char *lbsort_last_error(void);

/*
 * Autotuner (Section IV.C's several data sets at once, sorted with settings
 * picked by measurement).  Times candidate settings of one batched shape on
 * the current device and records the fastest in the tuning cache, keyed by
 * the device architecture, the key width, values or not, the instance size
 * (total_n / B, to a power of two), batched or not, and P.  Searched: the
 * radix tile (4096, 8192, and 16384 for 32-bit keys) and the handler schedule (LBSORT_HANDLER_PASSES
 * with each fan-in F = 2 .. 16 up to the power of two above P, and
 * LBSORT_HANDLER_ONE_PASS where it applies) with the default merge tile, then
 * the merge tile (1024, 2048, 4096; 2048 or 4096 for one pass) with the best
 * of those, then whether presorted blocks are looked for.  Every candidate must produce
 * the same bytes (keys, values, part_offsets) as the first, else
 * LBSORT_ERR_DEVICE.  The radix digit is 8 bits wide in every case.
 *
 * keys_in / vals_in / seg_offsets (device): the caller's batch, as for
 * lbsort_sort_batch (seg_offsets may be NULL for B = 1); tuning on it leaves
 * it unchanged.  keys_in == NULL: B synthetic instances of total_n / B
 * uniform random keys instead.  The tuner allocates its own outputs and
 * workspace (device memory) and frees them before returning; it synchronises.
 * cache_path (host): JSON file the whole table is written to (NULL: the
 * $LBSORT_TUNE_CACHE file, or none).  chosen (host, may be NULL) receives the
 * winning settings.  Later calls with fanin / merge_tile / radix_tile = 0 on
 * the same shape class use them.
 */
int lbsort_autotune(int key_type, int val_type, const void *keys_in, const void *vals_in,
                    const uint64_t *seg_offsets, uint32_t B, uint64_t total_n, uint32_t P,
                    const char *cache_path, lbsort_params *chosen);

/* Load a tuning cache written by lbsort_autotune (host path). */
int lbsort_load_tuning(const char *cache_path);

/*
 * The settings a sort call with these arguments would run with on the
 * current device (host only, nothing enqueued): P, s (the default budget
 * resolved), investigator, and fanin / merge_tile / radix_tile / handler /
 * presorted as given, else from the tuning cache, else the defaults.  out
 * (host) receives them.
 */
int lbsort_resolve_params(int key_type, int val_type, uint32_t B, uint64_t total_n,
                          const lbsort_params *params, lbsort_params *out);

/*
 * Measurement aid.  While enabled (on != 0), every kernel launch of the sort
 * calls is bracketed by two HIP events recorded on the call's stream.
 * lbsort_profile_read synchronises those events, writes one line per kernel
 * name, "name launches total_ms\n", into buf (host, len bytes, NUL
 * terminated) and returns the number of bytes needed (excluding the NUL).
 * With buf != NULL the records are cleared; a size query (buf == NULL)
 * keeps them.  Not thread safe; meant for benchmarks.
 */
int lbsort_profile_enable(int on);
int lbsort_profile_read(char *buf, size_t len);

#ifdef __cplusplus
}
#endif
#endif /* LBSORT_H */
