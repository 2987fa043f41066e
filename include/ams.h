/*
 * ams.h -- C ABI of the MI355X (gfx950) adaptive multi-level sample sort.
 *
 * Problem (Section 1, problem statement): permute n elements so that they are
 * sorted.  Equal keys keep their input order: the paper makes all keys unique
 * by breaking ties with the input position (Section 2 and Appendix D), which
 * on one array is the same as a stable sort.  The result is therefore unique:
 * output position i holds the element whose (ord(key), input position) pair is
 * the i-th smallest, keys are returned bit for bit and the payload follows its
 * key.  ord is the identity for unsigned integers and IEEE 754-2008 totalOrder
 * on the bit pattern for float32 (-NaN < -inf < ... < -0 < +0 < ... < +NaN);
 * no floating-point arithmetic is done on keys.
 *
 * Method (Section 6, AMS-sort): per level, a random sample of a*b*r keys is
 * sorted by all-pairs ranking (Section 4.2), b*r-1 splitters of equidistant
 * rank are taken from it, every key is classified into one of b*r buckets
 * (plus equality buckets for keys equal to a splitter, Appendix D), bucket
 * sizes are summed, the buckets are packed into at most r groups of minimal
 * maximum load (Section 6 and its lemma; Appendix C), and the keys are
 * scattered stably into their groups, which are the next level's
 * subproblems.  Groups small enough for one workgroup's LDS are finished by
 * an in-LDS split followed by all-pairs ranking (Section 4.2).
 *
 * Memory.  Every key/payload pointer is DEVICE memory owned by the caller;
 * the library never frees caller memory.  `stream` is a hipStream_t (NULL =
 * the default stream).  All sort calls only enqueue work on `stream` and
 * return; results are ready when the stream reaches that point.  A kernel
 * fault surfaces at the caller's next synchronisation.
 *
 * Errors.  Functions return 0 (AMS_OK) or a negative ams_status; no C++
 * exception crosses this boundary.  ams_last_error() gives a message for the
 * calling thread's last failure.  n = 0 and n = 1 are valid no-op-like sorts
 * (n = 1 still copies d_in to d_out).
 */
#ifndef AMS_H
#define AMS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  AMS_U32 = 1, /* uint32_t keys */
  AMS_U64 = 2, /* uint64_t keys (the paper's 64-bit integers, Section 7) */
  AMS_F32 = 3  /* float32 keys, ordered by totalOrder on their bits */
} ams_key_t;

typedef int ams_status;
#define AMS_OK 0
#define AMS_EINVAL (-1)       /* bad argument: NULL pointer with n > 0, unknown key type, ... */
#define AMS_ENOMEM (-2)       /* workspace too small / allocation failed / request can never fit */
#define AMS_EHIP (-3)         /* a HIP runtime call failed */
#define AMS_EAGAIN (-4)       /* server: pending queue full, try again */
#define AMS_EUNSUPPORTED (-5) /* size or option outside what the library supports */
#define AMS_ENOTFOUND (-6)    /* server: unknown or released ticket */
#define AMS_EDEVICE (-7)      /* the device raised an error (AMS_DEVERR_* bits): a table
                                 bound was exceeded and the output is not valid */

/* Largest segment (keys of one sort, of one batch segment or of one served
 * request): 2^32 - 2^20.  Payloads are 32-bit positions, and the kernels'
 * 32-bit tile arithmetic stays exact up to this size. */
#define AMS_MAX_SEGMENT ((1ull << 32) - (1ull << 20))

/* Device error bits.  Every table the kernels fill is sized on the host to an
 * upper bound of what the plan can produce; a kernel that would exceed one
 * (which means a bug, or the test hook AMS_FLAG_TEST_TINY_TABLES) skips the
 * write, keeps every access in bounds and raises one of these bits in the
 * run's counters and in the device's error word (ams_device_errors). */
#define AMS_DEVERR_TABLE 1u   /* the leaf list or an active-subproblem list was full */
#define AMS_DEVERR_ACTIVE 2u  /* more active subproblems than the level's table */
#define AMS_DEVERR_TILES 4u   /* more tiles, tile blocks or sample blocks than planned */
#define AMS_DEVERR_GROUPS 8u  /* a grouping gave more children than its table holds */
#define AMS_DEVERR_RANGE 16u  /* a scatter destination fell outside its child's range */
#define AMS_DEVERR_LEAF 32u   /* a leaf reached outside its segment */

/* Tuning parameters.  A zero field means "choose automatically": the
 * autotuner's choice for the call's shape class when ams_autotune has made
 * one, else the built-in defaults (k = 256, b = 4 for one sort; k = 128,
 * b = 2 for a batch of several segments, and b = 2 below the first level
 * when the planned leaves average at most 30% of the base case's capacity;
 * a = 8 samples per bucket at the first level and 2 below; cutoff 32; tiles
 * of 64 Ki keys from 2^27 keys, else 32 Ki); passing NULL means all
 * defaults.  Names follow the
 * paper: k is the number of groups per level (the paper's r), b the
 * overpartitioning factor, a the oversampling factor (Section 6). */
typedef struct {
  uint32_t levels;             /* partition levels before the base case */
  uint32_t k;                  /* groups per level r; power of two, 2..1024 */
  uint32_t overpartition_b;    /* buckets per group b; power of two, k*b <= 2048 */
  uint32_t samples_per_bucket; /* oversampling factor a */
  uint32_t tile_keys;          /* keys per workgroup tile in a level pass (multiple of 4096,
                                  at most 2^19) */
  uint32_t base_cutoff;        /* largest bucket handed to the all-pairs ranker, <= 1024 */
  uint64_t seed;               /* sampling seed (0 = fixed default) */
  uint32_t flags;              /* AMS_FLAG_* */
  uint32_t leaf_capacity;      /* test hook: subproblems larger than this are not finished in
                                  LDS (0 = the workgroup's capacity); lowering it forces the
                                  slow paths on small inputs */
} ams_params;

#define AMS_FLAG_EQ_ALWAYS 1u /* equality buckets on for every subproblem */
#define AMS_FLAG_STABLE_PARTITION 2u /* keys-only: partition levels keep input order inside
                                        every child (pairs always do); the sorted output is
                                        the same either way */
#define AMS_FLAG_SAMPLED_LEAF_SPLIT 4u /* base case: split every leaf by sampled splitters
                                          instead of first trying its key range; the sorted
                                          output is the same either way (test hook) */
#define AMS_FLAG_STRATIFIED 32u /* below the first level, each subproblem's splitters follow
                                   the buckets its group brought from the level above
                                   (Section 6: the overpartitioning exploited in the
                                   recursion): every bucket boundary is kept as a splitter
                                   and the buckets are shared among them in proportion to
                                   their exact sizes; the sorted output is the same */
#define AMS_FLAG_CHECK 8u /* the call waits for its stream before returning and returns
                             AMS_EDEVICE if its kernels raised a device error */
#define AMS_FLAG_TEST_TINY_TABLES 16u /* test hook: the leaf list holds one entry, so any
                                         sort with more than one leaf raises
                                         AMS_DEVERR_TABLE (its output is then invalid) */
#define AMS_FLAG_TEST_NO_PIECE_ROOM 64u /* test hook: the pieces of oversized leaves find the
                                           leaf list full and are finished by the remainder
                                           pass (the sorted output is the same) */

/* Bytes of device workspace a call with these arguments needs.  Returns 0 on
 * invalid arguments.  ams_sort_* accept d_ws = NULL, in which case they
 * allocate (stream-ordered) and free the workspace themselves. */
size_t ams_workspace_bytes(ams_key_t t, size_t n, int with_vals, const ams_params *p);

/* Workspace for ams_sort_batch; h_offsets is the host copy of the num+1
 * segment offsets. */
size_t ams_batch_workspace_bytes(ams_key_t t, const uint64_t *h_offsets, size_t num,
                                 int with_vals, const ams_params *p);

/* Sort n keys.  d_in (n keys) and d_out (n keys) may be the same buffer
 * (in-place).  n <= AMS_MAX_SEGMENT, else AMS_EUNSUPPORTED.  Section 6
 * (AMS-sort), Section 1 (output requirement). */
ams_status ams_sort_keys(ams_key_t t, const void *d_in, void *d_out, size_t n, void *d_ws,
                         size_t ws_bytes, void *stream, const ams_params *p);

/* Sort without allocating, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  The same sort as ams_sort_keys, with its workspace taken from
 * a fixed array of AMS_NOALLOC_SCRATCH_BYTES in device memory that the
 * library holds on every device it runs on until the process ends; the call
 * makes no hipMalloc, hipFree or other allocating call.  `stream` must
 * belong to the current device.  Returns AMS_EUNSUPPORTED when
 * ams_workspace_bytes(t, n, 0, p) exceeds the array (about 4.5 M uint64 or
 * 7.7 M 32-bit keys with the default parameters).  Every call on a device
 * shares that device's array, which keeps the last call's contents (each
 * call clears what it needs with its own kernels): calls that overlap on
 * one device, from different streams or threads, race and must be
 * serialised by the caller. */
#define AMS_NOALLOC_SCRATCH_BYTES (64ull << 20)
ams_status ams_sort_keys_noalloc(ams_key_t t, const void *d_in, void *d_out, size_t n,
                                 void *stream, const ams_params *p);

/* Stable key/payload sort: payload d_vin[i] follows key d_kin[i].  Output
 * arrays may alias the inputs.  Section 6; stability from the position
 * tie-break of Section 2 / Appendix D. */
ams_status ams_sort_pairs(ams_key_t t, const void *d_kin, const uint32_t *d_vin, void *d_kout,
                          uint32_t *d_vout, size_t n, void *d_ws, size_t ws_bytes, void *stream,
                          const ams_params *p);

/* ------------------------------------------------------------------------
 * RLM-sort: recurse-last multiway mergesort (Section 5), the paper's second
 * algorithm.  Every tile of tile_keys keys is sorted in LDS first (every PE
 * sorts locally); then level by level every group of sorted sequences is
 * split into `ways` parts of exactly equal size by multisequence selection
 * (Section 4.1, all boundaries of a level side by side), each part receives
 * its piece of every sequence and merges them, in slices of tile_keys keys,
 * into the sorted sequences of the next level.  Parts of at most one tile
 * are merged into the output.  The output is the same as ams_sort_keys'.
 * ------------------------------------------------------------------------ */
typedef struct {
  uint32_t ways;       /* parts per group and level (0 = 16) */
  uint32_t tile_keys;  /* keys per tile and per merged slice, multiple of 64, at most 4096
                          (0 = 4096) */
  uint64_t seed;       /* pivot seed (0 = fixed default); the output does not depend on it */
  uint32_t flags;      /* AMS_FLAG_CHECK */
  uint32_t reserved;
} ams_rlm_params;

/* Workspace of ams_rlm_sort_keys (0 on invalid arguments). */
size_t ams_rlm_workspace_bytes(ams_key_t t, size_t n, const ams_rlm_params *p);

/* RLM-sort of n keys (n <= AMS_MAX_SEGMENT); d_in and d_out may be the same
 * buffer.  d_ws = NULL allocates the workspace in stream order.  Section 5;
 * selection Section 4.1. */
ams_status ams_rlm_sort_keys(ams_key_t t, const void *d_in, void *d_out, size_t n, void *d_ws,
                             size_t ws_bytes, void *stream, const ams_rlm_params *p);

/* Batched sort: segment i = elements [h_offsets[i], h_offsets[i+1]) of the
 * key (and optional payload) arrays is sorted independently, each result
 * identical to sorting that segment alone.  h_offsets (host, num+1 entries,
 * non-decreasing, h_offsets[0] = 0) plans the work; d_offsets (device copy,
 * may be NULL) saves the upload.  d_vin/d_vout are NULL for keys-only.  All
 * segments run through the same level kernels together; no per-segment
 * launches.  Section 6 applied to many independent inputs. */
ams_status ams_sort_batch(ams_key_t t, const void *d_kin, const uint32_t *d_vin, void *d_kout,
                          uint32_t *d_vout, const uint64_t *h_offsets, const uint64_t *d_offsets,
                          size_t num, void *d_ws, size_t ws_bytes, void *stream,
                          const ams_params *p);

/* Autotuner.  Times candidate parameter sets (levels, k, overpartition_b,
 * base_cutoff, tile_keys; one changed at a time from the built-in defaults,
 * keeping each improvement) for sorting the num segments h_offsets describes
 * (num = 1, h_offsets = {0, n} for a single sort) of d_kin (and d_vin when
 * non-NULL), and writes the fastest to *best (its time per sort in ms to
 * *best_ms when non-NULL).  The input is only read: candidates sort into
 * buffers the tuner allocates (about twice the input) and frees.  Every
 * candidate's output must equal the first one's bit for bit, else AMS_EHIP.
 * At most max_trials candidates are timed (0 = 24), each three times.
 * Synchronises `stream`.  The choice is remembered for the process, keyed by
 * the shape class (key type, payload, floor(log2) of the total, of the
 * largest segment and of the segment count): later sort calls of that class
 * whose ams_params leave a tuned field zero (or pass NULL) use it.  The
 * workspace size of such a call follows the tuned parameters, so query
 * ams_*workspace_bytes after tuning.  Section 7 chooses levels and group
 * counts from the machine size; here they are measured. */
ams_status ams_autotune(ams_key_t t, const void *d_kin, const uint32_t *d_vin,
                        const uint64_t *h_offsets, size_t num, void *stream, uint32_t max_trials,
                        ams_params *best, double *best_ms);

/* Forget every autotuned choice of this process. */
void ams_autotune_clear(void);

/* Message for the calling thread's most recent error ("" if none). */
const char *ams_last_error(void);

/* Device errors.  Sort calls return once their kernels are enqueued, so an
 * error a kernel raises later cannot be their return value (unless the call
 * passed AMS_FLAG_CHECK).  Every such error is also ORed into a per-device
 * error word; this call waits for `stream` (a stream of the current device),
 * stores the word's AMS_DEVERR_* bits in *bits (0 = no error since the last
 * clear) and, when `clear` is nonzero, resets it. */
ams_status ams_device_errors(void *stream, uint32_t *bits, int clear);

/* Statistics of the last sort that ran in a caller-provided workspace d_ws
 * (its counters sit at the start of the workspace).  Waits for `stream`.
 * Level l's subproblems are what its partition pass read and wrote; keys
 * placed in final children (equality buckets, Appendix D) drop out of later
 * passes.  The imbalance of a subproblem is its grouping's maximum load L*
 * over the average ceil(W / r) of the W keys outside final children, the
 * ratio that the load-balance lemma of Section 6 bounds by 1 + eps. */
typedef struct {
  uint32_t device_errors;     /* AMS_DEVERR_* bits raised by the run */
  uint32_t levels;            /* partition levels of the plan */
  uint32_t subproblems[4];    /* subproblems level l partitioned */
  uint64_t keys[4];           /* keys in them */
  uint64_t final_keys[4];     /* keys level l placed in final children */
  uint32_t max_child[4];      /* largest regular child level l produced */
  uint32_t tiles[4];          /* tiles (workgroup items) of level l's passes */
  double imbalance_max[4];    /* largest L* / ceil(W / r) over level l's subproblems */
  double imbalance_mean[4];   /* its mean over the subproblems with W > 0 */
  uint32_t leaves;            /* leaves the base-case kernel processed */
  uint32_t big_leaves;        /* of those, larger than one workgroup's LDS: each is
                                 partitioned once more in HBM by its workgroup */
  uint64_t leaf_keys;         /* keys sorted in LDS by the base case */
  uint64_t copy_keys;         /* keys of final children copied to the output */
  uint64_t big_keys;          /* keys in oversized leaves */
  uint32_t merge_ranges;      /* pieces of oversized leaves still larger than one
                                 workgroup's LDS, sorted by the merge fallback */
  uint32_t reserved;
  uint64_t merge_keys;        /* keys in those pieces */
} ams_run_stats;
ams_status ams_workspace_stats(const void *d_ws, void *stream, ams_run_stats *out);

/* Per-kernel timing (tracing).  ams_trace_start() makes every later sort
 * call of the calling thread bracket each kernel launch with a pair of
 * hipEvents on the call's stream; ams_trace_stop() waits for them, sums the
 * elapsed times per kernel name (name.L<level> for level kernels) into `out`
 * (up to `max` entries) and returns the number of entries.  Tracing adds a
 * few microseconds per launch. */
typedef struct {
  char name[32];
  uint32_t launches;
  uint32_t reserved;
  double total_ms;
  double max_ms;
} ams_trace_entry;
ams_status ams_trace_start(void);
int ams_trace_stop(ams_trace_entry *out, int max);

/* Measurement aid: a plain streaming copy of `bytes` from d_src to d_dst
 * (both 16-byte aligned, not overlapping), enqueued on `stream`.  Its rate is
 * the practical HBM ceiling the level passes are measured against. */
ams_status ams_device_copy(const void *d_src, void *d_dst, size_t bytes, void *stream);

/* Library version string. */
const char *ams_version(void);

/* ------------------------------------------------------------------------
 * Serving: continuous batching of independent sort requests.
 *
 * A server owns worker streams on one device and a budget of device memory.
 * ams_submit queues a request whose keys (and optional payload) already sit
 * in device memory; requests are admitted while the bytes they need (result
 * buffers + workspace) fit in the budget, admitted requests are batched as
 * they arrive and sorted by ams_sort_batch-equivalent launches on the worker
 * streams, so batches overlap on the device.  Results stay on the device in
 * server-owned buffers until released.  Each result equals sorting that
 * request alone.
 * ------------------------------------------------------------------------ */
typedef struct ams_server ams_server;

typedef struct {
  uint64_t n;          /* keys in the request */
  int32_t key_type;    /* ams_key_t */
  int32_t status;      /* AMS_OK, or the error that ended the request */
  uint64_t batch_id;   /* batch the request ran in */
  uint32_t batch_size; /* requests in that batch */
  uint32_t reserved;
  double t_submit_us;  /* host clock (microseconds since server creation) */
  double t_admit_us;   /* admitted against the memory budget */
  double t_launch_us;  /* batch enqueued */
  double t_done_us;    /* completion observed */
  double gpu_ms;       /* device time of the batch (event pair) */
} ams_req_stats;

/* Create a server on `device` with `hbm_budget` bytes (0 = 80% of free
 * memory), at most `max_pending` queued + running requests (0 = 4096) and
 * `n_streams` worker streams (0 = 2).  Returns NULL and sets *st on failure. */
ams_server *ams_server_create(int device, size_t hbm_budget, uint32_t max_pending,
                              uint32_t n_streams, ams_status *st);

/* Queue a request.  d_keys must stay valid until the request completes.
 * Returns AMS_ENOMEM if the request alone can never fit the budget,
 * AMS_EAGAIN if max_pending requests are already queued or running and
 * AMS_EUNSUPPORTED for n > AMS_MAX_SEGMENT.  A request whose batch fails
 * (an allocation, a launch, or a device error its kernels raise) finishes
 * with that status in its ams_req_stats and from ams_wait; the server goes
 * on serving later requests. */
ams_status ams_submit(ams_server *srv, ams_key_t t, const void *d_keys, const uint32_t *d_vals,
                      size_t n, uint64_t *ticket);

/* Non-blocking completion check; *done = 1 when finished (stats filled). */
ams_status ams_poll(ams_server *srv, uint64_t ticket, int *done, ams_req_stats *stats);

/* Block until the request is finished. */
ams_status ams_wait(ams_server *srv, uint64_t ticket, ams_req_stats *stats);

/* Device pointers of a finished request's sorted keys / payload (NULL when
 * the request had none).  Valid until ams_release. */
ams_status ams_result(ams_server *srv, uint64_t ticket, void **d_keys, uint32_t **d_vals);

/* Copy a finished request's sorted keys / payload into caller device buffers
 * (either may be NULL), enqueued on `stream`. */
ams_status ams_result_copy(ams_server *srv, uint64_t ticket, void *d_keys, uint32_t *d_vals,
                           void *stream);

/* Free a finished request's result buffers and forget the ticket.  The
 * buffers are freed in stream order on a server stream: work of the caller
 * that reads them (ams_result pointers, an ams_result_copy) must have
 * completed, e.g. its stream synchronised, before this call. */
ams_status ams_release(ams_server *srv, uint64_t ticket);

/* Drain outstanding work, free everything. */
void ams_server_destroy(ams_server *srv);

/* Test hook for failure handling: the next `count` batches the server forms
 * fail as if their device allocation had failed, so their requests finish
 * with AMS_ENOMEM. */
ams_status ams_server_inject_alloc_failures(ams_server *srv, uint32_t count);

/* ------------------------------------------------------------------------
 * Step entry points: one step of the path on one subproblem, for checking
 * each kernel against its plain definition.  Keys here are ord values
 * (uint32 for AMS_U32/AMS_F32, uint64 for AMS_U64) unless stated.
 * ------------------------------------------------------------------------ */

/* Sample and splitters (Section 6; sample sorted by all-pairs rank, Section
 * 4.2).  Draws a*m positions of d_keys[0..n) with SplitMix64 keyed by (seed,
 * level 0, root 0, offset 0), ranks the sample, and writes the m-1 splitters
 * of rank j*a-1 (j = 1..m-1) as ord values to d_splitters.  m is a power of
 * two in 2..2048 and a*m <= 8192 (uint64) or 16384 (32-bit keys). */
ams_status ams_step_splitters(ams_key_t t, const void *d_keys, size_t n, uint32_t m, uint32_t a,
                              uint64_t seed, void *d_splitters, void *stream);

/* One level pass with given sorted splitters (ord values, m-1 of them):
 * classification (with equality buckets when two splitters are equal or
 * flags has AMS_FLAG_EQ_ALWAYS), bucket histogram (d_hist, 2m-1 uint32
 * entries; only the first m are written without equality buckets), bucket
 * grouping into at most r groups, children (d_children: 4 uint32 per child
 * = first id, end id, size, kind 0 regular / 1 final; *n_children set on the
 * host after the call synchronises `stream`), and the stable scatter of
 * d_in[0..n) into d_out (raw keys in, ord-ordered children out, keys
 * bit-identical).  Sections 6 and 4.3; Appendix C and D. */
ams_status ams_step_level(ams_key_t t, const void *d_in, void *d_out, size_t n,
                          const void *d_splitters, uint32_t m, uint32_t r, uint32_t flags,
                          uint32_t *d_hist, uint32_t *d_children, uint32_t *n_children,
                          void *stream);

/* Multisequence selection alone (Section 4.1), one RLM-sort level's
 * boundaries: d_runs holds n keys (raw bits) that are sorted within
 * consecutive runs of run_keys keys (the last run may be shorter); the
 * keys are ordered by (ord value, run, position).  For j = 0..parts, row j
 * of d_cuts (parts+1 rows of ceil(n / run_keys) uint32 entries, device)
 * receives, for every run, how many of its keys are among the
 * floor(j n / parts) smallest.  1 <= parts <= min(1024, n).  Synchronises
 * `stream`; AMS_EDEVICE if a selection did not finish.  Runs that are not
 * sorted give unspecified cuts (AMS_EDEVICE where the selection notices)
 * but every read stays inside its run. */
ams_status ams_step_multiselect(ams_key_t t, const void *d_runs, size_t n, uint32_t run_keys,
                                uint32_t parts, uint64_t seed, uint32_t *d_cuts, void *stream);

/* Bucket grouping alone (Section 6 and its lemma; Appendix C): w[0..nb)
 * weights -> d_out[0] = optimal maximum load L*, d_out[1] = number of groups
 * g, d_out[2..2+g) = start index of each greedy group under L*.  nb <= 4095;
 * the weights must sum to less than 2^32 (as bucket sizes of one subproblem
 * do); d_out holds nb + 2 words. */
ams_status ams_step_pack(const uint32_t *d_w, uint32_t nb, uint32_t r, uint32_t *d_out,
                         void *stream);

/* Base case alone: sort one array of n <= 8192 keys (and optional payload)
 * inside one workgroup by an in-LDS split followed by all-pairs ranking
 * (Section 4.2).  base_cutoff as in ams_params (0 = default). */
ams_status ams_step_base_case(ams_key_t t, const void *d_kin, const uint32_t *d_vin,
                              void *d_kout, uint32_t *d_vout, size_t n, uint32_t base_cutoff,
                              void *stream);

#ifdef __cplusplus
}
#endif

#endif /* AMS_H */
