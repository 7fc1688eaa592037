/*
 * swx.h -- MI355X (gfx950) Smith-Waterman-Gotoh alignment library, C ABI.
 *
 * What it computes (paper: "SSW Library: An SIMD Smith-Waterman C/C++ Library
 * for Use in Genomic Applications"; Introduction and method section
 * "Algorithm and implementation"): the optimal local alignment of a query
 * against a reference under a substitution matrix and affine gaps,
 *
 *   H(i,j) = max(0, H(i-1,j-1) + S(q_i, r_j), E(i,j), F(i,j))
 *   E(i,j) = max(E(i,j-1) - e, H(i,j-1) - o)   gap consuming reference (D)
 *   F(i,j) = max(F(i-1,j) - e, H(i-1,j) - o)   gap consuming query     (I)
 *
 * so a gap of length k costs o + (k-1)*e.  The Results section's API
 * description fixes the outputs: the optimal score, its end and begin on the
 * query and the reference, the detailed alignment (CIGAR), and the score and
 * end of the best suboptimal alignment, obtained as in the method section:
 * a per-column "max" array gives the end, a reversed pass from the end gives
 * the begin, a banded pass between begin and end gives the CIGAR, and the max
 * array with the primary alignment's region masked gives the second score.
 *
 * Ties (the paper leaves them open; every build of this library resolves them
 * the same way, so results are deterministic and independent of lane width,
 * batching or scheduling):
 *   end     smallest reference position, then smallest query position, among
 *           cells scoring score1;
 *   begin   among begins from which an alignment reaches that end with score
 *           score1: largest reference position, then largest query position;
 *   CIGAR   traceback of the global 3-state DP on [begin, end] preferring
 *           M, then D, then I, and inside a gap "open" before "extend";
 *   score2  largest max-array value outside columns
 *           [ref_begin1 - mask_len, ref_end1 + mask_len]; ref_end2 is its
 *           smallest column; mask_len < 0 selects max(qlen/2, 15).
 *   score1 == 0 means "no alignment": every coordinate is -1.
 *
 * Conventions: sequences are int8 symbol codes in [0, n); the matrix is
 * row-major n x n int8 indexed [query symbol][reference symbol]; gap_open and
 * gap_extend are positive magnitudes with gap_open >= gap_extend >= 0.
 * Coordinates are 0-based and inclusive.  CIGAR words are (length << 4) | op
 * with op 0 = M, 1 = I (consumes query), 2 = D (consumes reference), as in SAM.
 *
 * Errors: every call returns SWX_OK (0) or a negative status; no exception
 * crosses the ABI.  swx_last_error() returns a message for the calling
 * thread's last failure.  Inputs are validated before any alignment work; a
 * rejected call leaves outputs untouched.
 *
 * Threads: a context serialises its own calls; use one context per thread for
 * concurrency.  Profiles are immutable after creation and may be shared by
 * threads that use the same context.
 */
#ifndef SWX_H
#define SWX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define SWX_OK         0
#define SWX_EINVAL    -1   /* bad argument: null pointer, symbol >= n, o < e, n > 32, ... */
#define SWX_ENOMEM    -2   /* host or device allocation failed */
#define SWX_EDEVICE   -3   /* a HIP call failed (message in swx_last_error) */
#define SWX_EBUSY     -4   /* serving: admission refused (non-blocking submit) */
#define SWX_EOVERFLOW -5   /* a score could exceed the 32-bit lanes (query*max score >= 2^26) */
#define SWX_ERANGE    -6   /* caller's CIGAR arena too small; cigar_used holds the size needed */
#define SWX_EINTERNAL -7   /* an internal consistency check failed (a bug: please report) */

/* ---- flags --------------------------------------------------------------- */
#define SWX_BEGIN   1u     /* compute read_begin1 / ref_begin1 (reversed pass) */
#define SWX_CIGAR   2u     /* compute the CIGAR (banded pass); implies SWX_BEGIN */
#define SWX_SCORE2  4u     /* compute score2 / ref_end2; implies SWX_BEGIN */
#define SWX_ALL     7u
#define SWX_SUBOPT  8u     /* also the alignment behind score2 (method section; the dashed
                              path of Fig. 1): into swx_batch_out.sub_recs for batch calls,
                              swx_result.sub for swx_align; implies SWX_ALL.  Reading: it ends in column ref_end2 at the
                              smallest row whose H equals score2; its begin is T2 relative to
                              that end (among begins of alignments reaching the end with
                              score exactly score2: largest ref begin, then largest query
                              begin); its CIGAR is T3 on that rectangle.  Pairs with score2 ==
                              0 get -1 coordinates and no CIGAR. */

#define SWX_MEM_HOST   0u  /* buffers are host memory */
#define SWX_MEM_DEVICE 1u  /* buffers are device memory of the context's GPU */

typedef struct swx_ctx swx_ctx;
typedef struct swx_profile swx_profile;

/* One alignment result (56 bytes).  In batch output, cigar_off indexes the
 * batch's CIGAR arena; cigar_len is the number of CIGAR words. */
typedef struct {
  int32_t score1, score2;
  int32_t read_begin1, read_end1;
  int64_t ref_begin1, ref_end1, ref_end2;
  int64_t cigar_off;
  int32_t cigar_len;
  int32_t lane_bits;   /* lane width that produced the result (16 or 32); diagnostic only */
} swx_rec;

/* Single-pair result: the record plus a CIGAR owned by the result, and with
 * SWX_SUBOPT the suboptimal alignment's record (score1 = score2, begins and
 * end of that alignment; score2 0, ref_end2 -1) and CIGAR (release both with
 * swx_result_free; sub is zeroed and sub_cigar NULL without SWX_SUBOPT). */
typedef struct {
  swx_rec rec;
  uint32_t *cigar;
  swx_rec sub;
  uint32_t *sub_cigar;
} swx_result;

/* ---- context --------------------------------------------------------------
 * device: HIP device ordinal.  The context owns a stream and a device memory
 * pool that grows on demand and is reused across calls. */
int swx_ctx_create(int device, swx_ctx **out);
int swx_ctx_destroy(swx_ctx *ctx);

/* ---- profiles (method section: the query profile built once per query) ----
 * query: host codes [qlen], qlen >= 1.  matrix: host n x n, 1 <= n <= 32.
 * The profile copies everything it needs; the caller keeps ownership of its
 * buffers.  Errors: SWX_EINVAL (nulls, qlen < 1, n out of range, symbol >= n,
 * gap_open < gap_extend, gap_extend < 0, gap_open > 32767). */
int swx_profile_create(swx_ctx *ctx, const int8_t *query, int32_t qlen, const int8_t *matrix,
                       int32_t n, int32_t gap_open, int32_t gap_extend, swx_profile **out);
int swx_profile_destroy(swx_profile *p);

/* ---- one pair --------------------------------------------------------------
 * The paper's per-pair call (Results section, the library's API: a profile
 * aligned against one reference returns the optimal score, the suboptimal
 * score, both ends, both begins and the CIGAR; method section "Algorithm and
 * implementation" for how each is found).
 * p: a profile of this library (its context runs the call).  ref: [rlen]
 * codes in host memory, or device memory of the context's GPU when flags has
 * SWX_REF_DEVICE; the caller keeps ownership.  rlen == 0 is valid and yields
 * "no alignment".  flags: SWX_BEGIN | SWX_CIGAR | SWX_SCORE2 | SWX_SUBOPT
 * (+ SWX_REF_DEVICE);
 * mask_len as for swx_align_batch.  hip_stream: a hipStream_t of the
 * context's device, or NULL for the context's own stream; the call's device
 * work is queued on it, after whatever the caller queued there before (a
 * device-resident ref may be written by that earlier work).  Synchronous:
 * returns when out is filled (it waits for that stream, never for the whole
 * device).  out->cigar is malloc'd by the library (NULL when the CIGAR was
 * not requested or is empty; release with swx_result_free).  A pair of
 * qlen <= 4096 and rlen <= 65536 replays a graph of capacity one pair (the
 * chain of swx_graph_*, one pair spread over a wave) captured on first use
 * for its scoring scheme, flags, mask width and power-of-two size class and
 * kept on the context (at most 8, least recently used replaced); larger pairs,
 * and calls with SWX_SUBOPT, take the batch path.  Either way the result
 * equals swx_align_batch's.
 * Errors: SWX_EINVAL (null p or out, rlen < 0, unknown flag bits, a symbol
 * >= n: out untouched beyond being zeroed), SWX_EDEVICE, SWX_ENOMEM. */
#define SWX_REF_DEVICE (1u << 8)
int swx_align(const swx_profile *p, const int8_t *ref, int64_t rlen, uint32_t flags,
              int32_t mask_len, void *hip_stream, swx_result *out);
void swx_result_free(swx_result *r);

/* ---- many pairs ------------------------------------------------------------
 * The per-pair computation of swx_align (method section "Algorithm and
 * implementation": max array and end, reversed pass for the begin, banded
 * pass for the CIGAR, masked max array for score2; Results section for the
 * outputs), for many pairs in one call: the paper's callers align one query
 * against many references (database search) or many reads against their
 * windows (read mapping), which here share launches.
 * Queries and references are concatenated code arrays with offsets
 * (qoff[nq+1], roff[nr+1], non-decreasing, within [0, qcat_len] and
 * [0, rcat_len]); pair k aligns query pair_q[k] against reference pair_r[k].
 * in_mem says where qcat/qoff/rcat/roff/pair_q/pair_r live; matrix is always
 * host memory. */
typedef struct {
  const int8_t *matrix; int32_t n; int32_t gap_open; int32_t gap_extend;
  const int8_t *qcat; int64_t qcat_len; const int64_t *qoff; int64_t nq;
  const int8_t *rcat; int64_t rcat_len; const int64_t *roff; int64_t nr;
  const int64_t *pair_q; const int64_t *pair_r; int64_t npairs;
  uint32_t flags;      /* SWX_BEGIN | SWX_CIGAR | SWX_SCORE2 */
  int32_t mask_len;    /* < 0: max(qlen/2, 15) per pair */
  uint32_t in_mem;     /* SWX_MEM_HOST or SWX_MEM_DEVICE */
} swx_batch;

/* Output of a batch.  recs [npairs] and cigar [cigar_cap] are caller-owned and
 * live in out_mem.  On SWX_ERANGE the records are complete but the CIGARs did
 * not fit: cigar_used holds the number of words needed.  With SWX_SUBOPT,
 * sub_recs [npairs] (also in out_mem) receives each pair's suboptimal
 * alignment as a record -- score1 = score2, read/ref begin and end of that
 * alignment, score2 = 0, ref_end2 = -1 -- with its CIGAR in the same arena
 * after every primary CIGAR (cigar_off counts from the arena's start). */
typedef struct {
  swx_rec *recs;
  uint32_t *cigar;
  int64_t cigar_cap;
  int64_t cigar_used;  /* out */
  uint32_t out_mem;
  uint32_t pad_;
  swx_rec *sub_recs;   /* SWX_SUBOPT only; otherwise ignored (may be NULL) */
} swx_batch_out;

/* Aligns every pair.  hip_stream: a hipStream_t of the context's device, or
 * NULL for the context's own stream; every kernel and copy of the call is
 * queued on it (side streams of the context fork from it and join back into
 * it), after whatever the caller queued there before, so device-resident
 * inputs may be written by that earlier work.  Synchronous with respect to
 * the host: returns when the outputs are written (waiting for that stream,
 * never for the whole device).  Errors: SWX_EINVAL (null pointers, negative
 * counts, bad memory-space flag or flag bits, offsets, pair indices or
 * symbols out of range), SWX_EOVERFLOW, SWX_ERANGE (records complete, CIGARs
 * not copied), SWX_ENOMEM, SWX_EDEVICE, SWX_EINTERNAL. */
int swx_align_batch(swx_ctx *ctx, const swx_batch *b, swx_batch_out *out, void *hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * alignments as swx_align_batch (same arguments, same results), with every
 * scratch buffer of the call taken from one static device array of
 * SWX_NOALLOC_SCRATCH_BYTES that the library holds on each GPU it runs on
 * until the process ends.  The call makes no hipMalloc, hipFree, stream or
 * other allocating library call; the caller still provides the inputs and
 * outputs.  Side streams are not used.  All calls on one GPU share that
 * GPU's array and run one at a time (a call returns only after its device
 * work is done; overlapping calls from other threads wait); the array keeps
 * the last call's contents, and every call clears what it needs.  Limits:
 * npairs <= SWX_NOALLOC_MAX_PAIRS and, for host-memory inputs, the staged
 * inputs within half of the array (SWX_EINVAL otherwise, before any device
 * work); a batch whose work needs more scratch than the array fails with
 * SWX_ENOMEM (outputs then undefined).  About 4,000 pairs of 250 x 650 fit.
 * hip_stream: as for swx_align_batch. */
#define SWX_NOALLOC_SCRATCH_BYTES (64u << 20)
#define SWX_NOALLOC_MAX_PAIRS 65536
int swx_align_batch_noalloc(swx_ctx *ctx, const swx_batch *b, swx_batch_out *out,
                            void *hip_stream);

/* Upper bound on CIGAR words for a batch: sum over pairs of qlen + rlen + 1,
 * twice that with SWX_SUBOPT (host-memory batches only; returns -1 otherwise). */
int64_t swx_cigar_bound(const swx_batch *b);

/* ---- launch configuration ---------------------------------------------------
 * Knobs that move work between kernels.  Results never depend on them: every
 * setting computes the same alignments (rules above), only faster or slower.
 *   long_cells, long_rlen  a pair with qlen * rlen > long_cells or
 *                          rlen > long_rlen takes the intra-sequence path
 *                          (one pair spread over a wave, reference cut into
 *                          column chunks); others are batched, one pair per
 *                          16-bit lane half.  long_cells = -1 (the default)
 *                          derives the threshold from each call: twice the
 *                          call's cells per lane half of a full GPU, at least
 *                          2048.  long_cells >= -1, long_rlen >= 0.
 *   intra_jobs             target number of column chunks over all long pairs
 *                          of one call, >= 1.
 *   fill_rows              query rows per strip of the batched fill: 16, 24 or
 *                          32 (24 applies to alphabets of at most 4 symbols;
 *                          others use 32 instead).
 * Errors: SWX_EINVAL for null pointers or values out of range (ctx unchanged). */
typedef struct {
  int64_t long_cells;
  int64_t long_rlen;
  int64_t intra_jobs;
  int32_t fill_rows;
  int32_t side_streams;  /* 1: independent traceback launches run side by side on two
                            side streams of the context (made on first use); 0: all
                            on the context's stream (one hardware queue per context) */
  int32_t fill_sched;    /* order of the batched fill's tasks (tasks are sorted by size,
                            ascending): 0 in that order, one wave per task; 1 largest
                            first (default); 2 a grid of resident waves taking tasks
                            largest first from a device work queue */
  int32_t fill_coop;     /* 0 (default): a pass with fewer tasks than the device holds
                            waves runs each task on the four waves of a workgroup, which
                            take its strips round robin (a strip follows the one above
                            column group by column group); 1: never; 2: always */
  int32_t intra_bits;    /* lanes of the intra-sequence forward pass. 16: packed 16-bit
                            lanes, two column chunks per wave (on twice intra_jobs chunks),
                            for every long pair whose scores fit (smax * min(qlen, rlen)
                            + bias <= 32766), 32-bit for the others; 32: always 32-bit;
                            0 (default): as 16 when those 16-bit waves number at least
                            four per compute unit, else as 32 */
  int32_t pad_;          /* must be 0 */
} swx_tuning;
int swx_get_tuning(const swx_ctx *ctx, swx_tuning *out);
int swx_set_tuning(swx_ctx *ctx, const swx_tuning *t);

/* Autotuner: runs the first min(npairs, max_pairs) pairs of b under candidate
 * settings of each knob in turn (fill_rows, long_cells, intra_jobs, side_streams, fill_sched,
 * fill_coop, intra_bits;
 * each timed as the best of two runs after a warm-up, a change kept only if
 * at least 3% faster), installs the fastest in ctx and returns it in *out.
 * cache_path (may be NULL) names a text file of one JSON object per line,
 * keyed by the device architecture and a coarse workload signature (n, gaps,
 * log2 of the sample size and of its cells); a matching entry is installed
 * without timing (*from_cache = 1), a new result is appended.  Errors: those
 * of swx_align_batch; SWX_EINVAL for max_pairs < 1 or null pointers. */
int swx_autotune(swx_ctx *ctx, const swx_batch *b, int64_t max_pairs, const char *cache_path,
                 swx_tuning *out, int32_t *from_cache);

/* ---- graph mode -----------------------------------------------------------------
 * The batched path (forward fill, 32-bit re-run, reversed pass, banded
 * traceback, score2, records) captured once as a hipGraph for batches of a
 * fixed capacity and replayed per batch: no host round trips, no per-call
 * planning on the host.  Every run aligns exactly max_pairs pairs held in the
 * graph's own device buffers (swx_graph_io), which the caller fills before
 * each run (pad unused pair slots with an empty reference: roff[k] ==
 * roff[k+1]).  Requirements on the contents: qlen <= max_qlen, rlen <=
 * max_rlen, offsets non-decreasing within the code arrays, codes in [0, n)
 * over the whole code arrays (create fills them with 0).  Violations of the
 * validated ones are reported by swx_graph_run as SWX_EINVAL; lengths above
 * the capacities are the caller's error.  Every pair takes the route the
 * configuration names.  Results equal swx_align_batch's.
 * Errors: SWX_EINVAL (capacities < 1, flags), SWX_EOVERFLOW (scores could
 * exceed the lanes), SWX_ENOMEM, SWX_EDEVICE. */
typedef struct swx_graph swx_graph;

typedef struct {
  const int8_t *matrix; int32_t n; int32_t gap_open; int32_t gap_extend;   /* copied */
  int64_t max_pairs;
  int32_t max_qlen; int32_t pad_;
  int64_t max_rlen;
  int64_t qcat_cap, rcat_cap;   /* code array sizes */
  int64_t nq_cap, nr_cap;       /* numbers of queries / references (offsets hold cap + 1) */
  uint32_t flags;               /* SWX_BEGIN | SWX_CIGAR | SWX_SCORE2 */
  int32_t mask_len;
  int32_t route;                /* SWX_ROUTE_BATCHED: one pair per 16-bit lane half (best for
                                   many pairs); SWX_ROUTE_INTRA: every pair spread over a wave
                                   (lowest latency for few pairs) */
  int32_t pad2_;
} swx_graph_cfg;
#define SWX_ROUTE_BATCHED 0
#define SWX_ROUTE_INTRA 1

typedef struct {   /* device buffers owned by the graph (valid until swx_graph_destroy) */
  int8_t *qcat; int64_t *qoff; int8_t *rcat; int64_t *roff;   /* inputs, [cap], [cap + 1] */
  int64_t *pair_q, *pair_r;                                   /* inputs, [max_pairs] */
  swx_rec *recs;                                              /* output, [max_pairs] */
  uint32_t *cigar; int64_t cigar_cap;                         /* output CIGAR arena */
} swx_graph_io;

int swx_graph_create(swx_ctx *ctx, const swx_graph_cfg *cfg, swx_graph **out, swx_graph_io *io);
/* One replay on hip_stream (a hipStream_t of the context's device, or NULL for
 * the context's own stream), after the work queued there before; returns when
 * the outputs are ready (waiting for that stream only). */
int swx_graph_run(swx_graph *g, void *hip_stream);
/* The same chain issued kernel by kernel without the graph (for checking). */
int swx_graph_run_eager(swx_graph *g, void *hip_stream);
/* Copies a host-memory batch into the graph's input buffers, padding pair
 * slots past npairs with (query 0, reference nr), an empty reference: needs
 * npairs <= max_pairs, nq <= nq_cap, nr + 1 <= nr_cap, the code arrays
 * within their capacities, offsets non-decreasing within the code arrays,
 * pair indices in range, every pair within max_qlen and max_rlen and every
 * symbol code in [0, n) (SWX_EINVAL otherwise, checked on the host before any
 * copy, so a rejected load leaves the buffers as they were).  Contents written
 * straight into the device
 * buffers (swx_graph_io) are not checked beforehand: the run clamps every
 * index, offset and length into the buffers and capacities (so no kernel
 * leaves them), reports bad offsets, indices and codes afterwards as
 * SWX_EINVAL, and aligns a pair longer than the capacities truncated to
 * them (the caller's error, not reported). */
int swx_graph_load(swx_graph *g, const swx_batch *b);
/* Copies the records of the first npairs pairs, and the CIGAR words they
 * refer to, from the graph's output buffers to host memory (SWX_ERANGE when
 * out->cigar_cap is too small; cigar_used says how many words are needed). */
int swx_graph_read(swx_graph *g, int64_t npairs, swx_batch_out *out);
int swx_graph_destroy(swx_graph *g);

/* ---- serving ------------------------------------------------------------------
 * A request loop for a stream of alignment requests under one scoring scheme
 * (the paper's use in read mappers and search servers: many independent
 * queries against references, results as they complete).
 *   - Queries can be registered once (swx_server_register_query) and stay on
 *     the device for the server's lifetime; requests then name them by id.
 *   - Admission: every request carries an estimate of the device memory its
 *     work takes (sequences, boundary rows, max array, profile and traceback
 *     band); requests leave the queue only while the estimates of the work in
 *     flight stay within mem_budget, long requests within 3/4 of it so that
 *     short ones always find room.  A long request above that share starts
 *     only on an idle device: while one heads the long queue, no new short
 *     batch starts until the work in flight has drained, so it cannot be held
 *     back for good by steady short traffic.
 *   - Continuous batching: each of `workers` worker threads owns a context
 *     (own HIP stream and device pool); a free worker takes every queued
 *     request of one size class that fits (up to max_batch) as one batch, so
 *     requests arriving while batches run join the next batch and batches
 *     overlap on the GPU.  With two or more workers, worker 0 serves only
 *     short requests and the others prefer long ones (qlen * rlen >
 *     long_cells), so short requests do not wait behind long batches.  The
 *     device gives a process few hardware queues (four by default), and
 *     streams beyond that share them, so that a short batch queued behind a
 *     long kernel on a shared queue waits for it: keep workers at four or
 *     fewer, each on a single stream (side_streams off), for short-request
 *     latency.
 *   - Short batches may replay a captured graph on worker 0 (graph_batch);
 *     under a mix with long requests this is slower than the eager batch
 *     path, which is the default.
 *   - A request's result never depends on the batch it ran in.
 * Timestamps are CLOCK_MONOTONIC nanoseconds. */
typedef struct swx_server swx_server;

typedef struct {
  int device;
  const int8_t *matrix; int32_t n; int32_t gap_open; int32_t gap_extend;   /* copied */
  int64_t mem_budget;   /* bytes; <= 0: 4 GiB */
  int32_t max_pending;  /* submit accepts no more requests of a size class while this
                           many of that class wait; <= 0: 2^20 */
  int32_t workers;      /* concurrent batches (1..16); <= 0: 3 */
  int32_t max_batch;    /* requests per batch; <= 0: 65536 */
  uint32_t flags;       /* SWX_BEGIN | SWX_CIGAR | SWX_SCORE2 for every request */
  int32_t mask_len;     /* as for swx_align_batch */
  int64_t long_cells;   /* qlen * rlen above this: long class; <= 0: 2^22 */
  int32_t graph_batch;  /* > 0: worker 0 runs short batches through a captured graph (intra
                           route) of this many requests per replay; 0: eager batches */
  int32_t graph_max_qlen;   /* graph capacities (<= 0: 256 and 1536); requests beyond */
  int64_t graph_max_rlen;   /* them take the eager path */
  int32_t side_streams;     /* workers' side streams (swx_tuning.side_streams); < 0: off when
                               workers > 1, so that every worker holds one stream */
  int32_t pad_;
} swx_server_cfg;

typedef struct {
  int64_t query_id;     /* >= 0: a registered query; < 0: query[qlen] below (copied) */
  const int8_t *query; int32_t qlen;
  const int8_t *ref; int64_t rlen;   /* host codes, copied at submit; rlen may be 0 */
  uint64_t tag;         /* returned unchanged in the completion */
} swx_request;

typedef struct {
  uint64_t ticket, tag;
  int32_t status;       /* SWX_OK or the batch's error */
  int32_t batch_size;   /* requests in the batch this one ran in */
  swx_rec rec;          /* cigar_off is 0: the CIGAR is below */
  uint32_t *cigar;      /* rec.cigar_len words, malloc'd: release with swx_completion_free */
  int64_t t_submit_ns, t_start_ns, t_done_ns;
} swx_completion;

typedef struct {
  int64_t submitted, deferred;     /* requests accepted / refused with SWX_EBUSY */
  int64_t admitted, completed;     /* taken into a batch / finished */
  int64_t batches, max_batch_seen;
  int64_t graph_batches;           /* batches replayed through the captured graph */
  int64_t pending;                 /* waiting now */
  int64_t inflight_bytes, peak_inflight_bytes;
} swx_server_stats;

/* Errors: SWX_EINVAL (nulls, bad scoring, flags), SWX_EDEVICE, SWX_ENOMEM. */
int swx_server_create(const swx_server_cfg *cfg, swx_server **out);
/* Uploads a query once; *query_id names it in later requests.  SWX_EINVAL for
 * qlen < 1 or a symbol >= n. */
int swx_server_register_query(swx_server *s, const int8_t *query, int32_t qlen, int64_t *query_id);
/* Queues nreq requests in order; tickets[k] names request k.  The fields of
 * every request, and the symbols of those that fit the queues, are checked
 * first (SWX_EINVAL: none queued; requests past the fitting prefix are
 * neither checked nor copied).  When a request finds its
 * size class's queue full (max_pending waiting), it and the requests after it
 * are not queued: the first *naccepted are, and SWX_EBUSY is returned (a
 * caller that keeps short requests flowing submits the classes separately). */
int swx_server_submit(swx_server *s, const swx_request *rq, int32_t nreq, uint64_t *tickets,
                      int32_t *naccepted);
/* Moves up to max finished completions into done (waiting up to timeout_us
 * for the first one when none is ready); *ndone says how many. */
int swx_server_poll(swx_server *s, swx_completion *done, int32_t max, int32_t timeout_us,
                    int32_t *ndone);
/* Releases the CIGARs of n completions (their cigar pointers become NULL). */
void swx_completion_free(swx_completion *c, int32_t n);
int swx_server_stats_get(swx_server *s, swx_server_stats *out);
/* Finishes every queued request, then releases the server (completions not
 * polled are dropped). */
int swx_server_destroy(swx_server *s);

/* Discrete-event simulation of the serving policy on a virtual clock, with
 * no device: the arrival schedule is replayed against a modelled GPU on which
 * a batch of k requests holding C query x reference cells takes
 * batch_us + k * request_us + C / cells_per_us microseconds (batches do not
 * slow each other down: the model checks the policy, not performance).
 * Footprints, size classes, admission, the pending-queue limit (an arrival
 * that finds max_pending requests waiting is refused: status SWX_EBUSY) and
 * batch formation are the serving loop's own code.  Events are taken one at
 * a time, a completion before an arrival at the same time, and each is
 * followed by dispatch to the free workers in worker order.  Arrivals must
 * be in non-decreasing time order.  Fills out[k]
 * for every request and *stats (may be NULL).  Errors: SWX_EINVAL for null
 * pointers, n < 0, unsorted arrivals, negative lengths or a non-positive
 * cells_per_us. */
typedef struct {
  double arrival_us;
  int64_t qlen, rlen;
} swx_sim_request;

typedef struct {
  double cells_per_us;  /* modelled cell rate */
  double batch_us;      /* fixed cost of a batch */
  double request_us;    /* cost per request of a batch */
} swx_sim_model;

typedef struct {
  double start_us, done_us;   /* batch start and end (-1 if refused) */
  int64_t batch_id;           /* dispatch order, -1 if refused */
  int64_t footprint;          /* admission estimate, bytes */
  int32_t worker, batch_size; /* -1 / 0 if refused */
  int32_t cls, status;        /* size class (0 short, 1 long); SWX_OK or SWX_EBUSY */
} swx_sim_result;

int swx_server_simulate(const swx_server_cfg *cfg, const swx_sim_model *model,
                        const swx_sim_request *rq, int64_t n, swx_sim_result *out,
                        swx_server_stats *stats);

/* ---- diagnostics ------------------------------------------------------------ */
const char *swx_strerror(int status);
const char *swx_last_error(void);
/* Device time in milliseconds of each stage of the last batch on ctx, in the
 * order: prepare, fill, rerun32, reverse, traceback, score2, records.
 * Returns the number of stages written (at most cap). */
int swx_last_stage_ms(const swx_ctx *ctx, double *ms, int cap);
/* Lane-width probe (method section: narrow saturating lanes).  Runs the fill
 * recurrence -- biased H, E, F with the zero floor and the column max -- over
 * blocks x 256 threads of synthetic pairs (16 query rows x `columns`
 * reference columns each, DNA +2/-2, gap_open/gap_extend <= 60) at `bits`
 * = 8 (four SWAR byte lanes per register: gfx950 has no packed 8-bit add or
 * max) or 16 (two packed 16-bit lanes).  Pair p's query symbol of row r is a
 * hash of p*16 + r, so both widths align the same pairs: best[p] (host
 * array of blocks * 256 * 32/bits words) receives pair p's best score and
 * *ms the kernel time.  Errors: SWX_EINVAL for other widths, sizes < 1,
 * blocks > 2^20 or bad gaps. */
int swx_lane_probe(swx_ctx *ctx, int32_t bits, int64_t columns, int64_t blocks, int32_t gap_open,
                   int32_t gap_extend, uint32_t *best, double *ms);
/* Check of the hardware fact the batched fill's 16-bit lanes rely on (method
 * section: narrow saturating lanes): H, the largest of diagonal + score, E
 * and F, is taken with one packed f16 three-way maximum, which equals the
 * unsigned maximum only while every 16-bit pattern is below 0x7C00.  Runs
 * that operation (the fill's own lane helper) on the device over every pair
 * (a, b) below 0x7C00 with c from a fixed set of 8 values, in both halves,
 * and over 2^31 pseudo-random triples; *mismatches (host) receives the
 * number of results that differ from the unsigned maximum (0 expected) and
 * *checked the number of results compared.  Errors: SWX_EINVAL for null
 * arguments, SWX_EDEVICE on a device failure. */
int swx_check_max3(swx_ctx *ctx, uint64_t *mismatches, uint64_t *checked);

#ifdef __cplusplus
}
#endif
#endif /* SWX_H */
