// swx_internal.h -- structures shared by the HIP kernels and the host runtime.
//
// Coordinates: rows are query positions, columns are reference positions.
// A "pair view" names a (query, reference) pair by start offsets and lengths
// into concatenated code arrays; a reversed view reads both sequences from
// their last symbol backwards, which is how the reversed pass of the method
// section (begin position search) is run without copying sequences.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace swx {

// ---- inter-sequence fill ------------------------------------------------
// One wave (64 lanes) processes one task.  With 16-bit lanes each lane holds
// two pairs (low and high 16-bit halves): slot s -> lane s & 63, half s >> 6.
// With 32-bit lanes each lane holds one pair: slot s -> lane s.
constexpr int kWave = 64;
constexpr int kSlots16 = 128;
constexpr int kSlots32 = 64;

struct InterTask {
  int32_t nslots;     // occupied slots
  int32_t qp;         // padded rows: a multiple of the strip height R, or (no
                      // query profile) of R / 2, the last strip then half high
  int32_t rp;         // padded columns (multiple of 8)
  int32_t band;       // reversed pass: band half-width around the main diagonal (-1: none);
                      // columns j <= i + band of row i
  int32_t band_q;     // reversed pass: columns j >= i - band_q (-1: none; band_q <= band)
  int32_t pad_;
  int64_t slot_base;  // slots are slot_pair[slot_base + s]
  int64_t bnd_off;    // boundary planes at bnd + bnd_off: 3 planes of rp*64 dwords;
                      // packed reference symbols at rsym + rsym_offset(bnd_off)
  int64_t qdata_off;  // QGEN: profile bytes at prof + off
                      //       ((qp/R) strips * (n+1) symbols * halves * 64 lanes * R rows)
};

// Per-pair view of the sequences (indexed by pair id).
struct PairView {
  const int64_t *qstart;   // start of the query in qcat
  const int64_t *rstart;   // start of the reference in rcat
  const int32_t *qlen;
  const int64_t *rlen;
  const int8_t *qcat;
  const int8_t *rcat;
  int32_t reversed;        // read both sequences backwards (reversed pass)
};

// Forward/reversed fill results per pair (indexed by pair id).
struct FillOut {
  int32_t *score;      // best score (score1); saturated values are flagged
  int32_t *qend;       // T1 row (in the view's coordinates)
  int64_t *rend;       // T1 column
  uint8_t *overflow;   // 1 when the lane width saturated: re-run wider
  uint8_t *err;        // set when an internal check fails (may be null)
};

// Boundary plane layout.  Each plane (H of the strip's last row, F below it,
// column max) holds, per group of 4 columns, one 16-byte word per lane:
// dword (c & 3) of word [c / 4][lane].  A wave moves 4 columns of one plane
// with a single coalesced 1 KiB access.
__host__ __device__ inline int64_t bnd_index(int64_t c, int lane) {
  return (((c >> 2) * kWave + lane) << 2) + (c & 3);
}

// Packed reference symbols of a task, [rp/4][64 lanes] of 8 bytes: byte k of
// .x is the symbol of half 0 at column 4*g + k, .y the same for half 1 (the
// padding symbol n outside the pair).  A task's boundary planes take
// 192*rp dwords and its packed symbols 16*rp words, so the symbol offset is
// the plane offset / 12.
__host__ __device__ inline int64_t rsym_offset(int64_t bnd_off) { return bnd_off / 12; }

constexpr uint32_t kQSel = 0;    // n <= 4: per-row byte selectors + per-column LUT
constexpr uint32_t kQGen = 1;    // any n: per-slot biased profile rows in global memory

// Arguments of the inter-sequence fill.
struct InterArgs {
  const InterTask *tasks;
  int64_t ntasks;
  const int64_t *slot_pair;   // slot -> pair id
  PairView view;
  const uint8_t *prof;        // QGEN profile bytes (null: QSEL)
  uint32_t *bnd;              // boundary planes (H, F, CM)
  const uint2 *rsym;          // packed reference symbols
  uint32_t lut[8];            // QSEL: per reference symbol, biased scores of query symbols 0..3
  int32_t n, o, e, bias;
  int32_t rev;                // reversed pass: stop at target, band window, no CM plane
  int32_t clamp;              // scores may exceed the 16-bit value field: saturate the code
  int32_t pair3;              // 16-bit lanes, scores at most kInter16PairLimit: the column
                              // maximum takes two rows per packed three-way maximum
  int32_t code_top;           // row code of the first strip row (strip height - 1)
  const int8_t *dummy;        // readable bytes for empty slots
  const int32_t *target;      // reversed pass: per pair score to reach
  FillOut out;
  int32_t sched;              // task order: 0 grid ascending, 1 grid largest first,
                              // 2 resident waves on a device queue, largest first
  int32_t cus;                // compute units (sched 2 sizes its grid to them)
  unsigned long long *queue;  // sched 2: the queue's counter (zeroed by the launch)
  uint32_t anchor;            // reversed pass on 32-bit lanes: start value of the first cell
                              // (0: a local pass, every border starts from zero)
  int32_t lastcol;            // forward pass on 32-bit lanes: the best counts only the
                              // last column
  const uint8_t *qprof;       // QGEN, every pair of the pass on one query: that query's profile
                              // (null: per-task profile bytes at prof).  Forward: [sym][qp]
                              // biased scores, rows padded at the top as the tasks pad them.
                              // Reversed: 16 copies [c][sym][row], copy c shifted by c bytes,
                              // byte k of a row the biased score of query position qlen-1-k
  int64_t qprof_row;          // bytes per symbol row
  int64_t qprof_copy;         // reversed: bytes per shifted copy
  int32_t qprof_qlen;         // the query's length
  const int64_t *order;       // the tasks by ascending area (padded rows x columns), run from
                              // the end (largest first); null: the plan's order (by height,
                              // then width)
  int32_t coop;               // 1: one wave per task; 4: the four waves of a workgroup share
                              // a task, wave w taking strips w, w + 4, ... (a strip starts on
                              // a column group once the strip above has stored it)
};

// Strips per task that the cooperative mode pipelines (a task with more runs
// on one wave of its workgroup).
constexpr int kCoopMaxStrips = 512;
constexpr int kCoopWaves = 4;

// Largest score the 16-bit inter path represents exactly together with its
// 5-bit row code (value * 32 + code <= 65535).
constexpr int kInter16Limit = 2047;
// Largest score whose encoded form (value * 32 + code <= 0x7BFF) stays below
// 0x7C00, the range where the packed f16 maximum orders 16-bit patterns as
// unsigned integers.
constexpr int kInter16PairLimit = 991;

// ---- intra-sequence fill (long pairs) ------------------------------------
// One wave per job.  Lane k holds rows [k*RL, (k+1)*RL) of a strip of 64*RL
// query rows and computes column c - k at step c (a wavefront over lanes):
// the H and F leaving a lane's last row and the running column max move one
// lane down per step.  Queries taller than a strip take several strips, the
// strip's last row handed over through global memory.  A long reference is
// cut into jobs owning columns [c0, c1); each job starts from zero boundaries
// at cw <= c0, early enough that every positive value in the owned columns is
// exact (no positive-scoring path spans more than Lq + (smax*Lq - o)/e
// columns).
struct IntraJob {
  int64_t pair;      // pair id
  int64_t cw;        // first computed column
  int64_t c0, c1;    // owned columns: max array entries are written for these
  int64_t mc_off;    // forward: the pair's max array at maxcol + mc_off, [rlen] words
  int64_t bnd_off;   // hand-over rows at bnd + bnd_off: per strip boundary, H then F, (c1 - cw) words each
  int32_t kbits;     // row-code bits: max array word = value << kbits | (2^kbits - 1 - row)
  int32_t band;      // reversed pass: drift band half-width (-1: none)
};
// The strips of a job run on the waves of one workgroup (wave w: strips w,
// w + NW, ...), strip s consuming strip s - 1's hand-over row as soon as the
// columns it needs are published.

// Most strips of one intra-sequence job.
constexpr int kIntraMaxStrips = 256;

// Progress of one spread job (its strips on several workgroups), in global
// memory; intra_sync_init sets it before each launch.
struct IntraSync {
  int32_t prog[kIntraMaxStrips];     // columns published by strip s (from its window start)
  int32_t done[kIntraMaxStrips];     // strip s finished (its progress is final)
  int64_t rcol[kIntraMaxStrips];     // reversed pass: first column of strip s reaching the target (-1)
  int32_t rrow[kIntraMaxStrips];     // ... and its row (-1)
  unsigned long long best;           // reversed pass: smallest such column so far (~0: none)
  int32_t fin;                       // segments of the job that have finished
  int32_t pad_;
};

struct IntraArgs {
  const IntraJob *jobs;
  int64_t njobs;
  int32_t segs;              // workgroups per job (0 or 1: one; > 1: a spread launch, sync below)
  IntraSync *sync;           // spread launches: one per job
  PairView view;
  const int8_t *matrix;      // device n x n
  int32_t n, o, e, bias;
  uint32_t *maxcol;          // forward: encoded column maxima
  uint32_t *bnd;             // strip hand-over rows
  const int32_t *target;     // reversed pass: score to reach, per pair
  FillOut out;               // reversed pass: reached score, reversed row and column
  uint8_t *err;              // per pair: set when an internal check fails
};

}  // namespace swx
