// swx_internal.h -- structures shared by the HIP kernels and the host runtime.
//
// Coordinates: rows are query positions, columns are reference positions.
// A "pair view" names a (query, reference) pair by start offsets and lengths
// into concatenated code arrays; a reversed view reads both sequences from
// their last symbol backwards, which is how the reversed pass of the method
// section (begin position search) is run without copying sequences.
#pragma once
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
  int32_t qp;         // padded rows (multiple of the strip height)
  int32_t rp;         // padded columns (multiple of 8)
  int32_t band;       // reversed pass: band half-width around the main diagonal (-1: none)
  int64_t slot_base;  // slots are slot_pair[slot_base + s]
  int64_t bnd_off;    // boundary planes at bnd + bnd_off: 3 planes of rp*64 dwords
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
};

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
  uint32_t lut[8];            // QSEL: per reference symbol, biased scores of query symbols 0..3
  int32_t n, o, e, bias;
  int32_t rev;                // reversed pass: stop at target, band window, no CM plane
  int32_t clamp;              // scores may exceed the 16-bit value field: saturate the code
  int32_t code_top;           // row code of the first strip row (strip height - 1)
  const int8_t *dummy;        // readable bytes for empty slots
  const int32_t *target;      // reversed pass: per pair score to reach
  FillOut out;
};

// Largest score the 16-bit inter path represents exactly together with its
// 5-bit row code (value * 32 + code <= 65535).
constexpr int kInter16Limit = 2047;

// ---- intra-sequence fill (long references) -------------------------------
// One wave per job; a job is one or two column chunks of one pair (two with
// 16-bit lanes: low half = chunk A, high half = chunk B).  Lanes hold R rows
// each; a pass covers 64*R rows; longer queries take several passes with the
// bottom row handed over through global memory.
struct IntraJob {
  int64_t pair;        // pair id
  int64_t c0[2];       // first computed column of each chunk (-1: unused half)
  int64_t own0[2];     // first owned column (maxcol written from here)
  int64_t c1[2];       // one past the last column
  int64_t mc_base;     // maxcol array of the pair: mc + mc_base (int32 per column)
  int64_t hand_off;    // pass hand-over buffer (3 planes of ncols_max dwords), or -1
  int32_t target;      // reversed pass: stop once this score is reached (0: none)
  int32_t pad_;
};

struct IntraBest {      // per job and half: lexicographic best (score, -col, -row)
  int32_t score;
  int32_t row;
  int64_t col;
};

}  // namespace swx
