// swx_kernels.h -- launchers of the HIP kernels (internal to the library).
#pragma once
#include <hip/hip_runtime.h>

#include "swx_internal.h"

namespace swx {

// device copy of the public swx_rec (same layout)
struct swx_rec_dev {
  int32_t score1, score2;
  int32_t read_begin1, read_end1;
  int64_t ref_begin1, ref_end1, ref_end2;
  int64_t cigar_off;
  int32_t cigar_len;
  int32_t lane_bits;
};

struct PackArgs {            // QGEN profile construction
  const InterTask *tasks;
  int64_t ntasks;
  const int64_t *slot_pair;
  PairView view;
  uint8_t *prof;
  uint2 *rsym;            // packed reference symbols (k_inter_rsym)
  const int8_t *matrix;   // n x n, [query symbol][reference symbol], device
  int32_t n, bias, halves, strip_rows, rev;
};

struct BandArgs {
  int64_t npairs;
  const int32_t *score;
  const int32_t *qbeg, *qend;
  const int64_t *rbeg, *rend;
  const int64_t *qstart, *rstart;   // forward view
  const int32_t *qlen;
  const int64_t *rlen;
  const int8_t *qcat, *rcat;
  const int8_t *matrix;
  int32_t n, o, e, smax;
  uint8_t *dir;            const int64_t *dir_off;
  int32_t *rowbuf;         const int64_t *row_off;   // 2 rows (H, F) of row_cap ints
  uint32_t *cig;           const int64_t *cig_off;   // scratch runs
  int32_t *cig_len;
  uint8_t *err;
  const uint8_t *only;     // when set, only pairs with only[p] == 5 (wide bands)
};

struct Score2InterArgs {
  const InterTask *tasks;
  int64_t ntasks;
  const int64_t *slot_pair;
  const int64_t *rlen;
  const int32_t *qlen;
  const uint32_t *bnd;
  const int32_t *score1;
  const int64_t *rbeg, *rend;
  int32_t mask_len;       // < 0: per pair max(qlen/2, 15)
  int32_t halves;
  int32_t *score2;
  int64_t *rend2;
};

struct ValidateArgs {
  const int8_t *qcat; int64_t qcat_len; const int64_t *qoff; int64_t nq;
  const int8_t *rcat; int64_t rcat_len; const int64_t *roff; int64_t nr;
  const int64_t *pair_q, *pair_r; int64_t npairs;
  int32_t n;
  uint32_t *bad;          // bit flags: 1 offsets, 2 pair index, 4 query symbol, 8 reference symbol
};

// banded traceback
struct TbTask {
  int32_t nslots, rows, bw, pad_;
  int64_t slot_base;
  int64_t dir_off;     // dwords
};

constexpr int kTbwSlots = 16;
constexpr int kTbKeyBits = 23;  // traceback sort key: class (3 bits) above 20 bits of rows   // pairs per wide-band traceback task (four lanes each)

struct TbwTask {        // wide-band traceback task (kTbwSlots pairs)
  int32_t nslots, pad_;
  int64_t rows, wmax, dlo, width;
  int64_t slot_base;
  int64_t dir_off;      // dwords
  int64_t bnd_off;      // ints
};

// Safe band of the banded pass (method section: the band is set by the
// begin and the end).  m x w rectangle, score s1: every path of score s1 has
// at most G = floor((smax*(m+w) - 2o + 2e - 2*s1) / (smax + 2e)) gap symbols,
// so it stays on diagonals j - i in [min(0,D) - hw, max(0,D) + hw] with
// D = w - m and hw = floor((G - |D|) / 2).  Returns the lowest diagonal and
// the number of diagonals.
__host__ __device__ inline int64_t floor_div64(int64_t a, int64_t b) {
  int64_t q = a / b;
  if ((a % b != 0) && ((a < 0) != (b < 0))) --q;
  return q;
}

__host__ __device__ inline void safe_band(int64_t m, int64_t w, int64_t s1, int32_t smax, int32_t o,
                                          int32_t e, int64_t *dlo, int64_t *bw) {
  const int64_t D = w - m;
  const int64_t num = (int64_t)smax * (m + w) - 2 * o + 2 * e - 2 * s1;
  const int64_t den = (int64_t)smax + 2 * e;
  const int64_t G = den > 0 ? floor_div64(num, den) : (m + w);
  const int64_t aD = D < 0 ? -D : D;
  const int64_t hw = (G - aD) >= 0 ? (G - aD) / 2 : 0;
  *dlo = (D < 0 ? D : 0) - hw;
  *bw = ((D > 0 ? D : 0) + hw) - *dlo + 1;
}

// Pairs with more band cells than this take the wave-parallel traceback (one
// pair per workgroup) instead of one pair per lane; in a batch of at most
// kTbFewPairs pairs (less than one wave of lanes) the lower kWaveTbCellsFew.
constexpr int64_t kWaveTbCells = int64_t(1) << 18;
constexpr int64_t kWaveTbCellsFew = int64_t(1) << 14;
constexpr int64_t kTbFewPairs = 64;

// Wave-parallel traceback of one pair: rows in strips of 64 * RL (RL = 4, 8
// or 16 rows per lane), columns swept as a wavefront; choice codes stored per
// (strip, step, lane) as RL nibbles (2, 4 or 8 bytes).
struct TbWaveJob {
  int64_t pair;
  int64_t m, w;          // rectangle: query rows qbeg..qend, reference columns rbeg..rend
  int64_t dlo, bw;       // safe band (diagonals j - i, 1-based coordinates)
  int64_t dir_off;       // bytes: the pair's choice codes start there
  int64_t bnd_off;       // ints of the hand-over rows: per strip boundary (and the
                         // virtual top row) H then F, w + 1 each
};
__host__ __device__ inline int tb_code_bytes(int RL) { return RL / 2; }

// column window [clo, chi) of strip s (rows s*SH+1 .. (s+1)*SH, 1-based;
// column 0 is the virtual column left of the rectangle)
__host__ __device__ inline void tbw_window(int64_t s, int64_t SH, int64_t dlo, int64_t bw,
                                           int64_t w, int64_t *clo, int64_t *chi) {
  int64_t lo = s * SH + 1 + dlo;
  if (lo < 0) lo = 0;
  int64_t hi = (s + 1) * SH + dlo + bw;
  if (hi > w + 1) hi = w + 1;
  *clo = lo;
  *chi = hi > lo ? hi : lo;
}

struct TbArgs {
  const int32_t *score;
  const int32_t *qbeg, *qend;
  const int64_t *rbeg, *rend;
  const int64_t *qstart, *rstart;
  const int32_t *qlen;
  const int64_t *rlen;
  const int8_t *qcat, *rcat;
  const int8_t *matrix;
  int32_t n, o, e, smax;
  uint32_t *dir;
  uint32_t *cig;
  const int64_t *cig_off;
  int32_t *cig_len;
  uint8_t *err;
  int64_t wave_cells;    // wide bands with more cells go to the wave-parallel kernel
};

hipError_t tb_classify(const TbArgs &a, int64_t npairs, uint8_t *cls, uint64_t *key, int64_t *vals,
                       int64_t *ccap, hipStream_t st);
hipError_t tb_tasks(int64_t n0, int64_t n1, const int64_t *sorted, const TbArgs &a, int32_t bw,
                    TbTask *tasks, int64_t *dir_words, hipStream_t st);
hipError_t tb_offsets(int64_t ntasks, TbTask *tasks, const int64_t *off, hipStream_t st);
hipError_t tb_tasks_range(const int64_t *range, int64_t ntasks_cap, const int64_t *sorted,
                          const TbArgs &a, int32_t bw, TbTask *tasks, int64_t *dir_words,
                          hipStream_t st);
hipError_t tbw_tasks_range(const int64_t *range, int64_t ntasks_cap, const int64_t *sorted,
                           const TbArgs &a, TbwTask *tasks, int64_t *dir_words, int64_t *bnd_words,
                           hipStream_t st);
hipError_t tb_band(const TbArgs &a, const TbTask *tasks, int64_t ntasks, const int64_t *sorted,
                   int32_t bw, hipStream_t st);
hipError_t tbw_tasks(int64_t n0, int64_t n1, const int64_t *sorted, const TbArgs &a,
                     TbwTask *tasks, int64_t *dir_words, int64_t *bnd_words, hipStream_t st);
hipError_t tbw_offsets(int64_t ntasks, TbwTask *tasks, const int64_t *doff, const int64_t *boff,
                       hipStream_t st);
hipError_t tb_strip(const TbArgs &a, const TbwTask *tasks, int64_t ntasks, const int64_t *sorted,
                    int32_t *bndbuf, hipStream_t st);
// One-pair graphs: pair 0's wave job planned on the device (m = 0 when it has
// no alignment; its CIGAR scratch offset cig_off[0] = 0), and an upper bound
// of the code bytes of a pair of at most m rows and w columns
hipError_t tb_wave_job1(const TbArgs &a, TbWaveJob *job, int64_t *cig_off, hipStream_t st);
int64_t tb_wave_dir_bytes(int64_t m, int64_t w, int RL);
// segs > 1: each pair's strips spread over that many workgroups (sync: one
// record per pair), then a walk kernel; else the fill and the walk in one
hipError_t tb_wave(const TbArgs &a, const TbWaveJob *jobs, int64_t njobs, int RL, int waves,
                   int segs, IntraSync *sync, uint8_t *dirw, int32_t *bnd, hipStream_t st);
int tb_wave_waves(int64_t m, int n, int RL);   // waves per workgroup for a pair of m rows
int tb_wave_max_strips();
hipError_t fill_u8(int64_t n, uint8_t *p, uint8_t v, hipStream_t st);
hipError_t fill_i64(int64_t n, int64_t *p, int64_t v, hipStream_t st);
// lane-width probe: blocks x 256 threads, each 32/bits synthetic pairs of 16
// rows x cols columns; best[pair] = the pair's best score
// adds to *bad the results of VT<u16x2>::max3 that differ from the unsigned
// maximum over the check's operand set; *checked: the number of lane results
hipError_t max3_check(unsigned long long *bad, uint64_t *checked, hipStream_t st);
hipError_t lane_probe(int bits, int64_t cols, int64_t blocks, int32_t o, int32_t e, uint32_t *best,
                      hipStream_t st);
hipError_t class_ranges(const int64_t *counts, int64_t *ranges, hipStream_t st);
hipError_t count_classes(int64_t n, const uint8_t *cls, int64_t *counts, hipStream_t st);
// graph: the sort is recorded into a HIP graph (a form that issues no memset)
hipError_t sort_keys(int64_t n, uint64_t *keys, uint64_t *keys_alt, int64_t *vals,
                     int64_t *vals_alt, void *tmp, size_t *tmp_bytes, int64_t **sorted_out,
                     hipStream_t st, int end_bit = 64, bool graph = false);
hipError_t rev_prepare(int64_t npairs, const int32_t *score, const int32_t *qend,
                       const int64_t *rend, const uint8_t *lanebits, int32_t smax, int32_t o,
                       int32_t e, int32_t *band, int32_t *band_q, uint8_t *f16, uint8_t *f32,
                       hipStream_t st);

hipError_t inter_fill(const InterArgs &a, int lane_bits, int R, hipStream_t st);
// keys[t] = padded rows x swept columns of task t (a banded task's window of R +
// band_q + band columns per strip) / 256, vals[t] = t (for InterArgs::order; sorted on
// 24 key bits)
hipError_t inter_area_keys(const InterTask *tasks, int64_t ntasks, int32_t R, uint64_t *keys,
                           int64_t *vals, hipStream_t st);

// intra-sequence path (long pairs)
struct IntraPair {         // one long pair's forward max array
  int64_t pair;
  int64_t mc_off;          // words at maxcol + mc_off, [rlen]
  int32_t kbits;           // row-code bits
  int32_t sh;              // strip height of its forward jobs (padding rows = roundup(qlen, sh) - qlen)
};
struct IntraPairArgs {
  const IntraPair *pairs;
  const uint32_t *maxcol;
  const int32_t *qlen;
  const int64_t *rlen;
  int32_t *score;          // score1 (written by the end kernel, read by score2)
  int32_t *qend;
  int64_t *rend;
  uint8_t *overflow;
  const int64_t *rbeg;     // score2: begin of the primary alignment
  int32_t mask_len;
  int32_t *score2;
  int64_t *rend2;
  int32_t *part_v;         // per (pair, slice) partial bests: intra_slices() per pair
  int64_t *part_j;
};
size_t intra_lds_bytes(int n, int RL);
int intra_slices();
hipError_t intra_fill(const IntraArgs &a, int RL, int waves, bool rev, hipStream_t st);
// sets the progress records of a spread launch's jobs (before each launch)
hipError_t intra_sync_init(IntraSync *sync, int64_t njobs, hipStream_t st);
// forward pass on packed 16-bit lanes: jobs[2b] and jobs[2b + 1] (same padded
// height; pair -1: none) share workgroup b; a.njobs even
// m3: every pair's score bound plus bias is below 0x7C00 (one packed
// three-way maximum per row instead of two maxima)
hipError_t intra_fill16(const IntraArgs &a, int RL, int waves, bool m3, hipStream_t st);
size_t intra_lds_bytes16(int n, int RL);
int intra_max_strips();
int intra_max_waves();
hipError_t intra_jobs_chunked(int64_t B, int32_t nc, int64_t cw, const int32_t *qlen,
                              const int64_t *rlen, int32_t smax, int32_t o, int32_t e,
                              int32_t kbits, int32_t sh, int64_t mc_stride, int64_t bnd_stride,
                              IntraJob *jobs, IntraPair *pairs, hipStream_t st);
hipError_t intra_rev_jobs_fixed(int64_t B, const int32_t *score, const int64_t *rend,
                                const int32_t *band, int32_t kbits, int64_t bnd_stride,
                                IntraJob *jobs, hipStream_t st);
size_t intra_static_lds();
hipError_t intra_end(const IntraPairArgs &a, int64_t npairs, hipStream_t st);
hipError_t intra_score2(const IntraPairArgs &a, int64_t npairs, hipStream_t st);
hipError_t split_long(int64_t n, const int32_t *qlen, const int64_t *rlen, int64_t cells_thr,
                      int64_t rlen_thr, uint8_t *is_long, uint8_t *is_short, hipStream_t st);
hipError_t gather_pairs(int64_t n, const int64_t *ids, const int32_t *qlen, const int64_t *rlen,
                        const int32_t *score, const int32_t *qend, const int64_t *rend,
                        const int32_t *band, int64_t *out, hipStream_t st);
hipError_t clear_flags(int64_t n, const int64_t *ids, uint8_t *f1, uint8_t *f2, hipStream_t st);
hipError_t inter_pack(const PackArgs &a, hipStream_t st);
hipError_t inter_pack_ref(const PackArgs &a, hipStream_t st);

hipError_t launch_validate(const ValidateArgs &a, hipStream_t st);
// the shared query profile of a pass whose pairs all use one query (k_build_qprof)
hipError_t build_qprof(const int8_t *q, int32_t qlen, const int8_t *matrix, int32_t n, int32_t bias,
                       int32_t qp, uint8_t *fwd, int64_t rev_row, uint8_t *rev, hipStream_t st);
// bytes of a reversed row of the shared profile for strips of R rows
inline int64_t qprof_rev_row(int64_t qlen, int R) { return (2 * qlen + 2 * R + 16 + 15) / 16 * 16; }
hipError_t launch_pair_stats(int64_t n, const int32_t *qlen, const int64_t *rlen, int64_t *stats,
                             hipStream_t st);
hipError_t lens_to_i64(int64_t n, const int32_t *len, int64_t *out, hipStream_t st);
hipError_t mark_lanes(int64_t n, const int64_t *ids, uint8_t *lanebits, int v, hipStream_t st);
hipError_t mark_lanes_dev(int64_t cap, const int64_t *n_dev, const int64_t *ids, uint8_t *lanebits,
                          int v, hipStream_t st);
hipError_t launch_any_flag(int64_t n, const uint8_t *flag, int64_t *count, hipStream_t st);
// bounds the views are clamped into (see k_views)
struct ViewCaps {
  int64_t nq, nr, qcat_len, rcat_len;
  int32_t max_qlen, pad_;
  int64_t max_rlen;
};
hipError_t launch_views(int64_t npairs, const int64_t *qoff, const int64_t *roff,
                        const int64_t *pair_q, const int64_t *pair_r, const ViewCaps &caps,
                        int64_t *qstart, int32_t *qlen, int64_t *rstart, int64_t *rlen,
                        hipStream_t st);
hipError_t launch_rev_views(int64_t npairs, const int64_t *qstart, const int64_t *rstart,
                            const int32_t *qlen, const int64_t *rlen,
                            const int32_t *score, const int32_t *qend, const int64_t *rend,
                            int64_t *rqstart, int32_t *rqlen, int64_t *rrstart, int64_t *rrlen,
                            int32_t *target, uint8_t *err, hipStream_t st);
hipError_t launch_band_sizes(int64_t npairs, const int32_t *score, const int32_t *qbeg,
                             const int32_t *qend, const int64_t *rbeg, const int64_t *rend,
                             const int32_t *qlen, const int64_t *rlen, const uint8_t *only,
                             int32_t smax, int32_t o, int32_t e, int64_t *dir_size,
                             int64_t *cig_cap, int64_t *row_cap, hipStream_t st);
hipError_t launch_band_tb(const BandArgs &a, hipStream_t st);
// one launch for many clears: entry k sets n[k] elements of size[k] bytes
// (1, 4 or 8) at p[k] to v[k]
constexpr int kFillSetMax = 12;
struct FillSet {
  void *p[kFillSetMax];
  int64_t n[kFillSetMax];
  int64_t v[kFillSetMax];
  int32_t size[kFillSetMax];
  int32_t count;
  void add(void *ptr, int64_t count_, int32_t bytes, int64_t value) {
    p[count] = ptr; n[count] = count_; size[count] = bytes; v[count] = value; ++count;
  }
};
hipError_t fill_set(const FillSet &f, hipStream_t st);
// pair 0's CIGAR words and final offsets {0, length} (one-pair calls)
hipError_t cigar_one(const uint32_t *src, const int64_t *src_off, const int32_t *len,
                     int64_t *dst_off, uint32_t *dst, hipStream_t st);
hipError_t launch_cigar_compact(int64_t npairs, const uint32_t *src, const int64_t *src_off,
                                const int32_t *len, const int64_t *dst_off, uint32_t *dst,
                                hipStream_t st);
hipError_t launch_score2_inter(const Score2InterArgs &a, hipStream_t st);
hipError_t launch_score2_plain(int64_t p, const int32_t *maxcol, int64_t lr, const int32_t *score1,
                               const int64_t *rbeg, const int64_t *rend, int32_t mask_len,
                               const int32_t *qlen, int32_t *score2, int64_t *rend2,
                               hipStream_t st);
hipError_t launch_records(int64_t npairs, const int32_t *score1, const int32_t *score2,
                          const int32_t *qbeg, const int32_t *qend, const int64_t *rbeg,
                          const int64_t *rend, const int64_t *rend2, const int64_t *cig_off,
                          const int32_t *cig_len, const uint8_t *lane_bits, uint32_t flags,
                          swx_rec_dev *recs, hipStream_t st);
// the suboptimal alignment: window views, anchored reversed views, begins,
// and CIGAR offsets of records counted from the arena's start
hipError_t launch_sub_window(int64_t npairs, const int64_t *rstart, const int32_t *qlen,
                             const int32_t *score2, const int64_t *rend2, int32_t smax, int32_t o,
                             int32_t e, int64_t *wrstart, int64_t *wrlen, uint8_t *flag,
                             hipStream_t st);
hipError_t launch_sub_rev_views(int64_t npairs, const int64_t *qstart, const int64_t *rstart,
                                const int32_t *qlen, const int32_t *score2, const int64_t *rend2,
                                const int32_t *wscore, const int32_t *wqend, uint32_t anchor,
                                int64_t *rqstart, int32_t *rqlen, int64_t *rrstart, int64_t *rrlen,
                                int32_t *target, uint8_t *flag, uint8_t *err, hipStream_t st);
hipError_t launch_sub_begins(int64_t npairs, const int32_t *score2, const int64_t *rend2,
                             const int32_t *wqend, const uint8_t *flag, const int32_t *target,
                             const int32_t *rscore, const int32_t *rqend, const int64_t *rrend,
                             int32_t *sscore, int32_t *sqbeg, int32_t *sqend, int64_t *srbeg,
                             int64_t *srend, uint8_t *err, hipStream_t st);
hipError_t shift_cigar_offsets(int64_t npairs, int64_t base, swx_rec_dev *recs, hipStream_t st);
hipError_t launch_begins(int64_t npairs, const int32_t *score1, const int32_t *qend,
                         const int64_t *rend, const int32_t *rscore, const int32_t *rqend,
                         const int64_t *rrend, int32_t *qbeg, int64_t *rbeg, uint8_t *err,
                         hipStream_t st);
hipError_t plan_sort(int64_t n, const int64_t *n_dev, const int64_t *ids, const int32_t *qlen, const int64_t *rlen,
                     const int32_t *band, int32_t R, uint64_t *keys, uint64_t *keys_alt,
                     int64_t *vals, int64_t *vals_alt, void *tmp, size_t *tmp_bytes,
                     int64_t **sorted_out, hipStream_t st, bool graph = false);
hipError_t plan_tasks_dev(int64_t n, const int64_t *n_dev, int64_t ntasks, int32_t slots, int32_t R,
                          int64_t qdata_per_row, const int64_t *sorted, const int32_t *qlen,
                          const int64_t *rlen, const int32_t *band, const int32_t *band_q,
                          InterTask *tasks, int64_t *bnd_size, int64_t *qdata_size,
                          hipStream_t st);
hipError_t plan_offsets_dev(int64_t ntasks, InterTask *tasks, const int64_t *bnd_off,
                            const int64_t *qdata_off, hipStream_t st);
// f64[0 .. n) = flag != 0, f64[n] = 0 (n + 1 values, ready for an exclusive scan)
hipError_t flags_to_i64(int64_t n, const uint8_t *flag, int64_t *f64, hipStream_t st);
hipError_t compact_flags(int64_t n, const uint8_t *flag, const int64_t *pos, int64_t *out,
                         hipStream_t st);
hipError_t launch_exclusive_scan(const int64_t *in, int64_t *out, int64_t n, void *tmp,
                                 size_t *tmp_bytes, hipStream_t st);

}  // namespace swx
