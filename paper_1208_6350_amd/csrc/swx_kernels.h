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

struct PackArgs {
  const InterTask *tasks;
  int64_t ntasks;
  const int64_t *slot_pair;
  PairView view;
  uint4 *rsym;
  uint32_t *qsel;
  uint8_t *prof;
  const int8_t *matrix;   // n x n, [query symbol][reference symbol], device
  int32_t n, bias, halves, strip_rows, mode, rev;
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

hipError_t inter_fill(const InterArgs &a, int lane_bits, int R, hipStream_t st);
hipError_t inter_pack(const PackArgs &a, hipStream_t st);

hipError_t launch_validate(const ValidateArgs &a, hipStream_t st);
hipError_t launch_views(int64_t npairs, const int64_t *qoff, const int64_t *roff,
                        const int64_t *pair_q, const int64_t *pair_r, int64_t *qstart,
                        int32_t *qlen, int64_t *rstart, int64_t *rlen, hipStream_t st);
hipError_t launch_rev_views(int64_t npairs, const int64_t *qstart, const int64_t *rstart,
                            const int32_t *qlen, const int64_t *rlen,
                            const int32_t *score, const int32_t *qend, const int64_t *rend,
                            int64_t *rqstart, int32_t *rqlen, int64_t *rrstart, int64_t *rrlen,
                            int32_t *target, uint8_t *err, hipStream_t st);
hipError_t launch_band_sizes(int64_t npairs, const int32_t *score, const int32_t *qbeg,
                             const int32_t *qend, const int64_t *rbeg, const int64_t *rend,
                             const int32_t *qlen, const int64_t *rlen, int32_t smax, int32_t o, int32_t e, int64_t *dir_size,
                             int64_t *cig_cap, int64_t *row_cap, hipStream_t st);
hipError_t launch_band_tb(const BandArgs &a, hipStream_t st);
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
hipError_t launch_begins(int64_t npairs, const int32_t *score1, const int32_t *qend,
                         const int64_t *rend, const int32_t *rscore, const int32_t *rqend,
                         const int64_t *rrend, int32_t *qbeg, int64_t *rbeg, uint8_t *err,
                         hipStream_t st);
hipError_t launch_exclusive_scan(const int64_t *in, int64_t *out, int64_t n, void *tmp,
                                 size_t *tmp_bytes, hipStream_t st);

}  // namespace swx
