// runtime.cpp -- host side of the library: contexts, validation, planning of
// the inter-sequence tasks, and the alignment pipeline
//   forward fill -> 32-bit re-run of saturated pairs -> reversed pass (begin)
//   -> banded traceback (CIGAR) -> masked max array (score2) -> records,
// following the order of the paper's method section.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <numeric>
#include <string>
#include <vector>

#include "../../include/swx.h"
#include "swx_internal.h"
#include "swx_kernels.h"

namespace swx {

static thread_local std::string g_last_error;

static int fail(int code, const std::string &msg) {
  g_last_error = msg;
  return code;
}

#define HIP_TRY(expr)                                                                \
  do {                                                                               \
    hipError_t _e = (expr);                                                          \
    if (_e != hipSuccess)                                                            \
      return fail(SWX_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(_e));   \
  } while (0)

// ---- device memory pool ---------------------------------------------------
// Bump allocation from large blocks that are kept across calls; reset() makes
// the whole pool reusable.  Calls on one context are serialised, so a reset at
// the start of a call cannot free memory that a running call still uses.
class DevArena {
 public:
  ~DevArena() { release(); }
  void reset() {
    cur_ = 0;
    off_ = 0;
  }
  void release() {
    for (auto &b : blocks_) (void)hipFree(b.ptr);
    blocks_.clear();
    cur_ = 0;
    off_ = 0;
  }
  // returns nullptr on failure
  void *alloc(size_t bytes) {
    bytes = (bytes + 255) & ~size_t(255);
    if (bytes == 0) bytes = 256;
    while (cur_ < blocks_.size()) {
      Block &b = blocks_[cur_];
      if (off_ + bytes <= b.size) {
        void *p = (char *)b.ptr + off_;
        off_ += bytes;
        return p;
      }
      ++cur_;
      off_ = 0;
    }
    size_t sz = std::max(bytes, size_t(64) << 20);
    void *p = nullptr;
    if (hipMalloc(&p, sz) != hipSuccess) return nullptr;
    blocks_.push_back({p, sz});
    cur_ = blocks_.size() - 1;
    off_ = bytes;
    return p;
  }
  template <class T>
  T *get(int64_t count) {
    return (T *)alloc(sizeof(T) * (size_t)std::max<int64_t>(count, 1));
  }

 private:
  struct Block {
    void *ptr;
    size_t size;
  };
  std::vector<Block> blocks_;
  size_t cur_ = 0, off_ = 0;
};

}  // namespace swx

struct swx_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  swx::DevArena arena;
  std::mutex mu;
  hipEvent_t ev[8] = {};
  double stage_ms[8] = {};
  int nstages = 0;
};

struct swx_profile {
  swx_ctx *ctx = nullptr;
  std::vector<int8_t> query;
  std::vector<int8_t> matrix;
  int32_t n = 0, o = 0, e = 0;
};

namespace swx {

struct Scoring {
  int32_t n, o, e, bias, smax;
  const int8_t *dmat;       // device copy
  uint32_t lut[8];
  bool qsel;
};

static int make_scoring(const int8_t *mat, int32_t n, int32_t o, int32_t e, Scoring *sc) {
  if (!mat) return fail(SWX_EINVAL, "matrix is null");
  if (n < 1 || n > 32) return fail(SWX_EINVAL, "alphabet size n must be in [1, 32]");
  if (e < 0 || o < e) return fail(SWX_EINVAL, "gaps must satisfy gap_open >= gap_extend >= 0");
  if (o > 32767) return fail(SWX_EINVAL, "gap_open must be <= 32767");
  int mn = 127, mx = -128;
  for (int k = 0; k < n * n; ++k) {
    mn = std::min<int>(mn, mat[k]);
    mx = std::max<int>(mx, mat[k]);
  }
  sc->n = n;
  sc->o = o;
  sc->e = e;
  sc->bias = mn < 0 ? -mn : 0;
  sc->smax = mx;
  sc->qsel = (n <= 4);
  // QSEL column LUTs: lut[r] holds, for query symbols a = 0..3, the biased
  // score S(a, r) + bias in byte a; lut[pad] = 0 (pad scores -bias <= 0).
  for (int r = 0; r < 8; ++r) sc->lut[r] = 0;
  if (sc->qsel) {
    for (int r = 0; r < n; ++r) {
      uint32_t w = 0;
      for (int a = 0; a < n; ++a) w |= (uint32_t)(uint8_t)(mat[a * n + r] + sc->bias) << (8 * a);
      sc->lut[r] = w;
    }
  }
  return SWX_OK;
}

// ---- planning of inter-sequence tasks --------------------------------------
struct Plan {
  std::vector<InterTask> tasks;
  std::vector<int64_t> slot_pair;
  int64_t bnd_words = 0, sym_vecs = 0, qdata = 0;   // buffer sizes
  InterTask *d_tasks = nullptr;
  int64_t *d_slot_pair = nullptr;
  uint32_t *d_bnd = nullptr;
  uint4 *d_rsym = nullptr;
  uint32_t *d_qsel = nullptr;
  uint8_t *d_prof = nullptr;
  int lane_bits = 16, R = 32;
};

static inline int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

// ids: pairs of this pass; qlen/rlen/band indexed by pair id (band may be null)
static void plan_tasks(Plan &pl, const std::vector<int64_t> &ids, const int32_t *qlen,
                       const int64_t *rlen, const int32_t *band, int lane_bits, int R, int n,
                       bool qsel) {
  pl.lane_bits = lane_bits;
  pl.R = R;
  const int slots = lane_bits == 16 ? kSlots16 : kSlots32;
  const int halves = lane_bits == 16 ? 2 : 1;
  std::vector<int64_t> ord(ids);
  std::sort(ord.begin(), ord.end(), [&](int64_t a, int64_t b) {
    const int32_t ba = band ? band[a] : 0, bb = band ? band[b] : 0;
    if (ba != bb) return ba < bb;
    const int64_t qa = round_up(std::max(qlen[a], 1), R), qb = round_up(std::max(qlen[b], 1), R);
    if (qa != qb) return qa < qb;
    if (rlen[a] != rlen[b]) return rlen[a] < rlen[b];
    return a < b;
  });
  pl.tasks.clear();
  pl.slot_pair.clear();
  pl.bnd_words = pl.sym_vecs = pl.qdata = 0;
  for (size_t s0 = 0; s0 < ord.size(); s0 += slots) {
    const size_t s1 = std::min(ord.size(), s0 + slots);
    InterTask t{};
    t.nslots = (int32_t)(s1 - s0);
    int32_t mq = 1;
    int64_t mr = 1;
    int32_t mb = band ? 0 : -1;
    for (size_t k = s0; k < s1; ++k) {
      mq = std::max(mq, qlen[ord[k]]);
      mr = std::max(mr, rlen[ord[k]]);
      if (band) mb = (band[ord[k]] < 0 || mb < 0) ? -1 : std::max(mb, band[ord[k]]);
    }
    t.qp = (int32_t)round_up(mq, R);
    t.rp = (int32_t)round_up(mr, 8);
    t.band = mb;
    t.slot_base = (int64_t)pl.slot_pair.size();
    for (size_t k = s0; k < s1; ++k) pl.slot_pair.push_back(ord[k]);
    t.bnd_off = pl.bnd_words;
    pl.bnd_words += 3 * (int64_t)t.rp * 64;
    t.sym_off = pl.sym_vecs;
    pl.sym_vecs += (int64_t)(t.rp / 8) * 64;
    t.qdata_off = pl.qdata;
    if (qsel) pl.qdata += (int64_t)t.qp * 64;
    else pl.qdata += round_up((int64_t)t.qp * (n + 1) * halves * 64, 16);
    pl.tasks.push_back(t);
  }
}

static int upload_plan(swx_ctx *ctx, Plan &pl, bool qsel) {
  DevArena &A = ctx->arena;
  const int64_t nt = (int64_t)pl.tasks.size();
  pl.d_tasks = A.get<InterTask>(nt);
  pl.d_slot_pair = A.get<int64_t>((int64_t)pl.slot_pair.size());
  pl.d_bnd = A.get<uint32_t>(pl.bnd_words);
  pl.d_rsym = A.get<uint4>(pl.sym_vecs);
  if (qsel) {
    pl.d_qsel = A.get<uint32_t>(pl.qdata);
    pl.d_prof = nullptr;
  } else {
    pl.d_prof = A.get<uint8_t>(pl.qdata);
    pl.d_qsel = nullptr;
  }
  if (!pl.d_tasks || !pl.d_slot_pair || !pl.d_bnd || !pl.d_rsym || (!pl.d_qsel && !pl.d_prof))
    return fail(SWX_ENOMEM, "device pool exhausted while planning");
  if (nt) {
    HIP_TRY(hipMemcpyAsync(pl.d_tasks, pl.tasks.data(), sizeof(InterTask) * nt,
                           hipMemcpyHostToDevice, ctx->stream));
    HIP_TRY(hipMemcpyAsync(pl.d_slot_pair, pl.slot_pair.data(),
                           sizeof(int64_t) * pl.slot_pair.size(), hipMemcpyHostToDevice,
                           ctx->stream));
  }
  return SWX_OK;
}

// pack + fill for one plan
static int run_fill(swx_ctx *ctx, Plan &pl, const Scoring &sc, const PairView &view, bool rev,
                    const int32_t *d_target, FillOut out) {
  if (pl.tasks.empty()) return SWX_OK;
  int rc = upload_plan(ctx, pl, sc.qsel);
  if (rc) return rc;
  PackArgs pk{};
  pk.tasks = pl.d_tasks;
  pk.ntasks = (int64_t)pl.tasks.size();
  pk.slot_pair = pl.d_slot_pair;
  pk.view = view;
  pk.rsym = pl.d_rsym;
  pk.qsel = pl.d_qsel;
  pk.prof = pl.d_prof;
  pk.matrix = sc.dmat;
  pk.n = sc.n;
  pk.bias = sc.bias;
  pk.halves = pl.lane_bits == 16 ? 2 : 1;
  pk.strip_rows = pl.R;
  pk.mode = sc.qsel ? (int)kQSel : (int)kQGen;
  pk.rev = rev ? 1 : 0;
  HIP_TRY(inter_pack(pk, ctx->stream));
  InterArgs a{};
  a.tasks = pl.d_tasks;
  a.ntasks = (int64_t)pl.tasks.size();
  a.slot_pair = pl.d_slot_pair;
  a.view = view;
  a.rsym = pl.d_rsym;
  a.qsel = pl.d_qsel;
  a.prof = pl.d_prof;
  a.bnd = pl.d_bnd;
  for (int k = 0; k < 8; ++k) a.lut[k] = sc.lut[k];
  a.n = sc.n;
  a.o = sc.o;
  a.e = sc.e;
  a.bias = sc.bias;
  a.rev = rev ? 1 : 0;
  a.target = d_target;
  a.out = out;
  HIP_TRY(inter_fill(a, pl.lane_bits, pl.R, ctx->stream));
  return SWX_OK;
}

template <class T>
static int d2h(swx_ctx *ctx, std::vector<T> &dst, const T *src, int64_t n) {
  dst.resize((size_t)n);
  if (n) HIP_TRY(hipMemcpyAsync(dst.data(), src, sizeof(T) * n, hipMemcpyDeviceToHost, ctx->stream));
  return SWX_OK;
}

static int scan(swx_ctx *ctx, const int64_t *in, int64_t *out, int64_t n) {
  if (n == 0) return SWX_OK;
  size_t tmp = 0;
  HIP_TRY(launch_exclusive_scan(in, out, n, nullptr, &tmp, ctx->stream));
  void *t = ctx->arena.alloc(tmp);
  if (!t) return fail(SWX_ENOMEM, "device pool exhausted (scan)");
  HIP_TRY(launch_exclusive_scan(in, out, n, t, &tmp, ctx->stream));
  return SWX_OK;
}

// ---- the pipeline -----------------------------------------------------------
struct DeviceBatch {
  const int8_t *qcat, *rcat;
  const int64_t *qoff, *roff, *pair_q, *pair_r;
  int64_t qcat_len, rcat_len, nq, nr, npairs;
};

static int run_pipeline(swx_ctx *ctx, const Scoring &sc, const DeviceBatch &b, uint32_t flags,
                        int32_t mask_len, swx_batch_out *out) {
  DevArena &A = ctx->arena;
  hipStream_t st = ctx->stream;
  const int64_t np = b.npairs;
  if (flags & (SWX_CIGAR | SWX_SCORE2)) flags |= SWX_BEGIN;
  int stage = 0;
  auto mark = [&](int k) -> int {
    HIP_TRY(hipEventRecord(ctx->ev[k], st));
    stage = k;
    return SWX_OK;
  };
  int rc = mark(0);
  if (rc) return rc;

  // validation
  uint32_t *d_bad = A.get<uint32_t>(1);
  if (!d_bad) return fail(SWX_ENOMEM, "device pool exhausted");
  HIP_TRY(hipMemsetAsync(d_bad, 0, sizeof(uint32_t), st));
  ValidateArgs va{b.qcat, b.qcat_len, b.qoff, b.nq, b.rcat, b.rcat_len, b.roff, b.nr,
                  b.pair_q, b.pair_r, np, sc.n, d_bad};
  HIP_TRY(launch_validate(va, st));
  uint32_t bad = 0;
  HIP_TRY(hipMemcpyAsync(&bad, d_bad, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  if (bad & 1u) return fail(SWX_EINVAL, "offsets must be non-decreasing and within the code arrays");
  if (bad & 2u) return fail(SWX_EINVAL, "pair index out of range");
  if (bad & 12u) return fail(SWX_EINVAL, "symbol code outside [0, n)");

  // per-pair arrays
  int64_t *qstart = A.get<int64_t>(np), *rstart = A.get<int64_t>(np), *rlen = A.get<int64_t>(np);
  int32_t *qlen = A.get<int32_t>(np);
  int32_t *score = A.get<int32_t>(np), *qend = A.get<int32_t>(np);
  int64_t *rend = A.get<int64_t>(np);
  uint8_t *ovf = A.get<uint8_t>(np), *lanebits = A.get<uint8_t>(np), *err = A.get<uint8_t>(np);
  int32_t *qbeg = A.get<int32_t>(np), *score2 = A.get<int32_t>(np);
  int64_t *rbeg = A.get<int64_t>(np), *rend2 = A.get<int64_t>(np);
  if (!qstart || !rstart || !rlen || !qlen || !score || !qend || !rend || !ovf || !lanebits ||
      !err || !qbeg || !score2 || !rbeg || !rend2)
    return fail(SWX_ENOMEM, "device pool exhausted (pair arrays)");
  HIP_TRY(hipMemsetAsync(err, 0, np, st));
  HIP_TRY(hipMemsetAsync(lanebits, 16, np, st));
  HIP_TRY(launch_views(np, b.qoff, b.roff, b.pair_q, b.pair_r, qstart, qlen, rstart, rlen, st));
  std::vector<int32_t> hqlen;
  std::vector<int64_t> hrlen;
  if ((rc = d2h(ctx, hqlen, qlen, np))) return rc;
  if ((rc = d2h(ctx, hrlen, rlen, np))) return rc;
  HIP_TRY(hipStreamSynchronize(st));
  // a score can reach smax * min(qlen, rlen); the 32-bit lanes hold < 2^26
  for (int64_t p = 0; p < np; ++p) {
    if ((int64_t)std::max(sc.smax, 0) * std::min<int64_t>(hqlen[p], hrlen[p]) >= (1 << 26) - 1)
      return fail(SWX_EOVERFLOW, "a score could exceed the 32-bit lane range");
  }
  PairView fview{qstart, rstart, qlen, rlen, b.qcat, b.rcat, 0};
  FillOut fout{score, qend, rend, ovf};
  if ((rc = mark(1))) return rc;

  // forward fill, 16-bit lanes
  std::vector<int64_t> all(np);
  std::iota(all.begin(), all.end(), 0);
  const int R = 32;
  Plan p16;
  plan_tasks(p16, all, hqlen.data(), hrlen.data(), nullptr, 16, R, sc.n, sc.qsel);
  if ((rc = run_fill(ctx, p16, sc, fview, false, nullptr, fout))) return rc;
  if ((rc = mark(2))) return rc;

  // saturated pairs: exact re-run on 32-bit lanes
  std::vector<uint8_t> hovf;
  if ((rc = d2h(ctx, hovf, ovf, np))) return rc;
  HIP_TRY(hipStreamSynchronize(st));
  std::vector<int64_t> wide;
  for (int64_t p = 0; p < np; ++p)
    if (hovf[p]) wide.push_back(p);
  Plan p32;
  std::vector<uint8_t> is32(np, 0);
  if (!wide.empty()) {
    plan_tasks(p32, wide, hqlen.data(), hrlen.data(), nullptr, 32, R, sc.n, sc.qsel);
    if ((rc = run_fill(ctx, p32, sc, fview, false, nullptr, fout))) return rc;
    for (int64_t p : wide) is32[p] = 1;
    uint8_t *d32 = A.get<uint8_t>(np);
    if (!d32) return fail(SWX_ENOMEM, "device pool exhausted");
    std::vector<uint8_t> lb(np);
    for (int64_t p = 0; p < np; ++p) lb[p] = is32[p] ? 32 : 16;
    HIP_TRY(hipMemcpyAsync(lanebits, lb.data(), np, hipMemcpyHostToDevice, st));
    HIP_TRY(hipStreamSynchronize(st));
  }
  if ((rc = mark(3))) return rc;

  // reversed pass: begin
  if (flags & SWX_BEGIN) {
    int64_t *rqs = A.get<int64_t>(np), *rrs = A.get<int64_t>(np), *rrl = A.get<int64_t>(np);
    int32_t *rql = A.get<int32_t>(np), *tgt = A.get<int32_t>(np);
    int32_t *rsc = A.get<int32_t>(np), *rqe = A.get<int32_t>(np);
    int64_t *rre = A.get<int64_t>(np);
    uint8_t *rov = A.get<uint8_t>(np);
    if (!rqs || !rrs || !rrl || !rql || !tgt || !rsc || !rqe || !rre || !rov)
      return fail(SWX_ENOMEM, "device pool exhausted (reverse)");
    HIP_TRY(launch_rev_views(np, qstart, rstart, qlen, rlen, score, qend, rend, rqs, rql, rrs,
                             rrl, tgt, err, st));
    std::vector<int32_t> hs, hqe;
    std::vector<int64_t> hre;
    if ((rc = d2h(ctx, hs, score, np))) return rc;
    if ((rc = d2h(ctx, hqe, qend, np))) return rc;
    if ((rc = d2h(ctx, hre, rend, np))) return rc;
    HIP_TRY(hipStreamSynchronize(st));
    std::vector<int32_t> rq(np), bandv(np);
    std::vector<int64_t> rr(np);
    std::vector<int64_t> ids16, ids32;
    for (int64_t p = 0; p < np; ++p) {
      if (hs[p] <= 0) { rq[p] = 0; rr[p] = 0; bandv[p] = 0; continue; }
      rq[p] = hqe[p] + 1;
      rr[p] = hre[p] + 1;
      // every score1 alignment ending at the end cell stays within G' diagonals
      // of the reversed start: G' = (smax*min(qe+1, re+1) - o + e - score1) / e
      if (sc.e > 0) {
        const int64_t mlen = std::min<int64_t>(rq[p], rr[p]);
        int64_t g = ((int64_t)sc.smax * mlen - sc.o + sc.e - hs[p]) / sc.e;
        if (g < 0) g = 0;
        bandv[p] = (int32_t)std::min<int64_t>(g, 1 << 30);
      } else {
        bandv[p] = -1;
      }
      (is32[p] ? ids32 : ids16).push_back(p);
    }
    PairView rview{rqs, rrs, rql, rrl, b.qcat, b.rcat, 1};
    FillOut rout{rsc, rqe, rre, rov};
    HIP_TRY(hipMemsetAsync(rsc, 0, sizeof(int32_t) * np, st));
    Plan r16, r32;
    plan_tasks(r16, ids16, rq.data(), rr.data(), bandv.data(), 16, R, sc.n, sc.qsel);
    if ((rc = run_fill(ctx, r16, sc, rview, true, tgt, rout))) return rc;
    plan_tasks(r32, ids32, rq.data(), rr.data(), bandv.data(), 32, R, sc.n, sc.qsel);
    if ((rc = run_fill(ctx, r32, sc, rview, true, tgt, rout))) return rc;
    HIP_TRY(launch_begins(np, score, qend, rend, rsc, rqe, rre, qbeg, rbeg, err, st));
  }
  if ((rc = mark(4))) return rc;

  // banded traceback: CIGAR
  int64_t *cig_off_final = A.get<int64_t>(np + 1);
  int32_t *cig_len = A.get<int32_t>(np);
  if (!cig_off_final || !cig_len) return fail(SWX_ENOMEM, "device pool exhausted");
  HIP_TRY(hipMemsetAsync(cig_len, 0, sizeof(int32_t) * np, st));
  HIP_TRY(hipMemsetAsync(cig_off_final, 0, sizeof(int64_t) * (np + 1), st));
  int64_t cig_total = 0;
  if (flags & SWX_CIGAR) {
    int64_t *dsz = A.get<int64_t>(np + 1), *ccap = A.get<int64_t>(np + 1), *rcap = A.get<int64_t>(np + 1);
    int64_t *doff = A.get<int64_t>(np + 1), *coff = A.get<int64_t>(np + 1), *roff = A.get<int64_t>(np + 1);
    if (!dsz || !ccap || !rcap || !doff || !coff || !roff) return fail(SWX_ENOMEM, "device pool exhausted");
    HIP_TRY(hipMemsetAsync(dsz, 0, sizeof(int64_t) * (np + 1), st));
    HIP_TRY(hipMemsetAsync(ccap, 0, sizeof(int64_t) * (np + 1), st));
    HIP_TRY(hipMemsetAsync(rcap, 0, sizeof(int64_t) * (np + 1), st));
    HIP_TRY(launch_band_sizes(np, score, qbeg, qend, rbeg, rend, qlen, rlen, sc.smax, sc.o, sc.e,
                              dsz, ccap, rcap, st));
    if ((rc = scan(ctx, dsz, doff, np + 1))) return rc;
    if ((rc = scan(ctx, ccap, coff, np + 1))) return rc;
    if ((rc = scan(ctx, rcap, roff, np + 1))) return rc;
    int64_t tot[3];
    HIP_TRY(hipMemcpyAsync(&tot[0], doff + np, 8, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(&tot[1], coff + np, 8, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(&tot[2], roff + np, 8, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    uint8_t *dir = A.get<uint8_t>(tot[0]);
    uint32_t *cscr = A.get<uint32_t>(tot[1]);
    int32_t *rows = A.get<int32_t>(2 * tot[2]);
    if (!dir || !cscr || !rows) return fail(SWX_ENOMEM, "device pool exhausted (band)");
    BandArgs ba{};
    ba.npairs = np;
    ba.score = score;
    ba.qbeg = qbeg; ba.qend = qend; ba.rbeg = rbeg; ba.rend = rend;
    ba.qstart = qstart; ba.rstart = rstart;
    ba.qlen = qlen; ba.rlen = rlen;
    ba.qcat = b.qcat; ba.rcat = b.rcat;
    ba.matrix = sc.dmat;
    ba.n = sc.n; ba.o = sc.o; ba.e = sc.e; ba.smax = sc.smax;
    ba.dir = dir; ba.dir_off = doff;
    ba.rowbuf = rows; ba.row_off = roff;
    ba.cig = cscr; ba.cig_off = coff;
    ba.cig_len = cig_len;
    ba.err = err;
    HIP_TRY(launch_band_tb(ba, st));
    // compaction offsets
    int64_t *clen64 = A.get<int64_t>(np + 1);
    if (!clen64) return fail(SWX_ENOMEM, "device pool exhausted");
    std::vector<int32_t> hcl;
    if ((rc = d2h(ctx, hcl, cig_len, np))) return rc;
    HIP_TRY(hipStreamSynchronize(st));
    std::vector<int64_t> hoff(np + 1, 0);
    for (int64_t p = 0; p < np; ++p) hoff[p + 1] = hoff[p] + hcl[p];
    cig_total = hoff[np];
    HIP_TRY(hipMemcpyAsync(cig_off_final, hoff.data(), sizeof(int64_t) * (np + 1),
                           hipMemcpyHostToDevice, st));
    out->cigar_used = cig_total;
    if (cig_total > out->cigar_cap || (cig_total > 0 && !out->cigar)) {
      // records are still produced; CIGARs are not copied
      flags &= ~SWX_CIGAR;
      rc = SWX_ERANGE;
      g_last_error = "CIGAR arena too small";
    } else {
      uint32_t *dst = out->cigar;
      uint32_t *dtmp = nullptr;
      if (out->out_mem != SWX_MEM_DEVICE) {
        dtmp = A.get<uint32_t>(cig_total);
        if (!dtmp) return fail(SWX_ENOMEM, "device pool exhausted");
        dst = dtmp;
      }
      HIP_TRY(launch_cigar_compact(np, cscr, coff, cig_len, cig_off_final, dst, st));
      if (dtmp && cig_total)
        HIP_TRY(hipMemcpyAsync(out->cigar, dtmp, sizeof(uint32_t) * cig_total,
                               hipMemcpyDeviceToHost, st));
    }
  } else {
    out->cigar_used = 0;
  }
  int rc_range = rc;
  rc = mark(5);
  if (rc) return rc;

  // score2 from the max array (final CM plane of the forward tasks)
  if (flags & SWX_SCORE2) {
    Score2InterArgs s2{};
    s2.rlen = rlen; s2.qlen = qlen; s2.score1 = score; s2.rbeg = rbeg; s2.rend = rend;
    s2.mask_len = mask_len; s2.score2 = score2; s2.rend2 = rend2;
    s2.tasks = p16.d_tasks; s2.ntasks = (int64_t)p16.tasks.size(); s2.slot_pair = p16.d_slot_pair;
    s2.bnd = p16.d_bnd; s2.halves = 2;
    HIP_TRY(launch_score2_inter(s2, st));
    if (!p32.tasks.empty()) {
      s2.tasks = p32.d_tasks; s2.ntasks = (int64_t)p32.tasks.size(); s2.slot_pair = p32.d_slot_pair;
      s2.bnd = p32.d_bnd; s2.halves = 1;
      HIP_TRY(launch_score2_inter(s2, st));
    }
  }
  if ((rc = mark(6))) return rc;

  // records
  swx_rec_dev *drec = (out->out_mem == SWX_MEM_DEVICE) ? (swx_rec_dev *)out->recs
                                                       : A.get<swx_rec_dev>(np);
  if (!drec) return fail(SWX_ENOMEM, "device pool exhausted");
  HIP_TRY(launch_records(np, score, score2, qbeg, qend, rbeg, rend, rend2, cig_off_final, cig_len,
                         lanebits, flags, drec, st));
  if (out->out_mem != SWX_MEM_DEVICE && np)
    HIP_TRY(hipMemcpyAsync(out->recs, drec, sizeof(swx_rec) * np, hipMemcpyDeviceToHost, st));
  if ((rc = mark(7))) return rc;
  std::vector<uint8_t> herr;
  if ((rc = d2h(ctx, herr, err, np))) return rc;
  HIP_TRY(hipStreamSynchronize(st));
  ctx->nstages = 7;
  for (int k = 0; k < 7; ++k) {
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, ctx->ev[k], ctx->ev[k + 1]));
    ctx->stage_ms[k] = ms;
  }
  for (int64_t p = 0; p < np; ++p)
    if (herr[p]) return fail(SWX_EINTERNAL, "internal consistency check failed for pair " +
                                                std::to_string(p));
  (void)stage;
  return rc_range;
}

}  // namespace swx

using namespace swx;

// ============================================================================
// C ABI
// ============================================================================
extern "C" {

const char *swx_strerror(int status) {
  switch (status) {
    case SWX_OK: return "ok";
    case SWX_EINVAL: return "invalid argument";
    case SWX_ENOMEM: return "out of memory";
    case SWX_EDEVICE: return "device error";
    case SWX_EBUSY: return "busy";
    case SWX_EOVERFLOW: return "score range overflow";
    case SWX_ERANGE: return "output arena too small";
    case SWX_EINTERNAL: return "internal consistency check failed";
    default: return "unknown status";
  }
}

const char *swx_last_error(void) { return g_last_error.c_str(); }

int swx_ctx_create(int device, swx_ctx **out) {
  if (!out) return fail(SWX_EINVAL, "out is null");
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0)
    return fail(SWX_EDEVICE, "no HIP device available");
  if (device < 0 || device >= ndev) return fail(SWX_EINVAL, "device ordinal out of range");
  swx_ctx *c = new (std::nothrow) swx_ctx();
  if (!c) return fail(SWX_ENOMEM, "host allocation failed");
  c->device = device;
  if (hipSetDevice(device) != hipSuccess || hipStreamCreate(&c->stream) != hipSuccess) {
    delete c;
    return fail(SWX_EDEVICE, "could not create a stream");
  }
  for (auto &e : c->ev) {
    if (hipEventCreate(&e) != hipSuccess) {
      delete c;
      return fail(SWX_EDEVICE, "could not create events");
    }
  }
  *out = c;
  return SWX_OK;
}

int swx_ctx_destroy(swx_ctx *ctx) {
  if (!ctx) return fail(SWX_EINVAL, "ctx is null");
  {
    std::lock_guard<std::mutex> g(ctx->mu);
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    ctx->arena.release();
    for (auto &e : ctx->ev)
      if (e) (void)hipEventDestroy(e);
    (void)hipStreamDestroy(ctx->stream);
  }
  delete ctx;
  return SWX_OK;
}

int swx_last_stage_ms(const swx_ctx *ctx, double *ms, int cap) {
  if (!ctx || !ms || cap < 0) return fail(SWX_EINVAL, "bad arguments");
  int n = std::min(cap, ctx->nstages);
  for (int k = 0; k < n; ++k) ms[k] = ctx->stage_ms[k];
  return n;
}

int swx_profile_create(swx_ctx *ctx, const int8_t *query, int32_t qlen, const int8_t *matrix,
                       int32_t n, int32_t gap_open, int32_t gap_extend, swx_profile **out) {
  if (!out) return fail(SWX_EINVAL, "out is null");
  *out = nullptr;
  if (!query || !matrix) return fail(SWX_EINVAL, "null query or matrix");
  if (qlen < 1) return fail(SWX_EINVAL, "qlen must be >= 1");
  Scoring sc;
  int rc = make_scoring(matrix, n, gap_open, gap_extend, &sc);
  if (rc) return rc;
  for (int32_t i = 0; i < qlen; ++i)
    if (query[i] < 0 || query[i] >= n) return fail(SWX_EINVAL, "query symbol outside [0, n)");
  if (!ctx) return fail(SWX_EINVAL, "ctx is null");
  swx_profile *p = new (std::nothrow) swx_profile();
  if (!p) return fail(SWX_ENOMEM, "host allocation failed");
  p->ctx = ctx;
  p->query.assign(query, query + qlen);
  p->matrix.assign(matrix, matrix + (size_t)n * n);
  p->n = n;
  p->o = gap_open;
  p->e = gap_extend;
  *out = p;
  return SWX_OK;
}

int swx_profile_destroy(swx_profile *p) {
  if (!p) return fail(SWX_EINVAL, "profile is null");
  delete p;
  return SWX_OK;
}

void swx_result_free(swx_result *r) {
  if (!r) return;
  free(r->cigar);
  r->cigar = nullptr;
}

int64_t swx_cigar_bound(const swx_batch *b) {
  if (!b || b->in_mem != SWX_MEM_HOST || !b->qoff || !b->roff || !b->pair_q || !b->pair_r)
    return -1;
  int64_t s = 0;
  for (int64_t k = 0; k < b->npairs; ++k) {
    const int64_t qi = b->pair_q[k], ri = b->pair_r[k];
    if (qi < 0 || qi >= b->nq || ri < 0 || ri >= b->nr) return -1;
    s += (b->qoff[qi + 1] - b->qoff[qi]) + (b->roff[ri + 1] - b->roff[ri]) + 1;
  }
  return s;
}

static int align_batch_locked(swx_ctx *ctx, const swx_batch *b, swx_batch_out *out) {
  Scoring sc;
  int rc = make_scoring(b->matrix, b->n, b->gap_open, b->gap_extend, &sc);
  if (rc) return rc;
  if (b->npairs < 0 || b->nq < 0 || b->nr < 0 || b->qcat_len < 0 || b->rcat_len < 0)
    return fail(SWX_EINVAL, "negative count");
  if (!b->qoff || !b->roff || (b->npairs && (!b->pair_q || !b->pair_r)))
    return fail(SWX_EINVAL, "null offsets or pair arrays");
  if ((b->qcat_len && !b->qcat) || (b->rcat_len && !b->rcat))
    return fail(SWX_EINVAL, "null code arrays");
  if (!out || (b->npairs && !out->recs)) return fail(SWX_EINVAL, "null output");
  if (b->in_mem > 1 || out->out_mem > 1) return fail(SWX_EINVAL, "bad memory-space flag");
  if (b->flags & ~SWX_ALL) return fail(SWX_EINVAL, "unknown flag bits");
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(SWX_EDEVICE, "hipSetDevice failed");
  ctx->arena.reset();
  DevArena &A = ctx->arena;
  hipStream_t st = ctx->stream;
  int8_t *dmat = A.get<int8_t>((int64_t)sc.n * sc.n);
  if (!dmat) return fail(SWX_ENOMEM, "device pool exhausted");
  HIP_TRY(hipMemcpyAsync(dmat, b->matrix, (size_t)sc.n * sc.n, hipMemcpyHostToDevice, st));
  sc.dmat = dmat;
  DeviceBatch db{};
  db.qcat_len = b->qcat_len; db.rcat_len = b->rcat_len; db.nq = b->nq; db.nr = b->nr;
  db.npairs = b->npairs;
  if (b->in_mem == SWX_MEM_DEVICE) {
    db.qcat = b->qcat; db.rcat = b->rcat; db.qoff = b->qoff; db.roff = b->roff;
    db.pair_q = b->pair_q; db.pair_r = b->pair_r;
  } else {
    int8_t *qc = A.get<int8_t>(b->qcat_len), *rc8 = A.get<int8_t>(b->rcat_len);
    int64_t *qo = A.get<int64_t>(b->nq + 1), *ro = A.get<int64_t>(b->nr + 1);
    int64_t *pq = A.get<int64_t>(b->npairs), *pr = A.get<int64_t>(b->npairs);
    if (!qc || !rc8 || !qo || !ro || !pq || !pr) return fail(SWX_ENOMEM, "device pool exhausted");
    if (b->qcat_len) HIP_TRY(hipMemcpyAsync(qc, b->qcat, b->qcat_len, hipMemcpyHostToDevice, st));
    if (b->rcat_len) HIP_TRY(hipMemcpyAsync(rc8, b->rcat, b->rcat_len, hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(qo, b->qoff, 8 * (b->nq + 1), hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(ro, b->roff, 8 * (b->nr + 1), hipMemcpyHostToDevice, st));
    if (b->npairs) {
      HIP_TRY(hipMemcpyAsync(pq, b->pair_q, 8 * b->npairs, hipMemcpyHostToDevice, st));
      HIP_TRY(hipMemcpyAsync(pr, b->pair_r, 8 * b->npairs, hipMemcpyHostToDevice, st));
    }
    db.qcat = qc; db.rcat = rc8; db.qoff = qo; db.roff = ro; db.pair_q = pq; db.pair_r = pr;
  }
  if (b->npairs == 0) {
    out->cigar_used = 0;
    return SWX_OK;
  }
  return run_pipeline(ctx, sc, db, b->flags, b->mask_len, out);
}

int swx_align_batch(swx_ctx *ctx, const swx_batch *b, swx_batch_out *out) {
  if (!ctx || !b || !out) return fail(SWX_EINVAL, "null argument");
  std::lock_guard<std::mutex> g(ctx->mu);
  return align_batch_locked(ctx, b, out);
}

int swx_align(const swx_profile *p, const int8_t *ref, int64_t rlen, uint32_t flags,
              int32_t mask_len, swx_result *out) {
  if (!p || !out || (rlen > 0 && !ref)) return fail(SWX_EINVAL, "null argument");
  if (rlen < 0) return fail(SWX_EINVAL, "rlen must be >= 0");
  if (flags & ~(SWX_ALL | SWX_REF_DEVICE)) return fail(SWX_EINVAL, "unknown flag bits");
  swx_ctx *ctx = p->ctx;
  std::lock_guard<std::mutex> g(ctx->mu);
  memset(out, 0, sizeof(*out));
  std::vector<int8_t> href;
  const int8_t *rptr = ref;
  if (flags & SWX_REF_DEVICE) {
    href.resize((size_t)rlen);
    if (rlen && hipMemcpy(href.data(), ref, (size_t)rlen, hipMemcpyDeviceToHost) != hipSuccess)
      return fail(SWX_EDEVICE, "could not read the device reference");
    rptr = href.data();
  }
  const int64_t qoff[2] = {0, (int64_t)p->query.size()};
  const int64_t roff[2] = {0, rlen};
  const int64_t pq = 0, pr = 0;
  swx_batch b{};
  b.matrix = p->matrix.data(); b.n = p->n; b.gap_open = p->o; b.gap_extend = p->e;
  b.qcat = p->query.data(); b.qcat_len = (int64_t)p->query.size(); b.qoff = qoff; b.nq = 1;
  b.rcat = rptr; b.rcat_len = rlen; b.roff = roff; b.nr = 1;
  b.pair_q = &pq; b.pair_r = &pr; b.npairs = 1;
  b.flags = flags & SWX_ALL; b.mask_len = mask_len; b.in_mem = SWX_MEM_HOST;
  swx_rec rec{};
  std::vector<uint32_t> cig((size_t)(p->query.size() + rlen + 2));
  swx_batch_out bo{&rec, cig.data(), (int64_t)cig.size(), 0, SWX_MEM_HOST};
  int rc = align_batch_locked(ctx, &b, &bo);
  if (rc) return rc;
  out->rec = rec;
  out->cigar = nullptr;
  if (rec.cigar_len > 0) {
    out->cigar = (uint32_t *)malloc(sizeof(uint32_t) * rec.cigar_len);
    if (!out->cigar) return fail(SWX_ENOMEM, "host allocation failed");
    memcpy(out->cigar, cig.data() + rec.cigar_off, sizeof(uint32_t) * rec.cigar_len);
  }
  out->rec.cigar_off = 0;
  return SWX_OK;
}

}  // extern "C"
