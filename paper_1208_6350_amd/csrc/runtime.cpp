// runtime.cpp -- host side of the library: contexts, validation, planning of
// the inter-sequence tasks, and the alignment pipeline
//   forward fill -> 32-bit re-run of saturated pairs -> reversed pass (begin)
//   -> banded traceback (CIGAR) -> masked max array (score2) -> records,
// following the order of the paper's method section.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <functional>
#include <map>
#include <tuple>
#include <mutex>
#include <numeric>
#include <string>
#include <thread>
#include <vector>

#include "../../include/swx.h"
#include "runtime_internal.h"
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
// In fixed mode (use_fixed) every allocation comes from one given block and
// nothing is ever allocated from the device: a request past its end fails.
class DevArena {
 public:
  ~DevArena() { release(); }
  void reset() {
    cur_ = 0;
    off_ = 0;
    fixed_off_ = 0;
  }
  void use_fixed(void *p, size_t bytes) {
    fixed_ = p;
    fixed_size_ = bytes;
    fixed_off_ = 0;
    fixed_short_ = false;
  }
  void use_pool() { fixed_ = nullptr; }
  bool fixed_exhausted() const { return fixed_short_; }
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
    if (fixed_) {
      if (bytes > fixed_size_ - fixed_off_) {
        fixed_short_ = true;
        return nullptr;
      }
      void *p = (char *)fixed_ + fixed_off_;
      fixed_off_ += bytes;
      return p;
    }
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
  void *fixed_ = nullptr;
  size_t fixed_size_ = 0, fixed_off_ = 0;
  bool fixed_short_ = false;
};

// ---- static scratch of the entry point that allocates nothing ---------------
// One array per GPU (each device holds its own copy of a __device__ variable),
// kept until the process ends.  Host code never uses its name as an address:
// the device address comes from hipGetSymbolAddress, taken once per device
// with that device current (at the first context made on it).
static __device__ __align__(256) uint8_t scratch[SWX_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[kMaxDevices] = {};
static std::mutex g_scratch_use[kMaxDevices];   // one call at a time per device

// the device address of `scratch` on `device` (current), or nullptr
static void *scratch_address(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void *ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess) return nullptr;
    g_scratch_ptr[device] = ptr;
  }
  return g_scratch_ptr[device];
}

}  // namespace swx

struct swx_ctx {
  int device = 0;
  hipStream_t stream = nullptr;   // the stream of the running call (own, or the caller's)
  hipStream_t own = nullptr;      // the context's own stream
  swx::DevArena arena;
  std::mutex mu;
  hipEvent_t ev[8] = {};
  double stage_ms[8] = {};
  int nstages = 0;
  int64_t fill_cells = 0;   // cells of the last forward fill launch
  // routing of long pairs to the intra-sequence path and its launch shape
  int64_t long_cells = -1;                 // qlen * rlen above this (-1: from the batch) ...
  int64_t long_rlen = int64_t(1) << 16;    // ... or a reference longer than this
  int64_t intra_jobs = 2048;               // target column chunks over all long pairs
  int32_t fill_rows = 32;                  // strip height of the batched fill
  int32_t fill_sched = 1;                  // task order of the batched fill (InterArgs::sched)
  int32_t fill_coop = 0;                   // cooperative tasks: 0 automatic, 1 never, 2 always
  int32_t intra_bits = 0;                  // long pairs' lanes: 0 automatic, 16 where scores fit, 32
  int32_t cus = 0;                         // compute units of the device
  unsigned long long *queue = nullptr;     // work-queue counter of the batched fill
  // side streams (default priority) for independent kernels of one stage
  static constexpr int kAux = 3;   // side streams, created on first use
  bool side_streams = true;
  hipStream_t aux[kAux] = {};
  hipEvent_t fork_ev = nullptr;
  hipEvent_t join_ev[kAux] = {};
  // one-pair calls (swx_align): captured graphs of capacity one pair, one per
  // scoring scheme, flags and power-of-two size class, least recently used
  // evicted; pair_mu serialises their use (taken before mu, never inside it)
  struct PairGraph {
    std::vector<int8_t> matrix;
    int32_t n = 0, o = 0, e = 0, mask_len = 0;
    uint32_t flags = 0;
    int32_t qcap = 0;
    int64_t rcap = 0;
    swx_graph *g = nullptr;
    uint64_t last_use = 0;
  };
  std::mutex pair_mu;
  std::vector<PairGraph> pair_graphs;
  uint64_t pair_clock = 0;
  // pinned landing area of the small device-to-host reads between stages
  static constexpr int64_t kPinned = 512;   // int64 values
  int64_t *pinned = nullptr;
  void *scratch = nullptr;   // this device's static scratch (swx_align_batch_noalloc)
};

struct swx_profile {
  swx_ctx *ctx = nullptr;
  std::vector<int8_t> query;
  std::vector<int8_t> matrix;
  int32_t n = 0, o = 0, e = 0;
  // alphabets above 4 symbols: the query profile on the device, built once
  // (forward strips of 32 and of 16 rows, and the reversed table)
  uint8_t *dev = nullptr;
  uint8_t *fwd32 = nullptr, *fwd16 = nullptr, *rev = nullptr;
  int32_t qp32 = 0, qp16 = 0;
  int64_t rev_row = 0;
};

namespace swx {

// Runs a call on the caller's stream: while it lives, ctx->stream names
// `user` (when not null) instead of the context's own stream.  Every stage of
// a call issues its work on ctx->stream, so the call is ordered after the
// work the caller queued on that stream before it; side streams fork from it
// and join back into it.  Callers hold ctx->mu.
struct StreamScope {
  swx_ctx *c;
  hipStream_t saved;
  StreamScope(swx_ctx *c_, void *user) : c(c_), saved(c_->stream) {
    if (user) c->stream = (hipStream_t)user;
  }
  ~StreamScope() { c->stream = saved; }
  StreamScope(const StreamScope &) = delete;
  StreamScope &operator=(const StreamScope &) = delete;
};

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
  // the fills' bias: at least -min S, so that every biased score S + bias is
  // a byte >= 0; the gap open penalty where that qualifies, since the fill's
  // saturating H = hb - bias is then also its H - o (one instruction fewer
  // per cell)
  sc->bias = mn < 0 ? -mn : 0;
  if (o >= sc->bias && o + mx <= 255) sc->bias = o;
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

// The query profile of a batch whose pairs all use one query (k_build_qprof):
// forward strips of R rows, and the reversed table of 16 shifted copies.
struct SharedProf {
  const uint8_t *fwd = nullptr, *rev = nullptr;
  int64_t fwd_row = 0, rev_row = 0;
  int32_t qlen = 0, R = 0;
};

// ---- device-side planning of one fill pass ---------------------------------
struct Plan {
  int64_t n = 0, ntasks = 0;
  int lane_bits = 16, R = 32;
  InterTask *d_tasks = nullptr;
  int64_t *d_sorted = nullptr;   // slot -> pair id
  uint32_t *d_bnd = nullptr;
  uint2 *d_rsym = nullptr;       // packed reference symbols
  uint8_t *d_prof = nullptr;
};

static inline int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

// Waves per task of a batched fill pass: a pass with fewer tasks than the
// device holds waves (two per SIMD) leaves SIMDs idle and makes its largest
// task the critical path, so its tasks run on a workgroup's four waves each.
static int coop_waves(int32_t policy, int64_t ntasks, int32_t cus) {
  if (policy == 1) return 1;
  if (policy == 2) return kCoopWaves;
  return ntasks < (int64_t)cus * 4 * 2 ? kCoopWaves : 1;
}


// Wait for a stream by polling it.  A blocking wait sleeps until an interrupt
// wakes the thread, tens of microseconds after the stream has drained, and
// every host read between the stages of a call paid that with an idle device.
static hipError_t wait_stream(hipStream_t st) {
  for (;;) {
    const hipError_t e = hipStreamQuery(st);
    if (e != hipErrorNotReady) return e;
    std::this_thread::yield();
  }
}

template <class T>
static T *alloc_or_null(DevArena &A, int64_t n) { return A.get<T>(n); }

// Sort the pass's pairs by (band, padded query height, reference length) on
// the device, cut them into tasks, derive buffer offsets and allocate.
static int plan_pass(swx_ctx *ctx, const Scoring &sc, const int64_t *ids, int64_t n,
                     const int32_t *qlen, const int64_t *rlen, const int32_t *band,
                     const int32_t *band_q, int lane_bits, int R, Plan &pl,
                     const SharedProf *sp = nullptr) {
  DevArena &A = ctx->arena;
  hipStream_t st = ctx->stream;
  pl = Plan{};
  pl.n = n;
  pl.lane_bits = lane_bits;
  pl.R = R;
  if (n == 0) return SWX_OK;
  const int slots = lane_bits == 16 ? kSlots16 : kSlots32;
  const int halves = lane_bits == 16 ? 2 : 1;
  pl.ntasks = (n + slots - 1) / slots;
  uint64_t *k0 = A.get<uint64_t>(n), *k1 = A.get<uint64_t>(n);
  int64_t *v0 = A.get<int64_t>(n), *v1 = A.get<int64_t>(n);
  pl.d_tasks = A.get<InterTask>(pl.ntasks);
  int64_t *bsz = A.get<int64_t>(pl.ntasks + 1), *qsz = A.get<int64_t>(pl.ntasks + 1);
  int64_t *boff = A.get<int64_t>(pl.ntasks + 1), *qoff = A.get<int64_t>(pl.ntasks + 1);
  if (!k0 || !k1 || !v0 || !v1 || !pl.d_tasks || !bsz || !qsz || !boff || !qoff)
    return fail(SWX_ENOMEM, "device pool exhausted (plan)");
  size_t tmp_bytes = 0;
  HIP_TRY(plan_sort(n, nullptr, ids, qlen, rlen, band, R, k0, k1, v0, v1, nullptr, &tmp_bytes, nullptr, st));
  void *tmp = A.alloc(tmp_bytes);
  if (!tmp) return fail(SWX_ENOMEM, "device pool exhausted (sort)");
  HIP_TRY(plan_sort(n, nullptr, ids, qlen, rlen, band, R, k0, k1, v0, v1, tmp, &tmp_bytes, &pl.d_sorted, st));
  // profile bytes per padded row and task; -1: a profile shared by every task
  const int64_t per_row = sc.qsel ? 0 : (sp ? -1 : (int64_t)(sc.n + 1) * halves * 64);
  HIP_TRY(plan_tasks_dev(   // also clears bsz[ntasks], qsz[ntasks]
                         n, nullptr, pl.ntasks, slots, R, per_row, pl.d_sorted, qlen, rlen, band,
                         band_q, pl.d_tasks, bsz, qsz, st));
  size_t t1 = 0, t2 = 0;
  HIP_TRY(launch_exclusive_scan(bsz, boff, pl.ntasks + 1, nullptr, &t1, st));
  void *s1 = A.alloc(t1);
  if (!s1) return fail(SWX_ENOMEM, "device pool exhausted (scan)");
  HIP_TRY(launch_exclusive_scan(bsz, boff, pl.ntasks + 1, s1, &t1, st));
  HIP_TRY(launch_exclusive_scan(qsz, qoff, pl.ntasks + 1, nullptr, &t2, st));
  void *s2 = A.alloc(t2);
  if (!s2) return fail(SWX_ENOMEM, "device pool exhausted (scan)");
  HIP_TRY(launch_exclusive_scan(qsz, qoff, pl.ntasks + 1, s2, &t2, st));
  HIP_TRY(plan_offsets_dev(pl.ntasks, pl.d_tasks, boff, qoff, st));
  HIP_TRY(hipMemcpyAsync(ctx->pinned, boff + pl.ntasks, 8, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipMemcpyAsync(ctx->pinned + 1, qoff + pl.ntasks, 8, hipMemcpyDeviceToHost, st));
  HIP_TRY(wait_stream(st));
  const int64_t tot[2] = {ctx->pinned[0], ctx->pinned[1]};
  pl.d_bnd = A.get<uint32_t>(tot[0]);
  pl.d_rsym = A.get<uint2>(rsym_offset(tot[0]));
  if (!pl.d_bnd || !pl.d_rsym) return fail(SWX_ENOMEM, "device pool exhausted (boundary planes)");
  if (per_row > 0) {
    pl.d_prof = A.get<uint8_t>(tot[1]);
    if (!pl.d_prof) return fail(SWX_ENOMEM, "device pool exhausted (profiles)");
  }
  return SWX_OK;
}

// Runs independent launches side by side: each goes to a side stream that
// first waits for everything queued on the main stream, and the main stream
// then waits for all of them.  Launches come with a cost estimate (an
// estimated run time alone on the device) and are placed longest first on the
// least loaded of three side streams (the device gives a process four
// hardware queues: with the main stream, one each; measured: the benchmark's
// traceback stage 4.46 -> 4.28 ms against two).  A `lead` launch (one whose few,
// long waves leave most of the device to others) goes first, alone, and its
// stream is charged only kLeadShare of its cost: the launches beside it run
// mostly in its shadow.
struct SideLaunch {
  double cost;
  std::function<hipError_t(hipStream_t)> fn;
  bool lead = false;
};
constexpr double kLeadShare = 0.2;

// Side streams are made on first use, so a context that never needs them
// (short pairs only) holds a single stream and a single hardware queue.
// False when side streams are off or could not be made.
static bool have_side_streams(swx_ctx *ctx) {
  if (!ctx->side_streams) return false;
  bool have = true;
  for (int k = 0; k < swx_ctx::kAux; ++k)
    if (!ctx->aux[k] && hipStreamCreate(&ctx->aux[k]) != hipSuccess) {
      ctx->aux[k] = nullptr;
      have = false;
    }
  return have;
}

static int run_side_by_side(swx_ctx *ctx, std::vector<SideLaunch> &ls) {
  if (ls.empty()) return SWX_OK;
  if (ls.size() == 1 || !ctx->side_streams) {
    for (auto &l : ls) HIP_TRY(l.fn(ctx->stream));
    return SWX_OK;
  }
  constexpr int na = swx_ctx::kAux;
  if (!have_side_streams(ctx)) {   // no side streams: one after the other on the main stream
    for (auto &l : ls) HIP_TRY(l.fn(ctx->stream));
    return SWX_OK;
  }
  std::stable_sort(ls.begin(), ls.end(), [](const SideLaunch &x, const SideLaunch &y) {
    return x.lead != y.lead ? x.lead : x.cost > y.cost;
  });
  HIP_TRY(hipEventRecord(ctx->fork_ev, ctx->stream));
  for (int k = 0; k < na; ++k) HIP_TRY(hipStreamWaitEvent(ctx->aux[k], ctx->fork_ev, 0));
  // place every launch first, then submit stream by stream: the lead's
  // stream is filled before the other one starts (measured: interleaved
  // submission lets the other stream's first kernel take the device first)
  double load[na] = {};
  std::vector<int> where(ls.size());
  for (size_t x = 0; x < ls.size(); ++x) {
    int k = 0;
    for (int y = 1; y < na; ++y)
      if (load[y] < load[k]) k = y;
    load[k] += ls[x].lead ? kLeadShare * ls[x].cost : ls[x].cost;
    where[x] = k;
  }
  for (int k = 0; k < na; ++k)
    for (size_t x = 0; x < ls.size(); ++x)
      if (where[x] == k) HIP_TRY(ls[x].fn(ctx->aux[k]));
  for (int k = 0; k < na; ++k) {
    HIP_TRY(hipEventRecord(ctx->join_ev[k], ctx->aux[k]));
    HIP_TRY(hipStreamWaitEvent(ctx->stream, ctx->join_ev[k], 0));
  }
  return SWX_OK;
}

// profile (general alphabets) + fill for one plan; when mark_fill >= 0,
// events mark_fill and mark_fill + 1 bracket the fill kernel alone
static int run_fill(swx_ctx *ctx, Plan &pl, const Scoring &sc, const PairView &view, bool rev,
                    const int32_t *d_target, FillOut out, int64_t score_bound,
                    int mark_fill = -1, uint32_t anchor = 0, int lastcol = 0,
                    const SharedProf *sp = nullptr) {
  hipStream_t st = ctx->stream;
  if (pl.ntasks == 0) {
    if (mark_fill >= 0) {
      HIP_TRY(hipEventRecord(ctx->ev[mark_fill], st));
      HIP_TRY(hipEventRecord(ctx->ev[mark_fill + 1], st));
    }
    return SWX_OK;
  }
  PackArgs pk{};
  pk.tasks = pl.d_tasks;
  pk.ntasks = pl.ntasks;
  pk.slot_pair = pl.d_sorted;
  pk.view = view;
  pk.prof = pl.d_prof;
  pk.rsym = pl.d_rsym;
  pk.matrix = sc.dmat;
  pk.n = sc.n;
  pk.bias = sc.bias;
  pk.halves = pl.lane_bits == 16 ? 2 : 1;
  pk.strip_rows = pl.R;
  pk.rev = rev ? 1 : 0;
  HIP_TRY(inter_pack_ref(pk, st));
  if (!sc.qsel && !sp) HIP_TRY(inter_pack(pk, st));
  InterArgs a{};
  a.tasks = pl.d_tasks;
  a.ntasks = pl.ntasks;
  a.slot_pair = pl.d_sorted;
  a.view = view;
  a.prof = (sc.qsel || sp) ? nullptr : pl.d_prof;
  if (sp && !sc.qsel) {
    a.qprof = rev ? sp->rev : sp->fwd;
    a.qprof_row = rev ? sp->rev_row : sp->fwd_row;
    a.qprof_copy = (int64_t)(sc.n + 1) * sp->rev_row;
    a.qprof_qlen = sp->qlen;
  }
  a.bnd = pl.d_bnd;
  a.rsym = pl.d_rsym;
  for (int k = 0; k < 8; ++k) a.lut[k] = sc.lut[k];
  a.n = sc.n;
  a.o = sc.o;
  a.e = sc.e;
  a.bias = sc.bias;
  a.rev = rev ? 1 : 0;
  // without a possible score above the 16-bit value field the row code needs
  // no saturation (scores are at most smax * min(qlen, rlen))
  a.clamp = score_bound > kInter16Limit - 1 ? 1 : 0;
  a.pair3 = score_bound <= kInter16PairLimit ? 1 : 0;
  a.code_top = pl.R - 1;
  a.dummy = sc.dmat;   // any readable device bytes
  a.target = d_target;
  a.out = out;
  a.sched = ctx->fill_sched;
  a.cus = ctx->cus;
  a.queue = ctx->queue;
  a.anchor = anchor;
  a.lastcol = lastcol;
  a.coop = coop_waves(ctx->fill_coop, pl.ntasks, ctx->cus);
  // A pass runs its tasks by area (padded rows x swept columns, its cost),
  // largest first: the plan's order (by band, height, then width) leaves
  // mid-sized tasks of short, wide pairs for the end of the launch.  Passes
  // whose tasks all start at once (at most two per compute unit) keep the
  // plan's order and save the sort's launches.
  if (pl.ntasks > 2 * (int64_t)std::max(ctx->cus, 1)) {
    DevArena &A = ctx->arena;
    const int64_t nt = pl.ntasks;
    uint64_t *k0 = A.get<uint64_t>(nt), *k1 = A.get<uint64_t>(nt);
    int64_t *v0 = A.get<int64_t>(nt), *v1 = A.get<int64_t>(nt);
    if (!k0 || !k1 || !v0 || !v1) return fail(SWX_ENOMEM, "device pool exhausted (task order)");
    HIP_TRY(inter_area_keys(pl.d_tasks, nt, pl.R, k0, v0, st));
    size_t tb = 0;
    int64_t *order = nullptr;
    HIP_TRY(sort_keys(nt, k0, k1, v0, v1, nullptr, &tb, &order, st, 24));
    void *tmp = A.alloc(tb);
    if (!tmp) return fail(SWX_ENOMEM, "device pool exhausted (task order)");
    HIP_TRY(sort_keys(nt, k0, k1, v0, v1, tmp, &tb, &order, st, 24));
    a.order = order;
  }
  // A reversed pass over many tasks: its largest tasks (full rectangles of
  // weak alignments, no early exit) each take the four waves of a workgroup,
  // launched first beside the rest.  On one wave each they start first and
  // end last: on the benchmark workload the ~50 largest of 7,800 tasks ran
  // 2.0-3.1 ms against 2.1 ms of work per wave slot (the stage went 3.5 ->
  // 3.3 ms with the split).
  const int64_t nsplit = (rev && a.coop == 1 && ctx->fill_coop == 0 && ctx->side_streams &&
                          pl.ntasks >= (int64_t)ctx->cus * 8)
                             ? std::min<int64_t>(pl.ntasks / 16, ctx->cus / 2)
                             : 0;
  if (nsplit > 0 && mark_fill < 0) {
    InterArgs big = a, rest = a;
    big.order = a.order + (pl.ntasks - nsplit);   // the order lists the largest last
    big.ntasks = nsplit;
    big.coop = kCoopWaves;
    big.sched = 1;   // a grid of its own, all resident: no device queue
    rest.ntasks = pl.ntasks - nsplit;
    const int lb = pl.lane_bits, R = pl.R;
    std::vector<SideLaunch> ls;
    ls.push_back({2.0, [=](hipStream_t s_) { return inter_fill(big, lb, R, s_); }, true});
    ls.push_back({1.0, [=](hipStream_t s_) { return inter_fill(rest, lb, R, s_); }});
    return run_side_by_side(ctx, ls);
  }
  if (mark_fill >= 0) HIP_TRY(hipEventRecord(ctx->ev[mark_fill], st));
  HIP_TRY(inter_fill(a, pl.lane_bits, pl.R, st));
  if (mark_fill >= 0) HIP_TRY(hipEventRecord(ctx->ev[mark_fill + 1], st));
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

// n values from the device; small reads land in pinned memory (a direct copy,
// no staging through the runtime's own buffers).  Callers hold ctx->mu.
static int read_i64(swx_ctx *ctx, const int64_t *d, int64_t *h, int64_t n = 1) {
  const bool pin = n <= swx_ctx::kPinned;
  HIP_TRY(hipMemcpyAsync(pin ? ctx->pinned : h, d, 8 * n, hipMemcpyDeviceToHost, ctx->stream));
  HIP_TRY(wait_stream(ctx->stream));
  if (pin) memcpy(h, ctx->pinned, 8 * (size_t)n);
  return SWX_OK;
}

// ids of the pairs whose flag is set (device list) and their count (device)
static int select_flagged_dev(swx_ctx *ctx, const uint8_t *flag, int64_t np, int64_t **ids,
                              const int64_t **count_dev) {
  DevArena &A = ctx->arena;
  int64_t *f64 = A.get<int64_t>(np + 1), *pos = A.get<int64_t>(np + 1);
  *ids = A.get<int64_t>(np);
  if (!f64 || !pos || !*ids) return fail(SWX_ENOMEM, "device pool exhausted (select)");
  HIP_TRY(flags_to_i64(np, flag, f64, ctx->stream));   // also clears f64[np]
  int rc = scan(ctx, f64, pos, np + 1);
  if (rc) return rc;
  HIP_TRY(compact_flags(np, flag, pos, *ids, ctx->stream));
  *count_dev = pos + np;
  return SWX_OK;
}

// the same with the count read back to the host
static int select_flagged(swx_ctx *ctx, const uint8_t *flag, int64_t np, int64_t **ids,
                          int64_t *count) {
  const int64_t *cd = nullptr;
  int rc = select_flagged_dev(ctx, flag, np, ids, &cd);
  if (rc) return rc;
  return read_i64(ctx, cd, count);
}

// ---- banded traceback: classify by band width, one register kernel per
// width class, a general kernel for bands wider than 64 diagonals ------------
struct DeviceBatch {
  const int8_t *qcat, *rcat;
  const int64_t *qoff, *roff, *pair_q, *pair_r;
  int64_t qcat_len, rcat_len, nq, nr, npairs;
};

static int gather_info(swx_ctx *ctx, int64_t n, const int64_t *d_ids, const int32_t *qlen,
                       const int64_t *rlen, const int32_t *score, const int32_t *qend,
                       const int64_t *rend, const int32_t *band, std::vector<int64_t> &info);

// Shape of a wave traceback over m rows, w columns and a band of bw diagonals
// when `jobs` such pairs share the device (rl 0: too tall for every choice).
// Strip s starts SH + 128 steps after strip s - 1 and sweeps a window of
// SH + bw columns; the waves of a pair's workgroups run its strips in turn,
// and a step costs about 16 instructions per row of a lane plus 30: the
// cheapest of the longer of those two paths.  With fewer pairs than compute
// units a pair's strips spread over up to four waves in each of `segs`
// workgroups (at most one per compute unit, 32 per XCD), as in the
// intra-sequence fill.
struct TbShape {
  int rl, waves, segs;
  bool operator<(const TbShape &x) const {
    return rl != x.rl ? rl < x.rl : waves != x.waves ? waves < x.waves : segs < x.segs;
  }
  bool operator==(const TbShape &x) const { return rl == x.rl && waves == x.waves && segs == x.segs; }
};

static TbShape tb_wave_shape(int64_t m, int64_t w, int64_t bw, int n, int64_t jobs, int32_t cus) {
  jobs = std::max<int64_t>(jobs, 1);
  const int64_t segs_max =
      (cus <= 0 || jobs >= cus)
          ? 1
          : std::max<int64_t>(1, std::min<int64_t>(cus / jobs, 32 / ((jobs + 7) / 8)));
  TbShape best{0, 0, 0};
  double best_cost = 0;
  for (int RL : {4, 8, 16}) {
    const int64_t SH = 64 * RL, nstrips = (m + SH - 1) / SH;
    if (nstrips > tb_wave_max_strips()) continue;
    int64_t waves = tb_wave_waves(m, n, RL), g = 1;
    if (segs_max > 1) {
      const int64_t w4 = std::min<int64_t>(4, waves);
      g = std::min<int64_t>(segs_max, (nstrips + w4 - 1) / w4);
      if (g > 1) waves = w4;
    }
    const int64_t win = std::min<int64_t>(SH + bw, w + 1) + 63;
    const int64_t chain = (nstrips - 1) * (SH + 128) + win;
    const int64_t turns = (nstrips + waves * g - 1) / (waves * g) * win;
    const double cost = (double)std::max(chain, turns) * (16 * RL + 30) * (waves > 4 ? 1.5 : 1.0);
    if (best.rl == 0 || cost < best_cost) {
      best = TbShape{RL, (int)waves, (int)g};
      best_cost = cost;
    }
  }
  return best;
}

static int run_traceback(swx_ctx *ctx, const Scoring &sc, const DeviceBatch &b, int64_t np,
                         const int32_t *score, const int32_t *qbeg, const int32_t *qend,
                         const int64_t *rbeg, const int64_t *rend, const int64_t *qstart,
                         const int64_t *rstart, const int32_t *qlen, const int64_t *rlen,
                         int32_t *cig_len, int64_t *cig_off_final, uint8_t *err,
                         swx_batch_out *out, uint32_t *flags, int *rc_range) {
  DevArena &A = ctx->arena;
  hipStream_t st = ctx->stream;
  int rc;
  TbArgs ta{};
  ta.score = score; ta.qbeg = qbeg; ta.qend = qend; ta.rbeg = rbeg; ta.rend = rend;
  ta.qstart = qstart; ta.rstart = rstart; ta.qlen = qlen; ta.rlen = rlen;
  ta.qcat = b.qcat; ta.rcat = b.rcat; ta.matrix = sc.dmat;
  ta.n = sc.n; ta.o = sc.o; ta.e = sc.e; ta.smax = sc.smax;
  ta.cig_len = cig_len; ta.err = err;
  ta.wave_cells = np <= kTbFewPairs ? kWaveTbCellsFew : kWaveTbCells;
  uint8_t *cls = A.get<uint8_t>(np);
  uint64_t *k0 = A.get<uint64_t>(np), *k1 = A.get<uint64_t>(np);
  int64_t *v0 = A.get<int64_t>(np), *v1 = A.get<int64_t>(np);
  int64_t *ccap = A.get<int64_t>(np + 1), *coff = A.get<int64_t>(np + 1);
  int64_t *counts = A.get<int64_t>(8);
  if (!cls || !k0 || !k1 || !v0 || !v1 || !ccap || !coff || !counts)
    return fail(SWX_ENOMEM, "device pool exhausted (traceback)");
  HIP_TRY(hipMemsetAsync(ccap + np, 0, 8, st));
  HIP_TRY(hipMemsetAsync(counts, 0, 64, st));
  HIP_TRY(tb_classify(ta, np, cls, k0, v0, ccap, st));
  if ((rc = scan(ctx, ccap, coff, np + 1))) return rc;
  HIP_TRY(count_classes(np, cls, counts, st));
  size_t tmp_bytes = 0;
  int64_t *sorted = nullptr;
  HIP_TRY(sort_keys(np, k0, k1, v0, v1, nullptr, &tmp_bytes, &sorted, st, kTbKeyBits));
  void *tmp = A.alloc(tmp_bytes);
  if (!tmp) return fail(SWX_ENOMEM, "device pool exhausted (sort)");
  HIP_TRY(sort_keys(np, k0, k1, v0, v1, tmp, &tmp_bytes, &sorted, st, kTbKeyBits));
  // the class counts and the CIGAR scratch size in one read (class 7 is
  // never used)
  HIP_TRY(hipMemcpyAsync(counts + 7, coff + np, sizeof(int64_t), hipMemcpyDeviceToDevice, st));
  int64_t hc[8];
  if ((rc = read_i64(ctx, counts, hc, 8))) return rc;
  const int64_t capw = hc[7];
  uint32_t *cscr = A.get<uint32_t>(capw);
  if (!cscr) return fail(SWX_ENOMEM, "device pool exhausted (CIGAR scratch)");
  ta.cig = cscr;
  ta.cig_off = coff;
  // plan every class first, read all their buffer sizes back in one go, then
  // launch the classes' kernels side by side: the small classes would not
  // fill the GPU alone.  totals: [c - 1] code words of band class c, [3] and
  // [4] code and boundary words of the strip class.
  int64_t *totals = A.get<int64_t>(8);
  if (!totals) return fail(SWX_ENOMEM, "device pool exhausted (traceback sizes)");
  struct BandPlan { TbTask *tasks; int64_t nt; int32_t bw; };
  BandPlan bands[3];
  int nbands = 0;
  TbwTask *wtasks = nullptr;
  int64_t wnt = 0;
  int64_t pos = hc[0];
  for (int c = 1; c <= 3; ++c) {
    const int64_t nc = hc[c];
    if (nc == 0) continue;
    const int32_t bw = 8 << (c - 1);
    const int64_t nt = (nc + 63) / 64;
    TbTask *tasks = A.get<TbTask>(nt);
    int64_t *dsz = A.get<int64_t>(nt + 1), *doff = A.get<int64_t>(nt + 1);
    if (!tasks || !dsz || !doff) return fail(SWX_ENOMEM, "device pool exhausted (traceback tasks)");
    HIP_TRY(hipMemsetAsync(dsz + nt, 0, 8, st));
    HIP_TRY(tb_tasks(pos, pos + nc, sorted, ta, bw, tasks, dsz, st));
    if ((rc = scan(ctx, dsz, doff, nt + 1))) return rc;
    HIP_TRY(tb_offsets(nt, tasks, doff, st));
    HIP_TRY(hipMemcpyAsync(totals + (c - 1), doff + nt, sizeof(int64_t), hipMemcpyDeviceToDevice, st));
    bands[nbands++] = BandPlan{tasks, nt, bw};
    pos += nc;
  }
  if (hc[5] > 0) {   // bands wider than 64 diagonals: row strips, columns swept
    const int64_t nc = hc[5];
    const int64_t nt = (nc + kTbwSlots - 1) / kTbwSlots;
    TbwTask *tasks = A.get<TbwTask>(nt);
    int64_t *dsz = A.get<int64_t>(nt + 1), *doff = A.get<int64_t>(nt + 1);
    int64_t *bsz = A.get<int64_t>(nt + 1), *boff = A.get<int64_t>(nt + 1);
    if (!tasks || !dsz || !doff || !bsz || !boff)
      return fail(SWX_ENOMEM, "device pool exhausted (wide traceback tasks)");
    HIP_TRY(hipMemsetAsync(dsz + nt, 0, 8, st));
    HIP_TRY(hipMemsetAsync(bsz + nt, 0, 8, st));
    HIP_TRY(tbw_tasks(pos, pos + nc, sorted, ta, tasks, dsz, bsz, st));
    if ((rc = scan(ctx, dsz, doff, nt + 1))) return rc;
    if ((rc = scan(ctx, bsz, boff, nt + 1))) return rc;
    HIP_TRY(tbw_offsets(nt, tasks, doff, boff, st));
    HIP_TRY(hipMemcpyAsync(totals + 3, doff + nt, sizeof(int64_t), hipMemcpyDeviceToDevice, st));
    HIP_TRY(hipMemcpyAsync(totals + 4, boff + nt, sizeof(int64_t), hipMemcpyDeviceToDevice, st));
    wtasks = tasks;
    wnt = nt;
    pos += nc;
  }
  std::vector<SideLaunch> launches;
  if (nbands > 0 || wnt > 0) {
    int64_t ht[5];
    if ((rc = read_i64(ctx, totals, ht, 5))) return rc;
    for (int k = 0; k < nbands; ++k) {
      const BandPlan bp = bands[k];
      const int64_t words = ht[(bp.bw == 8 ? 1 : bp.bw == 16 ? 2 : 3) - 1];
      TbArgs tc = ta;
      tc.dir = A.get<uint32_t>(words);
      if (!tc.dir) return fail(SWX_ENOMEM, "device pool exhausted (choice codes)");
      // measured time per cell alone on the device, relative: 8-wide bands
      // pay the most per-row overhead per cell, 16-wide the least
      const double per_cell = bp.bw == 8 ? 2.0 : (bp.bw == 16 ? 1.2 : 1.5);
      launches.push_back({(double)words * 8 * per_cell, [=](hipStream_t s_) {
                            return tb_band(tc, bp.tasks, bp.nt, sorted, bp.bw, s_);
                          }});
    }
    if (wnt > 0) {
      TbArgs tc = ta;
      tc.dir = A.get<uint32_t>(ht[3]);
      int32_t *bnd = A.get<int32_t>(ht[4]);
      if (!tc.dir || !bnd) return fail(SWX_ENOMEM, "device pool exhausted (wide band)");
      launches.push_back({(double)ht[3] * 8 * 1.7,
                          [=](hipStream_t s_) { return tb_strip(tc, wtasks, wnt, sorted, bnd, s_); },
                          true});
    }
  }
  if (hc[6] > 0) {   // long pairs with wide bands: one pair per wave
    const int64_t nc = hc[6];
    std::vector<int64_t> info;
    // gather_pairs fields: qbeg, rbeg, score, qend, rend
    if ((rc = gather_info(ctx, nc, sorted + pos, qbeg, rbeg, score, qend, rend, nullptr, info)))
      return rc;
    std::vector<int64_t> ids(nc);
    if ((rc = read_i64(ctx, sorted + pos, ids.data(), nc))) return rc;
    std::vector<TbWaveJob> jobs(nc);
    std::vector<TbShape> shape(nc);
    int64_t dbytes = 0, bwords = 0;
    for (int64_t k = 0; k < nc; ++k) {
      TbWaveJob &jb = jobs[k];
      jb.pair = ids[k];
      jb.m = info[6 * k + 3] - info[6 * k + 0] + 1;
      jb.w = info[6 * k + 4] - info[6 * k + 1] + 1;
      safe_band(jb.m, jb.w, info[6 * k + 2], sc.smax, sc.o, sc.e, &jb.dlo, &jb.bw);
      shape[k] = tb_wave_shape(jb.m, jb.w, jb.bw, sc.n, nc, ctx->cus);
      const int RL = shape[k].rl;
      if (RL == 0) return fail(SWX_EINVAL, "alignment too long for the wave traceback");
      const int64_t SH = 64 * RL, nstrips = (jb.m + SH - 1) / SH;
      jb.dir_off = dbytes;
      jb.bnd_off = bwords;
      for (int64_t st_ = 0; st_ < nstrips; ++st_) {
        int64_t clo, chi;
        tbw_window(st_, SH, jb.dlo, jb.bw, jb.w, &clo, &chi);
        dbytes += ((chi - clo) + 63) * 64 * tb_code_bytes(RL);
      }
      dbytes = round_up(dbytes, 256);
      bwords += 2 * (jb.w + 1) * (nstrips + 1);
    }
    // launch groups of equal shape
    std::vector<int64_t> order(nc);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int64_t x, int64_t y) { return shape[x] < shape[y]; });
    std::vector<TbWaveJob> sorted_jobs(nc);
    for (int64_t k = 0; k < nc; ++k) sorted_jobs[k] = jobs[order[k]];
    TbWaveJob *dj = A.get<TbWaveJob>(nc);
    uint8_t *dirw = A.get<uint8_t>(std::max<int64_t>(dbytes, 256));
    int32_t *bnd = A.get<int32_t>(std::max<int64_t>(bwords, 1));
    int64_t nspread = 0;
    for (int64_t k = 0; k < nc; ++k) nspread += shape[k].segs > 1 ? 1 : 0;
    IntraSync *sync = nspread ? A.get<IntraSync>(nspread) : nullptr;
    if (!dj || !dirw || !bnd || (nspread && !sync))
      return fail(SWX_ENOMEM, "device pool exhausted (wave traceback)");
    HIP_TRY(hipMemcpyAsync(dj, sorted_jobs.data(), sizeof(TbWaveJob) * nc, hipMemcpyHostToDevice, st));
    HIP_TRY(hipStreamSynchronize(st));   // the host job table must outlive the copy
    for (int64_t k0 = 0; k0 < nc;) {
      int64_t k1 = k0;
      while (k1 < nc && shape[order[k1]] == shape[order[k0]]) ++k1;
      const TbShape sh = shape[order[k0]];
      const TbWaveJob *jp = dj + k0;
      const int64_t cnt = k1 - k0;
      IntraSync *gs = nullptr;
      if (sh.segs > 1) {   // one progress record per spread pair
        gs = sync;
        sync += cnt;
      }
      launches.push_back({(double)dbytes * 32, [=](hipStream_t s_) {
                            return tb_wave(ta, jp, cnt, sh.rl, sh.waves, sh.segs, gs, dirw, bnd, s_);
                          }});
      k0 = k1;
    }
    pos += nc;
  }
  if ((rc = run_side_by_side(ctx, launches))) return rc;
  // final CIGAR offsets and compaction into the caller's arena
  int64_t *len64 = A.get<int64_t>(np + 1);
  if (!len64) return fail(SWX_ENOMEM, "device pool exhausted");
  HIP_TRY(hipMemsetAsync(len64 + np, 0, 8, st));
  HIP_TRY(lens_to_i64(np, cig_len, len64, st));
  if ((rc = scan(ctx, len64, cig_off_final, np + 1))) return rc;
  int64_t total = 0;
  if ((rc = read_i64(ctx, cig_off_final + np, &total))) return rc;
  out->cigar_used = total;
  if (total > out->cigar_cap || (total > 0 && !out->cigar)) {
    *flags &= ~SWX_CIGAR;   // records are still produced; CIGARs are not copied
    *rc_range = SWX_ERANGE;
    g_last_error = "CIGAR arena too small";
    return SWX_OK;
  }
  uint32_t *dst = out->cigar, *dtmp = nullptr;
  if (out->out_mem != SWX_MEM_DEVICE) {
    dtmp = A.get<uint32_t>(total);
    if (!dtmp) return fail(SWX_ENOMEM, "device pool exhausted");
    dst = dtmp;
  }
  HIP_TRY(launch_cigar_compact(np, cscr, coff, cig_len, cig_off_final, dst, st));
  if (dtmp && total)
    HIP_TRY(hipMemcpyAsync(out->cigar, dtmp, sizeof(uint32_t) * total, hipMemcpyDeviceToHost, st));
  return SWX_OK;
}

// ---- the pipeline -----------------------------------------------------------

// ---- long pairs: intra-sequence path ----------------------------------------
struct LongPath {
  int64_t nlong = 0, nshort = 0;
  int64_t *d_long = nullptr;    // long pair ids (device)
  int64_t *d_short = nullptr;   // short pair ids (device; null: every pair is short)
  std::vector<int64_t> ids;     // long pair ids (host)
  std::vector<int64_t> info;    // gather_pairs fields per long pair
  std::vector<IntraPair> pairs;
  IntraPair *d_pairs = nullptr;
  uint32_t *d_maxcol = nullptr;
  int32_t *d_part_v = nullptr;  // partial bests of the max-array reductions
  int64_t *d_part_j = nullptr;
};

// Rows per lane of the intra kernel: the fewest instruction slots per column,
// counting padded rows and about 20 instructions of per-step overhead.
static int pick_rl(int64_t rows, int n) {
  int best = 4;
  int64_t best_cost = INT64_MAX;
  for (int RL : {4, 8, 16, 32}) {
    if (intra_lds_bytes(n, RL) + intra_static_lds() > 65536) continue;
    const int64_t strips = (rows + 64 * RL - 1) / (64 * RL);
    const int64_t cost = strips * (12 * RL + 20);
    if (cost < best_cost) { best_cost = cost; best = RL; }
  }
  return best;
}

// Pairs above this many cells go to the intra-sequence path.  In the batched
// path a pair occupies one 16-bit lane half for cells * t; a full GPU holds
// about 2048 waves * 128 halves, so a pair larger than twice the batch's
// average work per half would finish last -- it is faster spread over a wave.
// A batch of few tasks runs each on four waves (cooperative strips), which
// shortens a task's time about four times.
static int64_t long_threshold(const swx_ctx *ctx, int64_t total_cells, int64_t npairs) {
  if (ctx->long_cells >= 0) return ctx->long_cells;
  const int64_t base = std::max<int64_t>(2048, 2 * total_cells / (2048 * 128));
  const int64_t tasks = (npairs + kSlots16 - 1) / kSlots16;
  return coop_waves(ctx->fill_coop, tasks, ctx->cus) > 1 ? base * kCoopWaves : base;
}

static int code_bits(int64_t rows_padded) {
  int k = 1;
  while ((int64_t(1) << k) < rows_padded) ++k;
  return k;
}

static int gather_info(swx_ctx *ctx, int64_t n, const int64_t *d_ids, const int32_t *qlen,
                       const int64_t *rlen, const int32_t *score, const int32_t *qend,
                       const int64_t *rend, const int32_t *band, std::vector<int64_t> &info) {
  int64_t *d = ctx->arena.get<int64_t>(6 * n);
  if (!d) return fail(SWX_ENOMEM, "device pool exhausted (gather)");
  HIP_TRY(gather_pairs(n, d_ids, qlen, rlen, score, qend, rend, band, d, ctx->stream));
  info.resize(6 * n);
  return read_i64(ctx, d, info.data(), 6 * n);
}

static int split_pairs(swx_ctx *ctx, int64_t np, const int32_t *qlen, const int64_t *rlen,
                       int64_t total_cells, LongPath &lp) {
  DevArena &A = ctx->arena;
  uint8_t *fl = A.get<uint8_t>(np), *fs = A.get<uint8_t>(np);
  if (!fl || !fs) return fail(SWX_ENOMEM, "device pool exhausted (split)");
  HIP_TRY(split_long(np, qlen, rlen, long_threshold(ctx, total_cells, np), ctx->long_rlen, fl, fs,
                     ctx->stream));
  int rc;
  if ((rc = select_flagged(ctx, fl, np, &lp.d_long, &lp.nlong))) return rc;
  lp.nshort = np - lp.nlong;
  if (lp.nlong == 0) return SWX_OK;
  if ((rc = select_flagged(ctx, fs, np, &lp.d_short, &lp.nshort))) return rc;
  lp.ids.resize(lp.nlong);
  if ((rc = read_i64(ctx, lp.d_long, lp.ids.data(), lp.nlong))) return rc;
  return gather_info(ctx, lp.nlong, lp.d_long, qlen, rlen, nullptr, nullptr, nullptr, nullptr,
                     lp.info);
}

// Most column chunks per pair of a graph's intra-sequence forward pass.
constexpr int64_t kGraphMaxChunks = 16;

// Waves per workgroup of an intra job: one per strip, within the LDS budget
// (a profile of (n + 1) * 64 * RL bytes per wave) and the kernel's maximum.
static int intra_waves(int64_t nstrips, int n, int RL) {
  const int64_t per = (int64_t)intra_lds_bytes(n, RL);
  const int64_t room = (65536 - (int64_t)intra_static_lds()) / per;
  int64_t w = std::min<int64_t>({nstrips, (int64_t)intra_max_waves(), room});
  return (int)std::max<int64_t>(w, 1);
}

// Waves per workgroup of a 16-bit job pair (two profiles per wave in LDS).
static int intra_waves16(int64_t nstrips, int n, int RL) {
  const int64_t per = (int64_t)intra_lds_bytes16(n, RL);
  const int64_t room = (65536 - 4096) / per;
  int64_t w = std::min<int64_t>({nstrips, (int64_t)intra_max_waves(), room});
  return (int)std::max<int64_t>(w, 1);
}

// Widest span of a positive-scoring path (the warm-up of every chunk of a
// long pair): the reference length when gaps cost nothing to extend.
static int64_t intra_warmup(const Scoring &sc, int64_t Lq, int64_t Lr) {
  if (sc.e <= 0) return Lr;
  return Lq + std::max<int64_t>((int64_t)sc.smax * Lq - sc.o, 0) / sc.e + 1;
}

// Column chunk width of a long pair: its share (by reference length) of
// `target` chunks over all long pairs, at least 256 columns and half the
// warm-up, and the whole reference when the warm-up spans it.
static int64_t intra_chunk(const Scoring &sc, int64_t Lq, int64_t Lr, int64_t target,
                           int64_t total_r) {
  const int64_t W = intra_warmup(sc, Lq, Lr);
  if (W >= Lr) return std::max<int64_t>(Lr, 1);
  const int64_t want = std::max<int64_t>(1, target * Lr / std::max<int64_t>(total_r, 1));
  const int64_t C = (Lr + want - 1) / want;
  return std::max<int64_t>(C, std::max<int64_t>(256, W / 2));
}

// Packed 16-bit lanes hold a long pair when no score can pass 2^15 - 2 (the
// a-priori bound smax * min(qlen, rlen) with the bias added on the way: T6)
// and its padded height fits a 16-bit row code.
static bool intra_fits16(const Scoring &sc, int64_t Lq, int64_t Lr, int RL) {
  const int64_t bound = (int64_t)std::max(sc.smax, 0) * std::min(Lq, Lr);
  return bound + sc.bias <= 32766 && round_up(Lq, 64 * RL) <= 65536;
}

// Largest 16-bit lane value for which the packed f16 three-way maximum is the
// unsigned maximum (0x7C00 and above are f16 infinities and NaNs).
static constexpr int64_t kMax3Lane = 0x7BFF;

// 16-bit waves per compute unit from which the automatic choice takes them.
static constexpr int64_t kIntra16MinWavesPerCu = 4;

// Launch shape of intra-sequence jobs: rows per lane, waves per workgroup and
// workgroups per job (segs > 1: the job's strips spread over that many).
struct IntraShape {
  int rl, waves, segs;
  bool operator<(const IntraShape &o) const {
    return std::tie(rl, waves, segs) < std::tie(o.rl, o.waves, o.segs);
  }
};
typedef std::map<IntraShape, std::vector<IntraJob>> IntraGroups;

// Shape of a job of `rows` query rows over `width` columns (band >= 0: the
// reversed pass's strip windows, SH + 2 * band wide and SH apart) when `jobs`
// such jobs share the device.  With at least one job per compute unit the
// device is full: the fewest instructions over all strips (pick_rl).  With
// fewer, a job is as slow as its longer of two paths: the chain of strips,
// each starting about 128 columns (banded: SH + 128) after the one above, and
// the strips each wave runs in turn; a step costs about 12 instructions per
// row of a lane plus 20.  Those jobs spread over up to four waves per
// workgroup (one per SIMD) and as many workgroups as fit at once: at most one
// per compute unit, and 32 (the compute units of one XCD) per XCD.
static IntraShape intra_shape(int64_t rows, int64_t width, int32_t band, int n, int64_t jobs,
                              int32_t cus) {
  jobs = std::max<int64_t>(jobs, 1);
  if (jobs >= cus || cus <= 0) {
    const int RL = pick_rl(rows, n);
    return {RL, intra_waves((rows + 64 * RL - 1) / (64 * RL), n, RL), 1};
  }
  const int64_t segs_max =
      std::max<int64_t>(1, std::min<int64_t>(cus / jobs, 32 / ((jobs + 7) / 8)));
  IntraShape best{pick_rl(rows, n), 1, 1};
  double best_cost = -1;
  for (int RL : {4, 8, 16, 32}) {
    if (intra_lds_bytes(n, RL) + intra_static_lds() > 65536) continue;
    const int64_t SH = 64 * RL;
    const int64_t nstrips = std::max<int64_t>(1, (rows + SH - 1) / SH);
    if (nstrips > intra_max_strips()) continue;
    int64_t nw = std::min<int64_t>(4, intra_waves(nstrips, n, RL));
    const int64_t g = std::min<int64_t>(segs_max, (nstrips + nw - 1) / nw);
    if (g == 1) nw = intra_waves(nstrips, n, RL);
    const int64_t win = band >= 0 ? std::min<int64_t>(width, SH + 2 * (int64_t)band) : width;
    const int64_t lag = (band >= 0 ? SH : 0) + 128;
    const int64_t tw = g * nw;
    const int64_t chain = (nstrips - 1) * lag + win;
    const int64_t turns = (nstrips + tw - 1) / tw * (win + 63);
    // two waves share a SIMD beyond four per workgroup
    const double cost = (double)std::max(chain, turns) * (12 * RL + 20) * (nw > 4 ? 1.5 : 1.0);
    if (best_cost < 0 || cost < best_cost) {
      best_cost = cost;
      best = {RL, (int)nw, (int)g};
    }
  }
  return best;
}

// 16-bit forward jobs keyed by (rows per lane, strips): jobs of one key share
// their padded height, so any two of them can share a wave.
typedef std::map<std::pair<int, int64_t>, std::vector<IntraJob>> Jobs16;

// Upload the 16-bit jobs (each key's list padded to an even count with an
// empty job) and launch them, a pair of jobs per workgroup.
static int launch_intra16_jobs(swx_ctx *ctx, const Jobs16 &jobs, IntraArgs a, const Scoring &sc,
                               bool m3) {
  if (jobs.empty()) return SWX_OK;
  std::vector<IntraJob> all;
  std::vector<std::pair<int64_t, int64_t>> span;   // per key: first job, count
  for (const auto &kv : jobs) {
    const int64_t first = (int64_t)all.size();
    all.insert(all.end(), kv.second.begin(), kv.second.end());
    if (all.size() & 1) {
      IntraJob none{};
      none.pair = -1;
      all.push_back(none);
    }
    span.push_back({first, (int64_t)all.size() - first});
  }
  IntraJob *dj = ctx->arena.get<IntraJob>((int64_t)all.size());
  if (!dj) return fail(SWX_ENOMEM, "device pool exhausted (intra jobs)");
  HIP_TRY(hipMemcpyAsync(dj, all.data(), sizeof(IntraJob) * all.size(), hipMemcpyHostToDevice,
                         ctx->stream));
  size_t k = 0;
  for (const auto &kv : jobs) {
    const int RL = kv.first.first;
    a.jobs = dj + span[k].first;
    a.njobs = span[k].second;
    HIP_TRY(intra_fill16(a, RL, intra_waves16(kv.first.second, sc.n, RL), m3, ctx->stream));
    ++k;
  }
  HIP_TRY(hipStreamSynchronize(ctx->stream));   // the host job table must outlive the copy
  return SWX_OK;
}

// Upload jobs (grouped by launch shape) and launch them; bnd: the hand-over
// rows (null: allocated here, bnd_words of them).
static int launch_intra_jobs(swx_ctx *ctx, const IntraGroups &groups, IntraArgs a,
                             int64_t bnd_words, bool rev) {
  DevArena &A = ctx->arena;
  std::vector<IntraJob> all;
  int64_t nspread = 0;
  for (const auto &kv : groups) {
    all.insert(all.end(), kv.second.begin(), kv.second.end());
    if (kv.first.segs > 1) nspread += (int64_t)kv.second.size();
  }
  if (all.empty()) return SWX_OK;
  IntraJob *dj = A.get<IntraJob>((int64_t)all.size());
  IntraSync *sync = nspread ? A.get<IntraSync>(nspread) : nullptr;
  if (!a.bnd) a.bnd = A.get<uint32_t>(bnd_words > 0 ? bnd_words : 1);
  if (!dj || !a.bnd || (nspread && !sync))
    return fail(SWX_ENOMEM, "device pool exhausted (intra jobs)");
  HIP_TRY(hipMemcpyAsync(dj, all.data(), sizeof(IntraJob) * all.size(), hipMemcpyHostToDevice,
                         ctx->stream));
  if (nspread) HIP_TRY(intra_sync_init(sync, nspread, ctx->stream));
  int64_t off = 0, soff = 0;
  for (const auto &kv : groups) {
    a.jobs = dj + off;
    a.njobs = (int64_t)kv.second.size();
    a.segs = kv.first.segs;
    a.sync = kv.first.segs > 1 ? sync + soff : nullptr;
    HIP_TRY(intra_fill(a, kv.first.rl, kv.first.waves, rev, ctx->stream));
    off += a.njobs;
    if (kv.first.segs > 1) soff += a.njobs;
  }
  // the host job table must outlive the copy
  HIP_TRY(hipStreamSynchronize(ctx->stream));
  return SWX_OK;
}

// Forward pass of the long pairs: column chunks with a warm-up overlap, the
// encoded max array per pair, then the end (T1) of each pair.
static int run_intra_forward(swx_ctx *ctx, const Scoring &sc, LongPath &lp, const PairView &view,
                             const FillOut &out, uint8_t *err, uint8_t *lanebits) {
  DevArena &A = ctx->arena;
  int64_t total_r = 0;
  for (int64_t k = 0; k < lp.nlong; ++k) total_r += std::max<int64_t>(lp.info[6 * k + 1], 1);
  Jobs16 jobs16;
  std::vector<int64_t> ids16, ids32;
  lp.pairs.clear();
  // Packed 16-bit lanes run two chunks per wave, with half the waves per
  // workgroup (two profiles each in LDS), on twice the chunk target. Chosen
  // automatically only when those waves still cover every SIMD of the device:
  // a few long pairs in few chunks finish sooner on 32-bit lanes.
  bool auto16 = false;
  if (ctx->intra_bits == 0) {
    std::map<std::pair<int, int64_t>, int64_t> count;
    for (int64_t k = 0; k < lp.nlong; ++k) {
      const int64_t Lq = lp.info[6 * k], Lr = lp.info[6 * k + 1];
      const int RL = pick_rl(Lq, sc.n);
      if (Lr == 0 || !intra_fits16(sc, Lq, Lr, RL)) continue;
      const int64_t C = intra_chunk(sc, Lq, Lr, 2 * ctx->intra_jobs, total_r);
      count[{RL, round_up(Lq, 64 * RL) / (64 * RL)}] += (Lr + C - 1) / C;
    }
    int64_t waves = 0;
    for (const auto &kv : count)
      waves += (kv.second + 1) / 2 * intra_waves16(kv.first.second, sc.n, kv.first.first);
    auto16 = waves >= kIntra16MinWavesPerCu * (int64_t)ctx->cus;
  }
  // lanes of each pair, and the 32-bit jobs that will share the device
  std::vector<uint8_t> is16(lp.nlong);
  int64_t jobs32 = 0;
  for (int64_t k = 0; k < lp.nlong; ++k) {
    const int64_t Lq = lp.info[6 * k], Lr = lp.info[6 * k + 1];
    is16[k] = (ctx->intra_bits == 16 || auto16) && intra_fits16(sc, Lq, Lr, pick_rl(Lq, sc.n));
    if (!is16[k] && Lr > 0) {
      const int64_t C = intra_chunk(sc, Lq, Lr, ctx->intra_jobs, total_r);
      jobs32 += (Lr + C - 1) / C;
    }
  }
  IntraGroups groups;
  int64_t mc_words = 0, bnd_words = 0;
  bool m3 = true;   // every 16-bit pair's lane values below 0x7C00
  for (int64_t k = 0; k < lp.nlong; ++k) {
    const int64_t p = lp.ids[k], Lq = lp.info[6 * k], Lr = lp.info[6 * k + 1];
    const bool w16 = is16[k];
    const int64_t W = intra_warmup(sc, Lq, Lr);
    const int64_t C = intra_chunk(sc, Lq, Lr, (w16 ? 2 : 1) * ctx->intra_jobs, total_r);
    const IntraShape shape = w16 ? IntraShape{pick_rl(Lq, sc.n), 0, 1}
                                 : intra_shape(Lq, std::min(Lr, C + W), -1, sc.n, jobs32, ctx->cus);
    const int RL = shape.rl;
    const int64_t SH = 64 * RL;
    const int64_t qp = (Lq + SH - 1) / SH * SH;
    const int64_t bound = (int64_t)std::max(sc.smax, 0) * std::min(Lq, Lr);
    const int kb = w16 ? 16 : code_bits(qp);
    if (kb > 30 || bound >= (int64_t(1) << (32 - kb)))
      return fail(SWX_EOVERFLOW, "long pair: score range and query length exceed the max-array word");
    (w16 ? ids16 : ids32).push_back(p);
    if (w16 && bound + sc.bias > kMax3Lane) m3 = false;
    IntraPair ip{p, mc_words, kb, (int32_t)SH};
    lp.pairs.push_back(ip);
    if (Lr > 0) {
      const int64_t nstrips = qp / SH;
      if (nstrips > intra_max_strips())
        return fail(SWX_EINVAL, "query too long for the intra-sequence path");
      for (int64_t c0 = 0; c0 < Lr; c0 += C) {
        IntraJob jb{};
        jb.pair = p;
        jb.c0 = c0;
        jb.c1 = std::min(Lr, c0 + C);
        jb.cw = std::max<int64_t>(0, c0 - W);
        jb.mc_off = mc_words;
        jb.bnd_off = bnd_words;
        jb.kbits = kb;
        jb.band = -1;
        bnd_words += 2 * (jb.c1 - jb.cw) * (nstrips - 1);
        if (w16) jobs16[{RL, nstrips}].push_back(jb);
        else groups[shape].push_back(jb);
      }
    }
    mc_words += Lr;
  }
  lp.d_maxcol = A.get<uint32_t>(std::max<int64_t>(mc_words, 1));
  if (lp.d_maxcol && mc_words > 0)
    HIP_TRY(hipMemsetAsync(lp.d_maxcol, 0, sizeof(uint32_t) * mc_words, ctx->stream));
  lp.d_pairs = A.get<IntraPair>(lp.nlong);
  lp.d_part_v = A.get<int32_t>(lp.nlong * intra_slices());
  lp.d_part_j = A.get<int64_t>(lp.nlong * intra_slices());
  if (!lp.d_maxcol || !lp.d_pairs || !lp.d_part_v || !lp.d_part_j)
    return fail(SWX_ENOMEM, "device pool exhausted (max array)");
  HIP_TRY(hipMemcpyAsync(lp.d_pairs, lp.pairs.data(), sizeof(IntraPair) * lp.nlong,
                         hipMemcpyHostToDevice, ctx->stream));
  IntraArgs a{};
  a.view = view;
  a.matrix = sc.dmat;
  a.n = sc.n; a.o = sc.o; a.e = sc.e; a.bias = sc.bias;
  a.maxcol = lp.d_maxcol;
  a.err = err;
  a.bnd = A.get<uint32_t>(bnd_words > 0 ? bnd_words : 1);
  if (!a.bnd) return fail(SWX_ENOMEM, "device pool exhausted (hand-over rows)");
  int rc;
  if ((rc = launch_intra_jobs(ctx, groups, a, bnd_words, false))) return rc;
  if ((rc = launch_intra16_jobs(ctx, jobs16, a, sc, m3))) return rc;
  // lane widths of the long pairs (diagnostic)
  for (int w = 0; w < 2; ++w) {
    const std::vector<int64_t> &ids = w ? ids32 : ids16;
    if (ids.empty()) continue;
    int64_t *d = A.get<int64_t>((int64_t)ids.size());
    if (!d) return fail(SWX_ENOMEM, "device pool exhausted (lane widths)");
    HIP_TRY(hipMemcpyAsync(d, ids.data(), 8 * ids.size(), hipMemcpyHostToDevice, ctx->stream));
    HIP_TRY(mark_lanes((int64_t)ids.size(), d, lanebits, w ? 32 : 16, ctx->stream));
    HIP_TRY(hipStreamSynchronize(ctx->stream));   // the host list must outlive the copy
  }
  IntraPairArgs e{};
  e.pairs = lp.d_pairs; e.maxcol = lp.d_maxcol; e.qlen = view.qlen; e.rlen = view.rlen;
  e.score = out.score; e.qend = out.qend; e.rend = out.rend; e.overflow = out.overflow;
  e.part_v = lp.d_part_v; e.part_j = lp.d_part_j;
  HIP_TRY(intra_end(e, lp.nlong, ctx->stream));
  return SWX_OK;
}

// Reversed pass of the long pairs with a positive score: one job per pair.
static int run_intra_reverse(swx_ctx *ctx, const Scoring &sc, LongPath &lp, const PairView &rview,
                             const int32_t *score, const int32_t *qend, const int64_t *rend,
                             const int32_t *band, const int32_t *tgt, const FillOut &rout,
                             uint8_t *err) {
  std::vector<int64_t> info;
  int rc;
  if ((rc = gather_info(ctx, lp.nlong, lp.d_long, nullptr, nullptr, score, qend, rend, band, info)))
    return rc;
  IntraGroups groups;
  int64_t bnd_words = 0, njobs = 0;
  for (int64_t k = 0; k < lp.nlong; ++k) njobs += info[6 * k + 2] > 0;
  for (int64_t k = 0; k < lp.nlong; ++k) {
    if (info[6 * k + 2] <= 0) continue;
    const int64_t rows = info[6 * k + 3] + 1, cols = info[6 * k + 4] + 1;
    const IntraShape shape =
        intra_shape(rows, cols, (int32_t)info[6 * k + 5], sc.n, njobs, ctx->cus);
    const int RL = shape.rl;
    const int64_t SH = 64 * RL;
    const int64_t qp = (rows + SH - 1) / SH * SH;
    const int kb = code_bits(qp);
    if (kb > 30 || info[6 * k + 2] >= (int64_t(1) << (32 - kb)))
      return fail(SWX_EOVERFLOW, "long pair: score range and query length exceed the max-array word");
    const int64_t nstrips = qp / SH;
    if (nstrips > intra_max_strips())
      return fail(SWX_EINVAL, "query too long for the intra-sequence path");
    IntraJob jb{};
    jb.pair = lp.ids[k];
    jb.cw = 0; jb.c0 = 0; jb.c1 = cols;
    jb.mc_off = 0;
    jb.bnd_off = bnd_words;
    jb.kbits = kb;
    jb.band = (int32_t)info[6 * k + 5];
    bnd_words += 2 * cols * (nstrips - 1);
    groups[shape].push_back(jb);
  }
  IntraArgs a{};
  a.view = rview;
  a.matrix = sc.dmat;
  a.n = sc.n; a.o = sc.o; a.e = sc.e; a.bias = sc.bias;
  a.maxcol = nullptr;
  a.target = tgt;
  a.out = rout;
  a.err = err;
  return launch_intra_jobs(ctx, groups, a, bnd_words, true);
}

static int run_pipeline(swx_ctx *ctx, const Scoring &sc, const DeviceBatch &b, uint32_t flags,
                        int32_t mask_len, swx_batch_out *out, const swx_profile *prof) {
  DevArena &A = ctx->arena;
  hipStream_t st = ctx->stream;
  const int64_t np = b.npairs;
  if (flags & SWX_SUBOPT) flags |= SWX_ALL;
  if (flags & (SWX_CIGAR | SWX_SCORE2)) flags |= SWX_BEGIN;
  int rc;
  HIP_TRY(hipEventRecord(ctx->ev[0], st));

  // validation (before any alignment work)
  uint32_t *d_bad = A.get<uint32_t>(1);
  if (!d_bad) return fail(SWX_ENOMEM, "device pool exhausted");
  HIP_TRY(hipMemsetAsync(d_bad, 0, sizeof(uint32_t), st));
  ValidateArgs va{b.qcat, b.qcat_len, b.qoff, b.nq, b.rcat, b.rcat_len, b.roff, b.nr,
                  b.pair_q, b.pair_r, np, sc.n, d_bad};
  HIP_TRY(launch_validate(va, st));
  uint32_t bad = 0;
  HIP_TRY(hipMemcpyAsync(ctx->pinned, d_bad, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
  HIP_TRY(wait_stream(st));
  memcpy(&bad, ctx->pinned, sizeof(uint32_t));
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
  int64_t *stats = A.get<int64_t>(4);
  if (!qstart || !rstart || !rlen || !qlen || !score || !qend || !rend || !ovf || !lanebits ||
      !err || !qbeg || !score2 || !rbeg || !rend2 || !stats)
    return fail(SWX_ENOMEM, "device pool exhausted (pair arrays)");
  HIP_TRY(hipMemsetAsync(err, 0, np, st));
  HIP_TRY(hipMemsetAsync(lanebits, 16, np, st));
  {
    const ViewCaps vc{b.nq, b.nr, b.qcat_len, b.rcat_len, INT32_MAX, 0, INT64_MAX};
    HIP_TRY(launch_views(np, b.qoff, b.roff, b.pair_q, b.pair_r, vc, qstart, qlen, rstart, rlen,
                         st));
  }
  // a score can reach smax * min(qlen, rlen); the 32-bit lanes hold < 2^26
  HIP_TRY(hipMemsetAsync(stats, 0, 8 * 4, st));
  HIP_TRY(launch_pair_stats(np, qlen, rlen, stats, st));
  int64_t hstats[4];
  if ((rc = read_i64(ctx, stats, hstats, 4))) return rc;
  const int64_t score_bound = (int64_t)std::max(sc.smax, 0) * hstats[0];
  if (score_bound >= (1 << 26) - 1)
    return fail(SWX_EOVERFLOW, "a score could exceed the 32-bit lane range");
  PairView fview{qstart, rstart, qlen, rlen, b.qcat, b.rcat, 0};
  FillOut fout{score, qend, rend, ovf, err};

  // 24-row strips exist for the 4-symbol selector profile only
  const int R = (ctx->fill_rows == 24 && !sc.qsel) ? 32 : ctx->fill_rows;
  // every pair on one query (general alphabets): the query profile is built
  // once (or comes resident with the caller's profile) and every batched
  // pass reads it, instead of profile bytes per task
  SharedProf shp;
  const SharedProf *sp = nullptr;
  if (!sc.qsel && b.nq == 1) {
    if (prof && prof->dev) {
      shp.fwd = R == 32 ? prof->fwd32 : prof->fwd16;
      shp.fwd_row = R == 32 ? prof->qp32 : prof->qp16;
      shp.rev = prof->rev;
      shp.rev_row = prof->rev_row;
      shp.qlen = (int32_t)prof->query.size();
    } else {
      int64_t qo[2];
      HIP_TRY(hipMemcpyAsync(ctx->pinned, b.qoff, 16, hipMemcpyDeviceToHost, st));
      HIP_TRY(wait_stream(st));
      memcpy(qo, ctx->pinned, 16);
      const int64_t ql = qo[1] - qo[0];
      if (ql < 1 || ql > INT32_MAX / 4) return fail(SWX_EINVAL, "bad query length");
      shp.qlen = (int32_t)ql;
      shp.fwd_row = round_up(ql, R);
      shp.rev_row = qprof_rev_row(ql, 32);
      uint8_t *fw = A.get<uint8_t>((sc.n + 1) * shp.fwd_row);
      uint8_t *rv = A.get<uint8_t>(16 * (sc.n + 1) * shp.rev_row);
      if (!fw || !rv) return fail(SWX_ENOMEM, "device pool exhausted (query profile)");
      HIP_TRY(build_qprof(b.qcat + qo[0], shp.qlen, sc.dmat, sc.n, sc.bias, (int32_t)shp.fwd_row, fw,
                          shp.rev_row, rv, st));
      shp.fwd = fw;
      shp.rev = rv;
    }
    shp.R = R;
    sp = &shp;
  }

  // long pairs take the intra-sequence path, the rest the batched one
  LongPath lp;
  if ((rc = split_pairs(ctx, np, qlen, rlen, hstats[1], lp))) return rc;

  // forward fill, 16-bit lanes (events 1 and 2 bracket the fill kernels)
  Plan p16, p32;
  if ((rc = plan_pass(ctx, sc, lp.d_short, lp.nshort, qlen, rlen, nullptr, nullptr, 16, R, p16, sp)))
    return rc;
  // With both kinds of pairs, the long pairs' pass runs on a side stream
  // beside the batched one (each ends on its own largest tasks, the other
  // fills the device meanwhile; the outputs are disjoint).
  const bool beside = lp.nlong > 0 && p16.ntasks > 0 && have_side_streams(ctx);
  if (beside) {
    HIP_TRY(hipEventRecord(ctx->fork_ev, st));
    HIP_TRY(hipStreamWaitEvent(ctx->aux[0], ctx->fork_ev, 0));
  }
  if ((rc = run_fill(ctx, p16, sc, fview, false, nullptr, fout, score_bound, 1, 0, 0, sp))) return rc;
  if (lp.nlong > 0) {
    if (beside) {
      {
        StreamScope on_side(ctx, ctx->aux[0]);   // the pass's launches and waits go there
        rc = run_intra_forward(ctx, sc, lp, fview, fout, err, lanebits);
      }
      if (rc) {   // nothing of the call may still run when it returns
        (void)hipStreamSynchronize(ctx->aux[0]);
        return rc;
      }
      HIP_TRY(hipEventRecord(ctx->join_ev[0], ctx->aux[0]));
      HIP_TRY(hipStreamWaitEvent(st, ctx->join_ev[0], 0));
    } else if ((rc = run_intra_forward(ctx, sc, lp, fview, fout, err, lanebits))) {
      return rc;
    }
    HIP_TRY(hipEventRecord(ctx->ev[2], st));
  }

  // saturated pairs: exact re-run on 32-bit lanes
  int64_t *wide = nullptr, nwide = 0;
  if ((rc = select_flagged(ctx, ovf, np, &wide, &nwide))) return rc;
  if (nwide > 0) {
    if ((rc = plan_pass(ctx, sc, wide, nwide, qlen, rlen, nullptr, nullptr, 32, R, p32, sp))) return rc;
    if ((rc = run_fill(ctx, p32, sc, fview, false, nullptr, fout, score_bound, -1, 0, 0, sp))) return rc;
    HIP_TRY(mark_lanes(nwide, wide, lanebits, 32, st));
  }
  HIP_TRY(hipEventRecord(ctx->ev[3], st));

  // reversed pass: begin
  if (flags & SWX_BEGIN) {
    int64_t *rqs = A.get<int64_t>(np), *rrs = A.get<int64_t>(np), *rrl = A.get<int64_t>(np);
    int32_t *rql = A.get<int32_t>(np), *tgt = A.get<int32_t>(np), *band = A.get<int32_t>(np);
    int32_t *band_q = A.get<int32_t>(np), *rsc = A.get<int32_t>(np), *rqe = A.get<int32_t>(np);
    int64_t *rre = A.get<int64_t>(np);
    uint8_t *rov = A.get<uint8_t>(np), *f16 = A.get<uint8_t>(np), *f32 = A.get<uint8_t>(np);
    if (!rqs || !rrs || !rrl || !rql || !tgt || !band || !band_q || !rsc || !rqe || !rre || !rov ||
        !f16 || !f32)
      return fail(SWX_ENOMEM, "device pool exhausted (reverse)");
    HIP_TRY(launch_rev_views(np, qstart, rstart, qlen, rlen, score, qend, rend, rqs, rql, rrs,
                             rrl, tgt, err, st));
    HIP_TRY(rev_prepare(np, score, qend, rend, lanebits, sc.smax, sc.o, sc.e, band, band_q, f16,
                        f32, st));
    if (lp.nlong > 0) HIP_TRY(clear_flags(lp.nlong, lp.d_long, f16, f32, st));
    HIP_TRY(hipMemsetAsync(rsc, 0, sizeof(int32_t) * np, st));
    PairView rview{rqs, rrs, rql, rrl, b.qcat, b.rcat, 1};
    FillOut rout{rsc, rqe, rre, rov, err};
    // both lane widths' pair lists first, their counts in one read, so that
    // no read waits for a queued fill
    int64_t *rids[2] = {nullptr, nullptr}, rcnt[2] = {0, 0};
    const int64_t *rcd[2] = {nullptr, nullptr};
    int64_t *rc2 = A.get<int64_t>(2);
    if (!rc2) return fail(SWX_ENOMEM, "device pool exhausted (reverse counts)");
    for (int k = 0; k < 2; ++k) {
      if ((rc = select_flagged_dev(ctx, k == 0 ? f16 : f32, np, &rids[k], &rcd[k]))) return rc;
      HIP_TRY(hipMemcpyAsync(rc2 + k, rcd[k], sizeof(int64_t), hipMemcpyDeviceToDevice, st));
    }
    if ((rc = read_i64(ctx, rc2, rcnt, 2))) return rc;
    // as in the forward pass, the long pairs' reversed pass runs on a side
    // stream beside the batched one (16-bit lanes)
    const bool beside = lp.nlong > 0 && rcnt[0] > 0 && have_side_streams(ctx);
    bool long_done = false;
    for (int k = 0; k < 2; ++k) {
      if (rcnt[k] == 0) continue;
      Plan pr;
      if ((rc = plan_pass(ctx, sc, rids[k], rcnt[k], rql, rrl, band, band_q, k == 0 ? 16 : 32, R, pr,
                          sp)))
        return rc;
      if (k == 0 && beside) {
        HIP_TRY(hipEventRecord(ctx->fork_ev, st));
        HIP_TRY(hipStreamWaitEvent(ctx->aux[0], ctx->fork_ev, 0));
      }
      if ((rc = run_fill(ctx, pr, sc, rview, true, tgt, rout, score_bound, -1, 0, 0, sp))) return rc;
      if (k == 0 && beside) {
        {
          StreamScope on_side(ctx, ctx->aux[0]);
          rc = run_intra_reverse(ctx, sc, lp, rview, score, qend, rend, band, tgt, rout, err);
        }
        if (rc) {   // nothing of the call may still run when it returns
          (void)hipStreamSynchronize(ctx->aux[0]);
          return rc;
        }
        HIP_TRY(hipEventRecord(ctx->join_ev[0], ctx->aux[0]));
        long_done = true;
      }
    }
    if (long_done) {
      HIP_TRY(hipStreamWaitEvent(st, ctx->join_ev[0], 0));
    } else if (lp.nlong > 0 &&
               (rc = run_intra_reverse(ctx, sc, lp, rview, score, qend, rend, band, tgt, rout, err))) {
      return rc;
    }
    HIP_TRY(launch_begins(np, score, qend, rend, rsc, rqe, rre, qbeg, rbeg, err, st));
  }
  HIP_TRY(hipEventRecord(ctx->ev[4], st));

  // banded traceback: CIGAR
  int64_t *cig_off_final = A.get<int64_t>(np + 1);
  int32_t *cig_len = A.get<int32_t>(np);
  if (!cig_off_final || !cig_len) return fail(SWX_ENOMEM, "device pool exhausted");
  HIP_TRY(hipMemsetAsync(cig_len, 0, sizeof(int32_t) * np, st));
  HIP_TRY(hipMemsetAsync(cig_off_final, 0, sizeof(int64_t) * (np + 1), st));
  int rc_range = SWX_OK;
  if (flags & SWX_CIGAR) {
    if ((rc = run_traceback(ctx, sc, b, np, score, qbeg, qend, rbeg, rend, qstart, rstart, qlen,
                            rlen, cig_len, cig_off_final, err, out, &flags, &rc_range)))
      return rc;
  } else {
    out->cigar_used = 0;
  }
  HIP_TRY(hipEventRecord(ctx->ev[5], st));

  // score2 from the max array (final CM plane of the forward tasks)
  if (flags & SWX_SCORE2) {
    Score2InterArgs s2{};
    s2.rlen = rlen; s2.qlen = qlen; s2.score1 = score; s2.rbeg = rbeg; s2.rend = rend;
    s2.mask_len = mask_len; s2.score2 = score2; s2.rend2 = rend2;
    s2.tasks = p16.d_tasks; s2.ntasks = p16.ntasks; s2.slot_pair = p16.d_sorted;
    s2.bnd = p16.d_bnd; s2.halves = 2;
    HIP_TRY(launch_score2_inter(s2, st));
    if (p32.ntasks) {
      s2.tasks = p32.d_tasks; s2.ntasks = p32.ntasks; s2.slot_pair = p32.d_sorted;
      s2.bnd = p32.d_bnd; s2.halves = 1;
      HIP_TRY(launch_score2_inter(s2, st));
    }
    if (lp.nlong > 0) {
      IntraPairArgs e{};
      e.pairs = lp.d_pairs; e.maxcol = lp.d_maxcol; e.qlen = qlen; e.rlen = rlen;
      e.score = score; e.qend = qend; e.rend = rend; e.rbeg = rbeg;
      e.mask_len = mask_len; e.score2 = score2; e.rend2 = rend2;
      e.part_v = lp.d_part_v; e.part_j = lp.d_part_j;
      HIP_TRY(intra_score2(e, lp.nlong, st));
    }
  }
  HIP_TRY(hipEventRecord(ctx->ev[6], st));

  // The suboptimal alignment behind score2: its end row (a forward pass over
  // a window of the reference ending at ref_end2, best taken in the last
  // column only), its begin (the reversed pass anchored at that end, on
  // 32-bit lanes offset by kAnchor so that only alignments starting at the
  // anchor cell can reach the target), its CIGAR (the banded traceback),
  // placed in the arena after every primary CIGAR.
  if (flags & SWX_SUBOPT) {
    constexpr uint32_t kAnchor = 1u << 25;
    if (score_bound >= (int64_t(1) << 24))
      return fail(SWX_EOVERFLOW, "scores too large for the suboptimal alignment's anchored pass");
    int64_t *wrs = A.get<int64_t>(np), *wrl = A.get<int64_t>(np), *wre = A.get<int64_t>(np);
    int32_t *wsc = A.get<int32_t>(np), *wqe = A.get<int32_t>(np);
    uint8_t *wov = A.get<uint8_t>(np), *sfl = A.get<uint8_t>(np), *slb = A.get<uint8_t>(np);
    int64_t *rqs = A.get<int64_t>(np), *rrs = A.get<int64_t>(np), *rrl = A.get<int64_t>(np);
    int32_t *rql = A.get<int32_t>(np), *tgt = A.get<int32_t>(np), *rsc = A.get<int32_t>(np);
    int32_t *rqe = A.get<int32_t>(np);
    int64_t *rre = A.get<int64_t>(np);
    uint8_t *rov = A.get<uint8_t>(np);
    int32_t *s_score = A.get<int32_t>(np), *s_qbeg = A.get<int32_t>(np), *s_qend = A.get<int32_t>(np);
    int64_t *s_rbeg = A.get<int64_t>(np), *s_rend = A.get<int64_t>(np);
    int32_t *s_cig_len = A.get<int32_t>(np);
    int64_t *s_cig_off = A.get<int64_t>(np + 1);
    if (!wrs || !wrl || !wre || !wsc || !wqe || !wov || !sfl || !slb || !rqs || !rrs || !rrl ||
        !rql || !tgt || !rsc || !rqe || !rre || !rov || !s_score || !s_qbeg || !s_qend ||
        !s_rbeg || !s_rend || !s_cig_len || !s_cig_off)
      return fail(SWX_ENOMEM, "device pool exhausted (suboptimal)");
    HIP_TRY(launch_sub_window(np, rstart, qlen, score2, rend2, sc.smax, sc.o, sc.e, wrs, wrl, sfl,
                              st));
    HIP_TRY(hipMemsetAsync(wsc, 0, sizeof(int32_t) * np, st));
    HIP_TRY(hipMemsetAsync(wqe, 0xFF, sizeof(int32_t) * np, st));
    int64_t *ids = nullptr, cnt = 0;
    if ((rc = select_flagged(ctx, sfl, np, &ids, &cnt))) return rc;
    if (cnt > 0) {
      Plan pw;
      if ((rc = plan_pass(ctx, sc, ids, cnt, qlen, wrl, nullptr, nullptr, 32, R, pw, sp))) return rc;
      PairView wview{qstart, wrs, qlen, wrl, b.qcat, b.rcat, 0};
      FillOut wout{wsc, wqe, wre, wov, err};
      if ((rc = run_fill(ctx, pw, sc, wview, false, nullptr, wout, score_bound, -1, 0, 1, sp)))
        return rc;
    }
    HIP_TRY(launch_sub_rev_views(np, qstart, rstart, qlen, score2, rend2, wsc, wqe, kAnchor, rqs,
                                 rql, rrs, rrl, tgt, sfl, err, st));
    HIP_TRY(hipMemsetAsync(rsc, 0, sizeof(int32_t) * np, st));
    if ((rc = select_flagged(ctx, sfl, np, &ids, &cnt))) return rc;
    if (cnt > 0) {
      Plan pr;
      if ((rc = plan_pass(ctx, sc, ids, cnt, rql, rrl, nullptr, nullptr, 32, R, pr, sp))) return rc;
      PairView rview{rqs, rrs, rql, rrl, b.qcat, b.rcat, 1};
      FillOut rout{rsc, rqe, rre, rov, err};
      if ((rc = run_fill(ctx, pr, sc, rview, true, tgt, rout, score_bound + kAnchor, -1, kAnchor,
                         0, sp)))
        return rc;
    }
    HIP_TRY(launch_sub_begins(np, score2, rend2, wqe, sfl, tgt, rsc, rqe, rre, s_score, s_qbeg,
                              s_qend, s_rbeg, s_rend, err, st));
    // CIGARs after the primaries (cigar_used holds their total even when they did not fit)
    HIP_TRY(hipMemsetAsync(s_cig_len, 0, sizeof(int32_t) * np, st));
    HIP_TRY(hipMemsetAsync(s_cig_off, 0, sizeof(int64_t) * (np + 1), st));
    const int64_t base = out->cigar_used;
    swx_batch_out so = *out;
    so.cigar = (out->cigar && base <= out->cigar_cap) ? out->cigar + base : nullptr;
    so.cigar_cap = out->cigar_cap > base ? out->cigar_cap - base : 0;
    uint32_t sflags = SWX_BEGIN | SWX_CIGAR;
    int rc_sub = SWX_OK;
    if ((rc = run_traceback(ctx, sc, b, np, s_score, s_qbeg, s_qend, s_rbeg, s_rend, qstart,
                            rstart, qlen, rlen, s_cig_len, s_cig_off, err, &so, &sflags, &rc_sub)))
      return rc;
    out->cigar_used = base + so.cigar_used;
    if (rc_sub != SWX_OK) rc_range = rc_sub;
    if (!(flags & SWX_CIGAR)) sflags &= ~SWX_CIGAR;   // the primaries did not fit either
    HIP_TRY(hipMemsetAsync(slb, 32, np, st));
    swx_rec_dev *srec = (out->out_mem == SWX_MEM_DEVICE) ? (swx_rec_dev *)out->sub_recs
                                                         : A.get<swx_rec_dev>(np);
    if (!srec) return fail(SWX_ENOMEM, "device pool exhausted");
    HIP_TRY(launch_records(np, s_score, s_score, s_qbeg, s_qend, s_rbeg, s_rend, s_rend, s_cig_off,
                           s_cig_len, slb, sflags, srec, st));
    if (sflags & SWX_CIGAR) HIP_TRY(shift_cigar_offsets(np, base, srec, st));
    if (out->out_mem != SWX_MEM_DEVICE)
      HIP_TRY(hipMemcpyAsync(out->sub_recs, srec, sizeof(swx_rec) * np, hipMemcpyDeviceToHost, st));
  }

  // records
  swx_rec_dev *drec = (out->out_mem == SWX_MEM_DEVICE) ? (swx_rec_dev *)out->recs
                                                       : A.get<swx_rec_dev>(np);
  if (!drec) return fail(SWX_ENOMEM, "device pool exhausted");
  HIP_TRY(launch_records(np, score, score2, qbeg, qend, rbeg, rend, rend2, cig_off_final, cig_len,
                         lanebits, flags, drec, st));
  if (out->out_mem != SWX_MEM_DEVICE && np)
    HIP_TRY(hipMemcpyAsync(out->recs, drec, sizeof(swx_rec) * np, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipEventRecord(ctx->ev[7], st));
  // consistency: any per-pair error flag
  HIP_TRY(hipMemsetAsync(stats, 0, 8, st));
  HIP_TRY(launch_any_flag(np, err, stats, st));
  int64_t nerr = 0;
  if ((rc = read_i64(ctx, stats, &nerr))) return rc;
  ctx->nstages = 7;
  for (int k = 0; k < 7; ++k) {
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, ctx->ev[k], ctx->ev[k + 1]));
    ctx->stage_ms[k] = ms;
  }
  if (nerr) return fail(SWX_EINTERNAL, "internal consistency check failed for " +
                                           std::to_string(nerr) + " pairs");
  return rc_range;
}

// ============================================================================
// Fixed-capacity path for hipGraph capture.
//
// The same stages as run_pipeline, for batches of exactly B pairs with
// qlen <= QM and rlen <= RM, with every buffer sized from those capacities
// when the graph is made and every count that depends on the data (pairs
// re-run on 32-bit lanes, pairs per reversed pass, pairs per traceback class)
// kept on the device: plans take their pair count from device memory and
// form empty tasks past it, kernels skip empty tasks.  Nothing in it waits on
// the host, so the whole chain is captured once and replayed per batch.
// Long pairs are not routed to the intra-sequence path here (its job tables
// are built on the host), and wide bands stay on the strip kernel.
// ============================================================================
struct FixedPlan {
  int lane_bits = 16, R = 32, slots = 128;
  int64_t cap_n = 0, ntasks = 0;
  uint64_t *k0 = nullptr, *k1 = nullptr;
  int64_t *v0 = nullptr, *v1 = nullptr;
  void *sort_tmp = nullptr;
  size_t sort_bytes = 0;
  int64_t *sorted = nullptr;
  InterTask *tasks = nullptr;
  int64_t *bsz = nullptr, *boff = nullptr, *qsz = nullptr, *qoff = nullptr;
  uint32_t *bnd = nullptr;
  uint2 *rsym = nullptr;
  uint8_t *prof = nullptr;
};

struct FixedTb {   // one traceback class
  int64_t cap_tasks = 0;
  void *tasks = nullptr;     // TbTask or TbwTask
  int64_t *dsz = nullptr, *doff = nullptr, *bsz = nullptr, *boff = nullptr;
  uint32_t *dir = nullptr;
  int32_t *bnd = nullptr;
};

struct GraphState {
  swx_graph_cfg cfg{};
  int32_t fill_sched = 1, cus = 0;    // the creating context's fill schedule
  int32_t fill_coop = 0;
  unsigned long long *queue = nullptr;
  std::vector<int8_t> matrix;
  Scoring sc{};
  DevArena A;
  int64_t B = 0, QM = 0, RM = 0;
  bool clamp = false, need32 = false, pair3 = false;
  // inputs / outputs
  int8_t *qcat = nullptr, *rcat = nullptr;
  int64_t *qoff = nullptr, *roff = nullptr, *pair_q = nullptr, *pair_r = nullptr;
  swx_rec_dev *recs = nullptr;
  uint32_t *cigar = nullptr;
  int64_t cigar_cap = 0;
  // per pair
  int64_t *qstart, *rstart, *rlen, *rend, *rbeg, *rend2, *rqs, *rrs, *rrl, *rre;
  int32_t *qlen, *score, *qend, *qbeg, *score2, *rql, *tgt, *band, *band_q, *rsc, *rqe, *cig_len;
  uint8_t *ovf, *lanebits, *err, *rov, *f16, *f32, *cls;
  uint32_t *bad;
  int64_t *status;            // [0] pairs with an error flag
  // compaction of flagged pairs
  int64_t *f64, *pos, *ids;
  void *scan_tmp = nullptr;
  size_t scan_bytes = 0;
  FixedPlan p16, p32, r16, r32;
  // traceback
  uint64_t *tk0, *tk1;
  int64_t *tv0, *tv1, *ccap, *coff, *counts, *ranges, *len64, *cig_off_final;
  int64_t *tb_sorted = nullptr;
  void *tb_sort_tmp = nullptr;
  size_t tb_sort_bytes = 0;
  FixedTb tb[6];
  // one-pair graphs: the pair's traceback on the wave kernel, its job planned
  // on the device (instead of the class, sort and task kernels of a batch)
  bool tbw1 = false;
  int tbw_rl = 4, tbw_waves = 1;
  TbWaveJob *tbw_job = nullptr;
  uint8_t *tbw_dir = nullptr;
  int32_t *tbw_bnd = nullptr;
  uint32_t *cscr = nullptr;
  // intra route: every pair spread over a wave (one job per pair)
  bool intra = false;
  int RL = 16, waves = 1;
  int32_t kbits = 1, sh = 1024;
  int64_t bnd_stride = 0;      // reversed pass: hand-over rows per pair
  int32_t nc = 1;              // forward pass: column chunks per pair ...
  int64_t chunk = 0;           // ... of this many columns ...
  int64_t fbnd_stride = 0;     // ... and hand-over rows per chunk
  IntraJob *jobs = nullptr, *rjobs = nullptr;
  IntraPair *ipairs = nullptr;
  uint32_t *maxcol = nullptr, *ibnd = nullptr;
  int32_t *part_v = nullptr;
  int64_t *part_j = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

static int fixed_scan(GraphState &g, const int64_t *in, int64_t *out, int64_t n, hipStream_t st) {
  size_t need = 0;
  HIP_TRY(launch_exclusive_scan(in, out, n, nullptr, &need, st));
  if (need > g.scan_bytes) return fail(SWX_EINTERNAL, "scan scratch too small");
  size_t have = g.scan_bytes;
  HIP_TRY(launch_exclusive_scan(in, out, n, g.scan_tmp, &have, st));
  return SWX_OK;
}

// allocate a plan's buffers for up to cap_n pairs (create time)
static int fixed_plan_alloc(GraphState &g, FixedPlan &pl, int lane_bits, int R) {
  DevArena &A = g.A;
  pl.lane_bits = lane_bits;
  pl.R = R;
  pl.slots = lane_bits == 16 ? kSlots16 : kSlots32;
  pl.cap_n = g.B;
  pl.ntasks = (g.B + pl.slots - 1) / pl.slots;
  const int halves = lane_bits == 16 ? 2 : 1;
  pl.k0 = A.get<uint64_t>(g.B); pl.k1 = A.get<uint64_t>(g.B);
  pl.v0 = A.get<int64_t>(g.B); pl.v1 = A.get<int64_t>(g.B);
  pl.tasks = A.get<InterTask>(pl.ntasks);
  pl.bsz = A.get<int64_t>(pl.ntasks + 1); pl.boff = A.get<int64_t>(pl.ntasks + 1);
  pl.qsz = A.get<int64_t>(pl.ntasks + 1); pl.qoff = A.get<int64_t>(pl.ntasks + 1);
  const int64_t rp_cap = (g.RM + 7) / 8 * 8 + 8;
  const int64_t qp_cap = (g.QM + R - 1) / R * R + R;
  const int64_t bnd_words = pl.ntasks * 3 * 64 * rp_cap;
  pl.bnd = A.get<uint32_t>(bnd_words);
  pl.rsym = A.get<uint2>(rsym_offset(bnd_words) + 16);
  if (!g.sc.qsel) pl.prof = A.get<uint8_t>(pl.ntasks * qp_cap * (g.sc.n + 1) * halves * 64 + 16);
  size_t sb = 0;
  HIP_TRY(plan_sort(g.B, nullptr, nullptr, nullptr, nullptr, nullptr, R, pl.k0, pl.k1, pl.v0, pl.v1,
                    nullptr, &sb, nullptr, nullptr, true));
  pl.sort_bytes = sb;
  pl.sort_tmp = A.alloc(sb);
  if (!pl.k0 || !pl.k1 || !pl.v0 || !pl.v1 || !pl.tasks || !pl.bsz || !pl.boff || !pl.qsz ||
      !pl.qoff || !pl.bnd || !pl.rsym || (!g.sc.qsel && !pl.prof) || !pl.sort_tmp)
    return fail(SWX_ENOMEM, "device pool exhausted (graph plan)");
  return SWX_OK;
}

// plan + fill of one pass over ids[0 .. *n_dev) (ids null: all B pairs)
static int fixed_fill(GraphState &g, FixedPlan &pl, const int64_t *ids, const int64_t *n_dev,
                      const int32_t *qlen, const int64_t *rlen, const int32_t *band,
                      const int32_t *band_q, const PairView &view, bool rev,
                      const int32_t *target, FillOut out, hipStream_t st) {
  size_t sb = pl.sort_bytes;
  HIP_TRY(plan_sort(pl.cap_n, n_dev, ids, qlen, rlen, band, pl.R, pl.k0, pl.k1, pl.v0, pl.v1,
                    pl.sort_tmp, &sb, &pl.sorted, st, true));
  const int halves = pl.lane_bits == 16 ? 2 : 1;
  const int64_t per_row = g.sc.qsel ? 0 : (int64_t)(g.sc.n + 1) * halves * 64;
  HIP_TRY(plan_tasks_dev(   // also clears bsz[ntasks], qsz[ntasks]
                         pl.cap_n, n_dev, pl.ntasks, pl.slots, pl.R, per_row, pl.sorted, qlen, rlen,
                         band, band_q, pl.tasks, pl.bsz, pl.qsz, st));
  int rc;
  if ((rc = fixed_scan(g, pl.bsz, pl.boff, pl.ntasks + 1, st))) return rc;
  if ((rc = fixed_scan(g, pl.qsz, pl.qoff, pl.ntasks + 1, st))) return rc;
  HIP_TRY(plan_offsets_dev(pl.ntasks, pl.tasks, pl.boff, pl.qoff, st));
  PackArgs pk{};
  pk.tasks = pl.tasks; pk.ntasks = pl.ntasks; pk.slot_pair = pl.sorted; pk.view = view;
  pk.prof = pl.prof; pk.rsym = pl.rsym; pk.matrix = g.sc.dmat; pk.n = g.sc.n; pk.bias = g.sc.bias;
  pk.halves = halves; pk.strip_rows = pl.R; pk.rev = rev ? 1 : 0;
  HIP_TRY(inter_pack_ref(pk, st));
  if (!g.sc.qsel) HIP_TRY(inter_pack(pk, st));
  InterArgs a{};
  a.tasks = pl.tasks; a.ntasks = pl.ntasks; a.slot_pair = pl.sorted; a.view = view;
  a.prof = g.sc.qsel ? nullptr : pl.prof; a.bnd = pl.bnd; a.rsym = pl.rsym;
  for (int k = 0; k < 8; ++k) a.lut[k] = g.sc.lut[k];
  a.n = g.sc.n; a.o = g.sc.o; a.e = g.sc.e; a.bias = g.sc.bias;
  a.rev = rev ? 1 : 0;
  a.clamp = g.clamp ? 1 : 0;
  a.pair3 = g.pair3 ? 1 : 0;
  a.code_top = pl.R - 1;
  a.dummy = g.sc.dmat;
  a.target = target;
  a.out = out;
  a.sched = g.fill_sched;
  a.cus = g.cus;
  a.queue = g.queue;
  a.coop = coop_waves(g.fill_coop, pl.ntasks, g.cus);
  HIP_TRY(inter_fill(a, pl.lane_bits, pl.R, st));
  return SWX_OK;
}

// flagged pairs -> ids[0 .. *count) with the count on the device (pos[B])
static int fixed_select(GraphState &g, const uint8_t *flag, const int64_t **count, hipStream_t st) {
  HIP_TRY(flags_to_i64(g.B, flag, g.f64, st));   // also clears g.f64[B]
  int rc;
  if ((rc = fixed_scan(g, g.f64, g.pos, g.B + 1, st))) return rc;
  HIP_TRY(compact_flags(g.B, flag, g.pos, g.ids, st));
  *count = g.pos + g.B;
  return SWX_OK;
}

static int fixed_issue(GraphState &g, hipStream_t st) {
  const int64_t B = g.B;
  const uint32_t flags = g.cfg.flags & (SWX_CIGAR | SWX_SCORE2) ? (g.cfg.flags | SWX_BEGIN) : g.cfg.flags;
  int rc;
  if (g.intra) {
    // the intra route clears all its per-call buffers in one launch (the
    // lanes are 32-bit throughout)
    FillSet fs{};
    fs.add(g.bad, 1, 4, 0);
    fs.add(g.status, 1, 8, 0);
    fs.add(g.err, B, 1, 0);
    fs.add(g.lanebits, B, 1, 32);
    fs.add(g.maxcol, B * g.RM, 4, 0);
    fs.add(g.rsc, B, 4, 0);
    fs.add(g.cig_len, B, 4, 0);
    fs.add(g.cig_off_final, B + 1, 8, 0);
    fs.add(g.len64 + B, 1, 8, 0);
    HIP_TRY(fill_set(fs, st));
  } else {
    HIP_TRY(fill_u8(4, (uint8_t *)g.bad, 0, st));
    HIP_TRY(fill_i64(1, g.status, 0, st));
    HIP_TRY(fill_u8(B, g.err, 0, st));
    HIP_TRY(fill_u8(B, g.lanebits, 16, st));
  }
  ValidateArgs va{g.qcat, g.cfg.qcat_cap, g.qoff, g.cfg.nq_cap, g.rcat, g.cfg.rcat_cap, g.roff,
                  g.cfg.nr_cap, g.pair_q, g.pair_r, B, g.sc.n, g.bad};
  HIP_TRY(launch_validate(va, st));
  {
    const ViewCaps vc{g.cfg.nq_cap, g.cfg.nr_cap, g.cfg.qcat_cap, g.cfg.rcat_cap,
                      (int32_t)g.QM, 0, g.RM};
    HIP_TRY(launch_views(B, g.qoff, g.roff, g.pair_q, g.pair_r, vc, g.qstart, g.qlen, g.rstart,
                         g.rlen, st));
  }
  PairView fview{g.qstart, g.rstart, g.qlen, g.rlen, g.qcat, g.rcat, 0};
  FillOut fout{g.score, g.qend, g.rend, g.ovf, g.err};
  IntraArgs ia{};
  if (g.intra) {
    HIP_TRY(intra_jobs_chunked(B, g.nc, g.chunk, g.qlen, g.rlen, g.sc.smax, g.sc.o, g.sc.e,
                               g.kbits, g.sh, g.RM, g.fbnd_stride, g.jobs, g.ipairs, st));
    ia.jobs = g.jobs; ia.njobs = B * g.nc; ia.view = fview; ia.matrix = g.sc.dmat;
    ia.n = g.sc.n; ia.o = g.sc.o; ia.e = g.sc.e; ia.bias = g.sc.bias;
    ia.maxcol = g.maxcol; ia.bnd = g.ibnd; ia.err = g.err;
    HIP_TRY(intra_fill(ia, g.RL, g.waves, false, st));
    IntraPairArgs e{};
    e.pairs = g.ipairs; e.maxcol = g.maxcol; e.qlen = g.qlen; e.rlen = g.rlen;
    e.score = g.score; e.qend = g.qend; e.rend = g.rend; e.overflow = g.ovf;
    e.part_v = g.part_v; e.part_j = g.part_j;
    HIP_TRY(intra_end(e, B, st));
  } else if ((rc = fixed_fill(g, g.p16, nullptr, nullptr, g.qlen, g.rlen, nullptr, nullptr, fview, false,
                              nullptr, fout, st))) {
    return rc;
  }
  if (g.need32 && !g.intra) {
    const int64_t *nw = nullptr;
    if ((rc = fixed_select(g, g.ovf, &nw, st))) return rc;
    if ((rc = fixed_fill(g, g.p32, g.ids, nw, g.qlen, g.rlen, nullptr, nullptr, fview, false, nullptr,
                         fout, st)))
      return rc;
    HIP_TRY(mark_lanes_dev(B, nw, g.ids, g.lanebits, 32, st));
  }
  if (flags & SWX_BEGIN) {
    HIP_TRY(launch_rev_views(B, g.qstart, g.rstart, g.qlen, g.rlen, g.score, g.qend, g.rend, g.rqs,
                             g.rql, g.rrs, g.rrl, g.tgt, g.err, st));
    HIP_TRY(rev_prepare(B, g.score, g.qend, g.rend, g.lanebits, g.sc.smax, g.sc.o, g.sc.e, g.band,
                        g.band_q, g.f16, g.f32, st));
    if (!g.intra) HIP_TRY(fill_u8(4 * B, (uint8_t *)g.rsc, 0, st));
    PairView rview{g.rqs, g.rrs, g.rql, g.rrl, g.qcat, g.rcat, 1};
    FillOut rout{g.rsc, g.rqe, g.rre, g.rov, g.err};
    if (g.intra) {
      HIP_TRY(intra_rev_jobs_fixed(B, g.score, g.rend, g.band, g.kbits, g.bnd_stride, g.rjobs, st));
      IntraArgs ra = ia;
      ra.jobs = g.rjobs;
      ra.njobs = B;   // one reversed job per pair (the forward pass had g.nc per pair)
      ra.view = rview;
      ra.maxcol = nullptr;
      ra.target = g.tgt;
      ra.out = rout;
      HIP_TRY(intra_fill(ra, g.RL, g.waves, true, st));
    }
    const int64_t *n16 = nullptr;
    if (!g.intra && (rc = fixed_select(g, g.f16, &n16, st))) return rc;
    if (!g.intra && (rc = fixed_fill(g, g.r16, g.ids, n16, g.rql, g.rrl, g.band, g.band_q, rview,
                                     true, g.tgt, rout, st)))
      return rc;
    if (g.need32 && !g.intra) {
      const int64_t *n32 = nullptr;
      if ((rc = fixed_select(g, g.f32, &n32, st))) return rc;
      if ((rc = fixed_fill(g, g.r32, g.ids, n32, g.rql, g.rrl, g.band, g.band_q, rview, true,
                           g.tgt, rout, st)))
        return rc;
    }
    HIP_TRY(launch_begins(B, g.score, g.qend, g.rend, g.rsc, g.rqe, g.rre, g.qbeg, g.rbeg, g.err, st));
  }
  if (!g.intra) {
    HIP_TRY(fill_u8(4 * B, (uint8_t *)g.cig_len, 0, st));
    HIP_TRY(fill_i64(B + 1, g.cig_off_final, 0, st));
  }
  if (flags & SWX_CIGAR) {
    TbArgs ta{};
    ta.score = g.score; ta.qbeg = g.qbeg; ta.qend = g.qend; ta.rbeg = g.rbeg; ta.rend = g.rend;
    ta.qstart = g.qstart; ta.rstart = g.rstart; ta.qlen = g.qlen; ta.rlen = g.rlen;
    ta.qcat = g.qcat; ta.rcat = g.rcat; ta.matrix = g.sc.dmat;
    ta.n = g.sc.n; ta.o = g.sc.o; ta.e = g.sc.e; ta.smax = g.sc.smax;
    ta.cig_len = g.cig_len; ta.err = g.err;
    ta.wave_cells = INT64_MAX;   // no host-planned wave traceback in a graph
    ta.cig = g.cscr;
    ta.cig_off = g.coff;
    if (g.tbw1) {
      HIP_TRY(tb_wave_job1(ta, g.tbw_job, g.coff, st));
      HIP_TRY(tb_wave(ta, g.tbw_job, 1, g.tbw_rl, g.tbw_waves, 1, nullptr, g.tbw_dir, g.tbw_bnd, st));
    } else {
    HIP_TRY(fill_i64(1, g.ccap + B, 0, st));
    HIP_TRY(fill_i64(8, g.counts, 0, st));
    HIP_TRY(tb_classify(ta, B, g.cls, g.tk0, g.tv0, g.ccap, st));
    if ((rc = fixed_scan(g, g.ccap, g.coff, B + 1, st))) return rc;
    HIP_TRY(count_classes(B, g.cls, g.counts, st));
    size_t sb = g.tb_sort_bytes;
    HIP_TRY(sort_keys(B, g.tk0, g.tk1, g.tv0, g.tv1, g.tb_sort_tmp, &sb, &g.tb_sorted, st, kTbKeyBits,
                      true));
    HIP_TRY(class_ranges(g.counts, g.ranges, st));
    for (int c = 1; c <= 3; ++c) {
      FixedTb &t = g.tb[c];
      const int32_t bw = 8 << (c - 1);
      TbTask *tasks = (TbTask *)t.tasks;
      HIP_TRY(fill_i64(1, t.dsz + t.cap_tasks, 0, st));
      HIP_TRY(tb_tasks_range(g.ranges + 2 * c, t.cap_tasks, g.tb_sorted, ta, bw, tasks, t.dsz, st));
      if ((rc = fixed_scan(g, t.dsz, t.doff, t.cap_tasks + 1, st))) return rc;
      HIP_TRY(tb_offsets(t.cap_tasks, tasks, t.doff, st));
      TbArgs tc = ta;
      tc.dir = t.dir;
      HIP_TRY(tb_band(tc, tasks, t.cap_tasks, g.tb_sorted, bw, st));
    }
    {
      FixedTb &t = g.tb[5];
      TbwTask *tasks = (TbwTask *)t.tasks;
      HIP_TRY(fill_i64(1, t.dsz + t.cap_tasks, 0, st));
      HIP_TRY(fill_i64(1, t.bsz + t.cap_tasks, 0, st));
      HIP_TRY(tbw_tasks_range(g.ranges + 10, t.cap_tasks, g.tb_sorted, ta, tasks, t.dsz, t.bsz, st));
      if ((rc = fixed_scan(g, t.dsz, t.doff, t.cap_tasks + 1, st))) return rc;
      if ((rc = fixed_scan(g, t.bsz, t.boff, t.cap_tasks + 1, st))) return rc;
      HIP_TRY(tbw_offsets(t.cap_tasks, tasks, t.doff, t.boff, st));
      TbArgs tc = ta;
      tc.dir = t.dir;
      HIP_TRY(tb_strip(tc, tasks, t.cap_tasks, g.tb_sorted, t.bnd, st));
    }
    }
    if (B == 1) {
      HIP_TRY(cigar_one(g.cscr, g.coff, g.cig_len, g.cig_off_final, g.cigar, st));
    } else {
      if (!g.intra) HIP_TRY(fill_i64(1, g.len64 + B, 0, st));
      HIP_TRY(lens_to_i64(B, g.cig_len, g.len64, st));
      if ((rc = fixed_scan(g, g.len64, g.cig_off_final, B + 1, st))) return rc;
      HIP_TRY(launch_cigar_compact(B, g.cscr, g.coff, g.cig_len, g.cig_off_final, g.cigar, st));
    }
  }
  if ((flags & SWX_SCORE2) && g.intra) {
    IntraPairArgs e{};
    e.pairs = g.ipairs; e.maxcol = g.maxcol; e.qlen = g.qlen; e.rlen = g.rlen;
    e.score = g.score; e.qend = g.qend; e.rend = g.rend; e.rbeg = g.rbeg;
    e.mask_len = g.cfg.mask_len; e.score2 = g.score2; e.rend2 = g.rend2;
    e.part_v = g.part_v; e.part_j = g.part_j;
    HIP_TRY(intra_score2(e, B, st));
  } else if (flags & SWX_SCORE2) {
    Score2InterArgs s2{};
    s2.rlen = g.rlen; s2.qlen = g.qlen; s2.score1 = g.score; s2.rbeg = g.rbeg; s2.rend = g.rend;
    s2.mask_len = g.cfg.mask_len; s2.score2 = g.score2; s2.rend2 = g.rend2;
    s2.tasks = g.p16.tasks; s2.ntasks = g.p16.ntasks; s2.slot_pair = g.p16.sorted;
    s2.bnd = g.p16.bnd; s2.halves = 2;
    HIP_TRY(launch_score2_inter(s2, st));
    if (g.need32) {
      s2.tasks = g.p32.tasks; s2.ntasks = g.p32.ntasks; s2.slot_pair = g.p32.sorted;
      s2.bnd = g.p32.bnd; s2.halves = 1;
      HIP_TRY(launch_score2_inter(s2, st));
    }
  }
  HIP_TRY(launch_records(B, g.score, g.score2, g.qbeg, g.qend, g.rbeg, g.rend, g.rend2,
                         g.cig_off_final, g.cig_len, g.lanebits, flags, g.recs, st));
  HIP_TRY(launch_any_flag(B, g.err, g.status, st));
  return SWX_OK;
}

// Code bytes up to which a one-pair graph traces its pair on the wave kernel.
static constexpr int64_t kGraphWaveTbBytes = int64_t(64) << 20;

static int graph_alloc(GraphState &g) {
  DevArena &A = g.A;
  const int64_t B = g.B;
  g.queue = A.get<unsigned long long>(1);
  g.qcat = A.get<int8_t>(g.cfg.qcat_cap);
  g.rcat = A.get<int8_t>(g.cfg.rcat_cap);
  g.qoff = A.get<int64_t>(g.cfg.nq_cap + 1);
  g.roff = A.get<int64_t>(g.cfg.nr_cap + 1);
  g.pair_q = A.get<int64_t>(B);
  g.pair_r = A.get<int64_t>(B);
  g.recs = A.get<swx_rec_dev>(B);
  g.cigar_cap = B * (g.QM + g.RM + 2);
  g.cigar = A.get<uint32_t>(g.cigar_cap);
  g.cscr = A.get<uint32_t>(g.cigar_cap);
  bool per_pair = true;
  for (int64_t **p : {&g.qstart, &g.rstart, &g.rlen, &g.rend, &g.rbeg, &g.rend2, &g.rqs, &g.rrs,
                      &g.rrl, &g.rre, &g.tv0, &g.tv1})
    per_pair = (*p = A.get<int64_t>(B)) != nullptr && per_pair;
  for (int32_t **p : {&g.qlen, &g.score, &g.qend, &g.qbeg, &g.score2, &g.rql, &g.tgt, &g.band,
                      &g.band_q, &g.rsc, &g.rqe, &g.cig_len})
    per_pair = (*p = A.get<int32_t>(B)) != nullptr && per_pair;
  for (uint8_t **p : {&g.ovf, &g.lanebits, &g.err, &g.rov, &g.f16, &g.f32, &g.cls})
    per_pair = (*p = A.get<uint8_t>(B)) != nullptr && per_pair;
  if (!per_pair) return fail(SWX_ENOMEM, "device pool exhausted (graph)");
  g.bad = A.get<uint32_t>(1);
  g.status = A.get<int64_t>(1);
  g.f64 = A.get<int64_t>(B + 1);
  g.pos = A.get<int64_t>(B + 1);
  g.ids = A.get<int64_t>(B);
  g.tk0 = A.get<uint64_t>(B);
  g.tk1 = A.get<uint64_t>(B);
  g.ccap = A.get<int64_t>(B + 1);
  g.coff = A.get<int64_t>(B + 1);
  g.counts = A.get<int64_t>(8);
  g.ranges = A.get<int64_t>(16);
  g.len64 = A.get<int64_t>(B + 1);
  g.cig_off_final = A.get<int64_t>(B + 1);
  int rc;
  const int R = 32;
  if (g.intra) {
    g.RL = pick_rl(g.QM, g.sc.n);
    g.sh = 64 * g.RL;
    const int64_t qp = (g.QM + g.sh - 1) / g.sh * g.sh;
    const int64_t nstrips = qp / g.sh;
    if (nstrips > intra_max_strips()) return fail(SWX_EINVAL, "max_qlen too long for the intra route");
    g.kbits = code_bits(qp);
    const int64_t bound = (int64_t)std::max(g.sc.smax, 0) * std::min<int64_t>(g.QM, g.RM);
    if (g.kbits > 30 || bound >= (int64_t(1) << (32 - g.kbits)))
      return fail(SWX_EOVERFLOW, "score range and query length exceed the max-array word");
    g.waves = intra_waves(nstrips, g.sc.n, g.RL);
    g.bnd_stride = 2 * (nstrips - 1) * g.RM;
    // the forward pass cuts each reference into column chunks that start the
    // widest positive-scoring span early (for the capacity's query length;
    // a shorter query starts later), so that a pair spreads over several
    // workgroups instead of sweeping its reference on one
    g.nc = 1;
    g.chunk = std::max<int64_t>(g.RM, 1);
    int64_t wcap = g.RM;
    if (g.sc.e > 0) {
      wcap = g.QM + std::max<int64_t>((int64_t)g.sc.smax * g.QM - g.sc.o, 0) / g.sc.e + 1;
      // (a one-pair graph is latency-bound: its chunks only need to fill a
      // few compute units, so it takes the most of them)
      const int64_t C = B == 1 ? 128 : std::max<int64_t>(256, (wcap + 1) / 2);
      const int64_t nc = std::min<int64_t>(kGraphMaxChunks, (g.RM + C - 1) / C);
      if (nc > 1) {
        g.nc = (int32_t)nc;
        g.chunk = (g.RM + nc - 1) / nc;
      }
    }
    g.fbnd_stride = 2 * (nstrips - 1) * std::min<int64_t>(g.RM, g.chunk + wcap);
    g.jobs = A.get<IntraJob>(B * g.nc);
    g.rjobs = A.get<IntraJob>(B);
    g.ipairs = A.get<IntraPair>(B);
    g.maxcol = A.get<uint32_t>(B * std::max<int64_t>(g.RM, 1));
    g.ibnd = A.get<uint32_t>(std::max<int64_t>(
        {B * g.bnd_stride, B * g.nc * g.fbnd_stride, int64_t(1)}));
    g.part_v = A.get<int32_t>(B * intra_slices());
    g.part_j = A.get<int64_t>(B * intra_slices());
    if (!g.jobs || !g.rjobs || !g.ipairs || !g.maxcol || !g.ibnd || !g.part_v || !g.part_j)
      return fail(SWX_ENOMEM, "device pool exhausted (graph intra route)");
  } else {
    if ((rc = fixed_plan_alloc(g, g.p16, 16, R))) return rc;
    if ((rc = fixed_plan_alloc(g, g.r16, 16, R))) return rc;
  }
  if (g.need32 && !g.intra) {
    if ((rc = fixed_plan_alloc(g, g.p32, 32, R))) return rc;
    if ((rc = fixed_plan_alloc(g, g.r32, 32, R))) return rc;
  }
  // traceback classes: up to every pair in one class
  const int64_t capT = (B + 63) / 64;
  for (int c = 1; c <= 3; ++c) {
    FixedTb &t = g.tb[c];
    t.cap_tasks = capT;
    t.tasks = A.get<TbTask>(capT);
    t.dsz = A.get<int64_t>(capT + 1);
    t.doff = A.get<int64_t>(capT + 1);
    t.dir = A.get<uint32_t>(capT * (g.QM + 2) * ((8 << (c - 1)) / 8) * 64);
    if (!t.tasks || !t.dsz || !t.doff || !t.dir) return fail(SWX_ENOMEM, "device pool exhausted (graph traceback)");
  }
  {
    FixedTb &t = g.tb[5];
    const int64_t capW = (B + kTbwSlots - 1) / kTbwSlots;
    t.cap_tasks = capW;
    t.tasks = A.get<TbwTask>(capW);
    t.dsz = A.get<int64_t>(capW + 1); t.doff = A.get<int64_t>(capW + 1);
    t.bsz = A.get<int64_t>(capW + 1); t.boff = A.get<int64_t>(capW + 1);
    // a safe band is at most m + w + 1 diagonals wide; the union over a task's
    // pairs at most 2 (m + w) + 1; a strip of width W holds (W + 4) / 2 code
    // dwords per lane
    const int64_t W = 16 + 2 * (g.QM + g.RM) + 2;
    const int64_t nstrips = (g.QM + 15) / 16;
    t.dir = A.get<uint32_t>(capW * nstrips * ((W + 4) / 2) * 64);
    t.bnd = A.get<int32_t>(capW * 2 * (g.RM + 1) * kTbwSlots);
    if (!t.tasks || !t.dsz || !t.doff || !t.bsz || !t.boff || !t.dir || !t.bnd)
      return fail(SWX_ENOMEM, "device pool exhausted (graph traceback)");
  }
  if (B == 1) {
    // codes of at most QM rows over at most RM + 1 columns per strip
    const int RL = 4;
    const int64_t dbytes = tb_wave_dir_bytes(g.QM, g.RM, RL);
    const int64_t nstrips = (g.QM + 64 * RL - 1) / (64 * RL);
    if (dbytes <= kGraphWaveTbBytes && nstrips <= tb_wave_max_strips()) {
      g.tbw_rl = RL;
      g.tbw_waves = tb_wave_waves(g.QM, g.sc.n, RL);
      g.tbw_job = A.get<TbWaveJob>(1);
      g.tbw_dir = A.get<uint8_t>(dbytes);
      g.tbw_bnd = A.get<int32_t>(2 * (g.RM + 1) * (nstrips + 1));
      if (!g.tbw_job || !g.tbw_dir || !g.tbw_bnd)
        return fail(SWX_ENOMEM, "device pool exhausted (graph wave traceback)");
      g.tbw1 = true;
    }
  }
  size_t sb = 0;
  HIP_TRY(sort_keys(B, g.tk0, g.tk1, g.tv0, g.tv1, nullptr, &sb, &g.tb_sorted, nullptr, kTbKeyBits,
                    true));
  g.tb_sort_bytes = sb;
  g.tb_sort_tmp = A.alloc(sb);
  // scan scratch: the largest scan is over B + 1 elements
  size_t sc1 = 0;
  HIP_TRY(launch_exclusive_scan(g.f64, g.pos, B + 1, nullptr, &sc1, nullptr));
  g.scan_bytes = sc1 + 4096;
  g.scan_tmp = A.alloc(g.scan_bytes);
  if (!g.qcat || !g.rcat || !g.qoff || !g.roff || !g.pair_q || !g.pair_r || !g.recs || !g.cigar ||
      !g.cscr || !g.bad || !g.status || !g.f64 || !g.pos || !g.ids || !g.tk0 || !g.tk1 ||
      !g.ccap || !g.coff || !g.counts || !g.ranges || !g.len64 || !g.cig_off_final ||
      !g.tb_sort_tmp || !g.scan_tmp)
    return fail(SWX_ENOMEM, "device pool exhausted (graph)");
  return SWX_OK;
}

int internal_fail(int code, const char *msg) { return fail(code, msg); }
hipStream_t internal_stream(swx_ctx *ctx) { return ctx->stream; }
int internal_device(const swx_ctx *ctx) { return ctx->device; }

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

int swx_get_tuning(const swx_ctx *ctx, swx_tuning *out) {
  if (!ctx || !out) return fail(SWX_EINVAL, "null argument");
  swx_tuning t{};
  t.long_cells = ctx->long_cells;
  t.long_rlen = ctx->long_rlen;
  t.intra_jobs = ctx->intra_jobs;
  t.fill_rows = ctx->fill_rows;
  t.side_streams = ctx->side_streams ? 1 : 0;
  t.fill_sched = ctx->fill_sched;
  t.fill_coop = ctx->fill_coop;
  t.intra_bits = ctx->intra_bits;
  *out = t;
  return SWX_OK;
}

int swx_set_tuning(swx_ctx *ctx, const swx_tuning *t) {
  if (!ctx || !t) return fail(SWX_EINVAL, "null argument");
  if (t->long_cells < -1 || t->long_rlen < 0 || t->intra_jobs < 1 ||
      (t->side_streams != 0 && t->side_streams != 1) || t->fill_sched < 0 || t->fill_sched > 2 ||
      t->fill_coop < 0 || t->fill_coop > 2 || (t->intra_bits != 0 && t->intra_bits != 16 && t->intra_bits != 32) ||
      t->pad_ != 0 ||
      (t->fill_rows != 16 && t->fill_rows != 24 && t->fill_rows != 32))
    return fail(SWX_EINVAL, "tuning value out of range");
  std::lock_guard<std::mutex> g(ctx->mu);
  ctx->long_cells = t->long_cells;
  ctx->long_rlen = t->long_rlen;
  ctx->intra_jobs = t->intra_jobs;
  ctx->fill_rows = t->fill_rows;
  ctx->side_streams = t->side_streams != 0;
  ctx->fill_sched = t->fill_sched;
  ctx->fill_coop = t->fill_coop;
  ctx->intra_bits = t->intra_bits;
  return SWX_OK;
}

// frees whatever a context holds (also one that was only partly created)
static void release_ctx(swx_ctx *ctx) {
  (void)hipSetDevice(ctx->device);
  ctx->arena.release();
  if (ctx->queue) (void)hipFree(ctx->queue);
  if (ctx->pinned) (void)hipHostFree(ctx->pinned);
  for (auto &e : ctx->ev)
    if (e) (void)hipEventDestroy(e);
  for (int k = 0; k < swx_ctx::kAux; ++k) {
    if (ctx->aux[k]) (void)hipStreamDestroy(ctx->aux[k]);
    if (ctx->join_ev[k]) (void)hipEventDestroy(ctx->join_ev[k]);
  }
  if (ctx->fork_ev) (void)hipEventDestroy(ctx->fork_ev);
  if (ctx->own) (void)hipStreamDestroy(ctx->own);
  delete ctx;
}

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
  if (hipSetDevice(device) != hipSuccess || hipStreamCreate(&c->own) != hipSuccess) {
    release_ctx(c);
    return fail(SWX_EDEVICE, "could not create a stream");
  }
  c->stream = c->own;
  for (auto &e : c->ev) {
    if (hipEventCreate(&e) != hipSuccess) {
      release_ctx(c);
      return fail(SWX_EDEVICE, "could not create events");
    }
  }
  bool ok = hipEventCreateWithFlags(&c->fork_ev, hipEventDisableTiming) == hipSuccess;
  for (int k = 0; k < swx_ctx::kAux && ok; ++k)
    ok = hipEventCreateWithFlags(&c->join_ev[k], hipEventDisableTiming) == hipSuccess;
  if (!ok) {
    release_ctx(c);
    return fail(SWX_EDEVICE, "could not create side streams");
  }
  if (hipDeviceGetAttribute(&c->cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess ||
      c->cus < 1 || hipMalloc(&c->queue, 256) != hipSuccess ||
      hipHostMalloc(&c->pinned, 8 * swx_ctx::kPinned, hipHostMallocDefault) != hipSuccess) {
    release_ctx(c);
    return fail(SWX_EDEVICE, "could not query the device or allocate the work queue");
  }
  c->scratch = scratch_address(device);
  if (!c->scratch) {
    release_ctx(c);
    return fail(SWX_EDEVICE, "could not find the device address of the static scratch");
  }
  *out = c;
  return SWX_OK;
}

int swx_ctx_destroy(swx_ctx *ctx) {
  if (!ctx) return fail(SWX_EINVAL, "ctx is null");
  {
    std::lock_guard<std::mutex> lk(ctx->pair_mu);
    for (auto &pg : ctx->pair_graphs) swx_graph_destroy(pg.g);
    ctx->pair_graphs.clear();
  }
  {
    std::lock_guard<std::mutex> g(ctx->mu);
    (void)hipSetDevice(ctx->device);
    if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
    for (int k = 0; k < swx_ctx::kAux; ++k)
      if (ctx->aux[k]) (void)hipStreamSynchronize(ctx->aux[k]);
  }
  release_ctx(ctx);
  return SWX_OK;
}

int swx_last_stage_ms(const swx_ctx *ctx, double *ms, int cap) {
  if (!ctx || !ms || cap < 0) return fail(SWX_EINVAL, "bad arguments");
  int n = std::min(cap, ctx->nstages);
  for (int k = 0; k < n; ++k) ms[k] = ctx->stage_ms[k];
  return n;
}

int swx_lane_probe(swx_ctx *ctx, int32_t bits, int64_t columns, int64_t blocks, int32_t gap_open,
                   int32_t gap_extend, uint32_t *best, double *ms) {
  if (!ctx || !best || !ms) return fail(SWX_EINVAL, "null argument");
  if ((bits != 8 && bits != 16) || columns < 1 || blocks < 1 || blocks > (int64_t(1) << 20) ||
      gap_open < gap_extend || gap_extend < 0 || gap_open > 60)
    return fail(SWX_EINVAL, "bad probe arguments");
  std::lock_guard<std::mutex> g(ctx->mu);
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(SWX_EDEVICE, "hipSetDevice failed");
  ctx->arena.reset();
  const int64_t npairs = blocks * 256 * (32 / bits);
  uint32_t *d = ctx->arena.get<uint32_t>(npairs);
  if (!d) return fail(SWX_ENOMEM, "device pool exhausted (probe)");
  hipStream_t st = ctx->stream;
  HIP_TRY(hipEventRecord(ctx->ev[0], st));
  HIP_TRY(lane_probe(bits, columns, blocks, gap_open, gap_extend, d, st));
  HIP_TRY(hipEventRecord(ctx->ev[1], st));
  HIP_TRY(hipMemcpyAsync(best, d, sizeof(uint32_t) * (size_t)npairs, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  float t = 0;
  HIP_TRY(hipEventElapsedTime(&t, ctx->ev[0], ctx->ev[1]));
  *ms = t;
  return SWX_OK;
}

int swx_check_max3(swx_ctx *ctx, uint64_t *mismatches, uint64_t *checked) {
  if (!ctx || !mismatches || !checked) return fail(SWX_EINVAL, "null argument");
  std::lock_guard<std::mutex> g(ctx->mu);
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(SWX_EDEVICE, "hipSetDevice failed");
  ctx->arena.reset();
  unsigned long long *d = ctx->arena.get<unsigned long long>(1);
  if (!d) return fail(SWX_ENOMEM, "device pool exhausted (check)");
  hipStream_t st = ctx->stream;
  HIP_TRY(hipMemsetAsync(d, 0, sizeof(*d), st));
  HIP_TRY(max3_check(d, checked, st));
  unsigned long long h = 0;
  HIP_TRY(hipMemcpyAsync(&h, d, sizeof(h), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  *mismatches = h;
  return SWX_OK;
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
  if (!sc.qsel) {
    // the query profile on the device, once: forward strips of 32 and of 16
    // rows and the reversed table (alphabets of at most 4 symbols need none:
    // their fill builds two scores per instruction from a 4-byte table)
    p->qp32 = (int32_t)round_up(qlen, 32);
    p->qp16 = (int32_t)round_up(qlen, 16);
    p->rev_row = qprof_rev_row(qlen, 32);
    const int64_t n1 = n + 1;
    const int64_t f32b = n1 * p->qp32, f16b = n1 * p->qp16, rb = 16 * n1 * p->rev_row;
    const int64_t scratch = qlen + (int64_t)n * n;
    std::lock_guard<std::mutex> g(ctx->mu);
    hipStream_t st = ctx->stream;
    bool ok = hipSetDevice(ctx->device) == hipSuccess &&
              hipMalloc(&p->dev, (size_t)(f32b + f16b + rb + scratch + 64)) == hipSuccess;
    if (ok) {
      p->fwd32 = p->dev;
      p->fwd16 = p->fwd32 + f32b;
      p->rev = p->fwd16 + f16b;
      int8_t *dq = (int8_t *)(p->rev + rb), *dm = dq + qlen;
      ok = hipMemcpyAsync(dq, query, qlen, hipMemcpyHostToDevice, st) == hipSuccess &&
           hipMemcpyAsync(dm, matrix, (size_t)n * n, hipMemcpyHostToDevice, st) == hipSuccess &&
           build_qprof(dq, qlen, dm, n, sc.bias, p->qp32, p->fwd32, p->rev_row, p->rev, st) ==
               hipSuccess &&
           build_qprof(dq, qlen, dm, n, sc.bias, p->qp16, p->fwd16, 0, p->rev, st) == hipSuccess &&
           hipStreamSynchronize(st) == hipSuccess;
    }
    if (!ok) {
      if (p->dev) (void)hipFree(p->dev);
      delete p;
      return fail(SWX_EDEVICE, "could not build the device query profile");
    }
  }
  *out = p;
  return SWX_OK;
}

int swx_profile_destroy(swx_profile *p) {
  if (!p) return fail(SWX_EINVAL, "profile is null");
  if (p->dev) {
    std::lock_guard<std::mutex> g(p->ctx->mu);
    (void)hipSetDevice(p->ctx->device);
    (void)hipStreamSynchronize(p->ctx->stream);
    (void)hipFree(p->dev);
  }
  delete p;
  return SWX_OK;
}

void swx_result_free(swx_result *r) {
  if (!r) return;
  free(r->cigar);
  free(r->sub_cigar);
  r->cigar = nullptr;
  r->sub_cigar = nullptr;
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
  return (b->flags & SWX_SUBOPT) ? 2 * s : s;
}

static int align_batch_locked(swx_ctx *ctx, const swx_batch *b, swx_batch_out *out,
                              const swx_profile *prof = nullptr) {
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
  if (b->flags & ~(SWX_ALL | SWX_SUBOPT)) return fail(SWX_EINVAL, "unknown flag bits");
  if ((b->flags & SWX_SUBOPT) && b->npairs && !out->sub_recs)
    return fail(SWX_EINVAL, "SWX_SUBOPT needs sub_recs");
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
  return run_pipeline(ctx, sc, db, b->flags, b->mask_len, out, prof);
}

int swx_align_batch(swx_ctx *ctx, const swx_batch *b, swx_batch_out *out, void *hip_stream) {
  if (!ctx || !b || !out) return fail(SWX_EINVAL, "null argument");
  std::lock_guard<std::mutex> g(ctx->mu);
  StreamScope ss(ctx, hip_stream);
  return align_batch_locked(ctx, b, out);
}

int swx_align_batch_noalloc(swx_ctx *ctx, const swx_batch *b, swx_batch_out *out,
                            void *hip_stream) {
  if (!ctx || !b || !out) return fail(SWX_EINVAL, "null argument");
  if (b->npairs > SWX_NOALLOC_MAX_PAIRS)
    return fail(SWX_EINVAL, "batch above SWX_NOALLOC_MAX_PAIRS pairs");
  // host-memory inputs are staged in the scratch too
  if (b->in_mem == SWX_MEM_HOST) {
    const int64_t staged = b->qcat_len + b->rcat_len + 8 * (b->nq + b->nr + 2 + 2 * b->npairs);
    if (staged < 0 || staged > (int64_t)SWX_NOALLOC_SCRATCH_BYTES / 2)
      return fail(SWX_EINVAL, "inputs above half of the static scratch (SWX_NOALLOC_SCRATCH_BYTES)");
  }
  if (!ctx->scratch || ctx->device < 0 || ctx->device >= kMaxDevices)
    return fail(SWX_EDEVICE, "no static scratch on this device");
  std::lock_guard<std::mutex> dev(g_scratch_use[ctx->device]);
  std::lock_guard<std::mutex> g(ctx->mu);
  StreamScope ss(ctx, hip_stream);
  struct Restore {   // pool mode and side streams as they were, whatever happens
    swx_ctx *c;
    bool side;
    ~Restore() {
      c->arena.use_pool();
      c->side_streams = side;
    }
  } restore{ctx, ctx->side_streams};
  ctx->arena.use_fixed(ctx->scratch, SWX_NOALLOC_SCRATCH_BYTES);
  ctx->side_streams = false;   // making side streams would allocate
  int rc = align_batch_locked(ctx, b, out);
  const bool short_of_scratch = ctx->arena.fixed_exhausted();
  // the scratch is free for the next call only once this call's work is done
  if (wait_stream(ctx->stream) != hipSuccess && rc == SWX_OK)
    rc = fail(SWX_EDEVICE, "stream wait failed");
  if (rc == SWX_ENOMEM && short_of_scratch)
    rc = fail(SWX_ENOMEM, "the batch needs more device scratch than the static "
                          "SWX_NOALLOC_SCRATCH_BYTES; split it or use swx_align_batch");
  return rc;
}

// The one-pair call through a cached graph (intra route: the pair spread over
// a wave).  Returns 1 when no graph serves the pair (too large, or one could
// not be made): the caller then takes the batch path.
static constexpr int32_t kPairGraphMaxQ = 4096;
static constexpr int64_t kPairGraphMaxR = int64_t(1) << 16;
static constexpr size_t kPairGraphs = 8;

static int graph_run_on(swx_graph *gr, void *hip_stream);

static int align_pair_graph(const swx_profile *p, int64_t rlen, uint32_t flags,
                            int32_t mask_len, const swx_batch &b, void *hip_stream, swx_rec &rec,
                            std::vector<uint32_t> &cig) {
  swx_ctx *ctx = p->ctx;
  const int64_t ql = (int64_t)p->query.size();
  if (ql > kPairGraphMaxQ || rlen > kPairGraphMaxR) return 1;
  int32_t qcap = 64;
  while (qcap < ql) qcap *= 2;
  int64_t rcap = 256;
  while (rcap < rlen) rcap *= 2;
  std::lock_guard<std::mutex> lk(ctx->pair_mu);
  swx_ctx::PairGraph *hit = nullptr;
  for (auto &pg : ctx->pair_graphs)
    if (pg.n == p->n && pg.o == p->o && pg.e == p->e && pg.flags == flags &&
        pg.mask_len == mask_len && pg.qcap == qcap && pg.rcap == rcap && pg.matrix == p->matrix) {
      hit = &pg;
      break;
    }
  if (!hit) {
    if (ctx->pair_graphs.size() >= kPairGraphs) {   // evict the least recently used
      size_t old = 0;
      for (size_t k = 1; k < ctx->pair_graphs.size(); ++k)
        if (ctx->pair_graphs[k].last_use < ctx->pair_graphs[old].last_use) old = k;
      swx_graph_destroy(ctx->pair_graphs[old].g);
      ctx->pair_graphs.erase(ctx->pair_graphs.begin() + (std::ptrdiff_t)old);
    }
    swx_graph_cfg cfg{};
    cfg.matrix = p->matrix.data(); cfg.n = p->n; cfg.gap_open = p->o; cfg.gap_extend = p->e;
    cfg.max_pairs = 1; cfg.max_qlen = qcap; cfg.max_rlen = rcap;
    cfg.qcat_cap = qcap; cfg.rcat_cap = rcap; cfg.nq_cap = 1; cfg.nr_cap = 2;
    cfg.flags = flags; cfg.mask_len = mask_len; cfg.route = SWX_ROUTE_INTRA;
    swx_graph *gr = nullptr;
    swx_graph_io io{};
    if (swx_graph_create(ctx, &cfg, &gr, &io) != SWX_OK) return 1;
    swx_ctx::PairGraph pg;
    pg.matrix = p->matrix; pg.n = p->n; pg.o = p->o; pg.e = p->e;
    pg.flags = flags; pg.mask_len = mask_len; pg.qcap = qcap; pg.rcap = rcap; pg.g = gr;
    ctx->pair_graphs.push_back(std::move(pg));
    hit = &ctx->pair_graphs.back();
  }
  hit->last_use = ++ctx->pair_clock;
  int rc = swx_graph_load(hit->g, &b);
  if (rc == SWX_OK) rc = graph_run_on(hit->g, hip_stream);
  if (rc != SWX_OK) return rc;
  swx_batch_out bo{&rec, cig.data(), (int64_t)cig.size(), 0, SWX_MEM_HOST};
  return swx_graph_read(hit->g, 1, &bo);
}

int swx_align(const swx_profile *p, const int8_t *ref, int64_t rlen, uint32_t flags,
              int32_t mask_len, void *hip_stream, swx_result *out) {
  if (!p || !out || (rlen > 0 && !ref)) return fail(SWX_EINVAL, "null argument");
  if (rlen < 0) return fail(SWX_EINVAL, "rlen must be >= 0");
  if (flags & ~(SWX_ALL | SWX_SUBOPT | SWX_REF_DEVICE)) return fail(SWX_EINVAL, "unknown flag bits");
  swx_ctx *ctx = p->ctx;
  memset(out, 0, sizeof(*out));
  const bool subopt = (flags & SWX_SUBOPT) != 0;
  if (subopt) flags |= SWX_ALL;
  std::vector<int8_t> href;
  const int8_t *rptr = ref;
  if (flags & SWX_REF_DEVICE) {
    href.resize((size_t)rlen);
    // ordered after the caller's work on its stream (which may write ref)
    if (rlen) {
      if (hip_stream) {
        if (hipMemcpyAsync(href.data(), ref, (size_t)rlen, hipMemcpyDeviceToHost,
                           (hipStream_t)hip_stream) != hipSuccess ||
            wait_stream((hipStream_t)hip_stream) != hipSuccess)
          return fail(SWX_EDEVICE, "could not read the device reference");
      } else if (hipMemcpy(href.data(), ref, (size_t)rlen, hipMemcpyDeviceToHost) != hipSuccess) {
        return fail(SWX_EDEVICE, "could not read the device reference");
      }
    }
    rptr = href.data();
  }
  if (!subopt) {
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
    const int rc = align_pair_graph(p, rlen, flags & SWX_ALL, mask_len, b, hip_stream, rec, cig);
    if (rc < 0) return rc;
    if (rc == SWX_OK) {
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
  }
  std::lock_guard<std::mutex> g(ctx->mu);
  StreamScope ss(ctx, hip_stream);
  const int64_t qoff[2] = {0, (int64_t)p->query.size()};
  const int64_t roff[2] = {0, rlen};
  const int64_t pq = 0, pr = 0;
  swx_batch b{};
  b.matrix = p->matrix.data(); b.n = p->n; b.gap_open = p->o; b.gap_extend = p->e;
  b.qcat = p->query.data(); b.qcat_len = (int64_t)p->query.size(); b.qoff = qoff; b.nq = 1;
  b.rcat = rptr; b.rcat_len = rlen; b.roff = roff; b.nr = 1;
  b.pair_q = &pq; b.pair_r = &pr; b.npairs = 1;
  b.flags = flags & (SWX_ALL | SWX_SUBOPT); b.mask_len = mask_len; b.in_mem = SWX_MEM_HOST;
  swx_rec rec{}, sub{};
  // the suboptimal alignment's CIGAR goes to the same arena
  std::vector<uint32_t> cig((size_t)((subopt ? 2 : 1) * (p->query.size() + rlen + 2)));
  swx_batch_out bo{&rec, cig.data(), (int64_t)cig.size(), 0, SWX_MEM_HOST, 0, subopt ? &sub : nullptr};
  int rc = align_batch_locked(ctx, &b, &bo, p);
  if (rc) return rc;
  auto copy_out = [&](const swx_rec &r, swx_rec &dst, uint32_t *&dcig) {
    dst = r;
    dcig = nullptr;
    if (r.cigar_len > 0) {
      dcig = (uint32_t *)malloc(sizeof(uint32_t) * r.cigar_len);
      if (!dcig) return false;
      memcpy(dcig, cig.data() + r.cigar_off, sizeof(uint32_t) * r.cigar_len);
    }
    dst.cigar_off = 0;
    return true;
  };
  if (!copy_out(rec, out->rec, out->cigar) || (subopt && !copy_out(sub, out->sub, out->sub_cigar))) {
    swx_result_free(out);
    return fail(SWX_ENOMEM, "host allocation failed");
  }
  return SWX_OK;
}

}  // extern "C"

// ---- graph mode ---------------------------------------------------------------
struct swx_graph {
  swx_ctx *ctx = nullptr;
  swx::GraphState g;
};

extern "C" {

int swx_graph_create(swx_ctx *ctx, const swx_graph_cfg *cfg, swx_graph **out, swx_graph_io *io) {
  if (!ctx || !cfg || !out || !io) return fail(SWX_EINVAL, "null argument");
  *out = nullptr;
  if (cfg->max_pairs < 1 || cfg->max_qlen < 1 || cfg->max_rlen < 0 || cfg->qcat_cap < 0 ||
      cfg->rcat_cap < 0 || cfg->nq_cap < 1 || cfg->nr_cap < 1 || (cfg->flags & ~SWX_ALL))
    return fail(SWX_EINVAL, "bad graph capacities or flags");
  std::lock_guard<std::mutex> lk(ctx->mu);
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(SWX_EDEVICE, "hipSetDevice failed");
  swx_graph *gr = new (std::nothrow) swx_graph();
  if (!gr) return fail(SWX_ENOMEM, "host allocation failed");
  gr->ctx = ctx;
  GraphState &g = gr->g;
  g.cfg = *cfg;
  g.matrix.assign(cfg->matrix, cfg->matrix + (size_t)cfg->n * cfg->n);
  g.cfg.matrix = g.matrix.data();
  int rc = make_scoring(g.matrix.data(), cfg->n, cfg->gap_open, cfg->gap_extend, &g.sc);
  if (rc) { delete gr; return rc; }
  g.B = cfg->max_pairs;
  g.QM = cfg->max_qlen;
  g.RM = cfg->max_rlen;
  const int64_t bound = (int64_t)std::max(g.sc.smax, 0) * std::min<int64_t>(g.QM, g.RM);
  if (bound >= (1 << 26) - 1) { delete gr; return fail(SWX_EOVERFLOW, "scores could exceed the lane range"); }
  g.clamp = bound > kInter16Limit - 1;
  g.pair3 = bound <= kInter16PairLimit;
  g.need32 = bound >= kInter16Limit;
  g.intra = cfg->route == SWX_ROUTE_INTRA;
  g.fill_sched = ctx->fill_sched;
  g.fill_coop = ctx->fill_coop;
  g.cus = ctx->cus;
  int8_t *dmat = g.A.get<int8_t>((int64_t)g.sc.n * g.sc.n);
  if (!dmat) { delete gr; return fail(SWX_ENOMEM, "device pool exhausted"); }
  if (hipMemcpy(dmat, g.matrix.data(), (size_t)g.sc.n * g.sc.n, hipMemcpyHostToDevice) != hipSuccess) {
    delete gr;
    return fail(SWX_EDEVICE, "could not upload the matrix");
  }
  g.sc.dmat = dmat;
  if ((rc = graph_alloc(g))) { delete gr; return rc; }
  // valid empty contents: every code 0, every offset 0, every pair (0, 0)
  hipStream_t st = ctx->stream;
  bool ok = fill_u8(g.cfg.qcat_cap, (uint8_t *)g.qcat, 0, st) == hipSuccess &&
            fill_u8(g.cfg.rcat_cap, (uint8_t *)g.rcat, 0, st) == hipSuccess &&
            fill_i64(g.cfg.nq_cap + 1, g.qoff, 0, st) == hipSuccess &&
            fill_i64(g.cfg.nr_cap + 1, g.roff, 0, st) == hipSuccess &&
            fill_i64(g.B, g.pair_q, 0, st) == hipSuccess && fill_i64(g.B, g.pair_r, 0, st) == hipSuccess &&
            hipStreamSynchronize(st) == hipSuccess;
  if (!ok) { delete gr; return fail(SWX_EDEVICE, "could not clear the graph buffers"); }
  // capture the whole chain once
  if (hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    delete gr;
    return fail(SWX_EDEVICE, "could not begin stream capture");
  }
  rc = fixed_issue(g, st);
  hipGraph_t graph = nullptr;
  const hipError_t ce = hipStreamEndCapture(st, &graph);
  if (rc != SWX_OK || ce != hipSuccess || !graph) {
    if (graph) hipGraphDestroy(graph);
    delete gr;
    return rc != SWX_OK ? rc : fail(SWX_EDEVICE, "stream capture failed");
  }
  g.graph = graph;
  if (hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0) != hipSuccess) {
    hipGraphDestroy(graph);
    delete gr;
    return fail(SWX_EDEVICE, "could not instantiate the graph");
  }
  io->qcat = g.qcat; io->qoff = g.qoff; io->rcat = g.rcat; io->roff = g.roff;
  io->pair_q = g.pair_q; io->pair_r = g.pair_r;
  io->recs = (swx_rec *)g.recs;
  io->cigar = g.cigar;
  io->cigar_cap = g.cigar_cap;
  *out = gr;
  return SWX_OK;
}

// waits for the stream and reads the run's flags; the caller holds ctx->mu
static int graph_check(swx_graph *gr) {
  GraphState &g = gr->g;
  swx_ctx *ctx = gr->ctx;
  if (hipMemcpyAsync(ctx->pinned, g.bad, 4, hipMemcpyDeviceToHost, ctx->stream) != hipSuccess ||
      hipMemcpyAsync(ctx->pinned + 1, g.status, 8, hipMemcpyDeviceToHost, ctx->stream) != hipSuccess ||
      wait_stream(ctx->stream) != hipSuccess)
    return fail(SWX_EDEVICE, "could not read the graph status");
  uint32_t bad = 0;
  memcpy(&bad, ctx->pinned, 4);
  const int64_t nerr = ctx->pinned[1];
  if (bad & 1u) return fail(SWX_EINVAL, "offsets must be non-decreasing and within the code arrays");
  if (bad & 2u) return fail(SWX_EINVAL, "pair index out of range");
  if (bad & 12u) return fail(SWX_EINVAL, "symbol code outside [0, n)");
  if (nerr) return fail(SWX_EINTERNAL, "internal consistency check failed");
  return SWX_OK;
}

static int graph_run_on(swx_graph *gr, void *hip_stream) {
  std::lock_guard<std::mutex> lk(gr->ctx->mu);
  StreamScope ss(gr->ctx, hip_stream);
  if (hipSetDevice(gr->ctx->device) != hipSuccess) return fail(SWX_EDEVICE, "hipSetDevice failed");
  HIP_TRY(hipGraphLaunch(gr->g.exec, gr->ctx->stream));
  return graph_check(gr);
}

int swx_graph_run(swx_graph *gr, void *hip_stream) {
  if (!gr) return fail(SWX_EINVAL, "null argument");
  return graph_run_on(gr, hip_stream);
}

int swx_graph_run_eager(swx_graph *gr, void *hip_stream) {
  if (!gr) return fail(SWX_EINVAL, "null argument");
  std::lock_guard<std::mutex> lk(gr->ctx->mu);
  StreamScope ss(gr->ctx, hip_stream);
  if (hipSetDevice(gr->ctx->device) != hipSuccess) return fail(SWX_EDEVICE, "hipSetDevice failed");
  int rc = fixed_issue(gr->g, gr->ctx->stream);
  if (rc) return rc;
  return graph_check(gr);
}

int swx_graph_load(swx_graph *gr, const swx_batch *b) {
  if (!gr || !b) return fail(SWX_EINVAL, "null argument");
  GraphState &g = gr->g;
  if (b->in_mem != SWX_MEM_HOST) return fail(SWX_EINVAL, "swx_graph_load takes host memory");
  if (b->npairs < 0 || b->npairs > g.B || b->nq < 1 || b->nq > g.cfg.nq_cap ||
      b->nr < 0 || b->nr + 1 > g.cfg.nr_cap || b->qcat_len > g.cfg.qcat_cap ||
      b->rcat_len > g.cfg.rcat_cap || !b->qoff || !b->roff ||
      (b->npairs && (!b->pair_q || !b->pair_r)) || (b->qcat_len && !b->qcat) ||
      (b->rcat_len && !b->rcat))
    return fail(SWX_EINVAL, "batch does not fit the graph's capacities");
  // the host holds the whole batch here: offsets, pair indices and lengths
  // are checked before anything reaches the device
  for (int64_t k = 0; k < b->nq; ++k)
    if (b->qoff[k] < 0 || b->qoff[k] > b->qoff[k + 1] || b->qoff[k + 1] > b->qcat_len)
      return fail(SWX_EINVAL, "offsets must be non-decreasing and within the code arrays");
  for (int64_t k = 0; k < b->nr; ++k)
    if (b->roff[k] < 0 || b->roff[k] > b->roff[k + 1] || b->roff[k + 1] > b->rcat_len)
      return fail(SWX_EINVAL, "offsets must be non-decreasing and within the code arrays");
  for (int64_t k = 0; k < b->npairs; ++k) {
    const int64_t qi = b->pair_q[k], ri = b->pair_r[k];
    if (qi < 0 || qi >= b->nq || ri < 0 || ri >= b->nr)
      return fail(SWX_EINVAL, "pair index out of range");
    if (b->qoff[qi + 1] - b->qoff[qi] > g.QM || b->roff[ri + 1] - b->roff[ri] > g.RM)
      return fail(SWX_EINVAL, "a pair exceeds the graph's length capacities");
  }
  // symbols too: a rejected code must never reach the device buffers, where
  // it would outlive this load past the next, shorter one (every run checks
  // the whole code arrays)
  for (int64_t k = 0; k < b->qcat_len; ++k)
    if (b->qcat[k] < 0 || b->qcat[k] >= g.sc.n) return fail(SWX_EINVAL, "symbol code outside [0, n)");
  for (int64_t k = 0; k < b->rcat_len; ++k)
    if (b->rcat[k] < 0 || b->rcat[k] >= g.sc.n) return fail(SWX_EINVAL, "symbol code outside [0, n)");
  // offsets padded with their last value; pair slots past npairs take the
  // empty reference nr (roff[nr] == roff[nr + 1])
  std::vector<int64_t> qo(g.cfg.nq_cap + 1), ro(g.cfg.nr_cap + 1), pq(g.B, 0), pr(g.B, b->nr);
  for (int64_t k = 0; k <= g.cfg.nq_cap; ++k) qo[k] = b->qoff[std::min(k, b->nq)];
  for (int64_t k = 0; k <= g.cfg.nr_cap; ++k) ro[k] = b->roff[std::min(k, b->nr)];
  for (int64_t k = 0; k < b->npairs; ++k) { pq[k] = b->pair_q[k]; pr[k] = b->pair_r[k]; }
  std::lock_guard<std::mutex> lk(gr->ctx->mu);
  hipStream_t st = gr->ctx->stream;
  if (b->qcat_len) HIP_TRY(hipMemcpyAsync(g.qcat, b->qcat, b->qcat_len, hipMemcpyHostToDevice, st));
  if (b->rcat_len) HIP_TRY(hipMemcpyAsync(g.rcat, b->rcat, b->rcat_len, hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(g.qoff, qo.data(), 8 * qo.size(), hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(g.roff, ro.data(), 8 * ro.size(), hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(g.pair_q, pq.data(), 8 * pq.size(), hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(g.pair_r, pr.data(), 8 * pr.size(), hipMemcpyHostToDevice, st));
  HIP_TRY(wait_stream(st));   // the host vectors must outlive the copies
  return SWX_OK;
}

int swx_graph_read(swx_graph *gr, int64_t npairs, swx_batch_out *out) {
  if (!gr || !out || npairs < 0 || npairs > gr->g.B || (npairs && !out->recs))
    return fail(SWX_EINVAL, "bad arguments");
  GraphState &g = gr->g;
  std::lock_guard<std::mutex> lk(gr->ctx->mu);
  if (npairs == 0) { out->cigar_used = 0; return SWX_OK; }
  HIP_TRY(hipMemcpy(out->recs, g.recs, sizeof(swx_rec) * npairs, hipMemcpyDeviceToHost));
  int64_t used = 0;
  for (int64_t k = 0; k < npairs; ++k)
    used = std::max<int64_t>(used, out->recs[k].cigar_off + out->recs[k].cigar_len);
  out->cigar_used = used;
  if (used > out->cigar_cap || (used && !out->cigar)) return fail(SWX_ERANGE, "CIGAR arena too small");
  if (used) HIP_TRY(hipMemcpy(out->cigar, g.cigar, sizeof(uint32_t) * used, hipMemcpyDeviceToHost));
  return SWX_OK;
}

int swx_graph_destroy(swx_graph *gr) {
  if (!gr) return fail(SWX_EINVAL, "null argument");
  {
    std::lock_guard<std::mutex> lk(gr->ctx->mu);
    (void)hipSetDevice(gr->ctx->device);
    (void)hipStreamSynchronize(gr->ctx->stream);
    if (gr->g.exec) (void)hipGraphExecDestroy(gr->g.exec);
    if (gr->g.graph) (void)hipGraphDestroy(gr->g.graph);
    gr->g.A.release();
  }
  delete gr;
  return SWX_OK;
}

}  // extern "C"
