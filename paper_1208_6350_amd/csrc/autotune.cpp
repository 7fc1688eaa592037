// autotune.cpp -- picks the launch configuration (swx_tuning) by timing.
//
// The knobs only move work between kernels (results never change), so the
// tuner simply runs the batch path on a sample of the caller's pairs under
// each candidate setting and keeps the fastest: one knob at a time (strip
// height of the batched fill, routing threshold between the batched and the
// intra-sequence paths, column chunks of the intra path, side streams for the
// traceback launches, task order of the batched fill), each candidate
// timed as the best of a few runs after a warm-up.  Results are kept in a
// line-per-entry JSON cache keyed by the device and a coarse signature of the
// workload (alphabet, gaps, sample size and cell count), so a later call on
// similar work reuses them without timing.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/swx.h"
#include "runtime_internal.h"

namespace {

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

int log2_bucket(double x) { return x <= 1 ? 0 : (int)std::floor(std::log2(x)); }

// host copies of the sample's offsets and pair lists (for the signature)
int sample_cells(const swx_batch *b, int64_t np, double *cells) {
  std::vector<int64_t> qoff(b->nq + 1), roff(b->nr + 1), pq(np), pr(np);
  const hipMemcpyKind k = b->in_mem == SWX_MEM_DEVICE ? hipMemcpyDeviceToHost : hipMemcpyHostToHost;
  if (hipMemcpy(qoff.data(), b->qoff, 8 * (b->nq + 1), k) != hipSuccess ||
      hipMemcpy(roff.data(), b->roff, 8 * (b->nr + 1), k) != hipSuccess ||
      (np && hipMemcpy(pq.data(), b->pair_q, 8 * np, k) != hipSuccess) ||
      (np && hipMemcpy(pr.data(), b->pair_r, 8 * np, k) != hipSuccess))
    return SWX_EDEVICE;
  double c = 0;
  for (int64_t p = 0; p < np; ++p) {
    if (pq[p] < 0 || pq[p] >= b->nq || pr[p] < 0 || pr[p] >= b->nr) return SWX_EINVAL;
    c += (double)(qoff[pq[p] + 1] - qoff[pq[p]]) * (double)(roff[pr[p] + 1] - roff[pr[p]]);
  }
  *cells = c;
  return SWX_OK;
}

std::string make_key(int device, const swx_batch *b, int64_t np, double cells) {
  hipDeviceProp_t prop{};
  hipGetDeviceProperties(&prop, device);
  char buf[256];
  snprintf(buf, sizeof buf, "%s|n%d|o%d|e%d|np%d|cells%d", prop.gcnArchName, b->n, b->gap_open,
           b->gap_extend, log2_bucket((double)np), log2_bucket(cells));
  return buf;
}

bool parse_i64(const std::string &line, const char *field, int64_t *v) {
  const std::string pat = std::string("\"") + field + "\": ";
  const size_t k = line.find(pat);
  if (k == std::string::npos) return false;
  return sscanf(line.c_str() + k + pat.size(), "%lld", (long long *)v) == 1;
}

// the last cache entry for key, if any
bool cache_lookup(const char *path, const std::string &key, swx_tuning *t) {
  if (!path) return false;
  FILE *f = fopen(path, "r");
  if (!f) return false;
  char line[1024];
  bool found = false;
  const std::string kpat = "\"key\": \"" + key + "\"";
  while (fgets(line, sizeof line, f)) {
    std::string s(line);
    if (s.find(kpat) == std::string::npos) continue;
    int64_t fr, lc, lr, ij;
    if (parse_i64(s, "fill_rows", &fr) && parse_i64(s, "long_cells", &lc) &&
        parse_i64(s, "long_rlen", &lr) && parse_i64(s, "intra_jobs", &ij)) {
      t->fill_rows = (int32_t)fr;
      t->long_cells = lc;
      t->long_rlen = lr;
      t->intra_jobs = ij;
      int64_t ss = 1, fs = 1, fc = 0, ib = 0;
      (void)parse_i64(s, "side_streams", &ss);
      (void)parse_i64(s, "fill_sched", &fs);
      (void)parse_i64(s, "fill_coop", &fc);
      (void)parse_i64(s, "intra_bits", &ib);
      t->side_streams = ss ? 1 : 0;
      t->fill_sched = (fs >= 0 && fs <= 2) ? (int32_t)fs : 1;
      t->fill_coop = (fc >= 0 && fc <= 2) ? (int32_t)fc : 0;
      t->intra_bits = (ib == 16 || ib == 32) ? (int32_t)ib : 0;
      found = true;
    }
  }
  fclose(f);
  return found;
}

void cache_store(const char *path, const std::string &key, const swx_tuning &t, double ms) {
  if (!path) return;
  FILE *f = fopen(path, "a");
  if (!f) return;
  fprintf(f,
          "{\"key\": \"%s\", \"fill_rows\": %d, \"long_cells\": %lld, \"long_rlen\": %lld, "
          "\"intra_jobs\": %lld, \"side_streams\": %d, \"fill_sched\": %d, "
          "\"fill_coop\": %d, \"intra_bits\": %d, \"ms\": %.3f}\n",
          key.c_str(), t.fill_rows, (long long)t.long_cells, (long long)t.long_rlen,
          (long long)t.intra_jobs, t.side_streams, t.fill_sched, t.fill_coop,
          t.intra_bits, ms);
  fclose(f);
}

}  // namespace

extern "C" int swx_autotune(swx_ctx *ctx, const swx_batch *b, int64_t max_pairs,
                            const char *cache_path, swx_tuning *out, int32_t *from_cache) {
  if (!ctx || !b || !out) return swx::internal_fail(SWX_EINVAL, "null argument");
  if (max_pairs < 1) return swx::internal_fail(SWX_EINVAL, "max_pairs must be >= 1");
  swx_batch s = *b;
  s.npairs = b->npairs < max_pairs ? b->npairs : max_pairs;
  if (from_cache) *from_cache = 0;
  swx_tuning cur{};
  int rc = swx_get_tuning(ctx, &cur);
  if (rc) return rc;
  if (s.npairs == 0) { *out = cur; return SWX_OK; }
  double cells = 0;
  rc = sample_cells(&s, s.npairs, &cells);
  if (rc) return swx::internal_fail(rc, "could not read the batch's offsets");
  const std::string key = make_key(swx::internal_device(ctx), &s, s.npairs, cells);
  swx_tuning cached{};
  if (cache_lookup(cache_path, key, &cached)) {
    rc = swx_set_tuning(ctx, &cached);
    if (rc) return rc;
    *out = cached;
    if (from_cache) *from_cache = 1;
    return SWX_OK;
  }
  // outputs of the timing runs: host records and CIGAR words
  std::vector<swx_rec> recs((size_t)s.npairs);
  int64_t cap = swx_cigar_bound(&s);
  std::vector<uint32_t> cig;
  swx_batch_out bo{};
  bo.recs = recs.data();
  bo.out_mem = SWX_MEM_HOST;
  if (cap < 0) {   // device inputs: size the CIGAR arena from a first run
    bo.cigar = nullptr;
    bo.cigar_cap = 0;
    rc = swx_align_batch(ctx, &s, &bo, nullptr);
    if (rc != SWX_OK && rc != SWX_ERANGE) return rc;
    cap = bo.cigar_used;
  }
  cig.resize((size_t)(cap > 0 ? cap : 1));
  bo.cigar = cig.data();
  bo.cigar_cap = cap;
  auto timed = [&](const swx_tuning &t, double *ms) -> int {
    int r = swx_set_tuning(ctx, &t);
    if (r) return r;
    double best = 1e30;
    for (int k = 0; k < 3; ++k) {   // a warm-up, then the best of two
      const double t0 = now_s();
      r = swx_align_batch(ctx, &s, &bo, nullptr);
      if (r) return r;
      const double dt = (now_s() - t0) * 1e3;
      if (k > 0 && dt < best) best = dt;
    }
    *ms = best;
    return SWX_OK;
  };
  swx_tuning best = cur;
  double best_ms = 0;
  if ((rc = timed(best, &best_ms))) return rc;
  auto try_knob = [&](auto set, std::initializer_list<int64_t> vals) -> int {
    for (int64_t v : vals) {
      swx_tuning t = best;
      set(t, v);
      if (memcmp(&t, &best, sizeof t) == 0) continue;
      double ms = 0;
      const int r = timed(t, &ms);
      if (r) return r;
      if (ms < best_ms * 0.97) { best = t; best_ms = ms; }
    }
    return SWX_OK;
  };
  if ((rc = try_knob([](swx_tuning &t, int64_t v) { t.fill_rows = (int32_t)v; }, {16, 24, 32})))
    return rc;
  if ((rc = try_knob([](swx_tuning &t, int64_t v) { t.long_cells = v; },
                     {-1, int64_t(1) << 62, 0, int64_t(1) << 20, int64_t(1) << 24})))
    return rc;
  if ((rc = try_knob([](swx_tuning &t, int64_t v) { t.intra_jobs = v; }, {1024, 2048, 4096, 8192})))
    return rc;
  if ((rc = try_knob([](swx_tuning &t, int64_t v) { t.side_streams = (int32_t)v; }, {1, 0})))
    return rc;
  if ((rc = try_knob([](swx_tuning &t, int64_t v) { t.fill_sched = (int32_t)v; }, {1, 0, 2})))
    return rc;
  if ((rc = try_knob([](swx_tuning &t, int64_t v) { t.fill_coop = (int32_t)v; }, {0, 1, 2})))
    return rc;
  if ((rc = try_knob([](swx_tuning &t, int64_t v) { t.intra_bits = (int32_t)v; }, {0, 16, 32})))
    return rc;
  if ((rc = swx_set_tuning(ctx, &best))) return rc;
  cache_store(cache_path, key, best, best_ms);
  *out = best;
  return SWX_OK;
}
