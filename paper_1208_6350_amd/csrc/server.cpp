// server.cpp -- serving loop: resident queries, footprint admission and
// continuous batching on top of the batch path.
//
// Requests (a query -- registered once and kept on the device, or inline --
// and a reference) are queued by swx_server_submit, short and long ones
// (query x reference cells above long_cells) in separate FIFO queues.  Each of
// `workers` worker threads owns a library context (its own HIP stream and
// device pool); when a worker is free it takes every queued request of one
// class that fits the device-memory budget (up to max_batch), runs them as one
// batch and posts completions.
// Requests that arrive while batches run are picked up by the next free
// worker, so several batches of mixed sizes overlap on the GPU.  A request's
// results do not depend on the batch it lands in (the batch path is exact and
// batch-independent), which the tests check against the request run alone.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/swx.h"
#include "runtime_internal.h"
#include "serve_policy.h"

namespace {

int64_t now_ns() {
  return std::chrono::duration_cast<std::chrono::nanoseconds>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

struct Req {
  uint64_t ticket = 0, tag = 0;
  int cls = 0;                    // 0 short, 1 long (cells above the server's threshold)
  int64_t query_id = -1;          // registered query, or -1 (inline: qdata)
  std::vector<int8_t> qdata;
  std::vector<int8_t> rdata;
  int64_t footprint = 0;
  int64_t t_submit = 0;
};

// registered query: resident on the device, with a host copy for batches
// that go through a captured graph
struct RegQuery {
  int8_t *dev = nullptr;
  int32_t qlen = 0;
  std::vector<int8_t> host;
};

// growable device / pinned host buffers of one worker
struct Staging {
  void *d = nullptr;
  size_t dcap = 0;
  void *h = nullptr;
  size_t hcap = 0;
  int dev_reserve(size_t n) {
    if (n <= dcap) return 0;
    const size_t cap = std::max(n, dcap * 2);
    if (d) hipFree(d);
    d = nullptr;
    dcap = 0;
    if (hipMalloc(&d, cap) != hipSuccess) return -1;
    dcap = cap;
    return 0;
  }
  int host_reserve(size_t n) {
    if (n <= hcap) return 0;
    const size_t cap = std::max(n, hcap * 2);
    if (h) hipHostFree(h);
    h = nullptr;
    hcap = 0;
    if (hipHostMalloc(&h, cap, hipHostMallocDefault) != hipSuccess) return -1;
    hcap = cap;
    return 0;
  }
  void release() {
    if (d) hipFree(d);
    if (h) hipHostFree(h);
    d = h = nullptr;
    dcap = hcap = 0;
  }
};

}  // namespace

struct swx_server {
  swx_server_cfg cfg{};
  std::vector<int8_t> matrix;
  std::mutex mu;
  std::condition_variable cv_work;   // workers: pending work or stop
  std::condition_variable cv_done;   // pollers: completions
  std::deque<Req> pending[2];        // [0] short, [1] long requests, FIFO each
  std::deque<swx_completion> done;
  std::vector<RegQuery> queries;
  swx_sched::Budget budget;          // footprint of the work in flight
  uint64_t next_ticket = 1;
  bool stop = false;
  swx_server_stats stats{};
  std::vector<std::thread> threads;
  std::vector<swx_ctx *> ctxs;
};

namespace {

int64_t req_qlen(const swx_server *s, const Req &r) {
  return r.query_id >= 0 ? s->queries[r.query_id].qlen : (int64_t)r.qdata.size();
}

// A batch of short requests through the worker's captured graph (intra
// route: every request spread over a wave), in chunks of the graph's
// capacity.  Returns false when the requests do not fit the graph (or hold an
// empty query, which the eager path takes).
bool run_graph_batch(swx_server *s, swx_graph *g, std::vector<Req> &batch,
                     std::vector<swx_completion> &out, int64_t t_start) {
  const int64_t cap = s->cfg.graph_batch;
  for (const Req &r : batch) {
    const int64_t ql = req_qlen(s, r);
    if (ql < 1 || ql > s->cfg.graph_max_qlen || (int64_t)r.rdata.size() > s->cfg.graph_max_rlen)
      return false;
  }
  const int64_t nb = (int64_t)batch.size();
  out.resize(nb);
  for (int64_t c0 = 0; c0 < nb; c0 += cap) {
    const int64_t n = std::min(cap, nb - c0);
    std::vector<int8_t> qcat, rcat;
    std::vector<int64_t> qoff(n + 1), roff(n + 2), pq(n), pr(n);
    for (int64_t k = 0; k < n; ++k) {
      const Req &r = batch[c0 + k];
      qoff[k] = (int64_t)qcat.size();
      if (r.query_id >= 0) {
        const auto &h = s->queries[r.query_id].host;
        qcat.insert(qcat.end(), h.begin(), h.end());
      } else {
        qcat.insert(qcat.end(), r.qdata.begin(), r.qdata.end());
      }
      roff[k] = (int64_t)rcat.size();
      rcat.insert(rcat.end(), r.rdata.begin(), r.rdata.end());
      pq[k] = k;
      pr[k] = k;
    }
    qoff[n] = (int64_t)qcat.size();
    roff[n] = roff[n + 1] = (int64_t)rcat.size();   // reference n: empty, for padding
    swx_batch b{};
    b.matrix = s->matrix.data(); b.n = s->cfg.n;
    b.gap_open = s->cfg.gap_open; b.gap_extend = s->cfg.gap_extend;
    b.qcat = qcat.data(); b.qcat_len = (int64_t)qcat.size(); b.qoff = qoff.data(); b.nq = n;
    b.rcat = rcat.data(); b.rcat_len = (int64_t)rcat.size(); b.roff = roff.data(); b.nr = n;
    b.pair_q = pq.data(); b.pair_r = pr.data(); b.npairs = n;
    b.in_mem = SWX_MEM_HOST;
    std::vector<swx_rec> recs(n);
    std::vector<uint32_t> cig((size_t)std::max<int64_t>(qoff[n] + roff[n] + n, 1));
    swx_batch_out bo{};
    bo.recs = recs.data(); bo.cigar = cig.data(); bo.cigar_cap = (int64_t)cig.size();
    bo.out_mem = SWX_MEM_HOST;
    int status = swx_graph_load(g, &b);
    if (status == SWX_OK) status = swx_graph_run(g, nullptr);
    if (status == SWX_OK) status = swx_graph_read(g, n, &bo);
    const int64_t t_done = now_ns();
    for (int64_t k = 0; k < n; ++k) {
      swx_completion &c = out[c0 + k];
      memset(&c, 0, sizeof(c));
      c.ticket = batch[c0 + k].ticket;
      c.tag = batch[c0 + k].tag;
      c.status = status;
      c.t_submit_ns = batch[c0 + k].t_submit;
      c.t_start_ns = t_start;
      c.t_done_ns = t_done;
      c.batch_size = (int32_t)n;
      if (status == SWX_OK) {
        c.rec = recs[k];
        const int32_t cl = recs[k].cigar_len;
        if (cl > 0) {
          c.cigar = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)cl);
          if (c.cigar) memcpy(c.cigar, cig.data() + recs[k].cigar_off, sizeof(uint32_t) * cl);
          else c.status = SWX_ENOMEM;
        }
        c.rec.cigar_off = 0;
      }
    }
  }
  return true;
}

void finish_batch(swx_server *s, std::vector<Req> &batch, std::vector<swx_completion> &out) {
  int64_t fp = 0;
  for (const Req &r : batch) fp += r.footprint;
  const int64_t nb = (int64_t)batch.size();
  std::lock_guard<std::mutex> g(s->mu);
  swx_sched::release(s->budget, nb > 0 ? batch[0].cls : 0, fp);
  s->stats.batches += 1;
  s->stats.completed += nb;
  if (nb > s->stats.max_batch_seen) s->stats.max_batch_seen = nb;
  for (auto &c : out) s->done.push_back(c);
  s->cv_done.notify_all();
  s->cv_work.notify_all();
}

void run_batch(swx_server *s, swx_ctx *ctx, swx_graph *graph, std::vector<Req> &batch,
               Staging &stg) {
  const int64_t nb = (int64_t)batch.size();
  const int64_t t_start = now_ns();
  if (graph && nb > 0 && batch[0].cls == 0) {
    std::vector<swx_completion> gout;
    if (run_graph_batch(s, graph, batch, gout, t_start)) {
      std::lock_guard<std::mutex> g(s->mu);
      s->stats.graph_batches += 1;
    }
    if (!gout.empty()) {
      finish_batch(s, batch, gout);
      return;
    }
  }
  // layout: queries (registered ones gathered on the device, inline ones
  // copied from the host), references, offsets, pair lists
  std::vector<int64_t> qoff(nb + 1), roff(nb + 1), pq(nb), pr(nb);
  int64_t qtot = 0, rtot = 0;
  for (int64_t k = 0; k < nb; ++k) {
    const Req &r = batch[k];
    const int64_t ql = r.query_id >= 0 ? s->queries[r.query_id].qlen : (int64_t)r.qdata.size();
    qoff[k] = qtot;
    qtot += ql;
    roff[k] = rtot;
    rtot += (int64_t)r.rdata.size();
    pq[k] = k;
    pr[k] = k;
  }
  qoff[nb] = qtot;
  roff[nb] = rtot;
  auto align8 = [](int64_t x) { return (x + 7) & ~int64_t(7); };
  const int64_t o_q = 0, o_r = align8(qtot), o_qo = align8(o_r + rtot);
  const int64_t o_ro = o_qo + 8 * (nb + 1), o_pq = o_ro + 8 * (nb + 1), o_pr = o_pq + 8 * nb;
  const int64_t total = o_pr + 8 * nb;
  std::vector<swx_rec> recs(nb);
  int64_t cig_cap = qtot + rtot + nb;
  std::vector<uint32_t> cig((size_t)std::max<int64_t>(cig_cap, 1));
  int status = SWX_OK;
  hipStream_t st = nullptr;
  if (stg.dev_reserve((size_t)total) || stg.host_reserve((size_t)total)) {
    status = SWX_ENOMEM;
  } else {
    char *h = (char *)stg.h;
    for (int64_t k = 0; k < nb; ++k) {
      const Req &r = batch[k];
      if (r.query_id < 0 && !r.qdata.empty())
        memcpy(h + o_q + qoff[k], r.qdata.data(), r.qdata.size());
      if (!r.rdata.empty()) memcpy(h + o_r + roff[k], r.rdata.data(), r.rdata.size());
    }
    memcpy(h + o_qo, qoff.data(), 8 * (nb + 1));
    memcpy(h + o_ro, roff.data(), 8 * (nb + 1));
    memcpy(h + o_pq, pq.data(), 8 * nb);
    memcpy(h + o_pr, pr.data(), 8 * nb);
    st = swx::internal_stream(ctx);
    char *d = (char *)stg.d;
    if (hipMemcpyAsync(d, h, (size_t)total, hipMemcpyHostToDevice, st) != hipSuccess)
      status = SWX_EDEVICE;
    for (int64_t k = 0; k < nb && status == SWX_OK; ++k) {
      const Req &r = batch[k];
      if (r.query_id < 0) continue;
      const RegQuery &rq = s->queries[r.query_id];
      if (hipMemcpyAsync(d + o_q + qoff[k], rq.dev, (size_t)rq.qlen, hipMemcpyDeviceToDevice,
                         st) != hipSuccess)
        status = SWX_EDEVICE;
    }
    if (status == SWX_OK) {
      swx_batch b{};
      b.matrix = s->matrix.data();
      b.n = s->cfg.n;
      b.gap_open = s->cfg.gap_open;
      b.gap_extend = s->cfg.gap_extend;
      b.qcat = (const int8_t *)(d + o_q);
      b.qcat_len = qtot;
      b.qoff = (const int64_t *)(d + o_qo);
      b.nq = nb;
      b.rcat = (const int8_t *)(d + o_r);
      b.rcat_len = rtot;
      b.roff = (const int64_t *)(d + o_ro);
      b.nr = nb;
      b.pair_q = (const int64_t *)(d + o_pq);
      b.pair_r = (const int64_t *)(d + o_pr);
      b.npairs = nb;
      b.flags = s->cfg.flags;
      b.mask_len = s->cfg.mask_len;
      b.in_mem = SWX_MEM_DEVICE;
      swx_batch_out bo{};
      bo.recs = recs.data();
      bo.cigar = cig.data();
      bo.cigar_cap = cig_cap;
      bo.out_mem = SWX_MEM_HOST;
      status = swx_align_batch(ctx, &b, &bo, nullptr);
    }
  }
  const int64_t t_done = now_ns();
  std::vector<swx_completion> out(nb);
  for (int64_t k = 0; k < nb; ++k) {
    swx_completion &c = out[k];
    memset(&c, 0, sizeof(c));
    c.ticket = batch[k].ticket;
    c.tag = batch[k].tag;
    c.status = status;
    c.t_submit_ns = batch[k].t_submit;
    c.t_start_ns = t_start;
    c.t_done_ns = t_done;
    c.batch_size = (int32_t)nb;
    if (status == SWX_OK) {
      c.rec = recs[k];
      const int32_t cl = recs[k].cigar_len;
      if (cl > 0) {
        c.cigar = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)cl);
        if (c.cigar) memcpy(c.cigar, cig.data() + recs[k].cigar_off, sizeof(uint32_t) * cl);
        else c.status = SWX_ENOMEM;
      }
      c.rec.cigar_off = 0;
    }
  }
  finish_batch(s, batch, out);
}

void worker_main(swx_server *s, int w) {
  swx_ctx *ctx = s->ctxs[w];
  Staging stg;
  std::vector<Req> batch;
  // the short-request worker replays a captured graph
  swx_graph *graph = nullptr;
  if (w == 0 && s->cfg.graph_batch > 0) {
    swx_graph_cfg gc{};
    gc.matrix = s->matrix.data(); gc.n = s->cfg.n;
    gc.gap_open = s->cfg.gap_open; gc.gap_extend = s->cfg.gap_extend;
    gc.max_pairs = s->cfg.graph_batch;
    gc.max_qlen = s->cfg.graph_max_qlen;
    gc.max_rlen = s->cfg.graph_max_rlen;
    gc.qcat_cap = (int64_t)s->cfg.graph_batch * s->cfg.graph_max_qlen;
    gc.rcat_cap = (int64_t)s->cfg.graph_batch * s->cfg.graph_max_rlen + 8;
    gc.nq_cap = s->cfg.graph_batch + 1;
    gc.nr_cap = s->cfg.graph_batch + 2;
    gc.flags = s->cfg.flags;
    gc.mask_len = s->cfg.mask_len;
    gc.route = SWX_ROUTE_INTRA;
    swx_graph_io io{};
    if (swx_graph_create(ctx, &gc, &graph, &io) != SWX_OK) graph = nullptr;   // eager batches then
  }
  for (;;) {
    batch.clear();
    {
      std::unique_lock<std::mutex> lk(s->mu);
      auto next = [&] { return swx_sched::pick_class(s->cfg, s->budget, s->pending, w); };
      s->cv_work.wait(lk, [&] {
        return (s->stop && s->pending[0].empty() && s->pending[1].empty()) || next() >= 0;
      });
      const int c = next();
      if (c < 0) break;   // stopping, and nothing left for this worker
      swx_sched::take_batch(s->cfg, s->budget, s->pending[c], c, batch);
      s->stats.admitted += (int64_t)batch.size();
      if (s->budget.inflight > s->stats.peak_inflight_bytes)
        s->stats.peak_inflight_bytes = s->budget.inflight;
    }
    run_batch(s, ctx, graph, batch, stg);
  }
  if (graph) swx_graph_destroy(graph);
  stg.release();
}

}  // namespace

extern "C" {

int swx_server_create(const swx_server_cfg *cfg, swx_server **out) {
  if (!cfg || !out) return swx::internal_fail(SWX_EINVAL, "null argument");
  *out = nullptr;
  if (!cfg->matrix || cfg->n < 1 || cfg->n > 32 || cfg->gap_extend < 0 ||
      cfg->gap_open < cfg->gap_extend || (cfg->flags & ~SWX_ALL))
    return swx::internal_fail(SWX_EINVAL, "bad scoring or flags");
  swx_server *s = new (std::nothrow) swx_server();
  if (!s) return swx::internal_fail(SWX_ENOMEM, "host allocation failed");
  s->cfg = *cfg;
  swx_sched::apply_defaults(s->cfg);
  s->matrix.assign(cfg->matrix, cfg->matrix + (size_t)cfg->n * cfg->n);
  s->cfg.matrix = s->matrix.data();
  for (int w = 0; w < s->cfg.workers; ++w) {
    swx_ctx *c = nullptr;
    int rc = swx_ctx_create(cfg->device, &c);
    if (rc == SWX_OK) {
      swx_tuning t{};
      rc = swx_get_tuning(c, &t);
      t.side_streams = s->cfg.side_streams < 0 ? (s->cfg.workers > 1 ? 0 : 1)
                                               : (s->cfg.side_streams ? 1 : 0);
      if (rc == SWX_OK) rc = swx_set_tuning(c, &t);
      if (rc != SWX_OK) swx_ctx_destroy(c);
    }
    if (rc != SWX_OK) {
      for (swx_ctx *x : s->ctxs) swx_ctx_destroy(x);
      delete s;
      return rc;
    }
    s->ctxs.push_back(c);
  }
  for (int w = 0; w < s->cfg.workers; ++w) s->threads.emplace_back(worker_main, s, w);
  *out = s;
  return SWX_OK;
}

int swx_server_register_query(swx_server *s, const int8_t *query, int32_t qlen, int64_t *query_id) {
  if (!s || !query || !query_id) return swx::internal_fail(SWX_EINVAL, "null argument");
  if (qlen < 1) return swx::internal_fail(SWX_EINVAL, "qlen must be >= 1");
  for (int32_t k = 0; k < qlen; ++k)
    if (query[k] < 0 || query[k] >= s->cfg.n)
      return swx::internal_fail(SWX_EINVAL, "symbol code outside [0, n)");
  RegQuery rq;
  rq.qlen = qlen;
  rq.host.assign(query, query + qlen);
  if (hipSetDevice(s->cfg.device) != hipSuccess || hipMalloc((void **)&rq.dev, (size_t)qlen) != hipSuccess)
    return swx::internal_fail(SWX_ENOMEM, "device allocation failed");
  if (hipMemcpy(rq.dev, query, (size_t)qlen, hipMemcpyHostToDevice) != hipSuccess) {
    hipFree(rq.dev);
    return swx::internal_fail(SWX_EDEVICE, "could not upload the query");
  }
  std::lock_guard<std::mutex> g(s->mu);
  *query_id = (int64_t)s->queries.size();
  s->queries.push_back(rq);
  return SWX_OK;
}

int swx_server_submit(swx_server *s, const swx_request *rq, int32_t nreq, uint64_t *tickets,
                      int32_t *naccepted) {
  if (!s || (nreq > 0 && (!rq || !tickets)) || !naccepted || nreq < 0)
    return swx::internal_fail(SWX_EINVAL, "null argument");
  *naccepted = 0;
  // the fields of every request first; then, under the lock, the prefix that
  // fits its classes' queues.  Only that prefix is checked symbol by symbol
  // and copied (an overloaded server refuses most of a large call, and must
  // not spend its time copying what it refuses); a rejected call accepts
  // nothing.
  int64_t nq;
  int32_t nfit = 0;
  {
    std::lock_guard<std::mutex> g(s->mu);
    nq = (int64_t)s->queries.size();
    for (int32_t k = 0; k < nreq; ++k) {
      const swx_request &r = rq[k];
      if (r.rlen < 0 || (r.rlen > 0 && !r.ref)) return swx::internal_fail(SWX_EINVAL, "bad reference");
      if (r.query_id >= nq) return swx::internal_fail(SWX_EINVAL, "unknown query id");
      if (r.query_id < 0 && (r.qlen < 1 || !r.query)) return swx::internal_fail(SWX_EINVAL, "bad query");
    }
    int64_t room[2] = {s->cfg.max_pending - (int64_t)s->pending[0].size(),
                       s->cfg.max_pending - (int64_t)s->pending[1].size()};
    for (; nfit < nreq; ++nfit) {
      const swx_request &r = rq[nfit];
      const int64_t ql = r.query_id < 0 ? r.qlen : s->queries[r.query_id].qlen;
      const int c = swx_sched::size_class(ql, r.rlen, s->cfg.long_cells);
      if (room[c] <= 0) break;
      --room[c];
    }
  }
  for (int32_t k = 0; k < nfit; ++k) {
    const swx_request &r = rq[k];
    if (r.query_id < 0)
      for (int32_t i = 0; i < r.qlen; ++i)
        if (r.query[i] < 0 || r.query[i] >= s->cfg.n)
          return swx::internal_fail(SWX_EINVAL, "symbol code outside [0, n)");
    for (int64_t i = 0; i < r.rlen; ++i)
      if (r.ref[i] < 0 || r.ref[i] >= s->cfg.n)
        return swx::internal_fail(SWX_EINVAL, "symbol code outside [0, n)");
  }
  const int64_t t = now_ns();
  std::vector<Req> reqs;
  reqs.reserve((size_t)nfit);
  for (int32_t k = 0; k < nfit; ++k) {
    const swx_request &r = rq[k];
    Req q;
    q.tag = r.tag;
    q.query_id = r.query_id;
    int64_t ql;
    if (r.query_id < 0) {
      q.qdata.assign(r.query, r.query + r.qlen);
      ql = r.qlen;
    } else {
      std::lock_guard<std::mutex> g(s->mu);
      ql = s->queries[r.query_id].qlen;
    }
    if (r.rlen > 0) q.rdata.assign(r.ref, r.ref + r.rlen);
    q.footprint = swx_sched::footprint(ql, r.rlen, s->cfg.n);
    q.cls = swx_sched::size_class(ql, r.rlen, s->cfg.long_cells);
    q.t_submit = t;
    reqs.push_back(std::move(q));
  }
  std::lock_guard<std::mutex> g(s->mu);
  int32_t acc = 0;
  for (Req &q : reqs) {
    // each size class has its own queue limit: a backlog of long requests
    // never refuses short ones
    if ((int64_t)s->pending[q.cls].size() >= s->cfg.max_pending) break;
    q.ticket = s->next_ticket++;
    tickets[acc++] = q.ticket;
    s->pending[q.cls].push_back(std::move(q));
  }
  *naccepted = acc;
  s->stats.submitted += acc;
  s->stats.deferred += nreq - acc;
  s->cv_work.notify_all();
  if (acc < nreq) return swx::internal_fail(SWX_EBUSY, "pending queue full");
  return SWX_OK;
}

int swx_server_poll(swx_server *s, swx_completion *done, int32_t max, int32_t timeout_us,
                    int32_t *ndone) {
  if (!s || !ndone || (max > 0 && !done) || max < 0) return swx::internal_fail(SWX_EINVAL, "null argument");
  *ndone = 0;
  std::unique_lock<std::mutex> lk(s->mu);
  if (s->done.empty() && timeout_us > 0)
    s->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), [&] { return !s->done.empty(); });
  int32_t k = 0;
  while (k < max && !s->done.empty()) {
    done[k++] = s->done.front();
    s->done.pop_front();
  }
  *ndone = k;
  return SWX_OK;
}

void swx_completion_free(swx_completion *c, int32_t n) {
  if (!c) return;
  for (int32_t k = 0; k < n; ++k) {
    free(c[k].cigar);
    c[k].cigar = nullptr;
  }
}

int swx_server_stats_get(swx_server *s, swx_server_stats *out) {
  if (!s || !out) return swx::internal_fail(SWX_EINVAL, "null argument");
  std::lock_guard<std::mutex> g(s->mu);
  *out = s->stats;
  out->pending = (int64_t)(s->pending[0].size() + s->pending[1].size());
  out->inflight_bytes = s->budget.inflight;
  return SWX_OK;
}

int swx_server_destroy(swx_server *s) {
  if (!s) return swx::internal_fail(SWX_EINVAL, "null argument");
  {
    std::lock_guard<std::mutex> g(s->mu);
    s->stop = true;
  }
  s->cv_work.notify_all();
  for (auto &t : s->threads) t.join();
  for (swx_ctx *c : s->ctxs) swx_ctx_destroy(c);
  for (RegQuery &q : s->queries) hipFree(q.dev);
  for (swx_completion &c : s->done) free(c.cigar);
  delete s;
  return SWX_OK;
}

}  // extern "C"
