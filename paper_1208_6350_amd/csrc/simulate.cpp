// simulate.cpp -- the serving policy replayed on a virtual clock.
//
// A discrete-event loop over arrivals and batch completions drives the same
// policy code as the serving loop (footprints, size classes, admission,
// worker-to-class rule and FIFO batch formation) against a
// modelled GPU, so that admission and queueing can be checked on a host
// without a device, deterministically.
#include <cmath>
#include <deque>
#include <limits>
#include <vector>

#include "../../include/swx.h"
#include "runtime_internal.h"
#include "serve_policy.h"

namespace {

struct SimItem {
  int64_t idx;
  int64_t footprint;
};

struct SimWorker {
  bool busy = false;
  double done_us = 0;
  int cls = 0;
  int64_t fp = 0;
  std::vector<SimItem> batch;
};

}  // namespace

extern "C" int swx_server_simulate(const swx_server_cfg *cfg_in, const swx_sim_model *model,
                                   const swx_sim_request *rq, int64_t n, swx_sim_result *out,
                                   swx_server_stats *stats) {
  if (!cfg_in || !model || n < 0 || (n > 0 && (!rq || !out)))
    return swx::internal_fail(SWX_EINVAL, "null argument");
  if (!(model->cells_per_us > 0) || model->batch_us < 0 || model->request_us < 0)
    return swx::internal_fail(SWX_EINVAL, "bad model");
  for (int64_t k = 0; k < n; ++k) {
    if (rq[k].qlen < 0 || rq[k].rlen < 0 || !std::isfinite(rq[k].arrival_us))
      return swx::internal_fail(SWX_EINVAL, "bad request");
    if (k > 0 && rq[k].arrival_us < rq[k - 1].arrival_us)
      return swx::internal_fail(SWX_EINVAL, "arrivals out of order");
  }
  swx_server_cfg cfg = *cfg_in;
  swx_sched::apply_defaults(cfg);
  swx_server_stats st{};
  swx_sched::Budget budget;
  std::deque<SimItem> pending[2];
  std::vector<SimWorker> workers((size_t)cfg.workers);
  int64_t next_batch = 0;
  for (int64_t k = 0; k < n; ++k) {
    out[k] = swx_sim_result{};
    out[k].start_us = out[k].done_us = -1;
    out[k].batch_id = -1;
    out[k].worker = -1;
    out[k].footprint = swx_sched::footprint(rq[k].qlen, rq[k].rlen, cfg.n);
    out[k].cls = swx_sched::size_class(rq[k].qlen, rq[k].rlen, cfg.long_cells);
    out[k].status = SWX_OK;
  }

  auto dispatch = [&](double t) {
    for (int w = 0; w < cfg.workers; ++w) {
      SimWorker &wk = workers[(size_t)w];
      if (wk.busy) continue;
      const int c = swx_sched::pick_class(cfg, budget, pending, w);
      if (c < 0) continue;
      wk.batch.clear();
      wk.fp = swx_sched::take_batch(cfg, budget, pending[c], c, wk.batch);
      wk.cls = c;
      double cells = 0;
      for (const SimItem &it : wk.batch) cells += (double)rq[it.idx].qlen * (double)rq[it.idx].rlen;
      const double dur = model->batch_us + model->request_us * (double)wk.batch.size() +
                         cells / model->cells_per_us;
      wk.busy = true;
      wk.done_us = t + dur;
      for (const SimItem &it : wk.batch) {
        swx_sim_result &r = out[it.idx];
        r.start_us = t;
        r.done_us = wk.done_us;
        r.batch_id = next_batch;
        r.worker = w;
        r.batch_size = (int32_t)wk.batch.size();
      }
      ++next_batch;
      st.admitted += (int64_t)wk.batch.size();
      st.batches += 1;
      st.max_batch_seen = std::max<int64_t>(st.max_batch_seen, (int64_t)wk.batch.size());
      st.peak_inflight_bytes = std::max(st.peak_inflight_bytes, budget.inflight);
    }
  };

  const double inf = std::numeric_limits<double>::infinity();
  int64_t a = 0;
  for (;;) {
    int wdone = -1;
    double t_done = inf;
    for (int w = 0; w < cfg.workers; ++w)
      if (workers[(size_t)w].busy && workers[(size_t)w].done_us < t_done) {
        t_done = workers[(size_t)w].done_us;
        wdone = w;
      }
    const double t_arr = a < n ? rq[a].arrival_us : inf;
    if (wdone < 0 && a >= n) break;
    double t;
    if (wdone >= 0 && t_done <= t_arr) {   // a batch completes
      SimWorker &wk = workers[(size_t)wdone];
      swx_sched::release(budget, wk.cls, wk.fp);
      st.completed += (int64_t)wk.batch.size();
      wk.busy = false;
      t = t_done;
    } else {                                // a request arrives
      t = t_arr;
      if ((int64_t)pending[out[a].cls].size() >= cfg.max_pending) {
        out[a].status = SWX_EBUSY;
        st.deferred += 1;
      } else {
        pending[out[a].cls].push_back(SimItem{a, out[a].footprint});
        st.submitted += 1;
      }
      ++a;
    }
    dispatch(t);
  }
  st.pending = (int64_t)(pending[0].size() + pending[1].size());
  st.inflight_bytes = budget.inflight;
  if (stats) *stats = st;
  return SWX_OK;
}
