// serve_policy.h -- the serving policy: request footprints, size classes, admission
// against the device-memory budget and batch formation.  Host-only and free
// of device calls, so that the serving loop (server.cpp) and its
// discrete-event simulator (simulate.cpp) run exactly the same decisions.
#pragma once

#include <algorithm>
#include <cstdint>
#include <deque>
#include <vector>

#include "../../include/swx.h"

namespace swx_sched {

// Device bytes a request's work takes while it runs: sequences, boundary
// rows and max array (about 64 bytes per query or reference symbol), the
// query profile, and the traceback band (one nibble per cell of a band at
// most as wide as the query, plus slack).
inline int64_t footprint(int64_t qlen, int64_t rlen, int32_t n) {
  const int64_t band = std::min<int64_t>(rlen, qlen + 64);
  return 64 * (qlen + rlen) + (int64_t)(n + 1) * qlen + qlen * band / 2 + 4096;
}

// 0: short, 1: long (query x reference cells above the threshold)
inline int size_class(int64_t qlen, int64_t rlen, int64_t long_cells) {
  return qlen * rlen > long_cells ? 1 : 0;
}

// Footprint of the work in flight, in total and the part held by long requests.
struct Budget {
  int64_t inflight = 0;
  int64_t inflight_long = 0;
};

// Fills in the defaults of a server configuration (the documented ones).
inline void apply_defaults(swx_server_cfg &c) {
  if (c.mem_budget <= 0) c.mem_budget = int64_t(4) << 30;
  if (c.max_pending <= 0) c.max_pending = 1 << 20;
  if (c.workers <= 0) c.workers = 3;
  if (c.workers > 16) c.workers = 16;
  if (c.max_batch <= 0) c.max_batch = 1 << 16;
  if (c.long_cells <= 0) c.long_cells = int64_t(1) << 22;
  if (c.graph_batch < 0) c.graph_batch = 0;
  if (c.graph_batch > 0) {
    if (c.graph_max_qlen <= 0) c.graph_max_qlen = 256;
    if (c.graph_max_rlen <= 0) c.graph_max_rlen = 1536;
  }
}

// Can a request of footprint fp and class cls join a batch that already holds
// `extra` bytes?  Long requests may hold at most 3/4 of the budget, so short
// ones always find room; a request larger than its share still runs once
// nothing else does.
inline bool admissible(const swx_server_cfg &c, const Budget &b, int64_t fp, int cls,
                       int64_t extra) {
  if (b.inflight == 0 && extra == 0) return true;
  if (b.inflight + extra + fp > c.mem_budget) return false;
  return cls == 0 || b.inflight_long + extra + fp <= c.mem_budget / 4 * 3;
}

// A long request above the long requests' share can only start on an idle
// device: it needs the device alone.
inline bool needs_device_alone(const swx_server_cfg &c, int64_t fp) {
  return fp > c.mem_budget / 4 * 3;
}

// The class worker w serves next, or -1.  Worker 0 serves only short
// requests (when there are other workers), so a short request never waits
// behind a batch of long ones; the others prefer long requests and take
// short ones when no long request is admissible.  Drain: while the head of
// the long queue needs the device alone, no new batch of short requests
// starts, so that the work in flight drains and the long request runs on the
// idle device (otherwise steady short traffic would keep the device from
// ever being idle and hold it, and every long request behind it, back for
// good).  Q is a queue of items with a `footprint` member.
template <class Q>
int pick_class(const swx_server_cfg &c, const Budget &b, const Q pending[2], int w) {
  const bool drain = !pending[1].empty() && needs_device_alone(c, pending[1].front().footprint);
  auto ok = [&](int k) {
    if (k == 0 && drain) return false;
    return !pending[k].empty() && admissible(c, b, pending[k].front().footprint, k, 0);
  };
  if (w == 0 && c.workers > 1) return ok(0) ? 0 : -1;
  for (int k : {1, 0})
    if (ok(k)) return k;
  return -1;
}

// Moves the admissible head of queue `cls` (FIFO, up to max_batch requests)
// into `batch` and charges it to the budget.  Returns the bytes charged.
template <class Q, class V>
int64_t take_batch(const swx_server_cfg &c, Budget &b, Q &q, int cls, V &batch) {
  int64_t fp = 0;
  while (!q.empty() && (int64_t)batch.size() < c.max_batch &&
         admissible(c, b, q.front().footprint, cls, fp)) {
    fp += q.front().footprint;
    batch.push_back(std::move(q.front()));
    q.pop_front();
  }
  b.inflight += fp;
  if (cls == 1) b.inflight_long += fp;
  return fp;
}

// Returns a finished batch's bytes to the budget.
inline void release(Budget &b, int cls, int64_t fp) {
  b.inflight -= fp;
  if (cls == 1) b.inflight_long -= fp;
}

}  // namespace swx_sched
