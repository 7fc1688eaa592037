// Replays seeded arrival schedules through the serving policy's simulator
// (simulate.cpp and serve_policy.h, host code only) under several
// configurations -- few and many workers, a small memory budget, a short
// pending queue, long requests above their share -- and checks the
// schedule's basic invariants, so that an AddressSanitizer /
// UndefinedBehaviorSanitizer build reports any bad access or undefined
// operation in the policy code.  Test infrastructure only.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "../../include/swx.h"

namespace swx {
// the runtime's error hook (the simulator's only dependency on it)
static thread_local std::string g_err;
int internal_fail(int code, const char *msg) {
  g_err = msg;
  return code;
}
}  // namespace swx

static uint64_t rng = 0x243F6A8885A308D3ull;
static double unit() {
  rng ^= rng >> 12; rng ^= rng << 25; rng ^= rng >> 27;
  return (double)((rng * 0x2545F4914F6CDD1Dull) >> 11) / 9007199254740992.0;
}

int main() {
  int bad = 0;
  const int64_t counts[] = {0, 1, 50, 3000};
  for (int c = 0; c < 8; ++c) {
    for (int64_t n : counts) {
      std::vector<swx_sim_request> rq((size_t)n);
      double t = 0;
      for (int64_t k = 0; k < n; ++k) {
        t += -std::log(1.0 - unit()) * (c % 2 ? 2.0 : 20.0);
        const bool lng = unit() < 0.05;
        rq[(size_t)k] = {t, lng ? 10000 : 150, lng ? 20000 : (int64_t)(1000 + 50 * (k % 7))};
      }
      swx_server_cfg cfg{};
      cfg.n = 4;
      cfg.workers = 1 + c % 4;
      cfg.mem_budget = (c & 4) ? (int64_t(64) << 20) : 0;
      cfg.max_pending = (c & 2) ? 16 : 0;
      cfg.max_batch = (c & 1) ? 32 : 0;
      swx_sim_model model{2e5, 50.0, 0.5};
      std::vector<swx_sim_result> out((size_t)n + 1);
      swx_server_stats st{};
      const int rc = swx_server_simulate(&cfg, &model, rq.data(), n, out.data(), &st);
      if (rc != SWX_OK) { std::printf("cfg %d n %lld: rc %d\n", c, (long long)n, rc); ++bad; continue; }
      int64_t done = 0, refused = 0;
      for (int64_t k = 0; k < n; ++k) {
        const swx_sim_result &r = out[(size_t)k];
        if (r.status == SWX_EBUSY) { ++refused; continue; }
        ++done;
        if (r.start_us < rq[(size_t)k].arrival_us - 1e-9 || r.done_us < r.start_us || r.batch_size < 1 ||
            r.worker < 0 || r.worker >= cfg.workers)
          ++bad;
      }
      if (st.completed != done || st.deferred != refused) ++bad;
    }
  }
  // the error paths: null pointers, unsorted arrivals, a bad model
  swx_server_cfg cfg{};
  cfg.n = 4;
  swx_sim_model model{1e5, 10.0, 0.1};
  swx_sim_request two[2] = {{5.0, 10, 10}, {1.0, 10, 10}};
  swx_sim_result out2[2];
  if (swx_server_simulate(&cfg, &model, two, 2, out2, nullptr) != SWX_EINVAL) ++bad;
  if (swx_server_simulate(nullptr, &model, two, 0, out2, nullptr) != SWX_EINVAL) ++bad;
  swx_sim_model zero{0.0, 0.0, 0.0};
  if (swx_server_simulate(&cfg, &zero, two, 0, out2, nullptr) != SWX_EINVAL) ++bad;
  std::printf("simulator driver: %d failures\n", bad);
  return bad ? 1 : 0;
}
