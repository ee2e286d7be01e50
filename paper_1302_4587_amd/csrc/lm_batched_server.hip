// Batched serving loop: queued requests that fit the admission budget are
// solved together as one batch over their disjoint union.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <vector>

#include "lm.h"
#include "lm_runtime.h"
#include "lm_server_impl.h"

namespace lm {

struct BatchedState {
  int dummy = 0;
};

static void batch_loop(ServerCore* S) {
  std::vector<int64_t> vo, rp;
  std::vector<int32_t> col, mate;
  std::vector<float> w;
  std::vector<uint64_t> seeds;
  std::vector<int32_t> gph;
  for (;;) {
    std::vector<std::shared_ptr<Request>> take;
    {
      std::unique_lock<std::mutex> lk(S->mu);
      S->cv_work.wait(lk, [&] { return S->stopping || !S->queue.empty(); });
      if (S->queue.empty()) {
        if (S->stopping) return;
        continue;
      }
      size_t budget = 0;
      int64_t nsum = 0, esum = 0;
      while (!S->queue.empty() && (int)take.size() < S->opts.max_resident) {
        auto& r = S->queue.front();
        if (!take.empty() && (budget + r->footprint > S->opts.hbm_budget_bytes || nsum + r->n >= (1LL << 31) - 1 ||
                              esum + r->nnz >= (1LL << 31) - 65536))
          break;
        budget += r->footprint;
        nsum += r->n;
        esum += r->nnz;
        r->t_admit = std::chrono::steady_clock::now();
        S->running[r->ticket] = r;
        take.push_back(r);
        S->queue.pop_front();
      }
    }
    const int G = (int)take.size();
    vo.assign((size_t)G + 1, 0);
    seeds.resize((size_t)G);
    for (int g = 0; g < G; ++g) {
      vo[(size_t)g + 1] = vo[(size_t)g] + take[(size_t)g]->n;
      seeds[(size_t)g] = take[(size_t)g]->seed;
    }
    const int64_t N = vo[(size_t)G];
    int64_t E = 0;
    for (auto& r : take) E += r->nnz;
    rp.resize((size_t)N + 1);
    col.resize((size_t)std::max<int64_t>(E, 1));
    w.resize((size_t)std::max<int64_t>(E, 1));
    mate.assign((size_t)std::max<int64_t>(N, 1), -1);
    gph.assign((size_t)G, 0);
    int64_t eoff = 0;
    for (int g = 0; g < G; ++g) {
      const Request& r = *take[(size_t)g];
      for (int64_t v = 0; v < r.n; ++v) rp[(size_t)(vo[(size_t)g] + v)] = eoff + r.h_rp[v];
      if (r.nnz) {
        std::memcpy(col.data() + eoff, r.h_col, (size_t)r.nnz * 4);
        std::memcpy(w.data() + eoff, r.h_w, (size_t)r.nnz * 4);
      }
      eoff += r.nnz;
    }
    rp[(size_t)N] = E;
    lm_status st;
    {
      std::lock_guard<std::mutex> ck(mutex_of(S->ctx));
      lm_stats stats;
      std::memset(&stats, 0, sizeof(stats));
      st = solve_locked(S->ctx, N, E, G, vo.data(), rp.data(), col.data(), w.data(), seeds.data(), 1, mate.data(), 0u,
                        nullptr, &stats, gph.data());
    }
    for (int g = 0; g < G; ++g) {
      Request& r = *take[(size_t)g];
      if (st == LM_OK) {
        r.mate.assign(mate.begin() + vo[(size_t)g], mate.begin() + vo[(size_t)g + 1]);
        r.phases = gph[(size_t)g];
        int64_t m = 0;
        for (int32_t x : r.mate) m += (x >= 0);
        r.matched = m / 2;
      }
      S->finish(take[(size_t)g], st);
    }
  }
}

lm_status start_batched(ServerCore* s) {
  s->batched = new (std::nothrow) BatchedState();
  if (!s->batched) return LM_ENOMEM;
  s->worker = std::thread(batch_loop, s);
  return LM_OK;
}

void stop_batched(ServerCore* s) {
  delete s->batched;
  s->batched = nullptr;
}

}  // namespace lm
