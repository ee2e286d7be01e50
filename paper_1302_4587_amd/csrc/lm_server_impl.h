// Internal state of the request server (lm_server_* entry points).
#pragma once

#include <hip/hip_runtime.h>

#include <chrono>
#include <condition_variable>
#include <cstdint>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "lm.h"

namespace lm {

// Reusable pinned host blocks (pinning is far slower than copying): blocks
// are kept in power-of-two size classes up to a cached total.
struct PinnedPool {
  std::mutex mu;
  std::multimap<size_t, void*> free;  // capacity -> block
  size_t cached = 0;
  size_t limit = (size_t)8 << 30;
  void* get(size_t bytes, size_t* cap);
  void put(void* p, size_t cap);
  ~PinnedPool();
};

struct Request {
  uint64_t ticket = 0;
  int64_t n = 0, nnz = 0;
  uint64_t seed = 1;
  size_t footprint = 0;
  // pinned copy of the request graph: row_ptr, col, w in one block
  PinnedPool* pool = nullptr;
  void* block = nullptr;
  size_t block_cap = 0;
  int64_t* h_rp = nullptr;
  int32_t* h_col = nullptr;
  float* h_w = nullptr;
  std::vector<int32_t> mate;
  int32_t phases = 0;
  int64_t matched = 0;
  lm_status status = LM_OK;
  bool done = false;
  std::chrono::steady_clock::time_point t_submit, t_admit, t_solved, t_done;
  // batched mode: placement on the device
  int slot = -1;        // graph index in the resident tables
  int64_t vbase = 0;    // first vertex of the request in the server's vertex space
  int first_phase = 0;  // server phase in which the request was injected
  bool no_solo = false; // the single-graph path refused it (size): batch it
  // layout of the pinned block: row_ptr at 0, col at off_col, w at off_w
  size_t off_col = 0, off_w = 0, block_used = 0;
  // staging copy on the device (batched mode)
  int64_t stage_off = -1;
  hipEvent_t stage_ev = nullptr;
  ~Request();
};

struct BatchedState;  // lm_batched_server.hip

struct ServerCore {
  PinnedPool pinned;  // first member: outlives every request it lends to
  lm_ctx* ctx = nullptr;
  lm_server_opts opts{};
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<std::shared_ptr<Request>> queue;
  std::map<uint64_t, std::shared_ptr<Request>> running, finished, all;
  uint64_t next_ticket = 0;
  bool stopping = false;
  std::thread worker;
  lm_status worker_status = LM_OK;
  BatchedState* batched = nullptr;
  void finish(const std::shared_ptr<Request>& r, lm_status st);
};

// Device bytes one resident request may need at most.
inline size_t request_footprint(int64_t n, int64_t nnz) {
  return (size_t)n * (4 + 1 + 4 + 2 * 16) + (size_t)nnz * (2 * 8 + 8) + 4096;
}

// Resident-set capacity of the batched server for an HBM budget: vertices,
// entries and bytes of the device staging area for incoming requests; a
// request larger than any of them can never be admitted.
void server_caps(size_t budget, int64_t* n_cap, int64_t* e_cap, int64_t* stage_cap);

lm_status start_batched(ServerCore* s);
void stop_batched(ServerCore* s);

}  // namespace lm
