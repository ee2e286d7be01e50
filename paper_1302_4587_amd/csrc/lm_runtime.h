// Host-side runtime objects of the local-max matching library: the device
// memory pool with its HBM budget, the per-context solver state and the
// problem descriptor handed to the phase loop.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <mutex>
#include <string>
#include <vector>

#include "lm.h"
#include "lm_internal.h"

namespace lm {

constexpr int kLogCap = 1 << 16;  // device phase records kept per solve
constexpr int kGraphPhases = 12;  // phases in the captured graph (LM_GRAPH)
constexpr int kWeightSumMaxGrid = 1024;  // workgroups of the matched-weight sum (LM_WEIGHT_SUM)

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
};

// Grow-only device buffers, all charged against one budget.
struct Pool {
  size_t budget = 0;
  size_t used = 0;
  lm_status reserve(DevBuf& b, size_t bytes);
  void release(DevBuf& b);
};

// Device working buffers of one solve (beyond inputs and outputs): from the
// context's pool (Solver::pool_work) or carved from one caller-independent
// region (carve_work).
struct Work {
  int* C = nullptr;
  unsigned char* state = nullptr;
  int4* rows[2] = {nullptr, nullptr};
  int* ecol[2] = {nullptr, nullptr};
  float* ew[2] = {nullptr, nullptr};
  Run* runs[2] = {nullptr, nullptr};
  long long* epre[2] = {nullptr, nullptr};
  int* rpre[2] = {nullptr, nullptr};
  Ctl* ctl = nullptr;
  Part* parts = nullptr;
  BlockStat* bstat = nullptr;
  int* mcount = nullptr;
  int* gbase = nullptr;
  unsigned long long* gseed = nullptr;
  long long* vtxoff = nullptr;
  Totals* totals = nullptr;
  TailCtl* tail = nullptr;
  unsigned* mbits = nullptr;  // matched bits, (N + 31) / 32 words
};

// Lays the working buffers of a solve of N vertices, nnz entries and G graphs
// out from base (256-byte aligned pieces) and returns the bytes used; with
// base == nullptr only the size is computed.
size_t carve_work(int64_t N, int64_t nnz, int64_t G, void* base, Work* w);

// Device-resident problem: the union of G graphs (G = 1 for lm_match).
struct Problem {
  int64_t N = 0, nnz = 0, G = 1;
  const long long* row_ptr = nullptr;
  const int* col = nullptr;
  const float* w = nullptr;
  const long long* vtx_off = nullptr;  // device, G+1
  int* mate = nullptr;
  int* gphase = nullptr;  // optional per-graph phase counts
};

struct ContractState;  // buffers of lm_contract (lm_contract.hip)

struct Solver {
  int dev = -1;
  int num_cus = 0;
  std::string dev_name;
  hipStream_t own = nullptr;
  Pool pool;
  lm_tuning tun{};
  int bpc_stream = 1;  // resident compaction workgroups per CU
  int bpc_first = 1;   // resident first-argmax workgroups per CU
  int bpc_late = 1;    // resident late-compaction workgroups per CU
  int bpc_stream_u = 1, bpc_first_u = 1, bpc_late_u = 1;  // the same for unweighted graphs
  int bpc_tail = 1;              // resident tail workgroups per CU
  int bpc_first_csr = 1;         // the first argmax of one weighted graph read from its CSR
  int bpc_first_unw = 1;         // one-wave ranges per CU of the first argmax of one unweighted graph
  unsigned long long clock_khz = 100000;  // constant wall clock of the device (barrier time-outs)
  hipEvent_t e_async = nullptr;  // end of the last LM_ASYNC solve
  bool async_pending = false;    // an LM_ASYNC solve may still be running on the context's buffers
  bool busy_server = false;
  int last_phases = 0;

  DevBuf C, state, rows[2], ecol[2], ew[2], runs[2], epre[2], rpre[2];
  DevBuf ctl, parts, bstat, mcount;
  DevBuf gbase, gseed, vtxoff, gphase, totals, tailc, mbits;
  DevBuf in_rp, in_col, in_w, out_mate;
  DevBuf wsum;  // kWeightSumMaxGrid partial sums, then the total
  ContractState* contract = nullptr;

  Totals* h_totals = nullptr;
  // mapped pinned host memory the plan kernel writes: one record per live set
  // (the host loop reads it after the plan's event) and the phase log
  PhaseMirror* h_mir = nullptr;
  PhaseMirror* d_mir = nullptr;
  LogRec* h_log = nullptr;
  LogRec* d_log = nullptr;
  unsigned gen = 0;  // solves so far: tells this solve's mirror records from older ones
  // per-graph tables as last uploaded (base, premixed seed, vertex offsets),
  // the device buffers they went to, and their pinned staging area
  std::vector<int32_t> t_gbase;
  std::vector<uint64_t> t_gseed;
  std::vector<int64_t> t_vtxoff;
  const void* t_dev[3] = {nullptr, nullptr, nullptr};
  void* t_pinned = nullptr;
  size_t t_pinned_cap = 0;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipEvent_t e_order = nullptr;   // orders a captured solve after the legacy default stream
  hipEvent_t e_tables = nullptr;  // after the last per-graph table upload
  std::vector<hipEvent_t> evpool;

  lm_status init_device(int device, size_t budget);
  void shutdown();
  lm_status prepare(int64_t N, int64_t nnz, int64_t G, bool want_gphase);
  Work pool_work() const;  // the pool's buffers, after prepare
  lm_status run(const Problem& p, const Work& wk, hipStream_t s, uint32_t flags, lm_stats* st);
  hipEvent_t event(size_t i);
};

// Matched weight (LM_WEIGHT_SUM): partial sums go to scratch[0, grid) and the
// total to scratch[kWeightSumMaxGrid]; scratch holds kWeightSumMaxGrid + 1 doubles.
int weight_sum_grid(long long N);
hipError_t launch_weight_sum(const long long* row_ptr, const int* col, const float* w, const int* mate, long long N,
                             double* scratch, hipStream_t s);

const char* status_text(lm_status st);
// Frees the contraction's buffers (at context shutdown).
void contract_release(Solver& S);
// LM_CHECK_GRAPH on device input: offsets and duplicate entries within rows
// (LM_EGRAPH), with the contraction's grouping kernels. Synchronises s.
lm_status check_row_duplicates(Solver& S, int64_t n, int64_t nnz, const long long* rp, const int* col,
                               hipStream_t s);
// Looks up this device's copy of the allocation-free solve's scratch array
// (lm_match_noalloc); called once per device with that device current.
lm_status noalloc_setup(int dev);
lm_status dev_status(hipError_t e);
size_t solve_footprint(int64_t N, int64_t nnz, int64_t G);

// Entry points shared with the server and the autotuner; the caller holds
// the context lock.
lm_status solve_locked(lm_ctx* c, int64_t N, int64_t nnz, int64_t G, const int64_t* h_vtx_off, const int64_t* row_ptr,
                       const int32_t* col, const float* w, const uint64_t* seeds, uint64_t seed0, int32_t* mate,
                       uint32_t flags, void* stream, lm_stats* st, int32_t* graph_phases);
Solver& solver_of(lm_ctx* c);
lm_status host_check(int64_t n, const int64_t* rp, const int32_t* col, const float* w, int64_t nnz);
std::mutex& mutex_of(lm_ctx* c);

}  // namespace lm
