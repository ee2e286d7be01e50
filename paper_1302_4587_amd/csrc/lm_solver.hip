// Host driver and C ABI of the local-max matching library (see include/lm.h).
//
// A solve is: [optional input check] -> init (live set R_1 from the CSR) ->
// first argmax -> phases t = 1, 2, ...: mutual(t), compact(t). Phases are
// enqueued in chunks without host synchronisation; after each chunk the host
// reads one counter slot to see whether the live set is empty.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <atomic>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "lm.h"
#include "lm_internal.h"
#include "lm_key.h"
#include "lm_runtime.h"

using namespace lm;

namespace lm {

const char* status_text(lm_status st) {
  switch (st) {
    case LM_OK: return "ok";
    case LM_PENDING: return "pending";
    case LM_EINVAL: return "invalid argument";
    case LM_EGRAPH: return "graph violates the input contract";
    case LM_EWEIGHT: return "NaN or infinite weight";
    case LM_ENOMEM: return "device allocation failed";
    case LM_ETOOBIG: return "problem exceeds the HBM budget or the size limits";
    case LM_EAGAIN: return "server queue full";
    case LM_ENOTFOUND: return "unknown or retired ticket";
    case LM_EDEVICE: return "HIP device failure or no usable device";
    default: return "unknown status";
  }
}

lm_status dev_status(hipError_t e) {
  if (e == hipSuccess) return LM_OK;
  if (e == hipErrorOutOfMemory) return LM_ENOMEM;
  return LM_EDEVICE;
}

lm_status Pool::reserve(DevBuf& b, size_t bytes) {
  if (bytes == 0) bytes = 256;
  if (b.bytes >= bytes) return LM_OK;
  if (b.p) {
    (void)hipFree(b.p);
    used -= b.bytes;
    b.p = nullptr;
    b.bytes = 0;
  }
  if (used + bytes > budget) return LM_ETOOBIG;
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return e == hipErrorOutOfMemory ? LM_ENOMEM : LM_EDEVICE;
  }
  b.p = p;
  b.bytes = bytes;
  used += bytes;
  return LM_OK;
}

void Pool::release(DevBuf& b) {
  if (b.p) {
    (void)hipFree(b.p);
    used -= b.bytes;
  }
  b.p = nullptr;
  b.bytes = 0;
}

// Device bytes a solve needs beyond its inputs and outputs.
size_t solve_footprint(int64_t N, int64_t nnz, int64_t G) {
  size_t b = 0;
  b += (size_t)N * 4 + 256;                                // C
  b += (size_t)N + 256;                                    // state
  b += (size_t)((N + 31) / 32 + 16) * 4 + 256;             // matched bits
  b += 2 * (((size_t)N + 2 * kMaxBlocks + 16) * 16 + 256); // piece buffers
  b += 2 * 2 * ((size_t)nnz * 4 + 256);                    // entry ping-pong (col, w)
  b += 2 * ((size_t)kMaxBlocks * (sizeof(Run) + 8 + 4) + 1024);
  b += (size_t)kMaxFirstRanges * 2 * sizeof(Part) + (size_t)kMaxBlocks * (sizeof(BlockStat) + 4) + 1024;
  b += (size_t)G * 16 + (size_t)(G + 1) * 8 + 1024;
  b += 2 * sizeof(Ctl) + sizeof(Totals) + 1024;
  return b;
}

// ------------------------------------------------------------------ solve

lm_status Solver::prepare(int64_t N, int64_t nnz, int64_t G, bool want_gphase) {
  lm_status st;
#define RES(buf, bytes)                 \
  do {                                  \
    st = pool.reserve(buf, (bytes));    \
    if (st != LM_OK) return st;         \
  } while (0)
  RES(C, (size_t)N * 4);
  RES(state, (size_t)N);
  for (int i = 0; i < 2; ++i) {
    RES(rows[i], ((size_t)N + 2 * kMaxBlocks + 16) * 16);
    RES(ecol[i], (size_t)nnz * 4);
    RES(ew[i], (size_t)nnz * 4);
    RES(runs[i], (size_t)kMaxBlocks * sizeof(Run));
    RES(epre[i], (size_t)(kMaxBlocks + 1) * 8);
    RES(rpre[i], (size_t)(kMaxBlocks + 1) * 4);
  }
  RES(ctl, 2 * sizeof(Ctl));
  RES(parts, (size_t)kMaxFirstRanges * 2 * sizeof(Part));
  RES(bstat, (size_t)kMaxBlocks * sizeof(BlockStat));
  RES(mcount, (size_t)kMaxBlocks * 4);
  const size_t tb0 = gbase.bytes + gseed.bytes + vtxoff.bytes;
  RES(gbase, (size_t)G * 4);
  RES(gseed, (size_t)G * 8);
  RES(vtxoff, (size_t)(G + 1) * 8);
  if (gbase.bytes + gseed.bytes + vtxoff.bytes != tb0) t_dev[0] = t_dev[1] = t_dev[2] = nullptr;  // reallocated
  if (want_gphase) RES(gphase, (size_t)G * 4);
  RES(totals, sizeof(Totals));
  RES(tailc, sizeof(TailCtl));
  RES(mbits, (size_t)((N + 31) / 32 + 16) * 4);
#undef RES
  return LM_OK;
}

Work Solver::pool_work() const {
  Work w;
  w.C = (int*)C.p;
  w.state = (unsigned char*)state.p;
  for (int i = 0; i < 2; ++i) {
    w.rows[i] = (int4*)rows[i].p;
    w.ecol[i] = (int*)ecol[i].p;
    w.ew[i] = (float*)ew[i].p;
    w.runs[i] = (Run*)runs[i].p;
    w.epre[i] = (long long*)epre[i].p;
    w.rpre[i] = (int*)rpre[i].p;
  }
  w.ctl = (Ctl*)ctl.p;
  w.parts = (Part*)parts.p;
  w.bstat = (BlockStat*)bstat.p;
  w.mcount = (int*)mcount.p;
  w.gbase = (int*)gbase.p;
  w.gseed = (unsigned long long*)gseed.p;
  w.vtxoff = (long long*)vtxoff.p;
  w.totals = (Totals*)totals.p;
  w.tail = (TailCtl*)tailc.p;
  w.mbits = (unsigned*)mbits.p;
  return w;
}

size_t carve_work(int64_t N, int64_t nnz, int64_t G, void* base, Work* w) {
  size_t off = 0;
  auto take = [&](size_t bytes) -> void* {
    void* p = base ? (void*)((char*)base + off) : nullptr;
    off += (std::max<size_t>(bytes, 1) + 255) & ~(size_t)255;
    return p;
  };
  Work x;
  x.C = (int*)take((size_t)N * 4);
  x.state = (unsigned char*)take((size_t)N);
  for (int i = 0; i < 2; ++i) {
    x.rows[i] = (int4*)take(((size_t)N + 2 * kMaxBlocks + 16) * 16);
    x.ecol[i] = (int*)take((size_t)nnz * 4);
    x.ew[i] = (float*)take((size_t)nnz * 4);
    x.runs[i] = (Run*)take((size_t)kMaxBlocks * sizeof(Run));
    x.epre[i] = (long long*)take((size_t)(kMaxBlocks + 1) * 8);
    x.rpre[i] = (int*)take((size_t)(kMaxBlocks + 1) * 4);
  }
  x.ctl = (Ctl*)take(2 * sizeof(Ctl));
  x.parts = (Part*)take((size_t)kMaxFirstRanges * 2 * sizeof(Part));
  x.bstat = (BlockStat*)take((size_t)kMaxBlocks * sizeof(BlockStat));
  x.mcount = (int*)take((size_t)kMaxBlocks * 4);
  x.gbase = (int*)take((size_t)G * 4);
  x.gseed = (unsigned long long*)take((size_t)G * 8);
  x.vtxoff = (long long*)take((size_t)(G + 1) * 8);
  x.totals = (Totals*)take(sizeof(Totals));
  x.tail = (TailCtl*)take(sizeof(TailCtl));
  x.mbits = (unsigned*)take((size_t)((N + 31) / 32 + 16) * 4);
  if (w) *w = x;
  return off;
}

lm_status Solver::init_device(int device, size_t budget) {
  dev = device;
  pool.budget = budget;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || count <= 0 || device < 0 || device >= count) {
    (void)hipGetLastError();
    return LM_EDEVICE;
  }
  if (hipSetDevice(device) != hipSuccess) return LM_EDEVICE;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess) return LM_EDEVICE;
  num_cus = prop.multiProcessorCount;
  dev_name = prop.gcnArchName;
  if (hipStreamCreateWithFlags(&own, hipStreamNonBlocking) != hipSuccess) return LM_EDEVICE;
  if (hipHostMalloc((void**)&h_totals, sizeof(Totals)) != hipSuccess) return LM_EDEVICE;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return LM_EDEVICE;
  if (hipEventCreateWithFlags(&e_order, hipEventDisableTiming) != hipSuccess) return LM_EDEVICE;
  if (hipEventCreateWithFlags(&e_tables, hipEventDisableTiming) != hipSuccess) return LM_EDEVICE;
  if (hipEventCreateWithFlags(&e_async, hipEventDisableTiming) != hipSuccess) return LM_EDEVICE;
  int khz = 0;
  if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, device) == hipSuccess && khz > 0)
    clock_khz = (unsigned long long)khz;
  const unsigned mapped = hipHostMallocMapped | hipHostMallocCoherent;
  // one slot per live set of the ring, plus the tail kernel's final record
  if (hipHostMalloc((void**)&h_mir, sizeof(PhaseMirror) * (kMirrorSlots + 1), mapped) != hipSuccess) return LM_EDEVICE;
  if (hipHostMalloc((void**)&h_log, sizeof(LogRec) * (size_t)kLogCap, mapped) != hipSuccess) return LM_EDEVICE;
  std::memset(h_mir, 0, sizeof(PhaseMirror) * (kMirrorSlots + 1));
  if (hipHostGetDevicePointer((void**)&d_mir, h_mir, 0) != hipSuccess) return LM_EDEVICE;
  if (hipHostGetDevicePointer((void**)&d_log, h_log, 0) != hipSuccess) return LM_EDEVICE;
  if (noalloc_setup(device) != LM_OK) return LM_EDEVICE;
  bpc_stream = max_blocks_per_cu_stream(StreamKind::kCompact);
  bpc_first = max_blocks_per_cu_stream(StreamKind::kFirst);
  bpc_late = max_blocks_per_cu_stream(StreamKind::kLateCompact);
  bpc_stream_u = max_blocks_per_cu_stream(StreamKind::kCompact, true);
  bpc_first_u = max_blocks_per_cu_stream(StreamKind::kFirst, true);
  bpc_late_u = max_blocks_per_cu_stream(StreamKind::kLateCompact, true);
  bpc_tail = tail_blocks_per_cu();
  bpc_first_csr = first_csr_blocks_per_cu(false);
  bpc_first_unw = first_unw_ranges_per_cu();
  tun.block_entries = kCap;  // one batch: small phases still spread over every CU
  tun.grid_per_cu = 16;  // at most: the resident count of each kernel caps it
  tun.phases_per_sync = 1;  // phases queued past the live set the host checks
  tun.tail_entries = 1 << 20;  // live sets handed to the tail kernel (measured on RGG and R-MAT)
  return LM_OK;
}

void Solver::shutdown() {
  if (dev >= 0) (void)hipSetDevice(dev);
  if (own) (void)hipStreamSynchronize(own);
  if (e_async && async_pending) (void)hipEventSynchronize(e_async);
  async_pending = false;
  DevBuf* all[] = {&C,       &state,   &rows[0], &rows[1], &ecol[0], &ecol[1], &ew[0],   &ew[1],
                   &runs[0], &runs[1], &epre[0], &epre[1], &rpre[0], &rpre[1], &ctl,     &parts,
                   &bstat,   &mcount,  &gbase,   &gseed,   &vtxoff,  &gphase,  &totals,  &in_rp,
                   &in_col,  &in_w,    &out_mate, &wsum,   &tailc,   &mbits};
  for (DevBuf* b : all) pool.release(*b);
  contract_release(*this);
  for (hipEvent_t e : evpool) (void)hipEventDestroy(e);
  evpool.clear();
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (e_order) (void)hipEventDestroy(e_order);
  e_order = nullptr;
  if (e_tables) (void)hipEventDestroy(e_tables);
  e_tables = nullptr;
  if (e_async) (void)hipEventDestroy(e_async);
  e_async = nullptr;
  if (h_totals) (void)hipHostFree(h_totals);
  if (h_mir) (void)hipHostFree(h_mir);
  if (t_pinned) (void)hipHostFree(t_pinned);
  t_pinned = nullptr;
  t_pinned_cap = 0;
  if (h_log) (void)hipHostFree(h_log);
  h_mir = d_mir = nullptr;
  h_log = d_log = nullptr;

  if (own) (void)hipStreamDestroy(own);
  own = nullptr;
  h_totals = nullptr;
  e0 = e1 = nullptr;
}

hipEvent_t Solver::event(size_t i) {
  while (evpool.size() <= i) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    evpool.push_back(e);
  }
  return evpool[i];
}

// Runs the phase loop over a problem whose inputs are already on the device.
lm_status Solver::run(const Problem& p, const Work& wk, hipStream_t s, uint32_t flags, lm_stats* st) {
  const bool prof = (flags & LM_PROFILE) != 0;
  if (++gen == 0) gen = 1;  // 0 marks a never-written mirror slot
  const bool unweighted = p.w == nullptr;  // no weight array: every edge weighs 1
  // R_1 of a single graph is read straight from the input CSR: no 16-byte
  // piece records (k_init writes none, the first argmax, mutual check and
  // compaction take rows from row_ptr, the mutual check rewrites nothing). A
  // batch builds piece records, which carry each row's graph.
  const bool csr1 = p.G == 1;
  std::vector<std::pair<int, size_t>> marks;  // (kind, event index of start)
  size_t evn = 0;
  const uint32_t kmask = (st && st->profile_kinds) ? st->profile_kinds : ((1u << LM_K_KINDS) - 1);
  // Timing events {start, stop} for one launch of a profiled kind, stamped by
  // the dispatch itself; nullptr when the kind is not timed.
  hipEvent_t tev[2] = {nullptr, nullptr};
  bool tev_fail = false;
  auto timing = [&](int kind) -> hipEvent_t* {
    if (!prof || !((kmask >> kind) & 1u)) return nullptr;
    tev[0] = event(evn);
    tev[1] = event(evn + 1);
    if (!tev[0] || !tev[1]) {
      tev_fail = true;
      return nullptr;
    }
    marks.push_back({kind, evn});
    evn += 2;
    return tev;
  };
#define HIPCHK(x)                          \
  do {                                     \
    hipError_t _e = (x);                   \
    if (_e != hipSuccess) {                \
      (void)hipGetLastError();             \
      return dev_status(_e);               \
    }                                      \
  } while (0)

  // resident workgroups per CU of the kernels this solve uses
  const int bs = unweighted ? bpc_stream_u : bpc_stream;
  // (the weighted first argmax reads R_1 from the CSR for a batch too)
  const int bf = unweighted ? (csr1 ? bpc_first_unw : bpc_first_u) : bpc_first_csr;
  const int bl = unweighted ? bpc_late_u : bpc_late;
  const int pcap = std::max(1, std::min(kMaxBlocks, num_cus * std::max(1, std::min(tun.grid_per_cu, bs))));
  // R_1 feeds the first argmax and the first compaction, each split to its
  // own resident count; later live sets feed compactions with the wider piece
  // window, which fit fewer workgroups per CU
  const int pcap_first = std::max(1, std::min(kMaxFirstRanges, num_cus * std::max(1, bf)));
  const int pcap_late = std::max(1, std::min(kMaxBlocks, num_cus * std::max(1, std::min(tun.grid_per_cu, bl))));
  const int pmcap = std::max(1, std::min(kMaxBlocks, num_cus * 8));
  Ctl* dctl = wk.ctl;
  Totals* dtot = wk.totals;

  Common c;
  c.totals = dtot;
  c.n = (int)p.N;
  c.C = wk.C;
  c.state = wk.state;
  c.mate = p.mate;
  c.gbase = wk.gbase;
  c.gseed = wk.gseed;
  c.gphase = p.gphase;
  c.graphs = (int)p.G;
  c.guard = 0;
  c.renew = (flags & LM_RENEW_KEYS) ? 1 : 0;
  // one large graph: the compactions may read the matched state from bits,
  // if k_init's sample finds its neighbour ids scattered
  c.mbits = (p.G == 1 && p.N >= kBitsMinN) ? wk.mbits : nullptr;
  // A device-controlled solve (LM_GRAPH, LM_ASYNC) enqueues a fixed number of
  // guarded phases and then the tail kernel; the plan that produces a live set
  // of at most tail_at entries hands it to the tail, and the guarded phases
  // after it do nothing. A host-polled solve hands over from its loop.
  // (a stream-ordered solve is not captured: its graph would have to outlive the call)
  const bool use_graph = (flags & LM_GRAPH) != 0 && !prof && !(flags & LM_ASYNC);
  const bool dev_ctl = use_graph || (flags & LM_ASYNC) != 0;
  const long long tail_at = tun.tail_entries > 0 ? tun.tail_entries : (1ll << 20);

  auto live = [&](int t) {  // live set R_t
    const int i = (t - 1) & 1;
    LiveSet L;
    L.ctl = dctl + i;
    L.runs = wk.runs[i];
    L.epre = wk.epre[i];
    L.rpre = wk.rpre[i];
    L.rows = wk.rows[i];
    L.col = t == 1 ? p.col : wk.ecol[t & 1];
    L.w = t == 1 ? p.w : wk.ew[t & 1];
    L.csr_rp = (t == 1 && csr1) ? p.row_ptr : nullptr;
    return L;
  };
  auto plan_base = [&]() {
    PlanArgs a;
    std::memset(&a, 0, sizeof(a));
    a.c = c;
    a.pcap = pcap;
    a.pmcap = pmcap;
    a.min_per_block = std::max(kCap, tun.block_entries);
    a.pieces_per_block = kBlock * late_ppl(unweighted);
    a.nruns_new = -1;
    a.log = d_log;
    a.log_cap = kLogCap;
    a.mirror = d_mir;
    a.gen = gen;
    a.mcount = wk.mcount;
    a.tail_at = dev_ctl ? tail_at : 0;
    return a;
  };

  int64_t est_L = p.nnz, est_V = p.N;
  // Every launch returns its status; HIPCHK is not used between BeginCapture
  // and EndCapture so that a failed launch never leaves the stream capturing.
#define ENQ(x)                        \
  do {                                \
    hipError_t _e = (x);              \
    if (_e != hipSuccess) return _e;  \
  } while (0)
  // live set R_1 from the input and the first argmax over it
  auto enqueue_prologue = [&]() -> hipError_t {
    ENQ(launch_zero(dctl, 2, dtot, s, wk.tail));
    if (p.gphase) ENQ(launch_fill_i32(p.gphase, p.G, 0, s));
    if (flags & LM_CHECK_GRAPH) {
      CheckArgs ca{dtot, p.nnz, p.row_ptr, p.col, p.w, (int)p.N, (int)p.G, p.vtx_off};
      const int grid = (int)std::min<int64_t>(pmcap, (p.N + kBlock - 1) / kBlock + 1);
      ENQ(launch_check(ca, grid, s));
    }
    const int pi = (int)std::max<int64_t>(1, std::min<int64_t>(pcap, (p.N + 16383) / 16384));
    InitArgs ia;
    ia.c = c;
    ia.row_ptr = p.row_ptr;
    ia.nnz = p.nnz;
    ia.ebase = 0;
    ia.vfirst = 0;
    ia.vcount = p.N;
    ia.graphs = (int)p.G;
    ia.vtx_off = p.vtx_off;
    ia.slot_of = nullptr;
    ia.nblocks = pi;
    ia.rows_base = 0;
    ia.runs_base = 0;
    ia.runs_out = wk.runs[0];
    ia.rows_out = wk.rows[0];
    ia.csr = csr1 ? 1 : 0;
    ia.col = c.mbits ? p.col : nullptr;
    ia.bstat = wk.bstat;
    ENQ(launch_init(ia, s, timing(LM_K_INIT)));
    PlanArgs pa = plan_base();  // R_1: split for the first compaction and, apart, the first argmax
    pa.mode = kPlanPrefix;
    pa.pcap = pcap;
    pa.pcap_first = pcap_first;
    pa.pieces_per_block = kBlock;
    pa.ctl_prev = nullptr;
    pa.runs_new = wk.runs[0];
    pa.nruns_new = pi;
    pa.epre_new = wk.epre[0];
    pa.rpre_new = wk.rpre[0];
    pa.ctl_new = dctl + 0;
    pa.heads_of_runs = csr1 ? wk.bstat : nullptr;
    ENQ(launch_plan(pa, s, timing(LM_K_PLAN)));
    StreamArgs sa;
    std::memset(&sa, 0, sizeof(sa));
    sa.c = c;
    sa.in = live(1);
    // a weighted batch's first argmax also reads R_1 from the input CSR (the
    // union of the graphs; the kernel looks up each row's graph), while the
    // other kernels read its piece records
    if (!csr1 && !unweighted) sa.in.csr_rp = p.row_ptr;
    sa.parts = wk.parts;
    sa.bstat = wk.bstat;
    sa.cand_phase = 1;
    const int gx =
        (int)std::max<int64_t>(1, std::min<int64_t>(pcap_first, p.nnz / std::max(kCap, tun.block_entries) + 1));
    ENQ(launch_first_argmax(sa, gx, s, unweighted, timing(LM_K_ARGMAX), p.nnz));
    PlanArgs pf = plan_base();
    pf.mode = kPlanFix;
    pf.first = 1;
    pf.ctl_prev = dctl + 0;
    pf.parts = wk.parts;
    ENQ(launch_plan(pf, s, timing(LM_K_PLAN)));
    return hipSuccess;
  };
  // phase t: mutual check, compaction fused with the next argmax, plan
  int t = 1;
  auto enqueue_phase = [&]() -> hipError_t {
    const LiveSet in = live(t);
    MutualArgs ma;
    ma.c = c;
    ma.in = in;
    ma.mcount = wk.mcount;
    ma.census = 0;
    const int gm = (int)std::max<int64_t>(1, std::min<int64_t>(pmcap, est_V / kMutualRound + 1));
    ENQ(launch_mutual(ma, gm, s, timing(LM_K_MUTUAL)));
    const int lo = t & 1;
    StreamArgs sa;
    sa.c = c;
    sa.in = in;
    sa.runs_out = wk.runs[lo];
    sa.rows_out = wk.rows[lo];
    sa.dst_col = wk.ecol[(t + 1) & 1];
    sa.dst_w = wk.ew[(t + 1) & 1];
    sa.parts = wk.parts;
    sa.bstat = wk.bstat;
    sa.cand_phase = t + 1;  // the compaction of phase t computes the candidates of phase t + 1
    const bool late = t > 1;
    const int gx = (int)std::max<int64_t>(
        1, std::min<int64_t>(late ? pcap_late : pcap,
                             std::max<int64_t>(est_L / std::max(kCap, tun.block_entries),
                                               est_V / (kBlock * (late ? late_ppl(unweighted) : 1))) + 1));
    ENQ(launch_compact(sa, gx, s, late, unweighted, timing(LM_K_COMPACT)));
    PlanArgs pa = plan_base();  // sizes the next compaction, a late one
    pa.pcap = pcap_late;
    pa.mode = kPlanFix | kPlanPrefix | kPlanLog | kPlanTick;
    pa.ctl_prev = in.ctl;
    pa.parts = wk.parts;
    pa.bstat = wk.bstat;
    pa.rows_out = wk.rows[lo];
    pa.runs_new = wk.runs[lo];
    pa.epre_new = wk.epre[lo];
    pa.rpre_new = wk.rpre[lo];
    pa.ctl_new = dctl + lo;
    ENQ(launch_plan(pa, s, timing(LM_K_PLAN)));
    ++t;
    return hipSuccess;
  };
  // every remaining phase, from the live set the device phase counter names
  // at most half the resident capacity, so that two solves' tails on other
  // streams are resident together
  const int tail_cap = std::max(1, std::min(kTailMaxBlocks, num_cus * std::max(1, bpc_tail) / 2));
  auto enqueue_tail = [&](long long L_hint) -> hipError_t {
    TailArgs ta;
    std::memset(&ta, 0, sizeof(ta));
    ta.c = c;
    ta.c.guard = 0;
    ta.tc = wk.tail;
    for (int i = 0; i < 2; ++i) {
      ta.ctl[i] = dctl + i;
      ta.runs[i] = wk.runs[i];
      ta.epre[i] = wk.epre[i];
      ta.rpre[i] = wk.rpre[i];
      ta.rows[i] = wk.rows[i];
      ta.ecol[i] = wk.ecol[i];
      ta.ew[i] = unweighted ? nullptr : wk.ew[i];
    }
    ta.row_cap = (int)(p.N + 2 * kMaxBlocks + 16);
    ta.csr_rp = csr1 ? p.row_ptr : nullptr;
    ta.in_col = p.col;
    ta.in_w = p.w;
    ta.log = d_log;
    ta.log_cap = kLogCap;
    ta.final_rec = d_mir + kMirrorSlots;
    ta.gen = gen;
    ta.spin_ticks = clock_khz * 2000ull;  // 2 s
    // workgroups (1024 lanes each): about one per 16384 live entries
    const long long want = L_hint < 0 ? tail_cap : (L_hint + 16383) / 16384;
    const int grid = (int)std::max<long long>(1, std::min<long long>(tail_cap, want));
    ENQ(launch_tail(ta, grid, s, timing(LM_K_TAIL)));
    return hipSuccess;
  };
#undef ENQ

  HIPCHK(hipEventRecord(e0, s));
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  struct GraphGuard {
    hipGraph_t& g;
    hipGraphExec_t& x;
    ~GraphGuard() {
      if (x) (void)hipGraphExecDestroy(x);
      if (g) (void)hipGraphDestroy(g);
    }
  } guard{graph, gexec};
  constexpr int kRing = kMirrorSlots - 1;
  bool tail_queued = false;
  if (dev_ctl) {
    // Guarded phases until the live set is expected below tail_at (it shrinks
    // to about a third or less per phase), then the tail kernel, which runs
    // whatever is left. With LM_GRAPH the whole solve is one captured graph.
    int K = 0;
    for (double x = (double)p.nnz; x > (double)tail_at && K < 24; x /= 3.0) ++K;
    if (K > 0) ++K;  // one phase of margin: guarded phases after the hand-over do nothing
    auto enqueue_all = [&]() -> hipError_t {
      hipError_t e = enqueue_prologue();
      c.guard = 1;
      for (int j = 0; j < K && e == hipSuccess; ++j) e = enqueue_phase();
      c.guard = 0;
      if (e == hipSuccess) e = enqueue_tail(-1);
      return e;
    };
    if (use_graph) {
      HIPCHK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
      const hipError_t ce = enqueue_all();
      const hipError_t ee = hipStreamEndCapture(s, &graph);
      HIPCHK(ce);
      HIPCHK(ee);
      HIPCHK(hipGraphInstantiate(&gexec, graph, nullptr, nullptr, 0));
      HIPCHK(hipGraphLaunch(gexec, s));
    } else {
      HIPCHK(enqueue_all());
    }
    tail_queued = true;
    if (flags & LM_ASYNC) {
      HIPCHK(hipEventRecord(e_async, s));
      async_pending = true;
      return LM_OK;
    }
  } else {
    HIPCHK(enqueue_prologue());
    if (tun.tail_entries > 0 && p.nnz <= tun.tail_entries) {  // R_1 is already small
      HIPCHK(enqueue_tail(p.nnz));
      tail_queued = true;
    }
  }
  // rc: the live set R_rc the host checks next; the plan that produced it
  // leaves its record in h_mir[rc & kRing].
  int rc = 1;
  // Phase loop: phases rc .. rc + ahead - 1 stay queued while the host polls
  // the record of R_rc, so the device never idles on the host; the phases
  // queued past the empty live set are no-ops. No event is recorded between
  // phases: each one would put a bubble of a few microseconds on the stream.
  // Once R_rc is small the phases already queued run and the tail kernel
  // takes the rest.
  const int ahead = std::max(1, std::min(tun.phases_per_sync, kMirrorSlots / 2));
  const long long host_tail = tun.tail_entries > 0 ? 4ll * tun.tail_entries : -1;
  // Reads a record tagged for this solve and live set `idx` (idx < 0: the tail
  // kernel's final record, any live set). The tag is read before and after the
  // copy, so a record being rewritten is never taken.
  auto take_record = [&](const volatile PhaseMirror* slot, int idx, PhaseMirror& m) -> bool {
    const unsigned long long t0 = slot->tag;
    if ((unsigned)(t0 >> 32) != gen || (idx >= 0 && t0 != mirror_tag(gen, idx))) return false;
    std::atomic_thread_fence(std::memory_order_acquire);
    std::memcpy(&m, (const void*)slot, sizeof(m));
    std::atomic_thread_fence(std::memory_order_acquire);
    return slot->tag == t0 && m.tag == t0;
  };
  // 1: record of R_idx read; 0: the stream drained without it (an error flag
  // stopped the plan); -1: the stream failed
  auto wait_record = [&](int idx, PhaseMirror& m) -> int {
    const volatile PhaseMirror* slot = &h_mir[idx & kRing];
    for (unsigned spin = 1;; ++spin) {
      if (take_record(slot, idx, m)) return 1;
      if ((spin & 255u) == 0u) {
        const hipError_t q = hipStreamQuery(s);
        if (q == hipSuccess) return take_record(slot, idx, m) ? 1 : 0;
        if (q != hipErrorNotReady) return -1;
      }
    }
  };
  int64_t last_live = -1;
  bool stalled = false, no_record = false;
  PhaseMirror fin{};
  while (!tail_queued) {
    while (t < rc + ahead) HIPCHK(enqueue_phase());  // phase t - 1 queued: its plan produces R_t
    PhaseMirror m;
    const int got = wait_record(rc, m);
    if (got < 0) HIPCHK(hipStreamSynchronize(s));
    if (got <= 0) {
      no_record = true;
      break;
    }
    fin = m;
    if (m.err || m.L == 0) break;
    // every phase of a well-formed graph matches its globally heaviest live
    // edge; a phase without progress means asymmetric input
    if (m.L == last_live) {
      stalled = true;
      break;
    }
    last_live = m.L;
    est_L = m.L;
    est_V = m.pieces;
    if (m.L <= host_tail) {
      HIPCHK(enqueue_tail(m.L));
      tail_queued = true;
      break;
    }
    ++rc;
  }
  HIPCHK(hipEventRecord(e1, s));
  HIPCHK(hipEventSynchronize(e1));
  int tail_from = 0;  // the live set the tail kernel started from (0: no tail)
  if (tail_queued && !no_record && !stalled) {
    PhaseMirror m;
    if (take_record(&h_mir[kMirrorSlots], -1, m)) {
      fin = m;
      tail_from = m.pad;
    } else {
      no_record = true;  // the tail stopped on an error flag before its record
    }
  }
  Totals tot{};
  if (no_record) {
    HIPCHK(hipMemcpy(h_totals, dtot, sizeof(Totals), hipMemcpyDeviceToHost));
    tot = *h_totals;
  } else {
    tot.err = fin.err;
    tot.matched = fin.matched;
    tot.last_nonempty = fin.last_nonempty;
  }
  const unsigned err = tot.err;
  if (err) {
    if (err & kErrWeight) return LM_EWEIGHT;
    if (err & (kErrRowPtr | kErrColRange | kErrSelfLoop | kErrStall | kErrAsym)) return LM_EGRAPH;
    if (err & kErrDegree) return LM_ETOOBIG;
    return LM_EDEVICE;
  }
  if (stalled || no_record) return stalled ? LM_EGRAPH : LM_EDEVICE;
  if (tev_fail) return LM_ENOMEM;  // a timing event could not be created
  const int phases = tot.last_nonempty;
  last_phases = phases;
  if (st) {
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, e0, e1));
    st->phases = phases;
    st->matched_edges = (int64_t)(tot.matched / 2);
    st->device_ms = ms;
    for (int k = 0; k < LM_K_KINDS; ++k) {
      st->k_launches[k] = 0;
      st->k_ms[k] = 0.0;
      st->k_bytes[k] = 0.0;
    }
    for (auto& m : marks) {
      float km = 0.f;
      HIPCHK(hipEventElapsedTime(&km, event(m.second), event(m.second + 1)));
      st->k_launches[m.first] += 1;
      st->k_ms[m.first] += km;
    }
    // the records are read straight from the mapped log (complete once e1 has
    // passed); the record after the last one counts as empty
    const int nrec = std::min(phases, kLogCap);
    auto recs = [&](int i) -> LogRec { return i < nrec ? h_log[i] : LogRec{0, 0, 0, 0}; };
    st->log_len = 0;
    if (st->log && st->log_cap > 0) {
      const int nl = std::min(nrec, st->log_cap);
      if (nl > 0) std::memcpy(st->log, h_log, sizeof(LogRec) * (size_t)nl);
      st->log_len = nl;
    }
    // algorithmic bytes per kernel kind (what each must move, from the log).
    // A live row of R_1 costs a 16-byte piece record, written once and read by
    // the first argmax, mutual check (which rewrites it) and compaction; read
    // from the CSR it costs 8 bytes of row_ptr per vertex in the argmax and
    // the compaction (which adds state[v]), C[v] of every vertex in the mutual
    // check, and k_init clears C instead of writing records.
    const double N = (double)p.N;
    const double V1 = nrec > 0 ? (double)recs(0).live_rows : 0.0;
    const double L1 = nrec > 0 ? (double)recs(0).live_entries : 0.0;
    st->k_bytes[LM_K_INIT] = 8.0 * (N + 1.0) + (csr1 ? 9.0 * N : 5.0 * N + 16.0 * V1);
    const double eb = unweighted ? 4.0 : 8.0;  // bytes of one entry: col (+ w)
    st->k_bytes[LM_K_ARGMAX] = (csr1 ? 8.0 * (N + 1.0) : 16.0 * V1) + eb * L1 + 4.0 * V1;
    // Phases from tail_from on ran in the tail kernel: per phase a 16-byte row
    // record read twice (mutual check, compaction), C[v] and the C[C[v]]
    // gather, 5 bytes per matched vertex, the live entries of unmatched rows
    // with their neighbour's state, the survivors, and a 16-byte record plus
    // C[v] per next live row; starting from R_c with c >= 2 it first copies
    // the L_c entries to their virtual positions (a read and a write each) and
    // reads R_c's piece records.
    for (int i = 0; i < nrec; ++i) {
      const double L = (double)recs(i).live_entries, V = (double)recs(i).live_rows;
      const double mv = 2.0 * (double)recs(i).matched_edges, md = (double)recs(i).matched_entries;
      const double L2 = (double)recs(i + 1).live_entries, V2 = (double)recs(i + 1).live_rows;
      const bool from_csr = csr1 && i == 0;
      if (tail_from > 0 && i + 1 >= tail_from) {
        double b = 24.0 * V + 5.0 * mv + 16.0 * V + (eb + 1.0) * (L - md) + eb * L2 + 20.0 * V2;
        if (i + 1 == tail_from) b += (tail_from >= 2 ? 2.0 * eb * L : 0.0) + (from_csr ? 16.0 * N : 32.0 * V);
        st->k_bytes[LM_K_TAIL] += b;
        continue;
      }
      st->k_bytes[LM_K_MUTUAL] += from_csr ? 4.0 * N + 4.0 * V + 5.0 * mv : 24.0 * V + 9.0 * mv;
      st->k_bytes[LM_K_COMPACT] += (from_csr ? 9.0 * N : 16.0 * V) + (eb + 1.0) * (L - md) + eb * L2 + 20.0 * V2;
    }
    st->bytes_alg = 0.0;
    for (int k = 0; k < LM_K_KINDS; ++k) st->bytes_alg += st->k_bytes[k];
  }
#undef HIPCHK
  return LM_OK;
}

}  // namespace lm

// ==================================================================== C ABI

struct lm_ctx {
  Solver s;
  std::mutex mu;
};

static bool csr_shape_ok(const lm_csr* g) {
  if (!g) return false;
  if (g->n < 0 || g->nnz < 0) return false;
  if (g->n >= (int64_t)1 << 31) return false;
  if (!g->row_ptr) return false;
  if (g->nnz > 0 && !g->col) return false;  // w may be null: unweighted
  return true;
}

// Full host-side contract check of a graph (LM_CHECK_GRAPH on host input,
// and every request at server submit).
lm_status lm::host_check(int64_t n, const int64_t* rp, const int32_t* col, const float* w, int64_t nnz) {
  if (rp[0] != 0 || rp[n] != nnz) return LM_EINVAL;
  struct E {
    int32_t lo, hi;
    float w;
  };
  std::vector<E> es;
  es.reserve((size_t)nnz);
  for (int64_t v = 0; v < n; ++v) {
    if (rp[v + 1] < rp[v]) return LM_EINVAL;
    for (int64_t k = rp[v]; k < rp[v + 1]; ++k) {
      const int32_t u = col[k];
      if (u < 0 || u >= n || u == v) return LM_EGRAPH;
      const float x = w ? w[k] : 1.0f;  // no weight array: unweighted
      if (!(x == x) || x == 1.0f / 0.0f || x == -1.0f / 0.0f) return LM_EWEIGHT;
      es.push_back(E{(int32_t)std::min<int64_t>(v, u), (int32_t)std::max<int64_t>(v, u), x});
    }
  }
  std::sort(es.begin(), es.end(), [](const E& a, const E& b) {
    if (a.lo != b.lo) return a.lo < b.lo;
    if (a.hi != b.hi) return a.hi < b.hi;
    return a.w < b.w;
  });
  if (es.size() % 2) return LM_EGRAPH;
  for (size_t i = 0; i < es.size(); i += 2) {
    if (es[i].lo != es[i + 1].lo || es[i].hi != es[i + 1].hi) return LM_EGRAPH;  // missing twin
    if (!(es[i].w == es[i + 1].w)) return LM_EGRAPH;                             // unequal weights
    if (i + 2 < es.size() && es[i + 2].lo == es[i].lo && es[i + 2].hi == es[i].hi) return LM_EGRAPH;  // duplicate
  }
  return LM_OK;
}

extern "C" {

const char* lm_strerror(lm_status st) { return status_text(st); }

lm_status lm_create(int device, size_t hbm_budget_bytes, lm_ctx** out) {
  if (!out) return LM_EINVAL;
  *out = nullptr;
  lm_ctx* c = new (std::nothrow) lm_ctx();
  if (!c) return LM_ENOMEM;
  const size_t budget = hbm_budget_bytes ? hbm_budget_bytes : ((size_t)64 << 30);
  lm_status st = c->s.init_device(device, budget);
  if (st != LM_OK) {
    c->s.shutdown();
    delete c;
    return st;
  }
  *out = c;
  return LM_OK;
}

void lm_destroy(lm_ctx* c) {
  if (!c) return;
  c->s.shutdown();
  delete c;
}

lm_status lm_get_tuning(lm_ctx* c, lm_tuning* out) {
  if (!c || !out) return LM_EINVAL;
  *out = c->s.tun;
  return LM_OK;
}

lm_status lm_set_tuning(lm_ctx* c, const lm_tuning* t) {
  if (!c || !t) return LM_EINVAL;
  if (t->block_entries < 2048 || t->block_entries > (1 << 22)) return LM_EINVAL;
  if (t->grid_per_cu < 1 || t->grid_per_cu > 16) return LM_EINVAL;
  if (t->phases_per_sync < 1 || t->phases_per_sync > 64) return LM_EINVAL;
  if (t->tail_entries < 0 || t->tail_entries > (1 << 30)) return LM_EINVAL;
  c->s.tun = *t;
  return LM_OK;
}

// Shared body of lm_match and lm_match_batch.
static lm_status solve_common(lm_ctx* c, int64_t N, int64_t nnz, int64_t G, const int64_t* h_vtx_off,
                              const int64_t* row_ptr, const int32_t* col, const float* w, const uint64_t* seeds,
                              uint64_t seed0, int32_t* mate, uint32_t flags, void* stream, lm_stats* st,
                              int32_t* graph_phases) {
  const uint32_t known = LM_IN_DEVICE | LM_OUT_DEVICE | LM_CHECK_GRAPH | LM_PROFILE | LM_GRAPH | LM_WEIGHT_SUM |
                         LM_ASYNC | LM_RENEW_KEYS;
  if (flags & ~known) return LM_EINVAL;
  if (flags & LM_ASYNC) {  // stream-ordered: device buffers only, nothing to report back
    if ((flags & (LM_IN_DEVICE | LM_OUT_DEVICE)) != (LM_IN_DEVICE | LM_OUT_DEVICE)) return LM_EINVAL;
    if (flags & (LM_CHECK_GRAPH | LM_PROFILE | LM_WEIGHT_SUM)) return LM_EINVAL;
    if (st || graph_phases) return LM_EINVAL;
  }
  if (N < 0 || nnz < 0 || G < 1) return LM_EINVAL;
  if (N >= ((int64_t)1 << 31) || nnz >= ((int64_t)1 << 31) - 65536) return LM_ETOOBIG;
  if (N > 0 && (!row_ptr || !mate)) return LM_EINVAL;
  if (nnz > 0 && !col) return LM_EINVAL;  // w == nullptr: unweighted graph
  Solver& S = c->s;
  if (hipSetDevice(S.dev) != hipSuccess) return LM_EDEVICE;
  // the context's buffers belong to a pending stream-ordered solve until it ends
  if (S.async_pending) {
    if (hipEventSynchronize(S.e_async) != hipSuccess) return LM_EDEVICE;
    S.async_pending = false;
  }
  // The caller named the legacy default stream (or none): the solve runs on it,
  // after everything already queued there (for example the kernels that
  // produced device inputs). A captured graph needs a stream of its own, which
  // then waits for the default stream.
  const bool own_stream = !stream && (flags & LM_GRAPH) && !(flags & LM_PROFILE);
  hipStream_t s = stream ? (hipStream_t)stream : (own_stream ? S.own : nullptr);
  if (own_stream) {
    if (hipEventRecord(S.e_order, nullptr) != hipSuccess || hipStreamWaitEvent(s, S.e_order, 0) != hipSuccess) {
      (void)hipGetLastError();
      return LM_EDEVICE;
    }
  }
  const bool in_dev = (flags & LM_IN_DEVICE) != 0;
  const bool out_dev = (flags & LM_OUT_DEVICE) != 0;
  // host-side checks that need no device work
  if (!in_dev && N > 0) {
    if (row_ptr[0] != 0 || row_ptr[N] != nnz) return LM_EINVAL;
    if (flags & LM_CHECK_GRAPH) {
      for (int64_t g = 0; g < G; ++g) {
        const int64_t a = h_vtx_off ? h_vtx_off[g] : 0, b = h_vtx_off ? h_vtx_off[g + 1] : N;
        const int64_t e0 = row_ptr[a];
        std::vector<int64_t> rp((size_t)(b - a + 1));
        for (int64_t v = 0; v <= b - a; ++v) rp[(size_t)v] = row_ptr[a + v] - e0;
        lm_status hs = host_check(b - a, rp.data(), col + e0, w ? w + e0 : nullptr, rp[(size_t)(b - a)]);
        if (hs != LM_OK) return hs;
      }
    }
  }
  if (st) {
    st->phases = 0;
    st->matched_edges = 0;
    st->device_ms = 0.0;
    st->bytes_alg = 0.0;
    st->log_len = 0;
    st->matched_weight = 0.0;
  }
  if (graph_phases)
    for (int64_t g = 0; g < G; ++g) graph_phases[g] = 0;
  if (N == 0) return LM_OK;
  // memory: footprint plus staging of host inputs / outputs
  size_t need = solve_footprint(N, nnz, G);
  if (!in_dev) need += (size_t)(N + 1) * 8 + (size_t)nnz * (w ? 8 : 4) + 1024;
  if (!out_dev) need += (size_t)N * 4 + 256;
  if (need > S.pool.budget) return LM_ETOOBIG;
  lm_status rs = S.prepare(N, nnz, G, graph_phases != nullptr);
  if (rs != LM_OK) return rs;
  const int64_t* d_rp = row_ptr;
  const int32_t* d_col = col;
  const float* d_w = w;
  if (!in_dev) {
    if ((rs = S.pool.reserve(S.in_rp, (size_t)(N + 1) * 8)) != LM_OK) return rs;
    if ((rs = S.pool.reserve(S.in_col, (size_t)nnz * 4)) != LM_OK) return rs;
    if (w && (rs = S.pool.reserve(S.in_w, (size_t)nnz * 4)) != LM_OK) return rs;
    if (hipMemcpyAsync(S.in_rp.p, row_ptr, (size_t)(N + 1) * 8, hipMemcpyHostToDevice, s) != hipSuccess ||
        (nnz > 0 && hipMemcpyAsync(S.in_col.p, col, (size_t)nnz * 4, hipMemcpyHostToDevice, s) != hipSuccess) ||
        (w && nnz > 0 && hipMemcpyAsync(S.in_w.p, w, (size_t)nnz * 4, hipMemcpyHostToDevice, s) != hipSuccess))
      return LM_EDEVICE;
    d_rp = (const int64_t*)S.in_rp.p;
    d_col = (const int32_t*)S.in_col.p;
    d_w = w ? (const float*)S.in_w.p : nullptr;
  }
  int32_t* d_mate = mate;
  if (!out_dev) {
    if ((rs = S.pool.reserve(S.out_mate, (size_t)N * 4)) != LM_OK) return rs;
    d_mate = (int32_t*)S.out_mate.p;
  }
  // per-graph tables
  std::vector<int32_t> hb((size_t)G);
  std::vector<uint64_t> hs((size_t)G);
  std::vector<int64_t> hv((size_t)G + 1);
  for (int64_t g = 0; g < G; ++g) {
    hb[(size_t)g] = (int32_t)(h_vtx_off ? h_vtx_off[g] : 0);
    hs[(size_t)g] = premix_seed(seeds ? seeds[g] : seed0);
    hv[(size_t)g] = h_vtx_off ? h_vtx_off[g] : 0;
  }
  hv[(size_t)G] = h_vtx_off ? h_vtx_off[G] : N;
  // The tables live on the device between solves: upload only what changed
  // (repeated solves of one shape and seed upload nothing), from pinned memory.
  if (hb != S.t_gbase || hs != S.t_gseed || hv != S.t_vtxoff || S.t_dev[0] != S.gbase.p ||
      S.t_dev[1] != S.gseed.p || S.t_dev[2] != S.vtxoff.p) {
    const size_t bytes = (size_t)G * 4 + (size_t)G * 8 + (size_t)(G + 1) * 8 + 64;
    if (S.t_pinned_cap < bytes) {
      if (S.t_pinned) (void)hipHostFree(S.t_pinned);
      S.t_pinned = nullptr;
      S.t_pinned_cap = 0;
      if (hipHostMalloc(&S.t_pinned, bytes) != hipSuccess) return LM_ENOMEM;
      S.t_pinned_cap = bytes;
    }
    // the last copies out of the staging area must have landed before it is rewritten
    if (hipEventSynchronize(S.e_tables) != hipSuccess) return LM_EDEVICE;
    char* ph = (char*)S.t_pinned;
    int64_t* pv = (int64_t*)ph;
    uint64_t* ps = (uint64_t*)(ph + (size_t)(G + 1) * 8);
    int32_t* pb = (int32_t*)(ph + (size_t)(G + 1) * 8 + (size_t)G * 8);
    std::memcpy(pv, hv.data(), (size_t)(G + 1) * 8);
    std::memcpy(ps, hs.data(), (size_t)G * 8);
    std::memcpy(pb, hb.data(), (size_t)G * 4);
    S.t_dev[0] = S.t_dev[1] = S.t_dev[2] = nullptr;  // invalid until the copies are queued
    if (hipMemcpyAsync(S.gbase.p, pb, (size_t)G * 4, hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemcpyAsync(S.gseed.p, ps, (size_t)G * 8, hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemcpyAsync(S.vtxoff.p, pv, (size_t)(G + 1) * 8, hipMemcpyHostToDevice, s) != hipSuccess ||
        hipEventRecord(S.e_tables, s) != hipSuccess)
      return LM_EDEVICE;
    S.t_gbase = std::move(hb);
    S.t_gseed = std::move(hs);
    S.t_vtxoff = std::move(hv);
    S.t_dev[0] = S.gbase.p;
    S.t_dev[1] = S.gseed.p;
    S.t_dev[2] = S.vtxoff.p;
  }
  Problem p;
  p.N = N;
  p.nnz = nnz;
  p.G = G;
  p.row_ptr = (const long long*)d_rp;
  p.col = d_col;
  p.w = d_w;
  p.vtx_off = (const long long*)S.vtxoff.p;
  p.mate = d_mate;
  p.gphase = graph_phases ? (int*)S.gphase.p : nullptr;
  lm_stats local;
  std::memset(&local, 0, sizeof(local));
  lm_stats* sp = st ? st : &local;
  if (in_dev && (flags & LM_CHECK_GRAPH)) {  // host inputs were checked on the host
    rs = check_row_duplicates(S, N, nnz, p.row_ptr, p.col, s);
    if (rs != LM_OK) return rs;
  }
  rs = S.run(p, S.pool_work(), s, flags, sp);
  if (rs != LM_OK) return rs;
  if (flags & LM_ASYNC) return LM_OK;  // enqueued; the result lands in order on the stream
  double wsum = 0.0;
  const bool want_w = st && (flags & LM_WEIGHT_SUM);
  if (want_w) {  // after the solve's timed region
    if ((rs = S.pool.reserve(S.wsum, sizeof(double) * (kWeightSumMaxGrid + 1))) != LM_OK) return rs;
    double* ws = (double*)S.wsum.p;
    if (launch_weight_sum(p.row_ptr, p.col, p.w, p.mate, N, ws, s) != hipSuccess ||
        hipMemcpyAsync(&wsum, ws + kWeightSumMaxGrid, sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess) {
      (void)hipGetLastError();
      return LM_EDEVICE;
    }
  }
  if (!out_dev) {
    if (hipMemcpyAsync(mate, d_mate, (size_t)N * 4, hipMemcpyDeviceToHost, s) != hipSuccess) return LM_EDEVICE;
  }
  if (graph_phases) {
    if (hipMemcpyAsync(graph_phases, S.gphase.p, (size_t)G * 4, hipMemcpyDeviceToHost, s) != hipSuccess)
      return LM_EDEVICE;
  }
  if (hipStreamSynchronize(s) != hipSuccess) return LM_EDEVICE;
  if (want_w) st->matched_weight = wsum;
  return LM_OK;
}

lm_status lm_match(lm_ctx* c, const lm_csr* g, uint64_t seed, int32_t* mate, uint32_t flags, void* stream,
                   lm_stats* st) {
  if (!c || !csr_shape_ok(g)) return LM_EINVAL;
  std::lock_guard<std::mutex> lk(c->mu);
  if (c->s.busy_server) return LM_EINVAL;
  return solve_common(c, g->n, g->nnz, 1, nullptr, g->row_ptr, g->col, g->w, nullptr, seed, mate, flags, stream, st,
                      nullptr);
}

lm_status lm_match_batch(lm_ctx* c, int32_t graphs, const int64_t* vtx_off, int64_t nnz, const int64_t* row_ptr,
                         const int32_t* col, const float* w, const uint64_t* seeds, uint64_t seed0, int32_t* mate,
                         uint32_t flags, void* stream, lm_stats* st, int32_t* graph_phases) {
  if (!c || graphs < 1 || !vtx_off) return LM_EINVAL;
  if (vtx_off[0] != 0) return LM_EINVAL;
  for (int32_t g = 0; g < graphs; ++g)
    if (vtx_off[g + 1] < vtx_off[g]) return LM_EINVAL;
  std::lock_guard<std::mutex> lk(c->mu);
  if (c->s.busy_server) return LM_EINVAL;
  return solve_common(c, vtx_off[graphs], nnz, graphs, vtx_off, row_ptr, col, w, seeds, seed0, mate, flags, stream,
                      st, graph_phases);
}

}  // extern "C"

namespace lm {
// Used by the server and the autotuner (same translation-unit rules as the C
// ABI entry points: the caller holds the context lock).
lm_status solve_locked(lm_ctx* c, int64_t N, int64_t nnz, int64_t G, const int64_t* h_vtx_off, const int64_t* row_ptr,
                       const int32_t* col, const float* w, const uint64_t* seeds, uint64_t seed0, int32_t* mate,
                       uint32_t flags, void* stream, lm_stats* st, int32_t* graph_phases) {
  return solve_common(c, N, nnz, G, h_vtx_off, row_ptr, col, w, seeds, seed0, mate, flags, stream, st, graph_phases);
}
Solver& solver_of(lm_ctx* c) { return c->s; }
std::mutex& mutex_of(lm_ctx* c) { return c->mu; }
}  // namespace lm
