// Continuous batching for the request server (lm_server_* in batched mode).
//
// All resident graphs share one live set and every phase launch. A request
// joins at a phase boundary: its CSR is appended behind the live entries, its
// rows become new runs of the live set, and one first-argmax launch computes
// its candidates; from then on it goes through the same mutual / compaction /
// plan kernels as everything else. A graph leaves once it has no live row:
// its mate[] range is copied out, and its vertex range and table slot are
// reused. Keys use each graph's local ids and its own seed, and graphs share
// no edges, so every result equals solving that graph alone (paper, Section
// 2: a phase only looks at edges incident to a vertex).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <deque>
#include <cstring>
#include <iterator>
#include <map>
#include <vector>

#include "lm.h"
#include "lm_internal.h"
#include "lm_runtime.h"
#include "lm_server_impl.h"

namespace lm {

using Clock = std::chrono::steady_clock;

// Capacity of the resident set for an HBM budget: 50 % for the two entry
// buffers (col + w, 16 B per entry), 35 % for per-vertex state (C 4, state 1,
// mate 4, two piece buffers of 2 records per vertex 64, row staging 8 B) and
// 15 % for the staging area that receives requests while others compute.
void server_caps(size_t budget, int64_t* n_cap, int64_t* e_cap, int64_t* stage_cap) {
  const double b = (double)budget;
  int64_t e = (int64_t)(b * 0.50 / 16.0);
  int64_t n = (int64_t)(b * 0.35 / 81.0);
  e = std::min<int64_t>(e, ((int64_t)1 << 31) - 65536 - 1);
  n = std::min<int64_t>(n, (int64_t)1 << 29);
  *e_cap = std::max<int64_t>(e, 0);
  *n_cap = std::max<int64_t>(n, 0);
  *stage_cap = (int64_t)(b * 0.15) & ~(int64_t)255;
}

namespace {

struct SlotInit {
  int slot;
  int gbase;
  int gphase;
  int pad;
  unsigned long long gseed;
};

__global__ void k_slots(const SlotInit* in, int count, int* gbase, int* gphase, unsigned long long* gseed) {
  for (int i = threadIdx.x; i < count; i += blockDim.x) {
    const SlotInit x = in[i];
    gbase[x.slot] = x.gbase;
    gphase[x.slot] = x.gphase;
    gseed[x.slot] = x.gseed;
  }
}

}  // namespace

struct BatchedState {
  ServerCore* S = nullptr;
  int dev = 0, num_cus = 1, bpc = 1;
  lm_tuning tun{};
  hipStream_t s = nullptr;   // phase launches and admission
  hipStream_t cs = nullptr;  // host-to-device staging of queued requests
  Pool pool;
  int64_t n_cap = 0, e_cap = 0, rows_cap = 0, stage_cap = 0;
  DevBuf stage;
  // staged requests in arrival order and their byte ranges in `stage` (a ring)
  std::deque<std::shared_ptr<Request>> staged;
  std::deque<std::pair<int64_t, int64_t>> stage_ranges;
  size_t stage_release = 0;  // ranges freed at the next sync (admitted requests)
  std::vector<hipEvent_t> free_events;
  int s_cap = 0;
  DevBuf C, state, mate, rows[2], ecol[2], ew[2], runs[2], epre[2], rpre[2];
  DevBuf ctl, epre_t, rpre_t, parts, bstat, mcount, gbase, gseed, gphase, totals, st_rp, st_vo, st_slot, st_init;
  // pinned host mirrors
  Ctl* h_ctl = nullptr;  // 3
  Totals* h_tot = nullptr;
  int* h_gphase = nullptr;
  long long* h_vo = nullptr;
  int* h_slot = nullptr;
  SlotInit* h_init = nullptr;
  // residency
  std::vector<std::shared_ptr<Request>> slot_req;
  std::vector<int> free_slots;
  std::map<int64_t, int64_t> free_v;  // start -> length
  int t = 1;
  int64_t L_now = 0, pieces_now = 0, nruns_now = 0;
  int64_t phys_end = 0, rows_end = 0, n_res = 0;
  int resident = 0;
  int pcap = 1, pmcap = 1;

  bool stage_alloc(int64_t bytes, int64_t* off);
  hipEvent_t take_event();
  lm_status init(ServerCore* core);
  void shutdown();
  Common common() const;
  LiveSet live(int tt) const;
  lm_status admit(std::vector<std::shared_ptr<Request>>& group, int64_t v0);
  lm_status step(int k);
  lm_status sync_and_retire();
  void fail_all(lm_status st);
  void reset_live();
};

static int64_t vtake_at(std::map<int64_t, int64_t>& fr, int64_t at, int64_t len) {
  auto it = fr.find(at);
  const int64_t rest = it->second - len;
  fr.erase(it);
  if (rest > 0) fr[at + len] = rest;
  return at;
}

static void vgive(std::map<int64_t, int64_t>& fr, int64_t at, int64_t len) {
  if (len <= 0) return;
  auto nx = fr.lower_bound(at);
  if (nx != fr.end() && nx->first == at + len) {
    len += nx->second;
    nx = fr.erase(nx);
  }
  if (nx != fr.begin()) {
    auto pv = std::prev(nx);
    if (pv->first + pv->second == at) {
      pv->second += len;
      return;
    }
  }
  fr[at] = len;
}

// Ring allocation in arrival order; ranges are released in the same order.
bool BatchedState::stage_alloc(int64_t bytes, int64_t* off) {
  if (bytes > stage_cap) return false;
  int64_t at;
  if (stage_ranges.empty()) {
    at = 0;
  } else {
    const int64_t first = stage_ranges.front().first;
    const int64_t end = stage_ranges.back().first + stage_ranges.back().second;
    if (end > first) {  // not wrapped: free space is [end, cap) and [0, first)
      if (end + bytes <= stage_cap)
        at = end;
      else if (bytes <= first)
        at = 0;
      else
        return false;
    } else {  // wrapped: free space is [end, first)
      if (end + bytes <= first)
        at = end;
      else
        return false;
    }
  }
  stage_ranges.push_back({at, bytes});
  *off = at;
  return true;
}

hipEvent_t BatchedState::take_event() {
  if (!free_events.empty()) {
    hipEvent_t e = free_events.back();
    free_events.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return nullptr;
  return e;
}

lm_status BatchedState::init(ServerCore* core) {
  S = core;
  Solver& sv = solver_of(core->ctx);
  dev = sv.dev;
  num_cus = sv.num_cus;
  bpc = sv.bpc_stream;
  tun = sv.tun;
  if (hipSetDevice(dev) != hipSuccess) return LM_EDEVICE;
  if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return LM_EDEVICE;
  if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) return LM_EDEVICE;
  server_caps(core->opts.hbm_budget_bytes, &n_cap, &e_cap, &stage_cap);
  s_cap = std::max(2, core->opts.max_resident);
  rows_cap = 2 * n_cap + 2 * kMaxBlocks + 16;
  pool.budget = core->opts.hbm_budget_bytes + ((size_t)64 << 20);
  pcap = std::max(1, std::min(kMaxBlocks / 2, num_cus * std::max(1, std::min(tun.grid_per_cu, bpc))));
  pmcap = std::max(1, std::min(kMaxBlocks, num_cus * 8));
  lm_status st = LM_OK;
#define RES(buf, bytes)                 \
  do {                                  \
    st = pool.reserve(buf, (bytes));    \
    if (st != LM_OK) return st;         \
  } while (0)
  RES(C, (size_t)n_cap * 4);
  RES(state, (size_t)n_cap);
  RES(mate, (size_t)n_cap * 4);
  for (int i = 0; i < 2; ++i) {
    RES(rows[i], (size_t)rows_cap * 16);
    RES(ecol[i], (size_t)e_cap * 4);
    RES(ew[i], (size_t)e_cap * 4);
    RES(runs[i], (size_t)kMaxBlocks * sizeof(Run));
    RES(epre[i], (size_t)(kMaxBlocks + 1) * 8);
    RES(rpre[i], (size_t)(kMaxBlocks + 1) * 4);
  }
  RES(ctl, 3 * sizeof(Ctl));
  RES(epre_t, (size_t)(kMaxBlocks + 1) * 8);
  RES(rpre_t, (size_t)(kMaxBlocks + 1) * 4);
  RES(parts, (size_t)kMaxBlocks * 2 * sizeof(Part));
  RES(bstat, (size_t)kMaxBlocks * sizeof(BlockStat));
  RES(mcount, (size_t)kMaxBlocks * 4);
  RES(gbase, (size_t)s_cap * 4);
  RES(gseed, (size_t)s_cap * 8);
  RES(gphase, (size_t)s_cap * 4);
  RES(totals, sizeof(Totals));
  RES(st_rp, ((size_t)n_cap + 1) * 8);
  RES(st_vo, ((size_t)s_cap + 1) * 8);
  RES(st_slot, (size_t)s_cap * 4);
  RES(st_init, (size_t)s_cap * sizeof(SlotInit));
  RES(stage, (size_t)std::max<int64_t>(stage_cap, 256));
#undef RES
  if (hipHostMalloc((void**)&h_ctl, 3 * sizeof(Ctl)) != hipSuccess ||
      hipHostMalloc((void**)&h_tot, sizeof(Totals)) != hipSuccess ||
      hipHostMalloc((void**)&h_gphase, (size_t)s_cap * 4) != hipSuccess ||
      hipHostMalloc((void**)&h_vo, ((size_t)s_cap + 1) * 8) != hipSuccess ||
      hipHostMalloc((void**)&h_slot, (size_t)s_cap * 4) != hipSuccess ||
      hipHostMalloc((void**)&h_init, (size_t)s_cap * sizeof(SlotInit)) != hipSuccess)
    return LM_ENOMEM;
  slot_req.assign((size_t)s_cap, nullptr);
  for (int i = s_cap - 1; i >= 0; --i) free_slots.push_back(i);
  if (n_cap > 0) free_v[0] = n_cap;
  reset_live();
  if (hipStreamSynchronize(s) != hipSuccess) return LM_EDEVICE;
  return LM_OK;
}

void BatchedState::shutdown() {
  if (cs) (void)hipStreamSynchronize(cs);
  if (s) (void)hipStreamSynchronize(s);
  for (hipEvent_t e : free_events) (void)hipEventDestroy(e);
  free_events.clear();
  pool.release(stage);
  if (cs) (void)hipStreamDestroy(cs);
  cs = nullptr;
  DevBuf* all[] = {&C,       &state,   &mate,    &rows[0], &rows[1], &ecol[0], &ecol[1], &ew[0],  &ew[1],
                   &runs[0], &runs[1], &epre[0], &epre[1], &rpre[0], &rpre[1], &ctl,     &epre_t, &rpre_t,
                   &parts,   &bstat,   &mcount,  &gbase,   &gseed,   &gphase,  &totals,  &st_rp,  &st_vo,
                   &st_slot, &st_init};
  for (DevBuf* b : all) pool.release(*b);
  void* hp[] = {h_ctl, h_tot, h_gphase, h_vo, h_slot, h_init};
  for (void* p : hp)
    if (p) (void)hipHostFree(p);
  if (s) (void)hipStreamDestroy(s);
  s = nullptr;
}

Common BatchedState::common() const {
  Common c;
  c.totals = (Totals*)totals.p;
  c.n = (int)n_cap;
  c.C = (int*)C.p;
  c.state = (unsigned char*)state.p;
  c.mate = (int*)mate.p;
  c.gbase = (const int*)gbase.p;
  c.gseed = (const unsigned long long*)gseed.p;
  c.gphase = (int*)gphase.p;
  c.graphs = s_cap;  // >= 2: every piece looks up its graph's base and seed
  return c;
}

LiveSet BatchedState::live(int tt) const {
  const int i = (tt - 1) & 1;
  LiveSet L;
  L.ctl = (const Ctl*)ctl.p + i;
  L.runs = (const Run*)runs[i].p;
  L.epre = (const long long*)epre[i].p;
  L.rpre = (const int*)rpre[i].p;
  L.rows = (int4*)rows[i].p;
  L.col = (const int*)ecol[tt & 1].p;
  L.w = (const float*)ew[tt & 1].p;
  L.csr_rp = nullptr;  // every live set has piece records here
  return L;
}

void BatchedState::reset_live() {
  (void)launch_zero((Ctl*)ctl.p, 3, (Totals*)totals.p, s);  // device phase counter back to 1
  t = 1;
  L_now = pieces_now = nruns_now = 0;
  phys_end = rows_end = 0;
}

// Appends a group of requests (vertex range [v0, v0 + sum n)) to the live set
// R_t before phase t.
lm_status BatchedState::admit(std::vector<std::shared_ptr<Request>>& group, int64_t v0) {
  const int G = (int)group.size();
  const Common c = common();
  const int ti = (t - 1) & 1;
  int* dcol = (int*)ecol[t & 1].p;
  float* dw = (float*)ew[t & 1].p;
  long long* drp = (long long*)st_rp.p;
  const int64_t ebase = phys_end;
  int64_t xo = 0, eo = 0;
  auto fail = [&](hipError_t e) {
    (void)hipGetLastError();
    return dev_status(e);
  };
  for (int i = 0; i < G; ++i) {
    Request& r = *group[(size_t)i];
    // the request's graph is already in the staging area (copy stream):
    // wait for that copy, then move it into place on the device
    const char* src = (const char*)stage.p + r.stage_off;
    hipError_t e = hipStreamWaitEvent(s, r.stage_ev, 0);
    if (e == hipSuccess) e = hipMemcpyAsync(drp + xo, src, (size_t)(r.n + 1) * 8, hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess) e = launch_add_i64(drp + xo, r.n + 1, ebase + eo, s);
    if (e == hipSuccess && r.nnz > 0)
      e = hipMemcpyAsync(dcol + ebase + eo, src + r.off_col, (size_t)r.nnz * 4, hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess && r.nnz > 0)
      e = hipMemcpyAsync(dw + ebase + eo, src + r.off_w, (size_t)r.nnz * 4, hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return fail(e);
    h_vo[i] = xo;
    h_slot[i] = r.slot;
    SlotInit si;
    si.slot = r.slot;
    si.gbase = (int)(v0 + xo);
    si.gphase = t - 1;  // a graph without edges has no live row in phase t
    si.pad = 0;
    si.gseed = premix_seed(r.seed);
    h_init[i] = si;
    r.vbase = v0 + xo;
    r.first_phase = t;
    xo += r.n;
    eo += r.nnz;
  }
  h_vo[G] = xo;
  hipError_t e = hipMemcpyAsync(st_vo.p, h_vo, ((size_t)G + 1) * 8, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(st_slot.p, h_slot, (size_t)G * 4, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(st_init.p, h_init, (size_t)G * sizeof(SlotInit), hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return fail(e);
  hipLaunchKernelGGL(k_slots, dim3(1), dim3(256), 0, s, (const SlotInit*)st_init.p, G, (int*)gbase.p,
                     (int*)gphase.p, (unsigned long long*)gseed.p);
  if ((e = hipGetLastError()) != hipSuccess) return fail(e);
  if (xo == 0) return LM_OK;  // no vertices: nothing to add to the live set
  const int nb = (int)std::max<int64_t>(1, std::min<int64_t>(pcap, (xo + 16383) / 16384));
  Run* truns = (Run*)runs[ti].p;
  Ctl* dctl = (Ctl*)ctl.p;
  InitArgs ia;
  ia.c = c;
  ia.row_ptr = drp;
  ia.nnz = eo;
  ia.ebase = ebase;
  ia.vfirst = v0;
  ia.vcount = xo;
  ia.graphs = G;
  ia.vtx_off = (const long long*)st_vo.p;
  ia.slot_of = (const int*)st_slot.p;
  ia.nblocks = nb;
  ia.rows_base = (int)rows_end;
  ia.runs_base = (int)nruns_now;
  ia.runs_out = truns;
  ia.rows_out = (int4*)rows[ti].p;
  ia.csr = 0;
  ia.bstat = nullptr;
  if ((e = launch_init(ia, s)) != hipSuccess) return fail(e);
  PlanArgs pa;
  std::memset(&pa, 0, sizeof(pa));
  pa.c = c;
  pa.pcap = pcap;
  pa.pmcap = pmcap;
  pa.min_per_block = std::max(kCap, tun.block_entries);
  // run table of the new rows alone, for their first argmax
  pa.mode = kPlanPrefix;
  pa.runs_new = truns + nruns_now;
  pa.nruns_new = nb;
  pa.epre_new = (long long*)epre_t.p;
  pa.rpre_new = (int*)rpre_t.p;
  pa.ctl_new = dctl + 2;
  if ((e = launch_plan(pa, s)) != hipSuccess) return fail(e);
  StreamArgs sa;
  std::memset(&sa, 0, sizeof(sa));
  sa.c = c;
  sa.in.ctl = dctl + 2;
  sa.in.runs = truns + nruns_now;
  sa.in.epre = (const long long*)epre_t.p;
  sa.in.rpre = (const int*)rpre_t.p;
  sa.in.rows = (int4*)rows[ti].p;
  sa.in.col = dcol;
  sa.in.w = dw;
  sa.parts = (Part*)parts.p;
  sa.bstat = (BlockStat*)bstat.p;
  const int gx = (int)std::max<int64_t>(1, std::min<int64_t>(pcap, eo / std::max(kCap, tun.block_entries) + 1));
  if ((e = launch_first_argmax(sa, gx, s)) != hipSuccess) return fail(e);
  PlanArgs pf = pa;
  pf.mode = kPlanFix;
  pf.first = 1;
  pf.ctl_prev = dctl + 2;
  pf.parts = (Part*)parts.p;
  if ((e = launch_plan(pf, s)) != hipSuccess) return fail(e);
  // merged run table: the live runs followed by the new ones
  PlanArgs pm = pa;
  pm.runs_new = truns;
  pm.nruns_new = (int)(nruns_now + nb);
  pm.epre_new = (long long*)epre[ti].p;
  pm.rpre_new = (int*)rpre[ti].p;
  pm.ctl_new = dctl + ti;
  if ((e = launch_plan(pm, s)) != hipSuccess) return fail(e);
  nruns_now += nb;
  phys_end += eo;
  rows_end += xo;
  L_now += eo;
  pieces_now += xo;
  return LM_OK;
}

// k phases over the live set, then a census of the graphs that still have a
// live row.
lm_status BatchedState::step(int k) {
  const Common c = common();
  Ctl* dctl = (Ctl*)ctl.p;
  hipError_t e = hipSuccess;
  for (int j = 0; j < k && e == hipSuccess; ++j) {
    const LiveSet in = live(t);
    MutualArgs ma;
    ma.c = c;
    ma.in = in;
    ma.mcount = (int*)mcount.p;
    ma.census = 0;
    const int gm = (int)std::max<int64_t>(1, std::min<int64_t>(pmcap, pieces_now / kMutualRound + 1));
    e = launch_mutual(ma, gm, s);
    if (e != hipSuccess) break;
    const int lo = t & 1;
    StreamArgs sa;
    sa.c = c;
    sa.in = in;
    sa.cand_phase = t + 1;  // (fixed keys: unused)
    sa.runs_out = (Run*)runs[lo].p;
    sa.rows_out = (int4*)rows[lo].p;
    sa.dst_col = (int*)ecol[(t + 1) & 1].p;
    sa.dst_w = (float*)ew[(t + 1) & 1].p;
    sa.parts = (Part*)parts.p;
    sa.bstat = (BlockStat*)bstat.p;
    const int gx =
        (int)std::max<int64_t>(1, std::min<int64_t>(pcap, L_now / std::max(kCap, tun.block_entries) + 1));
    e = launch_compact(sa, gx, s);
    if (e != hipSuccess) break;
    PlanArgs pa;
    std::memset(&pa, 0, sizeof(pa));
    pa.c = c;
    pa.mode = kPlanFix | kPlanPrefix | kPlanTick;
    pa.ctl_prev = in.ctl;
    pa.parts = (Part*)parts.p;
    pa.bstat = (BlockStat*)bstat.p;
    pa.rows_out = (int4*)rows[lo].p;
    pa.runs_new = (const Run*)runs[lo].p;
    pa.nruns_new = -1;
    pa.epre_new = (long long*)epre[lo].p;
    pa.rpre_new = (int*)rpre[lo].p;
    pa.ctl_new = dctl + lo;
    pa.pcap = pcap;
    pa.pmcap = pmcap;
    pa.min_per_block = std::max(kCap, tun.block_entries);
    e = launch_plan(pa, s);
    ++t;
  }
  if (e == hipSuccess) {
    MutualArgs ma;
    ma.c = c;
    ma.in = live(t);
    ma.mcount = (int*)mcount.p;
    ma.census = 1;
    e = launch_mutual(ma, (int)std::max<int64_t>(1, std::min<int64_t>(pmcap, pieces_now / kMutualRound + 1)), s);
  }
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return dev_status(e);
  }
  return LM_OK;
}

lm_status BatchedState::sync_and_retire() {
  hipError_t e = hipMemcpyAsync(h_ctl, ctl.p, 2 * sizeof(Ctl), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipMemcpyAsync(h_tot, totals.p, sizeof(Totals), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipMemcpyAsync(h_gphase, gphase.p, (size_t)s_cap * 4, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return dev_status(e);
  }
  if (h_tot->err) {
    const unsigned err = h_tot->err;
    if (err & kErrWeight) return LM_EWEIGHT;
    if (err & (kErrRowPtr | kErrColRange | kErrSelfLoop)) return LM_EGRAPH;
    return LM_EDEVICE;
  }
  const Ctl& now = h_ctl[(t - 1) & 1];
  const Ctl& prev = h_ctl[t & 1];
  L_now = now.L;
  pieces_now = now.pieces;
  nruns_now = now.nruns;
  phys_end = prev.L;
  rows_end = (int64_t)prev.pieces + prev.P;
  for (int sl = 0; sl < s_cap; ++sl) {
    std::shared_ptr<Request> r = slot_req[(size_t)sl];
    if (!r || h_gphase[sl] >= t) continue;  // still has a live row in R_t
    r->t_solved = Clock::now();
    r->mate.resize((size_t)r->n);
    lm_status st = LM_OK;
    if (r->n > 0 &&
        hipMemcpy(r->mate.data(), (int*)mate.p + r->vbase, (size_t)r->n * 4, hipMemcpyDeviceToHost) != hipSuccess) {
      (void)hipGetLastError();
      st = LM_EDEVICE;
    }
    r->phases = std::max(0, h_gphase[sl] - r->first_phase + 1);
    int64_t m = 0;
    for (int32_t x : r->mate) m += (x >= 0);
    r->matched = m / 2;
    slot_req[(size_t)sl] = nullptr;
    free_slots.push_back(sl);
    vgive(free_v, r->vbase, r->n);
    n_res -= r->n;
    --resident;
    if (r->stage_ev) free_events.push_back(r->stage_ev);
    r->stage_ev = nullptr;
    S->finish(r, st);
  }
  if (resident == 0) {
    reset_live();
    return LM_OK;
  }
  // every phase matches the largest live edge of each graph, so a graph with
  // m edges needs at most m phases; more means its input broke the contract
  for (int sl = 0; sl < s_cap; ++sl) {
    const Request* r = slot_req[(size_t)sl].get();
    if (r && (int64_t)(t - r->first_phase) > r->nnz / 2 + 2) return LM_EGRAPH;
  }
  return LM_OK;
}

void BatchedState::fail_all(lm_status st) {
  (void)hipStreamSynchronize(cs);
  (void)hipStreamSynchronize(s);
  (void)hipGetLastError();
  for (int sl = 0; sl < s_cap; ++sl) {
    std::shared_ptr<Request> r = slot_req[(size_t)sl];
    if (!r) continue;
    slot_req[(size_t)sl] = nullptr;
    free_slots.push_back(sl);
    vgive(free_v, r->vbase, r->n);
    n_res -= r->n;
    --resident;
    if (r->stage_ev) free_events.push_back(r->stage_ev);
    r->stage_ev = nullptr;
    S->finish(r, st);
  }
  // staged requests that were not admitted yet fail too (their copies may
  // have failed); the staging area starts over
  for (auto& r : staged) {
    if (r->stage_ev) free_events.push_back(r->stage_ev);
    r->stage_ev = nullptr;
    {
      std::lock_guard<std::mutex> lk(S->mu);
      S->running[r->ticket] = r;
    }
    S->finish(r, st);
  }
  staged.clear();
  stage_ranges.clear();
  stage_release = 0;
  reset_live();
}

static void batch_loop(ServerCore* S) {
  BatchedState& B = *S->batched;
  (void)hipSetDevice(B.dev);
  const int k = std::max(1, S->opts.phases_per_step);
  for (;;) {
    std::vector<std::shared_ptr<Request>> fresh;
    std::shared_ptr<Request> solo;
    {
      std::unique_lock<std::mutex> lk(S->mu);
      if (B.resident == 0 && B.staged.empty())
        S->cv_work.wait(lk, [&] { return S->stopping || !S->queue.empty(); });
      if (S->stopping && S->queue.empty() && B.staged.empty() && B.resident == 0) return;
      // A request that finds the server idle (nothing resident, staged or
      // queued behind it) is solved alone on the single-graph path, with its
      // device tail and no phase steps shared with others: batching only
      // pays once requests wait for each other.
      if (B.resident == 0 && B.staged.empty() && S->queue.size() == 1 && !S->queue.front()->no_solo) {
        solo = S->queue.front();
        S->queue.pop_front();
        solo->t_admit = Clock::now();
        S->running[solo->ticket] = solo;
      }
      // start the host-to-device copies of queued requests while the staging
      // area has room; they overlap the phases of the resident graphs
      while (!solo && !S->queue.empty()) {
        auto& r = S->queue.front();
        int64_t off = 0;
        if (!B.stage_alloc((int64_t)r->block_used, &off)) break;
        r->stage_off = off;
        fresh.push_back(r);
        B.staged.push_back(r);
        S->queue.pop_front();
      }
    }
    if (solo) {
      lm_status st;
      {
        std::lock_guard<std::mutex> ck(mutex_of(S->ctx));
        lm_stats stats;
        std::memset(&stats, 0, sizeof(stats));
        solo->mate.assign((size_t)solo->n, -1);
        st = solve_locked(S->ctx, solo->n, solo->nnz, 1, nullptr, solo->h_rp, solo->h_col, solo->h_w, nullptr,
                          solo->seed, solo->mate.data(), 0u, (void*)solver_of(S->ctx).own, &stats, nullptr);
        solo->phases = stats.phases;
        solo->matched = stats.matched_edges;
      }
      if (st == LM_ETOOBIG || st == LM_ENOMEM) {  // beyond the context's pool: the batch takes it
        std::lock_guard<std::mutex> lk(S->mu);
        solo->no_solo = true;
        S->running.erase(solo->ticket);
        S->queue.push_front(solo);
        continue;
      }
      S->finish(solo, st);
      continue;
    }
    lm_status st = LM_OK;
    for (auto& r : fresh) {
      r->stage_ev = B.take_event();
      if (!r->stage_ev ||
          hipMemcpyAsync((char*)B.stage.p + r->stage_off, r->block, r->block_used, hipMemcpyHostToDevice, B.cs) !=
              hipSuccess ||
          hipEventRecord(r->stage_ev, B.cs) != hipSuccess) {
        (void)hipGetLastError();
        st = LM_EDEVICE;
      }
    }
    // admit staged requests in arrival order once their copy has landed (the
    // first one regardless when nothing is resident), while slots, one
    // contiguous vertex range, the entry buffer and the piece buffer have room
    std::vector<std::shared_ptr<Request>> group;
    int64_t v0 = -1;
    if (st == LM_OK) {
      int64_t best_at = -1, best_len = 0;
      for (auto& fr : B.free_v)
        if (fr.second > best_len) {
          best_at = fr.first;
          best_len = fr.second;
        }
      int64_t nsum = 0, esum = 0;
      while (!B.staged.empty() && group.size() < B.free_slots.size()) {
        auto& r = B.staged.front();
        const hipError_t q = hipEventQuery(r->stage_ev);
        if (q != hipSuccess) (void)hipGetLastError();  // not ready yet
        if (q != hipSuccess && !(B.resident == 0 && group.empty())) break;
        if (r->n > 0 && nsum + r->n > best_len) break;
        if (B.phys_end + esum + r->nnz > B.e_cap) break;
        if (B.rows_end + nsum + r->n > B.rows_cap) break;
        nsum += r->n;
        esum += r->nnz;
        group.push_back(r);
        B.staged.pop_front();
      }
      if (!group.empty()) {
        v0 = nsum > 0 ? vtake_at(B.free_v, best_at, nsum) : 0;
        std::lock_guard<std::mutex> lk(S->mu);
        for (auto& r : group) {
          r->t_admit = Clock::now();
          S->running[r->ticket] = r;
        }
      }
    }
    if (st == LM_OK && !group.empty()) {
      for (auto& r : group) {
        r->slot = B.free_slots.back();
        B.free_slots.pop_back();
        B.slot_req[(size_t)r->slot] = r;
        B.n_res += r->n;
        ++B.resident;
      }
      B.stage_release += group.size();
      st = B.admit(group, v0);
    }
    if (st == LM_OK && B.resident > 0) st = B.step(k);
    if (st == LM_OK && (B.resident > 0 || B.stage_release > 0)) st = B.sync_and_retire();
    if (st != LM_OK) {
      B.fail_all(st);
    } else {
      // the admitted requests' staging ranges are free once the stream has
      // passed their device-to-device copies (sync_and_retire waited for it)
      for (; B.stage_release > 0; --B.stage_release) B.stage_ranges.pop_front();
    }
  }
}

lm_status start_batched(ServerCore* s) {
  s->batched = new (std::nothrow) BatchedState();
  if (!s->batched) return LM_ENOMEM;
  lm_status st = s->batched->init(s);
  if (st != LM_OK) {
    s->batched->shutdown();
    delete s->batched;
    s->batched = nullptr;
    return st;
  }
  s->worker = std::thread(batch_loop, s);
  return LM_OK;
}

void stop_batched(ServerCore* s) {
  if (!s->batched) return;
  s->batched->shutdown();
  delete s->batched;
  s->batched = nullptr;
}

}  // namespace lm
