// Device-side tail of the phase loop of local-max matching (gfx950, wave64).
//
// Once the live set is small, a phase costs more in launches and host round
// trips than in work (Section 2: the work of a phase is linear in the live
// edges, and Section 3 notes that the GPU code of the paper was weak on small
// inputs for this reason). k_tail takes the live set R_c the phase kernels
// left behind and runs every remaining phase in one persistent launch:
//
//   mutual   every live vertex v with C[C[v]] = v is matched (mate, state);
//   -------- grid barrier
//   compact  every live row of an unmatched vertex keeps the entries whose
//            neighbour is unmatched, writes them to the same offset of the
//            other entry buffer and computes its new candidate C[v];
//   -------- grid barrier
//   log      the phase record (L_t, V_t, matched_t, matched entries_t).
//
// Nothing is counted through a shared global counter (atomics on one address
// serialise across the dies): workgroup b owns a segment of the next row list
// and reports its counts in a table (TailCtl::seg) that every workgroup reads
// after the barrier; within a workgroup rows are placed with LDS atomics. The
// row order is irrelevant to the result (the key order is strict, so every
// vertex has one candidate whatever the order of its entries). Once a live
// set is at most kTailSolo entries, workgroup 0 finishes alone and the grid
// barriers become workgroup barriers.
#include <hip/hip_ext.h>

#include "lm_device.h"
#include "lm_internal.h"
#include "lm_key.h"

namespace lm {

namespace {

constexpr long long kTailSolo = 16384;  // live entries workgroup 0 handles alone
constexpr int kTW = kTailBlock / 64;    // waves per workgroup
constexpr int kRunCache = kMaxBlocks + 1;

__device__ __forceinline__ unsigned ld_u32(const unsigned* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

struct TailSmem {
  int pre_s[kTailMaxBlocks + 1];  // short rows of the current list before segment b
  int pre_l[kTailMaxBlocks + 1];  // long rows before segment b
  int sbase[kTailMaxBlocks], scap[kTailMaxBlocks];
  long long red[3][kTW];
  long long sum[3];
  int cnt_s, cnt_l;  // rows this workgroup has placed in its segment
  unsigned ok;
  int rp[kRunCache];  // conversion: piece prefix of R_c's runs
};

// Barrier over the whole grid (every workgroup is resident: the host sizes
// the grid from the occupancy of this kernel). Workgroup b arrives at counter
// b % kTailArrive; the last arrival there arrives at the top counter, whose
// last arrival resets it and advances the generation. The workgroup barrier
// first waits for every lane's stores; lane 0 then makes them visible to the
// other dies (release) before it arrives, polls the generation with plain
// device-scope loads (an acquire per poll would invalidate the L2 under the
// workgroups still working) and invalidates its caches once (acquire) when the
// generation moves. A wait longer than `limit` ticks of the constant wall
// clock, or another workgroup's abort, makes every workgroup give up (false).
__device__ bool grid_sync(TailCtl* tc, unsigned nb, unsigned& gen, unsigned long long limit, Totals* tot,
                          TailSmem& sm) {
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned ok = 1u;
    const unsigned g = gen;
    const unsigned b = blockIdx.x;
    const unsigned k = b % kTailArrive;
    const unsigned members = nb / kTailArrive + (k < nb % kTailArrive ? 1u : 0u);
    const unsigned groups = nb < (unsigned)kTailArrive ? nb : (unsigned)kTailArrive;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");  // this die's stores reach the others
    bool last = false;
    if (__hip_atomic_fetch_add(&tc->arrive[k][0], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == members - 1) {
      __hip_atomic_store(&tc->arrive[k][0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      last = __hip_atomic_fetch_add(&tc->top[0], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == groups - 1;
    }
    if (last) {
      __hip_atomic_store(&tc->top[0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(&tc->gen[0], g + 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      const unsigned long long t0 = wall_clock64();
      while (__hip_atomic_load(&tc->gen[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == g) {
        if (ld_u32(&tc->abort[0])) {
          ok = 0u;
          break;
        }
        if (wall_clock64() - t0 > limit) {
          __hip_atomic_fetch_or(&tc->abort[0], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          atomicOr(&tot->err, (unsigned)kErrInternal);
          ok = 0u;
          break;
        }
        __builtin_amdgcn_s_sleep(2);
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");  // drop stale lines before the next step
    gen = g + 1u;
    sm.ok = ok;
  }
  __syncthreads();
  return sm.ok != 0u;
}

// Workgroup sums of three values; every lane gets them.
__device__ __forceinline__ void block_sum3(long long& x0, long long& x1, long long& x2, TailSmem& sm) {
  x0 = wave_incl_sum<long long>(x0);
  x1 = wave_incl_sum<long long>(x1);
  x2 = wave_incl_sum<long long>(x2);
  if (lane_id() == 63) {
    sm.red[0][wave_id()] = x0;
    sm.red[1][wave_id()] = x1;
    sm.red[2][wave_id()] = x2;
  }
  __syncthreads();
  if (threadIdx.x < 3) {
    long long s = 0;
#pragma unroll
    for (int i = 0; i < kTW; ++i) s += sm.red[threadIdx.x][i];
    sm.sum[threadIdx.x] = s;
  }
  __syncthreads();
  x0 = sm.sum[0];
  x1 = sm.sum[1];
  x2 = sm.sum[2];
  __syncthreads();
}

// Places the rows of the lanes with `es` (short, front of the segment) or `el`
// (long, back of the segment): one LDS atomic per wave and kind.
__device__ __forceinline__ void place_rows(bool es, bool el, int4 rec, int4* out, int base, int cap, TailSmem& sm) {
  const unsigned long long bs = __ballot(es), bl = __ballot(el);
  const unsigned long long lt = lanemask_lt();
  int ps = 0, pl = 0;
  if (lane_id() == 0) {
    if (bs) ps = atomicAdd(&sm.cnt_s, (int)__popcll(bs));
    if (bl) pl = atomicAdd(&sm.cnt_l, (int)__popcll(bl));
  }
  ps = __shfl(ps, 0, 64);
  pl = __shfl(pl, 0, 64);
  if (es) out[base + ps + (int)__popcll(bs & lt)] = rec;
  if (el) out[base + cap - 1 - (pl + (int)__popcll(bl & lt))] = rec;
}

__device__ __forceinline__ void graph_of(const Common& c, int g, int& base, unsigned long long& S) {
  if (c.graphs == 1) {
    base = 0;
    S = c.gseed[0];
  } else {
    base = c.gbase[g];
    S = c.gseed[g];
  }
}

// Row `i` of the short (long) rows of the current list.
__device__ __forceinline__ int4 short_row(const TailSmem& sm, int nseg, const int4* rows, int i) {
  int lo = 0, hi = nseg;  // largest b with pre_s[b] <= i
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (sm.pre_s[mid] <= i) lo = mid;
    else hi = mid;
  }
  return rows[sm.sbase[lo] + (i - sm.pre_s[lo])];
}
__device__ __forceinline__ int4 long_row(const TailSmem& sm, int nseg, const int4* rows, int j) {
  int lo = 0, hi = nseg;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (sm.pre_l[mid] <= j) lo = mid;
    else hi = mid;
  }
  return rows[sm.sbase[lo] + sm.scap[lo] - 1 - (j - sm.pre_l[lo])];
}

// Keeps the live entries of row r (unmatched vertex) in the next entry buffer
// and returns how many; best gets the largest key among them. One lane.
__device__ __forceinline__ int keep_row_lane(const Common& c, int4 r, int base, unsigned vloc, unsigned long long S,
                                             const int* col, const float* w, int* ncol, float* nw, Best& best) {
  const bool unw = w == nullptr;
  const int off = r.y, len = r.z;
  int kept = 0;
  for (int k0 = 0; k0 < len; k0 += 4) {
    int u[4];
    float x[4];
    bool ok[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      ok[q] = k0 + q < len;
      u[q] = ok[q] ? col[off + k0 + q] : 0;
      x[q] = (ok[q] && !unw) ? w[off + k0 + q] : 1.0f;
      ok[q] = ok[q] && u[q] >= 0 && (unsigned)(base + u[q]) < (unsigned)c.n;
    }
    unsigned char st[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) st[q] = ok[q] ? c.state[base + u[q]] : (unsigned char)1;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      if (st[q] == 0) {
        ncol[off + kept] = u[q];
        if (!unw) nw[off + kept] = x[q];
        ++kept;
        best_update(best, ord_weight_bits(__float_as_uint(x[q])), u[q], vloc, S);
      }
    }
  }
  return kept;
}

}  // namespace

// R_c (the live set the device phase counter names) in the piece layout of
// the phase kernels becomes the tail's first row list: one row per live
// vertex, its entries at the vertex's virtual position. Rows cut into several
// pieces are contiguous there, so for c >= 2 every run is copied to its
// virtual range first. R_1 needs no copy: its entries are the input rows.
__global__ __launch_bounds__(kTailBlock) void k_tail(TailArgs a) {
  __shared__ TailSmem sm;
  Common& c = a.c;
  Totals* tot = c.totals;
  TailCtl* tc = a.tc;
  const int tid = threadIdx.x, lane = lane_id(), wv = wave_id();
  const int b = blockIdx.x;
  if (tid == 0) sm.ok = tot->err == 0u ? 1u : 0u;
  __syncthreads();
  if (!sm.ok) return;  // every workgroup reads the same word: all leave
  const int c0 = tot->t;
  const int si = (c0 - 1) & 1;  // R_c's buffer set
  const Ctl ctl = *a.ctl[si];
  const int nb = (int)gridDim.x;
  const unsigned long long limit = a.spin_ticks;
  unsigned bgen = 0;
  const bool unw = a.ew[0] == nullptr;
  const bool csr = c0 == 1 && a.csr_rp != nullptr;
  int4* TA = a.rows[c0 & 1];
  int4* TB = a.rows[(c0 + 1) & 1];
  // ---- conversion: workgroup b takes pieces [P b / nb, P (b + 1) / nb), its
  // segment of the first row list starts at P b / nb
  const long long P = ctl.pieces;
  const int k0 = (int)(P * b / nb), k1 = (int)(P * (b + 1) / nb);
  if (tid == 0) {
    sm.cnt_s = 0;
    sm.cnt_l = 0;
  }
  if (!csr) {
    for (int i = tid; i <= ctl.nruns && i < kRunCache; i += kTailBlock) sm.rp[i] = a.rpre[si][i];
  }
  __syncthreads();
  const int* cur_col;
  const float* cur_w;
  int ni;  // the entry buffer phase c writes
  if (c0 == 1) {
    cur_col = a.in_col;
    cur_w = unw ? nullptr : a.in_w;
    ni = 1;
  } else {
    cur_col = a.ecol[(c0 + 1) & 1];
    cur_w = unw ? nullptr : a.ew[(c0 + 1) & 1];
    ni = c0 & 1;
  }
  if (csr) {  // piece k is vertex k (empty rows are pieces of length 0)
    for (int v0 = k0 + (tid & ~63); v0 < k1; v0 += kTailBlock) {
      const int v = v0 + lane;
      int4 r = make_int4(0, 0, 0, 0);
      bool es = false, el = false;
      if (v < k1) {
        const long long e0 = a.csr_rp[v], e1 = a.csr_rp[v + 1];
        const int len = (int)(e1 - e0);
        r = make_int4(v, (int)e0, len, 0);
        es = len > 0 && len <= kTailShort;
        el = len > kTailShort;
      }
      place_rows(es, el, r, TA, k0, k1 - k0, sm);
    }
  } else {
    const Run* runs = a.runs[si];
    const long long* epre = a.epre[si];
    const int4* pin = a.rows[si];
    if (c0 >= 2) {  // runs b, b + nb, ... to their virtual ranges
      const int* sc = a.ecol[c0 & 1];
      const float* sw = unw ? nullptr : a.ew[c0 & 1];
      int* dc = a.ecol[(c0 + 1) & 1];
      float* dw = unw ? nullptr : a.ew[(c0 + 1) & 1];
      for (int rn = b; rn < ctl.nruns; rn += nb) {
        const Run run = runs[rn];
        const long long vb = epre[rn];
        for (int e = tid; e < run.ent_count; e += kTailBlock) {
          dc[vb + e] = sc[run.phys_begin + e];
          if (!unw) dw[vb + e] = sw[run.phys_begin + e];
        }
      }
    }
    for (int q0 = k0 + (tid & ~63); q0 < k1; q0 += kTailBlock) {
      const int k = q0 + lane;
      int4 r = make_int4(0, 0, 0, 0);
      bool es = false, el = false;
      if (k < k1) {
        int lo = 0, hi = ctl.nruns;  // run of piece k: largest lo with rp[lo] <= k
        while (hi - lo > 1) {
          const int mid = (lo + hi) >> 1;
          if (sm.rp[mid] <= k) lo = mid;
          else hi = mid;
        }
        const Run run = runs[lo];
        const int4 rec = pin[run.row_begin + (k - sm.rp[lo])];
        if ((rec.w & kHeadBit) && rec.z > 0) {
          long long total = rec.z;
          // later pieces of the same vertex (its row was cut at a workgroup boundary)
          int j = k - sm.rp[lo] + 1, rr = lo;
          for (;;) {
            while (rr < ctl.nruns && j >= runs[rr].row_count) {
              ++rr;
              j = 0;
            }
            if (rr >= ctl.nruns) break;
            const int4 nx = pin[runs[rr].row_begin + j];
            if (nx.x != rec.x) break;
            total += nx.z;
            ++j;
          }
          r = make_int4(rec.x, (int)(epre[lo] + (rec.y - run.phys_begin)), (int)total, rec.w & kGraphMask);
          es = total <= kTailShort;
          el = !es;
        }
      }
      place_rows(es, el, r, TA, k0, k1 - k0, sm);
    }
  }
  __syncthreads();
  if (tid == 0) {
    TailSeg sg;
    sg.base = k0;
    sg.cap = k1 - k0;
    sg.ns = sm.cnt_s;
    sg.nl = sm.cnt_l;
    sg.kept = 0;
    sg.md = 0;
    sg.mv = 0;
    tc->seg[(c0 - 1) & 1][b] = sg;
  }
  if (!grid_sync(tc, nb, bgen, limit, tot, sm)) return;
  // ---- phases c, c + 1, ...
  const int4* rows = TA;
  int4* out = TB;
  int nseg = nb;  // segments of the current list
  bool solo = false;
  int t = c0;
  long long L = ctl.L, prevL = 0, prevV = 0;
  int last_nonempty = 0;
  unsigned long long matched_total = 0;
  if (b == 0 && tid == 0) {
    last_nonempty = tot->last_nonempty;
    matched_total = tot->matched;
  }
  for (;;) {
    // segment table of the current list (written by phase t - 1, or the conversion)
    {
      const TailSeg* tab = tc->seg[(t - 1) & 1];
      TailSeg sg;
      sg.ns = sg.nl = 0;
      sg.base = sg.cap = 0;
      sg.kept = sg.md = 0;
      sg.mv = 0;
      if (tid < nseg) sg = tab[tid];
      if (tid < nseg) {
        sm.sbase[tid] = sg.base;
        sm.scap[tid] = sg.cap;
      }
      // exclusive prefix of ns and nl over the segments (nseg <= 128: waves 0 and 1)
      const int is = (int)wave_incl_sum_u32((unsigned)sg.ns), il = (int)wave_incl_sum_u32((unsigned)sg.nl);
      if (lane == 63 && wv < 2) {
        sm.red[0][wv] = is;
        sm.red[1][wv] = il;
      }
      __syncthreads();
      if (wv < 2 && tid <= kTailMaxBlocks) {
        const int cs = wv == 1 ? (int)sm.red[0][0] : 0, cl = wv == 1 ? (int)sm.red[1][0] : 0;
        if (tid < nseg) {
          sm.pre_s[tid] = cs + is - sg.ns;
          sm.pre_l[tid] = cl + il - sg.nl;
        }
        if (tid == nseg - 1) {
          sm.pre_s[nseg] = cs + is;
          sm.pre_l[nseg] = cl + il;
        }
      }
      __syncthreads();
      long long kept = sg.kept, md = sg.md, mv = (long long)sg.mv;
      block_sum3(kept, md, mv, sm);
      if (t > c0) {
        L = kept;
        if (b == 0 && tid == 0) {  // the record of phase t - 1
          if (t - 1 >= 1 && t - 1 <= a.log_cap) {
            LogRec rec;
            rec.live_entries = prevL;
            rec.live_rows = prevV;
            rec.matched_edges = mv / 2;
            rec.matched_entries = md;
            a.log[t - 2] = rec;
          }
          last_nonempty = t - 1;
          matched_total += (unsigned long long)mv;
        }
        if (mv == 0) {  // nothing matched although edges were live: the input is not symmetric
          if (b == 0 && tid == 0) atomicOr(&tot->err, (unsigned)kErrStall);
          break;
        }
      }
    }
    const int S = sm.pre_s[nseg], Lg = sm.pre_l[nseg];
    const long long V = (long long)S + Lg;
    if (L == 0 || V == 0) break;
    if (!solo && L <= kTailSolo) {
      solo = true;
      if (b != 0) return;  // workgroup 0 finishes alone
    }
    const int nbe = solo ? 1 : nb;
    // this workgroup's short rows [lo, hi); long row j goes to wave j % (nbe * kTW)
    const int lo = (int)((long long)S * b / nbe), hi = (int)((long long)S * (b + 1) / nbe);
    const int nwaves = nbe * kTW, gw = b * kTW + wv;
    const int q = Lg / nwaves, rmd = Lg % nwaves;
    const int longs_mine = kTW * q + min(max(rmd - b * kTW, 0), kTW);
    const int longs_before = b * kTW * q + min(rmd, b * kTW);
    // ---- mutual check (rows striped over the workgroup's lanes)
    long long mv_b = 0;
    {
      const int nmine = (hi - lo) + longs_mine;
      for (int x = tid; x < nmine; x += kTailBlock) {
        int4 r;
        if (x < hi - lo) {
          r = short_row(sm, nseg, rows, lo + x);
        } else {
          // the y-th long row of this workgroup: wave w's m-th (the first
          // longs_mine - kTW q waves of the workgroup have q + 1, the rest q)
          const int y = x - (hi - lo);
          const int w = y % kTW, m = y / kTW;
          const int j = (b * kTW + w) + m * nwaves;
          if (j >= Lg) continue;
          r = long_row(sm, nseg, rows, j);
        }
        const int v = r.x;
        const int u = c.C[v];
        if (c.gphase) atomicMax(&c.gphase[r.w], t);
        if ((unsigned)u < (unsigned)c.n && c.C[u] == v) {
          int base;
          unsigned long long Sd;
          graph_of(c, r.w, base, Sd);
          c.mate[v] = u - base;
          c.state[v] = 1;
          ++mv_b;
        }
      }
    }
    {
      long long z0 = 0, z1 = 0;
      block_sum3(mv_b, z0, z1, sm);
    }
    if (solo) {
      __syncthreads();
    } else if (!grid_sync(tc, nb, bgen, limit, tot, sm)) {
      return;
    }
    // ---- compaction fused with the next candidates
    const int obase = lo + longs_before, ocap = (hi - lo) + longs_mine;
    if (tid == 0) {
      sm.cnt_s = 0;
      sm.cnt_l = 0;
    }
    __syncthreads();
    long long kept_b = 0, md_b = 0;
    int* ncol = a.ecol[ni];
    float* nw = unw ? nullptr : a.ew[ni];
    for (int i0 = lo + (tid & ~63); i0 < hi; i0 += kTailBlock) {
      const int i = i0 + lane;
      int4 r = make_int4(0, 0, 0, 0);
      bool es = false, el = false;
      if (i < hi) {
        r = short_row(sm, nseg, rows, i);
        if (c.state[r.x]) {
          md_b += r.z;
        } else {
          int base;
          unsigned long long Sd;
          graph_of(c, r.w, base, Sd);
          Sd = cand_seed(Sd, c.renew, t + 1);  // the candidates of phase t + 1
          const unsigned vloc = (unsigned)(r.x - base);
          Best best = best_ident();
          const int kept = keep_row_lane(c, r, base, vloc, Sd, cur_col, cur_w, ncol, nw, best);
          if (kept > 0) {
            c.C[r.x] = base + best.u;
            kept_b += kept;
            r.z = kept;
            es = kept <= kTailShort;
            el = !es;
          }
        }
      }
      place_rows(es, el, r, out, obase, ocap, sm);
    }
    for (int j = gw; j < Lg; j += nwaves) {  // long rows, a wave each
      const int4 r = long_row(sm, nseg, rows, j);
      const int v = r.x, off = r.y, len = r.z;
      if (c.state[v]) {
        if (lane == 0) md_b += len;
        continue;
      }
      int base;
      unsigned long long Sd;
      graph_of(c, r.w, base, Sd);
      Sd = cand_seed(Sd, c.renew, t + 1);  // the candidates of phase t + 1
      const unsigned vloc = (unsigned)(v - base);
      Best best = best_ident();
      int kept = 0;
      const unsigned long long lt = lanemask_lt();
      for (int e0 = 0; e0 < len; e0 += 64) {
        const int e = e0 + lane;
        bool ok = e < len;
        const int u = ok ? cur_col[off + e] : 0;
        const float x = (ok && !unw) ? cur_w[off + e] : 1.0f;
        ok = ok && u >= 0 && (unsigned)(base + u) < (unsigned)c.n;
        const bool keep = ok && c.state[base + u] == 0;
        const unsigned long long bal = __ballot(keep);
        if (keep) {
          const int at = off + kept + (int)__popcll(bal & lt);
          ncol[at] = u;
          if (!unw) nw[at] = x;
          best_update(best, ord_weight_bits(__float_as_uint(x)), u, vloc, Sd);
        }
        kept += (int)__popcll(bal);
      }
      const Key kb = wave_max_key(best_key(best, vloc, Sd));
      int4 rr = r;
      rr.z = kept;
      if (lane == 0 && kept > 0) {
        c.C[v] = base + kb.u;
        kept_b += kept;
      }
      const bool live = kept > 0 && lane == 0;
      place_rows(live && kept <= kTailShort, live && kept > kTailShort, rr, out, obase, ocap, sm);
    }
    {
      long long z = 0;
      block_sum3(kept_b, md_b, z, sm);
    }
    if (tid == 0) {
      TailSeg sg;
      sg.base = obase;
      sg.cap = ocap;
      sg.ns = sm.cnt_s;
      sg.nl = sm.cnt_l;
      sg.kept = kept_b;
      sg.md = md_b;
      sg.mv = (unsigned long long)mv_b;
      tc->seg[t & 1][b] = sg;
    }
    if (solo) {
      __syncthreads();
    } else if (!grid_sync(tc, nb, bgen, limit, tot, sm)) {
      return;
    }
    // next live set
    prevL = L;
    prevV = V;
    nseg = nbe;
    const int4* tmp = rows;
    rows = out;
    out = const_cast<int4*>(tmp);
    cur_col = ncol;
    cur_w = nw;
    ni ^= 1;
    ++t;
  }
  if (b == 0 && tid == 0) {
    tot->last_nonempty = last_nonempty;
    tot->matched = matched_total;
    tot->t = t;
    PhaseMirror m;
    m.L = L;
    m.matched = matched_total;
    m.pieces = 0;
    m.t = t;
    m.gen = a.gen;
    m.err = ld_u32(&tot->err);
    m.last_nonempty = last_nonempty;
    m.pad = c0;  // the live set the tail started from
    m.tag = 0ull;
    PhaseMirror* slot = a.final_rec;
    *(volatile unsigned long long*)&slot->tag = 0ull;
    __threadfence_system();
    *slot = m;
    __threadfence_system();
    *(volatile unsigned long long*)&slot->tag = mirror_tag(a.gen, t);
  }
}

hipError_t launch_tail(const TailArgs& a, int grid, hipStream_t s, hipEvent_t* ev) {
  if (grid < 1 || grid > kTailMaxBlocks) return hipErrorInvalidValue;
  if (ev)
    hipExtLaunchKernelGGL(k_tail, dim3(grid), dim3(kTailBlock), 0, s, ev[0], ev[1], 0, a);
  else
    hipLaunchKernelGGL(k_tail, dim3(grid), dim3(kTailBlock), 0, s, a);
  return hipGetLastError();
}

int tail_blocks_per_cu() {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_tail, kTailBlock, 0) != hipSuccess || nb < 1) nb = 1;
  return nb;
}

}  // namespace lm
