// Phase kernels of local-max matching for gfx950 (wave64).
//
// One phase (paper, Section 2, "Sequential Model", and the CREW phase steps of
// Section 2.1, re-planned for a GPU without atomics on the hot path):
//   argmax   every live vertex finds its live incident edge of largest key
//            (Lemma 3 form: a segmented max over the entry stream);
//   mutual   v is matched iff its candidate u has v as candidate (CREW step
//            3); the deletion flag of CREW step 4 lives on the vertex;
//   compact  a live entry survives iff both endpoints are unmatched; the
//            survivors are written contiguously (CREW steps 5-6) and the next
//            phase's argmax is computed in the same pass.
// The live-set layout (pieces grouped into runs) is described in
// lm_internal.h.
#include <hip/hip_ext.h>

#include <algorithm>
#include <climits>

#include "lm_device.h"
#include "lm_internal.h"
#include "lm_key.h"

namespace lm {

// Reads the error word once per workgroup so that every lane takes the same
// branch. A guarded launch (device-controlled solve) also stops once the tail
// kernel has taken the live set over.
__device__ __forceinline__ bool block_failed(const Common& c, unsigned* s) {
  if (threadIdx.x == 0) *s = c.totals->err | ((c.guard && c.totals->tail_from) ? 0x80000000u : 0u);
  __syncthreads();
  const bool f = *s != 0;
  __syncthreads();
  return f;
}

// ---------------------------------------------------------------- small

__global__ void k_zero(Ctl* ctl, int nctl, Totals* totals, TailCtl* tc) {
  int* p = reinterpret_cast<int*>(ctl);
  const int words = nctl * (int)(sizeof(Ctl) / 4);
  for (int i = threadIdx.x; i < words; i += blockDim.x) p[i] = 0;
  if (tc) {
    int* q = reinterpret_cast<int*>(tc);
    for (int i = threadIdx.x; i < (int)(sizeof(TailCtl) / 4); i += blockDim.x) q[i] = 0;
  }
  if (threadIdx.x == 0) {
    totals->err = 0;
    totals->last_nonempty = 0;
    totals->matched = 0;
    totals->t = 1;
    totals->tail_from = 0;
    totals->fp[0] = 0;
    totals->fp[1] = 0;
    totals->far = 0;
    totals->samp = 0;
  }
}

__global__ void k_fill_i32(int* p, long long n, int value) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    p[i] = value;
}

__global__ void k_add_i64(long long* p, long long n, long long delta) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    p[i] += delta;
}

// Fingerprint term of the entry (x, y) with weight bits wb of graph g: two
// rounds of the SplitMix64 output function. -0 and +0 give the same term.
__device__ __forceinline__ unsigned long long fp_term(long long g, long long x, long long y, unsigned wb) {
  if (wb == 0x80000000u) wb = 0u;
  const unsigned long long h = mix64((((unsigned long long)(unsigned)x << 32) | (unsigned)y) + 0x632BE59BD9B4E019ull);
  return mix64(h ^ (((unsigned long long)wb << 32) | (unsigned long long)(unsigned)g));
}

// Optional input check: ids in range, no self-loops, finite weights, and the
// symmetry of the entries with equal weights both ways: the sum (mod 2^64) of
// a hash of every entry (v, u, w) must equal the sum over the mirrors (u, v,
// w); the two multisets then agree except with probability about 2^-64.
// Duplicate entries are found by check_row_duplicates.
__global__ __launch_bounds__(kBlock) void k_check(CheckArgs a) {
  constexpr long long kLongRow = 64;  // rows longer than this are walked by the whole wave
  unsigned err = 0;
  unsigned long long f0 = 0, f1 = 0;
  auto entry = [&](long long k, long long vl, long long lim, long long gi) {
    const int u = a.col[k];
    if (u < 0 || u >= lim) err |= kErrColRange;
    if (u == vl) err |= kErrSelfLoop;
    unsigned wb = 0x3f800000u;
    if (a.w) {
      const float x = a.w[k];
      if (!(x == x) || x == __int_as_float(0x7f800000) || x == __int_as_float(0xff800000)) err |= kErrWeight;
      wb = __float_as_uint(x);
    }
    f0 += fp_term(gi, vl, u, wb);
    f1 += fp_term(gi, u, vl, wb);
  };
  const long long stride = (long long)gridDim.x * kBlock;
  const long long vend = ((a.n + stride - 1) / stride) * stride;  // every lane of a wave runs the same rounds
  for (long long v = (long long)blockIdx.x * kBlock + threadIdx.x; v < vend; v += stride) {
    long long base = 0, lim = a.n, gi = 0, b = 0, e = 0;
    if (v < a.n) {
      if (a.graphs > 1) {
        int lo = 0, hi = a.graphs - 1;
        while (lo < hi) {
          int mid = (lo + hi + 1) >> 1;
          if (a.vtx_off[mid] <= v) lo = mid;
          else hi = mid - 1;
        }
        base = a.vtx_off[lo];
        lim = a.vtx_off[lo + 1] - base;
        gi = lo;
      }
      b = a.row_ptr[v];
      e = a.row_ptr[v + 1];
      if (b < 0 || e > a.nnz || e < b) {
        err |= kErrRowPtr;
        b = e = 0;
      }
    }
    const bool lng = e - b > kLongRow;
    if (!lng)
      for (long long k = b; k < e; ++k) entry(k, v - base, lim, gi);
    // long rows: the wave walks each one together
    unsigned long long m = __ballot(lng);
    while (m) {
      const int l = __ffsll((long long)m) - 1;
      m &= m - 1;
      const long long vb = __shfl(b, l), ve = __shfl(e, l), vl = __shfl(v - base, l), lm = __shfl(lim, l),
                      g = __shfl(gi, l);
      for (long long k = vb + lane_id(); k < ve; k += 64) entry(k, vl, lm, g);
    }
  }
  f0 = wave_incl_sum_u64(f0);
  f1 = wave_incl_sum_u64(f1);
  if (lane_id() == 63) {
    atomicAdd(&a.totals->fp[0], f0);
    atomicAdd(&a.totals->fp[1], f1);
  }
  if (err) atomicOr(&a.totals->err, err);
}

__global__ void k_check_fp(Totals* t) {
  if (threadIdx.x == 0 && t->fp[0] != t->fp[1]) atomicOr(&t->err, (unsigned)kErrAsym);
}

// ---------------------------------------------------------------- init

// Live set R_1 straight from the input CSR: workgroup b covers vertices
// [vcount b / B, vcount (b+1) / B) of the group; every vertex with at least one
// entry becomes one head piece pointing at its input row, and the workgroup's
// pieces form one run (their rows are back to back in the entry buffer). Also
// clears mate and state and checks the offsets. Vertices are striped over the
// lanes (vertex c0 + jj * kBlock + lane) so that every load and store of a
// round is coalesced; wave ballots rank the non-empty rows. With a.csr no
// piece is written: the run covers every vertex of the workgroup, C is
// cleared, and the count of non-empty rows goes to bstat[b].
__global__ __launch_bounds__(kBlock) void k_init(InitArgs a) {
  __shared__ unsigned s_cnt[kItems * kWaves];
  const int tid = threadIdx.x;
  const int lane = lane_id(), wv = wave_id();
  const int b = blockIdx.x;
  const long long N = a.vcount;
  const long long vb = N * b / a.nblocks, ve = N * (b + 1) / a.nblocks;
  const long long eend = a.ebase + a.nnz;
  const unsigned long long lt = lanemask_lt();
  unsigned err = 0;
  int g = 0;  // graph of this lane's current vertex (group index)
  if (a.graphs > 1 && vb + tid < ve) {
    int lo = 0, hi = a.graphs - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (a.vtx_off[mid] <= vb + tid) lo = mid;
      else hi = mid - 1;
    }
    g = lo;
  }
  unsigned cursor = 0;
  for (long long c0 = vb; c0 < ve; c0 += kCap) {
    long long r0[kItems], r1[kItems];
#pragma unroll
    for (int jj = 0; jj < kItems; ++jj) {
      const long long v = c0 + (long long)jj * kBlock + tid;
      r0[jj] = v < ve ? a.row_ptr[v] : 0;
      r1[jj] = v < ve ? a.row_ptr[v + 1] : 0;
    }
    unsigned rank[kItems];
    unsigned okm = 0;
#pragma unroll
    for (int jj = 0; jj < kItems; ++jj) {
      const long long v = c0 + (long long)jj * kBlock + tid;
      const long long d = r1[jj] - r0[jj];
      bool ok = false;
      if (v < ve) {
        if (d < 0 || r0[jj] < a.ebase || r1[jj] > eend) err |= kErrRowPtr;
        if (d > 0x7fff0000LL) err |= kErrDegree;
        ok = d > 0 && d <= 0x7fff0000LL && r0[jj] >= a.ebase && r1[jj] <= eend;
      }
      const unsigned long long bal = __ballot(ok);
      rank[jj] = (unsigned)__popcll(bal & lt);
      if (jj == 0 && c0 == vb && a.col && a.c.mbits && wv == 0 && (b & 15) == 0) {
        // locality sample: the first entry of the non-empty rows of the first
        // wave of every 16th workgroup (two same-address atomics per wave)
        const long long vgs = a.vfirst + v;
        const int u = ok ? a.col[r0[0]] : 0;
        const long long dist = (long long)u - vgs;
        const unsigned long long farb = __ballot(ok && (dist >= (long long)kFarIds || dist <= -(long long)kFarIds));
        if (lane == 0 && bal) {
          atomicAdd(&a.c.totals->far, (unsigned)__popcll(farb));
          atomicAdd(&a.c.totals->samp, (unsigned)__popcll(bal));
        }
      }
      if (lane == 0) s_cnt[jj * kWaves + wv] = (unsigned)__popcll(bal);
      okm |= (ok ? 1u : 0u) << jj;
    }
    __syncthreads();
    const unsigned c = lane < kItems * kWaves ? s_cnt[lane] : 0u;
    const unsigned incl = wave_incl_sum_u32(c);
    const unsigned tot = (unsigned)__builtin_amdgcn_readlane((int)incl, 63);
    const unsigned excl = incl - c;
#pragma unroll
    for (int jj = 0; jj < kItems; ++jj) {
      const long long v = c0 + (long long)jj * kBlock + tid;
      const unsigned at = cursor + (unsigned)__builtin_amdgcn_readlane((int)excl, jj * kWaves + wv) + rank[jj];
      if (v < ve) {
        if (a.graphs > 1)
          while (a.vtx_off[g + 1] <= v) ++g;
        const long long vg = a.vfirst + v;
        a.c.mate[vg] = -1;
        a.c.state[vg] = 0;
        if (a.c.mbits && (vg & 31) == 0) a.c.mbits[vg >> 5] = 0u;
        if (a.csr) {
          a.c.C[vg] = -1;  // the mutual check reads C of every vertex, empty rows too
        } else if ((okm >> jj) & 1u) {
          const int slot = a.slot_of ? a.slot_of[g] : g;
          a.rows_out[a.rows_base + vb + at] =
              make_int4((int)vg, (int)r0[jj], (int)(r1[jj] - r0[jj]), (slot & kGraphMask) | kHeadBit);
        }
      }
    }
    cursor += tot;
    __syncthreads();  // s_cnt is rewritten by the next round
  }
  if (tid == 0) {
    Run r;
    r.row_begin = a.rows_base + (int)vb;
    r.row_count = a.csr ? (int)(ve - vb) : (int)cursor;  // from the CSR: every vertex is a piece
    if (a.csr) {
      BlockStat st;
      st.loaded = 0;
      st.matched_len = 0;
      st.pieces_out = (int)cursor;  // non-empty rows: the live rows of R_1
      st.pad = 0;
      a.bstat[b] = st;
    }
    const long long pb = vb < N ? a.row_ptr[vb] : eend;
    const long long pe = a.row_ptr[ve];
    r.phys_begin = (int)pb;
    r.ent_count = (int)(pe - pb);
    if (vb == 0 && pb != a.ebase) err |= kErrRowPtr;
    if (ve == N && pe != eend) err |= kErrRowPtr;
    if (pe < pb) err |= kErrRowPtr;
    a.runs_out[a.runs_base + b] = r;
  }
  if (err) atomicOr(&a.c.totals->err, err);
}

// ---------------------------------------------------------------- plan

// One workgroup of kPlanThreads lanes. Fixes the rows that the last
// compaction (or first argmax) cut at workgroup boundaries, scans the run
// table of the live set it produced, sizes the next launches and writes the
// phase log.
__global__ __launch_bounds__(kPlanThreads) void k_plan(PlanArgs a) {
  __shared__ unsigned s_err;
  __shared__ int s_extra;
  __shared__ long long s_e[kPlanThreads / 64];
  __shared__ int s_r[kPlanThreads / 64];
  __shared__ int s_h[kPlanThreads / 64];
  __shared__ long long s_red[4];
  const int tid = threadIdx.x;
  const Ctl prev = a.ctl_prev ? *a.ctl_prev : Ctl{0, 0, 0, 0, 0, 0, 0};
  // ranges of the launch being fixed: the first argmax may split R_1 its own way
  const int Pfix = (a.first && prev.Pf > 0) ? prev.Pf : prev.P;
  // The run table, the per-run live rows, the per-workgroup matched counts and
  // skipped entries, and (lane 0) the running totals are loaded here, before
  // the first barrier, so that the round trips overlap (the cut-row parts
  // follow in groups). None of it is written by this kernel before it is used.
  constexpr int kPer = kMaxBlocks / kPlanThreads;  // runs per lane in the scan
  const int nr = (a.mode & kPlanPrefix) ? (a.nruns_new >= 0 ? a.nruns_new : prev.P) : 0;
  long long le[kPer];
  int lr[kPer];
  int sh = 0;
#pragma unroll
  for (int i = 0; i < kPer; ++i) {
    const int r = tid * kPer + i;
    le[i] = 0;
    lr[i] = 0;
    if (r < nr) {
      const Run run = a.runs_new[r];
      le[i] = run.ent_count;
      lr[i] = run.row_count;
      if (a.heads_of_runs) sh += a.heads_of_runs[r].pieces_out;
    }
  }
  long long mc = 0, ml = 0;
  if (a.mode & kPlanLog) {  // (Pm, P <= kMaxBlocks: every load is issued before any is used)
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
      const int b = tid + i * kPlanThreads;
      if (b < prev.Pm) mc += a.mcount[b];
      if (b < prev.P) ml += a.bstat[b].matched_len;
    }
  }
  Totals tot;  // lane 0: the totals as the kernels before left them
  if (tid == 0) {
    tot = *a.c.totals;
    s_err = tot.err | ((a.c.guard && tot.tail_from) ? 0x80000000u : 0u);
    s_extra = 0;
    s_red[0] = s_red[1] = s_red[2] = 0;
  }
  __syncthreads();
  if (s_err) return;
  if (a.mode & kPlanFix) {
    // kFixG of the lane's ranges at a time: their parts (the last one of range
    // b and the first one of range b + 1, where a cut row continues) are all
    // loaded before any is used, so a chain of one step costs one round trip
    // per group; longer chains (rows over several ranges) load on.
    constexpr int kFixG = 4;
    Part none;
    none.v = -1;
    for (int b0 = tid; b0 < Pfix; b0 += kFixG * kPlanThreads) {
      Part plg[kFixG], pfg[kFixG];
#pragma unroll
      for (int g = 0; g < kFixG; ++g) {
        const int b = b0 + g * kPlanThreads;
        plg[g] = none;
        pfg[g] = none;
        if (b < Pfix) {
          plg[g] = a.parts[2 * b + 1];
          if (b + 1 < Pfix) pfg[g] = a.parts[2 * (b + 1)];
        }
      }
#pragma unroll
      for (int g = 0; g < kFixG; ++g) {
        const int b = b0 + g * kPlanThreads;
        const Part pl = plg[g];
        if (pl.v < 0) continue;  // block b does not own a cut row
        Key best;
        best.w = pl.w;
        best.hhi = pl.hhi;
        best.hlo = pl.hlo;
        best.u = pl.u;
        int head_row = pl.kept > 0 ? pl.out_row : -1;
        int pieces = pl.out_row >= 0 ? 1 : 0;
        Part pf = pfg[g];
        for (int b2 = b + 1; b2 < Pfix; ++b2) {
          if (b2 > b + 1) pf = a.parts[2 * b2];
          if (pf.v != pl.v) break;  // defensive: the chain always continues here
          Key k;
          k.w = pf.w;
          k.hhi = pf.hhi;
          k.hlo = pf.hlo;
          k.u = pf.u;
          best = key_max(best, k);
          if (pf.out_row >= 0) ++pieces;
          if (head_row < 0 && pf.kept > 0) head_row = pf.out_row;
          if (!(pf.flags & kPartSingle)) break;
        }
        if (best.u >= 0) a.c.C[pl.v] = best.u;
        if (!a.first) {
          if (head_row >= 0) atomicOr(&a.rows_out[head_row].w, kHeadBit);  // (no value returned: no wait)
          if (pieces > 1) atomicAdd(&s_extra, pieces - 1);
        }
      }
    }
  }
  __syncthreads();
  Ctl cn{0, 0, 0, 0, 0, 0, 0};  // lane 0: the live set just planned
  if (a.mode & kPlanPrefix) {
    // blocked scan over nr <= kMaxBlocks runs, kPer per lane
    long long se = 0;
    int sr = 0;
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
      se += le[i];
      sr += lr[i];
    }
    long long ie = wave_incl_sum<long long>(se);
    int ir = wave_incl_sum<int>(sr);
    const int ih = wave_incl_sum<int>(sh);
    if (lane_id() == 63) {
      s_e[tid >> 6] = ie;
      s_r[tid >> 6] = ir;
      s_h[tid >> 6] = ih;
    }
    __syncthreads();
    long long pe = 0, te = 0;
    int pr = 0, tr = 0, th = 0;
    for (int wv = 0; wv < kPlanThreads / 64; ++wv) {
      if (wv < (tid >> 6)) {
        pe += s_e[wv];
        pr += s_r[wv];
      }
      te += s_e[wv];
      tr += s_r[wv];
      th += s_h[wv];
    }
    long long ce = pe + ie - se;
    int cr = pr + ir - sr;
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
      const int r = tid * kPer + i;
      if (r <= nr) {
        a.epre_new[r] = ce;
        a.rpre_new[r] = cr;
      }
      ce += le[i];
      cr += lr[i];
    }
    if (tid == 0) {
      a.epre_new[nr] = te;
      a.rpre_new[nr] = tr;
      Ctl c;
      c.L = te;
      c.nruns = nr;
      c.pieces = tr;
      // live rows: pieces less the extra pieces of cut rows; for R_1 read from
      // the CSR (empty rows are pieces) the non-empty rows k_init counted
      c.heads = a.heads_of_runs ? th : tr - s_extra;
      // enough workgroups that each one sees a few full batches at most:
      // short rows fill a batch's piece window before its entry budget
      long long P = (te + a.min_per_block - 1) / a.min_per_block;
      if (a.pieces_per_block > 0) P = std::max<long long>(P, ((long long)tr + a.pieces_per_block - 1) / a.pieces_per_block);
      c.P = (int)std::max<long long>(te > 0 ? 1 : 0, std::min<long long>(P, a.pcap));
      c.Pf = a.pcap_first > 0 ? (int)std::max<long long>(te > 0 ? 1 : 0, std::min<long long>(P, a.pcap_first)) : 0;
      long long Pm = ((long long)tr + kMutualRound - 1) / kMutualRound;
      c.Pm = (int)std::max<long long>(tr > 0 ? 1 : 0, std::min<long long>(Pm, a.pmcap));
      *a.ctl_new = c;
      cn = c;
    }
  }
  if (a.mode & kPlanLog) {
    mc = wave_incl_sum<long long>(mc);
    ml = wave_incl_sum<long long>(ml);
    if (lane_id() == 63) {
      atomicAdd((unsigned long long*)&s_red[0], (unsigned long long)mc);
      atomicAdd((unsigned long long*)&s_red[1], (unsigned long long)ml);
    }
    __syncthreads();
    if (tid == 0) {
      const int t = tot.t;
      if (t >= 1 && t <= a.log_cap) {
        LogRec r;
        r.live_entries = prev.L;
        r.live_rows = prev.heads;
        r.matched_edges = s_red[0] / 2;
        r.matched_entries = s_red[1];
        a.log[t - 1] = r;
      }
      if (prev.heads > 0) tot.last_nonempty = t;
      tot.matched += (unsigned long long)s_red[0];
      a.c.totals->last_nonempty = tot.last_nonempty;
      a.c.totals->matched = tot.matched;
    }
  }
  if (a.mirror && (a.mode & kPlanPrefix) && tid == 0) {
    PhaseMirror m;
    m.L = cn.L;
    m.matched = tot.matched;
    m.pieces = cn.pieces;
    m.t = tot.t + ((a.mode & kPlanTick) ? 1 : 0);  // the live set for the next phase
    m.gen = a.gen;
    m.err = tot.err;
    m.last_nonempty = tot.last_nonempty;
    m.pad = 0;
    m.tag = 0ull;
    PhaseMirror* slot = &a.mirror[m.t & (kMirrorSlots - 1)];
    *(volatile unsigned long long*)&slot->tag = 0ull;  // the slot is being rewritten
    __threadfence_system();
    *slot = m;
    __threadfence_system();  // the record reaches host memory before it is tagged
    *(volatile unsigned long long*)&slot->tag = mirror_tag(a.gen, m.t);
  }
  if ((a.mode & kPlanTick) && tid == 0) a.c.totals->t = tot.t + 1;
  // a device-controlled solve leaves a small enough live set to the tail kernel
  if (a.tail_at > 0 && (a.mode & kPlanPrefix) && tid == 0 && cn.L <= a.tail_at)
    a.c.totals->tail_from = tot.t + ((a.mode & kPlanTick) ? 1 : 0);
}

// ---------------------------------------------------------------- run lookup

// rpre[c0 .. c0 + kBlock] and the first rows of runs c0 .. c0 + kBlock - 1,
// copied to LDS so that lanes find the run of a piece by a binary search in
// LDS instead of walking the run table in global memory (late live sets have
// many short runs).
struct RunCache {
  int rp[kBlock + 1];
  int rb[kBlock];
  int c0;
};

// Every lane of the workgroup; the caller synchronises before the first lookup.
__device__ __forceinline__ void run_cache_fill(const LiveSet& in, int nruns, int c0, RunCache& rc) {
  const int i = threadIdx.x;
  const int r = c0 + i;
  rc.rp[i] = r <= nruns ? in.rpre[r] : INT_MAX;
  rc.rb[i] = r < nruns ? in.runs[r].row_begin : 0;
  if (i == 0) {
    rc.rp[kBlock] = c0 + kBlock <= nruns ? in.rpre[c0 + kBlock] : INT_MAX;
    rc.c0 = c0;
  }
}

// Run r and row record of piece k when the cached runs hold it.
__device__ __forceinline__ bool run_cache_find(const RunCache& rc, long long k, int& r, int& row) {
  if (k < rc.rp[0] || k >= rc.rp[kBlock]) return false;
  int lo = 0;  // largest lo with rp[lo] <= k; then rp[lo + 1] > k, so run lo holds k
#pragma unroll
  for (int step = kBlock / 2; step > 0; step >>= 1)
    if (rc.rp[lo + step] <= k) lo += step;
  r = rc.c0 + lo;
  row = rc.rb[lo] + (int)(k - rc.rp[lo]);
  return true;
}

// ---------------------------------------------------------------- mutual

__global__ __launch_bounds__(kBlock) void k_mutual(MutualArgs a) {
  __shared__ unsigned s_err;
  __shared__ int s_lb[1];
  __shared__ unsigned s32[kWaves];
  __shared__ RunCache rc;
  if (block_failed(a.c, &s_err)) return;
  const bool use_bits = a.c.mbits != nullptr && bits_on(a.c.totals);
  const Ctl ctl = *a.in.ctl;
  const int t = a.c.totals->t;
  // R_1 read from the CSR: piece k is vertex k, every vertex is its own head,
  // and the matched flag lives in state only (C is -1 for empty rows)
  const bool csr = a.in.csr_rp != nullptr;
  for (int bb = blockIdx.x; bb < ctl.Pm; bb += gridDim.x) {
    const long long V = ctl.pieces;
    const long long p0 = V * bb / ctl.Pm, p1 = V * (bb + 1) / ctl.Pm;
    unsigned cnt = 0;
    if (p0 < p1) {
      // run containing piece p0: first r with rpre[r+1] > p0
      const int r0 = csr ? 0
                         : (int)block_lower_bound(
                               0, ctl.nruns, [&](long long r) { return (long long)a.in.rpre[r + 1] > p0; }, s_lb);
      if (!csr) run_cache_fill(a.in, ctl.nruns, r0, rc);
      __syncthreads();
      int r = r0;
      // kM pieces per lane per round; every load of a round is issued
      // unconditionally (clamped indices) so that the dependent chain piece ->
      // C[v] -> C[C[v]] is paid once per round, not once per piece
      constexpr int kM = kMutualRound / kBlock;
      for (long long base = p0; base < p1; base += (long long)kBlock * kM) {
        int row[kM];
#pragma unroll
        for (int i = 0; i < kM; ++i) {
          const long long pi = base + (long long)i * kBlock + threadIdx.x;
          row[i] = -1;
          if (csr) {
            row[i] = pi < p1 ? (int)pi : -1;
          } else if (pi < p1 && !run_cache_find(rc, pi, r, row[i])) {
            r = max(r, r0 + kBlock);  // past the cached runs: rpre[r0 + kBlock] <= pi
            while (r + 1 < ctl.nruns && (long long)a.in.rpre[r + 1] <= pi) ++r;
            row[i] = a.in.runs[r].row_begin + (int)(pi - a.in.rpre[r]);
          }
        }
        int4 rec[kM];
#pragma unroll
        for (int i = 0; i < kM; ++i)
          rec[i] = csr ? make_int4(row[i] >= 0 ? row[i] : 0, 0, 0, kHeadBit) : a.in.rows[row[i] >= 0 ? row[i] : 0];
        bool head[kM];
        int cv[kM];
#pragma unroll
        for (int i = 0; i < kM; ++i) {
          head[i] = row[i] >= 0 && (rec[i].w & kHeadBit) != 0;
          cv[i] = a.c.C[head[i] ? rec[i].x : 0];
        }
        int cu[kM];
        bool ok[kM];
#pragma unroll
        for (int i = 0; i < kM; ++i) {
          ok[i] = head[i] && !a.census && (unsigned)cv[i] < (unsigned)a.c.n;
          cu[i] = a.c.C[ok[i] ? cv[i] : 0];
        }
#pragma unroll
        for (int i = 0; i < kM; ++i) {
          if (ok[i] && cu[i] == rec[i].x) {
            const int v = rec[i].x;
            const int g = rec[i].w & kGraphMask;
            a.c.mate[v] = cv[i] - a.c.gbase[g];
            a.c.state[v] = 1;
            if (use_bits) atomicOr(&a.c.mbits[v >> 5], 1u << (v & 31));
            if (!csr) a.in.rows[row[i]].w = rec[i].w | kMatchedBit;
            ++cnt;
          }
        }
        if (a.c.gphase) {  // one atomic per distinct graph per wave
#pragma unroll
          for (int i = 0; i < kM; ++i) {
            // a live row: a head piece (read from the CSR: a vertex with a candidate)
            const bool live_row = head[i] && (!csr || cv[i] >= 0);
            const int g = live_row ? (rec[i].w & kGraphMask) : -1;
            unsigned long long active = __ballot(g >= 0);
            while (active) {
              const int leader = __ffsll((long long)active) - 1;
              const int gl = __shfl(g, leader, 64);
              const unsigned long long same = __ballot(g == gl);
              if (lane_id() == leader) atomicMax(&a.c.gphase[gl], t);
              active &= ~same;
            }
          }
        }
      }
    }
    unsigned tot;
    (void)block_excl_sum<unsigned>(cnt, s32, tot);
    if (threadIdx.x == 0) a.mcount[bb] = (int)tot;
  }
}

// ---------------------------------------------------------------- stream

// Compaction (and first argmax) over one virtual range [E0, E1) of the live
// set, in batches of at most kBlock * PPL pieces and kBlock * kItems loaded
// entries (kItems from stream_items: 4 to 8 by kernel kind):
//   1. lane j takes piece cur_k + j; a prefix scan decides which pieces fit;
//   2. continuity flags (a piece continuing the previous piece's vertex) and,
//      for every loaded position, the piece it belongs to;
//   3. coalesced loads of the loaded entries, the neighbour's state, and the
//      survivors written in order to the destination (ballot ranks);
//   4. the best candidate of every piece, one lane per piece (a wave per
//      piece longer than kLong);
//   5. vertex segments: the lane of a segment's last piece closes it (writes
//      C[v] and the next live set's piece record); the batch's last segment
//      stays open while its row may continue.
// Candidate keys travel as (ordered weight, local neighbour id): the 64-bit
// tie-break hash is a bijection of the neighbour for a fixed vertex, so the
// pair identifies the key and the hash is recomputed when a full key is due.

// Open vertex segment carried from one batch to the next.
struct Carry {
  int active;
  int v, g, base;  // vertex, graph, first vertex of the graph
  unsigned w;      // best ordered weight so far (0 = none)
  int u;           // best neighbour so far (local id) or -1
  int kept;        // survivors so far
  int out_start;   // destination offset of its first survivor, -1 if none
  int is_first;    // it is the segment that contains the range start
};

constexpr int kLong = 32;                        // longer pieces are reduced by a whole wave
constexpr int kTieLanes = 4;                     // more tied pieces per batch: striped tie-break
constexpr int kLongMax = kCap / (kLong + 1) + 1;  // long pieces per batch at most

// Entries per lane in a batch (measured on the shapes of RGG, R-MAT and the
// batch): the weighted first argmax 8 (4 workgroups per CU), weighted
// compactions 6 (5 per CU with one piece per lane), unweighted kernels 4 (6
// per CU): they hash every entry and gain most from resident waves.
template <bool FIRST, bool UNW>
constexpr int stream_items() { return UNW ? 4 : (FIRST ? 8 : 6); }

template <int W, int IT>  // pieces in a batch window, entries per lane
struct StreamSmem {
  int p_v[W];
  int p_delta[W];            // entry-buffer offset minus batch position of the piece's first entry
  int p_g[W];
  int p_base[W];             // first vertex of the piece's graph
  unsigned short p_vo[W];    // batch position of the piece's first loaded entry
  unsigned short p_ld[W];    // loaded entries of the piece
  unsigned p_w[W];           // best ordered weight of the piece (0 = none)
  int p_u[W];                // best neighbour of the piece (local id) or -1
  unsigned char p_cont[W];   // the piece continues the previous piece's vertex
  unsigned short rowof[kBlock * IT];     // piece of every loaded position
  unsigned short kpre[kBlock * IT + 2];  // survivors before every loaded position; [NLD] = total
  uint2 e_cw[kBlock * IT];               // {ordered weight or 0 when dropped, local neighbour id}
  unsigned long long s_scan[kWaves];
  unsigned s_max[kWaves];
  unsigned s_cnt[IT * kWaves];
  unsigned s_emit[kWaves];
  unsigned long long p_hash[W];  // largest tie-break hash per tied piece
  unsigned char p_tie[W];        // the piece's largest weight repeats
  unsigned char p_hit[W];        // the hash pass saw a candidate of the piece (UNW)
  unsigned s_lmax[kWaves];
  Key s_lkey[kWaves];
  int longlist[kLongMax];
  RunCache rc;  // runs after the window's first run, when the window reaches them
  int lb[1];
  Carry carry;
  Part pf;  // the range's first segment when its row began before E0
  int pf_valid;
  int cur_k, cur_o, cur_r;
  int run_rb, run_lo, run_hi;  // cached run cur_r: row_begin, rpre[cur_r], rpre[cur_r+1]
  long long pos;
  int out_cursor, row_cursor;
  int nt, nld, last_partial, next_cont, nlong;
  int open_left;
};

// How a stream kernel reads its live set: per-graph tables (several graphs),
// one graph with piece records, or R_1 of one graph straight from the CSR.
enum : int { kViewTables = 0, kViewOne = 1, kViewCsr = 2 };

// Piece record of row `row`; from the CSR made from row_ptr (vertex = row,
// graph 0, no head or matched bit: the matched flag is state[v]).
template <bool CSR>
__device__ __forceinline__ int4 piece_at(const LiveSet& in, int row) {
  if (CSR) {
    const long long b = in.csr_rp[row], e = in.csr_rp[row + 1];
    return make_int4(row, (int)b, (int)(e - b), 0);
  }
  return in.rows[row];
}

// First entry of the piece of row `row`.
template <bool CSR>
__device__ __forceinline__ long long piece_start(const LiveSet& in, int row) {
  return CSR ? in.csr_rp[row] : (long long)in.rows[row].y;
}

// Global row index of piece k, walking forward from run r (updated).
__device__ __forceinline__ int piece_row(const LiveSet& in, long long k, int& r, int nruns) {
  while (r + 1 < nruns && (long long)in.rpre[r + 1] <= k) ++r;
  return in.runs[r].row_begin + (int)(k - in.rpre[r]);
}

// Full key of the candidate (w, u) of vertex vloc (local ids).
__device__ __forceinline__ Key full_key(unsigned w, int u, unsigned vloc, unsigned long long S) {
  if (u < 0) return key_ident();
  const uint64_t h = edge_hash(S, vloc, (unsigned)u);
  Key k;
  k.w = w;
  k.hhi = (unsigned)(h >> 32);
  k.hlo = (unsigned)h;
  k.u = u;
  return k;
}

// Among the entries of one row piece whose ordered weight equals m (at
// least two), the neighbour with the largest tie-break hash.
__device__ __forceinline__ int tie_break(const uint2* e, int n, unsigned m, unsigned vloc, unsigned long long S) {
  uint64_t hb = 0;
  int ub = -1;
  for (int i = 0; i < n; ++i) {
    if (e[i].x != m) continue;
    const uint64_t h = edge_hash(S, vloc, e[i].y);
    if (ub < 0 || h > hb) {
      hb = h;
      ub = (int)e[i].y;
    }
  }
  return ub;
}

template <bool FIRST, typename Smem>
__device__ __forceinline__ void close_segment(const StreamArgs& a, Smem& sm, bool cut_left, int v, int g,
                                              int base, unsigned w, int u, unsigned long long S, int kept,
                                              int start, int slot) {
  if (cut_left) {  // the row began in the previous range: the plan kernel merges the parts
    const Key k = full_key(w, u, (unsigned)(v - base), S);
    Part p;
    p.v = v;
    p.flags = 0;
    p.kept = kept;
    p.out_row = slot;
    p.w = k.w;
    p.hhi = k.hhi;
    p.hlo = k.hlo;
    p.u = u >= 0 ? base + u : -1;
    sm.pf = p;
    sm.pf_valid = 1;
    if (!FIRST && slot >= 0) a.rows_out[slot] = make_int4(v, start, kept, g & kGraphMask);
    return;
  }
  if (u >= 0) a.c.C[v] = base + u;
  if (!FIRST && slot >= 0) a.rows_out[slot] = make_int4(v, start, kept, (g & kGraphMask) | kHeadBit);
}

// A batch looks at PPL pieces per lane. The first argmax and the first
// compaction take one: rows are long there, so the entry budget fills first.
// Later compactions see short rows and many pieces of rows matched in the
// phase (skipped without loading), and take kLatePPL (kLatePPLUnw when
// unweighted).
// UNW: an unweighted graph (no weight array; every edge weighs 1). Weights are
// neither loaded nor stored, every loaded piece is tied, the weight scans are
// skipped and the hash pass decides every piece.
// VIEW: kViewOne and kViewCsr hold one graph (vertex base 0, seed seed0), so
// pieces carry no per-graph base or seed and no table is read; kViewCsr reads
// R_1 from the input CSR, empty rows as pieces of length 0, and splits the
// ranges by entries plus a fixed cost per piece (kPieceCostFirst for the
// first argmax, kPieceCost for the compaction).
template <bool FIRST, int PPL, bool UNW, int VIEW>
__device__ void stream_range(const StreamArgs& a, const Ctl& ctl, int b, StreamSmem<kBlock * PPL, stream_items<FIRST, UNW>()>& sm,
                             unsigned long long seed0) {
  constexpr unsigned kUnitOrd = 0xBF800000u;  // ordered image of 1.0f (0x3f800000 | sign bit)
  // neighbour state from the matched bits (scattered ids of one large graph)
  const bool use_bits = !FIRST && a.c.mbits != nullptr && bits_on(a.c.totals);
  constexpr int kItems = stream_items<FIRST, UNW>();  // (shadows the defaults of the other kernels)
  constexpr int kCap = kBlock * kItems;
  constexpr int kPPL = PPL;
  constexpr int kW = kBlock * kPPL;  // pieces in a batch window
  const int tid = threadIdx.x;
  const int lane = lane_id(), wv = wave_id();
  constexpr bool single = VIEW != kViewTables;
  constexpr bool csr = VIEW == kViewCsr;
  long long E0, E1;
  if (csr) {
    constexpr int K = FIRST ? kPieceCostFirst : kPieceCost;
    const long long n = ctl.pieces, cost = ctl.L + (long long)K * n;
    E0 = csr_entry_at<K>(a.in, n, cost * b / ctl.P, sm.lb);
    E1 = csr_entry_at<K>(a.in, n, cost * (b + 1) / ctl.P, sm.lb);
  } else {
    E0 = ctl.L * b / ctl.P;
    E1 = ctl.L * (b + 1) / ctl.P;
  }
  if (E0 >= E1) {
    if (tid == 0) {
      if (!FIRST) {
        Run r;
        r.row_begin = 0;
        r.row_count = 0;
        r.phys_begin = (int)E0;
        r.ent_count = 0;
        a.runs_out[b] = r;
        BlockStat st;
        st.loaded = 0;
        st.matched_len = 0;
        st.pieces_out = 0;
        st.pad = 0;
        a.bstat[b] = st;
      }
      Part none;
      none.v = -1;
      a.parts[2 * b] = none;
      a.parts[2 * b + 1] = none;
    }
    return;
  }
  // ---- locate E0: run, then piece inside the run
  const int r0 = (int)block_lower_bound(
      0, ctl.nruns, [&](long long r) { return a.in.epre[r + 1] > E0; }, sm.lb);
  const Run run0 = a.in.runs[r0];
  const long long lo = E0 - a.in.epre[r0];
  const long long ip = block_lower_bound(
      0, run0.row_count,
      [&](long long i) { return piece_start<csr>(a.in, run0.row_begin + (int)i) - run0.phys_begin > lo; }, sm.lb);
  const int pidx = (int)ip - 1;
  const int k0 = a.in.rpre[r0] + pidx;
  if (tid == 0) {
    const int4 rec0 = piece_at<csr>(a.in, run0.row_begin + pidx);
    const int o0 = (int)(lo - (rec0.y - run0.phys_begin));
    // the range starts inside a row when it cuts a piece or when the previous
    // piece (of this run or of the last non-empty run before it) has the same vertex
    int open_left = o0 > 0;
    if (!csr && !open_left && k0 > 0) {  // (from the CSR every piece is a whole row)
      if (pidx > 0) {
        open_left = a.in.rows[run0.row_begin + pidx - 1].x == rec0.x;
      } else {
        int rr = r0 - 1;
        while (rr > 0 && a.in.runs[rr].row_count == 0) --rr;
        const Run rp = a.in.runs[rr];
        if (rp.row_count > 0) open_left = a.in.rows[rp.row_begin + rp.row_count - 1].x == rec0.x;
      }
    }
    sm.open_left = open_left;
    sm.cur_k = k0;
    sm.cur_o = o0;
    sm.cur_r = r0;
    sm.run_rb = run0.row_begin;
    sm.run_lo = a.in.rpre[r0];
    sm.run_hi = a.in.rpre[r0 + 1];
    sm.pos = E0;
    sm.out_cursor = (int)E0;
    sm.row_cursor = k0 + b;
    sm.carry.active = 0;
    sm.carry.v = -1;
    sm.pf_valid = 0;
  }
  __syncthreads();
  const bool open_left = sm.open_left != 0;
  const int row_start = k0 + b;
  long long loaded_total = 0;  // lane 0 only
  bool first_batch = true;
  for (;;) {
    const long long pos = sm.pos;
    if (pos >= E1) break;
    const int cur_k = sm.cur_k, cur_o = sm.cur_o;
    const int run_rb = sm.run_rb, run_lo = sm.run_lo, run_hi = sm.run_hi;
    const int out_base = sm.out_cursor, row_base = sm.row_cursor;
    const Carry carry = sm.carry;
    int rr = sm.cur_r;
    {
      unsigned* z = reinterpret_cast<unsigned*>(sm.rowof);
      for (int i = tid; i < kCap / 2; i += kBlock) z[i] = 0u;
    }
    if (tid == 0) {
      sm.nt = 0;
      sm.nlong = 0;
    }
    // ---- 1. window: lane t looks at pieces cur_k + kPPL t + h
    const bool span = (long long)cur_k + kW > run_hi && run_hi < ctl.pieces;  // beyond run cur_r
    if (span) {
      run_cache_fill(a.in, ctl.nruns, rr + 1, sm.rc);
      __syncthreads();
    }
    int4 rec[kPPL];
    bool mt[kPPL], valid[kPPL];
    int cov[kPPL], rrh[kPPL];
    unsigned long long lanesum = 0;
#pragma unroll
    for (int h = 0; h < kPPL; ++h) {
      const int j = tid * kPPL + h;
      const long long gk = (long long)cur_k + j;
      valid[h] = gk < ctl.pieces;
      rec[h] = make_int4(-1, 0, 0, 0);
      mt[h] = false;
      if (valid[h]) {
        int row;
        if (gk < run_hi) {
          row = run_rb + (int)(gk - run_lo);
        } else if (!run_cache_find(sm.rc, gk, rr, row)) {  // (span holds here)
          rr = max(rr, sm.rc.c0 + kBlock);  // past the cached runs: rpre[c0 + kBlock] <= gk
          row = piece_row(a.in, gk, rr, ctl.nruns);
        }
        rec[h] = piece_at<csr>(a.in, row);
        if (j == 0) {
          rec[h].y += cur_o;
          rec[h].z -= cur_o;
        }
        if (!FIRST) mt[h] = (rec[h].w & kHeadBit) ? (rec[h].w & kMatchedBit) != 0 : a.c.state[rec[h].x] != 0;
      }
      rrh[h] = rr;
      cov[h] = valid[h] ? rec[h].z : 0;
      lanesum += ((unsigned long long)(unsigned)cov[h] << 32) | (mt[h] ? 0u : (unsigned)cov[h]);
    }
    unsigned long long tot;
    const unsigned long long ex = block_excl_sum_1b<unsigned long long>(lanesum, sm.s_scan, tot);
    const long long Rrem = E1 - pos;
    // Whole pieces are taken while the range and the load budget last; the
    // last one may be cut. Matched pieces are skipped without loading.
    long long cp = (long long)(ex >> 32);        // virtual entries before the piece
    long long lp = (long long)(ex & 0xffffffffull);  // loadable entries before the piece
    // A piece is taken when it starts inside the range and the budget; an
    // empty row (R_1 read from the CSR) is taken with nothing to load.
    long long cpre[kPPL];
    int lpre[kPPL], take[kPPL], ldt[kPPL];
    bool tkn[kPPL];
#pragma unroll
    for (int h = 0; h < kPPL; ++h) {
      cpre[h] = cp;
      lpre[h] = (int)(lp < kCap ? lp : kCap);
      take[h] = 0;
      tkn[h] = valid[h] && cp < Rrem && lp < kCap;
      if (tkn[h]) {
        long long tk = cov[h] < Rrem - cp ? (long long)cov[h] : Rrem - cp;
        if (!mt[h] && tk > kCap - lp) tk = kCap - lp;
        take[h] = (int)tk;
      }
      ldt[h] = mt[h] ? 0 : take[h];
      cp += cov[h];
      lp += mt[h] ? 0 : cov[h];
    }
#pragma unroll
    for (int h = 0; h < kPPL; ++h) {
      const int j = tid * kPPL + h;
      if (tkn[h]) {
        bool next_taken;
        if (h + 1 < kPPL)
          next_taken = tkn[h + 1 < kPPL ? h + 1 : h];
        else
          next_taken = take[h] == cov[h] && j + 1 < kW && (long long)cur_k + j + 1 < ctl.pieces && cp < Rrem &&
                       lp < kCap;
        if (!next_taken) {  // this lane holds the batch's last piece
          sm.nt = j + 1;
          sm.nld = lpre[h] + ldt[h];
          sm.last_partial = take[h] < cov[h];
          sm.cur_r = rrh[h];
        }
        const int g = rec[h].w & kGraphMask;
        sm.p_delta[j] = rec[h].y - lpre[h];
        sm.p_g[j] = g;
        sm.p_base[j] = single ? 0 : a.c.gbase[g];
        sm.p_vo[j] = (unsigned short)lpre[h];
        sm.p_ld[j] = (unsigned short)ldt[h];
        if (ldt[h] > 0) sm.rowof[lpre[h]] = (unsigned short)j;
        if (ldt[h] > kLong) sm.longlist[atomicAdd(&sm.nlong, 1)] = j;
        if (UNW) {
          sm.p_hash[j] = 0ull;
          sm.p_hit[j] = 0;
        }
      }
      if (valid[h]) sm.p_v[j] = rec[h].x;
    }
    __syncthreads();
    const int nt = sm.nt;
    if (nt == 0) {  // nothing consumable: the live set is inconsistent; stop, never spin
      if (tid == 0) atomicOr(&a.c.totals->err, kErrInternal);
      break;
    }
    const int NLD = sm.nld;
    // ---- 2. vertex continuity; piece of every loaded position (prefix max)
    bool cont[kPPL];
#pragma unroll
    for (int h = 0; h < kPPL; ++h) {
      const int j = tid * kPPL + h;
      cont[h] = false;
      if (j < nt) {
        cont[h] = j == 0 ? (carry.active && carry.v == rec[h].x) : (sm.p_v[j - 1] == rec[h].x);
        sm.p_cont[j] = cont[h] ? 1 : 0;
      }
      if (j == nt) sm.next_cont = (valid[h] && sm.p_v[nt - 1] == rec[h].x) ? 1 : 0;
    }
    if (tid == 0 && nt == kW) sm.next_cont = -1;  // the window ended: unknown, keep the segment open
    {
      const int q0 = tid * kItems;
      unsigned runv = 0, vals[kItems];
#pragma unroll
      for (int i = 0; i < kItems; ++i) {
        runv = max(runv, (unsigned)sm.rowof[q0 + i]);
        vals[i] = runv;
      }
      const unsigned cin = block_excl_max_1b(runv, sm.s_max);
#pragma unroll
      for (int i = 0; i < kItems; ++i)
        if (q0 + i < NLD) sm.rowof[q0 + i] = (unsigned short)max(cin, vals[i]);
    }
    __syncthreads();
    // ---- 3. coalesced loads, neighbour state, survivors in order
    // Lanes past the loaded count repeat the last valid position, so every
    // load is unconditional and the compiler can issue them back to back.
    unsigned ktot = 0;
    if (NLD > 0) {
      int cc[kItems];
      float ww[kItems];
      int jp[kItems];
#pragma unroll
      for (int jj = 0; jj < kItems; ++jj) jp[jj] = sm.rowof[min(tid + kBlock * jj, NLD - 1)];
#pragma unroll
      for (int jj = 0; jj < kItems; ++jj) {
        const int addr = min(tid + kBlock * jj, NLD - 1) + sm.p_delta[jp[jj]];
        cc[jj] = a.in.col[addr];
        ww[jj] = UNW ? 1.0f : a.in.w[addr];
      }
      bool ok[kItems];
      unsigned ug[kItems];
#pragma unroll
      for (int jj = 0; jj < kItems; ++jj) {
        const int base = single ? 0 : sm.p_base[jp[jj]];
        ug[jj] = (unsigned)(base + cc[jj]);
        // ids outside the graph are dropped
        ok[jj] = tid + kBlock * jj < NLD && cc[jj] >= 0 && ug[jj] < (unsigned)a.c.n;
      }
      // The neighbours' matched flags: every gather is issued before any is
      // used (one branch around the loads, the bit extracted afterwards), so
      // the kItems round trips overlap.
      unsigned char st[kItems];
      if (!FIRST) {
        unsigned gw[kItems];
        if (use_bits) {
#pragma unroll
          for (int jj = 0; jj < kItems; ++jj) gw[jj] = a.c.mbits[(ok[jj] ? ug[jj] : 0u) >> 5];
        } else {
#pragma unroll
          for (int jj = 0; jj < kItems; ++jj) gw[jj] = a.c.state[ok[jj] ? ug[jj] : 0u];
        }
#pragma unroll
        for (int jj = 0; jj < kItems; ++jj)
          st[jj] = use_bits ? (unsigned char)((gw[jj] >> ((ok[jj] ? ug[jj] : 0u) & 31u)) & 1u) : (unsigned char)gw[jj];
      }
      unsigned rank[kItems];
      unsigned kpm = 0;
      const unsigned long long lt = lanemask_lt();
      if (UNW) {
        // Unweighted: every kept entry is a candidate of its piece, so the
        // lane hashes its kept entries here, keeps the largest hash while its
        // positions stay in one piece (a hub row spans every round), and
        // flushes it with an LDS atomic max when the piece changes; p_hit
        // marks the pieces that had a candidate at all.
        int cur_j = -1;
        unsigned long long cur_h = 0ull;
        bool cur_s = false;
#pragma unroll
        for (int jj = 0; jj < kItems; ++jj) {
          const int j = jp[jj];
          const bool hs = ok[jj] && (FIRST || st[jj] == 0);
          unsigned long long hh = 0ull;
          if (hs) {
            const unsigned long long S = single ? seed0 : cand_seed(a.c.gseed[sm.p_g[j]], a.c.renew, a.cand_phase);
            hh = edge_hash(S, (unsigned)(sm.p_v[j] - (single ? 0 : sm.p_base[j])), (unsigned)cc[jj]);
          }
          if (j != cur_j) {
            if (cur_s) {
              atomicMax(&sm.p_hash[cur_j], cur_h);
              sm.p_hit[cur_j] = 1;
            }
            cur_j = j;
            cur_h = hh;
            cur_s = hs;
          } else if (hs && (!cur_s || hh > cur_h)) {
            cur_h = hh;
            cur_s = true;
          }
        }
        if (__builtin_amdgcn_readfirstlane(cur_j) == __builtin_amdgcn_readlane(cur_j, 63)) {
          const bool any = __ballot(cur_s) != 0ull;  // the whole wave ends in one piece
          cur_h = wave_max_u64(cur_s ? cur_h : 0ull);
          if (lane == 0 && any) {
            atomicMax(&sm.p_hash[cur_j], cur_h);
            sm.p_hit[cur_j] = 1;
          }
        } else if (cur_s) {
          atomicMax(&sm.p_hash[cur_j], cur_h);
          sm.p_hit[cur_j] = 1;
        }
      }
#pragma unroll
      for (int jj = 0; jj < kItems; ++jj) {
        const int q = tid + kBlock * jj;
        const bool kp = ok[jj] && (FIRST || st[jj] == 0);
        if (!UNW && q < NLD)  // (unweighted pieces were decided above)
          sm.e_cw[q] = make_uint2(kp ? ord_weight_bits(__float_as_uint(ww[jj])) : 0u, (unsigned)cc[jj]);
        if (!FIRST) {
          const unsigned long long bal = __ballot(kp);
          rank[jj] = (unsigned)__popcll(bal & lt);
          if (lane == 0) sm.s_cnt[jj * kWaves + wv] = (unsigned)__popcll(bal);
          kpm |= (kp ? 1u : 0u) << jj;
        }
      }
      __syncthreads();
      if (!FIRST) {
        // survivors before (round jj, wave w), in position order q = tid + kBlock * jj
        const unsigned c = lane < kItems * kWaves ? sm.s_cnt[lane] : 0u;
        const unsigned incl = wave_incl_sum_u32(c);
        ktot = (unsigned)__builtin_amdgcn_readlane((int)incl, 63);
        const unsigned excl = incl - c;
#pragma unroll
        for (int jj = 0; jj < kItems; ++jj) {
          const int q = tid + kBlock * jj;
          const unsigned kq = (unsigned)__builtin_amdgcn_readlane((int)excl, jj * kWaves + wv) + rank[jj];
          if (q < NLD) sm.kpre[q] = (unsigned short)kq;
          if ((kpm >> jj) & 1u) {
            a.dst_col[out_base + (int)kq] = cc[jj];
            if (!UNW) a.dst_w[out_base + (int)kq] = ww[jj];
          }
        }
        if (tid == 0) sm.kpre[NLD] = (unsigned short)ktot;
      }
    } else if (tid == 0) {
      sm.kpre[0] = 0;
    }
    // ---- 4. best candidate per piece
    auto seed_of = [&](int h) -> unsigned long long {
      return single ? seed0 : cand_seed(a.c.gseed[rec[h].w & kGraphMask], a.c.renew, a.cand_phase);
    };
    auto vloc_of = [&](int h) -> unsigned {
      return (unsigned)(rec[h].x - (single ? 0 : sm.p_base[tid * kPPL + h]));
    };
    unsigned bw[kPPL];
    int bu[kPPL];
    bool tie[kPPL];
    bool anytie = false;
#pragma unroll
    for (int h = 0; h < kPPL; ++h) {
      const int j = tid * kPPL + h;
      bw[h] = 0u;
      bu[h] = -1;
      tie[h] = false;
      if (UNW) {
        // the hashes of step 3 are complete (barrier after step 3)
        if (j < nt && ldt[h] > 0 && sm.p_hit[j]) {
          bw[h] = kUnitOrd;
          bu[h] = hash_neighbour(sm.p_hash[j], seed_of(h), vloc_of(h));
        }
        if (j < nt) {
          sm.p_w[j] = bw[h];
          sm.p_u[j] = bu[h];
        }
      } else if (j < nt && ldt[h] <= kLong) {
        // largest ordered weight, its first neighbour, and whether it repeats;
        // only a repeated largest weight needs the tie-break hash
        unsigned m = 0u;
        int mu = -1, ties = 0;
#pragma unroll 4
        for (int i = 0; i < ldt[h]; ++i) {
          const uint2 e = sm.e_cw[lpre[h] + i];
          const bool gt = e.x > m;
          ties = gt ? 0 : ties + (e.x == m ? 1 : 0);
          mu = gt ? (int)e.y : mu;
          m = gt ? e.x : m;
        }
        tie[h] = m != 0u && ties > 0;
        bw[h] = m;
        bu[h] = mu;
        sm.p_w[j] = m;
        sm.p_u[j] = mu;
        if (tie[h]) sm.p_hash[j] = 0ull;
      }
      if (!UNW && j < nt && ldt[h] <= kLong) sm.p_tie[j] = tie[h] ? 1 : 0;  // long pieces: set below
      anytie = anytie || tie[h];
    }
    // Long pieces: largest ordered weight only (a wave per piece, or the whole
    // workgroup when there are fewer long pieces than waves); their winner is
    // found by the hash pass below like that of a tied short piece.
    const int nlong = sm.nlong;
    if (UNW) {
      // nothing: every loaded piece is tied at weight 1
    } else if (nlong > 0 && nlong < kWaves) {
      for (int li = 0; li < nlong; ++li) {
        const int j = sm.longlist[li];
        const int vo = sm.p_vo[j], ld = sm.p_ld[j];
        unsigned m = 0u;
        for (int i = tid; i < ld; i += kBlock) m = max(m, sm.e_cw[vo + i].x);
        m = (unsigned)__builtin_amdgcn_readlane((int)wave_incl_max_u32(m), 63);
        if (lane == 0) sm.s_lmax[wv] = m;
        __syncthreads();
        if (tid == 0) {
          unsigned mm = 0u;
#pragma unroll
          for (int x = 0; x < kWaves; ++x) mm = max(mm, sm.s_lmax[x]);
          sm.p_w[j] = mm;
          sm.p_u[j] = -1;
          sm.p_tie[j] = mm != 0u ? 1 : 0;
          sm.p_hash[j] = 0ull;
        }
        __syncthreads();  // s_lmax is rewritten for the next piece
      }
    } else {
      for (int li = wv; li < nlong; li += kWaves) {  // a wave per long piece
        const int j = sm.longlist[li];
        const int vo = sm.p_vo[j], ld = sm.p_ld[j];
        unsigned m = 0u;
        for (int i = lane; i < ld; i += 64) m = max(m, sm.e_cw[vo + i].x);
        m = (unsigned)__builtin_amdgcn_readlane((int)wave_incl_max_u32(m), 63);
        if (lane == 0) {
          sm.p_w[j] = m;
          sm.p_u[j] = -1;
          sm.p_tie[j] = m != 0u ? 1 : 0;
          sm.p_hash[j] = 0ull;
        }
      }
    }
    // A largest weight that repeats in a short piece, and the largest weight of
    // every long piece, is settled by the tie-break hash. With only a few tied
    // short pieces and no long one each lane rescans its own pieces; otherwise
    // all lanes hash the entries that reach their piece's largest weight in
    // striped order, keep the largest hash per piece with an LDS atomic max,
    // and each piece's lane recovers the neighbour by inverting the hash.
    const int ntie = UNW ? 0 : __syncthreads_count(anytie ? 1 : 0);
    if (UNW) {
      // decided in step 4's first loop
    } else if (nlong == 0 && ntie > 0 && ntie <= kTieLanes) {
#pragma unroll
      for (int h = 0; h < kPPL; ++h)
        if (tie[h]) {
          bu[h] = tie_break(sm.e_cw + lpre[h], ldt[h], bw[h], vloc_of(h), seed_of(h));
          sm.p_u[tid * kPPL + h] = bu[h];
        }
    } else if (NLD > 0 && (nlong > 0 || ntie > 0)) {  // (both need loaded entries)
      // each lane keeps the largest hash of its current piece while its
      // rounds stay inside that piece (a hub row spans every round) and
      // flushes it with an LDS atomic max when the piece changes
      int cur_j = -1;
      unsigned long long cur_h = 0ull;
#pragma unroll
      for (int jj = 0; jj < kItems; ++jj) {
        const int q = min(tid + kBlock * jj, NLD - 1);
        const int j = sm.rowof[q];
        unsigned long long hh = 0ull;
        if (tid + kBlock * jj < NLD && sm.p_tie[j]) {
          const uint2 e = sm.e_cw[q];
          if (e.x == sm.p_w[j]) {
            const unsigned long long S = single ? seed0 : cand_seed(a.c.gseed[sm.p_g[j]], a.c.renew, a.cand_phase);
            hh = edge_hash(S, (unsigned)(sm.p_v[j] - sm.p_base[j]), e.y);
          }
        }
        if (j != cur_j) {
          if (cur_h != 0ull) atomicMax(&sm.p_hash[cur_j], cur_h);
          cur_j = j;
          cur_h = hh;
        } else if (hh > cur_h) {
          cur_h = hh;
        }
      }
      if (__builtin_amdgcn_readfirstlane(cur_j) == __builtin_amdgcn_readlane(cur_j, 63)) {
        cur_h = wave_max_u64(cur_h);  // the whole wave ends in one piece
        if (lane == 0 && cur_h != 0ull) atomicMax(&sm.p_hash[cur_j], cur_h);
      } else if (cur_h != 0ull) {
        atomicMax(&sm.p_hash[cur_j], cur_h);
      }
      __syncthreads();
#pragma unroll
      for (int h = 0; h < kPPL; ++h) {
        const int j = tid * kPPL + h;
        if (j < nt && sm.p_tie[j]) {
          if (ldt[h] > kLong) bw[h] = sm.p_w[j];
          bu[h] = hash_neighbour(sm.p_hash[j], seed_of(h), vloc_of(h));
          sm.p_u[j] = bu[h];
        }
      }
    }
    __syncthreads();
    // ---- 5. vertex segments
    // The segment of piece j closes in this batch when piece j+1 starts another
    // vertex; the batch's last segment closes only when the next piece is known
    // to start another vertex. The carried segment closes before piece 0 when
    // piece 0 starts another vertex.
    const bool last_open = sm.last_partial || sm.next_cont != 0;
    const bool old_closes = carry.active && !sm.p_cont[0];
    bool closes[kPPL], shc[kPPL], sfirst[kPPL], emit[kPPL];
    int shead[kPPL], skept[kPPL];
    unsigned sw[kPPL];
    int su[kPPL];
    unsigned ne = 0;
#pragma unroll
    for (int h = 0; h < kPPL; ++h) {
      const int j = tid * kPPL + h;
      closes[h] = false;
      shc[h] = false;
      shead[h] = j;
      skept[h] = 0;
      sw[h] = bw[h];
      su[h] = bu[h];
      if (j < nt) {
        closes[h] = (j + 1 < nt) ? !sm.p_cont[j + 1] : !last_open;
        if (cont[h] && (closes[h] || j == nt - 1)) {
          // the vertex has several pieces here (its row was cut before): walk back
          const unsigned long long S = seed_of(h);
          const unsigned vl = vloc_of(h);
          Key k = full_key(bw[h], bu[h], vl, S);
          int jb = j;
          while (sm.p_cont[jb]) {
            if (jb == 0) {
              shc[h] = true;
              break;
            }
            --jb;
            k = key_max(k, full_key(sm.p_w[jb], sm.p_u[jb], vl, S));
          }
          if (shc[h]) k = key_max(k, full_key(carry.w, carry.u, vl, S));
          shead[h] = jb;
          sw[h] = k.w;
          su[h] = k.u;
        }
        if (!FIRST)
          skept[h] = (int)sm.kpre[lpre[h] + ldt[h]] - (int)sm.kpre[sm.p_vo[shead[h]]] + (shc[h] ? carry.kept : 0);
      }
      sfirst[h] = shc[h] ? carry.is_first != 0 : (first_batch && shead[h] == 0);
      emit[h] = !FIRST && j < nt && closes[h] && skept[h] > 0;
      ne += emit[h] ? 1u : 0u;
    }
    const bool emit_old = !FIRST && tid == 0 && old_closes && carry.kept > 0;
    ne += emit_old ? 1u : 0u;
    unsigned epre = 0, etot = 0;
    if (!FIRST) {  // slots of the emitted piece records, in piece order
      const unsigned inc = wave_incl_sum_u32(ne);
      if (lane == 63) sm.s_emit[wv] = inc;
      __syncthreads();
      epre = inc - ne;
#pragma unroll
      for (int i = 0; i < kWaves; ++i) {
        const unsigned x = sm.s_emit[i];
        if (i < wv) epre += x;
        etot += x;
      }
    }
    int slot = row_base + (int)epre;
    if (tid == 0 && old_closes) {
      close_segment<FIRST>(a, sm, carry.is_first && open_left, carry.v, carry.g, carry.base, carry.w, carry.u,
                           single ? seed0 : cand_seed(a.c.gseed[carry.g], a.c.renew, a.cand_phase), carry.kept, carry.out_start,
                           emit_old ? slot++ : -1);
    }
    int sstart[kPPL];
#pragma unroll
    for (int h = 0; h < kPPL; ++h) {
      const int j = tid * kPPL + h;
      sstart[h] = -1;
      if (!FIRST && j < nt && (closes[h] || j == nt - 1)) {
        const int bstart = out_base + (int)sm.kpre[sm.p_vo[shead[h]]];
        sstart[h] = shc[h] && carry.out_start >= 0 ? carry.out_start
                                                    : (skept[h] > (shc[h] ? carry.kept : 0) ? bstart : -1);
      }
      if (j < nt && closes[h]) {
        close_segment<FIRST>(a, sm, sfirst[h] && open_left, rec[h].x, rec[h].w & kGraphMask,
                             single ? 0 : sm.p_base[j], sw[h], su[h], seed_of(h), skept[h], sstart[h],
                             emit[h] ? slot++ : -1);
      }
    }
    // ---- 6. carry and advance (lane of the last piece)
    if (tid == (nt - 1) / kPPL) {
      const int hl = (nt - 1) - tid * kPPL;
      int4 rl = rec[0];
      int takel = take[0], covl = cov[0], skl = skept[0], ssl = sstart[0], rrl = rrh[0];
      long long cprel = cpre[0];
      unsigned swl = sw[0];
      int sul = su[0];
      bool sfl = sfirst[0];
#pragma unroll
      for (int h = 1; h < kPPL; ++h)
        if (hl == h) {
          rl = rec[h];
          takel = take[h];
          covl = cov[h];
          skl = skept[h];
          ssl = sstart[h];
          rrl = rrh[h];
          cprel = cpre[h];
          swl = sw[h];
          sul = su[h];
          sfl = sfirst[h];
        }
      Carry nc;
      nc.active = 0;
      nc.v = rl.x;
      if (last_open) {
        nc.active = 1;
        nc.g = rl.w & kGraphMask;
        nc.base = single ? 0 : sm.p_base[nt - 1];
        nc.w = swl;
        nc.u = sul;
        nc.kept = skl;
        nc.out_start = ssl;
        nc.is_first = sfl ? 1 : 0;
      }
      sm.carry = nc;
      sm.out_cursor = out_base + (int)ktot;
      sm.row_cursor = row_base + (int)etot;
      sm.pos = pos + cprel + takel;
      int nk, no;
      if (takel < covl) {
        nk = cur_k + nt - 1;
        no = (nt == 1 ? cur_o : 0) + takel;
      } else {
        nk = cur_k + nt;
        no = 0;
      }
      sm.cur_k = nk;
      sm.cur_o = no;
      if (nk >= run_hi && nk < ctl.pieces) {
        int r2 = rrl;
        (void)piece_row(a.in, nk, r2, ctl.nruns);
        sm.cur_r = r2;
        sm.run_rb = a.in.runs[r2].row_begin;
        sm.run_lo = a.in.rpre[r2];
        sm.run_hi = a.in.rpre[r2 + 1];
      }
    }
    if (tid == 0) loaded_total += NLD;
    first_batch = false;
    __syncthreads();
  }
  // ---- close the range: the open segment is cut iff its row continues at E1
  if (tid == 0) {
    Part pf_out, pl_out;
    pf_out.v = -1;
    pl_out.v = -1;
    if (sm.pf_valid) pf_out = sm.pf;
    const Carry c = sm.carry;
    if (c.active) {
      bool open_right = false;
      if (sm.cur_o > 0) {
        open_right = true;
      } else if (sm.cur_k < ctl.pieces) {
        int rr = sm.cur_r;
        open_right = piece_at<csr>(a.in, piece_row(a.in, sm.cur_k, rr, ctl.nruns)).x == c.v;
      }
      const bool cut_left = c.is_first && open_left;
      const int slot = (!FIRST && c.kept > 0) ? sm.row_cursor : -1;
      if (slot >= 0) {
        a.rows_out[slot] =
            make_int4(c.v, c.out_start, c.kept, (c.g & kGraphMask) | ((open_right || cut_left) ? 0 : kHeadBit));
        sm.row_cursor = slot + 1;
      }
      if (cut_left || open_right) {
        const Key k = full_key(c.w, c.u, (unsigned)(c.v - c.base), single ? seed0 : cand_seed(a.c.gseed[c.g], a.c.renew, a.cand_phase));
        Part p;
        p.v = c.v;
        p.flags = (cut_left && open_right) ? kPartSingle : 0;
        p.kept = c.kept;
        p.out_row = slot;
        p.w = k.w;
        p.hhi = k.hhi;
        p.hlo = k.hlo;
        p.u = c.u >= 0 ? c.base + c.u : -1;
        if (cut_left)
          pf_out = p;
        else
          pl_out = p;
      } else if (c.u >= 0) {
        a.c.C[c.v] = c.base + c.u;
      }
    }
    a.parts[2 * b] = pf_out;
    a.parts[2 * b + 1] = pl_out;
    if (!FIRST) {
      Run r;
      r.row_begin = row_start;
      r.row_count = sm.row_cursor - row_start;
      r.phys_begin = (int)E0;
      r.ent_count = sm.out_cursor - (int)E0;
      a.runs_out[b] = r;
      BlockStat st;
      st.loaded = loaded_total;
      st.matched_len = (E1 - E0) - loaded_total;
      st.pieces_out = r.row_count;
      st.pad = 0;
      a.bstat[b] = st;
    }
  }
}

template <bool FIRST, int PPL, bool UNW, int VIEW>
__global__ __launch_bounds__(kBlock, UNW ? (PPL > 1 ? 4 : 6) : (FIRST ? 4 : (PPL > 1 ? 3 : 5))) void k_stream(StreamArgs a) {
  __shared__ StreamSmem<kBlock * PPL, stream_items<FIRST, UNW>()> sm;
  __shared__ unsigned s_err;
  if (block_failed(a.c, &s_err)) return;
  Ctl ctl = *a.in.ctl;
  if (FIRST && ctl.Pf > 0) ctl.P = ctl.Pf;  // the first argmax's own split of R_1
  const unsigned long long seed0 = cand_seed(a.c.gseed[0], a.c.renew, a.cand_phase);
  for (int b = blockIdx.x; b < ctl.P; b += gridDim.x) {
    stream_range<FIRST, PPL, UNW, VIEW>(a, ctl, b, sm, seed0);
    __syncthreads();
  }
}

// ---------------------------------------------------------------- launchers

hipError_t launch_zero(Ctl* ctl, int nctl, Totals* totals, hipStream_t s, TailCtl* tc) {
  hipLaunchKernelGGL(k_zero, dim3(1), dim3(kBlock), 0, s, ctl, nctl, totals, tc);
  return hipGetLastError();
}
hipError_t launch_fill_i32(int* p, long long n, int value, hipStream_t s) {
  const long long blocks = std::min<long long>((n + kBlock - 1) / kBlock, 4096);
  hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)std::max<long long>(blocks, 1)), dim3(kBlock), 0, s, p, n, value);
  return hipGetLastError();
}
hipError_t launch_add_i64(long long* p, long long n, long long delta, hipStream_t s) {
  const long long blocks = std::min<long long>((n + kBlock - 1) / kBlock, 1024);
  hipLaunchKernelGGL(k_add_i64, dim3((unsigned)std::max<long long>(blocks, 1)), dim3(kBlock), 0, s, p, n, delta);
  return hipGetLastError();
}
hipError_t launch_check(const CheckArgs& a, int grid, hipStream_t s) {
  hipLaunchKernelGGL(k_check, dim3(grid), dim3(kBlock), 0, s, a);
  hipLaunchKernelGGL(k_check_fp, dim3(1), dim3(64), 0, s, a.totals);
  return hipGetLastError();
}
// With ev = {start, stop} the launch goes through hipExtLaunchKernelGGL and
// the dispatch itself stamps both events; otherwise a plain launch (the one
// HIP graph capture records).
template <typename K, typename A>
static hipError_t launch_timed(K kernel, dim3 grid, dim3 block, hipStream_t s, hipEvent_t* ev, const A& a) {
  if (ev)
    hipExtLaunchKernelGGL(kernel, grid, block, 0, s, ev[0], ev[1], 0, a);
  else
    hipLaunchKernelGGL(kernel, grid, block, 0, s, a);
  return hipGetLastError();
}

hipError_t launch_init(const InitArgs& a, hipStream_t s, hipEvent_t* ev) {
  return launch_timed(k_init, dim3(a.nblocks), dim3(kBlock), s, ev, a);
}
hipError_t launch_plan(const PlanArgs& a, hipStream_t s, hipEvent_t* ev) {
  return launch_timed(k_plan, dim3(1), dim3(kPlanThreads), s, ev, a);
}
// A live set of one graph (graphs == 1: vertex base 0) takes the kernels
// specialised for it (R_1 read from the CSR when the live set says so); every
// other live set the ones that read the tables.
template <bool FIRST, int PPL, bool UNW>
static hipError_t launch_stream(const StreamArgs& a, int grid, hipStream_t s, hipEvent_t* ev) {
  if constexpr (PPL == 1) {
    if (a.c.graphs == 1 && a.in.csr_rp)
      return launch_timed(k_stream<FIRST, PPL, UNW, kViewCsr>, dim3(grid), dim3(kBlock), s, ev, a);
  }
  if (a.in.csr_rp) return hipErrorInvalidValue;  // the CSR view is for R_1 of one graph only
  if (a.c.graphs == 1) return launch_timed(k_stream<FIRST, PPL, UNW, kViewOne>, dim3(grid), dim3(kBlock), s, ev, a);
  return launch_timed(k_stream<FIRST, PPL, UNW, kViewTables>, dim3(grid), dim3(kBlock), s, ev, a);
}
hipError_t launch_first_argmax(const StreamArgs& a, int grid, hipStream_t s, bool unweighted, hipEvent_t* ev,
                               long long nnz) {
  if (a.c.graphs > 1 && a.in.csr_rp && !unweighted) return launch_first_csr(a, grid, s, false, ev);  // a batch
  if (a.c.graphs == 1 && a.in.csr_rp) {
    if (unweighted) {
      const bool vec_ok = ((unsigned long long)a.in.col & 15ull) == 0ull && nnz >= first_unw_min_entries();
      return launch_first_unw(a, grid, s, vec_ok, ev);
    }
    return launch_first_csr(a, grid, s, false, ev);
  }
  if (unweighted) return launch_stream<true, 1, true>(a, grid, s, ev);
  return launch_stream<true, 1, false>(a, grid, s, ev);
}
hipError_t launch_compact(const StreamArgs& a, int grid, hipStream_t s, bool late, bool unweighted, hipEvent_t* ev) {
  if (unweighted) {
    if (late) return launch_stream<false, kLatePPLUnw, true>(a, grid, s, ev);
    return launch_stream<false, 1, true>(a, grid, s, ev);
  }
  if (late) return launch_stream<false, kLatePPL, false>(a, grid, s, ev);
  return launch_stream<false, 1, false>(a, grid, s, ev);
}
hipError_t launch_mutual(const MutualArgs& a, int grid, hipStream_t s, hipEvent_t* ev) {
  return launch_timed(k_mutual, dim3(grid), dim3(kBlock), s, ev, a);
}

template <typename K>
static int blocks_per_cu(K kernel) {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kernel, kBlock, 0) != hipSuccess || nb < 1) nb = 1;
  return nb;
}

// Resident workgroups of every specialisation a launch may take: the fewest.
template <bool FIRST, int PPL, bool UNW>
static int stream_blocks_per_cu() {
  int nb = std::min(blocks_per_cu(k_stream<FIRST, PPL, UNW, kViewOne>),
                    blocks_per_cu(k_stream<FIRST, PPL, UNW, kViewTables>));
  if constexpr (PPL == 1) nb = std::min(nb, blocks_per_cu(k_stream<FIRST, PPL, UNW, kViewCsr>));
  return nb;
}

int max_blocks_per_cu_stream(StreamKind kind, bool unweighted) {
  if (unweighted) {
    if (kind == StreamKind::kFirst) return stream_blocks_per_cu<true, 1, true>();
    if (kind == StreamKind::kCompact) return stream_blocks_per_cu<false, 1, true>();
    return stream_blocks_per_cu<false, kLatePPLUnw, true>();
  }
  if (kind == StreamKind::kFirst) return stream_blocks_per_cu<true, 1, false>();
  if (kind == StreamKind::kCompact) return stream_blocks_per_cu<false, 1, false>();
  return stream_blocks_per_cu<false, kLatePPL, false>();
}

uint64_t premix_seed(uint64_t seed) { return host_mix64(seed ^ kGoldenGamma); }

}  // namespace lm
