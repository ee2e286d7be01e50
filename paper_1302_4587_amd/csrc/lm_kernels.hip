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
#include <algorithm>

#include "lm_device.h"
#include "lm_internal.h"
#include "lm_key.h"

namespace lm {

// Reads the error word once per workgroup so that every lane takes the same
// branch.
__device__ __forceinline__ bool block_failed(Totals* t, unsigned* s) {
  if (threadIdx.x == 0) *s = t->err;
  __syncthreads();
  const bool f = *s != 0;
  __syncthreads();
  return f;
}

// ---------------------------------------------------------------- small

__global__ void k_zero(Ctl* ctl, int nctl, Totals* totals) {
  int* p = reinterpret_cast<int*>(ctl);
  const int words = nctl * (int)(sizeof(Ctl) / 4);
  for (int i = threadIdx.x; i < words; i += blockDim.x) p[i] = 0;
  if (threadIdx.x == 0) {
    totals->err = 0;
    totals->last_nonempty = 0;
    totals->matched = 0;
  }
}

__global__ void k_fill_i32(int* p, long long n, int value) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    p[i] = value;
}

// Optional input check: ids in range, no self-loops, finite weights.
__global__ __launch_bounds__(kBlock) void k_check(CheckArgs a) {
  unsigned err = 0;
  for (long long v = (long long)blockIdx.x * kBlock + threadIdx.x; v < a.n; v += (long long)gridDim.x * kBlock) {
    long long base = 0, lim = a.n;
    if (a.graphs > 1) {
      int lo = 0, hi = a.graphs - 1;
      while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (a.vtx_off[mid] <= v) lo = mid;
        else hi = mid - 1;
      }
      base = a.vtx_off[lo];
      lim = a.vtx_off[lo + 1] - base;
    }
    const long long b = a.row_ptr[v], e = a.row_ptr[v + 1];
    if (b < 0 || e > a.nnz || e < b) {
      err |= kErrRowPtr;
      continue;
    }
    for (long long k = b; k < e; ++k) {
      const int u = a.col[k];
      if (u < 0 || u >= lim) err |= kErrColRange;
      if (u == v - base) err |= kErrSelfLoop;
      const float x = a.w[k];
      if (!(x == x) || x == __int_as_float(0x7f800000) || x == __int_as_float(0xff800000)) err |= kErrWeight;
    }
  }
  if (err) atomicOr(&a.totals->err, err);
}

// ---------------------------------------------------------------- init

// Live set R_1 straight from the input CSR: workgroup b covers vertices
// [N b / B, N (b+1) / B); every vertex with at least one entry becomes one
// head piece pointing at its input row, and the workgroup's pieces form run
// b (their rows are back to back in the input). Also clears mate and state
// and checks the offsets.
__global__ __launch_bounds__(kBlock) void k_init(InitArgs a) {
  __shared__ unsigned s32[kWaves];
  const int tid = threadIdx.x;
  const int b = blockIdx.x;
  const long long N = a.c.n;
  const long long vb = N * b / a.nblocks, ve = N * (b + 1) / a.nblocks;
  unsigned err = 0;
  // graph of this lane's first vertex (lanes own kItems consecutive vertices)
  int g = 0;
  unsigned cursor = 0;
  for (long long c0 = vb; c0 < ve; c0 += kCap) {
    const long long v0 = c0 + (long long)tid * kItems;
    if (a.graphs > 1 && v0 < ve) {
      int lo = 0, hi = a.graphs - 1;
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (a.vtx_off[mid] <= v0) lo = mid;
        else hi = mid - 1;
      }
      g = lo;
    }
    long long rp[kItems + 1];
    unsigned cnt = 0;
#pragma unroll
    for (int i = 0; i <= kItems; ++i) {
      const long long v = v0 + i;
      rp[i] = (v <= ve && v <= N) ? a.row_ptr[v] : 0;
    }
#pragma unroll
    for (int i = 0; i < kItems; ++i) {
      const long long v = v0 + i;
      if (v < ve) {
        const long long d = rp[i + 1] - rp[i];
        if (d < 0 || rp[i] < 0 || rp[i + 1] > a.nnz) err |= kErrRowPtr;
        if (d > 0x7fff0000LL) err |= kErrDegree;
        if (d > 0) ++cnt;
      }
    }
    unsigned tot;
    unsigned ex = block_excl_sum<unsigned>(cnt, s32, tot);
    unsigned at = cursor + ex;
#pragma unroll
    for (int i = 0; i < kItems; ++i) {
      const long long v = v0 + i;
      if (v < ve) {
        if (a.graphs > 1)
          while (a.vtx_off[g + 1] <= v) ++g;
        a.c.mate[v] = -1;
        a.c.state[v] = 0;
        const long long d = rp[i + 1] - rp[i];
        if (d > 0 && d <= 0x7fff0000LL) {
          a.rows_out[vb + at] = make_int4((int)v, (int)rp[i], (int)d, (g & kGraphMask) | kHeadBit);
          ++at;
        }
      }
    }
    cursor += tot;
  }
  if (tid == 0) {
    Run r;
    r.row_begin = (int)vb;
    r.row_count = (int)cursor;
    const long long pb = vb < N ? a.row_ptr[vb] : a.nnz;
    const long long pe = a.row_ptr[ve];
    r.phys_begin = (int)pb;
    r.ent_count = (int)(pe - pb);
    if (vb == 0 && pb != 0) err |= kErrRowPtr;
    if (ve == N && pe != a.nnz) err |= kErrRowPtr;
    if (pe < pb) err |= kErrRowPtr;
    a.runs_out[b] = r;
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
  __shared__ long long s_red[4];
  const int tid = threadIdx.x;
  if (tid == 0) {
    s_err = a.c.totals->err;
    s_extra = 0;
    s_red[0] = s_red[1] = s_red[2] = 0;
  }
  __syncthreads();
  if (s_err) return;
  const Ctl prev = a.ctl_prev ? *a.ctl_prev : Ctl{0, 0, 0, 0, 0, 0, 0};
  if (a.mode & kPlanFix) {
    for (int b = tid; b < prev.P; b += kPlanThreads) {
      const Part pl = a.parts[2 * b + 1];
      if (pl.v < 0) continue;  // block b does not own a cut row
      Key best;
      best.w = pl.w;
      best.hhi = pl.hhi;
      best.hlo = pl.hlo;
      best.u = pl.u;
      int head_row = pl.kept > 0 ? pl.out_row : -1;
      int pieces = pl.out_row >= 0 ? 1 : 0;
      for (int b2 = b + 1; b2 < prev.P; ++b2) {
        const Part pf = a.parts[2 * b2];
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
        if (head_row >= 0) a.rows_out[head_row].w |= kHeadBit;
        if (pieces > 1) atomicAdd(&s_extra, pieces - 1);
      }
    }
  }
  __syncthreads();
  if (a.mode & kPlanPrefix) {
    const int nr = a.nruns_new >= 0 ? a.nruns_new : prev.P;
    // blocked scan over nr <= kMaxBlocks runs, 4 per lane
    constexpr int kPer = kMaxBlocks / kPlanThreads;
    long long le[kPer];
    int lr[kPer];
    long long se = 0;
    int sr = 0;
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
      const int r = tid * kPer + i;
      le[i] = 0;
      lr[i] = 0;
      if (r < nr) {
        const Run run = a.runs_new[r];
        le[i] = run.ent_count;
        lr[i] = run.row_count;
      }
      se += le[i];
      sr += lr[i];
    }
    long long ie = wave_incl_sum<long long>(se);
    int ir = wave_incl_sum<int>(sr);
    if (lane_id() == 63) {
      s_e[tid >> 6] = ie;
      s_r[tid >> 6] = ir;
    }
    __syncthreads();
    long long pe = 0, te = 0;
    int pr = 0, tr = 0;
    for (int wv = 0; wv < kPlanThreads / 64; ++wv) {
      if (wv < (tid >> 6)) {
        pe += s_e[wv];
        pr += s_r[wv];
      }
      te += s_e[wv];
      tr += s_r[wv];
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
      c.heads = tr - s_extra;
      long long P = (te + a.min_per_block - 1) / a.min_per_block;
      c.P = (int)std::max<long long>(te > 0 ? 1 : 0, std::min<long long>(P, a.pcap));
      long long Pm = ((long long)tr + kCap - 1) / kCap;
      c.Pm = (int)std::max<long long>(tr > 0 ? 1 : 0, std::min<long long>(Pm, a.pmcap));
      c.pad = 0;
      *a.ctl_new = c;
    }
  }
  if (a.mode & kPlanLog) {
    long long mc = 0, ml = 0;
    for (int b = tid; b < prev.Pm; b += kPlanThreads) mc += a.mcount[b];
    for (int b = tid; b < prev.P; b += kPlanThreads) ml += a.bstat[b].matched_len;
    mc = wave_incl_sum<long long>(mc);
    ml = wave_incl_sum<long long>(ml);
    if (lane_id() == 63) {
      atomicAdd((unsigned long long*)&s_red[0], (unsigned long long)mc);
      atomicAdd((unsigned long long*)&s_red[1], (unsigned long long)ml);
    }
    __syncthreads();
    if (tid == 0) {
      if (a.t >= 1 && a.t <= a.log_cap) {
        LogRec r;
        r.live_entries = prev.L;
        r.live_rows = prev.heads;
        r.matched_edges = s_red[0] / 2;
        r.matched_entries = s_red[1];
        a.log[a.t - 1] = r;
      }
      if (prev.heads > 0) a.c.totals->last_nonempty = a.t;
      a.c.totals->matched += (unsigned long long)s_red[0];
    }
  }
}

// ---------------------------------------------------------------- mutual

__global__ __launch_bounds__(kBlock) void k_mutual(MutualArgs a) {
  __shared__ unsigned s_err;
  __shared__ int s_lb[1];
  __shared__ unsigned s32[kWaves];
  if (block_failed(a.c.totals, &s_err)) return;
  const Ctl ctl = *a.in.ctl;
  for (int bb = blockIdx.x; bb < ctl.Pm; bb += gridDim.x) {
    const long long V = ctl.pieces;
    const long long p0 = V * bb / ctl.Pm, p1 = V * (bb + 1) / ctl.Pm;
    unsigned cnt = 0;
    if (p0 < p1) {
      // run containing piece p0: first r with rpre[r+1] > p0
      const int r0 = (int)block_lower_bound(
          0, ctl.nruns, [&](long long r) { return (long long)a.in.rpre[r + 1] > p0; }, s_lb);
      int r = r0;
      for (long long base = p0; base < p1; base += kBlock) {
        const long long pi = base + threadIdx.x;
        int g = -1;
        if (pi < p1) {
          while (r + 1 < ctl.nruns && (long long)a.in.rpre[r + 1] <= pi) ++r;
          const int row = a.in.runs[r].row_begin + (int)(pi - a.in.rpre[r]);
          const int4 rec = a.in.rows[row];
          if (rec.w & kHeadBit) {
            const int v = rec.x;
            g = rec.w & kGraphMask;
            const int u = a.c.C[v];
            if ((unsigned)u < (unsigned)a.c.n && a.c.C[u] == v) {
              a.c.mate[v] = u - a.c.gbase[g];
              a.c.state[v] = 1;
              a.in.rows[row].w = rec.w | kMatchedBit;
              ++cnt;
            }
          }
        }
        if (a.c.gphase) {  // one atomic per distinct graph per wave
          unsigned long long active = __ballot(g >= 0);
          while (active) {
            const int leader = __ffsll((long long)active) - 1;
            const int gl = __shfl(g, leader, 64);
            const unsigned long long same = __ballot(g == gl);
            if (lane_id() == leader) atomicMax(&a.c.gphase[gl], a.t);
            active &= ~same;
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

// Block-uniform state of one compaction workgroup while it walks its range.
struct Carry {
  int active;      // a segment is open from the previous batch
  int v, g;        // its vertex and graph
  unsigned w, hhi, hlo;
  int u;           // best neighbour so far (local id) or -1
  int kept;        // survivors so far
  int out_start;   // destination offset of its first survivor, -1 if none
  int is_first;    // it is the segment that contains the range start
};

struct StreamSmem {
  int p_v[kWin];
  int p_off[kWin];
  int p_g[kWin];
  int p_base[kWin];                  // first vertex of the piece's graph
  unsigned short p_vo[kWin];    // first loaded position of the piece in the batch
  unsigned short p_take[kWin];  // loaded entries of the piece in the batch
  unsigned short p_seg[kWin];   // segment id: head piece + 1, 0 = continuation
  unsigned char p_fl[kWin];     // kFl* flags
  unsigned short s_kst[kWin + 1];
  unsigned short s_kend[kWin + 1];
  int s_best[kWin + 1];         // best local id per segment
  unsigned short rowof[kCap];
  int e_col[kCap];
  unsigned e_w[kCap];
  unsigned long long s64[kWaves];
  unsigned s32[kWaves];
  SegKey sseg[kWaves];
  int lb[1];
  Key firstkey, lastkey;        // full keys of the batch's first and last segment
  // walk state
  Carry carry;
  int cur_k, cur_o, cur_r;
  int run_rb, run_lo, run_hi;  // cached run cur_r: row_begin, rpre[cur_r], rpre[cur_r+1]
  long long pos;
  int out_cursor, row_cursor;
  int nt, nld, consumed;
  int last_partial, last_take;
  int out_base_batch;
  int open_left;
};

enum : unsigned char { kFlHead = 1, kFlSegEnd = 2, kFlSegFirst = 4, kFlMatched = 8 };

// Global row index of piece k, walking forward from run r (updated).
__device__ __forceinline__ int piece_row(const LiveSet& in, long long k, int& r, int nruns) {
  while (r + 1 < nruns && (long long)in.rpre[r + 1] <= k) ++r;
  return in.runs[r].row_begin + (int)(k - in.rpre[r]);
}

template <bool FIRST>
__device__ void stream_range(const StreamArgs& a, const Ctl& ctl, int b, StreamSmem& sm,
                             unsigned long long seed0) {
  const int tid = threadIdx.x;
  const bool single = a.c.graphs == 1;
  const long long E0 = ctl.L * b / ctl.P;
  const long long E1 = ctl.L * (b + 1) / ctl.P;
  Part pf_out, pl_out;
  pf_out.v = -1;
  pl_out.v = -1;
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
      a.parts[2 * b] = pf_out;
      a.parts[2 * b + 1] = pl_out;
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
      [&](long long i) { return (long long)(a.in.rows[run0.row_begin + i].y - run0.phys_begin) > lo; }, sm.lb);
  const int pidx = (int)ip - 1;
  const int k0 = a.in.rpre[r0] + pidx;
  const int4 rec0 = a.in.rows[run0.row_begin + pidx];
  const int o0 = (int)(lo - (rec0.y - run0.phys_begin));
  if (tid == 0) {
    int open_left = o0 > 0;
    if (!open_left && k0 > 0) {
      int rr = 0;
      // run of piece k0-1: the last non-empty run before r0 (or r0 itself)
      if (pidx > 0) {
        open_left = a.in.rows[run0.row_begin + pidx - 1].x == rec0.x;
      } else {
        rr = r0 - 1;
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
    sm.carry.kept = 0;
    sm.carry.out_start = -1;
    sm.carry.u = -1;
    sm.carry.is_first = 0;
  }
  __syncthreads();
  const int row_start = k0 + b;
  long long loaded_total = 0, matched_total = 0;  // lane 0 only
  bool first_batch = true;
  for (;;) {
    const long long pos = sm.pos;
    if (pos >= E1) break;
    const int cur_k = sm.cur_k, cur_o = sm.cur_o;
    int rr = sm.cur_r;
    const int run_rb = sm.run_rb, run_lo = sm.run_lo, run_hi = sm.run_hi;
    const Carry carry = sm.carry;
    __syncthreads();
    // ---- 1. window of pieces: lane t owns pieces 2t, 2t+1
    int4 rec[2];
    long long cov[2];
    int ld[2];
    int rrh[2];
    bool mt[2], valid[2];
    unsigned long long mine = 0;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int j = 2 * tid + h;
      const long long gk = (long long)cur_k + j;
      valid[h] = gk < ctl.pieces;
      cov[h] = 0;
      ld[h] = 0;
      mt[h] = false;
      rec[h] = make_int4(-1, 0, 0, 0);
      rrh[h] = rr;
      if (valid[h]) {
        // pieces of the cached run need no run-table reads
        const int row = gk < run_hi ? run_rb + (int)(gk - run_lo) : piece_row(a.in, gk, rr, ctl.nruns);
        rec[h] = a.in.rows[row];
        rrh[h] = gk < run_hi ? rr : rr;
        const int sub = j == 0 ? cur_o : 0;
        rec[h].y += sub;
        rec[h].z -= sub;
        if (!FIRST)
          mt[h] = (rec[h].w & kHeadBit) ? (rec[h].w & kMatchedBit) != 0 : a.c.state[rec[h].x] != 0;
        cov[h] = rec[h].z;
      }
      mine += ((unsigned long long)cov[h] << 32) | (unsigned long long)(mt[h] ? 0 : (unsigned)cov[h]);
    }
    unsigned long long tot;
    const unsigned long long ex = block_excl_sum<unsigned long long>(mine, sm.s64, tot);
    const long long Rrem = E1 - pos;
    long long cpre = (long long)(ex >> 32);
    long long lpre = (long long)(ex & 0xffffffffull);
    int take[2];
    unsigned taken_cnt = 0, loaded = 0;
    long long consumed = 0;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      take[h] = 0;
      if (valid[h] && cpre < Rrem && lpre < kCap) {
        long long tk = std::min<long long>(cov[h], Rrem - cpre);
        if (!mt[h]) tk = std::min<long long>(tk, kCap - lpre);
        take[h] = (int)tk;
      }
      if (take[h] > 0) {
        ++taken_cnt;
        consumed += take[h];
        if (!mt[h]) loaded += (unsigned)take[h];
      }
      cpre += cov[h];
      lpre += mt[h] ? 0 : cov[h];
    }
    // counts: taken pieces and loaded entries (prefix), consumed (total)
    unsigned long long cnt2 = ((unsigned long long)consumed << 32) | ((unsigned long long)taken_cnt << 16) | loaded;
    unsigned long long tot2;
    const unsigned long long ex2 = block_excl_sum<unsigned long long>(cnt2, sm.s64, tot2);
    const int nt = (int)((tot2 >> 16) & 0xffffu);
    const int NLD = (int)(tot2 & 0xffffu);
    unsigned vo = (unsigned)(ex2 & 0xffffu);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int j = 2 * tid + h;
      if (take[h] > 0) {
        sm.p_v[j] = rec[h].x;
        sm.p_off[j] = rec[h].y;
        const int g = rec[h].w & kGraphMask;
        sm.p_g[j] = g;
        sm.p_base[j] = single ? 0 : a.c.gbase[g];
        sm.p_vo[j] = (unsigned short)vo;
        sm.p_take[j] = (unsigned short)(mt[h] ? 0 : take[h]);
        sm.p_fl[j] = mt[h] ? kFlMatched : 0;
        if (!mt[h]) vo += (unsigned)take[h];
        if (j == nt - 1) {
          sm.last_partial = take[h] < cov[h];
          sm.last_take = take[h];
          sm.cur_r = rrh[h];
        }
      }
    }
    if (nt == 0) {  // nothing consumable: the live set is inconsistent; stop, never spin
      if (tid == 0) atomicOr(&a.c.totals->err, kErrInternal);
      break;
    }
    if (tid == 0) {
      sm.nt = nt;
      sm.nld = NLD;
      sm.consumed = (int)(tot2 >> 32);
      sm.firstkey = key_ident();
      sm.lastkey = key_ident();
    }
    __syncthreads();
    // ---- 2. segment heads (by vertex) and segment ids
    unsigned hmax = 0;
    unsigned char hflag[2] = {0, 0};
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int j = 2 * tid + h;
      if (j < nt) {
        const int v = sm.p_v[j];
        const bool head = j == 0 ? !(carry.active && carry.v == v) : (sm.p_v[j - 1] != v);
        hflag[h] = head ? kFlHead : 0;
        if (head) hmax = (unsigned)(j + 1);
      }
    }
    // segment id of piece j = largest head index + 1 at or before j
    unsigned segs[2];
    {
      const unsigned carry_in = block_excl_max(hmax, sm.s32);
      unsigned run_seg = carry_in;
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int j = 2 * tid + h;
        if (hflag[h]) run_seg = (unsigned)(j + 1);
        segs[h] = run_seg;
      }
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int j = 2 * tid + h;
      if (j < nt) {
        sm.p_seg[j] = (unsigned short)segs[h];
        sm.p_fl[j] |= hflag[h];
      }
    }
    for (int s = tid; s <= nt; s += kBlock) {
      sm.s_kst[s] = 0;
      sm.s_kend[s] = 0;
      sm.s_best[s] = -1;
    }
    for (int q = tid; q < NLD; q += kBlock) sm.rowof[q] = 0;
    __syncthreads();
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int j = 2 * tid + h;
      if (j < nt) {
        const unsigned s = segs[h];
        const bool last_of_seg = (j + 1 >= nt) || (sm.p_seg[j + 1] != s);
        const bool first_of_seg = s == 0 ? (j == 0) : (j == (int)s - 1);
        unsigned char f = sm.p_fl[j];
        if (last_of_seg) f |= kFlSegEnd;
        if (first_of_seg) f |= kFlSegFirst;
        sm.p_fl[j] = f;
        if (sm.p_take[j] > 0) sm.rowof[sm.p_vo[j]] = (unsigned short)j;
      }
    }
    __syncthreads();
    // ---- 3. piece of every loaded position: prefix max of the piece heads
    {
      const int q0 = tid * kItems;
      unsigned runv = 0, vals[kItems];
#pragma unroll
      for (int i = 0; i < kItems; ++i) {
        const int q = q0 + i;
        if (q < NLD) runv = max(runv, (unsigned)sm.rowof[q]);
        vals[i] = runv;
      }
      const unsigned cin = block_excl_max(runv, sm.s32);
#pragma unroll
      for (int i = 0; i < kItems; ++i) {
        const int q = q0 + i;
        if (q < NLD) sm.rowof[q] = (unsigned short)max(cin, vals[i]);
      }
    }
    __syncthreads();
    // ---- 4. striped coalesced loads, neighbour state gather
    {
      int cc[kItems];
      float ww[kItems];
#pragma unroll
      for (int jj = 0; jj < kItems; ++jj) {
        const int q = tid + kBlock * jj;
        cc[jj] = 0;
        ww[jj] = 0.f;
        if (q < NLD) {
          const int j = sm.rowof[q];
          const int addr = sm.p_off[j] + (q - (int)sm.p_vo[j]);
          cc[jj] = a.in.col[addr];
          ww[jj] = a.in.w[addr];
        }
      }
#pragma unroll
      for (int jj = 0; jj < kItems; ++jj) {
        const int q = tid + kBlock * jj;
        if (q < NLD) {
          const int j = sm.rowof[q];
          unsigned col = (unsigned)cc[jj];
          const unsigned ug = (unsigned)(sm.p_base[j] + cc[jj]);
          if (cc[jj] < 0 || ug >= (unsigned)a.c.n)
            col |= kDropBit;  // id outside the graph: never a candidate
          else if (!FIRST && a.c.state[ug] != 0)
            col |= kDropBit;
          sm.e_col[q] = (int)col;
          sm.e_w[q] = __float_as_uint(ww[jj]);
        }
      }
    }
    __syncthreads();
    // ---- 5. blocked pass: kept counts, segmented argmax
    const int q0 = tid * kItems;
    unsigned mycol[kItems], myw[kItems];
    unsigned short myseg[kItems];
    unsigned char mypos[kItems];  // 1 = first entry of its segment, 2 = last entry
    unsigned kc = 0;
    SegKey agg;
    agg.f = 0;
    agg.k = key_ident();
    Key p1 = key_ident();
    int c0_seg = -1;
    bool c0_ends = false, head0 = false;
    {
      Best run = best_ident();
      int cur_s = -1;
      bool first_open = true;
      unsigned vloc = 0;
      unsigned long long S = 0;
#pragma unroll
      for (int i = 0; i < kItems; ++i) {
        const int q = q0 + i;
        myseg[i] = 0xffff;
        mypos[i] = 0;
        if (q >= NLD) continue;
        const int j = sm.rowof[q];
        const int s = sm.p_seg[j];
        const unsigned char fl = sm.p_fl[j];
        const bool seg_first = (fl & kFlSegFirst) && q == (int)sm.p_vo[j];
        const bool seg_last = (fl & kFlSegEnd) && q == (int)sm.p_vo[j] + (int)sm.p_take[j] - 1;
        if (s != cur_s) {
          S = single ? seed0 : a.c.gseed[sm.p_g[j]];
          vloc = (unsigned)(sm.p_v[j] - sm.p_base[j]);
          if (cur_s < 0) {
            c0_seg = s;
            head0 = seg_first && s >= 1;
            agg.f = head0 ? 1u : 0u;
          } else {
            agg.f = 1u;  // a segment starts inside this lane's items
          }
          cur_s = s;
          run = best_ident();
        }
        myseg[i] = (unsigned short)s;
        mypos[i] = (seg_first ? 1 : 0) | (seg_last ? 2 : 0);
        const unsigned col = (unsigned)sm.e_col[q];
        const unsigned wb = sm.e_w[q];
        mycol[i] = col;
        myw[i] = wb;
        if (!(col & kDropBit)) {
          ++kc;
          best_update(run, ord_weight_bits(wb), (int)col, vloc, S);
        }
        if (seg_last) {
          const Key k = best_key(run, vloc, S);
          if (first_open) {
            p1 = k;
            c0_ends = true;
            first_open = false;
          } else {
            sm.s_best[s] = k.u;
            if (q == NLD - 1) sm.lastkey = k;
          }
        }
      }
      if (cur_s >= 0) {
        if (first_open) p1 = best_key(run, vloc, S);
        agg.k = best_key(run, vloc, S);
      }
    }
    unsigned ktot;
    const unsigned kpre = block_excl_sum<unsigned>(kc, sm.s32, ktot);
    SegKey cin = block_excl_segscan(agg, sm.sseg);
    {
      // the open segment of the previous batch precedes every entry
      SegKey cel;
      cel.f = 0;
      cel.k = key_ident();
      if (carry.active && carry.u >= 0) {
        cel.k.w = carry.w;
        cel.k.hhi = carry.hhi;
        cel.k.hlo = carry.hlo;
        cel.k.u = carry.u;
      }
      cin = seg_combine(cel, cin);
    }
    if (c0_ends) {
      const Key k = head0 ? p1 : key_max(cin.k, p1);
      sm.s_best[c0_seg] = k.u;
      if (c0_seg == sm.p_seg[nt - 1] && sm.p_take[nt - 1] > 0) {
        // the batch's last segment ended in this lane's first segment
        sm.lastkey = k;
      }
      if (c0_seg == sm.p_seg[0]) sm.firstkey = k;
    }
    // kept positions of segment starts and ends
    {
      unsigned p = kpre;
#pragma unroll
      for (int i = 0; i < kItems; ++i) {
        if (myseg[i] == 0xffff) continue;
        if (mypos[i] & 1) sm.s_kst[myseg[i]] = (unsigned short)p;
        if (!(mycol[i] & kDropBit)) ++p;
        if (mypos[i] & 2) sm.s_kend[myseg[i]] = (unsigned short)p;
      }
    }
    // (the batch's first segment starts at q = 0, so it is always the first
    // segment of the lane where it ends: its full key was stored above)
    __syncthreads();
    // ---- 6. segment outputs
    // Segments of this batch in piece order: ids s_first = p_seg[0] ... ; the
    // segment of piece nt-1 stays open (new carry). The old carry closes
    // first when piece 0 starts a new segment.
    const int last_seg = sm.p_seg[nt - 1];
    const bool cont = (sm.p_seg[0] == 0);  // piece 0 continues the carry
    // per segment: finalize? kept>0? one lane per segment head (plus lane 0
    // for the continuation segment and the old carry)
    int my_out[2] = {0, 0};
    unsigned want = 0;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int j = 2 * tid + h;
      if (j < nt && (sm.p_fl[j] & kFlHead)) {
        const int s = j + 1;
        if (s != last_seg) {
          const int kept = (int)sm.s_kend[s] - (int)sm.s_kst[s];
          if (kept > 0 && !FIRST) {
            my_out[h] = 1;
            ++want;
          }
        }
      }
    }
    // lane 0: old carry (closed at batch start) and continuation segment
    int old_out = 0, cont_out = 0;
    if (tid == 0) {
      if (carry.active && !cont && carry.kept > 0 && !FIRST) old_out = 1;
      if (cont && last_seg != 0) {
        const int kept = carry.kept + ((int)sm.s_kend[0] - (int)sm.s_kst[0]);
        if (kept > 0 && !FIRST) cont_out = 1;
      }
      want += old_out + cont_out;
    }
    unsigned wtot;
    const unsigned wpre = block_excl_sum<unsigned>(want, sm.s32, wtot);
    const int out_base = sm.out_cursor;   // destination of this batch's first survivor
    const int row_base = sm.row_cursor;
    auto finalize = [&](int v, int g, int kept, int out_off, int u_local, const Key* full, int row_slot,
                        bool is_first_seg) {
      // row_slot: output piece index or -1; is_first_seg: segment containing E0
      const int gb = a.c.gbase[g];
      if (is_first_seg && sm.open_left) {
        Part p;
        p.v = v;
        p.flags = 0;
        p.kept = kept;
        p.out_row = row_slot;
        p.w = full ? full->w : 0u;
        p.hhi = full ? full->hhi : 0u;
        p.hlo = full ? full->hlo : 0u;
        p.u = (full && full->u >= 0) ? gb + full->u : -1;
        pf_out = p;
        if (!FIRST && row_slot >= 0) a.rows_out[row_slot] = make_int4(v, out_off, kept, g & kGraphMask);
        return;
      }
      if (u_local >= 0) a.c.C[v] = gb + u_local;
      if (!FIRST && row_slot >= 0) a.rows_out[row_slot] = make_int4(v, out_off, kept, (g & kGraphMask) | kHeadBit);
    };
    if (tid == 0) {
      unsigned at = wpre;
      if (carry.active && !cont) {
        // the previous batch's last segment ended with the previous batch
        Key full;
        full.w = carry.w;
        full.hhi = carry.hhi;
        full.hlo = carry.hlo;
        full.u = carry.u;
        const int slot = old_out ? row_base + (int)(at++) : -1;
        finalize(carry.v, carry.g, carry.kept, carry.out_start, carry.u, &full, slot, carry.is_first);
      }
      if (cont && last_seg != 0) {
        const int kb = (int)sm.s_kend[0] - (int)sm.s_kst[0];
        const int kept = carry.kept + kb;
        const int start = carry.out_start >= 0 ? carry.out_start : out_base + (int)sm.s_kst[0];
        const int slot = cont_out ? row_base + (int)(at++) : -1;
        finalize(sm.p_v[0], sm.p_g[0], kept, start, sm.s_best[0], &sm.firstkey, slot, carry.is_first);
      }
    }
    {
      unsigned at = wpre + (tid == 0 ? (unsigned)(old_out + cont_out) : 0u);
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int j = 2 * tid + h;
        if (j < nt && (sm.p_fl[j] & kFlHead)) {
          const int s = j + 1;
          if (s == last_seg) continue;
          const int kept = (int)sm.s_kend[s] - (int)sm.s_kst[s];
          const int slot = my_out[h] ? row_base + (int)(at++) : -1;
          const bool is_first_seg = first_batch && j == 0;
          finalize(sm.p_v[j], sm.p_g[j], kept, out_base + (int)sm.s_kst[s], sm.s_best[s],
                   is_first_seg ? &sm.firstkey : nullptr, slot, is_first_seg);
        }
      }
    }
    // in-place compaction of kept entries (all reads of e_* are done)
    if (!FIRST) {
      unsigned p = kpre;
#pragma unroll
      for (int i = 0; i < kItems; ++i) {
        if (myseg[i] == 0xffff || (mycol[i] & kDropBit)) continue;
        sm.e_col[p] = (int)(mycol[i] & ~kDropBit);
        sm.e_w[p] = myw[i];
        ++p;
      }
    }
    __syncthreads();
    if (!FIRST) {
      for (int p = tid; p < (int)ktot; p += kBlock) {
        a.dst_col[out_base + p] = sm.e_col[p];
        a.dst_w[out_base + p] = __uint_as_float(sm.e_w[p]);
      }
    }
    // ---- 7. new carry and advance
    if (tid == 0) {
      Carry nc;
      nc.active = 1;
      nc.v = sm.p_v[nt - 1];
      nc.g = sm.p_g[nt - 1];
      const bool has_entries = sm.p_take[nt - 1] > 0;
      const int kb = (int)sm.s_kend[last_seg] - (int)sm.s_kst[last_seg];
      Key lk = key_ident();
      if (has_entries) lk = sm.lastkey;
      if (last_seg == 0) {  // still the carried segment
        Key ck;
        ck.w = carry.w;
        ck.hhi = carry.hhi;
        ck.hlo = carry.hlo;
        ck.u = carry.u;
        if (carry.u < 0) ck = key_ident();
        lk = has_entries ? key_max(ck, lk) : ck;
        nc.kept = carry.kept + kb;
        nc.out_start = carry.out_start >= 0 ? carry.out_start : (kb > 0 ? out_base + (int)sm.s_kst[0] : -1);
        nc.is_first = carry.is_first;
      } else {
        nc.kept = kb;
        nc.out_start = kb > 0 ? out_base + (int)sm.s_kst[last_seg] : -1;
        nc.is_first = first_batch && last_seg == (int)sm.p_seg[0] && sm.p_seg[0] == 1;
      }
      nc.w = lk.w;
      nc.hhi = lk.hhi;
      nc.hlo = lk.hlo;
      nc.u = lk.u;
      sm.carry = nc;
      sm.out_cursor = out_base + (int)ktot;
      sm.row_cursor = row_base + (int)wtot;
      sm.pos = pos + sm.consumed;
      if (sm.last_partial) {
        sm.cur_k = cur_k + nt - 1;
        sm.cur_o = (nt == 1 ? cur_o : 0) + sm.last_take;
      } else {
        sm.cur_k = cur_k + nt;
        sm.cur_o = 0;
      }
      if (sm.cur_k >= sm.run_hi && sm.cur_k < ctl.pieces) {
        int r2 = sm.cur_r;
        (void)piece_row(a.in, sm.cur_k, r2, ctl.nruns);
        sm.cur_r = r2;
        sm.run_rb = a.in.runs[r2].row_begin;
        sm.run_lo = a.in.rpre[r2];
        sm.run_hi = a.in.rpre[r2 + 1];
      }
      loaded_total += NLD;
    }
    first_batch = false;
    __syncthreads();
  }
  // ---- close the range: the open segment is cut iff its row continues at E1
  if (tid == 0) {
    const Carry c = sm.carry;
    bool open_right = false;
    if (sm.cur_o > 0) {
      open_right = true;
    } else if (sm.cur_k < ctl.pieces) {
      int rr = sm.cur_r;
      open_right = a.in.rows[piece_row(a.in, sm.cur_k, rr, ctl.nruns)].x == c.v;
    }
    Key full;
    full.w = c.w;
    full.hhi = c.hhi;
    full.hlo = c.hlo;
    full.u = c.u;
    if (c.u < 0) full = key_ident();
    const int gb = a.c.gbase[c.g];
    const int slot = (!FIRST && c.kept > 0) ? sm.row_cursor : -1;
    if (!FIRST && slot >= 0) {
      const bool closed = !open_right && !(c.is_first && sm.open_left);
      a.rows_out[slot] = make_int4(c.v, c.out_start, c.kept, (c.g & kGraphMask) | (closed ? kHeadBit : 0));
      sm.row_cursor = slot + 1;
    }
    Part p;
    p.v = c.v;
    p.flags = 0;
    p.kept = c.kept;
    p.out_row = slot;
    p.w = full.w;
    p.hhi = full.hhi;
    p.hlo = full.hlo;
    p.u = full.u >= 0 ? gb + full.u : -1;
    if (c.is_first && sm.open_left) {
      p.flags = open_right ? kPartSingle : 0;
      pf_out = p;
    } else if (open_right) {
      pl_out = p;
    } else if (full.u >= 0) {
      a.c.C[c.v] = gb + full.u;
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

template <bool FIRST>
__global__ __launch_bounds__(kBlock, 4) void k_stream(StreamArgs a) {
  __shared__ StreamSmem sm;
  __shared__ unsigned s_err;
  if (block_failed(a.c.totals, &s_err)) return;
  const Ctl ctl = *a.in.ctl;
  const unsigned long long seed0 = a.c.gseed[0];
  for (int b = blockIdx.x; b < ctl.P; b += gridDim.x) {
    stream_range<FIRST>(a, ctl, b, sm, seed0);
    __syncthreads();
  }
}

// ---------------------------------------------------------------- launchers

hipError_t launch_zero(Ctl* ctl, int nctl, Totals* totals, hipStream_t s) {
  hipLaunchKernelGGL(k_zero, dim3(1), dim3(kBlock), 0, s, ctl, nctl, totals);
  return hipGetLastError();
}
hipError_t launch_fill_i32(int* p, long long n, int value, hipStream_t s) {
  const long long blocks = std::min<long long>((n + kBlock - 1) / kBlock, 4096);
  hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)std::max<long long>(blocks, 1)), dim3(kBlock), 0, s, p, n, value);
  return hipGetLastError();
}
hipError_t launch_check(const CheckArgs& a, int grid, hipStream_t s) {
  hipLaunchKernelGGL(k_check, dim3(grid), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}
hipError_t launch_init(const InitArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_init, dim3(a.nblocks), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}
hipError_t launch_plan(const PlanArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_plan, dim3(1), dim3(kPlanThreads), 0, s, a);
  return hipGetLastError();
}
hipError_t launch_first_argmax(const StreamArgs& a, int grid, hipStream_t s) {
  hipLaunchKernelGGL(k_stream<true>, dim3(grid), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}
hipError_t launch_compact(const StreamArgs& a, int grid, hipStream_t s) {
  hipLaunchKernelGGL(k_stream<false>, dim3(grid), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}
hipError_t launch_mutual(const MutualArgs& a, int grid, hipStream_t s) {
  hipLaunchKernelGGL(k_mutual, dim3(grid), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

int max_blocks_per_cu_stream() {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_stream<false>, kBlock, 0) != hipSuccess || nb < 1) nb = 1;
  return nb;
}

uint64_t premix_seed(uint64_t seed) { return host_mix64(seed + kGoldenGamma); }

}  // namespace lm
