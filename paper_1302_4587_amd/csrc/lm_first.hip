// First argmax of a single graph read straight from its CSR (R_1), gfx950:
// k_first_csr for a weighted graph, k_first_unw (further below) for an
// unweighted one.
//
// Every vertex v with a live entry gets C[v] = the neighbour u maximising the
// key (w, H(seed, lo, hi)) over its row (Section 2, first pass of the
// sequential model; the keys are those of Section 1's perturbed weights,
// fixed as a hash). The workgroup of a cost range (entries plus a fixed cost
// per row, as the plan kernel splits R_1) walks it in tiles of at most
// kFTile entries and kFRows rows. Each lane takes kFIt consecutive entries
// (two 16-byte loads) and reduces the runs of one row inside them in
// registers: a row whose entries all fall into one lane is finished there. A
// row that crosses lanes (or tiles) is combined in LDS in two passes: the
// largest ordered weight first, then the largest hash among the segments
// that reach it; the winner is the neighbour whose hash that is (the hash is
// a bijection of the neighbour for a fixed vertex). An unweighted graph skips
// the weight pass (k_first_unw is faster for those). Rows cut at range
// boundaries leave a partial result for the plan kernel, as the other stream
// kernels do.
#include <hip/hip_ext.h>

#include "lm_device.h"
#include "lm_internal.h"
#include "lm_key.h"

namespace lm {

namespace {

constexpr int kFIt = 8;                // entries per lane per tile
constexpr int kFTile = kBlock * kFIt;  // entries per tile at most
constexpr int kFRows = 256;            // rows per tile at most
static_assert(kFIt % 4 == 0, "entries are loaded 16 bytes at a time");

struct FirstSmem {
  long long wrp[kFRows + 1];       // row_ptr of the tile's rows vc .. vc + kFRows
  unsigned sw[kFRows];             // rows crossing lanes: largest ordered weight (unweighted: 1 = touched)
  unsigned long long sh[kFRows];   // largest hash among the segments at that weight
  unsigned c_w;                    // the row open at the tile's end: its partial key
  unsigned long long c_h;
  int c_valid;
  Part pf, pl;                     // the range's cut rows
  int lb[1];
  unsigned err;
  // several graphs (a batch): the graph of every row of the tile
  unsigned long long rseed[kFRows];  // its tie-break seed
  int rbase[kFRows];                 // its first vertex
  int rlim[kFRows];                  // its vertex count (local ids below it)
  int rgraph[kFRows + 1];            // its index; [kFRows]: the graph of row vc + kFRows
  int g_cur;                         // the graph of row vc
};

// A lane's running best over one row segment. Weighted: the largest ordered
// weight with its neighbour, the hash only once a tie needs it (Best).
// Unweighted: the largest hash and its neighbour.
template <bool UNW>
struct Seg;
template <>
struct Seg<false> {
  Best b;
  __device__ __forceinline__ void reset() { b = best_ident(); }
  // one entry's ordered weight w (0: no candidate) and neighbour u; the hash
  // only when w ties the best so far
  __device__ __forceinline__ void add_key(unsigned w, int u, unsigned v, unsigned long long S, unsigned long long) {
    if (w != 0u) best_update(b, w, u, v, S);
  }
  __device__ __forceinline__ int u() const { return b.u; }
  __device__ __forceinline__ unsigned w() const { return b.w; }
  __device__ __forceinline__ unsigned long long h(unsigned v, unsigned long long S) const {
    return b.hv ? b.h : edge_hash(S, v, (unsigned)b.u);
  }
  // this = c ? o : this, field by field (a select of whole structs would go
  // through private memory)
  __device__ __forceinline__ void pick(bool c, const Seg& o) {
    b.w = c ? o.b.w : b.w;
    b.u = c ? o.b.u : b.u;
    b.h = c ? o.b.h : b.h;
    b.hv = c ? o.b.hv : b.hv;
  }
};
template <>
struct Seg<true> {
  unsigned long long hb;
  int ub;
  __device__ __forceinline__ void reset() {
    hb = 0ull;
    ub = -1;
  }
  __device__ __forceinline__ void add_key(unsigned w, int u, unsigned, unsigned long long, unsigned long long h) {
    const bool gt = w != 0u && (ub < 0 || h > hb);
    hb = gt ? h : hb;
    ub = gt ? u : ub;
  }
  __device__ __forceinline__ int u() const { return ub; }
  __device__ __forceinline__ unsigned w() const { return 1u; }
  __device__ __forceinline__ unsigned long long h(unsigned, unsigned long long) const { return hb; }
  __device__ __forceinline__ void pick(bool c, const Seg& o) {
    hb = c ? o.hb : hb;
    ub = c ? o.ub : ub;
  }
};

// (v global; base: its graph's first vertex, whose local ids the hash takes)
__device__ __forceinline__ Part part_of(int v, int flags, unsigned w, unsigned long long h, unsigned long long S,
                                        int base = 0) {
  Part p;
  p.v = v;
  p.flags = flags;
  p.kept = 0;
  p.out_row = -1;
  p.w = w;
  p.hhi = (unsigned)(h >> 32);
  p.hlo = (unsigned)h;
  p.u = base + hash_neighbour(h, S, (unsigned)(v - base));
  return p;
}

// The lane's kFIt entries from s0 on (two 16-byte loads each when aligned
// and in bounds; otherwise only the entries in [lo, hi) are read).
template <bool UNW>
__device__ __forceinline__ void load_entries(const int* col, const float* wt, long long s0, long long lo, long long hi,
                                             long long nnz, bool vec, int (&cv)[kFIt], float (&wv)[kFIt]) {
  if (vec && s0 >= 0 && s0 + kFIt <= nnz) {
#pragma unroll
    for (int j = 0; j < kFIt; j += 4) {
      const int4 x = *reinterpret_cast<const int4*>(col + s0 + j);
      cv[j] = x.x;
      cv[j + 1] = x.y;
      cv[j + 2] = x.z;
      cv[j + 3] = x.w;
      if (!UNW) {
        const float4 y = *reinterpret_cast<const float4*>(wt + s0 + j);
        wv[j] = y.x;
        wv[j + 1] = y.y;
        wv[j + 2] = y.z;
        wv[j + 3] = y.w;
      }
    }
  } else {
#pragma unroll
    for (int j = 0; j < kFIt; ++j) {
      const long long q = s0 + j;
      const bool in = q >= lo && q < hi;
      cv[j] = in ? col[q] : 0;
      wv[j] = (!UNW && in) ? wt[q] : 1.0f;
    }
  }
}

// MULTI: the CSR is the disjoint union of a batch's graphs (a.c.graphs of
// them, graph k from vertex gbase[k] on, local neighbour ids, a seed each):
// every tile looks up the graph of each of its rows, walking on from the
// graph of its first row.
template <bool UNW, bool MULTI>
__device__ void first_range(const StreamArgs& a, const Ctl& ctl, int b, FirstSmem& sm, unsigned long long S,
                            bool vec) {
  constexpr unsigned kUnitOrd = 0xBF800000u;  // ordered image of 1.0f
  const int tid = threadIdx.x;
  const long long* rp = a.in.csr_rp;
  const int* col = a.in.col;
  const float* wt = a.in.w;
  const long long n = a.c.n;  // rows of the CSR (every vertex of the union)
  const int G = a.c.graphs;
  // per row slot of the current tile: graph seed, first vertex, vertex count
  auto seed_of = [&](int i) -> unsigned long long { return MULTI ? sm.rseed[i] : S; };
  auto base_of = [&](int i) -> int { return MULTI ? sm.rbase[i] : 0; };
  auto lim_of = [&](int i) -> long long { return MULTI ? (long long)sm.rlim[i] : n; };
  const long long nnz = rp[n];
  const long long cost = ctl.L + (long long)kPieceCostFirst * n;
  const long long E0 = csr_entry_at<kPieceCostFirst>(a.in, n, cost * b / ctl.P, sm.lb);
  const long long E1 = csr_entry_at<kPieceCostFirst>(a.in, n, cost * (b + 1) / ctl.P, sm.lb);
  Part none;
  none.v = -1;
  if (E0 >= E1) {
    if (tid == 0) {
      a.parts[2 * b] = none;
      a.parts[2 * b + 1] = none;
    }
    return;
  }
  // the row holding E0 (empty rows before it are skipped)
  const long long v0 = block_lower_bound(0, n, [&](long long v) { return rp[v + 1] > E0; }, sm.lb);
  const bool cut_left = rp[v0] < E0;
  long long vc = v0, e = E0;
  if (MULTI) {  // the graph of v0: the last graph starting at or before it
    const long long g1 = block_lower_bound(0, G, [&](long long g) { return (long long)a.c.gbase[g] > v0; }, sm.lb);
    if (tid == 0) sm.g_cur = (int)g1 - 1;
  }
  if (tid == 0) {
    sm.pf = none;
    sm.pl = none;
    sm.c_valid = 0;
  }
  __syncthreads();
  while (e < E1) {
    // ---- the tile's rows and their LDS slots
    for (int i = tid; i <= kFRows; i += kBlock) sm.wrp[i] = rp[min(vc + i, n)];
    for (int i = tid; i < kFRows; i += kBlock) {
      sm.sw[i] = 0u;
      sm.sh[i] = 0ull;
    }
    if (MULTI) {
      const int g0 = sm.g_cur;
      for (int i = tid; i <= kFRows; i += kBlock) {
        const long long v = min(vc + i, n - 1);
        int g = g0;
        while (g + 1 < G && (long long)a.c.gbase[g + 1] <= v) ++g;  // (graph boundaries inside the tile)
        sm.rgraph[i] = g;
        if (i < kFRows) {
          const int base = a.c.gbase[g];
          sm.rbase[i] = base;
          sm.rlim[i] = (g + 1 < G ? a.c.gbase[g + 1] : (int)n) - base;
          sm.rseed[i] = cand_seed(a.c.gseed[g], a.c.renew, a.cand_phase);
        }
      }
    }
    // the open row's partial key (from the previous tile): its weight joins
    // slot 0 in pass 1, its hash counts only if no segment of this tile
    // raises that weight
    const bool carry = sm.c_valid != 0;
    const unsigned cw_in = sm.c_w;
    const unsigned long long ch_in = sm.c_h;
    __syncthreads();
    const long long* wrp = sm.wrp;
    unsigned* sw = sm.sw;
    unsigned long long* sh = sm.sh;
    const long long e_al = e & ~3ll;
    const long long tend = min(min(E1, e_al + kFTile), wrp[kFRows]);
    const long long s0 = e_al + (long long)kFIt * tid;
    const long long lo = max(e, s0), hi = min(tend, s0 + kFIt);
    int cv[kFIt];
    float wv[kFIt];
    load_entries<UNW>(col, wt, s0, lo, hi, nnz, vec, cv, wv);
    // ---- stage 1: the row slot of each of the lane's positions (positions
    // outside [lo, hi) keep the slot before them) and whether it is a
    // candidate (the lane's, with an id inside the graph)
    int rs[kFIt];
    bool okv[kFIt];
    int r = 0;  // largest r with wrp[r] <= lo
    if (lo < hi) {
#pragma unroll
      for (int step = kFRows / 2; step > 0; step >>= 1)
        if (r + step < kFRows && wrp[r + step] <= lo) r += step;
    }
    {
      int rr = r;
#pragma unroll
      for (int i = 0; i < kFIt; ++i) {
        const long long q = s0 + i;
        const bool in = q >= lo && q < hi;
        if (in)
          while (q >= wrp[rr + 1]) ++rr;  // rows in between are empty
        rs[i] = rr;
        okv[i] = in && cv[i] >= 0 && cv[i] < lim_of(rr);
      }
    }
    // ---- stage 2: every entry's ordered weight (0: no candidate) and, for an
    // unweighted graph, its hash (all at once, out of masked branches)
    unsigned long long hv[kFIt];
    unsigned kw[kFIt];
#pragma unroll
    for (int i = 0; i < kFIt; ++i) {
      hv[i] = UNW ? keep(edge_hash(seed_of(rs[i]), (unsigned)(vc + rs[i] - base_of(rs[i])), (unsigned)cv[i])) : 0ull;
      kw[i] = okv[i] ? (UNW ? kUnitOrd : ord_weight_bits(__float_as_uint(wv[i]))) : 0u;
    }
    // ---- stage 3: segments. A row inside the lane is finished here; only the
    // lane's first segment (its row began before lo) and its last (its row
    // goes on past hi) can cross into other lanes.
    int rA = -1, rB = -1;  // slots of those two boundary segments
    Seg<UNW> sA, sB;
    sA.reset();
    sB.reset();
    if (lo < hi) {
      Seg<UNW> sg;
      sg.reset();
      Seg<UNW> empty;
      empty.reset();
      int cur = r;
      bool started = wrp[r] >= lo;
#pragma unroll
      for (int i = 0; i < kFIt; ++i) {
        const bool nw = rs[i] != cur;  // the position opens another row
        // the run before it ends: finished in the lane, or the lane's first segment
        if (nw && started && sg.u() >= 0) a.c.C[vc + cur] = base_of(cur) + sg.u();
        const bool fa = nw && !started;
        rA = fa ? cur : rA;
        sA.pick(fa, sg);
        started = started || nw;
        cur = rs[i];
        sg.pick(nw, empty);
        sg.add_key(kw[i], cv[i], (unsigned)(vc + rs[i] - base_of(rs[i])), seed_of(rs[i]), hv[i]);
      }
      const bool ends = wrp[cur + 1] <= hi;
      if (started && ends) {
        if (sg.u() >= 0) a.c.C[vc + cur] = base_of(cur) + sg.u();
      } else if (!started && ends) {
        rA = cur;
        sA = sg;
      } else {
        rB = cur;
        sB = sg;
      }
    }
    // ---- rows across lanes. When every lane of the wave holds a segment of
    // the same row (the tile lies inside a long row), the wave reduces first
    // and one lane updates the slot; otherwise each lane does.
    if (tid == 0) {
      sm.c_valid = 0;  // (read at the top of this tile; set again below)
      if (carry) {
        if (UNW) sw[0] = 1u;
        else atomicMax(&sw[0], cw_in);
      }
    }
    const int rB0 = __builtin_amdgcn_readfirstlane(rB);
    const bool waveB = rB0 >= 0 && __ballot(rB != rB0) == 0ull;
    // (a segment without a valid entry leaves its row untouched)
    if (waveB) {
      const unsigned wB = UNW ? (__ballot(sB.u() >= 0) ? 1u : 0u)
                              : (unsigned)__builtin_amdgcn_readlane((int)wave_incl_max_u32(sB.w()), 63);
      if (lane_id() == 0 && wB) {
        if (UNW) sw[rB0] = 1u;
        else atomicMax(&sw[rB0], wB);
      }
    } else if (rB >= 0 && sB.u() >= 0) {
      if (UNW) sw[rB] = 1u;
      else atomicMax(&sw[rB], sB.w());
    }
    // pass 1: the largest weight
    if (rA >= 0 && sA.u() >= 0) {
      if (UNW) sw[rA] = 1u;
      else atomicMax(&sw[rA], sA.w());
    }
    __syncthreads();
    // pass 2: the largest hash among the segments at that weight
    if (rA >= 0 && sA.u() >= 0 && (UNW || sA.w() == sw[rA]))
      atomicMax(&sh[rA], sA.h((unsigned)(vc + rA - base_of(rA)), seed_of(rA)));
    if (waveB) {
      const bool at = sB.u() >= 0 && (UNW || sB.w() == sw[rB0]);
      const unsigned long long hm =
          wave_max_u64(at ? sB.h((unsigned)(vc + rB0 - base_of(rB0)), seed_of(rB0)) : 0ull);
      const bool any = __ballot(at) != 0ull;  // (every lane takes part in the ballot)
      if (lane_id() == 0 && any) atomicMax(&sh[rB0], hm);
    } else if (rB >= 0 && sB.u() >= 0 && (UNW || sB.w() == sw[rB])) {
      atomicMax(&sh[rB], sB.h((unsigned)(vc + rB - base_of(rB)), seed_of(rB)));
    }
    __syncthreads();
    // ---- finish the rows that crossed lanes
    for (int i = tid; i < kFRows; i += kBlock) {
      if (sw[i] == 0u || wrp[i] >= tend) continue;
      const long long v = vc + i;
      const bool cutl = v == v0 && cut_left;
      const unsigned w = UNW ? kUnitOrd : sw[i];
      unsigned long long hh = sh[i];
      if (i == 0 && carry && sw[0] == cw_in) hh = max(hh, ch_in);
      const int bs = base_of(i);
      if (wrp[i + 1] <= tend) {  // the row ends in this tile
        if (cutl) sm.pf = part_of((int)v, 0, w, hh, seed_of(i), bs);
        else a.c.C[v] = bs + hash_neighbour(hh, seed_of(i), (unsigned)(v - bs));
      } else if (tend == E1) {  // the row goes on past the range
        const Part p = part_of((int)v, cutl ? kPartSingle : 0, w, hh, seed_of(i), bs);
        if (cutl) sm.pf = p;
        else sm.pl = p;
      } else {  // the row goes on in the next tile
        sm.c_w = sw[i];
        sm.c_h = hh;
        sm.c_valid = 1;
      }
    }
    int r2 = 0;  // the next tile starts at the row holding tend: largest r2 <= kFRows with wrp[r2] <= tend
#pragma unroll
    for (int step = kFRows; step > 0; step >>= 1)
      if (r2 + step <= kFRows && wrp[r2 + step] <= tend) r2 += step;
    if (MULTI && tid == 0) sm.g_cur = sm.rgraph[r2];
    __syncthreads();
    vc += r2;
    e = tend;
  }
  if (tid == 0) {
    a.parts[2 * b] = sm.pf;
    a.parts[2 * b + 1] = sm.pl;
  }
  __syncthreads();
}

// ---- unweighted first argmax of one graph: one wave per range ----
//
// Every entry is a candidate (all weights tie), so the row's winner is the
// neighbour of largest hash. A one-wave workgroup walks its range of R_1 in
// steps of kUStep consecutive entries, four per lane (one 16-byte load, the
// next step's issued before the current one is hashed). The rows of a step
// come from a window of 64 consecutive row ends held one per lane (the next
// 64 are loaded while this window is in use): a step never passes the
// window's last row. When the whole step lies in one row (long rows) every
// lane only folds its hashes into a running maximum held in registers; the
// row's lanes are combined once, when it ends. Otherwise each entry's row is
// found from boundary markers in LDS (a max-scan over the step), and every
// row that ends inside the step is combined by LDS 64-bit atomic max in a
// slot of its window row; the row still open at the step's end stays in
// the registers. No workgroup barrier couples waves.
constexpr int kUIt = 4;                // entries per lane per step
constexpr int kUStep = 64 * kUIt;      // entries per step
static_assert(kUIt % 4 == 0, "entries are loaded 16 bytes at a time");
constexpr int kUnwPerCu = 32;          // one-wave ranges per CU (8 per SIMD: at most 64 VGPRs)
constexpr int kUSlots = 64;            // the window's rows

struct UnwSmem {
  unsigned mark[kUStep];               // 1 + window index of the row starting at step position x, 0 none
  unsigned long long slot[kUSlots + 64];  // largest hash per row combined in LDS (+ a dummy per lane)
  unsigned hit[kUSlots + 64];             // the slot holds a hash
};

// Smallest i in [lo, hi) with pred(i) true (pred monotone), hi if none; every
// lane gets the answer. 64 points per round, one memory access per lane.
template <typename Pred>
__device__ __forceinline__ long long wave_lower_bound(long long lo, long long hi, Pred pred) {
  const int lane = lane_id();
  while (hi > lo) {
    const long long n = hi - lo;
    const long long step = (n + 63) >> 6;
    const long long idx = lo + (long long)lane * step;
    const bool p = idx < hi ? pred(idx) : true;
    const unsigned long long bal = __ballot(p);
    if (bal == 0ull) {  // false at every sampled point: the answer lies past the last one
      lo = lo + 63 * step + 1;
      continue;
    }
    const int f = __ffsll((long long)bal) - 1;
    if (f == 0) return lo;
    // false at lo + (f-1) step, true at lo + f step (or that point is past hi)
    const long long nhi = lo + (long long)f * step < hi ? lo + (long long)f * step : hi;
    lo = lo + (long long)(f - 1) * step + 1;
    hi = nhi;
  }
  return lo;
}

// The entry position of cost c over R_1 read from the CSR (the split of the
// other first-argmax kernels: kPieceCostFirst units per row, one per entry).
__device__ __forceinline__ long long wave_csr_entry_at(const long long* rp, long long n, long long c) {
  constexpr long long K = kPieceCostFirst;
  const long long v1 = wave_lower_bound(0, n + 1, [&](long long v) { return rp[v] + K * v > c; });
  const long long v = v1 - 1;
  const long long u = c - (rp[v] + K * v);
  if (u < K || v >= n) return rp[v];
  const long long deg = rp[v + 1] - rp[v];
  return rp[v] + min(u - K, deg);
}

struct UnwCols {
  int c[kUIt];
};

// The lane's kUIt entries of the step starting at s with 16-byte loads
// (the caller guarantees alignment and s + kUStep <= nnz).
__device__ __forceinline__ UnwCols unw_load_vec(const int* col, long long s) {
  const long long q = s + kUIt * lane_id();
  UnwCols r;
#pragma unroll
  for (int j = 0; j < kUIt; j += 4) {
    const int4 x = *reinterpret_cast<const int4*>(col + q + j);
    r.c[j] = x.x;
    r.c[j + 1] = x.y;
    r.c[j + 2] = x.z;
    r.c[j + 3] = x.w;
  }
  return r;
}

// The same one entry at a time, clamped to the last entry (positions past
// E1 are never used; nnz > 0 since the range is not empty).
__device__ __forceinline__ UnwCols unw_load_slow(const int* col, long long s, long long nnz) {
  const long long q = s + kUIt * lane_id();
  UnwCols r;
#pragma unroll
  for (int j = 0; j < kUIt; ++j) r.c[j] = col[min(q + j, nnz - 1)];
  return r;
}

__device__ __forceinline__ Part unw_part(long long v, int flags, bool any, unsigned long long h,
                                         unsigned long long S) {
  constexpr unsigned kUnitOrd = 0xBF800000u;  // ordered image of 1.0f
  Part p;
  p.v = (int)v;
  p.flags = flags;
  p.kept = 0;
  p.out_row = -1;
  p.w = any ? kUnitOrd : 0u;
  p.hhi = any ? (unsigned)(h >> 32) : 0u;
  p.hlo = any ? (unsigned)h : 0u;
  p.u = any ? hash_neighbour(h, S, (unsigned)v) : -1;
  return p;
}

// The workgroup is one wave: LDS accesses of its lanes are carried out in
// issue order, so lanes exchange data through LDS with no s_barrier and no
// wait for the stores; this only keeps the compiler from moving LDS accesses
// across the point.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// One lane to the left across the wave (lane 63 gets ident).
__device__ __forceinline__ unsigned dpp_wave_shl1(unsigned x, unsigned ident) {
  return (unsigned)__builtin_amdgcn_update_dpp((int)ident, (int)x, 0x130, 0xf, 0xf, false);
}

__device__ __forceinline__ long long rdl64(long long x, int l) {
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)x, l);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)((unsigned long long)x >> 32), l);
  return (long long)(((unsigned long long)hi << 32) | lo);
}

// VEC: 16-byte loads (an aligned entry array of at least kUStep entries);
// otherwise every step loads its entries one by one.
template <bool VEC>
__device__ void unw_range(const StreamArgs& a, const Ctl& ctl, int P, int b, UnwSmem& sm, unsigned long long S) {
  const int lane = lane_id();
  const long long* rp = a.in.csr_rp;
  const int* col = a.in.col;
  int* C = a.c.C;
  const long long n = ctl.pieces;
  const long long nnz = rp[n];
  const long long cost = ctl.L + (long long)kPieceCostFirst * n;
  const long long E0 = wave_csr_entry_at(rp, n, cost * b / P);
  const long long E1 = wave_csr_entry_at(rp, n, cost * (b + 1) / P);
  Part pf, pl;
  pf.v = pl.v = -1;
  pf.flags = pl.flags = 0;
  pf.kept = pl.kept = 0;
  pf.out_row = pl.out_row = -1;
  pf.w = pl.w = pf.hhi = pl.hhi = pf.hlo = pl.hlo = 0u;
  pf.u = pl.u = -1;
  if (E0 < E1) {
    // the row holding E0 (empty rows before it are skipped)
    const long long v0 = wave_lower_bound(0, n, [&](long long v) { return rp[v + 1] > E0; });
    const bool cut_left = rp[v0] < E0;
    long long R0 = v0 & ~63ll;                      // window: rows R0 .. R0 + 63, lane i holds the end of row R0 + i
    long long ce = rp[min(R0 + lane + 1, n)];
    long long ne = rp[min(R0 + 64 + lane + 1, n)];  // the next window
    long long pos = E0;
    long long orow = -1;                            // the row open at the end of the previous step
    unsigned long long acc = 0ull;                  // the lane's largest hash in it
    bool ahit = false;
    // a row of the range is finished: its winner, or its part when it began before E0
    auto finish = [&](long long r, bool any, unsigned long long h) {
      if (r == v0 && cut_left) {
        pf = unw_part(r, 0, any, h, S);
      } else if (any && lane == 0) {
        C[r] = hash_neighbour(h, S, (unsigned)r);
      }
    };
    // one step over the entries cv holds (loaded by the step before); the
    // next step's entries are loaded into nxt first. Two buffers alternate,
    // so a load in flight is never copied (a copy would wait for it).
    auto step = [&](UnwCols& cv, bool cvfast, UnwCols& nxt, bool& nxfast) {
      if (pos >= rdl64(ce, 63)) {  // the row of pos lies past the window
        R0 += 64;
        ce = ne;
        ne = rp[min(R0 + 64 + lane + 1, n)];
        while (pos >= rdl64(ce, 63)) {  // (64 or more empty rows)
          R0 += 64;
          ce = rp[min(R0 + lane + 1, n)];
          ne = rp[min(R0 + 64 + lane + 1, n)];
        }
      }
      const long long s = pos & ~3ll;
      const long long se = min(min(s + kUStep, E1), rdl64(ce, 63));
      // The next step's entries are loaded before this step's are used, by
      // the same single load on every path (a load on some paths only makes
      // every use wait for all loads): at the range's end, or where 16-byte
      // loads would not do, it reads the first kUStep entries instead and
      // the next step loads its own entries one by one, before that load.
      const long long sn = min(se, E1 - 1) & ~3ll;
      if (VEC) {
        if (!cvfast) cv = unw_load_slow(col, s, nnz);
        nxfast = sn + kUStep <= nnz;
        nxt = unw_load_vec(col, nxfast ? sn : 0ll);
      } else {
        nxt = unw_load_slow(col, sn, nnz);
      }
      const int xlo = (int)(pos - s), xhi = (int)(se - s);  // valid step positions [xlo, xhi)
      const int rpos = __popcll(__ballot(ce <= pos));       // window row of pos
      const int rlast = __popcll(__ballot(ce < se));        // window row of se - 1
      if (orow >= 0 && orow != R0 + rpos) {
        // the open row ended at pos (where a window or a range part ended):
        // its lanes' maxima meet in one wave reduction
        const bool any = __ballot(ahit) != 0ull;
        const unsigned long long h = any ? wave_max_u64(ahit ? acc : 0ull) : 0ull;
        finish(orow, any, h);
        acc = 0ull;
        ahit = false;
      }
      if (rpos == rlast) {
        // ---- the step lies in one row: fold into the running maximum
        const unsigned v = (unsigned)(R0 + rpos);
        unsigned long long hv[kUIt];
#pragma unroll
        for (int j = 0; j < kUIt; ++j) hv[j] = keep(edge_hash(S, v, (unsigned)cv.c[j]));
#pragma unroll
        for (int j = 0; j < kUIt; ++j) {
          const int x = kUIt * lane + j;
          const bool ok = x >= xlo && x < xhi && (unsigned)cv.c[j] < (unsigned)n;
          acc = ok && hv[j] > acc ? hv[j] : acc;
          ahit = ahit || ok;
        }
        orow = R0 + rpos;
      } else {
        // ---- rows from the boundary markers (all zero between steps)
        {
          // row R0 + lane + 1 starts at ce; only the last of several rows
          // starting there (the others are empty) marks it
          const long long cn = (long long)(((unsigned long long)dpp_wave_shl1((unsigned)((unsigned long long)ce >> 32), 0u) << 32) |
                                           dpp_wave_shl1((unsigned)ce, 0u));
          const bool last_start = lane == 63 || cn > ce;
          if (ce > pos && ce < se && last_start) sm.mark[(int)(ce - s)] = (unsigned)(lane + 2);
        }
        wave_lds_sync();
        unsigned m[kUIt];
#pragma unroll
        for (int j = 0; j < kUIt; j += 4) {
          const uint4 mk = *reinterpret_cast<const uint4*>(&sm.mark[kUIt * lane + j]);
          m[j] = mk.x;
          m[j + 1] = mk.y;
          m[j + 2] = mk.z;
          m[j + 3] = mk.w;
          *reinterpret_cast<uint4*>(&sm.mark[kUIt * lane + j]) = make_uint4(0u, 0u, 0u, 0u);  // (the lane's own)
        }
#pragma unroll
        for (int j = 1; j < kUIt; ++j) m[j] = max(m[j], m[j - 1]);
        const unsigned incl = wave_incl_max_u32(m[kUIt - 1]);
        const unsigned excl = dpp_wave_shr1(incl, 0u);
        int rr[kUIt];
        unsigned long long hv[kUIt];
        bool okv[kUIt];
#pragma unroll
        for (int j = 0; j < kUIt; ++j) {
          const unsigned mm = max(excl, m[j]);
          rr[j] = max(rpos, (int)mm - 1);  // window row of the entry
          const int x = kUIt * lane + j;
          okv[j] = x >= xlo && x < xhi && (unsigned)cv.c[j] < (unsigned)n;
          hv[j] = keep(edge_hash(S, (unsigned)(R0 + rr[j]), (unsigned)cv.c[j]));
        }
        // Runs of one row among the lane's entries (rows never decrease along
        // them). The lane's running maximum from earlier steps heads the
        // first run (it belongs to the row of pos, which ends in this step;
        // it is empty when that row began at pos). Every run but the one of the
        // step's last row, which stays open in the registers, ends in an LDS
        // atomic max on its row's slot; lanes with nothing to add write their
        // own dummy slot instead, so no branch splits the wave.
        const int dummy = kUSlots + lane;
        unsigned long long rm = acc;  // the current run's largest hash
        bool rh = ahit;               // the current run has one
        int prow = rpos;              // the current run's row
#pragma unroll
        for (int j = 0; j < kUIt; ++j) {
          const bool same = rr[j] == prow;
          const bool fl = !same && rh;  // the run before entry j ends (its row < rlast)
          atomicMax(&sm.slot[fl ? prow : dummy], rm);
          sm.hit[fl ? prow : dummy] = 1u;
          rm = same ? rm : 0ull;
          rh = same && rh;
          rm = okv[j] && hv[j] > rm ? hv[j] : rm;
          rh = rh || okv[j];
          prow = rr[j];
        }
        const bool lastopen = prow == rlast;
        {
          const bool fl = !lastopen && rh;
          atomicMax(&sm.slot[fl ? prow : dummy], rm);
          sm.hit[fl ? prow : dummy] = 1u;
        }
        const unsigned long long accl = lastopen ? rm : 0ull;
        const bool hitl = lastopen && rh;
        wave_lds_sync();
        // rows of the window that ended inside the step: rpos .. rlast - 1
        if (rpos < rlast) {
          // (the row of pos finishes here when the step goes past it)
          const bool mine = lane >= rpos && lane < rlast;
          const bool any = mine && sm.hit[lane] != 0u;
          const unsigned long long h = any ? sm.slot[lane] : 0ull;
          const long long r = R0 + lane;
          const bool firstcut = r == v0 && cut_left;
          if (any && !firstcut) C[r] = hash_neighbour(h, S, (unsigned)r);
          if (__ballot(mine && firstcut) != 0ull) {  // v0 is in this window: its part
            const int l0 = (int)(v0 - R0);
            const bool a0 = __builtin_amdgcn_readlane((int)(any ? 1 : 0), l0) != 0;
            const unsigned long long h0 =
                ((unsigned long long)(unsigned)__builtin_amdgcn_readlane((int)(unsigned)(h >> 32), l0) << 32) |
                (unsigned)__builtin_amdgcn_readlane((int)(unsigned)h, l0);
            pf = unw_part(v0, 0, a0, h0, S);
          }
          sm.slot[mine ? lane : kUSlots + lane] = 0ull;
          sm.hit[mine ? lane : kUSlots + lane] = 0u;
        }
        wave_lds_sync();  // the cleared slots before the next step's atomics
        acc = accl;
        ahit = hitl;
        orow = R0 + rlast;
      }
      pos = se;
    };
    bool fastA = VEC && (pos & ~3ll) + kUStep <= nnz, fastB = false;
    UnwCols bufA = VEC ? unw_load_vec(col, fastA ? pos & ~3ll : 0ll) : unw_load_slow(col, pos & ~3ll, nnz), bufB;
    for (;;) {
      step(bufA, fastA, bufB, fastB);
      if (pos >= E1) break;
      step(bufB, fastB, bufA, fastA);
      if (pos >= E1) break;
    }
    // the row open at the range's end
    const bool any = __ballot(ahit) != 0ull;
    const unsigned long long h = any ? wave_max_u64(ahit ? acc : 0ull) : 0ull;
    const long long er = rp[orow + 1];
    const bool cl = orow == v0 && cut_left;
    if (er > E1) {  // it goes on past the range
      const Part p = unw_part(orow, cl ? kPartSingle : 0, any, h, S);
      if (cl) pf = p;
      else pl = p;
    } else {
      finish(orow, any, h);
    }
  }
  if (lane == 0) {
    a.parts[2 * b] = pf;
    a.parts[2 * b + 1] = pl;
  }
}

}  // namespace

template <bool UNW, bool MULTI>
__global__ __launch_bounds__(kBlock) void k_first_csr(StreamArgs a) {
  __shared__ FirstSmem sm;
  if (threadIdx.x == 0) sm.err = a.c.totals->err;
  __syncthreads();
  if (sm.err) return;
  Ctl ctl = *a.in.ctl;
  if (ctl.Pf > 0) ctl.P = ctl.Pf;  // the first argmax's own split of R_1
  const unsigned long long S = cand_seed(a.c.gseed[0], a.c.renew, a.cand_phase);
  const bool vec = (((unsigned long long)a.in.col | (UNW ? 0ull : (unsigned long long)a.in.w)) & 15ull) == 0ull;
  for (int b = blockIdx.x; b < ctl.P; b += gridDim.x) first_range<UNW, MULTI>(a, ctl, b, sm, S, vec);
}

template <bool UNW, bool MULTI>
static hipError_t launch_first_csr_t(const StreamArgs& a, int grid, hipStream_t s, hipEvent_t* ev) {
  const auto kern = k_first_csr<UNW, MULTI>;
  if (ev) hipExtLaunchKernelGGL(kern, dim3(grid), dim3(kBlock), 0, s, ev[0], ev[1], 0, a);
  else hipLaunchKernelGGL(kern, dim3(grid), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_first_csr(const StreamArgs& a, int grid, hipStream_t s, bool unweighted, hipEvent_t* ev) {
  const bool multi = a.c.graphs > 1;
  if (unweighted) return multi ? launch_first_csr_t<true, true>(a, grid, s, ev) : launch_first_csr_t<true, false>(a, grid, s, ev);
  return multi ? launch_first_csr_t<false, true>(a, grid, s, ev) : launch_first_csr_t<false, false>(a, grid, s, ev);
}

// A failed solve, or a guarded launch whose phases the device tail took over.
__device__ __forceinline__ bool wave_failed(const Common& c) {
  return (c.totals->err | ((c.guard && c.totals->tail_from) ? 0x80000000u : 0u)) != 0u;
}

template <bool VEC>
__global__ __launch_bounds__(64, 8) void k_first_unw(StreamArgs a) {  // 8 waves per SIMD
  __shared__ UnwSmem sm;
  if (wave_failed(a.c)) return;
  Ctl ctl = *a.in.ctl;
  const int P = ctl.Pf > 0 ? ctl.Pf : ctl.P;  // the first argmax's own split of R_1
  const unsigned long long S = cand_seed(a.c.gseed[0], a.c.renew, a.cand_phase);
  for (int i = lane_id(); i < kUSlots; i += 64) {
    sm.slot[i] = 0ull;
    sm.hit[i] = 0u;
  }
  for (int i = lane_id(); i < kUStep; i += 64) sm.mark[i] = 0u;
  __syncthreads();
  for (int b = blockIdx.x; b < P; b += gridDim.x) unw_range<VEC>(a, ctl, P, b, sm, S);
}

// vec_ok: the entry array is 16-byte aligned and holds at least kUStep
// entries (what a step's placeholder load reads).
hipError_t launch_first_unw(const StreamArgs& a, int grid, hipStream_t s, bool vec_ok, hipEvent_t* ev) {
  if (vec_ok) {
    if (ev) hipExtLaunchKernelGGL(k_first_unw<true>, dim3(grid), dim3(64), 0, s, ev[0], ev[1], 0, a);
    else hipLaunchKernelGGL(k_first_unw<true>, dim3(grid), dim3(64), 0, s, a);
  } else {
    if (ev) hipExtLaunchKernelGGL(k_first_unw<false>, dim3(grid), dim3(64), 0, s, ev[0], ev[1], 0, a);
    else hipLaunchKernelGGL(k_first_unw<false>, dim3(grid), dim3(64), 0, s, a);
  }
  return hipGetLastError();
}

int first_unw_min_entries() { return kUStep; }

// kUnwPerCu, or fewer if the kernels' registers leave fewer waves resident
// (every range's wave is resident from the start).
int first_unw_ranges_per_cu() {
  int n1 = 0, n0 = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n1, k_first_unw<true>, 64, 0) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&n0, k_first_unw<false>, 64, 0) != hipSuccess) {
    (void)hipGetLastError();
    return 1;
  }
  return std::max(1, std::min(kUnwPerCu, std::min(n1, n0)));
}

// (the fewer of the one-graph and the batch instantiations)
int first_csr_blocks_per_cu(bool unweighted) {
  int n1 = 0, n2 = 0;
  const hipError_t e =
      unweighted ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&n1, (k_first_csr<true, false>), kBlock, 0)
                 : hipOccupancyMaxActiveBlocksPerMultiprocessor(&n1, (k_first_csr<false, false>), kBlock, 0);
  const hipError_t e2 =
      unweighted ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&n2, (k_first_csr<true, true>), kBlock, 0)
                 : hipOccupancyMaxActiveBlocksPerMultiprocessor(&n2, (k_first_csr<false, true>), kBlock, 0);
  if (e != hipSuccess || e2 != hipSuccess) {
    (void)hipGetLastError();
    return 1;
  }
  return std::max(1, std::min(n1, n2));
}

}  // namespace lm
