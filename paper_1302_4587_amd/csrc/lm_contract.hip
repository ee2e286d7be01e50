// Contraction of a graph by a matching (the coarsening step of multilevel
// partitioning, which contracts maximal matchings: Section 1 of the paper;
// its Section 3.1 runs local max on graph-contraction instances), gfx950.
//
// Result (lm_contract in lm.h): every matched pair {a, b}, a < b, and every
// free vertex a becomes one coarse vertex; coarse ids follow the smaller
// fine id (cmap); coarse row c lists each coarse neighbour once, in the
// order in which its first fine entry appears when a's row and then b's row
// are read; the weight of a coarse edge is the fp32 sum of the fine edges it
// merges (at most four in a simple graph) added in increasing order of the
// fine edge (min end, max end), the same order from both sides.
//
// Work: (1) a scan over the fine vertices numbers the pairs (cmap); (2) every
// coarse row whose bound deg(a) + deg(b) is at most kCS is merged in LDS: a
// workgroup takes the coarse rows of a range of fine vertices in tiles of at
// most kCT entries, maps each entry's neighbour through cmap, and groups the
// entries of one coarse neighbour in the row's own slots of an LDS hash
// table, with a list per slot; the first entry of a group (in row order)
// keeps it with the group's sum, and the kept entries are written compacted
// at the start of their fine row part. (3) Longer rows get a hash table of
// their own in device memory and the same grouping over all their entries at
// once. (4) A scan over the coarse rows gives their offsets and the kept
// entries are copied out in order. The fine graph's entries are read once;
// cmap is gathered once per entry.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <mutex>

#include "lm.h"
#include "lm_device.h"
#include "lm_internal.h"
#include "lm_runtime.h"

namespace lm {

namespace {

constexpr int kCV = 16;                 // fine vertices per lane in the numbering scans
constexpr int kCBlockV = kBlock * kCV;  // fine vertices per scan block
constexpr int kCT = 1024;               // tile capacity in entries
constexpr int kCS = 512;                // largest coarse-row bound merged in LDS
constexpr int kCStep = kCT - kCS;       // tiles take the rows that start in a window of this many entries
constexpr int kCTI = kCT / kBlock;      // tile entries per lane
constexpr int kCMaxDup = 4;             // fine edges one coarse edge merges at most in a simple graph
constexpr int kCCost = 4;               // cost of a fine vertex when ranges are split (entries cost 1)
constexpr int kCTopThreads = 1024;
constexpr int kCPackGrid = 4096;
constexpr unsigned long long kEmpty = ~0ull;
constexpr int kLB = 512;      // average entries of a long row's bucket
constexpr int kLBCap = 1024;  // entries a bucket may hold in LDS (more: the table path)
constexpr int kLC = 8192;     // entries of a long row per counting / scatter chunk
constexpr int kLHist = 4096;  // buckets a row may have for the chunks' LDS histograms

constexpr unsigned kCErrMate = 1u;    // mate is not an involution with -1 for free vertices
constexpr unsigned kCErrRowPtr = 2u;  // row_ptr is not a valid offset array
constexpr unsigned kCErrCol = 4u;     // a neighbour id outside [0, n)
constexpr unsigned kCErrDup = 8u;     // more than four fine edges in one coarse edge: duplicate entries

struct CTot {
  unsigned err;
  unsigned pad;
  long long nc;            // coarse vertices
  long long nnz_c;         // coarse entries
  long long nlong;         // coarse rows merged through device-memory tables
  long long long_entries;  // the sum of their bounds
  long long long_slots;    // hash slots their tables take
  long long long_buckets;  // LDS-sized buckets their entries are sorted into
  long long long_chunks;   // row-aligned chunks of kLC entries
  long long long_kept;     // their entries that are not the matched edge
  unsigned overflow;       // a bucket outgrew LDS: the long rows take the table path
  unsigned pad2;
};

struct LongRow {
  int a, b, c, dega;
  int ub;     // deg(a) + deg(b)
  int tbits;  // table of 2^tbits slots
  int nb;     // buckets of the row (about kLB entries each)
  int pad;
  long long eoff;  // first flat index of the row's entries among all long rows
  long long toff;  // first slot of its table
  long long boff;  // first bucket of the row
  long long coff;  // first chunk of the row (kLC entries each)
};

struct CArgs {
  long long n, nnz;
  const long long* rp;
  const int* col;
  const float* w;  // nullptr: every edge weighs 1
  const int* mate;
  const long long* vw;  // nullptr: every vertex weighs 1
  int* cmap;
  int* crep;  // coarse vertex -> its smaller fine vertex
  int* cnt;   // fine vertex -> coarse entries kept from its row part
  long long* cvw;  // nullptr: not wanted
  long long* bsum;
  CTot* tot;
  int2* scr;  // per fine entry: (coarse neighbour, summed weight bits) if kept, else (-1, 0)
  int* next;  // per fine entry of a long row: the previous entry of its table slot's list
  LongRow* lrows;
  long long lrow_cap;
  int2* table;  // (key, list head) per slot of the long rows' tables
  long long* bstart;  // per bucket: entry count, then (scanned) first record
  int* bfill;         // per bucket: records placed so far
  int* rec;           // fine entry indices of the long rows, grouped by bucket
  long long* crp;
  int* ccol;
  float* cw;
  int dup_limit;  // fine edges one coarse edge may merge (4; 1 for the duplicate check)
  int identity;   // every vertex free, cmap the identity (the duplicate check of LM_CHECK_GRAPH)
};

__device__ __forceinline__ unsigned long long tbl_hash(int d, int bits) {
  return (unsigned long long)(((unsigned)d * 0x9E3779B1u) >> (32 - bits));
}

// Exclusive prefix sum over a workgroup of kCTopThreads lanes.
__device__ __forceinline__ long long top_excl_sum(long long x, long long* sm, long long& total) {
  const long long incl = wave_incl_sum<long long>(x);
  if (lane_id() == 63) sm[wave_id()] = incl;
  __syncthreads();
  long long pre = 0, tot = 0;
#pragma unroll
  for (int i = 0; i < kCTopThreads / 64; ++i) {
    const long long v = sm[i];
    pre += (i < wave_id()) ? v : 0ll;
    tot += v;
  }
  __syncthreads();
  total = tot;
  return pre + incl - x;
}

// (1a) Checks mate and row_ptr and counts the pairs' smaller ends per block
// (vertex base + i * kBlock + lane: coalesced).
__global__ __launch_bounds__(kBlock) void k_c_count(CArgs a) {
  __shared__ long long sm[kWaves];
  const long long base = (long long)blockIdx.x * kCBlockV;
  unsigned err = 0;
  long long reps = 0;
  for (int i = 0; i < kCV; ++i) {
    const long long v = base + (long long)i * kBlock + threadIdx.x;
    if (v >= a.n) break;
    const int m = a.identity ? -1 : a.mate[v];
    if (m != -1) {
      if (m < 0 || m >= a.n || m == v)
        err |= kCErrMate;
      else if (a.mate[m] != (int)v)
        err |= kCErrMate;
    }
    reps += (m == -1 || v < m) ? 1 : 0;
    const long long r0 = a.rp[v], r1 = a.rp[v + 1];
    if (r1 < r0 || (v == 0 && r0 != 0) || (v == a.n - 1 && r1 != a.nnz)) err |= kCErrRowPtr;
  }
  long long total;
  (void)block_excl_sum<long long>(reps, sm, total);
  if (threadIdx.x == 0) a.bsum[blockIdx.x] = total;
  if (err) atomicOr(&a.tot->err, err);
}

// (1b, 4b) Exclusive scan of m block sums in place, one workgroup; the total
// goes to *total.
__global__ __launch_bounds__(kCTopThreads) void k_c_scan_top(long long* v, long long m, long long* total) {
  __shared__ long long sm[kCTopThreads / 64];
  long long carry = 0;
  for (long long base = 0; base < m; base += kCTopThreads) {
    const long long i = base + threadIdx.x;
    const long long x = i < m ? v[i] : 0ll;
    long long t;
    const long long e = top_excl_sum(x, sm, t);
    if (i < m) v[i] = carry + e;
    carry += t;
  }
  if (threadIdx.x == 0) *total = carry;
}

// In-place exclusive scan of a long array in three steps: per-workgroup sums
// of kSBlock consecutive values (k_c_scan_sums), the one-workgroup scan of
// those sums (k_c_scan_top), and each workgroup's scan from its prefix
// (k_c_scan_apply). A lane takes kSI consecutive values.
constexpr int kSI = 8;
constexpr int kSBlock = kBlock * kSI;

__global__ __launch_bounds__(kBlock) void k_c_scan_sums(const long long* v, long long m, long long* bs) {
  __shared__ long long sm[kWaves];
  const long long i0 = (long long)blockIdx.x * kSBlock + (long long)threadIdx.x * kSI;
  long long x = 0;
#pragma unroll
  for (int j = 0; j < kSI; ++j) x += i0 + j < m ? v[i0 + j] : 0ll;
  long long tot;
  (void)block_excl_sum<long long>(x, sm, tot);
  if (threadIdx.x == 0) bs[blockIdx.x] = tot;
}

__global__ __launch_bounds__(kBlock) void k_c_scan_apply(long long* v, long long m, const long long* bs) {
  __shared__ long long sm[kWaves];
  const long long i0 = (long long)blockIdx.x * kSBlock + (long long)threadIdx.x * kSI;
  long long x[kSI], s = 0;
#pragma unroll
  for (int j = 0; j < kSI; ++j) {
    x[j] = i0 + j < m ? v[i0 + j] : 0ll;
    s += x[j];
  }
  long long tot;
  long long run = bs[blockIdx.x] + block_excl_sum<long long>(s, sm, tot);
#pragma unroll
  for (int j = 0; j < kSI; ++j) {
    if (i0 + j < m) v[i0 + j] = run;
    run += x[j];
  }
}

// Exclusive prefix, in index order, of the kCBlockV values a block staged in
// val[] (value of index base + i * kBlock + lane at val[i * kBlock + lane]):
// every lane sums kCV consecutive values, the lanes are scanned, and val[]
// receives the prefixes. Returns the block total.
__device__ __forceinline__ long long block_stage_scan(long long* val, long long start, long long* sm) {
  long long s = 0;
  for (int j = 0; j < kCV; ++j) s += val[threadIdx.x * kCV + j];
  long long total;
  long long run = start + block_excl_sum<long long>(s, sm, total);  // ends after a barrier
  for (int j = 0; j < kCV; ++j) {
    const long long x = val[threadIdx.x * kCV + j];
    val[threadIdx.x * kCV + j] = run;
    run += x;
  }
  __syncthreads();
  return total;
}

// (1c) Numbers the coarse vertices, writes cmap, the coarse vertex weights,
// and clears the per-row-part counts.
__global__ __launch_bounds__(kBlock) void k_c_map(CArgs a) {
  __shared__ long long val[kCBlockV];
  __shared__ long long sm[kWaves];
  if (a.tot->err) return;
  const long long base = (long long)blockIdx.x * kCBlockV;
  int mm[kCV];
#pragma unroll
  for (int i = 0; i < kCV; ++i) {
    const long long v = base + (long long)i * kBlock + threadIdx.x;
    int m = -2, f = 0;
    if (v < a.n) {
      m = a.mate[v];
      f = (m == -1 || v < m) ? 1 : 0;
      a.cnt[v] = 0;
    }
    mm[i] = m;
    val[i * kBlock + threadIdx.x] = f;
  }
  __syncthreads();
  (void)block_stage_scan(val, a.bsum[blockIdx.x], sm);
#pragma unroll
  for (int i = 0; i < kCV; ++i) {
    const long long v = base + (long long)i * kBlock + threadIdx.x;
    const int m = mm[i];
    if (v >= a.n || !(m == -1 || v < m)) continue;
    const int c = (int)val[i * kBlock + threadIdx.x];
    a.cmap[v] = c;
    a.crep[c] = (int)v;
    if (m >= 0) a.cmap[m] = c;
    if (a.cvw) a.cvw[c] = (a.vw ? a.vw[v] : 1ll) + (m >= 0 ? (a.vw ? a.vw[m] : 1ll) : 0ll);
  }
}

// A fine vertex as the head of a coarse row.
struct RowHead {
  bool rep, lng;
  int m, c, dega, ub;
  long long ka, kb;
};
__device__ __forceinline__ RowHead row_head(const CArgs& a, long long v) {
  RowHead h;
  h.m = a.identity ? -1 : a.mate[v];
  h.rep = (h.m == -1 || v < h.m);
  h.c = 0;
  h.dega = h.ub = 0;
  h.ka = h.kb = 0;
  h.lng = false;
  if (h.rep) {
    h.c = a.identity ? (int)v : a.cmap[v];
    h.ka = a.rp[v];
    h.dega = (int)(a.rp[v + 1] - h.ka);
    h.ub = h.dega;
    if (h.m >= 0) {
      h.kb = a.rp[h.m];
      h.ub += (int)(a.rp[h.m + 1] - h.kb);
    }
    h.lng = h.ub > kCS;
  }
  return h;
}

// The fine vertices [vb, ve) of workgroup blockIdx.x: ranges split by
// entries plus kCCost per vertex.
__device__ __forceinline__ void wg_vertices(const CArgs& a, long long per_wg, long long& vb, long long& ve, int* lb) {
  const long long C = a.nnz + (long long)kCCost * a.n;
  const long long c0 = (long long)blockIdx.x * per_wg;
  const long long c1 = c0 + per_wg;
  vb = c0 >= C ? a.n
               : block_lower_bound(0, a.n + 1, [&](long long v) { return a.rp[v] + (long long)kCCost * v >= c0; },
                                   lb);
  ve = c1 >= C ? a.n
               : block_lower_bound(0, a.n + 1, [&](long long v) { return a.rp[v] + (long long)kCCost * v >= c1; },
                                   lb);
}

struct GroupSmem {
  int skey[2 * kCT];      // coarse neighbour of the slot, -1 if free
  int shead[2 * kCT];     // last tile position inserted into the slot's list
  int erank[kCT + 1];     // coarse neighbour, then exclusive rank among the kept entries
  short enext[kCT];
  short eslot[kCT];
  unsigned char erow[kCT];
  int st[kBlock + 1];  // chunk-local start of each row's entries; st[kBlock] = chunk total
  int ra[kBlock], rb[kBlock], rc[kBlock], rdega[kBlock], rut[kBlock];
  long long rka[kBlock], rkb[kBlock];
  int wcnt[kCTI * kWaves];
  int smi[kWaves];
  int lb[1];
};

// Last row r of the chunk with st[r] <= pos (rows with no tile entries share
// their start with the next row, so r is the row that holds pos).
__device__ __forceinline__ int row_of(const int* st, int pos) {
  int lo = 0, hi = kBlock;  // st[lo] <= pos; answer in [lo, hi)
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (st[mid] <= pos)
      lo = mid;
    else
      hi = mid;
  }
  return lo;
}
// Start of the first row whose start is at least t (the chunk total if none).
__device__ __forceinline__ int start_at(const int* st, int t) {
  if (st[0] >= t) return st[0];
  int lo = 0, hi = kBlock;  // st[lo] < t; smallest r in (lo, kBlock] with st[r] >= t
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (st[mid] >= t)
      hi = mid;
    else
      lo = mid;
  }
  return st[hi];
}

// Sums the fine edges of one group in increasing (min end, max end).
// Sums the n <= 4 fine edges of one group in increasing (min end, max end):
// slots n..3 hold ord = ~0 and sort last; a fixed sorting network keeps every
// index static (no dynamic register indexing).
static_assert(kCMaxDup == 4, "the sorting network below is for four slots");
__device__ __forceinline__ void cswap(unsigned long long& oa, float& wa, unsigned long long& ob, float& wb) {
  if (ob < oa) {
    const unsigned long long t = oa;
    oa = ob;
    ob = t;
    const float u = wa;
    wa = wb;
    wb = u;
  }
}
__device__ __forceinline__ float group_sum(unsigned long long* ord, float* wv, int n) {
  cswap(ord[0], wv[0], ord[1], wv[1]);
  cswap(ord[2], wv[2], ord[3], wv[3]);
  cswap(ord[0], wv[0], ord[2], wv[2]);
  cswap(ord[1], wv[1], ord[3], wv[3]);
  cswap(ord[1], wv[1], ord[2], wv[2]);
  float sum = wv[0];
  if (n > 1) sum += wv[1];
  if (n > 2) sum += wv[2];
  if (n > 3) sum += wv[3];
  return sum;
}

__device__ __forceinline__ unsigned long long edge_order(int s, int x) {
  return ((unsigned long long)(unsigned)min(s, x) << 32) | (unsigned)max(s, x);
}

constexpr int kWT = 256;           // wave tile capacity in entries
constexpr int kWS = 64;            // largest coarse-row bound one wave merges alone
constexpr int kWStep = kWT - kWS;  // wave tiles take the rows that start in a window of this many entries
constexpr int kWTI = kWT / 64;     // tile entries per lane

struct WaveSmem {
  int skey[2 * kWT];   // coarse neighbour of the slot, -1 if free
  int shead[2 * kWT];  // last tile position inserted into the slot's list
  short enext[kWT];
  short eslot[kWT];
  unsigned char erow[kWT];
  int st[65];  // wave-local start of each lane's row; st[64] = the wave's total
  int ra[64], rb[64], rc[64], rdega[64], rut[64];
  int rrk[64][2];  // kept entries of the tile before the row's a part and b part
  int rka[64], rkb[64];  // the row parts' first entries (nnz < 2^31: five workgroups fit a CU)
};

// Orders the wave's LDS accesses across lanes (a wave's LDS operations are
// performed in order; this keeps the compiler from moving them).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// Start of the first of the wave's rows whose start is at least t (the
// wave's total if none).
__device__ __forceinline__ int wstart_at(const int* st, int t) {
  if (st[0] >= t) return st[0];
  int lo = 0, hi = 64;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (st[mid] >= t)
      hi = mid;
    else
      lo = mid;
  }
  return st[hi];
}
__device__ __forceinline__ int wrow_of(const int* st, int pos) {
  int lo = 0, hi = 64;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (st[mid] <= pos)
      lo = mid;
    else
      hi = mid;
  }
  return lo;
}

// (2a) The coarse rows with bound <= kWS, one wave at a time with no
// workgroup barrier: each wave takes 64 fine vertices of every chunk of its
// workgroup's range, lays their rows out back to back and groups them in
// wave tiles of at most kWT entries (the same grouping as k_c_group, in the
// wave's own LDS); ranks in row order come from the tile's ballots.
__global__ __launch_bounds__(kBlock) void k_c_group_wave(CArgs a, long long per_wg) {
  __shared__ WaveSmem wsm[kWaves];
  __shared__ int lb[1];
  if (a.tot->err & (kCErrMate | kCErrRowPtr)) return;
  long long vb, ve;
  wg_vertices(a, per_wg, vb, ve, lb);
  WaveSmem& sm = wsm[wave_id()];
  const int l = lane_id();
  for (int i = l; i < 2 * kWT; i += 64) {
    sm.skey[i] = -1;
    sm.shead[i] = -1;
  }
  wave_sync();
  unsigned err = 0;
  for (long long cb = vb + (long long)wave_id() * 64; cb < ve; cb += kBlock) {
    const long long v = cb + l;
    RowHead h;
    h.rep = false;
    h.lng = false;
    h.m = -1;
    h.c = h.dega = h.ub = 0;
    h.ka = h.kb = 0;
    if (v < ve) h = row_head(a, v);
    const int ut = (h.rep && !h.lng && h.ub <= kWS) ? h.ub : 0;
    const int incl = wave_incl_sum<int>(ut);
    const int U = __shfl(incl, 63);
    sm.st[l] = incl - ut;
    if (l == 63) sm.st[64] = U;
    sm.ra[l] = (int)v;
    sm.rb[l] = h.m;
    sm.rc[l] = h.c;
    sm.rdega[l] = h.dega;
    sm.rut[l] = ut;
    sm.rka[l] = (int)h.ka;
    sm.rkb[l] = (int)h.kb;
    wave_sync();
    const int ntile = (U + kWStep - 1) / kWStep;
    for (int j = 0; j < ntile; ++j) {
      const int lo = wstart_at(sm.st, j * kWStep);
      const int hi = wstart_at(sm.st, (j + 1) * kWStep);
      const int len = hi - lo;
      if (len <= 0) continue;
      int Dr[kWTI], xr[kWTI], rr[kWTI];
      float wr[kWTI];
      long long kr[kWTI];
      // 1: load every entry of the lane, then map them all, then insert
#pragma unroll
      for (int i = 0; i < kWTI; ++i) {
        const int q = i * 64 + l;
        rr[i] = 0;
        kr[i] = -1;
        Dr[i] = -1;
        xr[i] = 0;
        wr[i] = 0.f;
        if (q < len) {
          const int pos = lo + q;
          const int r = wrow_of(sm.st, pos);
          const int off = pos - sm.st[r];
          const bool side = off >= sm.rdega[r];
          rr[i] = r;
          kr[i] = side ? sm.rkb[r] + (off - sm.rdega[r]) : sm.rka[r] + off;
          sm.erow[q] = (unsigned char)r;
        }
      }
#pragma unroll
      for (int i = 0; i < kWTI; ++i) {
        if (kr[i] < 0) continue;
        xr[i] = a.col[kr[i]];
        wr[i] = a.w ? a.w[kr[i]] : 1.0f;
      }
#pragma unroll
      for (int i = 0; i < kWTI; ++i) {
        if (kr[i] < 0) continue;
        if ((unsigned)xr[i] >= (unsigned)a.n)
          err |= kCErrCol;
        else
          Dr[i] = a.identity ? xr[i] : a.cmap[xr[i]];
      }
#pragma unroll
      for (int i = 0; i < kWTI; ++i) {
        const int q = i * 64 + l;
        const int r = rr[i];
        if (kr[i] < 0) continue;
        if (Dr[i] == sm.rc[r]) Dr[i] = -1;
        const int D = Dr[i];
        if (D >= 0) {
          const unsigned sb = 2u * (unsigned)(sm.st[r] - lo);
          const unsigned range = 2u * (unsigned)sm.rut[r];
          unsigned hh = (unsigned)(((unsigned long long)((unsigned)D * 0x9E3779B1u) * range) >> 32);
          for (;;) {
            const int old = atomicCAS(&sm.skey[sb + hh], -1, D);
            if (old == -1 || old == D) break;
            hh = hh + 1 == range ? 0u : hh + 1;
          }
          sm.eslot[q] = (short)(sb + hh);
          sm.enext[q] = (short)atomicExch(&sm.shead[sb + hh], q);
        }
      }
      wave_sync();
      // 2: the first entry of every group keeps it, with the group's sum
      bool keep[kWTI];
      float sumr[kWTI];
      unsigned long long bal[kWTI];
#pragma unroll
      for (int i = 0; i < kWTI; ++i) {
        const int q = i * 64 + l;
        keep[i] = false;
        sumr[i] = 0.f;
        if (q < len && Dr[i] >= 0) {
          int lst[kCMaxDup + 1];
          int nl = 0;
          int p = sm.shead[sm.eslot[q]];
          bool first = true;
#pragma unroll
          for (int t = 0; t <= kCMaxDup; ++t) {  // static indices: at most five nodes matter
            if (p >= 0) {
              lst[t] = p;
              nl = t + 1;
              first = first && p >= q;
              p = sm.enext[p];
            }
          }
          if (nl > a.dup_limit) err |= kCErrDup;
          if (first && nl <= a.dup_limit) {
            keep[i] = true;
            const int r = rr[i];
            if (nl == 1) {
              sumr[i] = wr[i];
            } else {
              unsigned long long ord[kCMaxDup];
              float wg[kCMaxDup];
#pragma unroll
              for (int t = 0; t < kCMaxDup; ++t) {
                ord[t] = ~0ull;
                wg[t] = 0.f;
                if (t >= nl) continue;
                const int pp = lst[t];
                const int off = lo + pp - sm.st[r];
                const bool side = off >= sm.rdega[r];
                const int s = side ? sm.rb[r] : sm.ra[r];
                int xp = xr[i];
                float wp = wr[i];
                if (pp != q) {
                  const long long kp = side ? sm.rkb[r] + (off - sm.rdega[r]) : sm.rka[r] + off;
                  xp = a.col[kp];
                  wp = a.w ? a.w[kp] : 1.0f;
                }
                ord[t] = edge_order(s, xp);
                wg[t] = wp;
              }
              sumr[i] = group_sum(ord, wg, nl);
            }
          }
        }
        bal[i] = __ballot(keep[i]);
      }
      // 3: kept entries before a tile position, from the ballots: every row's
      // lane finds its parts' starts, every kept entry its own rank
      int pre[kWTI];
      pre[0] = 0;
#pragma unroll
      for (int i = 1; i < kWTI; ++i) pre[i] = pre[i - 1] + (int)__popcll(bal[i - 1]);
      auto rank_at = [&](int pos) -> int {  // any tile position (row lanes only)
        const int ri = pos >> 6;
        int base = pre[kWTI - 1] + (int)__popcll(bal[kWTI - 1]);
        unsigned long long b = 0ull;
#pragma unroll
        for (int t = 0; t < kWTI; ++t)
          if (t == ri) {
            base = pre[t];
            b = bal[t];
          }
        return base + (int)__popcll(b & ((1ull << (pos & 63)) - 1ull));
      };
      const bool row_here = sm.rut[l] > 0 && sm.st[l] >= lo && sm.st[l] < hi;
      if (row_here) {
        const int s0 = sm.st[l] - lo;
        const int r0 = rank_at(s0), rb_ = rank_at(s0 + sm.rdega[l]);
        sm.rrk[l][0] = r0;
        sm.rrk[l][1] = rb_;
        if (a.cnt) {
          a.cnt[sm.ra[l]] = rb_ - r0;
          if (sm.rb[l] >= 0) a.cnt[sm.rb[l]] = rank_at(s0 + sm.rut[l]) - rb_;
        }
      }
      wave_sync();
      if (a.scr) {
#pragma unroll
        for (int i = 0; i < kWTI; ++i) {
          const int q = i * 64 + l;
          if (q >= len || !keep[i]) continue;
          const int r = rr[i];
          const int off = lo + q - sm.st[r];
          const bool side = off >= sm.rdega[r];
          const int own = pre[i] + (int)__popcll(bal[i] & lanemask_lt());
          a.scr[(side ? sm.rkb[r] : sm.rka[r]) + (own - sm.rrk[r][side ? 1 : 0])] =
              make_int2(Dr[i], __float_as_int(sumr[i]));
        }
      }
      for (int i = l; i < 2 * len; i += 64) {
        sm.skey[i] = -1;
        sm.shead[i] = -1;
      }
      wave_sync();
    }
    wave_sync();
  }
  if (err) atomicOr(&a.tot->err, err);
}

// (2b) Groups the entries of every medium coarse row (kWS < bound <= kCS) in LDS and
// keeps, compacted in place at the start of each row part, the first entry of
// every group with the group's sum; sets the parts' kept counts. Queues the
// long rows.
__global__ __launch_bounds__(kBlock) void k_c_group(CArgs a, long long per_wg) {
  __shared__ GroupSmem sm;
  if (a.tot->err & (kCErrMate | kCErrRowPtr)) return;
  const int tid = threadIdx.x;
  const int wv_id = wave_id();
  long long vb, ve;
  wg_vertices(a, per_wg, vb, ve, sm.lb);
  for (int i = tid; i < 2 * kCT; i += kBlock) {
    sm.skey[i] = -1;
    sm.shead[i] = -1;
  }
  unsigned err = 0;
  for (long long cb = vb; cb < ve; cb += kBlock) {
    const long long v = cb + tid;
    RowHead h;
    h.rep = false;
    h.lng = false;
    h.m = -1;
    h.c = h.dega = h.ub = 0;
    h.ka = h.kb = 0;
    if (v < ve) {
      h = row_head(a, v);
      if (h.rep && h.lng) {
        const unsigned long long idx = atomicAdd((unsigned long long*)&a.tot->nlong, 1ull);
        if ((long long)idx < a.lrow_cap) {
          LongRow L;
          L.a = (int)v;
          L.b = h.m;
          L.c = h.c;
          L.dega = h.dega;
          L.ub = h.ub;
          L.tbits = 0;
          L.eoff = 0;
          L.toff = 0;
          a.lrows[idx] = L;
        }
      }
    }
    const int ut = (h.rep && !h.lng && h.ub > kWS) ? h.ub : 0;  // shorter rows: k_c_group_wave
    int U;
    const int st = block_excl_sum<int>(ut, sm.smi, U);
    sm.st[tid] = st;
    if (tid == 0) sm.st[kBlock] = U;
    sm.ra[tid] = (int)v;
    sm.rb[tid] = h.m;
    sm.rc[tid] = h.c;
    sm.rdega[tid] = h.dega;
    sm.rut[tid] = ut;
    sm.rka[tid] = h.ka;
    sm.rkb[tid] = h.kb;
    __syncthreads();
    const int ntile = (U + kCStep - 1) / kCStep;
    for (int j = 0; j < ntile; ++j) {
      const int lo = start_at(sm.st, j * kCStep);
      const int hi = start_at(sm.st, (j + 1) * kCStep);
      const int len = hi - lo;
      if (len <= 0) continue;  // uniform across the workgroup
      int Dr[kCTI], xr[kCTI];
      float wr[kCTI];
      // 1: load every entry of the lane, then map them all, then insert (the
      // loads of all rounds are in flight together)
      int rr[kCTI];
      long long kr[kCTI];
#pragma unroll
      for (int i = 0; i < kCTI; ++i) {
        const int q = i * kBlock + tid;
        rr[i] = 0;
        kr[i] = -1;
        Dr[i] = -1;
        xr[i] = 0;
        wr[i] = 0.f;
        if (q < len) {
          const int pos = lo + q;
          const int r = row_of(sm.st, pos);
          const int off = pos - sm.st[r];
          const bool side = off >= sm.rdega[r];
          rr[i] = r;
          kr[i] = side ? sm.rkb[r] + (off - sm.rdega[r]) : sm.rka[r] + off;
          sm.erow[q] = (unsigned char)r;
        }
      }
#pragma unroll
      for (int i = 0; i < kCTI; ++i) {
        if (kr[i] < 0) continue;
        xr[i] = a.col[kr[i]];
        wr[i] = a.w ? a.w[kr[i]] : 1.0f;
      }
#pragma unroll
      for (int i = 0; i < kCTI; ++i) {
        if (kr[i] < 0) continue;
        if ((unsigned)xr[i] >= (unsigned)a.n)
          err |= kCErrCol;
        else
          Dr[i] = a.identity ? xr[i] : a.cmap[xr[i]];
      }
#pragma unroll
      for (int i = 0; i < kCTI; ++i) {
        const int q = i * kBlock + tid;
        const int r = rr[i];
        if (kr[i] < 0) continue;
        if (Dr[i] == sm.rc[r]) Dr[i] = -1;
        const int D = Dr[i];
        if (D >= 0) {
          // the row's own slots: 2 * (its bound) of them from 2 * (its tile start)
          const unsigned sb = 2u * (unsigned)(sm.st[r] - lo);
          const unsigned range = 2u * (unsigned)sm.rut[r];
          unsigned hh = (unsigned)(((unsigned long long)((unsigned)D * 0x9E3779B1u) * range) >> 32);
          for (;;) {
            const int old = atomicCAS(&sm.skey[sb + hh], -1, D);
            if (old == -1 || old == D) break;
            hh = hh + 1 == range ? 0u : hh + 1;
          }
          sm.eslot[q] = (short)(sb + hh);
          sm.enext[q] = (short)atomicExch(&sm.shead[sb + hh], q);
        }
      }
      __syncthreads();
      // 2: the first entry of every group keeps it, with the group's sum
      bool keep[kCTI];
      float sumr[kCTI];
#pragma unroll
      for (int i = 0; i < kCTI; ++i) {
        const int q = i * kBlock + tid;
        keep[i] = false;
        sumr[i] = 0.f;
        if (q < len && Dr[i] >= 0) {
          int lst[kCMaxDup + 1];
          int nl = 0;
          int p = sm.shead[sm.eslot[q]];
          bool first = true;
#pragma unroll
          for (int t = 0; t <= kCMaxDup; ++t) {  // static indices: at most five nodes matter
            if (p >= 0) {
              lst[t] = p;
              nl = t + 1;
              first = first && p >= q;
              p = sm.enext[p];
            }
          }
          if (nl > a.dup_limit) err |= kCErrDup;
          if (first && nl <= a.dup_limit) {
            keep[i] = true;
            const int r = sm.erow[q];
            if (nl == 1) {
              sumr[i] = wr[i];
            } else {
              unsigned long long ord[kCMaxDup];
              float wg[kCMaxDup];
#pragma unroll
              for (int t = 0; t < kCMaxDup; ++t) {
                ord[t] = ~0ull;
                wg[t] = 0.f;
                if (t >= nl) continue;
                const int pp = lst[t];
                const int off = lo + pp - sm.st[r];
                const bool side = off >= sm.rdega[r];
                const int s = side ? sm.rb[r] : sm.ra[r];
                int xp = xr[i];
                float wp = wr[i];
                if (pp != q) {
                  const long long kp = side ? sm.rkb[r] + (off - sm.rdega[r]) : sm.rka[r] + off;
                  xp = a.col[kp];
                  wp = a.w ? a.w[kp] : 1.0f;
                }
                ord[t] = edge_order(s, xp);
                wg[t] = wp;
              }
              sumr[i] = group_sum(ord, wg, nl);
            }
          }
        }
        const unsigned long long bal = __ballot(keep[i]);
        if (lane_id() == 0) sm.wcnt[i * kWaves + wv_id] = __popcll(bal);
        sm.erank[q] = (int)__popcll(bal & lanemask_lt());  // rank inside the wave for now
      }
      __syncthreads();
      // 3: exclusive ranks in tile order: the kept counts of the (round, wave)
      // groups are scanned across the wave's lanes, each lane takes its groups'
      {
        static_assert(kCTI * kWaves <= 64, "one lane per (round, wave) group");
        const int l = lane_id();
        const int cg = l < kCTI * kWaves ? sm.wcnt[l] : 0;
        const int incl = wave_incl_sum<int>(cg);
        const int excl = incl - cg;
        const int tot = __shfl(incl, kCTI * kWaves - 1);
#pragma unroll
        for (int i = 0; i < kCTI; ++i) {
          const int q = i * kBlock + tid;
          sm.erank[q] += __shfl(excl, i * kWaves + wv_id);
        }
        if (tid == 0) sm.erank[kCT] = tot;
      }
      __syncthreads();
      // 4: write the kept entries at the start of their row part; part counts
#pragma unroll
      for (int i = 0; i < kCTI; ++i) {
        const int q = i * kBlock + tid;
        if (q >= len || !keep[i] || !a.scr) continue;
        const int r = sm.erow[q];
        const int off = lo + q - sm.st[r];
        const bool side = off >= sm.rdega[r];
        const int ps = sm.st[r] - lo + (side ? sm.rdega[r] : 0);
        const int prank = sm.erank[q] - sm.erank[ps];
        a.scr[(side ? sm.rkb[r] : sm.rka[r]) + prank] = make_int2(Dr[i], __float_as_int(sumr[i]));
      }
      {
        const int r = tid;
        const int s0 = sm.st[r] - lo;
        if (a.cnt && sm.rut[r] > 0 && sm.st[r] >= lo && sm.st[r] < hi) {
          const int pb = s0 + sm.rdega[r];
          const int pe = s0 + sm.rut[r];
          const int rb_ = pe < len ? sm.erank[pe] : sm.erank[kCT];
          const int ra_ = pb < len ? sm.erank[pb] : sm.erank[kCT];
          a.cnt[sm.ra[r]] = ra_ - sm.erank[s0];
          if (sm.rb[r] >= 0) a.cnt[sm.rb[r]] = rb_ - ra_;
        }
      }
      for (int i = tid; i < 2 * len; i += kBlock) {
        sm.skey[i] = -1;
        sm.shead[i] = -1;
      }
      __syncthreads();
    }
  }
  if (err) atomicOr(&a.tot->err, err);
}

// (4d) Copies the kept entries of every short coarse row from the starts of
// its two row parts to the output.
__global__ __launch_bounds__(kBlock) void k_c_copy(CArgs a, long long per_wg) {
  __shared__ int pre[kBlock + 1];
  __shared__ int sca[kBlock];
  __shared__ long long ska[kBlock], skb[kBlock], sd0[kBlock];
  __shared__ int smi[kWaves];
  __shared__ int lb[1];
  if (a.tot->err) return;
  const int tid = threadIdx.x;
  long long vb, ve;
  wg_vertices(a, per_wg, vb, ve, lb);
  for (long long cb = vb; cb < ve; cb += kBlock) {
    const long long v = cb + tid;
    int len = 0, ca = 0;
    long long ka = 0, kb = 0, d0 = 0;
    if (v < ve) {
      const RowHead h = row_head(a, v);
      if (h.rep && !h.lng) {
        ca = a.cnt[v];
        len = ca + (h.m >= 0 ? a.cnt[h.m] : 0);
        ka = h.ka;
        kb = h.kb;
        d0 = a.crp[h.c];
      }
    }
    int T;
    const int p = block_excl_sum<int>(len, smi, T);
    pre[tid] = p;
    if (tid == 0) pre[kBlock] = T;
    sca[tid] = ca;
    ska[tid] = ka;
    skb[tid] = kb;
    sd0[tid] = d0;
    __syncthreads();
    for (int q = tid; q < T; q += kBlock) {
      const int r = row_of(pre, q);
      const int off = q - pre[r];
      const long long src = off < sca[r] ? ska[r] + off : skb[r] + (off - sca[r]);
      const int2 t = a.scr[src];
      a.ccol[sd0[r] + off] = t.x;
      a.cw[sd0[r] + off] = __int_as_float(t.y);
    }
    __syncthreads();
  }
}

// (3a') Sizes of the long rows: entries (their bound), table slots (the
// power of two at least twice the bound), buckets and chunks, and the
// offsets of each in row order. Workgroup g sums kLPRows rows
// (k_c_long_sums), one scan over the workgroup sums per quantity gives the
// totals (k_c_scan_top), and each workgroup writes its rows' offsets from its
// prefix (k_c_long_offs). The grid covers the row capacity; workgroups past
// the long rows counted write zero sums.
constexpr int kLP = 4;                 // long rows per lane in the prep kernels
constexpr int kLPRows = kBlock * kLP;  // long rows per workgroup

__device__ __forceinline__ void long_row_sizes(long long ub, int& bits, long long v[4]) {
  const long long t = 2 * ub;
  bits = t <= 2 ? 1 : 64 - __clzll((unsigned long long)(t - 1));  // smallest bits >= 1 with 2^bits >= 2 ub
  v[0] = ub;
  v[1] = 1ll << bits;
  v[2] = (ub + kLB - 1) / kLB;
  v[3] = (ub + kLC - 1) / kLC;
}

__global__ __launch_bounds__(kBlock) void k_c_long_sums(CArgs a, long long* lsum, long long nblk) {
  __shared__ long long sm[kWaves];
  const long long nl = a.tot->err ? 0 : (a.tot->nlong < a.lrow_cap ? a.tot->nlong : a.lrow_cap);
  long long su[4] = {0, 0, 0, 0};
  const long long i0 = (long long)blockIdx.x * kLPRows + (long long)threadIdx.x * kLP;
#pragma unroll
  for (int j = 0; j < kLP; ++j) {
    if (i0 + j >= nl) continue;
    int bits;
    long long v[4];
    long_row_sizes(a.lrows[i0 + j].ub, bits, v);
#pragma unroll
    for (int q = 0; q < 4; ++q) su[q] += v[q];
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    long long tot;
    (void)block_excl_sum<long long>(su[q], sm, tot);
    if (threadIdx.x == 0) lsum[q * nblk + blockIdx.x] = tot;
  }
}

__global__ __launch_bounds__(kBlock) void k_c_long_offs(CArgs a, const long long* lsum, long long nblk) {
  __shared__ long long sm[kWaves];
  if (a.tot->err) return;
  const long long nl = a.tot->nlong < a.lrow_cap ? a.tot->nlong : a.lrow_cap;
  if ((long long)blockIdx.x * kLPRows >= nl) return;  // (uniform)
  const long long i0 = (long long)blockIdx.x * kLPRows + (long long)threadIdx.x * kLP;
  int bits[kLP];
  long long v[kLP][4];
  long long su[4] = {0, 0, 0, 0};
#pragma unroll
  for (int j = 0; j < kLP; ++j) {
    bits[j] = 1;
#pragma unroll
    for (int q = 0; q < 4; ++q) v[j][q] = 0;
    if (i0 + j < nl) long_row_sizes(a.lrows[i0 + j].ub, bits[j], v[j]);
#pragma unroll
    for (int q = 0; q < 4; ++q) su[q] += v[j][q];
  }
  long long off[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    long long tot;
    off[q] = lsum[q * nblk + blockIdx.x] + block_excl_sum<long long>(su[q], sm, tot);
  }
#pragma unroll
  for (int j = 0; j < kLP; ++j) {
    if (i0 + j < nl) {
      LongRow& L = a.lrows[i0 + j];
      L.eoff = off[0];
      L.toff = off[1];
      L.tbits = bits[j];
      L.nb = (int)v[j][2];
      L.boff = off[2];
      L.coff = off[3];
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) off[q] += v[j][q];
  }
}

__global__ __launch_bounds__(kBlock) void k_c_fill(int2* t, long long m) {
  for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < m; i += (long long)gridDim.x * kBlock)
    t[i] = make_int2(-1, -1);
}

// The long row holding flat index i (largest eoff <= i).
__device__ __forceinline__ long long long_row_of(const LongRow* L, long long nl, long long i) {
  long long lo = 0, hi = nl;
  while (hi - lo > 1) {
    const long long mid = (lo + hi) >> 1;
    if (L[mid].eoff <= i)
      lo = mid;
    else
      hi = mid;
  }
  return lo;
}

// The long row of flat index i, searched forward from r0 (the row of the
// chunk's first index; rows are longer than a chunk's lane stride).
__device__ __forceinline__ long long long_row_from(const LongRow* L, long long nl, long long r0, long long i) {
  long long r = r0;
  while (r + 1 < nl && L[r + 1].eoff <= i) ++r;
  return r;
}

constexpr int kLI = 4;  // long-row entries per lane per round (their loads are in flight together)

// Where flat long-row index i lies: its row, fine entry and side.
struct LongAt {
  long long k;
  int r, off;
  bool side;
};
__device__ __forceinline__ LongAt long_at(const CArgs& a, long long nl, long long r0, long long i) {
  LongAt t;
  t.r = (int)long_row_from(a.lrows, nl, r0, i);
  const LongRow& L = a.lrows[t.r];
  t.off = (int)(i - L.eoff);
  t.side = t.off >= L.dega;
  t.k = t.side ? a.rp[L.b] + (t.off - L.dega) : a.rp[L.a] + t.off;
  return t;
}

// (3b) Inserts every entry of the long rows into its row's table.
__global__ __launch_bounds__(kBlock) void k_c_long_insert(CArgs a, long long nl, long long total) {
  unsigned err = 0;
  const long long step = (long long)gridDim.x * kBlock * kLI;
  for (long long i0 = (long long)blockIdx.x * kBlock * kLI; i0 < total; i0 += step) {
    const long long r0 = long_row_of(a.lrows, nl, i0);
    LongAt at[kLI];
    int x[kLI], D[kLI];
#pragma unroll
    for (int j = 0; j < kLI; ++j) {
      const long long i = i0 + (long long)j * kBlock + threadIdx.x;
      at[j].k = -1;
      if (i < total) at[j] = long_at(a, nl, r0, i);
    }
#pragma unroll
    for (int j = 0; j < kLI; ++j) x[j] = at[j].k >= 0 ? a.col[at[j].k] : -1;
#pragma unroll
    for (int j = 0; j < kLI; ++j) {
      D[j] = -1;
      if (at[j].k < 0) continue;
      if ((unsigned)x[j] >= (unsigned)a.n)
        err |= kCErrCol;
      else
        D[j] = a.identity ? x[j] : a.cmap[x[j]];
    }
#pragma unroll
    for (int j = 0; j < kLI; ++j) {
      if (D[j] < 0) continue;
      const LongRow& L = a.lrows[at[j].r];
      if (D[j] == L.c) continue;
      int2* tb = a.table + L.toff;
      const unsigned long long mask = (1ull << L.tbits) - 1;
      unsigned long long h = tbl_hash(D[j], L.tbits);
      for (;;) {
        const int old = atomicCAS(&tb[h].x, -1, D[j]);
        if (old == -1 || old == D[j]) break;
        h = (h + 1) & mask;
      }
      a.next[at[j].k] = atomicExch(&tb[h].y, (int)at[j].k);
    }
  }
  if (err) atomicOr(&a.tot->err, err);
}

// (3c) The first entry of every group of a long row keeps the group's sum
// (written at its own fine entry; the others write -1).
__global__ __launch_bounds__(kBlock) void k_c_long_keep(CArgs a, long long nl, long long total) {
  unsigned err = 0;
  const long long step = (long long)gridDim.x * kBlock * kLI;
  for (long long i0 = (long long)blockIdx.x * kBlock * kLI; i0 < total; i0 += step) {
    const long long r0 = long_row_of(a.lrows, nl, i0);
    LongAt at[kLI];
    int x[kLI], D[kLI];
    float wself[kLI];
#pragma unroll
    for (int j = 0; j < kLI; ++j) {
      const long long i = i0 + (long long)j * kBlock + threadIdx.x;
      at[j].k = -1;
      if (i < total) at[j] = long_at(a, nl, r0, i);
    }
#pragma unroll
    for (int j = 0; j < kLI; ++j) {
      x[j] = at[j].k >= 0 ? a.col[at[j].k] : -1;
      wself[j] = at[j].k >= 0 && a.w ? a.w[at[j].k] : 1.0f;
    }
#pragma unroll
    for (int j = 0; j < kLI; ++j) {
      D[j] = -1;
      if (at[j].k >= 0 && (unsigned)x[j] < (unsigned)a.n) D[j] = a.identity ? x[j] : a.cmap[x[j]];
      if (D[j] >= 0 && D[j] == a.lrows[at[j].r].c) D[j] = -1;
    }
    int2 slot[kLI];
#pragma unroll
    for (int j = 0; j < kLI; ++j) {
      slot[j] = make_int2(-1, -1);
      if (D[j] < 0) continue;
      const LongRow& L = a.lrows[at[j].r];
      const int2* tb = a.table + L.toff;
      const unsigned long long mask = (1ull << L.tbits) - 1;
      unsigned long long h = tbl_hash(D[j], L.tbits);
      int2 t = tb[h];
      while (t.x != D[j]) {
        h = (h + 1) & mask;
        t = tb[h];
      }
      slot[j] = t;
    }
    int nxt[kLI];
#pragma unroll
    for (int j = 0; j < kLI; ++j) nxt[j] = D[j] >= 0 ? a.next[slot[j].y] : -1;
#pragma unroll
    for (int j = 0; j < kLI; ++j) {
      if (at[j].k < 0) continue;
      if (D[j] < 0) {
        if (a.scr) a.scr[at[j].k] = make_int2(-1, 0);
        continue;
      }
      const LongRow& L = a.lrows[at[j].r];
      const long long ka = a.rp[L.a];
      const long long kb = L.b >= 0 ? a.rp[L.b] : 0;
      // the group's entries; row order is a's part, then b's part
      int lst[kCMaxDup + 1];
      int nlst = 0;
      int p = slot[j].y;
      int pn = nxt[j];
      bool first = true;
#pragma unroll
      for (int t = 0; t <= kCMaxDup; ++t) {  // static indices: at most five nodes matter
        if (p < 0) continue;
        lst[t] = p;
        nlst = t + 1;
        const bool pa = (long long)p >= ka && (long long)p < ka + L.dega;
        const long long pos_p = pa ? p - ka : L.dega + (p - kb);
        first = first && pos_p >= at[j].off;
        p = pn;
        if (p >= 0 && t < kCMaxDup) pn = a.next[p];
      }
      if (nlst > a.dup_limit) err |= kCErrDup;
      if (!a.scr) continue;
      if (!first || nlst > a.dup_limit) {
        a.scr[at[j].k] = make_int2(-1, 0);
        continue;
      }
      float sum = wself[j];
      if (nlst > 1) {
        unsigned long long ord[kCMaxDup];
        float wv[kCMaxDup];
#pragma unroll
        for (int t = 0; t < kCMaxDup; ++t) {
          ord[t] = ~0ull;
          wv[t] = 0.f;
          if (t >= nlst) continue;
          const int pp = lst[t];
          const bool pa = (long long)pp >= ka && (long long)pp < ka + L.dega;
          const int sp = pa ? L.a : L.b;
          const int xp = pp == at[j].k ? x[j] : a.col[pp];
          ord[t] = edge_order(sp, xp);
          wv[t] = pp == at[j].k ? wself[j] : (a.w ? a.w[pp] : 1.0f);
        }
        sum = group_sum(ord, wv, nlst);
      }
      a.scr[at[j].k] = make_int2(D[j], __float_as_int(sum));
      atomicAdd(&a.cnt[at[j].side ? L.b : L.a], 1);
    }
  }
  if (err) atomicOr(&a.tot->err, err);
}

// ---- long rows through LDS buckets: every entry of a long row goes to one
// of the row's buckets by a hash of its coarse neighbour (so a group never
// spans buckets), the entries are sorted by bucket (counts, scan, scatter of
// fine entry indices), and one workgroup groups each bucket in LDS.

__device__ __forceinline__ long long bucket_of(const LongRow& L, int D) {
  return L.boff + (long long)(((unsigned long long)((unsigned)D * 0x9E3779B1u) * (unsigned)L.nb) >> 32);
}

struct ChunkSmem {
  int hist[kLHist];      // per bucket of the row: entries of the chunk, then their first record
  unsigned erec[kLC];    // per chunk entry: bucket << 13 | rank in the bucket within the chunk
  int row;
  int lb;
};
static_assert(kLC <= (1 << 13) && kLHist <= (1 << 19), "bucket and rank fit the packed word");

// Workgroup g of G takes the contiguous items [m g / G, m (g + 1) / G) (chunks
// or buckets, in row order), so the row of each item is found by walking on
// from the row of the one before (one step at most, mostly none); the first
// item's row comes from one 256-way search over the long rows. Every lane
// calls it.
template <typename Off>
__device__ __forceinline__ long long first_item_row(long long nl, long long c0, Off off, int* sm) {
  return block_lower_bound(0, nl, [&](long long i) { return off(i) > c0; }, sm) - 1;  // largest off <= c0
}

// (3b') Maps every long-row entry (its coarse neighbour into next[k], -1 for
// the matched edge, whose output is written as dropped now) and counts the
// buckets. A workgroup takes a chunk of kLC entries of one row at a time and
// counts in LDS, so each (chunk, bucket) costs one device atomic (rows with
// more than kLHist buckets count straight in device memory).
__global__ __launch_bounds__(kBlock) void k_c_lb_count(CArgs a, long long nl, long long nchunks) {
  struct CountSmem {
    int hist[kLHist];
    int row;
  };
  __shared__ CountSmem sm;
  unsigned err = 0;
  const int tid = threadIdx.x;
  // chunks taken in strides: those of rows counted in device memory come in
  // runs, which contiguous ranges would leave to a few workgroups
  for (long long c = blockIdx.x; c < nchunks; c += gridDim.x) {
    if (tid == 0) {  // the row: largest coff <= c
      long long lo = 0, hi = nl;
      while (hi - lo > 1) {
        const long long mid = (lo + hi) >> 1;
        if (a.lrows[mid].coff <= c)
          lo = mid;
        else
          hi = mid;
      }
      sm.row = (int)lo;
    }
    __syncthreads();
    const LongRow L = a.lrows[sm.row];
    const bool lds = L.nb <= kLHist;
    if (lds)
      for (int i = tid; i < L.nb; i += kBlock) sm.hist[i] = 0;
    __syncthreads();
    const long long e0 = (c - L.coff) * kLC;
    const int ne = (int)min((long long)kLC, (long long)L.ub - e0);
    const long long ka = a.rp[L.a];
    const long long kb = L.b >= 0 ? a.rp[L.b] : 0;
    for (int q0 = 0; q0 < ne; q0 += kBlock * kLI) {
      long long k[kLI];
      int x[kLI];
#pragma unroll
      for (int j = 0; j < kLI; ++j) {
        const int q = q0 + j * kBlock + tid;
        const long long off = e0 + q;
        k[j] = q < ne ? (off < L.dega ? ka + off : kb + (off - L.dega)) : -1;
      }
#pragma unroll
      for (int j = 0; j < kLI; ++j) x[j] = k[j] >= 0 ? a.col[k[j]] : -1;
#pragma unroll
      for (int j = 0; j < kLI; ++j) {
        if (k[j] < 0) continue;
        int D = -1;
        if ((unsigned)x[j] >= (unsigned)a.n)
          err |= kCErrCol;
        else
          D = a.identity ? x[j] : a.cmap[x[j]];
        if (D == L.c) D = -1;
        a.next[k[j]] = D;
        if (D < 0) {
          a.scr[k[j]] = make_int2(-1, 0);
          continue;
        }
        const long long bb = bucket_of(L, D);
        if (lds)
          atomicAdd(&sm.hist[bb - L.boff], 1);
        else
          atomicAdd((unsigned long long*)&a.bstart[bb], 1ull);
      }
    }
    __syncthreads();
    if (lds)
      for (int i = tid; i < L.nb; i += kBlock)
        if (sm.hist[i]) atomicAdd((unsigned long long*)&a.bstart[L.boff + i], (unsigned long long)sm.hist[i]);
    __syncthreads();
  }
  if (err) atomicOr(&a.tot->err, err);
}

// (3c') Places every mapped long-row entry's index in its bucket: per chunk,
// ranks within (chunk, bucket) from LDS atomics, one device atomic per
// (chunk, bucket) for the range, then the writes.
__global__ __launch_bounds__(kBlock) void k_c_lb_scatter(CArgs a, long long nl, long long nchunks) {
  __shared__ ChunkSmem sm;
  const int tid = threadIdx.x;
  const long long c0 = nchunks * blockIdx.x / gridDim.x, c1 = nchunks * (blockIdx.x + 1) / gridDim.x;
  if (c0 >= c1) return;  // (uniform)
  long long row = first_item_row(nl, c0, [&](long long i) { return a.lrows[i].coff; }, &sm.lb);
  for (long long c = c0; c < c1; ++c) {
    if (tid == 0) {
      while (row + 1 < nl && a.lrows[row + 1].coff <= c) ++row;
      sm.row = (int)row;
    }
    __syncthreads();
    const LongRow L = a.lrows[sm.row];
    const bool lds = L.nb <= kLHist;
    if (lds)
      for (int i = tid; i < L.nb; i += kBlock) sm.hist[i] = 0;
    __syncthreads();
    const long long e0 = (c - L.coff) * kLC;
    const int ne = (int)min((long long)kLC, (long long)L.ub - e0);
    const long long ka = a.rp[L.a];
    const long long kb = L.b >= 0 ? a.rp[L.b] : 0;
    auto kof = [&](int q) {
      const long long off = e0 + q;
      return off < L.dega ? ka + off : kb + (off - L.dega);
    };
    for (int q0 = 0; q0 < ne; q0 += kBlock * kLI) {
      int D[kLI];
#pragma unroll
      for (int j = 0; j < kLI; ++j) {
        const int q = q0 + j * kBlock + tid;
        D[j] = q < ne ? a.next[kof(q)] : -1;
      }
#pragma unroll
      for (int j = 0; j < kLI; ++j) {
        const int q = q0 + j * kBlock + tid;
        if (D[j] < 0) {
          if (lds && q < ne) sm.erec[q] = ~0u;  // the matched edge: no record
          continue;
        }
        const long long bb = bucket_of(L, D[j]);
        if (lds) {
          const int lb = (int)(bb - L.boff);
          sm.erec[q] = ((unsigned)lb << 13) | (unsigned)atomicAdd(&sm.hist[lb], 1);
        } else {
          a.rec[a.bstart[bb] + atomicAdd(&a.bfill[bb], 1)] = (int)kof(q);
        }
      }
    }
    if (lds) {
      __syncthreads();
      for (int i = tid; i < L.nb; i += kBlock) {
        const int h = sm.hist[i];
        if (h) sm.hist[i] = (int)(a.bstart[L.boff + i] + atomicAdd(&a.bfill[L.boff + i], h));
      }
      __syncthreads();
      for (int q = tid; q < ne; q += kBlock) {
        const unsigned r = sm.erec[q];
        if (r == ~0u) continue;
        a.rec[sm.hist[r >> 13] + (int)(r & 8191u)] = (int)kof(q);
      }
    }
    __syncthreads();
  }
}

// (an entry's index is not kept: it follows from its position in the row
// and the row's two offsets, which keeps five workgroups resident per CU)
struct BucketSmem {
  int skey[2 * kLBCap];
  int shead[2 * kLBCap];
  int epos[kLBCap];
  int eD[kLBCap];
  short enext[kLBCap];
  short eslot[kLBCap];
  int kept[2];
  int row;
  int lb;
};

// (3d') Groups every bucket in LDS, one workgroup per bucket at a time: the
// first entry of a group in row order keeps it with the group's sum (written
// at its fine entry), the others are written as dropped; the parts' kept
// counts grow by the bucket's. A bucket above kLBCap entries sets overflow.
__global__ __launch_bounds__(kBlock) void k_c_lb_group(CArgs a, long long nl, long long nbk) {
  __shared__ BucketSmem sm;
  const int tid = threadIdx.x;
  for (int i = tid; i < 2 * kLBCap; i += kBlock) {
    sm.skey[i] = -1;
    sm.shead[i] = -1;
  }
  unsigned err = 0;
  const long long b0 = nbk * blockIdx.x / gridDim.x, b1 = nbk * (blockIdx.x + 1) / gridDim.x;
  long long row = b0 < b1 ? first_item_row(nl, b0, [&](long long i) { return a.lrows[i].boff; }, &sm.lb) : 0;
  // Consecutive buckets mostly share a row: its record and row offsets are
  // reloaded only when the row changes, the next row's first bucket only when
  // it is passed (thread 0), and a bucket's start is the previous one's end.
  long long next_boff = row + 1 < nl ? a.lrows[row + 1].boff : nbk;
  int cur = -1;
  LongRow L;
  long long ka = 0, kb = 0;
  long long s1n = b0 < b1 ? a.bstart[b0] : 0;
  for (long long b = b0; b < b1; ++b) {
    const long long s0 = s1n, s1 = a.bstart[b + 1];
    s1n = s1;
    const int ne = (int)(s1 - s0);
    if (ne == 0) continue;  // uniform
    if (ne > kLBCap) {
      if (tid == 0) atomicOr(&a.tot->overflow, 1u);
      continue;
    }
    if (tid == 0) {  // the row: largest boff <= b
      while (next_boff <= b) {
        ++row;
        next_boff = row + 1 < nl ? a.lrows[row + 1].boff : nbk;
      }
      sm.row = (int)row;
      sm.kept[0] = sm.kept[1] = 0;
    }
    __syncthreads();
    if (sm.row != cur) {  // (uniform)
      cur = sm.row;
      L = a.lrows[cur];
      ka = a.rp[L.a];
      kb = L.b >= 0 ? a.rp[L.b] : 0;
    }
    for (int q = tid; q < ne; q += kBlock) {
      const int k = a.rec[s0 + q];
      const int D = a.next[k];
      const bool pa = (long long)k >= ka && (long long)k < ka + L.dega;
      sm.epos[q] = pa ? (int)(k - ka) : L.dega + (int)(k - kb);
      sm.eD[q] = D;
      const unsigned h0 = (unsigned)D * 0x85EBCA77u;
      unsigned hh = (h0 ^ (h0 >> 15)) & (2u * kLBCap - 1u);
      for (;;) {
        const int old = atomicCAS(&sm.skey[hh], -1, D);
        if (old == -1 || old == D) break;
        hh = (hh + 1) & (2u * kLBCap - 1u);
      }
      sm.eslot[q] = (short)hh;
      sm.enext[q] = (short)atomicExch(&sm.shead[hh], q);
    }
    __syncthreads();
    auto entry_of = [&](int pos) { return (int)(pos < L.dega ? ka + pos : kb + (pos - L.dega)); };
    for (int q = tid; q < ne; q += kBlock) {
      const int my = sm.epos[q];
      const int k = entry_of(my);
      int lst[kCMaxDup + 1];
      int nlst = 0;
      int p = sm.shead[sm.eslot[q]];
      bool first = true;
#pragma unroll
      for (int t = 0; t <= kCMaxDup; ++t) {
        if (p >= 0) {
          lst[t] = p;
          nlst = t + 1;
          first = first && sm.epos[p] >= my;
          p = sm.enext[p];
        }
      }
      if (nlst > a.dup_limit) err |= kCErrDup;
      if (!first || nlst > a.dup_limit) {
        a.scr[k] = make_int2(-1, 0);
        continue;
      }
      float sum;
      if (nlst == 1) {
        sum = a.w ? a.w[k] : 1.0f;
      } else {
        unsigned long long ord[kCMaxDup];
        float wv[kCMaxDup];
#pragma unroll
        for (int t = 0; t < kCMaxDup; ++t) {
          ord[t] = ~0ull;
          wv[t] = 0.f;
          if (t >= nlst) continue;
          const int pp = lst[t];
          const int kp = entry_of(sm.epos[pp]);
          const int sp = sm.epos[pp] < L.dega ? L.a : L.b;
          ord[t] = edge_order(sp, a.col[kp]);
          wv[t] = a.w ? a.w[kp] : 1.0f;
        }
        sum = group_sum(ord, wv, nlst);
      }
      a.scr[k] = make_int2(sm.eD[q], __float_as_int(sum));
      atomicAdd(&sm.kept[my < L.dega ? 0 : 1], 1);
    }
    __syncthreads();
    if (tid == 0) {
      if (sm.kept[0]) atomicAdd(&a.cnt[L.a], sm.kept[0]);
      if (sm.kept[1]) atomicAdd(&a.cnt[L.b], sm.kept[1]);
    }
    for (int q = tid; q < ne; q += kBlock) {
      sm.skey[sm.eslot[q]] = -1;
      sm.shead[sm.eslot[q]] = -1;
    }
    __syncthreads();
  }
  if (err) atomicOr(&a.tot->err, err);
}

// Clears the kept counts of the long rows' parts (before the table path
// redoes them after a bucket overflow).
__global__ __launch_bounds__(kBlock) void k_c_long_clear_cnt(CArgs a, long long nl) {
  for (long long r = (long long)blockIdx.x * kBlock + threadIdx.x; r < nl; r += (long long)gridDim.x * kBlock) {
    a.cnt[a.lrows[r].a] = 0;
    if (a.lrows[r].b >= 0) a.cnt[a.lrows[r].b] = 0;
  }
}

__device__ __forceinline__ long long coarse_deg(const CArgs& a, long long c) {
  const int r = a.crep[c];
  const int m = a.mate[r];
  return (long long)a.cnt[r] + (m >= 0 ? a.cnt[m] : 0);
}

// (4a) Coarse row lengths, summed per block (coalesced).
__global__ __launch_bounds__(kBlock) void k_c_deg_count(CArgs a, long long nc) {
  __shared__ long long sm[kWaves];
  if (a.tot->err) return;
  const long long base = (long long)blockIdx.x * kCBlockV;
  long long s = 0;
  for (int i = 0; i < kCV; ++i) {
    const long long c = base + (long long)i * kBlock + threadIdx.x;
    if (c >= nc) break;
    s += coarse_deg(a, c);
  }
  long long total;
  (void)block_excl_sum<long long>(s, sm, total);
  if (threadIdx.x == 0) a.bsum[blockIdx.x] = total;
}

// (4c) Coarse row offsets.
__global__ __launch_bounds__(kBlock) void k_c_deg_write(CArgs a, long long nc) {
  __shared__ long long val[kCBlockV];
  __shared__ long long sm[kWaves];
  if (a.tot->err) return;
  const long long base = (long long)blockIdx.x * kCBlockV;
#pragma unroll
  for (int i = 0; i < kCV; ++i) {
    const long long c = base + (long long)i * kBlock + threadIdx.x;
    val[i * kBlock + threadIdx.x] = c < nc ? coarse_deg(a, c) : 0ll;
  }
  __syncthreads();
  (void)block_stage_scan(val, a.bsum[blockIdx.x], sm);
#pragma unroll
  for (int i = 0; i < kCV; ++i) {
    const long long c = base + (long long)i * kBlock + threadIdx.x;
    if (c < nc) a.crp[c] = val[i * kBlock + threadIdx.x];
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) a.crp[nc] = a.tot->nnz_c;
}

// (4d) Packs the kept entries of every long row part in order, one
// workgroup per part at a time.
__global__ __launch_bounds__(kBlock) void k_c_long_pack(CArgs a, long long nl) {
  __shared__ int smi[kWaves];
  if (a.tot->err) return;
  for (long long pi = blockIdx.x; pi < 2 * nl; pi += gridDim.x) {
    const LongRow L = a.lrows[pi >> 1];
    const bool side = (pi & 1) != 0;
    if (side && L.b < 0) continue;
    const int s = side ? L.b : L.a;
    const long long k0 = a.rp[s];
    const long long len = a.rp[s + 1] - k0;
    long long dest = a.crp[L.c] + (side ? a.cnt[L.a] : 0);
    for (long long base = 0; base < len; base += kBlock) {
      const long long j = base + threadIdx.x;
      int2 t = make_int2(-1, 0);
      if (j < len) t = a.scr[k0 + j];
      const int f = t.x >= 0 ? 1 : 0;
      int tot;
      const int e = block_excl_sum<int>(f, smi, tot);
      if (f) {
        a.ccol[dest + e] = t.x;
        a.cw[dest + e] = __int_as_float(t.y);
      }
      dest += tot;
    }
  }
}

int lb_group_blocks_per_cu() {
  static int cached = 0;
  if (cached) return cached;
  int nb = 1;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_c_lb_group, kBlock, 0) != hipSuccess || nb < 1) nb = 1;
  cached = nb;
  return nb;
}

int wave_blocks_per_cu() {
  static int cached = 0;
  if (cached) return cached;
  int nb = 1;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_c_group_wave, kBlock, 0) != hipSuccess || nb < 1) nb = 1;
  cached = nb;
  return nb;
}

int tile_blocks_per_cu() {
  static int cached = 0;
  if (cached) return cached;
  int nb = 1;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_c_group, kBlock, 0) != hipSuccess || nb < 1) nb = 1;
  cached = nb;
  return nb;
}

size_t a256(size_t b) { return (b + 255) & ~(size_t)255; }

}  // namespace

// The long rows' sizes and offsets (k_c_long_sums, four top scans, k_c_long_offs)
// over a grid that covers lrow_cap rows; lsum holds 4 * long_prep_blocks(lrow_cap).
static long long long_prep_blocks(long long lrow_cap) { return std::max<long long>(1, (lrow_cap + kLPRows - 1) / kLPRows); }
static void launch_long_prep(const CArgs& a, long long* lsum, hipStream_t s) {
  const long long nblk = long_prep_blocks(a.lrow_cap);
  hipLaunchKernelGGL(k_c_long_sums, dim3((unsigned)nblk), dim3(kBlock), 0, s, a, lsum, nblk);
  long long* totals[4] = {&a.tot->long_entries, &a.tot->long_slots, &a.tot->long_buckets, &a.tot->long_chunks};
  for (int q = 0; q < 4; ++q)
    hipLaunchKernelGGL(k_c_scan_top, dim3(1), dim3(kCTopThreads), 0, s, lsum + q * nblk, nblk, totals[q]);
  hipLaunchKernelGGL(k_c_long_offs, dim3((unsigned)nblk), dim3(kBlock), 0, s, a, (const long long*)lsum, nblk);
}

// Exclusive scan of v[0, m) in place, its total to *total. Arrays above one
// top-scan round's worth take the three-step scan, with the workgroup sums
// in tmp (tmp_cap values; the one-workgroup scan when they would not fit).
static void launch_scan(long long* v, long long m, long long* total, long long* tmp, long long tmp_cap,
                        hipStream_t s) {
  const long long nb = (m + kSBlock - 1) / kSBlock;
  if (m <= 8 * kCTopThreads || nb > tmp_cap) {
    hipLaunchKernelGGL(k_c_scan_top, dim3(1), dim3(kCTopThreads), 0, s, v, m, total);
    return;
  }
  hipLaunchKernelGGL(k_c_scan_sums, dim3((unsigned)nb), dim3(kBlock), 0, s, (const long long*)v, m, tmp);
  hipLaunchKernelGGL(k_c_scan_top, dim3(1), dim3(kCTopThreads), 0, s, tmp, nb, total);
  hipLaunchKernelGGL(k_c_scan_apply, dim3((unsigned)nb), dim3(kBlock), 0, s, v, m, (const long long*)tmp);
}

// Buffers of the contraction, kept in the context between calls.
struct ContractState {
  DevBuf bsum, tot, crep, cnt, scr, next, lrows, table, bstart, bfill, rec, lsum;
  DevBuf in_rp, in_col, in_w, in_mate, in_vw, o_cmap, o_crp, o_ccol, o_cw, o_cvw;
  CTot* h_tot = nullptr;
};

void contract_release(Solver& S) {
  ContractState* cs = S.contract;
  if (!cs) return;
  DevBuf* all[] = {&cs->bsum,  &cs->tot,    &cs->crep,  &cs->cnt,  &cs->scr,     &cs->next,  &cs->lrows,
                   &cs->table, &cs->bstart, &cs->bfill, &cs->rec,  &cs->in_rp,   &cs->in_col, &cs->in_w,
                   &cs->in_mate, &cs->in_vw, &cs->o_cmap, &cs->o_crp, &cs->o_ccol, &cs->o_cw, &cs->o_cvw,
                   &cs->lsum};
  for (DevBuf* b : all) S.pool.release(*b);
  if (cs->h_tot) (void)hipHostFree(cs->h_tot);
  delete cs;
  S.contract = nullptr;
}

Solver& solver_of(lm_ctx* c);
std::mutex& mutex_of(lm_ctx* c);

// Duplicate entries within rows, for LM_CHECK_GRAPH on device input: the
// grouping kernels of the contraction with every vertex free and a group
// limit of one entry (any neighbour seen twice in a row is an error). Also
// checks row_ptr. Synchronises the stream.
lm_status check_row_duplicates(Solver& S, int64_t n, int64_t nnz, const long long* rp, const int* col,
                               hipStream_t s) {
  if (n == 0) return LM_OK;
  if (!S.contract) S.contract = new ContractState();
  ContractState& cs = *S.contract;
  if (!cs.h_tot && hipHostMalloc((void**)&cs.h_tot, sizeof(CTot), hipHostMallocDefault) != hipSuccess)
    return LM_ENOMEM;
  Pool& P = S.pool;
  const long long nb_v = (n + kCBlockV - 1) / kCBlockV;
  const long long lrow_cap = nnz / (kCS + 1) + 1;
  lm_status rs;
  if ((rs = P.reserve(cs.bsum, a256(sizeof(long long) * (size_t)(nb_v + 1)))) != LM_OK) return rs;
  if ((rs = P.reserve(cs.tot, a256(sizeof(CTot)))) != LM_OK) return rs;
  if ((rs = P.reserve(cs.lrows, a256(sizeof(LongRow) * (size_t)lrow_cap))) != LM_OK) return rs;
  if ((rs = P.reserve(cs.lsum, a256(sizeof(long long) * 4 * (size_t)long_prep_blocks(lrow_cap)))) != LM_OK) return rs;
  CArgs a;
  std::memset(&a, 0, sizeof(a));
  a.n = n;
  a.nnz = nnz;
  a.rp = rp;
  a.col = col;
  a.bsum = (long long*)cs.bsum.p;
  a.tot = (CTot*)cs.tot.p;
  a.lrows = (LongRow*)cs.lrows.p;
  a.lrow_cap = lrow_cap;
  a.dup_limit = 1;
  a.identity = 1;
  if (hipMemsetAsync(a.tot, 0, sizeof(CTot), s) != hipSuccess) return LM_EDEVICE;
  hipLaunchKernelGGL(k_c_count, dim3((unsigned)nb_v), dim3(kBlock), 0, s, a);
  const long long cost = nnz + (long long)kCCost * n;
  long long grid = (long long)S.num_cus * tile_blocks_per_cu();
  grid = std::max<long long>(1, std::min<long long>(grid, (cost + 2 * kCT - 1) / (2 * kCT)));
  // (each grouping kernel takes its own resident count of workgroups)
  const long long gw = std::max<long long>(
      1, std::min<long long>((long long)S.num_cus * wave_blocks_per_cu(), (cost + 2 * kCT - 1) / (2 * kCT)));
  hipLaunchKernelGGL(k_c_group_wave, dim3((unsigned)gw), dim3(kBlock), 0, s, a, (cost + gw - 1) / gw);
  hipLaunchKernelGGL(k_c_group, dim3((unsigned)grid), dim3(kBlock), 0, s, a, (cost + grid - 1) / grid);
  launch_long_prep(a, (long long*)cs.lsum.p, s);
  if (hipGetLastError() != hipSuccess) return LM_EDEVICE;
  if (hipMemcpyAsync(cs.h_tot, a.tot, sizeof(CTot), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return LM_EDEVICE;
  const CTot t1 = *cs.h_tot;
  if (t1.err) return LM_EGRAPH;
  if (t1.nlong > 0) {
    if (t1.nlong > lrow_cap) return LM_EDEVICE;
    if ((rs = P.reserve(cs.next, a256(sizeof(int) * (size_t)nnz))) != LM_OK) return rs;
    if ((rs = P.reserve(cs.table, a256(sizeof(int2) * (size_t)t1.long_slots))) != LM_OK) return rs;
    a.next = (int*)cs.next.p;
    a.table = (int2*)cs.table.p;
    const long long fill_grid = std::min<long long>((t1.long_slots + kBlock - 1) / kBlock, 8192);
    hipLaunchKernelGGL(k_c_fill, dim3((unsigned)fill_grid), dim3(kBlock), 0, s, a.table, t1.long_slots);
    const long long lg = std::min<long long>((t1.long_entries + kBlock * kLI - 1) / (kBlock * kLI), 16384);
    hipLaunchKernelGGL(k_c_long_insert, dim3((unsigned)lg), dim3(kBlock), 0, s, a, t1.nlong, t1.long_entries);
    hipLaunchKernelGGL(k_c_long_keep, dim3((unsigned)lg), dim3(kBlock), 0, s, a, t1.nlong, t1.long_entries);
    if (hipGetLastError() != hipSuccess) return LM_EDEVICE;
    if (hipMemcpyAsync(cs.h_tot, a.tot, sizeof(CTot), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return LM_EDEVICE;
    if (cs.h_tot->err) return LM_EGRAPH;
  }
  return LM_OK;
}

}  // namespace lm

using namespace lm;

#define LMC_TRY(x)                    \
  do {                                \
    const lm_status st_ = (x);        \
    if (st_ != LM_OK) return st_;     \
  } while (0)
#define LMC_HIP(x)                                \
  do {                                            \
    const hipError_t e_ = (x);                    \
    if (e_ != hipSuccess) return dev_status(e_);  \
  } while (0)

extern "C" {

lm_status lm_contract(lm_ctx* ctx, const lm_csr* g, const int32_t* mate, const int64_t* vwgt, int32_t* cmap,
                      lm_coarse* out, uint32_t flags, void* stream, lm_contract_stats* st) {
  if (!ctx || !g || !out) return LM_EINVAL;
  if (flags & ~(LM_IN_DEVICE | LM_OUT_DEVICE)) return LM_EINVAL;
  const int64_t n = g->n, nnz = g->nnz;
  if (n < 0 || nnz < 0) return LM_EINVAL;
  if (n >= ((int64_t)1 << 31) || nnz >= ((int64_t)1 << 31) - 65536) return LM_ETOOBIG;
  if (!g->row_ptr || !out->row_ptr) return LM_EINVAL;
  if (n > 0 && (!mate || !cmap)) return LM_EINVAL;
  if (nnz > 0 && (!g->col || !out->col || !out->w)) return LM_EINVAL;
  std::lock_guard<std::mutex> lk(mutex_of(ctx));
  Solver& S = solver_of(ctx);
  if (S.busy_server) return LM_EINVAL;
  if (st) std::memset(st, 0, sizeof(*st));
  out->n = 0;
  out->nnz = 0;
  if (hipSetDevice(S.dev) != hipSuccess) return LM_EDEVICE;
  if (S.async_pending) {
    if (hipEventSynchronize(S.e_async) != hipSuccess) return LM_EDEVICE;
    S.async_pending = false;
  }
  hipStream_t s = (hipStream_t)stream;
  const bool din = (flags & LM_IN_DEVICE) != 0, dout = (flags & LM_OUT_DEVICE) != 0;
  if (n == 0) {
    const int64_t zero = 0;
    if (dout) {
      LMC_HIP(hipMemcpyAsync(out->row_ptr, &zero, sizeof(zero), hipMemcpyHostToDevice, s));
      LMC_HIP(hipStreamSynchronize(s));
    } else {
      out->row_ptr[0] = 0;
    }
    return LM_OK;
  }
  if (!S.contract) S.contract = new ContractState();
  ContractState& cs = *S.contract;
  if (!cs.h_tot) LMC_HIP(hipHostMalloc((void**)&cs.h_tot, sizeof(CTot), hipHostMallocDefault));
  Pool& P = S.pool;
  const long long nb_v = (n + kCBlockV - 1) / kCBlockV;
  const long long lrow_cap = nnz / (kCS + 1) + 1;
  LMC_TRY(P.reserve(cs.bsum, a256(sizeof(long long) * (size_t)(nb_v + 1))));
  LMC_TRY(P.reserve(cs.tot, a256(sizeof(CTot))));
  LMC_TRY(P.reserve(cs.crep, a256(sizeof(int) * (size_t)n)));
  LMC_TRY(P.reserve(cs.cnt, a256(sizeof(int) * (size_t)n)));
  LMC_TRY(P.reserve(cs.scr, a256(sizeof(int2) * (size_t)(nnz > 0 ? nnz : 1))));
  LMC_TRY(P.reserve(cs.lrows, a256(sizeof(LongRow) * (size_t)lrow_cap)));
  LMC_TRY(P.reserve(cs.lsum, a256(sizeof(long long) * 4 * (size_t)long_prep_blocks(lrow_cap))));

  CArgs a;
  std::memset(&a, 0, sizeof(a));
  a.n = n;
  a.nnz = nnz;
  // inputs
  if (din) {
    a.rp = (const long long*)g->row_ptr;
    a.col = g->col;
    a.w = g->w;
    a.mate = mate;
    a.vw = (const long long*)vwgt;
  } else {
    LMC_TRY(P.reserve(cs.in_rp, a256(sizeof(int64_t) * (size_t)(n + 1))));
    LMC_TRY(P.reserve(cs.in_col, a256(sizeof(int32_t) * (size_t)(nnz > 0 ? nnz : 1))));
    LMC_TRY(P.reserve(cs.in_mate, a256(sizeof(int32_t) * (size_t)n)));
    LMC_HIP(hipMemcpyAsync(cs.in_rp.p, g->row_ptr, sizeof(int64_t) * (size_t)(n + 1), hipMemcpyHostToDevice, s));
    if (nnz > 0)
      LMC_HIP(hipMemcpyAsync(cs.in_col.p, g->col, sizeof(int32_t) * (size_t)nnz, hipMemcpyHostToDevice, s));
    LMC_HIP(hipMemcpyAsync(cs.in_mate.p, mate, sizeof(int32_t) * (size_t)n, hipMemcpyHostToDevice, s));
    a.rp = (const long long*)cs.in_rp.p;
    a.col = (const int*)cs.in_col.p;
    a.mate = (const int*)cs.in_mate.p;
    if (g->w) {
      LMC_TRY(P.reserve(cs.in_w, a256(sizeof(float) * (size_t)(nnz > 0 ? nnz : 1))));
      if (nnz > 0) LMC_HIP(hipMemcpyAsync(cs.in_w.p, g->w, sizeof(float) * (size_t)nnz, hipMemcpyHostToDevice, s));
      a.w = (const float*)cs.in_w.p;
    }
    if (vwgt) {
      LMC_TRY(P.reserve(cs.in_vw, a256(sizeof(int64_t) * (size_t)n)));
      LMC_HIP(hipMemcpyAsync(cs.in_vw.p, vwgt, sizeof(int64_t) * (size_t)n, hipMemcpyHostToDevice, s));
      a.vw = (const long long*)cs.in_vw.p;
    }
  }
  // outputs (host outputs go through device buffers of the worst-case size)
  if (dout) {
    a.cmap = cmap;
    a.crp = (long long*)out->row_ptr;
    a.ccol = out->col;
    a.cw = out->w;
    a.cvw = (long long*)out->vwgt;
  } else {
    LMC_TRY(P.reserve(cs.o_cmap, a256(sizeof(int32_t) * (size_t)n)));
    LMC_TRY(P.reserve(cs.o_crp, a256(sizeof(int64_t) * (size_t)(n + 1))));
    LMC_TRY(P.reserve(cs.o_ccol, a256(sizeof(int32_t) * (size_t)(nnz > 0 ? nnz : 1))));
    LMC_TRY(P.reserve(cs.o_cw, a256(sizeof(float) * (size_t)(nnz > 0 ? nnz : 1))));
    a.cmap = (int*)cs.o_cmap.p;
    a.crp = (long long*)cs.o_crp.p;
    a.ccol = (int*)cs.o_ccol.p;
    a.cw = (float*)cs.o_cw.p;
    if (out->vwgt) {
      LMC_TRY(P.reserve(cs.o_cvw, a256(sizeof(int64_t) * (size_t)n)));
      a.cvw = (long long*)cs.o_cvw.p;
    }
  }
  a.crep = (int*)cs.crep.p;
  a.cnt = (int*)cs.cnt.p;
  a.bsum = (long long*)cs.bsum.p;
  a.tot = (CTot*)cs.tot.p;
  a.scr = (int2*)cs.scr.p;
  a.lrows = (LongRow*)cs.lrows.p;
  a.lrow_cap = lrow_cap;
  a.dup_limit = kCMaxDup;
  a.identity = 0;

  LMC_HIP(hipEventRecord(S.e0, s));
  LMC_HIP(hipMemsetAsync(a.tot, 0, sizeof(CTot), s));
  hipLaunchKernelGGL(k_c_count, dim3((unsigned)nb_v), dim3(kBlock), 0, s, a);
  hipLaunchKernelGGL(k_c_scan_top, dim3(1), dim3(kCTopThreads), 0, s, a.bsum, nb_v, &a.tot->nc);
  hipLaunchKernelGGL(k_c_map, dim3((unsigned)nb_v), dim3(kBlock), 0, s, a);
  const long long cost = nnz + (long long)kCCost * n;
  long long grid = (long long)S.num_cus * tile_blocks_per_cu();
  const long long by_cost = (cost + 2 * kCT - 1) / (2 * kCT);
  if (grid > by_cost) grid = by_cost;
  if (grid < 1) grid = 1;
  const long long per_wg = (cost + grid - 1) / grid;
  // (each grouping kernel takes its own resident count of workgroups)
  const long long gw = std::max<long long>(1, std::min<long long>((long long)S.num_cus * wave_blocks_per_cu(), by_cost));
  hipLaunchKernelGGL(k_c_group_wave, dim3((unsigned)gw), dim3(kBlock), 0, s, a, (cost + gw - 1) / gw);
  hipLaunchKernelGGL(k_c_group, dim3((unsigned)grid), dim3(kBlock), 0, s, a, per_wg);
  launch_long_prep(a, (long long*)cs.lsum.p, s);
  LMC_HIP(hipGetLastError());
  LMC_HIP(hipMemcpyAsync(cs.h_tot, a.tot, sizeof(CTot), hipMemcpyDeviceToHost, s));
  LMC_HIP(hipStreamSynchronize(s));
  CTot t1 = *cs.h_tot;
  if (t1.err & kCErrMate) return LM_EINVAL;
  if (t1.err) return LM_EGRAPH;
  const long long nc = t1.nc;
  const long long nl = t1.nlong;
  if (nl > lrow_cap) return LM_EDEVICE;  // cannot happen: the bounds of the rows sum to nnz
  long long overflow_rows = 0;
  if (nl > 0) {
    // long rows: entries sorted into LDS-sized buckets by a hash of their
    // coarse neighbour, each bucket grouped in LDS by one workgroup
    const long long nbk = t1.long_buckets;
    LMC_TRY(P.reserve(cs.next, a256(sizeof(int) * (size_t)nnz)));
    LMC_TRY(P.reserve(cs.bstart, a256(sizeof(long long) * (size_t)(nbk + 1))));
    LMC_TRY(P.reserve(cs.bfill, a256(sizeof(int) * (size_t)nbk)));
    LMC_TRY(P.reserve(cs.rec, a256(sizeof(int) * (size_t)t1.long_entries)));
    a.next = (int*)cs.next.p;
    a.bstart = (long long*)cs.bstart.p;
    a.bfill = (int*)cs.bfill.p;
    a.rec = (int*)cs.rec.p;
    LMC_HIP(hipMemsetAsync(a.bstart, 0, sizeof(long long) * (size_t)(nbk + 1), s));
    LMC_HIP(hipMemsetAsync(a.bfill, 0, sizeof(int) * (size_t)nbk, s));
    const long long lg = std::min<long long>((t1.long_entries + kBlock * kLI - 1) / (kBlock * kLI), 16384);
    const long long nch = t1.long_chunks;
    const long long cgd = std::max<long long>(1, std::min<long long>(nch, (long long)S.num_cus * 8));
    hipLaunchKernelGGL(k_c_lb_count, dim3((unsigned)cgd), dim3(kBlock), 0, s, a, nl, nch);
    // (lsum is free again: the long rows' offsets are written)
    launch_scan(a.bstart, nbk + 1, &a.tot->long_kept, (long long*)cs.lsum.p, 4 * long_prep_blocks(lrow_cap), s);
    hipLaunchKernelGGL(k_c_lb_scatter, dim3((unsigned)cgd), dim3(kBlock), 0, s, a, nl, nch);
    // every workgroup resident: each takes one contiguous range of buckets
    const long long gg = std::max<long long>(1, std::min<long long>(nbk, (long long)S.num_cus * lb_group_blocks_per_cu()));
    hipLaunchKernelGGL(k_c_lb_group, dim3((unsigned)gg), dim3(kBlock), 0, s, a, nl, nbk);
    LMC_HIP(hipGetLastError());
    LMC_HIP(hipMemcpyAsync(cs.h_tot, a.tot, sizeof(CTot), hipMemcpyDeviceToHost, s));
    LMC_HIP(hipStreamSynchronize(s));
    if (cs.h_tot->err & kCErrMate) return LM_EINVAL;
    if (cs.h_tot->err) return LM_EGRAPH;
    if (cs.h_tot->overflow) {  // a bucket outgrew LDS: every long row through per-row tables
      overflow_rows = nl;
      LMC_TRY(P.reserve(cs.table, a256(sizeof(int2) * (size_t)t1.long_slots)));
      a.table = (int2*)cs.table.p;
      const long long cg = std::min<long long>((nl + kBlock - 1) / kBlock, 4096);
      hipLaunchKernelGGL(k_c_long_clear_cnt, dim3((unsigned)cg), dim3(kBlock), 0, s, a, nl);
      const long long fill_grid = std::min<long long>((t1.long_slots + kBlock - 1) / kBlock, 8192);
      hipLaunchKernelGGL(k_c_fill, dim3((unsigned)fill_grid), dim3(kBlock), 0, s, a.table, t1.long_slots);
      hipLaunchKernelGGL(k_c_long_insert, dim3((unsigned)lg), dim3(kBlock), 0, s, a, nl, t1.long_entries);
      hipLaunchKernelGGL(k_c_long_keep, dim3((unsigned)lg), dim3(kBlock), 0, s, a, nl, t1.long_entries);
    }
  }
  const long long nb_c = (nc + kCBlockV - 1) / kCBlockV;
  if (nb_c > 0) {
    hipLaunchKernelGGL(k_c_deg_count, dim3((unsigned)nb_c), dim3(kBlock), 0, s, a, nc);
    hipLaunchKernelGGL(k_c_scan_top, dim3(1), dim3(kCTopThreads), 0, s, a.bsum, nb_c, &a.tot->nnz_c);
    hipLaunchKernelGGL(k_c_deg_write, dim3((unsigned)nb_c), dim3(kBlock), 0, s, a, nc);
  }
  hipLaunchKernelGGL(k_c_copy, dim3((unsigned)grid), dim3(kBlock), 0, s, a, per_wg);
  if (nl > 0) {
    const long long pg = std::min<long long>(2 * nl, kCPackGrid);
    hipLaunchKernelGGL(k_c_long_pack, dim3((unsigned)pg), dim3(kBlock), 0, s, a, nl);
  }
  LMC_HIP(hipGetLastError());
  LMC_HIP(hipEventRecord(S.e1, s));
  LMC_HIP(hipMemcpyAsync(cs.h_tot, a.tot, sizeof(CTot), hipMemcpyDeviceToHost, s));
  LMC_HIP(hipStreamSynchronize(s));
  const CTot t2 = *cs.h_tot;
  if (t2.err & kCErrMate) return LM_EINVAL;
  if (t2.err) return LM_EGRAPH;
  const long long nnz_c = t2.nnz_c;
  if (!dout) {
    LMC_HIP(hipMemcpy(cmap, a.cmap, sizeof(int32_t) * (size_t)n, hipMemcpyDeviceToHost));
    LMC_HIP(hipMemcpy(out->row_ptr, a.crp, sizeof(int64_t) * (size_t)(nc + 1), hipMemcpyDeviceToHost));
    if (nnz_c > 0) {
      LMC_HIP(hipMemcpy(out->col, a.ccol, sizeof(int32_t) * (size_t)nnz_c, hipMemcpyDeviceToHost));
      LMC_HIP(hipMemcpy(out->w, a.cw, sizeof(float) * (size_t)nnz_c, hipMemcpyDeviceToHost));
    }
    if (out->vwgt) LMC_HIP(hipMemcpy(out->vwgt, a.cvw, sizeof(int64_t) * (size_t)nc, hipMemcpyDeviceToHost));
  }
  out->n = nc;
  out->nnz = nnz_c;
  if (st) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, S.e0, S.e1) == hipSuccess) st->device_ms = ms;
    const double eb = g->w ? 8.0 : 4.0;
    st->bytes_alg = 8.0 * (n + 1) + 4.0 * n + (eb + 4.0) * nnz + 4.0 * n + 8.0 * (nc + 1) + 8.0 * nnz_c +
                    (vwgt ? 8.0 * n : 0.0) + (out->vwgt ? 8.0 * nc : 0.0);
    st->long_rows = nl;
    st->long_entries = t1.long_entries;
    st->table_rows = overflow_rows;
  }
  return LM_OK;
}

}  // extern "C"
