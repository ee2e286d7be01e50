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
// entries of one (coarse row, coarse neighbour) in an LDS hash table with a
// list per slot; the first entry of a group (in row order) sums the group
// and keeps it. (3) Longer rows get a hash table of their own in device
// memory and the same grouping over all their entries at once. (4) A scan
// over the coarse rows gives their offsets, and the kept entries of every
// row part are packed in order to the output. Every entry of the fine graph
// is read twice (grouping, packing); cmap is gathered once per entry.
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
constexpr int kCH = 2048;               // LDS hash slots (load at most 1/2)
constexpr int kCHBits = 11;
constexpr int kCMaxDup = 4;             // fine edges one coarse edge merges at most in a simple graph
constexpr int kCCost = 4;               // cost of a fine vertex when ranges are split (entries cost 1)
constexpr int kCTopThreads = 1024;
constexpr int kCPackGrid = 4096;
constexpr unsigned long long kEmpty = ~0ull;

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
};

struct LongRow {
  int a, b, c, dega;
  int ub;     // deg(a) + deg(b)
  int tbits;  // table of 2^tbits slots
  long long eoff;  // first flat index of the row's entries among all long rows
  long long toff;  // first slot of its table
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
  long long* crp;
  int* ccol;
  float* cw;
};

__device__ __forceinline__ unsigned lds_hash(int r, int d) {
  return ((unsigned)d * 0x9E3779B1u ^ (unsigned)r * 0x85EBCA77u) >> (32 - kCHBits);
}
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

// (1a) Checks mate and row_ptr, counts the pairs' smaller ends per block.
__global__ __launch_bounds__(kBlock) void k_c_count(CArgs a) {
  __shared__ long long sm[kWaves];
  const long long v0 = (long long)blockIdx.x * kCBlockV + (long long)threadIdx.x * kCV;
  unsigned err = 0;
  long long reps = 0;
  for (int i = 0; i < kCV; ++i) {
    const long long v = v0 + i;
    if (v >= a.n) break;
    const int m = a.mate[v];
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

// (1c) Numbers the coarse vertices, writes cmap, the coarse vertex weights,
// and clears the per-row-part counts.
__global__ __launch_bounds__(kBlock) void k_c_map(CArgs a) {
  __shared__ long long sm[kWaves];
  if (a.tot->err) return;
  const long long v0 = (long long)blockIdx.x * kCBlockV + (long long)threadIdx.x * kCV;
  long long reps = 0;
  for (int i = 0; i < kCV; ++i) {
    const long long v = v0 + i;
    if (v >= a.n) break;
    const int m = a.mate[v];
    reps += (m == -1 || v < m) ? 1 : 0;
  }
  long long total;
  long long id = a.bsum[blockIdx.x] + block_excl_sum<long long>(reps, sm, total);
  for (int i = 0; i < kCV; ++i) {
    const long long v = v0 + i;
    if (v >= a.n) break;
    a.cnt[v] = 0;
    const int m = a.mate[v];
    if (!(m == -1 || v < m)) continue;
    const int c = (int)id++;
    a.cmap[v] = c;
    a.crep[c] = (int)v;
    if (m >= 0) a.cmap[m] = c;
    if (a.cvw) a.cvw[c] = (a.vw ? a.vw[v] : 1ll) + (m >= 0 ? (a.vw ? a.vw[m] : 1ll) : 0ll);
  }
}

struct TileSmem {
  unsigned long long key[kCH];  // (row in chunk << 32 | coarse neighbour), kEmpty if free
  int head[kCH];                // last entry inserted into the slot's list
  int eD[kCT];                  // coarse neighbour of the entry, -1 for the matched edge
  int ex[kCT];                  // fine neighbour
  float ew[kCT];
  int ek[kCT];                  // fine entry index (pack: exclusive rank among kept entries)
  short enext[kCT];
  short eslot[kCT];
  unsigned char erow[kCT];
  int st[kBlock + 1];  // chunk-local start of each row's entries; st[kBlock] = chunk total
  int ra[kBlock], rb[kBlock], rc[kBlock], rdega[kBlock];
  int rcnt[2][kBlock];
  long long sm64[kWaves];
  int smi[kWaves];
  int lb[1];
};

// Last row r of the chunk with st[r] <= pos (rows with no tile entries share
// their start with the next row, so r is the row that holds pos).
__device__ __forceinline__ int row_of(const TileSmem& sm, int pos) {
  int lo = 0, hi = kBlock;  // st[lo] <= pos; answer in [lo, hi)
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (sm.st[mid] <= pos)
      lo = mid;
    else
      hi = mid;
  }
  return lo;
}
// Start of the first row whose start is at least t (the chunk total if none).
__device__ __forceinline__ int start_at(const TileSmem& sm, int t) {
  int lo = 0, hi = kBlock;  // smallest r in [0, kBlock] with st[r] >= t
  if (sm.st[0] >= t) return sm.st[0];
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (sm.st[mid] >= t)
      hi = mid;
    else
      lo = mid;
  }
  return sm.st[hi];
}

// (2) PASS 0: groups the entries of the short coarse rows and keeps the first
// of every group with the group's sum; queues the long rows. PASS 1: packs
// the kept entries of the short rows to the output in order.
template <int PASS>
__global__ __launch_bounds__(kBlock) void k_c_tiles(CArgs a, long long per_wg) {
  __shared__ TileSmem sm;
  if (a.tot->err & (kCErrMate | kCErrRowPtr)) return;
  const int tid = threadIdx.x;
  const long long C = a.nnz + (long long)kCCost * a.n;
  const long long c0 = (long long)blockIdx.x * per_wg;
  if (c0 >= C) return;
  const long long c1 = c0 + per_wg;
  const long long vb =
      block_lower_bound(0, a.n + 1, [&](long long v) { return a.rp[v] + (long long)kCCost * v >= c0; }, sm.lb);
  const long long ve = c1 >= C ? a.n
                               : block_lower_bound(0, a.n + 1,
                                                   [&](long long v) { return a.rp[v] + (long long)kCCost * v >= c1; },
                                                   sm.lb);
  if (PASS == 0) {
    for (int i = tid; i < kCH; i += kBlock) {
      sm.key[i] = kEmpty;
      sm.head[i] = -1;
    }
  }
  unsigned err = 0;
  for (long long cb = vb; cb < ve; cb += kBlock) {
    const long long v = cb + tid;
    int ut = 0;
    bool rep = false, lng = false;
    int m = -1, c = 0, dega = 0, ub = 0;
    if (v < ve) {
      m = a.mate[v];
      rep = (m == -1 || v < m);
      if (rep) {
        c = a.cmap[v];
        dega = (int)(a.rp[v + 1] - a.rp[v]);
        ub = dega + (m >= 0 ? (int)(a.rp[m + 1] - a.rp[m]) : 0);
        lng = ub > kCS;
        ut = lng ? 0 : ub;
        if (PASS == 0 && lng) {
          const unsigned long long idx = atomicAdd((unsigned long long*)&a.tot->nlong, 1ull);
          if ((long long)idx < a.lrow_cap) {
            LongRow L;
            L.a = (int)v;
            L.b = m;
            L.c = c;
            L.dega = dega;
            L.ub = ub;
            L.tbits = 0;
            L.eoff = 0;
            L.toff = 0;
            a.lrows[idx] = L;
          }
        }
      }
    }
    int U;
    const int st = block_excl_sum<int>(ut, sm.smi, U);
    sm.st[tid] = st;
    if (tid == 0) sm.st[kBlock] = U;
    sm.ra[tid] = (int)v;
    sm.rb[tid] = m;
    sm.rc[tid] = c;
    sm.rdega[tid] = dega;
    sm.rcnt[0][tid] = 0;
    sm.rcnt[1][tid] = 0;
    __syncthreads();
    const int ntile = (U + kCStep - 1) / kCStep;
    for (int j = 0; j < ntile; ++j) {
      const int lo = start_at(sm, j * kCStep);
      const int hi = start_at(sm, (j + 1) * kCStep);
      const int len = hi - lo;
      if (len <= 0) continue;  // uniform across the workgroup
      if (PASS == 0) {
#pragma unroll
        for (int i = 0; i < kCTI; ++i) {
          const int q = i * kBlock + tid;
          if (q >= len) break;
          const int pos = lo + q;
          const int r = row_of(sm, pos);
          const int off = pos - sm.st[r];
          const bool side = off >= sm.rdega[r];
          const int s = side ? sm.rb[r] : sm.ra[r];
          const long long k = a.rp[s] + (side ? off - sm.rdega[r] : off);
          const int x = a.col[k];
          int D = -1;
          if ((unsigned)x >= (unsigned)a.n)
            err |= kCErrCol;
          else
            D = a.cmap[x];
          if (D == sm.rc[r]) D = -1;
          sm.eD[q] = D;
          sm.ex[q] = x;
          sm.ew[q] = a.w ? a.w[k] : 1.0f;
          sm.ek[q] = (int)k;
          sm.erow[q] = (unsigned char)r;
          if (D >= 0) {
            const unsigned long long kk = ((unsigned long long)(unsigned)r << 32) | (unsigned)D;
            unsigned h = lds_hash(r, D);
            for (;;) {
              const unsigned long long old = atomicCAS(&sm.key[h], kEmpty, kk);
              if (old == kEmpty || old == kk) break;
              h = (h + 1) & (kCH - 1);
            }
            sm.eslot[q] = (short)h;
            sm.enext[q] = (short)atomicExch(&sm.head[h], q);
          }
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < kCTI; ++i) {
          const int q = i * kBlock + tid;
          if (q >= len) break;
          const int D = sm.eD[q];
          const long long k = sm.ek[q];
          if (D < 0) {
            a.scr[k] = make_int2(-1, 0);
            continue;
          }
          int lst[kCMaxDup + 1];
          int nl = 0;
          int p = sm.head[sm.eslot[q]];
          bool first = true;
          while (p >= 0 && nl <= kCMaxDup) {
            lst[nl++] = p;
            first = first && p >= q;
            p = sm.enext[p];
          }
          if (nl > kCMaxDup) err |= kCErrDup;
          if (!first || nl > kCMaxDup) {
            a.scr[k] = make_int2(-1, 0);
            continue;
          }
          const int r = sm.erow[q];
          // the group's fine edges in increasing (min end, max end)
          unsigned long long ord[kCMaxDup];
          float wv[kCMaxDup];
          for (int t = 0; t < nl; ++t) {
            const int pp = lst[t];
            const int off = lo + pp - sm.st[r];
            const int s = off >= sm.rdega[r] ? sm.rb[r] : sm.ra[r];
            const int x = sm.ex[pp];
            const unsigned lo_e = (unsigned)min(s, x), hi_e = (unsigned)max(s, x);
            unsigned long long o = ((unsigned long long)lo_e << 32) | hi_e;
            float ww = sm.ew[pp];
            int u = t;
            while (u > 0 && ord[u - 1] > o) {
              ord[u] = ord[u - 1];
              wv[u] = wv[u - 1];
              --u;
            }
            ord[u] = o;
            wv[u] = ww;
          }
          float sum = wv[0];
          for (int t = 1; t < nl; ++t) sum += wv[t];
          a.scr[k] = make_int2(D, __float_as_int(sum));
          const int off = lo + q - sm.st[r];
          atomicAdd(&sm.rcnt[off >= sm.rdega[r] ? 1 : 0][r], 1);
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < kCTI; ++i) {
          const int q = i * kBlock + tid;
          if (q >= len) break;
          if (sm.eD[q] >= 0) {
            sm.key[sm.eslot[q]] = kEmpty;
            sm.head[sm.eslot[q]] = -1;
          }
        }
        __syncthreads();
      } else {
        int flags[kCTI];
        int carry = 0;
#pragma unroll
        for (int i = 0; i < kCTI; ++i) {
          const int q = i * kBlock + tid;
          int f = 0;
          if (q < len) {
            const int pos = lo + q;
            const int r = row_of(sm, pos);
            const int off = pos - sm.st[r];
            const bool side = off >= sm.rdega[r];
            const int s = side ? sm.rb[r] : sm.ra[r];
            const long long k = a.rp[s] + (side ? off - sm.rdega[r] : off);
            const int2 t = a.scr[k];
            f = t.x >= 0 ? 1 : 0;
            sm.eD[q] = t.x;
            sm.ew[q] = __int_as_float(t.y);
            sm.erow[q] = (unsigned char)r;
          }
          flags[i] = f;
        }
#pragma unroll
        for (int i = 0; i < kCTI; ++i) {
          const int q = i * kBlock + tid;
          int tot;
          const int e = block_excl_sum<int>(flags[i], sm.smi, tot);
          if (q < kCT) sm.ek[q] = carry + e;
          carry += tot;
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < kCTI; ++i) {
          const int q = i * kBlock + tid;
          if (q >= len || !flags[i]) continue;
          const int r = sm.erow[q];
          const int off = lo + q - sm.st[r];
          const bool side = off >= sm.rdega[r];
          const int ps = sm.st[r] + (side ? sm.rdega[r] : 0) - lo;
          const int rank = sm.ek[q] - sm.ek[ps];
          const long long dest = a.crp[sm.rc[r]] + (side ? a.cnt[sm.ra[r]] : 0) + rank;
          a.ccol[dest] = sm.eD[q];
          a.cw[dest] = sm.ew[q];
        }
        __syncthreads();
      }
    }
    if (PASS == 0) {
      if (v < ve && rep && !lng) {
        a.cnt[v] = sm.rcnt[0][tid];
        if (m >= 0) a.cnt[m] = sm.rcnt[1][tid];
      }
    }
    __syncthreads();
  }
  if (err) atomicOr(&a.tot->err, err);
}

// (3a) Offsets of the long rows' entries and tables, one workgroup.
__global__ __launch_bounds__(kCTopThreads) void k_c_long_prep(CArgs a) {
  __shared__ long long sm[kCTopThreads / 64];
  if (a.tot->err) return;
  const long long nl = a.tot->nlong < a.lrow_cap ? a.tot->nlong : a.lrow_cap;
  long long ce = 0, cs = 0;
  for (long long base = 0; base < nl; base += kCTopThreads) {
    const long long i = base + threadIdx.x;
    long long ub = 0, slots = 0;
    int bits = 1;
    if (i < nl) {
      ub = a.lrows[i].ub;
      while ((1ll << bits) < 2 * ub) ++bits;
      slots = 1ll << bits;
    }
    long long te, ts;
    const long long ee = top_excl_sum(ub, sm, te);
    const long long es = top_excl_sum(slots, sm, ts);
    if (i < nl) {
      a.lrows[i].eoff = ce + ee;
      a.lrows[i].toff = cs + es;
      a.lrows[i].tbits = bits;
    }
    ce += te;
    cs += ts;
  }
  if (threadIdx.x == 0) {
    a.tot->long_entries = ce;
    a.tot->long_slots = cs;
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

// (3b) Inserts every entry of the long rows into its row's table.
__global__ __launch_bounds__(kBlock) void k_c_long_insert(CArgs a, long long nl, long long total) {
  unsigned err = 0;
  for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < total; i += (long long)gridDim.x * kBlock) {
    const LongRow L = a.lrows[long_row_of(a.lrows, nl, i)];
    const int off = (int)(i - L.eoff);
    const bool side = off >= L.dega;
    const int s = side ? L.b : L.a;
    const long long k = a.rp[s] + (side ? off - L.dega : off);
    const int x = a.col[k];
    if ((unsigned)x >= (unsigned)a.n) {
      err |= kCErrCol;
      continue;
    }
    const int D = a.cmap[x];
    if (D == L.c) continue;
    int2* tb = a.table + L.toff;
    const unsigned long long mask = (1ull << L.tbits) - 1;
    unsigned long long h = tbl_hash(D, L.tbits);
    for (;;) {
      const int old = atomicCAS(&tb[h].x, -1, D);
      if (old == -1 || old == D) break;
      h = (h + 1) & mask;
    }
    a.next[k] = atomicExch(&tb[h].y, (int)k);
  }
  if (err) atomicOr(&a.tot->err, err);
}

// (3c) The first entry of every group of a long row keeps the group's sum.
__global__ __launch_bounds__(kBlock) void k_c_long_keep(CArgs a, long long nl, long long total) {
  unsigned err = 0;
  for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < total; i += (long long)gridDim.x * kBlock) {
    const LongRow L = a.lrows[long_row_of(a.lrows, nl, i)];
    const int off = (int)(i - L.eoff);
    const bool side = off >= L.dega;
    const int s = side ? L.b : L.a;
    const long long ka = a.rp[L.a];
    const long long kb = L.b >= 0 ? a.rp[L.b] : 0;
    const long long k = (side ? kb : ka) + (side ? off - L.dega : off);
    const int x = a.col[k];
    if ((unsigned)x >= (unsigned)a.n) {
      a.scr[k] = make_int2(-1, 0);
      continue;
    }
    const int D = a.cmap[x];
    if (D == L.c) {
      a.scr[k] = make_int2(-1, 0);
      continue;
    }
    const int2* tb = a.table + L.toff;
    const unsigned long long mask = (1ull << L.tbits) - 1;
    unsigned long long h = tbl_hash(D, L.tbits);
    while (tb[h].x != D) h = (h + 1) & mask;
    // the group's entries; row order is a's part, then b's part
    int lst[kCMaxDup + 1];
    int nlst = 0;
    int p = tb[h].y;
    bool first = true;
    while (p >= 0 && nlst <= kCMaxDup) {
      lst[nlst++] = p;
      const bool pa = (long long)p >= ka && (long long)p < ka + L.dega;
      const long long pos_p = pa ? p - ka : L.dega + (p - kb);
      first = first && pos_p >= off;
      p = a.next[p];
    }
    if (nlst > kCMaxDup) err |= kCErrDup;
    if (!first || nlst > kCMaxDup) {
      a.scr[k] = make_int2(-1, 0);
      continue;
    }
    unsigned long long ord[kCMaxDup];
    float wv[kCMaxDup];
    for (int t = 0; t < nlst; ++t) {
      const int pp = lst[t];
      const bool pa = (long long)pp >= ka && (long long)pp < ka + L.dega;
      const int sp = pa ? L.a : L.b;
      const int xp = a.col[pp];
      const unsigned lo_e = (unsigned)min(sp, xp), hi_e = (unsigned)max(sp, xp);
      const unsigned long long o = ((unsigned long long)lo_e << 32) | hi_e;
      const float ww = a.w ? a.w[pp] : 1.0f;
      int u = t;
      while (u > 0 && ord[u - 1] > o) {
        ord[u] = ord[u - 1];
        wv[u] = wv[u - 1];
        --u;
      }
      ord[u] = o;
      wv[u] = ww;
    }
    float sum = wv[0];
    for (int t = 1; t < nlst; ++t) sum += wv[t];
    a.scr[k] = make_int2(D, __float_as_int(sum));
    atomicAdd(&a.cnt[s], 1);
  }
  if (err) atomicOr(&a.tot->err, err);
}

__device__ __forceinline__ long long coarse_deg(const CArgs& a, long long c) {
  const int r = a.crep[c];
  const int m = a.mate[r];
  return (long long)a.cnt[r] + (m >= 0 ? a.cnt[m] : 0);
}

// (4a) Coarse row lengths, summed per block.
__global__ __launch_bounds__(kBlock) void k_c_deg_count(CArgs a, long long nc) {
  __shared__ long long sm[kWaves];
  if (a.tot->err) return;
  const long long c0 = (long long)blockIdx.x * kCBlockV + (long long)threadIdx.x * kCV;
  long long s = 0;
  for (int i = 0; i < kCV; ++i) {
    const long long c = c0 + i;
    if (c >= nc) break;
    s += coarse_deg(a, c);
  }
  long long total;
  (void)block_excl_sum<long long>(s, sm, total);
  if (threadIdx.x == 0) a.bsum[blockIdx.x] = total;
}

// (4c) Coarse row offsets.
__global__ __launch_bounds__(kBlock) void k_c_deg_write(CArgs a, long long nc) {
  __shared__ long long sm[kWaves];
  if (a.tot->err) return;
  const long long c0 = (long long)blockIdx.x * kCBlockV + (long long)threadIdx.x * kCV;
  long long s = 0;
  for (int i = 0; i < kCV; ++i) {
    const long long c = c0 + i;
    if (c >= nc) break;
    s += coarse_deg(a, c);
  }
  long long total;
  long long off = a.bsum[blockIdx.x] + block_excl_sum<long long>(s, sm, total);
  for (int i = 0; i < kCV; ++i) {
    const long long c = c0 + i;
    if (c >= nc) break;
    a.crp[c] = off;
    off += coarse_deg(a, c);
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

int tile_blocks_per_cu() {
  static int cached = 0;
  if (cached) return cached;
  int nb = 1;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_c_tiles<0>, kBlock, 0) != hipSuccess || nb < 1) nb = 1;
  cached = nb;
  return nb;
}

size_t a256(size_t b) { return (b + 255) & ~(size_t)255; }

}  // namespace

// Buffers of the contraction, kept in the context between calls.
struct ContractState {
  DevBuf bsum, tot, crep, cnt, scr, next, lrows, table;
  DevBuf in_rp, in_col, in_w, in_mate, in_vw, o_cmap, o_crp, o_ccol, o_cw, o_cvw;
  CTot* h_tot = nullptr;
};

void contract_release(Solver& S) {
  ContractState* cs = S.contract;
  if (!cs) return;
  DevBuf* all[] = {&cs->bsum,  &cs->tot,    &cs->crep,    &cs->cnt,    &cs->scr,    &cs->next,   &cs->lrows,
                   &cs->table, &cs->in_rp,  &cs->in_col,  &cs->in_w,   &cs->in_mate, &cs->in_vw, &cs->o_cmap,
                   &cs->o_crp, &cs->o_ccol, &cs->o_cw,    &cs->o_cvw};
  for (DevBuf* b : all) S.pool.release(*b);
  if (cs->h_tot) (void)hipHostFree(cs->h_tot);
  delete cs;
  S.contract = nullptr;
}

Solver& solver_of(lm_ctx* c);
std::mutex& mutex_of(lm_ctx* c);

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
  hipLaunchKernelGGL(k_c_tiles<0>, dim3((unsigned)grid), dim3(kBlock), 0, s, a, per_wg);
  hipLaunchKernelGGL(k_c_long_prep, dim3(1), dim3(kCTopThreads), 0, s, a);
  LMC_HIP(hipGetLastError());
  LMC_HIP(hipMemcpyAsync(cs.h_tot, a.tot, sizeof(CTot), hipMemcpyDeviceToHost, s));
  LMC_HIP(hipStreamSynchronize(s));
  CTot t1 = *cs.h_tot;
  if (t1.err & kCErrMate) return LM_EINVAL;
  if (t1.err) return LM_EGRAPH;
  const long long nc = t1.nc;
  const long long nl = t1.nlong;
  if (nl > lrow_cap) return LM_EDEVICE;  // cannot happen: the bounds of the rows sum to nnz
  if (nl > 0) {
    LMC_TRY(P.reserve(cs.next, a256(sizeof(int) * (size_t)nnz)));
    LMC_TRY(P.reserve(cs.table, a256(sizeof(int2) * (size_t)t1.long_slots)));
    a.next = (int*)cs.next.p;
    a.table = (int2*)cs.table.p;
    const long long fill_grid = std::min<long long>((t1.long_slots + kBlock - 1) / kBlock, 8192);
    hipLaunchKernelGGL(k_c_fill, dim3((unsigned)fill_grid), dim3(kBlock), 0, s, a.table, t1.long_slots);
    const long long lg = std::min<long long>((t1.long_entries + kBlock - 1) / kBlock, 16384);
    hipLaunchKernelGGL(k_c_long_insert, dim3((unsigned)lg), dim3(kBlock), 0, s, a, nl, t1.long_entries);
    hipLaunchKernelGGL(k_c_long_keep, dim3((unsigned)lg), dim3(kBlock), 0, s, a, nl, t1.long_entries);
  }
  const long long nb_c = (nc + kCBlockV - 1) / kCBlockV;
  if (nb_c > 0) {
    hipLaunchKernelGGL(k_c_deg_count, dim3((unsigned)nb_c), dim3(kBlock), 0, s, a, nc);
    hipLaunchKernelGGL(k_c_scan_top, dim3(1), dim3(kCTopThreads), 0, s, a.bsum, nb_c, &a.tot->nnz_c);
    hipLaunchKernelGGL(k_c_deg_write, dim3((unsigned)nb_c), dim3(kBlock), 0, s, a, nc);
  }
  hipLaunchKernelGGL(k_c_tiles<1>, dim3((unsigned)grid), dim3(kBlock), 0, s, a, per_wg);
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
  }
  return LM_OK;
}

}  // extern "C"
