// Phase kernels of local-max matching for gfx950 (wave64).
//
// One phase (paper, Section 2, "Sequential Model" and the CREW phase steps of
// Section 2.1, re-planned for a GPU):
//   argmax   every live vertex v finds the live incident edge of largest key
//            (Lemma 3 form: a segmented reduction over the entry stream);
//   mutual   v is matched iff its candidate u has v as candidate (CREW step 3)
//            and marks itself (the deletion flag of CREW step 4 lives on the
//            vertex instead of being spread over its edges);
//   compact  every live entry whose endpoints are both unmatched survives and
//            is written contiguously (CREW steps 5-6); the argmax of the next
//            phase is computed in the same pass over the survivors.
//
// Layout of a live set R_t: a "short" list of rows (live degree <= short_max)
// that forms a dense CSR in list order, cut into tiles by a virtual position
// window of tile_width entries, and a "long" list of rows that get a
// workgroup each. All counters live in per-phase slots so that phases can be
// enqueued back to back without host synchronisation; kernels read their
// work sizes from device memory and stop when a phase is empty.
#include <algorithm>

#include "lm_internal.h"
#include "lm_key.h"

namespace lm {

// ---------------------------------------------------------------- helpers

__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }
__device__ __forceinline__ int wave_id() { return threadIdx.x >> 6; }
__device__ __forceinline__ unsigned long long lanemask_lt() {
  const int l = lane_id();
  return l == 0 ? 0ull : (~0ull >> (64 - l));
}

template <typename T>
__device__ __forceinline__ T wave_incl_sum(T x) {
  const int l = lane_id();
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    T y = __shfl_up(x, d, 64);
    if (l >= d) x += y;
  }
  return x;
}

// Exclusive prefix sum over the workgroup; total gets the sum of all lanes.
template <typename T>
__device__ __forceinline__ T block_excl_sum(T x, T* sm, T& total) {
  T incl = wave_incl_sum(x);
  if (lane_id() == 63) sm[wave_id()] = incl;
  __syncthreads();
  T pre = 0, tot = 0;
#pragma unroll
  for (int i = 0; i < kWaves; ++i) {
    T v = sm[i];
    pre += (i < wave_id()) ? v : T(0);
    tot += v;
  }
  __syncthreads();
  total = tot;
  return pre + incl - x;
}

// Exclusive prefix max over the workgroup (identity 0).
__device__ __forceinline__ unsigned block_excl_max(unsigned x, unsigned* sm) {
  const int l = lane_id();
  unsigned incl = x;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    unsigned y = __shfl_up(incl, d, 64);
    if (l >= d) incl = max(incl, y);
  }
  if (l == 63) sm[wave_id()] = incl;
  __syncthreads();
  unsigned pre = 0;
#pragma unroll
  for (int i = 0; i < kWaves; ++i)
    if (i < wave_id()) pre = max(pre, sm[i]);
  __syncthreads();
  unsigned ex = __shfl_up(incl, 1, 64);
  if (l == 0) ex = 0;
  return max(pre, ex);
}

// Segmented-scan element: f = a segment (row) starts inside, k = running best.
struct SegKey {
  unsigned f;
  Key k;
};

__device__ __forceinline__ SegKey seg_combine(const SegKey& a, const SegKey& b) {  // a precedes b
  SegKey r;
  r.f = a.f | b.f;
  r.k = b.f ? b.k : key_max(a.k, b.k);
  return r;
}

__device__ __forceinline__ SegKey shfl_up_seg(const SegKey& x, int d) {
  SegKey y;
  y.f = __shfl_up(x.f, d, 64);
  y.k.w = __shfl_up(x.k.w, d, 64);
  y.k.hhi = __shfl_up(x.k.hhi, d, 64);
  y.k.hlo = __shfl_up(x.k.hlo, d, 64);
  y.k.u = __shfl_up(x.k.u, d, 64);
  return y;
}

// Exclusive segmented max-scan over the workgroup.
__device__ __forceinline__ SegKey block_excl_segscan(SegKey x, SegKey* sm) {
  const int l = lane_id();
  SegKey incl = x;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    SegKey y = shfl_up_seg(incl, d);
    if (l >= d) incl = seg_combine(y, incl);
  }
  if (l == 63) sm[wave_id()] = incl;
  __syncthreads();
  SegKey carry;
  carry.f = 0;
  carry.k = key_ident();
  for (int i = 0; i < wave_id(); ++i) carry = seg_combine(carry, sm[i]);
  __syncthreads();
  SegKey ex = shfl_up_seg(incl, 1);
  if (l == 0) {
    ex.f = 0;
    ex.k = key_ident();
  }
  return seg_combine(carry, ex);
}

__device__ __forceinline__ Key shfl_xor_key(const Key& x, int m) {
  Key y;
  y.w = __shfl_xor(x.w, m, 64);
  y.hhi = __shfl_xor(x.hhi, m, 64);
  y.hlo = __shfl_xor(x.hlo, m, 64);
  y.u = __shfl_xor(x.u, m, 64);
  return y;
}

// Max key over the workgroup (every lane gets it).
__device__ __forceinline__ Key block_max_key(Key x, Key* sm) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) x = key_max(x, shfl_xor_key(x, m));
  if (lane_id() == 0) sm[wave_id()] = x;
  __syncthreads();
  Key r = sm[0];
#pragma unroll
  for (int i = 1; i < kWaves; ++i) r = key_max(r, sm[i]);
  __syncthreads();
  return r;
}

// Tiles of R_{t+1}: the row starting at virtual position vp with kept
// entries covers tile starts k*tw in [vp, vp+kept); tile k's first row is
// this row if it starts exactly there, else the next one.
__device__ __forceinline__ void write_tile_starts(int* tiles, long long cap, long long vp, long long kept, int row,
                                                  int tw) {
  long long k0 = (vp + tw - 1) / tw;
  long long k1 = (vp + kept - 1) / tw;
  if (k1 >= cap) k1 = cap - 1;  // only reachable from offsets that the init check rejects
  for (long long k = k0; k <= k1; ++k) tiles[k] = (k * tw == vp) ? row : row + 1;
}

// ---------------------------------------------------------------- zero

__global__ void k_zero(Slot* slots, Totals* totals) {
  unsigned* p = reinterpret_cast<unsigned*>(slots);
  const int words = kRing * (int)sizeof(Slot) / 4;
  for (int i = threadIdx.x; i < words; i += blockDim.x) p[i] = 0u;
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

// ---------------------------------------------------------------- init

struct InitSmem {
  unsigned long long s64[kWaves];
  unsigned s32[kWaves];
  unsigned long long bc;
  unsigned bcl;
};

// Builds R_1 from the input CSR: every vertex with degree 1..short_max joins
// the short list (packed counter gives list index and virtual position in one
// atomic), longer rows join the long list. Also clears mate and state and
// checks the offsets.
__global__ __launch_bounds__(kBlock) void k_init(InitArgs a) {
  __shared__ InitSmem sm;
  const int tid = threadIdx.x;
  const long long chunk = kCap;
  const long long nchunks = ((long long)a.n + chunk - 1) / chunk;
  unsigned err = 0;
  for (long long ch = blockIdx.x; ch < nchunks; ch += gridDim.x) {
    const long long v0 = ch * chunk;
    // graph of the first vertex of this lane
    int g = 0;
    if (a.graphs > 1) {
      long long vfirst = v0 + tid;
      int lo = 0, hi = a.graphs - 1;
      while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (a.vtx_off[mid] <= vfirst) lo = mid;
        else hi = mid - 1;
      }
      g = lo;
    }
    int vv[kItems], dd[kItems], gg[kItems];
    long long oo[kItems];
    unsigned cnt = 0, dsum = 0, lcnt = 0;
    unsigned long long lsum = 0;
#pragma unroll
    for (int j = 0; j < kItems; ++j) {
      const long long v = v0 + tid + (long long)kBlock * j;
      vv[j] = -1;
      dd[j] = 0;
      if (v < a.n) {
        if (a.graphs > 1)
          while (a.vtx_off[g + 1] <= v) ++g;
        const long long b = a.row_ptr[v], e = a.row_ptr[v + 1];
        if (v == 0 && b != 0) err |= kErrRowPtr;
        if (v == a.n - 1 && e != a.nnz) err |= kErrRowPtr;
        long long d = e - b;
        if (d < 0 || b < 0 || e > a.nnz) {
          err |= kErrRowPtr;
          d = 0;
        }
        if (d > 0x7fff0000LL) {
          err |= kErrDegree;
          d = 0;
        }
        a.mate[v] = -1;
        a.state[v] = 0;
        vv[j] = (int)v;
        dd[j] = (int)d;
        oo[j] = b;
        gg[j] = g;
        if (d >= 1 && d <= a.short_max) {
          ++cnt;
          dsum += (unsigned)d;
        } else if (d > a.short_max) {
          ++lcnt;
          lsum += (unsigned long long)d;
        }
      }
    }
    // short rows: one packed atomic per chunk
    unsigned long long mine = ((unsigned long long)cnt << 32) | dsum;
    unsigned long long tot;
    unsigned long long ex = block_excl_sum<unsigned long long>(mine, sm.s64, tot);
    if (tid == 0 && tot != 0) sm.bc = atomicAdd(&a.slot1->short_packed, tot);
    // long rows
    unsigned ltot;
    unsigned lex = block_excl_sum<unsigned>(lcnt, sm.s32, ltot);
    unsigned long long lsumtot;
    (void)block_excl_sum<unsigned long long>(lsum, sm.s64, lsumtot);
    if (tid == 0 && ltot != 0) {
      sm.bcl = atomicAdd(&a.slot1->long_rows, ltot);
      atomicAdd(&a.slot1->long_kept, lsumtot);
    }
    __syncthreads();
    const unsigned long long base = sm.bc;
    const unsigned rb = (unsigned)(base >> 32) + (unsigned)(ex >> 32);
    unsigned long long vp = (base & 0xffffffffull) + (ex & 0xffffffffull);
    unsigned ri = 0, li = 0;
#pragma unroll
    for (int j = 0; j < kItems; ++j) {
      if (vv[j] < 0) continue;
      const int d = dd[j];
      if (d >= 1 && d <= a.short_max) {
        const int row = (int)(rb + ri);
        a.short_out[row] = make_int4(vv[j], (int)oo[j], d, gg[j]);
        write_tile_starts(a.tiles_out, a.tiles_cap, (long long)vp, d, row, a.tile_width);
        vp += (unsigned)d;
        ++ri;
      } else if (d > a.short_max) {
        const unsigned long long at = (unsigned long long)sm.bcl + lex + li;
        if (at < (unsigned long long)a.long_cap) a.long_out[at] = make_int4(vv[j], (int)oo[j], d, gg[j]);
        else err |= kErrRowPtr;  // more long rows than nnz allows: offsets overlap
        ++li;
      }
    }
    __syncthreads();
  }
  if (err) atomicOr(&a.totals->err, err);
}

// Optional input check: ids in range, no self-loops, finite weights.
__global__ __launch_bounds__(kBlock) void k_check(CheckArgs a) {
  unsigned err = 0;
  const long long nnz = a.nnz;
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
    long long b = a.row_ptr[v], e = a.row_ptr[v + 1];
    if (b < 0 || e > nnz || e < b) {
      err |= kErrRowPtr;
      continue;
    }
    for (long long k = b; k < e; ++k) {
      int u = a.col[k];
      if (u < 0 || u >= lim) err |= kErrColRange;
      if (u == v - base) err |= kErrSelfLoop;
      float x = a.w[k];
      if (!(x == x) || x == __int_as_float(0x7f800000) || x == __int_as_float(0xff800000)) err |= kErrWeight;
    }
  }
  if (err) atomicOr(&a.totals->err, err);
}

// ---------------------------------------------------------------- tiles

struct TileSmem {
  int r_v[kMaxRowsPerTile];
  int r_offbest[kMaxRowsPerTile];  // physical offset while loading, then best local id
  int r_g[kMaxRowsPerTile];
  unsigned short r_vo[kMaxRowsPerTile + 1];
  unsigned short r_kst[kMaxRowsPerTile];
  unsigned short r_kend[kMaxRowsPerTile];
  unsigned short rowof[kCap];
  int e_col[kCap];
  unsigned e_w[kCap];  // raw float bits
  unsigned s32[kWaves];
  SegKey sseg[kWaves];
  unsigned long long bc;
};

struct LongSmem {
  int e_col[kCap];
  unsigned e_w[kCap];
  unsigned s32[kWaves];
  Key skey[kWaves];
  unsigned wcnt[kWaves];
  long long bc0;
  unsigned long long bc1;
};

union PhaseSmem {
  TileSmem tile;
  LongSmem lng;
};

// One tile of the short list: the rows whose virtual start lies in
// [k*tw, (k+1)*tw). All their entries fit one pass of kCap.
template <bool FIRST>
__device__ void tile_phase(const PhaseArgs& a, Slot* sout, int k, int ntiles, int nrows, TileSmem& sm) {
  const int tid = threadIdx.x;
  const int r0 = a.tiles_in[k];
  const int r1 = (k + 1 < ntiles) ? a.tiles_in[k + 1] : nrows;
  const int nr = r1 - r0;
  if (nr <= 0) return;  // uniform: every lane reads the same values
  // ---- rows of the tile; matched rows drop out without reading entries
  const int rpt = (nr + kBlock - 1) / kBlock;  // <= kMaxRowsPerTile / kBlock
  constexpr int kRpt = kMaxRowsPerTile / kBlock;
  int4 rec[kRpt];
  bool um[kRpt];
  unsigned cnt = 0, dsum = 0;
#pragma unroll
  for (int i = 0; i < kRpt; ++i) {
    const int j = tid * rpt + i;
    um[i] = false;
    if (i < rpt && j < nr) {
      rec[i] = a.short_in[r0 + j];
      um[i] = FIRST ? true : (a.state[rec[i].x] == 0);
      if (um[i]) {
        ++cnt;
        dsum += (unsigned)rec[i].z;
      }
    }
  }
  unsigned tot;
  unsigned ex = block_excl_sum<unsigned>((cnt << 16) | dsum, sm.s32, tot);
  const int NU = (int)(tot >> 16);
  const int NV = (int)(tot & 0xffffu);
  if (NV > kCap) {  // cannot happen for well-formed lists
    if (tid == 0) atomicOr(&a.totals->err, kErrTile);
    return;
  }
  {
    int c = (int)(ex >> 16);
    unsigned vo = ex & 0xffffu;
#pragma unroll
    for (int i = 0; i < kRpt; ++i) {
      if (!um[i]) continue;
      sm.r_v[c] = rec[i].x;
      sm.r_offbest[c] = rec[i].y;
      sm.r_g[c] = rec[i].w;
      sm.r_vo[c] = (unsigned short)vo;
      vo += (unsigned)rec[i].z;
      ++c;
    }
  }
  if (tid == 0) sm.r_vo[NU] = (unsigned short)NV;
  for (int q = tid; q < NV; q += kBlock) sm.rowof[q] = 0;
  __syncthreads();
  if (NU == 0) return;  // uniform
  for (int c = tid; c < NU; c += kBlock) sm.rowof[sm.r_vo[c]] = (unsigned short)c;
  __syncthreads();
  // ---- row of every virtual position: prefix max of the row heads
  {
    const int q0 = tid * kItems;
    unsigned run = 0, vals[kItems];
#pragma unroll
    for (int i = 0; i < kItems; ++i) {
      const int q = q0 + i;
      if (q < NV) run = max(run, (unsigned)sm.rowof[q]);
      vals[i] = run;
    }
    const unsigned carry = block_excl_max(run, sm.s32);
#pragma unroll
    for (int i = 0; i < kItems; ++i) {
      const int q = q0 + i;
      if (q < NV) sm.rowof[q] = (unsigned short)max(carry, vals[i]);
    }
  }
  __syncthreads();
  // ---- striped, coalesced loads of the live entries; neighbour state gather
  {
    int cc[kItems];
    float ww[kItems];
#pragma unroll
    for (int j = 0; j < kItems; ++j) {
      const int q = tid + kBlock * j;
      cc[j] = 0;
      ww[j] = 0.f;
      if (q < NV) {
        const int c = sm.rowof[q];
        const int addr = sm.r_offbest[c] + (q - (int)sm.r_vo[c]);
        cc[j] = a.src_col[addr];
        ww[j] = a.src_w[addr];
      }
    }
#pragma unroll
    for (int j = 0; j < kItems; ++j) {
      const int q = tid + kBlock * j;
      if (q < NV) {
        unsigned col = (unsigned)cc[j];
        const int c = sm.rowof[q];
        const unsigned ug = (unsigned)(a.gbase[sm.r_g[c]] + cc[j]);
        if (ug >= (unsigned)a.n || cc[j] < 0)
          col |= kDropBit;  // id outside the graph: never a candidate
        else if (!FIRST && a.state[ug] != 0)
          col |= kDropBit;
        sm.e_col[q] = (int)col;
        sm.e_w[q] = __float_as_uint(ww[j]);
      }
    }
  }
  __syncthreads();
  // ---- blocked pass: kept counts and segmented argmax per row
  const int q0 = tid * kItems;
  int myc[kItems];
  unsigned mycol[kItems], myw[kItems];
  unsigned kc = 0;
  SegKey agg;
  agg.f = 0;
  agg.k = key_ident();
  Key p1 = key_ident();
  int c0 = -1;
  bool c0_ends = false, head0 = false;
  if (q0 < NV) {
    int c = sm.rowof[q0];
    c0 = c;
    int rend = sm.r_vo[c + 1];
    head0 = ((int)sm.r_vo[c] == q0);
    bool first_open = true;
    unsigned f = head0 ? 1u : 0u;
    int g = sm.r_g[c];
    unsigned long long S = a.gseed[g];
    unsigned vloc = (unsigned)(sm.r_v[c] - a.gbase[g]);
    Run run = run_ident();
#pragma unroll
    for (int i = 0; i < kItems; ++i) {
      const int q = q0 + i;
      myc[i] = -1;
      if (q >= NV) continue;
      if (q == rend) {
        ++c;
        rend = sm.r_vo[c + 1];
        run = run_ident();
        f = 1u;
        g = sm.r_g[c];
        S = a.gseed[g];
        vloc = (unsigned)(sm.r_v[c] - a.gbase[g]);
      }
      myc[i] = c;
      const unsigned col = (unsigned)sm.e_col[q];
      const unsigned wb = sm.e_w[q];
      mycol[i] = col;
      myw[i] = wb;
      if (!(col & kDropBit)) {
        ++kc;
        run_update(run, ord_weight_bits(wb), (int)col, vloc, S);
      }
      if (q == rend - 1) {  // row c ends here
        if (first_open) {
          p1 = run_key(run, vloc, S);
          c0_ends = true;
          first_open = false;
        } else {
          sm.r_offbest[c] = run_key(run, vloc, S).u;
        }
      }
    }
    if (first_open) p1 = run_key(run, vloc, S);
    agg.f = f;
    agg.k = run_key(run, vloc, S);
  } else {
#pragma unroll
    for (int i = 0; i < kItems; ++i) myc[i] = -1;
  }
  // kept positions
  unsigned ktot;
  const unsigned kpre = block_excl_sum<unsigned>(kc, sm.s32, ktot);
  // carry of the row open at q0
  const SegKey carry = block_excl_segscan(agg, sm.sseg);
  if (c0 >= 0 && c0_ends) sm.r_offbest[c0] = (head0 ? p1 : key_max(carry.k, p1)).u;
  // row starts / ends in kept-position space
  {
    unsigned p = kpre;
#pragma unroll
    for (int i = 0; i < kItems; ++i) {
      const int c = myc[i];
      if (c < 0) continue;
      const int q = q0 + i;
      if (q == (int)sm.r_vo[c]) sm.r_kst[c] = (unsigned short)p;
      if (!(mycol[i] & kDropBit)) ++p;
      if (q == (int)sm.r_vo[c + 1] - 1) sm.r_kend[c] = (unsigned short)p;
    }
  }
  __syncthreads();
  if (FIRST) {
    for (int c = tid; c < NU; c += kBlock) {
      const int g = sm.r_g[c];
      const int b = sm.r_offbest[c];
      a.C[sm.r_v[c]] = b >= 0 ? a.gbase[g] + b : -1;
    }
    return;
  }
  // in-place compaction of kept entries (all reads of e_* are done)
  {
    unsigned p = kpre;
#pragma unroll
    for (int i = 0; i < kItems; ++i) {
      if (myc[i] < 0 || (mycol[i] & kDropBit)) continue;
      sm.e_col[p] = (int)mycol[i];
      sm.e_w[p] = myw[i];
      ++p;
    }
  }
  // surviving rows
  const int rpt2 = (NU + kBlock - 1) / kBlock;
  unsigned scount = 0;
  for (int i = 0; i < rpt2; ++i) {
    const int c = tid * rpt2 + i;
    if (c < NU && sm.r_kend[c] != sm.r_kst[c]) ++scount;
  }
  unsigned stot;
  const unsigned spre = block_excl_sum<unsigned>(scount, sm.s32, stot);
  if (tid == 0) {
    unsigned long long old = 0;
    if (stot != 0) old = atomicAdd(&sout->short_packed, ((unsigned long long)stot << 32) | ktot);
    sm.bc = old;
  }
  __syncthreads();
  const unsigned RB = (unsigned)(sm.bc >> 32);
  const long long EB = (long long)(sm.bc & 0xffffffffull);
  {
    unsigned s = spre;
    for (int i = 0; i < rpt2; ++i) {
      const int c = tid * rpt2 + i;
      if (c >= NU) break;
      const unsigned kst = sm.r_kst[c], kend = sm.r_kend[c];
      if (kend == kst) continue;
      const int row = (int)(RB + s);
      const int g = sm.r_g[c];
      const int v = sm.r_v[c];
      a.short_out[row] = make_int4(v, (int)(EB + kst), (int)(kend - kst), g);
      a.C[v] = a.gbase[g] + sm.r_offbest[c];
      write_tile_starts(a.tiles_out, a.tiles_cap, EB + kst, kend - kst, row, a.tile_width);
      ++s;
    }
  }
  for (int p = tid; p < (int)ktot; p += kBlock) {
    a.dst_col[EB + p] = sm.e_col[p];
    a.dst_w[EB + p] = __uint_as_float(sm.e_w[p]);
  }
}

// One long row (live degree > short_max), one workgroup.
template <bool FIRST>
__device__ void long_phase(const PhaseArgs& a, Slot* sout, int idx, LongSmem& sm) {
  const int tid = threadIdx.x;
  const int4 rec = a.long_in[idx];
  const int v = rec.x, off = rec.y, deg = rec.z, g = rec.w;
  if (!FIRST && a.state[v] != 0) return;  // uniform
  const int base = a.gbase[g];
  const unsigned long long S = a.gseed[g];
  const unsigned vloc = (unsigned)(v - base);
  const int npass = (deg + kCap - 1) / kCap;
  const bool multi = npass > 1;
  if (!FIRST && multi) {
    if (tid == 0) {
      unsigned long long old = atomicAdd(&sout->long_used, (unsigned long long)deg);
      sm.bc0 = a.dst_cap - (long long)old - deg;
    }
    __syncthreads();
  }
  const long long ob = (!FIRST && multi) ? sm.bc0 : 0;
  Run run = run_ident();
  unsigned running = 0;
  for (int p = 0; p < npass; ++p) {
    int cc[kItems];
    float ww[kItems];
    bool kp[kItems];
#pragma unroll
    for (int j = 0; j < kItems; ++j) {
      const int q = p * kCap + j * kBlock + tid;
      kp[j] = false;
      cc[j] = 0;
      ww[j] = 0.f;
      if (q < deg) {
        cc[j] = a.src_col[off + q];
        ww[j] = a.src_w[off + q];
      }
    }
#pragma unroll
    for (int j = 0; j < kItems; ++j) {
      const int q = p * kCap + j * kBlock + tid;
      if (q < deg) {
        const unsigned ug = (unsigned)(base + cc[j]);
        kp[j] = cc[j] >= 0 && ug < (unsigned)a.n && (FIRST || a.state[ug] == 0);
        if (kp[j]) run_update(run, ord_weight_bits(__float_as_uint(ww[j])), cc[j], vloc, S);
      }
    }
    if (FIRST) continue;
    // ballot positions: order (wave, item j, lane)
    unsigned long long mk[kItems];
    unsigned wtot = 0;
#pragma unroll
    for (int j = 0; j < kItems; ++j) {
      mk[j] = __ballot(kp[j]);
      wtot += (unsigned)__popcll(mk[j]);
    }
    if (lane_id() == 0) sm.wcnt[wave_id()] = wtot;
    __syncthreads();
    unsigned wpre = 0, ptot = 0;
#pragma unroll
    for (int i = 0; i < kWaves; ++i) {
      const unsigned x = sm.wcnt[i];
      wpre += (i < wave_id()) ? x : 0u;
      ptot += x;
    }
    __syncthreads();
    unsigned pos = wpre;
    const unsigned long long lt = lanemask_lt();
#pragma unroll
    for (int j = 0; j < kItems; ++j) {
      if (kp[j]) {
        const unsigned at = pos + (unsigned)__popcll(mk[j] & lt);
        if (multi) {
          a.dst_col[ob + running + at] = cc[j];
          a.dst_w[ob + running + at] = ww[j];
        } else {
          sm.e_col[at] = cc[j];
          sm.e_w[at] = __float_as_uint(ww[j]);
        }
      }
      pos += (unsigned)__popcll(mk[j]);
    }
    running += ptot;
  }
  const Key best = block_max_key(run_key(run, vloc, S), sm.skey);
  if (FIRST) {
    if (tid == 0) a.C[v] = best.u >= 0 ? base + best.u : -1;
    return;
  }
  const unsigned K = running;
  if (K == 0) return;  // every live neighbour was matched: the row drops
  if (multi) {
    if (tid == 0) {
      const unsigned li = atomicAdd(&sout->long_rows, 1u);
      if (li < a.long_cap) a.long_out[li] = make_int4(v, (int)ob, (int)K, g);
      atomicAdd(&sout->long_kept, (unsigned long long)K);
      a.C[v] = base + best.u;
    }
    return;
  }
  // single pass: survivors are staged in LDS
  if ((int)K <= a.short_max) {
    if (tid == 0) {
      const unsigned long long old = atomicAdd(&sout->short_packed, (1ull << 32) | K);
      const int row = (int)(old >> 32);
      const long long eb = (long long)(old & 0xffffffffull);
      a.short_out[row] = make_int4(v, (int)eb, (int)K, g);
      write_tile_starts(a.tiles_out, a.tiles_cap, eb, K, row, a.tile_width);
      a.C[v] = base + best.u;
      sm.bc0 = eb;
    }
  } else if (tid == 0) {
    const unsigned long long old = atomicAdd(&sout->long_used, (unsigned long long)K);
    const long long eb = a.dst_cap - (long long)old - K;
    const unsigned li = atomicAdd(&sout->long_rows, 1u);
    if (li < a.long_cap) a.long_out[li] = make_int4(v, (int)eb, (int)K, g);
    atomicAdd(&sout->long_kept, (unsigned long long)K);
    a.C[v] = base + best.u;
    sm.bc0 = eb;
  }
  __syncthreads();
  const long long eb = sm.bc0;
  for (int p = tid; p < (int)K; p += kBlock) {
    a.dst_col[eb + p] = sm.e_col[p];
    a.dst_w[eb + p] = __uint_as_float(sm.e_w[p]);
  }
}

// Persistent phase kernel: long rows first (they take longest), then tiles,
// handed out by an atomic ticket.
template <bool FIRST>
__global__ __launch_bounds__(kBlock) void k_phase(PhaseArgs a) {
  __shared__ PhaseSmem sm;
  __shared__ int s_item;
  __shared__ unsigned s_err;
  if (threadIdx.x == 0) s_err = a.totals->err;
  __syncthreads();
  if (s_err) return;  // a check failed: touch nothing that the check could not vouch for
  Slot* sin = &a.slots[a.t % kRing];
  Slot* sout = &a.slots[(a.t + 1) % kRing];
  const unsigned long long sp = sin->short_packed;
  const int nrows = (int)(sp >> 32);
  const long long sentries = (long long)(sp & 0xffffffffull);
  const int nlong = (int)sin->long_rows;
  const int ntiles = (int)((sentries + a.tile_width - 1) / a.tile_width);
  const int total = nlong + ntiles;
  if (!FIRST && blockIdx.x == 0 && threadIdx.x == 0 && a.t <= a.log_cap) {
    a.log[a.t - 1].matched_edges = sin->matched / 2;
    a.log[a.t - 1].matched_entries = (long long)sin->matched_deg;
  }
  unsigned* ticket = FIRST ? &sin->ticket_first : &sin->ticket;
  for (;;) {
    if (threadIdx.x == 0) s_item = (int)atomicAdd(ticket, 1u);
    __syncthreads();
    const int item = s_item;
    __syncthreads();
    if (item >= total) break;
    if (item < nlong)
      long_phase<FIRST>(a, sout, item, sm.lng);
    else
      tile_phase<FIRST>(a, sout, item - nlong, ntiles, nrows, sm.tile);
    __syncthreads();
  }
}

// ---------------------------------------------------------------- mutual

__global__ __launch_bounds__(kBlock) void k_mutual(PhaseArgs a) {
  __shared__ unsigned s32[kWaves];
  __shared__ unsigned long long s64[kWaves];
  __shared__ unsigned s_err;
  if (threadIdx.x == 0) s_err = a.totals->err;
  __syncthreads();
  if (s_err) return;
  Slot* sin = &a.slots[a.t % kRing];
  const unsigned long long sp = sin->short_packed;
  const long long nshort = (long long)(sp >> 32);
  const long long nlong = (long long)sin->long_rows;
  const long long nrows = nshort + nlong;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    if (a.t <= a.log_cap) {
      a.log[a.t - 1].live_entries = (long long)(sp & 0xffffffffull) + (long long)sin->long_kept;
      a.log[a.t - 1].live_rows = nrows;
    }
    if (nrows > 0) a.totals->last_nonempty = a.t;
    // the slot of phase t+1 is reused from phase t+1-kRing: clear it before
    // the compaction of this phase fills it
    unsigned* p = reinterpret_cast<unsigned*>(&a.slots[(a.t + 1) % kRing]);
    for (int i = 0; i < (int)(sizeof(Slot) / 4); ++i) p[i] = 0u;
  }
  if (nrows == 0) return;
  unsigned cnt = 0;
  unsigned long long dsum = 0;
  // wave-uniform trip count so that the ballots below see whole waves
  for (long long r0 = (long long)blockIdx.x * kBlock; r0 < nrows; r0 += (long long)gridDim.x * kBlock) {
    const long long r = r0 + threadIdx.x;
    int g = -1;
    if (r < nrows) {
      const int4 rec = (r < nshort) ? a.short_in[r] : a.long_in[r - nshort];
      const int v = rec.x;
      const int u = a.C[v];
      g = rec.w;
      if ((unsigned)u < (unsigned)a.n && a.C[u] == v) {
        a.mate[v] = u - a.gbase[g];
        a.state[v] = 1;
        ++cnt;
        dsum += (unsigned long long)rec.z;
      }
    }
    if (a.gphase) {  // one atomic per distinct graph per wave
      unsigned long long active = __ballot(g >= 0);
      while (active) {
        const int leader = __ffsll((long long)active) - 1;
        const int gl = __shfl(g, leader, 64);
        const unsigned long long same = __ballot(g == gl);
        if (lane_id() == leader) atomicMax(&a.gphase[gl], a.t);
        active &= ~same;
      }
    }
  }
  unsigned ctot;
  (void)block_excl_sum<unsigned>(cnt, s32, ctot);
  unsigned long long dtot;
  (void)block_excl_sum<unsigned long long>(dsum, s64, dtot);
  if (threadIdx.x == 0 && ctot != 0) {
    atomicAdd(&sin->matched, ctot);
    atomicAdd(&sin->matched_deg, dtot);
    atomicAdd(&a.totals->matched, (unsigned long long)ctot);
  }
}

// ---------------------------------------------------------------- launchers

hipError_t launch_zero(Slot* slots, Totals* totals, hipStream_t s) {
  hipLaunchKernelGGL(k_zero, dim3(1), dim3(kBlock), 0, s, slots, totals);
  return hipGetLastError();
}
hipError_t launch_fill_i32(int* p, long long n, int value, hipStream_t s) {
  const long long blocks = std::min<long long>((n + kBlock - 1) / kBlock, 4096);
  hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)std::max<long long>(blocks, 1)), dim3(kBlock), 0, s, p, n, value);
  return hipGetLastError();
}
hipError_t launch_init(const InitArgs& a, int grid, hipStream_t s) {
  hipLaunchKernelGGL(k_init, dim3(grid), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}
hipError_t launch_check(const CheckArgs& a, int grid, hipStream_t s) {
  hipLaunchKernelGGL(k_check, dim3(grid), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}
hipError_t launch_first_argmax(const PhaseArgs& a, int grid, hipStream_t s) {
  hipLaunchKernelGGL(k_phase<true>, dim3(grid), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}
hipError_t launch_mutual(const PhaseArgs& a, int grid, hipStream_t s) {
  hipLaunchKernelGGL(k_mutual, dim3(grid), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}
hipError_t launch_compact(const PhaseArgs& a, int grid, hipStream_t s) {
  hipLaunchKernelGGL(k_phase<false>, dim3(grid), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

int max_blocks_per_cu_compact() {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_phase<false>, kBlock, 0) != hipSuccess || nb < 1) nb = 1;
  return nb;
}
int max_blocks_per_cu_mutual() {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_mutual, kBlock, 0) != hipSuccess || nb < 1) nb = 4;
  return nb;
}

uint64_t premix_seed(uint64_t seed) { return host_mix64(seed + kGoldenGamma); }

}  // namespace lm
