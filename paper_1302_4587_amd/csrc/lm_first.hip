// First argmax of a single weighted graph read straight from its CSR (R_1),
// gfx950. (Unweighted graphs keep the piece-window kernel of lm_kernels.hip,
// which measured faster on R-MAT scale 24: 2.5 ms against 3.2 ms.)
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
// the weight pass. Rows cut at range boundaries leave a partial result for
// the plan kernel, as the other stream kernels do.
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
  __device__ __forceinline__ void add(unsigned w, int u, unsigned v, unsigned long long S) {
    best_update(b, w, u, v, S);
  }
  __device__ __forceinline__ void add_hash(unsigned long long, int) {}
  __device__ __forceinline__ int u() const { return b.u; }
  __device__ __forceinline__ unsigned w() const { return b.w; }
  __device__ __forceinline__ unsigned long long h(unsigned v, unsigned long long S) const {
    return b.hv ? b.h : edge_hash(S, v, (unsigned)b.u);
  }
};
template <>
struct Seg<true> {
  unsigned long long hb;
  int ub;
  __device__ __forceinline__ void add(unsigned, int, unsigned, unsigned long long) {}
  __device__ __forceinline__ void reset() {
    hb = 0ull;
    ub = -1;
  }
  __device__ __forceinline__ void add_hash(unsigned long long h, int u) {
    if (ub < 0 || h > hb) {
      hb = h;
      ub = u;
    }
  }
  __device__ __forceinline__ int u() const { return ub; }
  __device__ __forceinline__ unsigned w() const { return 1u; }
  __device__ __forceinline__ unsigned long long h(unsigned, unsigned long long) const { return hb; }
};

__device__ __forceinline__ Part part_of(int v, int flags, unsigned w, unsigned long long h, unsigned long long S) {
  Part p;
  p.v = v;
  p.flags = flags;
  p.kept = 0;
  p.out_row = -1;
  p.w = w;
  p.hhi = (unsigned)(h >> 32);
  p.hlo = (unsigned)h;
  p.u = hash_neighbour(h, S, (unsigned)v);
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

template <bool UNW>
__device__ void first_range(const StreamArgs& a, const Ctl& ctl, int b, FirstSmem& sm, unsigned long long S,
                            bool vec) {
  constexpr unsigned kUnitOrd = 0xBF800000u;  // ordered image of 1.0f
  const int tid = threadIdx.x;
  const long long* rp = a.in.csr_rp;
  const int* col = a.in.col;
  const float* wt = a.in.w;
  const long long n = ctl.pieces;
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
    // ---- stage 1: the row slot of each of the lane's entries (-1: not the lane's)
    int rs[kFIt];
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
        rs[i] = in && cv[i] >= 0 && cv[i] < n ? rr : -1;
      }
    }
    // ---- stage 2 (unweighted): every hash at once, independent of each other
    unsigned long long hv[kFIt];
    if (UNW) {
#pragma unroll
      for (int i = 0; i < kFIt; ++i) hv[i] = edge_hash(S, (unsigned)(vc + max(rs[i], 0)), (unsigned)cv[i]);
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
      int cur = r;
      bool started = wrp[r] >= lo;
#pragma unroll
      for (int i = 0; i < kFIt; ++i) {
        if (rs[i] < 0) continue;
        if (rs[i] != cur) {  // the entry opens another row
          if (started) {
            if (sg.u() >= 0) a.c.C[vc + cur] = sg.u();
          } else {
            rA = cur;
            sA = sg;
          }
          cur = rs[i];
          started = true;
          sg.reset();
        }
        if (UNW) sg.add_hash(hv[i], cv[i]);
        else sg.add(ord_weight_bits(__float_as_uint(wv[i])), cv[i], (unsigned)(vc + cur), S);
      }
      const bool ends = wrp[cur + 1] <= hi;
      if (started && ends) {
        if (sg.u() >= 0) a.c.C[vc + cur] = sg.u();
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
    if (rA >= 0 && sA.u() >= 0 && (UNW || sA.w() == sw[rA])) atomicMax(&sh[rA], sA.h((unsigned)(vc + rA), S));
    if (waveB) {
      const bool at = sB.u() >= 0 && (UNW || sB.w() == sw[rB0]);
      const unsigned long long hm = wave_max_u64(at ? sB.h((unsigned)(vc + rB0), S) : 0ull);
      const bool any = __ballot(at) != 0ull;  // (every lane takes part in the ballot)
      if (lane_id() == 0 && any) atomicMax(&sh[rB0], hm);
    } else if (rB >= 0 && sB.u() >= 0 && (UNW || sB.w() == sw[rB])) {
      atomicMax(&sh[rB], sB.h((unsigned)(vc + rB), S));
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
      if (wrp[i + 1] <= tend) {  // the row ends in this tile
        if (cutl) sm.pf = part_of((int)v, 0, w, hh, S);
        else a.c.C[v] = hash_neighbour(hh, S, (unsigned)v);
      } else if (tend == E1) {  // the row goes on past the range
        const Part p = part_of((int)v, cutl ? kPartSingle : 0, w, hh, S);
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

}  // namespace

template <bool UNW>
__global__ __launch_bounds__(kBlock) void k_first_csr(StreamArgs a) {
  __shared__ FirstSmem sm;
  if (threadIdx.x == 0) sm.err = a.c.totals->err;
  __syncthreads();
  if (sm.err) return;
  Ctl ctl = *a.in.ctl;
  if (ctl.Pf > 0) ctl.P = ctl.Pf;  // the first argmax's own split of R_1
  const unsigned long long S = cand_seed(a.c.gseed[0], a.c.renew, a.cand_phase);
  const bool vec = (((unsigned long long)a.in.col | (UNW ? 0ull : (unsigned long long)a.in.w)) & 15ull) == 0ull;
  for (int b = blockIdx.x; b < ctl.P; b += gridDim.x) first_range<UNW>(a, ctl, b, sm, S, vec);
}

hipError_t launch_first_csr(const StreamArgs& a, int grid, hipStream_t s, bool unweighted, hipEvent_t* ev) {
  if (unweighted) {
    if (ev) hipExtLaunchKernelGGL(k_first_csr<true>, dim3(grid), dim3(kBlock), 0, s, ev[0], ev[1], 0, a);
    else hipLaunchKernelGGL(k_first_csr<true>, dim3(grid), dim3(kBlock), 0, s, a);
  } else {
    if (ev) hipExtLaunchKernelGGL(k_first_csr<false>, dim3(grid), dim3(kBlock), 0, s, ev[0], ev[1], 0, a);
    else hipLaunchKernelGGL(k_first_csr<false>, dim3(grid), dim3(kBlock), 0, s, a);
  }
  return hipGetLastError();
}

int first_csr_blocks_per_cu(bool unweighted) {
  int nb = 0;
  const hipError_t e = unweighted
                           ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_first_csr<true>, kBlock, 0)
                           : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_first_csr<false>, kBlock, 0);
  if (e != hipSuccess || nb < 1) nb = 1;
  return nb;
}

}  // namespace lm
