// Workgroup-level primitives for the phase kernels (wave64, 256 lanes).
#pragma once

#include <hip/hip_runtime.h>

#include "lm_internal.h"
#include "lm_key.h"

namespace lm {

__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }

// The value, computed on every lane whatever later uses it: an empty asm
// statement (no instruction) that the compiler cannot move into the branch
// of a later select, so a lane's hashes run unmasked and interleaved instead
// of one exec-masked block each.
__device__ __forceinline__ unsigned long long keep(unsigned long long x) {
  asm volatile("" : "+v"(x));
  return x;
}
__device__ __forceinline__ int wave_id() { return threadIdx.x >> 6; }
__device__ __forceinline__ unsigned long long lanemask_lt() {
  const int l = lane_id();
  return l == 0 ? 0ull : (~0ull >> (64 - l));
}

// ---- wave64 scans with DPP (row_shr 1,2,4,8 inside rows of 16 lanes, then
// row_bcast 15 / 31 across rows). Lanes whose DPP source lies outside the
// pattern keep the identity passed as `old`.
__device__ __forceinline__ unsigned dpp_u32(unsigned x, unsigned ident, int ctrl_id) {
  switch (ctrl_id) {
    case 0: return (unsigned)__builtin_amdgcn_update_dpp((int)ident, (int)x, 0x111, 0xf, 0xf, false);
    case 1: return (unsigned)__builtin_amdgcn_update_dpp((int)ident, (int)x, 0x112, 0xf, 0xf, false);
    case 2: return (unsigned)__builtin_amdgcn_update_dpp((int)ident, (int)x, 0x114, 0xf, 0xf, false);
    case 3: return (unsigned)__builtin_amdgcn_update_dpp((int)ident, (int)x, 0x118, 0xf, 0xf, false);
    case 4: return (unsigned)__builtin_amdgcn_update_dpp((int)ident, (int)x, 0x142, 0xa, 0xf, false);
    default: return (unsigned)__builtin_amdgcn_update_dpp((int)ident, (int)x, 0x143, 0xc, 0xf, false);
  }
}
// one lane to the right across the whole wave (lane 0 gets ident)
__device__ __forceinline__ unsigned dpp_wave_shr1(unsigned x, unsigned ident) {
  return (unsigned)__builtin_amdgcn_update_dpp((int)ident, (int)x, 0x138, 0xf, 0xf, false);
}

__device__ __forceinline__ unsigned wave_incl_sum_u32(unsigned x) {
#pragma unroll
  for (int c = 0; c < 6; ++c) x += dpp_u32(x, 0u, c);
  return x;
}
__device__ __forceinline__ unsigned long long wave_incl_sum_u64(unsigned long long x) {
#pragma unroll
  for (int c = 0; c < 6; ++c) {
    const unsigned lo = dpp_u32((unsigned)x, 0u, c);
    const unsigned hi = dpp_u32((unsigned)(x >> 32), 0u, c);
    x += ((unsigned long long)hi << 32) | lo;
  }
  return x;
}
__device__ __forceinline__ unsigned wave_incl_max_u32(unsigned x) {
#pragma unroll
  for (int c = 0; c < 6; ++c) x = max(x, dpp_u32(x, 0u, c));
  return x;
}

// Largest 64-bit value of the wave, returned to every lane.
__device__ __forceinline__ unsigned long long wave_max_u64(unsigned long long x) {
#pragma unroll
  for (int c = 0; c < 6; ++c) {
    const unsigned lo = dpp_u32((unsigned)x, 0u, c);
    const unsigned hi = dpp_u32((unsigned)(x >> 32), 0u, c);
    const unsigned long long y = ((unsigned long long)hi << 32) | lo;
    x = y > x ? y : x;
  }
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)x, 63);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(x >> 32), 63);
  return ((unsigned long long)hi << 32) | lo;
}

__device__ __forceinline__ Key dpp_key(const Key& x, int c) {
  Key y;
  y.w = dpp_u32(x.w, 0u, c);
  y.hhi = dpp_u32(x.hhi, 0u, c);
  y.hlo = dpp_u32(x.hlo, 0u, c);
  y.u = (int)dpp_u32((unsigned)x.u, 0xffffffffu, c);
  return y;
}

// Largest key of the wave, returned to every lane.
__device__ __forceinline__ Key wave_max_key(Key k) {
#pragma unroll
  for (int c = 0; c < 6; ++c) k = key_max(dpp_key(k, c), k);
  Key r;
  r.w = (unsigned)__builtin_amdgcn_readlane((int)k.w, 63);
  r.hhi = (unsigned)__builtin_amdgcn_readlane((int)k.hhi, 63);
  r.hlo = (unsigned)__builtin_amdgcn_readlane((int)k.hlo, 63);
  r.u = __builtin_amdgcn_readlane(k.u, 63);
  return r;
}

template <typename T>
__device__ __forceinline__ T wave_incl_sum(T x);
template <>
__device__ __forceinline__ unsigned wave_incl_sum<unsigned>(unsigned x) {
  return wave_incl_sum_u32(x);
}
template <>
__device__ __forceinline__ int wave_incl_sum<int>(int x) {
  return (int)wave_incl_sum_u32((unsigned)x);
}
template <>
__device__ __forceinline__ unsigned long long wave_incl_sum<unsigned long long>(unsigned long long x) {
  return wave_incl_sum_u64(x);
}
template <>
__device__ __forceinline__ long long wave_incl_sum<long long>(long long x) {
  return (long long)wave_incl_sum_u64((unsigned long long)x);
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

// Single-barrier variants: `sm` (kWaves slots) is written before the barrier
// and only read after it, so the caller must not write it again before the
// workgroup has passed another barrier.
template <typename T>
__device__ __forceinline__ T block_excl_sum_1b(T x, T* sm, T& total) {
  const T incl = wave_incl_sum(x);
  if (lane_id() == 63) sm[wave_id()] = incl;
  __syncthreads();
  T pre = 0, tot = 0;
#pragma unroll
  for (int i = 0; i < kWaves; ++i) {
    const T v = sm[i];
    pre += (i < wave_id()) ? v : T(0);
    tot += v;
  }
  total = tot;
  return pre + incl - x;
}

__device__ __forceinline__ unsigned block_excl_max_1b(unsigned x, unsigned* sm) {
  const unsigned incl = wave_incl_max_u32(x);
  if (lane_id() == 63) sm[wave_id()] = incl;
  __syncthreads();
  unsigned pre = 0;
#pragma unroll
  for (int i = 0; i < kWaves; ++i)
    if (i < wave_id()) pre = max(pre, sm[i]);
  return max(pre, dpp_wave_shr1(incl, 0u));
}

// Exclusive prefix max over the workgroup (identity 0).
__device__ __forceinline__ unsigned block_excl_max(unsigned x, unsigned* sm) {
  const unsigned incl = wave_incl_max_u32(x);
  if (lane_id() == 63) sm[wave_id()] = incl;
  __syncthreads();
  unsigned pre = 0;
#pragma unroll
  for (int i = 0; i < kWaves; ++i)
    if (i < wave_id()) pre = max(pre, sm[i]);
  __syncthreads();
  return max(pre, dpp_wave_shr1(incl, 0u));
}

// Smallest index i in [lo, hi) with pred(i) true, assuming pred is monotone
// (false...false true...true); hi if none. Every lane gets the answer. Each
// round evaluates pred at 256 evenly spaced points, so an array of n entries
// takes ceil(log_256 n) rounds of one memory access per lane.
template <typename Pred>
__device__ __forceinline__ long long block_lower_bound(long long lo, long long hi, Pred pred, int* sm) {
  while (hi - lo > 1) {
    const long long n = hi - lo;
    const long long step = (n + kBlock - 1) / kBlock;
    const long long idx = lo + (long long)threadIdx.x * step;
    const bool p = idx < hi ? pred(idx) : true;
    if (threadIdx.x == 0) sm[0] = kBlock;
    __syncthreads();
    if (p) atomicMin(&sm[0], (int)threadIdx.x);
    __syncthreads();
    const int f = sm[0];
    __syncthreads();
    // pred false at lo + (f-1)*step (if f > 0), true at lo + f*step
    if (f == 0) return lo;  // pred(lo) is true
    const long long nlo = lo + (long long)(f - 1) * step;  // pred(nlo) false
    const long long nhi = f >= kBlock ? hi : (lo + (long long)f * step < hi ? lo + (long long)f * step : hi);
    lo = nlo + 1;
    hi = nhi;
    if (lo >= hi) return hi;
    if (hi - lo == 1) return pred(lo) ? lo : hi;
  }
  if (hi - lo == 1) return pred(lo) ? lo : hi;
  return hi;
}

// R_1 read from the CSR: the entry position of cost c, where vertex v's row
// spans the cost units [row_ptr[v] + K v, row_ptr[v+1] + K (v+1)) (K units
// for the piece, then one per entry). Monotone in c; c = 0 gives 0 and c =
// L + K n gives L. Every lane gets the same value.
template <int K>
__device__ __forceinline__ long long csr_entry_at(const LiveSet& in, long long n, long long c, int* sm) {
  const long long v1 = block_lower_bound(
      0, n + 1, [&](long long v) { return in.csr_rp[v] + (long long)K * v > c; }, sm);
  const long long v = v1 - 1;  // cost_start(0) = 0 <= c, so v1 >= 1
  const long long u = c - (in.csr_rp[v] + (long long)K * v);
  if (u < K || v >= n) return in.csr_rp[v];
  const long long deg = in.csr_rp[v + 1] - in.csr_rp[v];
  return in.csr_rp[v] + min(u - K, deg);
}

}  // namespace lm
