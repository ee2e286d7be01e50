// Total weight of the matching, w(M) = sum of w(e) over e in M (the quantity
// the approximation guarantee of Section 1 bounds: at least half of the
// maximum weight), computed after a solve on request (LM_WEIGHT_SUM).
//
// Every matched vertex v finds the entry (v, mate[v]) in its own input row and
// adds its weight, so each matched edge is counted from both endpoints and the
// total is halved (exact in binary). The additions follow a fixed order for a
// given vertex count: each lane adds its vertices in increasing order, a
// workgroup adds its lanes with a fixed tree, and one workgroup adds the
// workgroup sums the same way. Repeated calls therefore give identical values.
#include <hip/hip_runtime.h>

#include "lm_runtime.h"

namespace lm {
namespace {

constexpr int kWsBlock = 256;
constexpr int kLongRow = 64;  // longer rows are searched by the whole wave

__device__ __forceinline__ double block_sum_fixed(double x, double* s) {
  const int tid = threadIdx.x;
  s[tid] = x;
  __syncthreads();
  for (int o = kWsBlock / 2; o > 0; o >>= 1) {
    if (tid < o) s[tid] += s[tid + o];
    __syncthreads();
  }
  return s[0];
}

// Partial sums per workgroup. mate and col are in the graph's local ids
// (each graph of a batch), so a row entry matches when col == mate[v].
__global__ __launch_bounds__(kWsBlock) void k_weight_partial(const long long* row_ptr, const int* col, const float* w,
                                                             const int* mate, long long N, double* partial) {
  __shared__ double s[kWsBlock];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  double acc = 0.0;
  const long long stride = (long long)gridDim.x * kWsBlock;
  for (long long base = (long long)blockIdx.x * kWsBlock; base < N; base += stride) {
    const long long v = base + tid;
    const int u = v < N ? mate[v] : -1;
    long long e0 = 0, e1 = 0;
    if (u >= 0 && w) {
      e0 = row_ptr[v];
      e1 = row_ptr[v + 1];
    }
    const bool wide = e1 - e0 > kLongRow;
    if (u >= 0 && !w) {
      acc += 1.0;  // unweighted graph: every edge weighs 1
    } else if (u >= 0 && !wide) {
      for (long long e = e0; e < e1; ++e)
        if (col[e] == u) {
          acc += (double)w[e];
          break;
        }
    }
    // long rows: the wave searches each one together; the owner lane adds
    unsigned long long m = __ballot(u >= 0 && w && wide);
    while (m) {
      const int l = __ffsll((long long)m) - 1;
      m &= m - 1;
      const int uu = __shfl(u, l);
      const long long b0 = ((long long)__shfl((int)(e0 >> 32), l) << 32) | (unsigned)__shfl((int)e0, l);
      const long long b1 = ((long long)__shfl((int)(e1 >> 32), l) << 32) | (unsigned)__shfl((int)e1, l);
      float found = 0.f;
      bool hit = false;
      for (long long e = b0 + lane; e < b1; e += 64)
        if (!hit && col[e] == uu) {
          found = w[e];
          hit = true;
        }
      const unsigned long long hm = __ballot(hit);
      if (hm) {
        const float fw = __shfl(found, __ffsll((long long)hm) - 1);
        if (lane == l) acc += (double)fw;
      }
    }
  }
  const double t = block_sum_fixed(acc, s);
  if (tid == 0) partial[blockIdx.x] = t;
}

__global__ __launch_bounds__(kWsBlock) void k_weight_final(const double* partial, int nb, double* out) {
  __shared__ double s[kWsBlock];
  double acc = 0.0;
  for (int i = threadIdx.x; i < nb; i += kWsBlock) acc += partial[i];
  const double t = block_sum_fixed(acc, s);
  if (threadIdx.x == 0) out[0] = 0.5 * t;
}

}  // namespace

int weight_sum_grid(long long N) {
  const long long g = (N + kWsBlock - 1) / kWsBlock;
  return (int)std::max(1LL, std::min<long long>(g, kWeightSumMaxGrid));
}

hipError_t launch_weight_sum(const long long* row_ptr, const int* col, const float* w, const int* mate, long long N,
                             double* scratch, hipStream_t s) {
  const int nb = weight_sum_grid(N);
  hipLaunchKernelGGL(k_weight_partial, dim3(nb), dim3(kWsBlock), 0, s, row_ptr, col, w, mate, N, scratch);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_weight_final, dim3(1), dim3(kWsBlock), 0, s, scratch, nb, scratch + kWeightSumMaxGrid);
  return hipGetLastError();
}

}  // namespace lm
