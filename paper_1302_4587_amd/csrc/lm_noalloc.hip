// Allocation-free single-graph solve (lm_match_noalloc, include/lm.h).
//
// The working buffers of the solve (candidates, matched flags, the ping-pong
// live sets, run tables, per-workgroup partials and counters) are carved from
// one file-scope device array instead of the context's pool, so a call makes
// no device or pinned allocation. The array is per device: each GPU the
// library runs on holds its own copy, at its own address, until the process
// ends. Host code never passes the array's name to a kernel or a copy; it uses
// the device address that hipGetSymbolAddress returned for the current device
// at context creation.
#include <hip/hip_runtime.h>

#include <cstring>
#include <mutex>

#include "lm.h"
#include "lm_internal.h"
#include "lm_runtime.h"

namespace lm {

constexpr size_t kScratchBytes = (size_t)LM_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices];

// Called with `dev` current (lm_create): looks the array's device address up
// once per device.
lm_status noalloc_setup(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return LM_EDEVICE;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[dev]) return LM_OK;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p) {
    (void)hipGetLastError();
    return LM_EDEVICE;
  }
  g_scratch_ptr[dev] = p;
  return LM_OK;
}

static void* scratch_of(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  return g_scratch_ptr[dev];
}

// The single-graph tables (first vertex 0, premixed seed, vertex offsets
// {0, n}) written by one lane from kernel arguments: no host copy.
__global__ void k_single_tables(int* gbase, unsigned long long* gseed, long long* vtxoff, unsigned long long S,
                                long long n) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    gbase[0] = 0;
    gseed[0] = S;
    vtxoff[0] = 0;
    vtxoff[1] = n;
  }
}

}  // namespace lm

using namespace lm;

extern "C" lm_status lm_match_noalloc(lm_ctx* c, const lm_csr* g, uint64_t seed, int32_t* mate, uint32_t flags,
                                      void* stream, lm_stats* st) {
  if (!c || !g) return LM_EINVAL;
  const uint32_t need = LM_IN_DEVICE | LM_OUT_DEVICE;
  if ((flags & need) != need) return LM_EINVAL;  // host inputs would need staging buffers
  if (flags & ~(need | LM_CHECK_GRAPH)) return LM_EINVAL;
  const int64_t N = g->n, nnz = g->nnz;
  if (N < 0 || nnz < 0) return LM_EINVAL;
  if (N > 0 && (!g->row_ptr || !mate)) return LM_EINVAL;
  if (nnz > 0 && !g->col) return LM_EINVAL;  // w == NULL: unweighted graph
  if (N >= ((int64_t)1 << 31) || nnz >= ((int64_t)1 << 31) - 65536) return LM_ETOOBIG;
  if (carve_work(N, nnz, 1, nullptr, nullptr) > kScratchBytes) return LM_ETOOBIG;
  std::lock_guard<std::mutex> lk(mutex_of(c));
  Solver& S = solver_of(c);
  if (S.busy_server) return LM_EINVAL;
  if (st) {
    st->phases = 0;
    st->matched_edges = 0;
    st->device_ms = 0.0;
    st->bytes_alg = 0.0;
    st->log_len = 0;
    st->matched_weight = 0.0;
  }
  if (N == 0) return LM_OK;
  if (hipSetDevice(S.dev) != hipSuccess) return LM_EDEVICE;
  if (S.async_pending) {  // a stream-ordered solve may still use the context's mapped records
    if (hipEventSynchronize(S.e_async) != hipSuccess) return LM_EDEVICE;
    S.async_pending = false;
  }
  void* base = scratch_of(S.dev);
  if (!base) return LM_EDEVICE;
  Work wk;
  (void)carve_work(N, nnz, 1, base, &wk);
  hipStream_t s = (hipStream_t)stream;
  hipLaunchKernelGGL(k_single_tables, dim3(1), dim3(64), 0, s, wk.gbase, wk.gseed, wk.vtxoff,
                     (unsigned long long)premix_seed(seed), (long long)N);
  if (hipGetLastError() != hipSuccess) return LM_EDEVICE;
  Problem p;
  p.N = N;
  p.nnz = nnz;
  p.G = 1;
  p.row_ptr = (const long long*)g->row_ptr;
  p.col = g->col;
  p.w = g->w;
  p.vtx_off = wk.vtxoff;
  p.mate = mate;
  p.gphase = nullptr;
  lm_stats local;
  std::memset(&local, 0, sizeof(local));
  lm_stats* sp = st ? st : &local;
  return S.run(p, wk, s, flags, sp);
}
