// Edge key of local-max matching on the device: (weight, tie-break hash).
//
// The paper breaks weight ties by random perturbation (Section 1); the
// library fixes the perturbation as a hash of the edge so that every run and
// every schedule selects the same matching:
//   key({lo,hi}) = ( w as a number, H(seed, lo, hi) as uint64 ), lexicographic
//   H = mix( ((lo << 32) | hi) XOR mix(seed XOR gamma) )
// with mix the SplitMix64 output function. Weights are compared through an
// order-preserving map of the fp32 bit pattern (after folding -0 onto +0), so
// the compare is exact and independent of denormal flushing.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lm {

constexpr uint64_t kGoldenGamma = 0x9E3779B97F4A7C15ull;

__host__ __device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
inline uint64_t host_mix64(uint64_t z) { return mix64(z); }

// Inverse of mix64. Every step of the output function is a bijection on 64
// bits: an xor with the value shifted right by s >= 27 is undone by xoring the
// shifts by s and 2s, and the odd multipliers have inverses modulo 2^64.
__host__ __device__ __forceinline__ uint64_t unmix64(uint64_t z) {
  z = z ^ (z >> 31) ^ (z >> 62);
  z *= 0x319642B2D24D8EC3ull;  // 0x94D049BB133111EB^-1 mod 2^64
  z = z ^ (z >> 27) ^ (z >> 54);
  z *= 0x96DE1B173F119089ull;  // 0xBF58476D1CE4E5B9^-1 mod 2^64
  z = z ^ (z >> 30) ^ (z >> 60);
  return z;
}

// Order-preserving image of a finite fp32 bit pattern; 0 is below all of them.
__device__ __forceinline__ unsigned ord_weight_bits(unsigned b) {
  if (b == 0x80000000u) b = 0u;  // -0 == +0
  return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}

__device__ __forceinline__ uint64_t edge_hash(uint64_t S, unsigned a, unsigned b) {
  const unsigned lo = a < b ? a : b;
  const unsigned hi = a < b ? b : a;
  return mix64(((uint64_t)lo << 32 | (uint64_t)hi) ^ S);
}

// Renewed keys: the tie-break seed of phase t is the t-th output of a
// SplitMix64 stream started at the run's premixed seed S (the paper's Lemma 1
// draws fresh noise in every iteration), so H_t(lo, hi) = mix(pair XOR
// mix(S + t gamma)).
__host__ __device__ __forceinline__ uint64_t phase_seed(uint64_t S, int t) {
  return mix64(S + (uint64_t)t * kGoldenGamma);
}
__host__ __device__ __forceinline__ uint64_t cand_seed(uint64_t S, bool renew, int t) {
  return renew ? phase_seed(S, t) : S;
}

// The neighbour u of vertex vloc whose edge hash is h (the hash is a
// bijection of the pair, so it names the edge).
__device__ __forceinline__ int hash_neighbour(uint64_t h, uint64_t S, unsigned vloc) {
  const uint64_t pair = unmix64(h) ^ S;
  const unsigned lo = (unsigned)(pair >> 32), hi = (unsigned)pair;
  return (int)(lo == vloc ? hi : lo);
}

// A candidate with its full key; u = -1 is the dummy below every edge.
struct Key {
  unsigned w, hhi, hlo;
  int u;
};

__device__ __forceinline__ Key key_ident() {
  Key k;
  k.w = 0u;
  k.hhi = 0u;
  k.hlo = 0u;
  k.u = -1;
  return k;
}

__device__ __forceinline__ bool key_gt(const Key& a, const Key& b) {
  if (a.w != b.w) return a.w > b.w;
  if (a.hhi != b.hhi) return a.hhi > b.hhi;
  return a.hlo > b.hlo;
}

__device__ __forceinline__ Key key_max(const Key& a, const Key& b) { return key_gt(b, a) ? b : a; }

// Running best of one lane over consecutive entries of one row. The hash is
// evaluated only when a weight tie has to be decided.
struct Best {
  unsigned w;
  int u;
  uint64_t h;
  bool hv;
};

__device__ __forceinline__ Best best_ident() {
  Best r;
  r.w = 0u;
  r.u = -1;
  r.h = 0ull;
  r.hv = false;
  return r;
}

__device__ __forceinline__ void best_update(Best& r, unsigned w, int u, unsigned vloc, uint64_t S) {
  if (w > r.w) {
    r.w = w;
    r.u = u;
    r.hv = false;
  } else if (w == r.w) {  // r.u is a real edge: every real weight maps above 0
    const uint64_t h = edge_hash(S, vloc, (unsigned)u);
    if (!r.hv) {
      r.h = edge_hash(S, vloc, (unsigned)r.u);
      r.hv = true;
    }
    if (h > r.h) {
      r.u = u;
      r.h = h;
    }
  }
}

__device__ __forceinline__ Key best_key(const Best& r, unsigned vloc, uint64_t S) {
  if (r.u < 0) return key_ident();
  const uint64_t h = r.hv ? r.h : edge_hash(S, vloc, (unsigned)r.u);
  Key k;
  k.w = r.w;
  k.hhi = (unsigned)(h >> 32);
  k.hlo = (unsigned)h;
  k.u = r.u;
  return k;
}

}  // namespace lm
