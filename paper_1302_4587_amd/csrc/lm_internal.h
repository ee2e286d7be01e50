// Internal layout shared by the phase kernels and the host driver of the
// local-max matching library. Not part of the public C ABI (include/lm.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lm {

// Workgroup shape: 4 waves of 64 lanes; a tile pass covers kCap live entries
// (kItems per lane).
constexpr int kBlock = 256;
constexpr int kWaves = kBlock / 64;
constexpr int kItems = 8;
constexpr int kCap = kBlock * kItems;  // 2048
constexpr int kMaxRowsPerTile = kCap;  // every live row has >= 1 entry
constexpr int kRing = 4;               // phase counter slots in flight
constexpr unsigned kDropBit = 0x80000000u;

// Per-phase counters. Slot t % kRing describes the live set R_t (written by
// the kernel that built it) and holds the work counters of phase t.
struct alignas(64) Slot {
  unsigned long long short_packed;  // (rows << 32) | entries of R_t's short list
  unsigned long long long_used;     // entries reserved at the top of R_t's buffer
  unsigned long long long_kept;     // live entries held by R_t's long rows
  unsigned long long matched_deg;   // sum of live degree over rows matched in phase t
  unsigned int long_rows;           // rows in R_t's long list
  unsigned int matched;             // vertices matched in phase t
  unsigned int ticket;              // work tickets of the compaction in phase t
  unsigned int ticket_first;        // work tickets of the first argmax (R_1 only)
  unsigned int pad[4];
};

// Host-visible record, same layout as lm_phase_rec.
struct LogRec {
  long long live_entries;
  long long live_rows;
  long long matched_edges;
  long long matched_entries;
};

struct Totals {
  unsigned int err;              // LM_ERR_* bits found by the device checks
  int last_nonempty;             // largest phase index with a live row
  unsigned long long matched;    // vertices matched so far
};

enum : unsigned {
  kErrRowPtr = 1u,     // row_ptr not nondecreasing / wrong ends
  kErrDegree = 2u,     // a row too long for 32-bit offsets
  kErrColRange = 4u,   // neighbour id out of range
  kErrSelfLoop = 8u,   // self-loop
  kErrWeight = 16u,    // NaN or infinite weight
  kErrTile = 32u,      // internal: a tile exceeded its capacity
};

// A live row: global vertex id, physical offset of its first live entry in the
// current entry buffer, live degree, graph index.
// (int4: x = v, y = off, z = deg, w = g)

struct PhaseArgs {
  Slot* slots;
  LogRec* log;
  Totals* totals;
  int log_cap;
  int t;            // phase index, 1-based
  int short_max;    // rows of live degree <= short_max use the shared tiles
  int tile_width;   // virtual entries per tile start window = kCap - short_max

  int n;                   // vertices of the union; ids outside [0, n) are ignored
  long long long_cap;      // capacity of long_out
  long long tiles_cap;     // capacity of tiles_out
  int* C;                  // candidate partner per vertex (global id)
  unsigned char* state;    // 1 = matched
  int* mate;               // output, local ids
  const int* gbase;        // first global vertex of each graph
  const unsigned long long* gseed;  // per-graph premixed seed
  int* gphase;             // optional: last phase in which each graph had a live row

  // live set R_t
  const int4* short_in;
  const int4* long_in;
  const int* tiles_in;     // first row of each tile
  const int* src_col;
  const float* src_w;

  // live set R_{t+1}
  int4* short_out;
  int4* long_out;
  int* tiles_out;
  int* dst_col;
  float* dst_w;
  long long dst_cap;       // entries in dst_col / dst_w
};

struct InitArgs {
  Slot* slot1;
  Totals* totals;
  const long long* row_ptr;  // N+1
  long long nnz;
  int n;                     // N (vertices of the union)
  int graphs;
  const long long* vtx_off;  // graphs+1 (device)
  int short_max;
  int tile_width;
  int* mate;
  unsigned char* state;
  int4* short_out;
  int4* long_out;
  int* tiles_out;
  long long long_cap;
  long long tiles_cap;
};

struct CheckArgs {
  Totals* totals;
  long long nnz;             // entries the caller passed
  const long long* row_ptr;
  const int* col;
  const float* w;
  int n;
  int graphs;
  const long long* vtx_off;
};

// Kernel launchers (lm_kernels.hip).
hipError_t launch_zero(Slot* slots, Totals* totals, hipStream_t s);
hipError_t launch_fill_i32(int* p, long long n, int value, hipStream_t s);
hipError_t launch_init(const InitArgs& a, int grid, hipStream_t s);
hipError_t launch_check(const CheckArgs& a, int grid, hipStream_t s);
hipError_t launch_first_argmax(const PhaseArgs& a, int grid, hipStream_t s);
hipError_t launch_mutual(const PhaseArgs& a, int grid, hipStream_t s);
hipError_t launch_compact(const PhaseArgs& a, int grid, hipStream_t s);
// occupancy-derived persistent grid sizes per CU
int max_blocks_per_cu_compact();
int max_blocks_per_cu_mutual();

// Host mirror of the device tie-break premix (SplitMix64 first output).
uint64_t premix_seed(uint64_t seed);

}  // namespace lm
