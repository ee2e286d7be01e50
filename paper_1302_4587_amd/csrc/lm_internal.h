// Internal layout shared by the phase kernels and the host driver of the
// local-max matching library. Not part of the public C ABI (include/lm.h).
//
// Live set R_t of phase t
// -----------------------
// The live entries are a sequence of row *pieces*. A piece is a record
//   int4 { x = v (global vertex id), y = off (first entry in the entry buffer),
//          z = len (entries), w = g (graph index) | kHeadBit | kMatchedBit }
// and the pieces are grouped into *runs*: a run is a slice of the piece
// buffer whose pieces lie back to back in the entry buffer, in the same order.
// Concatenating the runs in index order gives a "virtual" entry sequence of
// length L_t. All pieces of one vertex are adjacent in that sequence and
// exactly one of them carries kHeadBit. A vertex has more than one piece only
// where a workgroup boundary cut its row in the previous phase.
//
// Phase kernels never allocate with atomics: workgroup b of a compaction owns
// the virtual range [L b / P, L (b+1) / P) and writes its survivors to the same
// range of the destination buffer, producing exactly one run. A single-block
// plan kernel stitches the rows that were cut at range boundaries and scans
// the run table for the next phase.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lm {

constexpr int kBlock = 256;            // lanes per workgroup (4 waves of 64)
constexpr int kWaves = kBlock / 64;
constexpr int kItems = 8;              // entries per lane per round of k_init (the stream kernels pick their own)
constexpr int kCap = kBlock * kItems;  // vertices per round of k_init; the smallest range a workgroup takes
constexpr int kLatePPL = 3;                 // pieces per lane in compactions after the first
constexpr int kLatePPLUnw = 2;              // the same for unweighted graphs (every entry hashed: more resident waves pay)
constexpr int late_ppl(bool unweighted) { return unweighted ? kLatePPLUnw : kLatePPL; }
constexpr int kMutualRound = kBlock * 4;    // pieces per mutual-check round of a workgroup
constexpr int kMaxBlocks = 4096;       // run table capacity
constexpr int kMaxFirstRanges = 8192;  // ranges of a first argmax (partial-result capacity)
constexpr int kPieceCost = 8;          // entries one piece weighs when R_1 is split from the CSR (compaction)
constexpr int kPieceCostFirst = 4;     // the same for the first argmax (measured on R-MAT and RGG)
constexpr int kPlanThreads = 1024;
constexpr unsigned kDropBit = 0x80000000u;
constexpr int kHeadBit = (int)0x80000000u;
constexpr int kMatchedBit = 0x40000000;
constexpr int kGraphMask = 0x3fffffff;

struct Run {
  int row_begin;   // first piece of the run in the piece buffer
  int row_count;   // pieces
  int phys_begin;  // entry-buffer offset of the run's first entry
  int ent_count;   // entries
};

// Description of a live set, written by the plan kernel.
struct Ctl {
  long long L;     // live entries
  int nruns;
  int pieces;      // pieces in all runs
  int heads;       // live vertices
  int P;           // workgroups for the compaction over this live set
  int Pm;          // workgroups for the mutual check over this live set
  int Pf;          // workgroups for the first argmax over this live set (R_1), 0: P
};

// A row cut by a workgroup boundary: the partial result of one side.
struct Part {
  int v;        // vertex (global), -1 = none
  int flags;    // kPartSingle: the segment spans the whole range of the block
  int kept;     // survivors of this part
  int out_row;  // piece written for it in the next live set, -1 = none
  unsigned w, hhi, hlo;
  int u;        // best neighbour (global id) or -1
};
enum : int { kPartSingle = 1 };

struct BlockStat {
  long long loaded;       // live entries read (unmatched pieces)
  long long matched_len;  // entries skipped because their row was matched
  int pieces_out;
  int pad;
};

struct LogRec {  // same layout as lm_phase_rec
  long long live_entries;
  long long live_rows;
  long long matched_edges;
  long long matched_entries;
};

struct Totals {
  unsigned int err;
  int last_nonempty;
  unsigned long long matched;
  int t;    // current phase (1-based): read by the mutual check, advanced by the plan kernel
  int tail_from;  // guarded phases: the live set R_t the tail kernel takes over (0 = none yet)
  unsigned long long fp[2];  // LM_CHECK_GRAPH: fingerprints of the entries and of their mirrors
  unsigned far, samp;        // sampled first entries of R_1 whose neighbour id is far from the row's
};

// One graph whose neighbour ids are mostly far from their row's id (sampled
// by k_init): the mutual check also sets a bit per matched vertex and the
// compactions read a neighbour's matched state from these bits (N / 8 bytes,
// which stay in L2) instead of the byte array.
constexpr long long kBitsMinN = 1ll << 22;  // smaller state arrays fit L2 as bytes
constexpr unsigned kFarIds = 1u << 15;      // "far": |u - v| at least this
__host__ __device__ __forceinline__ bool bits_on(const Totals* t) {
  return t->samp > 0 && 4ull * t->far > 3ull * t->samp;
}

// What the host loop needs after each plan, written by the plan kernel into
// mapped coherent pinned host memory: the record is stored, made visible to
// the system, and only then tagged (tag = gen << 32 | t), so the host polls the
// slot of R_t (t & (kMirrorSlots - 1)) with no event or copy on the stream.
// The tag names both the solve and the live set: a record left in the slot by
// the same solve kMirrorSlots phases earlier never passes for R_t. The tail
// kernel leaves the solve's final record in the extra slot kMirrorSlots.
struct PhaseMirror {
  long long L;                 // live entries of the live set just planned
  unsigned long long matched;  // matched entries so far (both directions)
  int pieces;                  // its pieces
  int t;                       // its index t (R_t)
  unsigned gen;                // solve that wrote the record
  unsigned err;                // error flags so far
  int last_nonempty;           // last phase that had live rows
  int pad;
  unsigned long long tag;      // (gen << 32) | t once the record is complete
};
constexpr int kMirrorSlots = 64;
__host__ __device__ inline unsigned long long mirror_tag(unsigned gen, int t) {
  return ((unsigned long long)gen << 32) | (unsigned)t;
}

enum : unsigned {
  kErrRowPtr = 1u,
  kErrDegree = 2u,
  kErrColRange = 4u,
  kErrSelfLoop = 8u,
  kErrWeight = 16u,
  kErrInternal = 32u,
  kErrStall = 64u,  // a phase removed nothing: the input is not symmetric
  kErrAsym = 128u,  // LM_CHECK_GRAPH: the entries and their mirrors differ (fingerprints)
};

// Inputs common to the phase kernels.
struct Common {
  Totals* totals;
  int n;                            // vertices of the union
  int* C;                           // candidate per vertex (global id)
  unsigned char* state;             // 1 = matched
  int* mate;                        // output, local ids
  const int* gbase;                 // first vertex of each graph
  const unsigned long long* gseed;  // premixed tie-break seed per graph
  int* gphase;                      // optional: last phase with a live row per graph
  int graphs;                       // 1: every piece belongs to graph 0 (no table lookups)
  int guard = 0;                    // phase kernels of a device-controlled solve: do nothing
                                    // once the tail kernel has taken the live set over
  unsigned* mbits = nullptr;        // matched bits (one graph, N >= kBitsMinN): cleared by k_init,
                                    // set by the mutual check while bits_on(totals)
  int renew = 0;                    // renewed keys: the candidates of phase t break ties with
                                    // phase_seed(seed, t) instead of the seed
};

// A live set as the kernels see it.
struct LiveSet {
  const Ctl* ctl;
  const Run* runs;
  const long long* epre;  // nruns+1 entry prefix
  const int* rpre;        // nruns+1 piece prefix
  int4* rows;
  const int* col;
  const float* w;
  const long long* csr_rp;  // R_1 read from the input CSR (its row_ptr), or nullptr: piece records
};

struct StreamArgs {
  Common c;
  LiveSet in;
  int cand_phase;    // the phase whose candidates this launch computes (renewed keys)
  // outputs (compaction only)
  Run* runs_out;
  int4* rows_out;
  int* dst_col;
  float* dst_w;
  Part* parts;       // 2 per workgroup: [first, last]
  BlockStat* bstat;
};

struct MutualArgs {
  Common c;
  LiveSet in;
  int* mcount;  // matched vertices per workgroup
  int census;   // only record gphase[g] = t for graphs with a live row (no matching)
};

struct PlanArgs {
  Common c;
  int mode;          // kPlanFix | kPlanPrefix | kPlanLog | kPlanTick
  int first;         // fixup after the first argmax (no pieces written)
  // fixup of the compaction (or first argmax) that just ran
  const Ctl* ctl_prev;  // live set it consumed
  Part* parts;
  BlockStat* bstat;
  int4* rows_out;
  // scan of the run table it produced
  const Run* runs_new;
  int nruns_new;         // -1: take ctl_prev->P
  long long* epre_new;
  int* rpre_new;
  Ctl* ctl_new;
  int pcap, pmcap;       // workgroup caps for the next phase
  int pcap_first;        // workgroup cap of the first argmax over the new live set (R_1), 0: none
  const BlockStat* heads_of_runs;  // kPlanPrefix, R_1 read from the CSR: live rows per run (pieces_out)
  int min_per_block;     // virtual entries per compaction workgroup at least
  int pieces_per_block;  // pieces per compaction workgroup at least (0: no bound)
  // log
  const int* mcount;
  LogRec* log;
  int log_cap;
  PhaseMirror* mirror;  // optional (kPlanPrefix): record of the live set just planned
  unsigned gen;
  long long tail_at;    // device-controlled solve: a planned live set of at most this many
                        // entries is left to the tail kernel (totals->tail_from); 0: never
};
// kPlanLog writes the log record of the phase totals->t; kPlanTick then
// advances totals->t (after the compaction of that phase).
enum : int { kPlanFix = 1, kPlanPrefix = 2, kPlanLog = 4, kPlanTick = 8 };

// R_1 of a single graph can instead be read straight from the input CSR: no
// piece records, piece k is vertex k (its row from row_ptr, empty rows as
// pieces of length 0), run b covers the vertices of init workgroup b, and the
// matched flag is state[v]. Workgroup ranges then split entries plus a fixed
// cost per piece (kPieceCost, kPieceCostFirst), so no range walks a long
// stretch of empty rows.
//
// Live-set construction for vertices [vfirst, vfirst + vcount) of the
// vertex space: row_ptr (vcount + 1 offsets into the entry buffer, from ebase
// to ebase + nnz) and vtx_off (graphs + 1 offsets, relative to vfirst) are
// indexed from vfirst. Pieces go to rows_out[rows_base ...], run b to
// runs_out[runs_base + b]; graph i of the group is table slot slot_of[i]
// (slot_of == nullptr: slot i).
struct InitArgs {
  Common c;
  const long long* row_ptr;
  long long nnz;
  long long ebase;
  long long vfirst, vcount;
  int graphs;
  const long long* vtx_off;
  const int* slot_of;
  int nblocks;        // workgroups (= runs produced)
  int rows_base, runs_base;
  Run* runs_out;
  int4* rows_out;
  const int* col = nullptr;  // with c.mbits: the input column ids, for the locality sample
  int csr;           // 1: no piece records (R_1 read from the CSR): C[v] = -1 for every vertex,
                     // bstat[b].pieces_out = non-empty rows of workgroup b
  BlockStat* bstat;
};

// Device-side tail of the phase loop (k_tail): one persistent launch runs
// every phase from the current live set R_c on, with software grid barriers
// between the mutual check and the compaction of each phase. Its live rows are
// records {v, entry offset, live length, graph}. Workgroup b writes the rows it
// keeps into a segment of its own of the next row list (rows of at most
// kTailShort live entries from the segment's front, one lane each next phase;
// longer ones from its back, one wave each), and its counts into a table that
// every workgroup reads after the barrier: no counter is shared. A row keeps
// its entry offset for the rest of the solve: phase t reads its entries from
// one entry buffer and writes the survivors to the same offset of the other.
constexpr int kTailBlock = 1024;
constexpr int kTailMaxBlocks = 128;
constexpr int kTailArrive = 16;  // barrier arrival counters (workgroup b uses b % kTailArrive)
constexpr int kTailShort = 16;

struct TailSeg {
  int base, cap;             // the segment: rows [base, base + cap) of the row buffer
  int ns, nl;                // short rows at [base, base + ns), long rows at [base + cap - nl, base + cap)
  long long kept;            // live entries of those rows
  long long md;              // entries of the rows this workgroup dropped as matched
  unsigned long long mv;     // vertices this workgroup matched
};

struct TailCtl {
  unsigned arrive[kTailArrive][32];  // one counter per 128-byte line
  unsigned top[32];
  unsigned gen[32];
  unsigned abort[32];
  TailSeg seg[2][kTailMaxBlocks];    // segment table of the list phase t writes: seg[t & 1]
};

struct TailArgs {
  Common c;
  TailCtl* tc;
  // both live-set buffers of the phase kernels: R_c is set (c - 1) & 1
  const Ctl* ctl[2];
  const Run* runs[2];
  const long long* epre[2];
  const int* rpre[2];
  int4* rows[2];       // R_c's piece records; afterwards the tail's row lists
  int row_cap;         // records per row buffer
  int* ecol[2];
  float* ew[2];        // nullptr: unweighted
  const long long* csr_rp;  // R_1 of one graph read from the input CSR, else nullptr
  const int* in_col;        // the input entries (R_1's)
  const float* in_w;
  LogRec* log;
  int log_cap;
  PhaseMirror* final_rec;  // the solve's final record
  unsigned gen;
  unsigned long long spin_ticks;  // a barrier wait longer than this (device wall clock) aborts the solve
};

struct CheckArgs {
  Totals* totals;
  long long nnz;
  const long long* row_ptr;
  const int* col;
  const float* w;
  int n;
  int graphs;
  const long long* vtx_off;
};

hipError_t launch_zero(Ctl* ctl, int nctl, Totals* totals, hipStream_t s, TailCtl* tc = nullptr);
hipError_t launch_fill_i32(int* p, long long n, int value, hipStream_t s);

hipError_t launch_add_i64(long long* p, long long n, long long delta, hipStream_t s);
hipError_t launch_check(const CheckArgs& a, int grid, hipStream_t s);
// Optional ev[2] = {start, stop} timing events: recorded by the dispatch itself
// (hipExtLaunchKernelGGL), so timing a launch adds no marker packet and no
// bubble to the stream.
hipError_t launch_init(const InitArgs& a, hipStream_t s, hipEvent_t* ev = nullptr);
hipError_t launch_plan(const PlanArgs& a, hipStream_t s, hipEvent_t* ev = nullptr);
// unweighted: the graph has no weight array (every edge weighs 1); the
// kernels then neither load nor store weights.
// nnz: entries of R_1 when it is read from the CSR of one graph (sizes the
// loads of the unweighted kernel), else unused.
hipError_t launch_first_argmax(const StreamArgs& a, int grid, hipStream_t s, bool unweighted = false,
                               hipEvent_t* ev = nullptr, long long nnz = 0);
hipError_t launch_compact(const StreamArgs& a, int grid, hipStream_t s, bool late = false, bool unweighted = false,
                          hipEvent_t* ev = nullptr);
// First argmax of R_1 of one graph read from its CSR (a.in.csr_rp set).
hipError_t launch_first_csr(const StreamArgs& a, int grid, hipStream_t s, bool unweighted, hipEvent_t* ev = nullptr);
int first_csr_blocks_per_cu(bool unweighted);
// First argmax of R_1 of one unweighted graph from its CSR: one-wave
// workgroups, one range each (first_unw_ranges_per_cu() ranges per CU).
// vec_ok: col is 16-byte aligned and nnz >= first_unw_min_entries().
hipError_t launch_first_unw(const StreamArgs& a, int grid, hipStream_t s, bool vec_ok, hipEvent_t* ev = nullptr);
int first_unw_ranges_per_cu();
int first_unw_min_entries();
hipError_t launch_mutual(const MutualArgs& a, int grid, hipStream_t s, hipEvent_t* ev = nullptr);
// grid must not exceed tail_blocks_per_cu() * CUs (every workgroup resident)
hipError_t launch_tail(const TailArgs& a, int grid, hipStream_t s, hipEvent_t* ev = nullptr);
int tail_blocks_per_cu();
enum class StreamKind { kFirst, kCompact, kLateCompact };
int max_blocks_per_cu_stream(StreamKind kind, bool unweighted = false);

uint64_t premix_seed(uint64_t seed);

}  // namespace lm
