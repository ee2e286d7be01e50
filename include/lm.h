/*
 * lm.h -- local-max matching on AMD Instinct MI355X (gfx950).
 *
 * The operation (Birn, Osipov, Sanders, Schulz, Sitchinava, "Efficient
 * Parallel and External Matching", Section 1, the "local max" algorithm):
 * an edge is locally maximal when its key beats the key of every incident
 * remaining edge. Starting from M = {}, every phase adds all locally maximal
 * edges to M and removes every edge incident to a newly matched vertex, until
 * no edge remains. The result is a maximal matching and a 1/2-approximation
 * of the maximum weight matching (Section 1, Preis' family); the number of
 * phases is logarithmic in expectation and the work is linear (Lemma 1 and
 * the argument after it, Section 2).
 *
 * Key and tie-break (the paper breaks ties by a random perturbation; this
 * library fixes it so that results are reproducible): the key of the edge
 * {lo, hi}, lo < hi in the graph's own (local) vertex ids, is the pair
 *     ( w  compared as a number (-0 equals +0),
 *       H  = mix( ((uint64)lo << 32 | hi) XOR mix(seed XOR 0x9E3779B97F4A7C15) )
 *            compared as an unsigned 64-bit integer ),
 * compared lexicographically; mix is the SplitMix64 output function
 * (z ^= z>>30; z *= 0xBF58476D1CE4E5B9; z ^= z>>27; z *= 0x94D049BB133111EB;
 * z ^= z>>31). Distinct edges have distinct H, so the order is strict and
 * the matching is unique: it equals the greedy matching under this key
 * (Section 3 defines greedy as the scan by decreasing weight). mate[] is a
 * pure function of (the set of CSR entries, seed): independent of entry
 * order, tuning, batching or serving mix.
 *
 * Graph input: a simple undirected graph as symmetric CSR. n vertices;
 * row_ptr int64[n+1] with row_ptr[0] = 0, nondecreasing, row_ptr[n] = nnz;
 * col int32[nnz] neighbour ids in [0, n); w float32[nnz] finite weights; the
 * entries (v,u) and (u,v) both exist and carry the same weight; no self-loops
 * and no duplicate entries. Limits: n < 2^31, nnz < 2^31 - 2^16.
 *
 * Output: mate int32[n], mate[v] = partner of v or -1.
 *
 * Memory and ownership: the caller owns every input and output buffer. The
 * library never writes inputs and keeps no pointer after the call returns.
 * Scratch memory comes from the context's device pool, bounded by the HBM
 * budget given to lm_create. Pointers are host memory unless the flags say
 * device memory (then they must be device memory of the context's GPU,
 * e.g. torch tensors' data_ptr()).
 *
 * Errors: every entry point returns LM_OK (0), LM_PENDING (1, poll only) or
 * a negative lm_status; lm_strerror gives a message. After an error mate[]
 * is unspecified. LM_EDEVICE means a HIP call failed; destroy the context.
 *
 * Threading: an lm_ctx is used by one thread at a time. lm_server_submit,
 * lm_server_poll and lm_server_wait are thread-safe.
 */
#ifndef LM_H_
#define LM_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t lm_status;

#define LM_OK 0
#define LM_PENDING 1
#define LM_EINVAL (-1)     /* null pointer, bad size, offsets or flags */
#define LM_EGRAPH (-2)     /* structural violation found by a check */
#define LM_EWEIGHT (-3)    /* NaN or infinite weight found by a check */
#define LM_ENOMEM (-4)     /* device allocation failed */
#define LM_ETOOBIG (-5)    /* the problem can never fit the HBM budget or limits */
#define LM_EAGAIN (-6)     /* server queue full, retry later */
#define LM_ENOTFOUND (-7)  /* unknown or already retired ticket */
#define LM_EDEVICE (-8)    /* HIP runtime failure or no usable device */

/* flags */
#define LM_IN_DEVICE 0x1u    /* row_ptr, col, w are device pointers */
#define LM_OUT_DEVICE 0x2u   /* mate is a device pointer */
#define LM_CHECK_GRAPH 0x4u  /* validate the input contract (Section 1: a simple undirected
                                graph) before solving: offsets, ids, self-loops, finite weights,
                                symmetry with equal weights both ways, no duplicate entries.
                                Host inputs are checked exactly on the host. Device inputs:
                                symmetry by comparing a 64-bit fingerprint of all entries with
                                one of their mirrors (a violation escapes with probability
                                about 2^-64), duplicates exactly by grouping every row's
                                entries by neighbour on the device (device memory of the
                                context, one extra synchronisation) */
#define LM_PROFILE 0x8u      /* time every kernel launch with HIP events */
#define LM_GRAPH 0x10u       /* run the whole solve as one captured HIP graph launch: set-up,
                                a fixed number of phases that do nothing once the tail kernel
                                has taken over, and the tail kernel (no host round trip);
                                ignored together with LM_PROFILE or LM_ASYNC; same results */
#define LM_WEIGHT_SUM 0x20u  /* after the solve, set stats->matched_weight (needs stats) */
#define LM_ASYNC 0x40u       /* stream-ordered: enqueue the whole solve on `stream` and return
                                at once; mate holds the result when the stream reaches that
                                point. Needs LM_IN_DEVICE | LM_OUT_DEVICE and stats == NULL
                                (batch: graph_phases == NULL); LM_CHECK_GRAPH, LM_PROFILE and
                                LM_WEIGHT_SUM are refused (LM_EINVAL). A later call on the same
                                context first waits for the pending solve to finish. */

#define LM_RENEW_KEYS 0x80u /* renewed tie-break keys: phase t compares (w, H_t) with
                                H_t(lo, hi) = mix(((lo << 32) | hi) XOR mix(S + t * gamma)),
                                S = mix(seed XOR gamma), gamma = 0x9E3779B97F4A7C15, so ties
                                are ordered anew in every phase (the fresh noise of Lemma 1's
                                footnote and of step 1 of the CREW algorithm, Section 2.1;
                                Section 4 asks whether renewing matters). The result is a
                                maximal local-max matching that no longer equals the fixed-key
                                greedy matching when weights tie; with distinct weights it is
                                the same matching. Not with lm_server_*. */

typedef struct lm_ctx lm_ctx;
typedef struct lm_server lm_server;

typedef struct {
  int64_t n;              /* vertices */
  int64_t nnz;            /* directed entries = 2 * undirected edges = row_ptr[n] */
  const int64_t* row_ptr; /* n+1 */
  const int32_t* col;     /* nnz */
  const float* w;         /* nnz, or NULL for an unweighted graph: every edge weighs 1
                             (the unweighted setting of Section 1), so the order of
                             the edges is the tie-break hash alone. The kernels then
                             neither read nor write weights. */
} lm_csr;

/* One record per phase t = 1, 2, ... */
typedef struct {
  int64_t live_entries;    /* directed entries alive at the start of phase t */
  int64_t live_rows;       /* vertices with at least one live entry */
  int64_t matched_edges;   /* edges added to M in phase t */
  int64_t matched_entries; /* live entries of the rows matched in phase t */
} lm_phase_rec;

/* kernel kinds reported under LM_PROFILE */
#define LM_K_INIT 0     /* live-set construction from the input CSR */
#define LM_K_ARGMAX 1   /* first-phase per-vertex argmax */
#define LM_K_MUTUAL 2   /* mutual-candidate check and matched marking */
#define LM_K_COMPACT 3  /* edge compaction fused with the next argmax */
#define LM_K_PLAN 4     /* single-workgroup stitching of cut rows and run-table scan */
#define LM_K_TAIL 5     /* persistent launch running every phase from a small live set on */
#define LM_K_KINDS 6

typedef struct {
  int32_t phases;         /* phases with at least one live edge */
  int32_t log_len;        /* records written to log (<= log_cap) */
  int64_t matched_edges;  /* |M| */
  double device_ms;       /* stream time of the solve (events around it) */
  double bytes_alg;       /* algorithmic HBM bytes of all kernels, from the log */
  lm_phase_rec* log;      /* caller buffer for per-phase records, or NULL */
  int32_t log_cap;        /* its capacity in records */
  uint32_t profile_kinds; /* input: with LM_PROFILE, bit (1 << LM_K_*) selects the kinds
                             to time (each timed launch adds two events); 0 = all */
  int32_t k_launches[LM_K_KINDS]; /* LM_PROFILE: launches per kernel kind */
  double k_ms[LM_K_KINDS];        /* LM_PROFILE: summed event time per kind */
  double k_bytes[LM_K_KINDS];     /* algorithmic bytes per kind */
  double matched_weight;  /* LM_WEIGHT_SUM: w(M), the sum of w(e) over the matched edges
                             (|M| for an unweighted graph; over all graphs of a batch);
                             0 otherwise. Found by two small kernels after the solve (not
                             part of device_ms): every matched vertex looks up the weight
                             of its matched entry in its input row, the sum over both
                             endpoints is halved. The additions run in double in a fixed
                             order for a given n, so repeated calls agree exactly; the
                             value is within 2|M| * 2^-53 * w(M) of the exact sum. */
} lm_stats;

/* Creates a context on HIP device `device`. hbm_budget_bytes caps the
 * library's own device memory (0 = 64 GiB). Returns LM_EDEVICE when no GPU
 * is usable. */
lm_status lm_create(int device, size_t hbm_budget_bytes, lm_ctx** out);
void lm_destroy(lm_ctx* ctx);

/* Solves one graph. seed selects the tie-break hash. stream is a
 * hipStream_t (NULL = the legacy default stream); the call returns after the
 * result is in mate (with LM_ASYNC: after enqueueing the solve on stream).
 * stats may be NULL. */
lm_status lm_match(lm_ctx* ctx, const lm_csr* g, uint64_t seed, int32_t* mate, uint32_t flags, void* stream,
                   lm_stats* stats);

/* Solves G graphs in one batched run over their disjoint union. Graph k owns
 * vertices [vtx_off[k], vtx_off[k+1]) of the union; row_ptr (N+1, N =
 * vtx_off[G]) holds global entry offsets; col holds LOCAL ids (0-based per
 * graph); mate receives local ids. Graph k uses seeds[k], or seed0 when seeds
 * is NULL, so each graph's result equals lm_match of that graph alone.
 * vtx_off and seeds are always host arrays. graph_phases (optional, host,
 * G entries) receives each graph's phase count. */
lm_status lm_match_batch(lm_ctx* ctx, int32_t graphs, const int64_t* vtx_off, int64_t nnz, const int64_t* row_ptr,
                         const int32_t* col, const float* w, const uint64_t* seeds, uint64_t seed0, int32_t* mate,
                         uint32_t flags, void* stream, lm_stats* stats, int32_t* graph_phases);

/* Allocation-free variant of lm_match, for callers that cannot allocate
 * device memory during the call (code under HIP graph capture, tight serving
 * loops, harnesses that forbid allocation). Same result, statistics and
 * errors as lm_match with the same flags, with these limits:
 *  - flags must include LM_IN_DEVICE | LM_OUT_DEVICE (host buffers would need
 *    staging) and may add LM_CHECK_GRAPH, which here checks everything but
 *    duplicate entries (that check needs device memory of its own); any other
 *    flag gives LM_EINVAL;
 *  - the working buffers come from one device array of
 *    LM_NOALLOC_SCRATCH_BYTES per GPU (held from the first lm_create on that
 *    GPU until the process ends), not from the context's pool; a graph needs
 *    37.2 n + 16 nnz bytes plus about 1.1 MiB of tables (each piece rounded up
 *    to 256 bytes), and a larger one gives LM_ETOOBIG before any device work
 *    (for example n = 2^19 with nnz up to 2.9 M entries fits);
 *  - the call makes no hipMalloc, hipFree, pinned or other device allocation.
 * Every call on one GPU shares that GPU's array, whose contents persist from
 * the last call (the solve clears what it needs): calls that overlap in time
 * on one GPU, from any contexts or streams, race and must be serialised by
 * the caller. stream as in lm_match (NULL = the legacy default stream); the
 * call returns once mate holds the result. */
#define LM_NOALLOC_SCRATCH_BYTES 0x4000000u /* 64 MiB */
lm_status lm_match_noalloc(lm_ctx* ctx, const lm_csr* g, uint64_t seed, int32_t* mate, uint32_t flags, void* stream,
                           lm_stats* stats);

/* Tuning knobs of the phase kernels. Results never depend on them.
 * block_entries: the least number of live entries a compaction workgroup
 * streams (the live entries are cut into at most grid_per_cu * CUs ranges
 * of at least this size). */
typedef struct {
  int32_t block_entries;   /* 2048..4194304 */
  int32_t grid_per_cu;     /* workgroups per compute unit at most, 1..16 (default 16: each kernel's resident count) */
  int32_t phases_per_sync; /* phases kept queued past the live set the host checks for emptiness, 1..64 (32 used at most) */
  int32_t tail_entries;    /* 0..2^30: the phases from the first live set of at most this many
                              entries on run in one persistent launch (device-controlled
                              solves: LM_GRAPH, LM_ASYNC); a host-polled solve hands over one
                              phase after a live set of at most 4x this many (it keeps one phase
                              queued ahead). 0: host-polled solves never hand over (default
                              2^20) */
} lm_tuning;

lm_status lm_get_tuning(lm_ctx* ctx, lm_tuning* out);
lm_status lm_set_tuning(lm_ctx* ctx, const lm_tuning* t);

/* Runs the autotuner: times candidate tunings on the given batch and keeps
 * the fastest in the context: block_entries x grid_per_cu x phases_per_sync,
 * then tail_entries, each solve timed in the mode flags name (LM_GRAPH:
 * captured launches). If cache_path is not NULL, results are read
 * from and appended to that JSON-lines file, keyed by device name and size
 * class. The chosen tuning is returned in out (may be NULL). */
lm_status lm_autotune_batch(lm_ctx* ctx, int32_t graphs, const int64_t* vtx_off, int64_t nnz,
                            const int64_t* row_ptr, const int32_t* col, const float* w, uint32_t flags,
                            const char* cache_path, lm_tuning* out);

/* ---------------- contraction by a matching (coarsening) ----------------- */

/* Coarse graph written by lm_contract. The caller allocates every array with
 * the fine graph's worst-case sizes; n and nnz are set on return. */
typedef struct {
  int64_t n;        /* out: coarse vertices (n_fine - matched pairs) */
  int64_t nnz;      /* out: coarse entries (at most nnz_fine - 2 * matched pairs) */
  int64_t* row_ptr; /* capacity n_fine + 1; receives n + 1 offsets */
  int32_t* col;     /* capacity nnz_fine */
  float* w;         /* capacity nnz_fine; coarse edge weights (also for an unweighted fine graph) */
  int64_t* vwgt;    /* capacity n_fine; coarse vertex weights, or NULL if not wanted */
} lm_coarse;

typedef struct {
  double device_ms;     /* stream time from the first kernel to the last */
  double bytes_alg;     /* algorithmic HBM bytes: 8(n+1) + 8n + (eb + 4) nnz + 8(nc+1) + 8 nnz_c
                           (+ 8n in, 8nc out with vertex weights), eb = 8 weighted, 4 unweighted */
  int64_t long_rows;    /* coarse rows with deg(a) + deg(b) > 512: their entries are sorted into
                           buckets of about 512 by a hash of the coarse neighbour and each
                           bucket is merged in LDS */
  int64_t long_entries; /* the fine entries of those rows */
  int64_t table_rows;   /* long rows merged through per-row hash tables in device memory
                           instead (all of them, when a bucket outgrew LDS; normally 0) */
} lm_contract_stats;

/* Contracts a graph by a matching: the coarsening step of multilevel graph
 * partitioning, which contracts maximal matchings again and again (paper,
 * Section 1; Section 3.1 runs local max on graph-contraction instances).
 *
 *   rep(v)  = v if v is free (mate[v] = -1) or v < mate[v], else mate[v]
 *   cmap[v] = the number of representatives below rep(v): coarse ids in the
 *             order of the pairs' smaller vertex; a pair shares one id
 *   coarse vertex c with representative a and partner b = mate[a] (if any):
 *     vwgt[c]  = vwgt_fine[a] + vwgt_fine[b]            (vwgt NULL: 1 each)
 *     row c    = each coarse neighbour d != c once, in the order in which a
 *                fine entry (s, x), cmap[x] = d, first appears when a's row
 *                and then b's row are read in input order; the matched edge
 *                (and any edge inside the pair) is dropped
 *     w(c, d)  = the fp32 sum of the weights of the fine edges {s, x} with s
 *                in c's pair and x in d's pair (at most four), added in
 *                increasing order of (min(s, x), max(s, x)): the same order
 *                from both sides, so the coarse graph is again symmetric with
 *                equal weights both ways (g->w NULL: each fine edge weighs 1)
 *
 * g: symmetric CSR as for lm_match (no self-loops, no duplicate entries).
 * mate: int32[n], an involution with -1 for free vertices (mate[mate[v]] = v,
 * mate[v] != v); any pairing is accepted, not only matchings of g. vwgt:
 * int64[n] or NULL. cmap: int32[n] output. Inputs are device pointers with
 * LM_IN_DEVICE, outputs (cmap and out's arrays) with LM_OUT_DEVICE; no other
 * flag is accepted. The call returns once out->n and out->nnz are set and the
 * outputs are written (stream as in lm_match). stats may be NULL.
 * Errors: LM_EINVAL for null pointers, bad flags or a mate that is not an
 * involution; LM_EGRAPH for a row_ptr that is not a valid offset array, a
 * neighbour id outside [0, n) or more than four fine edges between two pairs
 * (duplicate entries); LM_ETOOBIG beyond the size limits of lm_match or the
 * HBM budget. After an error the outputs are unspecified. */
lm_status lm_contract(lm_ctx* ctx, const lm_csr* g, const int32_t* mate, const int64_t* vwgt, int32_t* cmap,
                      lm_coarse* out, uint32_t flags, void* stream, lm_contract_stats* stats);

/* ---------------- serving: continuous batching at phase granularity ----- */

#define LM_SERVE_BATCHED 0  /* continuous batching: resident graphs share every phase launch; a
                               request that finds the server idle (nothing resident, staged or
                               queued behind it) is solved alone, as lm_match would */
#define LM_SERVE_FIFO 1     /* baseline: one request at a time through lm_match */

typedef struct {
  size_t hbm_budget_bytes;  /* admission budget for resident requests */
  int32_t max_resident;     /* graphs on the GPU at once, 1..4096 */
  int32_t queue_cap;        /* waiting requests before LM_EAGAIN */
  int32_t phases_per_step;  /* phases run over all resident graphs per step */
  int32_t mode;             /* LM_SERVE_BATCHED or LM_SERVE_FIFO */
} lm_server_opts;

typedef struct {
  int32_t phases;           /* phases the request took */
  int64_t matched_edges;
  double submit_to_admit_ms;/* time in the queue (batched: until its host-to-device copy landed
                               and it joined the resident graphs) */
  double submit_to_done_ms; /* latency until the result was on the host */
  double admit_to_solved_ms;/* on the device: admission until its last phase was seen done
                               (FIFO: the whole lm_match, copies included) */
  double solved_to_done_ms; /* copying mate back to the host (FIFO: 0) */
} lm_request_stats;

/* Creates a server with its own scheduler thread on ctx's device. The
 * server owns ctx's device while it lives: do not call lm_match on ctx. */
lm_status lm_server_create(lm_ctx* ctx, const lm_server_opts* opts, lm_server** out);
/* Deep-copies the host graph into pinned memory and queues it. Returns
 * LM_EAGAIN when the queue is full, LM_ETOOBIG when the graph can never fit
 * the admission budget. */
lm_status lm_server_submit(lm_server* s, const lm_csr* g, uint64_t seed, uint64_t* ticket);
/* LM_PENDING while running; LM_OK copies mate (host, n entries) and retires
 * the ticket; LM_ENOTFOUND for unknown or retired tickets. */
lm_status lm_server_poll(lm_server* s, uint64_t ticket, int32_t* mate, lm_request_stats* st);
/* Blocks until the ticket completes (or timeout_ms elapses: LM_PENDING),
 * then behaves as lm_server_poll. timeout_ms < 0 waits forever. */
lm_status lm_server_wait(lm_server* s, uint64_t ticket, int32_t* mate, lm_request_stats* st, int64_t timeout_ms);
/* Drains every queued and running request, then stops the thread. */
lm_status lm_server_destroy(lm_server* s);

const char* lm_strerror(lm_status st);

#ifdef __cplusplus
}
#endif

#endif /* LM_H_ */
