/*
 * CPU ORACLE for local-max matching -- TEST INFRASTRUCTURE ONLY.
 *
 * Only tests, the smoke check and the benchmark's CPU-baseline leg call this
 * code. The product path (the HIP library) never links or calls it, and this
 * file shares no code, header or constant table with it.
 *
 * Plain, single-threaded C99, no fast-math; weights are compared with the
 * ordinary numeric '>' on float (so -0 == +0).
 *
 * What is computed (paper, Section 1, "local max" definition; Section 2,
 * "Sequential Model"):
 *   An edge is locally maximal if its key beats the key of every incident
 *   remaining edge. Each iteration adds every locally maximal edge to M and
 *   removes all edges incident to newly matched vertices, until no edge is
 *   left. One iteration is three passes over the remaining edges:
 *     pass 1: every endpoint x keeps its candidate C[x], the best incident
 *             edge seen so far (C starts as a dummy edge below every key);
 *     pass 2: an edge e with C[u] = C[v] = e joins M;
 *     pass 3: an edge with a matched endpoint is removed; for every other
 *             edge the candidates of both endpoints go back to the dummy.
 *   C is initialised once, before the first iteration.
 *
 * Tie breaking (the paper perturbs equal weights randomly; the reading fixed
 * here): key(e) = (w(e), H(e)) compared lexicographically, w numerically and
 * H as an unsigned 64-bit integer, with H fixed for the whole run:
 *     S       = mix(seed XOR GAMMA)
 *     H(e)    = mix(((uint64)lo << 32 | hi) XOR S),   lo < hi the endpoints
 * where mix is the SplitMix64 output function (Steele, Lea & Flood, OOPSLA
 * 2014). mix and XOR with a constant are bijections, so distinct edges get
 * distinct H and the order on edges is strict.
 *
 * Renewed keys (lmo_local_max_ex with renew = 1; the paper's Lemma 1 draws
 * fresh random noise in every iteration, its footnote and Section 2.1 step 1):
 * iteration t compares (w(e), H_t(e)) with
 *     S_t     = mix(S + t * GAMMA)        (the t-th output of a SplitMix64
 *                                           stream started at S)
 *     H_t(e)  = mix(((uint64)lo << 32 | hi) XOR S_t)
 * so the order of tied edges is drawn anew each iteration. With distinct
 * weights the hash never decides and both modes give the same matching.
 *
 * Parity pins (checked by tests, not by this file): SplitMix64 published
 * output vectors pin mix; a sorted greedy scan under the same key, validity,
 * maximality, brute-force maximum weight matching (1/2 bound), closed forms
 * for paths/stars/triangles and the Lemma 1 removal fraction pin the loop.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define LMO_GAMMA 0x9E3779B97F4A7C15ULL
#define LMO_NONE (-1)

/* SplitMix64 output function. */
uint64_t lmo_mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

/* Per-run seed mix: the seed xored with the SplitMix64 increment, then mixed. */
uint64_t lmo_seed_mix(uint64_t seed) { return lmo_mix64(seed ^ LMO_GAMMA); }

/* Tie-break value of the undirected edge {lo, hi}, lo < hi, local ids. */
uint64_t lmo_edge_hash(uint64_t seed, int32_t lo, int32_t hi) {
  uint64_t pair = ((uint64_t)(uint32_t)lo << 32) | (uint64_t)(uint32_t)hi;
  return lmo_mix64(pair ^ lmo_seed_mix(seed));
}

typedef struct {
  int32_t lo, hi;
  float w;
  uint64_t h;
} lmo_edge;

/* key(a) > key(b): weight first, numerically; hash on equal weight. */
static int key_greater(const lmo_edge* a, const lmo_edge* b) {
  if (a->w > b->w) return 1;
  if (a->w < b->w) return 0;
  return a->h > b->h;
}

/* Error codes of the oracle entry points. */
#define LMO_EINVAL (-1)
#define LMO_ENOMEM (-2)

/* Builds the undirected edge list {lo < hi} from symmetric CSR. Entries with
 * v < u define the edges; a self-loop or an id out of range is an error. */
static int64_t edges_from_csr(int64_t n, const int64_t* row_ptr, const int32_t* col, const float* w, uint64_t seed,
                              lmo_edge** out) {
  if (n < 0 || !row_ptr) return LMO_EINVAL;
  int64_t nnz = row_ptr[n];
  int64_t m = 0;
  for (int64_t v = 0; v < n; ++v) {
    if (row_ptr[v + 1] < row_ptr[v]) return LMO_EINVAL;
    for (int64_t k = row_ptr[v]; k < row_ptr[v + 1]; ++k) {
      int32_t u = col[k];
      if (u < 0 || u >= n || u == v) return LMO_EINVAL;
      if (v < u) ++m;
    }
  }
  (void)nnz;
  lmo_edge* E = (lmo_edge*)malloc((size_t)(m > 0 ? m : 1) * sizeof(lmo_edge));
  if (!E) return LMO_ENOMEM;
  int64_t j = 0;
  for (int64_t v = 0; v < n; ++v)
    for (int64_t k = row_ptr[v]; k < row_ptr[v + 1]; ++k) {
      int32_t u = col[k];
      if (v < u) {
        E[j].lo = (int32_t)v;
        E[j].hi = u;
        E[j].w = w[k];
        E[j].h = lmo_edge_hash(seed, (int32_t)v, u);
        ++j;
      }
    }
  *out = E;
  return m;
}

/* Tie-break value of {lo, hi} in iteration t under renewed keys. */
uint64_t lmo_edge_hash_phase(uint64_t seed, int64_t t, int32_t lo, int32_t hi) {
  uint64_t pair = ((uint64_t)(uint32_t)lo << 32) | (uint64_t)(uint32_t)hi;
  uint64_t st = lmo_mix64(lmo_seed_mix(seed) + (uint64_t)t * LMO_GAMMA);
  return lmo_mix64(pair ^ st);
}

/*
 * Local-max matching of one graph given as symmetric CSR.
 *   mate[n]: output, partner id or -1.
 *   log (optional, log_cap rows of 3 int64): per iteration t = 1.. the number
 *   of remaining edges |E_t| at its start, the number of vertices with at least
 *   one remaining edge V_t, and the number of edges matched in it.
 * Returns the number of iterations (0 for an edgeless graph) or a negative
 * error code. Iterations beyond log_cap are still run, not logged.
 */
int64_t lmo_local_max_ex(int64_t n, const int64_t* row_ptr, const int32_t* col, const float* w, uint64_t seed,
                         int renew, int32_t* mate, int64_t* log, int64_t log_cap) {
  lmo_edge* E = NULL;
  int64_t m = edges_from_csr(n, row_ptr, col, w, seed, &E);
  if (m < 0) return m;
  int64_t* C = (int64_t*)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
  int64_t* seen = (int64_t*)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
  if (!C || !seen) {
    free(E);
    free(C);
    free(seen);
    return LMO_ENOMEM;
  }
  for (int64_t x = 0; x < n; ++x) {
    mate[x] = -1;
    C[x] = LMO_NONE; /* the dummy edge, below every key; set once */
    seen[x] = 0;
  }
  int64_t t = 0;
  while (m > 0) {
    ++t;
    if (renew) /* the keys of this iteration */
      for (int64_t j = 0; j < m; ++j) E[j].h = lmo_edge_hash_phase(seed, t, E[j].lo, E[j].hi);
    int64_t vt = 0;
    for (int64_t j = 0; j < m; ++j) {
      if (seen[E[j].lo] != t) {
        seen[E[j].lo] = t;
        ++vt;
      }
      if (seen[E[j].hi] != t) {
        seen[E[j].hi] = t;
        ++vt;
      }
    }
    /* pass 1: candidates */
    for (int64_t j = 0; j < m; ++j) {
      const lmo_edge* e = &E[j];
      if (C[e->lo] == LMO_NONE || key_greater(e, &E[C[e->lo]])) C[e->lo] = j;
      if (C[e->hi] == LMO_NONE || key_greater(e, &E[C[e->hi]])) C[e->hi] = j;
    }
    /* pass 2: mutual candidates join the matching */
    int64_t matched = 0;
    for (int64_t j = 0; j < m; ++j) {
      const lmo_edge* e = &E[j];
      if (C[e->lo] == j && C[e->hi] == j) {
        mate[e->lo] = e->hi;
        mate[e->hi] = e->lo;
        ++matched;
      }
    }
    /* pass 3: remove edges at matched vertices, reset the others' candidates */
    int64_t keep = 0;
    for (int64_t j = 0; j < m; ++j) {
      lmo_edge e = E[j];
      if (mate[e.lo] != -1 || mate[e.hi] != -1) continue;
      C[e.lo] = LMO_NONE;
      C[e.hi] = LMO_NONE;
      E[keep++] = e;
    }
    if (log && t <= log_cap) {
      log[3 * (t - 1) + 0] = m;
      log[3 * (t - 1) + 1] = vt;
      log[3 * (t - 1) + 2] = matched;
    }
    m = keep;
  }
  free(E);
  free(C);
  free(seen);
  return t;
}

/* Local max with keys fixed for the whole run. */
int64_t lmo_local_max(int64_t n, const int64_t* row_ptr, const int32_t* col, const float* w, uint64_t seed,
                      int32_t* mate, int64_t* log, int64_t log_cap) {
  return lmo_local_max_ex(n, row_ptr, col, w, seed, 0, mate, log, log_cap);
}

/*
 * Batch form: graphs g = 0..G-1 are solved one after another, each alone with
 * its own seed (seeds[g], or seed0 for all when seeds is NULL). Inputs as in
 * the batched library call: vtx_off[G+1], row_ptr[N+1] with global offsets,
 * col holding local ids. mate receives local ids. phases[g] (optional) gets
 * each graph's iteration count. Returns the largest count or an error.
 */
int64_t lmo_local_max_batch_ex(int64_t G, const int64_t* vtx_off, const int64_t* row_ptr, const int32_t* col,
                               const float* w, const uint64_t* seeds, uint64_t seed0, int renew, int32_t* mate,
                               int64_t* phases) {
  int64_t worst = 0;
  for (int64_t g = 0; g < G; ++g) {
    int64_t a = vtx_off[g], b = vtx_off[g + 1];
    int64_t n = b - a;
    int64_t e0 = row_ptr[a];
    int64_t* rp = (int64_t*)malloc((size_t)(n + 1) * sizeof(int64_t));
    if (!rp) return LMO_ENOMEM;
    for (int64_t v = 0; v <= n; ++v) rp[v] = row_ptr[a + v] - e0;
    int64_t t = lmo_local_max_ex(n, rp, col + e0, w + e0, seeds ? seeds[g] : seed0, renew, mate + a, NULL, 0);
    free(rp);
    if (t < 0) return t;
    if (phases) phases[g] = t;
    if (t > worst) worst = t;
  }
  return worst;
}

int64_t lmo_local_max_batch(int64_t G, const int64_t* vtx_off, const int64_t* row_ptr, const int32_t* col,
                            const float* w, const uint64_t* seeds, uint64_t seed0, int32_t* mate, int64_t* phases) {
  return lmo_local_max_batch_ex(G, vtx_off, row_ptr, col, w, seeds, seed0, 0, mate, phases);
}

/*
 * Greedy certificate check (test infrastructure; same key as above).
 *
 * The greedy matching -- scan edges by decreasing key, take an edge iff both
 * endpoints are free (paper, Section 3, the greedy competitor) -- is the
 * unique matching M such that every edge outside M touches an edge of M with
 * a larger key. With a strict key, local max reaches exactly this matching,
 * so the check decides bit-exact equality at any size in one pass.
 *
 * Returns the number of violations: mate not an involution or not an edge,
 * a free-free edge (maximality), or an edge outside M that beats every
 * matched edge at both its endpoints. Negative on bad input.
 */
int64_t lmo_greedy_certificate(int64_t n, const int64_t* row_ptr, const int32_t* col, const float* w, uint64_t seed,
                               const int32_t* mate) {
  if (n < 0 || !row_ptr) return LMO_EINVAL;
  float* mw = (float*)malloc((size_t)(n > 0 ? n : 1) * sizeof(float));
  int8_t* has = (int8_t*)calloc((size_t)(n > 0 ? n : 1), 1);
  if (!mw || !has) {
    free(mw);
    free(has);
    return LMO_ENOMEM;
  }
  int64_t bad = 0;
  for (int64_t v = 0; v < n; ++v) {
    int32_t p = mate[v];
    if (p == -1) continue;
    if (p < 0 || p >= n || p == v || mate[p] != v) {
      ++bad;
      continue;
    }
    for (int64_t k = row_ptr[v]; k < row_ptr[v + 1]; ++k)
      if (col[k] == p) {
        mw[v] = w[k];
        has[v] = 1;
        break;
      }
    if (!has[v]) ++bad;
  }
  for (int64_t v = 0; v < n; ++v) {
    for (int64_t k = row_ptr[v]; k < row_ptr[v + 1]; ++k) {
      int32_t u = col[k];
      if (u <= v) continue; /* each undirected edge once */
      if (mate[v] == u) continue;
      lmo_edge e = {(int32_t)v, u, w[k], lmo_edge_hash(seed, (int32_t)v, u)};
      int dominated = 0;
      int32_t ends[2] = {(int32_t)v, u};
      for (int s = 0; s < 2 && !dominated; ++s) {
        int32_t x = ends[s];
        if (!has[x]) continue;
        int32_t y = mate[x];
        lmo_edge f = {x < y ? x : y, x < y ? y : x, mw[x], 0};
        f.h = lmo_edge_hash(seed, f.lo, f.hi);
        if (key_greater(&f, &e)) dominated = 1;
      }
      if (!dominated) ++bad;
    }
  }
  free(mw);
  free(has);
  return bad;
}

/*
 * Contraction of a graph by a matching -- the coarsening step that multilevel
 * graph partitioning repeats with maximal matchings (paper, Section 1; its
 * Section 3.1 reports local max on graph-contraction instances). The paper
 * gives no layout for the coarse graph; the reading fixed here:
 *
 *   rep(v)  = v if v is free (mate[v] = -1) or v < mate[v], else mate[v]
 *   cmap[v] = the number of representatives r < rep(v): coarse ids follow
 *             the order of the representatives, a pair shares one id
 *   coarse vertex c with representative a and partner b = mate[a] (if any):
 *     cvw[c]  = vw[a] + vw[b]                          (vw NULL: 1 each)
 *     row c   = every coarse neighbour d != c once, in the order in which a
 *               fine entry (s, x) with cmap[x] = d first appears when a's
 *               row and then b's row are read in input order (entries with
 *               cmap[x] = c, the matched edge itself, are dropped)
 *     w(c, d) = the fp32 sum of the weights of the fine edges {s, x}, s in
 *               c's pair and x in d's pair, added in increasing order of
 *               (min(s, x), max(s, x)): the same order from both sides, so
 *               the coarse graph is symmetric with equal weights both ways
 *               (w NULL: every fine edge weighs 1).
 *
 * mate must be an involution (mate[mate[v]] = v, mate[v] != v) with -1 for
 * free vertices; any such pairing is accepted, not only matchings of the
 * graph. Output capacity: cmap n, crow_ptr n + 1, ccol and cw nnz, cvw n.
 * Returns the coarse nnz and sets *nc_out; LMO_EINVAL on a bad pairing.
 * Parity pins live in the tests: the coarse adjacency equals P^T A P with
 * the diagonal removed (P the fine-to-coarse membership matrix), weight
 * totals, identity when nothing is matched, closed forms on ladders and
 * cycles, hand-computed fp32 sums, and planted mistakes.
 */
typedef struct {
  int64_t slot; /* output position of the coarse neighbour */
  int32_t lo, hi;
  float w;
} lmo_contrib;

static int contrib_less(const void* pa, const void* pb) {
  const lmo_contrib* a = (const lmo_contrib*)pa;
  const lmo_contrib* b = (const lmo_contrib*)pb;
  if (a->slot != b->slot) return a->slot < b->slot ? -1 : 1;
  if (a->lo != b->lo) return a->lo < b->lo ? -1 : 1;
  if (a->hi != b->hi) return a->hi < b->hi ? -1 : 1;
  return 0;
}

int64_t lmo_contract(int64_t n, const int64_t* row_ptr, const int32_t* col, const float* w, const int32_t* mate,
                     const int64_t* vw, int32_t* cmap, int64_t* crow_ptr, int32_t* ccol, float* cw, int64_t* cvw,
                     int64_t* nc_out) {
  if (n < 0 || !row_ptr || !mate || !cmap || !crow_ptr) return LMO_EINVAL;
  for (int64_t v = 0; v < n; ++v) {
    int32_t m = mate[v];
    if (m == LMO_NONE) continue;
    if (m < 0 || m >= n || m == v || mate[m] != v) return LMO_EINVAL;
  }
  /* coarse ids in the order of the representatives */
  int64_t nc = 0;
  for (int64_t v = 0; v < n; ++v)
    if (mate[v] == LMO_NONE || v < mate[v]) cmap[v] = (int32_t)nc++;
  for (int64_t v = 0; v < n; ++v)
    if (mate[v] != LMO_NONE && v > mate[v]) cmap[v] = cmap[mate[v]];
  int64_t maxdeg2 = 0;
  for (int64_t v = 0; v < n; ++v) {
    int64_t d = row_ptr[v + 1] - row_ptr[v];
    if (mate[v] != LMO_NONE) d += row_ptr[mate[v] + 1] - row_ptr[mate[v]];
    if (d > maxdeg2) maxdeg2 = d;
  }
  int64_t* pos = (int64_t*)malloc((size_t)(nc > 0 ? nc : 1) * sizeof(int64_t));
  lmo_contrib* cb = (lmo_contrib*)malloc((size_t)(maxdeg2 > 0 ? maxdeg2 : 1) * sizeof(lmo_contrib));
  if (!pos || !cb) {
    free(pos);
    free(cb);
    return LMO_ENOMEM;
  }
  for (int64_t d = 0; d < nc; ++d) pos[d] = -1;
  int64_t out = 0;
  for (int64_t a = 0; a < n; ++a) {
    if (!(mate[a] == LMO_NONE || a < mate[a])) continue;
    const int64_t c = cmap[a];
    const int32_t b = mate[a];
    crow_ptr[c] = out;
    if (cvw) cvw[c] = (vw ? vw[a] : 1) + (b == LMO_NONE ? 0 : (vw ? vw[b] : 1));
    int64_t ncb = 0;
    const int64_t row0 = out;
    for (int side = 0; side < 2; ++side) {
      const int64_t s = side == 0 ? a : b;
      if (s == LMO_NONE) break;
      for (int64_t k = row_ptr[s]; k < row_ptr[s + 1]; ++k) {
        const int32_t x = col[k];
        const int64_t d = cmap[x];
        if (d == c) continue;
        if (pos[d] < 0) {
          pos[d] = out;
          ccol[out++] = (int32_t)d;
        }
        lmo_contrib e;
        e.slot = pos[d];
        e.lo = (int32_t)(s < x ? s : x);
        e.hi = (int32_t)(s < x ? x : s);
        e.w = w ? w[k] : 1.0f;
        cb[ncb++] = e;
      }
    }
    qsort(cb, (size_t)ncb, sizeof(lmo_contrib), contrib_less);
    for (int64_t i = 0; i < ncb; ++i) {
      if (i == 0 || cb[i].slot != cb[i - 1].slot)
        cw[cb[i].slot] = cb[i].w;
      else
        cw[cb[i].slot] += cb[i].w;
    }
    for (int64_t k = row0; k < out; ++k) pos[ccol[k]] = -1;
  }
  crow_ptr[nc] = out;
  free(pos);
  free(cb);
  *nc_out = nc;
  return out;
}

/*
 * Quality baselines of the paper's Section 3 (reporting only, not part of
 * the hot path):
 *
 * Heavy edge matching (HEM): the vertices are visited in a given order (the
 * caller passes a permutation, for the randomised variant a random one); an
 * unmatched vertex is matched to its heaviest unmatched neighbour (the first
 * one in row order among equal weights).
 *
 * Global path algorithm (GPA): the edges are scanned by decreasing weight
 * (ties by increasing (lo, hi)); an edge joins a subgraph G2 when both ends
 * have degree below two in G2 and it closes no odd cycle; then a maximum
 * weight matching of every path and even cycle of G2 is found by dynamic
 * programming along it.
 */
int64_t lmo_hem(int64_t n, const int64_t* row_ptr, const int32_t* col, const float* w, const int32_t* order,
                int32_t* mate) {
  if (n < 0 || !row_ptr || !order || !mate) return LMO_EINVAL;
  for (int64_t v = 0; v < n; ++v) mate[v] = LMO_NONE;
  int64_t m = 0;
  for (int64_t i = 0; i < n; ++i) {
    const int32_t v = order[i];
    if (v < 0 || v >= n) return LMO_EINVAL;
    if (mate[v] != LMO_NONE) continue;
    int32_t best = LMO_NONE;
    float bw = 0.0f;
    for (int64_t k = row_ptr[v]; k < row_ptr[v + 1]; ++k) {
      const int32_t u = col[k];
      if (u == v || mate[u] != LMO_NONE) continue;
      const float x = w ? w[k] : 1.0f;
      if (best == LMO_NONE || x > bw) {
        best = u;
        bw = x;
      }
    }
    if (best != LMO_NONE) {
      mate[v] = best;
      mate[best] = v;
      ++m;
    }
  }
  return m;
}

typedef struct {
  int32_t lo, hi;
  float w;
} lmo_wedge;

static int wedge_heavier(const void* pa, const void* pb) {
  const lmo_wedge* a = (const lmo_wedge*)pa;
  const lmo_wedge* b = (const lmo_wedge*)pb;
  if (a->w != b->w) return a->w > b->w ? -1 : 1;
  if (a->lo != b->lo) return a->lo < b->lo ? -1 : 1;
  if (a->hi != b->hi) return a->hi < b->hi ? -1 : 1;
  return 0;
}

static int32_t uf_find(int32_t* parent, int32_t x) {
  while (parent[x] != x) {
    parent[x] = parent[parent[x]];
    x = parent[x];
  }
  return x;
}

/* Maximum weight matching of the path x[0..len] with edge weights ew[0..len-1]
 * (edge i joins x[i] and x[i+1]), written into mate. */
static void path_dp(const int32_t* x, const float* ew, int64_t len, double* best, int8_t* take, int32_t* mate) {
  if (len <= 0) return;
  best[0] = 0.0;
  for (int64_t i = 1; i <= len; ++i) {
    const double skip = best[i - 1];
    const double with = (i >= 2 ? best[i - 2] : 0.0) + (double)ew[i - 1];
    take[i] = with > skip;
    best[i] = take[i] ? with : skip;
  }
  for (int64_t i = len; i >= 1;) {
    if (take[i]) {
      mate[x[i - 1]] = x[i];
      mate[x[i]] = x[i - 1];
      i -= 2;
    } else {
      i -= 1;
    }
  }
}

int64_t lmo_gpa(int64_t n, const int64_t* row_ptr, const int32_t* col, const float* w, int32_t* mate) {
  if (n < 0 || !row_ptr || !mate) return LMO_EINVAL;
  const int64_t nnz = n > 0 ? row_ptr[n] : 0;
  lmo_wedge* e = (lmo_wedge*)malloc((size_t)(nnz / 2 + 1) * sizeof(lmo_wedge));
  int32_t* adj = (int32_t*)malloc((size_t)(2 * n + 2) * sizeof(int32_t));   /* two G2 neighbours */
  float* adjw = (float*)malloc((size_t)(2 * n + 2) * sizeof(float));
  int32_t* parent = (int32_t*)malloc((size_t)(n + 1) * sizeof(int32_t));
  int64_t* cedges = (int64_t*)malloc((size_t)(n + 1) * sizeof(int64_t));  /* edges per component root */
  int32_t* seq = (int32_t*)malloc((size_t)(n + 2) * sizeof(int32_t));
  float* sw = (float*)malloc((size_t)(n + 2) * sizeof(float));
  double* best = (double*)malloc((size_t)(n + 2) * sizeof(double));
  int8_t* take = (int8_t*)malloc((size_t)(n + 2));
  int8_t* seen = (int8_t*)calloc((size_t)(n + 1), 1);
  if (!e || !adj || !adjw || !parent || !cedges || !seq || !sw || !best || !take || !seen) {
    free(e); free(adj); free(adjw); free(parent); free(cedges); free(seq); free(sw); free(best); free(take);
    free(seen);
    return LMO_ENOMEM;
  }
  int64_t m = 0;
  for (int64_t v = 0; v < n; ++v)
    for (int64_t k = row_ptr[v]; k < row_ptr[v + 1]; ++k)
      if (col[k] > v) {
        e[m].lo = (int32_t)v;
        e[m].hi = col[k];
        e[m].w = w ? w[k] : 1.0f;
        ++m;
      }
  qsort(e, (size_t)m, sizeof(lmo_wedge), wedge_heavier);
  for (int64_t v = 0; v < n; ++v) {
    adj[2 * v] = adj[2 * v + 1] = LMO_NONE;
    parent[v] = (int32_t)v;
    cedges[v] = 0;
    mate[v] = LMO_NONE;
  }
  for (int64_t i = 0; i < m; ++i) {
    const int32_t a = e[i].lo, b = e[i].hi;
    if (adj[2 * a + 1] != LMO_NONE || adj[2 * b + 1] != LMO_NONE) continue; /* degree two already */
    const int32_t ra = uf_find(parent, a), rb = uf_find(parent, b);
    if (ra == rb) {
      if (cedges[ra] % 2 == 0) continue; /* closing the path would make an odd cycle */
      cedges[ra] += 1;
    } else {
      parent[rb] = ra;
      cedges[ra] += cedges[rb] + 1;
    }
    adj[2 * a + (adj[2 * a] == LMO_NONE ? 0 : 1)] = b;
    adjw[2 * a + (adj[2 * a + 1] == b ? 1 : 0)] = e[i].w;
    adj[2 * b + (adj[2 * b] == LMO_NONE ? 0 : 1)] = a;
    adjw[2 * b + (adj[2 * b + 1] == a ? 1 : 0)] = e[i].w;
  }
  /* paths first (from an end), then the cycles that remain */
  for (int pass = 0; pass < 2; ++pass) {
    for (int64_t s = 0; s < n; ++s) {
      if (seen[s]) continue;
      const int deg = (adj[2 * s] != LMO_NONE) + (adj[2 * s + 1] != LMO_NONE);
      if (pass == 0 && deg == 2) continue;
      int64_t len = 0;
      int32_t prev = LMO_NONE, cur = (int32_t)s;
      seq[0] = cur;
      seen[cur] = 1;
      for (;;) {
        int32_t nxt = LMO_NONE;
        float nw = 0.0f;
        for (int j = 0; j < 2; ++j) {
          const int32_t u = adj[2 * cur + j];
          if (u != LMO_NONE && u != prev && !seen[u]) {
            nxt = u;
            nw = adjw[2 * cur + j];
            break;
          }
        }
        if (nxt == LMO_NONE) break;
        sw[len] = nw;
        seq[++len] = nxt;
        seen[nxt] = 1;
        prev = cur;
        cur = nxt;
      }
      if (pass == 0 || len == 0) {
        path_dp(seq, sw, len, best, take, mate);
        continue;
      }
      /* an even cycle seq[0..len] plus the closing edge (seq[len], seq[0]) */
      float wc = 0.0f;
      for (int j = 0; j < 2; ++j)
        if (adj[2 * seq[len] + j] == seq[0]) wc = adjw[2 * seq[len] + j];
      /* without the closing edge: the path as it is */
      path_dp(seq, sw, len, best, take, mate);
      const double without = best[len];
      /* with it: the path seq[1..len-1] plus the closing edge */
      double with_c = (double)wc;
      if (len >= 3) {
        path_dp(seq + 1, sw + 1, len - 2, best, take, mate); /* overwritten below if worse */
        with_c += best[len - 2];
      }
      if (with_c > without) {
        for (int64_t i = 0; i <= len; ++i) mate[seq[i]] = LMO_NONE;
        if (len >= 3) path_dp(seq + 1, sw + 1, len - 2, best, take, mate);
        mate[seq[0]] = seq[len];
        mate[seq[len]] = seq[0];
      } else {
        for (int64_t i = 0; i <= len; ++i) mate[seq[i]] = LMO_NONE;
        path_dp(seq, sw, len, best, take, mate);
      }
    }
  }
  int64_t matched = 0;
  for (int64_t v = 0; v < n; ++v) matched += mate[v] != LMO_NONE;
  free(e); free(adj); free(adjw); free(parent); free(cedges); free(seq); free(sw); free(best); free(take);
  free(seen);
  return matched / 2;
}
