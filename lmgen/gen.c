/*
 * Seeded synthetic graph generators for the local-max matching workloads.
 *
 * This file holds input generation only: random streams, graph shapes and CSR
 * assembly. It contains none of the matching method's arithmetic (no keys, no
 * edge hash, no phase logic) and is shared by the CPU oracle tests and the GPU
 * path tests alike.
 *
 * Random numbers come from SplitMix64 used as a counter-based stream: output
 * i of the stream with state s is mix(s + (i+1)*gamma) (Steele, Lea & Flood,
 * "Fast splittable pseudorandom number generators", OOPSLA 2014). Every value
 * is therefore addressable by index, so generation is parallel and still
 * deterministic.
 *
 * Families (paper, Section 3 "Implementations and Experiments"):
 *   - Erdos-Renyi G(n,m): m distinct non-loop pairs, uniform with rejection;
 *     the paper's random graphs with alpha*n edges and uniform weights.
 *   - 2-D random geometric graphs: n points in the unit square, edge iff the
 *     Euclidean distance is below r; weight 1 - distance.
 *   - R-MAT (Chakrabarti, Zhan & Faloutsos, SDM 2004): recursive quadrant
 *     sampling, self-loops dropped, duplicates removed, symmetrised; unit
 *     weights model the paper's unweighted case.
 * All outputs are symmetric CSR with rows sorted by neighbour id, no
 * self-loops, no duplicates, equal weights on both directions.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define LMG_GAMMA 0x9E3779B97F4A7C15ULL

typedef struct {
  int64_t n;
  int64_t nnz;
  int64_t* row_ptr; /* n+1 */
  int32_t* col;     /* nnz */
  float* w;         /* nnz */
} lmg_csr;

typedef struct {
  int64_t graphs;
  int64_t n_total;
  int64_t nnz_total;
  int64_t* vtx_off; /* graphs+1 */
  int64_t* row_ptr; /* n_total+1, global offsets */
  int32_t* col;     /* local ids */
  float* w;
} lmg_batch;

static inline uint64_t g_mix(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}
/* i-th output of the SplitMix64 stream with state s */
static inline uint64_t g_at(uint64_t s, uint64_t i) { return g_mix(s + (i + 1) * LMG_GAMMA); }
/* independent sub-stream state for a purpose tag */
static inline uint64_t g_sub(uint64_t seed, uint64_t tag) { return g_mix(seed ^ g_mix(tag * LMG_GAMMA + 0x632BE59BD9B4E019ULL)); }
static inline double g_u01(uint64_t r) { return (double)(r >> 11) * 0x1.0p-53; }
/* k * 2^-24 with k uniform in [1, 2^24]: uniform on (0,1], exact in fp32 */
static inline float g_wuni(uint64_t r) { return (float)((r >> 40) + 1) * 0x1.0p-24f; }
/* uniform integer in [0, n) from the high 32 bits (n < 2^32) */
static inline uint32_t g_below(uint64_t r, uint32_t n) { return (uint32_t)(((r >> 32) * (uint64_t)n) >> 32); }

enum { TAG_EDGE = 1, TAG_WEIGHT = 2, TAG_X = 3, TAG_Y = 4, TAG_RMAT = 5, TAG_GRAPH = 6 };
enum { W_UNIFORM = 0, W_UNIT = 1 };

void lmg_free(lmg_csr* g) {
  if (!g) return;
  free(g->row_ptr);
  free(g->col);
  free(g->w);
  memset(g, 0, sizeof(*g));
}
void lmg_batch_free(lmg_batch* b) {
  if (!b) return;
  free(b->vtx_off);
  free(b->row_ptr);
  free(b->col);
  free(b->w);
  memset(b, 0, sizeof(*b));
}

/* ---------------- CSR assembly ---------------- */

/* Undirected edges (eu[j] < ev[j]) sorted by (eu, ev): filling rows in that
 * order yields rows sorted by neighbour id (smaller neighbours arrive first,
 * in increasing order, then larger ones). */
static int csr_from_sorted_edges(int64_t n, int64_t m, const uint64_t* keys, const float* ew, int64_t* row_ptr,
                                 int32_t* col, float* w) {
  int64_t* fill = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
  if (!fill) return -1;
  for (int64_t j = 0; j < m; ++j) {
    fill[(int64_t)(keys[j] >> 32) + 1]++;
    fill[(int64_t)(keys[j] & 0xffffffffu) + 1]++;
  }
  row_ptr[0] = 0;
  for (int64_t v = 0; v < n; ++v) row_ptr[v + 1] = row_ptr[v] + fill[v + 1];
  for (int64_t v = 0; v < n; ++v) fill[v] = row_ptr[v];
  for (int64_t j = 0; j < m; ++j) {
    int64_t a = (int64_t)(keys[j] >> 32), b = (int64_t)(keys[j] & 0xffffffffu);
    float x = ew ? ew[j] : 1.0f;
    int64_t pa = fill[a]++, pb = fill[b]++;
    col[pa] = (int32_t)b;
    w[pa] = x;
    col[pb] = (int32_t)a;
    w[pb] = x;
  }
  free(fill);
  return 0;
}

/* LSD radix sort of 64-bit keys (bits [0, bits) significant), with an optional
 * float payload. Deterministic; parallel histograms when OpenMP is on. */
static int radix_sort_u64(uint64_t* keys, float* pay, int64_t m, int bits) {
  if (m <= 1) return 0;
  uint64_t* tk = (uint64_t*)malloc((size_t)m * sizeof(uint64_t));
  float* tp = pay ? (float*)malloc((size_t)m * sizeof(float)) : NULL;
  if (!tk || (pay && !tp)) {
    free(tk);
    free(tp);
    return -1;
  }
  int nthreads = 1;
#ifdef _OPENMP
  /* inside an enclosing parallel region (one graph per thread) sort serially */
  nthreads = omp_in_parallel() ? 1 : omp_get_max_threads();
  if (nthreads > 64) nthreads = 64;
#endif
  const int DIG = 16;
  const int64_t B = 1 << DIG;
  int64_t* hist = (int64_t*)malloc((size_t)nthreads * B * sizeof(int64_t));
  if (!hist) {
    free(tk);
    free(tp);
    return -1;
  }
  uint64_t* src = keys;
  uint64_t* dst = tk;
  float* ps = pay;
  float* pd = tp;
  int passes = (bits + DIG - 1) / DIG;
  for (int p = 0; p < passes; ++p) {
    int sh = p * DIG;
    memset(hist, 0, (size_t)nthreads * B * sizeof(int64_t));
#pragma omp parallel num_threads(nthreads)
    {
      int t = 0;
#ifdef _OPENMP
      t = omp_get_thread_num();
#endif
      int64_t lo = m * t / nthreads, hi = m * (t + 1) / nthreads;
      int64_t* h = hist + (int64_t)t * B;
      for (int64_t i = lo; i < hi; ++i) h[(src[i] >> sh) & (B - 1)]++;
    }
    int64_t run = 0;
    for (int64_t d = 0; d < B; ++d)
      for (int t = 0; t < nthreads; ++t) {
        int64_t c = hist[(int64_t)t * B + d];
        hist[(int64_t)t * B + d] = run;
        run += c;
      }
#pragma omp parallel num_threads(nthreads)
    {
      int t = 0;
#ifdef _OPENMP
      t = omp_get_thread_num();
#endif
      int64_t lo = m * t / nthreads, hi = m * (t + 1) / nthreads;
      int64_t* h = hist + (int64_t)t * B;
      for (int64_t i = lo; i < hi; ++i) {
        int64_t pos = h[(src[i] >> sh) & (B - 1)]++;
        dst[pos] = src[i];
        if (ps) pd[pos] = ps[i];
      }
    }
    uint64_t* tsw = src;
    src = dst;
    dst = tsw;
    float* psw = ps;
    ps = pd;
    pd = psw;
  }
  if (src != keys) {
    memcpy(keys, src, (size_t)m * sizeof(uint64_t));
    if (pay) memcpy(pay, ps, (size_t)m * sizeof(float));
  }
  free(hist);
  free(tk);
  free(tp);
  return 0;
}

static int alloc_csr(lmg_csr* out, int64_t n, int64_t nnz) {
  out->n = n;
  out->nnz = nnz;
  out->row_ptr = (int64_t*)malloc(((size_t)n + 1) * sizeof(int64_t));
  out->col = (int32_t*)malloc((size_t)(nnz > 0 ? nnz : 1) * sizeof(int32_t));
  out->w = (float*)malloc((size_t)(nnz > 0 ? nnz : 1) * sizeof(float));
  if (!out->row_ptr || !out->col || !out->w) {
    lmg_free(out);
    return -1;
  }
  return 0;
}

/* ---------------- Erdos-Renyi G(n, m) ---------------- */

/* Samples the edge keys of one G(n,m) graph into keys[0..m) (acceptance
 * order) and their weights. Returns 0, or -1 if m exceeds n(n-1)/2. */
static int er_sample(int64_t n, int64_t m, uint64_t seed, int wmode, uint64_t* keys, float* ew) {
  if (n < 2 && m > 0) return -1;
  if (m > n * (n - 1) / 2) return -1;
  if (m == 0) return 0;
  int64_t cap = 1;
  while (cap < 2 * m) cap <<= 1;
  uint64_t* table = (uint64_t*)malloc((size_t)cap * sizeof(uint64_t));
  if (!table) return -1;
  memset(table, 0xff, (size_t)cap * sizeof(uint64_t));
  uint64_t se = g_sub(seed, TAG_EDGE), sw = g_sub(seed, TAG_WEIGHT);
  int64_t got = 0;
  uint64_t k = 0;
  while (got < m) {
    uint32_t a = g_below(g_at(se, 2 * k), (uint32_t)n);
    uint32_t b = g_below(g_at(se, 2 * k + 1), (uint32_t)n);
    ++k;
    if (a == b) continue;
    uint64_t lo = a < b ? a : b, hi = a < b ? b : a;
    uint64_t key = (lo << 32) | hi;
    uint64_t h = g_mix(key) & (uint64_t)(cap - 1);
    int dup = 0;
    while (table[h] != ~0ULL) {
      if (table[h] == key) {
        dup = 1;
        break;
      }
      h = (h + 1) & (uint64_t)(cap - 1);
    }
    if (dup) continue;
    table[h] = key;
    keys[got] = key;
    ew[got] = wmode == W_UNIT ? 1.0f : g_wuni(g_at(sw, (uint64_t)got));
    ++got;
  }
  free(table);
  return 0;
}

int lmg_er(int64_t n, int64_t m, uint64_t seed, int wmode, lmg_csr* out) {
  memset(out, 0, sizeof(*out));
  if (n < 0 || m < 0 || n >= (1LL << 31)) return -1;
  uint64_t* keys = (uint64_t*)malloc((size_t)(m > 0 ? m : 1) * sizeof(uint64_t));
  float* ew = (float*)malloc((size_t)(m > 0 ? m : 1) * sizeof(float));
  if (!keys || !ew || er_sample(n, m, seed, wmode, keys, ew) != 0) {
    free(keys);
    free(ew);
    return -1;
  }
  int rc = radix_sort_u64(keys, ew, m, 64);
  if (rc == 0) rc = alloc_csr(out, n, 2 * m);
  if (rc == 0) rc = csr_from_sorted_edges(n, m, keys, ew, out->row_ptr, out->col, out->w);
  free(keys);
  free(ew);
  if (rc) lmg_free(out);
  return rc;
}

/* ---------------- 2-D random geometric graph ---------------- */

/* n points uniform in [0,1)^2 (fp64); edge iff d^2 < r^2; w = fp32(1 - d).
 * Vertex ids are assigned in grid-cell order (row-major cells of side >= r,
 * original index order inside a cell), which gives the locality of the
 * paper's rgg instances. */
int lmg_rgg(int64_t n, double r, uint64_t seed, lmg_csr* out) {
  memset(out, 0, sizeof(*out));
  if (n < 0 || n >= (1LL << 31) || !(r > 0.0)) return -1;
  int64_t G = (int64_t)floor(1.0 / r);
  if (G < 1) G = 1;
  if (G > 65536) G = 65536;
  const double cs = 1.0 / (double)G;
  uint64_t sx = g_sub(seed, TAG_X), sy = g_sub(seed, TAG_Y);
  double* px = (double*)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
  double* py = (double*)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
  double* qx = (double*)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
  double* qy = (double*)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
  int64_t* cell_start = (int64_t*)calloc((size_t)(G * G + 1), sizeof(int64_t));
  int64_t* deg = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
  if (!px || !py || !qx || !qy || !cell_start || !deg) goto fail;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    px[i] = g_u01(g_at(sx, (uint64_t)i));
    py[i] = g_u01(g_at(sy, (uint64_t)i));
  }
  /* counting sort of points by cell; stable in original index */
  for (int64_t i = 0; i < n; ++i) {
    int64_t cx = (int64_t)(px[i] * (double)G), cy = (int64_t)(py[i] * (double)G);
    if (cx >= G) cx = G - 1;
    if (cy >= G) cy = G - 1;
    cell_start[cy * G + cx + 1]++;
  }
  for (int64_t c = 0; c < G * G; ++c) cell_start[c + 1] += cell_start[c];
  {
    int64_t* pos = (int64_t*)malloc((size_t)(G * G) * sizeof(int64_t));
    if (!pos) goto fail;
    memcpy(pos, cell_start, (size_t)(G * G) * sizeof(int64_t));
    for (int64_t i = 0; i < n; ++i) {
      int64_t cx = (int64_t)(px[i] * (double)G), cy = (int64_t)(py[i] * (double)G);
      if (cx >= G) cx = G - 1;
      if (cy >= G) cy = G - 1;
      int64_t p = pos[cy * G + cx]++;
      qx[p] = px[i];
      qy[p] = py[i];
    }
    free(pos);
  }
  free(px);
  free(py);
  px = py = NULL;
  const double r2 = r * r;
  /* pass 1: degrees */
#pragma omp parallel for schedule(dynamic, 4096)
  for (int64_t i = 0; i < n; ++i) {
    int64_t cx = (int64_t)(qx[i] * (double)G), cy = (int64_t)(qy[i] * (double)G);
    if (cx >= G) cx = G - 1;
    if (cy >= G) cy = G - 1;
    int64_t d = 0;
    for (int64_t yy = cy - 1; yy <= cy + 1; ++yy) {
      if (yy < 0 || yy >= G) continue;
      for (int64_t xx = cx - 1; xx <= cx + 1; ++xx) {
        if (xx < 0 || xx >= G) continue;
        int64_t c = yy * G + xx;
        for (int64_t j = cell_start[c]; j < cell_start[c + 1]; ++j) {
          if (j == i) continue;
          double dx = qx[i] - qx[j], dy = qy[i] - qy[j];
          if (dx * dx + dy * dy < r2) ++d;
        }
      }
    }
    deg[i + 1] = d;
  }
  (void)cs;
  for (int64_t i = 0; i < n; ++i) deg[i + 1] += deg[i];
  if (alloc_csr(out, n, deg[n]) != 0) goto fail;
  memcpy(out->row_ptr, deg, ((size_t)n + 1) * sizeof(int64_t));
  /* pass 2: fill; cells are visited in increasing cell index and ids are
   * cell-major, so every row comes out sorted by neighbour id */
#pragma omp parallel for schedule(dynamic, 4096)
  for (int64_t i = 0; i < n; ++i) {
    int64_t cx = (int64_t)(qx[i] * (double)G), cy = (int64_t)(qy[i] * (double)G);
    if (cx >= G) cx = G - 1;
    if (cy >= G) cy = G - 1;
    int64_t p = out->row_ptr[i];
    for (int64_t yy = cy - 1; yy <= cy + 1; ++yy) {
      if (yy < 0 || yy >= G) continue;
      for (int64_t xx = cx - 1; xx <= cx + 1; ++xx) {
        if (xx < 0 || xx >= G) continue;
        int64_t c = yy * G + xx;
        for (int64_t j = cell_start[c]; j < cell_start[c + 1]; ++j) {
          if (j == i) continue;
          double dx = qx[i] - qx[j], dy = qy[i] - qy[j];
          double d2 = dx * dx + dy * dy;
          if (d2 < r2) {
            out->col[p] = (int32_t)j;
            out->w[p] = (float)(1.0 - sqrt(d2));
            ++p;
          }
        }
      }
    }
  }
  free(qx);
  free(qy);
  free(cell_start);
  free(deg);
  return 0;
fail:
  free(px);
  free(py);
  free(qx);
  free(qy);
  free(cell_start);
  free(deg);
  lmg_free(out);
  return -1;
}

/* ---------------- R-MAT ---------------- */

/* ef * 2^scale samples; each level picks a quadrant with probabilities
 * (a, b, c, 1-a-b-c) from a 16-bit uniform. Self-loops dropped, pairs
 * canonicalised to (min, max), sorted and deduplicated, then symmetrised. No
 * vertex permutation: hubs sit at low ids. wmode: unit or uniform (0,1]. */
int lmg_rmat(int scale, int64_t edge_factor, double a, double b, double c, uint64_t seed, int wmode, lmg_csr* out) {
  memset(out, 0, sizeof(*out));
  if (scale < 1 || scale > 30 || edge_factor < 0) return -1;
  int64_t n = 1LL << scale;
  int64_t S = edge_factor * n;
  uint64_t* keys = (uint64_t*)malloc((size_t)(S > 0 ? S : 1) * sizeof(uint64_t));
  if (!keys) return -1;
  const uint32_t ta = (uint32_t)floor(a * 65536.0 + 0.5);
  const uint32_t tb = (uint32_t)floor((a + b) * 65536.0 + 0.5);
  const uint32_t tc = (uint32_t)floor((a + b + c) * 65536.0 + 0.5);
  const uint64_t sr = g_sub(seed, TAG_RMAT);
  const int per = (scale + 3) / 4; /* 64-bit draws per sample */
#pragma omp parallel for schedule(static)
  for (int64_t k = 0; k < S; ++k) {
    uint64_t u = 0, v = 0;
    int lev = 0;
    for (int d = 0; d < per && lev < scale; ++d) {
      uint64_t r = g_at(sr, (uint64_t)k * (uint64_t)per + (uint64_t)d);
      for (int q = 0; q < 4 && lev < scale; ++q, ++lev) {
        uint32_t p = (uint32_t)((r >> (16 * q)) & 0xffffu);
        uint64_t bu = 0, bv = 0;
        if (p < ta) {
        } else if (p < tb) {
          bv = 1;
        } else if (p < tc) {
          bu = 1;
        } else {
          bu = 1;
          bv = 1;
        }
        u = (u << 1) | bu;
        v = (v << 1) | bv;
      }
    }
    if (u == v)
      keys[k] = ~0ULL;
    else
      keys[k] = u < v ? ((u << 32) | v) : ((v << 32) | u);
  }
  /* self-loop markers (all ones) sort last */
  if (radix_sort_u64(keys, NULL, S, 64) != 0) {
    free(keys);
    return -1;
  }
  int64_t m = 0;
  for (int64_t k = 0; k < S; ++k) {
    if (keys[k] == ~0ULL) break;
    if (m > 0 && keys[m - 1] == keys[k]) continue;
    keys[m++] = keys[k];
  }
  float* ew = NULL;
  if (wmode != W_UNIT) {
    ew = (float*)malloc((size_t)(m > 0 ? m : 1) * sizeof(float));
    if (!ew) {
      free(keys);
      return -1;
    }
    uint64_t sw = g_sub(seed, TAG_WEIGHT);
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < m; ++j) ew[j] = g_wuni(g_at(sw, (uint64_t)j));
  }
  int rc = alloc_csr(out, n, 2 * m);
  if (rc == 0) rc = csr_from_sorted_edges(n, m, keys, ew, out->row_ptr, out->col, out->w);
  free(keys);
  free(ew);
  if (rc) lmg_free(out);
  return rc;
}

/* ---------------- batch of G(n,m) graphs ---------------- */

/* Graph g draws, from its own sub-stream: n_g = round(2^(lg_lo + (lg_hi-lg_lo) U)),
 * average degree d_g uniform in [d_lo, d_hi], m_g = round(n_g d_g / 2) (capped
 * at n(n-1)/2), edges and weights as lmg_er. Output is one CSR over the
 * disjoint union with per-graph vertex offsets; col holds LOCAL ids. */
int lmg_er_batch(int64_t graphs, uint64_t seed, double lg_lo, double lg_hi, double d_lo, double d_hi, int wmode,
                 lmg_batch* out) {
  memset(out, 0, sizeof(*out));
  if (graphs < 0) return -1;
  int64_t* gn = (int64_t*)malloc((size_t)(graphs + 1) * sizeof(int64_t));
  int64_t* gm = (int64_t*)malloc((size_t)(graphs + 1) * sizeof(int64_t));
  int64_t* eoff = (int64_t*)calloc((size_t)graphs + 1, sizeof(int64_t));
  out->vtx_off = (int64_t*)calloc((size_t)graphs + 1, sizeof(int64_t));
  if (!gn || !gm || !eoff || !out->vtx_off) goto fail;
  const uint64_t sg = g_sub(seed, TAG_GRAPH);
  for (int64_t g = 0; g < graphs; ++g) {
    double U = g_u01(g_at(sg, 3 * (uint64_t)g));
    double V = g_u01(g_at(sg, 3 * (uint64_t)g + 1));
    int64_t n = (int64_t)llround(pow(2.0, lg_lo + (lg_hi - lg_lo) * U));
    if (n < 2) n = 2;
    double d = d_lo + (d_hi - d_lo) * V;
    int64_t m = (int64_t)llround((double)n * d / 2.0);
    if (m > n * (n - 1) / 2) m = n * (n - 1) / 2;
    gn[g] = n;
    gm[g] = m;
    out->vtx_off[g + 1] = out->vtx_off[g] + n;
    eoff[g + 1] = eoff[g] + 2 * m;
  }
  out->graphs = graphs;
  out->n_total = out->vtx_off[graphs];
  out->nnz_total = eoff[graphs];
  if (out->n_total >= (1LL << 31)) goto fail;
  out->row_ptr = (int64_t*)malloc(((size_t)out->n_total + 1) * sizeof(int64_t));
  out->col = (int32_t*)malloc((size_t)(out->nnz_total > 0 ? out->nnz_total : 1) * sizeof(int32_t));
  out->w = (float*)malloc((size_t)(out->nnz_total > 0 ? out->nnz_total : 1) * sizeof(float));
  if (!out->row_ptr || !out->col || !out->w) goto fail;
  out->row_ptr[out->n_total] = out->nnz_total;
  int failed = 0;
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t g = 0; g < graphs; ++g) {
    int64_t n = gn[g], m = gm[g];
    uint64_t gseed = g_at(sg, 3 * (uint64_t)g + 2);
    uint64_t* keys = (uint64_t*)malloc((size_t)(m > 0 ? m : 1) * sizeof(uint64_t));
    float* ew = (float*)malloc((size_t)(m > 0 ? m : 1) * sizeof(float));
    int64_t* rp = (int64_t*)malloc(((size_t)n + 1) * sizeof(int64_t));
    int rc = (!keys || !ew || !rp) ? -1 : er_sample(n, m, gseed, wmode, keys, ew);
    if (rc == 0) rc = radix_sort_u64(keys, ew, m, 64);
    if (rc == 0) rc = csr_from_sorted_edges(n, m, keys, ew, rp, out->col + eoff[g], out->w + eoff[g]);
    if (rc == 0)
      for (int64_t v = 0; v < n; ++v) out->row_ptr[out->vtx_off[g] + v] = eoff[g] + rp[v];
    if (rc) {
#pragma omp atomic write
      failed = 1;
    }
    free(keys);
    free(ew);
    free(rp);
  }
  if (failed) goto fail;
  free(gn);
  free(gm);
  free(eoff);
  return 0;
fail:
  free(gn);
  free(gm);
  free(eoff);
  lmg_batch_free(out);
  return -1;
}

/* ---------------- raw streams (for Python-side trace generation) -------- */

void lmg_stream_u01(uint64_t seed, uint64_t tag, int64_t first, int64_t count, double* out) {
  uint64_t s = g_sub(seed, tag);
  for (int64_t i = 0; i < count; ++i) out[i] = g_u01(g_at(s, (uint64_t)(first + i)));
}
