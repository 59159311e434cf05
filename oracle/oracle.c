/*
 * oracle.c -- sequential FP64 reference implementation of the Gauss-Seidel
 * cascadic multigrid (GS-CMG) Fiedler-vector solver of Gandhi, "Improvement of
 * the Cascadic Multigrid Algorithm with a Gauss Seidel Smoother to Efficiently
 * Compute the Fiedler Vector of a Graph Laplacian" (arXiv 1602.04386, 2015).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the checker for the HIP library: it
 * is built and called by the tests, by the smoke check and by the benchmark's
 * CPU-baseline leg, never by the library.  It shares no code, header, table or
 * helper with the HIP path.  It is deliberately plain: one thread, no blocking,
 * no fusion, every loop in the order the method states it, library primitives
 * limited to qsort, sqrt and fabs.
 *
 * Where the paper leaves a choice open, a fixed reading is taken; each
 * function below names the passage it follows and states the reading it takes.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_OK 0
#define OR_E_INVALID (-1)
#define OR_E_NOT_SYMMETRIC (-2)
#define OR_E_NOT_LAPLACIAN (-3)
#define OR_E_ISOLATED (-4)
#define OR_E_NOMEM (-5)
#define OR_E_NOT_CONVERGED (-7)

#define OR_MAX_LEVELS 64

/* ------------------------------------------------------------------------ */
/* Hashes and random numbers (published definitions, re-typed here).        */
/* ------------------------------------------------------------------------ */

/* SplitMix64 (Steele, Lea & Flood, OOPSLA 2014): draw k (k = 1, 2, ...) of the
 * stream seeded s is mix(s + k * 0x9E3779B97F4A7C15). */
static uint64_t or_splitmix64(uint64_t* state) {
  uint64_t z = (*state += 0x9E3779B97F4A7C15ULL);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

/* MurmurHash3 32-bit finaliser (Appleby, public domain). */
static uint32_t or_fmix32(uint32_t h) {
  h ^= h >> 16;
  h *= 0x85EBCA6BU;
  h ^= h >> 13;
  h *= 0xC2B2AE35U;
  h ^= h >> 16;
  return h;
}

/* Tie-break hash of the vertex pair a < b. */
uint32_t or_pair_hash(int32_t a, int32_t b) {
  return or_fmix32(or_fmix32((uint32_t)a) ^ (uint32_t)b);
}

/* Per-level colouring seed derived from the user's 64-bit colour seed. */
uint32_t or_level_seed(uint64_t colour_seed, int32_t level) {
  uint32_t lo = (uint32_t)colour_seed, hi = (uint32_t)(colour_seed >> 32);
  return or_fmix32(lo ^ or_fmix32(hi + (uint32_t)level));
}

/* Colouring priority of vertex v. */
uint32_t or_colour_priority(int32_t v, uint32_t level_seed) {
  return or_fmix32((uint32_t)v ^ level_seed);
}

/* ------------------------------------------------------------------------ */
/* Input: Definition 2.1 -- L(i,i) = weighted degree, L(i,j) = -w(i,j).      */
/* ------------------------------------------------------------------------ */

/* Binary search for column j in row i; returns the CSR position or -1. */
static int64_t or_find(const int32_t* rp, const int32_t* col, int32_t i, int32_t j) {
  int64_t lo = rp[i], hi = (int64_t)rp[i + 1] - 1;
  while (lo <= hi) {
    int64_t mid = lo + (hi - lo) / 2;
    if (col[mid] == j) return mid;
    if (col[mid] < j) lo = mid + 1; else hi = mid - 1;
  }
  return -1;
}

/*
 * Validates a CSR input and writes the off-diagonal weights W (w_ij > 0).
 * is_adjacency = 0: the input is L (Def. 2.1): off-diagonals < 0, a diagonal
 * entry per row equal to the weighted degree within 1e-12 max(1, L_ii).
 * is_adjacency = 1: the input is W: no diagonal, entries > 0.
 * Errors, by priority: structure (INVALID), signs/finiteness/diagonal
 * (NOT_LAPLACIAN), bitwise symmetry (NOT_SYMMETRIC), a vertex without edges
 * (ISOLATED).  out_* must hold nnz entries; *out_m receives the edge count.
 */
int32_t or_input_to_adjacency(int32_t n, int64_t nnz, const int32_t* rp, const int32_t* col,
                              const double* val, int32_t is_adjacency, int32_t* out_rp,
                              int32_t* out_col, double* out_w, int64_t* out_m) {
  if (n < 2 || nnz < 0 || nnz > 2147483647LL || !rp || (nnz > 0 && (!col || !val)))
    return OR_E_INVALID;
  if (rp[0] != 0 || (int64_t)rp[n] != nnz) return OR_E_INVALID;
  for (int32_t i = 0; i < n; ++i) {
    if (rp[i + 1] < rp[i]) return OR_E_INVALID;
    for (int64_t p = rp[i]; p < rp[i + 1]; ++p) {
      if (col[p] < 0 || col[p] >= n) return OR_E_INVALID;
      if (p > rp[i] && col[p] <= col[p - 1]) return OR_E_INVALID;
    }
  }
  for (int32_t i = 0; i < n; ++i) {
    int has_diag = 0;
    double diag = 0.0, deg = 0.0;
    for (int64_t p = rp[i]; p < rp[i + 1]; ++p) {
      double v = val[p];
      if (!isfinite(v)) return OR_E_NOT_LAPLACIAN;
      if (col[p] == i) {
        if (is_adjacency) return OR_E_NOT_LAPLACIAN;
        has_diag = 1;
        diag = v;
      } else {
        double wij = is_adjacency ? v : -v;
        if (!(wij > 0.0)) return OR_E_NOT_LAPLACIAN;
        deg += wij;
      }
    }
    if (!is_adjacency && rp[i + 1] > rp[i]) {
      if (!has_diag) return OR_E_NOT_LAPLACIAN;
      double tol = 1e-12 * (fabs(diag) > 1.0 ? fabs(diag) : 1.0);
      if (fabs(diag - deg) > tol) return OR_E_NOT_LAPLACIAN;
    }
  }
  for (int32_t i = 0; i < n; ++i)
    for (int64_t p = rp[i]; p < rp[i + 1]; ++p) {
      int32_t j = col[p];
      if (j == i) continue;
      int64_t t = or_find(rp, col, j, i);
      if (t < 0 || memcmp(&val[t], &val[p], sizeof(double)) != 0) return OR_E_NOT_SYMMETRIC;
    }
  int64_t m = 0;
  out_rp[0] = 0;
  for (int32_t i = 0; i < n; ++i) {
    int64_t start = m;
    for (int64_t p = rp[i]; p < rp[i + 1]; ++p) {
      if (col[p] == i) continue;
      out_col[m] = col[p];
      out_w[m] = is_adjacency ? val[p] : -val[p];
      ++m;
    }
    if (m == start) return OR_E_ISOLATED;
    out_rp[i + 1] = (int32_t)m;
  }
  *out_m = m;
  return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Heavy edge coarsening (Algorithm 1), deterministic reading.               */
/* ------------------------------------------------------------------------ */

/* The strict total order on undirected edges {a < b}: heavier first, then the
 * smaller pair hash, then the smaller a, then the smaller b.  It replaces the
 * random visiting order of Algorithm 1 and its first-index tie-break. */
typedef struct {
  double w;
  uint32_t h;
  int32_t a, b;
} or_edge;

static int or_edge_before(const or_edge* x, const or_edge* y) {
  if (x->w != y->w) return x->w > y->w;
  if (x->h != y->h) return x->h < y->h;
  if (x->a != y->a) return x->a < y->a;
  return x->b < y->b;
}

static int or_edge_cmp(const void* p, const void* q) {
  const or_edge* x = (const or_edge*)p;
  const or_edge* y = (const or_edge*)q;
  if (or_edge_before(x, y)) return -1;
  if (or_edge_before(y, x)) return 1;
  return 0;
}

static or_edge or_make_edge(int32_t u, int32_t v, double w) {
  or_edge e;
  e.a = u < v ? u : v;
  e.b = u < v ? v : u;
  e.w = w;
  e.h = or_pair_hash(e.a, e.b);
  return e;
}

/*
 * Heavy-edge matching: the greedy matching that takes the edges in the order
 * above and keeps an edge when both ends are still free.  mate[v] = partner or
 * -1.  (A locally-dominant parallel matching under the same strict order
 * produces exactly this set.)
 */
int32_t or_match(int32_t n, const int32_t* rp, const int32_t* col, const double* w,
                 int32_t* mate) {
  int64_t ne = 0;
  for (int32_t i = 0; i < n; ++i)
    for (int64_t p = rp[i]; p < rp[i + 1]; ++p)
      if (col[p] > i) ++ne;
  or_edge* e = (or_edge*)malloc(sizeof(or_edge) * (size_t)(ne > 0 ? ne : 1));
  if (!e) return OR_E_NOMEM;
  int64_t k = 0;
  for (int32_t i = 0; i < n; ++i)
    for (int64_t p = rp[i]; p < rp[i + 1]; ++p)
      if (col[p] > i) e[k++] = or_make_edge(i, col[p], w[p]);
  qsort(e, (size_t)ne, sizeof(or_edge), or_edge_cmp);
  for (int32_t v = 0; v < n; ++v) mate[v] = -1;
  for (int64_t t = 0; t < ne; ++t)
    if (mate[e[t].a] < 0 && mate[e[t].b] < 0) {
      mate[e[t].a] = e[t].b;
      mate[e[t].b] = e[t].a;
    }
  free(e);
  return OR_OK;
}

/*
 * Aggregates from a maximal matching (Algorithm 1, the branch where a vertex
 * joins the aggregate its heaviest neighbour already belongs to): a matched
 * pair is an aggregate; an unmatched vertex with edges joins the aggregate of
 * its best neighbour in the edge order (all its neighbours are matched, by
 * maximality); a vertex without edges stays alone.  Aggregates are numbered by
 * their smallest member, ascending.  Writes q[v] (the column index of the
 * interpolation matrix) and returns the number of aggregates, or < 0.
 */
int32_t or_aggregate(int32_t n, const int32_t* rp, const int32_t* col, const double* w,
                     const int32_t* mate, int32_t* q) {
  int32_t* root = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
  int32_t* minmem = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
  if (!root || !minmem) { free(root); free(minmem); return OR_E_NOMEM; }
  for (int32_t v = 0; v < n; ++v) root[v] = -1;
  for (int32_t v = 0; v < n; ++v)
    if (mate[v] >= 0) root[v] = v < mate[v] ? v : mate[v];
  for (int32_t v = 0; v < n; ++v) {
    if (mate[v] >= 0) continue;
    if (rp[v + 1] == rp[v]) { root[v] = v; continue; }
    or_edge best = or_make_edge(v, col[rp[v]], w[rp[v]]);
    int32_t bu = col[rp[v]];
    for (int64_t p = rp[v] + 1; p < rp[v + 1]; ++p) {
      or_edge c = or_make_edge(v, col[p], w[p]);
      if (or_edge_before(&c, &best)) { best = c; bu = col[p]; }
    }
    if (mate[bu] < 0) { free(root); free(minmem); return OR_E_INVALID; } /* not maximal */
    root[v] = bu < mate[bu] ? bu : mate[bu];
  }
  for (int32_t v = 0; v < n; ++v) minmem[v] = n;
  for (int32_t v = 0; v < n; ++v)
    if (v < minmem[root[v]]) minmem[root[v]] = v;
  int32_t nc = 0;
  int32_t* rank = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
  if (!rank) { free(root); free(minmem); return OR_E_NOMEM; }
  for (int32_t v = 0; v < n; ++v) rank[v] = -1;
  for (int32_t v = 0; v < n; ++v)
    if (minmem[root[v]] == v) rank[v] = nc++;
  for (int32_t v = 0; v < n; ++v) q[v] = rank[minmem[root[v]]];
  free(rank);
  free(root);
  free(minmem);
  return nc;
}

/*
 * Heavy edge coarsening as Algorithm 1 prints it (oracle-only mode, for
 * comparison with the deterministic matching): vertices are visited in the
 * order perm[0], perm[1], ...; a vertex not yet in an aggregate looks up its
 * heaviest neighbour (the most negative entry of its column of L; ties to
 * the smallest index, as MATLAB's min returns the first minimum) and either
 * opens a new aggregate with it, when that neighbour is free too, or joins the
 * neighbour's aggregate.  Aggregates are numbered in the order they are
 * opened.  Every aggregate has at least two vertices (each vertex is opened
 * with a neighbour or joins an existing aggregate).  Returns the number of
 * aggregates, or OR_E_ISOLATED for a vertex without neighbours.
 */
int32_t or_hec_random(int32_t n, const int32_t* rp, const int32_t* col, const double* w,
                      const int32_t* perm, int32_t* q) {
  for (int32_t v = 0; v < n; ++v) q[v] = -1;
  int32_t c = 0;
  for (int32_t t = 0; t < n; ++t) {
    const int32_t v = perm[t];
    if (q[v] >= 0) continue;
    if (rp[v + 1] == rp[v]) return OR_E_ISOLATED;
    int32_t m = -1;
    double best = 0.0;
    for (int64_t p = rp[v]; p < rp[v + 1]; ++p)
      if (m < 0 || w[p] > best || (w[p] == best && col[p] < m)) {
        m = col[p];
        best = w[p];
      }
    if (q[m] < 0) {
      q[m] = c;
      q[v] = c;
      ++c;
    } else {
      q[v] = q[m];
    }
  }
  return c;
}

/* A uniformly random permutation of 0..n-1 by the Fisher-Yates shuffle
 * (Knuth, TAOCP vol. 2, Algorithm P), drawing j uniform in [0, i] as
 * floor(u (i + 1)) from the 53-bit uniforms of SplitMix64(seed). */
void or_randperm(int32_t n, uint64_t seed, int32_t* perm) {
  uint64_t s = seed;
  for (int32_t i = 0; i < n; ++i) perm[i] = i;
  for (int32_t i = n - 1; i > 0; --i) {
    const double u = (double)(or_splitmix64(&s) >> 11) * (1.0 / 9007199254740992.0);
    int32_t j = (int32_t)(u * (double)(i + 1));
    if (j > i) j = i;
    const int32_t t = perm[i];
    perm[i] = perm[j];
    perm[j] = t;
  }
}

/* ------------------------------------------------------------------------ */
/* Galerkin coarse Laplacian L_c = I L I^T (Algorithm 3, Step 1).            */
/* ------------------------------------------------------------------------ */

typedef struct {
  int32_t A, B; /* coarse pair, A < B */
  int64_t seq;  /* position in the canonical fine-edge enumeration */
  double w;
} or_term;

static int or_term_cmp(const void* p, const void* q) {
  const or_term* x = (const or_term*)p;
  const or_term* y = (const or_term*)q;
  if (x->A != y->A) return x->A < y->A ? -1 : 1;
  if (x->B != y->B) return x->B < y->B ? -1 : 1;
  if (x->seq != y->seq) return x->seq < y->seq ? -1 : 1;
  return 0;
}

/*
 * Off-diagonal part of I L I^T: W_c(A,B) = sum of w_ij over fine edges {i<j}
 * with {q_i, q_j} = {A, B}, A != B, added in increasing (i, j) order (the same
 * order for (A,B) and (B,A), so W_c is bitwise symmetric).  Edges inside one
 * aggregate cancel against the diagonal and vanish.  The coarse diagonal is the
 * row sum, as at every level.  out_* must hold m_fine entries.
 */
int32_t or_galerkin(int32_t n, const int32_t* rp, const int32_t* col, const double* w,
                    const int32_t* q, int32_t nc, int32_t* out_rp, int32_t* out_col,
                    double* out_w, int64_t* out_m) {
  int64_t nt = 0;
  for (int32_t i = 0; i < n; ++i)
    for (int64_t p = rp[i]; p < rp[i + 1]; ++p)
      if (col[p] > i && q[i] != q[col[p]]) ++nt;
  or_term* t = (or_term*)malloc(sizeof(or_term) * (size_t)(nt > 0 ? nt : 1));
  int32_t* cnt = (int32_t*)calloc((size_t)nc + 1, sizeof(int32_t));
  if (!t || !cnt) { free(t); free(cnt); return OR_E_NOMEM; }
  int64_t k = 0;
  for (int32_t i = 0; i < n; ++i)
    for (int64_t p = rp[i]; p < rp[i + 1]; ++p) {
      int32_t j = col[p];
      if (j > i && q[i] != q[j]) {
        t[k].A = q[i] < q[j] ? q[i] : q[j];
        t[k].B = q[i] < q[j] ? q[j] : q[i];
        t[k].seq = k;
        t[k].w = w[p];
        ++k;
      }
    }
  qsort(t, (size_t)nt, sizeof(or_term), or_term_cmp);
  /* collapse runs: one upper-triangle entry per distinct (A,B) */
  int64_t nu = 0;
  for (int64_t s = 0; s < nt;) {
    int64_t e = s;
    double sum = 0.0;
    while (e < nt && t[e].A == t[s].A && t[e].B == t[s].B) { sum += t[e].w; ++e; }
    t[nu].A = t[s].A;
    t[nu].B = t[s].B;
    t[nu].w = sum;
    ++nu;
    s = e;
  }
  for (int64_t s = 0; s < nu; ++s) { cnt[t[s].A + 1]++; cnt[t[s].B + 1]++; }
  out_rp[0] = 0;
  for (int32_t c = 0; c < nc; ++c) out_rp[c + 1] = out_rp[c] + cnt[c + 1];
  int32_t* fill = (int32_t*)malloc(sizeof(int32_t) * (size_t)(nc > 0 ? nc : 1));
  if (!fill) { free(t); free(cnt); return OR_E_NOMEM; }
  for (int32_t c = 0; c < nc; ++c) fill[c] = out_rp[c];
  /* entries (B, A) with A < B come first in row B only if A is smaller than
   * every upper neighbour of B; fill lower parts first (ascending A since the
   * runs are sorted by A), then upper parts (ascending B). */
  for (int64_t s = 0; s < nu; ++s) {
    int32_t r = t[s].B;
    out_col[fill[r]] = t[s].A;
    out_w[fill[r]] = t[s].w;
    fill[r]++;
  }
  for (int64_t s = 0; s < nu; ++s) {
    int32_t r = t[s].A;
    out_col[fill[r]] = t[s].B;
    out_w[fill[r]] = t[s].w;
    fill[r]++;
  }
  *out_m = 2 * nu;
  free(fill);
  free(t);
  free(cnt);
  return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Colouring for the multicolour Gauss-Seidel order (Algorithm 2 visits the  */
/* rows in a fixed order; this reading visits colour classes in turn, the    */
/* rows of a class being independent of each other).                          */
/* ------------------------------------------------------------------------ */

typedef struct {
  uint32_t prio;
  int32_t v;
} or_prio;

static int or_prio_cmp(const void* p, const void* q) {
  const or_prio* x = (const or_prio*)p;
  const or_prio* y = (const or_prio*)q;
  if (x->prio != y->prio) return x->prio > y->prio ? -1 : 1;
  return x->v < y->v ? -1 : (x->v > y->v ? 1 : 0);
}

/*
 * Sequential first-fit colouring: vertices in decreasing priority (ties to
 * the smaller index) each take the smallest colour no coloured neighbour has.
 * Returns the number of colours.
 */
int32_t or_colour(int32_t n, const int32_t* rp, const int32_t* col, uint32_t level_seed,
                  int32_t* colour) {
  or_prio* o = (or_prio*)malloc(sizeof(or_prio) * (size_t)n);
  int32_t maxdeg = 0;
  for (int32_t i = 0; i < n; ++i)
    if (rp[i + 1] - rp[i] > maxdeg) maxdeg = rp[i + 1] - rp[i];
  char* used = (char*)calloc((size_t)maxdeg + 2, 1);
  if (!o || !used) { free(o); free(used); return OR_E_NOMEM; }
  for (int32_t v = 0; v < n; ++v) { o[v].prio = or_colour_priority(v, level_seed); o[v].v = v; }
  qsort(o, (size_t)n, sizeof(or_prio), or_prio_cmp);
  for (int32_t v = 0; v < n; ++v) colour[v] = -1;
  int32_t ncol = 0;
  for (int32_t t = 0; t < n; ++t) {
    int32_t v = o[t].v;
    for (int64_t p = rp[v]; p < rp[v + 1]; ++p) {
      int32_t c = colour[col[p]];
      if (c >= 0 && c <= maxdeg) used[c] = 1;
    }
    int32_t c = 0;
    while (used[c]) ++c;
    colour[v] = c;
    if (c + 1 > ncol) ncol = c + 1;
    for (int64_t p = rp[v]; p < rp[v + 1]; ++p) {
      int32_t cc = colour[col[p]];
      if (cc >= 0 && cc <= maxdeg) used[cc] = 0;
    }
  }
  free(o);
  free(used);
  return ncol;
}

/*
 * One iterated-greedy pass over a colouring (Culberson's iterated greedy,
 * one step): the colour classes are taken from the highest colour down, and
 * each vertex takes the smallest colour that no vertex recoloured before it
 * has among its neighbours.  A class is an independent set, so the order
 * inside a class does not matter, and first-fit in an order that keeps every
 * old class together never needs more colours than the old colouring.  Used
 * after or_colour: the small last classes that first-fit leaves are mostly
 * absorbed.  Returns the number of colours.
 */
int32_t or_recolour(int32_t n, const int32_t* rp, const int32_t* col, int32_t ncol,
                    int32_t* colour) {
  int32_t maxdeg = 0;
  for (int32_t i = 0; i < n; ++i)
    if (rp[i + 1] - rp[i] > maxdeg) maxdeg = rp[i + 1] - rp[i];
  char* used = (char*)calloc((size_t)maxdeg + 2, 1);
  int32_t* nw = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
  if (!used || !nw) { free(used); free(nw); return OR_E_NOMEM; }
  for (int32_t v = 0; v < n; ++v) nw[v] = -1;
  int32_t k = 0;
  for (int32_t c = ncol - 1; c >= 0; --c)
    for (int32_t v = 0; v < n; ++v) {
      if (colour[v] != c) continue;
      for (int64_t p = rp[v]; p < rp[v + 1]; ++p) {
        int32_t cc = nw[col[p]];
        if (cc >= 0 && cc <= maxdeg) used[cc] = 1;
      }
      int32_t t = 0;
      while (used[t]) ++t;
      nw[v] = t;
      if (t + 1 > k) k = t + 1;
      for (int64_t p = rp[v]; p < rp[v + 1]; ++p) {
        int32_t cc = nw[col[p]];
        if (cc >= 0 && cc <= maxdeg) used[cc] = 0;
      }
    }
  memcpy(colour, nw, sizeof(int32_t) * (size_t)n);
  free(nw);
  free(used);
  return k;
}

/*
 * Two-colouring of a bipartite level: breadth-first search from the smallest
 * unvisited vertex of each connected component, which takes colour 0, every
 * vertex at odd distance from it colour 1.  A connected bipartite graph has
 * exactly two proper 2-colourings, swapped, so fixing the colour of each
 * component's smallest vertex makes the result unique.  Returns the number of
 * colours (2, or 1 for a level without edges), or 0 when some edge joins two
 * vertices of the same colour (an odd cycle: the level is not bipartite, and
 * colour[] is then meaningless).  This is the optimal colouring of a bipartite
 * level: the classic red-black order of Gauss-Seidel on a 5-point grid.
 */
int32_t or_colour_two(int32_t n, const int32_t* rp, const int32_t* col, int32_t* colour) {
  int32_t* queue = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
  if (!queue) return OR_E_NOMEM;
  for (int32_t v = 0; v < n; ++v) colour[v] = -1;
  int32_t ncol = n > 0 ? 1 : 0;
  for (int32_t s = 0; s < n; ++s) {
    if (colour[s] >= 0) continue;
    int32_t head = 0, tail = 0;
    colour[s] = 0;
    queue[tail++] = s;
    while (head < tail) {
      const int32_t v = queue[head++];
      for (int64_t p = rp[v]; p < rp[v + 1]; ++p) {
        const int32_t u = col[p];
        if (colour[u] < 0) {
          colour[u] = 1 - colour[v];
          ncol = 2;
          queue[tail++] = u;
        }
      }
    }
  }
  free(queue);
  for (int32_t v = 0; v < n; ++v)
    for (int64_t p = rp[v]; p < rp[v + 1]; ++p)
      if (colour[col[p]] == colour[v]) return 0;
  return ncol;
}

/*
 * The colouring of a level for the smoother: on the finest level (two != 0)
 * the two-colouring when the level is bipartite; otherwise first-fit in
 * priority order followed by one iterated-greedy pass.  Coarse levels are not
 * tested: aggregation makes them non-bipartite in practice (an aggregate of
 * two neighbours and a common neighbour of both form a triangle).  Returns the
 * number of colours.
 */
int32_t or_level_colouring(int32_t n, const int32_t* rp, const int32_t* col, uint32_t level_seed,
                           int32_t two, int32_t* colour) {
  int32_t k = two ? or_colour_two(n, rp, col, colour) : 0;
  if (k != 0) return k;
  k = or_colour(n, rp, col, level_seed, colour);
  if (k > 0) k = or_recolour(n, rp, col, k, colour);
  return k;
}

/* ------------------------------------------------------------------------ */
/* Level operators.                                                          */
/* ------------------------------------------------------------------------ */

/* Shift sigma = 2 max_i d_i (Gershgorin bound on the spectrum of L). */
double or_sigma(int32_t n, const int32_t* rp, const double* w) {
  double mx = 0.0;
  for (int32_t i = 0; i < n; ++i) {
    double d = 0.0;
    for (int64_t p = rp[i]; p < rp[i + 1]; ++p) d += w[p];
    if (d > mx) mx = d;
  }
  return 2.0 * mx;
}

/* (L x)_i = sum_j w_ij (x_i - x_j), terms in CSR order. */
static double or_lap_row(const int32_t* rp, const int32_t* col, const double* w,
                         const double* x, int32_t i) {
  double s = 0.0;
  for (int64_t p = rp[i]; p < rp[i + 1]; ++p) s += w[p] * (x[i] - x[col[p]]);
  return s;
}

/* y = sigma x - L x: one power-iteration step on the shifted Laplacian. */
void or_pi_apply(int32_t n, const int32_t* rp, const int32_t* col, const double* w,
                 double sigma, const double* x, double* y) {
  for (int32_t i = 0; i < n; ++i) y[i] = sigma * x[i] - or_lap_row(rp, col, w, x, i);
}

/*
 * One Gauss-Seidel sweep (Algorithm 2) on (L - rho I) x = 0, the eigenproblem
 * written as a singular linear system with the current Rayleigh quotient as
 * the shift.  The splitting keeps Gauss-Seidel's own lower triangle D - W_l
 * and moves the shift to the right-hand side with the other known values:
 * (D - W_l) x' = (W_u + rho I) x.  Rows are visited colour by colour
 * (ascending colour, ascending index inside a colour), in place:
 *   x_i <- (1 - omega) x_i + omega (sum_j w_ij x_j + rho x_i) / d_i,
 * d_i = sum_j w_ij, both sums in CSR order, x_j the newest values and x_i the
 * row's value before its update.  An eigenvector with rho its eigenvalue is a
 * fixed point; rho = 0 gives the plain sweep on L x = 0; omega = 1 is
 * Gauss-Seidel.  Division is by d_i > 0 only, whatever rho is.
 */
void or_gs_sweep(int32_t n, const int32_t* rp, const int32_t* col, const double* w,
                 const int32_t* colour, int32_t ncolours, double rho, double omega, double* x) {
  for (int32_t c = 0; c < ncolours; ++c)
    for (int32_t i = 0; i < n; ++i) {
      if (colour[i] != c) continue;
      double num = 0.0, den = 0.0;
      for (int64_t p = rp[i]; p < rp[i + 1]; ++p) { num += w[p] * x[col[p]]; den += w[p]; }
      if (den > 0.0) {
        double g = (num + rho * x[i]) / den;
        x[i] = omega == 1.0 ? g : (1.0 - omega) * x[i] + omega * g;
      }
    }
}

/* The same sweep in the lexicographic order i = 1..n that Algorithm 2 prints
 * (oracle-only mode). */
void or_gs_sweep_lex(int32_t n, const int32_t* rp, const int32_t* col, const double* w,
                     double rho, double* x) {
  for (int32_t i = 0; i < n; ++i) {
    double num = 0.0, den = 0.0;
    for (int64_t p = rp[i]; p < rp[i + 1]; ++p) { num += w[p] * x[col[p]]; den += w[p]; }
    if (den > 0.0) x[i] = (num + rho * x[i]) / den;
  }
}

/* x <- (x - mean) / ||x - mean||_2: projection against the all-ones null
 * vector, then unit length. */
static void or_project_normalise(int32_t n, double* x) {
  double s = 0.0;
  for (int32_t i = 0; i < n; ++i) s += x[i];
  double mu = s / (double)n;
  double nn = 0.0;
  for (int32_t i = 0; i < n; ++i) { x[i] -= mu; nn += x[i] * x[i]; }
  double inv = 1.0 / sqrt(nn);
  for (int32_t i = 0; i < n; ++i) x[i] *= inv;
}

void or_project_normalise_export(int32_t n, double* x) { or_project_normalise(n, x); }

static double or_dot(int32_t n, const double* a, const double* b) {
  double s = 0.0;
  for (int32_t i = 0; i < n; ++i) s += a[i] * b[i];
  return s;
}

/*
 * Rayleigh quotient rho = sum_{i<j} w_ij (x_i - x_j)^2 / sum x_i^2 and
 * residual ||L x - rho x|| / ||x|| (finest-level eigenvalue estimate).
 */
void or_rq_residual(int32_t n, const int32_t* rp, const int32_t* col, const double* w,
                    const double* x, double* rho_out, double* res_out) {
  double num = 0.0, den = 0.0;
  for (int32_t i = 0; i < n; ++i) {
    double e = 0.0;
    for (int64_t p = rp[i]; p < rp[i + 1]; ++p) {
      double d = x[i] - x[col[p]];
      e += w[p] * d * d;
    }
    num += 0.5 * e;
    den += x[i] * x[i];
  }
  double rho = num / den;
  double r2 = 0.0;
  for (int32_t i = 0; i < n; ++i) {
    double r = or_lap_row(rp, col, w, x, i) - rho * x[i];
    r2 += r * r;
  }
  *rho_out = rho;
  *res_out = sqrt(r2 / den);
}

/* Random start on the coarsest level: x_i = 2 u_i - 1, u_i the i-th uniform
 * of SplitMix64(seed) with 53 bits. */
void or_random_start(int32_t n, uint64_t seed, double* x) {
  uint64_t s = seed;
  for (int32_t i = 0; i < n; ++i) {
    uint64_t z = or_splitmix64(&s);
    double u = (double)(z >> 11) * (1.0 / 9007199254740992.0);
    x[i] = 2.0 * u - 1.0;
  }
}

/*
 * Coarsest-level solve (Algorithm 3, Step 2; the text calls it a direct power
 * iteration): power iteration on B = sigma I - L with the all-ones vector
 * projected out, from the seeded random start.  Before each step the residual
 * ||L x - (x^T L x) x|| of the unit iterate is compared with tol * sigma (the
 * paper leaves the tolerance open; 1e-13 by default); the loop ends at or
 * below it or after max_it steps.  replay_it >= 0 forces exactly that many
 * steps instead.  Returns the number of steps taken.
 */
int32_t or_coarsest(int32_t n, const int32_t* rp, const int32_t* col, const double* w,
                    double sigma, uint64_t seed, int32_t max_it, int32_t replay_it,
                    double tol, double* x, int32_t* converged) {
  double* y = (double*)malloc(sizeof(double) * (size_t)n);
  double* lx = (double*)malloc(sizeof(double) * (size_t)n);
  or_random_start(n, seed, x);
  or_project_normalise(n, x);
  int32_t it = 0;
  *converged = 0;
  for (;;) {
    if (replay_it >= 0) {
      if (it >= replay_it) { *converged = 1; break; }
    } else {
      for (int32_t i = 0; i < n; ++i) lx[i] = or_lap_row(rp, col, w, x, i);
      double rho = or_dot(n, x, lx);
      double r2 = 0.0;
      for (int32_t i = 0; i < n; ++i) { double r = lx[i] - rho * x[i]; r2 += r * r; }
      if (sqrt(r2) <= tol * sigma) { *converged = 1; break; }
      if (it >= max_it) break;
    }
    or_pi_apply(n, rp, col, w, sigma, x, y);
    or_project_normalise(n, y);
    memcpy(x, y, sizeof(double) * (size_t)n);
    ++it;
  }
  free(y);
  free(lx);
  return it;
}

/* ------------------------------------------------------------------------ */
/* Hierarchy (Algorithm 3, Step 1).                                          */
/* ------------------------------------------------------------------------ */

typedef struct {
  int32_t n;
  int64_t m;
  int32_t* rp;
  int32_t* col;
  double* w;
  int32_t* q;      /* to the next level; NULL on the coarsest */
  int32_t* colour; /* NULL on the coarsest */
  int32_t ncolours;
  double sigma;
  double* mass;    /* aggregate sizes in finest vertices, M = I I^T; NULL on level 0 */
} or_level;

typedef struct {
  int32_t nlevels;
  or_level lv[OR_MAX_LEVELS];
} or_hier;

void or_hier_free(void* hp) {
  or_hier* h = (or_hier*)hp;
  if (!h) return;
  for (int32_t l = 0; l < h->nlevels; ++l) {
    free(h->lv[l].rp);
    free(h->lv[l].col);
    free(h->lv[l].w);
    free(h->lv[l].q);
    free(h->lv[l].colour);
    free(h->lv[l].mass);
  }
  free(h);
}

/*
 * Builds the hierarchy from the adjacency W of the finest graph: while the
 * level has more than n_coarse vertices, aggregate (matching + attach), form
 * the Galerkin coarse graph, and colour the level for the smoother (the
 * two-colouring of a bipartite finest level; otherwise first-fit in priority
 * order, then one iterated-greedy pass).  The loop
 * also stops when the next level would have fewer than 2 vertices or would not
 * be smaller, and at max_levels levels.
 */
void* or_hier_build_hec(int32_t n, const int32_t* rp, const int32_t* col, const double* w,
                        int32_t n_coarse, int32_t max_levels, uint64_t colour_seed,
                        uint64_t hec_seed, int32_t* status);

void* or_hier_build(int32_t n, const int32_t* rp, const int32_t* col, const double* w,
                    int32_t n_coarse, int32_t max_levels, uint64_t colour_seed,
                    int32_t* status) {
  return or_hier_build_hec(n, rp, col, w, n_coarse, max_levels, colour_seed, 0, status);
}

/* hec_seed != 0: every level is aggregated by or_hec_random in the order of
 * or_randperm(n_l, hec_seed + l) (the paper's randomised coarsening, an
 * oracle-only mode); 0: the deterministic matching and attachment. */
void* or_hier_build_hec(int32_t n, const int32_t* rp, const int32_t* col, const double* w,
                        int32_t n_coarse, int32_t max_levels, uint64_t colour_seed,
                        uint64_t hec_seed, int32_t* status) {
  or_hier* h = (or_hier*)calloc(1, sizeof(or_hier));
  if (!h) { *status = OR_E_NOMEM; return NULL; }
  if (max_levels < 1) max_levels = 1;
  if (max_levels > OR_MAX_LEVELS) max_levels = OR_MAX_LEVELS;
  int64_t m = rp[n];
  or_level* L0 = &h->lv[0];
  L0->n = n;
  L0->m = m;
  L0->rp = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n + 1));
  L0->col = (int32_t*)malloc(sizeof(int32_t) * (size_t)(m > 0 ? m : 1));
  L0->w = (double*)malloc(sizeof(double) * (size_t)(m > 0 ? m : 1));
  memcpy(L0->rp, rp, sizeof(int32_t) * (size_t)(n + 1));
  memcpy(L0->col, col, sizeof(int32_t) * (size_t)m);
  memcpy(L0->w, w, sizeof(double) * (size_t)m);
  h->nlevels = 1;
  int32_t l = 0;
  for (;;) {
    or_level* F = &h->lv[l];
    F->sigma = or_sigma(F->n, F->rp, F->w);
    if (F->n <= n_coarse || l + 1 >= max_levels) break;
    int32_t* mate = (int32_t*)malloc(sizeof(int32_t) * (size_t)F->n);
    int32_t* q = (int32_t*)malloc(sizeof(int32_t) * (size_t)F->n);
    int32_t nc;
    if (hec_seed) {
      or_randperm(F->n, hec_seed + (uint64_t)l, mate);  /* mate holds the order here */
      nc = or_hec_random(F->n, F->rp, F->col, F->w, mate, q);
    } else {
      int32_t st = or_match(F->n, F->rp, F->col, F->w, mate);
      nc = st == OR_OK ? or_aggregate(F->n, F->rp, F->col, F->w, mate, q) : st;
    }
    free(mate);
    if (nc < 0) { free(q); or_hier_free(h); *status = nc; return NULL; }
    if (nc < 2 || nc >= F->n) { free(q); break; }
    F->q = q;
    F->colour = (int32_t*)malloc(sizeof(int32_t) * (size_t)F->n);
    F->ncolours = or_level_colouring(F->n, F->rp, F->col, or_level_seed(colour_seed, l),
                                     l == 0, F->colour);
    or_level* C = &h->lv[l + 1];
    C->n = nc;
    C->rp = (int32_t*)malloc(sizeof(int32_t) * (size_t)(nc + 1));
    C->col = (int32_t*)malloc(sizeof(int32_t) * (size_t)(F->m > 0 ? F->m : 1));
    C->w = (double*)malloc(sizeof(double) * (size_t)(F->m > 0 ? F->m : 1));
    or_galerkin(F->n, F->rp, F->col, F->w, q, nc, C->rp, C->col, C->w, &C->m);
    /* mass of an aggregate: the finest vertices it holds (M_{l+1} = I M_l I^T) */
    C->mass = (double*)calloc((size_t)nc, sizeof(double));
    for (int32_t i = 0; i < F->n; ++i) C->mass[q[i]] += F->mass ? F->mass[i] : 1.0;
    h->nlevels = l + 2;
    ++l;
  }
  *status = OR_OK;
  return h;
}

int32_t or_hier_nlevels(const void* hp) { return ((const or_hier*)hp)->nlevels; }

/* info = {n, m, ncolours}; sigma returned. */
double or_hier_level_info(const void* hp, int32_t l, int64_t* info) {
  const or_level* L = &((const or_hier*)hp)->lv[l];
  info[0] = L->n;
  info[1] = L->m;
  info[2] = L->ncolours;
  return L->sigma;
}

void or_hier_level_copy(const void* hp, int32_t l, int32_t* rp, int32_t* col, double* w,
                        int32_t* q, int32_t* colour) {
  const or_level* L = &((const or_hier*)hp)->lv[l];
  memcpy(rp, L->rp, sizeof(int32_t) * (size_t)(L->n + 1));
  memcpy(col, L->col, sizeof(int32_t) * (size_t)L->m);
  memcpy(w, L->w, sizeof(double) * (size_t)L->m);
  if (q && L->q) memcpy(q, L->q, sizeof(int32_t) * (size_t)L->n);
  if (colour && L->colour) memcpy(colour, L->colour, sizeof(int32_t) * (size_t)L->n);
}

/* ------------------------------------------------------------------------ */
/* Solve (Algorithm 3, Steps 2 and 3, then the finest Rayleigh quotient).    */
/* ------------------------------------------------------------------------ */

typedef struct {
  uint64_t seed;
  double tol_cos;      /* stop a phase when (x_k, x_{k-1}) > 1 - tol_cos; <= 0: no
                          cosine stop, every phase runs to its cap */
  double tol_res;      /* > 0: repeat level-0 phases until residual <= tol_res */
  int32_t max_gs;      /* sweeps per smoothing phase */
  int32_t max_pi;      /* steps per power-iteration phase */
  int32_t max_outer;   /* extra level-0 rounds for tol_res */
  int32_t max_coarsest;
  int32_t gs_lexicographic; /* 1: paper's lexicographic order (oracle-only) */
  int32_t gs_unshifted;     /* 1: plain sweeps on L x = 0 (oracle-only) */
  double omega;             /* relaxation factor of the sweep; 1 = Gauss-Seidel */
  const int32_t* replay;    /* NULL, or the phase counts to execute exactly */
  int32_t replay_len;
  double tol_coarse;        /* coarsest stop: residual <= tol_coarse * sigma */
  /* Variants of the smoother and of the coarse problems (oracle-only modes
   * for comparison with the reading the library implements): */
  int32_t coarse_mass;      /* 1: coarse levels solve L_c y = lambda M_c y, M_c = I I^T */
  int32_t gs_rhs_y;         /* 1: the sweep solves L x = y with y the iterate before it */
  int32_t lanczos_k;        /* > 0: each smoothing phase is k Lanczos steps on sigma I - L */
  int32_t early_exit;       /* 1: end the finest rounds once the residual, falling by its
                               last factor each round, cannot reach tol_res within the
                               rounds max_outer leaves (or_can_reach) */
} or_solve_params;

/* The finest rounds' early exit (a serving policy beside Section 4's stop
 * rule): 1 when the residual res, multiplied round after round by its last
 * reduction factor q = res / res_prev, falls to tol within `left` more rounds
 * (the products taken one at a time, in double); 0 when it did not fall. */
int32_t or_can_reach(double res, double res_prev, double tol, int32_t left) {
  if (!(res < res_prev)) return 0;
  const double q = res / res_prev;
  double v = res;
  for (int32_t k = 0; k < left; ++k) {
    v *= q;
    if (v <= tol) return 1;
  }
  return 0;
}

/* Rayleigh quotient x^T L x / x^T x in the edge form of or_rq_residual. */
static double or_rq(int32_t n, const int32_t* rp, const int32_t* col, const double* w,
                    const double* x) {
  double num = 0.0, den = 0.0;
  for (int32_t i = 0; i < n; ++i) {
    double e = 0.0;
    for (int64_t p = rp[i]; p < rp[i + 1]; ++p) {
      double d = x[i] - x[col[p]];
      e += w[p] * d * d;
    }
    num += 0.5 * e;
    den += x[i] * x[i];
  }
  return num / den;
}

double or_rq_export(int32_t n, const int32_t* rp, const int32_t* col, const double* w,
                    const double* x) {
  return or_rq(n, rp, col, w, x);
}

/* ---- mass-weighted coarse problems (variant): L_c y = lambda M_c y ---------
 * M_c = I I^T is diagonal (aggregate sizes).  With it the coarse problem is the
 * Ritz projection of the fine one onto the aggregates' indicator vectors.
 * Inner products, means and norms are then M-weighted; m == NULL means M = I. */
static double or_mw(const double* m, int32_t i) { return m ? m[i] : 1.0; }

static double or_dot_m(int32_t n, const double* m, const double* a, const double* b) {
  double s = 0.0;
  for (int32_t i = 0; i < n; ++i) s += or_mw(m, i) * a[i] * b[i];
  return s;
}

/* x <- (x - mu 1) / ||x - mu 1||_M with mu the M-weighted mean: the projection
 * M-orthogonal to the null vector 1, then M-unit length. */
static void or_project_normalise_m(int32_t n, const double* m, double* x) {
  if (!m) { or_project_normalise(n, x); return; }
  double s = 0.0, sm = 0.0;
  for (int32_t i = 0; i < n; ++i) { s += m[i] * x[i]; sm += m[i]; }
  const double mu = s / sm;
  double nn = 0.0;
  for (int32_t i = 0; i < n; ++i) { x[i] -= mu; nn += m[i] * x[i] * x[i]; }
  const double inv = 1.0 / sqrt(nn);
  for (int32_t i = 0; i < n; ++i) x[i] *= inv;
}

/* sigma_M = 2 max_i d_i / m_i bounds the spectrum of M^{-1} L (Gershgorin). */
static double or_sigma_m(const or_level* L, const double* m) {
  if (!m) return L->sigma;
  double mx = 0.0;
  for (int32_t i = 0; i < L->n; ++i) {
    double d = 0.0;
    for (int64_t p = L->rp[i]; p < L->rp[i + 1]; ++p) d += L->w[p];
    if (d / m[i] > mx) mx = d / m[i];
  }
  return 2.0 * mx;
}

/* ---- Lanczos smoother (variant; the paper's conclusion names it) ----------
 * k steps of Lanczos on B = sigma I - L restricted to the complement of 1,
 * started from x, with full reorthogonalisation; x becomes the Ritz vector of
 * the largest Ritz value (the approximation of phi_2).  The k x k tridiagonal
 * eigenproblem is solved by cyclic Jacobi rotations (Golub & Van Loan, 8.5). */
static void or_jacobi_eig(int32_t k, double* A, double* V) {
  for (int32_t i = 0; i < k; ++i)
    for (int32_t j = 0; j < k; ++j) V[i * k + j] = i == j ? 1.0 : 0.0;
  for (int32_t sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0;
    for (int32_t i = 0; i < k; ++i)
      for (int32_t j = i + 1; j < k; ++j) off += A[i * k + j] * A[i * k + j];
    if (off < 1e-30) break;
    for (int32_t p = 0; p < k; ++p)
      for (int32_t q = p + 1; q < k; ++q) {
        const double apq = A[p * k + q];
        if (fabs(apq) < 1e-300) continue;
        const double theta = (A[q * k + q] - A[p * k + p]) / (2.0 * apq);
        const double t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
        const double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
        for (int32_t r = 0; r < k; ++r) {  /* A <- J^T A J, columns p and q */
          const double arp = A[r * k + p], arq = A[r * k + q];
          A[r * k + p] = c * arp - s * arq;
          A[r * k + q] = s * arp + c * arq;
        }
        for (int32_t r = 0; r < k; ++r) {  /* rows p and q */
          const double apr = A[p * k + r], aqr = A[q * k + r];
          A[p * k + r] = c * apr - s * aqr;
          A[q * k + r] = s * apr + c * aqr;
        }
        for (int32_t r = 0; r < k; ++r) {  /* V <- V J */
          const double vrp = V[r * k + p], vrq = V[r * k + q];
          V[r * k + p] = c * vrp - s * vrq;
          V[r * k + q] = s * vrp + c * vrq;
        }
      }
  }
}

static int32_t or_lanczos_phase(const or_level* L, int32_t k, double* x) {
  const int32_t n = L->n;
  if (k > n - 1) k = n - 1;
  if (k < 1) return 0;
  double* Q = (double*)malloc(sizeof(double) * (size_t)n * (size_t)(k + 1));
  double* T = (double*)calloc((size_t)k * (size_t)k, sizeof(double));
  double* V = (double*)malloc(sizeof(double) * (size_t)k * (size_t)k);
  double* z = (double*)malloc(sizeof(double) * (size_t)n);
  or_project_normalise(n, x);
  memcpy(Q, x, sizeof(double) * (size_t)n);
  int32_t steps = 0;
  for (int32_t j = 0; j < k; ++j) {
    const double* qj = Q + (size_t)j * n;
    or_pi_apply(n, L->rp, L->col, L->w, L->sigma, qj, z);
    /* full reorthogonalisation against 1 and q_0 .. q_j, twice (Gram-Schmidt
     * twice is enough, Giraud et al. 2005); alpha_j = q_j^T B q_j collects
     * both passes' coefficients on q_j, beta_{j-1} is set with q_j */
    for (int32_t pass = 0; pass < 2; ++pass) {
      double mu = 0.0;
      for (int32_t i = 0; i < n; ++i) mu += z[i];
      mu /= (double)n;
      for (int32_t i = 0; i < n; ++i) z[i] -= mu;
      for (int32_t r = 0; r <= j; ++r) {
        const double* qr = Q + (size_t)r * n;
        const double h = or_dot(n, qr, z);
        for (int32_t i = 0; i < n; ++i) z[i] -= h * qr[i];
        if (r == j) T[j * k + j] += h;
      }
    }
    steps = j + 1;
    const double beta = sqrt(or_dot(n, z, z));
    if (j + 1 == k || beta <= 1e-14 * L->sigma) break;
    T[j * k + j + 1] = T[(j + 1) * k + j] = beta;
    double* qn = Q + (size_t)(j + 1) * n;
    for (int32_t i = 0; i < n; ++i) qn[i] = z[i] / beta;
  }
  /* top Ritz pair of the leading steps x steps block */
  double* A = (double*)malloc(sizeof(double) * (size_t)steps * (size_t)steps);
  for (int32_t i = 0; i < steps; ++i)
    for (int32_t j = 0; j < steps; ++j) A[i * steps + j] = T[i * k + j];
  or_jacobi_eig(steps, A, V);
  int32_t best = 0;
  for (int32_t i = 1; i < steps; ++i) if (A[i * steps + i] > A[best * steps + best]) best = i;
  for (int32_t i = 0; i < n; ++i) {
    double v = 0.0;
    for (int32_t r = 0; r < steps; ++r) v += Q[(size_t)r * n + i] * V[r * steps + best];
    x[i] = v;
  }
  or_project_normalise(n, x);
  free(A);
  free(Q);
  free(T);
  free(V);
  free(z);
  return steps;
}

/* One smoothing phase: each sweep takes the Rayleigh quotient of the current
 * (unit, mean-free) iterate as its shift; sweeps continue until the cosine
 * test passes or the cap. */
static int32_t or_gs_phase(const or_level* L, const or_solve_params* P, int32_t forced,
                           double* x, double* xp, double* cos_out) {
  const double* m = P->coarse_mass ? L->mass : NULL;
  if (P->lanczos_k > 0) {
    /* variant: one Lanczos phase in place of the sweeps */
    memcpy(xp, x, sizeof(double) * (size_t)L->n);
    const int32_t k = or_lanczos_phase(L, forced >= 0 ? forced : P->lanczos_k, x);
    *cos_out = or_dot(L->n, x, xp);
    return k;
  }
  int32_t k = 0;
  double c = 0.0;
  for (;;) {
    if (k >= (forced >= 0 ? forced : P->max_gs)) break;
    memcpy(xp, x, sizeof(double) * (size_t)L->n);
    double rho = P->gs_unshifted ? 0.0 : or_rq(L->n, L->rp, L->col, L->w, x);
    if (m) rho *= or_dot(L->n, x, x) / or_dot_m(L->n, m, x, x);  /* x^T L x / x^T M x */
    if (P->gs_lexicographic) {
      or_gs_sweep_lex(L->n, L->rp, L->col, L->w, rho, x);
    } else if (m || P->gs_rhs_y) {
      /* the sweep on (L - rho M) x = 0 (mass-weighted) or on L x = y */
      for (int32_t cc = 0; cc < L->ncolours; ++cc)
        for (int32_t i = 0; i < L->n; ++i) {
          if (L->colour[i] != cc) continue;
          double num = 0.0, den = 0.0;
          for (int64_t p = L->rp[i]; p < L->rp[i + 1]; ++p) { num += L->w[p] * x[L->col[p]]; den += L->w[p]; }
          if (den > 0.0) {
            const double b = P->gs_rhs_y ? xp[i] : rho * or_mw(m, i) * x[i];
            const double g = (num + b) / den;
            x[i] = P->omega == 1.0 ? g : (1.0 - P->omega) * x[i] + P->omega * g;
          }
        }
    } else {
      or_gs_sweep(L->n, L->rp, L->col, L->w, L->colour, L->ncolours, rho, P->omega, x);
    }
    or_project_normalise_m(L->n, m, x);
    ++k;
    c = or_dot_m(L->n, m, x, xp);
    if (forced < 0 && P->tol_cos > 0.0 && c > 1.0 - P->tol_cos) break;
  }
  *cos_out = c;
  return k;
}

/* One power-iteration phase on B = sigma I - L (projected). */
static int32_t or_pi_phase(const or_level* L, const or_solve_params* P, int32_t forced,
                           double* x, double* y, double* cos_out) {
  const double* m = P->coarse_mass ? L->mass : NULL;
  const double sig = or_sigma_m(L, m);
  int32_t k = 0;
  double c = 0.0;
  for (;;) {
    if (k >= (forced >= 0 ? forced : P->max_pi)) break;
    if (m) /* y = sigma x - M^{-1} L x */
      for (int32_t i = 0; i < L->n; ++i) y[i] = sig * x[i] - or_lap_row(L->rp, L->col, L->w, x, i) / m[i];
    else
      or_pi_apply(L->n, L->rp, L->col, L->w, L->sigma, x, y);
    or_project_normalise_m(L->n, m, y);
    ++k;
    c = or_dot_m(L->n, m, x, y);
    memcpy(x, y, sizeof(double) * (size_t)L->n);
    if (forced < 0 && P->tol_cos > 0.0 && c > 1.0 - P->tol_cos) break;
  }
  *cos_out = c;
  return k;
}

/* Output sign: the first entry with |x_i| >= 1e-3 max|x| is made positive. */
void or_fix_sign(int32_t n, double* x) {
  double mx = 0.0;
  for (int32_t i = 0; i < n; ++i) if (fabs(x[i]) > mx) mx = fabs(x[i]);
  for (int32_t i = 0; i < n; ++i)
    if (fabs(x[i]) >= 1e-3 * mx) {
      if (x[i] < 0.0) for (int32_t j = 0; j < n; ++j) x[j] = -x[j];
      break;
    }
}

/*
 * Full solve on a built hierarchy.  counts receives the executed schedule:
 * [coarsest steps, (gs, pi) for levels J-1 .. 0, then (gs, pi) per extra
 * level-0 round]; scal = {lambda, residual, last cosine}.  Returns OR_OK, or
 * OR_E_NOT_CONVERGED when tol_res was not met or the coarsest solve hit its
 * cap (x and scal are filled either way).
 */
int32_t or_solve(const void* hp, const or_solve_params* P, double* x_out, double* scal,
                 int32_t* counts, int32_t counts_cap, int32_t* counts_len) {
  const or_hier* h = (const or_hier*)hp;
  int32_t J = h->nlevels - 1;
  int32_t nmax = h->lv[0].n;
  double* x = (double*)malloc(sizeof(double) * (size_t)nmax);
  double* y = (double*)malloc(sizeof(double) * (size_t)nmax);
  double* t = (double*)malloc(sizeof(double) * (size_t)nmax);
  if (!x || !y || !t) { free(x); free(y); free(t); return OR_E_NOMEM; }
  int32_t nc_out = 0;
  int32_t status = OR_OK;
  const int32_t* R = P->replay;
  int32_t ri = 0;
#define OR_NEXT_FORCED() ((R && ri < P->replay_len) ? R[ri++] : -1)
#define OR_PUSH(v) do { if (nc_out < counts_cap) counts[nc_out] = (v); ++nc_out; } while (0)
  const or_level* C = &h->lv[J];
  int32_t conv = 0;
  int32_t cit;
  if (P->coarse_mass && C->mass) {
    /* variant: power iteration on sigma I - M^{-1} L, M-projected, until the
     * M^{-1}-norm residual ||M^{-1} L x - rho x||_M <= tol_coarse sigma */
    const double sig = or_sigma_m(C, C->mass);
    const int32_t forced = OR_NEXT_FORCED();
    or_random_start(C->n, P->seed, x);
    or_project_normalise_m(C->n, C->mass, x);
    for (cit = 0;; ++cit) {
      for (int32_t i = 0; i < C->n; ++i) t[i] = or_lap_row(C->rp, C->col, C->w, x, i) / C->mass[i];
      if (forced >= 0) {
        if (cit >= forced) { conv = 1; break; }
      } else {
        const double rho = or_dot_m(C->n, C->mass, x, t);
        double r2 = 0.0;
        for (int32_t i = 0; i < C->n; ++i) { const double r = t[i] - rho * x[i]; r2 += C->mass[i] * r * r; }
        if (sqrt(r2) <= P->tol_coarse * sig) { conv = 1; break; }
        if (cit >= P->max_coarsest) break;
      }
      for (int32_t i = 0; i < C->n; ++i) y[i] = sig * x[i] - t[i];
      or_project_normalise_m(C->n, C->mass, y);
      memcpy(x, y, sizeof(double) * (size_t)C->n);
    }
  } else {
    cit = or_coarsest(C->n, C->rp, C->col, C->w, C->sigma, P->seed, P->max_coarsest,
                      OR_NEXT_FORCED(), P->tol_coarse, x, &conv);
  }
  if (!conv) status = OR_E_NOT_CONVERGED;
  OR_PUSH(cit);
  double cosv = 1.0;
  for (int32_t l = J - 1; l >= 0; --l) {
    const or_level* F = &h->lv[l];
    /* prolongation y^l = I^T y^{l+1}: x_f[i] = x_c[q(i)] */
    for (int32_t i = 0; i < F->n; ++i) y[i] = x[F->q[i]];
    memcpy(x, y, sizeof(double) * (size_t)F->n);
    or_project_normalise_m(F->n, P->coarse_mass ? F->mass : NULL, x);
    int32_t g = or_gs_phase(F, P, OR_NEXT_FORCED(), x, t, &cosv);
    int32_t p = or_pi_phase(F, P, OR_NEXT_FORCED(), x, y, &cosv);
    OR_PUSH(g);
    OR_PUSH(p);
  }
  const or_level* F0 = &h->lv[0];
  double rho, res;
  or_rq_residual(F0->n, F0->rp, F0->col, F0->w, x, &rho, &res);
  double res_prev = res;
  int32_t outer = 0;
  for (;;) {
    int32_t fg, fp;
    if (R) {
      if (ri >= P->replay_len) break;
      fg = OR_NEXT_FORCED();
      fp = OR_NEXT_FORCED();
    } else {
      if (!(P->tol_res > 0.0) || res <= P->tol_res || outer >= P->max_outer) break;
      if (P->early_exit && outer > 0 &&
          !or_can_reach(res, res_prev, P->tol_res, P->max_outer - outer))
        break;
      fg = fp = -1;
    }
    if (J == 0) break; /* a one-level hierarchy is solved by the coarsest solve */
    int32_t g = or_gs_phase(F0, P, fg, x, t, &cosv);
    int32_t p = or_pi_phase(F0, P, fp, x, y, &cosv);
    OR_PUSH(g);
    OR_PUSH(p);
    ++outer;
    res_prev = res;
    or_rq_residual(F0->n, F0->rp, F0->col, F0->w, x, &rho, &res);
  }
  if (!R && P->tol_res > 0.0 && res > P->tol_res) status = OR_E_NOT_CONVERGED;
  or_fix_sign(F0->n, x);
  memcpy(x_out, x, sizeof(double) * (size_t)F0->n);
  scal[0] = rho;
  scal[1] = res;
  scal[2] = cosv;
  *counts_len = nc_out;
#undef OR_NEXT_FORCED
#undef OR_PUSH
  free(x);
  free(y);
  free(t);
  return status;
}
