/*
 * CPU oracle for the per-tick spatial join of moving-object positions
 * against rectangular range queries (Lettich, Orlando, Silvestri, Jensen,
 * "Manycore processing of repeated range queries over massive moving
 * objects observations").
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  It shares no
 * source with the HIP path under paper_1411_3212_amd/csrc and includes none
 * of its headers.
 *
 * Every function is plain, sequential-by-definition C (OpenMP only splits
 * independent queries across threads).  Floating point: coordinates are
 * IEEE-754 binary32; the containment test is four comparisons and involves
 * no arithmetic, so result sets are exact.  The only float arithmetic is
 * the cell mapping of the index frame, which is one binary32 subtraction
 * followed by a multiplication by a power of two (exact), compiled with
 * -ffp-contract=off.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_L 16u /* bits per axis of the finest Morton grid */

/* ------------------------------------------------------------------ */
/* Tick batching (Section "Batch processing"): several updates of one   */
/* object inside a tick -> only the most recent counts; an object with  */
/* no update keeps its last known position.                             */
/* ------------------------------------------------------------------ */

/* Applies m updates in array order; a later entry overwrites an earlier
 * one.  Entries with id >= N or a non-finite coordinate are skipped and
 * counted in the return value. */
int64_t or_apply_updates(uint32_t N, float *px, float *py, uint8_t *has,
                         uint32_t m, const uint32_t *id, const float *x,
                         const float *y) {
  int64_t bad = 0;
  for (uint32_t k = 0; k < m; ++k) {
    if (id[k] >= N || !isfinite(x[k]) || !isfinite(y[k])) {
      ++bad;
      continue;
    }
    px[id[k]] = x[k];
    py[id[k]] = y[k];
    has[id[k]] = 1;
  }
  return bad;
}

/* The most recent query of each object within a tick is the one that is
 * answered; earlier queries with the same issuer are superseded.
 * live[k] = 1 iff query k is the last one carrying qid[k]. */
void or_live_queries(uint32_t N, uint32_t nq, const uint32_t *qid,
                     uint8_t *live) {
  uint8_t *seen = (uint8_t *)calloc(N ? N : 1, 1);
  for (uint32_t k = nq; k-- > 0;) {
    uint32_t q = qid[k];
    if (q < N && !seen[q]) {
      seen[q] = 1;
      live[k] = 1;
    } else {
      live[k] = 0;
    }
  }
  free(seen);
}

/* ------------------------------------------------------------------ */
/* Definition 1: res(q) = { o_j : x^a <= x_j <= x^b and y^a <= y_j <= y^b } */
/* closed on all four sides, brute force over queries x objects.        */
/* ------------------------------------------------------------------ */

static inline int or_inside(float x, float y, float xa, float ya, float xb,
                            float yb) {
  return xa <= x && x <= xb && ya <= y && y <= yb;
}

/* cnt[k] = |res(q_k)| (0 for superseded queries). Returns the sum. */
int64_t or_brute_counts(uint32_t N, const float *px, const float *py,
                        const uint8_t *has, uint32_t nq, const uint8_t *live,
                        const float *xa, const float *ya, const float *xb,
                        const float *yb, uint64_t *cnt) {
  int64_t total = 0;
#pragma omp parallel for schedule(dynamic, 16) reduction(+ : total)
  for (int64_t k = 0; k < (int64_t)nq; ++k) {
    uint64_t c = 0;
    if (live[k]) {
      for (uint32_t j = 0; j < N; ++j)
        if (has[j] && or_inside(px[j], py[j], xa[k], ya[k], xb[k], yb[k])) ++c;
    }
    cnt[k] = c;
    total += (int64_t)c;
  }
  return total;
}

/* Fills ids[off[k] .. off[k+1]) with res(q_k) in ascending id order. */
void or_brute_lists(uint32_t N, const float *px, const float *py,
                    const uint8_t *has, uint32_t nq, const uint8_t *live,
                    const float *xa, const float *ya, const float *xb,
                    const float *yb, const uint64_t *off, uint32_t *ids) {
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t k = 0; k < (int64_t)nq; ++k) {
    uint64_t w = off[k];
    if (!live[k]) continue;
    for (uint32_t j = 0; j < N; ++j)
      if (has[j] && or_inside(px[j], py[j], xa[k], ya[k], xb[k], yb[k]))
        ids[w++] = j;
  }
}

/* ------------------------------------------------------------------ */
/* Order-independent pair-set hash: H(q) = sum over id in res(q) of     */
/* mix64((qid << 32) | id) mod 2^64, where mix64 is the output function */
/* of SplitMix64 (Steele, Lea, Flood, OOPSLA 2014).                     */
/* ------------------------------------------------------------------ */

uint64_t or_mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
  return z ^ (z >> 31);
}

/* Brute-force count and hash per query. */
int64_t or_brute_hash(uint32_t N, const float *px, const float *py,
                      const uint8_t *has, uint32_t nq, const uint32_t *qid,
                      const uint8_t *live, const float *xa, const float *ya,
                      const float *xb, const float *yb, uint64_t *cnt,
                      uint64_t *hash) {
  int64_t total = 0;
#pragma omp parallel for schedule(dynamic, 16) reduction(+ : total)
  for (int64_t k = 0; k < (int64_t)nq; ++k) {
    uint64_t c = 0, h = 0;
    if (live[k]) {
      uint64_t hi = (uint64_t)qid[k] << 32;
      for (uint32_t j = 0; j < N; ++j)
        if (has[j] && or_inside(px[j], py[j], xa[k], ya[k], xb[k], yb[k])) {
          ++c;
          h += or_mix64(hi | j);
        }
    }
    cnt[k] = c;
    hash[k] = h;
    total += (int64_t)c;
  }
  return total;
}

/* ------------------------------------------------------------------ */
/* Second, independent CPU index: a plain uniform grid in double        */
/* precision whose cell side is a quarter of the largest query side     */
/* (at least 1/4096 of the objects' extent).  A query scans every cell  */
/* its corners' floors span, so no candidate is missed.  Same exact     */
/* containment test; used to check the brute force at scale and to      */
/* replace it where the brute force is too slow.                        */
/* ------------------------------------------------------------------ */

int64_t or_grid_hash(uint32_t N, const float *px, const float *py,
                     const uint8_t *has, uint32_t nq, const uint32_t *qid,
                     const uint8_t *live, const float *xa, const float *ya,
                     const float *xb, const float *yb, uint64_t *cnt,
                     uint64_t *hash) {
  double x0 = INFINITY, y0 = INFINITY, x1 = -INFINITY, y1 = -INFINITY;
  uint32_t npres = 0;
  for (uint32_t j = 0; j < N; ++j) {
    if (!has[j]) continue;
    ++npres;
    if (px[j] < x0) x0 = px[j];
    if (px[j] > x1) x1 = px[j];
    if (py[j] < y0) y0 = py[j];
    if (py[j] > y1) y1 = py[j];
  }
  if (npres == 0) {
    for (uint32_t k = 0; k < nq; ++k) cnt[k] = hash[k] = 0;
    return 0;
  }
  double side = 0.0;
  for (uint32_t k = 0; k < nq; ++k) {
    if (!live[k]) continue;
    double w = (double)xb[k] - (double)xa[k], h = (double)yb[k] - (double)ya[k];
    if (w > side && isfinite(w)) side = w;
    if (h > side && isfinite(h)) side = h;
  }
  double ext = fmax(x1 - x0, y1 - y0);
  side *= 0.25; /* cells of a quarter of the largest query side: fewer candidates */
  if (side < ext / 4096.0) side = ext / 4096.0; /* bound the cell count */
  if (!(side > 0.0)) side = 1.0;
  int64_t gx = (int64_t)floor((x1 - x0) / side) + 1;
  int64_t gy = (int64_t)floor((y1 - y0) / side) + 1;
  int64_t ncell = gx * gy;
  uint32_t *start = (uint32_t *)calloc((size_t)ncell + 1, sizeof(uint32_t));
  uint32_t *items = (uint32_t *)malloc(sizeof(uint32_t) * (npres ? npres : 1));
  int64_t *cellof = (int64_t *)malloc(sizeof(int64_t) * (N ? N : 1));
  for (uint32_t j = 0; j < N; ++j) {
    if (!has[j]) continue;
    int64_t cx = (int64_t)floor(((double)px[j] - x0) / side);
    int64_t cy = (int64_t)floor(((double)py[j] - y0) / side);
    if (cx >= gx) cx = gx - 1;
    if (cy >= gy) cy = gy - 1;
    cellof[j] = cy * gx + cx;
    start[cellof[j] + 1]++;
  }
  for (int64_t c = 0; c < ncell; ++c) start[c + 1] += start[c];
  /* positions are copied next to their ids in cell order, so a query scans
     its candidate cells sequentially */
  float *ix = (float *)malloc(sizeof(float) * (npres ? npres : 1));
  float *iy = (float *)malloc(sizeof(float) * (npres ? npres : 1));
  uint32_t *fill = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)ncell);
  memcpy(fill, start, sizeof(uint32_t) * (size_t)ncell);
  for (uint32_t j = 0; j < N; ++j)
    if (has[j]) {
      uint32_t t = fill[cellof[j]]++;
      items[t] = j;
      ix[t] = px[j];
      iy[t] = py[j];
    }
  free(fill);
  int64_t total = 0;
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : total)
  for (int64_t k = 0; k < (int64_t)nq; ++k) {
    uint64_t c = 0, h = 0;
    int ok = live[k] && xa[k] <= xb[k] && ya[k] <= yb[k];
    if (ok) {
      uint64_t hi = (uint64_t)qid[k] << 32;
      double fx0 = floor(((double)xa[k] - x0) / side);
      double fx1 = floor(((double)xb[k] - x0) / side);
      double fy0 = floor(((double)ya[k] - y0) / side);
      double fy1 = floor(((double)yb[k] - y0) / side);
      if (fx1 >= 0 && fy1 >= 0 && fx0 < gx + 1 && fy0 < gy + 1) {
        int64_t cx0 = fx0 < 0 ? 0 : (int64_t)fx0, cy0 = fy0 < 0 ? 0 : (int64_t)fy0;
        int64_t cx1 = fx1 >= gx ? gx - 1 : (int64_t)fx1;
        int64_t cy1 = fy1 >= gy ? gy - 1 : (int64_t)fy1;
        for (int64_t cy = cy0; cy <= cy1; ++cy)
          for (int64_t cx = cx0; cx <= cx1; ++cx) {
            int64_t cell = cy * gx + cx;
            for (uint32_t t = start[cell]; t < start[cell + 1]; ++t) {
              if (or_inside(ix[t], iy[t], xa[k], ya[k], xb[k], yb[k])) {
                ++c;
                h += or_mix64(hi | items[t]);
              }
            }
          }
      }
    }
    cnt[k] = c;
    hash[k] = h;
    total += (int64_t)c;
  }
  free(start);
  free(items);
  free(ix);
  free(iy);
  free(cellof);
  return total;
}

/* ------------------------------------------------------------------ */
/* Index frame and cell mapping (Definitions 2-4; mapping functions f  */
/* and g).  The frame is the square anchored at the lower-left corner  */
/* of the objects' MBR whose side is the smallest power of two that is */
/* >= the MBR's larger extent (extent taken as a binary32 difference),  */
/* never below 2^-100.  Cell index at the finest level L = 16:          */
/*   i = clamp(floor(fl32(x - x0) * 2^(L - e)), 0, 2^L - 1)             */
/* This function is monotone in x, so objects and query corners mapped  */
/* through it give sound covering decisions.                           */
/* ------------------------------------------------------------------ */

int or_frame(uint32_t N, const float *px, const float *py, const uint8_t *has,
             float *x0out, float *y0out, int32_t *eout) {
  float x0 = INFINITY, y0 = INFINITY, x1 = -INFINITY, y1 = -INFINITY;
  uint32_t npres = 0;
  for (uint32_t j = 0; j < N; ++j) {
    if (!has[j]) continue;
    ++npres;
    x0 = fminf(x0, px[j]);
    x1 = fmaxf(x1, px[j]);
    y0 = fminf(y0, py[j]);
    y1 = fmaxf(y1, py[j]);
  }
  if (npres == 0) {
    *x0out = 0.0f;
    *y0out = 0.0f;
    *eout = 0;
    return 0;
  }
  volatile float w = x1 - x0, h = y1 - y0;
  float m = w > h ? w : h;
  int e;
  if (!(m > 0.0f)) {
    e = -100;
  } else {
    int ex;
    float f = frexpf(m, &ex); /* m = f * 2^ex, f in [0.5, 1) */
    e = (f == 0.5f) ? ex - 1 : ex;
    if (e < -100) e = -100;
  }
  *x0out = x0;
  *y0out = y0;
  *eout = e;
  return (int)npres;
}

uint32_t or_cell(float v, float v0, int32_t e) {
  volatile float d = v - v0; /* one binary32 rounding */
  float t = d * ldexpf(1.0f, (int)OR_L - e); /* exact: power-of-two scale */
  if (!(t >= 0.0f)) return 0u;
  if (t >= 65536.0f) return 65535u;
  return (uint32_t)t;
}

/* Morton code (Z-order): bit b of i goes to bit 2b, bit b of j to bit
 * 2b + 1. */
uint32_t or_morton(uint32_t i, uint32_t j, uint32_t nbits) {
  uint32_t z = 0;
  for (uint32_t b = 0; b < nbits; ++b) {
    z |= ((i >> b) & 1u) << (2 * b);
    z |= ((j >> b) & 1u) << (2 * b + 1);
  }
  return z;
}

void or_demorton(uint32_t z, uint32_t nbits, uint32_t *i, uint32_t *j) {
  uint32_t a = 0, b = 0;
  for (uint32_t t = 0; t < nbits; ++t) {
    a |= ((z >> (2 * t)) & 1u) << t;
    b |= ((z >> (2 * t + 1)) & 1u) << t;
  }
  *i = a;
  *j = b;
}

/* ------------------------------------------------------------------ */
/* Algorithm 1 (GPU-based PR-quadtree construction), as plain CPU steps:*/
/*  1. Morton code of every object at the finest level, then a stable  */
/*     sort of the objects by code.                                    */
/*  2. I_A <- {root interval}, C <- {}, l <- 1.                        */
/*  3. while I_A is non-empty and l <= l_max: detect the four level-l  */
/*     child quadrants (sub-intervals) of every interval in I_A; a     */
/*     child with more than th objects and l < l_max goes to the next  */
/*     I_A, every other child (including empty ones) is a leaf of C.   */
/* Leaves are returned in Morton order: lvl, z (code at its level),    */
/* [beg, end) into the sorted object arrays.                           */
/* ------------------------------------------------------------------ */

static int or_cmp_u64(const void *a, const void *b) {
  uint64_t x = *(const uint64_t *)a, y = *(const uint64_t *)b;
  return (x > y) - (x < y);
}

/* Step 1: codes of present objects; (code, id) sorted by code then id
 * (== a stable sort of ids in ascending order).  Returns n_present. */
uint32_t or_sorted_codes(uint32_t N, const float *px, const float *py,
                         const uint8_t *has, float x0, float y0, int32_t e,
                         uint32_t *code_out, uint32_t *id_out) {
  uint64_t *kv = (uint64_t *)malloc(sizeof(uint64_t) * (N ? N : 1));
  uint32_t n = 0;
  for (uint32_t j = 0; j < N; ++j) {
    if (!has[j]) continue;
    uint32_t ci = or_cell(px[j], x0, e), cj = or_cell(py[j], y0, e);
    kv[n++] = ((uint64_t)or_morton(ci, cj, OR_L) << 32) | j;
  }
  qsort(kv, n, sizeof(uint64_t), or_cmp_u64);
  for (uint32_t t = 0; t < n; ++t) {
    code_out[t] = (uint32_t)(kv[t] >> 32);
    id_out[t] = (uint32_t)kv[t];
  }
  free(kv);
  return n;
}

typedef struct {
  uint32_t z, beg, end;
} or_iv;

typedef struct {
  uint64_t start; /* z << 2(L - l): first finest-level code of the leaf */
  uint32_t lvl, z, beg, end;
} or_leaf;

static int or_cmp_leaf(const void *a, const void *b) {
  uint64_t x = ((const or_leaf *)a)->start, y = ((const or_leaf *)b)->start;
  return (x > y) - (x < y);
}

/* Steps 2-3 over sorted codes.  Returns the number of leaves, or -1 if
 * more than cap leaves would be produced. */
int64_t or_quadtree(uint32_t n, const uint32_t *code, uint32_t th,
                    uint32_t l_max, uint64_t cap, uint32_t *lvl, uint32_t *z,
                    uint32_t *beg, uint32_t *end, uint32_t *l_deep_out) {
  size_t ia_cap = 16, next_cap = 16, leaf_cap = 64;
  or_iv *ia = (or_iv *)malloc(sizeof(or_iv) * ia_cap);
  or_iv *next = (or_iv *)malloc(sizeof(or_iv) * next_cap);
  or_leaf *leaves = (or_leaf *)malloc(sizeof(or_leaf) * leaf_cap);
  size_t n_ia = 1, n_leaf = 0;
  ia[0].z = 0;
  ia[0].beg = 0;
  ia[0].end = n;
  uint32_t l = 1, l_deep = 0;
  while (n_ia > 0 && l <= l_max) {
    size_t n_next = 0;
    uint32_t shift = 2 * (OR_L - l);
    for (size_t a = 0; a < n_ia; ++a) {
      /* detect quadrants: scan the parent's interval */
      uint32_t p = ia[a].beg;
      for (uint32_t k = 0; k < 4; ++k) {
        uint32_t cz = ia[a].z * 4 + k;
        uint32_t b = p;
        while (p < ia[a].end && (code[p] >> shift) == cz) ++p;
        uint32_t cnt = p - b;
        if (cnt > th && l < l_max) {
          if (n_next == next_cap) {
            next_cap *= 2;
            next = (or_iv *)realloc(next, sizeof(or_iv) * next_cap);
          }
          next[n_next].z = cz;
          next[n_next].beg = b;
          next[n_next].end = p;
          ++n_next;
        } else {
          if (n_leaf == leaf_cap) {
            leaf_cap *= 2;
            leaves = (or_leaf *)realloc(leaves, sizeof(or_leaf) * leaf_cap);
          }
          leaves[n_leaf].start = (uint64_t)cz << shift;
          leaves[n_leaf].lvl = l;
          leaves[n_leaf].z = cz;
          leaves[n_leaf].beg = b;
          leaves[n_leaf].end = p;
          ++n_leaf;
        }
      }
    }
    or_iv *t = ia;
    ia = next;
    next = t;
    size_t tc = ia_cap;
    ia_cap = next_cap;
    next_cap = tc;
    n_ia = n_next;
    l_deep = l;
    ++l;
  }
  free(ia);
  free(next);
  if (n_leaf > cap) {
    free(leaves);
    return -1;
  }
  qsort(leaves, n_leaf, sizeof(or_leaf), or_cmp_leaf);
  for (size_t t = 0; t < n_leaf; ++t) {
    lvl[t] = leaves[t].lvl;
    z[t] = leaves[t].z;
    beg[t] = leaves[t].beg;
    end[t] = leaves[t].end;
  }
  free(leaves);
  if (l_deep_out) *l_deep_out = l_deep;
  return (int64_t)n_leaf;
}

/* ------------------------------------------------------------------ */
/* Query splitting, mapping function g: a query is mapped to every     */
/* leaf whose finest-level cell range overlaps the query's corner-cell */
/* range [f(x^a), f(x^b)] x [f(y^a), f(y^b)], once per leaf.  A        */
/* subquery is covering when the leaf's cell range lies strictly inside*/
/* the corner-cell range on both axes (then every object of the leaf   */
/* is inside the query, by monotonicity of f), otherwise intersecting. */
/* Plain definition: every query is compared with every leaf.          */
/* Pass 1 (out == NULL): ni[k], nc[k] = counts per query.              */
/* Pass 2: for query k, writes leaf indices at out_i[oi[k]..] and       */
/* out_c[oc[k]..] in Morton order of the leaves.                        */
/* Queries with live[k] == 0 or an inverted / non-finite rectangle     */
/* have no subqueries.                                                  */
/* ------------------------------------------------------------------ */

void or_split(uint32_t nq, const uint8_t *live, const float *xa,
              const float *ya, const float *xb, const float *yb, float x0,
              float y0, int32_t e, uint32_t n_leaf, const uint32_t *lvl,
              const uint32_t *z, uint64_t *ni, uint64_t *nc,
              const uint64_t *oi, const uint64_t *oc, uint32_t *out_i,
              uint32_t *out_c) {
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t k = 0; k < (int64_t)nq; ++k) {
    uint64_t ci = 0, cc = 0;
    int ok = live[k] && xa[k] <= xb[k] && ya[k] <= yb[k] && isfinite(xa[k]) &&
             isfinite(xb[k]) && isfinite(ya[k]) && isfinite(yb[k]);
    if (ok) {
      uint32_t qi0 = or_cell(xa[k], x0, e), qi1 = or_cell(xb[k], x0, e);
      uint32_t qj0 = or_cell(ya[k], y0, e), qj1 = or_cell(yb[k], y0, e);
      for (uint32_t t = 0; t < n_leaf; ++t) {
        uint32_t zi, zj;
        or_demorton(z[t], lvl[t], &zi, &zj);
        uint32_t s = OR_L - lvl[t];
        uint32_t ilo = zi << s, ihi = ((zi + 1) << s) - 1;
        uint32_t jlo = zj << s, jhi = ((zj + 1) << s) - 1;
        if (ilo > qi1 || ihi < qi0 || jlo > qj1 || jhi < qj0) continue;
        int cov = qi0 < ilo && ihi < qi1 && qj0 < jlo && jhi < qj1;
        if (cov) {
          if (out_c) out_c[oc[k] + cc] = t;
          ++cc;
        } else {
          if (out_i) out_i[oi[k] + ci] = t;
          ++ci;
        }
      }
    }
    if (ni) ni[k] = ci;
    if (nc) nc[k] = cc;
  }
}

int or_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* Threads of the OpenMP loops over queries (n >= 1), e.g. 1 for a
 * single-core timing. */
void or_set_num_threads(int n) {
#ifdef _OPENMP
  if (n >= 1) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

/* ------------------------------------------------------------------ */
/* Uniform grid partitioning (Definition "MBR partitioning into a      */
/* uniform grid"; index creation and indexing of UG).  The frame is the */
/* same square as the quadtree's; it is cut into s columns and s rows   */
/* of (nearly) equal width along the finest-level cells of the frame:   */
/* finest cell i (0..2^16-1) belongs to column floor(i * s / 2^16).     */
/* Every column then spans floor or ceil of 2^16 / s finest cells (the  */
/* widths differ by at most one finest cell), the map is monotone, and  */
/* objects and query corners go through the same finest-cell function   */
/* (or_cell), so covering decisions stay sound.  A cell (i, j) is        */
/* identified by its Morton code over b bits per axis, b the smallest   */
/* with 2^b >= s (the paper numbers the grid cells by Morton codes).    */
/* ------------------------------------------------------------------ */

uint32_t or_ug_col(uint32_t fine, uint32_t s) {
  return (uint32_t)(((uint64_t)fine * s) >> OR_L);
}

uint32_t or_ug_bits(uint32_t s) {
  uint32_t b = 0;
  while ((1u << b) < s) ++b;
  return b;
}

/* Grid cell (Morton code) of every object with a position: cell[j]
 * (0xffffffff for objects without one). */
void or_ug_cells(uint32_t N, const float *px, const float *py, const uint8_t *has, float x0,
                 float y0, int32_t e, uint32_t s, uint32_t *cell) {
  uint32_t b = or_ug_bits(s);
  for (uint32_t j = 0; j < N; ++j) {
    if (!has[j]) {
      cell[j] = 0xffffffffu;
      continue;
    }
    uint32_t ci = or_ug_col(or_cell(px[j], x0, e), s);
    uint32_t cj = or_ug_col(or_cell(py[j], y0, e), s);
    cell[j] = or_morton(ci, cj, b);
  }
}

/* Query splitting over the grid (mapping function g): the query's corner
 * columns and rows [c(f(x^a)), c(f(x^b))] x [c(f(y^a)), c(f(y^b))] name
 * every cell it overlaps; a cell strictly inside that range on both axes
 * is covering, any other intersecting.  Plain definition: the nested loop
 * over the range.  Cells with no object (count[z] == 0) are skipped.
 * Pass 1 (out == NULL): counts; pass 2: Morton codes of the cells, in
 * row-then-column order. */
void or_ug_split(uint32_t nq, const uint8_t *live, const float *xa, const float *ya,
                 const float *xb, const float *yb, float x0, float y0, int32_t e, uint32_t s,
                 const uint32_t *count, uint64_t *ni, uint64_t *nc, const uint64_t *oi,
                 const uint64_t *oc, uint32_t *out_i, uint32_t *out_c) {
  uint32_t b = or_ug_bits(s);
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t k = 0; k < (int64_t)nq; ++k) {
    uint64_t ci = 0, cc = 0;
    int ok = live[k] && xa[k] <= xb[k] && ya[k] <= yb[k] && isfinite(xa[k]) &&
             isfinite(xb[k]) && isfinite(ya[k]) && isfinite(yb[k]);
    if (ok) {
      uint32_t i0 = or_ug_col(or_cell(xa[k], x0, e), s), i1 = or_ug_col(or_cell(xb[k], x0, e), s);
      uint32_t j0 = or_ug_col(or_cell(ya[k], y0, e), s), j1 = or_ug_col(or_cell(yb[k], y0, e), s);
      for (uint32_t j = j0; j <= j1; ++j)
        for (uint32_t i = i0; i <= i1; ++i) {
          uint32_t z = or_morton(i, j, b);
          if (count[z] == 0) continue;
          int cov = i0 < i && i < i1 && j0 < j && j < j1;
          if (cov) {
            if (out_c) out_c[oc[k] + cc] = z;
            ++cc;
          } else {
            if (out_i) out_i[oi[k] + ci] = z;
            ++ci;
          }
        }
    }
    if (ni) ni[k] = ci;
    if (nc) nc[k] = cc;
  }
}

/* ------------------------------------------------------------------ */
/* Repeated k-nearest-neighbour queries (the paper's stated future      */
/* work, Section "Conclusions"; the paper defines no semantics, so this */
/* is the reading both sides implement).  A query (qid, qx, qy) asks   */
/* for the k present objects with the smallest key (d2, id), where      */
/*   dx = fl32(px - qx), dy = fl32(py - qy),                             */
/*   d2 = fl32(fl32(dx * dx) + fl32(dy * dy)),                           */
/* evaluated in exactly that order in binary32 (no contraction), ties  */
/* broken by the smaller id.  Results are in ascending key order; a     */
/* query with fewer than k present objects gets all of them, the rest   */
/* of its k slots hold id 0xffffffff and d2 = +inf.  A query superseded */
/* by a later query of the same object in the tick is answered with    */
/* all slots empty (as a superseded range query has an empty result).  */
/* Brute force: every present object is scored, and a sorted list of    */
/* the k best keys so far is kept by insertion.                          */
/* ------------------------------------------------------------------ */

static inline float or_d2(float px, float py, float qx, float qy) {
  volatile float dx = px - qx, dy = py - qy;
  volatile float xx = dx * dx, yy = dy * dy;
  return xx + yy;
}

/* key = (binary32 bits of d2) << 32 | id; d2 >= +0, so the bit pattern   */
/* orders like the value.                                                 */
static inline uint64_t or_knn_key(float d2, uint32_t id) {
  uint32_t b;
  memcpy(&b, &d2, 4);
  return ((uint64_t)b << 32) | id;
}

void or_knn(uint32_t N, const float *px, const float *py, const uint8_t *has,
            uint32_t nq, const uint8_t *live, const float *qx, const float *qy,
            uint32_t k, uint32_t *out_id, float *out_d2) {
  if (k == 0) return;
#pragma omp parallel
  {
    uint64_t *best = (uint64_t *)malloc(sizeof(uint64_t) * k);
#pragma omp for schedule(dynamic, 4)
    for (int64_t q = 0; q < (int64_t)nq; ++q) {
      uint32_t nb = 0;
      if (live[q]) {
        for (uint32_t j = 0; j < N; ++j) {
          if (!has[j]) continue;
          const uint64_t key = or_knn_key(or_d2(px[j], py[j], qx[q], qy[q]), j);
          if (nb == k && key >= best[k - 1]) continue;
          uint32_t p = nb < k ? nb++ : k - 1;
          while (p > 0 && best[p - 1] > key) {
            best[p] = best[p - 1];
            --p;
          }
          best[p] = key;
        }
      }
      for (uint32_t i = 0; i < k; ++i) {
        if (i < nb) {
          const uint32_t b = (uint32_t)(best[i] >> 32);
          out_id[(uint64_t)q * k + i] = (uint32_t)best[i];
          memcpy(&out_d2[(uint64_t)q * k + i], &b, 4);
        } else {
          out_id[(uint64_t)q * k + i] = 0xffffffffu;
          out_d2[(uint64_t)q * k + i] = INFINITY;
        }
      }
    }
    free(best);
  }
}

/* The binary32 squared distance of the definition above, one pair. */
float or_knn_d2(float px, float py, float qx, float qy) { return or_d2(px, py, qx, qy); }
