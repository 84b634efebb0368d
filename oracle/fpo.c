/*
 * fpo.c -- plain serial CPU oracle of the patch-guided nested-dissection
 * ordering.  TEST INFRASTRUCTURE ONLY (see fpo.h): it defines the exact
 * result of the ordering; the GPU library shares nothing with it.
 *
 * Every decision below depends only on vertex ids, patch ids and integer
 * counts (never on CSR entry order), so the result is a function of the
 * pattern, the options and the seed.
 */
#include "fpo.h"

#include <stdlib.h>
#include <string.h>

#define NEW(T, k) ((T*)malloc(((size_t)(k) > 0 ? (size_t)(k) : 1) * sizeof(T)))
#define NEWZ(T, k) ((T*)calloc(((size_t)(k) > 0 ? (size_t)(k) : 1), sizeof(T)))

static int cmp_i32(const void* a, const void* b) {
  int32_t x = *(const int32_t*)a, y = *(const int32_t*)b;
  return (x > y) - (x < y);
}
static int cmp_i64(const void* a, const void* b) {
  int64_t x = *(const int64_t*)a, y = *(const int64_t*)b;
  return (x > y) - (x < y);
}

/* SplitMix64 (Steele, Lea, Flood, OOPSLA 2014): golden-ratio increment and
 * the variant-13 finaliser. */
uint64_t fpo_mix64(uint64_t seed, uint64_t i) {
  uint64_t z = seed + (i + 1) * 0x9E3779B97F4A7C15ULL;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

/* ------------------------------------------------------------------ */
/* O0: graph of A without its diagonal (Sec. 2; Sec. 4.1 Step 2).     */
/* Vertex k gathers the columns of DOF rows b*k..b*k+b-1 divided by b. */
/* ------------------------------------------------------------------ */

static int check_csr(int64_t n_dof, const int64_t* rowptr) {
  if (n_dof < 0 || !rowptr) return FPO_ERR_ARG;
  if (rowptr[0] != 0) return FPO_ERR_ARG;
  for (int64_t i = 0; i < n_dof; i++)
    if (rowptr[i + 1] < rowptr[i]) return FPO_ERR_ARG;
  return FPO_OK;
}

static int64_t gather_row(int64_t k, int32_t b, int64_t n_dof, const int64_t* rowptr,
                          const int32_t* colind, int32_t* buf, int* err) {
  int64_t len = 0;
  for (int64_t r = k * b; r < (k + 1) * b; r++)
    for (int64_t e = rowptr[r]; e < rowptr[r + 1]; e++) {
      int32_t c = colind[e];
      if (c < 0 || c >= n_dof) {
        *err = FPO_ERR_INDEX;
        return 0;
      }
      int32_t v = c / b;
      if (v != k) buf[len++] = v;
    }
  qsort(buf, (size_t)len, sizeof(int32_t), cmp_i32);
  int64_t u = 0;
  for (int64_t i = 0; i < len; i++)
    if (u == 0 || buf[u - 1] != buf[i]) buf[u++] = buf[i];
  return u;
}

static int64_t max_vertex_row(int64_t n_v, int32_t b, const int64_t* rowptr) {
  int64_t mx = 0;
  for (int64_t k = 0; k < n_v; k++) {
    int64_t l = rowptr[(k + 1) * b] - rowptr[k * b];
    if (l > mx) mx = l;
  }
  return mx;
}

int fpo_graph_count(int64_t n_dof, const int64_t* rowptr, const int32_t* colind,
                    int32_t b, int64_t* nnz_g) {
  if (b < 1 || n_dof % b) return FPO_ERR_ARG;
  int rc = check_csr(n_dof, rowptr);
  if (rc) return rc;
  int64_t n_v = n_dof / b;
  int32_t* buf = NEW(int32_t, max_vertex_row(n_v, b, rowptr));
  if (!buf) return FPO_ERR_OOM;
  int err = 0;
  int64_t tot = 0;
  for (int64_t k = 0; k < n_v && !err; k++) tot += gather_row(k, b, n_dof, rowptr, colind, buf, &err);
  free(buf);
  if (err) return err;
  *nnz_g = tot;
  return FPO_OK;
}

int fpo_graph_fill(int64_t n_dof, const int64_t* rowptr, const int32_t* colind,
                   int32_t b, int64_t* g_rowptr, int32_t* g_colind) {
  if (b < 1 || n_dof % b) return FPO_ERR_ARG;
  int rc = check_csr(n_dof, rowptr);
  if (rc) return rc;
  int64_t n_v = n_dof / b;
  int32_t* buf = NEW(int32_t, max_vertex_row(n_v, b, rowptr));
  if (!buf) return FPO_ERR_OOM;
  int err = 0;
  g_rowptr[0] = 0;
  for (int64_t k = 0; k < n_v && !err; k++) {
    int64_t l = gather_row(k, b, n_dof, rowptr, colind, buf, &err);
    memcpy(g_colind + g_rowptr[k], buf, (size_t)l * sizeof(int32_t));
    g_rowptr[k + 1] = g_rowptr[k] + l;
  }
  free(buf);
  return err;
}

/* ------------------------------------------------------------------ */
/* O1: patches (Sec. 4.1 Step 1; Lloyd's algorithm with target size S, */
/* Sec. 6).                                                            */
/* ------------------------------------------------------------------ */

int64_t fpo_grow(int32_t n, const int64_t* rp, const int32_t* ci, int32_t nseeds,
                 const int32_t* seeds, int32_t* label) {
  int32_t* front = NEW(int32_t, n);
  int32_t* next = NEW(int32_t, n);
  int32_t* cand = NEW(int32_t, n);
  for (int32_t v = 0; v < n; v++) {
    label[v] = -1;
    cand[v] = -1;
  }
  int64_t nf = 0;
  for (int32_t k = 0; k < nseeds; k++) {
    int32_t s = seeds[k];
    if (label[s] == -1) {
      label[s] = k;
      front[nf++] = s;
    } else if (k < label[s]) {
      label[s] = k;
    }
  }
  /* level by level: a vertex first reached from level l takes the smallest
   * label among its neighbours on level l */
  while (nf > 0) {
    int64_t nn = 0;
    for (int64_t f = 0; f < nf; f++) {
      int32_t v = front[f];
      for (int64_t e = rp[v]; e < rp[v + 1]; e++) {
        int32_t u = ci[e];
        if (label[u] != -1) continue;
        if (cand[u] == -1) {
          next[nn++] = u;
          cand[u] = label[v];
        } else if (label[v] < cand[u]) {
          cand[u] = label[v];
        }
      }
    }
    for (int64_t f = 0; f < nn; f++) {
      label[next[f]] = cand[next[f]];
      cand[next[f]] = -1;
    }
    int32_t* t = front;
    front = next;
    next = t;
    nf = nn;
  }
  int64_t un = 0;
  for (int32_t v = 0; v < n; v++) un += (label[v] == -1);
  free(front);
  free(next);
  free(cand);
  return un;
}

int fpo_patches(int32_t n, const int64_t* rp, const int32_t* ci, int32_t S,
                int32_t lloyd_iters, uint64_t seed, int32_t* gmap, int32_t* seeds_out) {
  if (S < 1 || n < 0 || lloyd_iters < 0) return FPO_ERR_ARG;
  if (n == 0) return 0;
  int32_t P0 = (int32_t)(((int64_t)n + S - 1) / S);
  int32_t* seeds = NEW(int32_t, n);
  /* one seed per block of S consecutive ids: smallest (hash, id) */
  for (int32_t b = 0; b < P0; b++) {
    int64_t lo = (int64_t)b * S, hi = lo + S < n ? lo + S : n;
    int32_t best = (int32_t)lo;
    uint64_t bk = fpo_mix64(seed, (uint64_t)lo);
    for (int64_t v = lo + 1; v < hi; v++) {
      uint64_t k = fpo_mix64(seed, (uint64_t)v);
      if (k < bk) {
        bk = k;
        best = (int32_t)v;
      }
    }
    seeds[b] = best;
  }
  int32_t P = P0;
  fpo_grow(n, rp, ci, P, seeds, gmap);
  /* components without a seed: the lowest unlabelled id seeds a new patch
   * that grows over its whole component */
  int32_t* queue = NEW(int32_t, n);
  for (int32_t v = 0; v < n; v++) {
    if (gmap[v] != -1) continue;
    seeds[P] = v;
    gmap[v] = P;
    int64_t qh = 0, qt = 0;
    queue[qt++] = v;
    while (qh < qt) {
      int32_t x = queue[qh++];
      for (int64_t e = rp[x]; e < rp[x + 1]; e++)
        if (gmap[ci[e]] == -1) {
          gmap[ci[e]] = P;
          queue[qt++] = ci[e];
        }
    }
    P++;
  }
  /* Lloyd: new seed = vertex farthest (in intra-patch hops) from the patch
   * boundary, ties to the lowest id; then regrow with the same ids */
  int32_t* dist = NEW(int32_t, n);
  int32_t* best = NEW(int32_t, P);
  uint8_t* hasb = NEW(uint8_t, P);
  for (int32_t it = 0; it < lloyd_iters; it++) {
    int64_t qh = 0, qt = 0;
    for (int32_t k = 0; k < P; k++) {
      hasb[k] = 0;
      best[k] = -1;
    }
    for (int32_t v = 0; v < n; v++) {
      dist[v] = -1;
      for (int64_t e = rp[v]; e < rp[v + 1]; e++)
        if (gmap[ci[e]] != gmap[v]) {
          dist[v] = 0;
          break;
        }
      if (dist[v] == 0) {
        queue[qt++] = v;
        hasb[gmap[v]] = 1;
      }
    }
    while (qh < qt) {
      int32_t x = queue[qh++];
      for (int64_t e = rp[x]; e < rp[x + 1]; e++) {
        int32_t u = ci[e];
        if (gmap[u] == gmap[x] && dist[u] == -1) {
          dist[u] = dist[x] + 1;
          queue[qt++] = u;
        }
      }
    }
    for (int32_t v = 0; v < n; v++) {
      int32_t k = gmap[v];
      if (!hasb[k]) continue;
      if (best[k] == -1 || dist[v] > dist[best[k]]) best[k] = v;
    }
    for (int32_t k = 0; k < P; k++)
      if (hasb[k]) seeds[k] = best[k];
    fpo_grow(n, rp, ci, P, seeds, gmap);
  }
  if (seeds_out) memcpy(seeds_out, seeds, (size_t)P * sizeof(int32_t));
  free(dist);
  free(best);
  free(hasb);
  free(queue);
  free(seeds);
  return P;
}

/* ------------------------------------------------------------------ */
/* O4: bisection of a quotient subgraph (Alg. 2 BiPartition).          */
/* BFS level structure from a pseudo-peripheral start (George & Liu,   */
/* 1979), ordered by (level, index), split at the weighted half and    */
/* clamped so that each child holds at most 2^(ceil(log2 m) - 1) nodes. */
/* ------------------------------------------------------------------ */

/* BFS from src; lev[] must be -1 on src's component.  Visit order goes to
 * queue; returns the number reached, eccentricity in *ecc. */
static int32_t bfs_local(const int64_t* arp, const int32_t* aci, int32_t src,
                         int32_t* lev, int32_t* queue, int32_t* ecc) {
  int32_t qh = 0, qt = 0;
  lev[src] = 0;
  queue[qt++] = src;
  int32_t e_max = 0;
  while (qh < qt) {
    int32_t x = queue[qh++];
    if (lev[x] > e_max) e_max = lev[x];
    for (int64_t e = arp[x]; e < arp[x + 1]; e++) {
      int32_t y = aci[e];
      if (lev[y] == -1) {
        lev[y] = lev[x] + 1;
        queue[qt++] = y;
      }
    }
  }
  *ecc = e_max;
  return qt;
}


int fpo_bisect(int32_t m, const int64_t* w, const int64_t* arp, const int32_t* aci,
               uint8_t* left) {
  if (m < 2) return FPO_ERR_ARG;
  int32_t* levA = NEW(int32_t, m);
  int32_t* levB = NEW(int32_t, m);
  int32_t* qA = NEW(int32_t, m);
  int32_t* qB = NEW(int32_t, m);
  uint8_t* seen = NEWZ(uint8_t, m);
  int32_t* Q = NEW(int32_t, m);
  int64_t* keys = NEW(int64_t, m);
  for (int32_t i = 0; i < m; i++) levA[i] = levB[i] = -1;
  int32_t qn = 0;
  for (int32_t r0 = 0; r0 < m; r0++) {
    if (seen[r0]) continue;
    /* components are taken in order of their lowest index */
    int32_t ecc_r, ecc_c;
    int32_t* lr = levA;
    int32_t* lc = levB;
    int32_t* qr = qA;
    int32_t* qc = qB;
    int32_t cnt = bfs_local(arp, aci, r0, lr, qr, &ecc_r);
    for (int round = 0; round < 8; round++) {
      /* candidate: least (degree, index) on the last level */
      int32_t c = -1;
      for (int32_t k = 0; k < cnt; k++) {
        int32_t x = qr[k];
        if (lr[x] != ecc_r) continue;
        int64_t dx = arp[x + 1] - arp[x];
        if (c == -1 || dx < arp[c + 1] - arp[c] || (dx == arp[c + 1] - arp[c] && x < c)) c = x;
      }
      bfs_local(arp, aci, c, lc, qc, &ecc_c);
      if (ecc_c > ecc_r) {
        /* accept: the candidate's level structure becomes current */
        for (int32_t k = 0; k < cnt; k++) lr[qr[k]] = -1;
        int32_t* t = lr;
        lr = lc;
        lc = t;
        t = qr;
        qr = qc;
        qc = t;
        ecc_r = ecc_c;
      } else {
        for (int32_t k = 0; k < cnt; k++) lc[qc[k]] = -1;
        break;
      }
    }
    for (int32_t k = 0; k < cnt; k++) {
      int32_t x = qr[k];
      keys[k] = (int64_t)lr[x] * m + x;
      seen[x] = 1;
    }
    qsort(keys, (size_t)cnt, sizeof(int64_t), cmp_i64);
    for (int32_t k = 0; k < cnt; k++) Q[qn++] = (int32_t)(keys[k] % m);
    for (int32_t k = 0; k < cnt; k++) lr[qr[k]] = -1;
  }
  int64_t W = 0;
  for (int32_t i = 0; i < m; i++) W += w[i];
  int32_t kstar;
  if (W == 0) {
    kstar = (m + 1) / 2;
  } else {
    kstar = m;
    int64_t pre = 0;
    for (int32_t k = 1; k <= m; k++) {
      pre += w[Q[k - 1]];
      if (2 * pre >= W) {
        kstar = k;
        break;
      }
    }
  }
  int32_t h = 0;
  while ((1LL << h) < m) h++;
  int32_t cap = 1 << (h - 1);
  int32_t lo = m - cap > 1 ? m - cap : 1;
  int32_t hi = m - 1 < cap ? m - 1 : cap;
  int32_t k = kstar < lo ? lo : (kstar > hi ? hi : kstar);
  for (int32_t i = 0; i < m; i++) left[i] = 0;
  for (int32_t i = 0; i < k; i++) left[Q[i]] = 1;
  free(levA);
  free(levB);
  free(qA);
  free(qB);
  free(seen);
  free(Q);
  free(keys);
  return FPO_OK;
}

/* ------------------------------------------------------------------ */
/* O2-O6: separator tree (Sec. 4.2 Step 3; Alg. 2; Sec. 5).             */
/* ------------------------------------------------------------------ */

static int64_t arc_index(const int64_t* qrp, const int32_t* qci, int32_t p, int32_t q) {
  int64_t lo = qrp[p], hi = qrp[p + 1];
  while (lo < hi) {
    int64_t mid = (lo + hi) / 2;
    if (qci[mid] < q)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}

/* RefineSeparator, refined reading: the smallest separator inside the
 * superset.  The two sides follow the patches (Alg. 2 induces the left and
 * right subgraphs from the patch bipartition), so a separator of node t is
 * any set of candidates that touches every crossing edge (an unmarked left
 * vertex joined to an unmarked right vertex): a vertex cover of the
 * bipartite crossing graph.  Its minimum is the size of a maximum matching
 * (Konig 1931).  Among the minimum covers the one taken is the refinement
 * of the one-sided separator: start from side s (the side the one-sided
 * rule marks), let Z be the vertices reachable from the s-vertices that the
 * matching leaves free along alternating paths (non-matching edges from s
 * to the other side, matching edges back); the cover is (s-side candidates
 * outside Z) plus (other-side candidates inside Z).  Z does not depend on
 * which maximum matching is found (Dulmage and Mendelsohn 1958: its s-side
 * part is the set of s-vertices that some maximum matching leaves free), so
 * the result is unique.  The matching is grown by augmenting paths found by
 * breadth-first search from every s-vertex in ascending id (Kuhn 1955). */
static int on_side(const int32_t* node_of, const int32_t* gmap, const int32_t* newnode,
                   int32_t u, int32_t child) {
  return node_of[u] == -1 && newnode[gmap[u]] == child;
}

static void refine_node(const int64_t* rp, const int32_t* ci, const int32_t* gmap,
                        const int32_t* node_of, const int32_t* newnode, int32_t t, int32_t s_child,
                        const int32_t* cv, int32_t ncv, int32_t* mate, int32_t* par,
                        int32_t* seen, int32_t* stamp, int32_t* queue, uint8_t* sep) {
  const int32_t o_child = (s_child & 1) ? s_child + 1 : s_child - 1;
  (void)t;
  for (int32_t i = 0; i < ncv; i++) mate[cv[i]] = -1;
  /* maximum matching: one augmenting-path search per s-vertex */
  for (int32_t i = 0; i < ncv; i++) {
    int32_t r = cv[i];
    if (newnode[gmap[r]] != s_child) continue;
    int32_t st = ++*stamp, qh = 0, qt = 0, found = -1;
    queue[qt++] = r;
    while (qh < qt && found < 0) {
      int32_t x = queue[qh++];
      for (int64_t e = rp[x]; e < rp[x + 1] && found < 0; e++) {
        int32_t u = ci[e];
        if (!on_side(node_of, gmap, newnode, u, o_child) || seen[u] == st) continue;
        seen[u] = st;
        par[u] = x;
        if (mate[u] == -1)
          found = u;
        else
          queue[qt++] = mate[u];
      }
    }
    /* flip the path: every other-side vertex on it takes its predecessor */
    for (int32_t u = found; u >= 0;) {
      int32_t x = par[u], next = mate[x];
      mate[x] = u;
      mate[u] = x;
      u = next;
    }
  }
  /* Z: alternating reachability from the free s-vertices */
  int32_t st = ++*stamp, qh = 0, qt = 0;
  for (int32_t i = 0; i < ncv; i++) {
    int32_t r = cv[i];
    if (newnode[gmap[r]] == s_child && mate[r] == -1) {
      seen[r] = st;
      queue[qt++] = r;
    }
  }
  while (qh < qt) {
    int32_t x = queue[qh++];
    for (int64_t e = rp[x]; e < rp[x + 1]; e++) {
      int32_t u = ci[e];
      if (!on_side(node_of, gmap, newnode, u, o_child) || seen[u] == st || mate[x] == u) continue;
      seen[u] = st;
      /* u is matched: a free u would end an augmenting path */
      int32_t y = mate[u];
      if (y >= 0 && seen[y] != st) {
        seen[y] = st;
        queue[qt++] = y;
      }
    }
  }
  for (int32_t i = 0; i < ncv; i++) {
    int32_t v = cv[i];
    int32_t in_z = seen[v] == st;
    sep[v] = newnode[gmap[v]] == s_child ? !in_z : in_z;
  }
}

int fpo_septree(int32_t n, const int64_t* rp, const int32_t* ci, int32_t P,
                const int32_t* gmap, int32_t nd_level, int32_t refine, int32_t* node_of,
                int32_t* pnode, int32_t* depth_out) {
  if (n < 0 || P < 0 || (n > 0 && P < 1) || nd_level < -1) return FPO_ERR_ARG;
  for (int32_t v = 0; v < n; v++)
    if (gmap[v] < 0 || gmap[v] >= P) return FPO_ERR_INDEX;
  int32_t D = 0;
  while ((1LL << D) < P) D++;
  if (D > 24) return FPO_ERR_SIZE;
  /* Sec. 4.2 Step 3: the recursion stops after nd_level levels; a leaf
   * then keeps the remaining vertices of all its patches */
  if (nd_level >= 0 && nd_level < D) D = nd_level;
  int32_t nn = (1 << (D + 1)) - 1;
  *depth_out = D;
  for (int32_t v = 0; v < n; v++) node_of[v] = -1;
  for (int32_t p = 0; p < P; p++) pnode[p] = 0;
  if (D == 0) {
    for (int32_t v = 0; v < n; v++) node_of[v] = 0;
    return FPO_OK;
  }

  /* quotient graph q (Sec. 2: nodes are patches, arcs join adjacent
   * patches), built once; its weights are recounted after every level */
  int64_t npair = 0;
  for (int32_t v = 0; v < n; v++)
    for (int64_t e = rp[v]; e < rp[v + 1]; e++)
      if (gmap[ci[e]] != gmap[v]) npair++;
  int64_t* pk = NEW(int64_t, npair);
  npair = 0;
  for (int32_t v = 0; v < n; v++)
    for (int64_t e = rp[v]; e < rp[v + 1]; e++)
      if (gmap[ci[e]] != gmap[v]) pk[npair++] = (int64_t)gmap[v] * P + gmap[ci[e]];
  qsort(pk, (size_t)npair, sizeof(int64_t), cmp_i64);
  int64_t na = 0;
  for (int64_t i = 0; i < npair; i++)
    if (na == 0 || pk[na - 1] != pk[i]) pk[na++] = pk[i];
  int64_t* qrp = NEWZ(int64_t, (int64_t)P + 1);
  int32_t* qci = NEW(int32_t, na);
  for (int64_t a = 0; a < na; a++) {
    qrp[pk[a] / P + 1]++;
    qci[a] = (int32_t)(pk[a] % P);
  }
  for (int32_t p = 0; p < P; p++) qrp[p + 1] += qrp[p];
  free(pk);

  int64_t* cnt = NEW(int64_t, na);     /* crossing edges between unmarked vertices */
  int64_t* w = NEW(int64_t, P);        /* unmarked vertices per patch */
  int32_t* newnode = NEW(int32_t, P);
  uint8_t* bis = NEWZ(uint8_t, nn);
  int64_t* cL = NEWZ(int64_t, nn);
  int64_t* cR = NEWZ(int64_t, nn);
  uint8_t* cand = NEW(uint8_t, n);
  int32_t* plist = NEW(int32_t, P);
  int32_t* pstart = NEW(int32_t, nn + 1);
  int32_t* loc = NEW(int32_t, P);
  int64_t* larp = NEW(int64_t, (int64_t)P + 1);
  int32_t* laci = NEW(int32_t, na);
  int64_t* lw = NEW(int64_t, P);
  uint8_t* lft = NEW(uint8_t, P);
  /* refinement scratch */
  int32_t* mate = NEW(int32_t, n);
  int32_t* par = NEW(int32_t, n);
  int32_t* seen = NEW(int32_t, n);
  int32_t* queue = NEW(int32_t, n);
  int32_t* cv = NEW(int32_t, n);
  int32_t* cstart = NEW(int32_t, nn + 1);
  uint8_t* sep = NEWZ(uint8_t, n);
  int32_t stamp = 0;
  for (int32_t v = 0; v < n; v++) seen[v] = 0;

  for (int32_t d = 0; d < D; d++) {
    /* weights as of the end of the previous level (Sec. 5: the separator
     * vertices are removed from node and edge weights) */
    for (int32_t p = 0; p < P; p++) w[p] = 0;
    for (int64_t a = 0; a < na; a++) cnt[a] = 0;
    for (int32_t v = 0; v < n; v++) {
      if (node_of[v] != -1) continue;
      w[gmap[v]]++;
      for (int64_t e = rp[v]; e < rp[v + 1]; e++) {
        int32_t u = ci[e];
        if (node_of[u] == -1 && gmap[u] != gmap[v]) cnt[arc_index(qrp, qci, gmap[v], gmap[u])]++;
      }
    }
    int32_t lo = (1 << d) - 1, hi = (1 << (d + 1)) - 1;
    /* patches of each depth-d node, ascending id */
    for (int32_t t = lo; t <= hi; t++) pstart[t] = 0;
    for (int32_t p = 0; p < P; p++)
      if (pnode[p] >= lo && pnode[p] < hi) pstart[pnode[p] + 1]++;
    pstart[lo] = 0;
    for (int32_t t = lo; t < hi; t++) pstart[t + 1] += pstart[t];
    {
      int32_t* fill = NEW(int32_t, hi - lo);
      for (int32_t t = lo; t < hi; t++) fill[t - lo] = pstart[t];
      for (int32_t p = 0; p < P; p++)
        if (pnode[p] >= lo && pnode[p] < hi) plist[fill[pnode[p] - lo]++] = p;
      free(fill);
    }
    for (int32_t p = 0; p < P; p++) newnode[p] = pnode[p];
    for (int32_t t = lo; t < hi; t++) {
      bis[t] = 0;
      int32_t m = pstart[t + 1] - pstart[t];
      if (m < 2) continue;
      const int32_t* pl = plist + pstart[t];
      for (int32_t i = 0; i < m; i++) loc[pl[i]] = i;
      /* sub-quotient graph: alive arcs among the node's patches */
      larp[0] = 0;
      for (int32_t i = 0; i < m; i++) {
        int32_t p = pl[i];
        int64_t k = larp[i];
        for (int64_t a = qrp[p]; a < qrp[p + 1]; a++)
          if (cnt[a] > 0 && pnode[qci[a]] == t) laci[k++] = loc[qci[a]];
        larp[i + 1] = k;
        lw[i] = w[p];
      }
      fpo_bisect(m, lw, larp, laci, lft);
      for (int32_t i = 0; i < m; i++) newnode[pl[i]] = lft[i] ? 2 * t + 1 : 2 * t + 2;
      bis[t] = 1;
      cL[t] = cR[t] = 0;
    }
    /* SuperSeparator: unmarked vertices of one side with an unmarked
     * neighbour on the other side.  RefineSeparator: keep the smaller of
     * the two candidate sets (ties to the left). */
    for (int32_t v = 0; v < n; v++) {
      cand[v] = 0;
      if (node_of[v] != -1) continue;
      int32_t t = pnode[gmap[v]];
      if (t < lo || !bis[t]) continue;
      int32_t c = newnode[gmap[v]];
      int32_t sib = (c & 1) ? c + 1 : c - 1;
      for (int64_t e = rp[v]; e < rp[v + 1]; e++) {
        int32_t u = ci[e];
        if (node_of[u] == -1 && newnode[gmap[u]] == sib) {
          cand[v] = 1;
          break;
        }
      }
      if (cand[v]) {
        if (c & 1)
          cL[t]++;
        else
          cR[t]++;
      }
    }
    if (!refine) {
      for (int32_t v = 0; v < n; v++) {
        if (!cand[v]) continue;
        int32_t t = pnode[gmap[v]];
        int32_t is_left = newnode[gmap[v]] & 1;
        int32_t mark_left = cL[t] <= cR[t];
        if (is_left == mark_left) node_of[v] = t;
      }
    } else {
      /* candidates of each node, ascending id; every node refined before
       * any vertex of this level is marked */
      for (int32_t t = lo; t <= hi; t++) cstart[t] = 0;
      for (int32_t v = 0; v < n; v++)
        if (cand[v]) cstart[pnode[gmap[v]] + 1]++;
      cstart[lo] = 0;
      for (int32_t t = lo; t < hi; t++) cstart[t + 1] += cstart[t];
      {
        int32_t* fill = NEW(int32_t, hi - lo);
        for (int32_t t = lo; t < hi; t++) fill[t - lo] = cstart[t];
        for (int32_t v = 0; v < n; v++)
          if (cand[v]) cv[fill[pnode[gmap[v]] - lo]++] = v;
        free(fill);
      }
      for (int32_t t = lo; t < hi; t++) {
        if (!bis[t] || cstart[t + 1] == cstart[t]) continue;
        int32_t s_child = cL[t] <= cR[t] ? 2 * t + 1 : 2 * t + 2;
        refine_node(rp, ci, gmap, node_of, newnode, t, s_child, cv + cstart[t],
                    cstart[t + 1] - cstart[t], mate, par, seen, &stamp, queue, sep);
      }
      for (int32_t t = lo; t < hi; t++)
        for (int32_t k = cstart[t]; k < cstart[t + 1]; k++)
          if (sep[cv[k]]) node_of[cv[k]] = t;
    }
    for (int32_t p = 0; p < P; p++) pnode[p] = newnode[p];
  }
  /* leaves keep the remaining vertices of their patch */
  for (int32_t v = 0; v < n; v++)
    if (node_of[v] == -1) node_of[v] = pnode[gmap[v]];

  free(qrp);
  free(qci);
  free(cnt);
  free(w);
  free(newnode);
  free(bis);
  free(cL);
  free(cR);
  free(cand);
  free(plist);
  free(pstart);
  free(loc);
  free(larp);
  free(laci);
  free(lw);
  free(lft);
  free(mate);
  free(par);
  free(seen);
  free(queue);
  free(cv);
  free(cstart);
  free(sep);
  return FPO_OK;
}

/* ------------------------------------------------------------------ */
/* O7: exact minimum degree (Sec. 4.3 Step 4 LocalOrder; the textbook   */
/* scheme of Tinney and Walker, one vertex per step).                  */
/* ------------------------------------------------------------------ */

static int popc64(uint64_t x) { return __builtin_popcountll(x); }

int fpo_md(int32_t m, const int64_t* rp, const int32_t* ci, int32_t* order) {
  if (m < 0) return FPO_ERR_ARG;
  if (m == 0) return FPO_OK;
  if (m > 65535) return FPO_ERR_SIZE;  /* the same node-size limit as the GPU library */
  int64_t W = (m + 63) / 64;
  uint64_t* adj = NEWZ(uint64_t, (int64_t)m * W);
  uint64_t* alive = NEWZ(uint64_t, W);
  uint64_t* nb = NEW(uint64_t, W);
  int32_t* deg = NEW(int32_t, m);
  if (!adj || !alive || !nb || !deg) {
    free(adj);
    free(alive);
    free(nb);
    free(deg);
    return FPO_ERR_OOM;
  }
  for (int32_t i = 0; i < m; i++) {
    alive[i >> 6] |= 1ULL << (i & 63);
    for (int64_t e = rp[i]; e < rp[i + 1]; e++) {
      int32_t j = ci[e];
      if (j == i || j < 0 || j >= m) continue;
      adj[(int64_t)i * W + (j >> 6)] |= 1ULL << (j & 63);
      adj[(int64_t)j * W + (i >> 6)] |= 1ULL << (i & 63);
    }
  }
  for (int32_t i = 0; i < m; i++) {
    int d = 0;
    for (int64_t k = 0; k < W; k++) d += popc64(adj[(int64_t)i * W + k]);
    deg[i] = d;
  }
  for (int32_t step = 0; step < m; step++) {
    int32_t p = -1;
    for (int32_t i = 0; i < m; i++)
      if ((alive[i >> 6] >> (i & 63)) & 1)
        if (p < 0 || deg[i] < deg[p]) p = i;
    order[step] = p;
    alive[p >> 6] &= ~(1ULL << (p & 63));
    for (int64_t k = 0; k < W; k++) nb[k] = adj[(int64_t)p * W + k] & alive[k];
    /* the neighbours of p become a clique; p leaves the graph */
    for (int64_t k = 0; k < W; k++) {
      uint64_t bits = nb[k];
      while (bits) {
        int32_t u = (int32_t)(k * 64 + __builtin_ctzll(bits));
        bits &= bits - 1;
        uint64_t* row = adj + (int64_t)u * W;
        int d = 0;
        for (int64_t j = 0; j < W; j++) {
          row[j] = (row[j] | nb[j]) & alive[j];
          if (j == (u >> 6)) row[j] &= ~(1ULL << (u & 63));
          d += popc64(row[j]);
        }
        deg[u] = d;
      }
    }
  }
  free(adj);
  free(alive);
  free(nb);
  free(deg);
  return FPO_OK;
}

/* ------------------------------------------------------------------ */
/* F3: approximate minimum degree (Sec. 4.3 Step 4 names AMD as the     */
/* local order; Amestoy, Davis and Duff, SIAM J. Matrix Anal. Appl.     */
/* 17(4), 1996).  Elimination on the quotient graph: variable i keeps   */
/* its variable neighbours A_i and its adjacent elements E_i; element e */
/* keeps its variables L_e.  Eliminating pivot p forms the element      */
/* L_p = (A_p + union of L_e over E_p) minus p, absorbs every element of */
/* E_p, and for each i in L_p sets A_i = A_i minus (L_p + p) and         */
/* E_i = (E_i minus E_p) + p.  The degree of i becomes the bound        */
/*   min( r - 1, dbar_i + |L_p \ i|,                                     */
/*        |A_i| + |L_p \ i| + sum over e in E_i \ p of |L_e \ L_p| )     */
/* with r the variables left after the step; |L_e \ L_p| is |L_e| less  */
/* the members of L_p that e touches.  The pivot is the least (dbar,    */
/* index).  Every variable is its own supervariable here: no mass       */
/* elimination and no aggressive absorption, so the order is defined by */
/* the bound alone.  dtrace (nullable, m*m): dtrace[k*m+i] = dbar_i when */
/* the k-th pivot is chosen, -1 once i is eliminated.                    */
/* ------------------------------------------------------------------ */
int fpo_amd(int32_t m, const int64_t* rp, const int32_t* ci, int32_t* order, int32_t* dtrace) {
  if (m < 0) return FPO_ERR_ARG;
  if (m == 0) return FPO_OK;
  if (m > 65535) return FPO_ERR_SIZE;
  /* A_i: distinct neighbours in 0..m-1 without i; E_i shares its row
   * capacity (at most one adjacent element per original neighbour) */
  int64_t* ro = NEW(int64_t, (int64_t)m + 1);
  int32_t* alen = NEW(int32_t, m);
  int32_t* elen = NEW(int32_t, m);
  int32_t* mark = NEW(int32_t, m);
  ro[0] = 0;
  for (int32_t i = 0; i < m; i++) ro[i + 1] = ro[i] + (rp[i + 1] - rp[i]);
  int32_t* arow = NEW(int32_t, ro[m] > 0 ? ro[m] : 1);
  int32_t* erow = NEW(int32_t, ro[m] > 0 ? ro[m] : 1);
  for (int32_t i = 0; i < m; i++) mark[i] = -1;
  for (int32_t i = 0; i < m; i++) {
    alen[i] = 0;
    elen[i] = 0;
    for (int64_t e = rp[i]; e < rp[i + 1]; e++) {
      int32_t j = ci[e];
      if (j == i || j < 0 || j >= m || mark[j] == i) continue;
      mark[j] = i;
      arow[ro[i] + alen[i]++] = j;
    }
  }
  int32_t** L = NEWZ(int32_t*, m); /* element lists, by pivot */
  int32_t* llen = NEWZ(int32_t, m);
  uint8_t* alive = NEW(uint8_t, m);
  int32_t* dbar = NEW(int32_t, m);
  int32_t* w = NEW(int32_t, m);
  int32_t* wst = NEW(int32_t, m);
  int32_t* lp = NEW(int32_t, m);
  for (int32_t i = 0; i < m; i++) {
    alive[i] = 1;
    dbar[i] = alen[i];
    mark[i] = -1;
    wst[i] = -1;
  }
  for (int32_t k = 0; k < m; k++) {
    if (dtrace)
      for (int32_t i = 0; i < m; i++) dtrace[(int64_t)k * m + i] = alive[i] ? dbar[i] : -1;
    int32_t p = -1;
    for (int32_t i = 0; i < m; i++)
      if (alive[i] && (p < 0 || dbar[i] < dbar[p])) p = i;
    order[k] = p;
    alive[p] = 0;
    /* L_p from A_p and the elements of E_p (k is this step's mark) */
    int32_t nl = 0;
    for (int32_t a = 0; a < alen[p]; a++) {
      int32_t v = arow[ro[p] + a];
      if (alive[v] && mark[v] != k) {
        mark[v] = k;
        lp[nl++] = v;
      }
    }
    for (int32_t a = 0; a < elen[p]; a++) {
      int32_t e = erow[ro[p] + a];
      for (int32_t q = 0; q < llen[e]; q++) {
        int32_t v = L[e][q];
        if (alive[v] && mark[v] != k) {
          mark[v] = k;
          lp[nl++] = v;
        }
      }
    }
    /* absorb E_p into p */
    for (int32_t a = 0; a < elen[p]; a++) {
      int32_t e = erow[ro[p] + a];
      free(L[e]);
      L[e] = NULL;
      llen[e] = -1; /* absorbed */
    }
    L[p] = NEW(int32_t, nl > 0 ? nl : 1);
    memcpy(L[p], lp, (size_t)nl * sizeof(int32_t));
    llen[p] = nl;
    /* quotient-graph update of every i in L_p */
    for (int32_t q = 0; q < nl; q++) {
      int32_t i = lp[q];
      int32_t na = 0;
      for (int32_t a = 0; a < alen[i]; a++) {
        int32_t v = arow[ro[i] + a];
        if (v != p && mark[v] != k) arow[ro[i] + na++] = v;
      }
      alen[i] = na;
      int32_t ne = 0;
      for (int32_t a = 0; a < elen[i]; a++) {
        int32_t e = erow[ro[i] + a];
        if (llen[e] >= 0) erow[ro[i] + ne++] = e;
      }
      erow[ro[i] + ne++] = p;
      elen[i] = ne;
    }
    /* |L_e \ L_p| for the other elements next to L_p */
    for (int32_t q = 0; q < nl; q++) {
      int32_t i = lp[q];
      for (int32_t a = 0; a < elen[i]; a++) {
        int32_t e = erow[ro[i] + a];
        if (e == p) continue;
        if (wst[e] != k) {
          wst[e] = k;
          w[e] = llen[e];
        }
        w[e]--;
      }
    }
    /* approximate degrees */
    int32_t r = m - (k + 1);
    for (int32_t q = 0; q < nl; q++) {
      int32_t i = lp[q];
      int64_t ext = 0;
      for (int32_t a = 0; a < elen[i]; a++) {
        int32_t e = erow[ro[i] + a];
        if (e != p) ext += w[e];
      }
      int64_t b1 = r - 1;
      int64_t b2 = (int64_t)dbar[i] + (nl - 1);
      int64_t b3 = (int64_t)alen[i] + (nl - 1) + ext;
      int64_t d = b1 < b2 ? b1 : b2;
      dbar[i] = (int32_t)(d < b3 ? d : b3);
    }
  }
  for (int32_t e = 0; e < m; e++) free(L[e]);
  free(L);
  free(llen);
  free(ro);
  free(alen);
  free(elen);
  free(mark);
  free(arow);
  free(erow);
  free(alive);
  free(dbar);
  free(w);
  free(wst);
  free(lp);
  return FPO_OK;
}

int fpo_brute_md(int32_t m, const int64_t* rp, const int32_t* ci, int32_t* order) {
  if (m < 0 || m > 2048) return FPO_ERR_SIZE;
  uint8_t* a = NEWZ(uint8_t, (int64_t)m * m);
  uint8_t* gone = NEWZ(uint8_t, m);
  for (int32_t i = 0; i < m; i++)
    for (int64_t e = rp[i]; e < rp[i + 1]; e++) {
      int32_t j = ci[e];
      if (j != i && j >= 0 && j < m) a[(int64_t)i * m + j] = a[(int64_t)j * m + i] = 1;
    }
  for (int32_t step = 0; step < m; step++) {
    int32_t best = -1, bd = 0;
    for (int32_t i = 0; i < m; i++) {
      if (gone[i]) continue;
      int32_t d = 0;
      for (int32_t j = 0; j < m; j++) d += (!gone[j] && a[(int64_t)i * m + j]);
      if (best < 0 || d < bd) {
        best = i;
        bd = d;
      }
    }
    order[step] = best;
    gone[best] = 1;
    for (int32_t x = 0; x < m; x++) {
      if (gone[x] || !a[(int64_t)best * m + x]) continue;
      for (int32_t y = 0; y < m; y++)
        if (y != x && !gone[y] && a[(int64_t)best * m + y]) a[(int64_t)x * m + y] = 1;
    }
  }
  free(a);
  free(gone);
  return FPO_OK;
}

/* ------------------------------------------------------------------ */
/* O9, O10: elimination tree and column counts of A(perm,perm).        */
/* ------------------------------------------------------------------ */

int fpo_etree(int32_t n, const int64_t* rp, const int32_t* ci, const int32_t* perm,
              const int32_t* iperm, int32_t* parent) {
  /* Liu's algorithm: row i links the current root of every earlier column
   * it touches to i; ancestors are path-compressed toward i */
  int32_t* anc = NEW(int32_t, n);
  for (int32_t i = 0; i < n; i++) {
    parent[i] = -1;
    anc[i] = -1;
    int32_t v = perm[i];
    for (int64_t e = rp[v]; e < rp[v + 1]; e++) {
      int32_t j = iperm[ci[e]];
      if (j >= i) continue;
      int32_t r = j;
      while (anc[r] != -1 && anc[r] != i) {
        int32_t nx = anc[r];
        anc[r] = i;
        r = nx;
      }
      if (anc[r] == -1) {
        anc[r] = i;
        parent[r] = i;
      }
    }
  }
  free(anc);
  return FPO_OK;
}

int fpo_colcount(int32_t n, const int64_t* rp, const int32_t* ci, const int32_t* perm,
                 const int32_t* iperm, const int32_t* parent, int32_t* colcount,
                 int64_t* nnzL) {
  /* L(i,k) != 0 for k < i exactly on the union of the etree paths from
   * each k with A(i,k) != 0 up to i (the row subtree of i) */
  int32_t* mark = NEW(int32_t, n);
  for (int32_t j = 0; j < n; j++) {
    colcount[j] = 1;
    mark[j] = -1;
  }
  for (int32_t i = 0; i < n; i++) {
    mark[i] = i;
    int32_t v = perm[i];
    for (int64_t e = rp[v]; e < rp[v + 1]; e++) {
      int32_t k = iperm[ci[e]];
      if (k >= i) continue;
      while (mark[k] != i) {
        colcount[k]++;
        mark[k] = i;
        k = parent[k];
      }
    }
  }
  int64_t s = 0;
  for (int32_t j = 0; j < n; j++) s += colcount[j];
  *nnzL = s;
  free(mark);
  return FPO_OK;
}

int fpo_brute_symbolic(int32_t n, const int64_t* rp, const int32_t* ci,
                       const int32_t* perm, int32_t* parent, int32_t* colcount,
                       int64_t* nnzL) {
  if (n < 0 || n > 16384) return FPO_ERR_SIZE;
  int64_t W = (n + 63) / 64;
  uint64_t* M = NEWZ(uint64_t, (int64_t)n * W);
  uint64_t* S = NEW(uint64_t, W);
  int32_t* ip = NEW(int32_t, n);
  for (int32_t i = 0; i < n; i++) ip[perm[i]] = i;
  for (int32_t i = 0; i < n; i++) {
    int32_t v = perm[i];
    for (int64_t e = rp[v]; e < rp[v + 1]; e++) {
      int32_t j = ip[ci[e]];
      if (j == i) continue;
      M[(int64_t)i * W + (j >> 6)] |= 1ULL << (j & 63);
      M[(int64_t)j * W + (i >> 6)] |= 1ULL << (i & 63);
    }
  }
  int64_t tot = 0;
  for (int32_t j = 0; j < n; j++) {
    /* struct(L(:,j)) = entries below the diagonal after eliminating 0..j-1 */
    int cntb = 0;
    int32_t first = -1;
    for (int64_t k = 0; k < W; k++) {
      uint64_t x = M[(int64_t)j * W + k];
      if (k < (j >> 6))
        x = 0;
      else if (k == (j >> 6))
        x &= ((j & 63) == 63) ? 0 : (~0ULL << ((j & 63) + 1));
      S[k] = x;
      cntb += popc64(x);
      if (first < 0 && x) first = (int32_t)(k * 64 + __builtin_ctzll(x));
    }
    colcount[j] = 1 + cntb;
    parent[j] = first;
    tot += colcount[j];
    for (int64_t k = 0; k < W; k++) {
      uint64_t bits = S[k];
      while (bits) {
        int32_t i = (int32_t)(k * 64 + __builtin_ctzll(bits));
        bits &= bits - 1;
        uint64_t* row = M + (int64_t)i * W;
        for (int64_t q = 0; q < W; q++) row[q] |= S[q];
      }
    }
  }
  *nnzL = tot;
  free(M);
  free(S);
  free(ip);
  return FPO_OK;
}

/* ------------------------------------------------------------------ */
/* F1: supernodal symbolic analysis.  The solver that consumes the       */
/* ordering needs the elimination tree for its symbolic analysis         */
/* (Sec. 1); a supernodal factorization groups columns into fundamental  */
/* supernodes (Liu, Ng and Peyton, SIAM J. Matrix Anal. Appl. 14(1),     */
/* 1993): column j+1 continues the supernode of column j exactly when    */
/* j is the only child of j+1 in the elimination tree and the structure  */
/* of column j is that of column j+1 plus j itself, which, given that    */
/* struct(L_j) minus j lies inside struct(L_parent(j)), is               */
/* colcount[j] == colcount[j+1] + 1 with parent[j] == j+1.               */
/* ------------------------------------------------------------------ */

int fpo_supernodes(int32_t n, const int32_t* parent, const int32_t* colcount, int64_t* Lp,
                   int32_t* super_of, int32_t* super_ptr, int32_t* super_parent, int64_t* Lx_ptr,
                   int32_t* n_super) {
  if (n < 0 || !parent || !colcount) return FPO_ERR_ARG;
  /* column pointers of L: column j occupies Lp[j] .. Lp[j+1]-1 */
  if (Lp) {
    Lp[0] = 0;
    for (int32_t j = 0; j < n; j++) Lp[j + 1] = Lp[j] + colcount[j];
  }
  /* number of children of every column in the elimination tree */
  int32_t* nchild = NEWZ(int32_t, n > 0 ? n : 1);
  for (int32_t j = 0; j < n; j++) {
    if (parent[j] < -1 || parent[j] >= n || (parent[j] >= 0 && parent[j] <= j)) {
      free(nchild);
      return FPO_ERR_INDEX;
    }
    if (parent[j] >= 0) nchild[parent[j]]++;
  }
  /* walk the columns: a new supernode starts wherever column j cannot
   * continue the supernode of column j-1 */
  int32_t ns = 0;
  for (int32_t j = 0; j < n; j++) {
    int cont = j > 0 && parent[j - 1] == j && nchild[j] == 1 && colcount[j - 1] == colcount[j] + 1;
    if (!cont) {
      if (super_ptr) super_ptr[ns] = j;
      ns++;
    }
    if (super_of) super_of[j] = ns - 1;
  }
  if (super_ptr) super_ptr[ns] = n;
  /* supernodal elimination tree: the parent of a supernode is the supernode
   * holding the etree parent of its last column */
  if (super_parent && super_ptr && super_of)
    for (int32_t s = 0; s < ns; s++) {
      int32_t last = super_ptr[s + 1] - 1;
      super_parent[s] = parent[last] < 0 ? -1 : super_of[parent[last]];
    }
  /* dense storage of a supernode: its first column's rows times its width */
  if (Lx_ptr && super_ptr) {
    Lx_ptr[0] = 0;
    for (int32_t s = 0; s < ns; s++) {
      int32_t f = super_ptr[s], w = super_ptr[s + 1] - f;
      Lx_ptr[s + 1] = Lx_ptr[s] + (int64_t)colcount[f] * w;
    }
  }
  *n_super = ns;
  free(nchild);
  return FPO_OK;
}

/* ------------------------------------------------------------------ */
/* O8 and the whole pipeline (Alg. 1; Alg. 3; Sec. 5 schedules).        */
/* ------------------------------------------------------------------ */

static void post_order(int32_t t, int32_t nn, int32_t* seq, int32_t* k) {
  if (t >= nn) return;
  post_order(2 * t + 1, nn, seq, k);
  post_order(2 * t + 2, nn, seq, k);
  seq[(*k)++] = t;
}

static int is_symmetric(int32_t n, const int64_t* rp, const int32_t* ci) {
  for (int32_t v = 0; v < n; v++)
    for (int64_t e = rp[v]; e < rp[v + 1]; e++) {
      int32_t u = ci[e];
      int64_t lo = rp[u], hi = rp[u + 1];
      while (lo < hi) {
        int64_t mid = (lo + hi) / 2;
        if (ci[mid] < v)
          lo = mid + 1;
        else
          hi = mid;
      }
      if (lo >= rp[u + 1] || ci[lo] != v) return 0;
    }
  return 1;
}

int fpo_order(int64_t n_dof, const int64_t* rowptr, const int32_t* colind,
              const int32_t* user_gmap, const fpo_opts* opts, fpo_out* out) {
  if (!opts || !out) return FPO_ERR_ARG;
  int32_t b = opts->block_size;
  if (b < 1 || opts->patch_size < 1 || opts->lloyd_iters < 0 || opts->nd_level < -1 ||
      (opts->refine != 0 && opts->refine != 1) || (opts->local_amd != 0 && opts->local_amd != 1))
    return FPO_ERR_ARG;
  if (opts->schedule != FPO_SCHED_LEVEL && opts->schedule != FPO_SCHED_POST) return FPO_ERR_ARG;
  if (n_dof < 0 || n_dof % b || n_dof >= (1LL << 31)) return FPO_ERR_ARG;
  int32_t n = (int32_t)(n_dof / b);
  int rc;
  int64_t nnz_g = 0;
  if ((rc = fpo_graph_count(n_dof, rowptr, colind, b, &nnz_g))) return rc;
  int64_t* rp = NEW(int64_t, (int64_t)n + 1);
  int32_t* ci = NEW(int32_t, nnz_g);
  if ((rc = fpo_graph_fill(n_dof, rowptr, colind, b, rp, ci))) goto done0;
  if (!is_symmetric(n, rp, ci)) {
    rc = FPO_ERR_ARG;
    goto done0;
  }

  int32_t* gmap = NEW(int32_t, n);
  int32_t P;
  if (user_gmap) {
    P = 0;
    for (int32_t v = 0; v < n; v++) {
      if (user_gmap[v] < 0 || user_gmap[v] >= n) {
        rc = FPO_ERR_INDEX;
        free(gmap);
        goto done0;
      }
      gmap[v] = user_gmap[v];
      if (gmap[v] + 1 > P) P = gmap[v] + 1;
    }
  } else {
    P = fpo_patches(n, rp, ci, opts->patch_size, opts->lloyd_iters, opts->seed, gmap, NULL);
    if (P < 0) {
      rc = P;
      free(gmap);
      goto done0;
    }
  }

  int32_t* node_of = NEW(int32_t, n);
  int32_t* pnode = NEW(int32_t, P);
  int32_t D = 0;
  if ((rc = fpo_septree(n, rp, ci, P, gmap, opts->nd_level, opts->refine, node_of, pnode, &D)))
    goto done1;
  int32_t nn = (1 << (D + 1)) - 1;

  /* group the vertices of each node by ascending id */
  int32_t* nstart = NEWZ(int32_t, nn + 1);
  int32_t* nvtx = NEW(int32_t, n);
  for (int32_t v = 0; v < n; v++) nstart[node_of[v] + 1]++;
  for (int32_t t = 0; t < nn; t++) nstart[t + 1] += nstart[t];
  {
    int32_t* fill = NEW(int32_t, nn);
    memcpy(fill, nstart, (size_t)nn * sizeof(int32_t));
    for (int32_t v = 0; v < n; v++) nvtx[fill[node_of[v]]++] = v;
    free(fill);
  }
  /* Alg. 3 step 1: local order of every node on its induced subgraph */
  int32_t* lorder = NEW(int32_t, n);
  int32_t* loc = NEW(int32_t, n);
  int32_t* lord = NEW(int32_t, n);
  int64_t* lrp = NEW(int64_t, (int64_t)n + 1);
  int32_t* lci = NEW(int32_t, nnz_g);
  for (int32_t t = 0; t < nn && !rc; t++) {
    int32_t m = nstart[t + 1] - nstart[t];
    if (m == 0) continue;
    const int32_t* V = nvtx + nstart[t];
    for (int32_t i = 0; i < m; i++) loc[V[i]] = i;
    lrp[0] = 0;
    for (int32_t i = 0; i < m; i++) {
      int64_t k = lrp[i];
      for (int64_t e = rp[V[i]]; e < rp[V[i] + 1]; e++)
        if (node_of[ci[e]] == t) lci[k++] = loc[ci[e]];
      lrp[i + 1] = k;
    }
    rc = opts->local_amd ? fpo_amd(m, lrp, lci, lord, NULL) : fpo_md(m, lrp, lci, lord);
    for (int32_t k = 0; k < m; k++) lorder[nstart[t] + k] = V[lord[k]];
  }
  if (rc) goto done2;

  /* Alg. 3 step 2: concatenate along the schedule; every child precedes
   * its parent in both schedules */
  int32_t* seq = NEW(int32_t, nn);
  int32_t ns = 0;
  if (opts->schedule == FPO_SCHED_LEVEL) {
    for (int32_t d = D; d >= 0; d--)
      for (int32_t t = (1 << d) - 1; t < (1 << (d + 1)) - 1; t++) seq[ns++] = t;
  } else {
    post_order(0, nn, seq, &ns);
  }
  int32_t* vperm = NEW(int32_t, n);
  int32_t* viperm = NEW(int32_t, n);
  int32_t* vbeg = NEW(int32_t, nn);
  int32_t pos = 0;
  for (int32_t s = 0; s < ns; s++) {
    int32_t t = seq[s];
    vbeg[t] = pos;
    for (int32_t k = nstart[t]; k < nstart[t + 1]; k++) vperm[pos++] = lorder[k];
  }
  for (int32_t i = 0; i < n; i++) viperm[vperm[i]] = i;

  int32_t* vpar = NEW(int32_t, n);
  int32_t* vcc = NEW(int32_t, n);
  int64_t vnnz = 0;
  fpo_etree(n, rp, ci, vperm, viperm, vpar);
  fpo_colcount(n, rp, ci, vperm, viperm, vpar, vcc, &vnnz);

  /* block expansion (Sec. 6.5): DOFs of a vertex stay consecutive */
  for (int32_t k = 0; k < n; k++)
    for (int32_t r = 0; r < b; r++) {
      int64_t j = (int64_t)k * b + r;
      out->perm[j] = vperm[k] * b + r;
      out->iperm[j] = viperm[k] * b + r;
      out->colcount[j] = b * vcc[k] - r;
      if (r < b - 1)
        out->parent[j] = (int32_t)(j + 1);
      else
        out->parent[j] = vpar[k] < 0 ? -1 : vpar[k] * b;
    }
  out->nnzL = (int64_t)b * b * vnnz - (int64_t)n * b * (b - 1) / 2;
  if (out->gmap) memcpy(out->gmap, gmap, (size_t)n * sizeof(int32_t));
  if (out->node_of) memcpy(out->node_of, node_of, (size_t)n * sizeof(int32_t));
  if (out->node_begin || out->node_size) {
    if (out->max_nodes < nn) {
      rc = FPO_ERR_SIZE;
    } else {
      for (int32_t t = 0; t < nn; t++) {
        if (out->node_begin) out->node_begin[t] = vbeg[t] * b;
        if (out->node_size) out->node_size[t] = (nstart[t + 1] - nstart[t]) * b;
      }
    }
  }
  out->n_patches = P;
  out->depth = D;
  out->n_nodes = nn;

  free(seq);
  free(vperm);
  free(viperm);
  free(vbeg);
  free(vpar);
  free(vcc);
done2:
  free(nstart);
  free(nvtx);
  free(lorder);
  free(loc);
  free(lord);
  free(lrp);
  free(lci);
done1:
  free(node_of);
  free(pnode);
  free(gmap);
done0:
  free(rp);
  free(ci);
  return rc;
}
