/*
 * fpo.h -- plain serial CPU oracle of the patch-guided nested-dissection
 * ordering (Zarebavani, Mahmoud et al., "Fast Sparse Matrix Permutation for
 * Mesh-Based Direct Solvers").
 *
 * TEST INFRASTRUCTURE ONLY.  This library defines the exact result that the
 * GPU path must reproduce; only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load it.  It shares no code, header,
 * table or helper with the GPU library.
 *
 * All arrays are host memory owned by the caller unless stated otherwise.
 * Graphs are CSR with int64 row pointers and int32 column indices.  Every
 * function returns FPO_OK (0) or a negative FPO_ERR_* code.
 *
 * Pins (checked by the CPU tests, not by re-typing the code):
 *   fpo_etree / fpo_colcount   -- dense symbolic elimination (fpo_brute_symbolic)
 *   fpo_md                     -- dense minimum degree (fpo_brute_md) + hand cases
 *   fpo_patches                -- nearest-seed definition by all-source BFS,
 *                                 connectivity, coverage
 *   fpo_bisect                 -- all-pairs-distance re-derivation of the
 *                                 pseudo-peripheral rule and the split
 *   fpo_septree                -- separator (nested-dissection) property at every
 *                                 node, heap capacity, candidate definition
 *   schedules                  -- equal fill for level and post order
 *   block expansion            -- symbolic analysis of the expanded DOF pattern
 *   fpo_supernodes             -- column structures of a dense symbolic
 *                                 elimination compared set by set
 *   fpo_amd                    -- exact minimum degree where the bound is exact
 *                                 (trees, cycles); the traced bound re-derived
 *                                 from the eliminated set's components
 *   nd_level, refine           -- the full tree cut at nd_level; matching
 *                                 numbers and the canonical cover (scipy)
 */
#ifndef FPO_H
#define FPO_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FPO_OK 0
#define FPO_ERR_ARG (-1)
#define FPO_ERR_INDEX (-2)
#define FPO_ERR_SIZE (-3)
#define FPO_ERR_OOM (-4)

#define FPO_SCHED_LEVEL 0
#define FPO_SCHED_POST 1

typedef struct {
  int32_t patch_size;   /* target patch size S (Sec. 4.1, Step 1; default 512) */
  int32_t lloyd_iters;  /* Lloyd re-centre iterations (Sec. 6: Lloyd's algorithm) */
  uint64_t seed;        /* seed of the seed-selection hash */
  int32_t schedule;     /* FPO_SCHED_LEVEL or FPO_SCHED_POST (Sec. 5) */
  int32_t block_size;   /* b >= 1: DOFs per mesh vertex (Sec. 4.1 Step 2, Sec. 6.5) */
  int32_t nd_level;     /* -1: full depth ceil(log2 P); else at most this many
                           levels, leaves holding several patches (Sec. 4.2 Step 3) */
  int32_t refine;       /* 0: one-sided separator (the smaller candidate side);
                           1: smallest separator inside the superset (Sec. 5) */
  int32_t local_amd;    /* 0: exact minimum degree local orders; 1: approximate
                           minimum degree (fpo_amd) */
} fpo_opts;

typedef struct {
  /* required outputs, n_dof entries each */
  int32_t* perm;      /* perm[new] = old */
  int32_t* iperm;     /* iperm[old] = new */
  int32_t* parent;    /* elimination tree of A(perm,perm); -1 for roots */
  int32_t* colcount;  /* nonzeros of column j of L, diagonal included */
  int64_t nnzL;       /* sum of colcount */
  /* optional outputs (NULL to skip), vertex-level */
  int32_t* gmap;      /* n_v: patch of each vertex */
  int32_t* node_of;   /* n_v: separator-tree node of each vertex */
  /* optional separator-tree ranges in DOF units, capacity max_nodes */
  int32_t* node_begin;
  int32_t* node_size;
  int32_t max_nodes;
  /* scalars written by fpo_order */
  int32_t n_patches;  /* P */
  int32_t depth;      /* D = ceil(log2 P) */
  int32_t n_nodes;    /* 2^(D+1) - 1 */
} fpo_out;

/* SplitMix64: output number i+1 of a generator seeded with `seed`. */
uint64_t fpo_mix64(uint64_t seed, uint64_t i);

/* O0: graph G of A without its diagonal, sorted and deduplicated (Sec. 2;
 * Sec. 4.1 Step 2).  For b > 1 DOF rows b*k..b*k+b-1 merge into vertex k.
 * Count pass returns nnz(G) in *nnz_g; fill pass writes g_rowptr[n_v+1] and
 * g_colind[nnz_g]. */
int fpo_graph_count(int64_t n_dof, const int64_t* rowptr, const int32_t* colind,
                    int32_t b, int64_t* nnz_g);
int fpo_graph_fill(int64_t n_dof, const int64_t* rowptr, const int32_t* colind,
                   int32_t b, int64_t* g_rowptr, int32_t* g_colind);

/* O1: patch partition (Sec. 4.1 Step 1; Lloyd's algorithm, Sec. 6).
 * Returns P (>= 0) or an error.  seeds_out (nullable, n entries) receives the
 * final seed of each patch. */
int fpo_patches(int32_t n, const int64_t* rp, const int32_t* ci, int32_t S,
                int32_t lloyd_iters, uint64_t seed, int32_t* gmap, int32_t* seeds_out);

/* Nearest-seed labelling by level-synchronous multi-source BFS: label[v] =
 * id of the seed nearest to v in hops, ties to the lowest id; -1 if no seed
 * reaches v.  seeds[k] is the seed vertex of id k.  Returns #unlabelled. */
int64_t fpo_grow(int32_t n, const int64_t* rp, const int32_t* ci, int32_t nseeds,
                 const int32_t* seeds, int32_t* label);

/* O2-O6: separator tree (Sec. 4.2 Step 3, Alg. 2, Sec. 5).  node_of[v]
 * receives the heap index of v's node, pnode[p] the final node of patch p.
 * *depth_out = D = min(ceil(log2 P), nd_level) (nd_level -1: no limit).
 * Capacity of the heap is 2^(D+1)-1.  refine selects the separator inside
 * the superset: 0 one side's candidates, 1 the minimum vertex cover of the
 * crossing edges (see refine_node). */
int fpo_septree(int32_t n, const int64_t* rp, const int32_t* ci, int32_t P,
                const int32_t* gmap, int32_t nd_level, int32_t refine, int32_t* node_of,
                int32_t* pnode, int32_t* depth_out);

/* O4: bisection of a quotient subgraph in local indices 0..m-1 (Alg. 2,
 * BiPartition).  w: node weights; (arp, aci): adjacency (symmetric, no self
 * loops, deduplicated).  left[i] = 1 for the left child, 0 for the right. */
int fpo_bisect(int32_t m, const int64_t* w, const int64_t* arp, const int32_t* aci,
               uint8_t* left);

/* O7: exact minimum-degree order of a graph on 0..m-1 (Sec. 4.3 Step 4,
 * LocalOrder): repeatedly eliminate the vertex of least current degree in the
 * elimination graph, ties to the lowest index.  order[k] = k-th vertex.
 * m <= 65535 (FPO_ERR_SIZE beyond), the GPU library's limit too. */
int fpo_md(int32_t m, const int64_t* rp, const int32_t* ci, int32_t* order);

/* F3: approximate minimum degree (Amestoy, Davis, Duff 1996) on the
 * quotient graph, each variable its own supervariable, pivot = least
 * (approximate degree, index).  dtrace (nullable, m*m ints): the
 * approximate degree of every variable when each pivot is chosen (-1 for
 * eliminated ones).  m <= 65535. */
int fpo_amd(int32_t m, const int64_t* rp, const int32_t* ci, int32_t* order, int32_t* dtrace);

/* O9: elimination tree of A(perm,perm) by Liu's algorithm with path
 * compression.  G is the graph of A (no diagonal). */
int fpo_etree(int32_t n, const int64_t* rp, const int32_t* ci, const int32_t* perm,
              const int32_t* iperm, int32_t* parent);

/* O10: column counts of L by row-subtree traversal; returns nnz(L) in *nnzL. */
int fpo_colcount(int32_t n, const int64_t* rp, const int32_t* ci, const int32_t* perm,
                 const int32_t* iperm, const int32_t* parent, int32_t* colcount,
                 int64_t* nnzL);

/* Pin: dense symbolic elimination of A(perm,perm) (n <= 16384). */
int fpo_brute_symbolic(int32_t n, const int64_t* rp, const int32_t* ci,
                       const int32_t* perm, int32_t* parent, int32_t* colcount,
                       int64_t* nnzL);

/* Pin: minimum degree with every degree recomputed from a dense adjacency
 * matrix at every step (m <= 2048). */
int fpo_brute_md(int32_t m, const int64_t* rp, const int32_t* ci, int32_t* order);

/* F1: supernodal symbolic analysis from the elimination tree and column
 * counts (the solver's symbolic phase, Sec. 1): fundamental supernodes
 * (Liu, Ng, Peyton 1993).  Lp[n+1]: column pointers of L; super_of[n]:
 * supernode of every column; super_ptr[ns+1]: first column of every
 * supernode, then n; super_parent[ns]: supernodal elimination tree (-1 for
 * roots); Lx_ptr[ns+1]: offsets of the dense supernode blocks (first column's
 * row count times width).  Any output may be NULL (super_parent and Lx_ptr
 * need super_ptr and super_of).  Capacities: n+1 for super_ptr and Lx_ptr,
 * n for super_parent. */
int fpo_supernodes(int32_t n, const int32_t* parent, const int32_t* colcount, int64_t* Lp,
                   int32_t* super_of, int32_t* super_ptr, int32_t* super_parent, int64_t* Lx_ptr,
                   int32_t* n_super);

/* The whole ordering (Alg. 1).  A is the matrix pattern (diagonal optional,
 * duplicates and column order irrelevant).  user_gmap (nullable, n_v entries)
 * replaces patching (Sec. 5, user-provided groups). */
int fpo_order(int64_t n_dof, const int64_t* rowptr, const int32_t* colind,
              const int32_t* user_gmap, const fpo_opts* opts, fpo_out* out);

#ifdef __cplusplus
}
#endif
#endif
