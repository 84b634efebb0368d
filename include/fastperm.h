/*
 * fastperm.h -- C ABI of the MI355X (gfx950) patch-guided nested-dissection
 * ordering library (libfastperm.so).
 *
 * What it computes (Zarebavani, Mahmoud et al., "Fast Sparse Matrix
 * Permutation for Mesh-Based Direct Solvers"): given the sparsity pattern
 * of a symmetric matrix A from a mesh (Sec. 4, "Inputs and outputs"), a
 * fill-reducing permutation built by patch-guided nested dissection
 * (Alg. 1-3), the separator tree it was built on (Sec. 4.2, stored as a heap
 * array), and the elimination tree and column counts of the Cholesky factor
 * of A(perm, perm) that a sparse Cholesky symbolic phase needs (Sec. 2).
 *
 * Conventions
 *   - All arrays passed to fp_order / fp_order_batch are DEVICE pointers
 *     owned by the caller; the library never frees them.  Server calls take
 *     host arrays (documented there).
 *   - `stream` is a hipStream_t passed as void* (NULL = default stream).
 *     fp_order, fp_order_static, fp_order_batch and fp_supernodes are
 *     asynchronous: they queue their kernels on `stream` (fp_order also on
 *     internal side streams that fork from `stream` with events and join
 *     back into it) and return without waiting for the device or reading
 *     anything back; the results are ready when `stream` reaches the end of
 *     the call.  Counts that only the device knows (patches, tree depth,
 *     frontier sizes) are read by the kernels themselves, so a call can be
 *     captured into a hipGraph.  Errors found by the device are read with
 *     fp_last_error / fp_error_detail (which synchronise `stream`) or from
 *     the status output.
 *   - perm[new] = old, iperm[old] = new.  parent[j] is the elimination-tree
 *     parent of column j of A(perm,perm), -1 for a root.  colcount[j] counts
 *     the nonzeros of column j of L including the diagonal; nnzL is their sum.
 *   - Block patterns (block_size b > 1): DOF b*k+r belongs to mesh vertex k;
 *     the ordering is computed on the vertex graph and expanded so that the
 *     b DOFs of a vertex stay consecutive (Sec. 6.5).  The expansion of the
 *     elimination tree and column counts is exact when every vertex-level
 *     nonzero is a dense b x b block.
 *   - No function throws; every entry point returns an fp_status.  A handle
 *     is not thread-safe: use one per host thread.
 */
#ifndef FASTPERM_H
#define FASTPERM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FP_ABI_VERSION 2

typedef enum {
  FP_OK = 0,
  FP_ERR_ARG = 1,          /* invalid scalar argument or null required pointer */
  FP_ERR_NOT_SYMMETRIC = 2,
  FP_ERR_INDEX = 3,        /* column index / row pointer out of range (device) */
  FP_ERR_SIZE = 4,         /* workspace too small or a device pool overflowed */
  FP_ERR_OOM = 5,          /* device allocation failed */
  FP_ERR_UNSUPPORTED = 6,  /* option value not implemented */
  FP_ERR_BUSY = 7,         /* server admission refused (slots or memory) */
  FP_ERR_HIP = 8,          /* a HIP runtime call failed */
  FP_ERR_DEVICE = 9        /* the device pipeline reported an internal failure */
} fp_status;

typedef struct fp_handle fp_handle;

#define FP_SCHED_LEVEL 0 /* level order: leaves first, then upward (Sec. 5) */
#define FP_SCHED_POST 1  /* post order: left, right, node (Sec. 5) */

/* Size limits: n < 2^31 vertices; every separator-tree node (a patch
 * interior or a separator) holds at most 65535 vertices, or the call reports
 * FP_ERR_SIZE (the oracle has the same limit). */
typedef struct {
  int32_t patch_size;   /* target patch size S (Sec. 6 uses 256; default 512) */
  int32_t nd_level;     /* -1: full depth ceil(log2 P), each leaf one patch; 0..30:
                           at most nd_level levels, a leaf then keeps the remaining
                           vertices of all its patches (Sec. 4.2 Step 3) */
  int32_t schedule;     /* FP_SCHED_LEVEL (default) or FP_SCHED_POST */
  int32_t block_size;   /* DOFs per mesh vertex, >= 1 (default 1) */
  int32_t lloyd_iters;  /* Lloyd re-centre iterations of patching (default 1) */
  uint64_t seed;        /* seed of the patch-seed hash (default 0) */
  uint32_t flags;       /* FP_FLAG_* bits, FP_FLAG_VALIDATE by default */
} fp_options;

/* flags: record the device time of every stage of the call on its stream
 * (read back with fp_stage_times) */
#define FP_FLAG_TIMING 1u
/* flags: check on the device that the pattern is symmetric, as the method
 * requires of its input (Sec. 4, "Inputs and outputs"): every entry (i, j)
 * must have its mirror (j, i) (in block mode, every coupled vertex pair both
 * ways).  A failure stops the ordering and is reported as
 * FP_ERR_NOT_SYMMETRIC.  Set by fp_options_default; a caller that clears it
 * saves one pass over the graph, and an asymmetric pattern then gives an
 * unspecified ordering. */
#define FP_FLAG_VALIDATE 2u
/* flags: refined separators (Sec. 5, separator refinement).  The two sides
 * of a split follow the patches, so the separator can be any set of the
 * superset's vertices that touches every edge between the sides; with this
 * flag it is the smallest such set (a minimum vertex cover of the crossing
 * edges, of the size of a maximum matching), namely the one closest to the
 * side the default rule marks: that side's candidates that every maximum
 * matching covers, plus the other-side neighbours of the rest.  Without it
 * the separator is the smaller side's candidate set (ties to the left).
 * Either way the result is unique. */
#define FP_FLAG_REFINE 4u
/* flags: approximate-minimum-degree local orders (Sec. 4.3 Step 4 names
 * AMD; the degree bound of Amestoy, Davis and Duff, SIAM J. Matrix Anal.
 * Appl. 17(4), 1996) instead of exact minimum degree: elimination on the
 * quotient graph with element absorption, each variable its own
 * supervariable, the pivot the least (bound, rank of the vertex id in the
 * node).  The result is unique. */
#define FP_FLAG_AMD 8u

/* Pattern of A in CSR form (device arrays).  Exactly one of rowptr32 /
 * rowptr64 is non-NULL (n+1 entries); colind has nnz entries in [0, n).
 * The pattern must be symmetric; the diagonal is optional; duplicates and
 * column order do not matter.  n < 2^31. */
typedef struct {
  int64_t n;
  int64_t nnz;
  const int32_t* rowptr32;
  const int64_t* rowptr64;
  const int32_t* colind;
} fp_csr;

/* Outputs (device arrays owned by the caller).  perm, iperm, parent and
 * colcount (n entries each) and nnzL (1 entry) are required; the rest are
 * optional (NULL skips them).  node_begin/node_size receive the separator
 * tree as a heap (node t has children 2t+1, 2t+2) in DOF units; their
 * capacity max_nodes comes from fp_query.  gmap (n/b entries) receives the
 * patch of every mesh vertex; n_nodes (1 entry) the heap size 2^(D+1)-1;
 * status (1 entry) the device error bits (0 = success). */
typedef struct {
  int32_t* perm;
  int32_t* iperm;
  int32_t* parent;
  int32_t* colcount;
  int64_t* nnzL;
  int32_t* node_begin;
  int32_t* node_size;
  int32_t* gmap;
  int32_t* n_nodes;
  uint32_t* status;
  int32_t max_nodes;
} fp_result;

int fp_version(void);
const char* fp_status_str(fp_status s);
void fp_options_default(fp_options* opts);

/* Create / destroy a handle bound to the current HIP device.  The handle
 * owns device properties, execution settings and its events;
 * fp_destroy(NULL) is a no-op.  The pipeline of one matrix forks work onto
 * three internal streams that every handle of the device shares (created on
 * first use, kept until the process ends), so the number of streams stays
 * within the device's hardware queues however many handles exist; calls of
 * several handles on several host threads stay correct and may wait on each
 * other's work on those streams. */
fp_status fp_create(fp_handle** h);
fp_status fp_destroy(fp_handle* h);

/* Host-side sizing, no device work: bytes of device workspace fp_order needs
 * for this pattern and options, and the capacity for node_begin/node_size. */
fp_status fp_query(fp_handle* h, const fp_csr* A, const fp_options* opts,
                   size_t* workspace_bytes, int32_t* max_nodes);

/* Order one matrix (Alg. 1).  user_gmap (device, n/b entries, nullable)
 * replaces patching with caller groups in [0, n/b) (Sec. 5).  workspace is
 * device memory of at least the fp_query size, owned by the caller and not
 * shared with another call in flight.  Asynchronous on `stream`. */
fp_status fp_order(fp_handle* h, const fp_csr* A, const int32_t* user_gmap,
                   const fp_options* opts, void* workspace, size_t ws_bytes,
                   fp_result* out, void* stream);

/* Order a matrix again after its pattern changed, on the same mesh
 * vertices, keeping an earlier call's patches: the reuse of the nested-
 * dissection hierarchy across pattern changes that the paper builds on
 * (Sec. 2, related work: reordering when the sparsity pattern changes over
 * time).  The result is exactly fp_order's with user_gmap = prev_gmap (the
 * gmap output of the earlier call); separator-tree nodes whose vertex set and
 * induced edges are unchanged take their local order (Sec. 4.3 Step 4) from
 * the earlier call instead of recomputing it, which is exact because that
 * order depends on nothing else.  prev_workspace is the earlier call's
 * workspace, unchanged since that call finished on the device (and not the
 * same buffer as `workspace`); a call whose sizes differ (another vertex
 * count, block size or tree size) reuses nothing and is still correct.
 * reused_vertices (device, 1 entry, nullable) receives the number of
 * vertices whose local order was reused.  Asynchronous like fp_order. */
fp_status fp_order_update(fp_handle* h, const fp_csr* A, const int32_t* prev_gmap,
                          const void* prev_workspace, const fp_options* opts, void* workspace,
                          size_t ws_bytes, fp_result* out, int32_t* reused_vertices,
                          void* stream);

/* fp_order for callers that cannot allocate device memory (code that must
 * not call hipMalloc: tight serving loops, harnesses that forbid it).  The
 * workspace is a static device array of the library, 256 MiB per device,
 * held from the library's first use on a device until the process ends;
 * the caller still passes the matrix and the output buffers.  A matrix whose
 * fp_query workspace exceeds 256 MiB gets FP_ERR_SIZE (no work is queued).
 * Every launch stays on `stream` and the call creates nothing: no memory,
 * streams or events.  Device error bits are written to out->status (pass a
 * non-NULL status to see them).  All calls on one device share that
 * device's array, and the last call's contents stay in it: two calls that
 * overlap on one device (different streams or host threads) race and give
 * wrong results, so serialise them.  Results equal fp_order's. */
fp_status fp_order_static(fp_handle* h, const fp_csr* A, const int32_t* user_gmap,
                          const fp_options* opts, fp_result* out, void* stream);

/* ---------------------------------------------------------------------
 * Supernodal symbolic analysis of the ordering's result, the first step of
 * the solver's symbolic phase, which needs the elimination tree (Sec. 1):
 * fundamental supernodes (Liu, Ng, Peyton, SIAM J. Matrix Anal. Appl.
 * 14(1), 1993).  Column j+1 continues the supernode of column j exactly when
 * parent[j] == j+1, j is the only child of j+1, and colcount[j] ==
 * colcount[j+1] + 1.  Inputs are the parent and colcount arrays that
 * fp_order wrote (n columns; device arrays).  Outputs (device arrays owned
 * by the caller):
 *   Lp[n+1]            column pointers of L (exclusive sums of colcount);
 *   super_ptr[n+1]     first column of every supernode, then n (the first
 *                      n_super+1 entries are written);
 *   n_super[1]         number of supernodes;
 *   super_of[n]        supernode of every column (nullable);
 *   super_parent[n]    supernodal elimination tree: the supernode of the
 *                      parent of its last column, -1 for roots (nullable);
 *   Lx_ptr[n+1]        offsets of dense supernode blocks, each the first
 *                      column's row count times the width (nullable);
 *   status[1]          1 if a parent entry is not -1 and not in (j, n)
 *                      (nullable; the other outputs are then unspecified).
 * Asynchronous on `stream`: nothing is read back to the host. */
typedef struct {
  int64_t* Lp;
  int32_t* super_ptr;
  int32_t* n_super;
  int32_t* super_of;
  int32_t* super_parent;
  int64_t* Lx_ptr;
  uint32_t* status;
} fp_super_result;

/* Bytes of device workspace fp_supernodes needs for n columns. */
fp_status fp_supernodes_query(int64_t n, size_t* workspace_bytes);
fp_status fp_supernodes(fp_handle* h, int64_t n, const int32_t* parent, const int32_t* colcount,
                        void* workspace, size_t ws_bytes, fp_super_result* out, void* stream);

/* Execution settings of the local-order stage (Sec. 4.3 Step 4), for an
 * autotuner: the LDS of each local-order workgroup (its size classes are a
 * quarter, half and all of it; 16 KB .. max_lds_bytes, a multiple of 1 KB;
 * 64 KB by default) and the workgroups launched per CU (1 .. 8; 2 by
 * default).  They change speed only: every result is the same under any
 * setting.  fp_get_tuning also reports the device's per-workgroup LDS limit. */
typedef struct {
  int32_t md_lds_bytes;
  int32_t md_blocks_per_cu;
  int32_t max_lds_bytes; /* fp_get_tuning only */
} fp_tuning;
fp_status fp_set_tuning(fp_handle* h, const fp_tuning* t);
fp_status fp_get_tuning(fp_handle* h, fp_tuning* t);

/* Synchronise `stream` and translate the device error bits of the last
 * call that used `workspace`. */
fp_status fp_last_error(fp_handle* h, void* workspace, void* stream);

/* Same, with the raw device error bits, the code of the first device check
 * that failed (0 if none; the FP_SITE_* values of the library's sources)
 * and one value it recorded (a node or vertex id).  Any output pointer may
 * be NULL. */
fp_status fp_error_detail(fp_handle* h, void* workspace, void* stream, uint32_t* bits,
                          int32_t* site, int32_t* arg);

/* Stages of one ordering, in order (the paper's breakdown into patching,
 * separators, local orders ... , Sec. 6.6): fp_stage_count() of them, named
 * by fp_stage_name(i).  fp_stage_times waits for the last call made with
 * FP_FLAG_TIMING on this handle and writes up to n stage times in
 * milliseconds (device time between consecutive stage boundaries on the
 * call's stream). */
int fp_stage_count(void);
const char* fp_stage_name(int i);
fp_status fp_stage_times(fp_handle* h, float* ms, int32_t n);

/* Time one kernel of the pipeline: every launch of the kernel named `name`
 * (e.g. "k_md"; NULL or "" stops) in later fp_order calls on this handle is
 * bracketed by events on the call's stream.  fp_kernel_time waits for the
 * last call's events and returns the summed device time and the number of
 * launches of that kernel in it. */
fp_status fp_time_kernel(fp_handle* h, const char* name);
fp_status fp_kernel_time(fp_handle* h, float* total_ms, int32_t* launches);

/* ---------------------------------------------------------------------
 * Batches: many independent matrices of uneven size (the paper orders meshes
 * from 1.5K to 1.8M vertices, Sec. 6) in one pass over the pipeline: every
 * kernel launch covers all matrices at once (each matrix takes the blocks
 * it would take alone, found by a block table the call uploads), and the
 * local orders of all separator-tree nodes of all matrices run in the same
 * launches.  Matrix i is A[i] with options opts[i], optional user grouping
 * user_gmap[i] (user_gmap itself may be NULL) and outputs out[i]; its result
 * is exactly what fp_order gives for it alone.  All pointers in A, out and
 * user_gmap are device pointers owned by the caller.
 * fp_query_batch: bytes of workspace for the batch (the matrices' own
 * workspaces, their descriptions and the block tables) and the largest
 * node_begin/node_size capacity among the matrices.
 * fp_order_batch: asynchronous like fp_order: queued on `stream`, nothing
 * read back; the descriptions and block tables are copied from pinned
 * memory the handle keeps (a later batch call on the same handle first
 * waits for that copy).  Device errors of matrix i are its out[i].status
 * bits (0 = success), valid when `stream` reaches the end of the batch.
 * To replay a batch without host work, record it with fp_graph_create: a
 * stream capture of this call would record the copy from the handle's
 * pinned memory, which a later batch call refills. */
fp_status fp_query_batch(fp_handle* h, int32_t n_mesh, const fp_csr* A, const fp_options* opts,
                         const int32_t* const* user_gmap, size_t* workspace_bytes,
                         int32_t* max_nodes);
fp_status fp_order_batch(fp_handle* h, int32_t n_mesh, const fp_csr* A,
                         const int32_t* const* user_gmap, const fp_options* opts, void* workspace,
                         size_t ws_bytes, fp_result* out, void* stream);

/* The same batch over concatenated arrays (device):
 *   rowptr  int64, mesh i's n_i + 1 row pointers at rowptr[vtx_off[i] + i],
 *           each mesh's starting at 0;
 *   colind  int32, mesh i's entries at colind[nnz_off[i] ..], column indices
 *           local to the mesh (0 .. n_i - 1);
 *   vtx_off, nnz_off  HOST arrays of n_mesh + 1 offsets (rows and entries);
 *   perm, iperm, parent, colcount  mesh i's local results at [vtx_off[i] ..];
 *   nnzL[i], status[i]  one per mesh (status nullable);
 *   node_begin, node_size  nullable; mesh i's separator tree at node_off[i]
 *           with capacity node_off[i+1] - node_off[i] (node_off is a HOST
 *           array that fp_query_batch_concat fills).
 * Sizes are in DOF units for block patterns (opts[i].block_size). */
fp_status fp_query_batch_concat(fp_handle* h, int32_t n_mesh, const int64_t* rowptr,
                                const int32_t* colind, const int64_t* vtx_off,
                                const int64_t* nnz_off, const fp_options* opts,
                                size_t* workspace_bytes, int64_t* node_off);
fp_status fp_order_batch_concat(fp_handle* h, int32_t n_mesh, const int64_t* rowptr,
                                const int32_t* colind, const int64_t* vtx_off,
                                const int64_t* nnz_off, const fp_options* opts, void* workspace,
                                size_t ws_bytes, int32_t* perm, int32_t* iperm, int32_t* parent,
                                int32_t* colcount, int64_t* nnzL, uint32_t* status,
                                int32_t* node_begin, int32_t* node_size, const int64_t* node_off,
                                void* stream);

/* ---------------------------------------------------------------------
 * Recorded orderings: the whole pipeline of one matrix (the fp_order path)
 * or of a batch (n_mesh > 1: the fp_order_batch path) recorded once into a
 * HIP graph and replayed by fp_graph_launch with a single host call and no
 * host work between the stages (Alg. 1 runs on the device end to end).
 *   fp_graph_create: arguments as fp_order_batch; workspace_bytes from
 *     fp_query_batch (for one matrix that is at least fp_query's).  The
 *     descriptions and block tables are written into the workspace with a
 *     synchronous copy before recording, so the workspace must be idle.
 *     FP_FLAG_TIMING gives FP_ERR_ARG; the
 *     handle's execution settings (fp_set_tuning) at this call are the
 *     graph's.  Nothing is queued; *g receives the graph.
 *   fp_graph_launch: queue one replay on `stream`.  Every replay reads the
 *     inputs anew, so their contents may change between replays as long as
 *     n and nnz stay those of the recording (the device checks every row
 *     range against nnz); the outputs and device errors (out[i].status, or
 *     fp_last_error on the workspace for one matrix) are those of the last
 *     replay.  The inputs, outputs and workspace must stay allocated while
 *     the graph exists; replays of one graph, and any other call on its
 *     workspace, must not overlap (they share the workspace).
 *   fp_graph_destroy: release the graph (NULL is a no-op); the caller makes
 *     sure no replay is still running. */
typedef struct fp_graph fp_graph;
fp_status fp_graph_create(fp_handle* h, int32_t n_mesh, const fp_csr* A,
                          const int32_t* const* user_gmap, const fp_options* opts, void* workspace,
                          size_t ws_bytes, fp_result* out, fp_graph** g);
fp_status fp_graph_launch(fp_graph* g, void* stream);
fp_status fp_graph_destroy(fp_graph* g);

/* ---------------------------------------------------------------------
 * Serving: a request loop that admits ordering requests of any size while
 * others run.  A request is admitted when one of max_slots worker slots is
 * free and its device footprint (input copy, workspace, outputs) fits in
 * what is left of hbm_budget bytes of device memory, which the server
 * allocates once at creation and keeps; the requests in flight overlap on
 * the device, each on its own stream.  Admission takes the oldest request
 * that fits among the 64 oldest waiting, so small requests need not queue
 * behind a large one that waits for memory; a request passed over 32 times
 * stops every later one until it fits.  Options as for fp_order (the
 * timing flag is ignored).
 * Inputs are HOST arrays; they must stay valid until fp_server_wait returns
 * for the ticket.  Results are the same as fp_order's for the matrix alone.
 */
typedef struct fp_server fp_server;

typedef struct {
  int64_t n;
  int64_t nnz;
  const int64_t* rowptr; /* host, n+1 entries */
  const int32_t* colind; /* host, nnz entries */
} fp_host_csr;

/* FP_ERR_OOM if hbm_budget cannot be allocated. */
fp_status fp_server_create(fp_handle* h, size_t hbm_budget, int32_t max_slots, fp_server** s);
/* Queue a request; FP_ERR_BUSY if its footprint exceeds the whole budget. */
fp_status fp_server_submit(fp_server* s, const fp_host_csr* A, const fp_options* opts,
                           uint64_t* ticket);
/* *done = 1 once the request has finished (no wait). */
fp_status fp_server_test(fp_server* s, uint64_t ticket, int32_t* done);
/* Wait for a request, copy its results to host arrays (n entries each; any
 * output pointer may be NULL) and release the ticket.  latency_s is the
 * time from submission to completion.  Returns the request's status. */
fp_status fp_server_wait(fp_server* s, uint64_t ticket, int32_t* perm, int32_t* iperm,
                         int32_t* parent, int32_t* colcount, int64_t* nnzL, double* latency_s);
/* Finish the requests in flight, release the device memory and threads.
 * Tickets not yet waited for are dropped. */
fp_status fp_server_destroy(fp_server* s);

#ifdef __cplusplus
}
#endif
#endif
