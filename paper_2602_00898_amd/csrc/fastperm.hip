// fastperm.hip -- gfx950 kernels of the patch-guided nested-dissection
// ordering and the C ABI declared in include/fastperm.h.
//
// Stages (one or a few kernels each, in stream order):
//   ingest -> patches (seeds, frontier growth, Lloyd) -> quotient graph ->
//   separator tree (per level: arc recount, bisection, separator marking) ->
//   grouping in schedule order -> local minimum-degree orders ->
//   elimination tree / column counts (per level) -> block expansion.
// The job description lives in the workspace and is read through a pointer;
// the host reads a few scalars between stages (patch count, frontier sizes).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>

#include "../../include/fastperm.h"
#include "fp_handle.h"
#include "fp_plan.h"
#include "fp_stages_sym.h"
#include "fp_stages_amd.h"

#define FP_CC_ROUNDS 4  // launched rounds of the orphan-component pass

// A launch can cover several meshes (a batch): the grid is the
// concatenation of every mesh's own grid, and g.boff[i] is the first block
// of mesh i (g.boff[nm] the total).  A block finds its mesh by binary search
// and then works as if it ran alone: fp_s.bx / fp_s.gx are its block index
// and grid size within that mesh.  A single mesh passes no table.
struct FpGrid {
  const FpMesh* ms;
  const int* boff;
  int nm;
};
struct FpSlot {
  int mi, bx, gx;
};
__device__ __forceinline__ FpSlot fp_slot(const FpGrid& g) {
  if (!g.boff) return FpSlot{0, (int)blockIdx.x, (int)gridDim.x};
  int lo = 0, hi = g.nm - 1;  // the last mesh whose first block is <= blockIdx.x
  const int b = (int)blockIdx.x;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (g.boff[mid] <= b)
      lo = mid;
    else
      hi = mid - 1;
  }
  lo = uni(lo);
  return FpSlot{lo, b - g.boff[lo], g.boff[lo + 1] - g.boff[lo]};
}
// grid-stride indices within the block's mesh
__device__ __forceinline__ int vt(const FpSlot& s) { return s.bx * (int)blockDim.x + (int)threadIdx.x; }
__device__ __forceinline__ int vs(const FpSlot& s) { return s.gx * (int)blockDim.x; }
__device__ __forceinline__ int vw(const FpSlot& s) { return uni(vt(s) >> 6); }
__device__ __forceinline__ int vn(const FpSlot& s) { return vs(s) >> 6; }

// The meshes' descriptions come in as a __restrict__ kernel argument: the
// kernels never write them, and without the qualifier the compiler would
// reload a description field after every store in a loop.
#define MESH0                                                  \
  const FpSlot fp_s = fp_slot(FpGrid{fp_ms, fp_boff, fp_nm});  \
  const FpMesh& M = fp_ms[fp_s.mi];                            \
  gptr<FpCtl> C = M.ctl;                                       \
  (void)C

// Every stage after ingest stops at once when an earlier one raised an
// error (its inputs may be unset).  A kernel on another stream may raise it
// while this one starts, so the error word is read once per wave (MESH:
// kernels whose waves never meet at a barrier) or once per workgroup and
// shared through LDS (MESH_WG: kernels with workgroup barriers, which a
// workgroup must reach whole).  MESH adds no LDS, so the kernels that take
// all of it keep it.
__device__ __forceinline__ bool wave_failed(gptr<FpCtl> C) { return uni((unsigned)C->err) != 0u; }
__device__ __forceinline__ bool wg_failed(gptr<FpCtl> C) {
  __shared__ unsigned fp_err_seen;
  if (threadIdx.x == 0) fp_err_seen = C->err;
  __syncthreads();
  return fp_err_seen != 0;
}
#define MESH \
  MESH0;     \
  if (wave_failed(C)) return
#define MESH_WG \
  MESH0;        \
  if (wg_failed(C)) return

// ==========================================================================
// generic helpers
// ==========================================================================
__global__ void k_fill(int* a, int n, int v) {
  for (int i = gtid(); i < n; i += gsize()) a[i] = v;
}
__global__ void k_copy(int* dst, const int* src, int n) {
  for (int i = gtid(); i < n; i += gsize()) dst[i] = src[i];
}
__global__ void k_put_mesh(FpMesh m, FpMesh* dst) {
  if (gtid() == 0) *dst = m;
}
__global__ void k_set(int* a, const int* v) {
  if (gtid() == 0) *a = *v;
}
// A count that only the device knows (a patch or arc count): the value at
// n_dev plus `add`, clamped to [0, cap]; without n_dev, cap itself.  Launch
// grids are sized on the host from capacities or expected values, and every
// loop runs to the count read here.
__device__ __forceinline__ int dcount(const int* n_dev, int add, int cap) {
  if (!n_dev) return cap;
  const int x = *n_dev + add;
  return x < 0 ? 0 : (x > cap ? cap : x);
}
__global__ void k_fill_n(int* a, const int* n_dev, int add, int cap, int v) {
  const int n = dcount(n_dev, add, cap);
  for (int i = gtid(); i < n; i += gsize()) a[i] = v;
}
__global__ void k_copy_n(int* dst, const int* src, const int* n_dev, int cap) {
  const int n = dcount(n_dev, 0, cap);
  for (int i = gtid(); i < n; i += gsize()) dst[i] = src[i];
}
// base[*idx] = *v, with *idx in [0, cap]
__global__ void k_set_at(int* base, const int* idx, int cap, const int* v) {
  if (gtid() == 0) base[dcount(idx, 0, cap)] = *v;
}

// exclusive scan, three passes: chunk sums, scan of the sums, chunk scans
__global__ void k_scan_part(const int* in, int cap, const int* n_dev, int chunk, int* part) {
  __shared__ int tmp[FP_WAVES + 2];
  const int n = dcount(n_dev, 0, cap);
  const int lo = min(n, (int)blockIdx.x * chunk), hi = min(n, lo + chunk);
  int s = 0;
  for (int i = lo + (int)threadIdx.x; i < hi; i += FP_WG) s += in[i];
  int tot;
  wg_excl_scan(s, tmp, &tot);
  if (threadIdx.x == 0) part[blockIdx.x] = tot;
}
__global__ void k_scan_top(int* part, int np, int* total) {
  __shared__ int tmp[FP_WAVES + 2];
  int base = 0;
  for (int c0 = 0; c0 < np; c0 += FP_WG) {
    const int i = c0 + (int)threadIdx.x;
    const int x = i < np ? part[i] : 0;
    int tt;
    const int ex = wg_excl_scan(x, tmp, &tt);
    if (i < np) part[i] = base + ex;
    base += tt;
  }
  if (threadIdx.x == 0) *total = base;
}
__global__ void k_scan_apply(const int* in, int* out, int cap, const int* n_dev, int chunk,
                             const int* part) {
  __shared__ int tmp[FP_WAVES + 2];
  const int n = dcount(n_dev, 0, cap);
  const int lo = min(n, (int)blockIdx.x * chunk), hi = min(n, lo + chunk);
  int base = part[blockIdx.x];
  for (int t0 = lo; t0 < hi; t0 += FP_WG) {
    const int i = t0 + (int)threadIdx.x;
    const int x = i < hi ? in[i] : 0;
    int tt;
    const int ex = wg_excl_scan(x, tmp, &tt);
    if (i < hi) out[i] = base + ex;
    base += tt;
  }
}

// ==========================================================================
// per-mesh generic passes: arrays and counts named by selectors, so that one
// launch serves every mesh of a batch
// ==========================================================================
enum : int { FA_PCNT, FA_GRP, FA_PPTR, FA_QPTR, FA_WP, FA_SBUF, FA_PROW };
enum : int { FN_N, FN_NNCAP, FN_P, FN_NN, FN_CCN };
enum : int { FT_NNZG, FT_TOT, FT_NQ, FT_NROOT };
__device__ __forceinline__ gptr<int> fa_arr(const FpMesh& M, int a) {
  switch (a) {
    case FA_PCNT: return M.pcnt;
    case FA_GRP: return M.grp;
    case FA_PPTR: return M.pptr;
    case FA_QPTR: return M.qptr;
    case FA_WP: return M.wp;
    case FA_SBUF: return M.sbuf;
    default: return M.prow;
  }
}
// capacity (host-known) and count (device) of a pass
__device__ __forceinline__ int fn_cap(const FpMesh& M, int f) {
  return f == FN_NNCAP || f == FN_NN ? M.NNcap : M.n;
}
__device__ __forceinline__ int fn_count(const FpMesh& M, int f) {
  const int cap = fn_cap(M, f);
  int x = cap;
  if (f == FN_P) x = M.ctl->P;
  if (f == FN_NN) x = M.ctl->nn;
  if (f == FN_CCN) x = M.ctl->ccn;
  return x < 0 ? 0 : (x > cap ? cap : x);
}
__device__ __forceinline__ gptr<int> ft_ptr(const FpMesh& M, int t) {
  FpCtl* C = M.ctl.p;
  switch (t) {
    case FT_NNZG: return gptr<int>(&C->nnz_g);
    case FT_NQ: return gptr<int>(&C->nq);
    case FT_NROOT: return gptr<int>(&C->nroot);
    default: return gptr<int>(&C->tot);
  }
}
// scan blocks of a pass with capacity `cap` (the host uses the same rule)
__host__ __device__ __forceinline__ int scan_blocks(int cap) {
  const int b = (cap + 4095) / 4096;
  return b < 1 ? 1 : (b > 1024 ? 1024 : b);
}
// exclusive scan of a per-mesh array, three launches: chunk sums, a scan of
// the sums (one block per mesh), chunk rescans; the total goes to `tdst`
__global__ void k_mscan_part(const FpMesh* __restrict__ fp_ms, const int* __restrict__ fp_boff, int fp_nm, int ain, int fcnt) {
  MESH;
  __shared__ int tmp[FP_WAVES + 2];
  const int cap = fn_cap(M, fcnt), n = fn_count(M, fcnt);
  const int chunk = max(1, (cap + fp_s.gx - 1) / fp_s.gx);
  gptr<const int> in = fa_arr(M, ain);
  const int lo = min(n, fp_s.bx * chunk), hi = min(n, lo + chunk);
  int sum = 0;
  for (int i = lo + (int)threadIdx.x; i < hi; i += FP_WG) sum += in[i];
  int tot;
  wg_excl_scan(sum, tmp, &tot);
  if (threadIdx.x == 0) C->part[fp_s.bx] = tot;
}
__global__ void k_mscan_top(const FpMesh* __restrict__ fp_ms, const int* __restrict__ fp_boff, int fp_nm, int fcnt, int tdst) {
  MESH;
  __shared__ int tmp[FP_WAVES + 2];
  const int np = scan_blocks(fn_cap(M, fcnt));
  int base = 0;
  for (int c0 = 0; c0 < np; c0 += FP_WG) {
    const int i = c0 + (int)threadIdx.x;
    const int x = i < np ? (int)C->part[i] : 0;
    int tt;
    const int ex = wg_excl_scan(x, tmp, &tt);
    if (i < np) C->part[i] = base + ex;
    base += tt;
  }
  if (threadIdx.x == 0) *ft_ptr(M, tdst) = base;
}
__global__ void k_mscan_apply(const FpMesh* __restrict__ fp_ms, const int* __restrict__ fp_boff, int fp_nm, int ain, int aout, int fcnt) {
  MESH;
  __shared__ int tmp[FP_WAVES + 2];
  const int cap = fn_cap(M, fcnt), n = fn_count(M, fcnt);
  const int chunk = max(1, (cap + fp_s.gx - 1) / fp_s.gx);
  gptr<const int> in = fa_arr(M, ain);
  gptr<int> out = fa_arr(M, aout);
  const int lo = min(n, fp_s.bx * chunk), hi = min(n, lo + chunk);
  int base = C->part[fp_s.bx];
  for (int t0 = lo; t0 < hi; t0 += FP_WG) {
    const int i = t0 + (int)threadIdx.x;
    const int x = i < hi ? (int)in[i] : 0;
    int tt;
    const int ex = wg_excl_scan(x, tmp, &tt);
    if (i < hi) out[i] = base + ex;
    base += tt;
  }
}
// out[count] = total (the last row pointer)
__global__ void k_mptr_end(const FpMesh* __restrict__ fp_ms, const int* __restrict__ fp_boff, int fp_nm, int aout, int fcnt, int tsrc) {
  MESH;
  if (vt(fp_s) == 0) fa_arr(M, aout)[fn_count(M, fcnt)] = *ft_ptr(M, tsrc);
}
__global__ void k_mcopy(const FpMesh* __restrict__ fp_ms, const int* __restrict__ fp_boff, int fp_nm, int adst, int asrc, int fcnt) {
  MESH;
  const int n = fn_count(M, fcnt);
  gptr<int> d = fa_arr(M, adst);
  gptr<const int> a = fa_arr(M, asrc);
  for (int i = vt(fp_s); i < n; i += vs(fp_s)) d[i] = a[i];
}
// control block of every mesh of a batch cleared before its pipeline
// starts: block i clears mesh i's
__global__ void k_ctl_clear_all(const FpMesh* __restrict__ ms) {
  gptr<int> w = ms[blockIdx.x].ctl.as<int>();
  const int words = (int)(sizeof(FpCtl) / 4);
  for (int i = (int)threadIdx.x; i < words; i += (int)blockDim.x) w[i] = 0;
}

// entries of a mesh row whose loads a lane issues together (rows have 4 to 8
// entries; longer ones take a loop for the rest)
#define FP_BFS_ROW 8

// ==========================================================================
// ingest: graph of A without its diagonal (Sec. 4.1 Step 2, Sec. 6.5)
// ==========================================================================
__global__ void k_ingest(const FpMesh* __restrict__ fp_ms, const int* __restrict__ fp_boff, int fp_nm, int fill) {
  MESH0;
  if (fill && wave_failed(C)) return;
  unsigned eb = 0;
  for (int v = vt(fp_s); v < M.n; v += vs(fp_s)) {
    if (fill) {
      gather_vertex_row(M, v, M.gci + M.grp[v], &eb);
    } else {
      const int c = gather_vertex_row(M, v, gptr<int>(nullptr), &eb);
      M.pcnt[v] = c < 0 ? 0 : c;
      if (c < 0) M.fb[atomicAdd(&C->nlong, 1)] = v;  // a long row: listed
    }
  }
  if (eb) fp_fail(C, eb, FP_SITE_INGEST, 0);
}
// rows of more than FP_ROW_SHORT input entries, a workgroup each
__global__ void k_ingest_long(const FpMesh* __restrict__ fp_ms, const int* __restrict__ fp_boff, int fp_nm, int fill) {
  MESH0;
  __shared__ int red;
  if (fill && wg_failed(C)) return;
  unsigned eb = 0;
  const int nl = C->nlong;
  for (int l = fp_s.bx; l < nl; l += fp_s.gx) {
    const int v = M.fb[l];
    const int c = ingest_long_row(M, v, fill ? M.gci + M.grp[v] : gptr<int>(nullptr), &eb, &red);
    if (!fill && threadIdx.x == 0) M.pcnt[v] = c;
  }
  if (eb) fp_fail(C, eb, FP_SITE_INGEST, 0);
}
// the vertex graph fits its capacity (an int32 count that overflowed reads
// negative); the fill pass and every later stage are gated on this
__global__ void k_check_graph(const FpMesh* __restrict__ fp_ms, const int* __restrict__ fp_boff, int fp_nm) {
  MESH0;
  if (vt(fp_s) == 0 && (C->nnz_g < 0 || (long long)C->nnz_g > M.Ecap))
    fp_fail(C, FP_E_SCRATCH, FP_SITE_GRAPH, C->nnz_g);
}
// every entry (v, u) of the graph has its mirror (u, v): the pattern of A is
// symmetric (Sec. 4, inputs), block by block in block mode
__global__ void k_validate(const FpMesh* __restrict__ fp_ms, const int* __restrict__ fp_boff, int fp_nm) {
  MESH0;
  if (!M.validate || wave_failed(C)) return;
  for (int v = vt(fp_s); v < M.n; v += vs(fp_s))
    for (int e = M.grp[v]; e < M.grp[v + 1]; e++)
      if (!row_has(M, M.gci[e], v)) {
        fp_fail(C, FP_E_ASYM, FP_SITE_ASYM, v);
        break;
      }
}

// ==========================================================================
// patches (Sec. 4.1 Step 1; Lloyd's algorithm, Sec. 6).  Growth computes,
// for every vertex, (hop distance to the nearest seed, id of the nearest
// seed with ties to the lowest id) as the fixed point of 64-bit keys
// (dist << 32 | id), one level per launch, atomicMin on the keys.
// ==========================================================================
__host__ __device__ __forceinline__ int fp_p0(long long n, int S) {
  return n > 0 ? (int)((n + S - 1) / S) : 0;
}
__global__ void k_seeds(const FpMesh* __restrict__ fp_ms, const int* __restrict__ fp_boff, int fp_nm) {
  MESH;
  const int P0 = fp_p0(M.n, M.S);
  const int n = M.n, S = M.S;
  for (int blk = vw(fp_s); blk < P0; blk += vn(fp_s)) {
    const long long lo = (long long)blk * S, hi = min((long long)n, lo + S);
    uint64_t bh = FP_UNSET;
    uint32_t bv = 0xFFFFFFFFu;
    for (long long v = lo + lane_id(); v < hi; v += 64) {
      const uint64_t h = fp_mix64(M.seed, (uint64_t)v);
      if (h < bh) {
        bh = h;
        bv = (uint32_t)v;
      }
    }
    const uint64_t hm = wave_min_u64(bh);
    const uint32_t vm = wave_min_u32(bh == hm ? bv : 0xFFFFFFFFu);
    if (lane_id() == 0) M.seeds[blk] = (int)vm;
  }
  if (vt(fp_s) == 0) {
    C->P0 = P0;
    C->P = P0;
  }
}
__global__ void k_key_unset(const FpMesh* __restrict__ fp_ms, const int* __restrict__ fp_boff, int fp_nm) {
  MESH;
  for (int v = vt(fp_s); v < M.n; v += vs(fp_s)) M.key[v] = FP_UNSET;
  for (int i = vt(fp_s); i < M.n + 16; i += vs(fp_s)) M.fcnt[i] = 0;
}
// all: every patch seed (the count is on the device); else the P0 seeds
__global__ void k_seed_push(const FpMesh* __restrict__ fp_ms, const int* __restrict__ fp_boff, int fp_nm, int all) {
  MESH;
  const int nseeds = all ? min(C->P, M.n) : fp_p0(M.n, M.S);
  for (int k = vt(fp_s); k < nseeds; k += vs(fp_s)) {
    const int s = M.seeds[k];
    atomicMin(&M.key[s], (unsigned long long)k);
    M.fa[k] = s;
  }
  if (vt(fp_s) == 0) M.fcnt[0] = nseeds;
}
// One frontier level: a lane per frontier vertex.  The loads of its first
// FP_BFS_ROW neighbours (columns, then keys) go out together, and the
// workgroup's claims are appended with one atomic (every wave taking one on
// the next frontier's single counter had serialised the large levels).
__global__ void __launch_bounds__(FP_WG) k_bfs_level(const FpMesh* __restrict__ fp_ms, const int* __restrict__ fp_boff, int fp_nm, int lvl) {
  MESH_WG;
  __shared__ int scan_tmp[FP_WAVES + 2];
  __shared__ int base_s;
  const int nf = M.fcnt[lvl];
  gptr<const int> cur = (lvl & 1) ? M.fb : M.fa;
  gptr<int> nxt = (lvl & 1) ? M.fa : M.fb;
  // the workgroup steps together (a barrier in each step)
  for (int b0 = fp_s.bx * FP_WG; b0 < nf; b0 += fp_s.gx * FP_WG) {
    const int f = b0 + (int)threadIdx.x;
    int e0 = 0, deg = 0;
    unsigned long long kv = 0;
    if (f < nf) {
      const int v = cur[f];
      kv = M.key[v] + (1ull << 32);
      e0 = M.grp[v];
      deg = M.grp[v + 1] - e0;
    }
    // the first FP_BFS_ROW neighbours: columns, then keys, then claims, each
    // round of loads issued at once; longer rows continue one by one
    int u[FP_BFS_ROW];
#pragma unroll
    for (int j = 0; j < FP_BFS_ROW; j++) u[j] = j < deg ? (int)M.gci[e0 + j] : -1;
    unsigned long long ku[FP_BFS_ROW];
#pragma unroll
    for (int j = 0; j < FP_BFS_ROW; j++) ku[j] = u[j] >= 0 ? (unsigned long long)M.key[u[j]] : 0ull;
    unsigned claims = 0u;
#pragma unroll
    for (int j = 0; j < FP_BFS_ROW; j++)
      if (u[j] >= 0 && ku[j] > kv && atomicMin(&M.key[u[j]], kv) == FP_UNSET) claims |= 1u << j;
    // one slot range per workgroup for all these claims
    const int c = __popc(claims);
    int tot;
    const int ex = wg_excl_scan(c, scan_tmp, &tot);
    if (threadIdx.x == 0 && tot) base_s = atomicAdd(&M.fcnt[lvl + 1], tot);
    __syncthreads();
    int o = (tot ? base_s : 0) + ex;
#pragma unroll
    for (int j = 0; j < FP_BFS_ROW; j++)
      if ((claims >> j) & 1u) nxt[o++] = u[j];
    // the rare longer rows: the remaining neighbours in lock step
    const int dmax = (int)wave_max_u32((uint32_t)deg);
    for (int j = FP_BFS_ROW; j < dmax; j++) {
      bool claim = false;
      int w = 0;
      if (j < deg) {
        w = M.gci[e0 + j];
        if (M.key[w] > kv) claim = atomicMin(&M.key[w], kv) == FP_UNSET;
      }
      const int slot = wave_append(&M.fcnt[lvl + 1], claim);
      if (claim) nxt[slot] = w;
    }
  }
}
// Levels past the last launched one, in one workgroup: a level at a time
// with a barrier between levels, until a frontier comes out empty (a BFS has
// fewer than n levels).  Only a BFS deeper than the launched levels does
// any work here; late frontiers are small.  The barrier between steps that
// share global memory within one workgroup: the release waits for the
// workgroup's stores and atomics (which complete in L2), the agent-scope
// acquire invalidates this CU's L1 so the next loads read L2.  No release
// at agent scope: that would write back the whole L2 of the XCD at every
// step, and nothing outside the workgroup reads these arrays before the
// kernel ends.
__device__ __forceinline__ void wg_level_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __syncthreads();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
}
// Levels of a BFS launched one by one before the tail takes over: one and a
// half times the side of a patch of S vertices on a triangle mesh, plus six,
// at most 64 (the growth from hashed seeds on the 1024 x 1024 torus at
// S = 512 takes 34 levels, the regrowth after Lloyd's step 27); the distance
// BFS of Lloyd's step runs inside patches (the side plus four).
__host__ __device__ __forceinline__ int fp_bfs_levels(int n, int S, bool inner) {
  int r = 1;
  while ((long long)r * r < (long long)S && r < 64) r++;
  const int L = inner ? r + 4 : (3 * r) / 2 + 6;
  return L < 64 ? (L < n ? L : n) : (64 < n ? 64 : n);
}
__global__ void __launch_bounds__(1024) k_bfs_tail(const FpMesh* __restrict__ fp_ms, const int* __restrict__ fp_boff, int fp_nm, int inner) {
  MESH_WG;
  const int lvl0 = fp_bfs_levels(M.n, M.S, inner != 0);
  wg_level_barrier();
  for (int lvl = lvl0; lvl < M.n + 15; lvl++) {
    const int nf = M.fcnt[lvl];
    if (nf == 0) break;
    gptr<const int> cur = (lvl & 1) ? M.fb : M.fa;
    gptr<int> nxt = (lvl & 1) ? M.fa : M.fb;
    for (int f = threadIdx.x; f < nf; f += blockDim.x) {
      const int v = cur[f];
      const unsigned long long kv = M.key[v] + (1ull << 32);
      for (int e = M.grp[v]; e < M.grp[v + 1]; e++) {
        const int u = M.gci[e];
        if (M.key[u] > kv && atomicMin(&M.key[u], kv) == FP_UNSET)
          nxt[atomicAdd(&M.fcnt[lvl + 1], 1)] = u;
      }
    }
    wg_level_barrier();
  }
}
__global__ void k_count_unset(const FpMesh* __restrict__ fp_ms, const int* __restrict__ fp_boff, int fp_nm) {
  MESH;
  int cnt = 0;
  for (int v = vt(fp_s); v < M.n; v += vs(fp_s)) cnt += (M.key[v] == FP_UNSET);
  cnt = wave_sum_i32(cnt);
  if (lane_id() == 0 && cnt) atomicAdd(&C->norphan, cnt);
}
// components without a seed: min-label fixed point, then ids P0 + rank of
// the component's lowest vertex
// Every kernel of this pass returns at once when growth left no vertex
// unlabelled.  Rounds of hooking and pointer jumping run as separate
// launches while the previous round changed a label; a one-workgroup tail
// finishes any component the rounds did not settle.
__global__ void k_cc_init(const FpMesh* __restrict__ fp_ms, const int* __restrict__ fp_boff, int fp_nm) {
  MESH;
  const bool any = C->norphan > 0;
  if (vt(fp_s) == 0) C->ccn = any ? M.n : 0;
  if (!any) return;
  for (int v = vt(fp_s); v < M.n; v += vs(fp_s)) M.fb[v] = (M.key[v] == FP_UNSET) ? v : -1;
}
__device__ __forceinline__ bool cc_hook_pass(const FpMesh& M, int i0, int di) {
  gptr<int> comp = M.fb;
  bool ch = false;
  for (int v = i0; v < M.n; v += di) {
    const int cv = comp[v];
    if (cv < 0) continue;
    for (int e = M.grp[v]; e < M.grp[v + 1]; e++) {
      const int cu = comp[M.gci[e]];
      if (cu >= 0 && cu < cv) {
        atomicMin(&comp[cv], cu);  // hook the larger label under the smaller
        atomicMin(&comp[v], cu);
        ch = true;
      }
    }
  }
  return ch;
}
__device__ __forceinline__ bool cc_jump_pass(const FpMesh& M, int i0, int di) {
  gptr<int> comp = M.fb;
  bool ch = false;
  for (int v = i0; v < M.n; v += di) {
    if (comp[v] < 0) continue;
    int c = comp[v];
    while (comp[c] != c) c = comp[c];
    if (c != comp[v]) {
      comp[v] = c;
      ch = true;
    }
  }
  return ch;
}
// round r runs while round r-1 changed something
__device__ __forceinline__ bool cc_round_live(gptr<FpCtl> C, int r) {
  return C->norphan > 0 && (r == 0 || C->ccchg[r - 1] != 0);
}
__global__ void k_cc_hook(const FpMesh* __restrict__ fp_ms, const int* __restrict__ fp_boff, int fp_nm, int r) {
  MESH;
  if (!cc_round_live(C, r)) return;
  if (cc_hook_pass(M, vt(fp_s), vs(fp_s))) atomicOr(&C->ccchg[r], 1);
}
__global__ void k_cc_jump(const FpMesh* __restrict__ fp_ms, const int* __restrict__ fp_boff, int fp_nm, int r) {
  MESH;
  if (!cc_round_live(C, r)) return;
  if (cc_jump_pass(M, vt(fp_s), vs(fp_s))) atomicOr(&C->ccchg[r], 1);
}
__global__ void __launch_bounds__(1024) k_cc_tail(const FpMesh* __restrict__ fp_ms, const int* __restrict__ fp_boff, int fp_nm, int r0) {
  MESH_WG;
  __shared__ int chg;
  if (!cc_round_live(C, r0)) return;
  if (threadIdx.x == 0) chg = 0;
  wg_level_barrier();
  while (true) {
    bool ch = cc_hook_pass(M, threadIdx.x, blockDim.x);
    wg_level_barrier();
    ch |= cc_jump_pass(M, threadIdx.x, blockDim.x);
    if (ch) atomicOr(&chg, 1);
    wg_level_barrier();
    const int c = chg;
    __syncthreads();  // every lane has read the flag before it is cleared
    if (threadIdx.x == 0) chg = 0;
    if (!c) break;
  }
}
__global__ void k_cc_flags(const FpMesh* __restrict__ fp_ms, const int* __restrict__ fp_boff, int fp_nm) {
  MESH;
  if (C->norphan == 0) return;
  for (int v = vt(fp_s); v < M.n; v += vs(fp_s)) M.pcnt[v] = (M.fb[v] == v) ? 1 : 0;
}
// ids P0 + rank of the component's lowest vertex; P grows by the count
__global__ void k_cc_label(const FpMesh* __restrict__ fp_ms, const int* __restrict__ fp_boff, int fp_nm) {
  MESH;
  if (C->norphan == 0) return;
  const int P0 = C->P0;
  for (int v = vt(fp_s); v < M.n; v += vs(fp_s)) {
    const int c = M.fb[v];
    if (c < 0) continue;
    const int id = P0 + M.pcnt[c];
    M.key[v] = (unsigned long long)id;
    if (c == v) M.seeds[id] = v;
  }
  if (vt(fp_s) == 0) C->P = P0 + C->nroot;
}
// Lloyd re-centre: new seed = vertex farthest from the patch boundary (the
// distance inside the patch equals the distance to the boundary set of the
// whole graph, because any path out of a patch passes its own boundary
// first), ties to the lowest id; patches without a boundary keep their seed.
__global__ void k_lloyd_gmap(const FpMesh* __restrict__ fp_ms, const int* __restrict__ fp_boff, int fp_nm) {
  MESH;
  const int P = C->P;
  for (int v = vt(fp_s); v < M.n; v += vs(fp_s)) M.gmap[v] = (int)(M.key[v] & 0xFFFFFFFFu);
  for (int p = vt(fp_s); p < P; p += vs(fp_s)) M.best[p] = 0;
  for (int i = vt(fp_s); i < M.n + 16; i += vs(fp_s)) M.fcnt[i] = 0;
}
// (the loops below step a whole workgroup at a time: wg_append holds a
// barrier, and a single list counter takes one atomic per workgroup)
// Patch-boundary flags of the vertices v = v0 + FP_WG k + threadIdx.x
// (k < FP_BND_K): bit k is set when v < n has a neighbour in another patch;
// g[k] is v's patch (0 past n).  The loads of a step go out together for
// all FP_BND_K vertices: patches and row ranges, the first FP_BFS_ROW
// columns of each row, then their patches.
#define FP_BND_K 8
__device__ __forceinline__ uint32_t boundary_flags(const FpMesh& M, int v0, int (&g)[FP_BND_K]) {
  int e0[FP_BND_K], dg[FP_BND_K];
#pragma unroll
  for (int k = 0; k < FP_BND_K; k++) {
    const int v = v0 + FP_WG * k + (int)threadIdx.x;
    const bool act = v < M.n;
    g[k] = act ? (int)M.gmap[v] : 0;
    e0[k] = act ? (int)M.grp[v] : 0;
    dg[k] = act ? (int)M.grp[v + 1] - e0[k] : 0;
  }
  int q[FP_BND_K][FP_BFS_ROW];
#pragma unroll
  for (int k = 0; k < FP_BND_K; k++)
#pragma unroll
    for (int j = 0; j < FP_BFS_ROW; j++) q[k][j] = j < dg[k] ? (int)M.gci[e0[k] + j] : -1;
#pragma unroll
  for (int k = 0; k < FP_BND_K; k++)
#pragma unroll
    for (int j = 0; j < FP_BFS_ROW; j++) q[k][j] = q[k][j] >= 0 ? (int)M.gmap[q[k][j]] : g[k];
  uint32_t fl = 0;
#pragma unroll
  for (int k = 0; k < FP_BND_K; k++) {
    bool b = false;
#pragma unroll
    for (int j = 0; j < FP_BFS_ROW; j++) b |= q[k][j] != g[k];
    for (int e = e0[k] + FP_BFS_ROW; e < e0[k] + dg[k] && !b; e++) b = M.gmap[M.gci[e]] != g[k];
    fl |= (uint32_t)b << k;
  }
  return fl;
}
// The flagged vertices of a step appended to list[*ctr]: one atomic per
// workgroup and step.  Every thread calls it (barriers inside).
template <class P, class L>
__device__ __forceinline__ void wg_append_flags(P ctr, L list, int v0, uint32_t fl, int* tmp, int* base_s) {
  int tot;
  const int ex = wg_excl_scan(popc32(fl), tmp, &tot);
  if (threadIdx.x == 0 && tot) *base_s = atomicAdd(ctr, tot);
  __syncthreads();
  if (!tot) return;
  int o = *base_s + ex;
#pragma unroll
  for (int k = 0; k < FP_BND_K; k++)
    if ((fl >> k) & 1u) list[o++] = v0 + FP_WG * k + (int)threadIdx.x;
}
// Lloyd step: the patch-boundary vertices start the distance BFS
__global__ void __launch_bounds__(FP_WG) k_lloyd_bnd(const FpMesh* __restrict__ fp_ms, const int* __restrict__ fp_boff, int fp_nm) {
  MESH_WG;
  __shared__ int tmp[FP_WAVES + 2];
  __shared__ int base_s;
  // the workgroup steps together (barriers in each step)
  for (int v0 = fp_s.bx * (FP_BND_K * FP_WG); v0 < M.n; v0 += fp_s.gx * (FP_BND_K * FP_WG)) {
    int g[FP_BND_K];
    const uint32_t fl = boundary_flags(M, v0, g);
#pragma unroll
    for (int k = 0; k < FP_BND_K; k++) {
      const int v = v0 + FP_WG * k + (int)threadIdx.x;
      if (v < M.n) M.key[v] = ((fl >> k) & 1u) ? 0ull : FP_UNSET;
    }
    wg_append_flags(&M.fcnt[0], M.fa, v0, fl, tmp, &base_s);
  }
}
// per patch, the candidate of largest distance (least vertex on ties); the
// lanes of a wave that share a patch take their maximum first, so a patch
// gets one atomic per wave instead of one per vertex
__global__ void k_lloyd_best(const FpMesh* __restrict__ fp_ms, const int* __restrict__ fp_boff, int fp_nm) {
  MESH;
  for (int v0 = vw(fp_s) * 64; v0 < M.n; v0 += vn(fp_s) * 64) {
    const int v = v0 + lane_id();
    const unsigned long long k = v < M.n ? M.key[v] : FP_UNSET;
    const bool act = k != FP_UNSET;
    const unsigned long long cand =
        act ? (((k >> 32) << 32) | (unsigned long long)(0xFFFFFFFFu - (unsigned)v) | (1ull << 63))
            : 0ull;
    const int g = act ? M.gmap[v] : -1;
    uint64_t pend = ballot64(act);
    while (pend) {
      const int l = __builtin_ctzll(pend);
      const int kg = wave_bcast(g, l);
      const uint64_t same = ballot64(g == kg) & pend;
      const unsigned long long mx = wave_max_u64(((same >> lane_id()) & 1ull) ? cand : 0ull);
      if (lane_id() == l) atomicMax(&M.best[kg], mx);
      pend &= ~same;
    }
  }
}
__global__ void k_lloyd_seed(const FpMesh* __restrict__ fp_ms, const int* __restrict__ fp_boff, int fp_nm) {
  MESH;
  const int P = C->P;
  for (int p = vt(fp_s); p < P; p += vs(fp_s)) {
    const unsigned long long bb = M.best[p];
    if (bb) M.seeds[p] = (int)(0xFFFFFFFFu - (unsigned)(bb & 0xFFFFFFFFu));
  }
}
__global__ void k_gmap_final(const FpMesh* __restrict__ fp_ms, const int* __restrict__ fp_boff, int fp_nm) {
  MESH;
  const int P = C->P;
  for (int v = vt(fp_s); v < M.n; v += vs(fp_s)) {
    const unsigned long long k = M.key[v];
    const int g = k == FP_UNSET ? -1 : (int)(k & 0xFFFFFFFFu);
    if (g < 0 || g >= P) fp_fail(C, FP_E_INTERNAL, FP_SITE_GMAP_LABEL, v);
    M.gmap[v] = (g < 0 || g >= P) ? 0 : g;
  }
}
__global__ void k_user_gmap(const FpMesh* __restrict__ fp_ms, const int* __restrict__ fp_boff, int fp_nm) {
  MESH;
  int mx = 0;
  for (int v = vt(fp_s); v < M.n; v += vs(fp_s)) {
    int g = M.user_gmap[v];
    if (g < 0 || g >= M.n) {
      fp_fail(C, FP_E_GMAP, FP_SITE_USER_GMAP, v);
      g = 0;
    }
    M.gmap[v] = g;
    mx = max(mx, g + 1);
  }
  mx = (int)wave_max_u32((uint32_t)mx);
  if (lane_id() == 0 && mx > 0) atomicMax(&C->P, mx);
}

// ==========================================================================
// patch members, boundary list, quotient graph (Sec. 2; built once, Sec. 5)
// ==========================================================================
__global__ void k_quot_init(const FpMesh* __restrict__ fp_ms, const int* __restrict__ fp_boff, int fp_nm) {
  MESH;
  const int P = min(C->P, M.n);
  for (int p = vt(fp_s); p <= P; p += vs(fp_s)) M.pcnt[p] = 0;
  if (vt(fp_s) == 0) C->nbnd = 0;
}
// patch sizes and the boundary list
__global__ void __launch_bounds__(FP_WG) k_patch_count(const FpMesh* __restrict__ fp_ms, const int* __restrict__ fp_boff, int fp_nm) {
  MESH_WG;
  __shared__ int tmp[FP_WAVES + 2];
  __shared__ int base_s;
  // the workgroup steps together (barriers in each step)
  for (int v0 = fp_s.bx * (FP_BND_K * FP_WG); v0 < M.n; v0 += fp_s.gx * (FP_BND_K * FP_WG)) {
    int g[FP_BND_K];
    const uint32_t fl = boundary_flags(M, v0, g);
#pragma unroll
    for (int k = 0; k < FP_BND_K; k++)
      (void)wave_append_keyed(M.pcnt, g[k], v0 + FP_WG * k + (int)threadIdx.x < M.n);
    wg_append_flags(&C->nbnd, M.bnd, v0, fl, tmp, &base_s);
  }
}
__global__ void k_patch_scatter(const FpMesh* __restrict__ fp_ms, const int* __restrict__ fp_boff, int fp_nm) {
  MESH;
  for (int v0 = vw(fp_s) * 64; v0 < M.n; v0 += vn(fp_s) * 64) {
    const int v = v0 + lane_id();
    const bool act = v < M.n;
    const int slot = wave_append_keyed(M.pcnt, act ? M.gmap[v] : 0, act);
    if (act) M.pvtx[slot] = v;
  }
}
// Quotient row of patch p: the sorted distinct patches next to it, one
// workgroup per patch.  With an LDS bitmap over the patch ids (bm_words
// words) the workgroup's threads mark the neighbours of the members, a row's
// loads issued together, and wave 0 reads the bitmap back in order; without
// it, wave 0 takes the smallest unseen neighbour patch per pass (a wave-wide
// minimum over the foreign neighbours of the members).
__global__ void __launch_bounds__(FP_WG) k_qrow(const FpMesh* __restrict__ fp_ms, const int* __restrict__ fp_boff, int fp_nm, int fill, int lds_words) {
  MESH_WG;
  FP_LDS_DECL;
  const int P = C->P;
  const int bm_words = (P + 31) / 32 <= lds_words ? (P + 31) / 32 : 0;
  uint32_t* bm = (uint32_t*)fp_lds;
  // the workgroup steps together (barriers in each step)
  for (int p = fp_s.bx; p < P; p += fp_s.gx) {
    const int a0 = M.pptr[p], a1 = M.pptr[p + 1];
    gptr<int> out = fill ? M.qci + M.qptr[p] : gptr<int>(nullptr);
    if (bm_words) {
      for (int w = threadIdx.x; w < bm_words; w += FP_WG) bm[w] = 0u;
      __syncthreads();
      for (int i = a0 + (int)threadIdx.x; i < a1; i += FP_WG) {
        const int v = M.pvtx[i];
        const int e0 = M.grp[v], deg = M.grp[v + 1] - e0;
        int u[FP_BFS_ROW];
#pragma unroll
        for (int j = 0; j < FP_BFS_ROW; j++) u[j] = j < deg ? (int)M.gci[e0 + j] : -1;
#pragma unroll
        for (int j = 0; j < FP_BFS_ROW; j++) {
          const int q = u[j] >= 0 ? (int)M.gmap[u[j]] : p;
          if (q != p) atomicOr(&bm[q >> 5], 1u << (q & 31));
        }
        for (int j = FP_BFS_ROW; j < deg; j++) {
          const int q = M.gmap[M.gci[e0 + j]];
          if (q != p) atomicOr(&bm[q >> 5], 1u << (q & 31));
        }
      }
      __syncthreads();
      if (wave_id() == 0) {
        int cnt = 0;
        for (int w0 = 0; w0 < bm_words; w0 += 64) {
          const int w = w0 + lane_id();
          uint32_t x = w < bm_words ? bm[w] : 0u;
          const int c = popc32(x);
          const int inc = wave_incl_scan(c);
          if (out) {
            int o = cnt + inc - c;
            while (x) {
              out[o++] = w * 32 + __ffs(x) - 1;
              x &= x - 1;
            }
          }
          cnt += wave_bcast(inc, 63);
        }
        if (!fill && lane_id() == 0) M.pcnt[p] = cnt;
      }
      __syncthreads();  // the bitmap is cleared for the next patch
    } else if (wave_id() == 0) {
      int cnt = 0, last = -1;
      while (true) {
        uint32_t m = 0xFFFFFFFFu;
        for (int i = a0 + lane_id(); i < a1; i += 64) {
          const int v = M.pvtx[i];
          for (int e = M.grp[v]; e < M.grp[v + 1]; e++) {
            const int q = M.gmap[M.gci[e]];
            if (q != p && q > last && (uint32_t)q < m) m = (uint32_t)q;
          }
        }
        m = wave_min_u32(m);
        if (m == 0xFFFFFFFFu) break;
        if (out && lane_id() == 0) out[cnt] = (int)m;
        cnt++;
        last = (int)m;
      }
      if (!fill && lane_id() == 0) M.pcnt[p] = cnt;
    }
  }
}

__global__ void k_check_arcs(const FpMesh* __restrict__ fp_ms, const int* __restrict__ fp_boff, int fp_nm) {
  MESH;
  if (vt(fp_s) == 0 && (C->nq < 0 || (long long)C->nq > M.Ecap))
    fp_fail(C, FP_E_SCRATCH, FP_SITE_QARCS, C->nq);
}

// ==========================================================================
// separator tree (Sec. 4.2 Step 3; Alg. 2; Sec. 5).  Level d: recount the
// alive quotient arcs from the boundary list, bisect every node of depth d,
// SuperSeparator (unmarked vertices with an unmarked neighbour across) and
// RefineSeparator (keep the smaller side, ties to the left).
// ==========================================================================
__global__ void k_sep_init(const FpMesh* __restrict__ fp_ms, const int* __restrict__ fp_boff, int fp_nm) {
  MESH;
  const int P = C->P;
  int D = 0;
  while ((1ll << D) < P) D++;
  // the recursion stops after nd_level levels (Sec. 4.2 Step 3)
  if (M.nd_level >= 0 && M.nd_level < D) D = M.nd_level;
  const int nn = (1 << (D + 1)) - 1;
  if (nn > M.NNcap) {  // never expected: NNcap holds the tree of n patches
    if (vt(fp_s) == 0) fp_fail(C, FP_E_SCRATCH, FP_SITE_TREE, nn);
    return;
  }
  if (vt(fp_s) == 0) {
    C->D = D;
    C->nn = nn;
  }
  for (int v = vt(fp_s); v < M.n; v += vs(fp_s)) M.node_of[v] = -1;
  for (int p = vt(fp_s); p < P; p += vs(fp_s)) {
    M.pnode[p] = 0;
    M.plist[p] = p;
  }
  for (int x = vt(fp_s); x < nn; x += vs(fp_s)) {
    M.cntL[x] = 0;
    M.cntR[x] = 0;
    M.segN[x] = 0;
    M.segS[x] = 0;
  }
  if (vt(fp_s) == 0) M.segN[0] = P;
}
// level d of the tree: alive arcs recounted from zero
__device__ __forceinline__ void lv_begin(const FpMesh& M, gptr<FpCtl> C, int d, int i0, int di) {
  (void)d;
  const int nq = min(C->nq, (int)M.Ecap);
  for (int a = i0; a < nq; a += di) M.qcnt[a] = 0;
}
__global__ void k_level_begin(const FpMesh* __restrict__ fp_ms, const int* __restrict__ fp_boff, int fp_nm, int d) {
  MESH;
  if (d >= C->D) return;
  lv_begin(M, C, d, vt(fp_s), vs(fp_s));
}
// arcs of a quotient row held in registers for the arc lookups of lv_arcs
#define FP_ARC_ROW 16
__device__ __forceinline__ void lv_arcs(const FpMesh& M, gptr<FpCtl> C, int d, int i0, int di) {
  (void)d;
  const int nb = C->nbnd;
  for (int i = i0; i < nb; i += di) {
    const int v = M.bnd[i];
    if (M.node_of[v] != -1) continue;
    const int gv = M.gmap[v];
    const int e0 = M.grp[v], deg = M.grp[v + 1] - e0;
    const int q0 = M.qptr[gv], qn = M.qptr[gv + 1] - q0;
    // the first FP_BFS_ROW neighbours' columns, marks and patches at once,
    // and v's quotient row (FP_ARC_ROW arcs) beside them: an arc is then
    // found by comparing in registers instead of a search of dependent loads
    int u[FP_BFS_ROW], nu[FP_BFS_ROW], gu[FP_BFS_ROW], qc[FP_ARC_ROW];
#pragma unroll
    for (int j = 0; j < FP_BFS_ROW; j++) u[j] = j < deg ? (int)M.gci[e0 + j] : -1;
#pragma unroll
    for (int k = 0; k < FP_ARC_ROW; k++) qc[k] = k < qn ? (int)M.qci[q0 + k] : -1;
#pragma unroll
    for (int j = 0; j < FP_BFS_ROW; j++) {
      nu[j] = u[j] >= 0 ? (int)M.node_of[u[j]] : 0;
      gu[j] = u[j] >= 0 ? (int)M.gmap[u[j]] : gv;
    }
#pragma unroll
    for (int j = 0; j < FP_BFS_ROW; j++) {
      if (nu[j] != -1 || gu[j] == gv) continue;
      int a = -1;
      if (qn <= FP_ARC_ROW) {
#pragma unroll
        for (int k = 0; k < FP_ARC_ROW; k++) a = qc[k] == gu[j] ? q0 + k : a;
      } else {
        a = arc_index(M, gv, gu[j]);
      }
      if (a >= 0) atomicAdd(&M.qcnt[a], 1);
    }
    for (int e = e0 + FP_BFS_ROW; e < e0 + deg; e++) {
      const int w = M.gci[e];
      if (M.node_of[w] != -1) continue;
      const int gw = M.gmap[w];
      if (gw == gv) continue;
      const int a = arc_index(M, gv, gw);
      if (a >= 0) atomicAdd(&M.qcnt[a], 1);
    }
  }
}
__global__ void k_arcs(const FpMesh* __restrict__ fp_ms, const int* __restrict__ fp_boff, int fp_nm, int d) {
  MESH;
  if (d >= C->D) return;
  lv_arcs(M, C, d, vt(fp_s), vs(fp_s));
}
__global__ void __launch_bounds__(FP_WG) k_bisect(const FpMesh* __restrict__ fp_ms, const int* __restrict__ fp_boff, int fp_nm, int d,
                                                   int lds_bytes) {
  MESH_WG;
  __shared__ BisectLds sh;
  FP_LDS_DECL;
  if (d >= C->D) return;
  const int lo = (1 << d) - 1, hi = (1 << (d + 1)) - 1;
  for (int t = lo + fp_s.bx; t < hi; t += fp_s.gx) {
    const int m = M.segN[t];
    if (m >= 2) wg_bisect(M, t, M.segS[t], m, &sh, fp_lds, lds_bytes);
  }
}
// Candidates of level d, counted per node and side.  The lanes of a wave
// hold consecutive indices (i0 and di as the callers pass them), so the loop
// runs wave by wave and a wave adds its candidates with one atomic per node
// and side present in it (at the root every candidate shares one counter).
__device__ __forceinline__ void lv_cand(const FpMesh& M, gptr<FpCtl> C, int d, int i0, int di) {
  const int hi = (1 << (d + 1)) - 1;
  const int nb = C->nbnd;
  for (int i = i0; i - lane_id() < nb; i += di) {
    bool is = false;
    int c = 0;
    if (i < nb) {
      const int v = M.bnd[i];
      c = M.node_of[v] == -1 ? (int)M.pnode[M.gmap[v]] : 0;
      if (c >= hi) {  // else the patch is not split at this level
        const int sib = (c & 1) ? c + 1 : c - 1;
        const int e0 = M.grp[v], deg = M.grp[v + 1] - e0;
        // the first FP_BFS_ROW neighbours' columns, marks and patches at once
        int u[FP_BFS_ROW], nu[FP_BFS_ROW], gu[FP_BFS_ROW];
#pragma unroll
        for (int j = 0; j < FP_BFS_ROW; j++) u[j] = j < deg ? (int)M.gci[e0 + j] : -1;
#pragma unroll
        for (int j = 0; j < FP_BFS_ROW; j++) {
          nu[j] = u[j] >= 0 ? (int)M.node_of[u[j]] : 0;
          gu[j] = u[j] >= 0 ? (int)M.gmap[u[j]] : 0;
        }
#pragma unroll
        for (int j = 0; j < FP_BFS_ROW; j++) is |= nu[j] == -1 && M.pnode[gu[j]] == sib;
        for (int e = e0 + FP_BFS_ROW; e < e0 + deg && !is; e++) {
          const int w = M.gci[e];
          is = (M.node_of[w] == -1 && M.pnode[M.gmap[w]] == sib);
        }
      }
      M.cand[i] = is ? 1 : 0;
    }
    const int t = is ? (c - 1) >> 1 : 0;
    (void)wave_append_keyed(M.cntL, t, is && (c & 1));
    (void)wave_append_keyed(M.cntR, t, is && !(c & 1));
  }
}
__global__ void k_cand(const FpMesh* __restrict__ fp_ms, const int* __restrict__ fp_boff, int fp_nm, int d) {
  MESH;
  if (d >= C->D) return;
  lv_cand(M, C, d, vt(fp_s), vs(fp_s));
}
__device__ __forceinline__ void lv_mark(const FpMesh& M, gptr<FpCtl> C, int d, int i0, int di) {
  (void)d;
  if (M.refine) return;  // the refinement marked the level
  const int nb = C->nbnd;
  for (int i = i0; i < nb; i += di) {
    if (!M.cand[i]) continue;
    const int v = M.bnd[i];
    const int c = M.pnode[M.gmap[v]];
    const int t = (c - 1) >> 1;
    const bool left = c & 1;
    const bool mark_left = M.cntL[t] <= M.cntR[t];
    if (left == mark_left) {
      M.node_of[v] = t;
      atomicSub(&M.wp[M.gmap[v]], 1);
    }
  }
}
__global__ void k_mark(const FpMesh* __restrict__ fp_ms, const int* __restrict__ fp_boff, int fp_nm, int d) {
  MESH;
  if (d >= C->D) return;
  lv_mark(M, C, d, vt(fp_s), vs(fp_s));
}
// --------------------------------------------------------------------------
// Refined separators (Sec. 5, separator refinement).  The sides of a split
// follow the patches, so a separator of node t is any set of candidates
// touching every crossing edge: a vertex cover of the bipartite crossing
// graph.  The smallest has the size of a maximum matching (Konig).  The one
// taken starts from side s (the side the one-sided rule marks): with Z the
// vertices reachable from the s-vertices a maximum matching leaves free,
// along alternating paths, the cover is (s-candidates outside Z) plus
// (other-side candidates in Z).  Z is the same for every maximum matching
// (Dulmage-Mendelsohn), so the parallel matching below, whose matching
// depends on timing, still gives a unique separator.
// --------------------------------------------------------------------------

// exclusive scan of the level's candidate counts into roff/rcur (one
// workgroup; sh: FP_WG ints of LDS)
__device__ __forceinline__ void lv_ref_place(const FpMesh& M, int d, int* sh) {
  const int lo = (1 << d) - 1, cnt = 1 << d;
  const int tid = (int)threadIdx.x, nt = (int)blockDim.x;
  const int chunk = (cnt + nt - 1) / nt;
  const int a = min(cnt, tid * chunk), b = min(cnt, a + chunk);
  int sum = 0;
  for (int x = a; x < b; x++) sum += M.cntL[lo + x] + M.cntR[lo + x];
  sh[tid] = sum;
  __syncthreads();
  if (tid == 0) {
    int run = 0;
    for (int i = 0; i < nt; i++) {
      const int v = sh[i];
      sh[i] = run;
      run += v;
    }
  }
  __syncthreads();
  int run = sh[tid];
  for (int x = a; x < b; x++) {
    M.roff[lo + x] = run;
    M.rcur[lo + x] = run;
    run += M.cntL[lo + x] + M.cntR[lo + x];
  }
  __syncthreads();
}
// every candidate into its node's segment; matching state cleared
__device__ __forceinline__ void lv_ref_scatter(const FpMesh& M, gptr<FpCtl> C, int d, int i0,
                                               int di) {
  (void)d;
  const int nb = C->nbnd;
  // lanes of a wave take consecutive entries (i0 is the lane's thread index,
  // di a multiple of 64), so one atomic per node and wave suffices
  for (int b = i0 - lane_id(); b < nb; b += di) {
    const int i = b + lane_id();
    const bool act = i < nb && M.cand[i];
    const int v = act ? M.bnd[i] : 0;
    const int t = act ? (M.pnode[M.gmap[v]] - 1) >> 1 : 0;
    const int slot = wave_append_keyed(M.rcur, t, act);
    if (act) {
      M.rlist[slot] = v;
      M.mate[v] = -1;
      M.seen[v] = 0;
    }
  }
}
// Node t by one workgroup: greedy matching, then phases of a breadth-first
// search from all free s-vertices at once that stop at the first level with
// free other-side vertices; one shortest augmenting path per search tree is
// flipped (the trees are vertex-disjoint).  A phase that finds none has
// reached exactly Z.  sh: 16 ints of LDS.
__device__ void wg_refine_node(const FpMesh& M, gptr<FpCtl> C, int t, int* sh) {
  const int k = M.cntL[t] + M.cntR[t];
  if (k == 0) return;
  const int k0 = M.roff[t];
  const int s_child = M.cntL[t] <= M.cntR[t] ? 2 * t + 1 : 2 * t + 2;
  const int o_child = (s_child & 1) ? s_child + 1 : s_child - 1;
  const gptr<int> L = M.rlist + k0;
  gptr<int> fa = M.rqa + k0, fb = M.rqb + k0;
  const int tid = (int)threadIdx.x, nt = (int)blockDim.x;
  auto other = [&](int u) { return M.node_of[u] == -1 && M.pnode[M.gmap[u]] == o_child; };
  auto s_side = [&](int v) { return M.pnode[M.gmap[v]] == s_child; };
  // greedy start: each s-vertex takes its first free neighbour across
  for (int i = tid; i < k; i += nt) {
    const int v = L[i];
    if (!s_side(v)) continue;
    for (int e = M.grp[v]; e < M.grp[v + 1]; e++) {
      const int u = M.gci[e];
      if (other(u) && atomicCAS(&M.mate[u], -1, v) == -1) {
        M.mate[v] = u;
        break;
      }
    }
  }
  wg_level_barrier();
  int stamp = 0;
  bool ok = true;
  while (true) {
    if (++stamp > k + 2) {  // each phase grows the matching: never expected
      ok = false;
      break;
    }
    if (tid == 0) {
      sh[0] = 0;  // frontier
      sh[2] = 0;  // free other-side vertices reached
    }
    __syncthreads();
    for (int i = tid; i < k; i += nt) {
      const int v = L[i];
      if (!s_side(v) || M.mate[v] != -1) continue;
      M.seen[v] = stamp;
      M.rpar[v] = -1;
      const int j = atomicAdd(&sh[0], 1);
      if (j < k) fa[j] = v;
    }
    wg_level_barrier();
    int nf = sh[0];
    while (nf > 0) {
      __syncthreads();
      if (tid == 0) sh[1] = 0;
      __syncthreads();
      for (int i = tid; i < nf; i += nt) {
        const int x = fa[i];
        const int mx = M.mate[x];
        for (int e = M.grp[x]; e < M.grp[x + 1]; e++) {
          const int u = M.gci[e];
          if (u == mx || !other(u)) continue;
          if (atomicMax(&M.seen[u], stamp) >= stamp) continue;  // reached already
          M.rpar[u] = x;
          const int y = M.mate[u];
          if (y == -1) {
            // endpoints fill the next frontier's buffer from its end: the
            // s-vertices appended from the front and the free vertices
            // reached are at most k together
            const int j = atomicAdd(&sh[2], 1);
            if (j < k) fb[k - 1 - j] = u;
          } else {
            M.seen[y] = stamp;
            M.rpar[y] = u;
            const int j = atomicAdd(&sh[1], 1);
            if (j < k) fb[j] = y;  // at most once per s-vertex: never past k
          }
        }
      }
      wg_level_barrier();
      if (sh[2] > 0) break;  // the shortest augmenting paths end at this level
      nf = sh[1];
      if (nf > k) {
        ok = false;
        break;
      }
      const gptr<int> tmp = fa;
      fa = fb;
      fb = tmp;
    }
    if (!ok) break;
    const int nep = min(sh[2], k);
    if (nep == 0) break;  // no augmenting path: the last search reached Z
    for (int j = tid; j < nep; j += nt) {
      const int end = fb[k - 1 - j];
      // paths alternate: an other-side vertex's predecessor is an s-vertex,
      // an s-vertex's is the other-side vertex matched to it (or -1: root);
      // both walks are bounded by the node's size
      int x = M.rpar[end], steps = 0;
      while (x >= 0 && M.rpar[x] != -1 && steps++ <= k) x = M.rpar[M.rpar[x]];
      if (x < 0 || steps > k) {
        fp_fail(C, FP_E_INTERNAL, FP_SITE_REFINE, t);
        continue;
      }
      // one path per search tree: the first to claim the root flips its path
      if (atomicCAS(&M.seen[x], stamp, -stamp) != stamp) continue;
      steps = 0;
      for (int u = end; u != -1 && steps++ <= k;) {
        const int y = M.rpar[u];
        const int next = M.rpar[y];
        M.mate[u] = y;
        M.mate[y] = u;
        u = next;
      }
    }
    wg_level_barrier();
  }
  if (!ok) {
    if (tid == 0) fp_fail(C, FP_E_INTERNAL, FP_SITE_REFINE, t);
    return;
  }
  for (int i = tid; i < k; i += nt) {
    const int v = L[i];
    const bool in_z = M.seen[v] == stamp;
    if (s_side(v) ? !in_z : in_z) {
      M.node_of[v] = t;
      atomicSub(&M.wp[M.gmap[v]], 1);
    }
  }
  wg_level_barrier();
}
// The same for a node small enough for one wave's LDS slice: the crossing
// graph in local candidate indices (CSR), matching, search stamps and
// predecessors all in LDS, each step wave-synchronous.  A candidate's local
// index is kept in rpar[v] while the adjacency is built.  Words of LDS:
// matching, stamps, predecessors, two frontiers and the endpoints of a
// phase's augmenting paths (6k), offsets (k + 1), the crossing entries and
// two counters.  Every phase flips one path per search tree that reached a
// free vertex, all of them.
__device__ __forceinline__ long long ref_wave_words(int k, long long ecross) {
  return 7ll * k + 1 + ecross + 2;
}
// crossing entries of node t (the sum of its candidates' graph degrees
// bounds them)
__device__ __forceinline__ long long ref_deg_sum(const FpMesh& M, int t) {
  const int k = M.cntL[t] + M.cntR[t], k0 = M.roff[t];
  long long e = 0;
  for (int i = lane_id(); i < k; i += 64) {
    const int v = M.rlist[k0 + i];
    e += M.grp[v + 1] - M.grp[v];
  }
  return wave_sum_i64(e);
}
__device__ void wave_refine_node(const FpMesh& M, gptr<FpCtl> C, int t, int* lds, long long ecap) {
  const int k = uni(M.cntL[t] + M.cntR[t]);
  const int k0 = uni(M.roff[t]);
  const int lane = lane_id();
  const int s_child = uni(M.cntL[t] <= M.cntR[t] ? 2 * t + 1 : 2 * t + 2);
  const int o_child = (s_child & 1) ? s_child + 1 : s_child - 1;
  const gptr<int> L = M.rlist + k0;
  int* mate = lds;
  int* seen = mate + k;
  int* par = seen + k;
  int* fr = par + k;       // two frontiers of k
  int* ep = fr + 2 * k;    // k endpoints
  int* off = ep + k;       // k + 1
  int* adj = off + k + 1;  // ecap
  int* cnt = adj + ecap;   // 2 counters
  auto side_of = [&](int v) { return M.pnode[M.gmap[v]]; };
  // local indices, then the crossing adjacency
  for (int i = lane; i < k; i += 64) M.rpar[L[i]] = i;
  wave_fence();
  int run = 0;
  for (int c = 0; c < k; c += 64) {
    const int i = c + lane;
    int n = 0;
    if (i < k) {
      const int v = L[i];
      const int oth = side_of(v) == s_child ? o_child : s_child;
      for (int e = M.grp[v]; e < M.grp[v + 1]; e++) {
        const int u = M.gci[e];
        n += M.node_of[u] == -1 && side_of(u) == oth;
      }
    }
    const int inc = wave_incl_scan(n);
    if (i < k) off[i] = run + inc - n;
    run += wave_bcast(inc, 63);
  }
  if (lane == 0) off[k] = run;
  wave_fence();
  for (int i = lane; i < k; i += 64) {
    const int v = L[i];
    const int oth = side_of(v) == s_child ? o_child : s_child;
    int q = off[i];
    for (int e = M.grp[v]; e < M.grp[v + 1]; e++) {
      const int u = M.gci[e];
      if (M.node_of[u] == -1 && side_of(u) == oth) adj[q++] = M.rpar[u];
    }
    mate[i] = -1;
    seen[i] = 0;
  }
  wave_fence();
  auto s_loc = [&](int i) { return side_of(L[i]) == s_child; };
  // greedy start
  for (int i = lane; i < k; i += 64) {
    if (!s_loc(i)) continue;
    for (int q = off[i]; q < off[i + 1]; q++)
      if (atomicCAS(&mate[adj[q]], -1, i) == -1) {
        mate[i] = adj[q];
        break;
      }
  }
  wave_fence();
  int stamp = 0;
  bool ok = true;
  while (true) {
    if (++stamp > k + 2) {  // each phase grows the matching: never expected
      ok = false;
      break;
    }
    int* fa = fr;
    int* fb = fr + k;
    int nf = 0;
    for (int c = 0; c < k; c += 64) {
      const int i = c + lane;
      const bool f = i < k && s_loc(i) && mate[i] == -1;
      const uint64_t bal = ballot64(f);
      if (f) {
        seen[i] = stamp;
        par[i] = -1;
        fa[nf + popc64(bal & lanemask_lt())] = i;
      }
      nf += popc64(bal);
    }
    if (lane == 0) cnt[1] = 0;  // endpoints found
    wave_fence();
    int nep = 0;
    while (nf > 0) {
      if (lane == 0) cnt[0] = 0;
      wave_fence();
      for (int c = 0; c < nf; c += 64) {
        const int f = c + lane;
        if (f >= nf) continue;
        const int x = fa[f];
        const int mx = mate[x];
        for (int q = off[x]; q < off[x + 1]; q++) {
          const int j = adj[q];
          if (j == mx) continue;
          if (atomicMax(&seen[j], stamp) >= stamp) continue;  // reached already
          par[j] = x;
          const int y = mate[j];
          if (y == -1) {
            const int e = atomicAdd(&cnt[1], 1);
            if (e < k) ep[e] = j;  // each free vertex once: never past k
          } else {
            seen[y] = stamp;
            par[y] = j;
            const int s2 = atomicAdd(&cnt[0], 1);
            if (s2 < k) fb[s2] = y;  // at most once per s-vertex: never past k
          }
        }
      }
      wave_fence();
      nep = uni(cnt[1]);
      if (nep > 0) break;  // the shortest augmenting paths end at this level
      nf = uni(cnt[0]);
      if (nf > k) {
        ok = false;
        break;
      }
      int* tmp = fa;
      fa = fb;
      fb = tmp;
    }
    if (!ok) break;
    nep = min(nep, k);
    if (nep == 0) break;  // no augmenting path: the last search reached Z
    for (int j = lane; j < nep; j += 64) {
      const int end = ep[j];
      int x = par[end], steps = 0;
      while (x >= 0 && par[x] != -1 && steps++ <= k) x = par[par[x]];
      if (x >= 0 && steps <= k && atomicCAS(&seen[x], stamp, -stamp) == stamp) {
        steps = 0;
        for (int u = end; u != -1 && steps++ <= k;) {
          const int y = par[u];
          const int next = par[y];
          mate[u] = y;
          mate[y] = u;
          u = next;
        }
      } else if (x < 0 || steps > k) {
        fp_fail(C, FP_E_INTERNAL, FP_SITE_REFINE, t);
      }
    }
    wave_fence();
  }
  if (!ok) {
    if (lane == 0) fp_fail(C, FP_E_INTERNAL, FP_SITE_REFINE, t);
    return;
  }
  for (int i = lane; i < k; i += 64) {
    const bool in_z = seen[i] == stamp;
    if (s_loc(i) ? !in_z : in_z) {
      const int v = L[i];
      M.node_of[v] = t;
      atomicSub(&M.wp[M.gmap[v]], 1);
    }
  }
  wave_fence();
}
// Which path refines node t: 0 a wave with a quarter of the per-node LDS,
// 1 a wave with the whole large LDS, 2 a workgroup in global memory.
__device__ __forceinline__ int ref_path(const FpMesh& M, long long words) {
  if (words <= M.lds_bytes / 4 / FP_WAVES) return 0;
  return words <= M.lds_big / 4 ? 1 : 2;
}
// nodes of path cls (0: four waves per workgroup, 1: one wave per
// workgroup of 64 threads), a wave each
__global__ void __launch_bounds__(FP_WG) k_refine_w(const FpMesh* __restrict__ fp_ms, const int* __restrict__ fp_boff, int fp_nm, int d, int cls) {
  MESH;
  FP_LDS_DECL;
  if (d >= C->D || !M.refine) return;
  const int lw = cls == 0 ? M.lds_bytes / 4 / FP_WAVES : M.lds_big / 4;
  int* lds = (int*)fp_lds + (cls == 0 ? lw * wave_id() : 0);
  const int lo = (1 << d) - 1, cnt = 1 << d;
  for (int x = vw(fp_s); x < cnt; x += vn(fp_s)) {
    const int t = lo + x;
    const int k = uni(M.cntL[t] + M.cntR[t]);
    if (k == 0) continue;
    const long long ec = ref_deg_sum(M, t);
    if (ref_path(M, ref_wave_words(k, ec)) == cls) wave_refine_node(M, C, t, lds, ec);
  }
}
__global__ void __launch_bounds__(FP_WG) k_ref_place(const FpMesh* __restrict__ fp_ms, const int* __restrict__ fp_boff, int fp_nm, int d) {
  MESH_WG;
  __shared__ int sh[FP_WG];
  if (d >= C->D || !M.refine) return;
  lv_ref_place(M, d, sh);
}
__global__ void k_ref_scatter(const FpMesh* __restrict__ fp_ms, const int* __restrict__ fp_boff, int fp_nm, int d) {
  MESH;
  if (d >= C->D || !M.refine) return;
  lv_ref_scatter(M, C, d, vt(fp_s), vs(fp_s));
}
__global__ void __launch_bounds__(FP_WG) k_refine(const FpMesh* __restrict__ fp_ms, const int* __restrict__ fp_boff, int fp_nm, int d) {
  MESH_WG;
  __shared__ int sh[16];
  if (d >= C->D || !M.refine) return;
  const int lo = (1 << d) - 1, hi = (2 << d) - 1;
  for (int t = lo + fp_s.bx; t < hi; t += fp_s.gx) {
    // nodes that fit a wave's LDS were refined by k_refine_w
    const int k = M.cntL[t] + M.cntR[t];
    if (k == 0) continue;
    long long ec = 0;
    if (threadIdx.x < 64) ec = ref_deg_sum(M, t);
    if (threadIdx.x == 0) sh[2] = ref_path(M, ref_wave_words(k, ec));
    __syncthreads();
    const int path = sh[2];
    __syncthreads();
    if (path == 2) wg_refine_node(M, C, t, sh);
  }
}
// One tree level in one workgroup: the steps of the level's separate
// launches in turn, with a barrier between steps.  Used for the levels past
// the expected depth, which only inputs with more patches than ⌈n/S⌉ (orphan
// components, more user groups) reach; for every other input it returns at
// once, one launch instead of five.
__device__ __forceinline__ void level_wg(const FpMesh& M, gptr<FpCtl> C, int d, BisectLds& sh,
                                         char* fp_lds, int lds_bytes) {
  const int i0 = (int)threadIdx.x, di = (int)blockDim.x;
  wg_level_barrier();
  lv_begin(M, C, d, i0, di);
  wg_level_barrier();
  lv_arcs(M, C, d, i0, di);
  wg_level_barrier();
  const int lo = (1 << d) - 1, hi = (1 << (d + 1)) - 1;
  for (int t = lo; t < hi; t++) {
    const int m = M.segN[t];
    if (m >= 2) wg_bisect(M, t, M.segS[t], m, &sh, fp_lds, lds_bytes);
  }
  wg_level_barrier();
  lv_cand(M, C, d, i0, di);
  wg_level_barrier();
  if (M.refine) {
    // the refinement's scratch comes from the dynamic LDS (the bisection
    // above is done with it)
    int* rsh = (int*)fp_lds;
    lv_ref_place(M, d, rsh);
    wg_level_barrier();
    lv_ref_scatter(M, C, d, i0, di);
    wg_level_barrier();
    for (int t = lo; t < hi; t++) wg_refine_node(M, C, t, rsh);
  } else {
    lv_mark(M, C, d, i0, di);
  }
}
// every level past the expected depth of the mesh, in turn (one launch)
__global__ void __launch_bounds__(FP_WG) k_level_wg(const FpMesh* __restrict__ fp_ms, const int* __restrict__ fp_boff, int fp_nm,
                                                    int lds_bytes) {
  MESH0;
  __shared__ BisectLds sh;
  __shared__ unsigned go;
  FP_LDS_DECL;
  for (int d = M.dexp + 1;; d++) {
    __syncthreads();
    if (threadIdx.x == 0) go = C->err == 0 && d < C->D;
    __syncthreads();
    if (!go) return;
    level_wg(M, C, d, sh, fp_lds, lds_bytes);
  }
}
// leaves keep the remaining vertices of their patch
__global__ void k_leaves(const FpMesh* __restrict__ fp_ms, const int* __restrict__ fp_boff, int fp_nm) {
  MESH;
  for (int v = vt(fp_s); v < M.n; v += vs(fp_s))
    if (M.node_of[v] == -1) M.node_of[v] = M.pnode[M.gmap[v]];
}

// ==========================================================================
// grouping in schedule order (Alg. 3)
// ==========================================================================
__global__ void k_nsize(const FpMesh* __restrict__ fp_ms, const int* __restrict__ fp_boff, int fp_nm) {
  MESH;
  const int nn = C->nn;
  for (int x = vt(fp_s); x < nn; x += vs(fp_s)) M.nsize[x] = 0;
  for (int v = vt(fp_s); v < M.n; v += vs(fp_s)) {
    if ((unsigned)M.node_of[v] >= (unsigned)nn) {  // never expected
      fp_fail(C, FP_E_INTERNAL, FP_SITE_NODE_OF, v);
      M.node_of[v] = 0;
    }
  }
}
// Node sizes and the scatter into node ranges, one contiguous chunk of
// vertices per workgroup: counts gather in an LDS histogram of the nodes
// (hcap entries; past that, per-wave keyed appends), and each workgroup
// adds its non-zero counts with one global atomic per node, so the top
// separators, whose vertices run through every chunk, take one atomic per
// workgroup instead of one per wave.
__device__ __forceinline__ void chunk_of(const FpSlot& s, int n, int* v0, int* v1) {
  const int ch = (n + s.gx - 1) / s.gx;
  *v0 = min(n, s.bx * ch);
  *v1 = min(n, *v0 + ch);
}
__global__ void __launch_bounds__(FP_WG) k_nsize_count(const FpMesh* __restrict__ fp_ms, const int* __restrict__ fp_boff, int fp_nm, int hcap) {
  MESH_WG;
  FP_LDS_DECL;
  const int nn = C->nn;
  int v0, v1;
  chunk_of(fp_s, M.n, &v0, &v1);
  if (nn > hcap) {
    for (int b = v0 + (int)threadIdx.x - lane_id(); b < v1; b += (int)blockDim.x) {
      const int v = b + lane_id();
      const bool act = v < v1;
      (void)wave_append_keyed(M.nsize, act ? M.node_of[v] : 0, act);
    }
    return;
  }
  int* h = (int*)fp_lds;
  for (int i = threadIdx.x; i < nn; i += blockDim.x) h[i] = 0;
  __syncthreads();
  for (int v = v0 + (int)threadIdx.x; v < v1; v += (int)blockDim.x) atomicAdd(&h[M.node_of[v]], 1);
  __syncthreads();
  for (int i = threadIdx.x; i < nn; i += blockDim.x)
    if (h[i]) atomicAdd(&M.nsize[i], h[i]);
}
__global__ void k_sched_place(const FpMesh* __restrict__ fp_ms, const int* __restrict__ fp_boff, int fp_nm) {
  MESH;
  const int nn = C->nn, D = C->D;
  for (int x = vt(fp_s); x < nn; x += vs(fp_s)) M.sbuf[sched_pos(x, D, M.sched)] = M.nsize[x];
}
__global__ void k_nbegin(const FpMesh* __restrict__ fp_ms, const int* __restrict__ fp_boff, int fp_nm) {
  MESH;
  const int nn = C->nn, D = C->D;
  for (int x = vt(fp_s); x < nn; x += vs(fp_s)) {
    const int b = M.sbuf[sched_pos(x, D, M.sched)];
    M.nbegin[x] = b;
    M.ncur[x] = b;
  }
}
// (the order of a node's vertices in its range does not matter: the local
// orders sort them by id)
__global__ void __launch_bounds__(FP_WG) k_scatter(const FpMesh* __restrict__ fp_ms, const int* __restrict__ fp_boff, int fp_nm, int hcap) {
  MESH_WG;
  FP_LDS_DECL;
  const int nn = C->nn;
  int v0, v1;
  chunk_of(fp_s, M.n, &v0, &v1);
  if (nn > hcap) {
    for (int b = v0 + (int)threadIdx.x - lane_id(); b < v1; b += (int)blockDim.x) {
      const int v = b + lane_id();
      const bool act = v < v1;
      const int slot = wave_append_keyed(M.ncur, act ? M.node_of[v] : 0, act);
      if (act) M.gbuf[slot] = v;
    }
    return;
  }
  // this chunk's counts, then one reservation per node, then the slots
  int* h = (int*)fp_lds;
  for (int i = threadIdx.x; i < nn; i += blockDim.x) h[i] = 0;
  __syncthreads();
  for (int v = v0 + (int)threadIdx.x; v < v1; v += (int)blockDim.x) atomicAdd(&h[M.node_of[v]], 1);
  __syncthreads();
  for (int i = threadIdx.x; i < nn; i += blockDim.x)
    if (h[i]) h[i] = atomicAdd(&M.ncur[i], h[i]);
  __syncthreads();
  for (int v = v0 + (int)threadIdx.x; v < v1; v += (int)blockDim.x) M.gbuf[atomicAdd(&h[M.node_of[v]], 1)] = v;
}

// ==========================================================================
// Reuse of an earlier call's local orders (update calls, patches kept): the
// local order of a node depends only on its vertex set and the edges among
// them (minimum degree with ties to the lowest local index, the rank of the
// vertex id), so a node whose vertex set and induced edges are both
// unchanged takes the earlier order as it is.  One wave per node; flags in
// segS (free once the tree is built) tell the task lists to skip it.
// ==========================================================================
__global__ void k_reuse(const FpMesh* __restrict__ fp_ms, const int* __restrict__ fp_boff, int fp_nm) {
  MESH;
  const FpMesh* O = M.prev;
  if (!O) return;
  const int nn = C->nn;
  const bool same = O->n == M.n && O->b == M.b && O->ctl->nn == nn && O->ctl->err == 0u;
  for (int t = vw(fp_s); t < nn; t += vn(fp_s)) {
    const int m = uni((int)M.nsize[t]);
    bool ok = same && m > 0 && O->nsize[t] == m;
    const int pos = uni((int)M.nbegin[t]);
    // the same vertices: every member was in node t before, and as many
    for (int k = lane_id(); ok && k < m; k += 64) ok = O->node_of[M.gbuf[pos + k]] == t;
    ok = ballot64(!ok) == 0;
    // the same induced edges: each member's row, restricted to the node, is
    // the same sorted list in both graphs
    for (int k = lane_id(); ok && k < m; k += 64) {
      const int v = M.gbuf[pos + k];
      int a = M.grp[v], ae = M.grp[v + 1], b = O->grp[v], be = O->grp[v + 1];
      while (ok) {
        while (a < ae && M.node_of[M.gci[a]] != t) a++;
        while (b < be && O->node_of[O->gci[b]] != t) b++;
        if (a == ae || b == be) {
          ok = a == ae && b == be;
          break;
        }
        ok = M.gci[a] == O->gci[b];
        a++;
        b++;
      }
    }
    ok = ballot64(!ok) == 0;
    if (ok) {
      const int opos = O->nbegin[t];
      for (int k = lane_id(); k < m; k += 64) {
        const int v = O->vperm[opos + k];
        M.vperm[pos + k] = v;
        M.viperm[v] = pos + k;
      }
      if (lane_id() == 0) atomicAdd(&C->vreuse, m);
    }
    if (lane_id() == 0) M.segS[t] = ok ? 1 : 0;
  }
}

// ==========================================================================
// local orders (Sec. 4.3 Step 4): one wave per node, LDS slice per wave
// ==========================================================================
// Task lists of the local orders, one per size class, largest nodes first
// (a counting sort on size / 16, one workgroup of 1024 threads, one per
// class and bucket): a class with more nodes than resident slots then ends
// with its smallest nodes, not its largest.
#define FP_TASK_BUCKETS 256
__global__ void __launch_bounds__(1024) k_md_tasks(const FpMesh* __restrict__ fp_ms, const int* __restrict__ fp_boff, int fp_nm, int ntop) {
  MESH_WG;
  const int nn = C->nn;
  __shared__ int hist[FP_MD_CLASSES * FP_TASK_BUCKETS];
  __shared__ int cmax[FP_MD_CLASSES];  // largest node of each class's slice
  __shared__ int wsum[32];
  for (int i = threadIdx.x; i < FP_MD_CLASSES * FP_TASK_BUCKETS; i += blockDim.x) hist[i] = 0;
  if (threadIdx.x < FP_MD_CLASSES)
    cmax[threadIdx.x] = md_bit_max(md_slice_bytes(threadIdx.x, M.lds_bytes, M.lds_md));
  if (threadIdx.x < 8) C->task_pop[threadIdx.x] = 0;
  __syncthreads();
  auto key = [&](int x) -> int {  // class * buckets + bucket, or -1
    const int m = M.nsize[x];
    if (m == 0 || (x < ntop && C->tearly[x])) return -1;  // top separators ordered already
    if (M.prev && M.segS[x]) return -1;                  // order reused
    const int c = m <= cmax[3] ? 3 : m <= cmax[2] ? 2 : m <= cmax[1] ? 1 : 0;
    return c * FP_TASK_BUCKETS + (FP_TASK_BUCKETS - 1) - min(m >> 4, FP_TASK_BUCKETS - 1);
  };
  for (int x = threadIdx.x; x < nn; x += blockDim.x) {
    const int k = key(x);
    if (k >= 0) atomicAdd(&hist[k], 1);
  }
  __syncthreads();
  // exclusive scan of each class's buckets: one thread per bucket (the
  // 1024 threads cover the four classes' 256 buckets), waves then classes
  {
    const int i = threadIdx.x;
    const int v = hist[i];
    const int inc = wave_incl_scan(v);
    if (lane_id() == 63) wsum[wave_id()] = inc;
    __syncthreads();
    // waves 4c .. 4c + 3 hold class c
    const int w = wave_id(), c0 = w & ~3;
    int before = 0;
    for (int q = c0; q < w; q++) before += wsum[q];
    hist[i] = before + inc - v;
    if ((w & 3) == 3 && lane_id() == 63) C->task_cnt[w >> 2] = before + inc;
  }
  __syncthreads();
  for (int x = threadIdx.x; x < nn; x += blockDim.x) {
    const int k = key(x);
    if (k >= 0) M.tasks[(k / FP_TASK_BUCKETS) * M.NNcap + atomicAdd(&hist[k], 1)] = x;
  }
}
__global__ void __launch_bounds__(FP_WG) k_md(const FpMesh* __restrict__ fp_ms, const int* __restrict__ fp_boff, int fp_nm, int c) {
  MESH;
  FP_LDS_DECL;
  const int nsl = md_slice_waves(c);
  const long long sb = uni(md_slice_bytes(c, M.lds_bytes, M.lds_md));
  const int cnt = uni(C->task_cnt[c]);
  if (wave_id() >= nsl) return;
  char* slice = fp_lds + sb * wave_id();
  while (true) {
    int k = 0;
    if (lane_id() == 0) k = atomicAdd(&C->task_pop[c], 1);
    k = wave_bcast(k, 0);
    if (k >= cnt) break;
    md_node(M, uni(M.tasks[c * M.NNcap + k]), slice, sb);
  }
}

// The top separators (depth < FP_TOP_LEVELS) are final as soon as their tree
// level is marked, and their level-order ranges follow from the sizes of the
// top levels alone: depth d fills the positions just before all shallower
// nodes, in heap order.  Their local orders, the longest serial chains of
// the stage, then run on a second stream while the rest of the tree and the
// grouping proceed.
// (counts and slots of the few depth-d nodes in an LDS array per chunk of
// vertices, as in k_nsize_count and k_scatter)
__global__ void __launch_bounds__(FP_WG) k_top_count(const FpMesh* __restrict__ fp_ms, const int* __restrict__ fp_boff, int fp_nm, int d) {
  MESH_WG;
  __shared__ int hc[1 << FP_TOP_LEVELS];
  if (d >= C->D) return;
  const int lo = (1 << d) - 1, cnt = 1 << d;
  int v0, v1;
  chunk_of(fp_s, M.n, &v0, &v1);
  if ((int)threadIdx.x < cnt) hc[threadIdx.x] = 0;
  __syncthreads();
  for (int v = v0 + (int)threadIdx.x; v < v1; v += (int)blockDim.x) {
    const int x = M.node_of[v] - lo;
    if (x >= 0 && x < cnt) atomicAdd(&hc[x], 1);
  }
  __syncthreads();
  if ((int)threadIdx.x < cnt && hc[threadIdx.x]) atomicAdd(&C->tcnt[lo + threadIdx.x], hc[threadIdx.x]);
}
__global__ void k_top_place(const FpMesh* __restrict__ fp_ms, const int* __restrict__ fp_boff, int fp_nm, int d) {
  MESH;
  if (vt(fp_s) != 0 || d >= C->D) return;
  const int lo = (1 << d) - 1, cnt = 1 << d;
  // A node that held a single patch at its level is a leaf: it gets that
  // patch's unmarked vertices only after the tree is done, and it also
  // shifts the ranges of all deeper levels.  Early orders stop there.
  for (int i = 0; i < cnt; i++)
    if (M.segN[lo + i] == 1) C->top_stop = 1;
  if (C->top_stop) return;
  int tot = 0;
  for (int i = 0; i < cnt; i++) tot += C->tcnt[lo + i];
  const int shallow = C->top_shallow;
  int pos = M.n - shallow - tot, off = shallow;
  for (int i = 0; i < cnt; i++) {
    const int t = lo + i;
    C->tpos[t] = pos;
    C->toff[t] = off;
    C->tcur[t] = off;
    C->tearly[t] = 1;
    pos += C->tcnt[t];
    off += C->tcnt[t];
  }
  C->top_shallow = shallow + tot;
}
__global__ void __launch_bounds__(FP_WG) k_top_scatter(const FpMesh* __restrict__ fp_ms, const int* __restrict__ fp_boff, int fp_nm, int d) {
  MESH_WG;
  __shared__ int hc[1 << FP_TOP_LEVELS];
  if (C->top_stop || d >= C->D) return;
  const int lo = (1 << d) - 1, cnt = 1 << d;
  int v0, v1;
  chunk_of(fp_s, M.n, &v0, &v1);
  if ((int)threadIdx.x < cnt) hc[threadIdx.x] = 0;
  __syncthreads();
  for (int v = v0 + (int)threadIdx.x; v < v1; v += (int)blockDim.x) {
    const int x = M.node_of[v] - lo;
    if (x >= 0 && x < cnt) atomicAdd(&hc[x], 1);
  }
  __syncthreads();
  if ((int)threadIdx.x < cnt && hc[threadIdx.x]) hc[threadIdx.x] = atomicAdd(&C->tcur[lo + threadIdx.x], hc[threadIdx.x]);
  __syncthreads();
  for (int v = v0 + (int)threadIdx.x; v < v1; v += (int)blockDim.x) {
    const int x = M.node_of[v] - lo;
    if (x >= 0 && x < cnt) M.tbuf[atomicAdd(&hc[x], 1)] = v;
  }
}
// one wave (and the whole LDS) per depth-d node
__global__ void __launch_bounds__(64) k_md_top(const FpMesh* __restrict__ fp_ms, const int* __restrict__ fp_boff, int fp_nm, int d) {
  MESH;
  FP_LDS_DECL;
  if (d >= uni(C->D)) return;
  const int t = uni((1 << d) - 1 + fp_s.bx);
  if (!uni(C->tearly[t])) return;
  const int m = uni(C->tcnt[t]), off = uni(C->toff[t]), pos0 = uni(C->tpos[t]);
  if (off < 0 || m < 0 || (long long)off + m > M.n) {
    if (lane_id() == 0) fp_fail(C, FP_E_INTERNAL, FP_SITE_TOP, t);
    return;
  }
  md_node_list(M, t, M.tbuf + off, m, pos0, fp_lds, uni(M.lds_md));
}
// the schedule's ranges must be the ones the early orders took
__global__ void k_top_check(const FpMesh* __restrict__ fp_ms, const int* __restrict__ fp_boff, int fp_nm, int ntop) {
  MESH;
  ntop = min(ntop, C->nn);
  for (int t = vt(fp_s); t < ntop; t += vs(fp_s))
    if (C->tearly[t] &&
        (M.nsize[t] != C->tcnt[t] || (M.nsize[t] > 0 && M.nbegin[t] != C->tpos[t])))
      fp_fail(C, FP_E_INTERNAL, FP_SITE_TOP, t);
}

// ==========================================================================
// elimination tree and column counts, bottom-up over the tree levels
// ==========================================================================
// The pool holds one level's node scratch at a time and the arena of parity
// d & 1 the records level d emits: the counters are reset with no launch of
// their own.  The pool's by the kernel before the first level (k_prow_deg),
// then by each level's emission (which allocates nothing; the scratch it
// reads stays in place, and the next level's prep allocates only after it);
// the arena's by the prep of level d (which reads the other parity, and
// which the emission of level d follows).
__global__ void __launch_bounds__(FP_WG) k_sym_prep(const FpMesh* __restrict__ fp_ms, const int* __restrict__ fp_boff, int fp_nm, int d) {
  MESH;
  FP_LDS_DECL;
  if (d > C->D) return;
  if (vt(fp_s) == 0) C->arena_top[d & 1] = 0;
  const int lw = M.lds_bytes / 4 / FP_WAVES;
  int* slice = (int*)fp_lds + lw * wave_id();
  const int lo = (1 << d) - 1, cnt = 1 << d;
  for (int x = vw(fp_s); x < cnt; x += vn(fp_s)) sym_prep(M, lo + x, d, slice, lw);
}
// Elimination of the nodes whose queue links and forward rows fit in an LDS
// slice: cls 0 with four waves per workgroup (a quarter of the per-node LDS
// each), cls 1 with one wave owning the large slice.
__global__ void __launch_bounds__(FP_WG) k_sym_elim(const FpMesh* __restrict__ fp_ms, const int* __restrict__ fp_boff, int fp_nm, int d, int cls) {
  MESH;
  FP_LDS_DECL;
  if (d > C->D) return;
  const int nsl = cls == 0 ? FP_WAVES : 1;
  if (wave_id() >= nsl) return;
  int* slice = (int*)fp_lds + (M.lds_bytes / 4 / nsl) * wave_id();
  const int lo = (1 << d) - 1, cnt = 1 << d;
  const int wv = uni(fp_s.bx * nsl + wave_id()), nw = fp_s.gx * nsl;
  const long long lw = cls == 0 ? M.lds_bytes / 4 / nsl : M.lds_big / 4;
  for (int x = wv; x < cnt; x += nw) sym_elim<true>(M, lo + x, cls, slice, lw);
}
// nodes too large for the whole LDS: links and rows in global memory
__global__ void __launch_bounds__(FP_WG) k_sym_elim_glb(const FpMesh* __restrict__ fp_ms, const int* __restrict__ fp_boff, int fp_nm, int d) {
  MESH;
  if (d > C->D) return;
  const int lo = (1 << d) - 1, cnt = 1 << d;
  for (int x = vw(fp_s); x < cnt; x += vn(fp_s)) sym_elim<false>(M, lo + x, 2, nullptr, 0);
}
__global__ void __launch_bounds__(FP_WG) k_sym_emit(const FpMesh* __restrict__ fp_ms, const int* __restrict__ fp_boff, int fp_nm, int d) {
  MESH;
  if (d > C->D) return;
  if (vt(fp_s) == 0) C->pool_top = 0;  // for the next level's prep
  const int lo = (1 << d) - 1, cnt = 1 << d;
  for (int x = vw(fp_s); x < cnt; x += vn(fp_s)) sym_emit(M, lo + x, d);
}
// One symbolic level in one workgroup (four waves), for the levels past the
// expected depth: initialisation, prep, elimination of the three classes and
// emission in turn, with a barrier between steps; wave w takes nodes w, w+4,
// ... in every step, and wave 0 the large-LDS class with all of the LDS.
// every level past the expected depth of the mesh, deepest first (one
// launch); the error word and depth are shared through the dynamic LDS (the
// large class takes all of it, so no static LDS here)
__device__ __forceinline__ void sym_level_wg(const FpMesh& M, gptr<FpCtl> C, int d, char* fp_lds);
__global__ void __launch_bounds__(FP_WG) k_sym_level_wg(const FpMesh* __restrict__ fp_ms, const int* __restrict__ fp_boff, int fp_nm) {
  MESH0;
  FP_LDS_DECL;
  if (threadIdx.x == 0) *(int*)fp_lds = C->err ? -1 : C->D;
  __syncthreads();
  const int D = *(volatile int*)fp_lds;
  __syncthreads();
  for (int d = D; d > M.dexp; d--) {
    if (threadIdx.x == 0) *(unsigned*)fp_lds = C->err;
    __syncthreads();
    const unsigned err = *(volatile unsigned*)fp_lds;
    __syncthreads();
    if (err) return;
    sym_level_wg(M, C, d, fp_lds);
    wg_level_barrier();
  }
  if (threadIdx.x == 0) C->pool_top = 0;  // for the first level launched after these
}
__device__ __forceinline__ void sym_level_wg(const FpMesh& M, gptr<FpCtl> C, int d, char* fp_lds) {
  if (threadIdx.x == 0) {
    C->arena_top[d & 1] = 0;
    C->pool_top = 0;
  }
  wg_level_barrier();
  const int lo = (1 << d) - 1, cnt = 1 << d;
  const int lw = M.lds_bytes / 4 / FP_WAVES;
  int* slice = (int*)fp_lds + lw * wave_id();
  const int w0 = uni(wave_id());
  for (int x = w0; x < cnt; x += FP_WAVES) sym_prep(M, lo + x, d, slice, lw);
  wg_level_barrier();
  for (int x = w0; x < cnt; x += FP_WAVES) sym_elim<true>(M, lo + x, 0, slice, lw);
  wg_level_barrier();
  if (w0 == 0)
    for (int x = 0; x < cnt; x++) sym_elim<true>(M, lo + x, 1, (int*)fp_lds, M.lds_big / 4);
  wg_level_barrier();
  for (int x = w0; x < cnt; x += FP_WAVES) sym_elim<false>(M, lo + x, 2, nullptr, 0);
  wg_level_barrier();
  for (int x = w0; x < cnt; x += FP_WAVES) sym_emit(M, lo + x, d);
}
// The permuted pattern by position, for the symbolic stage: row p lists the
// positions of the neighbours of vertex vperm[p].  One pass with a thread per
// position; the symbolic kernels then read contiguous rows instead of
// chasing vperm -> row pointers -> columns -> viperm per entry.
__global__ void k_prow_deg(const FpMesh* __restrict__ fp_ms, const int* __restrict__ fp_boff, int fp_nm) {
  MESH;
  if (vt(fp_s) == 0) C->pool_top = 0;  // the local orders are done with the pool
  for (int p = vt(fp_s); p < M.n; p += vs(fp_s)) {
    const int v = M.vperm[p];
    M.pcnt[p] = (unsigned)v < (unsigned)M.n ? M.grp[v + 1] - M.grp[v] : 0;
  }
}
__global__ void k_prow_fill(const FpMesh* __restrict__ fp_ms, const int* __restrict__ fp_boff, int fp_nm) {
  MESH;
  for (int p = vt(fp_s); p < M.n; p += vs(fp_s)) {
    const int v = M.vperm[p];
    if ((unsigned)v >= (unsigned)M.n) continue;
    const int o = M.prow[p], e0 = M.grp[v], deg = M.grp[v + 1] - e0;
    if (deg <= 0) continue;
    // the first FP_BFS_ROW columns, then their positions, loaded together
    // (indices past the row re-read its last entry; not stored)
    int u[FP_BFS_ROW];
#pragma unroll
    for (int j = 0; j < FP_BFS_ROW; j++) u[j] = M.gci[e0 + min(j, deg - 1)];
#pragma unroll
    for (int j = 0; j < FP_BFS_ROW; j++) u[j] = M.viperm[u[j]];
#pragma unroll
    for (int j = 0; j < FP_BFS_ROW; j++)
      if (j < deg) M.pent[o + j] = u[j];
    for (int e = FP_BFS_ROW; e < deg; e++) M.pent[o + e] = M.viperm[M.gci[e0 + e]];
  }
}
// nnz(L): the column counts summed per workgroup, one atomic each
__global__ void __launch_bounds__(FP_WG) k_nnzl(const FpMesh* __restrict__ fp_ms, const int* __restrict__ fp_boff, int fp_nm) {
  MESH_WG;
  __shared__ long long part[FP_WAVES];
  long long s = 0;
  for (int i = vt(fp_s); i < M.n; i += vs(fp_s)) s += M.vcc[i];
  s = wave_sum_i64(s);
  if (lane_id() == 0) part[wave_id()] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    long long t = 0;
    for (int w = 0; w < FP_WAVES; w++) t += part[w];
    if (t) atomicAdd((unsigned long long*)&C->nnzL, (unsigned long long)t);
  }
}

// ==========================================================================
// block expansion and outputs (Sec. 6.5)
// ==========================================================================
__global__ void k_expand(const FpMesh* __restrict__ fp_ms, const int* __restrict__ fp_boff, int fp_nm) {
  MESH;
  const int nn = C->nn;
  const int b = M.b;
  const long long nd = M.n_dof;
  for (long long j = vt(fp_s); j < nd; j += vs(fp_s)) {
    const int k = (int)(j / b), r = (int)(j - (long long)k * b);
    M.perm[j] = M.vperm[k] * b + r;
    M.iperm[j] = M.viperm[k] * b + r;
    M.colcount[j] = b * M.vcc[k] - r;
    M.parent[j] = r < b - 1 ? (int)(j + 1) : (M.vpar[k] < 0 ? -1 : M.vpar[k] * b);
  }
  if (M.gmap_out)
    for (int v = vt(fp_s); v < M.n; v += vs(fp_s)) M.gmap_out[v] = M.gmap[v];
  if ((M.node_begin_out || M.node_size_out) && nn <= M.max_nodes_out)
    for (int x = vt(fp_s); x < nn; x += vs(fp_s)) {
      if (M.node_begin_out) M.node_begin_out[x] = M.nbegin[x] * b;
      if (M.node_size_out) M.node_size_out[x] = M.nsize[x] * b;
    }
}
__global__ void k_finish(const FpMesh* __restrict__ fp_ms, const int* __restrict__ fp_boff, int fp_nm) {
  MESH0;
  if (vt(fp_s) != 0) return;
  const int nn = C->nn;
  if ((M.node_begin_out || M.node_size_out) && nn > M.max_nodes_out)
    fp_fail(C, FP_E_SCRATCH, FP_SITE_OUT_NODES, nn);
  *M.nnzL = (long long)M.b * M.b * C->nnzL - (long long)M.n * M.b * (M.b - 1) / 2;
  if (M.n_nodes_out) *M.n_nodes_out = nn;
  if (M.status_out) *M.status_out = C->err;
  if (M.reused_out) *M.reused_out = C->vreuse;
}

// ==========================================================================
// Static scratch of fp_order_static, for callers that cannot allocate
// device memory.  Each device holds its own copy of the array, from the
// first use of the library on it until the process ends.  Host code never
// uses the array's name as an address: the device address is looked up once
// per device (fp_create) and kept in g_scratch.
// ==========================================================================
#define FP_STATIC_SCRATCH_BYTES (256ull << 20)
#define FP_MAX_DEVICES 64
static __device__ __align__(256) char scratch[FP_STATIC_SCRATCH_BYTES];
static void* g_scratch[FP_MAX_DEVICES];
static bool g_scratch_tried[FP_MAX_DEVICES];
static std::mutex g_scratch_mu;

// with `device` current: its copy of the scratch array, looked up once
static void bind_scratch(int device) {
  if (device < 0 || device >= FP_MAX_DEVICES) return;
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (g_scratch_tried[device]) return;
  g_scratch_tried[device] = true;
  void* p = nullptr;
  if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) == hipSuccess)
    g_scratch[device] = p;
  else
    (void)hipGetLastError();  // fp_order_static then reports FP_ERR_HIP
}

// ==========================================================================
// host side
// ==========================================================================
static const char* const kStageNames[FP_NSTAGE] = {
    "ingest", "patches", "quotient", "septree", "group", "local_orders", "symbolic", "expand"};

namespace {

using fpplan::fill_mesh;
using fpplan::make_plan;
using fpplan::Plan;
using fpplan::align_up;

fp_status check_opts(const fp_options* o) {
  if (!o) return FP_ERR_ARG;
  if (o->patch_size < 1 || o->block_size < 1 || o->lloyd_iters < 0 || o->lloyd_iters > 64)
    return FP_ERR_ARG;
  if (o->schedule != FP_SCHED_LEVEL && o->schedule != FP_SCHED_POST) return FP_ERR_ARG;
  if (o->nd_level < -1 || o->nd_level > 30) return FP_ERR_ARG;
  if (o->flags & ~(FP_FLAG_TIMING | FP_FLAG_VALIDATE | FP_FLAG_REFINE | FP_FLAG_AMD))
    return FP_ERR_UNSUPPORTED;
  return FP_OK;
}

fp_status check_csr(const fp_csr* A, int b) {
  if (!A) return FP_ERR_ARG;
  if (A->n < 0 || A->nnz < 0 || A->n >= (1ll << 31)) return FP_ERR_ARG;
  if (!!A->rowptr32 == !!A->rowptr64) return FP_ERR_ARG;
  if (A->nnz > 0 && !A->colind) return FP_ERR_ARG;
  if (A->rowptr32 && A->nnz >= (1ll << 31)) return FP_ERR_ARG;
  if (A->n % b) return FP_ERR_ARG;
  return FP_OK;
}

fp_status map_err(unsigned e) {
  if (e & (FP_E_INDEX | FP_E_GMAP)) return FP_ERR_INDEX;
  if (e & FP_E_ASYM) return FP_ERR_NOT_SYMMETRIC;
  if (e & FP_E_SCRATCH) return FP_ERR_SIZE;
  if (e) return FP_ERR_DEVICE;
  return FP_OK;
}

// ==========================================================================
// The pipeline on the host.  One Pipe queues Alg. 1 for one mesh or for a
// batch of meshes: every launch covers all meshes at once (each mesh gets
// the blocks it would get alone; a mesh with no part in a launch gets none).
// The same code runs twice for a batch: a planning pass records the block
// table of every launch (no HIP calls), then the launching pass reads it
// back from device memory in the same order.  Nothing is read back to the
// host: counts known only on the device (patches, tree depth, arcs,
// frontier sizes) are read by the kernels, launch grids come from
// capacities or expected values, and every kernel returns at once after an
// earlier stage raised an error.
// ==========================================================================
static int ceil_log2(long long x) {
  int d = 0;
  while ((1ll << d) < x) d++;
  return d;
}

// host-known sizes of one mesh
struct MeshPlan {
  int n;
  long long n_dof;
  int S;
  int lloyd;
  bool user;      // user groups instead of patching
  bool validate;  // symmetry check
  bool refine;    // minimum-cover separators
  int sched;      // FP_SCHED_LEVEL or FP_SCHED_POST
  int P0, Pexp;   // seed blocks; expected patch count (exact without orphans)
  int Dpat;       // ceil(log2 Pexp): a depth-d node holds about 2^(Dpat-d) patches
  int Dexp, Dmax; // expected and largest possible tree depth (P <= n; nd_level)
  int NNcap;
  int Lg, Ld;     // launched levels of the growth and distance BFS
};

MeshPlan mesh_plan(const FpMesh& M, bool user) {
  MeshPlan m;
  m.n = M.n;
  m.n_dof = M.n_dof;
  m.S = M.S;
  m.lloyd = M.lloyd;
  m.user = user;
  m.validate = M.validate != 0;
  m.refine = M.refine != 0;
  m.sched = M.sched;
  m.P0 = fp_p0(M.n, M.S);
  m.Pexp = std::max(m.P0, 1);
  m.Dpat = ceil_log2(m.Pexp);
  m.Dexp = M.dexp;  // ceil(log2 Pexp), at most nd_level
  m.Dmax = ceil_log2(std::max(M.n, 1));
  if (M.nd_level >= 0) m.Dmax = std::min(m.Dmax, M.nd_level);
  m.NNcap = M.NNcap;
  m.Lg = fp_bfs_levels(M.n, M.S, false);
  m.Ld = fp_bfs_levels(M.n, M.S, true);
  return m;
}

struct Pipe {
  fp_handle* h;
  hipStream_t st;
  std::vector<MeshPlan> mp;
  const FpMesh* dm = nullptr;  // device array of the meshes' descriptions
  FpCtl* ctl0 = nullptr;       // control block of the single mesh
  bool single = true;          // one mesh: no block table; side streams and timing allowed
  bool plan = false;           // planning pass of a batch
  std::vector<int> tab;        // block tables, launch after launch (nm + 1 ints each)
  const int* dtab = nullptr;   // their device copy (launching pass)
  size_t tpos = 0;
  bool hip_failed = false;
  bool timing = false;
  bool update = false;     // an update call: local orders may be reused
  bool fixed = false;      // no side streams and no per-kernel events (static-scratch calls)
  bool side_open = false;  // work on the side stream not yet joined
  bool side2_open = false; // same for the second side stream
  int nm() const { return (int)mp.size(); }
  int ncu() const { return h->ncu; }

  long long blk(long long items, int per = FP_WG) const {
    const long long b = (items + per - 1) / per;
    return std::max(1ll, std::min(b, 8ll * h->ncu));
  }
  // timing of one kernel (fp_time_kernel): events around each of its launches
  bool tk(const char* name) const {
    return single && !fixed && h->tk_name[0] && strcmp(h->tk_name, name) == 0;
  }
  void tk_begin(hipStream_t ls) {
    if ((int)h->tk_ev.size() < 2 * (h->tk_n + 1)) {
      hipEvent_t a, b;
      if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) {
        h->tk_failed = true;
        return;
      }
      h->tk_ev.push_back(a);
      h->tk_ev.push_back(b);
    }
    if (hipEventRecord(h->tk_ev[2 * h->tk_n], ls) != hipSuccess) h->tk_failed = true;
  }
  void tk_end(hipStream_t ls) {
    if ((int)h->tk_ev.size() < 2 * (h->tk_n + 1)) return;
    if (hipEventRecord(h->tk_ev[2 * h->tk_n + 1], ls) != hipSuccess) h->tk_failed = true;
    h->tk_n++;
  }
  void mark(int i) {
    if (single && timing && hipEventRecord(h->ev[i], st) != hipSuccess) hip_failed = true;
  }
  // One launch: bl(i) blocks for mesh i (<= 0: none).
  template <class BL, class K, class... A>
  void go(const char* name, K kern, BL bl, dim3 T, size_t lds, hipStream_t s, A... args) {
    if (single) {
      const long long b = bl(0);
      if (b <= 0) return;
      const bool t = tk(name);
      if (t) tk_begin(s);
      hipLaunchKernelGGL(kern, dim3((unsigned)b), T, lds, s, dm, (const int*)nullptr, 1, args...);
      if (t) tk_end(s);
      return;
    }
    const int n = nm();
    if (plan) {
      long long o = 0;
      tab.push_back(0);
      for (int i = 0; i < n; i++) {
        o += std::max(0ll, (long long)bl(i));
        tab.push_back((int)std::min(o, (long long)INT32_MAX));
      }
      return;
    }
    const size_t at = tpos;
    tpos += n + 1;
    if (at + n >= tab.size()) {
      hip_failed = true;
      return;
    }
    const int tot = tab[at + n];
    if (tot <= 0) return;
    hipLaunchKernelGGL(kern, dim3((unsigned)tot), T, lds, s, dm, (const int*)(dtab + at), n, args...);
  }
  void check() {
    if (!plan && hipGetLastError() != hipSuccess) hip_failed = true;
  }
  // the call's stream waits for everything issued on the side streams
  void join_side() {
    if (side_open) {
      side_open = false;
      if (hipEventRecord(h->ev_join, h->side) != hipSuccess ||
          hipStreamWaitEvent(st, h->ev_join, 0) != hipSuccess)
        hip_failed = true;
    }
    if (side2_open) {  // both large-class streams
      side2_open = false;
      if (hipEventRecord(h->ev_join2, h->side2) != hipSuccess ||
          hipEventRecord(h->ev_join3, h->side3) != hipSuccess ||
          hipStreamWaitEvent(st, h->ev_join2, 0) != hipSuccess ||
          hipStreamWaitEvent(st, h->ev_join3, 0) != hipSuccess)
        hip_failed = true;
    }
  }
  // exclusive scan of array `ain` into `aout` over count `fcnt`, total to `tdst`
  void scan(int ain, int aout, int fcnt, int tdst) {
    auto cap = [&](int i) { return fcnt == FN_NNCAP || fcnt == FN_NN ? mp[i].NNcap : mp[i].n; };
    go("k_scan_part", k_mscan_part, [&](int i) { return scan_blocks(cap(i)); }, dim3(FP_WG), 0, st,
       ain, fcnt);
    go("k_scan_top", k_mscan_top, [&](int) { return 1; }, dim3(FP_WG), 0, st, fcnt, tdst);
    go("k_scan_apply", k_mscan_apply, [&](int i) { return scan_blocks(cap(i)); }, dim3(FP_WG), 0,
       st, ain, aout, fcnt);
    check();
  }
  // Frontier BFS from the level-0 frontier already in place: each mesh's
  // launched levels (a launch past its last level finds an empty frontier
  // and returns at once), then one workgroup per mesh continues until a
  // frontier comes out empty.  `on(i)`: mesh i takes part.
  template <class ON>
  void bfs(bool inner, ON on) {
    int L = 0;
    for (int i = 0; i < nm(); i++)
      if (on(i)) L = std::max(L, inner ? mp[i].Ld : mp[i].Lg);
    for (int k = 0; k < L; k++)
      go("k_bfs_level", k_bfs_level,
         [&](int i) { return on(i) && k < (inner ? mp[i].Ld : mp[i].Lg) ? blk(mp[i].n) : 0; },
         dim3(FP_WG), 0, st, k);
    go("k_bfs_tail", k_bfs_tail, [&](int i) { return on(i) ? 1 : 0; }, dim3(1024), 0, st,
       inner ? 1 : 0);
    check();
  }
};

#define FPG(...) P.go(__VA_ARGS__)

// The side streams: three per device for the whole process, shared by every
// handle on that device and created on first use.  A device has few hardware
// queues (four by default) and every stream takes one of them in turn; once
// a process holds more streams than queues, two streams can share a queue and
// then run one after the other, so handles that each created their own side
// streams (and streams made by others in between) would lose the overlap of
// the top separators' local orders with the rest of the pipeline.  A
// handle's events stay its own, so handles on several host threads can share
// the streams (their work interleaves in stream order, with no cross-handle
// waits).
struct FpSideStreams {
  bool ok = false;
  hipStream_t s[3] = {nullptr, nullptr, nullptr};
};
static std::mutex fp_side_mu;
static FpSideStreams fp_side[FP_MAX_DEVICES];

bool ensure_side(fp_handle* h) {
  if (h->side) return true;
  if (h->device < 0 || h->device >= FP_MAX_DEVICES) return false;
  {
    std::lock_guard<std::mutex> lk(fp_side_mu);
    FpSideStreams& S = fp_side[h->device];
    if (!S.ok) {
      int ns = 0;
      while (ns < 3 && hipStreamCreateWithFlags(&S.s[ns], hipStreamNonBlocking) == hipSuccess) ns++;
      if (ns < 3) {
        for (int j = 0; j < ns; j++) (void)hipStreamDestroy(S.s[j]);
        (void)hipGetLastError();
        return false;
      }
      S.ok = true;
    }
  }
  hipEvent_t* ev[7] = {&h->ev_top[0], &h->ev_top[1], &h->ev_top[2], &h->ev_join,
                       &h->ev_md,     &h->ev_join2,  &h->ev_join3};
  int ne = 0;
  while (ne < 7 && hipEventCreateWithFlags(ev[ne], hipEventDisableTiming) == hipSuccess) ne++;
  if (ne < 7) {
    for (int j = 0; j < ne; j++) (void)hipEventDestroy(*ev[j]);
    (void)hipGetLastError();
    return false;
  }
  const FpSideStreams& S = fp_side[h->device];
  h->side = S.s[0];
  h->side2 = S.s[1];
  h->side3 = S.s[2];
  return true;
}

// Queue Alg. 1 for every mesh of the pipe.  Levels of the separator tree and
// of the symbolic stage run to each mesh's largest possible depth
// (ceil(log2 n)); levels past the expected depth get one block.
fp_status run_pipe(Pipe& P) {
  hipStream_t st = P.st;
  const int nm = P.nm();
  auto& mp = P.mp;
  const dim3 T(FP_WG);
  auto per_n = [&](int i) { return P.blk(mp[i].n); };
  auto one = [&](int) { return 1ll; };
  int Dmax = 0, Lloyd = 0;
  bool any_patch = false, any_user = false;
  for (int i = 0; i < nm; i++) {
    Dmax = std::max(Dmax, mp[i].Dmax);
    if (mp[i].user) any_user = true;
    else if (mp[i].n > 0) {
      any_patch = true;
      Lloyd = std::max(Lloyd, mp[i].lloyd);
    }
  }
  auto patching = [&](int i) { return !mp[i].user && mp[i].n > 0; };

  // ingest
  P.mark(0);
  FPG("k_ingest", k_ingest, per_n, T, 0, st, 0);
  FPG("k_ingest_long", k_ingest_long, [&](int) { return (long long)P.ncu(); }, T, 0, st, 0);
  P.scan(FA_PCNT, FA_GRP, FN_N, FT_NNZG);
  FPG("k_check_graph", k_check_graph, one, dim3(64), 0, st);
  FPG("k_mptr_end", k_mptr_end, one, dim3(64), 0, st, (int)FA_GRP, (int)FN_N, (int)FT_NNZG);
  FPG("k_ingest", k_ingest, per_n, T, 0, st, 1);
  FPG("k_ingest_long", k_ingest_long, [&](int) { return (long long)P.ncu(); }, T, 0, st, 1);
  FPG("k_validate", k_validate, [&](int i) { return mp[i].validate ? P.blk(mp[i].n) : 0; }, T, 0,
      st);
  P.check();

  // patches
  P.mark(1);
  if (any_user)
    FPG("k_user_gmap", k_user_gmap, [&](int i) { return mp[i].user ? P.blk(mp[i].n) : 0; }, T, 0,
        st);
  if (any_patch) {
    auto pn = [&](int i) { return patching(i) ? P.blk(mp[i].n) : 0; };
    FPG("k_seeds", k_seeds, [&](int i) { return patching(i) ? P.blk(mp[i].P0, FP_WAVES) : 0; }, T,
        0, st);
    FPG("k_key_unset", k_key_unset, pn, T, 0, st);
    FPG("k_seed_push", k_seed_push, [&](int i) { return patching(i) ? P.blk(mp[i].P0) : 0; }, T, 0,
        st, 0);
    P.bfs(false, patching);
    FPG("k_count_unset", k_count_unset, pn, T, 0, st);
    // components growth did not reach (none on a connected mesh: every
    // kernel here then returns at once)
    FPG("k_cc_init", k_cc_init, pn, T, 0, st);
    for (int r = 0; r < FP_CC_ROUNDS; r++) {
      FPG("k_cc_hook", k_cc_hook, pn, T, 0, st, r);
      FPG("k_cc_jump", k_cc_jump, pn, T, 0, st, r);
    }
    FPG("k_cc_tail", k_cc_tail, [&](int i) { return patching(i) ? 1 : 0; }, dim3(1024), 0, st,
        FP_CC_ROUNDS);
    FPG("k_cc_flags", k_cc_flags, pn, T, 0, st);
    {
      // only patching meshes take part in the scan of their component roots
      auto cap = [&](int i) { return patching(i) ? scan_blocks(mp[i].n) : 0; };
      FPG("k_scan_part", k_mscan_part, cap, T, 0, st, (int)FA_PCNT, (int)FN_CCN);
      FPG("k_scan_top", k_mscan_top, [&](int i) { return patching(i) ? 1 : 0; }, T, 0, st,
          (int)FN_CCN, (int)FT_NROOT);
      FPG("k_scan_apply", k_mscan_apply, cap, T, 0, st, (int)FA_PCNT, (int)FA_PCNT, (int)FN_CCN);
    }
    FPG("k_cc_label", k_cc_label, pn, T, 0, st);
    P.check();
    for (int it = 0; it < Lloyd; it++) {
      auto on = [&](int i) { return patching(i) && it < mp[i].lloyd; };
      auto ln = [&](int i) { return on(i) ? P.blk(mp[i].n) : 0; };
      FPG("k_lloyd_gmap", k_lloyd_gmap, ln, T, 0, st);
      FPG("k_lloyd_bnd", k_lloyd_bnd,
          [&](int i) { return on(i) ? P.blk(mp[i].n, FP_BND_K * FP_WG) : 0; }, T, 0, st);
      P.check();
      P.bfs(true, on);
      FPG("k_lloyd_best", k_lloyd_best, ln, T, 0, st);
      FPG("k_lloyd_seed", k_lloyd_seed, [&](int i) { return on(i) ? P.blk(mp[i].Pexp) : 0; }, T, 0,
          st);
      FPG("k_key_unset", k_key_unset, ln, T, 0, st);
      FPG("k_seed_push", k_seed_push, [&](int i) { return on(i) ? P.blk(mp[i].Pexp) : 0; }, T, 0,
          st, 1);
      P.bfs(false, on);
    }
    FPG("k_gmap_final", k_gmap_final, pn, T, 0, st);
    P.check();
  }

  // quotient graph (P on the device)
  P.mark(2);
  FPG("k_quot_init", k_quot_init, [&](int i) { return P.blk(mp[i].Pexp + 1); }, T, 0, st);
  FPG("k_patch_count", k_patch_count, [&](int i) { return P.blk(mp[i].n, FP_BND_K * FP_WG); }, T,
      0, st);
  FPG("k_copy", k_mcopy, [&](int i) { return P.blk(mp[i].Pexp); }, T, 0, st, (int)FA_WP,
      (int)FA_PCNT, (int)FN_P);
  P.check();
  P.scan(FA_PCNT, FA_PPTR, FN_P, FT_TOT);
  FPG("k_set", k_mptr_end, one, dim3(64), 0, st, (int)FA_PPTR, (int)FN_P, (int)FT_TOT);
  FPG("k_copy", k_mcopy, [&](int i) { return P.blk(mp[i].Pexp); }, T, 0, st, (int)FA_PCNT,
      (int)FA_PPTR, (int)FN_P);
  FPG("k_patch_scatter", k_patch_scatter, per_n, T, 0, st);
  // a patch-id bitmap per workgroup when it fits in 64 KB of LDS (for the
  // expected patch count; the kernel checks the actual one)
  int qbw = 0;
  for (int i = 0; i < nm; i++) {
    const int w = (mp[i].Pexp + 31) / 32;
    if ((long long)w * 4 <= 65536) qbw = std::max(qbw, w);
  }
  auto qb = [&](int i) { return P.blk(mp[i].Pexp, 1); };
  FPG("k_qrow", k_qrow, qb, T, (size_t)qbw * 4, st, 0, qbw);
  P.check();
  P.scan(FA_PCNT, FA_QPTR, FN_P, FT_NQ);
  FPG("k_set", k_mptr_end, one, dim3(64), 0, st, (int)FA_QPTR, (int)FN_P, (int)FT_NQ);
  FPG("k_check_arcs", k_check_arcs, one, dim3(64), 0, st);
  FPG("k_qrow", k_qrow, qb, T, (size_t)qbw * 4, st, 1, qbw);
  P.check();

  // separator tree
  P.mark(3);
  FPG("k_sep_init", k_sep_init, per_n, T, 0, st);
  // top separators ordered early on the side streams (one mesh, level
  // order: there their ranges depend on the top levels alone)
  const int TL = P.single && !P.update && mp[0].n > 0 && mp[0].sched == FP_SCHED_LEVEL &&
                         P.h->side_ok && !P.fixed && ensure_side(P.h)
                     ? std::min(FP_TOP_LEVELS, mp[0].Dmax)
                     : 0;
  // a tree level of mesh i in separate launches up to its expected depth,
  // past it in one workgroup (k_level_wg)
  auto in_launches = [&](int d, int i) { return d < mp[i].Dmax && d <= mp[i].Dexp; };
  auto lvl = [&](int d, long long items) {
    return [&, d, items](int i) -> long long {
      return in_launches(d, i) ? P.blk(items > 0 ? items : mp[i].n) : 0;
    };
  };
  for (int d = 0; d < Dmax; d++) {
    FPG("k_level_begin", k_level_begin,
        [&, d](int i) -> long long { return in_launches(d, i) ? P.blk(8ll * mp[i].Pexp) : 0; }, T, 0,
        st, d);
    FPG("k_arcs", k_arcs, lvl(d, 0), T, 0, st, d);
    {
      // LDS for the local quotient subgraphs: a node at depth d holds about
      // 2^(Dexp-d) patches.  While the level has no more nodes than CUs,
      // each workgroup takes the large LDS (quotient degrees can pass 8);
      // deeper, about 8 alive arcs per patch, so several workgroups share a
      // CU (a node that does not fit runs from global memory).  The
      // kernel's static LDS comes on top.
      long long want = 0;
      for (int i = 0; i < nm; i++) {
        if (d >= mp[i].Dmax) continue;
        const long long cap = 1ll << std::max(0, mp[i].Dpat - d);
        want = std::max(want, (1ll << d) <= P.ncu() ? (long long)P.h->lds_big
                                                     : (4 * (13 * cap + 1) + 255) & ~255ll);
      }
      // (at least the refinement's scratch, which the one-workgroup
      // levels take from the same LDS)
      const int lb = (int)std::min<long long>(P.h->lds_big - 1024, std::max(want, 2048ll));
      FPG("k_bisect", k_bisect,
          [&, d](int i) -> long long {
            return in_launches(d, i) ? std::min(1 << std::min(d, 30), 4 * P.ncu()) : 0;
          },
          T, lb, st, d, lb);
      FPG("k_cand", k_cand, lvl(d, 0), T, 0, st, d);
      // refined separators: candidates grouped by node, then one workgroup
      // per node finds the minimum cover and marks it (k_mark then skips)
      auto ref = [&, d](long long b) {
        return [&, d, b](int i) -> long long { return in_launches(d, i) && mp[i].refine ? b : 0; };
      };
      FPG("k_ref_place", k_ref_place, ref(1), T, 0, st, d);
      FPG("k_ref_scatter", k_ref_scatter,
          [&, d](int i) -> long long {
            return in_launches(d, i) && mp[i].refine ? P.blk(mp[i].n) : 0;
          },
          T, 0, st, d);
      FPG("k_refine_w", k_refine_w,
          [&, d](int i) -> long long {
            return in_launches(d, i) && mp[i].refine
                       ? std::max(1ll, std::min((1ll << std::min(d, 30)) / FP_WAVES + 1,
                                                4ll * P.ncu()))
                       : 0;
          },
          T, P.h->lds_bytes, st, d, 0);
      FPG("k_refine_w", k_refine_w, ref(std::min(1 << std::min(d, 30), 2 * P.ncu())), dim3(64),
          P.h->lds_big, st, d, 1);
      FPG("k_refine", k_refine, ref(std::min(1 << std::min(d, 30), 4 * P.ncu())), T, 0, st, d);
      FPG("k_mark", k_mark, lvl(d, 0), T, 0, st, d);

    }
    if (d < TL) {
      const long long b = std::min(P.blk(mp[0].n), 2ll * P.ncu());
      FPG("k_top_count", k_top_count, [&](int) { return b; }, T, 0, st, d);
      FPG("k_top_place", k_top_place, one, dim3(64), 0, st, d);
      FPG("k_top_scatter", k_top_scatter, [&](int) { return b; }, T, 0, st, d);
      // one stream per level, so a level does not wait for the one above;
      // the large local-order classes follow on the second and third
      hipStream_t sd = d == 0 ? P.h->side : d == 1 ? P.h->side2 : P.h->side3;
      if (hipEventRecord(P.h->ev_top[d], st) != hipSuccess ||
          hipStreamWaitEvent(sd, P.h->ev_top[d], 0) != hipSuccess)
        P.hip_failed = true;
      if (d == 0)
        P.side_open = true;
      else
        P.side2_open = true;
      FPG("k_md_top", k_md_top, [&, d](int) { return 1ll << d; }, dim3(64), P.h->lds_md, sd, d);
    }
    P.check();
  }
  {
    // levels past the expected depth, in one workgroup per mesh
    const int lbw = P.h->lds_big - 1024;
    FPG("k_level_wg", k_level_wg,
        [&](int i) -> long long { return mp[i].Dmax > mp[i].Dexp + 1 ? 1 : 0; }, T, lbw, st, lbw);
  }
  FPG("k_leaves", k_leaves, per_n, T, 0, st);

  // grouping in schedule order (heap size nn on the device)
  P.mark(4);
  auto nnexp = [&](int i) { return P.blk((2ll << mp[i].Dexp) - 1); };
  FPG("k_nsize", k_nsize, per_n, T, 0, st);
  // node histograms in LDS: up to 16 K nodes (64 KB), a chunk of vertices
  // per workgroup
  const int hcap = 16384;
  auto chunks = [&](int i) { return std::min(P.blk(mp[i].n), 2ll * P.ncu()); };
  const int hbytes = 4 * std::min(hcap, [&] {
    int mx = 1;
    for (const auto& x : mp) mx = std::max(mx, (int)std::min<long long>(x.NNcap, hcap));
    return mx;
  }());
  FPG("k_nsize_count", k_nsize_count, chunks, T, hbytes, st, hcap);
  FPG("k_sched_place", k_sched_place, nnexp, T, 0, st);
  P.check();
  P.scan(FA_SBUF, FA_SBUF, FN_NN, FT_TOT);
  FPG("k_nbegin", k_nbegin, nnexp, T, 0, st);
  FPG("k_scatter", k_scatter, chunks, T, hbytes, st, hcap);
  const int ntop = (1 << TL) - 1;
  if (ntop) FPG("k_top_check", k_top_check, one, dim3(64), 0, st, ntop);
  if (P.update) FPG("k_reuse", k_reuse, [&](int i) { return P.blk((2ll << mp[i].Dexp) - 1, 64); }, T, 0, st);
  P.check();

  // local orders
  P.mark(5);
  FPG("k_md_tasks", k_md_tasks, one, dim3(1024), 0, st, ntop);
  {
    // The largest class (one wave per CU, the longest nodes) goes first on
    // this stream, so its workgroups take their CUs before the others fill
    // the rest; for one mesh, class 1 follows the depth-1 orders on the
    // second side stream, classes 2 and 3 the depth-2 orders on the third.
    const bool two = P.single && !P.fixed && P.h->side_ok && ensure_side(P.h);
    if (two) {
      if (hipEventRecord(P.h->ev_md, st) != hipSuccess ||
          hipStreamWaitEvent(P.h->side2, P.h->ev_md, 0) != hipSuccess ||
          hipStreamWaitEvent(P.h->side3, P.h->ev_md, 0) != hipSuccess)
        P.hip_failed = true;
      P.side2_open = true;
    }
    for (int c = 0; c < FP_MD_CLASSES; c++) {
      hipStream_t sc = !two || c == 0 ? st : c == 1 ? P.h->side2 : P.h->side3;
      // md_per_cu workgroups per CU (tuning) for one mesh; in a batch, a
      // share of that in proportion to the mesh's expected node count
      FPG("k_md", k_md,
          [&](int i) -> long long {
            const long long full = (long long)P.h->md_per_cu * P.ncu();
            if (P.single) return full;
            return std::max(1ll, std::min(full, (2ll * mp[i].Pexp + FP_WAVES - 1) / FP_WAVES));
          },
          T, c == 3 ? P.h->lds_bytes : P.h->lds_md, sc, c);
    }
  }
  if (P.single) P.join_side();
  P.check();

  // elimination tree and column counts, bottom-up over the tree levels (a
  // node whose local order failed raised an error: these kernels then return)
  P.mark(6);
  FPG("k_prow_deg", k_prow_deg, per_n, T, 0, st);
  P.scan(FA_PCNT, FA_PROW, FN_N, FT_TOT);
  FPG("k_set", k_mptr_end, one, dim3(64), 0, st, (int)FA_PROW, (int)FN_N, (int)FT_TOT);
  FPG("k_prow_fill", k_prow_fill, per_n, T, 0, st);
  // levels past the expected depth first, in one workgroup per mesh
  FPG("k_sym_level_wg", k_sym_level_wg,
      [&](int i) -> long long { return mp[i].Dmax > mp[i].Dexp ? 1 : 0; }, T, P.h->lds_big, st);
  for (int d = Dmax; d >= 0; d--) {
    const int cnt = 1 << d;
    // separate launches up to the expected depth, one workgroup past it
    auto G = [&, d, cnt](int i) -> long long {
      if (d > mp[i].Dmax || d > mp[i].Dexp) return 0;
      return std::max(1, std::min((cnt + FP_WAVES - 1) / FP_WAVES, 16 * P.ncu()));
    };
    auto G1 = [&, d, cnt](int i) -> long long {
      if (d > mp[i].Dmax || d > mp[i].Dexp) return 0;
      return std::max(1, std::min(cnt, 4 * P.ncu()));
    };
    FPG("k_sym_prep", k_sym_prep, G, T, P.h->lds_bytes, st, d);
    FPG("k_sym_elim", k_sym_elim, G, T, P.h->lds_bytes, st, d, 0);
    FPG("k_sym_elim", k_sym_elim, G1, T, P.h->lds_big, st, d, 1);
    FPG("k_sym_elim_glb", k_sym_elim_glb, G, T, 0, st, d);
    FPG("k_sym_emit", k_sym_emit, G, T, 0, st, d);
    P.check();
  }
  FPG("k_nnzl", k_nnzl, [&](int i) { return std::min(P.blk(mp[i].n), 2ll * P.ncu()); }, T, 0, st);

  // outputs
  P.mark(7);
  FPG("k_expand", k_expand,
      [&](int i) { return P.blk(std::max<long long>(mp[i].n_dof, (2ll << mp[i].Dexp) - 1)); }, T, 0,
      st);
  FPG("k_finish", k_finish, one, dim3(64), 0, st);
  P.mark(8);
  P.check();
  return P.hip_failed ? FP_ERR_HIP : FP_OK;
}

}  // namespace

extern "C" {

int fp_version(void) { return FP_ABI_VERSION; }

const char* fp_status_str(fp_status s) {
  switch (s) {
    case FP_OK: return "ok";
    case FP_ERR_ARG: return "invalid argument";
    case FP_ERR_NOT_SYMMETRIC: return "pattern not symmetric";
    case FP_ERR_INDEX: return "index out of range";
    case FP_ERR_SIZE: return "workspace or device pool too small";
    case FP_ERR_OOM: return "out of device memory";
    case FP_ERR_UNSUPPORTED: return "unsupported option";
    case FP_ERR_BUSY: return "server busy";
    case FP_ERR_HIP: return "HIP runtime error";
    case FP_ERR_DEVICE: return "device pipeline failure";
  }
  return "unknown status";
}

void fp_options_default(fp_options* o) {
  if (!o) return;
  o->patch_size = 512;
  o->nd_level = -1;
  o->schedule = FP_SCHED_LEVEL;
  o->block_size = 1;
  o->lloyd_iters = 1;
  o->seed = 0;
  o->flags = FP_FLAG_VALIDATE;
}

// LDS of the one-wave kernels for large nodes: what one workgroup may hold
// on this device (160 KB on gfx950), at least the per-node size
static int big_lds(int device) {
  // the default per-workgroup limit, or more where a kernel opts in (CDNA4:
  // 160 KB of LDS per CU, all of it to one workgroup)
  int lim = 0, optin = 0;
  if (hipDeviceGetAttribute(&lim, hipDeviceAttributeMaxSharedMemoryPerBlock, device) !=
      hipSuccess) {
    (void)hipGetLastError();
    return FP_LDS_BYTES;
  }
  if (hipDeviceGetAttribute(&optin, hipDeviceAttributeSharedMemPerBlockOptin, device) ==
      hipSuccess)
    lim = std::max(lim, optin);
  else
    (void)hipGetLastError();
  const int big = std::min(lim, 160 * 1024) & ~15;
  if (big <= FP_LDS_BYTES) return FP_LDS_BYTES;
  if (hipFuncSetAttribute((const void*)k_md, hipFuncAttributeMaxDynamicSharedMemorySize, big) !=
          hipSuccess ||
      hipFuncSetAttribute((const void*)k_md_top, hipFuncAttributeMaxDynamicSharedMemorySize,
                          big) != hipSuccess ||
      // the bisection keeps 1 KB for its static LDS
      hipFuncSetAttribute((const void*)k_bisect, hipFuncAttributeMaxDynamicSharedMemorySize,
                          big - 1024) != hipSuccess ||
      hipFuncSetAttribute((const void*)k_sym_elim, hipFuncAttributeMaxDynamicSharedMemorySize,
                          big) != hipSuccess ||
      hipFuncSetAttribute((const void*)k_level_wg, hipFuncAttributeMaxDynamicSharedMemorySize,
                          big - 1024) != hipSuccess ||
      hipFuncSetAttribute((const void*)k_refine_w, hipFuncAttributeMaxDynamicSharedMemorySize,
                          big) != hipSuccess ||
      hipFuncSetAttribute((const void*)k_sym_level_wg,
                          hipFuncAttributeMaxDynamicSharedMemorySize, big) != hipSuccess) {
    (void)hipGetLastError();
    return FP_LDS_BYTES;
  }
  return big;
}

fp_status fp_create(fp_handle** h) {
  if (!h) return FP_ERR_ARG;
  *h = nullptr;
  fp_handle* H = new (std::nothrow) fp_handle();
  if (!H) return FP_ERR_OOM;
  int ncu = 0;
  if (hipGetDevice(&H->device) != hipSuccess ||
      hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, H->device) !=
          hipSuccess) {
    delete H;
    return FP_ERR_HIP;
  }
  H->ncu = std::max(1, ncu);
  bind_scratch(H->device);
  H->lds_bytes = FP_LDS_BYTES;
  H->lds_big = big_lds(H->device);
  H->lds_md = std::min(H->lds_big, FP_MD_LDS);
  H->md_per_cu = 2;
  H->side_ok = true;
  H->tk_name[0] = 0;
  H->tk_n = 0;
  H->tk_failed = false;
  for (int i = 0; i <= FP_NSTAGE; i++)
    if (hipEventCreate(&H->ev[i]) != hipSuccess) {
      for (int j = 0; j < i; j++) (void)hipEventDestroy(H->ev[j]);
      delete H;
      return FP_ERR_HIP;
    }
  H->bstage = nullptr;
  H->bstage_cap = 0;
  H->bstage_busy = false;
  if (hipEventCreateWithFlags(&H->ev_bstage, hipEventDisableTiming) != hipSuccess) {
    for (int j = 0; j <= FP_NSTAGE; j++) (void)hipEventDestroy(H->ev[j]);
    delete H;
    return FP_ERR_HIP;
  }
  H->side = nullptr;  // created by the first call that uses it
  H->side2 = nullptr;
  H->side3 = nullptr;
  *h = H;
  return FP_OK;
}


fp_status fp_destroy(fp_handle* h) {
  if (!h) return FP_OK;
  if (h->side) {
    // the streams are shared by the device's handles and stay; this
    // handle's work on them is done before its events go
    for (hipEvent_t e : {h->ev_join, h->ev_join2, h->ev_join3}) (void)hipEventSynchronize(e);
    for (int i = 0; i < 3; i++) (void)hipEventDestroy(h->ev_top[i]);
    for (hipEvent_t e : {h->ev_join, h->ev_md, h->ev_join2, h->ev_join3}) (void)hipEventDestroy(e);
  }
  for (hipEvent_t e : h->tk_ev) (void)hipEventDestroy(e);
  for (int i = 0; i <= FP_NSTAGE; i++) (void)hipEventDestroy(h->ev[i]);
  if (h->bstage_busy) (void)hipEventSynchronize(h->ev_bstage);
  (void)hipEventDestroy(h->ev_bstage);
  if (h->bstage) (void)hipHostFree(h->bstage);
  delete h;
  return FP_OK;
}

fp_status fp_query(fp_handle* h, const fp_csr* A, const fp_options* opts, size_t* ws_bytes,
                   int32_t* max_nodes) {
  if (!h || !ws_bytes) return FP_ERR_ARG;
  fp_status s = check_opts(opts);
  if (s) return s;
  if ((s = check_csr(A, opts->block_size))) return s;
  Plan P;
  if (!make_plan(A->n, opts->block_size, A->nnz, opts->patch_size, &P)) return FP_ERR_ARG;
  *ws_bytes = P.total;
  if (max_nodes) *max_nodes = P.NNcap;
  return FP_OK;
}

}  // extern "C"

namespace {

// fp_order and fp_order_static: `fixed` keeps every launch on `stream`, with
// no side streams and no per-kernel timing events (nothing is created).
// the job description of one mesh: its workspace layout, input, options,
// outputs (host copy; the kernels read a device copy)
// (out == NULL: sizes only)
fp_status describe(fp_handle* h, const fp_csr* A, const int32_t* user_gmap,
                   const fp_options* opts, char* ws, size_t ws_bytes, const fp_result* out,
                   FpMesh* M, size_t* need) {
  if (!h) return FP_ERR_ARG;
  fp_status s = check_opts(opts);
  if (s) return s;
  if ((s = check_csr(A, opts->block_size))) return s;
  const fp_result none{};
  if (out) {
    if (!out->perm || !out->iperm || !out->parent || !out->colcount || !out->nnzL)
      return FP_ERR_ARG;
    if ((out->node_begin || out->node_size) && out->max_nodes < 1) return FP_ERR_ARG;
  } else {
    out = &none;
  }
  Plan P;
  if (!make_plan(A->n, opts->block_size, A->nnz, opts->patch_size, &P)) return FP_ERR_ARG;
  if (need) *need = P.total;
  if (ws && ws_bytes < P.total) return FP_ERR_SIZE;
  memset(M, 0, sizeof(*M));
  fill_mesh(P, ws, M);
  M->rp32 = A->rowptr32;
  M->rp64 = (const long long*)A->rowptr64;
  M->ci_in = A->colind;
  M->nnz_in = A->nnz;
  M->user_gmap = user_gmap;
  M->S = opts->patch_size;
  M->lloyd = opts->lloyd_iters;
  M->sched = opts->schedule;
  M->seed = opts->seed;
  M->validate = (opts->flags & FP_FLAG_VALIDATE) != 0;
  M->nd_level = opts->nd_level;
  {  // expected tree depth: ceil(log2 P0), at most nd_level
    int dx = 0;
    while ((1ll << dx) < std::max(fp_p0(M->n, opts->patch_size), 1)) dx++;
    M->dexp = opts->nd_level >= 0 ? std::min(dx, opts->nd_level) : dx;
  }
  M->refine = (opts->flags & FP_FLAG_REFINE) != 0;
  M->amd = (opts->flags & FP_FLAG_AMD) != 0;
  M->perm = out->perm;
  M->iperm = out->iperm;
  M->parent = out->parent;
  M->colcount = out->colcount;
  M->nnzL = (long long*)out->nnzL;
  M->node_begin_out = out->node_begin;
  M->node_size_out = out->node_size;
  M->gmap_out = out->gmap;
  M->n_nodes_out = out->n_nodes;
  M->status_out = out->status;
  M->max_nodes_out = out->max_nodes;
  M->lds_bytes = h->lds_bytes;
  M->lds_big = h->lds_big;
  M->lds_md = h->lds_md;
  return FP_OK;
}

fp_status order_impl(fp_handle* h, const fp_csr* A, const int32_t* user_gmap,
                     const fp_options* opts, void* workspace, size_t ws_bytes, fp_result* out,
                     void* stream, bool fixed, const void* prev_ws = nullptr,
                     int32_t* reused = nullptr) {
  if (!h || !out || !workspace) return FP_ERR_ARG;
  FpMesh M;
  char* ws = (char*)workspace;
  fp_status s = describe(h, A, user_gmap, opts, ws, ws_bytes, out, &M, nullptr);
  if (s) return s;
  Plan PL;
  make_plan(A->n, opts->block_size, A->nnz, opts->patch_size, &PL);
  // the earlier call's description sits at the same offset of its workspace
  // (the control block, then the description, lead every layout)
  M.prev = prev_ws ? (const FpMesh*)((const char*)prev_ws + PL.o_mesh) : nullptr;
  M.reused_out = reused;
  Pipe P;
  P.h = h;
  P.st = (hipStream_t)stream;
  P.mp.push_back(mesh_plan(M, user_gmap != nullptr));
  P.dm = (const FpMesh*)(ws + PL.o_mesh);
  P.single = true;
  P.fixed = fixed;
  P.update = prev_ws != nullptr;
  P.timing = !fixed && (opts->flags & FP_FLAG_TIMING) != 0;
  h->timed = false;
  h->tk_n = 0;
  h->tk_failed = false;
  // control block cleared, job description copied in as a kernel argument
  // (so no host buffer has to outlive the call)
  const int words = (int)(sizeof(FpCtl) / 4);
  hipLaunchKernelGGL(k_fill, dim3((words + FP_WG - 1) / FP_WG), dim3(FP_WG), 0, P.st,
                     (int*)(FpCtl*)M.ctl, words, 0);
  hipLaunchKernelGGL(k_put_mesh, dim3(1), dim3(64), 0, P.st, M, (FpMesh*)P.dm);
  if (hipGetLastError() != hipSuccess) return FP_ERR_HIP;
  s = run_pipe(P);
  P.join_side();  // a call that stopped early still leaves no work behind it
  h->timed = P.timing && s == FP_OK;
  return s;
}

// ---------------------------------------------------------------- batches
// Workspace of a batch: the meshes' descriptions (device array), the block
// tables of every launch, then each mesh's own workspace.
struct BatchLayout {
  size_t o_desc, o_tab, total;
  std::vector<size_t> o_ws, ws;
  std::vector<FpMesh> desc;
  std::vector<int> tab;
};

fp_status batch_layout(fp_handle* h, int32_t n_mesh, const fp_csr* A,
                       const int32_t* const* user_gmap, const fp_options* opts,
                       const fp_result* out, char* base, BatchLayout* L) {
  L->o_ws.resize(n_mesh);
  L->ws.resize(n_mesh);
  L->desc.resize(n_mesh);
  size_t o = align_up(sizeof(FpMesh) * (size_t)std::max(n_mesh, 1));
  L->o_desc = 0;
  std::vector<size_t> need(n_mesh);
  for (int32_t i = 0; i < n_mesh; i++) {
    Plan PL;
    fp_status s = check_opts(&opts[i]);
    if (s) return s;
    if ((s = check_csr(&A[i], opts[i].block_size))) return s;
    if (!make_plan(A[i].n, opts[i].block_size, A[i].nnz, opts[i].patch_size, &PL))
      return FP_ERR_ARG;
    need[i] = align_up(PL.total);
  }
  // the planning pass sizes the block tables (it needs only the sizes)
  Pipe P;
  P.h = h;
  P.single = false;
  P.plan = true;
  for (int32_t i = 0; i < n_mesh; i++) {
    const int32_t* ug = user_gmap ? user_gmap[i] : nullptr;
    FpMesh M;
    fp_status s = describe(h, &A[i], ug, &opts[i], nullptr, 0, nullptr, &M, nullptr);
    if (s) return s;
    P.mp.push_back(mesh_plan(M, ug != nullptr));
  }
  (void)run_pipe(P);
  L->tab = std::move(P.tab);
  L->o_tab = o;
  o = align_up(o + 4 * L->tab.size());
  for (int32_t i = 0; i < n_mesh; i++) {
    L->o_ws[i] = o;
    L->ws[i] = need[i];
    o += need[i];
  }
  L->total = o;
  if (base)
    for (int32_t i = 0; i < n_mesh; i++) {
      const int32_t* ug = user_gmap ? user_gmap[i] : nullptr;
      fp_status s = describe(h, &A[i], ug, &opts[i], base + L->o_ws[i], L->ws[i], &out[i],
                             &L->desc[i], nullptr);
      if (s) return s;
    }
  return FP_OK;
}

// host staging of a batch's descriptions and block tables: pinned memory of
// the handle, reused once the previous batch's copy has completed
fp_status stage_batch(fp_handle* h, const void* a, size_t na, const void* b, size_t nb,
                      hipStream_t st, void* dst_a, void* dst_b) {
  if (h->bstage_busy && hipEventSynchronize(h->ev_bstage) != hipSuccess) return FP_ERR_HIP;
  h->bstage_busy = false;
  const size_t need = align_up(na) + nb;
  if (need > h->bstage_cap) {
    if (h->bstage) (void)hipHostFree(h->bstage);
    h->bstage = nullptr;
    h->bstage_cap = 0;
    if (hipHostMalloc(&h->bstage, need, hipHostMallocDefault) != hipSuccess) {
      (void)hipGetLastError();
      return FP_ERR_OOM;
    }
    h->bstage_cap = need;
  }
  char* p = (char*)h->bstage;
  memcpy(p, a, na);
  memcpy(p + align_up(na), b, nb);
  if (hipMemcpyAsync(dst_a, p, na, hipMemcpyHostToDevice, st) != hipSuccess ||
      (nb && hipMemcpyAsync(dst_b, p + align_up(na), nb, hipMemcpyHostToDevice, st) !=
                 hipSuccess) ||
      hipEventRecord(h->ev_bstage, st) != hipSuccess)
    return FP_ERR_HIP;
  h->bstage_busy = true;
  return FP_OK;
}

fp_status batch_impl(fp_handle* h, int32_t n_mesh, const fp_csr* A,
                     const int32_t* const* user_gmap, const fp_options* opts, void* workspace,
                     size_t ws_bytes, fp_result* out, void* stream, bool staged = false) {
  if (!h || n_mesh < 0) return FP_ERR_ARG;
  if (n_mesh == 0) return FP_OK;
  if (!A || !opts || !out || !workspace) return FP_ERR_ARG;
  BatchLayout L;
  char* base = (char*)workspace;
  fp_status s = batch_layout(h, n_mesh, A, user_gmap, opts, nullptr, nullptr, &L);
  if (s) return s;
  if (ws_bytes < L.total) return FP_ERR_SIZE;
  if ((s = batch_layout(h, n_mesh, A, user_gmap, opts, out, base, &L))) return s;
  Pipe P;
  P.h = h;
  P.st = (hipStream_t)stream;
  P.single = false;
  for (int32_t i = 0; i < n_mesh; i++) {
    P.mp.push_back(mesh_plan(L.desc[i], user_gmap && user_gmap[i]));
  }
  P.dm = (const FpMesh*)(base + L.o_desc);
  P.tab = L.tab;
  P.dtab = (const int*)(base + L.o_tab);
  // (a recorded batch has its descriptions and tables in place already)
  if (!staged &&
      (s = stage_batch(h, L.desc.data(), sizeof(FpMesh) * n_mesh, L.tab.data(), 4 * L.tab.size(),
                       P.st, base + L.o_desc, base + L.o_tab)))
    return s;
  // every mesh's control block cleared (one block each), then the pipeline
  hipLaunchKernelGGL(k_ctl_clear_all, dim3((unsigned)n_mesh), dim3(FP_WG), 0, P.st, P.dm);
  if (hipGetLastError() != hipSuccess) return FP_ERR_HIP;
  return run_pipe(P);
}

}  // namespace

extern "C" {

fp_status fp_order(fp_handle* h, const fp_csr* A, const int32_t* user_gmap,
                   const fp_options* opts, void* workspace, size_t ws_bytes, fp_result* out,
                   void* stream) {
  return order_impl(h, A, user_gmap, opts, workspace, ws_bytes, out, stream, false);
}

fp_status fp_order_update(fp_handle* h, const fp_csr* A, const int32_t* prev_gmap,
                          const void* prev_workspace, const fp_options* opts, void* workspace,
                          size_t ws_bytes, fp_result* out, int32_t* reused_vertices,
                          void* stream) {
  if (!h || !prev_gmap || !prev_workspace || !workspace || prev_workspace == workspace)
    return FP_ERR_ARG;
  return order_impl(h, A, prev_gmap, opts, workspace, ws_bytes, out, stream, false,
                    prev_workspace, reused_vertices);
}

fp_status fp_order_static(fp_handle* h, const fp_csr* A, const int32_t* user_gmap,
                          const fp_options* opts, fp_result* out, void* stream) {
  if (!h || !opts || !A) return FP_ERR_ARG;
  if (h->device < 0 || h->device >= FP_MAX_DEVICES) return FP_ERR_ARG;
  void* ws = g_scratch[h->device];
  if (!ws) return FP_ERR_HIP;
  size_t need = 0;
  fp_status s = fp_query(h, A, opts, &need, nullptr);
  if (s != FP_OK) return s;
  if (need > FP_STATIC_SCRATCH_BYTES) return FP_ERR_SIZE;
  return order_impl(h, A, user_gmap, opts, ws, FP_STATIC_SCRATCH_BYTES, out, stream, true);
}

fp_status fp_query_batch(fp_handle* h, int32_t n_mesh, const fp_csr* A, const fp_options* opts,
                         const int32_t* const* user_gmap, size_t* workspace_bytes,
                         int32_t* max_nodes) {
  if (!h || n_mesh < 0 || (n_mesh > 0 && (!A || !opts)) || !workspace_bytes) return FP_ERR_ARG;
  BatchLayout L;
  fp_status s = batch_layout(h, n_mesh, A, user_gmap, opts, nullptr, nullptr, &L);
  if (s) return s;
  *workspace_bytes = std::max<size_t>(L.total, 256);
  if (max_nodes) {
    int32_t mx = 1;
    for (int32_t i = 0; i < n_mesh; i++) {
      Plan PL;
      make_plan(A[i].n, opts[i].block_size, A[i].nnz, opts[i].patch_size, &PL);
      mx = std::max(mx, PL.NNcap);
    }
    *max_nodes = mx;
  }
  return FP_OK;
}

fp_status fp_order_batch(fp_handle* h, int32_t n_mesh, const fp_csr* A,
                         const int32_t* const* user_gmap, const fp_options* opts, void* workspace,
                         size_t ws_bytes, fp_result* out, void* stream) {
  return batch_impl(h, n_mesh, A, user_gmap, opts, workspace, ws_bytes, out, stream);
}

// the concatenated form: per-mesh views into the caller's arrays
static fp_status concat_views(int32_t n_mesh, const int64_t* rowptr, const int32_t* colind,
                              const int64_t* vtx_off, const int64_t* nnz_off,
                              const fp_options* opts, std::vector<fp_csr>* A) {
  if (n_mesh < 0 || (n_mesh > 0 && (!rowptr || !vtx_off || !nnz_off || !opts))) return FP_ERR_ARG;
  A->resize(n_mesh);
  for (int32_t i = 0; i < n_mesh; i++) {
    const int64_t n = vtx_off[i + 1] - vtx_off[i], nnz = nnz_off[i + 1] - nnz_off[i];
    if (n < 0 || nnz < 0 || (nnz > 0 && !colind)) return FP_ERR_ARG;
    (*A)[i] = fp_csr{n, nnz, nullptr, rowptr + vtx_off[i] + i, nnz ? colind + nnz_off[i] : nullptr};
  }
  return FP_OK;
}

fp_status fp_query_batch_concat(fp_handle* h, int32_t n_mesh, const int64_t* rowptr,
                                const int32_t* colind, const int64_t* vtx_off,
                                const int64_t* nnz_off, const fp_options* opts,
                                size_t* workspace_bytes, int64_t* node_off) {
  std::vector<fp_csr> A;
  fp_status s = concat_views(n_mesh, rowptr, colind, vtx_off, nnz_off, opts, &A);
  if (s) return s;
  if ((s = fp_query_batch(h, n_mesh, A.data(), opts, nullptr, workspace_bytes, nullptr))) return s;
  if (node_off) {
    node_off[0] = 0;
    for (int32_t i = 0; i < n_mesh; i++) {
      Plan PL;
      make_plan(A[i].n, opts[i].block_size, A[i].nnz, opts[i].patch_size, &PL);
      node_off[i + 1] = node_off[i] + PL.NNcap;
    }
  }
  return FP_OK;
}

fp_status fp_order_batch_concat(fp_handle* h, int32_t n_mesh, const int64_t* rowptr,
                                const int32_t* colind, const int64_t* vtx_off,
                                const int64_t* nnz_off, const fp_options* opts, void* workspace,
                                size_t ws_bytes, int32_t* perm, int32_t* iperm, int32_t* parent,
                                int32_t* colcount, int64_t* nnzL, uint32_t* status,
                                int32_t* node_begin, int32_t* node_size, const int64_t* node_off,
                                void* stream) {
  std::vector<fp_csr> A;
  fp_status s = concat_views(n_mesh, rowptr, colind, vtx_off, nnz_off, opts, &A);
  if (s) return s;
  if (n_mesh > 0 && (!perm || !iperm || !parent || !colcount || !nnzL)) return FP_ERR_ARG;
  if ((node_begin || node_size) && !node_off) return FP_ERR_ARG;
  std::vector<fp_result> R(n_mesh);
  for (int32_t i = 0; i < n_mesh; i++) {
    const int64_t o = vtx_off[i];
    fp_result& r = R[i];
    r = fp_result{};
    r.perm = perm + o;
    r.iperm = iperm + o;
    r.parent = parent + o;
    r.colcount = colcount + o;
    r.nnzL = nnzL + i;
    r.status = status ? status + i : nullptr;
    if (node_begin || node_size) {
      r.node_begin = node_begin ? node_begin + node_off[i] : nullptr;
      r.node_size = node_size ? node_size + node_off[i] : nullptr;
      r.max_nodes = (int32_t)(node_off[i + 1] - node_off[i]);
    }
  }
  return batch_impl(h, n_mesh, A.data(), nullptr, opts, workspace, ws_bytes, R.data(), stream);
}

fp_status fp_graph_create(fp_handle* h, int32_t n_mesh, const fp_csr* A,
                          const int32_t* const* user_gmap, const fp_options* opts, void* workspace,
                          size_t ws_bytes, fp_result* out, fp_graph** g) {
  if (!h || !g || n_mesh < 1 || !A || !opts || !out || !workspace) return FP_ERR_ARG;
  *g = nullptr;
  for (int32_t i = 0; i < n_mesh; i++)
    if (opts[i].flags & ~FP_FLAG_VALIDATE) return FP_ERR_ARG;
  // host-side checks and sizes first: nothing is recorded for a bad batch
  BatchLayout L;
  char* base = (char*)workspace;
  fp_status s = batch_layout(h, n_mesh, A, user_gmap, opts, nullptr, nullptr, &L);
  if (s) return s;
  if (ws_bytes < L.total) return FP_ERR_SIZE;
  if (n_mesh > 1) {
    if ((s = batch_layout(h, n_mesh, A, user_gmap, opts, out, base, &L))) return s;
    if (hipMemcpy(base + L.o_desc, L.desc.data(), sizeof(FpMesh) * n_mesh,
                  hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(base + L.o_tab, L.tab.data(), 4 * L.tab.size(), hipMemcpyHostToDevice) !=
            hipSuccess)
      return FP_ERR_HIP;
  }
  // streams and events of the pipeline exist before recording starts; the
  // recording uses streams of its own (the device's shared side streams may
  // carry other handles' work meanwhile), which the graph does not keep; the
  // kernel timing switch is off while recording
  hipStream_t rec[3] = {nullptr, nullptr, nullptr}, shared[3] = {h->side, h->side2, h->side3};
  const bool side = h->side_ok && ensure_side(h);
  if (side) {
    shared[0] = h->side;
    shared[1] = h->side2;
    shared[2] = h->side3;
    for (int j = 0; j < 3; j++)
      if (hipStreamCreateWithFlags(&rec[j], hipStreamNonBlocking) != hipSuccess) {
        for (int q = 0; q < j; q++) (void)hipStreamDestroy(rec[q]);
        return FP_ERR_HIP;
      }
    h->side = rec[0];
    h->side2 = rec[1];
    h->side3 = rec[2];
  }
  auto restore = [&]() {
    if (!side) return;
    h->side = shared[0];
    h->side2 = shared[1];
    h->side3 = shared[2];
    for (int j = 0; j < 3; j++) (void)hipStreamDestroy(rec[j]);
  };
  hipStream_t cs = nullptr;
  if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) {
    restore();
    return FP_ERR_HIP;
  }
  char tk_saved[sizeof(h->tk_name)];
  memcpy(tk_saved, h->tk_name, sizeof(tk_saved));
  h->tk_name[0] = 0;
  hipGraph_t graph = nullptr;
  if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    (void)hipStreamDestroy(cs);
    memcpy(h->tk_name, tk_saved, sizeof(tk_saved));
    restore();
    return FP_ERR_HIP;
  }
  s = n_mesh == 1 ? order_impl(h, A, user_gmap ? user_gmap[0] : nullptr, opts, workspace,
                               ws_bytes, out, cs, false)
                  : batch_impl(h, n_mesh, A, user_gmap, opts, workspace, ws_bytes, out, cs, true);
  const hipError_t ec = hipStreamEndCapture(cs, &graph);
  memcpy(h->tk_name, tk_saved, sizeof(tk_saved));
  (void)hipStreamDestroy(cs);
  restore();
  if (s == FP_OK && (ec != hipSuccess || !graph)) s = FP_ERR_HIP;
  hipGraphExec_t exec = nullptr;
  if (s == FP_OK && hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess)
    s = FP_ERR_HIP;
  if (s != FP_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    (void)hipGetLastError();
    return s;
  }
  fp_graph* G = new (std::nothrow) fp_graph;
  if (!G) {
    (void)hipGraphExecDestroy(exec);
    (void)hipGraphDestroy(graph);
    return FP_ERR_OOM;
  }
  G->graph = graph;
  G->exec = exec;
  *g = G;
  return FP_OK;
}

fp_status fp_graph_launch(fp_graph* g, void* stream) {
  if (!g) return FP_ERR_ARG;
  return hipGraphLaunch(g->exec, (hipStream_t)stream) == hipSuccess ? FP_OK : FP_ERR_HIP;
}

fp_status fp_graph_destroy(fp_graph* g) {
  if (!g) return FP_OK;
  const bool ok = hipGraphExecDestroy(g->exec) == hipSuccess && hipGraphDestroy(g->graph) == hipSuccess;
  delete g;
  return ok ? FP_OK : FP_ERR_HIP;
}

fp_status fp_set_tuning(fp_handle* h, const fp_tuning* t) {
  if (!h || !t) return FP_ERR_ARG;
  if (t->md_lds_bytes < 16 * 1024 || t->md_lds_bytes > h->lds_big || (t->md_lds_bytes & 1023) ||
      t->md_blocks_per_cu < 1 || t->md_blocks_per_cu > 8)
    return FP_ERR_ARG;
  h->lds_md = t->md_lds_bytes;
  h->md_per_cu = t->md_blocks_per_cu;
  return FP_OK;
}

fp_status fp_get_tuning(fp_handle* h, fp_tuning* t) {
  if (!h || !t) return FP_ERR_ARG;
  t->md_lds_bytes = h->lds_md;
  t->md_blocks_per_cu = h->md_per_cu;
  t->max_lds_bytes = h->lds_big;
  return FP_OK;
}

fp_status fp_time_kernel(fp_handle* h, const char* name) {
  if (!h) return FP_ERR_ARG;
  if (!name) name = "";
  if (strlen(name) >= sizeof(h->tk_name)) return FP_ERR_ARG;
  strcpy(h->tk_name, name);
  h->tk_n = 0;
  return FP_OK;
}

fp_status fp_kernel_time(fp_handle* h, float* total_ms, int32_t* launches) {
  if (!h || !total_ms) return FP_ERR_ARG;
  if (h->tk_failed) return FP_ERR_HIP;
  float tot = 0.f;
  for (int i = 0; i < h->tk_n; i++) {
    float ms = 0.f;
    if (hipEventSynchronize(h->tk_ev[2 * i + 1]) != hipSuccess ||
        hipEventElapsedTime(&ms, h->tk_ev[2 * i], h->tk_ev[2 * i + 1]) != hipSuccess)
      return FP_ERR_HIP;
    tot += ms;
  }
  *total_ms = tot;
  if (launches) *launches = h->tk_n;
  return FP_OK;
}

int fp_stage_count(void) { return FP_NSTAGE; }

const char* fp_stage_name(int i) { return (i >= 0 && i < FP_NSTAGE) ? kStageNames[i] : ""; }

fp_status fp_stage_times(fp_handle* h, float* ms, int32_t n) {
  if (!h || !ms || n < 0) return FP_ERR_ARG;
  if (!h->timed) return FP_ERR_ARG;
  if (hipEventSynchronize(h->ev[FP_NSTAGE]) != hipSuccess) return FP_ERR_HIP;
  for (int i = 0; i < std::min(n, FP_NSTAGE); i++)
    if (hipEventElapsedTime(&ms[i], h->ev[i], h->ev[i + 1]) != hipSuccess) return FP_ERR_HIP;
  return FP_OK;
}

fp_status fp_error_detail(fp_handle* h, void* workspace, void* stream, uint32_t* bits,
                          int32_t* site, int32_t* arg) {
  if (!h || !workspace) return FP_ERR_ARG;
  if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess) return FP_ERR_HIP;
  const FpCtl* C = (const FpCtl*)workspace;
  unsigned e = 0;
  int s[2] = {0, 0};
  if (hipMemcpy(&e, &C->err, sizeof(e), hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemcpy(s, &C->site, sizeof(s), hipMemcpyDeviceToHost) != hipSuccess)
    return FP_ERR_HIP;
  if (bits) *bits = e;
  if (site) *site = s[0];
  if (arg) *arg = s[1];
  return FP_OK;
}

fp_status fp_last_error(fp_handle* h, void* workspace, void* stream) {
  if (!h || !workspace) return FP_ERR_ARG;
  if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess) return FP_ERR_HIP;
  unsigned e = 0;
  if (hipMemcpy(&e, &((FpCtl*)workspace)->err, sizeof(e), hipMemcpyDeviceToHost) != hipSuccess)
    return FP_ERR_HIP;
  return map_err(e);
}

}  // extern "C"
