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

#define FP_CC_ROUNDS 4  // launched rounds of the orphan-component pass

#define MESH0            \
  const FpMesh& M = *Mp; \
  gptr<FpCtl> C = M.ctl; \
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
// ingest: graph of A without its diagonal (Sec. 4.1 Step 2, Sec. 6.5)
// ==========================================================================
__global__ void k_ingest(const FpMesh* __restrict__ Mp, int fill) {
  MESH0;
  if (fill && wave_failed(C)) return;
  unsigned eb = 0;
  for (int v = gtid(); v < M.n; v += gsize()) {
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
__global__ void k_ingest_long(const FpMesh* __restrict__ Mp, int fill) {
  MESH0;
  __shared__ int red;
  if (fill && wg_failed(C)) return;
  unsigned eb = 0;
  const int nl = C->nlong;
  for (int l = blockIdx.x; l < nl; l += gridDim.x) {
    const int v = M.fb[l];
    const int c = ingest_long_row(M, v, fill ? M.gci + M.grp[v] : gptr<int>(nullptr), &eb, &red);
    if (!fill && threadIdx.x == 0) M.pcnt[v] = c;
  }
  if (eb) fp_fail(C, eb, FP_SITE_INGEST, 0);
}
// the vertex graph fits its capacity (an int32 count that overflowed reads
// negative); the fill pass and every later stage are gated on this
__global__ void k_check_graph(const FpMesh* __restrict__ Mp) {
  MESH0;
  if (gtid() == 0 && (C->nnz_g < 0 || (long long)C->nnz_g > M.Ecap))
    fp_fail(C, FP_E_SCRATCH, FP_SITE_GRAPH, C->nnz_g);
}
// every entry (v, u) of the graph has its mirror (u, v): the pattern of A is
// symmetric (Sec. 4, inputs), block by block in block mode
__global__ void k_validate(const FpMesh* __restrict__ Mp) {
  MESH0;
  if (wave_failed(C)) return;
  for (int v = gtid(); v < M.n; v += gsize())
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
__global__ void k_seeds(const FpMesh* __restrict__ Mp, int P0) {
  MESH;
  const int n = M.n, S = M.S;
  for (int blk = gwave(); blk < P0; blk += nwaves()) {
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
  if (gtid() == 0) {
    C->P0 = P0;
    C->P = P0;
  }
}
__global__ void k_key_unset(const FpMesh* __restrict__ Mp) {
  MESH;
  for (int v = gtid(); v < M.n; v += gsize()) M.key[v] = FP_UNSET;
  for (int i = gtid(); i < M.n + 16; i += gsize()) M.fcnt[i] = 0;
}
// nseeds < 0: every patch seed (the count is on the device)
__global__ void k_seed_push(const FpMesh* __restrict__ Mp, int nseeds) {
  MESH;
  if (nseeds < 0) nseeds = min(C->P, M.n);
  for (int k = gtid(); k < nseeds; k += gsize()) {
    const int s = M.seeds[k];
    atomicMin(&M.key[s], (unsigned long long)k);
    M.fa[k] = s;
  }
  if (gtid() == 0) M.fcnt[0] = nseeds;
}
// One frontier level: a lane per frontier vertex.  The loads of its first
// FP_BFS_ROW neighbours (columns, then keys) go out together, and the wave's
// claims are appended with one atomic.
#define FP_BFS_ROW 8
__global__ void k_bfs_level(const FpMesh* __restrict__ Mp, int lvl) {
  MESH;
  const int nf = M.fcnt[lvl];
  gptr<const int> cur = (lvl & 1) ? M.fb : M.fa;
  gptr<int> nxt = (lvl & 1) ? M.fa : M.fb;
  for (int f0 = gwave() * 64; f0 < nf; f0 += nwaves() * 64) {
    const int f = f0 + lane_id();
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
    // one slot range per wave for all these claims
    const int c = __popc(claims);
    const int inc = wave_incl_scan(c);
    const int tot = wave_bcast(inc, 63);
    int base = 0;
    if (tot) {
      if (lane_id() == 0) base = atomicAdd(&M.fcnt[lvl + 1], tot);
      base = wave_bcast(base, 0);
    }
    int o = base + inc - c;
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
// any work here; late frontiers are small.  The agent-scope fences around
// each barrier make the level's claims and appends (in L2) visible to every
// lane's next loads, which would otherwise be served from this CU's L1.
__device__ __forceinline__ void wg_level_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
  __syncthreads();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
}
__global__ void __launch_bounds__(1024) k_bfs_tail(const FpMesh* __restrict__ Mp, int lvl0) {
  MESH_WG;
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
__global__ void k_count_unset(const FpMesh* __restrict__ Mp) {
  MESH;
  int cnt = 0;
  for (int v = gtid(); v < M.n; v += gsize()) cnt += (M.key[v] == FP_UNSET);
  cnt = wave_sum_i32(cnt);
  if (lane_id() == 0 && cnt) atomicAdd(&C->norphan, cnt);
}
// components without a seed: min-label fixed point, then ids P0 + rank of
// the component's lowest vertex
// Every kernel of this pass returns at once when growth left no vertex
// unlabelled.  Rounds of hooking and pointer jumping run as separate
// launches while the previous round changed a label; a one-workgroup tail
// finishes any component the rounds did not settle.
__global__ void k_cc_init(const FpMesh* __restrict__ Mp) {
  MESH;
  const bool any = C->norphan > 0;
  if (gtid() == 0) C->ccn = any ? M.n : 0;
  if (!any) return;
  for (int v = gtid(); v < M.n; v += gsize()) M.fb[v] = (M.key[v] == FP_UNSET) ? v : -1;
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
__global__ void k_cc_hook(const FpMesh* __restrict__ Mp, int r) {
  MESH;
  if (!cc_round_live(C, r)) return;
  if (cc_hook_pass(M, gtid(), gsize())) atomicOr(&C->ccchg[r], 1);
}
__global__ void k_cc_jump(const FpMesh* __restrict__ Mp, int r) {
  MESH;
  if (!cc_round_live(C, r)) return;
  if (cc_jump_pass(M, gtid(), gsize())) atomicOr(&C->ccchg[r], 1);
}
__global__ void __launch_bounds__(1024) k_cc_tail(const FpMesh* __restrict__ Mp, int r0) {
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
__global__ void k_cc_flags(const FpMesh* __restrict__ Mp) {
  MESH;
  if (C->norphan == 0) return;
  for (int v = gtid(); v < M.n; v += gsize()) M.pcnt[v] = (M.fb[v] == v) ? 1 : 0;
}
// ids P0 + rank of the component's lowest vertex; P grows by the count
__global__ void k_cc_label(const FpMesh* __restrict__ Mp) {
  MESH;
  if (C->norphan == 0) return;
  const int P0 = C->P0;
  for (int v = gtid(); v < M.n; v += gsize()) {
    const int c = M.fb[v];
    if (c < 0) continue;
    const int id = P0 + M.pcnt[c];
    M.key[v] = (unsigned long long)id;
    if (c == v) M.seeds[id] = v;
  }
  if (gtid() == 0) C->P = P0 + C->nroot;
}
// Lloyd re-centre: new seed = vertex farthest from the patch boundary (the
// distance inside the patch equals the distance to the boundary set of the
// whole graph, because any path out of a patch passes its own boundary
// first), ties to the lowest id; patches without a boundary keep their seed.
__global__ void k_lloyd_gmap(const FpMesh* __restrict__ Mp) {
  MESH;
  const int P = C->P;
  for (int v = gtid(); v < M.n; v += gsize()) M.gmap[v] = (int)(M.key[v] & 0xFFFFFFFFu);
  for (int p = gtid(); p < P; p += gsize()) M.best[p] = 0;
  for (int i = gtid(); i < M.n + 16; i += gsize()) M.fcnt[i] = 0;
}
// (the loops below step a whole workgroup at a time: wg_append holds a
// barrier, and a single list counter takes one atomic per workgroup)
__global__ void k_lloyd_bnd(const FpMesh* __restrict__ Mp) {
  MESH_WG;
  __shared__ int lds2[2];
  for (int v0 = (int)(blockIdx.x * blockDim.x); v0 < M.n; v0 += (int)(gridDim.x * blockDim.x)) {
    const int v = v0 + (int)threadIdx.x;
    bool isb = false;
    if (v < M.n) {
      const int g = M.gmap[v];
      for (int e = M.grp[v]; e < M.grp[v + 1] && !isb; e++) isb = (M.gmap[M.gci[e]] != g);
      M.key[v] = isb ? 0ull : FP_UNSET;
    }
    const int slot = wg_append(&M.fcnt[0], isb, lds2);
    if (isb) M.fa[slot] = v;
  }
}
// per patch, the candidate of largest distance (least vertex on ties); the
// lanes of a wave that share a patch take their maximum first, so a patch
// gets one atomic per wave instead of one per vertex
__global__ void k_lloyd_best(const FpMesh* __restrict__ Mp) {
  MESH;
  for (int v0 = gwave() * 64; v0 < M.n; v0 += nwaves() * 64) {
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
__global__ void k_lloyd_seed(const FpMesh* __restrict__ Mp) {
  MESH;
  const int P = C->P;
  for (int p = gtid(); p < P; p += gsize()) {
    const unsigned long long bb = M.best[p];
    if (bb) M.seeds[p] = (int)(0xFFFFFFFFu - (unsigned)(bb & 0xFFFFFFFFu));
  }
}
__global__ void k_gmap_final(const FpMesh* __restrict__ Mp) {
  MESH;
  const int P = C->P;
  for (int v = gtid(); v < M.n; v += gsize()) {
    const unsigned long long k = M.key[v];
    const int g = k == FP_UNSET ? -1 : (int)(k & 0xFFFFFFFFu);
    if (g < 0 || g >= P) fp_fail(C, FP_E_INTERNAL, FP_SITE_GMAP_LABEL, v);
    M.gmap[v] = (g < 0 || g >= P) ? 0 : g;
  }
}
__global__ void k_user_gmap(const FpMesh* __restrict__ Mp) {
  MESH;
  int mx = 0;
  for (int v = gtid(); v < M.n; v += gsize()) {
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
__global__ void k_patch_count(const FpMesh* __restrict__ Mp) {
  MESH_WG;
  __shared__ int lds2[2];
  for (int v0 = (int)(blockIdx.x * blockDim.x); v0 < M.n; v0 += (int)(gridDim.x * blockDim.x)) {
    const int v = v0 + (int)threadIdx.x;
    const bool act = v < M.n;
    const int g = act ? M.gmap[v] : 0;
    bool isb = false;
    if (act)
      for (int e = M.grp[v]; e < M.grp[v + 1] && !isb; e++) isb = (M.gmap[M.gci[e]] != g);
    (void)wave_append_keyed(M.pcnt, g, act);
    const int slot = wg_append(&C->nbnd, isb, lds2);
    if (isb) M.bnd[slot] = v;
  }
}
__global__ void k_patch_scatter(const FpMesh* __restrict__ Mp) {
  MESH;
  for (int v0 = gwave() * 64; v0 < M.n; v0 += nwaves() * 64) {
    const int v = v0 + lane_id();
    const bool act = v < M.n;
    const int slot = wave_append_keyed(M.pcnt, act ? M.gmap[v] : 0, act);
    if (act) M.pvtx[slot] = v;
  }
}
// distinct neighbour patches of patch p, ascending, by repeated wave-wide
// minimum over the foreign neighbours of its members
// Quotient row of patch p: the sorted distinct patches next to it.  With an
// LDS bitmap over the patch ids (bm_words words per wave) one pass over the
// members marks the neighbours, their loads issued a row at a time, and the
// bitmap is read back in order; without it, one pass per neighbour.
__global__ void k_qrow(const FpMesh* __restrict__ Mp, int fill, int lds_words) {
  MESH;
  FP_LDS_DECL;
  const int P = C->P;
  const int bm_words = (P + 31) / 32 <= lds_words ? (P + 31) / 32 : 0;
  uint32_t* bm = (uint32_t*)fp_lds + (long long)bm_words * wave_id();
  for (int p = gwave(); p < P; p += nwaves()) {
    const int a0 = M.pptr[p], a1 = M.pptr[p + 1];
    gptr<int> out = fill ? M.qci + M.qptr[p] : gptr<int>(nullptr);
    int cnt = 0;
    if (bm_words) {
      for (int w = lane_id(); w < bm_words; w += 64) bm[w] = 0u;
      wave_fence();
      for (int i = a0 + lane_id(); i < a1; i += 64) {
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
      wave_fence();
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
      wave_fence();
    } else {
      int last = -1;
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
    }
    if (!fill && lane_id() == 0) M.pcnt[p] = cnt;
  }
}

__global__ void k_check_arcs(const FpMesh* __restrict__ Mp) {
  MESH;
  if (gtid() == 0 && (C->nq < 0 || (long long)C->nq > M.Ecap))
    fp_fail(C, FP_E_SCRATCH, FP_SITE_QARCS, C->nq);
}

// ==========================================================================
// separator tree (Sec. 4.2 Step 3; Alg. 2; Sec. 5).  Level d: recount the
// alive quotient arcs from the boundary list, bisect every node of depth d,
// SuperSeparator (unmarked vertices with an unmarked neighbour across) and
// RefineSeparator (keep the smaller side, ties to the left).
// ==========================================================================
__global__ void k_sep_init(const FpMesh* __restrict__ Mp) {
  MESH;
  const int P = C->P;
  int D = 0;
  while ((1ll << D) < P) D++;
  const int nn = (1 << (D + 1)) - 1;
  if (nn > M.NNcap) {  // never expected: NNcap holds the tree of n patches
    if (gtid() == 0) fp_fail(C, FP_E_SCRATCH, FP_SITE_TREE, nn);
    return;
  }
  if (gtid() == 0) {
    C->D = D;
    C->nn = nn;
  }
  for (int v = gtid(); v < M.n; v += gsize()) M.node_of[v] = -1;
  for (int p = gtid(); p < P; p += gsize()) {
    M.pnode[p] = 0;
    M.plist[p] = p;
  }
  for (int x = gtid(); x < nn; x += gsize()) {
    M.cntL[x] = 0;
    M.cntR[x] = 0;
    M.segN[x] = 0;
    M.segS[x] = 0;
  }
  if (gtid() == 0) M.segN[0] = P;
}
// level d of the tree: alive arcs recounted from zero
__global__ void k_level_begin(const FpMesh* __restrict__ Mp, int d) {
  MESH;
  if (d >= C->D) return;
  const int nq = min(C->nq, (int)M.Ecap);
  for (int a = gtid(); a < nq; a += gsize()) M.qcnt[a] = 0;
}
__global__ void k_arcs(const FpMesh* __restrict__ Mp, int d) {
  MESH;
  if (d >= C->D) return;
  const int nb = C->nbnd;
  for (int i = gtid(); i < nb; i += gsize()) {
    const int v = M.bnd[i];
    if (M.node_of[v] != -1) continue;
    const int gv = M.gmap[v];
    const int e0 = M.grp[v], deg = M.grp[v + 1] - e0;
    // the first FP_BFS_ROW neighbours' columns, marks and patches at once
    int u[FP_BFS_ROW], nu[FP_BFS_ROW], gu[FP_BFS_ROW];
#pragma unroll
    for (int j = 0; j < FP_BFS_ROW; j++) u[j] = j < deg ? (int)M.gci[e0 + j] : -1;
#pragma unroll
    for (int j = 0; j < FP_BFS_ROW; j++) {
      nu[j] = u[j] >= 0 ? (int)M.node_of[u[j]] : 0;
      gu[j] = u[j] >= 0 ? (int)M.gmap[u[j]] : gv;
    }
#pragma unroll
    for (int j = 0; j < FP_BFS_ROW; j++) {
      if (nu[j] != -1 || gu[j] == gv) continue;
      const int a = arc_index(M, gv, gu[j]);
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
__global__ void __launch_bounds__(FP_WG) k_bisect(const FpMesh* __restrict__ Mp, int d,
                                                   int lds_bytes) {
  MESH_WG;
  __shared__ BisectLds sh;
  FP_LDS_DECL;
  if (d >= C->D) return;
  const int lo = (1 << d) - 1, hi = (1 << (d + 1)) - 1;
  for (int t = lo + (int)blockIdx.x; t < hi; t += (int)gridDim.x) {
    const int m = M.segN[t];
    if (m >= 2) wg_bisect(M, t, M.segS[t], m, &sh, fp_lds, lds_bytes);
  }
}
__global__ void k_cand(const FpMesh* __restrict__ Mp, int d) {
  MESH;
  if (d >= C->D) return;
  const int hi = (1 << (d + 1)) - 1;
  const int nb = C->nbnd;
  for (int i = gtid(); i < nb; i += gsize()) {
    const int v = M.bnd[i];
    M.cand[i] = 0;
    if (M.node_of[v] != -1) continue;
    const int c = M.pnode[M.gmap[v]];
    if (c < hi) continue;  // patch not split at this level
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
    bool is = false;
#pragma unroll
    for (int j = 0; j < FP_BFS_ROW; j++) is |= nu[j] == -1 && M.pnode[gu[j]] == sib;
    for (int e = e0 + FP_BFS_ROW; e < e0 + deg && !is; e++) {
      const int w = M.gci[e];
      is = (M.node_of[w] == -1 && M.pnode[M.gmap[w]] == sib);
    }
    if (is) {
      M.cand[i] = 1;
      atomicAdd((c & 1) ? &M.cntL[(c - 1) >> 1] : &M.cntR[(c - 1) >> 1], 1);
    }
  }
}
__global__ void k_mark(const FpMesh* __restrict__ Mp, int d) {
  MESH;
  if (d >= C->D) return;
  const int nb = C->nbnd;
  for (int i = gtid(); i < nb; i += gsize()) {
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
// leaves keep the remaining vertices of their patch
__global__ void k_leaves(const FpMesh* __restrict__ Mp) {
  MESH;
  for (int v = gtid(); v < M.n; v += gsize())
    if (M.node_of[v] == -1) M.node_of[v] = M.pnode[M.gmap[v]];
}

// ==========================================================================
// grouping in schedule order (Alg. 3)
// ==========================================================================
__global__ void k_nsize(const FpMesh* __restrict__ Mp) {
  MESH;
  const int nn = C->nn;
  for (int x = gtid(); x < nn; x += gsize()) M.nsize[x] = 0;
  for (int v = gtid(); v < M.n; v += gsize()) {
    if ((unsigned)M.node_of[v] >= (unsigned)nn) {  // never expected
      fp_fail(C, FP_E_INTERNAL, FP_SITE_NODE_OF, v);
      M.node_of[v] = 0;
    }
  }
}
__global__ void k_nsize_count(const FpMesh* __restrict__ Mp) {
  MESH;
  for (int v0 = gwave() * 64; v0 < M.n; v0 += nwaves() * 64) {
    const int v = v0 + lane_id();
    const bool act = v < M.n;
    (void)wave_append_keyed(M.nsize, act ? M.node_of[v] : 0, act);
  }
}
__global__ void k_sched_place(const FpMesh* __restrict__ Mp) {
  MESH;
  const int nn = C->nn, D = C->D;
  for (int x = gtid(); x < nn; x += gsize()) M.sbuf[sched_pos(x, D, M.sched)] = M.nsize[x];
}
__global__ void k_nbegin(const FpMesh* __restrict__ Mp) {
  MESH;
  const int nn = C->nn, D = C->D;
  for (int x = gtid(); x < nn; x += gsize()) {
    const int b = M.sbuf[sched_pos(x, D, M.sched)];
    M.nbegin[x] = b;
    M.ncur[x] = b;
  }
}
__global__ void k_scatter(const FpMesh* __restrict__ Mp) {
  MESH;
  for (int v0 = gwave() * 64; v0 < M.n; v0 += nwaves() * 64) {
    const int v = v0 + lane_id();
    const bool act = v < M.n;
    const int slot = wave_append_keyed(M.ncur, act ? M.node_of[v] : 0, act);
    if (act) M.gbuf[slot] = v;
  }
}

// ==========================================================================
// local orders (Sec. 4.3 Step 4): one wave per node, LDS slice per wave
// ==========================================================================
// Task lists of the local orders, one per size class, largest nodes first
// (a counting sort on size / 16, one workgroup): a class with more nodes
// than resident slots then ends with its smallest nodes, not its largest.
#define FP_TASK_BUCKETS 256
__global__ void __launch_bounds__(1024) k_md_tasks(const FpMesh* __restrict__ Mp, int ntop) {
  MESH_WG;
  const int nn = C->nn;
  __shared__ int hist[FP_MD_CLASSES * FP_TASK_BUCKETS];
  for (int i = threadIdx.x; i < FP_MD_CLASSES * FP_TASK_BUCKETS; i += blockDim.x) hist[i] = 0;
  __syncthreads();
  auto key = [&](int x) -> int {  // class * buckets + bucket, or -1
    const int m = M.nsize[x];
    if (m == 0 || (x < ntop && C->tearly[x])) return -1;  // top separators ordered already
    const int c = md_class(m, M.lds_bytes, M.lds_md);
    return c * FP_TASK_BUCKETS + (FP_TASK_BUCKETS - 1) - min(m >> 4, FP_TASK_BUCKETS - 1);
  };
  for (int x = threadIdx.x; x < nn; x += blockDim.x) {
    const int k = key(x);
    if (k >= 0) atomicAdd(&hist[k], 1);
  }
  __syncthreads();
  if (threadIdx.x < FP_MD_CLASSES) {
    int run = 0;
    for (int b = 0; b < FP_TASK_BUCKETS; b++) {
      const int v = hist[threadIdx.x * FP_TASK_BUCKETS + b];
      hist[threadIdx.x * FP_TASK_BUCKETS + b] = run;
      run += v;
    }
    C->task_cnt[threadIdx.x] = run;
  }
  __syncthreads();
  for (int x = threadIdx.x; x < nn; x += blockDim.x) {
    const int k = key(x);
    if (k >= 0) M.tasks[(k / FP_TASK_BUCKETS) * M.NNcap + atomicAdd(&hist[k], 1)] = x;
  }
}
__global__ void __launch_bounds__(FP_WG) k_md(const FpMesh* __restrict__ Mp, int c) {
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
__global__ void k_top_count(const FpMesh* __restrict__ Mp, int d) {
  MESH;
  if (d >= C->D) return;
  const int lo = (1 << d) - 1, hi = (2 << d) - 1;
  for (int v0 = gwave() * 64; v0 < M.n; v0 += nwaves() * 64) {
    const int v = v0 + lane_id();
    const int t = v < M.n ? M.node_of[v] : -1;
    const bool act = t >= lo && t < hi;
    (void)wave_append_keyed(&C->tcnt[0], act ? t : 0, act);
  }
}
__global__ void k_top_place(const FpMesh* __restrict__ Mp, int d) {
  MESH;
  if (gtid() != 0 || d >= C->D) return;
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
__global__ void k_top_scatter(const FpMesh* __restrict__ Mp, int d) {
  MESH;
  if (C->top_stop || d >= C->D) return;
  const int lo = (1 << d) - 1, hi = (2 << d) - 1;
  for (int v0 = gwave() * 64; v0 < M.n; v0 += nwaves() * 64) {
    const int v = v0 + lane_id();
    const int t = v < M.n ? M.node_of[v] : -1;
    const bool act = t >= lo && t < hi;
    const int slot = wave_append_keyed(&C->tcur[0], act ? t : 0, act);
    if (act) M.tbuf[slot] = v;
  }
}
// one wave (and the whole LDS) per depth-d node
__global__ void __launch_bounds__(64) k_md_top(const FpMesh* __restrict__ Mp, int d) {
  MESH;
  FP_LDS_DECL;
  if (d >= uni(C->D)) return;
  const int t = uni((1 << d) - 1 + (int)blockIdx.x);
  if (!uni(C->tearly[t])) return;
  const int m = uni(C->tcnt[t]), off = uni(C->toff[t]), pos0 = uni(C->tpos[t]);
  if (off < 0 || m < 0 || (long long)off + m > M.n) {
    if (lane_id() == 0) fp_fail(C, FP_E_INTERNAL, FP_SITE_TOP, t);
    return;
  }
  md_node_list(M, t, M.tbuf + off, m, pos0, fp_lds, uni(M.lds_md));
}
// the schedule's ranges must be the ones the early orders took
__global__ void k_top_check(const FpMesh* __restrict__ Mp, int ntop) {
  MESH;
  ntop = min(ntop, C->nn);
  for (int t = gtid(); t < ntop; t += gsize())
    if (C->tearly[t] &&
        (M.nsize[t] != C->tcnt[t] || (M.nsize[t] > 0 && M.nbegin[t] != C->tpos[t])))
      fp_fail(C, FP_E_INTERNAL, FP_SITE_TOP, t);
}

// ==========================================================================
// elimination tree and column counts, bottom-up over the tree levels
// ==========================================================================
__global__ void k_sym_init(const FpMesh* __restrict__ Mp, int d) {
  MESH;
  if (gtid() == 0 && d <= C->D) {
    C->arena_top[d & 1] = 0;
    C->pool_top = 0;  // the pool holds one level's node scratch at a time
  }
}
__global__ void __launch_bounds__(FP_WG) k_sym_prep(const FpMesh* __restrict__ Mp, int d) {
  MESH;
  FP_LDS_DECL;
  if (d > C->D) return;
  const int lw = M.lds_bytes / 4 / FP_WAVES;
  int* slice = (int*)fp_lds + lw * wave_id();
  const int lo = (1 << d) - 1, cnt = 1 << d;
  for (int x = gwave(); x < cnt; x += nwaves()) sym_prep(M, lo + x, d, slice, lw);
}
// Elimination of the nodes whose queue links and forward rows fit in an LDS
// slice: cls 0 with four waves per workgroup (a quarter of the per-node LDS
// each), cls 1 with one wave owning the large slice.
__global__ void __launch_bounds__(FP_WG) k_sym_elim(const FpMesh* __restrict__ Mp, int d, int cls) {
  MESH;
  FP_LDS_DECL;
  if (d > C->D) return;
  const int nsl = cls == 0 ? FP_WAVES : 1;
  if (wave_id() >= nsl) return;
  int* slice = (int*)fp_lds + (M.lds_bytes / 4 / nsl) * wave_id();
  const int lo = (1 << d) - 1, cnt = 1 << d;
  const int wv = uni((int)blockIdx.x * nsl + wave_id()), nw = (int)gridDim.x * nsl;
  const long long lw = cls == 0 ? M.lds_bytes / 4 / nsl : M.lds_big / 4;
  for (int x = wv; x < cnt; x += nw) sym_elim<true>(M, lo + x, cls, slice, lw);
}
// nodes too large for the whole LDS: links and rows in global memory
__global__ void __launch_bounds__(FP_WG) k_sym_elim_glb(const FpMesh* __restrict__ Mp, int d) {
  MESH;
  if (d > C->D) return;
  const int lo = (1 << d) - 1, cnt = 1 << d;
  for (int x = gwave(); x < cnt; x += nwaves()) sym_elim<false>(M, lo + x, 2, nullptr, 0);
}
__global__ void __launch_bounds__(FP_WG) k_sym_emit(const FpMesh* __restrict__ Mp, int d) {
  MESH;
  if (d > C->D) return;
  const int lo = (1 << d) - 1, cnt = 1 << d;
  for (int x = gwave(); x < cnt; x += nwaves()) sym_emit(M, lo + x, d);
}
// The permuted pattern by position, for the symbolic stage: row p lists the
// positions of the neighbours of vertex vperm[p].  One pass with a thread per
// position; the symbolic kernels then read contiguous rows instead of
// chasing vperm -> row pointers -> columns -> viperm per entry.
__global__ void k_prow_deg(const FpMesh* __restrict__ Mp) {
  MESH;
  for (int p = gtid(); p < M.n; p += gsize()) {
    const int v = M.vperm[p];
    M.pcnt[p] = (unsigned)v < (unsigned)M.n ? M.grp[v + 1] - M.grp[v] : 0;
  }
}
__global__ void k_prow_fill(const FpMesh* __restrict__ Mp) {
  MESH;
  for (int p = gtid(); p < M.n; p += gsize()) {
    const int v = M.vperm[p];
    if ((unsigned)v >= (unsigned)M.n) continue;
    int o = M.prow[p];
    for (int e = M.grp[v]; e < M.grp[v + 1]; e++) M.pent[o++] = M.viperm[M.gci[e]];
  }
}
// nnz(L): the column counts summed per workgroup, one atomic each
__global__ void __launch_bounds__(FP_WG) k_nnzl(const FpMesh* __restrict__ Mp) {
  MESH_WG;
  __shared__ long long part[FP_WAVES];
  long long s = 0;
  for (int i = gtid(); i < M.n; i += gsize()) s += M.vcc[i];
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
__global__ void k_expand(const FpMesh* __restrict__ Mp) {
  MESH;
  const int nn = C->nn;
  const int b = M.b;
  const long long nd = M.n_dof;
  for (long long j = gtid(); j < nd; j += gsize()) {
    const int k = (int)(j / b), r = (int)(j - (long long)k * b);
    M.perm[j] = M.vperm[k] * b + r;
    M.iperm[j] = M.viperm[k] * b + r;
    M.colcount[j] = b * M.vcc[k] - r;
    M.parent[j] = r < b - 1 ? (int)(j + 1) : (M.vpar[k] < 0 ? -1 : M.vpar[k] * b);
  }
  if (M.gmap_out)
    for (int v = gtid(); v < M.n; v += gsize()) M.gmap_out[v] = M.gmap[v];
  if ((M.node_begin_out || M.node_size_out) && nn <= M.max_nodes_out)
    for (int x = gtid(); x < nn; x += gsize()) {
      if (M.node_begin_out) M.node_begin_out[x] = M.nbegin[x] * b;
      if (M.node_size_out) M.node_size_out[x] = M.nsize[x] * b;
    }
}
__global__ void k_finish(const FpMesh* __restrict__ Mp) {
  MESH0;
  if (gtid() != 0) return;
  const int nn = C->nn;
  if ((M.node_begin_out || M.node_size_out) && nn > M.max_nodes_out)
    fp_fail(C, FP_E_SCRATCH, FP_SITE_OUT_NODES, nn);
  *M.nnzL = (long long)M.b * M.b * C->nnzL - (long long)M.n * M.b * (M.b - 1) / 2;
  if (M.n_nodes_out) *M.n_nodes_out = nn;
  if (M.status_out) *M.status_out = C->err;
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

fp_status check_opts(const fp_options* o) {
  if (!o) return FP_ERR_ARG;
  if (o->patch_size < 1 || o->block_size < 1 || o->lloyd_iters < 0 || o->lloyd_iters > 64)
    return FP_ERR_ARG;
  if (o->schedule != FP_SCHED_LEVEL && o->schedule != FP_SCHED_POST) return FP_ERR_ARG;
  if (o->nd_level != -1 || (o->flags & ~(FP_FLAG_TIMING | FP_FLAG_VALIDATE)))
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

// one ordering job: launches in stream order, reads scalars through the
// handle's pinned buffer
// every launch of the pipeline goes through these, so that one kernel can be
// timed with events on the call's stream (fp_time_kernel)
#define FP_LAUNCH_(JOB, k, g, b, l, s, ...)                 \
  do {                                                     \
    const bool tk_ = (JOB).tk(#k);                         \
    if (tk_) (JOB).tk_begin(s);                            \
    hipLaunchKernelGGL(k, g, b, l, s, __VA_ARGS__);        \
    if (tk_) (JOB).tk_end(s);                              \
  } while (0)
#define FPLM(...) FP_LAUNCH_(*this, __VA_ARGS__)
#define FPL(...) FP_LAUNCH_(J, __VA_ARGS__)

struct Job {
  fp_handle* h;
  hipStream_t st;
  FpMesh hm;         // host copy of the job description
  const FpMesh* dm;  // device copy
  FpCtl* ctl;
  bool hip_failed = false;
  bool timing = false;
  bool validate = false;    // symmetry check of the pattern
  bool fixed = false;       // no side streams and no per-kernel events (static-scratch calls)
  bool side_open = false;   // work on the side stream not yet joined
  bool side2_open = false;  // same for the second side stream

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

  // timing of one kernel (fp_time_kernel): events around each of its launches
  bool tk(const char* name) const {
    return !fixed && h->tk_name[0] && strcmp(h->tk_name, name) == 0;
  }
  // the events go on the launch's own stream
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
    if (timing && hipEventRecord(h->ev[i], st) != hipSuccess) hip_failed = true;
  }
  int blocks(long long items, int per = FP_WG) const {
    long long b = (items + per - 1) / per;
    return (int)std::max(1ll, std::min(b, 8ll * h->ncu));
  }
  void check() {
    if (hipGetLastError() != hipSuccess) hip_failed = true;
  }
  // read `count` ints of the control block starting at `field`
  void read(const void* field, int count) {
    if (hipMemcpyAsync(h->host, field, 4 * count, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
      hip_failed = true;
  }
  int read1(const int* field) {
    read(field, 1);
    return hip_failed ? 0 : h->host[0];
  }
  unsigned err() {
    read(&ctl->err, 1);
    return hip_failed ? 0xFFFFFFFFu : (unsigned)h->host[0];
  }
  // exclusive scan of in[0..count) into out, total to *total; count is cap
  // or, with n_dev, the device value clamped to cap
  void scan(const int* in, int* out, int cap, int* total, const int* n_dev = nullptr) {
    const int np = std::max(1, std::min(1024, (cap + 4095) / 4096));
    const int chunk = std::max(1, (cap + np - 1) / np);
    FPLM(k_scan_part, dim3(np), dim3(FP_WG), 0, st, in, cap, n_dev, chunk, ctl->part);
    FPLM(k_scan_top, dim3(1), dim3(FP_WG), 0, st, ctl->part, np, total);
    FPLM(k_scan_apply, dim3(np), dim3(FP_WG), 0, st, in, out, cap, n_dev, chunk, ctl->part);
    check();
  }
  // Frontier BFS from the level-0 frontier already in place: `levels`
  // launches of a level each (a launch past the last level finds an empty
  // frontier and returns at once), then one workgroup continues from there
  // until a frontier comes out empty.  Nothing is read back.
  void bfs(int levels) {
    const int n = hm.n;
    const int L = std::max(0, std::min(levels, n));
    for (int k = 0; k < L; k++) FPLM(k_bfs_level, dim3(blocks(n)), dim3(FP_WG), 0, st, dm, k);
    FPLM(k_bfs_tail, dim3(1), dim3(1024), 0, st, dm, L);
    check();
  }
  // nseeds < 0: the device patch count
  void grow(int nseeds, int nseeds_exp, int levels) {
    const int n = hm.n;
    FPLM(k_key_unset, dim3(blocks(n)), dim3(FP_WG), 0, st, dm);
    FPLM(k_seed_push, dim3(blocks(nseeds_exp)), dim3(FP_WG), 0, st, dm, nseeds);
    check();
    bfs(levels);
  }
};

// The side stream and its events, created on first use: every stream takes
// one of the device's hardware queues in turn, so a handle that never uses
// it (a lane of the batched calls) should not hold one.
bool ensure_side(fp_handle* h) {
  if (h->side) return true;
  hipStream_t s[3] = {nullptr, nullptr, nullptr};
  int ns = 0;
  while (ns < 3 && hipStreamCreateWithFlags(&s[ns], hipStreamNonBlocking) == hipSuccess) ns++;
  hipEvent_t* ev[7] = {&h->ev_top[0], &h->ev_top[1], &h->ev_top[2], &h->ev_join,
                       &h->ev_md,     &h->ev_join2,  &h->ev_join3};
  int ne = 0;
  while (ns == 3 && ne < 7 && hipEventCreateWithFlags(ev[ne], hipEventDisableTiming) == hipSuccess)
    ne++;
  if (ns < 3 || ne < 7) {
    for (int j = 0; j < ne; j++) (void)hipEventDestroy(*ev[j]);
    for (int j = 0; j < ns; j++) (void)hipStreamDestroy(s[j]);
    (void)hipGetLastError();
    return false;
  }
  h->side = s[0];
  h->side2 = s[1];
  h->side3 = s[2];
  return true;
}

// Levels of a growth BFS launched one by one before the tail takes over:
// about twice the radius of a patch of S vertices on a triangle mesh, at
// most 64.  The distance BFS of Lloyd's step runs inside patches (half).
static int bfs_levels(int S, bool inner) {
  const int r = (int)std::ceil(std::sqrt((double)std::max(S, 1)));
  return std::min(64, (inner ? r : 2 * r) + 4);
}
static int ceil_log2(long long x) {
  int d = 0;
  while ((1ll << d) < x) d++;
  return d;
}

// Queue the whole pipeline on J.st (and the side streams, joined back).
// Nothing is read back to the host: counts known only on the device (patches,
// tree depth, arcs, frontier sizes) are read there, launch grids come from
// capacities or expected values, and every kernel returns at once once an
// earlier stage has raised an error.  The tree depth D is at most
// ceil(log2 n); levels past the expected depth get small grids.
fp_status run_job(Job& J) {
  const int n = J.hm.n;
  const FpMesh* dm = J.dm;
  hipStream_t st = J.st;
  FpCtl* C = J.ctl;
  auto B = [&](long long items) { return dim3(J.blocks(items)); };
  const dim3 T(FP_WG);
  const int P0 = n > 0 ? (int)(((long long)n + J.hm.S - 1) / J.hm.S) : 0;
  const int Pexp = std::max(P0, 1);            // expected patch count (exact without orphans)
  const int Dexp = ceil_log2(Pexp);             // expected tree depth
  const int Dmax = ceil_log2(std::max(n, 1));   // P <= n
  auto BL = [&](int d, long long items) {       // grid of a tree level
    return d <= Dexp ? B(items) : dim3(1);
  };

  // ingest
  J.mark(0);
  FPL(k_ingest, B(n), T, 0, st, dm, 0);
  FPL(k_ingest_long, dim3(J.h->ncu), T, 0, st, dm, 0);
  J.scan(J.hm.pcnt, J.hm.grp, n, &C->nnz_g);
  FPL(k_check_graph, dim3(1), dim3(64), 0, st, dm);
  FPL(k_set, dim3(1), dim3(1), 0, st, J.hm.grp + n, &C->nnz_g);
  FPL(k_ingest, B(n), T, 0, st, dm, 1);
  FPL(k_ingest_long, dim3(J.h->ncu), T, 0, st, dm, 1);
  if (J.validate) FPL(k_validate, B(n), T, 0, st, dm);
  J.check();

  // patches
  J.mark(1);
  if (J.hm.user_gmap) {
    FPL(k_user_gmap, B(n), T, 0, st, dm);
    J.check();
  } else if (n > 0) {
    const int Lg = bfs_levels(J.hm.S, false), Ld = bfs_levels(J.hm.S, true);
    FPL(k_seeds, dim3(J.blocks(P0, FP_WAVES)), T, 0, st, dm, P0);
    J.check();
    J.grow(P0, P0, Lg);
    FPL(k_count_unset, B(n), T, 0, st, dm);
    // components growth did not reach (none on a connected mesh: every
    // kernel here then returns at once)
    FPL(k_cc_init, B(n), T, 0, st, dm);
    for (int r = 0; r < FP_CC_ROUNDS; r++) {
      FPL(k_cc_hook, B(n), T, 0, st, dm, r);
      FPL(k_cc_jump, B(n), T, 0, st, dm, r);
    }
    FPL(k_cc_tail, dim3(1), dim3(1024), 0, st, dm, FP_CC_ROUNDS);
    FPL(k_cc_flags, B(n), T, 0, st, dm);
    J.scan(J.hm.pcnt, J.hm.pcnt, n, &C->nroot, &C->ccn);
    FPL(k_cc_label, B(n), T, 0, st, dm);
    J.check();
    for (int it = 0; it < J.hm.lloyd; it++) {
      FPL(k_lloyd_gmap, B(n), T, 0, st, dm);
      FPL(k_lloyd_bnd, B(n), T, 0, st, dm);
      J.check();
      J.bfs(Ld);
      FPL(k_lloyd_best, B(n), T, 0, st, dm);
      FPL(k_lloyd_seed, B(Pexp), T, 0, st, dm);
      J.check();
      J.grow(-1, Pexp, Lg);
    }
    FPL(k_gmap_final, B(n), T, 0, st, dm);
    J.check();
  }

  // quotient graph (P on the device)
  J.mark(2);
  FPL(k_fill_n, B(Pexp + 1), T, 0, st, J.hm.pcnt, &C->P, 1, n + 1, 0);
  FPL(k_fill, dim3(1), dim3(64), 0, st, &C->nbnd, 1, 0);
  FPL(k_patch_count, B(n), T, 0, st, dm);
  FPL(k_copy_n, B(Pexp), T, 0, st, J.hm.wp, J.hm.pcnt, &C->P, n);
  J.check();
  J.scan(J.hm.pcnt, J.hm.pptr, n, &C->tot, &C->P);
  FPL(k_set_at, dim3(1), dim3(1), 0, st, J.hm.pptr, &C->P, n, &C->tot);
  FPL(k_copy_n, B(Pexp), T, 0, st, J.hm.pcnt, J.hm.pptr, &C->P, n);
  FPL(k_patch_scatter, B(n), T, 0, st, dm);
  // a patch-id bitmap per wave when four of them fit in 64 KB of LDS (for
  // the expected patch count; the kernel checks the actual one)
  const int qbw = (long long)(Pexp + 31) / 32 * 4 * FP_WAVES <= 65536 ? (Pexp + 31) / 32 : 0;
  FPL(k_qrow, dim3(J.blocks(Pexp, FP_WAVES)), T, qbw * 4 * FP_WAVES, st, dm, 0, qbw);
  J.check();
  J.scan(J.hm.pcnt, J.hm.qptr, n, &C->nq, &C->P);
  FPL(k_set_at, dim3(1), dim3(1), 0, st, J.hm.qptr, &C->P, n, &C->nq);
  FPL(k_check_arcs, dim3(1), dim3(64), 0, st, dm);
  FPL(k_qrow, dim3(J.blocks(Pexp, FP_WAVES)), T, qbw * 4 * FP_WAVES, st, dm, 1, qbw);
  J.check();

  // separator tree
  J.mark(3);
  FPL(k_sep_init, B(n), T, 0, st, dm);
  // top separators ordered early on the side streams (level order only:
  // there their ranges depend on the top levels alone)
  const int TL = J.hm.sched == 0 && !J.fixed && J.h->side_ok && ensure_side(J.h)
                     ? std::min(FP_TOP_LEVELS, Dmax)
                     : 0;
  const int ntop = (1 << TL) - 1;
  for (int d = 0; d < Dmax; d++) {
    FPL(k_level_begin, BL(d, 8ll * Pexp), T, 0, st, dm, d);
    FPL(k_arcs, BL(d, n), T, 0, st, dm, d);
    {
      // LDS for the local quotient subgraphs: a node at depth d holds about
      // 2^(Dexp-d) patches.  While the level has no more nodes than CUs,
      // each workgroup takes the large LDS (quotient degrees can pass 8);
      // deeper, about 8 alive arcs per patch, so several workgroups share a
      // CU (a node that does not fit runs from global memory).  The
      // kernel's static LDS comes on top.
      const long long cap = 1ll << std::max(0, Dexp - d);
      const long long want =
          (1ll << d) <= J.h->ncu ? J.h->lds_big : (4 * (13 * cap + 1) + 255) & ~255ll;
      const int lb = (int)std::min<long long>(J.h->lds_big - 1024, want);
      const dim3 gb = d <= Dexp ? dim3(std::min(1 << std::min(d, 30), 4 * J.h->ncu)) : dim3(1);
      FPL(k_bisect, gb, T, lb, st, dm, d, lb);
    }
    FPL(k_cand, BL(d, n), T, 0, st, dm, d);
    FPL(k_mark, BL(d, n), T, 0, st, dm, d);
    if (d < TL) {
      FPL(k_top_count, B(n), T, 0, st, dm, d);
      FPL(k_top_place, dim3(1), dim3(64), 0, st, dm, d);
      FPL(k_top_scatter, B(n), T, 0, st, dm, d);
      // one stream per level, so a level does not wait for the one above;
      // the large local-order classes follow on the second and third
      hipStream_t sd = d == 0 ? J.h->side : d == 1 ? J.h->side2 : J.h->side3;
      if (hipEventRecord(J.h->ev_top[d], st) != hipSuccess ||
          hipStreamWaitEvent(sd, J.h->ev_top[d], 0) != hipSuccess)
        J.hip_failed = true;
      if (d == 0)
        J.side_open = true;
      else
        J.side2_open = true;
      FPL(k_md_top, dim3(1 << d), dim3(64), J.h->lds_md, sd, dm, d);
    }
    J.check();
  }
  FPL(k_leaves, B(n), T, 0, st, dm);

  // grouping in schedule order (heap size nn on the device)
  J.mark(4);
  const int NNexp = (2 << Dexp) - 1;
  FPL(k_nsize, B(n), T, 0, st, dm);
  FPL(k_nsize_count, B(n), T, 0, st, dm);
  FPL(k_sched_place, B(NNexp), T, 0, st, dm);
  J.check();
  J.scan(J.hm.sbuf, J.hm.sbuf, J.hm.NNcap, &C->tot, &C->nn);
  FPL(k_nbegin, B(NNexp), T, 0, st, dm);
  FPL(k_scatter, B(n), T, 0, st, dm);
  if (ntop) FPL(k_top_check, dim3(1), dim3(64), 0, st, dm, ntop);
  J.check();

  // local orders
  J.mark(5);
  FPL(k_fill, dim3(1), dim3(64), 0, st, C->task_cnt, 16, 0);
  FPL(k_md_tasks, dim3(1), dim3(1024), 0, st, dm, ntop);
  {
    // The largest class (one wave per CU, the longest nodes) goes first on
    // this stream, so its workgroups take their CUs before the others fill
    // the rest; class 1 follows the depth-1 orders on the second side
    // stream, classes 2 and 3 the depth-2 orders on the third.
    const bool two = !J.fixed && J.h->side_ok && ensure_side(J.h);
    if (two) {
      if (hipEventRecord(J.h->ev_md, st) != hipSuccess ||
          hipStreamWaitEvent(J.h->side2, J.h->ev_md, 0) != hipSuccess ||
          hipStreamWaitEvent(J.h->side3, J.h->ev_md, 0) != hipSuccess)
        J.hip_failed = true;
      J.side2_open = true;
    }
    for (int c = 0; c < FP_MD_CLASSES; c++) {
      hipStream_t sc = !two || c == 0 ? st : c == 1 ? J.h->side2 : J.h->side3;
      FPL(k_md, dim3(2 * J.h->ncu), T, c == 3 ? J.h->lds_bytes : J.h->lds_md, sc, dm, c);
    }
  }
  J.join_side();
  J.check();

  // elimination tree and column counts, bottom-up over the tree levels (a
  // node whose local order failed raised an error: these kernels then return)
  J.mark(6);
  FPL(k_prow_deg, B(n), T, 0, st, dm);
  J.scan(J.hm.pcnt, J.hm.prow, n, &C->tot);
  FPL(k_set, dim3(1), dim3(1), 0, st, J.hm.prow + n, &C->tot);
  FPL(k_prow_fill, B(n), T, 0, st, dm);
  for (int d = Dmax; d >= 0; d--) {
    const int cnt = 1 << d;
    const bool big = d <= Dexp;
    const dim3 G(big ? std::max(1, std::min((cnt + FP_WAVES - 1) / FP_WAVES, 16 * J.h->ncu)) : 1);
    FPL(k_sym_init, dim3(1), dim3(64), 0, st, dm, d);
    FPL(k_sym_prep, G, T, J.h->lds_bytes, st, dm, d);
    const dim3 G1(big ? std::max(1, std::min(cnt, 4 * J.h->ncu)) : 1);
    FPL(k_sym_elim, G, T, J.h->lds_bytes, st, dm, d, 0);
    FPL(k_sym_elim, G1, T, J.h->lds_big, st, dm, d, 1);
    FPL(k_sym_elim_glb, G, T, 0, st, dm, d);
    FPL(k_sym_emit, G, T, 0, st, dm, d);
    J.check();
  }
  FPL(k_nnzl, dim3(std::min(J.blocks(n), 2 * J.h->ncu)), T, 0, st, dm);

  // outputs
  J.mark(7);
  FPL(k_expand, B(std::max<long long>(J.hm.n_dof, NNexp)), T, 0, st, dm);
  FPL(k_finish, dim3(1), dim3(64), 0, st, dm);
  J.mark(8);
  J.check();
  return J.hip_failed ? FP_ERR_HIP : FP_OK;
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
                          big) != hipSuccess) {
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
          hipSuccess ||
      hipHostMalloc((void**)&H->host, 8192, hipHostMallocDefault) != hipSuccess) {
    delete H;
    return FP_ERR_HIP;
  }
  H->ncu = std::max(1, ncu);
  bind_scratch(H->device);
  H->lds_bytes = FP_LDS_BYTES;
  H->lds_big = big_lds(H->device);
  H->lds_md = std::min(H->lds_big, FP_MD_LDS);
  H->side_ok = true;
  H->tk_name[0] = 0;
  H->tk_n = 0;
  H->tk_failed = false;
  for (int i = 0; i <= FP_NSTAGE; i++)
    if (hipEventCreate(&H->ev[i]) != hipSuccess) {
      for (int j = 0; j < i; j++) (void)hipEventDestroy(H->ev[j]);
      (void)hipHostFree(H->host);
      delete H;
      return FP_ERR_HIP;
    }
  if (hipEventCreateWithFlags(&H->ev_bfs, hipEventDisableTiming) != hipSuccess) {
    for (int j = 0; j <= FP_NSTAGE; j++) (void)hipEventDestroy(H->ev[j]);
    (void)hipHostFree(H->host);
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
  for (FpLane& L : h->lanes) {
    (void)hipStreamSynchronize(L.st);
    (void)hipStreamDestroy(L.st);
    (void)fp_destroy(L.h);
  }
  h->lanes.clear();
  if (h->side) {
    for (hipStream_t s : {h->side, h->side2, h->side3}) {
      (void)hipStreamSynchronize(s);
      (void)hipStreamDestroy(s);
    }
    for (int i = 0; i < 3; i++) (void)hipEventDestroy(h->ev_top[i]);
    for (hipEvent_t e : {h->ev_join, h->ev_md, h->ev_join2, h->ev_join3}) (void)hipEventDestroy(e);
  }
  for (hipEvent_t e : h->tk_ev) (void)hipEventDestroy(e);
  for (int i = 0; i <= FP_NSTAGE; i++) (void)hipEventDestroy(h->ev[i]);
  (void)hipEventDestroy(h->ev_bfs);
  if (h->host) (void)hipHostFree(h->host);
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
fp_status order_impl(fp_handle* h, const fp_csr* A, const int32_t* user_gmap,
                     const fp_options* opts, void* workspace, size_t ws_bytes, fp_result* out,
                     void* stream, bool fixed) {
  if (!h || !out || !workspace) return FP_ERR_ARG;
  fp_status s = check_opts(opts);
  if (s) return s;
  if ((s = check_csr(A, opts->block_size))) return s;
  if (!out->perm || !out->iperm || !out->parent || !out->colcount || !out->nnzL) return FP_ERR_ARG;
  if ((out->node_begin || out->node_size) && out->max_nodes < 1) return FP_ERR_ARG;
  Plan P;
  if (!make_plan(A->n, opts->block_size, A->nnz, opts->patch_size, &P)) return FP_ERR_ARG;
  if (ws_bytes < P.total) return FP_ERR_SIZE;
  Job J;
  J.h = h;
  J.st = (hipStream_t)stream;
  FpMesh& M = J.hm;
  memset(&M, 0, sizeof(M));
  char* ws = (char*)workspace;
  fill_mesh(P, ws, &M);
  M.rp32 = A->rowptr32;
  M.rp64 = (const long long*)A->rowptr64;
  M.ci_in = A->colind;
  M.nnz_in = A->nnz;
  M.user_gmap = user_gmap;
  M.S = opts->patch_size;
  M.lloyd = opts->lloyd_iters;
  M.sched = opts->schedule;
  M.seed = opts->seed;
  M.perm = out->perm;
  M.iperm = out->iperm;
  M.parent = out->parent;
  M.colcount = out->colcount;
  M.nnzL = (long long*)out->nnzL;
  M.node_begin_out = out->node_begin;
  M.node_size_out = out->node_size;
  M.gmap_out = out->gmap;
  M.n_nodes_out = out->n_nodes;
  M.status_out = out->status;
  M.max_nodes_out = out->max_nodes;
  M.lds_bytes = h->lds_bytes;
  M.lds_big = h->lds_big;
  M.lds_md = h->lds_md;
  J.ctl = M.ctl;
  J.dm = (const FpMesh*)(ws + P.o_mesh);
  J.fixed = fixed;
  J.timing = !fixed && (opts->flags & FP_FLAG_TIMING) != 0;
  J.validate = (opts->flags & FP_FLAG_VALIDATE) != 0;
  h->timed = false;
  h->tk_n = 0;
  h->tk_failed = false;
  // control block cleared, job description copied in as a kernel argument
  // (so no host buffer has to outlive the call)
  const int words = (int)(sizeof(FpCtl) / 4);
  hipLaunchKernelGGL(k_fill, dim3((words + FP_WG - 1) / FP_WG), dim3(FP_WG), 0, J.st, (int*)(FpCtl*)M.ctl,
                     words, 0);
  hipLaunchKernelGGL(k_put_mesh, dim3(1), dim3(64), 0, J.st, M, (FpMesh*)J.dm);
  if (hipGetLastError() != hipSuccess) return FP_ERR_HIP;
  s = run_job(J);
  J.join_side();  // a call that stopped early still leaves no work behind it
  h->timed = J.timing && s == FP_OK;
  return s;
}

}  // namespace

extern "C" {

fp_status fp_order(fp_handle* h, const fp_csr* A, const int32_t* user_gmap,
                   const fp_options* opts, void* workspace, size_t ws_bytes, fp_result* out,
                   void* stream) {
  return order_impl(h, A, user_gmap, opts, workspace, ws_bytes, out, stream, false);
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
