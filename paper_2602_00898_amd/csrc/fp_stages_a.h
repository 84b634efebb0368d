// fp_stages_a.h -- graph ingest, patching, patch structures and the quotient
// graph, as team-wide device stages.  Every result is a fixed point or a
// set function of the input (integer min/max/add atomics only), so it does
// not depend on thread or workgroup order.
#pragma once

#include "fp_device.h"
#include "fp_mesh.h"

#define FP_UNSET 0xFFFFFFFFFFFFFFFFull

// SplitMix64 (Steele, Lea, Flood, OOPSLA 2014): output i+1 of the generator
// seeded with `seed` -- the seed-selection hash of the patching stage.
__device__ __forceinline__ uint64_t fp_mix64(uint64_t seed, uint64_t i) {
  uint64_t z = seed + (i + 1) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__device__ __forceinline__ long long rp_at(const FpMesh& M, long long r) {
  return M.rp64 ? M.rp64[r] : (long long)M.rp32[r];
}

// --------------------------------------------------------------------------
// Ingest: graph of A without its diagonal; block rows b*v..b*v+b-1 merge
// into vertex v (Sec. 4.1 Step 2, Sec. 6.5).  Duplicates are dropped for
// rows up to 512 entries; every later stage treats rows as sets, so longer
// rows may keep duplicates.
// --------------------------------------------------------------------------
__device__ int gather_vertex_row(const FpMesh& M, int v, int* out, unsigned* eb) {
  const int b = M.b;
  const long long r0 = (long long)v * b;
  long long e0 = rp_at(M, r0), e1 = rp_at(M, r0 + b);
  if (e0 < 0 || e1 < e0 || e1 > M.nnz_in) {
    *eb |= FP_E_INDEX;
    return 0;
  }
  const bool dedup = (e1 - e0) <= 512;
  int cnt = 0;
  for (long long e = e0; e < e1; e++) {
    int c = M.ci_in[e];
    if (c < 0 || (long long)c >= M.n_dof) {
      *eb |= FP_E_INDEX;
      continue;
    }
    int u = c / b;
    if (u == v) continue;
    bool dup = false;
    if (dedup)
      for (long long f = e0; f < e; f++) {
        int c2 = M.ci_in[f];
        if (c2 >= 0 && (long long)c2 < M.n_dof && c2 / b == u) {
          dup = true;
          break;
        }
      }
    if (dup) continue;
    if (out) out[cnt] = u;
    cnt++;
  }
  return cnt;
}

__device__ void stage_ingest(const Team& T, const FpMesh& M, int* lds_tmp) {
  FpCtl* C = M.ctl;
  unsigned eb = 0;
  for (int v = T.gtid(); v < M.n; v += T.gsize()) M.pcnt[v] = gather_vertex_row(M, v, nullptr, &eb);
  if (eb) atomicOr(&C->err, eb);
  T.sync();
  team_excl_scan(T, M.pcnt, M.grp, M.n, C->part, &C->nnz_g, lds_tmp);
  if (C->nnz_g > M.Ecap || C->nnz_g < 0) {
    if (T.gtid() == 0) atomicOr(&C->err, FP_E_SCRATCH);
    return;
  }
  if (T.gtid() == 0) M.grp[M.n] = C->nnz_g;
  eb = 0;
  for (int v = T.gtid(); v < M.n; v += T.gsize()) gather_vertex_row(M, v, M.gci + M.grp[v], &eb);
  T.sync();
}

// --------------------------------------------------------------------------
// Patching (Sec. 4.1 Step 1; Lloyd's algorithm, Sec. 6).
// Growth computes, for every vertex, (hop distance to the nearest seed, id
// of the nearest seed with ties to the lowest id) as a 64-bit key fixed
// point: level-synchronous frontiers with atomicMin on (dist << 32 | id).
// --------------------------------------------------------------------------

// frontier BFS over the whole graph from the vertices in M.fa[0..nf) whose
// keys are already set; keys of newly reached vertices become
// key(parent) + (1 << 32) minimised over parents.  Returns when no vertex
// was reached.  Counters C->fcount rotate over three slots.
__device__ void team_bfs_keys(const Team& T, const FpMesh& M, unsigned long long* key, int nf0) {
  FpCtl* C = M.ctl;
  int* cur = M.fa;
  int* nxt = M.fb;
  int nf = nf0;
  int lvl = 0;
  if (T.gtid() == 0) {
    C->fcount[1] = 0;
    C->fcount[2] = 0;
  }
  T.sync();
  while (nf > 0 && !T.failed()) {
    int* cnt_next = &C->fcount[(lvl + 1) % 3];
    if (T.gtid() == 0) C->fcount[(lvl + 2) % 3] = 0;
    for (int f = T.gtid(); f < nf; f += T.gsize()) {
      int v = cur[f];
      unsigned long long kv = key[v] + (1ull << 32);
      for (int e = M.grp[v]; e < M.grp[v + 1]; e++) {
        int u = M.gci[e];
        if (key[u] <= kv) continue;
        unsigned long long old = atomicMin(&key[u], kv);
        if (old == FP_UNSET) nxt[atomicAdd(cnt_next, 1)] = u;
      }
    }
    T.sync();
    nf = *cnt_next;
    int* t = cur;
    cur = nxt;
    nxt = t;
    lvl++;
  }
  T.sync();
}

__device__ void grow_from_seeds(const Team& T, const FpMesh& M, int nseeds) {
  for (int v = T.gtid(); v < M.n; v += T.gsize()) M.key[v] = FP_UNSET;
  T.sync();
  for (int k = T.gtid(); k < nseeds; k += T.gsize()) {
    int s = M.seeds[k];
    atomicMin(&M.key[s], (unsigned long long)k);
    M.fa[k] = s;
  }
  T.sync();
  team_bfs_keys(T, M, M.key, nseeds);
}

__device__ void stage_patches(const Team& T, const FpMesh& M, int* lds_tmp) {
  FpCtl* C = M.ctl;
  const int n = M.n;
  if (M.user_gmap) {
    // user-provided groups (Sec. 5): ids must lie in [0, n)
    int mx = -1;
    for (int v = T.gtid(); v < n; v += T.gsize()) {
      int g = M.user_gmap[v];
      if (g < 0 || g >= n) {
        atomicOr(&C->err, FP_E_GMAP);
        g = 0;
      }
      M.gmap[v] = g;
      mx = max(mx, g);
    }
    mx = (int)wave_max_u32((uint32_t)(mx + 1));
    if (lane_id() == 0 && mx > 0) atomicMax(&C->P, mx);
    T.sync();
    return;
  }
  const int S = M.S;
  const int P0 = (int)(((long long)n + S - 1) / S);
  // one seed per block of S consecutive ids: least (hash, id)
  for (int blk = T.gwave(); blk < P0; blk += T.nwaves()) {
    const long long lo = (long long)blk * S, hi = min((long long)n, lo + S);
    uint64_t bh = FP_UNSET;
    uint32_t bv = 0xFFFFFFFFu;
    for (long long v = lo + lane_id(); v < hi; v += 64) {
      uint64_t h = fp_mix64(M.seed, (uint64_t)v);
      if (h < bh) {
        bh = h;
        bv = (uint32_t)v;
      }
    }
    uint64_t hm = wave_min_u64(bh);
    uint32_t vm = wave_min_u32(bh == hm ? bv : 0xFFFFFFFFu);
    if (lane_id() == 0) M.seeds[blk] = (int)vm;
  }
  if (T.gtid() == 0) {
    C->P0 = P0;
    C->norphan = 0;
    C->nroot = 0;
  }
  T.sync();
  grow_from_seeds(T, M, P0);

  // components without a seed become patches: min-label fixed point over the
  // unlabelled vertices, ids P0 + rank of the component's lowest vertex
  int cnt = 0;
  for (int v = T.gtid(); v < n; v += T.gsize()) cnt += (M.key[v] == FP_UNSET);
  cnt = wave_sum_i32(cnt);
  if (lane_id() == 0 && cnt) atomicAdd(&C->norphan, cnt);
  T.sync();
  int P = P0;
  if (C->norphan > 0) {
    int* comp = M.fb;
    for (int v = T.gtid(); v < n; v += T.gsize()) comp[v] = (M.key[v] == FP_UNSET) ? v : -1;
    T.sync();
    if (T.gtid() == 0) C->chg[0] = C->chg[1] = C->chg[2] = 0;
    T.sync();
    for (int it = 0; it < (1 << 30); it++) {
      if (T.gtid() == 0) C->chg[(it + 1) % 3] = 0;
      int ch = 0;
      for (int v = T.gtid(); v < n; v += T.gsize()) {
        if (comp[v] < 0) continue;
        int cv = comp[v];
        for (int e = M.grp[v]; e < M.grp[v + 1]; e++) {
          int u = M.gci[e];
          int cu = comp[u];
          if (cu >= 0 && cu < cv) {
            atomicMin(&comp[cv], cu);  // hook the larger root under the smaller
            atomicMin(&comp[v], cu);
            ch = 1;
          }
        }
      }
      T.sync();
      for (int v = T.gtid(); v < n; v += T.gsize()) {
        if (comp[v] < 0) continue;
        int c = comp[v];
        while (comp[c] != c) c = comp[c];
        if (c != comp[v]) {
          comp[v] = c;
          ch = 1;
        }
      }
      if (ch) C->chg[it % 3] = 1;
      T.sync();
      if (!C->chg[it % 3] || T.failed()) break;
    }
    // rank roots by id
    for (int v = T.gtid(); v < n; v += T.gsize()) M.pcnt[v] = (comp[v] == v) ? 1 : 0;
    T.sync();
    team_excl_scan(T, M.pcnt, M.pcnt, n, C->part, &C->nroot, lds_tmp);
    for (int v = T.gtid(); v < n; v += T.gsize()) {
      if (comp[v] < 0) continue;
      int id = P0 + M.pcnt[comp[v]];
      M.key[v] = (unsigned long long)id;
      if (comp[v] == v) M.seeds[id] = v;
    }
    T.sync();
    P = P0 + C->nroot;
  }

  // Lloyd re-centre: new seed = vertex farthest from the patch boundary
  // (the distance inside the patch equals the distance to the boundary set
  // of the whole graph, because any path out of a patch passes its own
  // boundary first), ties to the lowest id; patches without a boundary keep
  // their seed; then regrow with the same ids.
  for (int it = 0; it < M.lloyd; it++) {
    for (int v = T.gtid(); v < n; v += T.gsize()) M.gmap[v] = (int)(M.key[v] & 0xFFFFFFFFu);
    for (int p = T.gtid(); p < P; p += T.gsize()) M.best[p] = 0;
    if (T.gtid() == 0) C->fcount[3] = 0;
    T.sync();
    for (int v = T.gtid(); v < n; v += T.gsize()) {
      int g = M.gmap[v];
      bool isb = false;
      for (int e = M.grp[v]; e < M.grp[v + 1] && !isb; e++) isb = (M.gmap[M.gci[e]] != g);
      M.key[v] = isb ? 0ull : FP_UNSET;
      if (isb) M.fa[atomicAdd(&C->fcount[3], 1)] = v;
    }
    T.sync();
    team_bfs_keys(T, M, M.key, C->fcount[3]);
    for (int v = T.gtid(); v < n; v += T.gsize()) {
      unsigned long long k = M.key[v];
      if (k == FP_UNSET) continue;
      unsigned long long cand = ((k >> 32) << 32) | (unsigned long long)(0xFFFFFFFFu - (unsigned)v);
      atomicMax(&M.best[M.gmap[v]], cand | (1ull << 63));
    }
    T.sync();
    for (int p = T.gtid(); p < P; p += T.gsize()) {
      unsigned long long bb = M.best[p];
      if (bb) M.seeds[p] = (int)(0xFFFFFFFFu - (unsigned)(bb & 0xFFFFFFFFu));
    }
    T.sync();
    grow_from_seeds(T, M, P);
  }
  for (int v = T.gtid(); v < n; v += T.gsize()) {
    const unsigned long long k = M.key[v];
    if (k == FP_UNSET) atomicOr(&C->err, FP_E_INTERNAL);
    M.gmap[v] = k == FP_UNSET ? 0 : (int)(k & 0xFFFFFFFFu);
  }
  if (T.gtid() == 0) C->P = P;
  T.sync();
}

// --------------------------------------------------------------------------
// Patch members, boundary list and the quotient graph (Sec. 2: nodes are
// patches, arcs join patches adjacent in G), built once (Sec. 5).
// --------------------------------------------------------------------------
__device__ void stage_quotient(const Team& T, const FpMesh& M, int* lds_tmp) {
  FpCtl* C = M.ctl;
  const int n = M.n;
  const int P = C->P;
  for (int p = T.gtid(); p <= P; p += T.gsize()) M.pcnt[p] = 0;
  if (T.gtid() == 0) {
    C->nbnd = 0;
  }
  T.sync();
  for (int v = T.gtid(); v < n; v += T.gsize()) {
    int g = M.gmap[v];
    atomicAdd(&M.pcnt[g], 1);
    bool isb = false;
    for (int e = M.grp[v]; e < M.grp[v + 1] && !isb; e++) isb = (M.gmap[M.gci[e]] != g);
    if (isb) M.bnd[atomicAdd(&C->nbnd, 1)] = v;
  }
  T.sync();
  for (int p = T.gtid(); p < P; p += T.gsize()) M.wp[p] = M.pcnt[p];
  team_excl_scan(T, M.pcnt, M.pptr, P, C->part, &C->tot, lds_tmp);
  for (int p = T.gtid(); p < P; p += T.gsize()) M.pcnt[p] = M.pptr[p];
  if (T.gtid() == 0) M.pptr[P] = n;
  T.sync();
  for (int v = T.gtid(); v < n; v += T.gsize()) M.pvtx[atomicAdd(&M.pcnt[M.gmap[v]], 1)] = v;
  T.sync();
  // distinct neighbour patches of patch p, ascending, by repeated wave-wide
  // minimum over the foreign neighbours of its members
  for (int pass = 0; pass < 2; pass++) {
    for (int p = T.gwave(); p < P; p += T.nwaves()) {
      const int a0 = M.pptr[p], a1 = M.pptr[p + 1];
      int last = -1, cnt = 0;
      int* out = pass ? M.qci + M.qptr[p] : nullptr;
      while (true) {
        uint32_t m = 0xFFFFFFFFu;
        for (int i = a0 + lane_id(); i < a1; i += 64) {
          int v = M.pvtx[i];
          for (int e = M.grp[v]; e < M.grp[v + 1]; e++) {
            int q = M.gmap[M.gci[e]];
            if (q != p && q > last && (uint32_t)q < m) m = (uint32_t)q;
          }
        }
        m = wave_min_u32(m);
        if (m == 0xFFFFFFFFu) break;
        if (out && lane_id() == 0) out[cnt] = (int)m;
        cnt++;
        last = (int)m;
      }
      if (!pass && lane_id() == 0) M.pcnt[p] = cnt;
    }
    T.sync();
    if (!pass) {
      team_excl_scan(T, M.pcnt, M.qptr, P, C->part, &C->nq, lds_tmp);
      if (T.gtid() == 0) M.qptr[P] = C->nq;
      if (C->nq > M.Ecap) {
        if (T.gtid() == 0) atomicOr(&C->err, FP_E_SCRATCH);
        return;
      }
      T.sync();
    }
  }
}

// arc index of (p, q) in the sorted quotient row of p, -1 if absent
__device__ __forceinline__ int arc_index(const FpMesh& M, int p, int q) {
  int lo = M.qptr[p], hi = M.qptr[p + 1];
  while (lo < hi) {
    int mid = (lo + hi) >> 1;
    if (M.qci[mid] < q)
      lo = mid + 1;
    else
      hi = mid;
  }
  return (lo < M.qptr[p + 1] && M.qci[lo] == q) ? lo : -1;
}
