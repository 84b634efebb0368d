// fp_stages_amd.h -- approximate-minimum-degree local orders (Sec. 4.3 Step
// 4 names AMD as the local order; the degree bound of Amestoy, Davis and
// Duff, SIAM J. Matrix Anal. Appl. 17(4), 1996).
//
// Elimination on the quotient graph of the node's induced subgraph: a
// variable i keeps its variable neighbours A_i and adjacent elements E_i,
// an element e its variables L_e.  Eliminating the pivot p forms
//   L_p = (A_p + union of L_e over e in E_p) minus p,
// absorbs every element of E_p, sets A_i = A_i minus (L_p + p) and
// E_i = (E_i minus E_p) + p for each i in L_p, and bounds the degree of i by
//   min( r - 1, dbar_i + |L_p| - 1, |A_i| + |L_p| - 1 + sum_{e in E_i, e != p} |L_e \ L_p| )
// with r the variables left; |L_e \ L_p| is |L_e| less the members of L_p
// that touch e.  Each variable is its own supervariable (no mass
// elimination, no aggressive absorption); the pivot is the least
// (bound, local index), the local index being the vertex's rank in the node.
//
// One wave owns a node; the quotient graph sits in a slice of the global
// pool: rows A_i and E_i with the vertex's graph degree as capacity (an
// element next to i holds one of i's original neighbours, so |E_i| never
// passes it), element lists in an arena of sum-of-degrees + 2m words that is
// compacted in creation order when the next L_p might not fit (the live
// lists never hold more than the sum of degrees).  The pivot search keeps
// per-64 group minima of the keys (bound << 16 | index); only the groups
// whose keys changed are refreshed.
#pragma once

#include "fp_stages_md.h"

// a load served by L2, for words other lanes changed with atomics (which
// complete in L2; the wave's L1 may still hold the line)
template <class T>
__device__ __forceinline__ T ld_l2(FP_GLOBAL T* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

struct AmdState {
  int m, G, DW;
  long long acap;
  gptr<int> ro;                       // m+1 row offsets
  gptr<int> arow, erow;               // rows A_i and E_i
  gptr<int> alen, elen, dbar, mark;   // m each
  gptr<int> w, wst, llen, loff, ord;  // m each (w, wst, llen, loff by element = pivot)
  gptr<unsigned> key;                 // m: bound << 16 | index, ~0 once eliminated
  gptr<unsigned> gmin;                // G group minima
  gptr<unsigned> dirty;               // DW words: groups to refresh
  gptr<int> arena;                    // element lists
};

__device__ __forceinline__ void amd_refresh_group(const AmdState& S, int g) {
  const int i = g * 64 + lane_id();
  const uint32_t k = i < S.m ? S.key[i] : 0xFFFFFFFFu;
  const uint32_t mn = wave_min_u32(k);
  if (lane_id() == 0) S.gmin[g] = mn;
}

// Append the live, not yet marked entries of list[0..len) to the arena at
// top + *nl (marks them with step k).
__device__ __forceinline__ void amd_gather(const AmdState& S, gptr<const int> list, int len, int k,
                                           long long top, int* nl) {
  for (int c = 0; c < len; c += 64) {
    const int j = c + lane_id();
    int v = -1;
    bool take = false;
    if (j < len) {
      v = list[j];
      take = S.key[v] != 0xFFFFFFFFu && S.mark[v] != k;
    }
    const uint64_t bal = ballot64(take);
    if (take) {
      S.mark[v] = k;
      S.arena[top + *nl + popc64(bal & lanemask_lt())] = v;
    }
    *nl += popc64(bal);
    wave_fence();
  }
}

// Local order of node t's m vertices V (ascending ids; M.lidx holds their
// ranks) at positions pos0 ..
__device__ void md_amd_node(const FpMesh& M, int t, gptr<const int> V, int m, int pos0) {
  const int lane = lane_id();
  // row capacities: the vertices' graph degrees
  int R = 0;
  for (int c = 0; c < m; c += 64) {
    const int i = c + lane;
    const int d = i < m ? M.grp[V[i] + 1] - M.grp[V[i]] : 0;
    R += wave_sum_i32(d);
  }
  AmdState S;
  S.m = m;
  S.G = (m + 63) / 64;
  S.DW = (S.G + 31) / 32;
  S.acap = (long long)R + 2ll * m + 64;
  const unsigned long long words = (unsigned long long)(m + 1) + 2ull * R + 10ull * m + m + S.G +
                                   S.DW + (unsigned long long)S.acap + 64;
  gptr<unsigned> base = pool_alloc(M, words);
  if (!base) return;  // pool_alloc raised the error
  {
    gptr<unsigned> q = base;
    auto take = [&](long long n) {
      gptr<unsigned> r = q;
      q = q + n;
      return r;
    };
    S.ro = take(m + 1).as<int>();
    S.arow = take(R).as<int>();
    S.erow = take(R).as<int>();
    S.alen = take(m).as<int>();
    S.elen = take(m).as<int>();
    S.dbar = take(m).as<int>();
    S.mark = take(m).as<int>();
    S.w = take(m).as<int>();
    S.wst = take(m).as<int>();
    S.llen = take(m).as<int>();
    S.loff = take(m).as<int>();
    S.ord = take(m).as<int>();
    S.key = take(m);
    S.gmin = take(S.G);
    S.dirty = take(S.DW);
    S.arena = take(S.acap).as<int>();
  }
  // row offsets, then A_i from the induced subgraph
  {
    int run = 0;
    for (int c = 0; c < m; c += 64) {
      const int i = c + lane;
      const int d = i < m ? M.grp[V[i] + 1] - M.grp[V[i]] : 0;
      const int inc = wave_incl_scan(d);
      if (i < m) S.ro[i] = run + inc - d;
      run += wave_bcast(inc, 63);
    }
    if (lane == 0) S.ro[m] = run;
  }
  wave_fence();
  for (int i = lane; i < m; i += 64) {
    const int v = V[i], r0 = S.ro[i];
    int na = 0;
    for (int e = M.grp[v]; e < M.grp[v + 1]; e++) {
      const int u = M.gci[e];
      if (M.node_of[u] != t) continue;
      const int j = M.lidx[u];
      if (j != i) S.arow[r0 + na++] = j;
    }
    S.alen[i] = na;
    S.elen[i] = 0;
    S.dbar[i] = na;
    S.mark[i] = -1;
    S.wst[i] = -1;
    S.llen[i] = -2;  // not an element
    S.key[i] = ((uint32_t)na << 16) | (uint32_t)i;
  }
  for (int g = lane; g < S.DW; g += 64) S.dirty[g] = 0u;
  wave_fence();
  for (int g = 0; g < S.G; g++) amd_refresh_group(S, g);
  wave_fence();

  long long top = 0;
  for (int k = 0; k < m; k++) {
    // pivot: least key
    uint32_t mn = 0xFFFFFFFFu;
    for (int c = 0; c < S.G; c += 64) {
      const int g = c + lane;
      if (g < S.G) mn = min(mn, (uint32_t)S.gmin[g]);
    }
    mn = wave_min_u32(mn);
    const int p = (int)(mn & 0xFFFFu);
    if (mn == 0xFFFFFFFFu || p >= m) {  // never expected: the call reports it
      if (lane == 0) fp_fail(M.ctl, FP_E_INTERNAL, FP_SITE_MD_PIVOT, t);
      return;
    }
    if (lane == 0) {
      const int v = V[p];
      M.vperm[pos0 + k] = v;
      M.viperm[v] = pos0 + k;
      S.ord[k] = p;
      S.key[p] = 0xFFFFFFFFu;
      atomicOr(&S.dirty[(p >> 6) >> 5], 1u << ((p >> 6) & 31));
    }
    wave_fence();
    // room for L_p (at most m entries): compact the live lists in creation
    // order when the arena's tail is short
    if (top + m > S.acap) {
      long long nt = 0;
      for (int kk = 0; kk < k; kk++) {
        const int e = uni(S.ord[kk]);
        const int len = uni(S.llen[e]);
        if (len < 0) continue;
        const long long from = uni(S.loff[e]);
        for (int c = 0; c < len; c += 64) {
          const int j = c + lane;
          const int x = j < len ? S.arena[from + j] : 0;
          wave_fence();
          if (j < len) S.arena[nt + j] = x;
          wave_fence();
        }
        if (lane == 0) S.loff[e] = (int)nt;
        nt += len;
      }
      top = nt;
      wave_fence();
      if (top + m > S.acap) {  // never expected: the live lists fit by bound
        if (lane == 0) fp_fail(M.ctl, FP_E_SCRATCH, FP_SITE_MD_POOL, t);
        return;
      }
    }
    // L_p
    int nl = 0;
    const int rp0 = uni(S.ro[p]);
    amd_gather(S, S.arow + rp0, uni(S.alen[p]), k, top, &nl);
    const int ep = uni(S.elen[p]);
    for (int a = 0; a < ep; a++) {
      const int e = uni(S.erow[rp0 + a]);
      amd_gather(S, S.arena + uni(S.loff[e]), uni(S.llen[e]), k, top, &nl);
    }
    // absorb E_p; p becomes an element
    for (int a = lane; a < ep; a += 64) S.llen[S.erow[rp0 + a]] = -1;
    if (lane == 0) {
      S.loff[p] = (int)top;
      S.llen[p] = nl;
    }
    wave_fence();
    const gptr<int> Lp = S.arena + top;
    top += nl;
    // quotient-graph update of each i in L_p
    bool bad = false;
    for (int q = lane; q < nl; q += 64) {
      const int i = Lp[q];
      const int r0 = S.ro[i], cap = S.ro[i + 1] - r0;
      int na = 0;
      const int la = S.alen[i];
      for (int a = 0; a < la; a++) {
        const int v = S.arow[r0 + a];
        if (v != p && S.mark[v] != k) S.arow[r0 + na++] = v;
      }
      S.alen[i] = na;
      int ne = 0;
      const int le = S.elen[i];
      for (int a = 0; a < le; a++) {
        const int e = S.erow[r0 + a];
        if (S.llen[e] >= 0) S.erow[r0 + ne++] = e;
      }
      if (ne < cap)
        S.erow[r0 + ne++] = p;
      else
        bad = true;
      S.elen[i] = ne;
    }
    if (ballot64(bad)) {  // never expected: |E_i| is bounded by the degree
      if (lane == 0) fp_fail(M.ctl, FP_E_INTERNAL, FP_SITE_MD_PIVOT, t);
      return;
    }
    wave_fence();
    // |L_e \ L_p| for the other elements next to L_p: |L_e|, less one per
    // member of L_p
    for (int q = lane; q < nl; q += 64) {
      const int i = Lp[q], r0 = S.ro[i], le = S.elen[i];
      for (int a = 0; a < le; a++) {
        const int e = S.erow[r0 + a];
        if (e != p) S.w[e] = S.llen[e];
      }
    }
    wave_fence();
    for (int q = lane; q < nl; q += 64) {
      const int i = Lp[q], r0 = S.ro[i], le = S.elen[i];
      for (int a = 0; a < le; a++) {
        const int e = S.erow[r0 + a];
        if (e != p) atomicSub(&S.w[e], 1);
      }
    }
    wave_fence();
    // the bound
    const int r = m - (k + 1);
    for (int q = lane; q < nl; q += 64) {
      const int i = Lp[q], r0 = S.ro[i], le = S.elen[i];
      long long ext = 0;
      for (int a = 0; a < le; a++) {
        const int e = S.erow[r0 + a];
        if (e != p) ext += ld_l2(&S.w[e]);
      }
      const long long b1 = r - 1;
      const long long b2 = (long long)S.dbar[i] + (nl - 1);
      const long long b3 = (long long)S.alen[i] + (nl - 1) + ext;
      const int d = (int)min(b1, min(b2, b3));
      S.dbar[i] = d;
      S.key[i] = ((uint32_t)d << 16) | (uint32_t)i;
      atomicOr(&S.dirty[(i >> 6) >> 5], 1u << ((i >> 6) & 31));
    }
    wave_fence();
    // refresh the groups whose keys changed
    for (int c = 0; c < S.DW; c += 64) {
      const int wi = c + lane;
      const uint32_t x = wi < S.DW ? ld_l2(&S.dirty[wi]) : 0u;
      uint64_t bal = ballot64(x != 0u);
      while (bal) {
        const int l = __builtin_ctzll(bal);
        bal &= bal - 1;
        uint32_t word = (uint32_t)wave_bcast((int)x, l);
        if (lane == 0) S.dirty[c + l] = 0u;
        while (word) {
          const int b = __builtin_ctz(word);
          word &= word - 1;
          amd_refresh_group(S, (c + l) * 32 + b);
        }
      }
    }
    wave_fence();
  }
}
