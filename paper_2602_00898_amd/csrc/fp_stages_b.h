// fp_stages_b.h -- workgroup bisection of a separator-tree node on the
// quotient graph, and schedule positions of tree nodes.
#pragma once

#include "fp_stages_a.h"

// --------------------------------------------------------------------------
// Workgroup BFS on the quotient subgraph of tree node t (alive arcs whose
// both ends lie in t).  Local index i <-> patch pid[i]; ploc maps back.
// lev[] must be -1 on the component of src.  The visit order goes to
// queue[]; ls[L] = first queue slot of level L, ls[ecc+1] = count.
// Returns the number of nodes reached; *ecc_out = eccentricity of src.
// --------------------------------------------------------------------------
struct BisectLds {
  int tmp[FP_WAVES + 2];
  int tail;
  int r0;
  int lvcnt[3];  // claims of the next level, rotating over three levels
  int sink[64];  // per lane: the target of compare-swaps that must fail (0)
  unsigned long long red[FP_WAVES];
};

__device__ __forceinline__ int wg_bfs(const FpMesh& M, int t, gptr<const int> pid, int src, gptr<int> lev,
                                      gptr<int> queue, gptr<int> ls, int* ecc_out, BisectLds* sh) {
  if (threadIdx.x == 0) {
    lev[src] = 0;
    queue[0] = src;
    ls[0] = 0;
    sh->tail = 1;
  }
  __syncthreads();
  int head = 0, tail = 1, L = 0;
  while (true) {
    for (int i = head + (int)threadIdx.x; i < tail; i += FP_WG) {
      const int x = queue[i];
      const int p = pid[x];
      for (int a = M.qptr[p]; a < M.qptr[p + 1]; a++) {
        if (M.qcnt[a] <= 0) continue;
        const int q = M.qci[a];
        if (M.pnode[q] != t) continue;
        const int y = M.ploc[q];
        if (atomicCAS(&lev[y], -1, L + 1) == -1) queue[atomicAdd(&sh->tail, 1)] = y;
      }
    }
    __syncthreads();
    const int nt = sh->tail;
    __syncthreads();
    if (nt == tail) break;
    L++;
    if (threadIdx.x == 0) ls[L] = tail;
    head = tail;
    tail = nt;
  }
  if (threadIdx.x == 0) ls[L + 1] = tail;
  __syncthreads();
  *ecc_out = L;
  return tail;
}

// The same BFS on the node's quotient subgraph held as a local CSR (lrow,
// lcol: local indices) with its levels and queue in LDS.  A level is latency
// bound: a lane reads its vertex's first FP_BIS_ROW neighbours and their
// levels at once, and each wave reserves its claims' queue slots with one
// LDS atomic on the level's own counter.  The counters rotate over three
// levels, so that one barrier per level suffices: the one for level L+2 is
// cleared while level L runs, after every thread has read it.  The loads
// and compare-swaps are branch free (a lane with nothing to claim swaps on
// its sink word, which never holds -1), so that they are all in flight
// together.  The order inside a level depends on timing; the levels and
// their sets do not.
#define FP_BIS_ROW 8
__device__ __forceinline__ int wg_bfs_lds(const int* lrow, const int* lcol, int src, int* lev,
                                          int* queue, gptr<int> ls, int* ecc_out, BisectLds* sh) {
  if (threadIdx.x == 0) {
    lev[src] = 0;
    queue[0] = src;
    ls[0] = 0;
    sh->lvcnt[1] = 0;
  }
  if (threadIdx.x < 64) sh->sink[threadIdx.x] = 0;
  __syncthreads();
  int head = 0, tail = 1, L = 0;
  while (true) {
    if (threadIdx.x == 0) sh->lvcnt[(L + 2) % 3] = 0;
    int* ctr = &sh->lvcnt[(L + 1) % 3];
    for (int i = head + (int)threadIdx.x; i - (int)threadIdx.x < tail; i += FP_WG) {
      int y[FP_BIS_ROW];
      unsigned claims = 0;
      int a0 = 0, a1 = 0;
      {
        // a lane past the level reads vertex 0's row and claims nothing
        const int x = i < tail ? queue[i] : 0;
        a0 = lrow[x];
        a1 = i < tail ? lrow[x + 1] : a0;
        // lcol[a0 + j] past the row stays inside the LDS arrays (the
        // level arrays follow lcol)
#pragma unroll
        for (int j = 0; j < FP_BIS_ROW; j++) y[j] = lcol[a0 + j];
#pragma unroll
        for (int j = 0; j < FP_BIS_ROW; j++) y[j] = a0 + j < a1 ? y[j] : -1;
        int ly[FP_BIS_ROW];
#pragma unroll
        for (int j = 0; j < FP_BIS_ROW; j++) ly[j] = lev[y[j] >= 0 ? y[j] : 0];
        int r[FP_BIS_ROW];
#pragma unroll
        for (int j = 0; j < FP_BIS_ROW; j++)
          r[j] = atomicCAS(y[j] >= 0 && ly[j] == -1 ? &lev[y[j]] : &sh->sink[lane_id()], -1, L + 1);
#pragma unroll
        for (int j = 0; j < FP_BIS_ROW; j++) claims |= (unsigned)(r[j] == -1) << j;
      }
      const int c = __popc(claims);
      const int inc = wave_incl_scan(c);
      const int tot = wave_bcast(inc, 63);
      int base = 0;
      if (tot) {
        if (lane_id() == 63) base = atomicAdd(ctr, tot);
        base = wave_bcast(base, 63);
      }
      int o = tail + base + inc - c;
#pragma unroll
      for (int j = 0; j < FP_BIS_ROW; j++)
        if (claims & (1u << j)) queue[o++] = y[j];
      // rows longer than FP_BIS_ROW (rare on a patch quotient graph)
      for (int a = a0 + FP_BIS_ROW; a < a1; a++) {
        const int z = lcol[a];
        if (lev[z] == -1 && atomicCAS(&lev[z], -1, L + 1) == -1) queue[tail + atomicAdd(ctr, 1)] = z;
      }
    }
    __syncthreads();
    const int nc = sh->lvcnt[(L + 1) % 3];
    if (nc == 0) break;
    L++;
    if (threadIdx.x == 0) ls[L] = tail;
    head = tail;
    tail += nc;
  }
  if (threadIdx.x == 0) ls[L + 1] = tail;
  __syncthreads();
  *ecc_out = L;
  return tail;
}

__device__ __forceinline__ unsigned long long wg_min_u64(unsigned long long x, BisectLds* sh) {
  x = wave_min_u64(x);
  if (lane_id() == 0) sh->red[wave_id()] = x;
  __syncthreads();
  unsigned long long m = sh->red[0];
  for (int w = 1; w < FP_WAVES; w++) m = sh->red[w] < m ? sh->red[w] : m;
  __syncthreads();
  return m;
}

// Bisection of tree node t (Alg. 2 BiPartition; METIS is replaced by a BFS
// level structure from a pseudo-peripheral start, George & Liu 1979).  The
// node's patches are plist[s..s+m), ascending ids.  Writes the two child
// segments back into plist (left ascending, then right ascending) and moves
// each patch to its child in pnode.
//
// When the node's local CSR, two level arrays and two queues fit in the
// workgroup's dynamic LDS (lds, lds_bytes), the BFS sweeps run there.
template <bool kLds, class PT>
__device__ __forceinline__ void wg_bisect_body(const FpMesh& M, int t, int s, int m, BisectLds* sh,
                                               PT levA, PT levB, PT qA, PT qB, const int* lrow,
                                               const int* lcol) {
  gptr<int> pid = M.bs[0] + s;
  gptr<int> deg = M.bs[1] + s;
  // level starts need up to m+1 entries: node t's region is shifted by its
  // rank inside its depth, so regions of one depth stay disjoint
  const int rank_in_depth = t - ((1 << (31 - __clz(t + 1))) - 1);
  gptr<int> lsA = M.bs[6] + s + rank_in_depth;
  gptr<int> lsB = M.bs[7] + s + rank_in_depth;
  gptr<int> Q = M.bs[8] + s;
  gptr<int> flag = M.bs[9] + s;
  int base = 0, r0 = 0;
  while (base < m) {
    // the next component starts at its lowest unseen local index
    unsigned long long cand = 0xFFFFFFFFFFFFFFFFull;
    for (int i = r0 + (int)threadIdx.x; i < m; i += FP_WG)
      if (!flag[i]) {
        cand = (unsigned long long)i;
        break;
      }
    r0 = (int)wg_min_u64(cand, sh);
    int eccA, eccB;
    int cnt = kLds ? wg_bfs_lds(lrow, lcol, r0, (int*)levA, (int*)qA, lsA, &eccA, sh)
                   : wg_bfs(M, t, pid, r0, (gptr<int>)levA, (gptr<int>)qA, lsA, &eccA, sh);
    for (int round = 0; round < 8; round++) {
      // least (degree, index) on the last level
      unsigned long long best = 0xFFFFFFFFFFFFFFFFull;
      for (int i = lsA[eccA] + (int)threadIdx.x; i < cnt; i += FP_WG) {
        int x = qA[i];
        unsigned long long k = ((unsigned long long)deg[x] << 32) | (unsigned)x;
        best = k < best ? k : best;
      }
      const int c = (int)(wg_min_u64(best, sh) & 0xFFFFFFFFu);
      if (kLds)
        wg_bfs_lds(lrow, lcol, c, (int*)levB, (int*)qB, lsB, &eccB, sh);
      else
        wg_bfs(M, t, pid, c, (gptr<int>)levB, (gptr<int>)qB, lsB, &eccB, sh);
      const bool accept = eccB > eccA;
      PT clr_lev = accept ? levA : levB;
      PT clr_q = accept ? qA : qB;
      for (int i = threadIdx.x; i < cnt; i += FP_WG) clr_lev[clr_q[i]] = -1;
      __syncthreads();
      if (!accept) break;
      PT tp;
      tp = levA; levA = levB; levB = tp;
      tp = qA; qA = qB; qB = tp;
      gptr<int> tl = lsA; lsA = lsB; lsB = tl;
      eccA = eccB;
    }
    // order by (level, index): rank inside the level by counting smaller
    // ids, eight queue entries read together per step
    for (int i = threadIdx.x; i < cnt; i += FP_WG) {
      const int x = qA[i];
      const int L = levA[x];
      const int a = lsA[L], b = lsA[L + 1];
      int r = 0, j = a;
      for (; j + 8 <= b; j += 8) {
        int q[8];
#pragma unroll
        for (int u = 0; u < 8; u++) q[u] = qA[j + u];
#pragma unroll
        for (int u = 0; u < 8; u++) r += (q[u] < x);
      }
      for (; j < b; j++) r += (qA[j] < x);
      Q[base + a + r] = x;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < cnt; i += FP_WG) {
      const int x = qA[i];
      flag[x] = 1;
      levA[x] = -1;
    }
    __syncthreads();
    base += cnt;
  }
  // weighted split: k* = least k with 2 * (weight of Q[0..k)) >= W, then
  // clamp to the heap capacity of the children
  long long W = 0;
  for (int i = threadIdx.x; i < m; i += FP_WG) W += M.wp[pid[i]];
  W = wg_sum_i64(W, (int64_t*)sh->red);
  int kstar;
  if (W == 0) {
    kstar = (m + 1) / 2;
  } else {
    unsigned long long first = 0xFFFFFFFFFFFFFFFFull;
    long long run = 0;
    for (int c0 = 0; c0 < m; c0 += FP_WG) {
      const int i = c0 + (int)threadIdx.x;
      const int w = i < m ? M.wp[pid[Q[i]]] : 0;
      int tt;
      const int ex = wg_excl_scan(w, sh->tmp, &tt);
      if (i < m && 2 * (run + ex + w) >= W && (unsigned long long)i < first) first = i;
      run += tt;
    }
    first = wg_min_u64(first, sh);
    kstar = first == 0xFFFFFFFFFFFFFFFFull ? m : (int)first + 1;
  }
  int h = 0;
  while ((1 << h) < m) h++;
  const int cap = 1 << (h - 1);
  const int lo = max(1, m - cap), hi = min(m - 1, cap);
  const int k = min(max(kstar, lo), hi);
  for (int i = threadIdx.x; i < m; i += FP_WG) flag[Q[i]] = (i < k) ? 1 : 2;
  __syncthreads();
  // stable split in ascending id order
  int rl = 0, rr = 0;
  for (int c0 = 0; c0 < m; c0 += FP_WG) {
    const int i = c0 + (int)threadIdx.x;
    const int f = i < m ? flag[i] : 0;
    int tl, tr;
    const int el = wg_excl_scan(f == 1, sh->tmp, &tl);
    const int er = wg_excl_scan(f == 2, sh->tmp, &tr);
    if (f == 1) {
      M.plist[s + rl + el] = pid[i];
      M.pnode[pid[i]] = 2 * t + 1;
    } else if (f == 2) {
      M.plist[s + k + rr + er] = pid[i];
      M.pnode[pid[i]] = 2 * t + 2;
    }
    rl += tl;
    rr += tr;
  }
  if (threadIdx.x == 0) {
    if (rl != k || rr != m - k) fp_fail(M.ctl, FP_E_INTERNAL, FP_SITE_BISECT_SPLIT, t);
    M.segS[2 * t + 1] = s;
    M.segN[2 * t + 1] = k;
    M.segS[2 * t + 2] = s + k;
    M.segN[2 * t + 2] = m - k;
  }
  __syncthreads();
}

__device__ __forceinline__ void wg_bisect(const FpMesh& M, int t, int s, int m, BisectLds* sh,
                                          char* lds, long long lds_bytes) {
  gptr<int> pid = M.bs[0] + s;
  gptr<int> deg = M.bs[1] + s;
  gptr<int> levA = M.bs[2] + s;
  gptr<int> levB = M.bs[3] + s;
  gptr<int> qA = M.bs[4] + s;
  gptr<int> qB = M.bs[5] + s;
  gptr<int> flag = M.bs[9] + s;
  const int P = M.ctl->P;
  for (int i = threadIdx.x; i < m; i += FP_WG) {
    int p = M.plist[s + i];
    if (p < 0 || p >= P) {  // never expected: keep every later index in range
      fp_fail(M.ctl, FP_E_INTERNAL, FP_SITE_BISECT_PATCH, p);
      p = 0;
    }
    pid[i] = p;
    M.ploc[p] = i;
    levA[i] = -1;
    levB[i] = -1;
    flag[i] = 0;
  }
  __syncthreads();
  // degrees inside t: the first FP_BIS_ROW arcs' loads go out together
  for (int i = threadIdx.x; i < m; i += FP_WG) {
    const int p = pid[i];
    const int a0 = M.qptr[p], a1 = M.qptr[p + 1];
    int q[FP_BIS_ROW], c[FP_BIS_ROW];
#pragma unroll
    for (int j = 0; j < FP_BIS_ROW; j++) {
      q[j] = a0 + j < a1 ? (int)M.qci[a0 + j] : -1;
      c[j] = a0 + j < a1 ? (int)M.qcnt[a0 + j] : 0;
    }
    int d = 0;
#pragma unroll
    for (int j = 0; j < FP_BIS_ROW; j++) d += (c[j] > 0 && (q[j] >= 0 ? (int)M.pnode[q[j]] : -1) == t);
    for (int a = a0 + FP_BIS_ROW; a < a1; a++) d += (M.qcnt[a] > 0 && M.pnode[M.qci[a]] == t);
    deg[i] = d;
  }
  __syncthreads();
  // the node's quotient subgraph as a local CSR in LDS, with two level
  // arrays and two queues, when it fits
  if (4ll * (5ll * m + 1) <= lds_bytes) {
    int* lrow = (int*)lds;
    int run = 0;
    for (int c0 = 0; c0 < m; c0 += FP_WG) {
      const int i = c0 + (int)threadIdx.x;
      const int dd = i < m ? deg[i] : 0;
      int tot;
      const int ex = wg_excl_scan(dd, sh->tmp, &tot);
      if (i < m) lrow[i] = run + ex;
      run += tot;
    }
    if (threadIdx.x == 0) lrow[m] = run;
    __syncthreads();
    if (4ll * (5ll * m + 1 + run) <= lds_bytes) {
      int* lcol = lrow + (m + 1);
      int* lA = lcol + run;
      int* lB = lA + m;
      int* qa = lB + m;
      int* qb = qa + m;
      for (int i = threadIdx.x; i < m; i += FP_WG) {
        const int p = pid[i];
        int o = lrow[i];
        const int a0 = M.qptr[p], a1 = M.qptr[p + 1];
        int q[FP_BIS_ROW], c[FP_BIS_ROW], pn[FP_BIS_ROW], pl[FP_BIS_ROW];
#pragma unroll
        for (int j = 0; j < FP_BIS_ROW; j++) {
          q[j] = a0 + j < a1 ? (int)M.qci[a0 + j] : -1;
          c[j] = a0 + j < a1 ? (int)M.qcnt[a0 + j] : 0;
        }
#pragma unroll
        for (int j = 0; j < FP_BIS_ROW; j++) {
          pn[j] = q[j] >= 0 ? (int)M.pnode[q[j]] : -1;
          pl[j] = q[j] >= 0 ? (int)M.ploc[q[j]] : 0;
        }
#pragma unroll
        for (int j = 0; j < FP_BIS_ROW; j++)
          if (c[j] > 0 && pn[j] == t) lcol[o++] = pl[j];
        for (int a = a0 + FP_BIS_ROW; a < a1; a++) {
          const int qq = M.qci[a];
          if (M.qcnt[a] > 0 && M.pnode[qq] == t) lcol[o++] = M.ploc[qq];
        }
        lA[i] = -1;
        lB[i] = -1;
      }
      __syncthreads();
      wg_bisect_body<true, int*>(M, t, s, m, sh, lA, lB, qa, qb, lrow, lcol);
      return;
    }
  }
  wg_bisect_body<false, gptr<int>>(M, t, s, m, sh, levA, levB, qA, qB, nullptr, nullptr);
}

// --------------------------------------------------------------------------
// Schedule position of tree node t (Alg. 3, Sec. 5).  Level order: depth
// descending, heap index ascending.  Post order: left subtree, right
// subtree, node.
// --------------------------------------------------------------------------
__device__ __forceinline__ int sched_pos(int t, int D, int sched) {
  int d = 31 - __clz(t + 1);
  if (sched == 0) return ((1 << (D + 1)) - (1 << (d + 1))) + (t - ((1 << d) - 1));
  // post order: start of t's subtree block plus its size minus one
  int start = 0;
  const int path = t + 1;
  for (int i = d - 1; i >= 0; i--) {
    const int depth_child = d - i;  // depth of the node reached by this step
    if ((path >> i) & 1) start += (1 << (D - depth_child + 1)) - 1;  // skip left sibling subtree
  }
  return start + (1 << (D - d + 1)) - 2;
}

