// fp_stages_md.h -- local orders: exact minimum degree on the subgraph
// induced by each separator-tree node (Sec. 4.3 Step 4, LocalOrder; the
// textbook one-vertex-per-step scheme of Tinney and Walker, ties to the
// lowest local index = rank of the vertex id inside the node).
//
// One wave64 owns a node.  The elimination graph lives in LDS:
//   BIT    -- adjacency bitsets (m x ceil(m/32) words); neighbours of the
//             pivot are found word-wise and only the nonzero words of the
//             pivot row are OR-ed into each neighbour row,
//   SPARSE -- fixed-capacity rows of 16-bit local ids, for large nodes of
//             low degree (separators are path-like); when the remaining
//             vertices fit the BIT layout and a pivot has more than four
//             neighbours, or a row would overflow, the state is re-indexed
//             (rank order kept, so tie-breaking is unchanged) into BIT form,
//   BITG   -- BIT layout in a global-memory pool, for nodes too big for LDS.
// The pivot is the minimum of keys (degree << 16 | index) found through a
// 64-ary min tree: per-64 group minima are refreshed only for groups whose
// keys changed, then reduced across the wave.
#pragma once

#include "fp_stages_b.h"

#define FP_KEY_INF 0xFFFFFFFFu
#define FP_MD_MAXM 65535  // 16-bit local ids

// device-wide bump allocation from the fallback pool (32-bit words)
__device__ __forceinline__ gptr<unsigned> pool_alloc(const FpMesh& M, unsigned long long words) {
  unsigned long long off = 0;
  if (lane_id() == 0) {
    words = (words + 63) & ~63ull;
    off = atomicAdd(&M.ctl->pool_top, words);
    if (off + words > M.pool_words) {
      fp_fail(M.ctl, FP_E_SCRATCH, FP_SITE_MD_POOL, (int)(words >> 6));
      off = ~0ull;
    }
  }
  off = __shfl((unsigned long long)off, 0, 64);
  return off == ~0ull ? gptr<unsigned>(nullptr) : M.pool + off;
}

__device__ __forceinline__ int md_words(int m) { return (m + 31) >> 5; }
__device__ __forceinline__ int md_groups(int m) { return (m + 63) >> 6; }

// LDS bytes of the BIT layout for m vertices
__device__ __forceinline__ long long md_bit_bytes(int m) {
  const long long W = md_words(m), G = md_groups(m);
  return 4ll * m * W + 12ll * W + 8ll * m + 12ll * G + 64;
}
__device__ __forceinline__ int md_bit_max(long long bytes) {
  int lo = 0, hi = FP_MD_MAXM;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (md_bit_bytes(mid) <= bytes)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

struct MdBit {
  uint32_t* rows;
  uint32_t* alive;
  uint32_t* nbm;
  int* nzw;
  int* nbl;
  uint32_t* key;
  uint32_t* gmin;
  int* dl;  // dirty groups: flags [0,G) then list [G,2G)
  int m, W, G;
};

__device__ __forceinline__ void md_bit_carve(MdBit& B, char* mem, int m) {
  B.m = m;
  B.W = md_words(m);
  B.G = md_groups(m);
  char* p = mem;
  B.rows = (uint32_t*)p;
  p += 4ll * m * B.W;
  B.alive = (uint32_t*)p;
  p += 4 * B.W;
  B.nbm = (uint32_t*)p;
  p += 4 * B.W;
  B.nzw = (int*)p;
  p += 4 * B.W;
  B.nbl = (int*)p;
  p += 4ll * m;
  B.key = (uint32_t*)p;
  p += 4ll * m;
  B.gmin = (uint32_t*)p;
  p += 4 * B.G;
  B.dl = (int*)p;
}

__device__ __forceinline__ void md_refresh_all_groups(MdBit& B) {
  for (int g = 0; g < B.G; g++) {
    const int i = g * 64 + lane_id();
    uint32_t k = i < B.m ? B.key[i] : FP_KEY_INF;
    k = wave_min_u32(k);
    if (lane_id() == 0) B.gmin[g] = k;
    if (lane_id() == 0) B.dl[g] = 0;
  }
  wave_fence();
}

__device__ __forceinline__ uint32_t md_argmin(const uint32_t* gmin, int G) {
  uint32_t km = FP_KEY_INF;
  for (int g = lane_id(); g < G; g += 64) km = min(km, gmin[g]);
  return wave_min_u32(km);
}

// refresh the minima of the groups flagged in dl[0..G) and clear the flags
__device__ __forceinline__ void md_refresh_dirty(uint32_t* key, uint32_t* gmin, int* dl, int m,
                                                 int G) {
  int nd = 0;
  for (int g0 = 0; g0 < G; g0 += 64) {
    const int g = g0 + lane_id();
    const bool d = g < G && dl[g];
    const uint64_t bal = ballot64(d);
    if (d) {
      dl[G + nd + popc64(bal & lanemask_lt())] = g;
      dl[g] = 0;
    }
    nd += popc64(bal);
  }
  wave_fence();
  for (int j = 0; j < nd; j++) {
    const int g = uni(dl[G + j]);
    const int i = g * 64 + lane_id();
    uint32_t k = i < m ? key[i] : FP_KEY_INF;
    k = wave_min_u32(k);
    if (lane_id() == 0) gmin[g] = k;
  }
  wave_fence();
}

// The pivot steps store the pivot's local index into vperm (a store that
// waits for nothing); md_map_order then turns the positions
// [pos0, pos0 + count) into vertex ids through vmap (local index -> vertex,
// mlim entries) and fills viperm, all lanes at once.
__device__ __forceinline__ void md_map_order(const FpMesh& M, gptr<const int> vmap, int mlim, int pos0,
                                             int count) {
  wave_fence();
  for (int s = lane_id(); s < count; s += 64) {
    const int p = M.vperm[pos0 + s];
    const int v = (unsigned)p < (unsigned)mlim ? vmap[p] : -1;
    M.vperm[pos0 + s] = v;
    if ((unsigned)v < (unsigned)M.n) M.viperm[v] = pos0 + s;
  }
  wave_fence();
}

// Run minimum degree steps on a BIT layout until every vertex is ordered.
// vmap[i] = vertex id of current index i; outputs go to positions
// pos0, pos0+1, ...
//
// Rows of at most 64 words (m <= 2048, so at most 32 groups): the group
// minima and the live set live in registers (lane g holds group g's
// minimum, lane w word w of the live set), lane w holds word w of the
// pivot's live row, the neighbours are listed from the lanes' bits with one
// prefix sum, and the clique update takes one lane per (neighbour, nonzero
// word) pair, each adding the bits it set to the neighbour's key with one
// LDS atomic.  The groups to refresh are those of the pivot's nonzero words
// (a group is two words) and the pivot's own; each 16-lane row of the wave
// refreshes one of them.
__device__ __forceinline__ void md_bit_run64(const FpMesh& M, MdBit& B, gptr<const int> vmap,
                                             int pos0, int nsteps) {
  const int lane = lane_id();
  const int W = B.W, G = B.G;
  uint32_t gm = lane < G ? B.gmin[lane] : FP_KEY_INF;
  uint32_t aw = lane < W ? B.alive[lane] : 0u;  // lane w holds word w of the live set
  const int row = lane >> 4, q = lane & 15;
  for (int s = 0; s < nsteps; s++) {
    const uint32_t km = wave_min_u32(gm);
    const int p = (int)(km & 0xFFFFu);
    if (km == FP_KEY_INF || p >= B.m) {  // never expected: stop before any wild index
      if (lane == 0) fp_fail(M.ctl, FP_E_INTERNAL, FP_SITE_MD_PIVOT, pos0);
      md_map_order(M, vmap, B.m, pos0, s);
      return;
    }
    if (lane == 0) {
      M.vperm[pos0 + s] = p;
      B.key[p] = FP_KEY_INF;
    }
    if (lane == (p >> 5)) aw &= ~(1u << (p & 31));
    wave_fence();
    const uint32_t* rp = B.rows + (long long)p * W;
    const uint32_t x = lane < W ? (rp[lane] & aw) : 0u;
    const uint64_t nzm = ballot64(x != 0u);
    const int nnzw = popc64(nzm);
    const int c = popc32(x);
    const int inc = wave_incl_scan(c);
    const int k = wave_bcast(inc, 63);
    {
      int off = inc - c;
      uint32_t y = x;
      while (y) {
        const int bit = __ffs(y) - 1;
        y &= y - 1;
        B.nbl[off] = lane * 32 + bit;
        off++;
      }
    }
    if (x) {
      B.nzw[popc64(nzm & lanemask_lt())] = lane;
      B.nbm[lane] = x;
    }
    wave_fence();
    // the neighbours become a clique: OR the pivot's live row into theirs
    // pairs (i, j) at qq = i * 2^sh + j, the words padded to a power of two
    // so no lane divides
    const int sh = nnzw <= 1 ? 0 : 32 - __builtin_clz(nnzw - 1);
    const int npair = k << sh;
    for (int q0 = 0; q0 < npair; q0 += 64) {
      const int qq = q0 + lane;
      const int i = qq >> sh, j = qq & ((1 << sh) - 1);
      if (qq < npair && j < nnzw) {
        const int u = B.nbl[i], w = B.nzw[j];
        uint32_t* ru = B.rows + (long long)u * W;
        const uint32_t old = ru[w];
        uint32_t nv = old | B.nbm[w];
        if (w == (u >> 5)) nv &= ~(1u << (u & 31));
        ru[w] = nv;
        // u's degree gains the bits its row gained and loses p (counted
        // once, on the pair of u's first word): one atomic on the key's
        // degree field, exact in wrapping 32-bit arithmetic
        const int d = popc32(nv & ~old) - (j == 0);
        if (d) atomicAdd(&B.key[u], (uint32_t)d << 16);
      }
    }
    wave_fence();
    // groups to refresh: the pivot's, and those of its nonzero words
    uint64_t dg = 1ull << (p >> 6);
    for (uint64_t b = nzm; b; b &= b - 1) dg |= 1ull << (__builtin_ctzll(b) >> 1);
    while (dg) {
      int gs[4];
#pragma unroll
      for (int r = 0; r < 4; r++) {
        gs[r] = dg ? __builtin_ctzll(dg) : -1;
        if (dg) dg &= dg - 1;
      }
      const int g = row == 0 ? gs[0] : row == 1 ? gs[1] : row == 2 ? gs[2] : gs[3];
      uint32_t kk = FP_KEY_INF;
      {
        // four keys per lane, all loads issued before the first use (the
        // index clamped into the array, the values past m masked)
        const int b = (g >= 0 ? g : 0) * 64 + q * 4;
        uint32_t kv[4];
#pragma unroll
        for (int a = 0; a < 4; a++) kv[a] = B.key[min(b + a, B.m - 1)];
#pragma unroll
        for (int a = 0; a < 4; a++)
          if (g >= 0 && b + a < B.m) kk = min(kk, kv[a]);
      }
      const int I = -1;  // identity of the unsigned minimum
      kk = min(kk, (uint32_t)dpp_shr((int)kk, I, 1));
      kk = min(kk, (uint32_t)dpp_shr((int)kk, I, 2));
      kk = min(kk, (uint32_t)dpp_shr((int)kk, I, 4));
      kk = min(kk, (uint32_t)dpp_shr((int)kk, I, 8));
#pragma unroll
      for (int r = 0; r < 4; r++) {  // lane 15 of row r holds group gs[r]'s minimum
        const uint32_t v = (uint32_t)wave_bcast((int)kk, 16 * r + 15);
        if (gs[r] >= 0 && lane == gs[r]) gm = v;
      }
    }
  }
  if (lane < W) B.alive[lane] = aw;
  md_map_order(M, vmap, B.m, pos0, nsteps);
}

__device__ __forceinline__ void md_bit_run(const FpMesh& M, MdBit& B, gptr<const int> vmap, int pos0,
                                           int nsteps) {
  if (B.W <= 64) {
    md_bit_run64(M, B, vmap, pos0, nsteps);
    return;
  }
  const int lane = lane_id();
  const int W = B.W;
  for (int s = 0; s < nsteps; s++) {
    const uint32_t km = md_argmin(B.gmin, B.G);
    const int p = (int)(km & 0xFFFFu);
    if (km == FP_KEY_INF || p >= B.m) {  // never expected: stop before any wild index
      if (lane == 0) fp_fail(M.ctl, FP_E_INTERNAL, FP_SITE_MD_PIVOT, pos0);
      md_map_order(M, vmap, B.m, pos0, s);
      return;
    }
    if (lane == 0) {
      M.vperm[pos0 + s] = p;
      B.alive[p >> 5] &= ~(1u << (p & 31));
      B.key[p] = FP_KEY_INF;
      B.dl[p >> 6] = 1;
    }
    wave_fence();
    // neighbours of p among the remaining vertices, word by word
    int nnzw = 0;
    const uint32_t* rp = B.rows + (long long)p * W;
    for (int w0 = 0; w0 < W; w0 += 64) {
      const int w = w0 + lane;
      const uint32_t x = (w < W) ? (rp[w] & B.alive[w]) : 0u;
      if (w < W) B.nbm[w] = x;
      const uint64_t bal = ballot64(x != 0);
      if (x) B.nzw[nnzw + popc64(bal & lanemask_lt())] = w;
      nnzw += popc64(bal);
    }
    wave_fence();
    int k = 0;
    for (int j0 = 0; j0 < nnzw; j0 += 64) {
      const int j = j0 + lane;
      uint32_t x = j < nnzw ? B.nbm[B.nzw[j]] : 0u;
      const int w = j < nnzw ? B.nzw[j] : 0;
      const int c = popc32(x);
      const int inc = wave_incl_scan(c);
      int off = k + inc - c;
      while (x) {
        const int bit = __ffs(x) - 1;
        x &= x - 1;
        B.nbl[off++] = w * 32 + bit;
      }
      k += wave_bcast(inc, 63);
    }
    wave_fence();
    // the neighbours become a clique: OR the pivot row into theirs
    for (int i = lane; i < k; i += 64) {
      const int u = B.nbl[i];
      uint32_t* ru = B.rows + (long long)u * W;
      const int uw = u >> 5;
      const uint32_t ubit = 1u << (u & 31);
      int added = 0;
      for (int j = 0; j < nnzw; j++) {
        const int w = B.nzw[j];
        const uint32_t old = ru[w];
        uint32_t nv = old | B.nbm[w];
        if (w == uw) nv &= ~ubit;
        added += popc32(nv & ~old);
        ru[w] = nv;
      }
      const uint32_t deg = (B.key[u] >> 16) + added - 1;
      B.key[u] = (deg << 16) | (uint32_t)u;
      B.dl[u >> 6] = 1;
    }
    wave_fence();
    md_refresh_dirty(B.key, B.gmin, B.dl, B.m, B.G);
  }
  md_map_order(M, vmap, B.m, pos0, nsteps);
}

// ---------------------------------------------------------------- SPARSE
// The pivot of the sparse layout is found through degree buckets: bucket d
// is a bitmap of the remaining vertices of degree d (degrees stay <= C here),
// cnt[d] its population; the pivot is the lowest vertex of the lowest
// non-empty bucket, the (degree, index) minimum, found with two ballots.
struct MdSp {
  uint16_t* rows;   // m*C
  uint16_t* len;    // m: degree = row length
  uint32_t* alive;  // MW: remaining vertices (set up front and at conversion)
  uint32_t* bk;     // (C+1) x MW: vertices by degree
  int* cnt;         // C+1
  int* nbl;         // 64: the pivot's neighbours
  int m, C, MW;
};

__device__ __forceinline__ long long md_sp_bytes(int m, int C) {
  const long long MW = (m + 31) / 32;
  return 2ll * m * C + 2ll * m + 4 * MW + 4 * (C + 1) * MW + 4ll * (C + 1) + 4 * 64 + 64;
}

__device__ __forceinline__ void md_sp_carve(MdSp& S, char* mem, int m, int C) {
  S.m = m;
  S.C = C;
  S.MW = (m + 31) >> 5;
  char* p = mem;
  S.bk = (uint32_t*)p;
  p += 4ll * (C + 1) * S.MW;
  S.alive = (uint32_t*)p;
  p += 4ll * S.MW;
  S.cnt = (int*)p;
  p += 4ll * (C + 1);
  S.nbl = (int*)p;
  p += 4 * 64;
  S.len = (uint16_t*)p;
  p += 2ll * m;
  p = mem + ((p - mem + 15) & ~15ll);  // mem is 16-byte aligned; keeps the LDS address space
  S.rows = (uint16_t*)p;
}

// ---------------------------------------------------------------- driver
// sort the node's vertex ids (LDS bitonic sort over the next power of two)
template <class P>  // an LDS or a global int array
__device__ __forceinline__ void wave_sort_ids(P a, int m, int np2) {
  for (int i = m + lane_id(); i < np2; i += 64) a[i] = 0x7FFFFFFF;
  wave_fence();
  for (int k = 2; k <= np2; k <<= 1)
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = lane_id(); i < np2; i += 64) {
        const int ixj = i ^ j;
        if (ixj > i) {
          const int x = a[i], y = a[ixj];
          const bool up = (i & k) == 0;
          if ((x > y) == up) {
            a[i] = y;
            a[ixj] = x;
          }
        }
      }
      wave_fence();
    }
}

// Build BIT rows for the vertices vmap[0..m) of node t straight from G.
__device__ __forceinline__ void md_bit_build(const FpMesh& M, MdBit& B, int t, gptr<const int> vmap) {
  const int m = B.m, W = B.W;
  for (long long i = lane_id(); i < (long long)m * W; i += 64) B.rows[i] = 0u;
  for (int w = lane_id(); w < W; w += 64) {
    const int hi = min(32, m - w * 32);
    B.alive[w] = hi >= 32 ? 0xFFFFFFFFu : ((1u << hi) - 1u);
  }
  for (int g = lane_id(); g < 2 * B.G; g += 64) B.dl[g] = 0;
  wave_fence();
  for (int i = lane_id(); i < m; i += 64) {
    const int v = vmap[i];
    uint32_t* ri = B.rows + (long long)i * W;
    for (int e = M.grp[v]; e < M.grp[v + 1]; e++) {
      const int u = M.gci[e];
      if (M.node_of[u] != t) continue;
      const int j = M.lidx[u];
      if (j != i) ri[j >> 5] |= 1u << (j & 31);
    }
    int d = 0;
    for (int w = 0; w < W; w++) d += popc32(ri[w]);
    B.key[i] = ((uint32_t)d << 16) | (uint32_t)i;
  }
  wave_fence();
  md_refresh_all_groups(B);
}

// One node, one wave.  slice/slice_bytes: this wave's LDS.
// Re-index the na remaining vertices of a sparse state (rows srows/slen,
// new index ni[i] or -1 if ordered) into a BIT layout carved from mem and
// finish the node there.
__device__ __forceinline__ void md_sp_to_bit(const FpMesh& M, char* mem, int na, int m, int C,
                                             gptr<const uint16_t> srows, gptr<const uint16_t> slen,
                                             gptr<const int> ni, gptr<const int> vm2, int pos) {
  MdBit B;
  md_bit_carve(B, mem, na);
  for (long long i = lane_id(); i < (long long)na * B.W; i += 64) B.rows[i] = 0u;
  for (int w = lane_id(); w < B.W; w += 64) {
    const int hi = min(32, na - w * 32);
    B.alive[w] = hi >= 32 ? 0xFFFFFFFFu : ((1u << hi) - 1u);
  }
  for (int g = lane_id(); g < 2 * B.G; g += 64) B.dl[g] = 0;
  wave_fence();
  for (int i = lane_id(); i < m; i += 64) {
    const int r = ni[i];
    if (r < 0) continue;
    uint32_t* rr = B.rows + (long long)r * B.W;
    const int l = slen[i];
    for (int q = 0; q < l; q++) {
      const int x = ni[srows[(long long)i * C + q]];
      if (x >= 0) rr[x >> 5] |= 1u << (x & 31);
    }
    B.key[r] = ((uint32_t)l << 16) | (uint32_t)r;
  }
  wave_fence();
  md_refresh_all_groups(B);
  md_bit_run(M, B, vm2, pos, na);
}

// Local order of node t: its m vertices listed at V (sorted there in place)
// take positions pos0 .. pos0+m-1.
// approximate-minimum-degree local order (fp_stages_amd.h)
__device__ void md_amd_node(const FpMesh& M, int t, gptr<const int> V, int m, int pos0);

__device__ __forceinline__ void md_node_list(const FpMesh& M, int t, gptr<int> V, int m, int pos0,
                                             char* slice, long long slice_bytes) {
  if (m == 0) return;
  // the node's vertex list must hold vertices of this node only
  {
    bool bad = pos0 < 0 || m < 0 || (long long)pos0 + m > M.n;
    for (int i = lane_id(); i < m && !bad; i += 64) {
      const int v = V[i];
      bad = (unsigned)v >= (unsigned)M.n || M.node_of[v] != t;
    }
    if (ballot64(bad)) {
      if (lane_id() == 0) fp_fail(M.ctl, FP_E_INTERNAL, FP_SITE_MD_VERTEX, t);
      return;
    }
  }
  if (m > FP_MD_MAXM) {
    // beyond 16-bit local ids: keep id order (flagged as unsupported)
    if (lane_id() == 0) fp_fail(M.ctl, FP_E_SCRATCH, FP_SITE_MD_MAXM, t);
    for (int i = lane_id(); i < m; i += 64) {
      M.vperm[pos0 + i] = V[i];
      M.viperm[V[i]] = pos0 + i;
    }
    return;
  }
  // 1. sort ids (LDS when it fits, else in a pool buffer)
  int np2 = 1;
  while (np2 < m) np2 <<= 1;
  if (4ll * np2 <= slice_bytes) {
    int* a = (int*)slice;
    for (int i = lane_id(); i < m; i += 64) a[i] = V[i];
    wave_fence();
    wave_sort_ids(a, m, np2);
    for (int i = lane_id(); i < m; i += 64) V[i] = a[i];
  } else {
    gptr<int> a = pool_alloc(M, np2).as<int>();
    if (!a) return;
    for (int i = lane_id(); i < m; i += 64) a[i] = V[i];
    wave_fence();
    wave_sort_ids(a, m, np2);
    for (int i = lane_id(); i < m; i += 64) V[i] = a[i];
  }
  wave_fence();
  for (int i = lane_id(); i < m; i += 64) M.lidx[V[i]] = i;
  wave_fence();
  if (M.amd) {  // approximate minimum degree (the quotient graph in the pool)
    md_amd_node(M, t, V, m, pos0);
    return;
  }

  const int mbit = md_bit_max(slice_bytes);
  if (m <= mbit) {
    MdBit B;
    md_bit_carve(B, slice, m);
    md_bit_build(M, B, t, V);
    md_bit_run(M, B, V, pos0, m);
    return;
  }
  // SPARSE when the rows fit with a useful capacity
  int C = 0;
  {
    const long long MW = (m + 31) / 32;
    const long long fixed = md_sp_bytes(m, 0) + 16;
    C = (int)min(63ll, (slice_bytes - fixed) / (2ll * m + 4 * MW + 4));
  }
  bool sparse_ok = C >= 6;
  MdSp S;
  if (sparse_ok) {
    md_sp_carve(S, slice, m, C);
    int over = 0;
    for (long long i = lane_id(); i < (long long)(C + 1) * S.MW; i += 64) S.bk[i] = 0u;
    for (int i = lane_id(); i <= C; i += 64) S.cnt[i] = 0;
    for (int w = lane_id(); w < S.MW; w += 64) {
      const int hi = min(32, m - w * 32);
      S.alive[w] = hi >= 32 ? 0xFFFFFFFFu : ((1u << hi) - 1u);
    }
    wave_fence();
    for (int i = lane_id(); i < m; i += 64) {
      const int v = V[i];
      uint16_t* ri = S.rows + (long long)i * C;
      int len = 0;
      for (int e = M.grp[v]; e < M.grp[v + 1]; e++) {
        const int u = M.gci[e];
        if (M.node_of[u] != t) continue;
        const int j = M.lidx[u];
        if (j == i) continue;
        bool dup = false;
        for (int q = 0; q < len && q < C; q++) dup |= (ri[q] == j);
        if (dup) continue;
        if (len < C) ri[len] = (uint16_t)j;
        len++;
      }
      if (len > C) over = 1;
      const int d = min(len, C);
      S.len[i] = (uint16_t)d;
      atomicOr(&S.bk[(long long)d * S.MW + (i >> 5)], 1u << (i & 31));
      atomicAdd(&S.cnt[d], 1);
    }
    wave_fence();
    sparse_ok = !ballot64(over);
  }
  int done = 0;           // vertices already ordered
  int na = m;             // vertices remaining
  gptr<const int> vmap = V;
  if (sparse_ok) {
    // bucket sizes live in registers from here on: lane d counts degree d
    int creg = lane_id() <= C ? S.cnt[lane_id()] : 0;
    const int lane = lane_id();
    while (na > 0) {
      // pivot: lowest vertex of the lowest non-empty degree bucket
      const uint64_t nz = ballot64(creg > 0);
      const int d = uni(nz ? (int)__builtin_ctzll(nz) : -1);
      int p = -1;
      if (d >= 0) {
        // 128 words per round, both halves read at once
        const uint32_t* row = S.bk + (long long)d * S.MW;
        for (int w0 = 0; w0 < S.MW; w0 += 128) {
          const int wa = w0 + lane, wb = w0 + 64 + lane;
          const uint32_t xa = wa < S.MW ? row[wa] : 0u;
          const uint32_t xb = wb < S.MW ? row[wb] : 0u;
          const uint64_t ba = ballot64(xa != 0u);
          if (ba) {
            const int l = __builtin_ctzll(ba);
            p = (w0 + l) * 32 + __ffs(wave_bcast_u32(xa, l)) - 1;
            break;
          }
          const uint64_t bb = ballot64(xb != 0u);
          if (bb) {
            const int l = __builtin_ctzll(bb);
            p = (w0 + 64 + l) * 32 + __ffs(wave_bcast_u32(xb, l)) - 1;
            break;
          }
        }
      }
      p = uni(p);
      // p's row and length are read together, before the check (the
      // address clamped to row 0 until p is known to be in range)
      const int pc = p >= 0 && p < m ? p : 0;
      const uint16_t* rpv = S.rows + (long long)pc * C;
      const int rpl0 = lane < 8 ? (int)rpv[min(lane, C - 1)] : -1;
      const int lenp = uni((int)S.len[pc]);
      if (p < 0 || p >= m || lenp != d) {  // never expected: stop before any wild index
        if (lane == 0) fp_fail(M.ctl, FP_E_INTERNAL, FP_SITE_MD_PIVOT_SP, t);
        md_map_order(M, vmap, m, pos0, done);
        goto fail;
      }
      const int kp = d;
      // dense steps once the rest fits the slice and the pivots have more
      // than four neighbours (the dense layout starts over from p)
      if (na <= mbit && kp > 4) break;
      if (kp <= 4) {
        // One 16-lane row per neighbour u of p; a lane covers the slots
        // q = lane % 16 + 16 s of u's row.  p's neighbours sit in scalar
        // registers, each row's result gathers in its lane 15.
        const int rpl = lane < kp ? rpl0 : -1;
        int rp[4];
#pragma unroll
        for (int a = 0; a < 4; a++) rp[a] = wave_bcast(rpl, a);
        const int g = lane >> 4, q0 = lane & 15;
        const int u = g == 0 ? rp[0] : g == 1 ? rp[1] : g == 2 ? rp[2] : rp[3];
        const bool act = g < kp;
        const uint16_t* ru = S.rows + (long long)(act ? u : 0) * C;
        const int x0 = (int)ru[min(q0, C - 1)];
        const int lu = act ? (int)S.len[u] : 0;
        uint32_t pk = 0u;
        for (int q = q0; q < lu; q += 16) {
          const int x = q == q0 ? x0 : (int)ru[q];
#pragma unroll
          for (int a = 0; a < 4; a++)
            if (a < kp && x == rp[a]) pk |= 1u << a;
          if (x == p) pk |= (uint32_t)(q + 1) << 8;
          if (q == lu - 1) pk |= (uint32_t)x << 16;
        }
        pk |= (uint32_t)dpp_shr((int)pk, 0, 1);
        pk |= (uint32_t)dpp_shr((int)pk, 0, 2);
        pk |= (uint32_t)dpp_shr((int)pk, 0, 4);
        pk |= (uint32_t)dpp_shr((int)pk, 0, 8);
        const bool lead = act && q0 == 15;  // lane 16g+15 holds group g's result
        const uint32_t missing = ((1u << kp) - 1u) & ~pk & ~(1u << g);
        const int hole = (int)((pk >> 8) & 0xFFu) - 1;
        const int nl = lu - 1 + __popc(missing);
        if (ballot64(lead && hole < 0)) {  // p missing from a neighbour's row
          if (lane == 0) fp_fail(M.ctl, FP_E_INTERNAL, FP_SITE_MD_PIVOT_SP, t);
          md_map_order(M, vmap, m, pos0, done);
          goto fail;
        }
        if (ballot64(lead && nl > C)) break;  // convert with p still present
        if (lane == 0) {
          M.vperm[pos0 + done] = p;  // local index; mapped below
          atomicAnd(&S.bk[(long long)d * S.MW + (p >> 5)], ~(1u << (p & 31)));
        }
        if (lead) {
          uint16_t* rw = S.rows + (long long)u * C;
          if (hole != lu - 1) rw[hole] = (uint16_t)(pk >> 16);
#pragma unroll
          for (int a = 0; a < 4; a++)
            if ((missing >> a) & 1u) rw[lu - 1 + __popc(missing & ((1u << a) - 1u))] = (uint16_t)rp[a];
          S.len[u] = (uint16_t)nl;
          if (nl != lu) {
            const uint32_t bit = 1u << (u & 31);
            atomicAnd(&S.bk[(long long)lu * S.MW + (u >> 5)], ~bit);
            atomicOr(&S.bk[(long long)nl * S.MW + (u >> 5)], bit);
          }
        }
        creg -= lane == d;
        // u of group a moves from bucket lu to bucket nl: both in one word
        const int mv = lu | (nl << 16);
#pragma unroll
        for (int a = 0; a < 4; a++)
          if (a < kp) {
            const int v = wave_bcast(mv, 16 * a + 15);
            creg += (lane == (v >> 16)) - (lane == (v & 0xFFFF));
          }
        wave_fence();
      } else if (kp <= 8) {
        // One group of 8 lanes per neighbour u of p; a lane covers the slots
        // q = lane % 8 + 8 s of u's row.  p's neighbours sit in registers.
        const int rpl = lane < kp ? rpl0 : -1;
        int rp[8];  // p's neighbours (-1 past kp), in scalar registers
#pragma unroll
        for (int a = 0; a < 8; a++) rp[a] = wave_bcast(rpl, a);
        const int g = lane >> 3, q0 = lane & 7;
        int u = 0;
#pragma unroll
        for (int a = 0; a < 8; a++) u = g == a ? rp[a] : u;
        const bool act = g < kp;
        // u's length and its slot q0 are read together (u = 0 for the
        // groups past kp, whose length counts as 0)
        const uint16_t* ru = S.rows + (long long)(act ? u : 0) * C;
        const int x0 = (int)ru[min(q0, C - 1)];
        const int lu = act ? (int)S.len[u] : 0;
        // found bits (which neighbours of p u already has), the slot of p
        // (+1) and the value in u's last slot, packed for one OR reduction
        uint32_t pk = 0u;
        for (int q = q0; q < lu; q += 8) {
          const int x = q == q0 ? x0 : (int)ru[q];
#pragma unroll
          for (int a = 0; a < 8; a++)
            if (a < kp && x == rp[a]) pk |= 1u << a;
          if (x == p) pk |= (uint32_t)(q + 1) << 8;
          if (q == lu - 1) pk |= (uint32_t)x << 16;
        }
        pk |= (uint32_t)dpp_shr((int)pk, 0, 1);
        pk |= (uint32_t)dpp_shr((int)pk, 0, 2);
        pk |= (uint32_t)dpp_shr((int)pk, 0, 4);
        const bool lead = act && q0 == 7;  // lane 8g+7 holds group g's result
        const uint32_t missing = ((1u << kp) - 1u) & ~pk & ~(1u << g);
        const int hole = (int)((pk >> 8) & 0xFFu) - 1;
        const int nl = lu - 1 + __popc(missing);
        if (ballot64(lead && hole < 0)) {  // p missing from a neighbour's row
          if (lane == 0) fp_fail(M.ctl, FP_E_INTERNAL, FP_SITE_MD_PIVOT_SP, t);
          md_map_order(M, vmap, m, pos0, done);
          goto fail;
        }
        if (ballot64(lead && nl > C)) break;  // convert with p still present
        if (lane == 0) {
          M.vperm[pos0 + done] = p;  // local index; mapped below
          atomicAnd(&S.bk[(long long)d * S.MW + (p >> 5)], ~(1u << (p & 31)));
        }
        if (lead) {
          uint16_t* rw = S.rows + (long long)u * C;
          if (hole != lu - 1) rw[hole] = (uint16_t)(pk >> 16);
#pragma unroll
          for (int a = 0; a < 8; a++)
            if ((missing >> a) & 1u) rw[lu - 1 + __popc(missing & ((1u << a) - 1u))] = (uint16_t)rp[a];
          S.len[u] = (uint16_t)nl;
          if (nl != lu) {
            const uint32_t bit = 1u << (u & 31);
            atomicAnd(&S.bk[(long long)lu * S.MW + (u >> 5)], ~bit);
            atomicOr(&S.bk[(long long)nl * S.MW + (u >> 5)], bit);
          }
        }
        creg -= lane == d;
#pragma unroll
        for (int a = 0; a < 8; a++)
          if (a < kp) {  // u of group a moves from bucket lu to bucket nl
            const int o = wave_bcast(lu, 8 * a + 7), n2 = wave_bcast(nl, 8 * a + 7);
            creg += (lane == n2) - (lane == o);
          }
        wave_fence();
      } else {
        // dry run: would any neighbour row overflow?
        int over = 0;
        for (int i = lane; i < kp; i += 64) {
          const int u = rpv[i];
          const uint16_t* ru = S.rows + (long long)u * C;
          const int lu = S.len[u];
          int add = -1;  // p leaves the row
          for (int a = 0; a < kp; a++) {
            const int x = rpv[a];
            if (x == u) continue;
            bool f = false;
            for (int q = 0; q < lu; q++) f |= (ru[q] == x);
            add += !f;
          }
          if (lu + add > C) over = 1;
        }
        if (ballot64(over)) break;  // convert with p still present
        if (lane == 0) {
          M.vperm[pos0 + done] = p;  // local index; mapped below
          atomicAnd(&S.bk[(long long)d * S.MW + (p >> 5)], ~(1u << (p & 31)));
        }
        for (int i = lane; i < kp; i += 64) S.nbl[i] = rpv[i];
        wave_fence();
        // the neighbours become a clique; their degrees move between buckets
        int d1 = 0, d2 = 0;
        for (int i = lane; i < kp; i += 64) {
          const int u = S.nbl[i];
          uint16_t* ru = S.rows + (long long)u * C;
          d1 = S.len[u];
          int lu = d1;
          for (int q = 0; q < lu; q++)
            if (ru[q] == p) {
              ru[q] = ru[lu - 1];
              lu--;
              break;
            }
          for (int a = 0; a < kp; a++) {
            const int x = S.nbl[a];
            if (x == u) continue;
            bool f = false;
            for (int q = 0; q < lu; q++) f |= (ru[q] == x);
            if (!f) ru[lu++] = (uint16_t)x;
          }
          d2 = lu;
          S.len[u] = (uint16_t)lu;
          if (lu != d1) {
            const uint32_t bit = 1u << (u & 31);
            atomicAnd(&S.bk[(long long)d1 * S.MW + (u >> 5)], ~bit);
            atomicOr(&S.bk[(long long)lu * S.MW + (u >> 5)], bit);
          }
        }
        creg -= lane == d;
        for (int a = 0; a < kp; a++) {  // kp <= C < 64: one neighbour per lane
          const int o = wave_bcast(d1, a), n2 = wave_bcast(d2, a);
          if (o != n2) creg += (lane == n2) - (lane == o);
        }
        wave_fence();
      }
      done++;
      na--;
    }
    md_map_order(M, vmap, m, pos0, done);
    if (na == 0) return;
    // re-index the remaining vertices (rank order) into BIT form; stage the
    // sparse state in the pool first since the BIT layout reuses the slice
    gptr<unsigned> st = pool_alloc(M, (unsigned long long)m * C / 2 + 2ull * m + 64);
    if (!st) goto fail;
    // the live set is the union of the degree buckets (the steps keep only
    // the buckets)
    for (int w = lane_id(); w < S.MW; w += 64) {
      uint32_t x = 0u;
      for (int dd = 0; dd <= C; dd++) x |= S.bk[(long long)dd * S.MW + w];
      S.alive[w] = x;
    }
    wave_fence();
    {
      const long long wrows = ((long long)m * C + 1) / 2, wlen = (m + 1) / 2;
      gptr<uint16_t> srows = st.as<uint16_t>();
      gptr<uint16_t> slen = (st + wrows).as<uint16_t>();
      gptr<int> ni = (st + wrows + wlen).as<int>();
      for (long long i = lane_id(); i < (long long)m * C; i += 64) srows[i] = S.rows[i];
      int run = 0;
      for (int i0 = 0; i0 < m; i0 += 64) {
        const int i = i0 + lane_id();
        const bool al = i < m && ((S.alive[i >> 5] >> (i & 31)) & 1u);
        if (i < m) slen[i] = S.len[i];
        const uint64_t bal = ballot64(al);
        if (i < m) ni[i] = al ? run + popc64(bal & lanemask_lt()) : -1;
        run += popc64(bal);
      }
      wave_fence();
      gptr<int> vm2 = pool_alloc(M, na).as<int>();
      if (!vm2) goto fail;
      for (int i = lane_id(); i < m; i += 64)
        if (ni[i] >= 0) vm2[ni[i]] = vmap[i];
      wave_fence();
      // two call sites, so each keeps one address space (LDS or global)
      if (na <= mbit) {
        md_sp_to_bit(M, slice, na, m, C, srows, slen, ni, vm2, pos0 + done);
      } else {
        const long long bytes = md_bit_bytes(na);
        char* mem = (char*)(unsigned*)pool_alloc(M, (bytes + 3) / 4);
        if (!mem) goto fail;
        md_sp_to_bit(M, mem, na, m, C, srows, slen, ni, vm2, pos0 + done);
      }
      return;
    }
  } else {
    // too large for LDS: BIT layout in the pool
    const long long bytes = md_bit_bytes(m);
    char* mem = (char*)(unsigned*)pool_alloc(M, (bytes + 3) / 4);
    if (!mem) goto fail;
    MdBit B;
    md_bit_carve(B, mem, m);
    md_bit_build(M, B, t, V);
    md_bit_run(M, B, V, pos0, m);
    return;
  }
fail:
  // keep perm a bijection: remaining vertices in index order
  {
    int run = 0;
    for (int i0 = 0; i0 < m; i0 += 64) {
      const int i = i0 + lane_id();
      bool rem = false;
      if (i < m) {
        const int v = V[i];
        rem = true;
        for (int q = 0; q < done; q++) rem &= (M.vperm[pos0 + q] != v);
      }
      const uint64_t bal = ballot64(rem);
      if (rem) {
        const int pos = pos0 + done + run + popc64(bal & lanemask_lt());
        M.vperm[pos] = V[i];
        M.viperm[V[i]] = pos;
      }
      run += popc64(bal);
    }
  }
}

// node t at its range in the schedule, vertices as the grouping listed them
__device__ __forceinline__ void md_node(const FpMesh& M, int t, char* slice, long long slice_bytes) {
  const int m = uni(M.nsize[t]);
  const int pos0 = uni(M.nbegin[t]);
  md_node_list(M, t, M.gbuf + pos0, m, pos0, slice, slice_bytes);
}

// Size classes of the local orders, by the LDS the dense layout needs:
//   3: a quarter of the per-node LDS (four waves per workgroup),
//   2: a quarter of the large LDS, 1: half of it, 0: all of it (one wave;
//      also every node too large for the dense layout).
// A node goes to the highest class whose slice holds its dense layout
// (m <= md_bit_max of the slice), else to class 0.  Slices sized to the
// node keep several waves per CU on the mid-size nodes.
#define FP_MD_CLASSES 4
__device__ __forceinline__ int md_slice_waves(int c) { return c == 0 ? 1 : c == 1 ? 2 : 4; }
__device__ __forceinline__ long long md_slice_bytes(int c, long long lds, long long big) {
  return ((c == 3 ? lds : big) / md_slice_waves(c)) & ~15ll;
}

