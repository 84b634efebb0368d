// fp_stages_sym.h -- elimination tree and column counts of A(perm, perm)
// (the symbolic data sparse Cholesky needs, Sec. 2; the paper hands this to
// the solver, Sec. 6), computed bottom-up over the separator tree.
//
// Node t owns the contiguous positions [b, b+m) of perm; every vertex that
// precedes it and touches it lies in t's subtree, every later neighbour in
// t or an ancestor.  The children summarise their eliminated subtrees as
// *elements*: one per connected component, carrying its boundary (later
// positions adjacent to the component).  Eliminating position k of t:
//   struct(k) = (later neighbours of k in A)  U  (boundaries of live elements
//               that contain k), minus positions <= k,
//   colcount(k) = 1 + |struct(k)|,  parent(k) = min struct(k) (or -1),
// the absorbed elements die and struct(k) becomes a new element.  This is
// symbolic elimination in quotient-graph form (George & Liu), exact for any
// order, so it agrees with the row-subtree definition of the column counts.
// Boundaries are bitsets over F = t's positions followed by the sorted later
// positions t can reach, held in the wave's LDS slice (pool when larger).
#pragma once

#include "fp_stages_md.h"

struct SymLay {
  int* bd;        // sorted later positions, capacity ncand
  int* optr;      // m+1
  int* oent;      // forward neighbours, F-local
  uint32_t* sw;   // struct work bitset, FW words
  uint32_t* slots;  // nslot x FW
  int* live;      // nslot
  int* freel;     // nslot
  int* tmp;       // 128 ints
  int m, FW, nslot, ncand, nent;
};

__device__ __forceinline__ int lower_bound_i(const int* a, int n, int x) {
  int lo = 0, hi = n;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (a[mid] < x)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}

// F-local index of position q (t's own range first, then the sorted list of
// later positions); -1 if q is in neither, which the callers report
__device__ __forceinline__ int sym_findex(int q, int b0, int e0, int m, const int* bd, int nbd) {
  if (q >= b0 && q < e0) return q - b0;
  if (q < e0) return -1;
  const int i = lower_bound_i(bd, nbd, q);
  return (i < nbd && bd[i] == q) ? m + i : -1;
}

// a failed internal check: record it, leave no elements for the parent
__device__ __forceinline__ bool sym_abort(const FpMesh& M, int t, int site) {
  if (lane_id() == 0) {
    fp_fail(M.ctl, FP_E_INTERNAL, site, t);
    M.eoff[3 * t] = 0;
    M.eoff[3 * t + 1] = 0;
    M.eoff[3 * t + 2] = 0;
  }
  return true;
}

// returns bytes needed (0 if nslot would be < 1)
__device__ __forceinline__ long long sym_bytes(int m, int ncand, int nent, int FW, int nslot) {
  return 4ll * ncand + 4ll * (m + 1) + 4ll * nent + 4ll * FW + (4ll * FW + 8) * nslot + 512 + 64;
}

// Process node t at depth d.  Returns false if the given memory was too
// small (the caller retries with pool memory).
__device__ __forceinline__ bool sym_node_try(const FpMesh& M, int t, int d, char* mem, long long bytes,
                             bool full) {
  FpCtl* Cc = M.ctl;
  const int m = M.nsize[t];
  const int b0 = M.nbegin[t], e0 = b0 + m;
  const int nn = Cc->nn;
  const int* src = M.arena[(d + 1) & 1];
  // child element records: [len, pos...] ...
  int cst[2] = {0, 0}, cin[2] = {0, 0}, crec[2] = {0, 0};
  for (int c = 0; c < 2; c++) {
    const int ch = 2 * t + 1 + c;
    if (ch < nn) {
      cst[c] = M.eoff[3 * ch];
      cin[c] = M.eoff[3 * ch + 1];
      crec[c] = M.eoff[3 * ch + 2];
    }
  }
  const int nce = crec[0] + crec[1];
  // inputs in range: t's positions hold vertices placed there by the local
  // orders, child records hold positions of t or later.  An earlier failure
  // can leave them unset; then t is skipped instead of indexing wildly.
  {
    bool bad = b0 < 0 || m < 0 || e0 > M.n;
    for (int k = lane_id(); k < m && !bad; k += 64) {
      const int v = M.vperm[b0 + k];
      bad = (unsigned)v >= (unsigned)M.n || M.viperm[v] != b0 + k;
    }
    bad = ballot64(bad) != 0;
    int site = bad ? FP_SITE_SYM_VERTEX : 0;
    for (int c = 0; c < 2 && !bad; c++) {
      site = FP_SITE_SYM_RECORD;
      if (cst[c] < 0 || cin[c] < 0 || (long long)cst[c] + cin[c] > M.acap || crec[c] < 0) {
        bad = true;
        break;
      }
      int off = cst[c];
      const int end = cst[c] + cin[c];
      int nrec = 0;
      while (off < end) {  // uniform: every lane walks the same records
        const int len = src[off];
        if (len < 0 || off + 1 + len > end) {
          bad = true;
          break;
        }
        for (int i = lane_id(); i < len; i += 64) {
          const int q = src[off + 1 + i];
          if (q < b0 || q >= M.n) bad = true;
        }
        off += 1 + len;
        nrec++;
      }
      if (nrec != crec[c]) bad = true;
      bad = ballot64(bad) != 0;
    }
    if (bad) {
      if (lane_id() == 0) {
        fp_fail(Cc, FP_E_INTERNAL, site, t);
        M.eoff[3 * t] = 0;
        M.eoff[3 * t + 1] = 0;
        M.eoff[3 * t + 2] = 0;
      }
      return true;
    }
  }
  // count forward neighbours and later (ancestor) candidates
  int nfw = 0, nanc = 0;
  for (int k = lane_id(); k < m; k += 64) {
    const int v = M.vperm[b0 + k];
    for (int e = M.grp[v]; e < M.grp[v + 1]; e++) {
      const int q = M.viperm[M.gci[e]];
      if (q > b0 + k) {
        nfw++;
        nanc += (q >= e0);
      }
    }
  }
  nfw = wave_sum_i32(nfw);
  nanc = wave_sum_i32(nanc);
  const int nchild_ents = cin[0] + cin[1] - nce;
  int ncand = nanc + nchild_ents;
  if (ncand < 0 || ncand > (1 << 29)) return sym_abort(M, t, FP_SITE_SYM_RECORD);
  int np2 = 1;
  while (np2 < ncand) np2 <<= 1;
  ncand = max(np2, 64);
  // F is at most m + ncand
  const int FWmax = (m + ncand + 31) >> 5;
  int nslot = full ? (nce + m + 1) : 0;
  if (!full) {
    const long long fixed = sym_bytes(m, ncand, nfw, FWmax, 0);
    if (fixed > bytes) return false;
    nslot = (int)min((long long)(nce + m + 1), (bytes - fixed) / (4ll * FWmax + 8));
    if (nslot < nce + 1) return false;
  } else if (sym_bytes(m, ncand, nfw, FWmax, nslot) > bytes) {
    return false;
  }
  SymLay L;
  {
    char* p = mem;
    L.tmp = (int*)p;
    p += 512;
    L.bd = (int*)p;
    p += 4ll * ncand;
    L.optr = (int*)p;
    p += 4ll * (m + 1);
    L.oent = (int*)p;
    p += 4ll * nfw;
    L.sw = (uint32_t*)p;
    p += 4ll * FWmax;
    L.live = (int*)p;
    p += 4ll * nslot;
    L.freel = (int*)p;
    p += 4ll * nslot;
    p = mem + ((p - mem + 15) & ~15ll);  // mem is 16-byte aligned; keeps the LDS address space
    L.slots = (uint32_t*)p;
  }
  L.m = m;
  L.nslot = nslot;
  L.ncand = ncand;
  // 1. later positions reachable from t: child boundaries and t's own rows
  int nc = 0;
  for (int c = 0; c < 2; c++) {
    int off = cst[c];
    const int end = cst[c] + cin[c];
    while (off < end) {
      const int len = src[off];
      for (int i = lane_id(); i < len; i += 64) {
        const int q = src[off + 1 + i];
        L.bd[nc + i] = q >= e0 ? q : 0x7FFFFFFF;
      }
      nc += len;
      off += 1 + len;
    }
  }
  {
    int run = nc;
    for (int k0 = 0; k0 < m; k0 += 64) {
      const int k = k0 + lane_id();
      int cnt = 0;
      if (k < m) {
        const int v = M.vperm[b0 + k];
        for (int e = M.grp[v]; e < M.grp[v + 1]; e++) cnt += (M.viperm[M.gci[e]] >= e0);
      }
      const int inc = wave_incl_scan(cnt);
      int o = run + inc - cnt;
      if (k < m) {
        const int v = M.vperm[b0 + k];
        for (int e = M.grp[v]; e < M.grp[v + 1]; e++) {
          const int q = M.viperm[M.gci[e]];
          if (q >= e0) L.bd[o++] = q;
        }
      }
      run += __shfl(inc, 63, 64);
    }
    nc = run;
  }
  for (int i = nc + lane_id(); i < ncand; i += 64) L.bd[i] = 0x7FFFFFFF;
  __threadfence_block();
  wave_sort_ids(L.bd, ncand, ncand);
  // unique
  int nbd = 0;
  for (int i0 = 0; i0 < ncand; i0 += 64) {
    const int i = i0 + lane_id();
    const int x = i < ncand ? L.bd[i] : 0x7FFFFFFF;
    const bool keep = x != 0x7FFFFFFF && (i == 0 || L.bd[i - 1] != x);
    const uint64_t bal = ballot64(keep);
    // compaction in place is safe: writes go to index <= read index
    const int dst = nbd + popc64(bal & lanemask_lt());
    __threadfence_block();
    if (keep) L.bd[dst] = x;
    __threadfence_block();
    nbd += popc64(bal);
  }
  const int F = m + nbd;
  const int FW = (F + 31) >> 5;
  L.FW = FW;
  // 2. forward rows in F-local indices
  {
    bool bad = nbd > ncand;
    int run = 0;
    for (int k0 = 0; k0 < m; k0 += 64) {
      const int k = k0 + lane_id();
      int cnt = 0;
      if (k < m) {
        const int v = M.vperm[b0 + k];
        for (int e = M.grp[v]; e < M.grp[v + 1]; e++) cnt += (M.viperm[M.gci[e]] > b0 + k);
      }
      const int inc = wave_incl_scan(cnt);
      int o = run + inc - cnt;
      if (k < m) {
        L.optr[k] = o;
        const int v = M.vperm[b0 + k];
        for (int e = M.grp[v]; e < M.grp[v + 1]; e++) {
          const int q = M.viperm[M.gci[e]];
          if (q > b0 + k) {
            const int f = sym_findex(q, b0, e0, m, L.bd, nbd);
            bad |= f < 0;
            L.oent[o++] = f < 0 ? m : f;
          }
        }
      }
      run += __shfl(inc, 63, 64);
    }
    if (lane_id() == 0) L.optr[m] = run;
    if (ballot64(bad) || run != nfw) return sym_abort(M, t, FP_SITE_SYM_LOOKUP);
  }
  // 3. child elements become slots
  int nlive = 0;
  bool bad3 = nce > nslot;
  for (int c = 0; c < 2 && !bad3; c++) {
    int off = cst[c];
    const int end = cst[c] + cin[c];
    while (off < end) {
      const int len = src[off];
      uint32_t* sl = L.slots + (long long)nlive * FW;
      for (int w = lane_id(); w < FW; w += 64) sl[w] = 0u;
      __threadfence_block();
      for (int i = lane_id(); i < len; i += 64) {
        const int q = src[off + 1 + i];
        const int f = sym_findex(q, b0, e0, m, L.bd, nbd);
        if (f < 0)
          bad3 = true;
        else
          atomicOr(&sl[f >> 5], 1u << (f & 31));
      }
      if (lane_id() == 0) L.live[nlive] = nlive;
      nlive++;
      off += 1 + len;
    }
  }
  if (ballot64(bad3) || nlive != nce) return sym_abort(M, t, FP_SITE_SYM_LOOKUP);
  int nfree = 0;
  for (int i = nlive + lane_id(); i < nslot; i += 64) L.freel[i - nlive] = i;
  nfree = nslot - nlive;
  __threadfence_block();
  // 4. eliminate t's positions in order
  for (int k = 0; k < m; k++) {
    const int kw = k >> 5;
    if (nlive < 0 || nlive > nslot || nfree < 0 || nfree > nslot) return sym_abort(M, t, FP_SITE_SYM_LIVE);
    bool bad4 = false;
    // live elements containing k
    int nab = 0;
    for (int j0 = 0; j0 < nlive; j0 += 64) {
      const int j = j0 + lane_id();
      int sidx = j < nlive ? L.live[j] : 0;
      if ((unsigned)sidx >= (unsigned)nslot) {
        bad4 = true;
        sidx = 0;
      }
      const bool has = j < nlive && ((L.slots[(long long)sidx * FW + kw] >> (k & 31)) & 1u);
      const uint64_t bal = ballot64(has);
      if (has) L.tmp[nab + popc64(bal & lanemask_lt())] = j;  // live-list slot index
      nab += popc64(bal);
      if (nab > 48) break;  // many absorptions: handled below in chunks
    }
    __threadfence_block();
    // struct = union of absorbed boundaries and the forward row, bits > k
    for (int w = kw + lane_id(); w < FW; w += 64) {
      uint32_t x = 0;
      for (int a = 0; a < min(nab, 48); a++) {
        const int j = L.tmp[a];
        const int sj = (unsigned)j < (unsigned)nlive ? L.live[j] : -1;
        if ((unsigned)sj < (unsigned)nslot)
          x |= L.slots[(long long)sj * FW + w];
        else
          bad4 = true;
      }
      L.sw[w] = x;
    }
    __threadfence_block();
    if (nab > 48) {
      // rare: scan every live element directly
      for (int w = kw + lane_id(); w < FW; w += 64) {
        uint32_t x = L.sw[w];
        for (int j = 0; j < nlive; j++) {
          const int s = L.live[j];
          if ((unsigned)s >= (unsigned)nslot) {
            bad4 = true;
            continue;
          }
          const uint32_t* sl = L.slots + (long long)s * FW;
          if ((sl[kw] >> (k & 31)) & 1u) x |= sl[w];
        }
        L.sw[w] = x;
      }
      __threadfence_block();
    }
    const int r0 = L.optr[k], r1 = L.optr[k + 1];
    bad4 |= r0 < 0 || r1 < r0 || r1 > nfw;
    if (ballot64(bad4)) return sym_abort(M, t, FP_SITE_SYM_LIVE);
    for (int e = r0 + lane_id(); e < r1; e += 64) {
      const int f = L.oent[e];
      if (f > k && f < F) atomicOr(&L.sw[f >> 5], 1u << (f & 31));
      else bad4 = true;
    }
    if (ballot64(bad4)) return sym_abort(M, t, FP_SITE_SYM_ROWS);
    __threadfence_block();
    if (lane_id() == 0) {
      const uint32_t msk = (k & 31) == 31 ? 0u : (0xFFFFFFFFu << ((k & 31) + 1));
      L.sw[kw] &= msk;
    }
    __threadfence_block();
    int cnt = 0;
    uint32_t first = 0xFFFFFFFFu;
    for (int w = kw + lane_id(); w < FW; w += 64) {
      const uint32_t x = L.sw[w];
      cnt += popc32(x);
      if (x && first == 0xFFFFFFFFu) first = (uint32_t)(w * 32 + __ffs(x) - 1);
    }
    cnt = wave_sum_i32(cnt);
    first = wave_min_u32(first);
    if (first != 0xFFFFFFFFu && (first <= (uint32_t)k || first >= (uint32_t)F))
      return sym_abort(M, t, FP_SITE_SYM_PIVOT);
    if (lane_id() == 0) {
      M.vcc[b0 + k] = 1 + cnt;
      int par = -1;
      if (first != 0xFFFFFFFFu) par = (int)first < m ? b0 + (int)first : L.bd[first - m];
      M.vpar[b0 + k] = par;
    }
    // remove absorbed elements from the live list, recycle their slots
    {
      int nl = 0;
      int nf_add = 0;
      for (int j0 = 0; j0 < nlive; j0 += 64) {
        const int j = j0 + lane_id();
        bool absorbed = false;
        int sidx = 0;
        if (j < nlive) {
          sidx = L.live[j];
          if ((unsigned)sidx >= (unsigned)nslot) {
            bad4 = true;
            sidx = 0;
          }
          absorbed = (L.slots[(long long)sidx * FW + kw] >> (k & 31)) & 1u;
        }
        const uint64_t bk = ballot64(j < nlive && !absorbed);
        const uint64_t ba = ballot64(absorbed);
        __threadfence_block();
        if (j < nlive && !absorbed) L.live[nl + popc64(bk & lanemask_lt())] = sidx;
        if (absorbed) L.freel[nfree + nf_add + popc64(ba & lanemask_lt())] = sidx;
        __threadfence_block();
        nl += popc64(bk);
        nf_add += popc64(ba);
      }
      nlive = nl;
      nfree += nf_add;
    }
    if (ballot64(bad4) || nlive + nfree != nslot) return sym_abort(M, t, FP_SITE_SYM_LIVE);
    if (cnt > 0) {
      if (nfree == 0) return false;  // out of slots
      const int sidx = L.freel[nfree - 1];
      nfree--;
      if ((unsigned)sidx >= (unsigned)nslot) return sym_abort(M, t, FP_SITE_SYM_LIVE);
      uint32_t* sl = L.slots + (long long)sidx * FW;
      for (int w = lane_id(); w < FW; w += 64) sl[w] = w >= kw ? L.sw[w] : 0u;
      if (lane_id() == 0) L.live[nlive] = sidx;
      nlive++;
    }
    __threadfence_block();
  }
  // 5. surviving elements (boundaries beyond t) go to the parent
  int total = 0;
  for (int j = 0; j < nlive; j++) {
    const uint32_t* sl = L.slots + (long long)L.live[j] * FW;
    int c = 0;
    for (int w = lane_id(); w < FW; w += 64) c += popc32(sl[w]);
    total += 1 + wave_sum_i32(c);
  }
  int base = 0;
  if (lane_id() == 0) {
    base = atomicAdd(&Cc->arena_top[d & 1], total);
    if ((long long)base + total > M.acap) {
      fp_fail(Cc, FP_E_SCRATCH, FP_SITE_SYM_ARENA, t);
      base = -1;
    }
  }
  base = __shfl(base, 0, 64);
  if (base < 0) {
    if (lane_id() == 0) {
      M.eoff[3 * t] = 0;
      M.eoff[3 * t + 1] = 0;
      M.eoff[3 * t + 2] = 0;
    }
    return true;
  }
  int* dst = M.arena[d & 1];
  int off = base;
  for (int j = 0; j < nlive; j++) {
    const uint32_t* sl = L.slots + (long long)L.live[j] * FW;
    int len = 0;
    for (int w0 = 0; w0 < FW; w0 += 64) {
      const int w = w0 + lane_id();
      uint32_t x = w < FW ? sl[w] : 0u;
      const int c = popc32(x);
      const int inc = wave_incl_scan(c);
      int o = off + 1 + len + inc - c;
      while (x) {
        const int f = w * 32 + __ffs(x) - 1;
        x &= x - 1;
        dst[o++] = f < m ? b0 + f : L.bd[f - m];
      }
      len += __shfl(inc, 63, 64);
    }
    if (lane_id() == 0) dst[off] = len;
    off += 1 + len;
  }
  if (lane_id() == 0) {
    M.eoff[3 * t] = base;
    M.eoff[3 * t + 1] = total;
    M.eoff[3 * t + 2] = nlive;
  }
  return true;
}

__device__ __forceinline__ void sym_node(const FpMesh& M, int t, int d, char* slice, long long sb) {
  if (sym_node_try(M, t, d, slice, sb, false)) return;
  // pool memory sized for the worst case of this node
  const int m = M.nsize[t];
  long long words = 0;
  {
    // generous bound: F <= m + later candidates; nslot = children + m + 1
    int cin = 0, crec = 0;
    for (int c = 0; c < 2; c++) {
      const int ch = 2 * t + 1 + c;
      if (ch < M.ctl->nn) {
        cin += M.eoff[3 * ch + 1];
        crec += M.eoff[3 * ch + 2];
      }
    }
    int nfw = 0;
    for (int k = lane_id(); k < m; k += 64) {
      const int v = M.vperm[M.nbegin[t] + k];
      nfw += M.grp[v + 1] - M.grp[v];
    }
    nfw = wave_sum_i32(nfw);
    long long nc = 1;
    while (nc < (long long)nfw + cin) nc <<= 1;
    nc = max(nc, 64ll);
    const long long FW = (m + nc + 31) / 32;
    words = (sym_bytes(m, (int)nc, nfw, (int)FW, crec + m + 1) + 3) / 4 + 64;
  }
  char* mem = (char*)pool_alloc(M, words);
  if (!mem) return;
  if (!sym_node_try(M, t, d, mem, words * 4, true))
    if (lane_id() == 0) fp_fail(M.ctl, FP_E_INTERNAL, FP_SITE_SYM_SLOTS, t);
}

