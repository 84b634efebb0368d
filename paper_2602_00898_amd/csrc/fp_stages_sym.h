// fp_stages_sym.h -- elimination tree and column counts of A(perm, perm)
// (the symbolic data sparse Cholesky needs, Sec. 2; the paper hands this to
// the solver, Sec. 6), computed bottom-up over the separator tree.
//
// Node t owns the contiguous positions [b, b+m) of perm; every vertex that
// precedes it and touches it lies in t's subtree, every later neighbour in
// t or an ancestor.  Column k of L has the structure
//   struct(k) = adj+(k)  U  (struct(j) for the columns j whose etree parent
//               is k)  minus positions <= k,
// parent(k) = min struct(k) (-1 if empty) and colcount(k) = 1 + |struct(k)|
// (the column-structure recurrence of the elimination tree, Liu 1990).
// Columns of t's subtree whose parent lies beyond t reach t as *elements*:
// records [len, positions...] written by the children into an arena.
//
// Per tree level, three kernels, one wave per node, all scratch in a global
// pool (reset per level):
//   prep -- the node's index space F = t's positions followed by the sorted
//           later positions it can reach; forward rows in F indices; every
//           incoming element as a bitset row, queued on the column that
//           absorbs it (its least position) or passed through;
//   elim -- columns in order: OR of the rows queued on k and k's forward
//           row; the new row is queued on its parent or leaves t;
//   emit -- the rows that leave t become the parent's element records.
#pragma once

#include <type_traits>

#include "fp_stages_md.h"

// node scratch header (32-bit words at the start of the node's pool block)
enum {
  SH_M = 0,
  SH_NBD,     // later positions in the index space
  SH_NFW,     // forward entries
  SH_FW,      // words of a row in use
  SH_ROWS,    // m + incoming elements
  SH_NCE,     // incoming elements
  SH_NP2,     // capacity of the later-position list
  SH_STRIDE,  // words per row
  SH_NOUT,    // rows leaving t
  SH_OK,      // 1 when prep finished
  SH_WORDS = 16
};

struct SymView {
  gptr<int> hdr;
  gptr<int> bd;      // np2: sorted later positions
  gptr<int> optr;    // m+1
  gptr<int> oent;    // nfw: forward entries, F indices
  gptr<int> head;    // m: first row queued on column k, -1 if none
  gptr<int> next;    // rows: next row in the same queue
  gptr<int> outl;    // rows: rows that leave t
  gptr<uint32_t> rows;  // rows x stride words
};

__device__ __forceinline__ long long sym_words(int m, int np2, int nfw, int rows, int stride) {
  return SH_WORDS + (long long)np2 + (m + 1) + nfw + m + 2ll * rows + (long long)rows * stride + 4;
}

__device__ __forceinline__ SymView sym_view(gptr<unsigned> base, int m, int np2, int nfw, int rows) {
  SymView V;
  gptr<int> p = base.as<int>();
  V.hdr = p;
  p += SH_WORDS;
  V.bd = p;
  p += np2;
  V.optr = p;
  p += m + 1;
  V.oent = p;
  p += nfw;
  V.head = p;
  p += m;
  V.next = p;
  p += rows;
  V.outl = p;
  p += rows;
  V.rows = p.as<uint32_t>();
  return V;
}

// node t produces no elements for its parent and no scratch for the later
// kernels of this level; `site` != 0 also records a failed check
__device__ __forceinline__ void sym_drop(const FpMesh& M, int t, int site) {
  if (lane_id() == 0) {
    if (site) fp_fail(M.ctl, FP_E_INTERNAL, site, t);
    M.sdesc[t] = -1;
    M.eoff[3 * t] = 0;
    M.eoff[3 * t + 1] = 0;
    M.eoff[3 * t + 2] = 0;
  }
}

// ---------------------------------------------------------------- prep
// The permuted rows of a node's columns, 256 columns per step: lane l takes
// columns k0 + l + 64 u (u < 4) and holds the first FP_PREP_ROW entries of
// each row in registers, every load of the step issued at once (mesh rows
// have 4 to 8 entries), so a step costs two memory round trips; entries past
// FP_PREP_ROW are read from memory when visited.
#define FP_PREP_ROW 8
#define FP_PREP_COLS 4
struct PrepRows {
  int e0[FP_PREP_COLS], deg[FP_PREP_COLS];
  int q[FP_PREP_COLS][FP_PREP_ROW];
};
// rows k of a CSR (rp, ent), k = k0 + lane + 64 u < m, position base + k
__device__ __forceinline__ void csr_rows(gptr<const int> rp, gptr<const int> ent, int base, int m,
                                         int k0, PrepRows& r) {
#pragma unroll
  for (int u = 0; u < FP_PREP_COLS; u++) {
    const int k = k0 + lane_id() + 64 * u;
    const bool act = k < m;
    r.e0[u] = act ? rp[base + k] : 0;
    r.deg[u] = act ? rp[base + k + 1] - r.e0[u] : 0;
  }
#pragma unroll
  for (int u = 0; u < FP_PREP_COLS; u++)
#pragma unroll
    for (int j = 0; j < FP_PREP_ROW; j++) r.q[u][j] = j < r.deg[u] ? ent[r.e0[u] + j] : 0;
}
__device__ __forceinline__ void prep_rows(const FpMesh& M, int b0, int m, int k0, PrepRows& r) {
  csr_rows(M.prow, M.pent, b0, m, k0, r);
}
// fn(q) for every entry q of the row of column k0 + lane + 64 u
template <class Fn>
__device__ __forceinline__ void csr_each(gptr<const int> ent, const PrepRows& r, int u, Fn fn) {
#pragma unroll
  for (int j = 0; j < FP_PREP_ROW; j++)
    if (j < r.deg[u]) fn(r.q[u][j]);
  for (int j = FP_PREP_ROW; j < r.deg[u]; j++) fn((int)ent[r.e0[u] + j]);
}
template <class Fn>
__device__ __forceinline__ void prep_each(const FpMesh& M, const PrepRows& r, int u, Fn fn) {
  csr_each(M.pent, r, u, fn);
}

// Sizes and child records of a node, for the second half of the prep.
struct PrepIn {
  int m, b0, e0, na, BW, np2, nfw, nanc, nce, rows, stride;
  int cst[2], cin[2];
};

// Bit of each later position q[j] in the bitmap over the ancestors' ranges
// (anc: begin, size, bit offset per ancestor, begins increasing), or -1.
// The search is branch free with a step count set by na alone (top: the
// largest power of two <= na, 0 if na == 0), so the N lookups run side by
// side: each step is one LDS round trip for all of them.
template <int N>
__device__ __forceinline__ void anc_bits(const int* anc, int na, int top, const int (&q)[N],
                                         int (&bit)[N]) {
  int c[N];  // ancestors beginning at or before q[j]
#pragma unroll
  for (int j = 0; j < N; j++) c[j] = 0;
  for (int st = top; st > 0; st >>= 1) {
    int bg[N];
#pragma unroll
    for (int j = 0; j < N; j++) bg[j] = anc[3 * (min(c[j] + st, na) - 1)];
#pragma unroll
    for (int j = 0; j < N; j++) c[j] += (c[j] + st <= na && bg[j] <= q[j]) ? st : 0;
  }
  int beg[N], sz[N], off[N];
#pragma unroll
  for (int j = 0; j < N; j++) {
    const int f = max(c[j] - 1, 0);
    beg[j] = anc[3 * f];
    sz[j] = anc[3 * f + 1];
    off[j] = anc[3 * f + 2];
  }
#pragma unroll
  for (int j = 0; j < N; j++)
    bit[j] = c[j] > 0 && q[j] < beg[j] + sz[j] ? off[j] + (q[j] - beg[j]) : -1;
}

// Second half of the prep: the later positions (marked in a bitmap over the
// ancestors' ranges and read back in order), the forward rows in F
// indices, and the incoming element rows.  bm and pre (BW words each) and
// rbuf (stride words) live in LDS or in the pool (P a plain or a global
// pointer).  The F index of a later position is m plus its rank in the
// bitmap: the prefix count of its word plus the set bits below it.
template <class P>
__device__ __forceinline__ void sym_prep_tail(const FpMesh& M, int t, const SymView& V,
                                              gptr<unsigned> base, gptr<const int> src,
                                              const int* anc, const PrepIn& in, P bm, P pre,
                                              P rbuf) {
  const int m = in.m, b0 = in.b0, e0 = in.e0, na = in.na, BW = in.BW, np2 = in.np2;
  const int lane = lane_id();
  int top = 0;
  if (na > 0)
    for (top = 1; (top << 1) <= na;) top <<= 1;
  for (int w = lane; w < BW; w += 64) bm[w] = 0u;
  wave_fence();
  // F index of each q[j] (t's own range first, then the later positions in
  // order; -1 if q[j] is in neither, which the callers report), the lookups
  // of a call side by side.  Reads the bitmap only when a lane needs it.
  auto findex_n = [&](const auto& q, auto& f) {
    constexpr int N = std::extent<std::remove_reference_t<decltype(q)>>::value;
    bool later = false;
#pragma unroll
    for (int j = 0; j < N; j++) {
      f[j] = q[j] >= b0 && q[j] < e0 ? q[j] - b0 : -1;
      later |= q[j] >= e0;
    }
    if (ballot64(later)) {
      int bit[N];
      anc_bits<N>(anc, na, top, q, bit);
      uint32_t x[N];
      int pr[N];
#pragma unroll
      for (int j = 0; j < N; j++) {
        const int wd = max(bit[j], 0) >> 5;
        x[j] = bm[wd];
        pr[j] = pre[wd];
      }
#pragma unroll
      for (int j = 0; j < N; j++) {
        const uint32_t b = 1u << (bit[j] & 31);
        if (q[j] >= e0 && bit[j] >= 0 && (x[j] & b)) f[j] = m + pr[j] + popc32(x[j] & (b - 1u));
      }
    }
  };
  auto findex = [&](int q) -> int {
    const int qa[1] = {q};
    int fa[1];
    findex_n(qa, fa);
    return fa[0];
  };
  // 1. mark the later positions of the child records and of t's own rows
  bool bad1 = false;
  // mark every q[j] >= e0 (the others are skipped)
  auto mark_n = [&](const auto& q) {
    constexpr int N = std::extent<std::remove_reference_t<decltype(q)>>::value;
    bool need = false;
#pragma unroll
    for (int j = 0; j < N; j++) need |= q[j] >= e0;
    if (!ballot64(need)) return;
    int bit[N];
    anc_bits<N>(anc, na, top, q, bit);
#pragma unroll
    for (int j = 0; j < N; j++) {
      if (q[j] < e0) continue;
      if (bit[j] < 0)
        bad1 = true;
      else
        atomicOr(&bm[bit[j] >> 5], 1u << (bit[j] & 31));
    }
  };
  // the positions of a child record, four per lane loaded together
  // (-1 past its end)
  auto record_round = [&](int off, int len, int i0, int (&q)[FP_PREP_COLS]) {
#pragma unroll
    for (int u = 0; u < FP_PREP_COLS; u++) {
      const int i = i0 + lane + 64 * u;
      q[u] = i < len ? src[off + 1 + i] : -1;
    }
  };
  for (int c = 0; c < 2; c++) {
    int off = in.cst[c];
    const int end = in.cst[c] + in.cin[c];
    while (off < end) {
      const int len = uni(src[off]);
      for (int i0 = 0; i0 < len; i0 += 64 * FP_PREP_COLS) {
        int q[FP_PREP_COLS];
        record_round(off, len, i0, q);
        mark_n(q);
      }
      off += 1 + len;
    }
  }
  // (t's rows reach no later position when the count found none)
  for (int k0 = 0; k0 < (in.nanc ? m : 0); k0 += 64 * FP_PREP_COLS) {
    PrepRows R;
    prep_rows(M, b0, m, k0, R);
#pragma unroll
    for (int u = 0; u < FP_PREP_COLS; u++) {
      int q[FP_PREP_ROW];
#pragma unroll
      for (int j = 0; j < FP_PREP_ROW; j++) q[j] = j < R.deg[u] ? R.q[u][j] : -1;
      mark_n(q);
      for (int j = FP_PREP_ROW; j < R.deg[u]; j++) {
        const int q1[1] = {(int)M.pent[R.e0[u] + j]};
        mark_n(q1);
      }
    }
  }
  if (ballot64(bad1)) {
    sym_drop(M, t, FP_SITE_SYM_LOOKUP);
    return;
  }
  wave_fence();
  // read the bitmap back: positions in increasing order, and the rank
  // prefix of every word.  A lane finds the ancestor of its word's first
  // set bit, then steps forward through the ancestors as its bits rise.
  int nbd = 0;
  for (int w0 = 0; w0 < BW; w0 += 64) {
    const int w = w0 + lane;
    uint32_t x = w < BW ? bm[w] : 0u;
    const int c = popc32(x);
    const int inc = wave_incl_scan(c);
    int o = nbd + inc - c;
    if (w < BW) pre[w] = o;
    if (x) {
      const int b1 = w * 32 + __ffs(x) - 1;
      int lo = 0, hi = na - 1, f = 0;
      while (lo <= hi) {  // the ancestor whose bit range holds b1
        const int mid = (lo + hi) >> 1;
        if (anc[3 * mid + 2] <= b1) {
          f = mid;
          lo = mid + 1;
        } else {
          hi = mid - 1;
        }
      }
      int fbeg = anc[3 * f], foff = anc[3 * f + 2];
      int nxt = f + 1 < na ? anc[3 * (f + 1) + 2] : INT_MAX;
      while (x) {
        const int b = w * 32 + __ffs(x) - 1;
        x &= x - 1;
        while (b >= nxt) {
          f++;
          fbeg = anc[3 * f];
          foff = nxt;
          nxt = f + 1 < na ? anc[3 * (f + 1) + 2] : INT_MAX;
        }
        if (o < np2) V.bd[o] = fbeg + (b - foff);
        o++;
      }
    }
    nbd += wave_bcast(inc, 63);
  }
  if (nbd > np2) {
    sym_drop(M, t, FP_SITE_SYM_LOOKUP);
    return;
  }
  wave_fence();
  const int F = m + nbd;
  const int FW = (F + 31) >> 5;
  // 2. forward rows in F indices
  {
    bool bad = false;
    int run = 0;
    for (int k1 = 0; k1 < m; k1 += 64 * FP_PREP_COLS) {
      PrepRows R;
      prep_rows(M, b0, m, k1, R);
#pragma unroll
      for (int u = 0; u < FP_PREP_COLS; u++) {
        if (k1 + 64 * u >= m) break;
        const int k = k1 + 64 * u + lane;
        const int p = b0 + k;
        int cnt = 0;
        prep_each(M, R, u, [&](int q) { cnt += q > p; });
        const int inc = wave_incl_scan(cnt);
        int o = run + inc - cnt;
        // F indices of the first FP_PREP_ROW entries, looked up together
        int q[FP_PREP_ROW], fi[FP_PREP_ROW];
#pragma unroll
        for (int j = 0; j < FP_PREP_ROW; j++) q[j] = j < R.deg[u] && k < m ? R.q[u][j] : -1;
        findex_n(q, fi);
        if (k < m) {
          V.optr[k] = o;
#pragma unroll
          for (int j = 0; j < FP_PREP_ROW; j++) {
            if (q[j] > p) {
              const bool ok = fi[j] > k && fi[j] < F;
              bad |= !ok;
              V.oent[o++] = ok ? fi[j] : k + 1;
            }
          }
        }
        // entries past FP_PREP_ROW one at a time (findex takes the whole
        // wave, so the loop runs to the longest row of the wave)
        const int dl = k < m ? R.deg[u] : 0;
        const int dmax = (int)wave_max_u32((uint32_t)dl);
        for (int j = FP_PREP_ROW; j < dmax; j++) {
          const int qj = j < dl ? (int)M.pent[R.e0[u] + j] : -1;
          const int f = findex(qj);
          if (qj > p) {
            const bool ok = f > k && f < F;
            bad |= !ok;
            V.oent[o++] = ok ? f : k + 1;
          }
        }
        run += wave_bcast(inc, 63);
      }
    }
    if (lane == 0) V.optr[m] = run;
    if (ballot64(bad) || run != in.nfw) {
      sym_drop(M, t, FP_SITE_SYM_LOOKUP);
      return;
    }
  }
  for (int k = lane; k < m; k += 64) V.head[k] = -1;
  wave_fence();
  // 3. incoming elements: one row each, gathered in rbuf and stored whole,
  // queued on their least position
  int npass = 0, e = 0;
  bool bad3 = false;
  for (int c = 0; c < 2; c++) {
    int off = in.cst[c];
    const int end = in.cst[c] + in.cin[c];
    while (off < end) {
      const int len = uni(src[off]);
      const int r = m + e;
      for (int w = lane; w < FW; w += 64) rbuf[w] = 0u;
      wave_fence();
      uint32_t fmin = 0xFFFFFFFFu;
      for (int i0 = 0; i0 < len; i0 += 64 * FP_PREP_COLS) {
        int q[FP_PREP_COLS], f[FP_PREP_COLS];
        record_round(off, len, i0, q);
        findex_n(q, f);
#pragma unroll
        for (int u = 0; u < FP_PREP_COLS; u++) {
          if (i0 + lane + 64 * u >= len) continue;
          if (f[u] < 0) {
            bad3 = true;
          } else {
            atomicOr(&rbuf[f[u] >> 5], 1u << (f[u] & 31));
            fmin = min(fmin, (uint32_t)f[u]);
          }
        }
      }
      fmin = wave_min_u32(fmin);
      wave_fence();
      const gptr<uint32_t> row = V.rows + (long long)r * in.stride;
      for (int w = lane; w < FW; w += 64) row[w] = rbuf[w];
      if (fmin != 0xFFFFFFFFu) {
        if ((int)fmin < m) {
          if (lane == 0) {
            V.next[r] = V.head[fmin];
            V.head[fmin] = r;
          }
        } else {
          if (lane == 0) V.outl[npass] = r;
          npass++;
        }
      }
      wave_fence();
      e++;
      off += 1 + len;
    }
  }
  if (ballot64(bad3) || e != in.nce) {
    sym_drop(M, t, FP_SITE_SYM_LOOKUP);
    return;
  }
  if (lane == 0) {
    V.hdr[SH_M] = m;
    V.hdr[SH_NBD] = nbd;
    V.hdr[SH_NFW] = in.nfw;
    V.hdr[SH_FW] = FW;
    V.hdr[SH_ROWS] = in.rows;
    V.hdr[SH_NCE] = in.nce;
    V.hdr[SH_NP2] = np2;
    V.hdr[SH_STRIDE] = in.stride;
    V.hdr[SH_NOUT] = npass;
    V.hdr[SH_OK] = 1;
    M.sdesc[t] = (long long)(base - M.pool);
  }
}

// lds / lwords: this wave's LDS slice, which holds the ancestor table and,
// when they fit, the later-position bitmap, its rank prefix and a row buffer
__device__ __forceinline__ void sym_prep(const FpMesh& M, int t, int d, int* lds, int lwords) {
  gptr<FpCtl> C = M.ctl;
  const int m = uni(M.nsize[t]);
  const int b0 = uni(M.nbegin[t]), e0 = b0 + m;
  const int nn = uni(C->nn);
  gptr<const int> src = M.arena[(d + 1) & 1];
  // child element records: [len, pos...] ...
  int cst[2] = {0, 0}, cin[2] = {0, 0}, crec[2] = {0, 0};
  for (int c = 0; c < 2; c++) {
    const int ch = 2 * t + 1 + c;
    if (ch < nn) {
      cst[c] = uni(M.eoff[3 * ch]);
      cin[c] = uni(M.eoff[3 * ch + 1]);
      crec[c] = uni(M.eoff[3 * ch + 2]);
    }
  }
  const int nce = crec[0] + crec[1];
  // inputs in range: t's positions hold vertices placed there by the local
  // orders, child records hold positions of t or later.  The vertex check
  // shares its rounds with the count of forward entries and later
  // positions: four columns per lane and round, every load of a round
  // issued before the first use.
  int nfw = 0, nanc = 0;
  {
    bool bad = b0 < 0 || m < 0 || e0 > M.n;
    if (!bad) {
      for (int k0 = 0; k0 < m; k0 += 64 * FP_PREP_COLS) {
        int v[FP_PREP_COLS];
#pragma unroll
        for (int u = 0; u < FP_PREP_COLS; u++) {
          const int k = k0 + lane_id() + 64 * u;
          v[u] = k < m ? M.vperm[b0 + k] : 0;
        }
        PrepRows R;
        prep_rows(M, b0, m, k0, R);
        int w[FP_PREP_COLS];
#pragma unroll
        for (int u = 0; u < FP_PREP_COLS; u++) {
          const int k = k0 + lane_id() + 64 * u;
          const bool in = k < m && (unsigned)v[u] < (unsigned)M.n;
          bad |= k < m && !in;
          w[u] = in ? M.viperm[v[u]] : 0;
        }
#pragma unroll
        for (int u = 0; u < FP_PREP_COLS; u++) {
          const int p = b0 + k0 + lane_id() + 64 * u;
          prep_each(M, R, u, [&](int q) {
            if (q > p) {
              nfw++;
              nanc += (q >= e0);
            }
          });
        }
#pragma unroll
        for (int u = 0; u < FP_PREP_COLS; u++) {
          const int k = k0 + lane_id() + 64 * u;
          bad |= k < m && w[u] != b0 + k;
        }
      }
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
        const int len = uni(src[off]);
        if (len < 0 || off + 1 + len > end) {
          bad = true;
          break;
        }
        for (int i0 = 0; i0 < len; i0 += 256) {
          int q[4];
#pragma unroll
          for (int u = 0; u < 4; u++) {
            const int i = i0 + lane_id() + 64 * u;
            q[u] = i < len ? src[off + 1 + i] : b0;
          }
#pragma unroll
          for (int u = 0; u < 4; u++) bad |= q[u] < b0 || q[u] >= M.n;
        }
        off += 1 + len;
        nrec++;
      }
      if (nrec != crec[c]) bad = true;
      bad = ballot64(bad) != 0;
    }
    if (bad) {
      sym_drop(M, t, site);
      return;
    }
  }
  nfw = wave_sum_i32(nfw);
  nanc = wave_sum_i32(nanc);
  const int ncand = nanc + (cin[0] + cin[1] - nce);
  if (ncand < 0 || ncand > (1 << 29)) {
    sym_drop(M, t, FP_SITE_SYM_RECORD);
    return;
  }
  // Every later position lies in an ancestor of t (the separator property),
  // and t's ancestors, nearest first, occupy increasing positions.  Marking
  // the positions in a bitmap over the ancestors' ranges, concatenated in
  // that order, and reading the bitmap back gives them sorted and unique.
  // lane i holds the i-th ancestor (nearest first): its size and start,
  // read at once; the depth of t bounds their count
  int dep = 0;
  for (int a = t; a > 0; a = (a - 1) >> 1) dep++;
  int asz = 0, abeg = 0;
  if (lane_id() < dep) {
    const int a = ((t + 1) >> (lane_id() + 1)) - 1;
    asz = M.nsize[a];
    abeg = M.nbegin[a];
  }
  const uint64_t nzm = ballot64(lane_id() < dep && asz > 0);
  const int na = popc64(nzm);
  const long long B = wave_sum_i64(lane_id() < dep && asz > 0 ? (long long)asz : 0ll);
  if (dep > 64 || na > 32 || B > (1 << 29)) {
    sym_drop(M, t, FP_SITE_SYM_RECORD);
    return;
  }
  const int cap = (int)min((long long)max(ncand, 1), max(B, 1ll));  // later positions at most
  const int BW = (int)((B + 31) >> 5);
  const int stride = (m + cap + 31) >> 5;
  const int rows = m + nce;
  const long long words = sym_words(m, cap, nfw, rows, stride);
  // the bitmap, its rank prefix and a row buffer: in the LDS slice after
  // the ancestor table when they fit, else in the pool after the scratch
  const bool lmode = 96 + 2ll * BW + stride <= lwords;
  const long long extra = lmode ? 0 : 2ll * BW + stride;
  gptr<unsigned> base = pool_alloc(M, (unsigned long long)(words + extra + 96));
  if (!base) {  // pool_alloc raised the error
    sym_drop(M, t, 0);
    return;
  }
  const int np2 = cap;  // capacity of the later-position list
  const SymView V = sym_view(base, m, np2, nfw, rows);
  int* anc = lds;  // per ancestor: begin, size, bit offset (at most 32 ancestors)
  {
    // the non-empty ancestors in order, their bit offsets by a prefix sum
    const bool ne = lane_id() < dep && asz > 0;
    const int i = popc64(nzm & lanemask_lt());
    const int inc = wave_incl_scan(ne ? asz : 0);
    if (ne) {
      anc[3 * i] = abeg;
      anc[3 * i + 1] = asz;
      anc[3 * i + 2] = inc - asz;
    }
  }
  wave_fence();
  const PrepIn in{m, b0, e0, na, BW, np2, nfw, nanc, nce, rows, stride, {cst[0], cst[1]}, {cin[0], cin[1]}};
  if (lmode) {
    uint32_t* l = (uint32_t*)(lds + 96);
    sym_prep_tail(M, t, V, base, src, anc, in, l, l + BW, l + 2 * BW);
  } else {
    const gptr<uint32_t> g = base.as<uint32_t>() + words;
    sym_prep_tail(M, t, V, base, src, anc, in, g, g + BW, g + 2 * BW);
  }
}

// scratch of node t after prep, or false if it has none
__device__ __forceinline__ bool sym_load(const FpMesh& M, int t, SymView* V, int* h) {
  const long long so = uni(M.sdesc[t]);
  if (so < 0 || (unsigned long long)so >= M.pool_words) return false;
  gptr<unsigned> base = M.pool + so;
  for (int i = 0; i < SH_WORDS; i++) h[i] = uni(base.as<int>()[i]);
  if (h[SH_OK] != 1) return false;
  *V = sym_view(base, h[SH_M], h[SH_NP2], h[SH_NFW], h[SH_ROWS]);
  return true;
}

// ---------------------------------------------------------------- elim
// The columns of a node are a sequential chain of dependent steps, so their
// latency decides the time of the top tree levels.  A step builds the
// column's row, finds its least entry (the parent, found by ballot) to queue
// the row on, and counts its entries (one DPP reduction).  The queue links
// are copied into the wave's LDS slice when they fit (kLds), and every lane
// keeps its words of the last column in registers: the next column is most
// often that column's parent, and then its row needs no memory read.
#define FP_SYM_REGW 4  // words per lane kept in registers (rows up to 256 words)
#ifndef FP_SYM_ENTW
#define FP_SYM_ENTW 4  // forward entries per lane in the register window
#endif

// entry q * 64 + l of the window, q and l wave-uniform: one readlane per
// register and a scalar select, so the window is never indexed dynamically
// (which would move it to scratch memory)
__device__ __forceinline__ int sym_ent(const int (&a)[FP_SYM_ENTW], int q, int l) {
  int r = __builtin_amdgcn_readlane(a[0], l);
#pragma unroll
  for (int i = 1; i < FP_SYM_ENTW; i++) {
    const int v = __builtin_amdgcn_readlane(a[i], l);
    r = q == i ? v : r;
  }
  return r;
}

// the row of column k, word w: queued rows OR forward entries, bits > k
template <class NP, class OP>
__device__ __forceinline__ uint32_t sym_word(const SymView& V, NP next, OP oent,
                                             int k, int w, int q0, int r0, int r1, int rows,
                                             int stride, bool use_prev, uint32_t prev, bool* bad) {
  uint32_t x = 0u;
  const int kw = k >> 5;
  if (w < kw) return 0u;
  int j = q0, steps = 0;
  while (j >= 0 && j < rows && steps < rows) {
    x |= (use_prev && j == k - 1) ? prev : V.rows[(long long)j * stride + w];
    j = next[j];
    steps++;
  }
  *bad |= j >= 0;  // a queue that leaves the rows or does not end
  for (int e = r0; e < r1; e++) {
    const int f = oent[e];
    if ((f >> 5) == w) x |= 1u << (f & 31);
  }
  if (w == kw) x &= (k & 31) == 31 ? 0u : (0xFFFFFFFFu << ((k & 31) + 1));
  return x;
}

// Rows wider than the register window (F > 64 * 32 * FP_SYM_REGW): every row
// goes through memory.
template <class IP>
__device__ __forceinline__ void sym_elim_wide(const FpMesh& M, int t, const SymView& V, const int* h,
                                              IP head, IP next, gptr<int> optr, gptr<int> oent,
                                              int s0, int nout) {
  const int m = h[SH_M], nbd = h[SH_NBD], FW = h[SH_FW], rows = h[SH_ROWS];
  const int stride = h[SH_STRIDE];
  const int F = m + nbd;
  const bool regs = FW <= 64 * FP_SYM_REGW;
  const int b0 = M.nbegin[t];
  uint32_t prev[FP_SYM_REGW];
#pragma unroll
  for (int i = 0; i < FP_SYM_REGW; i++) prev[i] = 0u;
  int my_cc = 0, my_par = -1;  // column count and parent of column k with k % 64 == lane
  for (int k = s0; k < m; k++) {
    const int r0 = optr[k], r1 = optr[k + 1];
    const int q0 = head[k];
    gptr<uint32_t> rk = V.rows + (long long)k * stride;
    bool bad = false;
    uint32_t first = 0xFFFFFFFFu;
    int cnt = 0;
#pragma unroll
    for (int i = 0; i < FP_SYM_REGW; i++) {
      if (i * 64 < FW) {
        const int w = lane_id() + 64 * i;
        uint32_t x = 0u;
        if (w < FW) {
          x = sym_word(V, next, oent, k, w, q0, r0, r1, rows, stride, regs, prev[i], &bad);
          if (!regs) rk[w] = x;
        }
        prev[i] = x;
        cnt += popc32(x);
        // least set bit: lowest word with a bit, found by ballot
        const uint64_t b = ballot64(x != 0u);
        if (first == 0xFFFFFFFFu && b) {
          const int l = __builtin_ctzll(b);
          const uint32_t xv = wave_bcast_u32(x, l);
          first = (uint32_t)((l + 64 * i) * 32 + __ffs(xv) - 1);
        }
      }
    }
    if (!regs) {  // rows wider than the register window: the rest from memory
      uint32_t f2 = 0xFFFFFFFFu;
      for (int w = lane_id() + 64 * FP_SYM_REGW; w < FW; w += 64) {
        const uint32_t x = sym_word(V, next, oent, k, w, q0, r0, r1, rows, stride, false, 0u, &bad);
        rk[w] = x;
        cnt += popc32(x);
        if (x && f2 == 0xFFFFFFFFu) f2 = (uint32_t)(w * 32 + __ffs(x) - 1);
      }
      f2 = wave_min_u32(f2);
      if (first == 0xFFFFFFFFu) first = f2;
    }
    if (ballot64(bad) || (first != 0xFFFFFFFFu && (first <= (uint32_t)k || first >= (uint32_t)F))) {
      if (lane_id() == 0) {
        fp_fail(M.ctl, FP_E_INTERNAL, FP_SITE_SYM_LIVE, t);
        V.hdr[SH_OK] = 0;
      }
      return;
    }
    // The row is read again only by its parent: from registers when that is
    // the next column, else from memory (a later column, or the parent node
    // for a row that leaves t).  Skipping the store keeps a chain of columns
    // free of global stores, so no wait for a later load has to drain them.
    if (regs && first != 0xFFFFFFFFu && !(first == (uint32_t)(k + 1) && (int)first < m)) {
#pragma unroll
      for (int i = 0; i < FP_SYM_REGW; i++) {
        const int w = lane_id() + 64 * i;
        if (i * 64 < FW && w < FW) rk[w] = prev[i];
      }
    }
    cnt = wave_sum_i32(cnt);
    int par = -1;
    if (first != 0xFFFFFFFFu) par = (int)first < m ? b0 + (int)first : V.bd[first - m];
    if (lane_id() == 0 && first != 0xFFFFFFFFu) {
      if ((int)first < m) {
        next[k] = head[first];
        head[first] = k;
      } else {
        V.outl[nout] = k;
      }
    }
    if (first != 0xFFFFFFFFu && (int)first >= m) nout++;
    // counts and parents leave in one 64-column store
    if (lane_id() == (k & 63)) {
      my_cc = 1 + cnt;
      my_par = par;
    }
    if ((k & 63) == 63 || k == m - 1) {
      const int c = (k & ~63) + lane_id();
      if (c >= s0 && c <= k) {
        M.vcc[b0 + c] = my_cc;
        M.vpar[b0 + c] = my_par;
      }
    }
    wave_fence();  // queue links and outl reach every lane of the wave
  }
  if (lane_id() == 0) V.hdr[SH_NOUT] = nout;
}

// ---------------------------------------------------------------- chain
// Most separator nodes eliminate as chains: column k's parent is k + 1.
// Take a run of columns s.. that starts with nothing carried in (s = 0, or
// column s - 1 has another parent).  While the run is a chain, column k's
// structure is every index b > k that some column j in s..k holds among
// its forward entries or queued rows (a row joins at the column it is
// queued on).  With intro(b) the least such column, the run goes on through
// column k + 1 exactly when intro(k + 1) <= k (by induction over k: column
// k's parent is its least index above k), so the run ends at the first
// column e whose test fails, or at m - 1.  The count of column k in s..e is
// one plus the number of b with intro(b) <= k < b: a difference array and a
// prefix sum, all lanes at once.  Column e's structure, the b > e with
// intro(b) <= e, goes to its parent as a queued row (or leaves t), and the
// next run starts at e + 1.  A node with many breaks hands the columns left
// after FP_CHAIN_RUNS runs to the sequential walk.
#define FP_CHAIN_MIN 32
#ifndef FP_CHAIN_RUNS
#define FP_CHAIN_RUNS 8
#endif
// intro (F words) and diff (m words): the wave's LDS slice or global scratch.
// Returns the first column left for the sequential walk (m when done), or
// -1 after raising an error; *nout receives the count of rows leaving t.
template <class SP>
__device__ __forceinline__ int sym_elim_chain(const FpMesh& M, int t, const SymView& V,
                                              const int* h, SP intro, SP diff, int* nout_out) {
  const int m = h[SH_M], nbd = h[SH_NBD], rows = h[SH_ROWS], FW = h[SH_FW];
  const int stride = h[SH_STRIDE];
  const int F = m + nbd;
  const gptr<const int> optr = V.optr, oent = V.oent;
  const gptr<int> head = V.head, next = V.next;
  const int lane = lane_id();
  const int b0 = uni(M.nbegin[t]);
  int nout = h[SH_NOUT];
  int s = 0;
  for (int run_no = 0; run_no < FP_CHAIN_RUNS && s < m; run_no++) {
    for (int b = s + lane; b < F; b += 64) intro[b] = 0x7FFFFFFF;
    wave_fence();
    // forward entries of the columns s..
    bool bad = false;
    for (int k0 = s; k0 < m; k0 += 64 * FP_PREP_COLS) {
      PrepRows R;
      csr_rows(optr, oent, 0, m, k0, R);
#pragma unroll
      for (int u = 0; u < FP_PREP_COLS; u++) {
        const int k = k0 + lane + 64 * u;
        csr_each(oent, R, u, [&](int f) {
          if (f <= k || f >= F)
            bad = true;
          else
            atomicMin(&intro[f], k);
        });
      }
    }
    // Queued rows are few but wide (a child's last row holds most of its
    // structure), so each is taken by the whole wave.  The columns with a
    // queue are listed in diff first (cleared afterwards).
    int nq = 0;
    for (int k0 = s; k0 < m; k0 += 64 * FP_PREP_COLS) {
      int hj[FP_PREP_COLS];
#pragma unroll
      for (int u = 0; u < FP_PREP_COLS; u++) {
        const int k = k0 + lane + 64 * u;
        hj[u] = k < m ? head[k] : -1;
      }
#pragma unroll
      for (int u = 0; u < FP_PREP_COLS; u++) {
        const uint64_t bal = ballot64(hj[u] >= 0);
        if (hj[u] >= 0) diff[nq + popc64(bal & lanemask_lt())] = k0 + lane + 64 * u;
        nq += popc64(bal);
      }
    }
    wave_fence();
    for (int q = 0; q < nq; q++) {
      const int k = uni(diff[q]);
      const int kw = k >> 5;
      const uint32_t kmask = (k & 31) == 31 ? 0u : (0xFFFFFFFFu << ((k & 31) + 1));
      int j = uni(head[k]), steps = 0;
      while (j >= 0 && j < rows && steps < rows) {
        const gptr<const uint32_t> rj = V.rows + (long long)j * stride;
        for (int w = kw + lane; w < FW; w += 64) {
          uint32_t x = rj[w];
          if (w == kw) x &= kmask;
          while (x) {
            const int b = w * 32 + __ffs(x) - 1;
            x &= x - 1;
            if (b < F) atomicMin(&intro[b], k);
          }
        }
        j = uni(next[j]);
        steps++;
      }
      bad |= j >= 0;  // a queue that leaves the rows or does not end
    }
    wave_fence();
    for (int k = lane; k < m; k += 64) diff[k] = 0;
    if (ballot64(bad)) {
      if (lane == 0) {
        fp_fail(M.ctl, FP_E_INTERNAL, FP_SITE_SYM_LIVE, t);
        V.hdr[SH_OK] = 0;
      }
      return -1;
    }
    wave_fence();
    // the run's last column: the first k >= s with intro(k + 1) > k
    int e = m - 1;
    for (int k0 = s; k0 + 1 < m; k0 += 64) {
      const int k = k0 + lane;
      const uint64_t br = ballot64(k + 1 < m && intro[k + 1] > k);
      if (br) {
        e = k0 + __builtin_ctzll(br);
        break;
      }
    }
    // every b with intro(b) in s..e holds on the columns intro(b) .. b - 1,
    // or up to e; the least such b above e is the parent of e.  The +1 side
    // aggregates runs of equal intro over consecutive lanes: the bits of one
    // queued row share their intro, and one atomic per run replaces up to 64
    // on the same LDS word.
    uint32_t pl = 0xFFFFFFFFu;
    for (int g = s; g < F; g += 64) {
      const int b = g + lane;
      const int i = b < F ? intro[b] : 0x7FFFFFFF;
      const bool v = i <= e;  // intro(b) >= s for every b marked in this run
      if (v && b <= e) atomicAdd(&diff[b], -1);
      if (v && b > e) pl = min(pl, (uint32_t)b);
      const int ip = __shfl_up(i, 1, 64);
      const uint64_t heads = ballot64(lane == 0 || i != ip);
      if (v && ((heads >> lane) & 1)) {
        const uint64_t after = lane == 63 ? 0ull : heads >> (lane + 1);
        atomicAdd(&diff[i], after ? __builtin_ctzll(after) + 1 : 64 - lane);
      }
    }
    pl = wave_min_u32(pl);
    wave_fence();
    const int pe = pl == 0xFFFFFFFFu ? -1 : (int)pl < m ? b0 + (int)pl : uni(V.bd[pl - m]);
    int acc = 0;
    for (int k0 = s; k0 <= e; k0 += 64) {
      const int k = k0 + lane;
      const int c = k <= e ? (int)diff[k] : 0;
      const int inc = wave_incl_scan(c);
      if (k <= e) {
        M.vcc[b0 + k] = 1 + acc + inc;
        M.vpar[b0 + k] = k < e ? b0 + k + 1 : pe;
      }
      acc += wave_bcast(inc, 63);
    }
    if (pl != 0xFFFFFFFFu) {
      // the row of e, 64 bits at a time from one ballot: words 2g, 2g + 1
      const gptr<uint32_t> rl = V.rows + (long long)e * stride;
      const int g0 = (e + 1) >> 6;
      for (int w = lane; w < 2 * g0 && w < FW; w += 64) rl[w] = 0u;
      for (int g = g0; 64 * g < F; g++) {
        const int b = 64 * g + lane;
        const uint64_t bal = ballot64(b > e && b < F && intro[b] <= e);
        const int w = 2 * g + lane;
        if (lane < 2 && w < FW) rl[w] = lane == 0 ? (uint32_t)bal : (uint32_t)(bal >> 32);
      }
      if ((int)pl < m) {
        if (lane == 0) {  // queued on its parent, a column of a later run
          next[e] = head[pl];
          head[pl] = e;
        }
      } else {
        if (lane == 0) V.outl[nout] = e;
        nout++;
      }
    }
    // the queue links and the row reach every lane (the next run, or the
    // sequential walk, reads them)
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
    s = e + 1;
  }
  *nout_out = nout;
  if (lane == 0) V.hdr[SH_NOUT] = nout;
  return s;
}

// The sequential walk over a node's columns, rows of up to 64 NW words
// held NW words per lane.
// With the links in LDS (IP a plain pointer), rb is an LDS buffer of FW
// zero words that gathers each column's forward entries.
template <int NW, class IP>
__device__ __forceinline__ void sym_elim_cols(const FpMesh& M, int t, const SymView& V,
                                              const int* h, IP head, IP next,
                                              const gptr<int> optr, const gptr<int> oent,
                                              uint32_t* rb, int s0, int nout) {
  constexpr bool kRb = std::is_same<IP, int*>::value;
  const int m = h[SH_M], nbd = h[SH_NBD], FW = h[SH_FW], rows = h[SH_ROWS];
  const int stride = h[SH_STRIDE];
  const int F = m + nbd;
  // Columns go in blocks of 64.  A block's queue heads, row pointers and
  // forward entries are read once into registers (lane i holds column k0+i),
  // and a column whose parent is the next column hands its row over in
  // registers instead of a queue: a chain of such columns, the common case
  // in separators, runs without any LDS or global round trip.
  const int lane = lane_id();
  const int b0 = M.nbegin[t];
  uint32_t x[NW];  // the row being built, word lane + 64 i in x[i]
#pragma unroll
  for (int i = 0; i < NW; i++) x[i] = 0u;
  int cnt = 0;
  bool chain = false;          // the previous column's parent is this column
  int my_cc = 0, my_par = -1;  // results of column k0 + lane, stored per block
  uint32_t pf[NW];             // row pfj, loaded one column ahead
  int pfj = -1;
#pragma unroll
  for (int i = 0; i < NW; i++) pf[i] = 0u;
  for (int k0 = s0; k0 < m; k0 += 64) {
    const int kn = min(64, m - k0);
    int hreg = lane < kn ? head[k0 + lane] : -1;
    const int oreg = lane < kn ? optr[k0 + lane] : 0;
    const int e1 = uni(optr[k0 + kn]);
    // a window of the block's forward entries in registers: entries wb ..
    // wb + 64 FP_SYM_ENTW - 1, moved up to a column's first entry when that
    // column's entries run past it
    int wb = uni(optr[k0]);
    int ent[FP_SYM_ENTW];
#pragma unroll
    for (int q = 0; q < FP_SYM_ENTW; q++) {
      const int e = wb + lane + 64 * q;
      ent[q] = e < e1 ? oent[e] : 0;
    }
    vm_wait();
    for (int kk = 0; kk < kn; kk++) {
      const int k = k0 + kk;
      const int r0 = wave_bcast(oreg, kk);
      const int r1 = kk + 1 < kn ? wave_bcast(oreg, kk + 1) : e1;
      // The carried row: after a chain step the previous column's row (its
      // entries > k-1, k among them), else empty.  cnt counts its entries
      // > k, and every bit added below is counted where it is set, so the
      // row is never counted over again.
      if (chain) {
        cnt -= 1;  // k, the previous column's parent, is not an entry of k
      } else {
#pragma unroll
        for (int i = 0; i < NW; i++) x[i] = 0u;
        cnt = 0;
      }
      const int kw = k >> 5;
      const uint32_t kmask = (k & 31) == 31 ? 0u : (0xFFFFFFFFu << ((k & 31) + 1));
      // rows queued on k (columns other than k-1, and rows from below); the
      // first of them was loaded into pf at the previous column
      bool bad = false;
      int add = 0;  // bits set in x below, summed over the wave once
      int j = wave_bcast(hreg, kk), steps = 0;
      if (j >= 0 && j == pfj) {
#pragma unroll
        for (int i = 0; i < NW; i++) {
          const int w = lane + 64 * i;
          uint32_t y = w >= kw && w < FW ? pf[i] : 0u;
          if (w == kw) y &= kmask;
          add += popc32(y & ~x[i]);
          x[i] |= y;
        }
        j = uni(next[j]);
        steps = 1;
      }
      // the first row queued on k + 1 (that queue is complete: this column
      // hands its own row to k + 1 in registers), loaded while k goes on
      {
        const int jn = kk + 1 < kn ? wave_bcast(hreg, kk + 1) : (k + 1 < m ? uni(head[k + 1]) : -1);
        pfj = -1;
        if (jn >= 0 && jn < rows) {
          pfj = jn;
          const gptr<const uint32_t> rn = V.rows + (long long)jn * stride;
#pragma unroll
          for (int i = 0; i < NW; i++) pf[i] = rn[min(lane + 64 * i, FW - 1)];
        }
      }
      while (j >= 0 && j < rows && steps < rows) {
        const gptr<const uint32_t> rj = V.rows + (long long)j * stride;
#pragma unroll
        for (int i = 0; i < NW; i++) {
          const int w = lane + 64 * i;
          if (i * 64 < FW && w < FW && w >= kw) {
            uint32_t y = rj[w];
            if (w == kw) y &= kmask;
            add += popc32(y & ~x[i]);
            x[i] |= y;
          }
        }
        j = uni(next[j]);
        steps++;
      }
      bad = j >= 0;  // a queue that leaves the rows or does not end
      // forward entries of column k: a bit test in the owning lane
      if (r1 > wb + 64 * FP_SYM_ENTW && r1 - r0 <= 64 * FP_SYM_ENTW) {
        wb = r0;
#pragma unroll
        for (int q = 0; q < FP_SYM_ENTW; q++) {
          const int e = wb + lane + 64 * q;
          ent[q] = e < e1 ? oent[e] : 0;
        }
        vm_wait();
      }
      const bool ereg = r1 <= wb + 64 * FP_SYM_ENTW;
      uint32_t fm[NW];
#pragma unroll
      for (int i = 0; i < NW; i++) fm[i] = 0u;
      if (kRb) {
        // the lanes that hold the column's entries set their bits in the
        // LDS row buffer; each lane then takes (and clears) its own words
        if (r1 > r0) {
          if (ereg) {
            const int p0 = r0 - wb, p1 = r1 - wb;
#pragma unroll
            for (int q = 0; q < FP_SYM_ENTW; q++) {
              if (64 * q < p1 && 64 * q + 64 > p0) {
                const int p = lane + 64 * q;
                const int f = ent[q];
                if (p >= p0 && p < p1) {
                  bad |= f <= k || f >= F;
                  if (f > k && f < F) atomicOr(&rb[f >> 5], 1u << (f & 31));
                }
              }
            }
          } else {
            for (int e = r0 + lane; e < r1; e += 64) {
              const int f = oent[e];
              bad |= f <= k || f >= F;
              if (f > k && f < F) atomicOr(&rb[f >> 5], 1u << (f & 31));
            }
          }
          wave_fence();
#pragma unroll
          for (int i = 0; i < NW; i++) {
            const int w = lane + 64 * i;
            if (i * 64 < FW && w < FW) {
              fm[i] = rb[w];
              rb[w] = 0u;
            }
          }
        }
      } else {
        // every entry is broadcast and each lane keeps the bits of its own
        // words: straight-line vector work
        for (int e = r0; e < r1; e++) {
          int f;
          if (ereg) {
            const int q = (e - wb) >> 6, l = (e - wb) & 63;
            f = sym_ent(ent, q, l);
          } else {
            f = uni(oent[e]);
          }
          bad |= f <= k || f >= F;
          const int fw = f >> 5;
          const uint32_t bit = 1u << (f & 31);
#pragma unroll
          for (int i = 0; i < NW; i++) fm[i] |= lane + 64 * i == fw ? bit : 0u;
        }
      }
#pragma unroll
      for (int i = 0; i < NW; i++) {
        add += popc32(fm[i] & ~x[i]);
        x[i] |= fm[i];
      }
      cnt += wave_sum_i32(add);
      // keep entries > k; the row is stored at once (its parent, unless that
      // is the next column, reads it back from memory), so the store is done
      // by the time a later column waits for its loads
      const gptr<uint32_t> rk = V.rows + (long long)k * stride;
#pragma unroll
      for (int i = 0; i < NW; i++) {
        const int w = lane + 64 * i;
        if (w < kw || w >= FW) x[i] = 0u;
        if (w == kw) x[i] &= kmask;
        if (i * 64 < FW && w < FW) rk[w] = x[i];
      }
      // least entry by ballot
      uint32_t first = 0xFFFFFFFFu;
#pragma unroll
      for (int i = 0; i < NW; i++) {
        if (i * 64 < FW) {
          const uint64_t b = ballot64(x[i] != 0u);
          if (first == 0xFFFFFFFFu && b) {
            const int l = __builtin_ctzll(b);
            first = (uint32_t)((l + 64 * i) * 32 + __ffs(wave_bcast_u32(x[i], l)) - 1);
          }
        }
      }
      if (ballot64(bad) || (first != 0xFFFFFFFFu && (first <= (uint32_t)k || first >= (uint32_t)F))) {
        if (lane == 0) {
          fp_fail(M.ctl, FP_E_INTERNAL, FP_SITE_SYM_LIVE, t);
          V.hdr[SH_OK] = 0;
        }
        return;
      }
      const bool to_next = first == (uint32_t)(k + 1) && (int)first < m;
      int par = -1;
      if (first != 0xFFFFFFFFu) par = (int)first < m ? b0 + (int)first : uni(V.bd[first - m]);
      if (first != 0xFFFFFFFFu && !to_next) {
        if ((int)first < m) {
          // queue k on its parent column, in LDS and in this block's registers
          const int hf = (int)first < k0 + kn ? wave_bcast(hreg, (int)first - k0) : 0;
          if (lane == 0) {
            next[k] = (int)first < k0 + kn ? hf : head[first];
            head[first] = k;
          }
          if (lane == (int)first - k0) hreg = k;
        } else {
          if (lane == 0) V.outl[nout] = k;
          nout++;
        }
      }
      chain = to_next;
      if (lane == kk) {
        my_cc = 1 + cnt;
        my_par = par;
      }
      wave_fence();  // queue links and outl reach every lane of the wave
    }
    if (lane < kn) {  // counts and parents leave in one store per block
      M.vcc[b0 + k0 + lane] = my_cc;
      M.vpar[b0 + k0 + lane] = my_par;
    }
  }
  if (lane == 0) V.hdr[SH_NOUT] = nout;
}

template <bool kLds>
__device__ __forceinline__ void sym_elim_run(const FpMesh& M, int t, const SymView& V,
                                             const int* h, int* lds, long long lds_words) {
  const int m = h[SH_M], nbd = h[SH_NBD], FW = h[SH_FW], rows = h[SH_ROWS];
  const int F = m + nbd;
  // chain runs first (section above): their arrays in the LDS slice when
  // they fit, else in pool scratch; the sequential walk takes the columns
  // they leave
  int s0 = 0, nout = h[SH_NOUT];
  if (m >= FP_CHAIN_MIN && rows > m) {  // a node with no incoming rows is a leaf
    if (kLds && (long long)F + m <= lds_words) {
      s0 = sym_elim_chain(M, t, V, h, lds, lds + F, &nout);
    } else {
      const gptr<unsigned> sc = pool_alloc(M, (unsigned long long)F + m + 64);
      if (!sc) return;  // pool_alloc raised the error
      s0 = sym_elim_chain(M, t, V, h, sc.as<int>(), sc.as<int>() + F, &nout);
    }
    if (s0 < 0 || s0 >= m) return;
  }
  // queue links: the wave's LDS slice, or global memory; the forward rows
  // are read from global memory once per block of 64 columns
  using IP = typename std::conditional<kLds, int*, gptr<int>>::type;
  IP head = V.head;
  IP next = V.next;
  const gptr<int> optr = V.optr;
  const gptr<int> oent = V.oent;
  uint32_t* rb = nullptr;
  if constexpr (kLds) {
    head = lds;
    next = head + m;
    rb = (uint32_t*)(lds + m + rows);
    for (int i = lane_id(); i < m; i += 64) head[i] = V.head[i];
    for (int i = lane_id(); i < rows; i += 64) next[i] = V.next[i];
    for (int i = lane_id(); i < FW; i += 64) rb[i] = 0u;
    wave_fence();
  }
  if (FW > 64 * FP_SYM_REGW) {
    sym_elim_wide(M, t, V, h, head, next, optr, oent, s0, nout);
    return;
  }
  if (FW <= 64)
    sym_elim_cols<1>(M, t, V, h, head, next, optr, oent, rb, s0, nout);
  else if (FW <= 128)
    sym_elim_cols<2>(M, t, V, h, head, next, optr, oent, rb, s0, nout);
  else
    sym_elim_cols<4>(M, t, V, h, head, next, optr, oent, rb, s0, nout);
}

// LDS words of a node's elimination: the chain form's intro and diff
// arrays, or the sequential walk's queue links (heads and next pointers)
// and forward-entry row buffer
__device__ __forceinline__ long long sym_elim_lds_words(const int* h) {
  const long long chain = 2ll * h[SH_M] + h[SH_NBD];
  const long long walk = (long long)h[SH_M] + h[SH_ROWS] + h[SH_FW];
  return chain > walk ? chain : walk;
}

// 0: the links fit a quarter of the per-node LDS (four waves per workgroup),
// 1: the large one-wave slice, 2: neither (global memory)
__device__ __forceinline__ int sym_elim_class(const FpMesh& M, const int* h) {
  const long long need = sym_elim_lds_words(h);
  if (need <= (long long)uni(M.lds_bytes) / 4 / FP_WAVES) return 0;
  if (need <= (long long)uni(M.lds_big) / 4) return 1;
  return 2;
}

template <bool kLds>
__device__ __forceinline__ void sym_elim(const FpMesh& M, int t, int cls, int* lds,
                                         long long lds_words) {
  SymView V;
  int h[SH_WORDS];
  if (!sym_load(M, t, &V, h)) return;
  if (sym_elim_class(M, h) == cls) sym_elim_run<kLds>(M, t, V, h, lds, lds_words);
}

// ---------------------------------------------------------------- emit
__device__ __forceinline__ void sym_emit(const FpMesh& M, int t, int d) {
  SymView V;
  int h[SH_WORDS];
  if (!sym_load(M, t, &V, h)) {
    if (M.sdesc[t] >= 0) sym_drop(M, t, 0);  // elim failed after prep
    return;
  }
  const int m = h[SH_M], nbd = h[SH_NBD], FW = h[SH_FW], rows = h[SH_ROWS];
  const int stride = h[SH_STRIDE], nout = h[SH_NOUT];
  if (nout < 0 || nout > rows) {
    sym_drop(M, t, FP_SITE_SYM_LIVE);
    return;
  }
  // record sizes, four rows per step with their loads issued together
  int total = 0;
  for (int i0 = 0; i0 < nout; i0 += 4) {
    int r[4];
    bool bad = false;
#pragma unroll
    for (int u = 0; u < 4; u++) {
      r[u] = i0 + u < nout ? uni(V.outl[i0 + u]) : 0;
      bad |= (unsigned)r[u] >= (unsigned)rows;
    }
    if (bad) {
      sym_drop(M, t, FP_SITE_SYM_LIVE);
      return;
    }
    int c[4] = {0, 0, 0, 0};
    for (int w = lane_id(); w < FW; w += 64) {
      uint32_t x[4];
#pragma unroll
      for (int u = 0; u < 4; u++) x[u] = V.rows[(long long)r[u] * stride + w];
#pragma unroll
      for (int u = 0; u < 4; u++) c[u] += i0 + u < nout ? popc32(x[u]) : 0;
    }
#pragma unroll
    for (int u = 0; u < 4; u++) total += i0 + u < nout ? 1 + wave_sum_i32(c[u]) : 0;
  }
  int base = 0;
  if (lane_id() == 0) {
    base = atomicAdd(&M.ctl->arena_top[d & 1], total);
    if ((long long)base + total > M.acap) {
      fp_fail(M.ctl, FP_E_SCRATCH, FP_SITE_SYM_ARENA, t);
      base = -1;
    }
  }
  base = wave_bcast(base, 0);
  if (base < 0) {
    sym_drop(M, t, 0);
    return;
  }
  gptr<int> dst = M.arena[d & 1];
  const int b0 = uni(M.nbegin[t]);
  int off = base;
  bool bad = false;
  for (int i = 0; i < nout; i++) {
    gptr<const uint32_t> row = V.rows + (long long)uni(V.outl[i]) * stride;
    int len = 0;
    for (int w0 = 0; w0 < FW; w0 += 64) {
      const int w = w0 + lane_id();
      uint32_t x = w < FW ? row[w] : 0u;
      const int c = popc32(x);
      const int inc = wave_incl_scan(c);
      int o = off + 1 + len + inc - c;
      // eight set bits per step, their positions loaded together
      while (x) {
        int f[8], q[8];
#pragma unroll
        for (int u = 0; u < 8; u++) {
          f[u] = x ? w * 32 + __ffs(x) - 1 : -1;
          x &= x - 1;
        }
#pragma unroll
        for (int u = 0; u < 8; u++) {
          const bool ok = f[u] >= m && f[u] < m + nbd;  // elements only hold later positions
          q[u] = V.bd[ok ? f[u] - m : 0];
        }
#pragma unroll
        for (int u = 0; u < 8; u++) {
          if (f[u] < 0) continue;
          const bool ok = f[u] >= m && f[u] < m + nbd;
          bad |= !ok;
          dst[o++] = ok ? q[u] : b0;
        }
      }
      len += wave_bcast(inc, 63);
    }
    if (lane_id() == 0) dst[off] = len;
    off += 1 + len;
  }
  if (ballot64(bad)) {
    sym_drop(M, t, FP_SITE_SYM_LOOKUP);
    return;
  }
  if (lane_id() == 0) {
    M.eoff[3 * t] = base;
    M.eoff[3 * t + 1] = total;
    M.eoff[3 * t + 2] = nout;
  }
}
