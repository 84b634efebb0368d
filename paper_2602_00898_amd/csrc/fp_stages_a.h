// fp_stages_a.h -- per-item helpers of graph ingest, patching and the
// quotient graph.
#pragma once

#include "fp_device.h"
#include "fp_mesh.h"

#define FP_UNSET 0xFFFFFFFFFFFFFFFFull

// raise error bits; the first failing site and one value are kept
__device__ __forceinline__ void fp_fail(gptr<FpCtl> C, unsigned bits, int site, int arg) {
  atomicOr(&C->err, bits);
  if (atomicCAS(&C->site, 0, site) == 0) atomicExch(&C->site_arg, arg);
}

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
// into vertex v (Sec. 4.1 Step 2, Sec. 6.5).  Every row of the graph comes
// out sorted ascending and without duplicates, whatever the order and
// multiplicity of the input entries.  A lane per vertex handles rows of up
// to FP_ROW_SHORT input entries; longer rows are listed and handled by a
// whole workgroup each (ingest_long_row).
// --------------------------------------------------------------------------
#define FP_ROW_SHORT 512

// input entries of vertex v's block rows: [*e0, *e1); false on a bad range
__device__ __forceinline__ bool vertex_row_range(const FpMesh& M, int v, long long* e0,
                                                 long long* e1) {
  const long long r0 = (long long)v * M.b;
  *e0 = rp_at(M, r0);
  *e1 = rp_at(M, r0 + M.b);
  return *e0 >= 0 && *e1 >= *e0 && *e1 <= M.nnz_in;
}

// vertex of input entry e, or -1 for the diagonal block and bad indices
__device__ __forceinline__ int entry_vertex(const FpMesh& M, long long e, int v, unsigned* eb) {
  const int c = M.ci_in[e];
  if (c < 0 || (long long)c >= M.n_dof) {
    *eb |= FP_E_INDEX;
    return -1;
  }
  const int u = c / M.b;
  return u == v ? -1 : u;
}

// Rows of up to FP_ROW_REG input entries (mesh rows): the entries are
// loaded together and deduplicated and ranked in registers.
#define FP_ROW_REG 16
__device__ __forceinline__ int gather_vertex_row_reg(const FpMesh& M, int v, long long e0, long long e1,
                                                     gptr<int> out, unsigned* eb) {
  if (e1 == e0) return 0;
  int u[FP_ROW_REG];  // entries past the row re-read its last one (ignored)
#pragma unroll
  for (int j = 0; j < FP_ROW_REG; j++) u[j] = M.ci_in[min(e0 + j, e1 - 1)];
  bool bad = false;
#pragma unroll
  for (int j = 0; j < FP_ROW_REG; j++) {
    const int c = u[j];
    const bool in = e0 + j < e1;
    const bool ok = c >= 0 && (long long)c < M.n_dof;
    bad |= in && !ok;
    const int w = M.b == 1 ? c : c / M.b;
    u[j] = in && ok && w != v ? w : -1;  // -1: the diagonal block or a bad index
  }
  if (bad) *eb |= FP_E_INDEX;
  // an entry counts if no earlier entry names the same vertex
#pragma unroll
  for (int j = 1; j < FP_ROW_REG; j++) {
    bool dup = false;
#pragma unroll
    for (int i = 0; i < j; i++) dup |= u[i] == u[j];
    if (dup) u[j] = -1;
  }
  int cnt = 0;
#pragma unroll
  for (int j = 0; j < FP_ROW_REG; j++) cnt += u[j] >= 0;
  if (out) {
    // rank of each distinct vertex among the others: its slot in the
    // ascending row
#pragma unroll
    for (int j = 0; j < FP_ROW_REG; j++) {
      int r = 0;
#pragma unroll
      for (int i = 0; i < FP_ROW_REG; i++) r += u[i] >= 0 && u[i] < u[j];
      if (u[j] >= 0) out[r] = u[j];
    }
  }
  return cnt;
}

// Short rows (one lane): the distinct neighbours of v; with `out`, written
// there in ascending order.  Returns their count, or -1 for a long row.
__device__ __forceinline__ int gather_vertex_row(const FpMesh& M, int v, gptr<int> out, unsigned* eb) {
  long long e0, e1;
  if (!vertex_row_range(M, v, &e0, &e1)) {
    *eb |= FP_E_INDEX;
    return 0;
  }
  if (e1 - e0 > FP_ROW_SHORT) return -1;
  if (e1 - e0 <= FP_ROW_REG) return gather_vertex_row_reg(M, v, e0, e1, out, eb);
  int cnt = 0;
  for (long long e = e0; e < e1; e++) {
    const int u = entry_vertex(M, e, v, eb);
    if (u < 0) continue;
    bool dup = false;
    for (long long f = e0; f < e && !dup; f++) {
      const int c2 = M.ci_in[f];
      dup = c2 >= 0 && (long long)c2 < M.n_dof && c2 / M.b == u;
    }
    if (dup) continue;
    if (out) {
      // insertion into the sorted prefix out[0..cnt)
      int k = cnt;
      while (k > 0 && out[k - 1] > u) {
        out[k] = out[k - 1];
        k--;
      }
      out[k] = u;
    }
    cnt++;
  }
  return cnt;
}

// Long rows (one workgroup, blockDim.x threads): an entry counts if no
// earlier entry of the row names the same vertex.  Without `out`, returns the
// number of distinct vertices to every thread.  With `out`, the distinct
// vertices are appended there and then sorted in place by a bitonic network
// whose first step of every merge compares mirrored positions, so every
// comparison puts the smaller value first and positions past the count act
// as +infinity that never moves.  `red` is one LDS word.
__device__ __forceinline__ int ingest_long_row(const FpMesh& M, int v, gptr<int> out, unsigned* eb,
                                               int* red) {
  long long e0, e1;
  if (!vertex_row_range(M, v, &e0, &e1)) {
    *eb |= FP_E_INDEX;
    return 0;
  }
  if (threadIdx.x == 0) *red = 0;
  __syncthreads();
  for (long long e = e0 + threadIdx.x; e < e1; e += blockDim.x) {
    const int u = entry_vertex(M, e, v, eb);
    if (u < 0) continue;
    bool first = true;
    for (long long f = e0; f < e && first; f++) {
      const int c2 = M.ci_in[f];
      first = !(c2 >= 0 && (long long)c2 < M.n_dof && c2 / M.b == u);
    }
    if (!first) continue;
    const int slot = atomicAdd(red, 1);
    if (out) out[slot] = u;
  }
  __syncthreads();
  const int cnt = *red;
  if (out && cnt > 1) {
    int pw = 1;
    while (pw < cnt) pw <<= 1;
    for (int k = 2; k <= pw; k <<= 1) {
      const int h = k >> 1;
      for (int i = threadIdx.x; i < pw / 2; i += blockDim.x) {
        const int a = (i / h) * k + (i % h), b = (i / h) * k + (k - 1 - (i % h));
        if (b < cnt) {
          const int x = out[a], y = out[b];
          if (x > y) {
            out[a] = y;
            out[b] = x;
          }
        }
      }
      __syncthreads();
      for (int j = h >> 1; j >= 1; j >>= 1) {
        for (int i = threadIdx.x; i < pw / 2; i += blockDim.x) {
          const int a = (i / j) * 2 * j + (i % j), b = a + j;
          if (b < cnt) {
            const int x = out[a], y = out[b];
            if (x > y) {
              out[a] = y;
              out[b] = x;
            }
          }
        }
        __syncthreads();
      }
    }
  }
  __syncthreads();
  return cnt;
}

// true if the sorted row of u holds v
__device__ __forceinline__ bool row_has(const FpMesh& M, int u, int v) {
  int lo = M.grp[u], hi = M.grp[u + 1];
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (M.gci[mid] < v)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo < M.grp[u + 1] && M.gci[lo] == v;
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
