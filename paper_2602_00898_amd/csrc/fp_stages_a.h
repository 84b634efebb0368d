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
// into vertex v (Sec. 4.1 Step 2, Sec. 6.5).  Duplicates are dropped for
// rows up to 512 entries; every later stage treats rows as sets, so longer
// rows may keep duplicates.
// --------------------------------------------------------------------------
__device__ __forceinline__ int gather_vertex_row(const FpMesh& M, int v, gptr<int> out, unsigned* eb) {
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
