// fp_pipeline.h -- block expansion of the outputs and the stage sequence
// that a team runs for one mesh.
#pragma once

#include "fp_stages_sym.h"

// --------------------------------------------------------------------------
// block expansion and outputs (Sec. 6.5: expand the vertex ordering, its
// elimination tree and column counts to the b DOFs of every vertex)
// --------------------------------------------------------------------------
__device__ void stage_expand(const Team& T, const FpMesh& M) {
  FpCtl* C = M.ctl;
  const int b = M.b;
  const long long nd = M.n_dof;
  for (long long j = T.gtid(); j < nd; j += T.gsize()) {
    const int k = (int)(j / b), r = (int)(j - (long long)k * b);
    M.perm[j] = M.vperm[k] * b + r;
    M.iperm[j] = M.viperm[k] * b + r;
    M.colcount[j] = b * M.vcc[k] - r;
    M.parent[j] = r < b - 1 ? (int)(j + 1) : (M.vpar[k] < 0 ? -1 : M.vpar[k] * b);
  }
  if (M.gmap_out)
    for (int v = T.gtid(); v < M.n; v += T.gsize()) M.gmap_out[v] = M.gmap[v];
  const int nn = C->nn;
  if (M.node_begin_out || M.node_size_out) {
    if (nn > M.max_nodes_out) {
      if (T.gtid() == 0) atomicOr(&C->err, FP_E_SCRATCH);
    } else {
      for (int x = T.gtid(); x < nn; x += T.gsize()) {
        if (M.node_begin_out) M.node_begin_out[x] = M.nbegin[x] * b;
        if (M.node_size_out) M.node_size_out[x] = M.nsize[x] * b;
      }
    }
  }
  T.sync();
  if (T.gtid() == 0) {
    *M.nnzL = (long long)b * b * C->nnzL - (long long)M.n * b * (b - 1) / 2;
    if (M.n_nodes_out) *M.n_nodes_out = nn;
  }
}

__device__ void pipeline(const Team& T, const FpMesh& M, char* lds, int* lds_tmp) {
  FpCtl* C = M.ctl;
  stage_ingest(T, M, lds_tmp);
  if (C->nnz_g > M.Ecap || C->nnz_g < 0) return;
  stage_patches(T, M, lds_tmp);
  stage_quotient(T, M, lds_tmp);
  if (C->nq > M.Ecap) return;
  if (!stage_septree(T, M, lds)) return;
  stage_group(T, M, lds_tmp);
  FP_DBG(T, M, 1);
  stage_local_orders(T, M, lds);
  FP_DBG(T, M, 2);
  stage_symbolic(T, M, lds);
  stage_expand(T, M);
}

