// fp_plan.h -- host-side workspace layout of one ordering job: byte offsets
// of every device array inside the caller's workspace buffer.
#pragma once

#include <algorithm>
#include <cstddef>

#include "fp_mesh.h"


namespace fpplan {

struct Plan {
  long long n_dof;
  int b;
  int n;
  long long Ecap;
  int NNcap;
  long long acap;
  unsigned long long pool_words;
  size_t total;
  // byte offsets
  size_t o_ctl, o_mesh, o_fcnt, o_grp, o_gci, o_key, o_best, o_fa, o_fb, o_gmap, o_seeds, o_pcnt, o_pptr, o_pvtx,
      o_bnd, o_qptr, o_qci, o_qcnt, o_wp, o_pnode, o_plist, o_ploc, o_node_of, o_cand, o_bs[10],
      o_nsize, o_nbegin, o_ncur, o_segS, o_segN, o_cntL, o_cntR, o_sbuf, o_eoff, o_tasks, o_gbuf,
      o_lidx, o_vperm, o_viperm, o_vpar, o_vcc, o_arena[2], o_sdesc, o_tbuf, o_prow, o_pent, o_pool,
      o_rlist, o_mate, o_rpar, o_seen, o_rqa, o_rqb, o_roff, o_rcur;
};

size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

// S: target patch size (bounds the per-level scratch of the symbolic stage)
bool make_plan(long long n_dof, int b, long long nnz, int S, Plan* P) {
  if (b < 1 || n_dof < 0 || n_dof % b) return false;
  const long long n = n_dof / b;
  if (n >= (1ll << 31) - 2) return false;
  P->n_dof = n_dof;
  P->b = b;
  P->n = (int)n;
  P->Ecap = std::max(nnz, 1ll);
  if (P->Ecap >= (1ll << 31) - 1) P->Ecap = (1ll << 31) - 2;
  int d = 0;
  while ((1ll << d) < std::max(n, 1ll)) d++;
  P->NNcap = (int)std::min((1ll << (d + 1)) + 2, (1ll << 31) - 1);
  P->acap = P->Ecap + 3 * n + 4096;
  // one pool serves the local orders, then each level of the symbolic stage
  // in turn: per vertex of a level a bitset row over the node's positions
  // and later positions (about 2S + 1024 bits for patch-sized nodes)
  const long long Se = std::max(1ll, std::min((long long)std::max(S, 1), n));
  P->pool_words = std::max(1ull << 24, (unsigned long long)(16 * n + 4 * P->Ecap +
                                                            n * ((2 * Se + 1024) / 32) + (1 << 20)));
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t r = o;
    o = align_up(o + bytes);
    return r;
  };
  const size_t N1 = (size_t)n + 1, E = (size_t)P->Ecap, NN = (size_t)P->NNcap;
  P->o_ctl = take(sizeof(FpCtl));
  P->o_mesh = take(sizeof(FpMesh));
  P->o_fcnt = take(4 * (N1 + 16));
  P->o_grp = take(4 * N1);
  P->o_gci = take(4 * E);
  P->o_key = take(8 * N1);
  P->o_best = take(8 * N1);
  P->o_fa = take(4 * N1);
  P->o_fb = take(4 * N1);
  P->o_gmap = take(4 * N1);
  P->o_seeds = take(4 * N1);
  P->o_pcnt = take(4 * (N1 + 1));
  P->o_pptr = take(4 * (N1 + 1));
  P->o_pvtx = take(4 * N1);
  P->o_bnd = take(4 * N1);
  P->o_qptr = take(4 * (N1 + 1));
  P->o_qci = take(4 * E);
  P->o_qcnt = take(4 * E);
  P->o_wp = take(4 * N1);
  P->o_pnode = take(4 * N1);
  P->o_plist = take(4 * N1);
  P->o_ploc = take(4 * N1);
  P->o_node_of = take(4 * N1);
  P->o_cand = take(4 * N1);
  for (int i = 0; i < 10; i++) P->o_bs[i] = take(4 * (2 * N1 + 2));
  P->o_nsize = take(4 * NN);
  P->o_nbegin = take(4 * NN);
  P->o_ncur = take(4 * NN);
  P->o_segS = take(4 * NN);
  P->o_segN = take(4 * NN);
  P->o_cntL = take(4 * NN);
  P->o_cntR = take(4 * NN);
  P->o_sbuf = take(4 * NN);
  P->o_eoff = take(12 * NN);
  P->o_tasks = take(32 * NN);
  P->o_gbuf = take(4 * N1);
  P->o_lidx = take(4 * N1);
  P->o_vperm = take(4 * N1);
  P->o_viperm = take(4 * N1);
  P->o_vpar = take(4 * N1);
  P->o_vcc = take(4 * N1);
  P->o_arena[0] = take(4 * (size_t)P->acap);
  P->o_arena[1] = take(4 * (size_t)P->acap);
  P->o_sdesc = take(8 * NN);
  P->o_tbuf = take(4 * N1);
  P->o_rlist = take(4 * N1);
  P->o_mate = take(4 * N1);
  P->o_rpar = take(4 * N1);
  P->o_seen = take(4 * N1);
  P->o_rqa = take(4 * N1);
  P->o_rqb = take(4 * N1);
  P->o_roff = take(4 * NN);
  P->o_rcur = take(4 * NN);
  P->o_prow = take(4 * (N1 + 1));
  P->o_pent = take(4 * (size_t)P->Ecap);
  P->o_pool = take(4 * (size_t)P->pool_words);
  P->total = o;
  return true;
}

void fill_mesh(const Plan& P, char* ws, FpMesh* M) {
  M->n = P.n;
  M->n_dof = P.n_dof;
  M->b = P.b;
  M->Ecap = P.Ecap;
  M->NNcap = P.NNcap;
  M->acap = P.acap;
  M->pool_words = P.pool_words;
  M->ctl = (FpCtl*)(ws + P.o_ctl);
  M->grp = (int*)(ws + P.o_grp);
  M->gci = (int*)(ws + P.o_gci);
  M->key = (unsigned long long*)(ws + P.o_key);
  M->best = (unsigned long long*)(ws + P.o_best);
  M->fa = (int*)(ws + P.o_fa);
  M->fcnt = (int*)(ws + P.o_fcnt);
  M->fb = (int*)(ws + P.o_fb);
  M->gmap = (int*)(ws + P.o_gmap);
  M->seeds = (int*)(ws + P.o_seeds);
  M->pcnt = (int*)(ws + P.o_pcnt);
  M->pptr = (int*)(ws + P.o_pptr);
  M->pvtx = (int*)(ws + P.o_pvtx);
  M->bnd = (int*)(ws + P.o_bnd);
  M->qptr = (int*)(ws + P.o_qptr);
  M->qci = (int*)(ws + P.o_qci);
  M->qcnt = (int*)(ws + P.o_qcnt);
  M->wp = (int*)(ws + P.o_wp);
  M->pnode = (int*)(ws + P.o_pnode);
  M->plist = (int*)(ws + P.o_plist);
  M->ploc = (int*)(ws + P.o_ploc);
  M->node_of = (int*)(ws + P.o_node_of);
  M->cand = (int*)(ws + P.o_cand);
  for (int i = 0; i < 10; i++) M->bs[i] = (int*)(ws + P.o_bs[i]);
  M->nsize = (int*)(ws + P.o_nsize);
  M->nbegin = (int*)(ws + P.o_nbegin);
  M->ncur = (int*)(ws + P.o_ncur);
  M->segS = (int*)(ws + P.o_segS);
  M->segN = (int*)(ws + P.o_segN);
  M->cntL = (int*)(ws + P.o_cntL);
  M->cntR = (int*)(ws + P.o_cntR);
  M->sbuf = (int*)(ws + P.o_sbuf);
  M->eoff = (int*)(ws + P.o_eoff);
  M->tasks = (int*)(ws + P.o_tasks);
  M->gbuf = (int*)(ws + P.o_gbuf);
  M->lidx = (int*)(ws + P.o_lidx);
  M->vperm = (int*)(ws + P.o_vperm);
  M->viperm = (int*)(ws + P.o_viperm);
  M->vpar = (int*)(ws + P.o_vpar);
  M->vcc = (int*)(ws + P.o_vcc);
  M->arena[0] = (int*)(ws + P.o_arena[0]);
  M->arena[1] = (int*)(ws + P.o_arena[1]);
  M->sdesc = (long long*)(ws + P.o_sdesc);
  M->tbuf = (int*)(ws + P.o_tbuf);
  M->rlist = (int*)(ws + P.o_rlist);
  M->mate = (int*)(ws + P.o_mate);
  M->rpar = (int*)(ws + P.o_rpar);
  M->seen = (int*)(ws + P.o_seen);
  M->rqa = (int*)(ws + P.o_rqa);
  M->rqb = (int*)(ws + P.o_rqb);
  M->roff = (int*)(ws + P.o_roff);
  M->rcur = (int*)(ws + P.o_rcur);
  M->prow = (int*)(ws + P.o_prow);
  M->pent = (int*)(ws + P.o_pent);
  M->pool = (unsigned*)(ws + P.o_pool);
}

}  // namespace fpplan
