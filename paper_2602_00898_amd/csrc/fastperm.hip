// fastperm.hip -- the persistent gfx950 ordering kernel and the C ABI
// declared in include/fastperm.h.
//
// One launch orders one matrix: a team made of every workgroup of the grid
// (one 512-thread workgroup per CU, 160 KiB LDS each) runs the stages in
// sequence, separated by team barriers:
//   ingest -> patches -> quotient graph -> separator tree -> grouping ->
//   local orders -> elimination tree / column counts -> block expansion.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <new>

#include "../../include/fastperm.h"
#include "fp_pipeline.h"
#include "fp_plan.h"

__global__ void __launch_bounds__(FP_WG) fp_plain_kernel(FpMesh M) {
  extern __shared__ __align__(16) char lds[];
  __shared__ int lds_tmp[FP_WAVES + 8];
  Team T{(int)blockIdx.x, (int)gridDim.x, M.ctl->bar, &M.ctl->err};
  pipeline(T, M, lds, lds_tmp);
  T.sync();
  if (T.gtid() == 0 && M.status_out) *M.status_out = M.ctl->err;
}

__global__ void fp_ctl_init(unsigned* ctl, int words) {
  for (int i = threadIdx.x + blockIdx.x * blockDim.x; i < words; i += blockDim.x * gridDim.x)
    ctl[i] = 0u;
}

// --------------------------------------------------------------------------
// host side
// --------------------------------------------------------------------------
struct fp_handle {
  int device;
  int ncu;
  int lds_bytes;
  int grid;
};

namespace {

using fpplan::Plan;
using fpplan::make_plan;
using fpplan::fill_mesh;

fp_status check_opts(const fp_options* o) {
  if (!o) return FP_ERR_ARG;
  if (o->patch_size < 1 || o->block_size < 1 || o->lloyd_iters < 0 || o->lloyd_iters > 64)
    return FP_ERR_ARG;
  if (o->schedule != FP_SCHED_LEVEL && o->schedule != FP_SCHED_POST) return FP_ERR_ARG;
  if (o->nd_level != -1 || o->flags != 0) return FP_ERR_UNSUPPORTED;
  return FP_OK;
}

fp_status check_csr(const fp_csr* A, int b) {
  if (!A) return FP_ERR_ARG;
  if (A->n < 0 || A->nnz < 0 || A->n >= (1ll << 31)) return FP_ERR_ARG;
  if (!!A->rowptr32 == !!A->rowptr64) return FP_ERR_ARG;
  if (A->nnz > 0 && !A->colind) return FP_ERR_ARG;
  if (A->rowptr32 && A->nnz >= (1ll << 31)) return FP_ERR_ARG;
  if (A->n % b) return FP_ERR_ARG;
  return FP_OK;
}

}  // namespace

extern "C" {

int fp_version(void) { return FP_ABI_VERSION; }

const char* fp_status_str(fp_status s) {
  switch (s) {
    case FP_OK: return "ok";
    case FP_ERR_ARG: return "invalid argument";
    case FP_ERR_NOT_SYMMETRIC: return "pattern not symmetric";
    case FP_ERR_INDEX: return "index out of range";
    case FP_ERR_SIZE: return "workspace or device pool too small";
    case FP_ERR_OOM: return "out of device memory";
    case FP_ERR_UNSUPPORTED: return "unsupported option";
    case FP_ERR_BUSY: return "server busy";
    case FP_ERR_HIP: return "HIP runtime error";
    case FP_ERR_DEVICE: return "device pipeline failure";
  }
  return "unknown status";
}

void fp_options_default(fp_options* o) {
  if (!o) return;
  o->patch_size = 512;
  o->nd_level = -1;
  o->schedule = FP_SCHED_LEVEL;
  o->block_size = 1;
  o->lloyd_iters = 1;
  o->seed = 0;
  o->flags = 0;
}

fp_status fp_create(fp_handle** h) {
  if (!h) return FP_ERR_ARG;
  *h = nullptr;
  fp_handle* H = new (std::nothrow) fp_handle();
  if (!H) return FP_ERR_OOM;
  if (hipGetDevice(&H->device) != hipSuccess) {
    delete H;
    return FP_ERR_HIP;
  }
  int ncu = 0, maxsh = 0;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, H->device) != hipSuccess ||
      hipDeviceGetAttribute(&maxsh, hipDeviceAttributeMaxSharedMemoryPerBlock, H->device) !=
          hipSuccess) {
    delete H;
    return FP_ERR_HIP;
  }
  H->ncu = ncu;
  const int static_lds = (int)sizeof(int) * (FP_WAVES + 8);
  H->lds_bytes = std::min(FP_LDS_BYTES, maxsh - static_lds - 64) & ~255;
  if (hipFuncSetAttribute((const void*)fp_plain_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                          H->lds_bytes) != hipSuccess) {
    delete H;
    return FP_ERR_HIP;
  }
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fp_plain_kernel, FP_WG,
                                                   H->lds_bytes) != hipSuccess ||
      per_cu < 1) {
    delete H;
    return FP_ERR_HIP;
  }
  H->grid = ncu * std::min(per_cu, 1);
  *h = H;
  return FP_OK;
}

fp_status fp_destroy(fp_handle* h) {
  delete h;
  return FP_OK;
}

fp_status fp_query(fp_handle* h, const fp_csr* A, const fp_options* opts, size_t* ws_bytes,
                   int32_t* max_nodes) {
  if (!h || !ws_bytes) return FP_ERR_ARG;
  fp_status s = check_opts(opts);
  if (s) return s;
  if ((s = check_csr(A, opts->block_size))) return s;
  Plan P;
  if (!make_plan(A->n, opts->block_size, A->nnz, &P)) return FP_ERR_ARG;
  *ws_bytes = P.total;
  if (max_nodes) *max_nodes = P.NNcap;
  return FP_OK;
}

fp_status fp_order(fp_handle* h, const fp_csr* A, const int32_t* user_gmap,
                   const fp_options* opts, void* workspace, size_t ws_bytes, fp_result* out,
                   void* stream) {
  if (!h || !out || !workspace) return FP_ERR_ARG;
  fp_status s = check_opts(opts);
  if (s) return s;
  if ((s = check_csr(A, opts->block_size))) return s;
  if (!out->perm || !out->iperm || !out->parent || !out->colcount || !out->nnzL) return FP_ERR_ARG;
  if ((out->node_begin || out->node_size) && out->max_nodes < 1) return FP_ERR_ARG;
  Plan P;
  if (!make_plan(A->n, opts->block_size, A->nnz, &P)) return FP_ERR_ARG;
  if (ws_bytes < P.total) return FP_ERR_SIZE;
  hipStream_t st = (hipStream_t)stream;
  FpMesh M;
  memset(&M, 0, sizeof(M));
  fill_mesh(P, (char*)workspace, &M);
  M.rp32 = A->rowptr32;
  M.rp64 = (const long long*)A->rowptr64;
  M.ci_in = A->colind;
  M.nnz_in = A->nnz;
  M.user_gmap = user_gmap;
  M.S = opts->patch_size;
  M.lloyd = opts->lloyd_iters;
  M.sched = opts->schedule;
  M.seed = opts->seed;
  M.perm = out->perm;
  M.iperm = out->iperm;
  M.parent = out->parent;
  M.colcount = out->colcount;
  M.nnzL = (long long*)out->nnzL;
  M.node_begin_out = out->node_begin;
  M.node_size_out = out->node_size;
  M.gmap_out = out->gmap;
  M.n_nodes_out = out->n_nodes;
  M.status_out = out->status;
  M.max_nodes_out = out->max_nodes;
  M.lds_bytes = h->lds_bytes;
  const int words = (int)(sizeof(FpCtl) / 4);
  hipLaunchKernelGGL(fp_ctl_init, dim3(1), dim3(1024), 0, st, (unsigned*)M.ctl, words);
  hipLaunchKernelGGL(fp_plain_kernel, dim3(h->grid), dim3(FP_WG), h->lds_bytes, st, M);
  if (hipGetLastError() != hipSuccess) return FP_ERR_HIP;
  return FP_OK;
}

fp_status fp_last_error(fp_handle* h, void* workspace, void* stream) {
  if (!h || !workspace) return FP_ERR_ARG;
  if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess) return FP_ERR_HIP;
  unsigned e = 0;
  if (hipMemcpy(&e, &((FpCtl*)workspace)->err, sizeof(e), hipMemcpyDeviceToHost) != hipSuccess)
    return FP_ERR_HIP;
  if (e & FP_E_INDEX) return FP_ERR_INDEX;
  if (e & (FP_E_SCRATCH)) return FP_ERR_SIZE;
  if (e & FP_E_GMAP) return FP_ERR_INDEX;
  if (e) return FP_ERR_DEVICE;
  return FP_OK;
}

}  // extern "C"
