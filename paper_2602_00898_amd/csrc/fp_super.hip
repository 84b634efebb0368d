// fp_super.hip -- supernodal symbolic analysis on the ordering's outputs
// (the solver's symbolic phase, which needs the elimination tree, Sec. 1).
//
// Fundamental supernodes (Liu, Ng and Peyton, SIAM J. Matrix Anal. Appl.
// 14(1), 1993): column j+1 continues the supernode of column j exactly when
// parent[j] == j+1, j is the only child of j+1 and colcount[j] ==
// colcount[j+1] + 1.  Every step is a vertex-parallel pass over the columns
// or the supernodes (HBM-bound), plus 64-bit scans for the column pointers
// of L and the offsets of the dense supernode blocks.  Nothing is read back
// to the host: the supernode count stays on the device and the passes over
// supernodes read it there.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "../../include/fastperm.h"
#include "fp_device.h"
#include "fp_handle.h"

#define SN_PER_THREAD 16
#define SN_CHUNK (FP_WG * SN_PER_THREAD)  // elements per scan block

namespace {

// control words of one call, at the start of its workspace
struct SnCtl {
  unsigned err;  // 1: a parent out of range or not after its column
  int ns;        // supernodes
  int bad;       // first offending column
};

__global__ void k_sn_init(SnCtl* c, int* nchild, int n) {
  for (int i = gtid(); i < n; i += gsize()) nchild[i] = 0;
  if (gtid() == 0) {
    c->err = 0;
    c->ns = 0;
    c->bad = -1;
  }
}

// children per column; a parent must lie after its column (etree of a
// permuted matrix: parent[j] > j) or be -1
__global__ void k_sn_child(const int* __restrict__ parent, int n, int* nchild, SnCtl* c) {
  for (int j = gtid(); j < n; j += gsize()) {
    const int p = parent[j];
    if (p < -1 || p >= n || (p >= 0 && p <= j)) {
      atomicOr(&c->err, 1u);
      atomicMax(&c->bad, j);
    } else if (p >= 0) {
      atomicAdd(&nchild[p], 1);
    }
  }
}

// 1 where a supernode starts
__global__ void k_sn_flag(const int* __restrict__ parent, const int* __restrict__ cc,
                          const int* __restrict__ nchild, int n, int* flag) {
  for (int j = gtid(); j < n; j += gsize()) {
    const bool cont =
        j > 0 && parent[j - 1] == j && nchild[j] == 1 && cc[j - 1] == cc[j] + 1;
    flag[j] = cont ? 0 : 1;
  }
}

// ---------------------------------------------------------------- scans
// Exclusive 64-bit scan of in[0..n) into out[0..n], out[n] = total; n is
// the host value `n_host` or, when n_dev is given, the device value (at most
// n_host).  Blocks of SN_CHUNK elements: block sums, a scan of the sums,
// then each block rescans its chunk (SN_PER_THREAD consecutive elements per
// thread, a workgroup scan of the thread sums in LDS).
template <class T>
__device__ __forceinline__ long long sn_val(const T* in, long long i) {
  return (long long)in[i];
}

__device__ __forceinline__ long long wg_excl_scan64(long long x, long long* tmp, long long* total) {
  tmp[threadIdx.x] = x;
  __syncthreads();
  for (int o = 1; o < FP_WG; o <<= 1) {
    const long long y = threadIdx.x >= (unsigned)o ? tmp[threadIdx.x - o] : 0;
    __syncthreads();
    tmp[threadIdx.x] += y;
    __syncthreads();
  }
  const long long inc = tmp[threadIdx.x];
  *total = tmp[FP_WG - 1];
  __syncthreads();
  return inc - x;
}

template <class T>
__global__ void k_scan64_part(const T* __restrict__ in, int n_host, const int* n_dev,
                              long long* part) {
  __shared__ long long tmp[FP_WG];
  const int n = n_dev ? min(*n_dev, n_host) : n_host;
  const long long lo = (long long)blockIdx.x * SN_CHUNK;
  long long s = 0;
  for (long long i = lo + threadIdx.x; i < min((long long)n, lo + SN_CHUNK); i += FP_WG)
    s += sn_val(in, i);
  long long tot;
  wg_excl_scan64(s, tmp, &tot);
  if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

__global__ void k_scan64_top(long long* part, int nb, int n_host, const int* n_dev,
                             long long* out) {
  __shared__ long long tmp[FP_WG];
  long long base = 0;
  for (int c0 = 0; c0 < nb; c0 += FP_WG) {
    const int i = c0 + (int)threadIdx.x;
    const long long x = i < nb ? part[i] : 0;
    long long tt;
    const long long ex = wg_excl_scan64(x, tmp, &tt);
    if (i < nb) part[i] = base + ex;
    base += tt;
  }
  const int n = n_dev ? min(*n_dev, n_host) : n_host;
  if (threadIdx.x == 0) out[n] = base;
}

template <class T>
__global__ void k_scan64_apply(const T* __restrict__ in, int n_host, const int* n_dev,
                               const long long* part, long long* out) {
  __shared__ long long tmp[FP_WG];
  const int n = n_dev ? min(*n_dev, n_host) : n_host;
  const long long lo = (long long)blockIdx.x * SN_CHUNK + (long long)threadIdx.x * SN_PER_THREAD;
  long long v[SN_PER_THREAD];
  long long s = 0;
#pragma unroll
  for (int k = 0; k < SN_PER_THREAD; k++) {
    v[k] = lo + k < n ? sn_val(in, lo + k) : 0;
    s += v[k];
  }
  long long tot;
  long long run = part[blockIdx.x] + wg_excl_scan64(s, tmp, &tot);
#pragma unroll
  for (int k = 0; k < SN_PER_THREAD; k++) {
    if (lo + k < n) out[lo + k] = run;
    run += v[k];
  }
}

// first column of every supernode; ns and super_ptr[ns] = n
__global__ void k_sn_ptr(const int* __restrict__ flag, const int* __restrict__ sof, int n,
                         int* sptr, SnCtl* c, int* ns_out) {
  for (int j = gtid(); j < n; j += gsize())
    if (flag[j]) sptr[sof[j]] = j;
  if (gtid() == 0) {
    const int ns = n > 0 ? sof[n - 1] + 1 : 0;
    c->ns = ns;
    sptr[ns] = n;
    if (ns_out) *ns_out = ns;
  }
}

// super_of[j] = (inclusive count of starts up to j) - 1
__global__ void k_sn_of(const int* __restrict__ flag, const long long* __restrict__ excl, int n,
                        int* sof) {
  for (int j = gtid(); j < n; j += gsize()) sof[j] = (int)(excl[j] + flag[j]) - 1;
}

// supernodal tree and dense block sizes (first column's rows x width)
__global__ void k_sn_tree(const int* __restrict__ parent, const int* __restrict__ cc,
                          const int* __restrict__ sptr, const int* __restrict__ sof, int n,
                          const SnCtl* c, int* spar, long long* rw) {
  const int ns = c->ns;
  for (int s = gtid(); s < ns; s += gsize()) {
    const int f = sptr[s], e = sptr[s + 1];
    const int p = parent[e - 1];
    if (spar) spar[s] = p < 0 || p >= n ? -1 : sof[p];
    rw[s] = (long long)cc[f] * (e - f);
  }
}

__global__ void k_sn_status(const SnCtl* c, uint32_t* status) {
  if (gtid() == 0 && status) *status = c->err;
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// workspace: control, nchild, flag, super_of (when the caller gives none),
// 64-bit scratch (exclusive scan of the flags, then rows x width per
// supernode), scan partials
struct SnPlan {
  size_t o_ctl, o_nchild, o_flag, o_sof, o_tmp, o_part, total;
  int nb;
};

SnPlan sn_plan(long long n) {
  SnPlan p;
  size_t o = 0;
  auto take = [&](size_t b) {
    const size_t r = o;
    o = align256(o + b);
    return r;
  };
  const size_t N = (size_t)std::max(n, 1ll);
  p.nb = (int)std::max(1ll, (n + SN_CHUNK - 1) / SN_CHUNK);
  p.o_ctl = take(sizeof(SnCtl));
  p.o_nchild = take(4 * N);
  p.o_flag = take(4 * N);
  p.o_sof = take(4 * N);
  p.o_tmp = take(8 * (N + 1));
  p.o_part = take(8 * (size_t)p.nb);
  p.total = o;
  return p;
}

}  // namespace

extern "C" {

fp_status fp_supernodes_query(int64_t n, size_t* workspace_bytes) {
  if (n < 0 || n >= (1ll << 31) - 1 || !workspace_bytes) return FP_ERR_ARG;
  *workspace_bytes = sn_plan(n).total;
  return FP_OK;
}

fp_status fp_supernodes(fp_handle* h, int64_t n64, const int32_t* parent, const int32_t* colcount,
                        void* workspace, size_t ws_bytes, fp_super_result* out, void* stream) {
  if (!h || !out || n64 < 0 || n64 >= (1ll << 31) - 1) return FP_ERR_ARG;
  if (n64 > 0 && (!parent || !colcount)) return FP_ERR_ARG;
  if (!out->Lp || !out->super_ptr || !out->n_super) return FP_ERR_ARG;
  const SnPlan P = sn_plan(n64);
  if (!workspace || ws_bytes < P.total) return FP_ERR_SIZE;
  const int n = (int)n64;
  char* ws = (char*)workspace;
  SnCtl* c = (SnCtl*)(ws + P.o_ctl);
  int* nchild = (int*)(ws + P.o_nchild);
  int* flag = (int*)(ws + P.o_flag);
  int* sof = out->super_of ? out->super_of : (int*)(ws + P.o_sof);
  int* sptr = out->super_ptr;
  long long* tmp = (long long*)(ws + P.o_tmp);
  long long* part = (long long*)(ws + P.o_part);
  hipStream_t st = (hipStream_t)stream;
  const dim3 T(FP_WG);
  const dim3 G((unsigned)std::max(1ll, std::min<long long>((n64 + FP_WG - 1) / FP_WG, 8ll * h->ncu)));
  const dim3 NB((unsigned)P.nb);

  hipLaunchKernelGGL(k_sn_init, G, T, 0, st, c, nchild, n);
  hipLaunchKernelGGL(k_sn_child, G, T, 0, st, parent, n, nchild, c);
  hipLaunchKernelGGL(k_sn_flag, G, T, 0, st, parent, colcount, nchild, n, flag);
  // super_of from the exclusive scan of the start flags
  hipLaunchKernelGGL(k_scan64_part<int>, NB, T, 0, st, flag, n, nullptr, part);
  hipLaunchKernelGGL(k_scan64_top, dim3(1), T, 0, st, part, P.nb, n, nullptr, tmp);
  hipLaunchKernelGGL(k_scan64_apply<int>, NB, T, 0, st, flag, n, nullptr, part, tmp);
  hipLaunchKernelGGL(k_sn_of, G, T, 0, st, flag, tmp, n, sof);
  hipLaunchKernelGGL(k_sn_ptr, G, T, 0, st, flag, sof, n, sptr, c, out->n_super);
  // column pointers of L
  hipLaunchKernelGGL(k_scan64_part<int>, NB, T, 0, st, colcount, n, nullptr, part);
  hipLaunchKernelGGL(k_scan64_top, dim3(1), T, 0, st, part, P.nb, n, nullptr, (long long*)out->Lp);
  hipLaunchKernelGGL(k_scan64_apply<int>, NB, T, 0, st, colcount, n, nullptr, part,
                     (long long*)out->Lp);
  // supernodal tree, dense block offsets
  hipLaunchKernelGGL(k_sn_tree, G, T, 0, st, parent, colcount, sptr, sof, n, c, out->super_parent,
                     tmp);
  if (out->Lx_ptr) {
    hipLaunchKernelGGL(k_scan64_part<long long>, NB, T, 0, st, tmp, n, &c->ns, part);
    hipLaunchKernelGGL(k_scan64_top, dim3(1), T, 0, st, part, P.nb, n, &c->ns,
                       (long long*)out->Lx_ptr);
    hipLaunchKernelGGL(k_scan64_apply<long long>, NB, T, 0, st, tmp, n, &c->ns, part,
                       (long long*)out->Lx_ptr);
  }
  hipLaunchKernelGGL(k_sn_status, dim3(1), dim3(64), 0, st, c, out->status);
  return hipGetLastError() == hipSuccess ? FP_OK : FP_ERR_HIP;
}

}  // extern "C"
