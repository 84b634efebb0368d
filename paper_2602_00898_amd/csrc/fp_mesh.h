// fp_mesh.h -- per-mesh job description and workspace layout shared by the
// host API and the device stages.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#define FP_GLOBAL __attribute__((address_space(1)))

// A pointer into device global memory.  Element access through it compiles
// to global (not flat) loads and stores: a flat access also counts against
// the LDS counter, so every wait for an LDS result would wait for the
// outstanding global stores as well.  It converts to a plain pointer where
// one is needed.
template <class T>
struct gptr {
  T* p;
  gptr() = default;
  __host__ __device__ constexpr gptr(T* q) : p(q) {}
  template <class U>  // int -> const int and the like
  __host__ __device__ constexpr gptr(gptr<U> o) : p(o.p) {}
  template <class U>  // the same memory seen as another element type
  __host__ __device__ constexpr gptr<U> as() const {
    return gptr<U>((U*)p);
  }
  __host__ __device__ constexpr operator T*() const { return p; }
  __device__ __forceinline__ FP_GLOBAL T& operator[](long long i) const {
    return ((FP_GLOBAL T*)p)[i];
  }
  __device__ __forceinline__ FP_GLOBAL T& operator*() const { return *(FP_GLOBAL T*)p; }
  __device__ __forceinline__ FP_GLOBAL T* operator->() const { return (FP_GLOBAL T*)p; }
  template <class I, class = typename std::enable_if<std::is_integral<I>::value>::type>
  __host__ __device__ constexpr gptr operator+(I i) const {
    return gptr(p + i);
  }
  template <class I, class = typename std::enable_if<std::is_integral<I>::value>::type>
  __host__ __device__ constexpr gptr operator-(I i) const {
    return gptr(p - i);
  }
  __host__ __device__ constexpr long long operator-(gptr o) const { return p - o.p; }
  template <class I>
  __host__ __device__ gptr& operator+=(I i) {
    p += i;
    return *this;
  }
};

// device-scope relaxed atomics on global memory (the semantics of HIP's
// atomicAdd family), taking the pointers that gptr element access yields
template <class T>
__device__ __forceinline__ T atomicAdd(FP_GLOBAL T* p, T v) {
  return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <class T>
__device__ __forceinline__ T atomicSub(FP_GLOBAL T* p, T v) {
  return __hip_atomic_fetch_add(p, (T)(0 - v), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <class T>
__device__ __forceinline__ T atomicOr(FP_GLOBAL T* p, T v) {
  return __hip_atomic_fetch_or(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <class T>
__device__ __forceinline__ T atomicAnd(FP_GLOBAL T* p, T v) {
  return __hip_atomic_fetch_and(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <class T>
__device__ __forceinline__ T atomicMin(FP_GLOBAL T* p, T v) {
  return __hip_atomic_fetch_min(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <class T>
__device__ __forceinline__ T atomicMax(FP_GLOBAL T* p, T v) {
  return __hip_atomic_fetch_max(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <class T>
__device__ __forceinline__ T atomicExch(FP_GLOBAL T* p, T v) {
  return __hip_atomic_exchange(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <class T>
__device__ __forceinline__ T atomicCAS(FP_GLOBAL T* p, T cmp, T v) {
  __hip_atomic_compare_exchange_strong(p, &cmp, v, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
  return cmp;
}

// control block at the start of every mesh workspace (device memory,
// cleared by fp_ctl_init before the pipeline starts)
struct FpCtl {
  unsigned err;          // FP_E_* bits
  int P;                 // patches
  int P0;                // seed blocks
  int D;                 // separator-tree depth
  int nn;                // heap nodes 2^(D+1)-1
  int nnz_g;             // entries of the vertex graph
  int nbnd;              // boundary-list length
  int nq;                // quotient arcs
  int norphan;           // unlabelled vertices after growth
  int nroot;             // orphan components
  int nlong;             // vertex rows of more than FP_ROW_SHORT input entries
  int ccn;               // vertices the orphan-component pass covers (n, or 0 without orphans)
  int vreuse;            // vertices whose local order came from the previous call
  int ccchg[8];          // orphan components: 1 if round r changed a label
  int chg;               // fixed-point iteration flag
  int tot;               // scan total
  int task_cnt[8];       // local-order task counts per size class
  int task_pop[8];       // task dispensers
  int arena_top[2];      // element arena bump pointers (ping-pong per level)
  unsigned long long pool_top;  // global fallback pool bump pointer (words)
  long long nnzL;        // sum of vertex column counts
  int site;              // FP_SITE_* of the first failure raised, 0 = none
  // top separators whose local orders start early: vertex counts, list
  // offsets and cursors in tbuf, first positions (heap index < 8)
  int tcnt[8];
  int tcur[8];
  int toff[8];
  int tpos[8];
  int top_shallow;       // vertices in the top levels placed so far
  int top_stop;          // a top node kept a patch (a leaf): no early orders from its level on
  int tearly[8];         // 1: this top node's local order runs early
  int site_arg;          // a value that failure recorded (node, count ...)
  int part[1040];        // scan partials
};

// description of one ordering job; the host fills it and copies it into the
// workspace, kernels read it through a pointer
struct FpMesh {
  // input pattern (device)
  long long n_dof;
  int b;
  gptr<const int> rp32;
  gptr<const long long> rp64;
  gptr<const int> ci_in;
  long long nnz_in;
  gptr<const int> user_gmap;
  // options
  int S;
  int lloyd;
  int sched;
  unsigned long long seed;
  int validate;   // check that the pattern is symmetric
  int nd_level;   // -1: full tree depth; else at most this many levels
  int dexp;       // expected tree depth (levels past it run in one workgroup)
  int refine;     // separators: 0 one side's candidates, 1 minimum cover
  int amd;        // local orders: 0 exact minimum degree, 1 approximate
  // outputs (device; optional ones may be null)
  gptr<int> perm;
  gptr<int> iperm;
  gptr<int> parent;
  gptr<int> colcount;
  gptr<long long> nnzL;
  gptr<int> node_begin_out;
  gptr<int> node_size_out;
  gptr<int> gmap_out;
  gptr<int> n_nodes_out;
  gptr<unsigned> status_out;
  gptr<int> reused_out;  // vertices whose local order was reused (update calls)
  int max_nodes_out;
  // sizes
  int n;          // vertices
  long long Ecap; // capacity of the vertex graph
  int NNcap;      // capacity of heap arrays
  int lds_bytes;  // dynamic LDS of the per-node kernels
  int lds_big;    // LDS of the one-wave kernels for large nodes (>= lds_bytes)
  int lds_md;     // LDS of the local orders' large classes (<= lds_big)
  // workspace
  gptr<FpCtl> ctl;
  gptr<int> grp;       // n+1
  gptr<int> gci;       // Ecap
  gptr<unsigned long long> key;  // n
  gptr<unsigned long long> best; // n
  gptr<int> fa;        // n
  gptr<int> fcnt;      // n+16: frontier size of every BFS level
  gptr<int> fb;        // n
  gptr<int> gmap;      // n
  gptr<int> seeds;     // n
  gptr<int> pcnt;      // n+1
  gptr<int> pptr;      // n+1
  gptr<int> pvtx;      // n
  gptr<int> bnd;       // n
  gptr<int> qptr;      // n+1
  gptr<int> qci;       // Ecap
  gptr<int> qcnt;      // Ecap
  gptr<int> wp;        // n
  gptr<int> pnode;     // n
  gptr<int> plist;     // n
  gptr<int> ploc;      // n
  gptr<int> node_of;   // n
  gptr<int> cand;      // n
  gptr<int> bs[10];    // bisection scratch, 2n+2 each
  gptr<int> nsize;     // NNcap
  gptr<int> nbegin;    // NNcap
  gptr<int> ncur;      // NNcap
  gptr<int> segS;      // NNcap
  gptr<int> segN;      // NNcap
  gptr<int> cntL;      // NNcap
  gptr<int> cntR;      // NNcap
  gptr<int> sbuf;      // NNcap
  gptr<int> eoff;      // 3*NNcap: element records: start, ints, records
  gptr<int> tasks;     // 8*NNcap
  gptr<int> gbuf;      // n
  gptr<int> lidx;      // n
  gptr<int> vperm;     // n
  gptr<int> viperm;    // n
  gptr<int> vpar;      // n
  gptr<int> vcc;       // n
  gptr<int> arena[2];  // element arenas, acap each
  long long acap;
  gptr<long long> sdesc;  // NNcap: pool word offset of a node's symbolic scratch, -1 if none
  gptr<int> tbuf;      // n: vertex lists of the top separators
  // refined separators: candidates grouped by node, matching and search state
  gptr<int> rlist;     // n: candidates of each node at roff[t]
  gptr<int> mate;      // n: matched partner, -1 if free
  gptr<int> rpar;      // n: search tree: predecessor of a vertex
  gptr<int> seen;      // n: phase stamp of the last search that reached a vertex
  gptr<int> rqa;       // n: search frontiers, at roff[t]
  gptr<int> rqb;       // n
  gptr<int> roff;      // NNcap: first candidate of each node
  gptr<int> rcur;      // NNcap: fill cursor
  gptr<int> prow;      // n+1: the permuted pattern by position: row pointers
  gptr<int> pent;      // Ecap: its entries, as positions
  gptr<unsigned> pool; // fallback pool (32-bit words)
  // update calls: the description of the earlier call whose local orders
  // may be reused (its workspace, unchanged since), else null
  const FpMesh* prev;
  unsigned long long pool_words;
};
