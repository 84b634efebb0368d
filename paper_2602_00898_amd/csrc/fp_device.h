// fp_device.h -- device-side building blocks for the gfx950 ordering path:
// wave64 reductions and scans and workgroup scans.  CDNA4 only (wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define FP_WG 256                // threads per workgroup
#define FP_WAVES (FP_WG / 64)    // waves per workgroup
#define FP_LDS_BYTES (64 * 1024) // dynamic LDS of the per-node kernels
// large LDS of the local orders: two such workgroups share a CU, which
// measured faster than one wave per CU holding the whole 160 KB
#define FP_MD_LDS (64 * 1024)
#define FP_TOP_LEVELS 3          // tree levels whose separators are ordered early (at most 3)

// error bits raised on the device; surfaced by fp_get_error
#define FP_E_INDEX 0x1u       // column index out of range
#define FP_E_SCRATCH 0x4u     // a workspace pool overflowed
#define FP_E_GMAP 0x8u        // user group id out of range
#define FP_E_INTERNAL 0x10u   // an internal consistency check failed
#define FP_E_ASYM 0x20u       // the pattern is not symmetric (validation)

// where a failure was raised (the first one is kept with one value)
enum {
  FP_SITE_NONE = 0,
  FP_SITE_INGEST = 1,       // column index / row pointer out of range
  FP_SITE_GMAP_LABEL = 2,   // a vertex left without a patch
  FP_SITE_USER_GMAP = 3,    // user group id out of range
  FP_SITE_BISECT_PATCH = 4, // patch id out of range in a node's list
  FP_SITE_BISECT_SPLIT = 5, // split counts disagree with the split point
  FP_SITE_NODE_OF = 6,      // vertex assigned to no valid node
  FP_SITE_MD_VERTEX = 7,    // node vertex list holds a foreign vertex
  FP_SITE_MD_POOL = 8,      // fallback pool exhausted
  FP_SITE_MD_MAXM = 9,      // node beyond 16-bit local ids
  FP_SITE_MD_PIVOT = 10,    // no valid pivot (dense layout)
  FP_SITE_MD_PIVOT_SP = 11, // no valid pivot (sparse layout)
  FP_SITE_SYM_VERTEX = 12,  // position list holds a vertex out of range
  FP_SITE_SYM_RECORD = 13,  // child element record out of range
  FP_SITE_SYM_ARENA = 14,   // element arena full
  FP_SITE_SYM_SLOTS = 15,   // element slots exhausted even in the pool
  FP_SITE_OUT_NODES = 16,   // node_begin/node_size capacity too small
  FP_SITE_SYM_LOOKUP = 17,  // a later position missing from the node's list
  FP_SITE_SYM_ROWS = 18,    // forward-row pointers out of order
  FP_SITE_SYM_LIVE = 19,    // element slot or list index out of range
  FP_SITE_SYM_PIVOT = 20,   // parent position outside the node's index space
  FP_SITE_TOP = 21,         // early top-separator range differs from the schedule's
  FP_SITE_ASYM = 22,        // entry (v, u) without its mirror (u, v); the value is v
  FP_SITE_GRAPH = 23,       // vertex graph larger than its capacity
  FP_SITE_QARCS = 24,       // quotient graph larger than its capacity
  FP_SITE_TREE = 25,        // separator tree larger than its capacity
  FP_SITE_REFINE = 26,      // separator refinement past its phase bound
};

// the dynamic LDS array of every kernel that uses one
#define FP_LDS_DECL extern __shared__ __align__(16) char fp_lds[]

// A value every lane of the wave holds alike (a node id, a size read from
// memory at one address), moved into a scalar register.  The compiler treats
// whatever a vector load returns as varying per lane; loops and branches on
// such values then run under exec masks with vector counters.  Passing them
// through readfirstlane makes them scalar, and the loops scalar too.
__device__ __forceinline__ int uni(int x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ __forceinline__ unsigned uni(unsigned x) {
  return (unsigned)__builtin_amdgcn_readfirstlane((int)x);
}
__device__ __forceinline__ long long uni(long long x) {
  const unsigned lo = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)x);
  const unsigned hi = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)((unsigned long long)x >> 32));
  return (long long)(((unsigned long long)hi << 32) | lo);
}

__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }
__device__ __forceinline__ int wave_id() { return threadIdx.x >> 6; }

// Orders memory operations between the lanes of one wave (code where a wave
// owns its data: the per-node stages).  The lanes of a wave issue their
// memory operations together and in program order, so this scope needs no
// wait for outstanding stores, unlike a workgroup fence.
__device__ __forceinline__ void wave_fence() { __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront"); }

// Waits until every vector memory operation the wave has issued is done
// (vmcnt 0; expcnt and lgkmcnt left alone).  Placed right after loads whose
// registers a loop reads many times: the compiler then knows they have
// arrived, instead of waiting for every outstanding load and store (a
// store's completion takes hundreds of cycles) at each use in the loop.
__device__ __forceinline__ void vm_wait() { __builtin_amdgcn_s_waitcnt(0x0F70); }

// ---------------------------------------------------------------- wave64
// Reductions and scans run on DPP row shifts (within each 16-lane row,
// register to register) and combine the four rows through readlane, instead
// of LDS-routed lane permutes.  All lanes of the wave must be active.
// Value of `x` in lane `l` (l the same in every lane), broadcast to all.
__device__ __forceinline__ int wave_bcast(int x, int l) { return __builtin_amdgcn_readlane(x, l); }
__device__ __forceinline__ uint32_t wave_bcast_u32(uint32_t x, int l) {
  return (uint32_t)__builtin_amdgcn_readlane((int)x, l);
}
// row_shr:n of x, `fill` where the source lane is before the row start
__device__ __forceinline__ int dpp_shr(int x, int fill, int n) {
  switch (n) {
    case 1: return __builtin_amdgcn_update_dpp(fill, x, 0x111, 0xf, 0xf, false);
    case 2: return __builtin_amdgcn_update_dpp(fill, x, 0x112, 0xf, 0xf, false);
    case 4: return __builtin_amdgcn_update_dpp(fill, x, 0x114, 0xf, 0xf, false);
    default: return __builtin_amdgcn_update_dpp(fill, x, 0x118, 0xf, 0xf, false);
  }
}
__device__ __forceinline__ uint32_t wave_min_u32(uint32_t x) {
  const int I = -1;  // 0xFFFFFFFF, the identity of the unsigned minimum
  x = min(x, (uint32_t)dpp_shr((int)x, I, 1));
  x = min(x, (uint32_t)dpp_shr((int)x, I, 2));
  x = min(x, (uint32_t)dpp_shr((int)x, I, 4));
  x = min(x, (uint32_t)dpp_shr((int)x, I, 8));
  // lane 15 of each row now holds the row's minimum
  const uint32_t a = min(wave_bcast_u32(x, 15), wave_bcast_u32(x, 31));
  const uint32_t b = min(wave_bcast_u32(x, 47), wave_bcast_u32(x, 63));
  return min(a, b);
}
__device__ __forceinline__ uint32_t wave_max_u32(uint32_t x) {
  x = max(x, (uint32_t)dpp_shr((int)x, 0, 1));
  x = max(x, (uint32_t)dpp_shr((int)x, 0, 2));
  x = max(x, (uint32_t)dpp_shr((int)x, 0, 4));
  x = max(x, (uint32_t)dpp_shr((int)x, 0, 8));
  const uint32_t a = max(wave_bcast_u32(x, 15), wave_bcast_u32(x, 31));
  const uint32_t b = max(wave_bcast_u32(x, 47), wave_bcast_u32(x, 63));
  return max(a, b);
}
__device__ __forceinline__ uint64_t wave_min_u64(uint64_t x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    uint64_t y = __shfl_xor((unsigned long long)x, o, 64);
    x = y < x ? y : x;
  }
  return x;
}
__device__ __forceinline__ uint64_t wave_max_u64(uint64_t x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    uint64_t y = __shfl_xor((unsigned long long)x, o, 64);
    x = y > x ? y : x;
  }
  return x;
}
__device__ __forceinline__ int wave_sum_i32(int x) {
  x += dpp_shr(x, 0, 1);
  x += dpp_shr(x, 0, 2);
  x += dpp_shr(x, 0, 4);
  x += dpp_shr(x, 0, 8);
  return (wave_bcast(x, 15) + wave_bcast(x, 31)) + (wave_bcast(x, 47) + wave_bcast(x, 63));
}
__device__ __forceinline__ int64_t wave_sum_i64(int64_t x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x += (int64_t)__shfl_xor((long long)x, o, 64);
  return x;
}
// inclusive prefix sum over the wave: scans of the 16-lane rows, then the
// totals of the rows before
__device__ __forceinline__ int wave_incl_scan(int x) {
  x += dpp_shr(x, 0, 1);
  x += dpp_shr(x, 0, 2);
  x += dpp_shr(x, 0, 4);
  x += dpp_shr(x, 0, 8);
  const int t0 = wave_bcast(x, 15), t1 = wave_bcast(x, 31), t2 = wave_bcast(x, 47);
  const int row = lane_id() >> 4;
  return x + (row > 0 ? t0 : 0) + (row > 1 ? t1 : 0) + (row > 2 ? t2 : 0);
}
__device__ __forceinline__ uint64_t ballot64(bool p) { return __ballot(p); }
__device__ __forceinline__ int popc64(uint64_t x) { return __popcll(x); }
__device__ __forceinline__ int popc32(uint32_t x) { return __popc(x); }
__device__ __forceinline__ uint64_t lanemask_lt() {
  const int l = lane_id();
  return l ? (~0ull >> (64 - l)) : 0ull;
}

// Append to a list whose length is *ctr: one atomic per wave instead of one
// per item.  Call with the whole wave; returns the slot of a lane with `pred`.
template <class P>
__device__ __forceinline__ int wave_append(P ctr, bool pred) {
  const uint64_t bal = ballot64(pred);
  int base = 0;
  if (bal) {
    const int leader = __builtin_ctzll(bal);
    if (lane_id() == leader) base = atomicAdd(ctr, (int)popc64(bal));
    base = wave_bcast(base, leader);
  }
  return base + popc64(bal & lanemask_lt());
}

// Append for a whole workgroup: one global atomic per workgroup and call.
// Every thread of the workgroup must call it (a barrier inside); lds2 is two
// ints of LDS the workgroup owns.
template <class P>
__device__ __forceinline__ int wg_append(P ctr, bool pred, int* lds2) {
  const uint64_t bal = ballot64(pred);
  const int c = popc64(bal);
  if (threadIdx.x == 0) lds2[0] = 0;
  __syncthreads();
  int off = 0;
  if (lane_id() == 0 && c) off = atomicAdd(&lds2[0], c);
  off = wave_bcast(off, 0);
  __syncthreads();
  if (threadIdx.x == 0) lds2[1] = lds2[0] ? atomicAdd(ctr, lds2[0]) : 0;
  __syncthreads();
  const int base = lds2[1];
  __syncthreads();  // lds2 is free again for the next call
  return base + off + popc64(bal & lanemask_lt());
}

// Same for per-key counters ctr[key]: one atomic per distinct key present
// in the wave (mesh vertices of a wave mostly share a few patches or nodes).
template <class P>
__device__ __forceinline__ int wave_append_keyed(P ctr, int key, bool pred) {
  uint64_t pending = ballot64(pred);
  int slot = 0;
  while (pending) {
    const int leader = __builtin_ctzll(pending);
    const int lk = wave_bcast(key, leader);
    const uint64_t grp = ballot64(pred && key == lk) & pending;
    int base = 0;
    if (lane_id() == leader) base = atomicAdd(&ctr[lk], (int)popc64(grp));
    base = wave_bcast(base, leader);
    if ((grp >> lane_id()) & 1ull) slot = base + popc64(grp & lanemask_lt());
    pending &= ~grp;
  }
  return slot;
}

// ---------------------------------------------------------------- workgroup
// exclusive scan of one value per thread over the workgroup; returns the
// exclusive prefix, *total receives the sum.  `tmp` holds FP_WAVES ints.
__device__ __forceinline__ int wg_excl_scan(int x, int* tmp, int* total) {
  int inc = wave_incl_scan(x);
  if (lane_id() == 63) tmp[wave_id()] = inc;
  __syncthreads();
  int base = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < FP_WAVES; w++) {
    int v = tmp[w];
    if (w < wave_id()) base += v;
    tot += v;
  }
  __syncthreads();
  if (total) *total = tot;
  return base + inc - x;
}

__device__ __forceinline__ int64_t wg_sum_i64(int64_t x, int64_t* tmp) {
  x = wave_sum_i64(x);
  if (lane_id() == 0) tmp[wave_id()] = x;
  __syncthreads();
  int64_t s = 0;
#pragma unroll
  for (int w = 0; w < FP_WAVES; w++) s += tmp[w];
  __syncthreads();
  return s;
}

// grid-stride helpers of the one-thread-per-item kernels
__device__ __forceinline__ int gtid() { return (int)(blockIdx.x * blockDim.x + threadIdx.x); }
__device__ __forceinline__ int gsize() { return (int)(gridDim.x * blockDim.x); }
__device__ __forceinline__ int gwave() { return uni((int)((blockIdx.x * blockDim.x + threadIdx.x) >> 6)); }
__device__ __forceinline__ int nwaves() { return (int)((gridDim.x * blockDim.x) >> 6); }
