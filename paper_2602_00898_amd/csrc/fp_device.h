// fp_device.h -- device-side building blocks for the gfx950 ordering path:
// wave64 reductions and scans, the team barrier that lets a group of
// co-resident workgroups run one mesh through all stages, and team-wide
// prefix sums.  CDNA4 only (wave64, 160 KiB LDS per CU).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define FP_WG 512                // threads per workgroup of the persistent kernel
#define FP_WAVES (FP_WG / 64)    // waves per workgroup
#define FP_LDS_BYTES (160 * 1024) // dynamic LDS per workgroup (one workgroup per CU)

// error bits raised on the device; surfaced by fp_get_error
#define FP_E_INDEX 0x1u       // column index out of range
#define FP_E_BARRIER 0x2u     // a team barrier timed out
#define FP_E_SCRATCH 0x4u     // a workspace pool overflowed
#define FP_E_GMAP 0x8u        // user group id out of range
#define FP_E_INTERNAL 0x10u   // an internal consistency check failed

#define FP_SPIN_LIMIT (1u << 24)

// debug hook: empty in device builds
#ifndef FP_DBG
#define FP_DBG(...)
#endif
#ifndef FP_DBGP
#define FP_DBGP(...)
#endif

__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }
__device__ __forceinline__ int wave_id() { return threadIdx.x >> 6; }

// ---------------------------------------------------------------- wave64
__device__ __forceinline__ uint32_t wave_min_u32(uint32_t x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x = min(x, (uint32_t)__shfl_xor((int)x, o, 64));
  return x;
}
__device__ __forceinline__ uint32_t wave_max_u32(uint32_t x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x = max(x, (uint32_t)__shfl_xor((int)x, o, 64));
  return x;
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
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
  return x;
}
__device__ __forceinline__ int64_t wave_sum_i64(int64_t x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x += (int64_t)__shfl_xor((long long)x, o, 64);
  return x;
}
// inclusive prefix sum over the wave
__device__ __forceinline__ int wave_incl_scan(int x) {
  const int l = lane_id();
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    int y = __shfl_up(x, o, 64);
    if (l >= o) x += y;
  }
  return x;
}
__device__ __forceinline__ uint64_t ballot64(bool p) { return __ballot(p); }
__device__ __forceinline__ int popc64(uint64_t x) { return __popcll(x); }
__device__ __forceinline__ int popc32(uint32_t x) { return __popc(x); }

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

// ---------------------------------------------------------------- team
// A team is `size` co-resident workgroups that work on one mesh.  sync() is
// a counting barrier with a generation word; an agent-scope fence on both
// sides makes every global store before it visible to every workgroup of the
// team after it, across XCDs.  A barrier that cannot complete within
// FP_SPIN_LIMIT polls raises FP_E_BARRIER and releases the team, so every
// wave exits.
struct Team {
  int rank;
  int size;
  unsigned* bar;  // [0] arrivals, [1] generation
  unsigned* err;  // error bits of the mesh the team works on

  __device__ __forceinline__ int gtid() const { return rank * FP_WG + (int)threadIdx.x; }
  __device__ __forceinline__ int gsize() const { return size * FP_WG; }
  __device__ __forceinline__ int gwave() const { return rank * FP_WAVES + wave_id(); }
  __device__ __forceinline__ int nwaves() const { return size * FP_WAVES; }
  __device__ __forceinline__ bool failed() const {
    return __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & FP_E_BARRIER;
  }

  __device__ void sync() const {
    __syncthreads();
    if (size > 1) {
      if (threadIdx.x == 0 && !(__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & FP_E_BARRIER)) {
        __threadfence();
        unsigned gen = __hip_atomic_load(&bar[1], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
        unsigned a = __hip_atomic_fetch_add(&bar[0], 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        if (a == (unsigned)size - 1) {
          __hip_atomic_store(&bar[0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          __hip_atomic_fetch_add(&bar[1], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        } else {
          unsigned spins = 0;
          while (__hip_atomic_load(&bar[1], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == gen) {
            __builtin_amdgcn_s_sleep(2);
            if (++spins > FP_SPIN_LIMIT ||
                (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & FP_E_BARRIER)) {
              atomicOr(err, FP_E_BARRIER);
              break;
            }
          }
        }
        __threadfence();
      }
      __syncthreads();
    }
  }
};

// team-wide exclusive scan of int32 counts (in place allowed: out may equal
// in).  Workgroup r owns the r-th chunk; chunk sums are exchanged through
// `part` (team.size + 1 ints).  *total (global) receives the sum.  Two team
// barriers.  lds_tmp holds FP_WAVES + 1 ints.
__device__ void team_excl_scan(const Team& T, const int* in, int* out, int n, int* part,
                               int* total, int* lds_tmp) {
  const int chunk = (n + T.size - 1) / T.size;
  const int lo = min(n, T.rank * chunk), hi = min(n, lo + chunk);
  // pass 1: chunk sum
  int s = 0;
  for (int i = lo + (int)threadIdx.x; i < hi; i += FP_WG) s += in[i];
  int tot;
  wg_excl_scan(s, lds_tmp, &tot);
  if (threadIdx.x == 0) part[T.rank] = tot;
  T.sync();
  // pass 2: base of this chunk, then scan the chunk in tiles of FP_WG
  int base = 0, all = 0;
  for (int r = 0; r < T.size; r++) {
    int v = part[r];
    if (r < T.rank) base += v;
    all += v;
  }
  for (int t0 = lo; t0 < hi; t0 += FP_WG) {
    int i = t0 + (int)threadIdx.x;
    int x = i < hi ? in[i] : 0;
    int tt;
    int ex = wg_excl_scan(x, lds_tmp, &tt);
    if (i < hi) out[i] = base + ex;
    base += tt;
  }
  if (T.rank == 0 && threadIdx.x == 0) *total = all;
  T.sync();
}
