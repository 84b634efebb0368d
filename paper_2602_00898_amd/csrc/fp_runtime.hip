// fp_runtime.hip -- host runtime of the request server declared in
// include/fastperm.h: slots (an internal stream with its own handle) driven
// by host worker threads, and a device-memory arena.  No kernels here:
// every request goes through fp_order on its slot's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/fastperm.h"
#include "fp_handle.h"

namespace {

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

fp_status new_lane(int device, FpLane* L) {
  if (hipSetDevice(device) != hipSuccess) return FP_ERR_HIP;
  fp_handle* h = nullptr;
  fp_status s = fp_create(&h);
  if (s != FP_OK) return s;
  hipStream_t st = nullptr;
  if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
    fp_destroy(h);
    return FP_ERR_HIP;
  }
  h->side_ok = false;  // slots run side by side already
  L->h = h;
  L->st = st;
  return FP_OK;
}

void free_lane(FpLane& L) {
  (void)hipStreamSynchronize(L.st);
  (void)hipStreamDestroy(L.st);
  (void)fp_destroy(L.h);
}

}  // namespace

// ===========================================================================
// request server
// ===========================================================================
namespace {

struct FpRequest {
  uint64_t ticket;
  fp_host_csr A;
  fp_options o;
  size_t ws_bytes;
  size_t bytes;  // device footprint
  size_t off;    // offset in the arena while in flight
  std::chrono::steady_clock::time_point t_submit, t_done;
  int bypassed;  // later requests admitted ahead of this one
  bool done;
  fp_status status;
  int64_t nnzL;
  std::vector<int32_t> perm, iperm, parent, colcount;
};

// first-fit allocator over [0, size) in 256-byte units
struct FpArena {
  std::map<size_t, size_t> free_blocks;  // offset -> bytes
  void init(size_t size) {
    free_blocks.clear();
    if (size) free_blocks[0] = size;
  }
  bool alloc(size_t bytes, size_t* off) {
    for (auto it = free_blocks.begin(); it != free_blocks.end(); ++it) {
      if (it->second < bytes) continue;
      *off = it->first;
      const size_t rest = it->second - bytes;
      const size_t o2 = it->first + bytes;
      free_blocks.erase(it);
      if (rest) free_blocks[o2] = rest;
      return true;
    }
    return false;
  }
  bool fits(size_t bytes) const {
    for (const auto& b : free_blocks)
      if (b.second >= bytes) return true;
    return false;
  }
  void release(size_t off, size_t bytes) {
    auto it = free_blocks.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != free_blocks.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_blocks.erase(nx);
    }
    if (it != free_blocks.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_blocks.erase(it);
      }
    }
  }
};

size_t request_bytes(const fp_host_csr& A, size_t ws) {
  const size_t n = (size_t)A.n;
  return align256(8 * (n + 1)) + align256(4 * (size_t)std::max<int64_t>(A.nnz, 1)) + align256(ws) +
         4 * align256(4 * std::max<size_t>(n, 1)) + 3 * 256;
}

}  // namespace

struct fp_server {
  fp_handle* h;
  int device;
  size_t budget;
  char* arena_mem;
  FpArena arena;
  std::vector<FpLane> lanes;
  std::mutex mu;
  std::condition_variable cv;
  std::deque<FpRequest*> queue;
  std::unordered_map<uint64_t, FpRequest*> reqs;
  uint64_t next_ticket;
  bool stop;
  std::vector<std::thread> workers;
};

namespace {

// Admission: the oldest request that fits, looking at most FP_BYPASS_WINDOW
// requests deep; a request that has been passed FP_BYPASS_MAX times blocks
// every later one until it fits (so a large request waits for memory to
// free up, but small ones need not queue behind it meanwhile).  Returns the
// queue index to admit, or -1.  Called under the server lock.
#define FP_BYPASS_WINDOW 64
#define FP_BYPASS_MAX 32
int pick_request(fp_server* S) {
  const size_t lim = std::min<size_t>(S->queue.size(), FP_BYPASS_WINDOW);
  for (size_t i = 0; i < lim; i++) {
    FpRequest* r = S->queue[i];
    if (S->arena.fits(r->bytes)) return (int)i;
    if (r->bypassed >= FP_BYPASS_MAX) return -1;  // no one passes it any more
  }
  return -1;
}

// one slot: admit a request (pick_request), order it on this slot's lane,
// copy the results back, release the memory
void server_worker(fp_server* S, int w) {
  FpLane& L = S->lanes[w];
  const bool dev_ok = hipSetDevice(S->device) == hipSuccess;
  while (true) {
    FpRequest* r = nullptr;
    {
      std::unique_lock<std::mutex> lk(S->mu);
      int at = -1;
      S->cv.wait(lk, [&] {
        if (S->stop && S->queue.empty()) return true;
        at = S->queue.empty() ? -1 : pick_request(S);
        return at >= 0;
      });
      if (at < 0) return;  // stopping
      r = S->queue[at];
      if (!S->arena.alloc(r->bytes, &r->off)) continue;  // cannot happen: it fit under the lock
      for (int i = 0; i < at; i++) S->queue[i]->bypassed++;
      S->queue.erase(S->queue.begin() + at);
    }
    fp_status st = dev_ok ? FP_OK : FP_ERR_HIP;
    const size_t n = (size_t)r->A.n, nnz = (size_t)std::max<int64_t>(r->A.nnz, 0);
    char* p = S->arena_mem + r->off;
    int64_t* d_rp = (int64_t*)p;
    p += align256(8 * (n + 1));
    int32_t* d_ci = (int32_t*)p;
    p += align256(4 * std::max<size_t>(nnz, 1));
    void* ws = p;
    p += align256(r->ws_bytes);
    int32_t* d_out[4];
    for (int k = 0; k < 4; k++) {
      d_out[k] = (int32_t*)p;
      p += align256(4 * std::max<size_t>(n, 1));
    }
    int64_t* d_nnzL = (int64_t*)p;
    p += 256;
    uint32_t* d_status = (uint32_t*)p;
    if (st == FP_OK &&
        (hipMemcpyAsync(d_rp, r->A.rowptr, 8 * (n + 1), hipMemcpyHostToDevice, L.st) != hipSuccess ||
         (nnz && hipMemcpyAsync(d_ci, r->A.colind, 4 * nnz, hipMemcpyHostToDevice, L.st) !=
                     hipSuccess)))
      st = FP_ERR_HIP;
    if (st == FP_OK) {
      fp_csr dA{r->A.n, r->A.nnz, nullptr, d_rp, nnz ? d_ci : nullptr};
      fp_result R{d_out[0], d_out[1], d_out[2], d_out[3], d_nnzL, nullptr, nullptr, nullptr,
                  nullptr, d_status, 0};
      st = fp_order(L.h, &dA, nullptr, &r->o, ws, r->ws_bytes, &R, L.st);
      if (st == FP_OK) st = fp_last_error(L.h, ws, L.st);
    }
    if (st == FP_OK) {
      r->perm.resize(n);
      r->iperm.resize(n);
      r->parent.resize(n);
      r->colcount.resize(n);
      int32_t* dst[4] = {r->perm.data(), r->iperm.data(), r->parent.data(), r->colcount.data()};
      for (int k = 0; k < 4 && st == FP_OK; k++)
        if (n && hipMemcpyAsync(dst[k], d_out[k], 4 * n, hipMemcpyDeviceToHost, L.st) != hipSuccess)
          st = FP_ERR_HIP;
      if (st == FP_OK &&
          (hipMemcpyAsync(&r->nnzL, d_nnzL, 8, hipMemcpyDeviceToHost, L.st) != hipSuccess ||
           hipStreamSynchronize(L.st) != hipSuccess))
        st = FP_ERR_HIP;
    } else {
      (void)hipStreamSynchronize(L.st);
    }
    {
      std::lock_guard<std::mutex> g(S->mu);
      S->arena.release(r->off, r->bytes);
      r->status = st;
      r->t_done = std::chrono::steady_clock::now();
      r->done = true;
    }
    S->cv.notify_all();
  }
}

}  // namespace

extern "C" {

fp_status fp_server_create(fp_handle* h, size_t hbm_budget, int32_t max_slots, fp_server** s) {
  if (!h || !s || max_slots < 1 || max_slots > 64 || hbm_budget < 4096) return FP_ERR_ARG;
  *s = nullptr;
  fp_server* S = new (std::nothrow) fp_server();
  if (!S) return FP_ERR_OOM;
  S->h = h;
  S->device = h->device;
  S->budget = hbm_budget & ~(size_t)255;
  S->next_ticket = 1;
  S->stop = false;
  if (hipSetDevice(S->device) != hipSuccess) {
    delete S;
    return FP_ERR_HIP;
  }
  if (hipMalloc((void**)&S->arena_mem, S->budget) != hipSuccess) {
    delete S;
    return FP_ERR_OOM;
  }
  S->arena.init(S->budget);
  for (int w = 0; w < max_slots; w++) {
    FpLane L;
    fp_status st = new_lane(S->device, &L);
    if (st != FP_OK) {
      for (FpLane& x : S->lanes) free_lane(x);
      (void)hipFree(S->arena_mem);
      delete S;
      return st;
    }
    S->lanes.push_back(L);
  }
  for (int w = 0; w < max_slots; w++) S->workers.emplace_back(server_worker, S, w);
  *s = S;
  return FP_OK;
}

fp_status fp_server_submit(fp_server* S, const fp_host_csr* A, const fp_options* opts,
                           uint64_t* ticket) {
  if (!S || !A || !opts || !ticket || A->n < 0 || A->nnz < 0 || !A->rowptr ||
      (A->nnz > 0 && !A->colind))
    return FP_ERR_ARG;
  fp_csr probe{A->n, A->nnz, nullptr, (const int64_t*)A->rowptr, A->colind};
  size_t ws = 0;
  fp_status st = fp_query(S->h, &probe, opts, &ws, nullptr);
  if (st != FP_OK) return st;
  FpRequest* r = new (std::nothrow) FpRequest();
  if (!r) return FP_ERR_OOM;
  r->A = *A;
  r->o = *opts;
  r->o.flags &= ~FP_FLAG_TIMING;  // no per-stage timing inside the server
  r->ws_bytes = ws;
  r->bytes = request_bytes(*A, ws);
  r->done = false;
  r->bypassed = 0;
  r->status = FP_OK;
  r->nnzL = 0;
  if (r->bytes > S->budget) {
    delete r;
    return FP_ERR_BUSY;
  }
  {
    std::lock_guard<std::mutex> g(S->mu);
    if (S->stop) {
      delete r;
      return FP_ERR_ARG;
    }
    r->ticket = S->next_ticket++;
    r->t_submit = std::chrono::steady_clock::now();
    S->reqs[r->ticket] = r;
    S->queue.push_back(r);
    *ticket = r->ticket;
  }
  S->cv.notify_all();
  return FP_OK;
}

fp_status fp_server_test(fp_server* S, uint64_t ticket, int32_t* done) {
  if (!S || !done) return FP_ERR_ARG;
  std::lock_guard<std::mutex> g(S->mu);
  auto it = S->reqs.find(ticket);
  if (it == S->reqs.end()) return FP_ERR_ARG;
  *done = it->second->done ? 1 : 0;
  return FP_OK;
}

fp_status fp_server_wait(fp_server* S, uint64_t ticket, int32_t* perm, int32_t* iperm,
                         int32_t* parent, int32_t* colcount, int64_t* nnzL, double* latency_s) {
  if (!S) return FP_ERR_ARG;
  FpRequest* r = nullptr;
  {
    std::unique_lock<std::mutex> lk(S->mu);
    auto it = S->reqs.find(ticket);
    if (it == S->reqs.end()) return FP_ERR_ARG;
    r = it->second;
    S->cv.wait(lk, [&] { return r->done; });
    S->reqs.erase(it);
  }
  const fp_status st = r->status;
  if (st == FP_OK) {
    const size_t n = (size_t)r->A.n;
    if (perm) memcpy(perm, r->perm.data(), 4 * n);
    if (iperm) memcpy(iperm, r->iperm.data(), 4 * n);
    if (parent) memcpy(parent, r->parent.data(), 4 * n);
    if (colcount) memcpy(colcount, r->colcount.data(), 4 * n);
    if (nnzL) *nnzL = r->nnzL;
  }
  if (latency_s) latency_s[0] = std::chrono::duration<double>(r->t_done - r->t_submit).count();
  delete r;
  return st;
}

fp_status fp_server_destroy(fp_server* S) {
  if (!S) return FP_OK;
  {
    std::lock_guard<std::mutex> g(S->mu);
    S->stop = true;
  }
  S->cv.notify_all();
  for (auto& t : S->workers) t.join();
  for (FpLane& L : S->lanes) free_lane(L);
  for (auto& kv : S->reqs) delete kv.second;
  (void)hipFree(S->arena_mem);
  delete S;
  return FP_OK;
}

}  // extern "C"
