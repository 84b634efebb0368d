// fp_handle.h -- the handle behind the C ABI (host side): device properties,
// the pinned buffer scalars are read through, stage timing events, and the
// lanes (internal streams with their own handles) of the batched and served
// calls.
#pragma once

#include <hip/hip_runtime.h>

#include <mutex>
#include <vector>

#define FP_NSTAGE 8

struct fp_handle;

// one lane: a handle of its own (pinned buffer, events) and a stream
struct FpLane {
  fp_handle* h;
  hipStream_t st;
};

struct fp_handle {
  int device;
  int ncu;
  int lds_bytes;
  int lds_big;
  int lds_md;  // the local orders' large LDS (at most FP_MD_LDS)
  int* host;  // pinned: scalars read back between stages, and the job copy
  // second stream: local orders of the top separators, started while the
  // separator tree is still being built; events order it after the call's
  // stream and back
  hipStream_t side;
  hipStream_t side2;  // the two large size classes of the local orders,
  hipStream_t side3;  // one stream each
  hipEvent_t ev_md;
  hipEvent_t ev_join2;
  hipEvent_t ev_join3;
  bool side_ok;  // off for the lanes of batched and served calls: they overlap already
  hipEvent_t ev_top[3];
  hipEvent_t ev_join;
  hipEvent_t ev[FP_NSTAGE + 1];
  hipEvent_t ev_bfs;  // a BFS frontier size has reached the host buffer
  bool timed;  // the last call recorded stage events
  std::mutex lanes_mu;
  std::vector<FpLane> lanes;  // created on demand by the batched calls
  // kernel timing: events around every launch of the kernel named tk_name
  char tk_name[64];
  std::vector<hipEvent_t> tk_ev;  // pairs (begin, end)
  int tk_n;                       // launches timed in the last call
  bool tk_failed;
};
