// fp_handle.h -- the handle behind the C ABI (host side): device properties,
// side streams and their events, stage and kernel timing events, and the
// pinned staging buffer of batched calls.
#pragma once

#include <hip/hip_runtime.h>

#include <mutex>
#include <vector>

#define FP_NSTAGE 8

struct fp_handle;

// a recorded ordering: the graph and its executable form
struct fp_graph {
  hipGraph_t graph;
  hipGraphExec_t exec;
};

// one lane of the request server: a handle of its own and a stream
struct FpLane {
  fp_handle* h;
  hipStream_t st;
};

struct fp_handle {
  int device;
  int ncu;
  int lds_bytes;
  int lds_big;
  int lds_md;     // the local orders' large LDS (tuning; FP_MD_LDS by default)
  int md_per_cu;  // local-order workgroups per CU (tuning; 2 by default)
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
  bool timed;  // the last call recorded stage events
  // kernel timing: events around every launch of the kernel named tk_name
  char tk_name[64];
  std::vector<hipEvent_t> tk_ev;  // pairs (begin, end)
  int tk_n;                       // launches timed in the last call
  bool tk_failed;
  // pinned staging of a batch's mesh descriptions and block tables, and the
  // event after their copy (the buffer is reused once that copy is done)
  void* bstage;
  size_t bstage_cap;
  bool bstage_busy;
  hipEvent_t ev_bstage;
};
