// fp_mesh.h -- per-mesh job description and workspace layout shared by the
// host API and the device stages.
#pragma once

#include <stdint.h>

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
  int chg;               // fixed-point iteration flag
  int tot;               // scan total
  int task_cnt[8];       // local-order task counts per size class
  int task_pop[8];       // task dispensers
  int arena_top[2];      // element arena bump pointers (ping-pong per level)
  unsigned long long pool_top;  // global fallback pool bump pointer (words)
  long long nnzL;        // sum of vertex column counts
  int site;              // FP_SITE_* of the first failure raised, 0 = none
  int site_arg;          // a value that failure recorded (node, count ...)
  int part[1040];        // scan partials
};

// description of one ordering job; the host fills it and copies it into the
// workspace, kernels read it through a pointer
struct FpMesh {
  // input pattern (device)
  long long n_dof;
  int b;
  const int* rp32;
  const long long* rp64;
  const int* ci_in;
  long long nnz_in;
  const int* user_gmap;
  // options
  int S;
  int lloyd;
  int sched;
  unsigned long long seed;
  // outputs (device; optional ones may be null)
  int* perm;
  int* iperm;
  int* parent;
  int* colcount;
  long long* nnzL;
  int* node_begin_out;
  int* node_size_out;
  int* gmap_out;
  int* n_nodes_out;
  unsigned* status_out;
  int max_nodes_out;
  // sizes
  int n;          // vertices
  long long Ecap; // capacity of the vertex graph
  int NNcap;      // capacity of heap arrays
  int lds_bytes;  // dynamic LDS of the per-node kernels
  int lds_big;    // LDS of the one-wave kernels for large nodes (>= lds_bytes)
  // workspace
  FpCtl* ctl;
  int* grp;       // n+1
  int* gci;       // Ecap
  unsigned long long* key;  // n
  unsigned long long* best; // n
  int* fa;        // n
  int* fcnt;      // n+16: frontier size of every BFS level
  int* fb;        // n
  int* gmap;      // n
  int* seeds;     // n
  int* pcnt;      // n+1
  int* pptr;      // n+1
  int* pvtx;      // n
  int* bnd;       // n
  int* qptr;      // n+1
  int* qci;       // Ecap
  int* qcnt;      // Ecap
  int* wp;        // n
  int* pnode;     // n
  int* plist;     // n
  int* ploc;      // n
  int* node_of;   // n
  int* cand;      // n
  int* bs[10];    // bisection scratch, 2n+2 each
  int* nsize;     // NNcap
  int* nbegin;    // NNcap
  int* ncur;      // NNcap
  int* segS;      // NNcap
  int* segN;      // NNcap
  int* cntL;      // NNcap
  int* cntR;      // NNcap
  int* sbuf;      // NNcap
  int* eoff;      // 3*NNcap: element records: start, ints, records
  int* tasks;     // 8*NNcap
  int* gbuf;      // n
  int* lidx;      // n
  int* vperm;     // n
  int* viperm;    // n
  int* vpar;      // n
  int* vcc;       // n
  int* arena[2];  // element arenas, acap each
  long long acap;
  long long* sdesc;  // NNcap: pool word offset of a node's symbolic scratch, -1 if none
  unsigned* pool; // fallback pool (32-bit words)
  unsigned long long pool_words;
};
