// qmc_persist.h -- host-side launch interface of the persistent segmented step (qmc_persist.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

// Largest packed step table the persistent kernel takes (it keeps the table in LDS); batches
// with larger tables run on the streamed kernels.
constexpr uint32_t kPersistTableBytes = 8192;

struct PersistLaunch {
  uint64_t* ck;         // canonical store (read at batch start, rewritten by a re-split)
  int2* cv;
  uint64_t* pk_prev;    // AB2: N(step0 - 1), sorted, count in counters->n_prev; else null
  int2* pv_prev;        // (a re-split in the kernel rewrites it with N(s))
  void* counters;
  uint32_t cur;
  uint64_t* sk;         // segments [nbuf][P][segcap]
  int2* sv;
  uint64_t segcap;
  uint32_t* seg_n;      // [nbuf][P]
  uint32_t nbuf;        // 2 (Euler) or 3 (AB2: N(s) and N(s-1) survive a failed step)
  uint64_t* ik;         // inboxes [2][P][incap]
  int2* iv;
  uint32_t incap;
  uint32_t* in_n;       // [2][P]
  const uint64_t* split;  // [P] first composite key of each workgroup's range
  uint64_t* split_w;      // the same array, written by the preparation kernel and by the
                          // cost-weighted re-splits inside the fused kernel
  uint32_t P;
  const uint8_t* tab_base;
  const uint32_t* tab_off;   // [nsteps] byte offsets of the step tables (first / only term)
  const uint32_t* tabB_off;  // AB2: [nsteps] offsets of the second-term tables; else null
  uint32_t step0, nsteps;
  uint64_t seed;
  uint32_t kbits;
  uint64_t init_min;    // initiator threshold in walkers (0 = off)
  uint32_t n_circuits;  // circuits of the batch: tab_off holds n_circuits offsets per step
  uint32_t rep_per;     // replicas per circuit (segments = n_circuits * rep_per)
  uint32_t n_replicas;
  const int64_t* qshift;     // per-replica Q32 shifts of the first / only term
  const int64_t* qshiftB;    // AB2: of the second term
  uint64_t* slots;      // [2][P][4] epoch-tagged per-workgroup barrier slots (zeroed once)
  uint64_t epoch0;      // first barrier epoch of the launch
  uint64_t cap_store;
  uint64_t cap_inbox;
  uint32_t rebal_min;
  uint32_t max_rebal;   // re-splits done inside one launch (one circuit); 0: stop instead
  uint32_t* done;       // [2]
};

extern "C" {
int qmcp_max_segments(int* P);
// Zero the inbox counts and error flags and compute the splitters of the canonical store.
int qmcp_prepare(hipStream_t st, const PersistLaunch* L);
// The cooperative launch of the persistent step kernel (after qmcp_prepare).
int qmcp_launch(hipStream_t st, const PersistLaunch* L);
// One empty cooperative launch (the runtime's one-time set-up of cooperative launches).
int qmcp_warm(hipStream_t st);
// Segment buffer `buf` (N(step0 + j) after j steps is in buffer j mod nbuf) -> the sorted store
// (out_k, out_v) with its record count written to *out_count (device pointers).
int qmcp_gather(hipStream_t st, const PersistLaunch* L, uint32_t buf, uint64_t* out_k,
                int2* out_v, uint64_t* out_count);
}
