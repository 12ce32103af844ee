// qmc_persist.h -- host-side launch interface of the persistent segmented step (qmc_persist.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

// Largest packed step table the persistent kernel takes (it keeps the table in LDS); batches
// with larger tables run on the streamed kernels.
constexpr uint32_t kPersistTableBytes = 8192;

struct PersistLaunch {
  const uint64_t* ck;   // canonical store (read at batch start)
  const int2* cv;
  uint64_t* ck_w;       // canonical store (written by the gather)
  int2* cv_w;
  void* counters;
  uint32_t cur;
  uint64_t* sk;         // segments [2][P][segcap]
  int2* sv;
  uint64_t segcap;
  uint32_t* seg_n;      // [2][P]
  uint64_t* ik;         // inboxes [2][P][incap]
  int2* iv;
  uint32_t incap;
  uint32_t* in_n;       // [2][P]
  const uint64_t* split;
  uint64_t* split_w;
  uint32_t P;
  const uint8_t* tab_base;
  const uint32_t* tab_off;  // [nsteps] byte offsets of the step tables
  uint32_t step0, nsteps;
  uint64_t seed;
  uint32_t kbits;
  uint32_t n_replicas;
  const int64_t* qshift;
  uint64_t* slots;      // [P][4] epoch-tagged per-workgroup barrier slots (zeroed once)
  uint64_t epoch0;      // first barrier epoch of the launch
  uint64_t cap_store;
  uint64_t cap_inbox;
  uint32_t rebal_min;
  uint32_t* done;       // [2]
};

extern "C" {
int qmcp_max_segments(int* P);
// Zero the inbox counts and error flags and compute the splitters of the canonical store.
int qmcp_prepare(hipStream_t st, const PersistLaunch* L);
// The cooperative launch of the persistent step kernel (after qmcp_prepare).
int qmcp_launch(hipStream_t st, const PersistLaunch* L);
int qmcp_gather(hipStream_t st, const PersistLaunch* L, uint32_t par);
}
