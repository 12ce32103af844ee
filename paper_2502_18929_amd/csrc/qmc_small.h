// qmc_small.h -- host-side launch interface of the LDS-resident step for small stores
// (qmc_small.hip): one workgroup per replica, a batch of steps per launch.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

constexpr int kSmallCap = 1024;    // occupied keys of one replica the step holds in LDS
constexpr int kSmallNew = 1024;    // records per replica and step landing on unoccupied keys
constexpr int kSmallStats = 5;     // per-replica statistics: walkers, keys, records, outputs,
                                   // death records (summed over the batch's steps)
constexpr uint32_t kSmallBatch = 64;   // steps per launch of a chain

struct SmallLaunch {
  const uint64_t* ck;       // canonical store, n_store[cur] records of all segments, or null:
  const int2* cv;           //   the input is the segments (ik, iv, in_n)
  void* counters;
  uint32_t cur;
  const uint64_t* ik;       // input segments [n_segments][segcap], counts in_n
  const int2* iv;
  const uint32_t* in_n;
  uint64_t* ok;             // output segments [n_segments][segcap], counts out_n
  int2* ov;
  uint32_t* out_n;
  uint64_t segcap;
  const uint8_t* tab_base;
  const uint32_t* tab_off;  // [nsteps][n_circuits] table offsets
  uint32_t n_circuits, rep_per, n_segments;
  uint32_t step0, nsteps;
  uint64_t seed;
  uint32_t kbits;
  uint64_t init_min;
  const int64_t* qshift;    // per-segment Q32 shifts
  uint64_t cap_store;       // keys per replica allowed (capped at kSmallCap)
  uint64_t cap_spawn;       // records per replica and step allowed
  unsigned long long* stop; // the chain's stop word: (epoch << 32) | ~(first step not taken)
  uint32_t epoch;           // this chain's epoch (distinct from every earlier one, not 0)
  uint64_t* stats;          // [n_segments][kSmallStats] of this batch
};

extern "C" {
// Launches one batch (one workgroup per segment); it does nothing once the chain stopped.
int qmcs_launch(hipStream_t st, const SmallLaunch* L);
// The end of a chain: gathers segments [0, n_segments) (stride segcap, counts seg_n) into the
// canonical store, writes its size to *count and adds nrows rows of per-segment batch statistics
// to the counters, unless the chain of `epoch` stopped (stop == null: always); with stop given it
// also copies the stop word into the counters (Counters::small_stop), so that one read of the
// counters returns both.  n_blocks = 1 (at most 64 segments): one workgroup, and with a mirror
// (device address of host-visible memory, room for a Counters) the workgroup then writes
// a copy of the whole Counters there, which the host reads after the stream synchronization.
int qmcs_finish(hipStream_t st, const uint64_t* sk, const int2* sv, const uint32_t* seg_n,
                uint64_t segcap, uint32_t n_segments, uint64_t* ck, int2* cv, uint64_t* count,
                void* counters, const uint64_t* stats, uint32_t nrows,
                const unsigned long long* stop, uint32_t epoch, uint32_t n_blocks,
                void* mirror);
}
