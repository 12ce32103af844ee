// qmc_kernels.h -- host-callable launch wrappers of the HIP kernels in qmc_kernels.hip.
// Every wrapper enqueues on the given stream and returns the hipError_t of the launch.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

// Spawn proposal (End Matter, spawn step: the multinomial over a column's (target, Re/Im)
// channels, importance weighted): kind 0 = the comb (no proposal), 1 uniform, 2 heat-bath, 3 the
// int8 MLP scores of the key bits, 4 the deeper int8 network of the key bits and the step's
// active weight channels; k samples per parent (a power of two).  Kind 3: sizes
// kPropIn x kPropHidden x kPropOut (w1 [hidden][in], w2 [out][hidden]).  Kind 4: kDeepIn inputs,
// two layers of kDeepHidden units, kDeepOut scores (w1 [hidden][in], w2 [hidden][hidden],
// w3 [out][hidden]).  Weights in device memory.
constexpr int kPropIn = 64, kPropHidden = 32, kPropOut = 64;
constexpr int kDeepIn = 128, kDeepHidden = 128, kDeepOut = 64;
struct QmcProposal {
  uint32_t kind;
  uint32_t k;
  uint32_t nbits;   // key bits fed to the network (2n)
  uint32_t s1;      // first hidden layer's shift
  const int8_t* w1;
  const int32_t* b1;
  const int8_t* w2;
  const int32_t* b2;
  const int8_t* w3;   // kind 4: output layer, and the second hidden layer's shift
  const int32_t* b3;
  uint32_t s2;
  // Spawn-event log of the plain comb (null: off): every nonzero off-diagonal child drawn is
  // appended as one event while fewer than log_cap are stored; *log_count counts them all.
  struct SpawnEvent* log;
  uint64_t log_cap;
  unsigned long long* log_count;
};
// One logged spawn: the parent's composite key, the step, the column group, the child's counts.
struct SpawnEvent {
  uint64_t key;
  uint32_t step;
  uint32_t group;
  int32_t re;
  int32_t im;
};
static_assert(sizeof(SpawnEvent) == 24, "24-byte events");

extern "C" {
uint32_t qmck_sort_passes(uint32_t key_bits);
int qmck_batch_begin(hipStream_t st, void* counters, uint64_t* status, uint64_t n_status,
                     uint64_t* sort_status, uint64_t n_sort_status, uint32_t* ghist,
                     uint32_t n_ghist);
// Records of step `step` from the n = *count parents (pk, pv), Philox stream `stream`: the death
// delta of each parent (diagonal of its column plus the per-replica Q32 shift qsh) and its
// children, appended at n_child[step & 1] with the digit histograms of their sort in ghist.  init_min > 0: initiator approximation, record keys carry the non-initiator flag
// below the composite key.
// The tables are tab_base + tab_off[c] for circuit c (rep_per replicas per circuit).
int qmck_spawn(hipStream_t st, const uint64_t* pk, const int2* pv, void* counters,
               const uint64_t* count, const uint8_t* tab_base, const uint32_t* tab_off,
               uint32_t rep_per, uint32_t step, uint64_t seed,
               uint32_t kbits, uint64_t init_min, uint32_t stream, const int64_t* qsh,
               uint64_t* ck, int2* cv, uint64_t cap_child, uint64_t max_parents, uint32_t* ghist,
               uint32_t passes, const QmcProposal* prop);
int qmck_digit_hist(hipStream_t st, const uint64_t* keys, void* counters, uint32_t nsel,
                    uint32_t passes, uint32_t* ghist, uint64_t max_items);
int qmck_sort(hipStream_t st, uint64_t* k0, int2* v0, uint64_t* k1, int2* v1, void* counters,
              uint32_t nsel, uint32_t passes, const uint32_t* ghist, uint64_t* sort_status,
              uint32_t step, uint32_t src, uint64_t max_items, uint32_t ipt);
// The same sort of one step's records without look-back (per-tile digit counts, a scan over
// tiles and a scatter per pass); hist_a and hist_b hold qmck_step_sort_hist_words(max_items)
// words each and need no initial contents.  The result lands in pair src ^ (passes & 1).
uint64_t qmck_step_sort_hist_words(uint64_t max_items);
int qmck_sort_step(hipStream_t st, uint64_t* k0, int2* v0, uint64_t* k1, int2* v1, void* counters,
                   uint32_t nsel, uint32_t passes, const uint32_t* ghist, uint32_t* hist_a,
                   uint32_t* hist_b, uint32_t step, uint32_t src, uint64_t max_items);
// Records per thread of a sort tile that qmck_sort supports (8, 12, 16, 24): nonzero if ok.
int qmck_sort_tile_ok(uint32_t ipt);
// n synthetic records (keys masked to `mask`, values (1, 0)) for timing the sort.
int qmck_fill_sort_probe(hipStream_t st, uint64_t* k, int2* v, uint64_t n, uint64_t mask,
                         uint64_t salt);
// Annihilation of step `step`: the parents (pk, pv) (n_store[cur]) merged with the sorted
// records (ck, cv) (n_child[csel]) into the new store (ok, ov), whose size goes to
// n_store[cur ^ 1]: tile split points (splits, max tiles + 1), tile output counts and offsets
// (tile_off: max tiles words, max tiles / 256 + 1 words of block offsets, then max tiles + 1
// int32 count adjustments, which must hold zeros on entry and hold zeros again on return),
// with mpos (room for max_items - cap_store words) the records' merged positions, then the
// tiles; sidx holds the parents' search index on entry and the new store's on return.  Also clears the next step's record counter
// and digit histograms (ghist_next), which the records of step + 1 (qmck_spawn) fill.  With
// toff_next (the tables of step + 1 for circuit c at tab_base + toff_next[c], shifts qshift),
// every new store record whose comb can fire in step + 1 (Philox stream 0) is appended to
// (act_k, act_v) (room for cap_store records; their number in Counters::n_active), the parents
// a qmck_spawn of step + 1 draws from.
int qmck_merge(hipStream_t st, const uint64_t* pk, const int2* pv, const uint64_t* ck,
               const int2* cv, void* counters, uint32_t cur, uint32_t csel, uint2* splits,
               uint64_t* tile_off, uint32_t step, uint32_t kbits, uint64_t init_min, uint64_t* ok,
               int2* ov, uint64_t cap_store, uint64_t max_items, uint32_t* ghist_next,
               const uint8_t* tab_base, const uint32_t* toff_next, uint32_t rep_per,
               const int64_t* qshift, uint64_t seed, uint64_t* act_k, int2* act_v,
               uint32_t* mpos, uint64_t* sidx);
// The search index of the sorted keys[0, *count): sidx[i] = keys[256 i] (room for
// max_items / 256 + 1 words).  qmck_merge reads the index of its parents from sidx (its
// k_merge_delta searches the store through it) and then writes the index of the new store there.
int qmck_store_index(hipStream_t st, const uint64_t* keys, const uint64_t* count,
                     uint64_t* sidx, uint64_t max_items);
// out[0..1] (device) = the index range of the sorted keys[0, *count) within [lo, hi].
int qmck_key_range(hipStream_t st, const uint64_t* keys, const uint64_t* count, uint64_t lo,
                   uint64_t hi, uint64_t* out);
// Ideal Pauli pulse: circuit c of the store (rep_per replicas each) takes X^x Z^z with
// (x, z) = (pxz[2c], pxz[2c+1]) (device); with any_x the records go to (ck, cv) for a re-sort.
int qmck_pulse(hipStream_t st, uint64_t* pk, int2* pv, void* counters, uint32_t cur, uint32_t n,
               uint32_t kbits, uint32_t rep_per, const uint64_t* pxz, int any_x, uint64_t* ck,
               int2* cv, uint32_t csel, uint64_t max_parents);
// Copies *count records (a device counter) from (ki, vi) to (ko, vo).
int qmck_copy_store(hipStream_t st, const uint64_t* ki, const int2* vi, uint64_t* ko, int2* vo,
                    const uint64_t* count, uint64_t max_items);
int qmck_observe(hipStream_t st, const uint64_t* pk, const int2* pv, void* counters, uint32_t cur,
                 uint32_t n, uint32_t kbits, uint32_t nrep, uint32_t n_pauli, const uint64_t* pxz,
                 uint32_t want_eps, unsigned long long* out, uint32_t out_stride,
                 uint64_t max_per_replica);
int qmck_lookup(hipStream_t st, const uint64_t* pk, const int2* pv, void* counters, uint32_t cur,
                uint32_t kbits, const uint64_t* keys, uint32_t nk, uint32_t nrep, int64_t* out);
// out[r] (device, nrep + 1 words) = first record of replica r of the sorted store whose size is
// n_store[0] of the Counters image at `counters`; out[nrep] = that size.
int qmck_replica_bounds(hipStream_t st, const uint64_t* keys, const void* counters,
                        uint32_t kbits, uint32_t nrep, uint64_t* out);
}
