// qmc_device.hpp -- device primitives and shared layouts of libqmc (gfx950, wave64).
//
// Composite walker key: ck = (replica << 2n) | key, key = (bra << n) | ket.  The store of all
// replicas is one array sorted ascending by ck, so every replica is a contiguous segment.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace qmc {

constexpr int kBlock = 256;          // threads per block (4 waves of 64)
constexpr int kWave = 64;
constexpr int kWaves = kBlock / kWave;
constexpr int kMaxGroups = 255;      // off-diagonal column groups per step
constexpr int kMaxTerms = 4096;      // merged terms per step table
constexpr int kMergeIpt = 4;         // merged items per thread
constexpr int kMergeTile = kBlock * kMergeIpt;
constexpr int kMergeSlack = kMaxGroups + 1;  // a key's run of children is at most one per group
constexpr int kIdxShift = 8;                  // the store's search index: every 256th key
constexpr uint32_t kIdxStride = 1u << kIdxShift;
constexpr int kMergeCap = kMergeTile + kMergeSlack + 8;
constexpr int kSpawnSeg = 256;       // per-wave LDS staging of child records in k_spawn
constexpr int kSpawnRound = 1024;    // parents k_spawn loads at once
constexpr int kMergeActive = kBlock + kWave;  // spawn queue of active parents: < 64 + one chunk
constexpr int kMergeQueue = kBlock;  // merge's queue of next-step parents (flushed when full)
constexpr int kRadixBits = 11;       // digit width of the onesweep passes
constexpr int kRadixBins = 1 << kRadixBits;
constexpr int kMaxPasses = 6;        // ceil(64 / 11)
constexpr int kSortIpt = 16;         // records per thread of a sort tile
constexpr int kSortTile = kBlock * kSortIpt;
constexpr int kPersistBlocks = 512;  // grid of the persistent (tile-ticket) kernels
constexpr int kMergeBlocks = 1536;   // k_merge: at most six workgroups per CU (26 KB of LDS each)
constexpr int kMaxSegments = 512;    // key ranges (workgroups) of the segmented step
constexpr int kMaxCircuits = kMaxSegments;  // circuits of one batch (each needs a key range)
constexpr int kInboxMax = 4096;      // records per segment inbox (sorted in LDS)
constexpr int kTermPad = 4;          // terms per group are a multiple of this in a packed table

// Device error bits (counters.err).
enum : uint32_t {
  kErrSpawnCap = 1u,
  kErrStoreCap = 2u,
  kErrOverflow = 4u,
  kErrLookback = 8u,   // a bounded wait expired (look-back, grid barrier) or a layout check failed
  kErrSegCap = 16u,    // one key range outgrew its segment (cured by rebalancing)
  kErrInbox = 32u,     // one key range received more records than its inbox holds
};

// One quantized term of a step table: sign mask and Q32 coefficient.
struct Term {
  uint64_t zmask;
  int32_t qre, qim;
};

// Packed per-step table (host-built, 16-byte aligned):
//   TableHeader | uint64 gx[n_groups] | uint32 gs[n_groups + 1] (padded to 16 B) | Term t[n_terms]
// Group 0 is the diagonal group (gx[0] == 0, possibly empty); groups 1.. are off-diagonal in
// increasing xmask order.  Every group's term range is padded with zero terms to a nonzero
// multiple of kTermPad terms (a zero term adds nothing whatever its sign).  q_off / q_diag bound sum(|c_re| + |c_im|) over all off-diagonal
// groups / over the diagonal group of any key.
struct TableHeader {
  uint32_t n_groups;
  uint32_t n_terms;
  uint32_t gx_off;    // byte offsets from the start of the table
  uint32_t gs_off;
  uint32_t t_off;
  uint32_t bytes;
  uint64_t q_off;
  uint64_t q_diag;
  uint64_t active[2];  // bit m: weight channel m of the step (H monomials, then Lindblad
                       // operators of the circuit) is nonzero; channels past 127 not kept
  uint64_t pad;
};
static_assert(sizeof(TableHeader) % 16 == 0, "the group masks follow at a 16-byte offset");

struct Counters {
  uint64_t n_store[2];     // occupied keys of the current / next store (by step parity)
  uint64_t n_prev;         // occupied keys of N(s-1) (AB2)
  uint64_t n_child[2];     // child records of the step with the same parity
  uint64_t walker_steps;   // running sum of N^tot over the parents of every step
  uint64_t key_steps;      // running sum of occupied keys over the parents of every step
  uint64_t child_steps;    // running sum of child records of every step
  uint64_t out_steps;      // running sum of annihilated output keys of every step
  uint64_t death_steps;    // running sum of nonzero diagonal (death/cloning) records of every
                           // step; child_steps - death_steps are the off-diagonal children
  uint64_t n_active;       // parents of the next step queued by the merge (their combs can fire)
  uint32_t err;
  uint32_t err_step;
  uint32_t tile_counter;   // (unused)
  uint32_t resplits;       // key ranges re-cut inside the fused kernel (running sum)
  uint32_t sort_ticket[2][kMaxPasses + 2];  // onesweep tile tickets per step parity and pass
  uint64_t small_stop;     // the LDS-resident chain's stop word, as its finishing kernel saw it
};

// Epoch tags of the look-back status words (never 0, distinct within a batch of <= 8000 steps).
__host__ __device__ inline uint32_t sort_epoch(uint32_t step, uint32_t pass) {
  return 1u + (step * 8u + pass) % 65535u;
}

// Lane exchanges inside rows of 16 lanes (DPP, gfx9 encodings); lanes with no source read 0.
template <int Ctrl, int RowMask = 0xF>
__device__ __forceinline__ uint32_t dpp(uint32_t x) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, Ctrl, RowMask, 0xF, false);
}

// Sum over aligned groups of T lanes (T a power of two <= 64, wave-uniform), in every lane of
// the group; all lanes active.
__device__ __forceinline__ uint32_t team_sum(uint32_t x, uint32_t T) {
  if (T >= 2) x += dpp<0xB1>(x);    // quad_perm [1, 0, 3, 2]
  if (T >= 4) x += dpp<0x4E>(x);    // quad_perm [2, 3, 0, 1]
  if (T >= 8) x += dpp<0x141>(x);   // row_half_mirror: a lane of the other quad of its 8
  if (T >= 16) x += dpp<0x140>(x);  // row_mirror: a lane of the other half of its row
  if (T >= 32) x += (uint32_t)__builtin_amdgcn_ds_swizzle((int)x, 0x401F);  // lane ^ 16
  if (T >= 64) x += __shfl_xor(x, 32);
  return x;
}

// Inclusive prefix sum over aligned groups of T lanes (lt = lane index in the group); all lanes
// active.
__device__ __forceinline__ uint32_t team_scan(uint32_t x, uint32_t T, uint32_t lt) {
  if (T >= 2) { const uint32_t y = dpp<0x111>(x); if (lt >= 1) x += y; }  // row_shr 1
  if (T >= 4) { const uint32_t y = dpp<0x112>(x); if (lt >= 2) x += y; }  // row_shr 2
  if (T >= 8) { const uint32_t y = dpp<0x114>(x); if (lt >= 4) x += y; }  // row_shr 4
  if (T >= 16) { const uint32_t y = dpp<0x118>(x); if (lt >= 8) x += y; } // row_shr 8
  if (T >= 32) x += dpp<0x142, 0xA>(x);  // rows 1 and 3 add lane 15 of rows 0 and 2
  if (T >= 64) x += dpp<0x143, 0xC>(x);  // rows 2 and 3 add lane 31
  return x;
}

__device__ __forceinline__ void philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                              uint32_t k0, uint32_t k1, uint32_t out[4]) {
  // Salmon et al., SC'11: ten rounds, multipliers 0xD2511F53 / 0xCD9E8D57, Weyl key bumps.
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
    // three-way exclusive or in one instruction (bitop3 truth table 0x96)
    const uint32_t n0 = __builtin_amdgcn_bitop3_b32((uint32_t)(p1 >> 32), c1, k0, 0x96);
    const uint32_t n2 = __builtin_amdgcn_bitop3_b32((uint32_t)(p0 >> 32), c3, k1, 0x96);
    c1 = (uint32_t)p1;
    c3 = (uint32_t)p0;
    c0 = n0;
    c2 = n2;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
    // The key is wave-uniform (the run's seed): each round's key is bumped in scalar registers
    // as the rounds go, rather than all twenty precomputed and held (or spilled) for the loop.
    asm volatile("" : "+s"(k0), "+s"(k1));
  }
  out[0] = c0;
  out[1] = c1;
  out[2] = c2;
  out[3] = c3;
}

__device__ __forceinline__ uint32_t parity64(uint64_t v) {
  return (__popcll(v)) & 1u;
}

__device__ __forceinline__ uint64_t uabs64(int64_t v) {
  return v < 0 ? (uint64_t)0 - (uint64_t)v : (uint64_t)v;
}

// One step of the systematic comb: returns the signed count for x and advances r (< 2^32).
__device__ __forceinline__ int64_t comb_step(uint64_t& r, int64_t x) {
  const uint64_t t = r + uabs64(x);
  r = t & 0xFFFFFFFFull;
  const int64_t c = (int64_t)(t >> 32);
  return x < 0 ? -c : c;
}

// s * q + U < 2^32 (s = |a| + |b|, q bounds the column coefficients) means every output of a
// comb started at U is zero: the comb only emits when its running sum crosses 2^32.
__device__ __forceinline__ bool comb_all_zero(uint64_t s, uint64_t q, uint32_t U) {
  // the usual case: s q + U in one 32 x 32 + 32 -> 64 multiply-add (zero s or q give U < 2^32)
  if (((s | q) >> 32) == 0) return (((uint64_t)(uint32_t)s * (uint32_t)q + U) >> 32) == 0;
  if (q == 0 || s == 0) return true;
  if (__umul64hi(s, q) != 0) return false;
  return s * q < (1ull << 32) - (uint64_t)U;
}

__device__ __forceinline__ uint64_t lanemask_lt() {
  const uint32_t lane = __lane_id();
  return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

__device__ __forceinline__ uint32_t mbcnt64(uint64_t m) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                   __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

__device__ __forceinline__ void wave_lds_fence() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ uint64_t atomic_load_agent(const uint64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void atomic_store_agent(uint64_t* p, uint64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Step tables are read-only while any kernel runs and every lane of a wave reads the same
// entry, so they are addressed in the constant address space: the loads go through the scalar
// unit and cache, and the values arrive in scalar registers.
// A kernel that copies the table into LDS first reads it there instead (lptr).
template <class T>
using cptr = const __attribute__((address_space(4))) T*;
template <class T>
using lptr = const T*;

template <template <class> class Ptr>
struct TableViewT {
  Ptr<TableHeader> h;
  Ptr<uint64_t> gx;
  Ptr<uint32_t> gs;
  Ptr<Term> t;
};
using TableView = TableViewT<cptr>;

template <template <class> class Ptr = cptr>
__device__ __forceinline__ TableViewT<Ptr> table_view(const uint8_t* tab) {
  const Ptr<uint8_t> b = (Ptr<uint8_t>)tab;
  TableViewT<Ptr> v;
  v.h = (Ptr<TableHeader>)b;
  v.gx = (Ptr<uint64_t>)(b + v.h->gx_off);
  v.gs = (Ptr<uint32_t>)(b + v.h->gs_off);
  v.t = (Ptr<Term>)(b + v.h->t_off);
  return v;
}

// The step tables of one step for a batch of circuits: circuit c's table starts at base + off[c];
// segment s of the store (composite key >> 2n: replica rep of circuit c is s = c * rep_per + r)
// takes its circuit's table.  One circuit (the usual case) has a single table for all replicas.
struct TabSet {
  const uint8_t* base;
  const uint32_t* off;  // [circuits] offsets for this step, or null: no table
  uint32_t rep_per;     // replicas per circuit
  __device__ __forceinline__ bool valid() const { return off != nullptr; }
  __device__ __forceinline__ const uint8_t* of_segment(uint32_t seg) const {
    return base + off[seg / rep_per];
  }
};

struct KeyLayout {
  uint32_t kbits;     // 2n
  uint64_t kmask;     // (1 << 2n) - 1
  // Initiator approximation (End Matter on simulation methodology): with it on (ish = 1) a
  // routed record's key is (composite key << 1) | flag, flag = its parent is not an initiator
  // (population below init_min); a flagged record only lands on a key that has a parent.
  uint32_t ish;       // 0 or 1
  uint64_t init_min;  // initiator threshold in walkers (0 with ish = 0)
  __device__ __forceinline__ uint64_t key(uint64_t ck) const { return ck & kmask; }
  __device__ __forceinline__ uint32_t replica(uint64_t ck) const {
    return kbits >= 64 ? 0u : (uint32_t)(ck >> kbits);
  }
  // routed-record key of composite key ck spawned by a parent of population sab
  __device__ __forceinline__ uint64_t rkey(uint64_t ck, uint64_t sab) const {
    return (ck << ish) | (sab < init_min ? 1ull : 0ull);
  }
  // composite key of a routed record
  __device__ __forceinline__ uint64_t ckey(uint64_t rk) const { return rk >> ish; }
  // whether a routed record counts on a key with / without a parent
  __device__ __forceinline__ bool keep(uint64_t rk, bool has_parent) const {
    return has_parent || (rk & 1ull & (uint64_t)ish) == 0;
  }
};

// Philox block of a walker: counter (key, step, (replica << 8) | stream), key = the seed.
// Stream 0 draws for N(s) (Euler, first AB2 term), stream 1 for N(s-1) (second AB2 term).
__device__ __forceinline__ void walker_random(uint64_t key, uint32_t step, uint32_t replica,
                                              uint64_t seed, uint32_t stream, uint32_t w[4]) {
  philox4x32_10((uint32_t)key, (uint32_t)(key >> 32), step, (replica << 8) | stream,
                (uint32_t)seed, (uint32_t)(seed >> 32), w);
}

// Group coefficient c = sum_t (-1)^parity(zmask_t & key) q_t; |c_re| + |c_im| < 2^31, so every
// partial sum fits int32.  [b, e) is a padded group range: a nonzero multiple of kTermPad terms.
template <class TP>
__device__ __forceinline__ void group_coeff(TP t, uint32_t b, uint32_t e, uint64_t key,
                                            int32_t& cre, int32_t& cim) {
  int32_t re = 0, im = 0;
  uint32_t i = b;
  do {
#pragma unroll
    for (int u = 0; u < kTermPad; ++u) {
      const uint64_t zm = t[i + u].zmask;
      const int32_t qre = t[i + u].qre, qim = t[i + u].qim;
      const int32_t s = -(int32_t)parity64(zm & key);  // 0 or -1
      re += (qre ^ s) - s;
      im += (qim ^ s) - s;
    }
    i += kTermPad;
  } while (i < e);
  cre = re;
  cim = im;
}

// The same sum over the terms [b, e) (a multiple of kTermPad, possibly empty) of one group: a
// slice of its terms.
template <typename TP>
__device__ __forceinline__ void group_coeff_part(TP t, uint32_t b, uint32_t e, uint64_t key,
                                                 int32_t& cre, int32_t& cim) {
  int32_t re = 0, im = 0;
  for (uint32_t i = b; i < e; i += kTermPad) {
#pragma unroll
    for (int u = 0; u < kTermPad; ++u) {
      const uint64_t zm = t[i + u].zmask;
      const int32_t qre = t[i + u].qre, qim = t[i + u].qim;
      const int32_t s = -(int32_t)parity64(zm & key);  // 0 or -1
      re += (qre ^ s) - s;
      im += (qim ^ s) - s;
    }
  }
  cre = re;
  cim = im;
}

__device__ __forceinline__ void cmul_q32(int64_t a, int64_t b, int32_t cre, int32_t cim,
                                         int64_t& xre, int64_t& xim) {
  xre = a * (int64_t)cre - b * (int64_t)cim;
  xim = a * (int64_t)cim + b * (int64_t)cre;
}

__device__ __forceinline__ uint32_t digit_of(uint64_t k, uint32_t shift) {
  return (uint32_t)(k >> shift) & (kRadixBins - 1);
}

// Lanes of the wave (among `active`) holding the same radix digit.
__device__ __forceinline__ uint64_t match_digit(uint32_t d, uint64_t active) {
  uint64_t peers = active;
#pragma unroll
  for (int b = 0; b < kRadixBits; ++b) {
    const uint64_t bm = __ballot((d >> b) & 1u);
    peers &= ((d >> b) & 1u) ? bm : ~bm;
  }
  return peers;
}

// Merge of parents (unique keys) with sorted child records, parents first on equal keys.
template <class KA, class KB>
__device__ __forceinline__ uint32_t merge_path(const KA& A, uint32_t na, const KB& B, uint32_t nb,
                                               uint32_t d) {
  uint32_t lo = d > nb ? d - nb : 0u;
  uint32_t hi = d < na ? d : na;
  while (lo < hi) {
    const uint32_t mid = (lo + hi) >> 1;
    if (A(mid) <= B(d - 1 - mid))
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}

// Split at diagonal d moved forward past the run of the key just before it.
template <class KA, class KB>
__device__ __forceinline__ void run_split(const KA& A, uint32_t na, const KB& B, uint32_t nb,
                                          uint32_t d, uint32_t& i, uint32_t& j) {
  i = merge_path(A, na, B, nb, d);
  j = d - i;
  if (d == 0 || d >= na + nb) return;
  uint64_t last = 0;
  if (i > 0) last = A(i - 1);
  if (j > 0) {
    const uint64_t c = B(j - 1);
    if (i == 0 || c > last) last = c;
  }
  // Only children can continue the run (a parent equal to `last` would precede it); most
  // splits do not fall inside a run, which the first probe settles.
  if (j >= nb || B(j) > last) return;
  uint32_t lo = j + 1, hi = nb;
  if (hi - j > (uint32_t)kMergeSlack) hi = j + kMergeSlack;
  while (lo < hi) {
    const uint32_t mid = (lo + hi) >> 1;
    if (B(mid) <= last)
      lo = mid + 1;
    else
      hi = mid;
  }
  j = lo;
}

}  // namespace qmc
