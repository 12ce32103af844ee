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
constexpr int kSpawnSeg = 512;       // per-wave LDS staging segment for child records
constexpr int kRadixBits = 8;
constexpr int kRadixBins = 1 << kRadixBits;
constexpr int kSortBlocks = 256;     // fixed grid of the radix passes

// Device error bits (counters.err).
enum : uint32_t {
  kErrSpawnCap = 1u,
  kErrStoreCap = 2u,
  kErrOverflow = 4u,
  kErrLookback = 8u,
};

// One quantized term of a step table: sign mask and Q32 coefficient.
struct Term {
  uint64_t zmask;
  int32_t qre, qim;
};

// Packed per-step table (host-built, 16-byte aligned):
//   TableHeader | uint64 gx[n_groups] | uint32 gs[n_groups + 1] (padded to 16 B) | Term t[n_terms]
// Group 0 is the diagonal group (gx[0] == 0, possibly empty); groups 1.. are off-diagonal in
// increasing xmask order.  q_off / q_diag bound sum(|c_re| + |c_im|) over all off-diagonal
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
  uint64_t pad;
};

struct Counters {
  uint64_t n_store[2];     // occupied keys of the store buffer 0 / 1
  uint64_t n_child[2];     // child records of the step with the same parity
  uint64_t walker_steps;   // running sum of N^tot over the parents of every step
  uint64_t key_steps;      // running sum of occupied keys over the parents of every step
  uint64_t child_steps;    // running sum of child records of every step
  uint64_t out_steps;      // running sum of annihilated output keys of every step
  uint32_t err;
  uint32_t err_step;
  uint32_t tile_counter;
  uint32_t pad;
};

__device__ __forceinline__ void philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                              uint32_t k0, uint32_t k1, uint32_t out[4]) {
  // Salmon et al., SC'11: ten rounds, multipliers 0xD2511F53 / 0xCD9E8D57, Weyl key bumps.
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint32_t lo0 = 0xD2511F53u * c0;
    const uint32_t hi0 = __umulhi(0xD2511F53u, c0);
    const uint32_t lo1 = 0xCD9E8D57u * c2;
    const uint32_t hi1 = __umulhi(0xCD9E8D57u, c2);
    const uint32_t n0 = hi1 ^ c1 ^ k0;
    const uint32_t n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
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
  if (q == 0 || s == 0) return true;
  if (__umul64hi(s, q) != 0) return false;
  const uint64_t p = s * q;
  return p < (1ull << 32) - (uint64_t)U;
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

}  // namespace qmc
