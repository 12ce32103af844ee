// qmc_persist.hip -- the population-dynamics step as one persistent, key-range-segmented
// cooperative kernel per batch of steps (gfx950, wave64).
//
// The sorted store (all replicas, composite keys) is cut by P splitter keys taken from the store
// itself into P key ranges; workgroup p owns range p for the whole batch: its parents live in a
// sorted segment, and every record destined to its range (spawned children, and the death/cloning
// delta of each of its own parents) arrives in its inbox.  One step of workgroup p:
//   1. sort the inbox in LDS (bitonic);
//   2. stream the parents of the segment through LDS in tiles, merge them with the inbox, sum every
//      key in int64 (annihilation, End Matter), drop empty keys, write the new segment;
//   3. for every new parent draw Philox once (step s+1) and, only for the parents whose column
//      can produce a nonzero amount (|a|+|b|)*sum|q| + U >= 2^32, evaluate the death delta
//      (diagonal of the column applied to N(s+1)) and the off-diagonal children, and route each
//      record to the inbox of the workgroup owning its key (one atomic per destination);
//   4. grid barrier.
// The batch starts with the same pass over the canonical store with an empty inbox, which copies
// each workgroup's slice into its segment and draws the first step.  One grid barrier per step,
// no global sort passes, parents read and written once per step.
#include "qmc_device.hpp"
#include "qmc_persist.h"

namespace qmc {

constexpr int kPBlock = 512;               // threads per workgroup
constexpr int kPWaves = kPBlock / kWave;   // 8
constexpr int kPTile = 1024;               // parents per tile (staged in LDS)
constexpr int kActCap = kPBlock + kWave;   // block list of active new parents
constexpr int kStage = 256;                // per-wave staging of routed records

struct PersistArgs {
  // canonical store: sorted records of all replicas (read by the first pass; a re-split in
  // the kernel writes it through ckw / cvw, the same arrays)
  const uint64_t* ck;
  const int2* cv;
  uint64_t* ckw;
  int2* cvw;
  Counters* cnt;
  uint32_t cur;
  // AB2: N(step0 - 1), sorted (its records draw the second term of step0), or null
  const uint64_t* pk_prev;
  const int2* pv_prev;
  uint64_t* pkw;          // the same array, rewritten by an AB2 re-split in the kernel (N(s))
  int2* pvw;
  // segments [nbuf][P][segcap] and counts [nbuf][P]; pass k reads buffer k mod nbuf and
  // writes buffer (k + 1) mod nbuf (three buffers keep N(s) and N(s-1) while N(s+1) is written)
  uint64_t* sk;
  int2* sv;
  uint64_t segcap;
  uint32_t* seg_n;
  uint32_t nbuf;
  // inboxes [2][P][incap] and counts [2][P]
  uint64_t* ik;
  int2* iv;
  uint32_t incap;
  uint32_t* in_n;
  // key ranges: split[p] <= key < split[p+1]
  const uint64_t* split;
  uint64_t* splitw;       // the same array, rewritten by a re-split in the kernel
  uint32_t P;
  // per-step tables of the batch: step k of circuit c at tab_base + tab_off[k * n_circuits + c]
  const uint8_t* tab_base;
  const uint32_t* tab_off;
  const uint32_t* tabB_off;  // AB2 (one circuit): tables of the second term, or null (Euler)
  uint32_t n_circuits;
  uint32_t rep_per;          // replicas per circuit
  uint32_t step0, nsteps;
  uint64_t seed;
  KeyLayout kl;
  uint32_t n_replicas;
  const int64_t* qshift;    // per-replica Q32 shifts of the first term (Euler: the only one)
  const int64_t* qshiftB;   // AB2: of the second term
  // synchronization and reporting
  uint64_t* slots;        // [2][P][4] barrier slots by epoch parity: keys out, inbox records,
                          // error bits, each tagged with the epoch
  uint64_t cap_store;     // total occupied keys allowed
  uint64_t cap_inbox;     // total inbox records allowed per step
  uint32_t max_rebal;     // re-splits the kernel may do itself (one circuit), then it stops
  uint32_t rebal_min;     // stop to rebalance when the largest range exceeds 1.25 x the larger
                          // of the mean and the launch's first largest range, + this
  uint64_t epoch0;        // first barrier epoch of this launch (epochs only grow)
  uint32_t* done;         // [0] steps completed, [1] stop reason (0 end, 1 rebalance, 2 error)
};

struct Shared {
  uint64_t split[kMaxSegments];
  uint64_t in_k[kInboxMax];
  int2 in_v[kInboxMax];
  uint64_t pa_k[kPTile];
  int2 pa_v[kPTile];
  uint32_t scan[kPBlock];
  uint32_t xsplit[kPBlock];  // merge-path split of each thread: parent index | inbox index << 16
  uint64_t act_k[kActCap];   // active new parents: key, value, comb words (w0, w1), shift
  int2 act_v[kActCap];
  uint2 act_w[kActCap];
  int64_t act_s[kActCap];
  uint64_t st_k[kPWaves][kStage];
  int2 st_v[kPWaves][kStage];
  uint64_t red[kPWaves];
  uint64_t xch[kPWaves][4];
  uint64_t dec[4];        // reduced totals of the last barrier: keys, max segment, inbox, errors
  uint32_t nouts[2][kMaxSegments];  // keys out of every workgroup, by barrier epoch parity
  uint4 tab[kPersistTableBytes / 16];   // the step table of the spawns drawn in this pass
  uint4 tabB[kPersistTableBytes / 16];  // AB2: the table of their second term
  uint32_t err;           // error bits this workgroup raised in the current step
  uint32_t ndiag;         // diagonal records this workgroup routed in the current pass
};
using LTable = TableViewT<lptr>;

// Cross-workgroup data (inbox records and counts, barrier slots) is written and read only with
// agent-scope atomic accesses: on gfx950 these go through to the device coherence point and never
// leave dirty or stale lines in an XCD's L2, so the barrier needs no L2 writeback or invalidate,
// only the completion of the workgroup's own stores (s_waitcnt vmcnt(0)).
__device__ __forceinline__ void st_agent(uint64_t* p, uint64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_agent(int2* p, int2 v) {
  const uint64_t u = (uint64_t)(uint32_t)v.x | ((uint64_t)(uint32_t)v.y << 32);
  __hip_atomic_store(reinterpret_cast<uint64_t*>(p), u, __ATOMIC_RELAXED,
                     __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_agent(uint32_t* p, uint32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t ld_agent(const uint64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int2 ld_agent(const int2* p) {
  const uint64_t u = __hip_atomic_load(reinterpret_cast<const uint64_t*>(p), __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
  return make_int2((int32_t)(uint32_t)u, (int32_t)(uint32_t)(u >> 32));
}
__device__ __forceinline__ uint32_t ld_agent(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// Wait until every memory access this wave issued has completed (for the atomic stores above:
// reached the coherence point).  The signal fences keep the compiler from moving accesses across.
__device__ __forceinline__ void wait_mem() {
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __builtin_amdgcn_s_waitcnt(0);
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

// Errors go to the context's flags (reported to the host) and to this workgroup's error word of
// the current step, which the next barrier reduces over all workgroups: every workgroup decides
// to stop from the reduced value only, so the decision is identical everywhere.
__device__ __forceinline__ void raise_err(Counters* cnt, uint32_t* my_err, uint32_t bit,
                                          uint32_t step) {
  atomicOr(&cnt->err, bit);
  atomicMin(&cnt->err_step, step);
  atomicOr(my_err, bit);
}

// Grid-wide barrier with reduction over the co-resident workgroups of a cooperative launch.
// Each workgroup publishes (keys out, inbox records, error bits) in its own slot and then reads
// every slot itself (one thread per slot) until all carry this epoch, reducing the values
// locally: two memory round trips, no master workgroup, identical totals everywhere (S.dec).
// Every slot word carries the low 32 bits of the epoch above its 32-bit value, so a word is
// valid on its own and the three are published without ordering waits; slots alternate between
// two buffers by epoch parity, so a workgroup that has passed this barrier and publishes the
// next one never overwrites a slot another workgroup may still be reading.  All cross-workgroup
// writes before the barrier are agent-scope atomics, so publishing only waits for their
// completion.  Waits are bounded: on expiry the totals carry kErrLookback and false is returned.
__device__ __forceinline__ bool grid_sync(Shared& S, const PersistArgs& A, uint64_t epoch,
                                          uint64_t nout, uint64_t nin) {
  const uint32_t t = threadIdx.x, p = blockIdx.x, P = A.P;
  wait_mem();
  __syncthreads();
  const uint64_t tag = (epoch & 0xFFFFFFFFull) << 32;
  uint64_t* const buf = A.slots + (epoch & 1u) * 4 * (uint64_t)P;
  if (t == 0) {
    uint64_t* sl = buf + 4 * (uint64_t)p;
    st_agent(&sl[0], tag | (nout < 0xFFFFFFFFull ? nout : 0xFFFFFFFFull));
    st_agent(&sl[1], tag | (nin < 0xFFFFFFFFull ? nin : 0xFFFFFFFFull));
    st_agent(&sl[2], tag | (uint64_t)S.err);
  }
  uint64_t tot = 0, mx = 0, nn = 0, er = 0;
  for (uint32_t q = t; q < P; q += kPBlock) {
    const uint64_t* sl = buf + 4 * (uint64_t)q;
    uint32_t spins = 0;
    uint64_t v0, v1, v2;
    // the workgroup's own slot: the values it has just published (the last workgroup to arrive
    // then needs no round trip through the coherence point for its own store)
    if (q == p) {
      v0 = tag | (nout < 0xFFFFFFFFull ? nout : 0xFFFFFFFFull);
      v1 = tag | (nin < 0xFFFFFFFFull ? nin : 0xFFFFFFFFull);
      v2 = tag | (uint64_t)S.err;
    }
    while (q != p) {
      v0 = ld_agent(&sl[0]);
      v1 = ld_agent(&sl[1]);
      v2 = ld_agent(&sl[2]);
      if (((v0 ^ tag) | (v1 ^ tag) | (v2 ^ tag)) >> 32 == 0) break;
      __builtin_amdgcn_s_sleep(1);
      if (++spins > (1u << 24)) {
        er |= kErrLookback;
        break;
      }
    }
    v0 &= 0xFFFFFFFFull;
    S.nouts[epoch & 1u][q] = (uint32_t)v0;
    tot += v0;
    mx = v0 > mx ? v0 : mx;
    nn += v1 & 0xFFFFFFFFull;
    er |= v2 & 0xFFFFFFFFull;
  }
  for (int o = 32; o > 0; o >>= 1) {
    tot += __shfl_xor(tot, o);
    const uint64_t m2 = __shfl_xor(mx, o);
    mx = m2 > mx ? m2 : mx;
    nn += __shfl_xor(nn, o);
    er |= __shfl_xor(er, o);
  }
  if (__lane_id() == 0) {
    S.xch[t / kWave][0] = tot;
    S.xch[t / kWave][1] = mx;
    S.xch[t / kWave][2] = nn;
    S.xch[t / kWave][3] = er;
  }
  __syncthreads();
  if (t == 0) {
    for (int w = 1; w < kPWaves; ++w) {
      tot += S.xch[w][0];
      mx = S.xch[w][1] > mx ? S.xch[w][1] : mx;
      nn += S.xch[w][2];
      er |= S.xch[w][3];
    }
    S.dec[0] = tot;
    S.dec[1] = mx;
    S.dec[2] = nn;
    S.dec[3] = er;
    if (er & kErrLookback) raise_err(A.cnt, &S.err, kErrLookback, A.step0);
    S.err = 0;  // the next step starts clean
  }
  __syncthreads();
  return (S.dec[3] & kErrLookback) == 0;
}

// Off-diagonal bound and group count of the step table held in LDS.
__device__ __forceinline__ uint64_t tn_qoff(const Shared& S) {
  return reinterpret_cast<const TableHeader*>(S.tab)->q_off;
}
__device__ __forceinline__ uint32_t tn_groups(const Shared& S) {
  return reinterpret_cast<const TableHeader*>(S.tab)->n_groups;
}

__device__ __forceinline__ uint32_t upper_bound_lds(const uint64_t* a, uint32_t n, uint64_t v) {
  uint32_t lo = 0, hi = n;
  while (lo < hi) {
    const uint32_t mid = (lo + hi) >> 1;
    if (a[mid] <= v)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}

__device__ __forceinline__ uint64_t lower_bound_glb(const uint64_t* a, uint64_t n, uint64_t v,
                                                   bool coherent = false) {
  uint64_t lo = 0, hi = n;
  while (lo < hi) {
    const uint64_t mid = (lo + hi) >> 1;
    if ((coherent ? ld_agent(&a[mid]) : a[mid]) < v)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}

// Inbox order: by key, and among equal keys a padding record (value (0, 0), which no routed
// record carries) after the real ones, so that the first c sorted records are the c real ones
// even when a real key equals the padding key ~0.
__device__ __forceinline__ bool inbox_less(uint64_t ka, int2 va, uint64_t kb, int2 vb) {
  if (ka != kb) return ka < kb;
  const bool pa = (va.x | va.y) == 0, pb = (vb.x | vb.y) == 0;
  return !pa && pb;
}

// Bitonic sort of 64 words held one per lane, ascending along the lanes (descending if `desc`,
// as the first levels of a longer bitonic network need for odd chunks).
__device__ __forceinline__ uint64_t wave_sort64(uint64_t k, bool desc) {
  const uint32_t lane = __lane_id();
  for (uint32_t size = 2; size <= (uint32_t)kWave; size <<= 1) {
    for (uint32_t stride = size >> 1; stride > 0; stride >>= 1) {
      const uint64_t pk = __shfl_xor(k, (int)stride);
      const bool asc = size == (uint32_t)kWave ? !desc : (lane & size) == 0;
      const bool lower = (lane & stride) == 0;
      if ((asc == lower) ? (pk < k) : (pk > k)) k = pk;
    }
  }
  return k;
}

// Sorts the c real records of the inbox in LDS (then m - c padding records, m a power of two).
// When the composite keys leave 12 bits free, the sort runs on one 64-bit word per record,
// (key << 12) | index, and the values follow by index at the end:
//  - up to 1024 records: every wave sorts 64-word chunks in registers (lane shuffles); the final
//    position of a word is the number of smaller words over all chunks (words are distinct),
//    found by binary search in each sorted chunk;
//  - up to 4096 records: a bitonic network on the words in place, whose strides below 64 run in
//    registers per 64-word chunk and only the larger strides go through LDS.
// Wider keys take a bitonic network on the records in LDS.
__device__ __forceinline__ void sort_inbox(Shared& S, uint32_t m, uint32_t c, bool packed) {
  const uint32_t t = threadIdx.x, wave = t / kWave, lane = __lane_id();
  if (packed && c <= (uint32_t)kWave) {
    // one chunk: wave 0 sorts it in registers and puts the records in place
    if (wave == 0) {
      const uint64_t wd = wave_sort64(lane < c ? (S.in_k[lane] << 12) | lane : ~0ull, false);
      const int2 v = lane < c ? S.in_v[wd & 0xFFFu] : make_int2(0, 0);
      if (lane < c) {
        S.in_k[lane] = wd >> 12;
        S.in_v[lane] = v;
      }
    }
    __syncthreads();
    return;
  }
  if (packed && c <= 2u * kPBlock) {
    const uint32_t nch = (c + kWave - 1) / kWave;  // <= 16 chunks of 64 words in S.pa_k
    for (uint32_t ch = wave; ch < nch; ch += kPWaves) {
      const uint32_t i = ch * kWave + lane;
      const uint64_t k = i < c ? (S.in_k[i] << 12) | i : ~0ull;
      S.pa_k[i] = wave_sort64(k, false);
    }
    __syncthreads();
    uint64_t wd[2];
    uint32_t rank[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const uint32_t i = t + h * kPBlock;
      wd[h] = i < nch * kWave ? S.pa_k[i] : ~0ull;
      rank[h] = 0;
      if (wd[h] != ~0ull) {
        for (uint32_t ch = 0; ch < nch; ++ch) {
          const uint64_t* a = S.pa_k + ch * kWave;
          uint32_t pos = 0;
#pragma unroll
          for (uint32_t st = kWave / 2; st > 0; st >>= 1)
            if (a[pos + st - 1] < wd[h]) pos += st;
          if (a[pos] < wd[h]) ++pos;  // the search leaves pos <= 63; this counts the last word
          rank[h] += pos;
        }
      }
    }
    int2 v[2];
#pragma unroll
    for (int h = 0; h < 2; ++h)
      v[h] = wd[h] != ~0ull ? S.in_v[wd[h] & 0xFFFu] : make_int2(0, 0);
    __syncthreads();
#pragma unroll
    for (int h = 0; h < 2; ++h)
      if (wd[h] != ~0ull) {
        S.in_k[rank[h]] = wd[h] >> 12;
        S.in_v[rank[h]] = v[h];
      }
    __syncthreads();
    return;
  }
  if (packed) {
    // m in (1024, 4096]: words in place in S.in_k
    for (uint32_t i = t; i < m; i += kPBlock) S.in_k[i] = i < c ? (S.in_k[i] << 12) | i : ~0ull;
    __syncthreads();
    const uint32_t nch = m / kWave;
    for (uint32_t ch = wave; ch < nch; ch += kPWaves) {
      const uint32_t i = ch * kWave + lane;
      S.in_k[i] = wave_sort64(S.in_k[i], (ch & 1u) != 0);
    }
    __syncthreads();
    for (uint32_t size = 2 * kWave; size <= m; size <<= 1) {
      for (uint32_t stride = size >> 1; stride >= (uint32_t)kWave; stride >>= 1) {
        for (uint32_t x = t; x < (m >> 1); x += kPBlock) {
          const uint32_t lo = 2 * x - (x & (stride - 1));
          const uint32_t hi = lo + stride;
          const uint64_t a = S.in_k[lo], b = S.in_k[hi];
          if ((a > b) == ((lo & size) == 0)) {
            S.in_k[lo] = b;
            S.in_k[hi] = a;
          }
        }
        __syncthreads();
      }
      for (uint32_t ch = wave; ch < nch; ch += kPWaves) {
        const uint32_t i = ch * kWave + lane;
        uint64_t k = S.in_k[i];
        for (uint32_t stride = kWave / 2; stride > 0; stride >>= 1) {
          const uint64_t pk = __shfl_xor(k, (int)stride);
          const bool asc = (i & size) == 0, lower = (lane & stride) == 0;
          if ((asc == lower) ? (pk < k) : (pk > k)) k = pk;
        }
        S.in_k[i] = k;
      }
      __syncthreads();
    }
    uint64_t wd[kInboxMax / kPBlock];
    int2 v[kInboxMax / kPBlock];
#pragma unroll
    for (int h = 0; h < kInboxMax / kPBlock; ++h) {
      const uint32_t i = t + h * kPBlock;
      wd[h] = i < c ? S.in_k[i] : ~0ull;
      v[h] = i < c ? S.in_v[wd[h] & 0xFFFu] : make_int2(0, 0);
    }
    __syncthreads();
#pragma unroll
    for (int h = 0; h < kInboxMax / kPBlock; ++h) {
      const uint32_t i = t + h * kPBlock;
      if (i < c) {
        S.in_k[i] = wd[h] >> 12;
        S.in_v[i] = v[h];
      }
    }
    __syncthreads();
    return;
  }
  for (uint32_t size = 2; size <= m; size <<= 1) {
    for (uint32_t stride = size >> 1; stride > 0; stride >>= 1) {
      for (uint32_t i = t; i < (m >> 1); i += kPBlock) {
        const uint32_t lo = 2 * i - (i & (stride - 1));
        const uint32_t hi = lo + stride;
        const bool asc = (lo & size) == 0;
        const uint64_t a = S.in_k[lo], b = S.in_k[hi];
        const int2 va = S.in_v[lo], vb = S.in_v[hi];
        if (asc ? inbox_less(b, vb, a, va) : inbox_less(a, va, b, vb)) {
          S.in_k[lo] = b;
          S.in_k[hi] = a;
          S.in_v[lo] = vb;
          S.in_v[hi] = va;
        }
      }
      __syncthreads();
    }
  }
}

// Routed emission.  Records are staged per wave in LDS; a flush finds the workgroup owning each
// key (fixed-length binary search in the splitters, all chunks interleaved), groups the records
// of each destination, and reserves inbox space with one atomic per distinct destination, all
// issued by one instruction, so a flush costs one atomic round trip.
struct Router {
  uint32_t* in_n;          // [2][P]
  uint64_t* ik;            // [2][P][incap]
  int2* iv;
  uint32_t incap;
  Counters* cnt;
  const uint64_t* split;   // LDS copy
  uint32_t P, pbits;
  uint32_t par;            // inbox parity of the destination step
  uint32_t step;           // destination step (for error reports)
  uint32_t* my_err;        // this workgroup's error word (LDS)
  uint32_t ish;            // initiator flag bit below each routed key (0 or 1)
  uint64_t* sk;            // this wave's LDS staging
  int2* sv;
  uint32_t fill;           // wave-uniform
  uint32_t* ndiag;         // LDS count of the diagonal (death/cloning) records routed this pass

  __device__ __forceinline__ void flush() {
    if (fill == 0) return;
    wave_lds_fence();
    const uint32_t lane = __lane_id();
    const uint64_t lt = lanemask_lt();
    constexpr int NC = kStage / kWave;
    uint64_t key[NC];
    int2 val[NC];
    uint32_t q[NC];
    bool has[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const uint32_t i = c * kWave + lane;
      has[c] = i < fill;
      key[c] = has[c] ? sk[i] : 0;
      val[c] = has[c] ? sv[i] : make_int2(0, 0);
      q[c] = 0;
    }
    // destination: the largest p with split[p] <= key (split[0] == 0); chunks past the fill
    // are skipped (wave-uniform)
    for (uint32_t st = pbits ? 1u << (pbits - 1) : 0u; st > 0; st >>= 1) {
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        if ((uint32_t)c * kWave >= fill) break;
        const uint32_t cand = q[c] + st;
        if (cand < P && split[cand] <= (key[c] >> ish)) q[c] = cand;
      }
    }
    wave_lds_fence();  // the staging area becomes the table of distinct destinations
    uint32_t* pq = reinterpret_cast<uint32_t*>(sk);            // [kStage] destination
    uint32_t* pc = reinterpret_cast<uint32_t*>(sv);            // [kStage] records
    uint32_t* pb = reinterpret_cast<uint32_t*>(sv) + kStage;   // [kStage] reserved base
    uint32_t np = 0;  // distinct (chunk, destination) pairs so far, wave-uniform
    uint32_t rank[NC], pidx[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      rank[c] = pidx[c] = 0;
      if ((uint32_t)c * kWave >= fill) continue;
      uint64_t peers = __ballot(has[c]);
      for (uint32_t b = 0; b < pbits; ++b) {
        const uint64_t bm = __ballot((q[c] >> b) & 1u);
        peers &= ((q[c] >> b) & 1u) ? bm : ~bm;
      }
      rank[c] = (uint32_t)__popcll(peers & lt);
      const bool lead = has[c] && rank[c] == 0;
      const uint64_t lm = __ballot(lead);
      const uint32_t my = np + (uint32_t)__popcll(lm & lt);
      if (lead) {
        pq[my] = q[c];
        pc[my] = (uint32_t)__popcll(peers);
      }
      const int leader = has[c] ? __ffsll((unsigned long long)peers) - 1 : 0;
      pidx[c] = __shfl(my, leader);
      np += (uint32_t)__popcll(lm);
    }
    wave_lds_fence();
    for (uint32_t j = lane; j < np; j += kWave)
      pb[j] = atomicAdd(&in_n[par * P + pq[j]], pc[j]);
    wave_lds_fence();
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      if (has[c]) {
        const uint32_t pos = pb[pidx[c]] + rank[c];
        if (pos < incap) {
          const uint64_t off = ((uint64_t)par * P + q[c]) * incap + pos;
          st_agent(&ik[off], key[c]);
          st_agent(&iv[off], val[c]);
        } else {
          raise_err(cnt, my_err, kErrInbox, step);
        }
      }
    }
    wave_lds_fence();
    fill = 0;
  }

  // All lanes of the wave call; lanes with `has` stage (key, val).
  __device__ __forceinline__ void emit(bool has, uint64_t key, int2 val) {
    const uint64_t m = __ballot(has);
    if (m == 0) return;
    if (has) {
      const uint32_t pos = fill + mbcnt64(m);
      sk[pos] = key;
      sv[pos] = val;
    }
    fill += (uint32_t)__popcll(m);
    if (fill > kStage - kWave) flush();
  }

  // The same for a parent's diagonal (death/cloning) record, counted apart from the children.
  __device__ __forceinline__ void emit_diag(bool has, uint64_t key, int2 val) {
    const uint64_t m = __ballot(has);
    if (m != 0 && __lane_id() == 0) atomicAdd(ndiag, (uint32_t)__popcll(m));
    emit(has, key, val);
  }
};

// Death delta and children of the n <= 64 active parents at list offset b (one per lane).
__device__ __forceinline__ void process_active(const PersistArgs& A, Shared& S, Router& R,
                                               const LTable& tn, uint32_t b, uint32_t n) {
  const uint32_t lane = __lane_id();
  const bool valid = lane < n;
  const uint64_t ck = valid ? S.act_k[b + lane] : 0;
  const int2 v = valid ? S.act_v[b + lane] : make_int2(0, 0);
  const uint2 w = valid ? S.act_w[b + lane] : make_uint2(0, 0);
  const int64_t qs = valid ? S.act_s[b + lane] : 0;
  const uint64_t key = A.kl.key(ck);
  const uint64_t sab = uabs64(v.x) + uabs64(v.y);
  // Death/cloning delta from the diagonal group (applied to N(t) in the next merge).
  {
    const bool act = valid && !comb_all_zero(sab, tn.h->q_diag + uabs64(qs), w.y);
    int2 d = make_int2(0, 0);
    if (__ballot(act)) {
      if (act) {
        int32_t dre, dim;
        group_coeff(tn.t, 0, tn.gs[1], key, dre, dim);
        int64_t xre, xim;
        cmul_q32(v.x, v.y, dre + (int32_t)qs, dim, xre, xim);
        uint64_t r = w.y;
        d.x = (int32_t)comb_step(r, xre);
        d.y = (int32_t)comb_step(r, xim);
      }
      R.emit_diag((d.x | d.y) != 0, A.kl.rkey(ck, sab), d);
    }
  }
  // Children into every off-diagonal target, one comb over all groups (Re, Im) in order.
  const uint32_t G = tn.h->n_groups;
  const bool act = valid && G > 1 && !comb_all_zero(sab, tn.h->q_off, w.x);
  if (__ballot(act) == 0) return;
  uint64_t r = w.x;
  uint32_t gb = tn.gs[1];
  for (uint32_t g = 1; g < G; ++g) {
    const uint32_t ge = tn.gs[g + 1];
    const uint64_t gxm = tn.gx[g];
    int2 child = make_int2(0, 0);
    if (act) {
      int32_t cre, cim;
      group_coeff(tn.t, gb, ge, key, cre, cim);
      int64_t xre, xim;
      cmul_q32(v.x, v.y, cre, cim, xre, xim);
      child.x = (int32_t)comb_step(r, xre);
      child.y = (int32_t)comb_step(r, xim);
    }
    R.emit((child.x | child.y) != 0, A.kl.rkey(ck ^ gxm, sab), child);
    gb = ge;
  }
}

// Death deltas and children of the whole active list [0, nl) when it holds at most kPWaves / 2
// batches of 64 parents, with J = kPWaves / batches waves on each batch: wave j of a batch takes
// the j-th slice of the diagonal group's terms and of the off-diagonal groups.  The partial
// diagonal coefficients are summed over the slices (integer sums, exact), and the comb of slice
// j starts where the comb over all earlier groups would stand: the uniform plus their amounts,
// mod 2^32 (the remainder after any run of comb steps is that sum mod 2^32), so every record
// equals the one the single-wave comb in group order gives.  Block-uniform; uses the parent tile
// area of LDS for the partial sums.
__device__ __forceinline__ void process_wide(const PersistArgs& A, Shared& S, Router& R,
                                             const LTable& tn, uint32_t nl) {
  static_assert(sizeof(S.pa_v) >= kPBlock * sizeof(int2), "partial coefficients");
  static_assert(sizeof(S.pa_k) >= kPBlock * sizeof(uint32_t), "partial comb amounts");
  const uint32_t wave = threadIdx.x / kWave, lane = __lane_id();
  const uint32_t nb = (nl + kWave - 1) / kWave;
  const uint32_t J = kPWaves / nb;
  const uint32_t b = wave / J, j = wave % J;
  const bool mine = b < nb;  // wave-uniform
  int2* dpart = S.pa_v;
  uint32_t* cpart = reinterpret_cast<uint32_t*>(S.pa_k);
  const uint32_t i = b * kWave + lane;
  const bool valid = mine && i < nl;
  const uint64_t ck = valid ? S.act_k[i] : 0;
  const int2 v = valid ? S.act_v[i] : make_int2(0, 0);
  const uint2 w = valid ? S.act_w[i] : make_uint2(0, 0);
  const int64_t qs = valid ? S.act_s[i] : 0;
  const uint64_t key = A.kl.key(ck);
  const uint64_t sab = uabs64(v.x) + uabs64(v.y);
  const uint32_t G = tn.h->n_groups;
  const bool dact = valid && !comb_all_zero(sab, tn.h->q_diag + uabs64(qs), w.y);
  const bool act = valid && G > 1 && !comb_all_zero(sab, tn.h->q_off, w.x);
  const uint32_t nd = tn.gs[1] / kTermPad;
  const uint32_t d0 = nd * j / J * kTermPad, d1 = nd * (j + 1) / J * kTermPad;
  const uint32_t g0 = 1 + (G - 1) * j / J, g1 = 1 + (G - 1) * (j + 1) / J;
  int32_t pre = 0, pim = 0;
  if (__ballot(dact) && dact) group_coeff_part(tn.t, d0, d1, key, pre, pim);
  uint32_t amt = 0;
  if (__ballot(act) && act) {
    for (uint32_t g = g0; g < g1; ++g) {
      int32_t cre, cim;
      group_coeff(tn.t, tn.gs[g], tn.gs[g + 1], key, cre, cim);
      int64_t xre, xim;
      cmul_q32(v.x, v.y, cre, cim, xre, xim);
      amt += (uint32_t)uabs64(xre) + (uint32_t)uabs64(xim);
    }
  }
  if (mine) {
    dpart[wave * kWave + lane] = make_int2(pre, pim);
    cpart[wave * kWave + lane] = amt;
  }
  __syncthreads();
  if (mine && j == 0 && __ballot(dact)) {
    int2 d = make_int2(0, 0);
    if (dact) {
      int32_t dre = 0, dim = 0;
      for (uint32_t jj = 0; jj < J; ++jj) {
        const int2 pp = dpart[(b * J + jj) * kWave + lane];
        dre += pp.x;
        dim += pp.y;
      }
      int64_t xre, xim;
      cmul_q32(v.x, v.y, dre + (int32_t)qs, dim, xre, xim);
      uint64_t r = w.y;
      d.x = (int32_t)comb_step(r, xre);
      d.y = (int32_t)comb_step(r, xim);
    }
    R.emit_diag((d.x | d.y) != 0, A.kl.rkey(ck, sab), d);
  }
  if (mine && __ballot(act)) {
    uint32_t r0 = w.x;
    for (uint32_t jj = 0; jj < j; ++jj) r0 += cpart[(b * J + jj) * kWave + lane];
    uint64_t r = r0;
    for (uint32_t g = g0; g < g1; ++g) {
      int2 child = make_int2(0, 0);
      if (act) {
        int32_t cre, cim;
        group_coeff(tn.t, tn.gs[g], tn.gs[g + 1], key, cre, cim);
        int64_t xre, xim;
        cmul_q32(v.x, v.y, cre, cim, xre, xim);
        child.x = (int32_t)comb_step(r, xre);
        child.y = (int32_t)comb_step(r, xim);
      }
      R.emit((child.x | child.y) != 0, A.kl.rkey(ck ^ tn.gx[g], sab), child);
    }
  }
  __syncthreads();
}

// Draw Philox (stream `stream`) for the records [o0, o1) of (seg_k, seg_v) at step `step` and
// route their diagonal deltas and children under table tn with shifts qsh.  The parents that can produce a nonzero amount are
// compacted over the whole workgroup into a list, which is processed in full 64-parent batches
// spread over the waves (a batch costs the same whatever its lane count), so a busy key range
// needs few batches and they run on different SIMDs.  Block-uniform control flow.
__device__ __forceinline__ void advance(const PersistArgs& A, Shared& S, Router& R,
                                        const LTable& tn, const int64_t* qsh, uint32_t stream,
                                        const uint64_t* seg_k, const int2* seg_v, uint64_t o0,
                                        uint64_t o1, uint32_t step,
                                        bool coherent = false) {
  const uint32_t t = threadIdx.x, wave = t / kWave, lane = __lane_id();
  const KeyLayout kl = A.kl;
  const uint64_t q_diag = tn.h->q_diag, q_off = tn.h->n_groups > 1 ? tn.h->q_off : 0;
  uint32_t nl = 0;  // entries in the list (block-uniform)
  for (uint64_t base = o0; base < o1; base += kPBlock) {
    const uint64_t i = base + t;
    const bool valid = i < o1;
    uint64_t ck = 0;
    int2 v = make_int2(0, 0);
    bool act = false;
    uint32_t w[4] = {0, 0, 0, 0};
    int64_t qs = 0;
    if (valid) {
      ck = coherent ? ld_agent(&seg_k[i]) : seg_k[i];
      v = coherent ? ld_agent(&seg_v[i]) : seg_v[i];
      const uint32_t rep = kl.replica(ck);
      qs = qsh[rep];
      walker_random(kl.key(ck), step, rep, A.seed, stream, w);
      const uint64_t sab = uabs64(v.x) + uabs64(v.y);
      act = !comb_all_zero(sab, q_diag + uabs64(qs), w[1]) || !comb_all_zero(sab, q_off, w[0]);
    }
    // workgroup-wide compaction of the active parents, in index order
    const uint64_t m = __ballot(act);
    if (lane == 0) S.scan[wave] = (uint32_t)__popcll(m);
    __syncthreads();
    uint32_t off = 0, tot = 0;
    for (uint32_t x = 0; x < (uint32_t)kPWaves; ++x) {
      const uint32_t cnt = S.scan[x];
      off += x < wave ? cnt : 0u;
      tot += cnt;
    }
    if (act) {
      const uint32_t at = nl + off + mbcnt64(m);
      S.act_k[at] = ck;
      S.act_v[at] = v;
      S.act_w[at] = make_uint2(w[0], w[1]);
      S.act_s[at] = qs;
    }
    nl += tot;
    __syncthreads();
    const bool end = base + kPBlock >= o1;
    if (end || nl >= (uint32_t)kPBlock) {
      // full batches now (all of them at the end), the rest moves to the front of the list
      const uint32_t nb = end ? (nl + kWave - 1) / kWave : nl / kWave;
      if (end && nb <= (uint32_t)kPWaves / 2) {
        if (nb > 0) process_wide(A, S, R, tn, nl);  // few batches: several waves on each
      } else {
        for (uint32_t b = wave; b < nb; b += kPWaves) {
          const uint32_t b0 = b * kWave;
          process_active(A, S, R, tn, b0,
                         nl - b0 < (uint32_t)kWave ? nl - b0 : (uint32_t)kWave);
        }
      }
      const uint32_t done = nb * kWave < nl ? nb * kWave : nl;
      const uint32_t rest = nl - done;
      __syncthreads();
      uint64_t rk = 0;
      int2 rv = make_int2(0, 0);
      uint2 rw = make_uint2(0, 0);
      int64_t rs = 0;
      if (t < rest) {
        rk = S.act_k[done + t];
        rv = S.act_v[done + t];
        rw = S.act_w[done + t];
        rs = S.act_s[done + t];
      }
      __syncthreads();
      if (t < rest) {
        S.act_k[t] = rk;
        S.act_v[t] = rv;
        S.act_w[t] = rw;
        S.act_s[t] = rs;
      }
      nl = rest;
      __syncthreads();
    }
  }
  R.flush();
}

// Merge one segment's parents (sorted, global) with its sorted inbox (LDS), sum per key,
// write the surviving keys to the output segment, and (if `spawn`) draw the next step from them
// (and, if `spawnB`, the next step's second AB2 term from the parents).
// The parents go through LDS in tiles of kPTile; each tile takes the inbox records up to its last
// parent (the last tile takes the rest), and the merged items of the tile are split evenly over
// the threads by a merge-path search that never cuts a key's run.  Returns the number of keys
// written in S.red[0] and the walker sum of the parents in S.red[1] (block-uniform).
__device__ __forceinline__ void merge_segment(const PersistArgs& A, Shared& S, const uint64_t* pk,
                                              const int2* pv, uint64_t np, uint32_t c, uint64_t* ok,
                                              int2* ov, uint32_t step, bool spawn, bool spawnB,
                                              Router R, const LTable tn, const LTable tnB,
                                              uint32_t nstep, bool coherent = false) {
  const uint32_t t = threadIdx.x;
  uint64_t out_run = 0;   // block-uniform
  uint64_t wsum = 0;
  uint32_t jb = 0;        // first inbox record not yet merged (block-uniform)
  const uint64_t ntile = np > 0 ? (np + kPTile - 1) / kPTile : (c > 0 ? 1 : 0);
  for (uint64_t tt = 0; tt < ntile; ++tt) {
    const uint64_t f = tt * kPTile;
    const uint32_t pn = np > f ? (uint32_t)((np - f) < (uint64_t)kPTile ? (np - f) : kPTile) : 0u;
    for (uint32_t i = t; i < pn; i += kPBlock) {
      // parents written by other workgroups in this launch (a re-split store) bypass the caches
      S.pa_k[i] = coherent ? ld_agent(&pk[f + i]) : pk[f + i];
      const int2 v = coherent ? ld_agent(&pv[f + i]) : pv[f + i];
      S.pa_v[i] = v;
      wsum += uabs64(v.x) + uabs64(v.y);
    }
    __syncthreads();
    // inbox window of this tile: records up to its last parent, or all the rest on the last tile
    const bool last_tile = tt + 1 == ntile;
    const uint32_t je =
        last_tile ? c : upper_bound_lds(S.in_k, c, (S.pa_k[pn - 1] << A.kl.ish) | A.kl.ish);
    const uint32_t cn = je - jb;
    const uint64_t* ck = S.in_k + jb;
    const int2* cv = S.in_v + jb;
    // this thread's share of the tile's merged items
    auto KA = [&](uint32_t x) { return S.pa_k[x]; };
    auto KB = [&](uint32_t x) { return A.kl.ckey(ck[x]); };
    const uint32_t tot = pn + cn;
    const uint32_t per = (tot + kPBlock - 1) / kPBlock;
    uint32_t d0 = t * per;
    if (d0 > tot) d0 = tot;
    // this thread's end is the next thread's start (one search per thread)
    uint32_t i0, j0, i1, j1;
    run_split(KA, pn, KB, cn, d0, i0, j0);
    S.xsplit[t] = i0 | (j0 << 16);
    __syncthreads();
    if (t + 1 < (uint32_t)kPBlock) {
      const uint32_t nx = S.xsplit[t + 1];
      i1 = nx & 0xFFFFu;
      j1 = nx >> 16;
    } else {
      i1 = pn;
      j1 = cn;
    }
    auto walk = [&](auto&& out) __attribute__((always_inline)) {
      uint32_t i = i0, j = j0;
      while (i < i1 || j < j1) {
        uint64_t key;
        int64_t re = 0, im = 0;
        bool hp = false;
        if (j >= j1 || (i < i1 && S.pa_k[i] <= A.kl.ckey(ck[j]))) {
          key = S.pa_k[i];
          re = S.pa_v[i].x;
          im = S.pa_v[i].y;
          hp = true;
          ++i;
        } else {
          key = A.kl.ckey(ck[j]);
        }
        while (j < j1 && A.kl.ckey(ck[j]) == key) {
          if (A.kl.keep(ck[j], hp)) {
            re += cv[j].x;
            im += cv[j].y;
          }
          ++j;
        }
        out(key, re, im);
      }
    };
    // Pass 1: count the nonzero sums.
    uint32_t count = 0;
    bool overflow = false;
    walk([&](uint64_t, int64_t re, int64_t im) __attribute__((always_inline)) {
      if (re < INT32_MIN || re > INT32_MAX || im < INT32_MIN || im > INT32_MAX) overflow = true;
      count += (re != 0 || im != 0) ? 1u : 0u;
    });
    if (overflow) raise_err(A.cnt, &S.err, kErrOverflow, step);
    // Block exclusive scan of the counts: inclusive scan within each wave, then wave totals.
    uint32_t incl = count;
    for (int o = 1; o < kWave; o <<= 1) {
      const uint32_t x = __shfl_up(incl, o);
      if (__lane_id() >= (uint32_t)o) incl += x;
    }
    if (__lane_id() == kWave - 1) S.scan[t / kWave] = incl;
    __syncthreads();
    uint32_t wpre = 0, agg = 0;
    for (uint32_t w = 0; w < (uint32_t)kPWaves; ++w) {
      const uint32_t v = S.scan[w];
      wpre += w < t / kWave ? v : 0u;
      agg += v;
    }
    const uint32_t excl = wpre + incl - count;
    const uint64_t o0 = out_run;
    if (o0 + agg > A.segcap) {
      if (t == 0) raise_err(A.cnt, &S.err, kErrSegCap, step);
    } else {
      // Pass 2: write.
      uint64_t o = o0 + excl;
      walk([&](uint64_t key, int64_t re, int64_t im) __attribute__((always_inline)) {
        if (re != 0 || im != 0) {
          ok[o] = key;
          ov[o] = make_int2((int32_t)re, (int32_t)im);
          ++o;
        }
      });
    }
    out_run = o0 + agg;
    jb = je;
    __syncthreads();  // this tile's outputs are visible to the whole workgroup
    if (spawn && o0 + agg <= A.segcap)
      advance(A, S, R, tn, A.qshift, 0u, ok, ov, o0, o0 + agg, nstep);
    // AB2: the second term of the next step from this tile's parents N(s)
    if (spawnB) advance(A, S, R, tnB, A.qshiftB, 1u, pk + f, pv + f, 0, pn, nstep);
    __syncthreads();
  }
  // block reduction of the walker sum
  for (int o = 32; o > 0; o >>= 1) wsum += __shfl_xor(wsum, o);
  if (__lane_id() == 0) S.red[t / kWave] = wsum;
  __syncthreads();
  if (t == 0) {
    uint64_t s = 0;
    for (int w = 0; w < kPWaves; ++w) s += S.red[w];
    S.red[0] = out_run;
    S.red[1] = s;
  }
  __syncthreads();
}

__global__ __launch_bounds__(kPBlock) void k_persist(PersistArgs A) {
  __shared__ Shared S;
  const uint32_t t = threadIdx.x, p = blockIdx.x;
  const uint32_t P = A.P;
  Counters* cnt = A.cnt;
  uint32_t pbits = 0;
  while ((1u << pbits) < P) ++pbits;
  // composite keys below 2^52: the inbox sort can pack a 12-bit record index under the key
  uint32_t rbits = 0;
  while ((1ull << rbits) < (uint64_t)A.n_replicas) ++rbits;
  const bool packed = A.kl.kbits + rbits + A.kl.ish <= 52;
  for (uint32_t i = t; i < P; i += kPBlock) S.split[i] = A.split[i];
  if (t == 0) {
    S.err = 0;
    // this workgroup's slice of the canonical store
    const uint64_t n_can = cnt->n_store[A.cur];
    S.red[0] = lower_bound_glb(A.ck, n_can, A.split[p]);
    S.red[1] = p + 1 < P ? lower_bound_glb(A.ck, n_can, A.split[p + 1]) : n_can;
    // and of N(step0 - 1) (AB2)
    const uint64_t n_prev = A.pk_prev ? cnt->n_prev : 0;
    S.red[2] = A.pk_prev ? lower_bound_glb(A.pk_prev, n_prev, A.split[p]) : 0;
    S.red[3] = A.pk_prev && p + 1 < P ? lower_bound_glb(A.pk_prev, n_prev, A.split[p + 1])
                                      : n_prev;
  }
  __syncthreads();
  const uint64_t cb = S.red[0], ce = S.red[1], qb = S.red[2], qe = S.red[3];
  __syncthreads();

  // Pass k = -1 merges the canonical slice with an empty inbox into segment buffer 0 and draws
  // step0 from it (and, with AB2, the second term of step0 from N(step0 - 1)); pass k >= 0 is
  // step step0 + k: segment buffer k mod nbuf and inbox parity k & 1 in, buffer (k + 1) mod nbuf
  // and parity (k & 1) ^ 1 out, and draws step s + 1 from its outputs (first AB2 term) and its
  // parents (second term).
  uint64_t epoch = A.epoch0 - 1;
  uint64_t st_w = 0, st_k = 0, st_c = 0, st_o = 0;  // statistics of this workgroup (thread 0)
  uint64_t st_d = 0;     // diagonal records among the routed records of the steps run
  uint32_t pend_d = 0;   // diagonal records routed by the last pass (consumed by the next one)
  uint32_t reason = 0, kdone = A.nsteps;
  uint64_t tot_last = 0, tot_prev = 0;  // keys of the last two passes' outputs
  uint64_t mx_ref = 0;  // largest key range right after the split (circuit-aligned ranges)
  const uint32_t rebal_max =
      A.n_circuits == 1 && (A.nbuf == 2 || A.pkw != nullptr) ? A.max_rebal : 0u;
  uint32_t rebal_left = rebal_max;
  static_assert(kPersistTableBytes / 16 == kPBlock, "one table word per thread");
  // table offsets of the current pass, loaded one pass ahead; the table of pass k is the one of
  // step s + 1 (step0 on the first pass, step s itself on the last, which spawns nothing)
  auto tab_index = [&](int32_t kk) -> uint32_t {
    return kk + 1 == (int32_t)A.nsteps ? (uint32_t)kk : (uint32_t)(kk + 1);
  };
  // this workgroup's circuit (its key range lies within one circuit)
  const uint32_t circ = A.kl.replica(S.split[p]) / A.rep_per;
  uint32_t offA = A.tab_off[tab_index(-1) * A.n_circuits + circ];
  uint32_t offB = A.tabB_off && A.nsteps > 0 ? A.tabB_off[0] : 0u;
  uint64_t np_next = 0;  // keys this workgroup wrote in the previous pass
  for (int32_t k = -1; k < (int32_t)A.nsteps; ++k) {
    const bool first = k < 0;
    const uint32_t s = first ? A.step0 : A.step0 + (uint32_t)k;
    if (t == 0) S.ndiag = 0;  // counted by this pass's router (after the inbox barrier below)
    const uint32_t par = (uint32_t)k & 1u;  // 1 for the first pass
    const bool last = k + 1 == (int32_t)A.nsteps;
    const uint32_t ob = (uint32_t)(k + 1) % A.nbuf, ib = (ob + A.nbuf - 1) % A.nbuf;
    const bool two = A.tabB_off && !last && (!first || A.pk_prev);
    // One round of independent loads: the inbox count with the first kPBlock inbox records
    // (read before the count is known; the ones past it are dropped), the step tables (a whole
    // table area per thread block: the device area has that much slack past its end) and the
    // table offsets of the next pass.
    const uint64_t* ibk = A.ik + ((uint64_t)par * P + p) * A.incap;
    const int2* ibv = A.iv + ((uint64_t)par * P + p) * A.incap;
    const uint32_t c_raw = ld_agent(&A.in_n[par * P + p]);
    uint64_t k0 = 0;
    int2 v0 = make_int2(0, 0);
    if (t < A.incap) {
      k0 = ld_agent(&ibk[t]);
      v0 = ld_agent(&ibv[t]);
    }
    S.tab[t] = reinterpret_cast<const uint4*>(A.tab_base + offA)[t];
    if (two) S.tabB[t] = reinterpret_cast<const uint4*>(A.tab_base + offB)[t];
    if (k + 1 < (int32_t)A.nsteps) {
      offA = A.tab_off[tab_index(k + 1) * A.n_circuits + circ];
      if (A.tabB_off && k + 2 < (int32_t)A.nsteps) offB = A.tabB_off[k + 2];
    }
    // inbox of this step -> LDS, sorted (empty on the first pass: zeroed before the launch)
    const uint32_t c = c_raw < A.incap ? c_raw : A.incap;
    if (t == 0 && c_raw > A.incap) raise_err(cnt, &S.err, kErrInbox, s);
    uint32_t m2 = 1;
    while (m2 < c) m2 <<= 1;
    if (t < m2) {
      S.in_k[t] = t < c ? k0 : ~0ull;
      S.in_v[t] = t < c ? v0 : make_int2(0, 0);
    }
    for (uint32_t i = t + kPBlock; i < m2; i += kPBlock) {
      S.in_k[i] = i < c ? ld_agent(&ibk[i]) : ~0ull;
      S.in_v[i] = i < c ? ld_agent(&ibv[i]) : make_int2(0, 0);
    }
    __syncthreads();
    if (t == 0) st_agent(&A.in_n[par * P + p], 0u);  // refilled during pass k+1 (for k+2)
    if (c > 1) sort_inbox(S, m2, c, packed);  // the c real records first, then the padding
    // parents: the canonical slice, or the segment written by the previous pass
    const uint64_t np_k = first ? ce - cb : np_next;
    const uint64_t* pk = first ? A.ck + cb : A.sk + ((uint64_t)ib * P + p) * A.segcap;
    const int2* pv = first ? A.cv + cb : A.sv + ((uint64_t)ib * P + p) * A.segcap;
    uint64_t* okp = A.sk + ((uint64_t)ob * P + p) * A.segcap;
    int2* ovp = A.sv + ((uint64_t)ob * P + p) * A.segcap;
    const uint32_t nstep = first ? A.step0 : s + 1;
    const LTable tn = table_view<lptr>(reinterpret_cast<const uint8_t*>(S.tab));
    const LTable tnB = table_view<lptr>(reinterpret_cast<const uint8_t*>(S.tabB));
    Router R{A.in_n, A.ik, A.iv, A.incap, cnt, S.split, P, pbits, par ^ 1u, nstep, &S.err,
             A.kl.ish, S.st_k[t / kWave], S.st_v[t / kWave], 0u, &S.ndiag};
    merge_segment(A, S, pk, pv, np_k, c, okp, ovp, s, !last, two && !first, R, tn, tnB, nstep);
    const uint64_t nout = S.red[0], wsum = S.red[1];
    if (two && first) {
      // the second AB2 term of step0 from this range of N(step0 - 1)
      advance(A, S, R, tnB, A.qshiftB, 1u, A.pk_prev + qb, A.pv_prev + qb, 0, qe - qb, nstep);
      __syncthreads();
    }
    np_next = nout <= A.segcap ? nout : 0;
    if (t == 0) {
      A.seg_n[ob * P + p] = (uint32_t)np_next;
      if (!first) {
        st_w += wsum;
        st_k += np_k;
        st_c += c;
        st_o += nout;
        st_d += pend_d;
      }
      pend_d = S.ndiag;
    }
    ++epoch;
    if (!grid_sync(S, A, epoch, nout, c)) {
      reason = 2;
      kdone = first ? 0u : (uint32_t)k;
      break;
    }
    // every workgroup reads the same reduced totals and takes the same decision
    const uint64_t tot = S.dec[0], mx = S.dec[1], nin = S.dec[2], ebits = S.dec[3];
    tot_prev = tot_last;
    tot_last = tot;
    const bool cap_store = tot > A.cap_store, cap_in = nin > A.cap_inbox;
    if (ebits || cap_store || cap_in) {
      if (p == 0 && t == 0) {
        if (cap_store) raise_err(cnt, &S.err, kErrStoreCap, s);
        if (cap_in) raise_err(cnt, &S.err, kErrSpawnCap, s);
      }
      reason = 2;
      kdone = first ? 0u : (uint32_t)k;  // refined by the host from err_step
      break;
    }
    if (first) mx_ref = mx;
    const uint64_t ref = tot / P > mx_ref ? tot / P : mx_ref;
    if (!first && !last && mx > ref + ref / 4 + A.rebal_min) {
      if (rebal_left == 0) {
        reason = 1;
        kdone = (uint32_t)k + 1;
        break;
      }
      // Re-split in the kernel (one circuit): N(s+1) of every range goes to the canonical
      // store at its prefix (with AB2 also N(s), this pass's parents, to the N(s-1) array, which
      // only the first pass reads), the records already routed for step s+1 are dropped, the
      // ranges are re-cut at even positions of the estimated cost of N(s+1) (below), and step
      // s+1 is drawn again from the new slices (with AB2 its second term from each range's slice
      // of N(s)) into the same segment buffer and inbox parity; pass k + 1 then runs as usual.
      // The draws are keyed on the walkers, so the records are the same; only their owners
      // change.
      --rebal_left;
      const bool two_rs = A.nbuf == 3 && two;
      {
        // exclusive prefix over the workgroups of the counts of barrier parity `par_b` (64-bit:
        // the counts of all workgroups together may pass 2^32)
        auto prefix_of = [&](uint32_t par_b) -> uint64_t {
          uint64_t mine = t < p ? S.nouts[par_b][t] : 0u;
          for (int o = 32; o > 0; o >>= 1) mine += __shfl_xor(mine, o);
          __syncthreads();
          if (__lane_id() == 0) S.red[t / kWave] = mine;
          __syncthreads();
          uint64_t pre = 0;
          for (int w = 0; w < kPWaves; ++w) pre += S.red[w];
          __syncthreads();
          return pre;
        };
        const uint64_t prefix = prefix_of(epoch & 1u);
        const uint64_t* sk_o = A.sk + ((uint64_t)ob * P + p) * A.segcap;
        const int2* sv_o = A.sv + ((uint64_t)ob * P + p) * A.segcap;
        for (uint64_t i = t; i < nout; i += kPBlock) {
          st_agent(&A.ckw[prefix + i], sk_o[i]);
          st_agent(&A.cvw[prefix + i], sv_o[i]);
        }
        if (two_rs) {
          // N(s): this pass's parents, counted at the previous barrier
          const uint64_t prefix_s = prefix_of((epoch - 1) & 1u);
          const uint64_t* sk_i = A.sk + ((uint64_t)ib * P + p) * A.segcap;
          const int2* sv_i = A.sv + ((uint64_t)ib * P + p) * A.segcap;
          for (uint64_t i = t; i < np_k; i += kPBlock) {
            st_agent(&A.pkw[prefix_s + i], sk_i[i]);
            st_agent(&A.pvw[prefix_s + i], sv_i[i]);
          }
        }
        if (t == 0) st_agent(&A.in_n[(par ^ 1u) * P + p], 0u);
      }
      // The new ranges hold equal estimated cost rather than equal key counts.  A key costs
      // 4 + 3 min(e, G - 1): e = (|a| + |b|) q_off / 2^32 is its expected number of spawned
      // walkers in step s+1, and it routes at most one record per off-diagonal group (a key
      // takes ~29 ns, a routed record ~21 ns).  Each workgroup publishes the cost of its N(s+1);
      // the boundaries r W / P (W the total) that fall in its slice it places at the key whose
      // running cost crosses them; then every workgroup reads the new splitters.
      const uint64_t wq_off = tn_qoff(S);
      const uint32_t wcap = tn_groups(S) > 1 ? tn_groups(S) - 1 : 0u;
      const uint64_t* wsk = A.sk + ((uint64_t)ob * P + p) * A.segcap;
      const int2* wsv = A.sv + ((uint64_t)ob * P + p) * A.segcap;
      auto key_cost = [&](uint64_t i) -> uint32_t {
        const int2 v = wsv[i];
        const uint64_t sab = uabs64(v.x) + uabs64(v.y);
        const uint64_t hi = __umul64hi(sab, wq_off), lo = sab * wq_off;
        const uint64_t e = hi != 0 ? ~0ull : (lo >> 32);
        return 4u + 3u * (uint32_t)(e < wcap ? e : wcap);
      };
      uint64_t wmine = 0;
      for (uint64_t i = t; i < nout; i += kPBlock) wmine += key_cost(i);
      for (int o = 32; o > 0; o >>= 1) wmine += __shfl_xor(wmine, o);
      __syncthreads();
      if (__lane_id() == 0) S.red[t / kWave] = wmine;
      __syncthreads();
      wmine = 0;
      for (int w = 0; w < kPWaves; ++w) wmine += S.red[w];
      wmine = wmine < 0xFFFFFFFFull ? wmine : 0xFFFFFFFFull;  // as the barrier publishes it
      __syncthreads();
      ++epoch;
      if (!grid_sync(S, A, epoch, wmine, 0)) {
        reason = 2;
        kdone = (uint32_t)k + 1;
        break;
      }
      {
        const uint64_t wtot = S.dec[0];
        // cost of the slices before this one (64-bit: the total may pass 2^32)
        uint64_t mine = t < p ? S.nouts[epoch & 1u][t] : 0u;
        for (int o = 32; o > 0; o >>= 1) mine += __shfl_xor(mine, o);
        __syncthreads();
        if (__lane_id() == 0) S.red[t / kWave] = mine;
        __syncthreads();
        uint64_t wpre = 0;
        for (int w = 0; w < kPWaves; ++w) wpre += S.red[w];
        // thread t places boundary t (0 < t < P) at cost t W / P if it falls in this slice
        const uint64_t bnd = t < P ? ((uint64_t)t * wtot) / P : 0;
        const bool own = t > 0 && t < P && bnd >= wpre && bnd < wpre + wmine;
        uint64_t carry = wpre;  // running cost before the current chunk
        for (uint64_t c0 = 0; c0 < nout; c0 += kPBlock) {
          // inclusive scan of this chunk's key costs
          const uint32_t wi = c0 + t < nout ? key_cost(c0 + t) : 0u;
          uint32_t incl = wi;
          for (int o = 1; o < kWave; o <<= 1) {
            const uint32_t x = __shfl_up(incl, o);
            if (__lane_id() >= (uint32_t)o) incl += x;
          }
          __syncthreads();
          if (__lane_id() == kWave - 1) S.scan[t / kWave] = incl;
          __syncthreads();
          uint32_t wbefore = 0, ctot = 0;
          for (int w = 0; w < kPWaves; ++w) {
            wbefore += w < (int)(t / kWave) ? S.scan[w] : 0u;
            ctot += S.scan[w];
          }
          S.xsplit[t] = wbefore + incl;
          __syncthreads();
          if (own && bnd >= carry && bnd < carry + ctot) {
            // the first key of the chunk whose inclusive running cost exceeds the boundary
            const uint32_t tgt = (uint32_t)(bnd - carry);
            uint32_t lo = 0, hi = kPBlock - 1;
            while (lo < hi) {
              const uint32_t mid = (lo + hi) >> 1;
              if (S.xsplit[mid] > tgt)
                hi = mid;
              else
                lo = mid + 1;
            }
            st_agent(&A.splitw[t], wsk[c0 + lo]);
          }
          carry += ctot;
          __syncthreads();
        }
      }
      ++epoch;
      if (!grid_sync(S, A, epoch, 0, 0)) {
        reason = 2;
        kdone = (uint32_t)k + 1;
        break;
      }
      for (uint32_t q = t; q < P; q += kPBlock)
        S.split[q] = q == 0 ? 0ull : ld_agent(&A.splitw[q]);
      __syncthreads();
      uint64_t nout2 = 0;
      if (t == 0) {
        S.red[2] = p == 0 ? 0 : lower_bound_glb(A.ckw, tot, S.split[p], true);
        S.red[3] = p + 1 < P ? lower_bound_glb(A.ckw, tot, S.split[p + 1], true) : tot;
        S.ndiag = 0;  // the records of step s+1 are drawn again
      }
      __syncthreads();
      const uint64_t rb = S.red[2], re = S.red[3];
      __syncthreads();
      {
        uint64_t* okp = A.sk + ((uint64_t)ob * P + p) * A.segcap;
        int2* ovp = A.sv + ((uint64_t)ob * P + p) * A.segcap;
        const LTable tn = table_view<lptr>(reinterpret_cast<const uint8_t*>(S.tab));
        Router R{A.in_n, A.ik, A.iv, A.incap, cnt, S.split, P, pbits, par ^ 1u, s + 1, &S.err,
                 A.kl.ish, S.st_k[t / kWave], S.st_v[t / kWave], 0u, &S.ndiag};
        merge_segment(A, S, A.ckw + rb, A.cvw + rb, re - rb, 0, okp, ovp, s + 1, true, false, R,
                      tn, tn, s + 1, true);
        nout2 = S.red[0];
        if (two_rs) {
          // the second AB2 term of step s+1 from this range's slice of N(s) (tot_prev keys)
          if (t == 0) {
            S.red[2] = p == 0 ? 0 : lower_bound_glb(A.pkw, tot_prev, S.split[p], true);
            S.red[3] = p + 1 < P ? lower_bound_glb(A.pkw, tot_prev, S.split[p + 1], true)
                                 : tot_prev;
          }
          __syncthreads();
          const uint64_t sb = S.red[2], se = S.red[3];
          __syncthreads();
          const LTable tnB = table_view<lptr>(reinterpret_cast<const uint8_t*>(S.tabB));
          advance(A, S, R, tnB, A.qshiftB, 1u, A.pkw + sb, A.pvw + sb, 0, se - sb, s + 1, true);
          __syncthreads();
        }
      }
      np_next = nout2 <= A.segcap ? nout2 : 0;
      if (t == 0) {
        A.seg_n[ob * P + p] = (uint32_t)np_next;
        pend_d = S.ndiag;
      }
      ++epoch;
      if (!grid_sync(S, A, epoch, nout2, 0)) {
        reason = 2;
        kdone = (uint32_t)k + 1;
        break;
      }
      if (S.dec[3]) {
        reason = 2;
        kdone = (uint32_t)k + 1;
        break;
      }
      mx_ref = S.dec[1];
      tot_last = S.dec[0];
    }
  }
  if (t == 0) {
    atomicAdd((unsigned long long*)&cnt->walker_steps, (unsigned long long)st_w);
    atomicAdd((unsigned long long*)&cnt->key_steps, (unsigned long long)st_k);
    atomicAdd((unsigned long long*)&cnt->child_steps, (unsigned long long)st_c);
    atomicAdd((unsigned long long*)&cnt->out_steps, (unsigned long long)st_o);
    atomicAdd((unsigned long long*)&cnt->death_steps, (unsigned long long)st_d);
    if (p == 0) {
      A.done[0] = kdone;
      A.done[1] = reason;
      atomicAdd(&cnt->resplits, rebal_max - rebal_left);
      if (reason != 2 && kdone > 0) {
        // sizes of the stores the host gathers: N(step0 + kdone), and N(step0 + kdone - 1)
        cnt->n_store[A.cur] = tot_last;
        if (A.nbuf == 3) cnt->n_prev = tot_prev;
      }
    }
  }
}

// Splitters, aligned to circuits (a key range then needs one circuit's table): the first
// workgroup of circuit c starts at its lowest composite key (c * rep_per) << kbits, circuit c gets
// 1 + floor((P - C) * n_c / n) workgroups (the rest to the largest circuit) and its other splits
// sit at even positions of its keys.  One circuit: split[p] = the key at index p * n / P.
// One workgroup of kPBlock threads.
__global__ void k_splitters(const uint64_t* __restrict__ ck, const Counters* __restrict__ cnt,
                            uint32_t cur, uint32_t P, uint32_t C, uint32_t rep_per,
                            uint32_t kbits, uint64_t* __restrict__ split) {
  __shared__ uint64_t s_off[kMaxCircuits + 1];
  __shared__ uint32_t s_first[kMaxCircuits + 1];
  const uint32_t t = threadIdx.x;
  const uint64_t n = cnt->n_store[cur];
  auto base_key = [&](uint32_t c) -> uint64_t {
    return kbits >= 64 ? 0ull : ((uint64_t)c * rep_per) << kbits;
  };
  for (uint32_t c = t; c <= C; c += blockDim.x)
    s_off[c] = c == C ? n : (c == 0 ? 0 : lower_bound_glb(ck, n, base_key(c)));
  __syncthreads();
  if (t == 0) {
    uint32_t used = 0, big = 0;
    uint64_t bign = 0;
    for (uint32_t c = 0; c < C; ++c) {
      const uint64_t nc = s_off[c + 1] - s_off[c];
      s_first[c] = used;
      used += 1 + (n ? (uint32_t)(((uint64_t)(P - C) * nc) / n) : 0u);
      if (c == 0 || nc > bign) {
        big = c;
        bign = nc;
      }
    }
    const uint32_t extra = P - used;
    for (uint32_t c = big + 1; c < C; ++c) s_first[c] += extra;
    s_first[C] = P;
  }
  __syncthreads();
  for (uint32_t p = t; p < P; p += blockDim.x) {
    uint32_t lo = 0, hi = C;  // the circuit c with s_first[c] <= p < s_first[c + 1]
    while (hi - lo > 1) {
      const uint32_t mid = (lo + hi) >> 1;
      if (s_first[mid] <= p)
        lo = mid;
      else
        hi = mid;
    }
    const uint32_t c = lo, j = p - s_first[c], a = s_first[c + 1] - s_first[c];
    const uint64_t nc = s_off[c + 1] - s_off[c];
    split[p] = (j == 0 || nc == 0) ? base_key(c) : ck[s_off[c] + (j * nc) / a];
  }
}

// Batch prologue: empty inboxes of the first step, error flags reset.
__global__ void k_persist_prep(Counters* cnt, uint32_t* in_n, uint32_t P, uint32_t* done) {
  const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  for (uint32_t i = t; i < 2 * P; i += gridDim.x * blockDim.x) in_n[i] = 0;
  if (t == 0) {
    done[0] = 0;
    done[1] = 0;
    cnt->err = 0;
    cnt->err_step = 0xFFFFFFFFu;
  }
}

// Segments of buffer `par` -> a sorted store (concatenation in segment order is sorted) whose
// record count goes to *count.
__global__ __launch_bounds__(256) void k_gather(const uint64_t* __restrict__ sk,
                                                const int2* __restrict__ sv,
                                                const uint32_t* __restrict__ seg_n, uint32_t par,
                                                uint32_t P, uint64_t segcap,
                                                uint64_t* __restrict__ ck, int2* __restrict__ cv,
                                                uint64_t* __restrict__ count) {
  __shared__ uint64_t s_off;
  const uint32_t p = blockIdx.x;
  if (threadIdx.x == 0) {
    uint64_t o = 0;
    for (uint32_t q = 0; q < p; ++q) o += seg_n[par * P + q];
    s_off = o;
    if (p == P - 1) *count = o + seg_n[par * P + p];
  }
  __syncthreads();
  const uint64_t off = s_off;
  const uint64_t n = seg_n[par * P + p];
  const uint64_t* k = sk + ((uint64_t)par * P + p) * segcap;
  const int2* v = sv + ((uint64_t)par * P + p) * segcap;
  for (uint64_t i = threadIdx.x; i < n; i += 256) {
    ck[off + i] = k[i];
    cv[off + i] = v[i];
  }
}

// An empty cooperative kernel: the runtime sets up cooperative launches on their first use in
// a process (about 5 ms), which belongs to set-up rather than to the first fused step.
__global__ void k_coop_warm() {}

PersistArgs make_args(const PersistLaunch* L) {
  PersistArgs a;
  a.ck = L->ck;
  a.cv = L->cv;
  a.ckw = L->ck;
  a.cvw = L->cv;
  a.cnt = (Counters*)L->counters;
  a.cur = L->cur;
  a.pk_prev = L->pk_prev;
  a.pv_prev = L->pv_prev;
  a.pkw = L->pk_prev;
  a.pvw = L->pv_prev;
  a.nbuf = L->nbuf;
  a.tabB_off = L->tabB_off;
  a.n_circuits = L->n_circuits;
  a.rep_per = L->rep_per;
  a.qshiftB = L->qshiftB;
  a.sk = L->sk;
  a.sv = L->sv;
  a.segcap = L->segcap;
  a.seg_n = L->seg_n;
  a.ik = L->ik;
  a.iv = L->iv;
  a.incap = L->incap;
  a.in_n = L->in_n;
  a.split = L->split;
  a.P = L->P;
  a.tab_base = L->tab_base;
  a.tab_off = L->tab_off;
  a.step0 = L->step0;
  a.nsteps = L->nsteps;
  a.seed = L->seed;
  a.kl = KeyLayout{L->kbits, L->kbits >= 64 ? ~0ull : ((1ull << L->kbits) - 1),
                   L->init_min ? 1u : 0u, L->init_min};
  a.n_replicas = L->n_replicas;
  a.qshift = L->qshift;
  a.slots = L->slots;
  a.epoch0 = L->epoch0;
  a.cap_store = L->cap_store;
  a.cap_inbox = L->cap_inbox;
  a.rebal_min = L->rebal_min;
  a.max_rebal = L->max_rebal;
  a.splitw = L->split_w;
  a.done = L->done;
  return a;
}

}  // namespace qmc

using namespace qmc;

extern "C" {

int qmcp_max_segments(int* P) {
  int dev = 0, ncu = 0, nb = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  if (e == hipSuccess)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, reinterpret_cast<const void*>(k_persist),
                                                     kPBlock, 0);
  if (e != hipSuccess) return (int)e;
  long long tot = (long long)ncu * (nb > 0 ? nb : 0);
  if (tot > kMaxSegments) tot = kMaxSegments;
  *P = (int)tot;
  return 0;
}

int qmcp_prepare(hipStream_t st, const PersistLaunch* L) {
  hipLaunchKernelGGL(k_persist_prep, dim3(1), dim3(256), 0, st, (Counters*)L->counters, L->in_n,
                     L->P, L->done);
  hipLaunchKernelGGL(k_splitters, dim3(1), dim3(kPBlock), 0, st, L->ck,
                     (const Counters*)L->counters, L->cur, L->P, L->n_circuits, L->rep_per,
                     L->kbits, L->split_w);
  return (int)hipGetLastError();
}

int qmcp_warm(hipStream_t st) {
  void* args[] = {nullptr};
  hipError_t e = hipLaunchCooperativeKernel(reinterpret_cast<const void*>(k_coop_warm), dim3(1),
                                            dim3(kWave), args, 0, st);
  if (e != hipSuccess) return (int)e;
  return (int)hipGetLastError();
}

int qmcp_launch(hipStream_t st, const PersistLaunch* L) {
  PersistArgs a = make_args(L);
  void* args[] = {&a};
  hipError_t e = hipLaunchCooperativeKernel(reinterpret_cast<const void*>(k_persist), dim3(a.P),
                                            dim3(kPBlock), args, 0, st);
  if (e != hipSuccess) return (int)e;
  return (int)hipGetLastError();
}

int qmcp_gather(hipStream_t st, const PersistLaunch* L, uint32_t buf, uint64_t* out_k,
                int2* out_v, uint64_t* out_count) {
  hipLaunchKernelGGL(k_gather, dim3(L->P), dim3(256), 0, st, L->sk, L->sv, L->seg_n, buf, L->P,
                     L->segcap, out_k, out_v, out_count);
  return (int)hipGetLastError();
}

}  // extern "C"
