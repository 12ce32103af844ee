// qmc_small.hip -- the population-dynamics step for stores small enough that one workgroup holds
// a whole replica (gfx950, wave64).
//
// Replicas are independent samples (eq. (3)): walkers of one replica only ever spawn onto keys of
// the same replica.  While every replica has at most kSmallCap occupied keys, workgroup r keeps
// replica (store segment) r in LDS and advances it through a batch of steps alone -- no
// grid-wide synchronization, no global memory traffic but the step tables.  One step of a
// workgroup, for its sorted parents N(s):
//   1. Philox once per parent (step s, its replica, stream 0): w0 (spawn comb), w1 (death comb);
//      the parents whose death or spawn comb can fire are listed;
//   2. each listed parent is taken by a team of T lanes (T = the largest power of two up to 64
//      that gives every parent a team): the diagonal group's terms are split over the team and
//      the partial coefficients added up (integer sums, exact); lane 0 applies the death comb
//      started at w1 to N(s) (End Matter, spawn step, the walker's own key included).  The
//      off-diagonal groups are split over the team in table order; a lane's comb starts at w0
//      plus the amounts of the earlier lanes' groups, mod 2^32, which is where the single comb
//      over all groups in order stands (a comb's remainder after any run of steps is its start
//      plus their amounts, mod 2^32), so every child equals the one of the plain sequential comb.
//      A child landing on an occupied key is added to that key's delta (binary search in LDS,
//      LDS atomics); one landing elsewhere goes to a list of new records (dropped if its parent
//      is not an initiator);
//   3. the new records are sorted (rank by counting) and merged with the parents plus their
//      deltas: int64 sums, int32 range check, (0, 0) dropped (annihilation, End Matter) -> N(s+1).
// A workgroup whose replica outgrows the key limit, produces more than kSmallNew new records in
// one step, or leaves int32 records the step in the chain's stop word and stops.  The host
// launches a call's steps as a chain of batches of at most kSmallBatch steps, each reading the
// segments the one before wrote, then the gather of the last batch's segments into the canonical
// store and the commit of the statistics; a workgroup takes no step at or after the step the stop
// word records, and the chain's gather and commit do nothing once it is set, so after a stop the
// recorded step is the earliest at which any replica failed, the last complete batch's segments
// hold the state, and the host gathers them, runs the steps up to the stop again from there (the
// results are the same, the draws being keyed on the walkers) and continues with the other step
// paths.  The stop word is
// (chain epoch << 32) | ~step, raised with atomicMax: it belongs to a chain only when it carries
// that chain's epoch (no reset between chains), and within a chain it keeps the earliest step.
#include "qmc_device.hpp"
#include "qmc_persist.h"
#include "qmc_small.h"

namespace qmc {

constexpr int kSBlock = 512;
constexpr int kSWaves = kSBlock / kWave;
constexpr int kSTab = kPersistTableBytes / 16;  // uint4 words of a step table
constexpr uint32_t kActIdx = 0xFFFFu;           // active-list entry: parent index, comb flags
constexpr uint32_t kActD = 1u << 16;
constexpr uint32_t kActS = 1u << 17;
static_assert(kSmallCap <= (int)kActIdx + 1, "parent index in 16 bits");
static_assert(kSmallCap < 65536 && kSmallNew < 65536, "merge split points in 16 bits");

struct SmallArgs {
  const uint64_t* ck;       // canonical store (all segments, sorted), n_store[cur] records; or
  const int2* cv;           // null: the input is segment `seg` of (ik, iv, in_n)
  const Counters* cnt;
  uint32_t cur;
  const uint64_t* ik;       // input segments [R][segcap], counts in_n
  const int2* iv;
  const uint32_t* in_n;
  uint64_t* ok;             // output segments [R][segcap], counts out_n
  int2* ov;
  uint32_t* out_n;
  uint64_t segcap;
  const uint8_t* tab_base;  // step k of circuit c at tab_base + tab_off[k * n_circuits + c]
  const uint32_t* tab_off;
  uint32_t n_circuits, rep_per;
  uint32_t step0, nsteps;
  uint64_t seed;
  KeyLayout kl;
  const int64_t* qshift;    // per-segment Q32 shifts
  uint32_t cap_store;       // keys per replica allowed (at most kSmallCap)
  uint64_t cap_spawn;       // records (children and death deltas) per replica and step allowed
  uint32_t check_spawn;     // nonzero: cap_spawn can be reached, count each step's records
  unsigned long long* stop; // the chain's stop word (see above)
  uint32_t epoch;
  uint64_t* stats;          // [R][kSmallStats] of this batch
};

__device__ __forceinline__ bool chain_stopped(const unsigned long long* stop, uint32_t epoch) {
  return (uint32_t)(__hip_atomic_load(stop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >> 32) ==
         epoch;
}

__device__ __forceinline__ void chain_stop(unsigned long long* stop, uint32_t epoch,
                                           uint32_t step) {
  atomicMax(stop, ((unsigned long long)epoch << 32) | (0xFFFFFFFFu - step));
}

// Whether stop word `w` stops this chain at or before step s: step s and the later ones are then
// dropped anyway.  A workgroup still before the recorded step must go on, since one of its own
// steps before it may be the chain's earliest stop (workgroups advance at different speeds).
__device__ __forceinline__ bool stopped_by(unsigned long long w, uint32_t epoch, uint32_t s) {
  return (uint32_t)(w >> 32) == epoch && 0xFFFFFFFFu - (uint32_t)w <= s;
}

struct SmallShared {
  uint64_t pk[2][kSmallCap];
  int2 pv[2][kSmallCap];
  unsigned long long dre[kSmallCap];   // int64 deltas (two's complement) of the parents
  unsigned long long dim[kSmallCap];
  uint64_t ak[kSmallCap];              // parents whose death or spawn comb can fire: key,
  int2 av[kSmallCap];                  // value, Philox words (x spawn, y death),
  uint2 aw[kSmallCap];                 // index | comb flags
  uint32_t ai[kSmallCap];
  uint64_t nk[kSmallNew];              // new records: composite key, value
  int2 nv[kSmallNew];
  uint64_t sk[kSmallNew];              // the same, sorted
  int2 sv[kSmallNew];
  uint4 tab[2][kSTab];
  uint32_t xsplit[kSBlock];
  uint32_t scan[kSWaves];
  uint64_t red[3 * kSWaves];
  // per step, by step parity (step k resets the words of step k + 1 after its first barrier,
  // when every thread is done with those of step k - 1): new records, listed parents, records
  // of the step (when the spawn capacity is checked), a limit exceeded
  uint32_t nnew[2];
  uint32_t nact[2];
  uint32_t nrec[2];
  uint32_t flag[2];
  uint32_t toff[kSmallBatch];          // table offsets of the batch's steps (this circuit)
};
static_assert(kSTab == kSBlock, "one 16-byte word of a step table per thread");

__global__ __launch_bounds__(kSBlock) void k_small(SmallArgs A) {
  __shared__ SmallShared S;
  const uint32_t t = threadIdx.x, wave = t / kWave, lane = __lane_id();
  const uint32_t seg = blockIdx.x;
  const KeyLayout kl = A.kl;
  const uint32_t circ = seg / A.rep_per;
  const int64_t qs = A.qshift[seg];
  // this replica's input records; nothing at all once the chain stopped at or before the first
  // step of this batch
  if (t == 0) {
    const uint32_t stop = stopped_by(
        __hip_atomic_load(A.stop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT), A.epoch, A.step0);
    uint64_t a = 0, e = 0;
    if (!stop && A.ck) {
      const uint64_t n_can = A.cnt->n_store[A.cur];
      const uint64_t lo = kl.kbits >= 64 ? 0 : ((uint64_t)seg << kl.kbits);
      uint64_t x = 0, y = n_can;
      while (x < y) {
        const uint64_t m = (x + y) >> 1;
        if (A.ck[m] < lo) x = m + 1; else y = m;
      }
      a = x;
      e = n_can;
      if (kl.kbits < 64) {
        const uint64_t hi = (uint64_t)(seg + 1) << kl.kbits;
        y = n_can;
        while (x < y) {
          const uint64_t m = (x + y) >> 1;
          if (A.ck[m] < hi) x = m + 1; else y = m;
        }
        e = x;
      }
    } else if (!stop) {
      a = (uint64_t)seg * A.segcap;
      e = a + A.in_n[seg];
    }
    S.red[0] = a;
    S.red[1] = e;
    S.flag[0] = stop;
  }
  __syncthreads();
  if (S.flag[0]) return;
  const uint64_t base = S.red[0];
  if (S.red[1] - base > (uint64_t)A.cap_store) {
    if (t == 0) chain_stop(A.stop, A.epoch, A.step0);
    return;
  }
  uint32_t n = (uint32_t)(S.red[1] - base);
  const uint64_t* srck = A.ck ? A.ck : A.ik;
  const int2* srcv = A.ck ? A.cv : A.iv;
  for (uint32_t i = t; i < n; i += kSBlock) {
    S.pk[0][i] = srck[base + i];
    S.pv[0][i] = srcv[base + i];
  }
  // Step tables go through registers: thread t loads the t-th 16 bytes of the next step's table
  // (a table area of kPersistTableBytes bytes; the table memory has that much slack past its
  // end) at the start of a step and stores them to LDS at its end, so no LDS access of the step
  // waits for the load.  The tables may sit in host memory: the batch's table offsets are read
  // once, into LDS, so each step's prefetch is one read.
  if (t < A.nsteps) S.toff[t] = A.tab_off[(size_t)t * A.n_circuits + circ];
  auto table_word = [&](uint32_t kk) {
    return reinterpret_cast<const uint4*>(A.tab_base + S.toff[kk])[t];
  };
  if (A.nsteps > 0) S.tab[0][t] = reinterpret_cast<const uint4*>(A.tab_base + A.tab_off[circ])[t];
  __syncthreads();  // every thread has read the start flag; the table offsets are in LDS
  if (t == 0) {
    S.nnew[0] = 0;
    S.nact[0] = 0;
    S.nrec[0] = 0;
    S.flag[0] = 0;
  }
  // statistics, per thread over the batch (walkers, death records, children); keys and outputs
  // in thread 0
  uint64_t st_w = 0, st_k = 0, st_o = 0;
  uint32_t st_d = 0, st_c = 0;
  uint32_t b = 0;  // parent buffer
  uint32_t kdone = 0;
  // The chain's stop word, read by thread 0 during each step and looked at one step later (the
  // load's latency hidden; the recorded step only moves earlier, so an old value is safe): once
  // another workgroup has stopped the chain at or before the step this one is about to take,
  // the rest of this workgroup's batch is dropped anyway, so it halts.
  unsigned long long seen = 0;
  bool halted = false;
  for (uint32_t k = 0; k < A.nsteps; ++k) {
    const uint32_t s = A.step0 + k;
    const uint32_t p = k & 1;
    if (t == 0 && k > 0 && stopped_by(seen, A.epoch, s)) S.flag[p] = 3;
    __syncthreads();  // the parents, this step's table and counters
    if (S.flag[p] == 3) {  // block-uniform
      halted = true;
      break;
    }
    if (t == 0) {
      S.nnew[p ^ 1] = 0;
      S.nact[p ^ 1] = 0;
      S.nrec[p ^ 1] = 0;
      S.flag[p ^ 1] = 0;
    }
    const bool more = k + 1 < A.nsteps;
    const uint4 tnext = more ? table_word(k + 1) : make_uint4(0, 0, 0, 0);
    if (t == 0) seen = __hip_atomic_load(A.stop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const TableViewT<lptr> tv = table_view<lptr>(reinterpret_cast<const uint8_t*>(S.tab[k & 1]));
    const uint32_t G = tv.h->n_groups;
    const uint64_t q_off = G > 1 ? tv.h->q_off : 0, q_diag = tv.h->q_diag + uabs64(qs);
    // 1: Philox, walker statistics, deltas cleared, list of the parents that can fire
    for (uint32_t i0 = 0; i0 < n; i0 += kSBlock) {  // block-uniform
      const uint32_t i = i0 + t;
      bool dact = false, sact = false;
      uint64_t ck = 0;
      int2 v = make_int2(0, 0);
      uint32_t r4[4] = {0, 0, 0, 0};
      if (i < n) {
        ck = S.pk[b][i];
        v = S.pv[b][i];
        walker_random(kl.key(ck), s, seg, A.seed, 0u, r4);
        const uint64_t sab = uabs64(v.x) + uabs64(v.y);
        st_w += sab;
        dact = !comb_all_zero(sab, q_diag, r4[1]);
        sact = !comb_all_zero(sab, q_off, r4[0]);
        S.dre[i] = 0;
        S.dim[i] = 0;
      }
      const bool act = dact || sact;
      const uint64_t m = __ballot(act);
      if (m) {  // wave-uniform
        uint32_t at = 0;
        if (lane == 0) at = atomicAdd(&S.nact[p], (uint32_t)__popcll(m));
        at = __shfl(at, 0);
        if (act) {
          const uint32_t j = at + (uint32_t)__popcll(m & lanemask_lt());
          S.ak[j] = ck;
          S.av[j] = v;
          S.aw[j] = make_uint2(r4[0], r4[1]);
          S.ai[j] = i | (dact ? kActD : 0u) | (sact ? kActS : 0u);
        }
      }
    }
    __syncthreads();
    // 2: death deltas and children, a team of T lanes per listed parent
    const uint32_t nact = S.nact[p];
    uint32_t T = 1;
    while (T < (uint32_t)kWave && 2 * T * nact <= (uint32_t)kSBlock) T *= 2;
    const uint32_t lt = t & (T - 1), nteam = kSBlock / T, team = t / T;
    const uint32_t nd = tv.gs[1] / kTermPad;
    const uint32_t d0 = nd * lt / T * kTermPad, d1 = nd * (lt + 1) / T * kTermPad;
    const uint32_t g0 = 1 + (G - 1) * lt / T, g1 = 1 + (G - 1) * (lt + 1) / T;
    uint32_t nrec = 0;  // records of this thread in this step
    for (uint32_t a0 = 0; a0 < nact; a0 += nteam) {  // block-uniform
      const uint32_t ai = a0 + team;
      const bool has = ai < nact;  // team-uniform
      const uint32_t e = has ? S.ai[ai] : 0u;
      const uint32_t i = e & kActIdx;
      const bool dact = (e & kActD) != 0, sact = (e & kActS) != 0;
      const uint64_t ck = has ? S.ak[ai] : 0;
      const int2 v = has ? S.av[ai] : make_int2(0, 0);
      const uint2 w = has ? S.aw[ai] : make_uint2(0, 0);
      const uint64_t key = kl.key(ck);
      // death: partial diagonal coefficients over the team's slices of the group 0 terms
      int32_t pre = 0, pim = 0;
      if (dact) group_coeff_part(tv.t, d0, d1, key, pre, pim);
      pre = (int32_t)team_sum((uint32_t)pre, T);
      pim = (int32_t)team_sum((uint32_t)pim, T);
      if (dact && lt == 0) {
        int64_t xre, xim;
        cmul_q32(v.x, v.y, pre + (int32_t)qs, pim, xre, xim);
        uint64_t r = w.y;
        const int64_t dx = comb_step(r, xre), dy = comb_step(r, xim);
        if ((dx | dy) != 0) {
          atomicAdd(&S.dre[i], (unsigned long long)dx);
          atomicAdd(&S.dim[i], (unsigned long long)dy);
          ++st_d;
          ++nrec;
        }
      }
      // spawn: the comb of lane lt starts after the amounts of the team's earlier lanes; the
      // lane's first group keeps its amounts from the first pass
      int64_t x0re = 0, x0im = 0;
      uint32_t amt = 0;
      if (sact && T > 1) {
        for (uint32_t g = g0; g < g1; ++g) {
          int32_t cre, cim;
          group_coeff(tv.t, tv.gs[g], tv.gs[g + 1], key, cre, cim);
          int64_t xre, xim;
          cmul_q32(v.x, v.y, cre, cim, xre, xim);
          if (g == g0) {
            x0re = xre;
            x0im = xim;
          }
          amt += (uint32_t)uabs64(xre) + (uint32_t)uabs64(xim);
        }
      }
      const uint32_t incl = team_scan(amt, T, lt);
      if (sact) {
        const bool initiator = uabs64(v.x) + uabs64(v.y) >= kl.init_min;
        uint64_t r = (uint32_t)(w.x + (incl - amt));
        for (uint32_t g = g0; g < g1; ++g) {
          int64_t xre, xim;
          if (g == g0 && T > 1) {
            xre = x0re;
            xim = x0im;
          } else {
            int32_t cre, cim;
            group_coeff(tv.t, tv.gs[g], tv.gs[g + 1], key, cre, cim);
            cmul_q32(v.x, v.y, cre, cim, xre, xim);
          }
          const int64_t nre = comb_step(r, xre), nim = comb_step(r, xim);
          if ((nre | nim) == 0) continue;
          ++st_c;
          ++nrec;
          const uint64_t tk = ck ^ tv.gx[g];
          uint32_t lo = 0, hi = n;
          while (lo < hi) {
            const uint32_t m = (lo + hi) >> 1;
            if (S.pk[b][m] < tk) lo = m + 1; else hi = m;
          }
          if (lo < n && S.pk[b][lo] == tk) {
            atomicAdd(&S.dre[lo], (unsigned long long)nre);
            atomicAdd(&S.dim[lo], (unsigned long long)nim);
          } else if (initiator) {
            const uint32_t at = atomicAdd(&S.nnew[p], 1u);
            if (at < (uint32_t)kSmallNew) {
              S.nk[at] = tk;
              S.nv[at] = make_int2((int32_t)nre, (int32_t)nim);
            } else {
              S.flag[p] = 1;
            }
          }
        }
      }
    }
    if (A.check_spawn) {  // records of the step against the spawn capacity
      const uint32_t wr = team_sum(nrec, kWave);
      if (lane == 0 && wr) atomicAdd(&S.nrec[p], wr);
    }
    if (t == 0) st_k += n;
    __syncthreads();
    const uint32_t nn = S.nnew[p] < (uint32_t)kSmallNew ? S.nnew[p] : (uint32_t)kSmallNew;
    if (S.flag[p] || S.nrec[p] > A.cap_spawn) break;  // block-uniform: the step does not fit
    // 3a: the new records in key order (rank = smaller keys, then equal keys of smaller index)
    for (uint32_t i = t; i < nn; i += kSBlock) {
      const uint64_t ki = S.nk[i];
      uint32_t rank = 0;
      for (uint32_t j = 0; j < nn; ++j) {
        const uint64_t kj = S.nk[j];
        rank += (kj < ki || (kj == ki && j < i)) ? 1u : 0u;
      }
      S.sk[rank] = ki;
      S.sv[rank] = S.nv[i];
    }
    __syncthreads();
    // 3b: merge of the parents (plus deltas) with the sorted new records, split over the threads
    // at run ends (a run is one parent or a run of new records of one key: at most one child of
    // a key per off-diagonal group, fewer than the split's search window)
    const uint32_t tot = n + nn;
    const uint32_t per = (tot + kSBlock - 1) / kSBlock;
    auto KA = [&](uint32_t x) { return S.pk[b][x]; };
    auto KB = [&](uint32_t x) { return S.sk[x]; };
    uint32_t d = t * per;
    if (d > tot) d = tot;
    uint32_t i0, j0;
    run_split(KA, n, KB, nn, d, i0, j0);
    S.xsplit[t] = i0 | (j0 << 16);
    __syncthreads();
    uint32_t i1, j1;
    if (t + 1 < (uint32_t)kSBlock) {
      i1 = S.xsplit[t + 1] & 0xFFFFu;
      j1 = S.xsplit[t + 1] >> 16;
    } else {
      i1 = n;
      j1 = nn;
    }
    auto walk = [&](auto&& out) __attribute__((always_inline)) {
      uint32_t i = i0, j = j0;
      while (i < i1 || j < j1) {
        uint64_t key;
        int64_t re, im;
        if (j >= j1 || (i < i1 && S.pk[b][i] <= S.sk[j])) {
          key = S.pk[b][i];
          re = (int64_t)S.pv[b][i].x + (int64_t)S.dre[i];
          im = (int64_t)S.pv[b][i].y + (int64_t)S.dim[i];
          ++i;
        } else {
          key = S.sk[j];
          re = im = 0;
        }
        while (j < j1 && S.sk[j] == key) {
          re += S.sv[j].x;
          im += S.sv[j].y;
          ++j;
        }
        out(key, re, im);
      }
    };
    uint32_t count = 0;
    bool over = false;
    walk([&](uint64_t, int64_t re, int64_t im) __attribute__((always_inline)) {
      if (re < INT32_MIN || re > INT32_MAX || im < INT32_MIN || im > INT32_MAX) over = true;
      count += (re != 0 || im != 0) ? 1u : 0u;
    });
    const uint32_t incl = team_scan(count, kWave, lane);
    if (over) S.flag[p] = 2;
    if (lane == kWave - 1) S.scan[wave] = incl;
    __syncthreads();
    uint32_t wpre = 0, agg = 0;
    for (uint32_t x = 0; x < (uint32_t)kSWaves; ++x) {
      wpre += x < wave ? S.scan[x] : 0u;
      agg += S.scan[x];
    }
    if (S.flag[p] || agg > A.cap_store) break;  // block-uniform
    uint32_t o = wpre + incl - count;
    walk([&](uint64_t key, int64_t re, int64_t im) __attribute__((always_inline)) {
      if (re != 0 || im != 0) {
        S.pk[b ^ 1][o] = key;
        S.pv[b ^ 1][o] = make_int2((int32_t)re, (int32_t)im);
        ++o;
      }
    });
    if (more) S.tab[(k + 1) & 1][t] = tnext;
    if (t == 0) st_o += agg;
    n = agg;
    b ^= 1;
    kdone = k + 1;
  }
  if (kdone < A.nsteps) {
    // this replica could not take step step0 + kdone (more keys or new records than the LDS
    // holds, a population outside int32, or more records than the spawn capacity), or another
    // one stopped the chain first
    if (t == 0 && !halted) chain_stop(A.stop, A.epoch, A.step0 + kdone);
    return;
  }
  __syncthreads();  // the last step's outputs
  uint64_t* ok = A.ok + (uint64_t)seg * A.segcap;
  int2* ov = A.ov + (uint64_t)seg * A.segcap;
  for (uint32_t i = t; i < n; i += kSBlock) {
    ok[i] = S.pk[b][i];
    ov[i] = S.pv[b][i];
  }
  // the batch's statistics: block sums of the per-thread ones
  for (int o = 32; o > 0; o >>= 1) {
    st_w += __shfl_xor(st_w, o);
    st_d += __shfl_xor(st_d, o);
    st_c += __shfl_xor(st_c, o);
  }
  if (lane == 0) {
    S.red[wave] = st_w;
    S.red[kSWaves + wave] = st_d;
    S.red[2 * kSWaves + wave] = st_c;
  }
  __syncthreads();
  if (t == 0) {
    uint64_t w = 0, dd = 0, cc = 0;
    for (int x = 0; x < kSWaves; ++x) {
      w += S.red[x];
      dd += S.red[kSWaves + x];
      cc += S.red[2 * kSWaves + x];
    }
    A.out_n[seg] = n;
    uint64_t* st = A.stats + (uint64_t)seg * kSmallStats;
    st[0] = w;
    st[1] = st_k;
    st[2] = cc + dd;
    st[3] = st_o;
    st[4] = dd;
  }
}

// The end of a chain (one launch): the last batch's segments into the canonical store and the
// statistics of the completed batches into the counters (by workgroup 0) -- neither when the
// chain stopped (stop == null: always); workgroup 0 also copies the stop word into the counters,
// for the host's one read of them.  Either one workgroup per segment, or one workgroup for all
// of at most kFinishSegs segments (their records copied in one flattened pass), which, given a
// mirror, then writes the whole counters there (host-visible memory, system-scope stores).
constexpr uint32_t kFinishSegs = 64;

__global__ __launch_bounds__(256) void k_small_finish(const uint64_t* __restrict__ sk,
                                                      const int2* __restrict__ sv,
                                                      const uint32_t* __restrict__ seg_n,
                                                      uint64_t segcap, uint32_t n_seg,
                                                      uint64_t* __restrict__ ck,
                                                      int2* __restrict__ cv, uint64_t* count,
                                                      Counters* cnt, const uint64_t* stats,
                                                      uint32_t nrows,
                                                      const unsigned long long* stop,
                                                      uint32_t epoch, uint64_t* mirror) {
  __shared__ uint64_t s_pre[kFinishSegs + 1];
  __shared__ uint32_t s_skip;
  __shared__ unsigned long long s_sum[kSmallStats];
  const uint32_t b = blockIdx.x, t = threadIdx.x;
  if (t == 0) {
    s_skip = stop && chain_stopped(stop, epoch);
    if (stop && b == 0) cnt->small_stop = *stop;
  }
  if (b == 0 && t < (uint32_t)kSmallStats) s_sum[t] = 0;
  if (gridDim.x == 1 && t < n_seg) s_pre[t + 1] = seg_n[t];
  __syncthreads();
  const bool skip = s_skip;
  if (!skip && gridDim.x == 1) {
    // all segments here: offsets first, then every record of every segment at once
    if (t == 0) {
      s_pre[0] = 0;
      for (uint32_t q = 0; q < n_seg; ++q) s_pre[q + 1] += s_pre[q];
      *count = s_pre[n_seg];
    }
    __syncthreads();
    const uint64_t total = s_pre[n_seg];
    for (uint64_t i = t; i < total; i += 256) {
      uint32_t lo = 0, hi = n_seg;  // the segment q with s_pre[q] <= i < s_pre[q + 1]
      while (hi - lo > 1) {
        const uint32_t m = (lo + hi) >> 1;
        if (s_pre[m] <= i) lo = m; else hi = m;
      }
      const uint64_t src = (uint64_t)lo * segcap + (i - s_pre[lo]);
      ck[i] = sk[src];
      cv[i] = sv[src];
    }
  } else if (!skip) {
    // segment b: its offset is the sum of the counts before it
    const uint32_t p = b;
    __shared__ uint64_t s_off;
    if (t == 0) {
      uint64_t o = 0;
      for (uint32_t q = 0; q < p; ++q) o += seg_n[q];
      s_off = o;
      if (p == n_seg - 1) *count = o + seg_n[p];
    }
    __syncthreads();
    const uint64_t off = s_off, n = seg_n[p];
    const uint64_t* k = sk + (uint64_t)p * segcap;
    const int2* v = sv + (uint64_t)p * segcap;
    for (uint64_t i = t; i < n; i += 256) {
      ck[off + i] = k[i];
      cv[off + i] = v[i];
    }
  }
  if (b != 0) return;  // block-uniform
  if (!skip) {
    for (uint32_t i = t; i < nrows * (uint32_t)kSmallStats; i += blockDim.x)
      atomicAdd(&s_sum[i % kSmallStats], (unsigned long long)stats[i]);
    __syncthreads();
    if (t == 0) {
      cnt->walker_steps += s_sum[0];
      cnt->key_steps += s_sum[1];
      cnt->child_steps += s_sum[2];
      cnt->out_steps += s_sum[3];
      cnt->death_steps += s_sum[4];
    }
  }
  if (mirror && gridDim.x == 1) {
    // every counter write of the chain is done: the earlier kernels', and thread 0's here
    // (fenced at device scope before the barrier)
    __threadfence();
    __syncthreads();
    const uint64_t* w = reinterpret_cast<const uint64_t*>(cnt);
    constexpr uint32_t kWords = (uint32_t)(sizeof(Counters) / 8);
    for (uint32_t i = t; i < kWords; i += blockDim.x)
      __hip_atomic_store(&mirror[i],
                         __hip_atomic_load(&w[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT),
                         __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
  }
}

}  // namespace qmc

using namespace qmc;

extern "C" {

int qmcs_launch(hipStream_t st, const SmallLaunch* L) {
  if (L->nsteps > kSmallBatch) return (int)hipErrorInvalidValue;  // the batch's offsets in LDS
  SmallArgs a;
  a.ck = L->ck;
  a.cv = L->cv;
  a.cnt = (const Counters*)L->counters;
  a.cur = L->cur;
  a.ik = L->ik;
  a.iv = L->iv;
  a.in_n = L->in_n;
  a.ok = L->ok;
  a.ov = L->ov;
  a.out_n = L->out_n;
  a.segcap = L->segcap;
  a.tab_base = L->tab_base;
  a.tab_off = L->tab_off;
  a.n_circuits = L->n_circuits;
  a.rep_per = L->rep_per;
  a.step0 = L->step0;
  a.nsteps = L->nsteps;
  a.seed = L->seed;
  a.kl = KeyLayout{L->kbits, L->kbits >= 64 ? ~0ull : ((1ull << L->kbits) - 1), 0u,
                   L->init_min};
  a.qshift = L->qshift;
  a.cap_store = (uint32_t)(L->cap_store < (uint64_t)kSmallCap ? L->cap_store : kSmallCap);
  a.cap_spawn = L->cap_spawn;
  // a step has at most (keys) x (groups) records: no count needed below that
  a.check_spawn = L->cap_spawn < (uint64_t)a.cap_store * (uint64_t)(kMaxGroups + 1);
  a.stop = L->stop;
  a.epoch = L->epoch;
  a.stats = L->stats;
  hipLaunchKernelGGL(k_small, dim3(L->n_segments), dim3(kSBlock), 0, st, a);
  return (int)hipGetLastError();
}

int qmcs_finish(hipStream_t st, const uint64_t* sk, const int2* sv, const uint32_t* seg_n,
                uint64_t segcap, uint32_t n_segments, uint64_t* ck, int2* cv, uint64_t* count,
                void* counters, const uint64_t* stats, uint32_t nrows,
                const unsigned long long* stop, uint32_t epoch, uint32_t n_blocks,
                void* mirror) {
  // one workgroup for all only up to kFinishSegs segments, else one per segment
  const uint32_t g = n_blocks == 1 && n_segments <= kFinishSegs ? 1u : n_segments;
  hipLaunchKernelGGL(k_small_finish, dim3(g), dim3(256), 0, st, sk, sv, seg_n, segcap,
                     n_segments, ck, cv, count, (Counters*)counters, stats, nrows, stop, epoch,
                     g == 1 ? (uint64_t*)mirror : nullptr);
  return (int)hipGetLastError();
}

}  // extern "C"
