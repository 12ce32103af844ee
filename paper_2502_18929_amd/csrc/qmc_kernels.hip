// qmc_kernels.hip -- HIP kernels of one population-dynamics time step (gfx950, wave64).
//
// Step s (End Matter, spawn and annihilation; Euler solver):
//   k_spawn          parents N(s) -> child records (key ^ mask, comb-rounded dt L N), unsorted
//   k_radix_*        LSD radix sort of the child records by composite key (LDS ranking)
//   k_merge_part     merge-path split points of (parents, sorted children), moved to run ends
//   k_merge          death/cloning of each parent (diagonal of the column, applied to N(s)),
//                    merge with the children, int64 segmented sum per key, drop (0, 0),
//                    decoupled look-back for the compacted output offset -> N(s+1)
// plus k_pulse (ideal Pauli conjugation), k_observe / k_lookup (estimator numerators) and
// small utility kernels.  Every kernel reads its problem sizes from device memory, so a whole
// batch of steps is enqueued without host synchronization.
#include "qmc_device.hpp"
#include "qmc_kernels.h"

namespace qmc {

struct TableView {
  const TableHeader* h;
  const uint64_t* gx;
  const uint32_t* gs;
  const Term* t;
};

__device__ __forceinline__ TableView table_view(const uint8_t* tab) {
  TableView v;
  v.h = reinterpret_cast<const TableHeader*>(tab);
  v.gx = reinterpret_cast<const uint64_t*>(tab + v.h->gx_off);
  v.gs = reinterpret_cast<const uint32_t*>(tab + v.h->gs_off);
  v.t = reinterpret_cast<const Term*>(tab + v.h->t_off);
  return v;
}

struct KeyLayout {
  uint32_t kbits;   // 2n
  uint64_t kmask;   // (1 << 2n) - 1
  __device__ __forceinline__ uint64_t key(uint64_t ck) const { return ck & kmask; }
  __device__ __forceinline__ uint32_t replica(uint64_t ck) const {
    return kbits >= 64 ? 0u : (uint32_t)(ck >> kbits);
  }
};

__device__ __forceinline__ void walker_random(uint64_t key, uint32_t step, uint32_t replica,
                                              uint64_t seed, uint32_t w[4]) {
  philox4x32_10((uint32_t)key, (uint32_t)(key >> 32), step, replica << 8, (uint32_t)seed,
                (uint32_t)(seed >> 32), w);
}

// Group coefficient c = sum_t (-1)^parity(zmask_t & key) q_t; |c_re| + |c_im| < 2^31.
__device__ __forceinline__ void group_coeff(const Term* __restrict__ t, uint32_t b, uint32_t e,
                                            uint64_t key, int32_t& cre, int32_t& cim) {
  int32_t re = 0, im = 0;
  for (uint32_t i = b; i < e; ++i) {
    const Term tm = t[i];
    const int32_t s = -(int32_t)parity64(tm.zmask & key);  // 0 or -1
    re += (tm.qre ^ s) - s;
    im += (tm.qim ^ s) - s;
  }
  cre = re;
  cim = im;
}

__device__ __forceinline__ void cmul_q32(int64_t a, int64_t b, int32_t cre, int32_t cim,
                                         int64_t& xre, int64_t& xim) {
  xre = a * (int64_t)cre - b * (int64_t)cim;
  xim = a * (int64_t)cim + b * (int64_t)cre;
}

// ---------------------------------------------------------------------------------------------
// k_spawn: one lane per parent; child records are staged per wave in LDS and flushed to the
// child buffer with one global atomic per flush.
// ---------------------------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_spawn(
    const uint64_t* __restrict__ pk, const int2* __restrict__ pv, Counters* __restrict__ cnt,
    uint32_t cur, const uint8_t* __restrict__ tab, uint32_t step, uint64_t seed, KeyLayout kl,
    uint64_t* __restrict__ ck_out, int2* __restrict__ cv_out, uint64_t cap_child) {
  __shared__ uint64_t s_key[kWaves][kSpawnSeg];
  __shared__ int2 s_val[kWaves][kSpawnSeg];
  if (cnt->err) return;
  const uint64_t np = cnt->n_store[cur];
  const TableView tv = table_view(tab);
  const uint32_t G = tv.h->n_groups;
  const uint64_t q_off = tv.h->q_off;
  const uint32_t wave = threadIdx.x / kWave, lane = __lane_id();
  uint32_t fill = 0;  // wave-uniform
  uint64_t* my_key = s_key[wave];
  int2* my_val = s_val[wave];
  const uint64_t stride = (uint64_t)gridDim.x * kBlock;

  auto flush = [&]() {
    wave_lds_fence();
    uint64_t base = 0;
    if (lane == 0) base = atomicAdd((unsigned long long*)&cnt->n_child[step & 1], (unsigned long long)fill);
    base = __shfl(base, 0);
    if (base + fill > cap_child) {
      if (lane == 0) {
        atomicOr(&cnt->err, kErrSpawnCap);
        atomicMin(&cnt->err_step, step);
      }
    } else {
      for (uint32_t i = lane; i < fill; i += kWave) {
        ck_out[base + i] = my_key[i];
        cv_out[base + i] = my_val[i];
      }
    }
    wave_lds_fence();
    fill = 0;
  };

  if (G > 1) {
    for (uint64_t wbase = (uint64_t)blockIdx.x * kBlock + wave * kWave; wbase < np;
         wbase += stride) {
      const uint64_t p = wbase + lane;
      const bool valid = p < np;
      uint64_t ck = 0;
      int2 v = make_int2(0, 0);
      uint32_t w[4] = {0, 0, 0, 0};
      bool active = false;
      if (valid) {
        ck = pk[p];
        v = pv[p];
        walker_random(kl.key(ck), step, kl.replica(ck), seed, w);
        const uint64_t s = uabs64(v.x) + uabs64(v.y);
        active = !comb_all_zero(s, q_off, w[0]);
      }
      if (__ballot(active) == 0) continue;
      const uint64_t key = kl.key(ck);
      uint64_t r = w[0];
      for (uint32_t g = 1; g < G; ++g) {
        int2 child = make_int2(0, 0);
        if (active) {
          int32_t cre, cim;
          group_coeff(tv.t, tv.gs[g], tv.gs[g + 1], key, cre, cim);
          int64_t xre, xim;
          cmul_q32(v.x, v.y, cre, cim, xre, xim);
          child.x = (int32_t)comb_step(r, xre);
          child.y = (int32_t)comb_step(r, xim);
        }
        const bool has = (child.x | child.y) != 0;
        const uint64_t m = __ballot(has);
        if (m == 0) continue;
        if (has) {
          const uint32_t pos = fill + mbcnt64(m);
          my_key[pos] = ck ^ tv.gx[g];
          my_val[pos] = child;
        }
        fill += (uint32_t)__popcll(m);
        if (fill > kSpawnSeg - kWave) flush();
      }
    }
  }
  if (fill) flush();
}

// ---------------------------------------------------------------------------------------------
// LSD radix sort of (key, value) records, 8-bit digits, fixed grid of kSortBlocks blocks, each
// owning one contiguous chunk; per-pass: digit histogram, exclusive scan, stable scatter.
// ---------------------------------------------------------------------------------------------
__device__ __forceinline__ void chunk_range(uint64_t n, uint64_t& b, uint64_t& e) {
  const uint64_t per = ((n + kSortBlocks - 1) / kSortBlocks + kBlock - 1) / kBlock * kBlock;
  b = per * blockIdx.x;
  e = b + per;
  if (b > n) b = n;
  if (e > n) e = n;
}

__global__ __launch_bounds__(kBlock) void k_radix_hist(const uint64_t* __restrict__ keys,
                                                       const Counters* __restrict__ cnt,
                                                       uint32_t nsel, uint32_t shift,
                                                       uint32_t* __restrict__ hist) {
  __shared__ uint32_t h[kRadixBins];
  if (cnt->err) return;
  const uint64_t n = cnt->n_child[nsel];
  h[threadIdx.x] = 0;
  __syncthreads();
  uint64_t b, e;
  chunk_range(n, b, e);
  for (uint64_t i = b + threadIdx.x; i < e; i += kBlock)
    atomicAdd(&h[(uint32_t)(keys[i] >> shift) & (kRadixBins - 1)], 1u);
  __syncthreads();
  hist[threadIdx.x * kSortBlocks + blockIdx.x] = h[threadIdx.x];
}

// Exclusive scan of kRadixBins * kSortBlocks counts (digit-major), one block of 1024 threads.
__global__ __launch_bounds__(1024) void k_radix_scan(uint32_t* __restrict__ hist,
                                                     const Counters* __restrict__ cnt) {
  constexpr int N = kRadixBins * kSortBlocks;
  constexpr int PER = N / 1024;
  __shared__ uint32_t part[1024];
  if (cnt->err) return;
  uint32_t loc[PER];
  uint32_t s = 0;
  const int base = threadIdx.x * PER;
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    loc[i] = hist[base + i];
    s += loc[i];
  }
  part[threadIdx.x] = s;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    uint32_t v = threadIdx.x >= (unsigned)off ? part[threadIdx.x - off] : 0u;
    __syncthreads();
    part[threadIdx.x] += v;
    __syncthreads();
  }
  uint32_t run = part[threadIdx.x] - s;
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    hist[base + i] = run;
    run += loc[i];
  }
}

__global__ __launch_bounds__(kBlock) void k_radix_scatter(
    const uint64_t* __restrict__ kin, const int2* __restrict__ vin, uint64_t* __restrict__ kout,
    int2* __restrict__ vout, const Counters* __restrict__ cnt, uint32_t nsel, uint32_t shift,
    const uint32_t* __restrict__ hist) {
  __shared__ uint32_t off[kRadixBins];
  __shared__ uint32_t wcnt[kWaves][kRadixBins];
  if (cnt->err) return;
  const uint64_t n = cnt->n_child[nsel];
  const uint32_t wave = threadIdx.x / kWave;
  off[threadIdx.x] = hist[threadIdx.x * kSortBlocks + blockIdx.x];
  for (int w = 0; w < kWaves; ++w) wcnt[w][threadIdx.x] = 0;
  __syncthreads();
  uint64_t b, e;
  chunk_range(n, b, e);
  const uint64_t lt = lanemask_lt();
  for (uint64_t base = b; base < e; base += kBlock) {
    const uint64_t i = base + threadIdx.x;
    const bool valid = i < e;
    uint64_t k = 0;
    int2 v = make_int2(0, 0);
    uint32_t d = 0;
    if (valid) {
      k = kin[i];
      v = vin[i];
      d = (uint32_t)(k >> shift) & (kRadixBins - 1);
    }
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int bit = 0; bit < kRadixBits; ++bit) {
      const uint64_t bm = __ballot((d >> bit) & 1u);
      peers &= ((d >> bit) & 1u) ? bm : ~bm;
    }
    const uint32_t rank = (uint32_t)__popcll(peers & lt);
    if (valid && rank == 0) wcnt[wave][d] = (uint32_t)__popcll(peers);
    __syncthreads();
    if (valid) {
      uint32_t pos = off[d] + rank;
      for (uint32_t w = 0; w < wave; ++w) pos += wcnt[w][d];
      kout[pos] = k;
      vout[pos] = v;
    }
    __syncthreads();
    {
      const uint32_t dd = threadIdx.x;
      uint32_t add = 0;
      for (int w = 0; w < kWaves; ++w) {
        add += wcnt[w][dd];
        wcnt[w][dd] = 0;
      }
      off[dd] += add;
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------------------------
// Merge of parents (unique keys) with sorted children, split into tiles whose boundaries never
// cut a key's run (parents win ties, so a run is [parent] children...).
// ---------------------------------------------------------------------------------------------
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
  // Only children can continue the run (a parent equal to `last` would precede it).
  uint32_t lo = j, hi = nb;
  if (hi - lo > (uint32_t)kMergeSlack) hi = lo + kMergeSlack;
  while (lo < hi) {
    const uint32_t mid = (lo + hi) >> 1;
    if (B(mid) <= last)
      lo = mid + 1;
    else
      hi = mid;
  }
  j = lo;
}

__global__ __launch_bounds__(kBlock) void k_merge_part(const uint64_t* __restrict__ pk,
                                                       const uint64_t* __restrict__ ckeys,
                                                       Counters* __restrict__ cnt, uint32_t cur,
                                                       uint32_t csel, uint2* __restrict__ splits,
                                                       uint32_t max_tiles) {
  if (cnt->err) return;
  const uint32_t np = (uint32_t)cnt->n_store[cur];
  const uint32_t nc = (uint32_t)cnt->n_child[csel];
  const uint32_t total = np + nc;
  const uint32_t ntiles = (total + kMergeTile - 1) / kMergeTile;
  const uint32_t t = blockIdx.x * kBlock + threadIdx.x;
  if (t == 0) {
    cnt->tile_counter = 0;
    cnt->n_child[csel ^ 1] = 0;  // counter of the next step's children (last used two steps ago)
  }
  if (t > ntiles || t > max_tiles) return;
  uint32_t d = t * kMergeTile;
  if (d > total) d = total;
  auto A = [&](uint32_t x) { return pk[x]; };
  auto B = [&](uint32_t x) { return ckeys[x]; };
  uint32_t i, j;
  run_split(A, np, B, nc, d, i, j);
  splits[t] = make_uint2(i, j);
}

// Look-back status word: epoch (16) | flag (2) | value (46).
__device__ __forceinline__ uint64_t lb_pack(uint32_t epoch, uint32_t flag, uint64_t v) {
  return ((uint64_t)(epoch & 0xFFFFu) << 48) | ((uint64_t)flag << 46) | (v & ((1ull << 46) - 1));
}

__global__ __launch_bounds__(kBlock) void k_merge(
    const uint64_t* __restrict__ pk, const int2* __restrict__ pv,
    const uint64_t* __restrict__ ckeys, const int2* __restrict__ cvals, Counters* __restrict__ cnt,
    uint32_t cur, uint32_t csel, const uint2* __restrict__ splits, uint64_t* __restrict__ status,
    uint32_t epoch, const uint8_t* __restrict__ tab, const int64_t* __restrict__ qshift,
    uint32_t step, uint64_t seed, KeyLayout kl, uint64_t* __restrict__ ok,
    int2* __restrict__ ov, uint64_t cap_store) {
  constexpr int CAP = kMergeTile + kMergeSlack + 8;
  __shared__ uint64_t s_pk[CAP];
  __shared__ int64_t s_pre[CAP];
  __shared__ int64_t s_pim[CAP];
  __shared__ uint64_t s_ck[CAP];
  __shared__ int2 s_cv[CAP];
  __shared__ uint32_t s_scan[kBlock];
  __shared__ uint32_t s_tile;
  __shared__ uint64_t s_base;
  __shared__ uint64_t s_ws[kWaves];

  if (cnt->err) return;
  const uint32_t np = (uint32_t)cnt->n_store[cur];
  const uint32_t nc = (uint32_t)cnt->n_child[csel];
  const uint32_t total = np + nc;
  const uint32_t ntiles = (total + kMergeTile - 1) / kMergeTile;
  if (threadIdx.x == 0) {
    s_tile = atomicAdd(&cnt->tile_counter, 1u);
    if (ntiles == 0 && blockIdx.x == 0) cnt->n_store[cur ^ 1] = 0;
  }
  __syncthreads();
  const uint32_t tile = s_tile;
  if (tile >= ntiles) return;
  const uint2 s0 = splits[tile], s1 = splits[tile + 1];
  if (s1.x < s0.x || s1.y < s0.y || (s1.x - s0.x) + (s1.y - s0.y) > (uint32_t)CAP ||
      s1.x > np || s1.y > nc) {
    // cannot happen for runs shorter than the slack; refuse rather than overrun LDS
    if (threadIdx.x == 0) {
      atomicOr(&cnt->err, kErrLookback);
      atomicMin(&cnt->err_step, step);
      atomic_store_agent(&status[tile], lb_pack(epoch, 2, 0));
    }
    return;
  }
  const uint32_t pa = s0.x, pn = s1.x - s0.x;
  const uint32_t ca = s0.y, cn = s1.y - s0.y;

  // Load parents with their death/cloning update (diagonal of the column, applied to N(s)).
  const TableView tv = table_view(tab);
  const uint32_t d_end = tv.h->n_groups > 0 ? tv.gs[1] : 0u;
  const uint64_t q_diag = tv.h->q_diag;
  uint64_t wsum = 0;
  for (uint32_t x = threadIdx.x; x < pn; x += kBlock) {
    const uint64_t ck = pk[pa + x];
    const int2 v = pv[pa + x];
    const uint32_t rep = kl.replica(ck);
    const int64_t qs = qshift[rep];
    int64_t a = v.x, b = v.y;
    uint32_t w[4];
    walker_random(kl.key(ck), step, rep, seed, w);
    const uint64_t sab = uabs64(a) + uabs64(b);
    wsum += sab;
    if (!comb_all_zero(sab, q_diag + uabs64(qs), w[1])) {
      int32_t dre, dim;
      group_coeff(tv.t, 0, d_end, kl.key(ck), dre, dim);
      int64_t xre, xim;
      cmul_q32(a, b, dre + (int32_t)qs, dim, xre, xim);
      uint64_t r = w[1];
      const int64_t nre = comb_step(r, xre);
      const int64_t nim = comb_step(r, xim);
      a += nre;
      b += nim;
    }
    s_pk[x] = ck;
    s_pre[x] = a;
    s_pim[x] = b;
  }
  for (uint32_t x = threadIdx.x; x < cn; x += kBlock) {
    s_ck[x] = ckeys[ca + x];
    s_cv[x] = cvals[ca + x];
  }
  // walker statistics of the parents of this step
  for (int o = 32; o > 0; o >>= 1) wsum += __shfl_xor(wsum, o);
  if (__lane_id() == 0) s_ws[threadIdx.x / kWave] = wsum;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint64_t t = 0;
    for (int w = 0; w < kWaves; ++w) t += s_ws[w];
    atomicAdd((unsigned long long*)&cnt->walker_steps, (unsigned long long)t);
    atomicAdd((unsigned long long*)&cnt->key_steps, (unsigned long long)pn);
  }

  // Per-thread ranges of the local merge, cut only at run ends.
  auto A = [&](uint32_t x) { return s_pk[x]; };
  auto B = [&](uint32_t x) { return s_ck[x]; };
  const uint32_t tot = pn + cn;
  uint32_t d0 = threadIdx.x * kMergeIpt, d1 = d0 + kMergeIpt;
  if (d0 > tot) d0 = tot;
  if (d1 > tot) d1 = tot;
  uint32_t i0, j0, i1, j1;
  run_split(A, pn, B, cn, d0, i0, j0);
  run_split(A, pn, B, cn, d1, i1, j1);
  if (threadIdx.x == kBlock - 1) {
    i1 = pn;
    j1 = cn;
  }
  if (i1 + j1 < i0 + j0) {  // an earlier thread's run already covers this range
    i1 = i0;
    j1 = j0;
  }

  // Pass 1: count nonzero outputs.
  uint32_t count = 0;
  bool overflow = false;
  {
    uint32_t i = i0, j = j0;
    while (i < i1 || j < j1) {
      uint64_t k;
      int64_t re = 0, im = 0;
      if (j >= j1 || (i < i1 && s_pk[i] <= s_ck[j])) {
        k = s_pk[i];
        re = s_pre[i];
        im = s_pim[i];
        ++i;
      } else {
        k = s_ck[j];
      }
      while (j < j1 && s_ck[j] == k) {
        re += s_cv[j].x;
        im += s_cv[j].y;
        ++j;
      }
      if (re < INT32_MIN || re > INT32_MAX || im < INT32_MIN || im > INT32_MAX) overflow = true;
      count += (re != 0 || im != 0) ? 1u : 0u;
    }
  }
  if (overflow) {
    atomicOr(&cnt->err, kErrOverflow);
    atomicMin(&cnt->err_step, step);
  }

  // Block exclusive scan of counts.
  s_scan[threadIdx.x] = count;
  __syncthreads();
  for (int o = 1; o < kBlock; o <<= 1) {
    const uint32_t v = threadIdx.x >= (unsigned)o ? s_scan[threadIdx.x - o] : 0u;
    __syncthreads();
    s_scan[threadIdx.x] += v;
    __syncthreads();
  }
  const uint32_t excl = s_scan[threadIdx.x] - count;
  const uint32_t agg = s_scan[kBlock - 1];

  // Decoupled look-back (Merrill & Garland) for the tile's output offset.
  if (threadIdx.x == 0) {
    uint64_t prefix = 0;
    if (tile == 0) {
      atomic_store_agent(&status[0], lb_pack(epoch, 2, agg));
    } else {
      atomic_store_agent(&status[tile], lb_pack(epoch, 1, agg));
      int32_t j = (int32_t)tile - 1;
      uint32_t spins = 0;
      while (j >= 0) {
        const uint64_t sw = atomic_load_agent(&status[j]);
        const uint32_t ep = (uint32_t)(sw >> 48), fl = (uint32_t)(sw >> 46) & 3u;
        if (ep != (epoch & 0xFFFFu) || fl == 0) {
          if (++spins > (1u << 24)) {
            atomicOr(&cnt->err, kErrLookback);
            atomicMin(&cnt->err_step, step);
            break;
          }
          __builtin_amdgcn_s_sleep(1);
          continue;
        }
        prefix += sw & ((1ull << 46) - 1);
        if (fl == 2) break;
        --j;
      }
      atomic_store_agent(&status[tile], lb_pack(epoch, 2, prefix + agg));
    }
    s_base = prefix;
    if (tile == ntiles - 1) {
      cnt->n_store[cur ^ 1] = prefix + agg;
      atomicAdd((unsigned long long*)&cnt->child_steps, (unsigned long long)nc);
      atomicAdd((unsigned long long*)&cnt->out_steps, (unsigned long long)(prefix + agg));
      if (prefix + agg > cap_store) {
        atomicOr(&cnt->err, kErrStoreCap);
        atomicMin(&cnt->err_step, step);
      }
    }
  }
  __syncthreads();
  const uint64_t base = s_base + excl;

  // Pass 2: write the annihilated, compacted records.
  {
    uint32_t i = i0, j = j0;
    uint64_t o = base;
    while (i < i1 || j < j1) {
      uint64_t k;
      int64_t re = 0, im = 0;
      if (j >= j1 || (i < i1 && s_pk[i] <= s_ck[j])) {
        k = s_pk[i];
        re = s_pre[i];
        im = s_pim[i];
        ++i;
      } else {
        k = s_ck[j];
      }
      while (j < j1 && s_ck[j] == k) {
        re += s_cv[j].x;
        im += s_cv[j].y;
        ++j;
      }
      if (re != 0 || im != 0) {
        if (o < cap_store) {
          ok[o] = k;
          ov[o] = make_int2((int32_t)re, (int32_t)im);
        }
        ++o;
      }
    }
  }
}

// ---------------------------------------------------------------------------------------------
// Utility and estimator kernels.
// ---------------------------------------------------------------------------------------------
__global__ void k_batch_begin(Counters* cnt, uint32_t step, uint64_t* status, uint32_t n_status) {
  const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t == 0) {
    cnt->n_child[0] = 0;
    cnt->n_child[1] = 0;
    cnt->err = 0;
    cnt->err_step = 0xFFFFFFFFu;
  }
  for (uint32_t i = t; i < n_status; i += gridDim.x * blockDim.x) status[i] = 0;
}

__global__ void k_reset_child(Counters* cnt, uint32_t sel) {
  if (threadIdx.x == 0 && blockIdx.x == 0) cnt->n_child[sel] = 0;
}

// In-place sign flips of an ideal diagonal Pauli pulse, or key transform into (ck, cv) for a
// pulse with x != 0 (sorted afterwards).
__global__ __launch_bounds__(kBlock) void k_pulse(uint64_t* __restrict__ pk, int2* __restrict__ pv,
                                                  Counters* __restrict__ cnt, uint32_t cur,
                                                  uint32_t n, uint64_t x, uint64_t z,
                                                  uint64_t* __restrict__ ck_out,
                                                  int2* __restrict__ cv_out, uint32_t csel) {
  const uint64_t np = cnt->n_store[cur];
  const uint64_t qm = n >= 32 ? 0xFFFFFFFFull : ((1ull << n) - 1);
  const uint64_t kx = (x << n) | x;
  for (uint64_t p = (uint64_t)blockIdx.x * kBlock + threadIdx.x; p < np;
       p += (uint64_t)gridDim.x * kBlock) {
    const uint64_t ck = pk[p];
    int2 v = pv[p];
    const uint64_t i = ck & qm, j = (ck >> n) & qm;
    const bool neg = ((__popcll(z & i) + __popcll(z & j)) & 1) != 0;
    if (neg) {
      if (v.x == INT32_MIN || v.y == INT32_MIN) atomicOr(&cnt->err, kErrOverflow);
      v.x = -v.x;
      v.y = -v.y;
    }
    if (x == 0) {
      pv[p] = v;
    } else {
      ck_out[p] = ck ^ kx;
      cv_out[p] = v;
    }
  }
  if (x != 0 && blockIdx.x == 0 && threadIdx.x == 0) cnt->n_child[csel] = np;
}

__global__ __launch_bounds__(kBlock) void k_copy_store(const uint64_t* __restrict__ ki,
                                                       const int2* __restrict__ vi,
                                                       uint64_t* __restrict__ ko,
                                                       int2* __restrict__ vo,
                                                       const Counters* __restrict__ cnt,
                                                       uint32_t csel) {
  const uint64_t n = cnt->n_child[csel];
  for (uint64_t p = (uint64_t)blockIdx.x * kBlock + threadIdx.x; p < n;
       p += (uint64_t)gridDim.x * kBlock) {
    ko[p] = ki[p];
    vo[p] = vi[p];
  }
}

// Per-replica estimator numerators; blockIdx.y is the replica, whose segment of the sorted
// store is found by binary search.  Output per replica (int64 words):
//   [0] n_tot, [1] ndiag_re, [2] ndiag_im, [3] eps2_lo, [4] eps2_hi, [5..] pauli re/im pairs.
__device__ __forceinline__ uint64_t lower_bound64(const uint64_t* __restrict__ a, uint64_t n,
                                                  uint64_t v) {
  uint64_t lo = 0, hi = n;
  while (lo < hi) {
    const uint64_t mid = (lo + hi) >> 1;
    if (a[mid] < v)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}

__device__ __forceinline__ void add_u128(unsigned long long* lo, unsigned long long* hi,
                                         uint64_t v) {
  if (v == 0) return;
  const unsigned long long old = atomicAdd(lo, (unsigned long long)v);
  if (old + v < old) atomicAdd(hi, 1ull);
}

__global__ __launch_bounds__(kBlock) void k_observe(const uint64_t* __restrict__ pk,
                                                    const int2* __restrict__ pv,
                                                    const Counters* __restrict__ cnt, uint32_t cur,
                                                    uint32_t n, KeyLayout kl, uint32_t n_pauli,
                                                    const uint64_t* __restrict__ pxz,
                                                    uint32_t want_eps,
                                                    unsigned long long* __restrict__ out,
                                                    uint32_t out_stride) {
  extern __shared__ unsigned long long s_acc[];
  const uint64_t np = cnt->n_store[cur];
  const uint32_t rep = blockIdx.y;
  const uint64_t lo_ck = kl.kbits >= 64 ? 0 : ((uint64_t)rep << kl.kbits);
  const uint64_t seg_b = lower_bound64(pk, np, lo_ck);
  const uint64_t seg_e = (kl.kbits >= 64) ? np : lower_bound64(pk, np, (uint64_t)(rep + 1) << kl.kbits);
  for (uint32_t i = threadIdx.x; i < out_stride; i += kBlock) s_acc[i] = 0;
  __syncthreads();
  const uint64_t qm = n >= 32 ? 0xFFFFFFFFull : ((1ull << n) - 1);
  for (uint64_t p = seg_b + (uint64_t)blockIdx.x * kBlock + threadIdx.x; p < seg_e;
       p += (uint64_t)gridDim.x * kBlock) {
    const uint64_t ck = pk[p];
    const int2 v = pv[p];
    const uint64_t key = kl.key(ck);
    const uint64_t i = key & qm, j = (key >> n) & qm;
    atomicAdd(&s_acc[0], (unsigned long long)(uabs64(v.x) + uabs64(v.y)));
    if (i == j) {
      atomicAdd(&s_acc[1], (unsigned long long)(int64_t)v.x);
      atomicAdd(&s_acc[2], (unsigned long long)(int64_t)v.y);
    }
    for (uint32_t k = 0; k < n_pauli; ++k) {
      if ((i ^ j) != pxz[2 * k]) continue;
      const bool neg = (__popcll(pxz[2 * k + 1] & i) & 1) != 0;
      atomicAdd(&s_acc[5 + 2 * k], (unsigned long long)(int64_t)(neg ? -(int64_t)v.x : v.x));
      atomicAdd(&s_acc[6 + 2 * k], (unsigned long long)(int64_t)(neg ? -(int64_t)v.y : v.y));
    }
    if (want_eps) {
      const uint64_t kt = (ck & ~kl.kmask) | ((i << n) | j);
      const uint64_t q = lower_bound64(pk + seg_b, seg_e - seg_b, kt) + seg_b;
      int64_t c = 0, d = 0;
      const bool found = q < seg_e && pk[q] == kt;
      if (found) {
        c = pv[q].x;
        d = pv[q].y;
      }
      const uint64_t u = uabs64((int64_t)v.x - c), w = uabs64((int64_t)v.y + d);
      add_u128(&s_acc[3], &s_acc[4], u * u);
      add_u128(&s_acc[3], &s_acc[4], w * w);
      if (!found) {
        const uint64_t aa = uabs64(v.x), bb = uabs64(v.y);
        add_u128(&s_acc[3], &s_acc[4], aa * aa);
        add_u128(&s_acc[3], &s_acc[4], bb * bb);
      }
    }
  }
  __syncthreads();
  unsigned long long* o = out + (uint64_t)rep * out_stride;
  if (threadIdx.x == 0) {
    // 128-bit (lo, hi) pair: carry of the low word into the high word
    add_u128(&o[3], &o[4], s_acc[3]);
    if (s_acc[4]) atomicAdd(&o[4], s_acc[4]);
  }
  for (uint32_t i = threadIdx.x; i < out_stride; i += kBlock) {
    if (i == 3 || i == 4) continue;
    if (s_acc[i]) atomicAdd(&o[i], s_acc[i]);
  }
}

// Values at given keys of every replica: out[(rep * nk + k) * 2 + {0,1}].
__global__ __launch_bounds__(kBlock) void k_lookup(const uint64_t* __restrict__ pk,
                                                   const int2* __restrict__ pv,
                                                   const Counters* __restrict__ cnt, uint32_t cur,
                                                   KeyLayout kl, const uint64_t* __restrict__ keys,
                                                   uint32_t nk, uint32_t nrep,
                                                   int64_t* __restrict__ out) {
  const uint64_t np = cnt->n_store[cur];
  const uint64_t t = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
  if (t >= (uint64_t)nk * nrep) return;
  const uint32_t rep = (uint32_t)(t / nk), k = (uint32_t)(t % nk);
  const uint64_t ck = (kl.kbits >= 64 ? 0 : ((uint64_t)rep << kl.kbits)) | keys[k];
  const uint64_t q = lower_bound64(pk, np, ck);
  int64_t a = 0, b = 0;
  if (q < np && pk[q] == ck) {
    a = pv[q].x;
    b = pv[q].y;
  }
  out[2 * t] = a;
  out[2 * t + 1] = b;
}

// ---------------------------------------------------------------------------------------------
// Host-side launch wrappers.
// ---------------------------------------------------------------------------------------------
static inline uint32_t grid_for(uint64_t n, uint32_t cap_blocks) {
  uint64_t g = (n + kBlock - 1) / kBlock;
  if (g < 1) g = 1;
  if (g > cap_blocks) g = cap_blocks;
  return (uint32_t)g;
}

}  // namespace qmc

using namespace qmc;

extern "C" {

int qmck_batch_begin(hipStream_t st, void* counters, uint32_t step, uint64_t* status,
                     uint32_t n_status) {
  uint32_t g = grid_for(n_status, 1024);
  hipLaunchKernelGGL(k_batch_begin, dim3(g), dim3(kBlock), 0, st, (Counters*)counters, step,
                     status, n_status);
  return (int)hipGetLastError();
}

int qmck_spawn(hipStream_t st, const uint64_t* pk, const int2* pv, void* counters, uint32_t cur,
               const uint8_t* tab, uint32_t step, uint64_t seed, uint32_t kbits,
               uint64_t* ck, int2* cv, uint64_t cap_child, uint64_t max_parents) {
  KeyLayout kl{kbits, kbits >= 64 ? ~0ull : ((1ull << kbits) - 1)};
  uint32_t g = grid_for(max_parents, 4096);
  hipLaunchKernelGGL(k_spawn, dim3(g), dim3(kBlock), 0, st, pk, pv, (Counters*)counters, cur, tab,
                     step, seed, kl, ck, cv, cap_child);
  return (int)hipGetLastError();
}

// Sorts n_child[nsel] records found in (k0, v0); returns in *in_second whether the result is in
// (k1, v1).
int qmck_sort(hipStream_t st, uint64_t* k0, int2* v0, uint64_t* k1, int2* v1, void* counters,
              uint32_t nsel, uint32_t key_bits, uint32_t* hist, int* in_second) {
  uint32_t passes = (key_bits + kRadixBits - 1) / kRadixBits;
  uint64_t* ka = k0;
  int2* va = v0;
  uint64_t* kb = k1;
  int2* vb = v1;
  for (uint32_t p = 0; p < passes; ++p) {
    const uint32_t shift = p * kRadixBits;
    hipLaunchKernelGGL(k_radix_hist, dim3(kSortBlocks), dim3(kBlock), 0, st, ka,
                       (const Counters*)counters, nsel, shift, hist);
    hipLaunchKernelGGL(k_radix_scan, dim3(1), dim3(1024), 0, st, hist, (const Counters*)counters);
    hipLaunchKernelGGL(k_radix_scatter, dim3(kSortBlocks), dim3(kBlock), 0, st, ka, va, kb, vb,
                       (const Counters*)counters, nsel, shift, hist);
    uint64_t* tk = ka;
    ka = kb;
    kb = tk;
    int2* tv = va;
    va = vb;
    vb = tv;
  }
  *in_second = (passes & 1) ? 1 : 0;
  return (int)hipGetLastError();
}

int qmck_merge(hipStream_t st, const uint64_t* pk, const int2* pv, const uint64_t* ck,
               const int2* cv, void* counters, uint32_t cur, uint32_t csel, uint2* splits,
               uint64_t* status, uint32_t epoch, const uint8_t* tab, const int64_t* qshift,
               uint32_t step, uint64_t seed, uint32_t kbits, uint64_t* ok, int2* ov,
               uint64_t cap_store, uint64_t max_items) {
  KeyLayout kl{kbits, kbits >= 64 ? ~0ull : ((1ull << kbits) - 1)};
  const uint32_t max_tiles = (uint32_t)((max_items + kMergeTile - 1) / kMergeTile);
  hipLaunchKernelGGL(k_merge_part, dim3(grid_for((uint64_t)max_tiles + 1, 1u << 20)), dim3(kBlock),
                     0, st, pk, ck, (Counters*)counters, cur, csel, splits, max_tiles);
  hipLaunchKernelGGL(k_merge, dim3(max_tiles > 0 ? max_tiles : 1), dim3(kBlock), 0, st, pk, pv,
                     ck, cv, (Counters*)counters, cur, csel, splits, status, epoch, tab, qshift,
                     step, seed, kl, ok, ov, cap_store);
  return (int)hipGetLastError();
}

int qmck_reset_child(hipStream_t st, void* counters, uint32_t sel) {
  hipLaunchKernelGGL(k_reset_child, dim3(1), dim3(64), 0, st, (Counters*)counters, sel);
  return (int)hipGetLastError();
}

int qmck_pulse(hipStream_t st, uint64_t* pk, int2* pv, void* counters, uint32_t cur, uint32_t n,
               uint64_t x, uint64_t z, uint64_t* ck, int2* cv, uint32_t csel,
               uint64_t max_parents) {
  uint32_t g = grid_for(max_parents, 8192);
  hipLaunchKernelGGL(k_pulse, dim3(g), dim3(kBlock), 0, st, pk, pv, (Counters*)counters, cur, n,
                     x, z, ck, cv, csel);
  return (int)hipGetLastError();
}

int qmck_copy_store(hipStream_t st, const uint64_t* ki, const int2* vi, uint64_t* ko, int2* vo,
                    void* counters, uint32_t csel, uint64_t max_items) {
  uint32_t g = grid_for(max_items, 8192);
  hipLaunchKernelGGL(k_copy_store, dim3(g), dim3(kBlock), 0, st, ki, vi, ko, vo,
                     (const Counters*)counters, csel);
  return (int)hipGetLastError();
}

int qmck_observe(hipStream_t st, const uint64_t* pk, const int2* pv, void* counters, uint32_t cur,
                 uint32_t n, uint32_t kbits, uint32_t nrep, uint32_t n_pauli,
                 const uint64_t* pxz, uint32_t want_eps, unsigned long long* out,
                 uint32_t out_stride, uint64_t max_per_replica) {
  KeyLayout kl{kbits, kbits >= 64 ? ~0ull : ((1ull << kbits) - 1)};
  uint32_t gx = grid_for(max_per_replica, 1024);
  hipLaunchKernelGGL(k_observe, dim3(gx, nrep), dim3(kBlock),
                     out_stride * sizeof(unsigned long long), st, pk, pv,
                     (const Counters*)counters, cur, n, kl, n_pauli, pxz, want_eps, out,
                     out_stride);
  return (int)hipGetLastError();
}

int qmck_lookup(hipStream_t st, const uint64_t* pk, const int2* pv, void* counters, uint32_t cur,
                uint32_t kbits, const uint64_t* keys, uint32_t nk, uint32_t nrep, int64_t* out) {
  KeyLayout kl{kbits, kbits >= 64 ? ~0ull : ((1ull << kbits) - 1)};
  uint64_t tot = (uint64_t)nk * nrep;
  if (tot == 0) return 0;
  uint32_t g = (uint32_t)((tot + kBlock - 1) / kBlock);
  hipLaunchKernelGGL(k_lookup, dim3(g), dim3(kBlock), 0, st, pk, pv, (const Counters*)counters,
                     cur, kl, keys, nk, nrep, out);
  return (int)hipGetLastError();
}

}  // extern "C"
