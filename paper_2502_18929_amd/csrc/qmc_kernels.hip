// qmc_kernels.hip -- HIP kernels of one population-dynamics time step (gfx950, wave64).
//
// Step s (End Matter, spawn and annihilation; Euler solver):
//   records(s)       from N(s): the death/cloning delta of each parent (diagonal of its
//                    column, the parent's own key) and its children (key ^ mask), comb-rounded
//                    dt L N, unsorted, with the radix digit histograms of every pass
//                    accumulated while they are written
//   k_onesweep x P   single-pass LSD radix sort of the records by composite key: per tile,
//                    wave-local stable ranking in LDS, decoupled look-back per digit, scatter
//   k_merge_part     merge-path split points of (parents, sorted records), moved to run ends
//   k_merge          merge of parents and records, int64 segmented sum per key, drop (0, 0),
//                    decoupled look-back for the compacted output offset -> N(s+1); then the
//                    records of step s+1 are made from the outputs still in LDS
// The first step of a batch spawns with k_spawn.  Plus k_pulse (ideal Pauli conjugation),
// k_observe / k_lookup (estimator numerators) and small utility kernels.  Every kernel reads its
// problem sizes from device memory, so a batch of steps is enqueued without host sync.
#include "qmc_device.hpp"
#include "qmc_kernels.h"

namespace qmc {

// Spawn emitter: per-wave LDS staging of child records, flushed to the child buffer with one
// atomic per flush; every flushed record is also counted into the digit histograms of all
// radix passes of the next sort (wave-aggregated atomics).
struct Emitter {
  uint64_t* s_key;      // this wave's staging segment
  int2* s_val;
  uint32_t seg;         // segment capacity (records)
  uint32_t fill;        // wave-uniform
  Counters* cnt;
  uint32_t nsel;        // child counter parity
  uint32_t step;        // the step the children belong to
  uint64_t* ck_out;
  int2* cv_out;
  uint64_t cap;
  uint32_t* ghist;      // [passes][kRadixBins]
  uint32_t passes;
  uint32_t ndiag = 0;   // wave-uniform: diagonal (death) records emitted so far (the owner adds
                        // them to cnt->death_steps once, when it is done)

  __device__ void flush() {
    const uint32_t lane = __lane_id();
    wave_lds_fence();
    uint64_t base = 0;
    if (lane == 0)
      base = atomicAdd((unsigned long long*)&cnt->n_child[nsel], (unsigned long long)fill);
    base = __shfl(base, 0);
    const bool ok = base + fill <= cap;
    if (!ok && lane == 0) {
      atomicOr(&cnt->err, kErrSpawnCap);
      atomicMin(&cnt->err_step, step);
    }
    for (uint32_t i0 = 0; i0 < fill; i0 += kWave) {
      const uint32_t i = i0 + lane;
      const bool v = i < fill;
      uint64_t k = 0;
      if (v) {
        k = s_key[i];
        if (ok) {
          ck_out[base + i] = k;
          cv_out[base + i] = s_val[i];
        }
      }
      const uint64_t act = __ballot(v);
      for (uint32_t p = 0; p < passes; ++p) {
        const uint32_t d = digit_of(k, p * kRadixBits);
        const uint64_t peers = match_digit(d, act);
        if (v && (peers & lanemask_lt()) == 0)
          atomicAdd(&ghist[p * kRadixBins + d], (uint32_t)__popcll(peers));
      }
    }
    wave_lds_fence();
    fill = 0;
  }

  // All lanes call; lanes with has == true append (key, val).
  __device__ __forceinline__ void emit(bool has, uint64_t key, int2 val) {
    const uint64_t m = __ballot(has);
    if (m == 0) return;
    if (has) {
      const uint32_t pos = fill + mbcnt64(m);
      s_key[pos] = key;
      s_val[pos] = val;
    }
    fill += (uint32_t)__popcll(m);
    if (fill > seg - kWave) flush();
  }

  // The same for a parent's diagonal (death/cloning) record, counted apart from the children.
  __device__ __forceinline__ void emit_diag(bool has, uint64_t key, int2 val) {
    ndiag += (uint32_t)__popcll(__ballot(has));
    emit(has, key, val);
  }

  // A record of this step does not fit int32.
  __device__ __forceinline__ void overflow() {
    atomicOr(&cnt->err, kErrOverflow);
    atomicMin(&cnt->err_step, step);
  }
};

typedef int32_t v16i32 __attribute__((ext_vector_type(16)));

// Hidden layer of the proposal MLP for the 64 keys of a wave (lane l holds key l; every lane
// calls): h[l][j] = min(127, max(0, a) >> s1), a = b1[j] + sum_b w1[j][b] x_b, with x_b = +1 where
// bit b of the key is set and -1 where it is clear for b < nbits, 0 past.  Two int8 MFMA products
// (32 keys x 16 inputs by 16 inputs x 32 units, four input blocks each) accumulate in int32;
// lane l of an MFMA holds unit l % 32 of keys 8 (i / 4) + 4 (l / 32) + i % 4 in its i-th
// accumulator.  The units go to hid[key][unit] (LDS, 64 x 32 bytes).
__device__ __forceinline__ void mlp_hidden(const QmcProposal& pr, uint64_t key, uint8_t* hid) {
  const uint32_t lane = __lane_id(), col = lane & 31u, half = lane >> 5;
#pragma unroll
  for (int rb = 0; rb < 2; ++rb) {
    const uint64_t kr = __shfl(key, rb * 32 + (int)col);  // key of A-operand row col
    v16i32 acc = {};
#pragma unroll
    for (int kb = 0; kb < kPropIn / 16; ++kb) {
      const uint32_t b0 = kb * 16 + half * 8;
      uint64_t a = 0;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const uint32_t b = b0 + e;
        const uint64_t f = b < pr.nbits ? (((kr >> b) & 1u) ? 0x01ull : 0xFFull) : 0ull;
        a |= f << (8 * e);
      }
      const uint64_t w = *reinterpret_cast<const uint64_t*>(pr.w1 + col * kPropIn + b0);
      acc = __builtin_amdgcn_mfma_i32_32x32x16_i8((long)a, (long)w, acc, 0, 0, 0);
    }
    const int32_t bias = pr.b1[col];
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const uint32_t row = 8 * (i / 4) + 4 * half + (i % 4);
      const int32_t v = acc[i] + bias;
      int32_t h = v > 0 ? (v >> pr.s1) : 0;
      h = h > 127 ? 127 : h;
      hid[(rb * 32 + row) * kPropHidden + col] = (uint8_t)h;
    }
  }
  wave_lds_fence();
}

// Hidden layers of the deeper proposal network (kind 4) for the 64 keys of a wave (lane l holds
// key l; every lane calls).  Input of a key: +1 / -1 for key bits b < nbits, then 1 / 0 for the
// step's weight channels that are nonzero / zero (bits of `active`), 0 past kDeepIn.  Layer 1:
// h1 = min(127, max(0, b1 + w1 x) >> s1), 128 units, as int8 MFMA 32x32x16 products (32 keys x 16
// inputs by 16 inputs x 32 units, eight input blocks per product) accumulated in int32; h1 goes
// to LDS (64 x 128 bytes) and layer 2 reads it the same way: h2 = min(127, max(0, b2 + w2 h1) >>
// s2) into the second 64 x 128 bytes.  Lane l of a product holds unit 32 cb + l % 32 of keys
// 8 (i / 4) + 4 (l / 32) + i % 4 in its i-th accumulator.
__device__ __forceinline__ void mlp_deep(const QmcProposal& pr, uint64_t key, uint64_t act0,
                                         uint64_t act1, uint8_t* hid) {
  const uint32_t lane = __lane_id(), col = lane & 31u, half = lane >> 5;
  uint8_t* h1 = hid;
  uint8_t* h2 = hid + kWave * kDeepHidden;
  const uint32_t nb = pr.nbits < (uint32_t)kDeepIn ? pr.nbits : (uint32_t)kDeepIn;
  auto layer = [&](const int8_t* w, const int32_t* bias, uint32_t sh, uint8_t* out,
                   auto&& operand) __attribute__((always_inline)) {
#pragma unroll 1
    for (int rb = 0; rb < 2; ++rb) {
      uint64_t a[kDeepIn / 16];
#pragma unroll
      for (int kb = 0; kb < kDeepIn / 16; ++kb) a[kb] = operand(rb, kb * 16 + half * 8);
#pragma unroll 1
      for (int cb = 0; cb < kDeepHidden / 32; ++cb) {
        const uint32_t unit = cb * 32 + col;
        v16i32 acc = {};
#pragma unroll
        for (int kb = 0; kb < kDeepIn / 16; ++kb) {
          const uint64_t wv =
              *reinterpret_cast<const uint64_t*>(w + unit * kDeepIn + kb * 16 + half * 8);
          acc = __builtin_amdgcn_mfma_i32_32x32x16_i8((long)a[kb], (long)wv, acc, 0, 0, 0);
        }
        const int32_t b = bias[unit];
#pragma unroll
        for (int i = 0; i < 16; ++i) {
          const uint32_t row = 8 * (i / 4) + 4 * half + (i % 4);
          const int32_t v = acc[i] + b;
          int32_t h = v > 0 ? (v >> sh) : 0;
          h = h > 127 ? 127 : h;
          out[(rb * 32 + row) * kDeepHidden + unit] = (uint8_t)h;
        }
      }
    }
    wave_lds_fence();
  };
  // layer 1: the A operand of key row `col` of block rb, inputs b0 .. b0 + 7
  layer(pr.w1, pr.b1, pr.s1, h1, [&](int rb, uint32_t b0) __attribute__((always_inline)) {
    const uint64_t kr = __shfl(key, rb * 32 + (int)col);
    uint64_t v = 0;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const uint32_t i = b0 + e;
      uint64_t x;
      if (i < nb) {
        x = ((kr >> i) & 1u) ? 0x01ull : 0xFFull;
      } else {
        const uint32_t m = i - nb;
        x = ((m < 64 ? act0 >> m : act1 >> (m - 64)) & 1u) ? 0x01ull : 0x00ull;
      }
      v |= x << (8 * e);
    }
    return v;
  });
  // layer 2: the A operand is a row of h1
  layer(pr.w2, pr.b2, pr.s2, h2, [&](int rb, uint32_t b0) __attribute__((always_inline)) {
    return *reinterpret_cast<const uint64_t*>(h1 + (rb * 32 + col) * kDeepHidden + b0);
  });
}

__device__ __forceinline__ uint32_t bitlen64(uint64_t v) {
  return v ? 64u - (uint32_t)__clzll(v) : 0u;
}

// Off-diagonal records of one parent per lane under a spawn proposal (End Matter, spawn step:
// the multinomial over the column's (target, Re/Im) channels, with importance weights); every
// lane of the wave calls.  Channel ch = 2 (g - 1) + comp of group g >= 1; thresholds P_ch sum to
// 2^32: a floor F = floor(2^32 / (16 nch)) each, the rest M shared in proportion to the weights
// W_ch (all zero: as all one), the remainder to the last channel.  Sample k draws Philox stream
// 0x40 + k: u = word 0 picks the channel whose interval [C, C + P) holds it, j = word 1 mod K, and
// the channel's Q32 amount x gives floor(|x| / (K P)) walkers plus one where j P + (u - C) <
// |x| mod (K P), with the sign of x -- a uniform on [0, K P), so the rounding is exact.
// Weights: uniform 1; heat-bath |x_ch| >> sh, sh = max(0, bitlen(|a| + |b|) + bitlen(q_off) - 24);
// MLP min(2^24, max(0, score_g)) for both components, score_g = b2[g-1] + w2[g-1] . h (0 past
// kPropOut groups); kind 4 the same with score_g = b3[g-1] + w3[g-1] . h2 (0 past kDeepOut).
__device__ __forceinline__ void spawn_proposal(Emitter& em, const TableView& tv, bool valid,
                                               uint64_t ck, int2 v, const KeyLayout& kl,
                                               const QmcProposal& pr, uint32_t step,
                                               uint64_t seed, uint8_t* hid) {
  const uint32_t lane = __lane_id();
  const uint64_t key = kl.key(ck);
  if (pr.kind == 3) mlp_hidden(pr, key, hid);
  if (pr.kind == 4) mlp_deep(pr, key, tv.h->active[0], tv.h->active[1], hid);
  const uint32_t G = valid ? tv.h->n_groups : 0u;
  const bool act = valid && G > 1;
  if (__ballot(act) == 0) return;
  // the lane's hidden units feeding the scores, four per word: kind 3 h in registers, kind 4 h2
  // read from its LDS row as the scores need it
  uint32_t hw[kPropHidden / 4];
#pragma unroll
  for (int q = 0; q < kPropHidden / 4; ++q)
    hw[q] = pr.kind == 3 ? reinterpret_cast<const uint32_t*>(hid + lane * kPropHidden)[q] : 0u;
  const uint4* h2row = reinterpret_cast<const uint4*>(hid + (kWave + lane) * kDeepHidden);
  const uint64_t sab = uabs64(v.x) + uabs64(v.y);
  const uint32_t nch = act ? 2 * (G - 1) : 2u;
  const uint64_t T32 = 1ull << 32, F = T32 / (16ull * nch), M = T32 - (uint64_t)nch * F;
  uint32_t sh = 0;
  if (pr.kind == 2) {
    const uint32_t bl = bitlen64(sab) + bitlen64(tv.h->q_off);
    sh = bl > 24 ? bl - 24 : 0u;
  }
  auto weights = [&](uint32_t g, uint64_t& wr, uint64_t& wi) __attribute__((always_inline)) {
    if (pr.kind == 2) {
      int32_t cre, cim;
      group_coeff(tv.t, tv.gs[g], tv.gs[g + 1], key, cre, cim);
      int64_t xre, xim;
      cmul_q32(v.x, v.y, cre, cim, xre, xim);
      wr = uabs64(xre) >> sh;
      wi = uabs64(xim) >> sh;
    } else {
      int32_t sc = 0;
      if (pr.kind == 4) {
        if (g - 1 < (uint32_t)kDeepOut) {
          const uint4* w3r = reinterpret_cast<const uint4*>(pr.w3 + (g - 1) * kDeepHidden);
          sc = pr.b3[g - 1];
#pragma unroll
          for (int q = 0; q < kDeepHidden / 16; ++q) {
            const uint4 h = h2row[q], w = w3r[q];
            sc = __builtin_amdgcn_sdot4((int)h.x, (int)w.x, sc, false);
            sc = __builtin_amdgcn_sdot4((int)h.y, (int)w.y, sc, false);
            sc = __builtin_amdgcn_sdot4((int)h.z, (int)w.z, sc, false);
            sc = __builtin_amdgcn_sdot4((int)h.w, (int)w.w, sc, false);
          }
        }
      } else if (g - 1 < (uint32_t)kPropOut) {
        const uint32_t* w2r = reinterpret_cast<const uint32_t*>(pr.w2 + (g - 1) * kPropHidden);
        sc = pr.b2[g - 1];
#pragma unroll
        for (int q = 0; q < kPropHidden / 4; ++q)
          sc = __builtin_amdgcn_sdot4((int)hw[q], (int)w2r[q], sc, false);
      }
      const uint64_t w = sc <= 0 ? 0ull : (sc > (1 << 24) ? (1ull << 24) : (uint64_t)sc);
      wr = wi = w;
    }
  };
  uint64_t S = 0;
  if (pr.kind >= 2 && act)
    for (uint32_t g = 1; g < G; ++g) {
      uint64_t wr, wi;
      weights(g, wr, wi);
      S += wr + wi;
    }
  const uint64_t St = S ? S : nch;
  const uint32_t rep = kl.replica(ck);
  // The draws of one sample: channel ch with interval [C, C + P) holding u, and its record.
  auto emit_draw = [&](uint32_t ch, uint64_t C, uint64_t P, uint64_t u, uint32_t j)
      __attribute__((always_inline)) {
    const uint32_t g = act ? 1 + ch / 2 : 1u;
    int2 rec = make_int2(0, 0);
    bool over = false;
    if (act) {
      int32_t cre, cim;
      group_coeff(tv.t, tv.gs[g], tv.gs[g + 1], key, cre, cim);
      int64_t xre, xim;
      cmul_q32(v.x, v.y, cre, cim, xre, xim);
      const int64_t x = (ch & 1u) ? xim : xre;
      const uint64_t a = uabs64(x), D = (uint64_t)pr.k * P;
      const uint64_t U = (uint64_t)(j & (pr.k - 1)) * P + (u - C);
      const uint64_t m = a / D + (U < a % D ? 1u : 0u);
      if (m > 0x7FFFFFFFull) {
        over = true;
      } else {
        const int32_t n = x < 0 ? -(int32_t)m : (int32_t)m;
        rec = (ch & 1u) ? make_int2(0, n) : make_int2(n, 0);
      }
    }
    if (over) em.overflow();
    em.emit((rec.x | rec.y) != 0, kl.rkey(ck ^ (act ? tv.gx[g] : 0ull), sab), rec);
  };
  if (pr.kind == 1) {
    const uint64_t P0 = F + M / nch;
    for (uint32_t k = 0; k < pr.k; ++k) {
      uint32_t q[4] = {0, 0, 0, 0};
      if (act) walker_random(key, step, rep, seed, 0x40u + k, q);
      uint32_t ch = (uint32_t)((uint64_t)q[0] / P0);
      if (ch > nch - 1) ch = nch - 1;
      const uint64_t C = (uint64_t)ch * P0;
      emit_draw(ch, C, ch + 1 < nch ? P0 : T32 - C, q[0], q[1]);
    }
    return;
  }
  // Weighted proposals: the samples in blocks of kSamp, each block's channels found in one scan
  // over the groups (the thresholds are recomputed from the weights on the way).
  constexpr int kSamp = 8;
  for (uint32_t k0 = 0; k0 < pr.k; k0 += kSamp) {
    uint32_t su[kSamp], sj[kSamp], sch[kSamp];
    uint64_t sC[kSamp], sP[kSamp];
    bool sf[kSamp];
#pragma unroll
    for (int b = 0; b < kSamp; ++b) {
      uint32_t q[4] = {0, 0, 0, 0};
      if (act && k0 + b < pr.k) walker_random(key, step, rep, seed, 0x40u + k0 + b, q);
      su[b] = q[0];
      sj[b] = q[1];
      sch[b] = 0;
      sC[b] = 0;
      sP[b] = 1;
      sf[b] = !(act && k0 + b < pr.k);
    }
    if (act) {
      uint64_t C = 0;
      for (uint32_t g = 1; g < G; ++g) {
        uint64_t wr, wi;
        weights(g, wr, wi);
#pragma unroll
        for (uint32_t comp = 0; comp < 2; ++comp) {
          const uint32_t c2 = 2 * (g - 1) + comp;
          const uint64_t w = S ? (comp ? wi : wr) : 1ull;
          const uint64_t p = c2 + 1 == nch ? T32 - C : F + (w * M) / St;
#pragma unroll
          for (int b = 0; b < kSamp; ++b)
            if (!sf[b] && (uint64_t)su[b] < C + p) {
              sch[b] = c2;
              sC[b] = C;
              sP[b] = p;
              sf[b] = true;
            }
          C += p;
        }
      }
    }
#pragma unroll
    for (int b = 0; b < kSamp; ++b)
      if (k0 + b < pr.k) emit_draw(sch[b], sC[b], sP[b], su[b], sj[b]);
  }
}

// Death/cloning record and children of one parent per lane, every lane of the wave calling
// (`valid` lanes hold a parent; (w0, w1) its spawn and death comb words).  The lane's table is its
// circuit's (tv); tables of different circuits may have different group counts, so the group
// loop runs to the largest count in the wave.  The death delta is a record of the parent's own
// key, summed into the next store by the merge like the children; qsh holds the per-segment Q32
// shifts of the table.
template <bool kProp>
__device__ __forceinline__ void spawn_records(Emitter& em, const TableView& tv, bool valid,
                                              uint64_t ck, int2 v, uint32_t w0, uint32_t w1,
                                              const KeyLayout& kl, const int64_t* qsh,
                                              const QmcProposal& pr, uint32_t step,
                                              uint64_t seed, uint8_t* hid) {
  const uint64_t key = kl.key(ck);
  const uint64_t sab = uabs64(v.x) + uabs64(v.y);
  {
    const int64_t qs = valid ? qsh[kl.replica(ck)] : 0;
    const bool dact = valid && !comb_all_zero(sab, tv.h->q_diag + uabs64(qs), w1);
    if (__ballot(dact)) {
      int2 d = make_int2(0, 0);
      if (dact) {
        int32_t dre, dim;
        group_coeff(tv.t, 0, tv.gs[1], key, dre, dim);
        int64_t xre, xim;
        cmul_q32(v.x, v.y, dre + (int32_t)qs, dim, xre, xim);
        uint64_t r = w1;
        d.x = (int32_t)comb_step(r, xre);
        d.y = (int32_t)comb_step(r, xim);
      }
      em.emit_diag((d.x | d.y) != 0, kl.rkey(ck, sab), d);
    }
  }
  if constexpr (kProp) {
    spawn_proposal(em, tv, valid, ck, v, kl, pr, step, seed, hid);
    return;
  }
  const uint32_t G = valid ? tv.h->n_groups : 0u;
  const bool act = valid && G > 1 && !comb_all_zero(sab, tv.h->q_off, w0);
  uint64_t r = w0;
  for (uint32_t g = 1; __ballot(act && g < G) != 0; ++g) {
    int2 child = make_int2(0, 0);
    uint64_t target = ck;
    if (act && g < G) {
      int32_t cre, cim;
      group_coeff(tv.t, tv.gs[g], tv.gs[g + 1], key, cre, cim);
      int64_t xre, xim;
      cmul_q32(v.x, v.y, cre, cim, xre, xim);
      child.x = (int32_t)comb_step(r, xre);
      child.y = (int32_t)comb_step(r, xim);
      target = ck ^ tv.gx[g];
      if (pr.log && (child.x | child.y) != 0) {
        const unsigned long long at = atomicAdd(pr.log_count, 1ull);
        if (at < pr.log_cap) pr.log[at] = SpawnEvent{ck, step, g, child.x, child.y};
      }
    }
    em.emit((child.x | child.y) != 0, kl.rkey(target, sab), child);
  }
}

// Records of one parent per lane drawn from Philox stream `stream` at step `step`.
template <bool kProp = false>
__device__ __forceinline__ void spawn_parent(Emitter& em, const TabSet& ts, bool valid,
                                             uint64_t ck, int2 v, uint32_t step, uint64_t seed,
                                             const KeyLayout& kl, uint32_t stream,
                                             const int64_t* qsh, const QmcProposal& pr = {},
                                             uint8_t* hid = nullptr) {
  uint32_t w[4] = {0, 0, 0, 0};
  if (valid) walker_random(kl.key(ck), step, kl.replica(ck), seed, stream, w);
  const TableView tv = table_view(ts.of_segment(valid ? kl.replica(ck) : 0u));
  spawn_records<kProp>(em, tv, valid, ck, v, w[0], w[1], kl, qsh, pr, step, seed, hid);
}

// Records of up to 64 queued parents (lane < n holds one, with the comb words drawn when it was
// queued).
template <bool kProp>
__device__ __forceinline__ void spawn_batch(Emitter& em, const TabSet& ts, const int64_t* qsh,
                                            const uint64_t* ak, const int2* av, const uint2* aw,
                                            uint32_t n, const KeyLayout& kl,
                                            const QmcProposal& pr, uint32_t step, uint64_t seed,
                                            uint8_t* hid) {
  const uint32_t lane = __lane_id();
  const bool valid = lane < n;
  const uint64_t ck = valid ? ak[lane] : 0;
  const int2 v = valid ? av[lane] : make_int2(0, 0);
  const uint2 w = valid ? aw[lane] : make_uint2(0, 0);
  const TableView tv = table_view(ts.of_segment(valid ? kl.replica(ck) : 0u));
  spawn_records<kProp>(em, tv, valid, ck, v, w.x, w.y, kl, qsh, pr, step, seed, hid);
}

// Death/cloning records and children of the n <= 64 queued parents (one per lane) with all the
// block's waves on the one batch: wave j takes the j-th of kWaves slices of each lane's diagonal
// terms and of its off-diagonal groups.  The partial diagonal coefficients are summed over the
// slices (integer sums, exact), and the comb of slice j starts where the comb over all earlier
// groups would stand: the uniform plus their amounts, mod 2^32 (what a run of comb steps leaves),
// so every record equals the one the single-wave comb in group order gives.  A short list of
// parents that all emit (the merge's queue) then costs a quarter of the group loop per batch.
// Block-uniform; dpart and cpart are kBlock entries of LDS that no one else uses meanwhile.
__device__ __forceinline__ void spawn_team(Emitter& em, const TabSet& ts, const int64_t* qsh,
                                           const uint64_t* ak, const int2* av, const uint2* aw,
                                           uint32_t n, const KeyLayout& kl, const QmcProposal& pr,
                                           uint32_t step, int2* dpart, uint32_t* cpart) {
  constexpr uint32_t J = kWaves;
  const uint32_t lane = __lane_id(), j = threadIdx.x / kWave;
  const bool valid = lane < n;
  const uint64_t ck = valid ? ak[lane] : 0;
  const int2 v = valid ? av[lane] : make_int2(0, 0);
  const uint2 w = valid ? aw[lane] : make_uint2(0, 0);
  const TableView tv = table_view(ts.of_segment(valid ? kl.replica(ck) : 0u));
  const uint64_t key = kl.key(ck);
  const uint64_t sab = uabs64(v.x) + uabs64(v.y);
  const int64_t qs = valid ? qsh[kl.replica(ck)] : 0;
  const uint32_t G = valid ? tv.h->n_groups : 0u;
  const bool dact = valid && !comb_all_zero(sab, tv.h->q_diag + uabs64(qs), w.y);
  const bool act = valid && G > 1 && !comb_all_zero(sab, tv.h->q_off, w.x);
  const uint32_t nd = valid ? tv.gs[1] / kTermPad : 0u;
  const uint32_t d0 = nd * j / J * kTermPad, d1 = nd * (j + 1) / J * kTermPad;
  const uint32_t g0 = G > 1 ? 1 + (G - 1) * j / J : 1u;
  const uint32_t g1 = G > 1 ? 1 + (G - 1) * (j + 1) / J : 1u;
  int32_t pre = 0, pim = 0;
  if (dact) group_coeff_part(tv.t, d0, d1, key, pre, pim);
  uint32_t amt = 0;  // this slice's comb amounts, mod 2^32
  if (act) {
    for (uint32_t g = g0; g < g1; ++g) {
      int32_t cre, cim;
      group_coeff(tv.t, tv.gs[g], tv.gs[g + 1], key, cre, cim);
      int64_t xre, xim;
      cmul_q32(v.x, v.y, cre, cim, xre, xim);
      amt += (uint32_t)uabs64(xre) + (uint32_t)uabs64(xim);
    }
  }
  dpart[threadIdx.x] = make_int2(pre, pim);
  cpart[threadIdx.x] = amt;
  __syncthreads();
  if (j == 0 && __ballot(dact)) {
    int2 d = make_int2(0, 0);
    if (dact) {
      int32_t dre = 0, dim = 0;
      for (uint32_t jj = 0; jj < J; ++jj) {
        const int2 pp = dpart[jj * kWave + lane];
        dre += pp.x;
        dim += pp.y;
      }
      int64_t xre, xim;
      cmul_q32(v.x, v.y, dre + (int32_t)qs, dim, xre, xim);
      uint64_t r = w.y;
      d.x = (int32_t)comb_step(r, xre);
      d.y = (int32_t)comb_step(r, xim);
    }
    em.emit_diag((d.x | d.y) != 0, kl.rkey(ck, sab), d);
  }
  uint32_t r0 = w.x;
  for (uint32_t jj = 0; jj < j; ++jj) r0 += cpart[jj * kWave + lane];
  uint64_t r = r0;
  for (uint32_t g = g0; __ballot(act && g < g1) != 0; ++g) {
    int2 child = make_int2(0, 0);
    uint64_t target = ck;
    if (act && g < g1) {
      int32_t cre, cim;
      group_coeff(tv.t, tv.gs[g], tv.gs[g + 1], key, cre, cim);
      int64_t xre, xim;
      cmul_q32(v.x, v.y, cre, cim, xre, xim);
      child.x = (int32_t)comb_step(r, xre);
      child.y = (int32_t)comb_step(r, xim);
      target = ck ^ tv.gx[g];
      if (pr.log && (child.x | child.y) != 0) {
        const unsigned long long at = atomicAdd(pr.log_count, 1ull);
        if (at < pr.log_cap) pr.log[at] = SpawnEvent{ck, step, g, child.x, child.y};
      }
    }
    em.emit((child.x | child.y) != 0, kl.rkey(target, sab), child);
  }
  __syncthreads();  // every wave has read the partials
}

// ---------------------------------------------------------------------------------------------
// k_spawn: the records of step `step` from the n = *count parents (pk, pv) and Philox stream
// `stream` (0: N(s), the Euler step and the first AB2 term; 1: N(s-1), the second AB2 term):
// the death/cloning record of every parent whose diagonal comb fires and its children.  One
// Philox draw per parent decides whether any of its combs can fire ((|a|+|b|) sum|q| + U >=
// 2^32); only those parents are queued (compacted over the workgroup) and processed in full
// 64-parent batches, so the group loop runs for parents that emit (most do not at small dt).
// ---------------------------------------------------------------------------------------------
template <bool kProp>
__global__ __launch_bounds__(kBlock) void k_spawn(
    const uint64_t* __restrict__ pk, const int2* __restrict__ pv, Counters* __restrict__ cnt,
    const uint64_t* __restrict__ count, TabSet ts, uint32_t step,
    uint64_t seed, KeyLayout kl, uint32_t stream, const int64_t* __restrict__ qsh,
    uint64_t* __restrict__ ck_out, int2* __restrict__ cv_out, uint64_t cap_child,
    uint32_t* __restrict__ ghist, uint32_t passes, QmcProposal pr) {
  __shared__ uint64_t s_key[kWaves][kSpawnSeg];
  __shared__ int2 s_val[kWaves][kSpawnSeg];
  // proposal networks: kind 3 uses 64 x kPropHidden bytes per wave, kind 4 two 64 x kDeepHidden
  __shared__ uint8_t s_hid[kProp ? kWaves : 1][kProp ? 2 * kWave * kDeepHidden : 4];
  __shared__ uint64_t s_ak[kMergeActive];  // queued parents: key, value, comb words
  __shared__ int2 s_av[kMergeActive];
  __shared__ uint2 s_aw[kMergeActive];
  __shared__ uint32_t s_cnt[kWaves];
  __shared__ uint64_t s_pk[kSpawnRound];   // the parents of one round, loaded all at once
  __shared__ int2 s_pv[kSpawnRound];
  if (cnt->err) return;
  const uint64_t np = *count;
  const uint32_t wave = threadIdx.x / kWave, lane = __lane_id();
  Emitter em{s_key[wave], s_val[wave], kSpawnSeg, 0, cnt, step & 1u, step, ck_out, cv_out,
             cap_child, ghist, passes};
  uint32_t nl = 0;  // queued parents (block-uniform)
  // Records of the first nb * 64 queued parents (at most nl), the rest moved to the front.
  auto drain = [&](uint32_t nb) __attribute__((always_inline)) {
    for (uint32_t b = wave; b < nb; b += kWaves) {
      const uint32_t b0 = b * kWave;
      spawn_batch<kProp>(em, ts, qsh, s_ak + b0, s_av + b0, s_aw + b0,
                         nl - b0 < (uint32_t)kWave ? nl - b0 : (uint32_t)kWave, kl, pr, step,
                         seed, s_hid[kProp ? wave : 0]);
    }
    const uint32_t done = nb * kWave < nl ? nb * kWave : nl;
    const uint32_t rest = nl - done;
    __syncthreads();
    uint64_t rk = 0;
    int2 rv = make_int2(0, 0);
    uint2 rw = make_uint2(0, 0);
    if (threadIdx.x < rest) {
      rk = s_ak[done + threadIdx.x];
      rv = s_av[done + threadIdx.x];
      rw = s_aw[done + threadIdx.x];
    }
    __syncthreads();
    if (threadIdx.x < rest) {
      s_ak[threadIdx.x] = rk;
      s_av[threadIdx.x] = rv;
      s_aw[threadIdx.x] = rw;
    }
    nl = rest;
    __syncthreads();
  };
  // table bounds of the segment of the last parent seen (parents are sorted by segment)
  uint32_t h_seg = ~0u;
  uint64_t h_qoff = 0, h_qdiag = 0;
  // Rounds of R parents: all of a round's loads in flight at once (LDS-direct dword loads, no
  // registers), then kBlock parents at a time from LDS.  R is kSpawnRound for long lists and
  // shrinks when the list would leave workgroups idle: a short list of parents that all emit
  // (the merge's queue) is spread over the grid rather than over a few workgroups.  At most one
  // 64-parent batch per workgroup (team): each drained at once with every wave of the workgroup
  // on it (spawn_team).
  uint64_t R = (np + gridDim.x - 1) / gridDim.x;
  const bool team = !kProp && R <= (uint64_t)kWave;
  R = (R + kBlock - 1) / kBlock * kBlock;
  if (R > (uint64_t)kSpawnRound) R = kSpawnRound;
  if (R < (uint64_t)kBlock) R = kBlock;
  if (team) R = kWave;
  const uint64_t stride = (uint64_t)gridDim.x * R;
  for (uint64_t rbase = (uint64_t)blockIdx.x * R; rbase < np; rbase += stride) {
    const uint32_t rn = (uint32_t)(np - rbase < R ? np - rbase : R);
    {
      const uint32_t* ks = reinterpret_cast<const uint32_t*>(pk + rbase);
      const uint32_t* vs = reinterpret_cast<const uint32_t*>(pv + rbase);
      uint32_t* kd = reinterpret_cast<uint32_t*>(s_pk);
      uint32_t* vd = reinterpret_cast<uint32_t*>(s_pv);
      for (uint32_t c = wave; c * kWave < 2 * rn; c += kWaves) {
        const uint32_t x = c * kWave + lane;
        if (x < 2 * rn) {
          __builtin_amdgcn_global_load_lds(ks + x, kd + c * kWave, 4, 0, 0);
          __builtin_amdgcn_global_load_lds(vs + x, vd + c * kWave, 4, 0, 0);
        }
      }
      __builtin_amdgcn_s_waitcnt(0);
    }
    __syncthreads();
    for (uint32_t sub = 0; sub < rn; sub += kBlock) {
      const uint32_t p = sub + threadIdx.x;
      bool act = false;
      uint64_t ck = 0;
      int2 v = make_int2(0, 0);
      uint32_t w[4] = {0, 0, 0, 0};
      if (p < rn) {
        ck = s_pk[p];
        v = s_pv[p];
        const uint32_t rep = kl.replica(ck);
        if (rep != h_seg) {
          const TableHeader* h = reinterpret_cast<const TableHeader*>(ts.of_segment(rep));
          h_qoff = h->n_groups > 1 ? h->q_off : 0;
          h_qdiag = h->q_diag + uabs64(qsh[rep]);
          h_seg = rep;
        }
        walker_random(kl.key(ck), step, rep, seed, stream, w);
        const uint64_t sab = uabs64(v.x) + uabs64(v.y);
        // a proposal draws for every parent of a column with off-diagonal groups
        act = (kProp ? h_qoff != 0 : !comb_all_zero(sab, h_qoff, w[0])) ||
              !comb_all_zero(sab, h_qdiag, w[1]);
      }
      const uint64_t m = __ballot(act);
      if (lane == 0) s_cnt[wave] = (uint32_t)__popcll(m);
      __syncthreads();
      uint32_t off = 0, tot = 0;
      for (uint32_t x = 0; x < (uint32_t)kWaves; ++x) {
        const uint32_t c = s_cnt[x];
        off += x < wave ? c : 0u;
        tot += c;
      }
      __syncthreads();
      if (nl + tot > (uint32_t)kMergeActive) drain(nl / kWave);
      if (act) {
        const uint32_t at = nl + off + mbcnt64(m);
        s_ak[at] = ck;
        s_av[at] = v;
        s_aw[at] = make_uint2(w[0], w[1]);
      }
      nl += tot;
      __syncthreads();
    }
    if (team && nl > 0) {  // the round's batch, drained at once (the round's LDS is free now)
      spawn_team(em, ts, qsh, s_ak, s_av, s_aw, nl, kl, pr, step, s_pv,
                 reinterpret_cast<uint32_t*>(s_pk));
      nl = 0;
    }
  }
  if (nl > 0) drain((nl + kWave - 1) / kWave);
  if (em.fill) em.flush();
  if (lane == 0 && em.ndiag)
    atomicAdd((unsigned long long*)&cnt->death_steps, (unsigned long long)em.ndiag);
}

// Digit histograms of n_child[nsel] records (used where records did not come from a spawn).
__global__ __launch_bounds__(kBlock) void k_digit_hist(const uint64_t* __restrict__ keys,
                                                       const Counters* __restrict__ cnt,
                                                       uint32_t nsel, uint32_t passes,
                                                       uint32_t* __restrict__ ghist) {
  if (cnt->err) return;
  const uint64_t n = cnt->n_child[nsel];
  for (uint64_t base = (uint64_t)blockIdx.x * kBlock + (threadIdx.x & ~63u); base < n;
       base += (uint64_t)gridDim.x * kBlock) {
    const uint64_t i = base + __lane_id();
    const bool v = i < n;
    const uint64_t k = v ? keys[i] : 0;
    const uint64_t act = __ballot(v);
    for (uint32_t p = 0; p < passes; ++p) {
      const uint32_t d = digit_of(k, p * kRadixBits);
      const uint64_t peers = match_digit(d, act);
      if (v && (peers & lanemask_lt()) == 0)
        atomicAdd(&ghist[p * kRadixBins + d], (uint32_t)__popcll(peers));
    }
  }
}

// ---------------------------------------------------------------------------------------------
// k_onesweep: one LSD radix pass.  Tiles of kBlock * IPT records are taken in order from a ticket
// counter; wave w of a block ranks records [w*64*IPT, (w+1)*64*IPT) of the tile stably in LDS; the
// tile's per-digit counts are published and the exclusive prefix over earlier tiles is found by
// decoupled look-back (Merrill & Garland), one status word per (tile, digit).
// ---------------------------------------------------------------------------------------------
__device__ __forceinline__ uint64_t lb_pack(uint32_t epoch, uint32_t flag, uint64_t v) {
  return ((uint64_t)(epoch & 0xFFFFu) << 48) | ((uint64_t)flag << 46) | (v & ((1ull << 46) - 1));
}
__device__ __forceinline__ uint32_t lb_epoch(uint64_t s) { return (uint32_t)(s >> 48); }
__device__ __forceinline__ uint32_t lb_flag(uint64_t s) { return (uint32_t)(s >> 46) & 3u; }
__device__ __forceinline__ uint64_t lb_value(uint64_t s) { return s & ((1ull << 46) - 1); }

__device__ __forceinline__ uint64_t wave_sum64(uint64_t v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// Merge-path split for diagonal d computed by one wave with 64-ary search (few dependent
// rounds instead of log2 of them): the number of A elements among the first d of the merge,
// A winning ties.
template <class KA, class KB>
__device__ uint32_t merge_path_wave(const KA& A, uint32_t na, const KB& B, uint32_t nb,
                                    uint32_t d) {
  const uint32_t lane = __lane_id();
  uint32_t lo = d > nb ? d - nb : 0u;
  uint32_t hi = d < na ? d : na;
  // invariant: answer in [lo, hi]; pred(p) = A[p] <= B[d-1-p] holds exactly for p < answer
  while (hi - lo > 64) {
    const uint32_t step = (hi - lo + 63) / 64;
    const uint32_t p = lo + lane * step;
    const bool t = p < hi && A(p) <= B(d - 1 - p);
    const uint32_t c = (uint32_t)__popcll(__ballot(t));
    const uint32_t nlo = c ? lo + (c - 1) * step + 1 : lo;
    const uint32_t nhi = lo + c * step < hi ? lo + c * step : hi;
    lo = nlo;
    hi = nhi;
  }
  const uint32_t p = lo + lane;
  const bool t = p < hi && A(p) <= B(d - 1 - p);
  return lo + (uint32_t)__popcll(__ballot(t));
}

// Stable ranks of one wave's slice of a sort tile: record k of the lane is
// kin[tbase + k * 64 + lane] (absent past n); rk[k] counts the slice's earlier records with the
// same digit, and wcnt[d] (this wave's row of LDS counters, zero on entry) ends as the slice's
// count of digit d.
template <int IPT>
__device__ __forceinline__ void rank_slice(const uint64_t* __restrict__ kin,
                                           const int2* __restrict__ vin, uint64_t n,
                                           uint64_t tbase, uint32_t shift, uint32_t* wcnt,
                                           uint64_t (&key)[IPT], int2 (&val)[IPT],
                                           uint32_t (&rk)[IPT]) {
  const uint32_t lane = __lane_id();
  const uint64_t lt = lanemask_lt();
#pragma unroll
  for (int k = 0; k < IPT; ++k) {
    const uint64_t i = tbase + (uint64_t)k * kWave + lane;
    const bool v = i < n;
    key[k] = v ? kin[i] : 0;
    val[k] = v ? vin[i] : make_int2(0, 0);
    const uint32_t d = digit_of(key[k], shift);
    const uint64_t peers = match_digit(d, __ballot(v));
    const uint32_t before = (uint32_t)__popcll(peers & lt);
    uint32_t seen = 0;
    if (v) seen = wcnt[d];
    rk[k] = seen + before;
    wave_lds_fence();
    if (v && before == 0) wcnt[d] = seen + (uint32_t)__popcll(peers);
    wave_lds_fence();
  }
}

// Per digit of thread tid (digits tid * DPT ...): the waves' counts become exclusive prefixes
// over the waves, and tot[i] the tile's count.
template <int DPT>
__device__ __forceinline__ void wave_digit_prefix(uint32_t (*wcnt)[kRadixBins], uint32_t tid,
                                                  uint32_t (&tot)[DPT]) {
#pragma unroll
  for (int i = 0; i < DPT; ++i) {
    const uint32_t d = tid * DPT + i;
    uint32_t run = 0;
    for (int w = 0; w < kWaves; ++w) {
      const uint32_t c = wcnt[w][d];
      wcnt[w][d] = run;
      run += c;
    }
    tot[i] = run;
  }
}

template <int IPT>
__global__ __launch_bounds__(kBlock) void k_onesweep(
    const uint64_t* __restrict__ kin, const int2* __restrict__ vin, uint64_t* __restrict__ kout,
    int2* __restrict__ vout, Counters* __restrict__ cnt, uint32_t nsel, uint32_t pass,
    const uint32_t* __restrict__ ghist, uint64_t* __restrict__ status, uint32_t epoch,
    uint32_t step) {
  constexpr int DPT = kRadixBins / kBlock;  // digits per thread
  constexpr int TILE = kBlock * IPT;        // records per tile
  __shared__ uint32_t s_gbase[kRadixBins];
  __shared__ uint32_t s_wcnt[kWaves][kRadixBins];
  __shared__ uint32_t s_pref[kRadixBins];
  __shared__ uint32_t s_part[kBlock];
  __shared__ uint32_t s_tile;
  if (cnt->err) return;
  const uint64_t n = cnt->n_child[nsel];
  const uint32_t ntiles = (uint32_t)((n + TILE - 1) / TILE);
  const uint32_t shift = pass * kRadixBits;
  const uint32_t tid = threadIdx.x, wave = tid / kWave, lane = __lane_id();
  const uint32_t* gh = ghist + pass * kRadixBins;
  uint32_t* ticket = &cnt->sort_ticket[nsel][pass];
  (void)lane;

  // First ticket before the prologue, so blocks without a tile leave at once.
  if (tid == 0) s_tile = atomicAdd(ticket, 1u);
  __syncthreads();
  if (s_tile >= ntiles) return;
  // Global exclusive digit offsets of this pass (thread t owns digits t*DPT .. t*DPT+DPT-1).
  {
    uint32_t loc[DPT], s = 0;
#pragma unroll
    for (int i = 0; i < DPT; ++i) {
      loc[i] = gh[tid * DPT + i];
      s += loc[i];
    }
    s_part[tid] = s;
    __syncthreads();
    for (int o = 1; o < kBlock; o <<= 1) {
      const uint32_t v = tid >= (uint32_t)o ? s_part[tid - o] : 0u;
      __syncthreads();
      s_part[tid] += v;
      __syncthreads();
    }
    uint32_t run = s_part[tid] - s;
#pragma unroll
    for (int i = 0; i < DPT; ++i) {
      s_gbase[tid * DPT + i] = run;
      run += loc[i];
    }
  }
  bool first_tile = true;

  while (true) {
    if (tid == 0 && !first_tile) s_tile = atomicAdd(ticket, 1u);
    first_tile = false;
#pragma unroll
    for (int i = 0; i < DPT; ++i)
      for (int w = 0; w < kWaves; ++w) s_wcnt[w][tid * DPT + i] = 0;
    __syncthreads();
    const uint32_t tile = s_tile;
    if (tile >= ntiles) break;
    const uint64_t tbase = (uint64_t)tile * TILE + (uint64_t)wave * (IPT * kWave);
    uint64_t key[IPT];
    int2 val[IPT];
    uint32_t rk[IPT];
    rank_slice<IPT>(kin, vin, n, tbase, shift, s_wcnt[wave], key, val, rk);
    __syncthreads();
    // Per digit: exclusive prefix over waves, and the tile total.
    uint32_t tot[DPT];
    wave_digit_prefix<DPT>(s_wcnt, tid, tot);
    // Publish and look back (all DPT digits of a thread advance through predecessors together).
    uint64_t* row = status + (uint64_t)tile * kRadixBins + tid * DPT;
#pragma unroll
    for (int i = 0; i < DPT; ++i)
      atomic_store_agent(&row[i], lb_pack(epoch, tile == 0 ? 2 : 1, tot[i]));
    uint32_t pref[DPT];
#pragma unroll
    for (int i = 0; i < DPT; ++i) pref[i] = 0;
    if (tile > 0) {
      uint32_t done = 0;  // bit i: digit i has reached an inclusive predecessor
      int32_t j = (int32_t)tile - 1;
      uint32_t spins = 0;
      while (done != (1u << DPT) - 1 && j >= 0) {
        const uint64_t* prow = status + (uint64_t)j * kRadixBins + tid * DPT;
        uint64_t sw[DPT];
        bool ready = true;
#pragma unroll
        for (int i = 0; i < DPT; ++i) {
          sw[i] = ((done >> i) & 1u) ? 0 : atomic_load_agent(&prow[i]);
          if (!((done >> i) & 1u) &&
              (lb_epoch(sw[i]) != (epoch & 0xFFFFu) || lb_flag(sw[i]) == 0))
            ready = false;
        }
        if (!ready) {
          if (++spins > (1u << 22)) {
            atomicOr(&cnt->err, kErrLookback);
            atomicMin(&cnt->err_step, step);
            break;
          }
          __builtin_amdgcn_s_sleep(1);
          continue;
        }
#pragma unroll
        for (int i = 0; i < DPT; ++i) {
          if ((done >> i) & 1u) continue;
          pref[i] += (uint32_t)lb_value(sw[i]);
          if (lb_flag(sw[i]) == 2) done |= 1u << i;
        }
        --j;
      }
#pragma unroll
      for (int i = 0; i < DPT; ++i)
        atomic_store_agent(&row[i], lb_pack(epoch, 2, pref[i] + tot[i]));
    }
#pragma unroll
    for (int i = 0; i < DPT; ++i) s_pref[tid * DPT + i] = s_gbase[tid * DPT + i] + pref[i];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < IPT; ++k) {
      const uint64_t i = tbase + (uint64_t)k * kWave + lane;
      if (i < n) {
        const uint32_t d = digit_of(key[k], shift);
        const uint32_t pos = s_pref[d] + s_wcnt[wave][d] + rk[k];
        if (pos < n) {
          kout[pos] = key[k];
          vout[pos] = val[k];
        } else {
          atomicOr(&cnt->err, kErrLookback);  // inconsistent digit histogram: refuse the write
          atomicMin(&cnt->err_step, step);
        }
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------------------------
// Step sort without look-back.  A pass over tiles of kStepSortTile records needs, per tile and
// digit, the number of the pass's records with that digit in earlier tiles.  k_tile_hist counts
// the first pass's digits per tile; k_sort_scan turns a pass's per-tile counts into per-tile
// offsets (digit base plus the earlier tiles' counts, one thread per digit and segment of
// tiles) and clears the next pass's counts; k_sort_scatter ranks each tile in LDS, writes its
// records at those offsets and counts the next pass's digits per output tile with one atomic
// per record.  No tile waits for another, so a pass costs three short dependent launches
// instead of a look-back chain through every tile.
// ---------------------------------------------------------------------------------------------
constexpr int kStepSortIpt = 8;
constexpr int kStepSortTile = kBlock * kStepSortIpt;
constexpr int kScanSegs = 16;  // tile segments per digit in k_sort_scan (one wave each)
constexpr int kScanDigits = kWave;  // digits per block of k_sort_scan (one per lane)

__global__ __launch_bounds__(kBlock) void k_tile_hist(const uint64_t* __restrict__ keys,
                                                      const Counters* __restrict__ cnt,
                                                      uint32_t nsel, uint32_t* __restrict__ hist) {
  __shared__ uint32_t s_h[kRadixBins];
  if (cnt->err) return;
  const uint64_t n = cnt->n_child[nsel];
  const uint32_t ntiles = (uint32_t)((n + kStepSortTile - 1) / kStepSortTile);
  for (uint32_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    for (uint32_t d = threadIdx.x; d < (uint32_t)kRadixBins; d += kBlock) s_h[d] = 0;
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kStepSortIpt; ++k) {
      const uint64_t i = (uint64_t)tile * kStepSortTile + (uint64_t)k * kBlock + threadIdx.x;
      if (i < n) atomicAdd(&s_h[digit_of(keys[i], 0)], 1u);
    }
    __syncthreads();
    uint32_t* row = hist + (uint64_t)tile * kRadixBins;
    for (uint32_t d = threadIdx.x; d < (uint32_t)kRadixBins; d += kBlock) row[d] = s_h[d];
    __syncthreads();
  }
}

// Block b: digits [64 b, 64 b + 64) (lane), wave w: tiles [w T / 16, (w + 1) T / 16).  In place,
// hist[t][d] becomes base(d) + sum over t' < t of hist[t'][d], where base(d) is the count of
// smaller digits in the pass (ghist); with next set, next[t][d] = 0 for every tile t.
__global__ __launch_bounds__(kScanSegs * kScanDigits) void k_sort_scan(
    const Counters* __restrict__ cnt, uint32_t nsel, const uint32_t* __restrict__ ghist,
    uint32_t* __restrict__ hist, uint32_t* __restrict__ next) {
  constexpr int kThreads = kScanSegs * kScanDigits;
  constexpr int kBatch = 16;  // loads in flight per thread
  __shared__ uint32_t s_seg[kScanSegs][kScanDigits];
  __shared__ uint32_t s_below[kScanSegs];
  if (cnt->err) return;
  const uint64_t n = cnt->n_child[nsel];
  const uint32_t ntiles = (uint32_t)((n + kStepSortTile - 1) / kStepSortTile);
  const uint32_t seg = threadIdx.x / kScanDigits, lane = __lane_id();
  const uint32_t d0 = blockIdx.x * kScanDigits, d = d0 + lane;
  // base(d): the pass's records with digits below d0, then the lower lanes of this block
  uint32_t below = 0;
  for (uint32_t x = threadIdx.x; x < d0; x += kThreads) below += ghist[x];
  below = team_sum(below, kWave);
  if (lane == 0) s_below[seg] = below;
  const uint32_t mine = ghist[d];
  const uint32_t base_lane = team_scan(mine, kWave, lane) - mine;
  // this segment's tiles and their column sum
  const uint32_t t0 = (uint32_t)(((uint64_t)seg * ntiles) / kScanSegs);
  const uint32_t t1 = (uint32_t)(((uint64_t)(seg + 1) * ntiles) / kScanSegs);
  uint32_t sum = 0;
  for (uint32_t t = t0; t < t1; t += kBatch) {
    uint32_t h[kBatch];
#pragma unroll
    for (int u = 0; u < kBatch; ++u)
      h[u] = t + u < t1 ? hist[(uint64_t)(t + u) * kRadixBins + d] : 0u;
#pragma unroll
    for (int u = 0; u < kBatch; ++u) sum += h[u];
  }
  s_seg[seg][lane] = sum;
  __syncthreads();
  uint32_t run = base_lane;
  for (int w = 0; w < kScanSegs; ++w) run += s_below[w];
  for (uint32_t w = 0; w < seg; ++w) run += s_seg[w][lane];
  for (uint32_t t = t0; t < t1; t += kBatch) {
    uint32_t h[kBatch];
#pragma unroll
    for (int u = 0; u < kBatch; ++u)
      h[u] = t + u < t1 ? hist[(uint64_t)(t + u) * kRadixBins + d] : 0u;
#pragma unroll
    for (int u = 0; u < kBatch; ++u) {
      if (t + u < t1) {
        hist[(uint64_t)(t + u) * kRadixBins + d] = run;
        if (next) next[(uint64_t)(t + u) * kRadixBins + d] = 0;
      }
      run += h[u];
    }
  }
}

// One pass: tile t's records ranked in LDS and written at off[t][digit] + rank; with next set,
// next[output tile][digit of the next pass] counts every record written.
__global__ __launch_bounds__(kBlock) void k_sort_scatter(
    const uint64_t* __restrict__ kin, const int2* __restrict__ vin, uint64_t* __restrict__ kout,
    int2* __restrict__ vout, Counters* __restrict__ cnt, uint32_t nsel, uint32_t shift,
    const uint32_t* __restrict__ off, uint32_t* __restrict__ next, uint32_t next_shift,
    uint32_t step) {
  constexpr int IPT = kStepSortIpt;
  constexpr int DPT = kRadixBins / kBlock;
  __shared__ uint32_t s_wcnt[kWaves][kRadixBins];
  __shared__ uint32_t s_pref[kRadixBins];
  if (cnt->err) return;
  const uint64_t n = cnt->n_child[nsel];
  const uint32_t ntiles = (uint32_t)((n + kStepSortTile - 1) / kStepSortTile);
  const uint32_t tid = threadIdx.x, wave = tid / kWave, lane = __lane_id();
  for (uint32_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
#pragma unroll
    for (int i = 0; i < DPT; ++i)
      for (int w = 0; w < kWaves; ++w) s_wcnt[w][tid * DPT + i] = 0;
    __syncthreads();
    const uint64_t tbase = (uint64_t)tile * kStepSortTile + (uint64_t)wave * (IPT * kWave);
    uint64_t key[IPT];
    int2 val[IPT];
    uint32_t rk[IPT];
    rank_slice<IPT>(kin, vin, n, tbase, shift, s_wcnt[wave], key, val, rk);
    __syncthreads();
    uint32_t tot[DPT];
    wave_digit_prefix<DPT>(s_wcnt, tid, tot);
    const uint32_t* orow = off + (uint64_t)tile * kRadixBins + tid * DPT;
#pragma unroll
    for (int i = 0; i < DPT; ++i) s_pref[tid * DPT + i] = orow[i];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < IPT; ++k) {
      const uint64_t i = tbase + (uint64_t)k * kWave + lane;
      if (i < n) {
        const uint32_t d = digit_of(key[k], shift);
        const uint64_t pos = (uint64_t)s_pref[d] + s_wcnt[wave][d] + rk[k];
        if (pos < n) {
          kout[pos] = key[k];
          vout[pos] = val[k];
          if (next)
            atomicAdd(&next[(pos / kStepSortTile) * kRadixBins + digit_of(key[k], next_shift)],
                      1u);
        } else {
          atomicOr(&cnt->err, kErrLookback);  // inconsistent digit counts: refuse the write
          atomicMin(&cnt->err_step, step);
        }
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------------------------
// Merge of parents (unique keys) with sorted children, split into tiles whose boundaries never
// cut a key's run (parents win ties, so a run is [parent] children...).
// ---------------------------------------------------------------------------------------------
// The search index of a sorted store: sidx[i] = keys[i kIdxStride] for every i kIdxStride below
// *count.  k_merge writes it for the store it produces; this kernel builds it for a store that
// came from elsewhere (the first step of a streamed run).
__global__ __launch_bounds__(kBlock) void k_store_index(const uint64_t* __restrict__ keys,
                                                        const uint64_t* __restrict__ count,
                                                        uint64_t* __restrict__ sidx) {
  const uint64_t n = *count, m = (n + kIdxStride - 1) >> kIdxShift;
  for (uint64_t i = blockIdx.x * (uint64_t)kBlock + threadIdx.x; i < m;
       i += (uint64_t)gridDim.x * kBlock)
    sidx[i] = keys[i << kIdxShift];
}

// Split points (one thread per tile boundary, from the records' merged positions that
// k_merge_delta wrote), plus the per-step resets of the counters the next step's kernels use.
__global__ __launch_bounds__(kBlock) void k_merge_part(const uint64_t* __restrict__ pk,
                                                       const uint64_t* __restrict__ ckeys,
                                                       Counters* __restrict__ cnt, uint32_t cur,
                                                       uint32_t csel, uint2* __restrict__ splits,
                                                       uint32_t max_tiles,
                                                       uint32_t* __restrict__ ghist_next,
                                                       uint32_t ish,
                                                       const uint32_t* __restrict__ mpos) {
  if (cnt->err) return;
  const uint32_t gt = blockIdx.x * kBlock + threadIdx.x;
  // The next step's child counter, sort tickets and digit histograms were last used two steps
  // ago; this step's merge, which spawns the next step's children, runs after this kernel.
  for (uint32_t i = gt; i < (uint32_t)(kMaxPasses * kRadixBins); i += gridDim.x * kBlock)
    ghist_next[i] = 0;
  if (gt == 0) {
    cnt->n_child[csel ^ 1] = 0;
    cnt->n_active = 0;
    for (int p = 0; p < kMaxPasses + 2; ++p) cnt->sort_ticket[csel ^ 1][p] = 0;
  }
  const uint32_t np = (uint32_t)cnt->n_store[cur];
  const uint32_t nc = (uint32_t)cnt->n_child[csel];
  const uint32_t total = np + nc;
  const uint32_t ntiles = (total + kMergeTile - 1) / kMergeTile;
  auto A = [&](uint32_t x) { return pk[x]; };
  auto B = [&](uint32_t x) { return ckeys[x] >> ish; };  // composite key of a routed record
  // One thread per tile boundary: the records among the first d merged items are the ones whose
  // merged position is below d (a binary search over the records' positions, a small array that
  // stays in the caches, instead of one over the store), then the boundary moves past the
  // records that continue the run of the last key before it.
  for (uint32_t t = gt; t <= ntiles && t <= max_tiles; t += gridDim.x * kBlock) {
    uint32_t d = t * kMergeTile;
    if (d > total) d = total;
    uint32_t lo = 0, hi = nc;
    while (lo < hi) {
      const uint32_t mid = (lo + hi) >> 1;
      if (mpos[mid] < d)
        lo = mid + 1;
      else
        hi = mid;
    }
    uint32_t j = lo;
    const uint32_t i = d - j;
    if (d > 0 && d < total) {
      uint64_t last = 0;
      if (i > 0) last = A(i - 1);
      if (j > 0) {
        const uint64_t c = B(j - 1);
        if (i == 0 || c > last) last = c;
      }
      // records continuing the run of `last` (at most kMergeSlack of them)
      const uint32_t jmax = nc - j < (uint32_t)kMergeSlack ? nc : j + (uint32_t)kMergeSlack;
      while (j < jmax && B(j) <= last) ++j;
    }
    splits[t] = make_uint2(i, j);
  }
}

// Output count of every merge tile, from its records alone: each of the tile's parents survives
// unless its records annihilate it, so the count is the parents, plus the record keys without a
// parent whose sum is nonzero, minus the parents whose sum with their records is zero.
// k_merge_delta (first of the class): one thread per record; the one at the start of a key's run
// finds the key's place a among the parents (binary search over the store), sums the run, writes
// every record's merged position (a, plus one with a parent, plus its own index) for
// k_merge_part, and adds +1 / -1 to tdelta[tile] for the tile of the run's first merged item,
// a + j (tile boundaries move only to run ends, so a key's parent and its records fall in that
// tile).  k_merge_count: one thread per tile, count = parents + delta (then clears the delta for
// the next step), and an exclusive scan over the 256 tiles of each block: tinfo[tile] =
// (count << 32) | first output counted from the block's first, bsum[b] = the block's outputs
// (k_merge_scan turns them into offsets).
__global__ __launch_bounds__(kBlock) void k_merge_delta(const uint64_t* __restrict__ pk,
                                                        const int2* __restrict__ pv,
                                                        const uint64_t* __restrict__ ckeys,
                                                        const int2* __restrict__ cvals,
                                                        const Counters* __restrict__ cnt,
                                                        uint32_t cur, uint32_t csel,
                                                        uint32_t* __restrict__ mpos,
                                                        int32_t* __restrict__ tdelta,
                                                        KeyLayout kl,
                                                        const uint64_t* __restrict__ sidx) {
  if (cnt->err) return;
  const uint32_t np = (uint32_t)cnt->n_store[cur];
  const uint32_t nc = (uint32_t)cnt->n_child[csel];
  const uint32_t ntiles = (np + nc + kMergeTile - 1) / kMergeTile;
  const uint32_t nidx = (np + kIdxStride - 1) >> kIdxShift;  // entries of the store's index
  for (uint32_t j = blockIdx.x * kBlock + threadIdx.x; j < nc; j += gridDim.x * kBlock) {
    const uint64_t k = kl.ckey(ckeys[j]);
    if (j > 0 && kl.ckey(ckeys[j - 1]) == k) continue;  // not the start of its run
    // The index (every kIdxStride-th parent key, a few MB that stay in the caches) narrows the
    // search to one block of parents: with x entries below k, the parents below k number more
    // than (x - 1) kIdxStride (entry x - 1 is one of them) and at most x kIdxStride (entry x,
    // if any, is not).
    uint32_t x = 0, y = nidx;
    while (x < y) {
      const uint32_t mid = (x + y) >> 1;
      if (sidx[mid] < k)
        x = mid + 1;
      else
        y = mid;
    }
    uint32_t a = x == 0 ? 0u : ((x - 1) << kIdxShift) + 1;  // parents below k
    uint32_t b = (x << kIdxShift) < np ? (x << kIdxShift) : np;
    while (a < b) {
      const uint32_t mid = (a + b) >> 1;
      if (pk[mid] < k)
        a = mid + 1;
      else
        b = mid;
    }
    const bool hp = a < np && pk[a] == k;
    int64_t re = 0, im = 0;
    if (hp) {
      const int2 v = pv[a];
      re = v.x;
      im = v.y;
    }
    const uint32_t before = a + (hp ? 1u : 0u);  // parents ahead of each of the run's records
    for (uint32_t q = j; q < nc; ++q) {
      const uint64_t rk = ckeys[q];
      if (kl.ckey(rk) != k) break;
      mpos[q] = before + q;
      if (kl.keep(rk, hp)) {
        const int2 v = cvals[q];
        re += v.x;
        im += v.y;
      }
    }
    const uint32_t tile = (a + j) / kMergeTile;
    if (tile >= ntiles) continue;  // cannot happen: a + j < np + nc
    const bool nz = re != 0 || im != 0;
    if (!hp && nz) atomicAdd(&tdelta[tile], 1);
    if (hp && !nz) atomicAdd(&tdelta[tile], -1);
  }
}

constexpr int kCountTiles = kBlock;  // tiles per block of k_merge_count
__global__ __launch_bounds__(kBlock) void k_merge_count(const Counters* __restrict__ cnt,
                                                        uint32_t cur, uint32_t csel,
                                                        const uint2* __restrict__ splits,
                                                        int32_t* __restrict__ tdelta,
                                                        uint64_t* __restrict__ tinfo,
                                                        uint64_t* __restrict__ bsum) {
  __shared__ uint32_t s_w[kWaves];
  if (cnt->err) return;
  const uint32_t np = (uint32_t)cnt->n_store[cur];
  const uint32_t nc = (uint32_t)cnt->n_child[csel];
  const uint32_t ntiles = (np + nc + kMergeTile - 1) / kMergeTile;
  if (blockIdx.x * kCountTiles >= ntiles) return;  // block-uniform
  const uint32_t tile = blockIdx.x * kCountTiles + threadIdx.x;
  const uint32_t wave = threadIdx.x / kWave, lane = __lane_id();
  uint32_t count = 0;
  if (tile < ntiles) {
    const uint2 s0 = splits[tile], s1 = splits[tile + 1];
    if (s1.x >= s0.x && s1.y >= s0.y && s1.x <= np && s1.y <= nc)  // else k_merge reports it
      count = (uint32_t)((int32_t)(s1.x - s0.x) + tdelta[tile]);
    tdelta[tile] = 0;  // zero again for the next step's k_merge_delta
  }
  const uint32_t incl = team_scan(count, kWave, lane);
  if (lane == kWave - 1) s_w[wave] = incl;
  __syncthreads();
  uint32_t wpre = 0;
  for (uint32_t x = 0; x < wave; ++x) wpre += s_w[x];
  if (tile < ntiles) tinfo[tile] = ((uint64_t)count << 32) | (wpre + incl - count);
  if (threadIdx.x == kBlock - 1) bsum[blockIdx.x] = wpre + incl;
}

// Exclusive prefix of the block sums of k_merge_count, in place (bsum[b] becomes the first output
// of block b's tiles; bsum[nblocks] the new store size), and the step's counters.  One
// workgroup.
constexpr int kScanBlock = 1024;
__global__ __launch_bounds__(kScanBlock) void k_merge_scan(uint64_t* __restrict__ bsum,
                                                           Counters* __restrict__ cnt,
                                                           uint32_t cur, uint32_t csel,
                                                           uint64_t cap_store, uint32_t step) {
  __shared__ uint64_t s_part[kScanBlock];
  if (cnt->err) return;
  const uint32_t np = (uint32_t)cnt->n_store[cur];
  const uint32_t nc = (uint32_t)cnt->n_child[csel];
  const uint32_t ntiles = (np + nc + kMergeTile - 1) / kMergeTile;
  const uint32_t nb = (ntiles + kCountTiles - 1) / kCountTiles;
  const uint32_t t = threadIdx.x;
  const uint32_t per = (nb + kScanBlock - 1) / kScanBlock;
  const uint32_t b = t * per < nb ? t * per : nb;
  const uint32_t e = b + per < nb ? b + per : nb;
  uint64_t sum = 0;
  for (uint32_t i = b; i < e; ++i) sum += bsum[i];
  s_part[t] = sum;
  __syncthreads();
  for (int o = 1; o < kScanBlock; o <<= 1) {  // inclusive scan of the thread sums
    const uint64_t x = t >= (uint32_t)o ? s_part[t - o] : 0;
    __syncthreads();
    s_part[t] += x;
    __syncthreads();
  }
  uint64_t run = s_part[t] - sum;
  for (uint32_t i = b; i < e; ++i) {
    const uint64_t c = bsum[i];
    bsum[i] = run;
    run += c;
  }
  if (t == kScanBlock - 1) {
    const uint64_t total = s_part[t];
    bsum[nb] = total;
    cnt->n_store[cur ^ 1] = total;
    cnt->child_steps += nc;
    cnt->out_steps += total;
    if (total > cap_store) {
      atomicOr(&cnt->err, kErrStoreCap);
      atomicMin(&cnt->err_step, step);
    }
  }
}

struct MergeArgs {
  const uint64_t* pk;
  const int2* pv;
  const uint64_t* ckeys;
  const int2* cvals;
  Counters* cnt;
  uint32_t cur, csel;
  const uint2* splits;
  const uint64_t* tinfo;     // per tile: (outputs << 32) | first output within its count block
  const uint64_t* boff;      // first output of every count block (k_merge_scan)
  uint32_t step;
  KeyLayout kl;
  uint64_t* ok;
  int2* ov;
  uint64_t cap_store;
  // With tab_next valid: every output whose comb can fire in step s+1 under these tables (Philox
  // stream 0, shifts qshift) is appended to (act_k, act_v) (cnt->n_active of them, at most
  // cap_store), the parents from which k_spawn draws that step's records.
  TabSet tab_next;
  const int64_t* qshift;
  uint64_t seed;
  uint64_t* act_k;
  int2* act_v;
  uint64_t* sidx;  // index of the new store: key of every kIdxStride-th record
};

// Annihilation: every tile's parents and sorted records go to LDS together (LDS-direct loads:
// a wave instruction moves 256 contiguous bytes and no registers hold the data, so all of a
// tile's loads are in flight at once), are merged with int64 sums per key, and the nonzero sums
// are written to the new store at the tile's offset.  The tiles are independent (their offsets
// come from k_merge_count and k_merge_scan): block b of G takes the contiguous tiles
// [b T / G, (b + 1) T / G).  As soon as a tile's records are in registers, the loads of the
// block's next tile are issued, so they are in flight while this tile's records are written and
// its next-step draws are made.
__global__ __launch_bounds__(kBlock) void k_merge(MergeArgs A) {
  constexpr int CAP = kMergeCap;
  __shared__ uint64_t s_pk[CAP];   // parents, then the tile's records behind them
  __shared__ int2 s_pv[CAP];
  __shared__ uint32_t s_scan[kWaves];
  __shared__ uint32_t s_xsplit[kBlock];  // merge-path split of each thread: parent | child << 16
  __shared__ uint64_t s_ws[kWaves];
  __shared__ uint64_t s_qk[kMergeQueue];  // outputs that can fire in step s+1, not yet appended
  __shared__ int2 s_qv[kMergeQueue];
  __shared__ uint64_t s_qbase;

  Counters* cnt = A.cnt;
  if (cnt->err) return;
  const uint32_t np = (uint32_t)cnt->n_store[A.cur];
  const uint32_t nc = (uint32_t)cnt->n_child[A.csel];
  const uint32_t ntiles = (np + nc + kMergeTile - 1) / kMergeTile;
  const uint32_t wave = threadIdx.x / kWave, lane = __lane_id();
  const KeyLayout kl = A.kl;
  uint64_t st_keys = 0;  // parents (thread 0), added once at the end
  uint64_t wsum = 0;     // walkers of the parents this thread's merge ranges held, over all tiles
  const bool draw = A.tab_next.valid();
  uint32_t nq = 0;  // queued outputs (block-uniform)
  // Appends the queue to the list of step s+1's parents (one atomic per flush).
  auto flush_queue = [&]() __attribute__((always_inline)) {
    if (threadIdx.x == 0)
      s_qbase = atomicAdd((unsigned long long*)&cnt->n_active, (unsigned long long)nq);
    __syncthreads();
    const uint64_t qb = s_qbase;
    for (uint32_t i = threadIdx.x; i < nq; i += kBlock)
      if (qb + i < A.cap_store) {
        A.act_k[qb + i] = s_qk[i];
        A.act_v[qb + i] = s_qv[i];
      }
    __syncthreads();
    nq = 0;
  };
  // table bounds of the segment of the last output seen (outputs are sorted by segment)
  uint32_t h_seg = ~0u;
  uint64_t h_qoff = 0, h_qdiag = 0;
  // A tile's parents [pa, pa + pn) and records [ca, ca + cn) from its split points; false if they
  // are inconsistent (cannot happen for runs shorter than the slack; reported, never loaded).
  auto geometry = [&](uint2 s0, uint2 s1, uint32_t& pa, uint32_t& pn, uint32_t& ca,
                      uint32_t& cn) __attribute__((always_inline)) -> bool {
    if (s1.x < s0.x || s1.y < s0.y || (s1.x - s0.x) + (s1.y - s0.y) > (uint32_t)CAP ||
        s1.x > np || s1.y > nc)
      return false;
    pa = s0.x;
    pn = s1.x - s0.x;
    ca = s0.y;
    cn = s1.y - s0.y;
    return true;
  };
  auto issue = [&](uint32_t pa, uint32_t pn, uint32_t ca, uint32_t cn)
      __attribute__((always_inline)) {
    auto to_lds = [&](const void* src, void* dst, uint32_t ndw) __attribute__((always_inline)) {
      const uint32_t* s32 = reinterpret_cast<const uint32_t*>(src);
      uint32_t* d32 = reinterpret_cast<uint32_t*>(dst);
      for (uint32_t c = wave; c * kWave < ndw; c += kWaves) {
        const uint32_t x = c * kWave + lane;
        if (x < ndw) __builtin_amdgcn_global_load_lds(s32 + x, d32 + c * kWave, 4, 0, 0);
      }
    };
    to_lds(A.pk + pa, s_pk, 2 * pn);
    to_lds(A.pv + pa, s_pv, 2 * pn);
    to_lds(A.ckeys + ca, s_pk + pn, 2 * cn);
    to_lds(A.cvals + ca, s_pv + pn, 2 * cn);
  };
  auto report = [&]() __attribute__((always_inline)) {
    if (threadIdx.x == 0) {
      atomicOr(&cnt->err, kErrLookback);
      atomicMin(&cnt->err_step, A.step);
    }
  };

  // this block's tiles: a contiguous run (a run crosses few replica boundaries, each of which
  // costs its threads a table-header load)
  const uint32_t t_end = (uint32_t)(((uint64_t)(blockIdx.x + 1) * ntiles) / gridDim.x);
  uint32_t pa = 0, pn = 0, ca = 0, cn = 0;
  bool ok = false;
  uint32_t tile = (uint32_t)(((uint64_t)blockIdx.x * ntiles) / gridDim.x);
  if (tile < t_end) {
    ok = geometry(A.splits[tile], A.splits[tile + 1], pa, pn, ca, cn);
    if (ok) issue(pa, pn, ca, cn);
  }
  for (; tile < t_end; ++tile) {
    const uint32_t next = tile + 1;
    const uint64_t ti = A.tinfo[tile];
    const uint64_t gbase = A.boff[tile / kCountTiles] + (uint32_t)ti, nout = ti >> 32;
    uint2 n0 = make_uint2(0, 0), n1 = make_uint2(0, 0);
    if (next < t_end) {
      n0 = A.splits[next];
      n1 = A.splits[next + 1];
    }
    __builtin_amdgcn_s_waitcnt(0);  // this tile's LDS data (and the loads above)
    __syncthreads();
    uint32_t npa = 0, npn = 0, nca = 0, ncn = 0;
    const bool nok = next < t_end && geometry(n0, n1, npa, npn, nca, ncn);
    if (!ok) {
      report();
      if (nok) issue(npa, npn, nca, ncn);
      pa = npa, pn = npn, ca = nca, cn = ncn, ok = nok;
      continue;
    }
    const uint64_t* const s_ck = s_pk + pn;
    const int2* const s_cv = s_pv + pn;
    if (threadIdx.x == 0) st_keys += pn;

    // Per-thread ranges of the local merge, cut only at run ends.
    auto KA = [&](uint32_t x) { return s_pk[x]; };
    auto KB = [&](uint32_t x) { return kl.ckey(s_ck[x]); };
    const uint32_t tot = pn + cn;
    uint32_t d0 = threadIdx.x * kMergeIpt;
    if (d0 > tot) d0 = tot;
    // this thread's end is the next thread's start (one search per thread)
    uint32_t i0, j0, i1, j1;
    run_split(KA, pn, KB, cn, d0, i0, j0);
    s_xsplit[threadIdx.x] = i0 | (j0 << 16);
    __syncthreads();
    if (threadIdx.x + 1 < (uint32_t)kBlock) {
      const uint32_t nx = s_xsplit[threadIdx.x + 1];
      i1 = nx & 0xFFFFu;
      j1 = nx >> 16;
    } else {
      i1 = pn;
      j1 = cn;
    }

    // One pass: the annihilated records of this thread's range, held in registers.  A range is
    // kMergeIpt merged items moved to run ends, and only the run of its last key can extend it,
    // so it holds at most kMergeIpt distinct keys; its parents lie between merge-path splits
    // kMergeIpt diagonals apart, so there are at most kMergeIpt of them.  The slots start as the
    // range's parents in key order; each run of equal-key records then adds its kept sum to its
    // key's parent or, with no parent and a nonzero sum, is inserted in key order.  Slots whose
    // sum is zero drop out of `live` (bit u: slot u is an output).  With records sparse, most
    // ranges hold none and their parents pass straight through.
    uint64_t rk[kMergeIpt];
    int2 rv[kMergeIpt];
    uint32_t live = 0;
    bool overflow = false, too_many = false;
    if (i1 - i0 > (uint32_t)kMergeIpt) {
      too_many = true;  // cannot happen (see above)
    } else {
      uint32_t used = i1 - i0;  // slots in use, in key order
#pragma unroll
      for (int u = 0; u < kMergeIpt; ++u) {
        const uint32_t x = i0 + u < (uint32_t)CAP ? i0 + (uint32_t)u : (uint32_t)CAP - 1;
        rk[u] = s_pk[x];
        rv[u] = s_pv[x];
        if ((uint32_t)u < used) wsum += uabs64(rv[u].x) + uabs64(rv[u].y);
      }
      live = (1u << used) - 1u;
      uint32_t j = j0;
      while (j < j1) {
        const uint64_t key = kl.ckey(s_ck[j]);
        // the key's parent among the slots (a record run never meets a key inserted by an
        // earlier run: runs have distinct keys), and the slots below the key
        uint32_t at = (uint32_t)kMergeIpt, below = 0;
#pragma unroll
        for (int u = 0; u < kMergeIpt; ++u)
          if ((uint32_t)u < used) {
            if (rk[u] == key) at = (uint32_t)u;
            below += rk[u] < key ? 1u : 0u;
          }
        const bool hp = at < (uint32_t)kMergeIpt;
        int64_t re = 0, im = 0;
        while (j < j1) {
          const uint64_t r = s_ck[j];
          if (kl.ckey(r) != key) break;
          if (kl.keep(r, hp)) {
            re += s_cv[j].x;
            im += s_cv[j].y;
          }
          ++j;
        }
        if (hp) {
#pragma unroll
          for (int u = 0; u < kMergeIpt; ++u)
            if ((uint32_t)u == at) {
              re += rv[u].x;
              im += rv[u].y;
              rv[u] = make_int2((int32_t)re, (int32_t)im);
            }
          if (re == 0 && im == 0) live &= ~(1u << at);
        } else if (re != 0 || im != 0) {
          if (used == (uint32_t)kMergeIpt) {
            too_many = true;  // cannot happen (see above); refuse rather than drop a record
          } else {
            // slots [below, used) move up by one, the new key takes slot `below`
#pragma unroll
            for (int u = kMergeIpt - 1; u > 0; --u)
              if ((uint32_t)u > below && (uint32_t)u <= used) {
                rk[u] = rk[u - 1];
                rv[u] = rv[u - 1];
              }
#pragma unroll
            for (int u = 0; u < kMergeIpt; ++u)
              if ((uint32_t)u == below) {
                rk[u] = key;
                rv[u] = make_int2((int32_t)re, (int32_t)im);
              }
            const uint32_t lo = live & ((1u << below) - 1u);
            live = lo | ((live & ~((1u << below) - 1u)) << 1) | (1u << below);
            ++used;
          }
        }
        if (re < INT32_MIN || re > INT32_MAX || im < INT32_MIN || im > INT32_MAX) overflow = true;
      }
    }
    const uint32_t count = (uint32_t)__popc(live);
    if (overflow) {
      atomicOr(&cnt->err, kErrOverflow);
      atomicMin(&cnt->err_step, A.step);
    }
    if (too_many) {  // cannot happen (see above); refuse rather than drop a record
      atomicOr(&cnt->err, kErrLookback);
      atomicMin(&cnt->err_step, A.step);
    }
    // Block exclusive scan of the counts: inclusive scan within each wave, then wave totals.
    const uint32_t incl = team_scan(count, kWave, lane);
    if (lane == kWave - 1) s_scan[wave] = incl;
    __syncthreads();  // also: every thread has finished reading the tile's LDS data
    uint32_t wpre = 0, agg = 0;
    for (uint32_t x = 0; x < (uint32_t)kWaves; ++x) {
      const uint32_t v = s_scan[x];
      wpre += x < wave ? v : 0u;
      agg += v;
    }
    // (the count pass must agree with the merge; a disagreement is an internal error, reported
    // rather than written)
    if (agg != nout) {
      report();
      agg = 0;
    }
    // The tile's records go through LDS once more, in output order, so that each store below
    // writes contiguous lanes (a thread's own records would leave gaps of its neighbours' counts
    // between lanes).  At most kMergeTile of them: a thread's range holds at most kMergeIpt keys.
    if (agg) {
      uint32_t at = wpre + incl - count;
#pragma unroll
      for (int u = 0; u < kMergeIpt; ++u)
        if ((live >> u) & 1u) {
          s_pk[at] = rk[u];
          s_pv[at] = rv[u];
          ++at;
        }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < kMergeIpt; ++u) {
      const uint32_t x = threadIdx.x + (uint32_t)u * kBlock;
      if (x < agg) {
        rk[u] = s_pk[x];
        rv[u] = s_pv[x];
      }
    }
    __syncthreads();  // the staged records are in registers
    // the next tile's loads, in flight during the rest of this one
    if (nok) issue(npa, npn, nca, ncn);
    // The tile's records to the new store at its offset, record x of the tile by thread
    // x mod kBlock; with the next step's tables, Philox once per record and the ones whose combs
    // can fire are queued.
    uint32_t nact = 0;
    bool act[kMergeIpt];
#pragma unroll
    for (int u = 0; u < kMergeIpt; ++u) {
      act[u] = false;
      if (threadIdx.x + (uint32_t)u * kBlock < agg) {
        const uint64_t o = gbase + threadIdx.x + (uint32_t)u * kBlock;
        if (o < A.cap_store) {
          A.ok[o] = rk[u];
          A.ov[o] = rv[u];
          if ((o & (kIdxStride - 1)) == 0) A.sidx[o >> kIdxShift] = rk[u];
        }
        if (draw) {
          const uint32_t rep = kl.replica(rk[u]);
          if (rep != h_seg) {
            const TableHeader* h =
                reinterpret_cast<const TableHeader*>(A.tab_next.of_segment(rep));
            h_qoff = h->n_groups > 1 ? h->q_off : 0;
            h_qdiag = h->q_diag + uabs64(A.qshift[rep]);
            h_seg = rep;
          }
          uint32_t w[4];
          walker_random(kl.key(rk[u]), A.step + 1, rep, A.seed, 0u, w);
          const uint64_t sab = uabs64(rv[u].x) + uabs64(rv[u].y);
          act[u] = !comb_all_zero(sab, h_qoff, w[0]) || !comb_all_zero(sab, h_qdiag, w[1]);
          nact += act[u] ? 1u : 0u;
        }
      }
    }
    if (draw) {
      // block exclusive scan of the queued counts, then the records into the queue (or, when
      // more than it holds, straight into the list)
      const uint32_t ai = team_scan(nact, kWave, lane);
      if (lane == kWave - 1) s_scan[wave] = ai;  // (read for the counts two barriers ago)
      __syncthreads();
      uint32_t apre = 0, atot = 0;
      for (uint32_t x = 0; x < (uint32_t)kWaves; ++x) {
        const uint32_t v = s_scan[x];
        apre += x < wave ? v : 0u;
        atot += v;
      }
      if (atot > 0) {
        if (nq + atot > (uint32_t)kMergeQueue) flush_queue();
        uint32_t at = apre + ai - nact;
        if (atot > (uint32_t)kMergeQueue) {
          if (threadIdx.x == 0)
            s_qbase = atomicAdd((unsigned long long*)&cnt->n_active, (unsigned long long)atot);
          __syncthreads();
          const uint64_t qb = s_qbase;
#pragma unroll
          for (int u = 0; u < kMergeIpt; ++u)
            if (act[u]) {
              if (qb + at < A.cap_store) {
                A.act_k[qb + at] = rk[u];
                A.act_v[qb + at] = rv[u];
              }
              ++at;
            }
          __syncthreads();
        } else {
#pragma unroll
          for (int u = 0; u < kMergeIpt; ++u)
            if (act[u]) {
              s_qk[nq + at] = rk[u];
              s_qv[nq + at] = rv[u];
              ++at;
            }
          nq += atot;
        }
      }
    }
    pa = npa, pn = npn, ca = nca, cn = ncn, ok = nok;
  }
  __syncthreads();
  if (draw && nq > 0) flush_queue();
  // the block's walker sum: per wave, then thread 0 over the waves
  for (int o = 32; o > 0; o >>= 1) wsum += __shfl_xor(wsum, o);
  if (lane == 0) s_ws[wave] = wsum;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint64_t st_w = 0;
    for (int w = 0; w < kWaves; ++w) st_w += s_ws[w];
    if (st_keys) atomicAdd((unsigned long long*)&cnt->key_steps, (unsigned long long)st_keys);
    if (st_w) atomicAdd((unsigned long long*)&cnt->walker_steps, (unsigned long long)st_w);
  }
}

// ---------------------------------------------------------------------------------------------
// Utility and estimator kernels.
// ---------------------------------------------------------------------------------------------
__global__ void k_batch_begin(Counters* cnt, uint64_t* status, uint64_t n_status,
                              uint64_t* sort_status, uint64_t n_sort_status, uint32_t* ghist,
                              uint32_t n_ghist) {
  const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  if (t == 0) {
    cnt->n_child[0] = 0;
    cnt->n_child[1] = 0;
    cnt->err = 0;
    cnt->err_step = 0xFFFFFFFFu;
    cnt->tile_counter = 0;
    for (int s = 0; s < 2; ++s)
      for (int p = 0; p < kMaxPasses + 2; ++p) cnt->sort_ticket[s][p] = 0;
  }
  for (uint64_t i = t; i < n_status; i += stride) status[i] = 0;
  for (uint64_t i = t; i < n_sort_status; i += stride) sort_status[i] = 0;
  for (uint64_t i = t; i < n_ghist; i += stride) ghist[i] = 0;
}

// In-place sign flips of an ideal diagonal Pauli pulse, or key transform into (ck, cv) for a
// pulse with x != 0 (sorted afterwards).
__global__ __launch_bounds__(kBlock) void k_pulse(uint64_t* __restrict__ pk, int2* __restrict__ pv,
                                                  Counters* __restrict__ cnt, uint32_t cur,
                                                  uint32_t n, KeyLayout kl, uint32_t rep_per,
                                                  const uint64_t* __restrict__ pxz, bool any_x,
                                                  uint64_t* __restrict__ ck_out,
                                                  int2* __restrict__ cv_out, uint32_t csel) {
  const uint64_t np = cnt->n_store[cur];
  const uint64_t qm = n >= 32 ? 0xFFFFFFFFull : ((1ull << n) - 1);
  for (uint64_t p = (uint64_t)blockIdx.x * kBlock + threadIdx.x; p < np;
       p += (uint64_t)gridDim.x * kBlock) {
    const uint64_t ck = pk[p];
    int2 v = pv[p];
    // the Pauli of this record's circuit
    const uint32_t c = kl.replica(ck) / rep_per;
    const uint64_t x = pxz[2 * c], z = pxz[2 * c + 1];
    const uint64_t i = ck & qm, j = (ck >> n) & qm;
    const bool neg = ((__popcll(z & i) + __popcll(z & j)) & 1) != 0;
    if (neg) {
      if (v.x == INT32_MIN || v.y == INT32_MIN) atomicOr(&cnt->err, kErrOverflow);
      v.x = -v.x;
      v.y = -v.y;
    }
    if (!any_x) {
      pv[p] = v;
    } else {
      ck_out[p] = ck ^ ((x << n) | x);
      cv_out[p] = v;
    }
  }
  if (any_x && blockIdx.x == 0 && threadIdx.x == 0) cnt->n_child[csel] = np;
}

// [out[0], out[1]) = the records of the sorted keys[0, *count) with lo <= key <= hi (one
// thread: two binary searches).
__global__ void k_key_range(const uint64_t* __restrict__ keys, const uint64_t* __restrict__ count,
                            uint64_t lo, uint64_t hi, uint64_t* __restrict__ out) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  const uint64_t n = *count;
  uint64_t a = 0, b = n;
  while (a < b) {
    const uint64_t m = a + (b - a) / 2;
    if (keys[m] < lo)
      a = m + 1;
    else
      b = m;
  }
  uint64_t c = a, d = n;
  while (c < d) {
    const uint64_t m = c + (d - c) / 2;
    if (keys[m] <= hi)
      c = m + 1;
    else
      d = m;
  }
  out[0] = a;
  out[1] = c;
}

__global__ __launch_bounds__(kBlock) void k_copy_store(const uint64_t* __restrict__ ki,
                                                       const int2* __restrict__ vi,
                                                       uint64_t* __restrict__ ko,
                                                       int2* __restrict__ vo,
                                                       const uint64_t* __restrict__ count) {
  const uint64_t n = *count;
  for (uint64_t p = (uint64_t)blockIdx.x * kBlock + threadIdx.x; p < n;
       p += (uint64_t)gridDim.x * kBlock) {
    ko[p] = ki[p];
    vo[p] = vi[p];
  }
}

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

// Per-replica estimator numerators; blockIdx.y is the replica, whose segment of the sorted
// store is found by binary search.  Output per replica (int64 words):
//   [0] n_tot, [1] ndiag_re, [2] ndiag_im, [3] eps2_lo, [4] eps2_hi, [5..] pauli re/im pairs.
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
  const uint64_t seg_e =
      (kl.kbits >= 64) ? np : lower_bound64(pk, np, (uint64_t)(rep + 1) << kl.kbits);
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

// out[r] = the first record of replica r in the sorted composite keys[0, *count), r < nrep, and
// out[nrep] = *count (one binary search per thread).
__global__ void k_replica_bounds(const uint64_t* __restrict__ keys,
                                 const uint64_t* __restrict__ count, uint32_t kbits,
                                 uint32_t nrep, uint64_t* __restrict__ out) {
  const uint32_t r = blockIdx.x * blockDim.x + threadIdx.x;
  const uint64_t n = *count;
  if (r > nrep) return;
  if (r == nrep || (r > 0 && kbits >= 64)) {
    out[r] = n;
    return;
  }
  out[r] = r == 0 ? 0 : lower_bound64(keys, n, (uint64_t)r << kbits);
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

// Workgroups of a kernel with kBlock threads that are resident on the whole device at once (at
// most cap): kernels whose tiles are strided over the grid launch no more, since a workgroup that
// had to wait for a free slot would run all of its tiles after the others finished theirs.
// Taken once per device and slot from the occupancy the compiled kernel reaches (its LDS and
// registers).
template <class K>
static uint32_t resident_blocks(K kernel, int slot, uint32_t cap) {
  constexpr int kDevices = 64, kSlots = 4;
  static uint32_t cached[kSlots][kDevices] = {};
  int dev = 0;
  if (slot < 0 || slot >= kSlots || hipGetDevice(&dev) != hipSuccess || dev < 0 ||
      dev >= kDevices)
    return 256;
  if (cached[slot][dev] == 0) {
    int per_cu = 0, cus = 0;
    uint32_t g = 256;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, kBlock, 0) == hipSuccess &&
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
        per_cu > 0 && cus > 0)
      g = (uint32_t)per_cu * (uint32_t)cus;
    cached[slot][dev] = g < cap ? g : cap;
  }
  return cached[slot][dev];
}
static uint32_t merge_blocks() { return resident_blocks(k_merge, 0, (uint32_t)kMergeBlocks); }

static inline uint32_t grid_for(uint64_t n, uint32_t cap_blocks) {
  uint64_t g = (n + kBlock - 1) / kBlock;
  if (g < 1) g = 1;
  if (g > cap_blocks) g = cap_blocks;
  return (uint32_t)g;
}

// init_min > 0 turns the initiator approximation on (one flag bit below each routed key).
static inline KeyLayout key_layout(uint32_t kbits, uint64_t init_min = 0) {
  return KeyLayout{kbits, kbits >= 64 ? ~0ull : ((1ull << kbits) - 1), init_min ? 1u : 0u,
                   init_min};
}

}  // namespace qmc

using namespace qmc;

extern "C" {

uint32_t qmck_sort_passes(uint32_t key_bits) {
  return key_bits == 0 ? 1u : (key_bits + kRadixBits - 1) / kRadixBits;
}

int qmck_batch_begin(hipStream_t st, void* counters, uint64_t* status, uint64_t n_status,
                     uint64_t* sort_status, uint64_t n_sort_status, uint32_t* ghist,
                     uint32_t n_ghist) {
  uint64_t big = n_status > n_sort_status ? n_status : n_sort_status;
  uint32_t g = grid_for(big, 2048);
  hipLaunchKernelGGL(k_batch_begin, dim3(g), dim3(kBlock), 0, st, (Counters*)counters, status,
                     n_status, sort_status, n_sort_status, ghist, n_ghist);
  return (int)hipGetLastError();
}

int qmck_spawn(hipStream_t st, const uint64_t* pk, const int2* pv, void* counters,
               const uint64_t* count, const uint8_t* tab_base, const uint32_t* tab_off,
               uint32_t rep_per, uint32_t step, uint64_t seed,
               uint32_t kbits, uint64_t init_min, uint32_t stream, const int64_t* qsh,
               uint64_t* ck, int2* cv, uint64_t cap_child, uint64_t max_parents, uint32_t* ghist,
               uint32_t passes, const QmcProposal* prop) {
  uint32_t g = grid_for(max_parents, 1024);
  const QmcProposal pr = prop ? *prop : QmcProposal{};
  if (pr.kind)
    hipLaunchKernelGGL(k_spawn<true>, dim3(g), dim3(kBlock), 0, st, pk, pv, (Counters*)counters,
                       count, TabSet{tab_base, tab_off, rep_per}, step, seed,
                       key_layout(kbits, init_min), stream, qsh, ck, cv, cap_child, ghist, passes,
                       pr);
  else
    hipLaunchKernelGGL(k_spawn<false>, dim3(g), dim3(kBlock), 0, st, pk, pv, (Counters*)counters,
                       count, TabSet{tab_base, tab_off, rep_per}, step, seed,
                       key_layout(kbits, init_min), stream, qsh, ck, cv, cap_child, ghist, passes,
                       pr);
  return (int)hipGetLastError();
}

int qmck_digit_hist(hipStream_t st, const uint64_t* keys, void* counters, uint32_t nsel,
                    uint32_t passes, uint32_t* ghist, uint64_t max_items) {
  uint32_t g = grid_for(max_items, 1024);
  hipLaunchKernelGGL(k_digit_hist, dim3(g), dim3(kBlock), 0, st, keys, (const Counters*)counters,
                     nsel, passes, ghist);
  return (int)hipGetLastError();
}

// Sorts n_child[nsel] records found in buffer pair `src` (0/1 of (k0,v0)/(k1,v1)); the result
// lands in pair src ^ (passes & 1).
int qmck_sort_tile_ok(uint32_t ipt) {
  return ipt == 8 || ipt == 12 || ipt == 16 || ipt == 24;
}

extern "C++" template <int IPT>
static void sort_passes(hipStream_t st, uint64_t* const* kb, int2* const* vb, void* counters,
                        uint32_t nsel, uint32_t passes, const uint32_t* ghist,
                        uint64_t* sort_status, uint32_t step, uint32_t src, uint64_t max_items) {
  const uint64_t tile = (uint64_t)kBlock * IPT;
  const uint64_t max_tiles = (max_items + tile - 1) / tile;
  const uint32_t g = (uint32_t)(max_tiles < (uint64_t)kPersistBlocks ? (max_tiles ? max_tiles : 1)
                                                                       : kPersistBlocks);
  uint32_t s = src;
  for (uint32_t p = 0; p < passes; ++p) {
    hipLaunchKernelGGL(k_onesweep<IPT>, dim3(g), dim3(kBlock), 0, st, kb[s], vb[s], kb[s ^ 1],
                       vb[s ^ 1], (Counters*)counters, nsel, p, ghist, sort_status,
                       sort_epoch(step, p), step);
    s ^= 1;
  }
}

uint64_t qmck_step_sort_hist_words(uint64_t max_items) {
  return ((max_items + kStepSortTile - 1) / kStepSortTile + 1) * (uint64_t)kRadixBins;
}

int qmck_sort_step(hipStream_t st, uint64_t* k0, int2* v0, uint64_t* k1, int2* v1, void* counters,
                   uint32_t nsel, uint32_t passes, const uint32_t* ghist, uint32_t* hist_a,
                   uint32_t* hist_b, uint32_t step, uint32_t src, uint64_t max_items) {
  uint64_t* kb[2] = {k0, k1};
  int2* vb[2] = {v0, v1};
  const uint64_t max_tiles = (max_items + kStepSortTile - 1) / kStepSortTile;
  const uint32_t cap = (uint32_t)(max_tiles ? (max_tiles < 4096 ? max_tiles : 4096) : 1);
  const uint32_t gh = std::min(resident_blocks(k_tile_hist, 1, 4096), cap);
  const uint32_t gs = std::min(resident_blocks(k_sort_scatter, 2, 4096), cap);
  Counters* cnt = (Counters*)counters;
  hipLaunchKernelGGL(k_tile_hist, dim3(gh), dim3(kBlock), 0, st, kb[src], cnt, nsel, hist_a);
  uint32_t* h[2] = {hist_a, hist_b};
  uint32_t s = src;
  for (uint32_t p = 0; p < passes; ++p) {
    uint32_t* nx = p + 1 < passes ? h[(p + 1) & 1] : nullptr;
    hipLaunchKernelGGL(k_sort_scan, dim3(kRadixBins / kScanDigits),
                       dim3(kScanSegs * kScanDigits), 0, st, cnt, nsel,
                       ghist + (size_t)p * kRadixBins, h[p & 1], nx);
    hipLaunchKernelGGL(k_sort_scatter, dim3(gs), dim3(kBlock), 0, st, kb[s], vb[s], kb[s ^ 1],
                       vb[s ^ 1], cnt, nsel, p * kRadixBits, h[p & 1], nx,
                       (p + 1) * kRadixBits, step);
    s ^= 1;
  }
  return (int)hipGetLastError();
}

int qmck_sort(hipStream_t st, uint64_t* k0, int2* v0, uint64_t* k1, int2* v1, void* counters,
              uint32_t nsel, uint32_t passes, const uint32_t* ghist, uint64_t* sort_status,
              uint32_t step, uint32_t src, uint64_t max_items, uint32_t ipt) {
  uint64_t* kb[2] = {k0, k1};
  int2* vb[2] = {v0, v1};
  switch (ipt) {
    case 8:
      sort_passes<8>(st, kb, vb, counters, nsel, passes, ghist, sort_status, step, src, max_items);
      break;
    case 12:
      sort_passes<12>(st, kb, vb, counters, nsel, passes, ghist, sort_status, step, src,
                      max_items);
      break;
    case 24:
      sort_passes<24>(st, kb, vb, counters, nsel, passes, ghist, sort_status, step, src,
                      max_items);
      break;
    default:
      sort_passes<16>(st, kb, vb, counters, nsel, passes, ghist, sort_status, step, src,
                      max_items);
      break;
  }
  return (int)hipGetLastError();
}

// Synthetic records for timing the sort: keys from a 64-bit mix of the index (the splitmix64
// finalizer), masked to the composite-key bits, value (1, 0).
__global__ __launch_bounds__(kBlock) void k_fill_sort_probe(uint64_t* __restrict__ k,
                                                            int2* __restrict__ v, uint64_t n,
                                                            uint64_t mask, uint64_t salt) {
  for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * kBlock) {
    uint64_t z = (i + salt) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    k[i] = z & mask;
    v[i] = make_int2(1, 0);
  }
}

int qmck_fill_sort_probe(hipStream_t st, uint64_t* k, int2* v, uint64_t n, uint64_t mask,
                         uint64_t salt) {
  hipLaunchKernelGGL(k_fill_sort_probe, dim3(grid_for(n, 2048)), dim3(kBlock), 0, st, k, v, n,
                     mask, salt);
  return (int)hipGetLastError();
}

int qmck_merge(hipStream_t st, const uint64_t* pk, const int2* pv, const uint64_t* ck,
               const int2* cv, void* counters, uint32_t cur, uint32_t csel, uint2* splits,
               uint64_t* tile_off, uint32_t step, uint32_t kbits, uint64_t init_min, uint64_t* ok,
               int2* ov, uint64_t cap_store, uint64_t max_items, uint32_t* ghist_next,
               const uint8_t* tab_base, const uint32_t* toff_next, uint32_t rep_per,
               const int64_t* qshift, uint64_t seed, uint64_t* act_k, int2* act_v,
               uint32_t* mpos, uint64_t* sidx) {
  const uint32_t max_tiles = (uint32_t)((max_items + kMergeTile - 1) / kMergeTile);
  const KeyLayout kl = key_layout(kbits, init_min);
  const uint32_t nblk = (max_tiles + kCountTiles - 1) / kCountTiles;
  uint64_t* bsum = tile_off + max_tiles;  // count blocks' sums, then offsets (nblk + 1 words)
  int32_t* tdelta = reinterpret_cast<int32_t*>(bsum + nblk + 1);  // max_tiles + 1 words
  hipLaunchKernelGGL(k_merge_delta, dim3(grid_for(max_items, 2048)), dim3(kBlock), 0, st, pk,
                     pv, ck, cv, (const Counters*)counters, cur, csel, mpos, tdelta, kl, sidx);
  hipLaunchKernelGGL(k_merge_part,
                     dim3(grid_for((uint64_t)max_tiles + 1, 2048)), dim3(kBlock), 0,
                     st, pk, ck, (Counters*)counters, cur, csel, splits, max_tiles, ghist_next,
                     kl.ish, mpos);
  hipLaunchKernelGGL(k_merge_count, dim3(nblk ? nblk : 1), dim3(kBlock), 0, st,
                     (const Counters*)counters, cur, csel, splits, tdelta, tile_off, bsum);
  hipLaunchKernelGGL(k_merge_scan, dim3(1), dim3(kScanBlock), 0, st, bsum, (Counters*)counters,
                     cur, csel, cap_store, step);
  MergeArgs a;
  a.pk = pk;
  a.pv = pv;
  a.ckeys = ck;
  a.cvals = cv;
  a.cnt = (Counters*)counters;
  a.cur = cur;
  a.csel = csel;
  a.splits = splits;
  a.tinfo = tile_off;
  a.boff = bsum;
  a.step = step;
  a.kl = kl;
  a.ok = ok;
  a.ov = ov;
  a.cap_store = cap_store;
  a.tab_next = TabSet{tab_base, toff_next, rep_per};
  a.qshift = qshift;
  a.seed = seed;
  a.act_k = act_k;
  a.act_v = act_v;
  a.sidx = sidx;
  const uint32_t mb = merge_blocks();
  hipLaunchKernelGGL(k_merge, dim3(max_tiles < mb ? (max_tiles ? max_tiles : 1) : mb),
                     dim3(kBlock), 0, st, a);
  return (int)hipGetLastError();
}

int qmck_store_index(hipStream_t st, const uint64_t* keys, const uint64_t* count,
                     uint64_t* sidx, uint64_t max_items) {
  hipLaunchKernelGGL(k_store_index, dim3(grid_for((max_items >> kIdxShift) + 1, 1024)),
                     dim3(kBlock), 0, st, keys, count, sidx);
  return (int)hipGetLastError();
}

int qmck_key_range(hipStream_t st, const uint64_t* keys, const uint64_t* count, uint64_t lo,
                   uint64_t hi, uint64_t* out) {
  hipLaunchKernelGGL(k_key_range, dim3(1), dim3(64), 0, st, keys, count, lo, hi, out);
  return (int)hipGetLastError();
}

int qmck_pulse(hipStream_t st, uint64_t* pk, int2* pv, void* counters, uint32_t cur, uint32_t n,
               uint32_t kbits, uint32_t rep_per, const uint64_t* pxz, int any_x, uint64_t* ck,
               int2* cv, uint32_t csel, uint64_t max_parents) {
  uint32_t g = grid_for(max_parents, 8192);
  hipLaunchKernelGGL(k_pulse, dim3(g), dim3(kBlock), 0, st, pk, pv, (Counters*)counters, cur, n,
                     key_layout(kbits), rep_per, pxz, any_x != 0, ck, cv, csel);
  return (int)hipGetLastError();
}

int qmck_copy_store(hipStream_t st, const uint64_t* ki, const int2* vi, uint64_t* ko, int2* vo,
                    const uint64_t* count, uint64_t max_items) {
  uint32_t g = grid_for(max_items, 8192);
  hipLaunchKernelGGL(k_copy_store, dim3(g), dim3(kBlock), 0, st, ki, vi, ko, vo, count);
  return (int)hipGetLastError();
}

int qmck_observe(hipStream_t st, const uint64_t* pk, const int2* pv, void* counters, uint32_t cur,
                 uint32_t n, uint32_t kbits, uint32_t nrep, uint32_t n_pauli,
                 const uint64_t* pxz, uint32_t want_eps, unsigned long long* out,
                 uint32_t out_stride, uint64_t max_per_replica) {
  uint32_t gx = grid_for(max_per_replica, 1024);
  hipLaunchKernelGGL(k_observe, dim3(gx, nrep), dim3(kBlock),
                     out_stride * sizeof(unsigned long long), st, pk, pv,
                     (const Counters*)counters, cur, n, key_layout(kbits), n_pauli, pxz, want_eps,
                     out, out_stride);
  return (int)hipGetLastError();
}

int qmck_replica_bounds(hipStream_t st, const uint64_t* keys, const void* counters,
                        uint32_t kbits, uint32_t nrep, uint64_t* out) {
  const uint32_t g = (nrep + 1 + kBlock - 1) / kBlock;
  hipLaunchKernelGGL(k_replica_bounds, dim3(g), dim3(kBlock), 0, st, keys,
                     &((const Counters*)counters)->n_store[0], kbits, nrep, out);
  return (int)hipGetLastError();
}

int qmck_lookup(hipStream_t st, const uint64_t* pk, const int2* pv, void* counters, uint32_t cur,
                uint32_t kbits, const uint64_t* keys, uint32_t nk, uint32_t nrep, int64_t* out) {
  uint64_t tot = (uint64_t)nk * nrep;
  if (tot == 0) return 0;
  uint32_t g = (uint32_t)((tot + kBlock - 1) / kBlock);
  hipLaunchKernelGGL(k_lookup, dim3(g), dim3(kBlock), 0, st, pk, pv, (const Counters*)counters,
                     cur, key_layout(kbits), keys, nk, nrep, out);
  return (int)hipGetLastError();
}

}  // extern "C"
