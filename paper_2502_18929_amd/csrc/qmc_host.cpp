// qmc_host.cpp -- host runtime of libqmc: the C ABI of include/qmc.h.
//
// Responsibilities: validate the problem, compile the model of eq. (1) into Liouville-space
// source terms (eq. (2)), quantize them per step into Q32 tables with exact integer merging and
// the per-group bound, carve the caller's device workspace, enqueue the kernels of each step on
// the caller's stream, and turn device error flags into status codes with rollback to the last
// good step.  No device memory is allocated here; pinned host staging is.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <thread>
#include <vector>

#include "../../include/qmc.h"
#include "qmc_device.hpp"
#include "qmc_kernels.h"
#include "qmc_persist.h"
#include "qmc_small.h"

namespace {

constexpr uint32_t kMaxPauli = 256;
constexpr uint32_t kMaxLookup = 4096;
constexpr size_t kTableArea = 32u << 20;  // device bytes for the step tables of one window
// spawn-proposal MLP weights on the device: w1 int8 [hidden][in], b1 int32, w2 int8 [out][hidden],
// b2 int32 (each part a multiple of 8 bytes, so the int8 rows stay 8-byte aligned)
constexpr size_t kMlpW1 = (size_t)kPropHidden * kPropIn, kMlpB1 = (size_t)kPropHidden * 4,
                 kMlpW2 = (size_t)kPropOut * kPropHidden, kMlpB2 = (size_t)kPropOut * 4;
constexpr size_t kMlpBytes = kMlpW1 + kMlpB1 + kMlpW2 + kMlpB2;
// the deeper network (kind 4): w1, b1, w2, b2, w3, b3
constexpr size_t kDeepW1 = (size_t)kDeepHidden * kDeepIn, kDeepB1 = (size_t)kDeepHidden * 4,
                 kDeepW2 = (size_t)kDeepHidden * kDeepHidden, kDeepB2 = (size_t)kDeepHidden * 4,
                 kDeepW3 = (size_t)kDeepOut * kDeepHidden, kDeepB3 = (size_t)kDeepOut * 4;
constexpr size_t kDeepBytes = kDeepW1 + kDeepB1 + kDeepW2 + kDeepB2 + kDeepW3 + kDeepB3;
// sort tiles: kBlock x (8, 12, 16 or 24) records; 16 unless qmc_tune_sort picks another
constexpr uint64_t kSortTileMin = (uint64_t)qmc::kBlock * 8;
constexpr uint32_t kSortIpts[] = {8, 12, 16, 24};
constexpr uint32_t kMaxChunkSteps = 8000;  // look-back epochs stay distinct within a chunk
constexpr uint32_t kTableThreads = 8;      // host threads building the step tables of a call
constexpr uint32_t kSegBuffers = 3;        // segment buffers: N(s-1), N(s), N(s+1) for AB2
constexpr int kProfClasses = 6;            // kernel classes qmc_profile times
constexpr size_t kPinMirror = 1024;        // pinned bytes of the counters' copy
static_assert(sizeof(qmc::Counters) <= kPinMirror && sizeof(qmc::Counters) % 8 == 0,
              "the counters' copy is written in 8-byte words");
constexpr uint32_t kFinishOne = 16;        // segments up to which one workgroup ends a chain
constexpr uint32_t kHeadMax = 16;          // steps of a chain's early first batch, at most
constexpr uint32_t kSmallAutoKeys = 384;   // default of qmc_small_limit
// batches of the LDS-resident step in one chain (a window of steps)
constexpr uint32_t kSmallBatches = (kMaxChunkSteps + kSmallBatch - 1) / kSmallBatch;

size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

// A Liouville-space source term: rho -> w(t) * kappa0 * A rho B, acting on key k as
// k -> k ^ xmask with sign (-1)^parity(zmask & k) (the key-independent sign of the right factor
// is folded into kappa0).
struct SrcTerm {
  uint64_t xmask, zmask;
  double kre, kim;
  uint32_t weight_kind;  // 0: s_m, 1: gamma_k
  uint32_t weight_index;
};

struct QTerm {
  uint64_t xmask, zmask;
  int64_t qre, qim;
};

// A model's source terms laid out for the per-step table build (the same table as build_table,
// faster): per term its constant and its weight channel (H monomials first, then Lindblad
// operators), and the runs of terms with equal (xmask, zmask).
struct TermPlan {
  const std::vector<SrcTerm>* src = nullptr;
  uint32_t nh = 0;                    // channels below nh are H weights, the rest rates
  std::vector<double> kre, kim;
  std::vector<uint32_t> ch;           // weight channel of each term
  std::vector<uint32_t> run;          // run r: terms [run[r], run[r + 1])
  std::vector<uint64_t> rx, rz;       // masks of run r
  std::vector<uint32_t> used;         // the channels some term reads
};


struct Layout {
  size_t counters, sk0, sv0, ck0, ck1, cv0, cv1, ghist, sort_status, status, splits, tab, qshift,
      obs_out, obs_in, look_keys, look_out, seg_k, seg_v, seg_n, pk, pv, in_k, in_v, in_n, split,
      tab_off, tabB_off, slots, done, pulse, mlp, small_fail, small_stats, thist, mpos, sidx, total;
  uint64_t cap_store, cap_child, cap_sort, n_sort_status, max_tiles, status_words;
  uint32_t P;          // key ranges / workgroups of the persistent step
  uint64_t segcap;     // records per segment
  uint32_t incap;      // records per inbox
};

int pc_parity(uint64_t v) { return __builtin_popcountll(v) & 1; }

uint32_t replica_bits(uint32_t R) {
  uint32_t b = 0;
  while ((1ull << b) < R) ++b;
  return b;
}

// c.n_replicas counts store segments (circuits x replicas per circuit).
bool compute_layout(const qmc_config& c, uint32_t P, uint32_t n_circuits, Layout& L) {
  const uint64_t S = c.store_capacity * (uint64_t)c.n_replicas;
  const uint64_t C = c.spawn_capacity * (uint64_t)c.n_replicas;
  if (S == 0 || C == 0 || S >= (1ull << 31) || C >= (1ull << 31) || P == 0) return false;
  L.cap_store = S;
  L.cap_child = C;
  // the child buffers hold one step's children, or the whole store when a pulse with x != 0
  // re-sorts it
  L.cap_sort = std::max(S, C);
  // look-back status words of the sort, (tile, digit), for the smallest tile it can use
  L.n_sort_status = ((L.cap_sort + kSortTileMin - 1) / kSortTileMin) * qmc::kRadixBins;
  L.max_tiles = (S + C + qmc::kMergeTile - 1) / qmc::kMergeTile;
  L.P = P;
  L.segcap = std::max<uint64_t>(4096, (2 * S + P - 1) / P);
  L.incap = qmc::kInboxMax;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o = align256(o + bytes);
    return at;
  };
  L.counters = take(sizeof(qmc::Counters));
  L.sk0 = take(S * 8);
  L.sv0 = take(S * 8);
  L.ck0 = take(L.cap_sort * 8);
  L.ck1 = take(L.cap_sort * 8);
  L.cv0 = take(L.cap_sort * 8);
  L.cv1 = take(L.cap_sort * 8);
  L.ghist = take((size_t)2 * qmc::kMaxPasses * qmc::kRadixBins * 4);
  L.sort_status = take(L.n_sort_status * 8);
  // merge tile counts and offsets (max_tiles words), the count blocks' sums and offsets (one
  // block per 256 tiles, plus the total), then the tiles' int32 count adjustments
  L.status_words = (L.max_tiles + (L.max_tiles + 255) / 256 + 1) + (L.max_tiles + 2) / 2;
  L.status = take(L.status_words * 8);
  L.splits = take((L.max_tiles + 1) * 8);
  L.tab = take(kTableArea + kPersistTableBytes);  // slack: the fused kernel reads 8 KB
  L.qshift = take((size_t)c.n_replicas * 2 * 8);  // first / only term, then the second AB2 term
  L.obs_out = take((size_t)c.n_replicas * (5 + 2 * kMaxPauli) * 8);
  L.obs_in = take((size_t)kMaxPauli * 16);
  L.look_keys = take((size_t)kMaxLookup * 8);
  L.look_out = take((size_t)c.n_replicas * kMaxLookup * 16);
  L.seg_k = take((size_t)kSegBuffers * P * L.segcap * 8);
  L.seg_v = take((size_t)kSegBuffers * P * L.segcap * 8);
  L.seg_n = take((size_t)kSegBuffers * P * 4);
  L.pk = take(S * 8);  // N(s-1) (AB2)
  L.pv = take(S * 8);
  L.in_k = take((size_t)2 * P * L.incap * 8);
  L.in_v = take((size_t)2 * P * L.incap * 8);
  L.in_n = take((size_t)2 * P * 4);
  L.split = take((size_t)P * 8);
  L.tab_off = take((size_t)kMaxChunkSteps * 4 * n_circuits);
  L.tabB_off = take((size_t)kMaxChunkSteps * 4);
  L.slots = take((size_t)2 * P * 4 * 8);
  L.done = take(8);
  L.pulse = take((size_t)n_circuits * 16);
  L.mlp = take(kMlpBytes + kDeepBytes);
  L.small_fail = take(8);
  L.small_stats = take((size_t)kSmallBatches * c.n_replicas * kSmallStats * 8);
  // per-tile digit counts of the step sort, two buffers (a pass reads one, counts into the other)
  L.thist = take((size_t)2 * qmck_step_sort_hist_words(C) * 4);
  L.mpos = take(C * 4);  // merged positions of one step's records
  L.sidx = take(((S >> 8) + 2) * 8);  // the store's search index (every 256th key)
  L.total = o;
  return true;
}

// Workgroups of the persistent step that can be co-resident on the current device.
int persist_segments(uint32_t* P) {
  int p = 0;
  if (qmcp_max_segments(&p) != 0 || p <= 0) return QMC_ERR_HIP;
  *P = (uint32_t)p;
  return QMC_OK;
}

}  // namespace

struct qmc_ctx {
  qmc_config cfg{};
  // R = store segments = circuits x replicas per circuit (one circuit: R = the replicas)
  uint32_t n = 0, R = 0, kbits = 0, rbits = 0;
  uint32_t C = 1, Rc = 0;           // circuits of a batch, replicas per circuit
  uint32_t n_h = 0, n_l = 0;        // weights per step, all circuits together
  std::vector<std::vector<SrcTerm>> terms;  // per circuit
  std::vector<TermPlan> plans;               // per circuit, over `terms`
  std::vector<uint32_t> wh_off, wl_off;      // a circuit's first weight in a step's s / gamma
  Layout L{};
  uint8_t* ws = nullptr;
  hipStream_t stream = nullptr;
  uint32_t step = 0;
  uint32_t cur = 0;
  std::vector<double> shift;
  std::vector<int64_t> nd0_re;
  std::vector<int64_t> qshift_dev;  // the Q32 shifts last uploaded to the device (both terms)
  std::vector<uint8_t> shift_on;     // variable shift: the replica has reached shift_target
  std::vector<uint64_t> shift_ref;   // variable shift: N^tot at the last update
  uint8_t* pinned = nullptr;     // table staging: kTableArea bytes, then the window offsets
  uint8_t* pinned_small = nullptr;  // counters and estimator staging
  // Device addresses of the two pinned buffers: the LDS-resident step reads its step tables
  // straight from the staging area, and its finishing kernel writes a copy of the counters into
  // the last kPinMirror bytes of pinned_small (pin_mirror), so neither needs a copy on the stream.
  uint8_t* pinned_dev = nullptr;
  uint8_t* pinned_small_dev = nullptr;
  size_t pin_mirror = 0;
  // The table offsets of a chain's early first batch (kHeadMax steps x C circuits), in pinned
  // memory of their own right after the counters' copy: that batch runs while the host still
  // writes the call's other offsets, and no cache line it reads may hold any of those.
  size_t pin_head = 0;
  size_t pinned_small_bytes = 0;
  std::string err;
  bool broken = false;
  int32_t prof_class = -1;
  uint64_t epoch = 0;               // last barrier epoch used by the persistent step
  int32_t path = 0;                 // 0 automatic, 1 fused persistent kernel only, 2 streamed only
  int32_t integrator = 0;           // 0 Euler, 1 AB2
  uint64_t init_min = 0;            // initiator threshold in walkers (0 = off)
  QmcProposal prop{};               // spawn proposal (kind 0: the comb); weights on the device
  uint32_t sort_ipt = 16;           // records per thread of a sort tile
  bool use_graph = false;           // streamed chunks captured into a HIP graph and replayed
  hipGraphExec_t gexec = nullptr;   // the executable graph of the last captured chunk
  hipStream_t gstream = nullptr;    // the stream chunks are captured from (default priority)
  bool have_prev = false;           // AB2: N(s-1) (device) and w_prev are valid
  std::vector<double> w_prev;       // AB2: weights of step s-1 (s then gamma)
  uint64_t n_occ = 0;               // occupied keys (all replicas) after the last device sync
  uint32_t streamed_until = 0;      // automatic mode: steps before this one run streamed
  bool small_off = false;           // automatic mode: a replica outgrew the LDS-resident step
  uint32_t small_limit = kSmallAutoKeys;  // automatic mode: keys per replica it runs up to
  uint32_t small_epoch = 0;         // epoch of the last LDS-resident chain
  std::vector<hipEvent_t> prof_ev;   // start/stop pairs, one pair per step of a chunk
  // Whole-launch timings are read back lazily (qmc_profile_read): reading an event's time right
  // after the launch costs the step call up to tens of microseconds.  Each entry: class, start
  // and stop event, launches; the events return to ev_free once read.
  struct PendingTime {
    int cls;
    hipEvent_t a, b;
    uint64_t launches;
  };
  std::vector<PendingTime> ev_pending;
  std::vector<hipEvent_t> ev_free;
  // per kernel class: summed milliseconds and launches of the timed launches
  double prof_ms[kProfClasses] = {};
  uint64_t prof_launches[kProfClasses] = {};
  uint64_t relaunches = 0;  // fused launches that stopped to re-cut the key ranges
  qmc_stats prof_cover[kProfClasses] = {};  // counter deltas of the steps each class ran
  // the whole-step classes (3 fused, 4 LDS-resident) are timed together
  bool prof_whole() const { return prof_class == 3 || prof_class == 4; }
  qmc::Counters last_hc{};           // counters at the last device read

  template <class T>
  T* at(size_t off) const { return reinterpret_cast<T*>(ws + off); }
  // The store: always in the canonical buffer between calls.  The streamed step alternates
  // between it and the segment area of the persistent step (at least 4x the store capacity).
  uint64_t* sk(uint32_t) const { return at<uint64_t>(L.sk0); }
  int2* sv(uint32_t) const { return at<int2>(L.sv0); }
  uint64_t* alt_k(uint32_t i = 0) const {
    return at<uint64_t>(L.seg_k) + (size_t)i * L.cap_store;
  }
  int2* alt_v(uint32_t i = 0) const { return at<int2>(L.seg_v) + (size_t)i * L.cap_store; }
  uint64_t* pk() const { return at<uint64_t>(L.pk); }  // N(s-1), AB2
  int2* pv() const { return at<int2>(L.pv); }
  uint64_t* ck(uint32_t b) const { return at<uint64_t>(b ? L.ck1 : L.ck0); }
  int2* cv(uint32_t b) const { return at<int2>(b ? L.cv1 : L.cv0); }
  qmc::Counters* counters() const { return at<qmc::Counters>(L.counters); }
  uint32_t* ghist(uint32_t parity) const {
    return at<uint32_t>(L.ghist) + (size_t)parity * qmc::kMaxPasses * qmc::kRadixBins;
  }
  uint32_t* thist(uint32_t which) const {
    return at<uint32_t>(L.thist) + (size_t)which * qmck_step_sort_hist_words(L.cap_child);
  }
};

namespace {

int fail(qmc_ctx* c, int code, const std::string& msg) {
  if (c) c->err = msg;
  return code;
}

int hip_fail(qmc_ctx* c, hipError_t e, const char* what) {
  if (c) {
    c->err = std::string(what) + ": " + hipGetErrorString(e);
    c->broken = true;
  }
  return QMC_ERR_HIP;
}

#define HIPCHK(ctx, expr)                                  \
  do {                                                     \
    hipError_t e_ = (hipError_t)(expr);                    \
    if (e_ != hipSuccess) return hip_fail(ctx, e_, #expr); \
  } while (0)

// Source terms of eqs. (1)-(2): -i H rho, +i rho H, gamma L rho L^dagger and
// -(gamma/2){L^dagger L, rho} for L_k = sum_a c_a X^xa Z^za.  The FP64 expressions are part of
// the arithmetic contract (the same operation order as the CPU oracle).
void compile_model(const qmc_model& m, uint32_t n, std::vector<SrcTerm>& out) {
  out.clear();
  auto emit = [&](uint64_t xm, uint64_t zm, double re, double im, uint32_t kind, uint32_t idx) {
    out.push_back(SrcTerm{xm, zm, re, im, kind, idx});
  };
  for (uint32_t i = 0; i < m.n_h; ++i) {
    const qmc_monomial& h = m.h[i];
    // left factor: kappa = -i h
    emit(h.x, h.z, h.im, -h.re, 0, i);
    // right factor: kappa = +i h times (-1)^popc(x & z)
    const double f = pc_parity(h.x & h.z) ? -1.0 : 1.0;
    emit(h.x << n, h.z << n, f * -h.im, f * h.re, 0, i);
  }
  for (uint32_t k = 0; k < m.n_l; ++k) {
    for (uint32_t a = m.l_off[k]; a < m.l_off[k + 1]; ++a) {
      for (uint32_t b = m.l_off[k]; b < m.l_off[k + 1]; ++b) {
        const qmc_monomial& A = m.l[a];
        const qmc_monomial& B = m.l[b];
        // gamma c_a conj(c_b) P_a rho P_b^dagger
        emit((B.x << n) | A.x, (B.z << n) | A.z, A.re * B.re + A.im * B.im,
             A.im * B.re - A.re * B.im, 1, k);
        // -(gamma/2) mu M rho and -(gamma/2) mu rho M, mu = conj(c_a) c_b * sign
        const double sg = ((__builtin_popcountll(A.x & A.z) + __builtin_popcountll(A.z & B.x)) & 1)
                              ? -1.0 : 1.0;
        const double mre = sg * (A.re * B.re + A.im * B.im);
        const double mim = sg * (A.re * B.im - A.im * B.re);
        const uint64_t x = A.x ^ B.x, z = A.z ^ B.z;
        emit(x, z, -0.5 * mre, -0.5 * mim, 1, k);
        const double f = pc_parity(x & z) ? -1.0 : 1.0;
        emit(x << n, z << n, f * (-0.5 * mre), f * (-0.5 * mim), 1, k);
      }
    }
  }
  // Terms of equal (xmask, zmask) adjacent, diagonal first: a step table then merges runs by
  // integer addition (order-free) without sorting again.
  std::stable_sort(out.begin(), out.end(), [](const SrcTerm& a, const SrcTerm& b) {
    return a.xmask != b.xmask ? a.xmask < b.xmask : a.zmask < b.zmask;
  });
}

// Q32 of scale * dt * w * kappa0: the product w * kappa0 first, then dt, then the integrator's
// factor (1 for Euler; 3/2 and -1/2 for the two AB2 terms), exact scaling by 2^32, round half to
// even.
bool quantize(double dt, double w, double k, double scale, int64_t& q) {
  // multiplying by 2^32 is exact (as ldexp); |v| < 2^51 rounds half to even by adding and
  // subtracting 1.5 * 2^52 in the default rounding mode, larger values go through llrint
  const double v = scale * (dt * (w * k)) * 4294967296.0;
  if (!(std::fabs(v) < 4611686018427387904.0)) return false;  // also NaN and infinities
  constexpr double kMagic = 6755399441055744.0;
  q = std::fabs(v) < 2251799813685248.0 ? (int64_t)((v + kMagic) - kMagic)
                                         : (int64_t)std::llrint(v);
  return true;
}

uint64_t uabs(int64_t v) { return v < 0 ? (uint64_t)0 - (uint64_t)v : (uint64_t)v; }

// Quantized, merged, grouped table for one step.
struct HostTable {
  std::vector<QTerm> t;          // grouped: diagonal first, then xmask ascending
  std::vector<uint64_t> gx;      // group masks (gx[0] = 0)
  std::vector<uint32_t> gs;      // group starts, size n_groups + 1
  uint64_t q_off = 0, q_diag = 0;
  uint64_t active[2] = {0, 0};   // nonzero weight channels of the step (proposal input)
};

int group_table(HostTable& T, std::string& why);

// The step's weight channels that are nonzero (the proposal network's input): H monomials
// m < nh, then Lindblad operators.
void active_channels(const double* s, const double* g, uint32_t nh, uint32_t nl, HostTable& T) {
  T.active[0] = T.active[1] = 0;
  for (uint32_t m = 0; m < nh + nl && m < 128; ++m) {
    const double w = m < nh ? s[m] : g[m - nh];
    if (w != 0.0) T.active[m >> 6] |= 1ull << (m & 63);
  }
}

int build_table(const std::vector<SrcTerm>& src, double dt, const double* s, const double* g,
                double scale, HostTable& T, std::string& why, uint32_t nh = 0, uint32_t nl = 0) {
  active_channels(s, g, nh, nl, T);
  // src is sorted by (xmask, zmask): each run of equal terms is one merged Q32 term.
  T.t.clear();
  T.t.reserve(src.size());
  for (size_t i = 0; i < src.size();) {
    QTerm acc{src[i].xmask, src[i].zmask, 0, 0};
    size_t j = i;
    for (; j < src.size() && src[j].xmask == acc.xmask && src[j].zmask == acc.zmask; ++j) {
      const SrcTerm& st = src[j];
      const double w = st.weight_kind == 0 ? s[st.weight_index] : g[st.weight_index];
      if (!std::isfinite(w)) {
        why = "non-finite weight";
        return QMC_ERR_ARG;
      }
      int64_t qre, qim;
      if (!quantize(dt, w, st.kre, scale, qre) || !quantize(dt, w, st.kim, scale, qim)) {
        why = "coefficient too large for Q32";
        return QMC_ERR_DT;
      }
      acc.qre += qre;
      acc.qim += qim;
    }
    if (acc.qre != 0 || acc.qim != 0) T.t.push_back(acc);
    i = j;
  }
  return group_table(T, why);
}

// Groups of a table's merged terms (diagonal first, then xmask ascending), their bound check and
// the Q32 sums of the diagonal and the off-diagonal groups.
int group_table(HostTable& T, std::string& why) {
  T.gx.assign(1, 0);
  T.gs.assign(1, 0);
  for (size_t i = 0; i < T.t.size(); ++i) {
    if (T.t[i].xmask == 0) continue;
    if (i == 0 || T.t[i].xmask != T.t[i - 1].xmask) {
      T.gs.push_back((uint32_t)i);
      T.gx.push_back(T.t[i].xmask);
    }
  }
  T.gs.push_back((uint32_t)T.t.size());
  if (T.gx.size() - 1 > (size_t)qmc::kMaxGroups || T.t.size() > (size_t)qmc::kMaxTerms) {
    why = "too many column groups or terms in one step table";
    return QMC_ERR_ARG;
  }
  T.q_off = T.q_diag = 0;
  for (size_t g2 = 0; g2 + 1 < T.gs.size(); ++g2) {
    uint64_t sum = 0;
    for (uint32_t i = T.gs[g2]; i < T.gs[g2 + 1]; ++i) sum += uabs(T.t[i].qre) + uabs(T.t[i].qim);
    if (sum >= (1ull << 31)) {
      why = "dt * |column group| >= 1/2: Q32 bound violated";
      return QMC_ERR_DT;
    }
    if (g2 == 0)
      T.q_diag = sum;
    else
      T.q_off += sum;
  }
  return QMC_OK;
}

size_t pack_table(const HostTable& T, uint8_t* dst) {
  // device layout: every group's terms padded with zero terms to a nonzero multiple of kTermPad
  const uint32_t G = (uint32_t)T.gx.size();
  auto padded = [&](uint32_t g) -> uint32_t {
    const uint32_t len = T.gs[g + 1] - T.gs[g];
    return len == 0 ? (uint32_t)qmc::kTermPad
                    : (len + qmc::kTermPad - 1) / qmc::kTermPad * qmc::kTermPad;
  };
  uint32_t NT = 0;
  for (uint32_t g = 0; g < G; ++g) NT += padded(g);
  qmc::TableHeader h{};
  h.n_groups = G;
  h.n_terms = NT;
  h.gx_off = (uint32_t)sizeof(qmc::TableHeader);
  h.gs_off = h.gx_off + 8 * G;
  h.t_off = (uint32_t)((h.gs_off + 4 * (G + 1) + 15) & ~15u);
  h.bytes = (uint32_t)((h.t_off + sizeof(qmc::Term) * NT + 15) & ~15u);
  h.q_off = T.q_off;
  h.q_diag = T.q_diag;
  h.active[0] = T.active[0];
  h.active[1] = T.active[1];
  if (!dst) return h.bytes;
  std::memset(dst, 0, h.bytes);
  std::memcpy(dst, &h, sizeof(h));
  std::memcpy(dst + h.gx_off, T.gx.data(), 8 * G);
  uint32_t* gs = reinterpret_cast<uint32_t*>(dst + h.gs_off);
  qmc::Term* tt = reinterpret_cast<qmc::Term*>(dst + h.t_off);
  uint32_t at = 0;
  for (uint32_t g = 0; g < G; ++g) {
    gs[g] = at;
    for (uint32_t i = T.gs[g]; i < T.gs[g + 1]; ++i) {
      qmc::Term& o = tt[at + (i - T.gs[g])];
      o.zmask = T.t[i].zmask;
      o.qre = (int32_t)T.t[i].qre;
      o.qim = (int32_t)T.t[i].qim;
    }
    at += padded(g);
  }
  gs[G] = at;
  return h.bytes;
}

void make_plan(const std::vector<SrcTerm>& src, uint32_t nh, TermPlan& P) {
  P.src = &src;
  P.nh = nh;
  P.kre.clear();
  P.kim.clear();
  P.ch.clear();
  P.run.clear();
  P.rx.clear();
  P.rz.clear();
  std::vector<uint32_t> ch;
  for (size_t i = 0; i < src.size(); ++i) {
    const SrcTerm& t = src[i];
    P.kre.push_back(t.kre);
    P.kim.push_back(t.kim);
    P.ch.push_back(t.weight_kind == 0 ? t.weight_index : nh + t.weight_index);
    if (i == 0 || t.xmask != src[i - 1].xmask || t.zmask != src[i - 1].zmask) {
      P.run.push_back((uint32_t)i);
      P.rx.push_back(t.xmask);
      P.rz.push_back(t.zmask);
    }
  }
  P.run.push_back((uint32_t)src.size());
  P.used = P.ch;
  std::sort(P.used.begin(), P.used.end());
  P.used.erase(std::unique(P.used.begin(), P.used.end()), P.used.end());
}

// build_table through the plan: the weights of the used channels checked once, every term
// quantized in one pass (the same FP64 expression; round half to even by the bit pattern of
// v + 1.5 * 2^52, exact for |v| < 2^51), run sums, then the same grouping.  A non-finite weight
// or a coefficient of 2^51 or more goes through build_table itself (the same result and error).
int build_table_plan(const TermPlan& P, double dt, const double* s, const double* g,
                     double scale, HostTable& T, std::string& why, uint32_t nh = 0,
                     uint32_t nl = 0) {
  thread_local std::vector<double> W;
  thread_local std::vector<int64_t> Q;
  const uint32_t nch = P.used.empty() ? 0u : P.used.back() + 1;
  W.resize(nch);
  bool slow = false;
  for (const uint32_t c : P.used) {
    const double w = c < P.nh ? s[c] : g[c - P.nh];
    W[c] = w;
    slow |= !std::isfinite(w);
  }
  const size_t M = P.kre.size();
  Q.resize(2 * M);
  if (!slow) {
    constexpr double kMagic = 6755399441055744.0;  // 1.5 * 2^52
    int64_t mbits;
    std::memcpy(&mbits, &kMagic, 8);
    const double* kre = P.kre.data();
    const double* kim = P.kim.data();
    const uint32_t* ch = P.ch.data();
    int64_t* q = Q.data();
    const double* w = W.data();
    uint32_t big = 0;
    for (size_t i = 0; i < M; ++i) {
      const double wi = w[ch[i]];
      const double vr = scale * (dt * (wi * kre[i])) * 4294967296.0;
      const double vi = scale * (dt * (wi * kim[i])) * 4294967296.0;
      big |= !(std::fabs(vr) < 2251799813685248.0) | !(std::fabs(vi) < 2251799813685248.0);
      const double rr = vr + kMagic, ri = vi + kMagic;
      int64_t br, bi;
      std::memcpy(&br, &rr, 8);
      std::memcpy(&bi, &ri, 8);
      q[2 * i] = br - mbits;
      q[2 * i + 1] = bi - mbits;
    }
    slow = big != 0;
  }
  if (slow) return build_table(*P.src, dt, s, g, scale, T, why, nh, nl);
  active_channels(s, g, nh, nl, T);
  T.t.clear();
  T.t.reserve(P.rx.size());
  const int64_t* q = Q.data();
  for (size_t r = 0; r + 1 < P.run.size(); ++r) {
    int64_t re = 0, im = 0;
    for (uint32_t i = P.run[r]; i < P.run[r + 1]; ++i) {
      re += q[2 * i];
      im += q[2 * i + 1];
    }
    if (re != 0 || im != 0) T.t.push_back(QTerm{P.rx[r], P.rz[r], re, im});
  }
  return group_table(T, why);
}

int check_records(uint32_t n, const uint64_t* keys, const int32_t* re, const int32_t* im,
                  uint64_t n0, std::string& why) {
  const uint64_t kmask = n >= 32 ? ~0ull : ((1ull << (2 * n)) - 1);
  for (uint64_t i = 0; i < n0; ++i) {
    if (keys[i] & ~kmask) {
      why = "key outside 2n bits";
      return QMC_ERR_ARG;
    }
    if (i && keys[i] <= keys[i - 1]) {
      why = "keys not sorted ascending and unique";
      return QMC_ERR_ARG;
    }
    if (re[i] == 0 && im[i] == 0) {
      why = "empty (0,0) record";
      return QMC_ERR_ARG;
    }
  }
  return QMC_OK;
}

int validate(const qmc_config* cfg, const qmc_model* m, std::string& why) {
  if (!cfg || !m) {
    why = "null config or model";
    return QMC_ERR_ARG;
  }
  if (cfg->n_qubits < 1 || cfg->n_qubits > 32 || cfg->n_replicas < 1 ||
      cfg->n_replicas >= (1u << 24)) {
    why = "n_qubits must be 1..32 and n_replicas 1..2^24-1";
    return QMC_ERR_ARG;
  }
  if (2 * cfg->n_qubits + replica_bits(cfg->n_replicas) > 64) {
    why = "2n + ceil(log2 R) must not exceed 64";
    return QMC_ERR_ARG;
  }
  if (!(cfg->dt > 0.0) || !std::isfinite(cfg->dt)) {
    why = "dt must be positive and finite";
    return QMC_ERR_ARG;
  }
  if (cfg->shift_mode > 1 ||
      (cfg->shift_mode == 1 && (cfg->shift_period == 0 || !std::isfinite(cfg->shift_zeta) ||
                                cfg->shift_zeta < 0.0))) {
    why = "shift_mode 0 or 1; a variable shift needs shift_period >= 1 and shift_zeta >= 0";
    return QMC_ERR_ARG;
  }
  const uint64_t qmask = cfg->n_qubits >= 32 ? 0xFFFFFFFFull : ((1ull << cfg->n_qubits) - 1);
  for (uint32_t i = 0; i < m->n_h; ++i)
    if ((m->h[i].x | m->h[i].z) & ~qmask) {
      why = "H monomial mask outside n bits";
      return QMC_ERR_ARG;
    }
  if (m->n_l && !m->l_off) {
    why = "missing l_off";
    return QMC_ERR_ARG;
  }
  for (uint32_t k = 0; k < m->n_l; ++k)
    if (m->l_off[k + 1] < m->l_off[k]) {
      why = "l_off not monotone";
      return QMC_ERR_ARG;
    }
  for (uint32_t a = 0; m->n_l && a < m->l_off[m->n_l]; ++a)
    if ((m->l[a].x | m->l[a].z) & ~qmask) {
      why = "L monomial mask outside n bits";
      return QMC_ERR_ARG;
    }
  Layout L;
  if (!compute_layout(*cfg, 1, 1, L)) {
    why = "capacities must be nonzero and R*(store+spawn) < 2^31";
    return QMC_ERR_ARG;
  }
  return QMC_OK;
}

// Upload the records of all replicas (sorted composite keys) into store buffer `b`.
int upload_store(qmc_ctx* c, uint32_t b, const std::vector<uint64_t>& ck,
                 const std::vector<int2>& cv) {
  const uint64_t n = ck.size();
  if (n > c->L.cap_store) return fail(c, QMC_ERR_STORE_CAP, "store capacity too small");
  if (n) {
    HIPCHK(c, hipMemcpyAsync(c->sk(b), ck.data(), n * 8, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->sv(b), cv.data(), n * 8, hipMemcpyHostToDevice, c->stream));
  }
  HIPCHK(c, hipMemcpyAsync(&c->counters()->n_store[b], &n, 8, hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  c->n_occ = n;
  return QMC_OK;
}

int download_store(qmc_ctx* c, std::vector<uint64_t>& ck, std::vector<int2>& cv) {
  uint64_t n = 0;
  HIPCHK(c, hipMemcpyAsync(&n, &c->counters()->n_store[c->cur], 8, hipMemcpyDeviceToHost,
                           c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  ck.resize(n);
  cv.resize(n);
  if (n) {
    HIPCHK(c, hipMemcpyAsync(ck.data(), c->sk(c->cur), n * 8, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(cv.data(), c->sv(c->cur), n * 8, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
  }
  return QMC_OK;
}

int read_counters(qmc_ctx* c, qmc::Counters& out) {
  HIPCHK(c, hipMemcpyAsync(c->pinned_small, c->counters(), sizeof(qmc::Counters),
                           hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  std::memcpy(&out, c->pinned_small, sizeof(out));
  c->last_hc = out;
  return QMC_OK;
}

// The counters as the last finishing kernel of the LDS-resident step left them in pinned memory.
int read_mirror(qmc_ctx* c, qmc::Counters& out) {
  HIPCHK(c, hipStreamSynchronize(c->stream));
  std::memcpy(&out, c->pinned_small + c->pin_mirror, sizeof(out));
  c->last_hc = out;
  return QMC_OK;
}

int upload_qshift(qmc_ctx* c, const std::vector<int64_t>& qs) {
  if (qs == c->qshift_dev) return QMC_OK;  // the device already holds these shifts
  c->qshift_dev.clear();
  std::memcpy(c->pinned_small, qs.data(), qs.size() * 8);
  HIPCHK(c, hipMemcpyAsync(c->at<int64_t>(c->L.qshift), c->pinned_small, qs.size() * 8,
                           hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  c->qshift_dev = qs;
  return QMC_OK;
}

// Per-replica Q32 shifts for a table with the integrator's factor `scale`.
int shifts_q32(const qmc_ctx* c, double scale, std::vector<int64_t>& qs) {
  qs.resize(c->R);
  for (uint32_t r = 0; r < c->R; ++r)
    if (!quantize(c->cfg.dt, 1.0, c->shift[r], scale, qs[r])) return QMC_ERR_DT;
  return QMC_OK;
}

}  // namespace

extern "C" {

namespace {

// The configuration of the store: n_replicas counts segments (circuits x replicas per circuit).
qmc_config segment_config(const qmc_config* cfg, uint32_t n_circuits) {
  qmc_config s = *cfg;
  s.n_replicas = cfg->n_replicas * n_circuits;
  return s;
}

int validate_batch(const qmc_config* cfg, uint32_t n_circuits, const qmc_model* models,
                   std::string& why) {
  if (!cfg || !models || n_circuits < 1 || n_circuits > (uint32_t)qmc::kMaxCircuits) {
    why = "1..512 circuits with a model each";
    return QMC_ERR_ARG;
  }
  if ((uint64_t)cfg->n_replicas * n_circuits >= (1u << 24)) {
    why = "circuits x replicas must stay below 2^24";
    return QMC_ERR_ARG;
  }
  const qmc_config s = segment_config(cfg, n_circuits);
  for (uint32_t ci = 0; ci < n_circuits; ++ci) {
    int rc = validate(&s, &models[ci], why);
    if (rc) {
      why = "circuit " + std::to_string(ci) + ": " + why;
      return rc;
    }
  }
  return QMC_OK;
}

}  // namespace

int qmc_workspace_bytes_batch(const qmc_config* cfg, uint32_t n_circuits,
                              const qmc_model* models, size_t* bytes) {
  std::string why;
  int rc = validate_batch(cfg, n_circuits, models, why);
  if (rc) return rc;
  uint32_t P = 0;
  rc = persist_segments(&P);
  if (rc) return rc;
  Layout L;
  compute_layout(segment_config(cfg, n_circuits), P, n_circuits, L);
  if (bytes) *bytes = L.total;
  return QMC_OK;
}

int qmc_workspace_bytes(const qmc_config* cfg, const qmc_model* model, size_t* bytes) {
  return qmc_workspace_bytes_batch(cfg, 1, model, bytes);
}

int qmc_init_batch(const qmc_config* cfg, uint32_t n_circuits, const qmc_model* models,
                   const uint64_t* const* keys, const int32_t* const* re,
                   const int32_t* const* im, const uint64_t* n0, void* d_workspace,
                   size_t ws_bytes, void* hip_stream, qmc_ctx** out) {
  if (!out) return QMC_ERR_ARG;
  *out = nullptr;
  std::string why;
  int rc = validate_batch(cfg, n_circuits, models, why);
  if (rc) return rc;
  if (!keys || !re || !im || !n0) return QMC_ERR_ARG;
  for (uint32_t ci = 0; ci < n_circuits; ++ci) {
    rc = check_records(cfg->n_qubits, keys[ci], re[ci], im[ci], n0[ci], why);
    if (rc) return rc;
    if (n0[ci] > cfg->store_capacity) return QMC_ERR_ARG;
  }
  uint32_t P = 0;
  if (persist_segments(&P)) return QMC_ERR_HIP;
  if (n_circuits > P) return QMC_ERR_ARG;  // every circuit needs a key range of its own
  qmc_ctx* c = new qmc_ctx();
  c->cfg = segment_config(cfg, n_circuits);
  c->n = cfg->n_qubits;
  c->C = n_circuits;
  c->Rc = cfg->n_replicas;
  c->R = c->C * c->Rc;
  c->kbits = 2 * c->n;
  c->rbits = replica_bits(c->R);
  c->n_h = c->n_l = 0;
  c->terms.resize(c->C);
  for (uint32_t ci = 0; ci < c->C; ++ci) {
    c->wh_off.push_back(c->n_h);
    c->wl_off.push_back(c->n_l);
    c->n_h += models[ci].n_h;
    c->n_l += models[ci].n_l;
    compile_model(models[ci], c->n, c->terms[ci]);
  }
  c->plans.resize(c->C);
  for (uint32_t ci = 0; ci < c->C; ++ci) make_plan(c->terms[ci], models[ci].n_h, c->plans[ci]);
  compute_layout(c->cfg, P, c->C, c->L);
  if (!d_workspace || ws_bytes < c->L.total || ((uintptr_t)d_workspace & 255)) {
    delete c;
    return QMC_ERR_ARG;
  }
  c->ws = (uint8_t*)d_workspace;
  c->stream = (hipStream_t)hip_stream;
  c->shift.assign(c->R, 0.0);
  c->shift_on.assign(c->R, 0);
  c->shift_ref.assign(c->R, 0);
  c->nd0_re.assign(c->R, 0);
  for (uint32_t ci = 0; ci < c->C; ++ci) {
    int64_t nd = 0;
    for (uint64_t i = 0; i < n0[ci]; ++i) {
      const uint64_t kk = keys[ci][i];
      const uint64_t ket = kk & ((c->n >= 32) ? 0xFFFFFFFFull : ((1ull << c->n) - 1));
      const uint64_t bra = c->n >= 32 ? kk >> 32 : kk >> c->n;
      if (ket == bra) nd += re[ci][i];
    }
    for (uint32_t r = 0; r < c->Rc; ++r) c->nd0_re[(size_t)ci * c->Rc + r] = nd;
  }
  hipError_t e = hipHostMalloc((void**)&c->pinned,
                               kTableArea + (size_t)kMaxChunkSteps * 4 * (c->C + 1),
                               hipHostMallocDefault);
  c->pinned_small_bytes = std::max<size_t>(1 << 16, (size_t)c->R * kMaxLookup * 16 + 4096);
  c->pinned_small_bytes = std::max<size_t>(c->pinned_small_bytes, (size_t)c->C * 16 + 4096);
  c->pin_mirror = align256(c->pinned_small_bytes);
  c->pin_head = c->pin_mirror + kPinMirror;
  if (e == hipSuccess)
    e = hipHostMalloc((void**)&c->pinned_small,
                      c->pin_head + align256((size_t)kHeadMax * c->C * 4), hipHostMallocDefault);
  if (e == hipSuccess) e = hipHostGetDevicePointer((void**)&c->pinned_dev, c->pinned, 0);
  if (e == hipSuccess)
    e = hipHostGetDevicePointer((void**)&c->pinned_small_dev, c->pinned_small, 0);
  if (e != hipSuccess) {
    qmc_destroy(c);
    return QMC_ERR_HIP;
  }
  // zero counters, then the initial store (segment tag in the high bits)
  e = hipMemsetAsync(c->counters(), 0, sizeof(qmc::Counters), c->stream);
  if (e == hipSuccess)
    e = hipMemsetAsync(c->at<uint64_t>(c->L.slots), 0, (size_t)2 * c->L.P * 4 * 8, c->stream);
  if (e == hipSuccess)  // the LDS-resident step's stop word: no epoch yet
    e = hipMemsetAsync(c->at<uint64_t>(c->L.small_fail), 0, 8, c->stream);
  // One copy each way between the pinned staging and the table area, of a size the runtime
  // hands to its DMA engines: their first use in a process costs several milliseconds, which
  // belongs to set-up rather than to the first qmc_step that uploads a window of tables.
  constexpr size_t kWarmCopy = 1u << 20;
  if (e == hipSuccess)
    e = hipMemcpyAsync(c->at<uint8_t>(c->L.tab), c->pinned, kWarmCopy, hipMemcpyHostToDevice,
                       c->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(c->pinned, c->at<uint8_t>(c->L.tab), kWarmCopy, hipMemcpyDeviceToHost,
                       c->stream);
  if (e == hipSuccess) e = (hipError_t)qmcp_warm(c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) {
    qmc_destroy(c);
    return QMC_ERR_HIP;
  }
  std::vector<uint64_t> ck;
  std::vector<int2> cv;
  for (uint32_t ci = 0; ci < c->C; ++ci)
    for (uint32_t r = 0; r < c->Rc; ++r) {
      const uint64_t seg = (uint64_t)ci * c->Rc + r;
      for (uint64_t i = 0; i < n0[ci]; ++i) {
        ck.push_back((c->kbits >= 64 ? 0 : (seg << c->kbits)) | keys[ci][i]);
        cv.push_back(make_int2(re[ci][i], im[ci][i]));
      }
    }
  c->cur = 0;
  rc = upload_store(c, 0, ck, cv);
  if (!rc) {
    std::vector<int64_t> qs(2 * (size_t)c->R, 0);
    rc = upload_qshift(c, qs);
  }
  if (rc) {
    qmc_destroy(c);
    return rc;
  }
  *out = c;
  return QMC_OK;
}

int qmc_init(const qmc_config* cfg, const qmc_model* model, const uint64_t* keys,
             const int32_t* re, const int32_t* im, uint64_t n0, void* d_workspace,
             size_t ws_bytes, void* hip_stream, qmc_ctx** out) {
  return qmc_init_batch(cfg, 1, model, &keys, &re, &im, &n0, d_workspace, ws_bytes, hip_stream,
                        out);
}

namespace {

// Adds the running-sum deltas between two counter reads to a kernel class's coverage.
void add_cover(qmc_ctx* c, int cls, const qmc::Counters& a, const qmc::Counters& b,
               uint32_t steps) {
  qmc_stats& v = c->prof_cover[cls];
  v.step += steps;
  v.walker_steps += b.walker_steps - a.walker_steps;
  v.key_steps += b.key_steps - a.key_steps;
  v.child_steps += b.child_steps - a.child_steps;
  v.out_steps += b.out_steps - a.out_steps;
  v.spawn_steps += (b.child_steps - b.death_steps) - (a.child_steps - a.death_steps);
  v.rebalances += b.resplits - a.resplits;
}

// Two events for a deferred whole-launch timing.
int timing_pair(qmc_ctx* c, hipEvent_t& a, hipEvent_t& b) {
  while (c->ev_free.size() < 2) {
    hipEvent_t ev;
    HIPCHK(c, hipEventCreate(&ev));
    c->ev_free.push_back(ev);
  }
  a = c->ev_free.back();
  c->ev_free.pop_back();
  b = c->ev_free.back();
  c->ev_free.pop_back();
  return QMC_OK;
}

// The pending timings into the class totals (the events completed: every step call ends with a
// stream synchronization).
int settle_timings(qmc_ctx* c) {
  for (const qmc_ctx::PendingTime& t : c->ev_pending) {
    float ms = 0.f;
    HIPCHK(c, hipEventElapsedTime(&ms, t.a, t.b));
    c->prof_ms[t.cls] += ms;
    c->prof_launches[t.cls] += t.launches;
    c->ev_free.push_back(t.a);
    c->ev_free.push_back(t.b);
  }
  c->ev_pending.clear();
  return QMC_OK;
}

// Records a timing to be read later; many of them are settled at once.
void defer_timing(qmc_ctx* c, int cls, hipEvent_t a, hipEvent_t b, uint64_t launches) {
  c->ev_pending.push_back(qmc_ctx::PendingTime{cls, a, b, launches});
  if (c->ev_pending.size() >= 256) (void)settle_timings(c);
}

constexpr uint64_t kFusedKeysPerSegment = 8192;  // automatic mode: larger stores run streamed
constexpr uint32_t kStreamedWindow = 256;         // steps run streamed after a fused overflow
constexpr uint32_t kKernelResplits = 64;          // re-splits the fused kernel does by itself

// One chunk of steps [step, step + nst): device tables at dtab (+ offsA / offsB), and whether
// the chunk integrates with AB2 from a known N(s-1) (`two`; the tables B exist).
struct Chunk {
  uint8_t* dtab;                 // the device table area
  uint32_t first;                // index of the chunk's first step in the device offset arrays
  uint32_t nst;
  bool two;
};

// Steps of the chunk as one launch of the fused persistent kernel.  On return kd = completed
// steps, reason = the kernel's stop reason (0 end, 1 rebalance, 2 error), hc = the counters; the
// store (and N(s-1) for AB2) and c->step reflect kd.
int run_fused(qmc_ctx* c, const Chunk& ch, uint32_t& kd, uint32_t& reason, qmc::Counters& hc) {
  const qmc::Counters before = c->last_hc;
  // the kernel's done flags go to pinned memory past the counters, which read_counters copies
  // to the start of the same buffer
  constexpr size_t kPinDone = (sizeof(qmc::Counters) + 255) / 256 * 256;
  static_assert(kPinDone >= sizeof(qmc::Counters) && kPinDone + 8 <= (1u << 16),
                "done flags must not overlap the counters in the pinned staging buffer");
  uint32_t* pin_done = reinterpret_cast<uint32_t*>(c->pinned_small + kPinDone);
  const uint32_t nst = ch.nst;
  PersistLaunch pl;
  pl.ck = c->sk(0);
  pl.cv = c->sv(0);
  pl.pk_prev = ch.two ? c->pk() : nullptr;
  pl.pv_prev = ch.two ? c->pv() : nullptr;
  pl.counters = c->counters();
  pl.cur = c->cur;
  pl.sk = c->at<uint64_t>(c->L.seg_k);
  pl.sv = c->at<int2>(c->L.seg_v);
  pl.segcap = c->L.segcap;
  pl.seg_n = c->at<uint32_t>(c->L.seg_n);
  pl.nbuf = c->integrator == 1 ? 3u : 2u;
  pl.ik = c->at<uint64_t>(c->L.in_k);
  pl.iv = c->at<int2>(c->L.in_v);
  pl.incap = c->L.incap;
  pl.in_n = c->at<uint32_t>(c->L.in_n);
  pl.split = c->at<uint64_t>(c->L.split);
  pl.split_w = c->at<uint64_t>(c->L.split);
  pl.P = c->L.P;
  pl.tab_base = ch.dtab;
  pl.tab_off = c->at<uint32_t>(c->L.tab_off) + (size_t)ch.first * c->C;
  pl.tabB_off = ch.two ? c->at<uint32_t>(c->L.tabB_off) + ch.first : nullptr;
  pl.n_circuits = c->C;
  pl.rep_per = c->Rc;
  pl.step0 = c->step;
  pl.nsteps = nst;
  pl.seed = c->cfg.seed;
  pl.kbits = c->kbits;
  pl.init_min = c->init_min;
  pl.n_replicas = c->R;
  pl.qshift = c->at<int64_t>(c->L.qshift);
  pl.qshiftB = c->at<int64_t>(c->L.qshift) + c->R;
  pl.slots = c->at<uint64_t>(c->L.slots);
  pl.max_rebal = c->C == 1 ? kKernelResplits : 0u;
  pl.epoch0 = c->epoch + 1;
  // barriers of this launch: batch start, one per step, three per re-split
  c->epoch += (uint64_t)nst + 1 + 3ull * pl.max_rebal;
  pl.cap_store = c->L.cap_store;
  pl.cap_inbox = c->L.cap_child;
  pl.rebal_min = 64;
  pl.done = c->at<uint32_t>(c->L.done);
  const bool prof = c->prof_whole();
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  if (prof) {
    int rc = timing_pair(c, ev0, ev1);
    if (rc) return rc;
  }
  HIPCHK(c, qmcp_prepare(c->stream, &pl));
  if (prof) HIPCHK(c, hipEventRecord(ev0, c->stream));
  HIPCHK(c, qmcp_launch(c->stream, &pl));
  if (prof) HIPCHK(c, hipEventRecord(ev1, c->stream));
  HIPCHK(c, hipMemcpyAsync(pin_done, pl.done, 8, hipMemcpyDeviceToHost, c->stream));
  int rc = read_counters(c, hc);  // synchronizes the stream
  if (rc) return rc;
  if (prof) defer_timing(c, 3, ev0, ev1, 1);
  kd = pin_done[0];
  reason = pin_done[1];
  if (reason == 1) {
    c->relaunches += 1;
    if (prof) c->prof_cover[3].rebalances += 1;
  }
  bool sized = true;  // the kernel wrote the sizes of the stores gathered below
  if (reason == 2 || hc.err) {
    sized = false;
    const uint32_t es = hc.err_step;
    if (es < pl.step0 || es > pl.step0 + pl.nsteps) {
      c->broken = true;
      return fail(c, QMC_ERR_HIP, "device error flag without a valid step");
    }
    kd = es - pl.step0;
  }
  // N(step0 + j) is in segment buffer j mod nbuf; kd = 0 leaves the stores untouched.
  if (kd > 0) {
    qmc::Counters* dcnt = c->counters();
    if (c->integrator == 1)
      HIPCHK(c, qmcp_gather(c->stream, &pl, (kd - 1) % pl.nbuf, c->pk(), c->pv(),
                            &dcnt->n_prev));
    HIPCHK(c, qmcp_gather(c->stream, &pl, kd % pl.nbuf, c->sk(0), c->sv(0),
                          &dcnt->n_store[c->cur]));
    if (!sized) {
      rc = read_counters(c, hc);
      if (rc) return rc;
    }
  }
  c->step = pl.step0 + kd;
  c->n_occ = hc.n_store[c->cur];
  if (prof) add_cover(c, 3, before, hc, kd);
  return QMC_OK;
}

// The first batch of a small chain, launched while the rest of the call's tables are still being
// built (the host's table build overlaps the batch): steps [0, steps) of the first chunk, chain
// epoch `epoch`, the profiling events around it (or null).
struct SmallHead {
  uint32_t steps = 0;
  uint32_t epoch = 0;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
};

// The launch fields of the LDS-resident step that stay the same over a chain; its step tables
// are read from the pinned staging area (dtab, device address).
void small_setup(qmc_ctx* c, const uint8_t* dtab, SmallLaunch& sl) {
  sl = SmallLaunch{};
  sl.counters = c->counters();
  sl.cur = c->cur;
  sl.segcap = c->L.segcap;
  sl.tab_base = dtab;
  sl.n_circuits = c->C;
  sl.rep_per = c->Rc;
  sl.n_segments = c->R;
  sl.seed = c->cfg.seed;
  sl.kbits = c->kbits;
  sl.init_min = c->init_min;
  sl.qshift = c->at<int64_t>(c->L.qshift);
  sl.cap_store = std::min<uint64_t>(c->cfg.store_capacity,
                                    c->path == 3 ? (uint64_t)kSmallCap : c->small_limit);
  sl.cap_spawn = c->cfg.spawn_capacity;
  sl.stop = c->at<unsigned long long>(c->L.small_fail);
}

// Batch j of a chain: steps [first, first + steps) of the chunk whose first table is entry
// tfirst of the offsets and whose first step is step0, from the canonical store (j = 0) or from
// segment buffer (j - 1) & 1, into segment buffer j & 1, statistics into row block j.  The
// table offsets are the window's in pinned staging, or those at head_off (device address, the
// batch's own steps from its first) when given.
int small_batch(qmc_ctx* c, SmallLaunch& sl, uint32_t tfirst, uint32_t step0, uint32_t j,
                uint32_t first, uint32_t steps, const uint32_t* head_off = nullptr) {
  const uint64_t segcap = c->L.segcap, P = c->L.P;
  uint64_t* seg_k = c->at<uint64_t>(c->L.seg_k);
  int2* seg_v = c->at<int2>(c->L.seg_v);
  uint32_t* seg_n = c->at<uint32_t>(c->L.seg_n);
  const uint32_t ib = (j + 1) & 1, ob = j & 1;
  sl.ck = j == 0 ? c->sk(0) : nullptr;
  sl.cv = j == 0 ? c->sv(0) : nullptr;
  sl.ik = seg_k + ib * P * segcap;
  sl.iv = seg_v + ib * P * segcap;
  sl.in_n = seg_n + ib * P;
  sl.ok = seg_k + ob * P * segcap;
  sl.ov = seg_v + ob * P * segcap;
  sl.out_n = seg_n + ob * P;
  // the window's table offsets, staged in pinned memory right after the table staging area
  sl.tab_off = head_off ? head_off
                       : reinterpret_cast<const uint32_t*>(c->pinned_dev + kTableArea) +
                             (size_t)(tfirst + first) * c->C;
  sl.step0 = step0 + first;
  sl.nsteps = steps;
  sl.stats = c->at<uint64_t>(c->L.small_stats) + (size_t)j * c->R * kSmallStats;
  return qmcs_launch(c->stream, &sl);
}

// Steps of the chunk with the LDS-resident step, one workgroup per store segment (Euler, the
// comb).  A segment that outgrows what the step holds stops the launch at the first such step F;
// the steps before F are then run again from the unchanged canonical store (the results are the
// same) and the automatic mode leaves the small step for this trajectory.  On return kd =
// completed steps (0 if not even the first step fits) and the store reflects them.  A head batch
// (head->steps > 0) is the chain's first batch, already launched.
int run_small(qmc_ctx* c, const Chunk& ch, uint32_t& kd, qmc::Counters& hc,
              const SmallHead* head) {
  const qmc::Counters before = c->last_hc;
  const uint32_t step0 = c->step, nst = ch.nst;
  const uint64_t segcap = c->L.segcap, P = c->L.P;
  uint64_t* seg_k = c->at<uint64_t>(c->L.seg_k);
  int2* seg_v = c->at<int2>(c->L.seg_v);
  uint32_t* seg_n = c->at<uint32_t>(c->L.seg_n);
  unsigned long long* dstop = c->at<unsigned long long>(c->L.small_fail);
  uint64_t* dstats = c->at<uint64_t>(c->L.small_stats);
  const uint64_t rows = (uint64_t)c->R;  // statistics rows of one batch
  qmc::Counters* dcnt = c->counters();
  SmallLaunch sl;
  small_setup(c, c->pinned_dev, sl);
  auto batch = [&](uint32_t j, uint32_t first, uint32_t steps) {
    return small_batch(c, sl, ch.first, step0, j, first, steps);
  };
  // the segments batch jd - 1 wrote into the canonical store and the statistics of batches
  // [0, jd) into the counters; gated on the stop word of `epoch` when stop is given
  // With few segments one workgroup does it all and leaves a copy of the counters in pinned
  // memory (read_mirror), so the call's end needs no copy on the stream.
  const bool one = c->R <= kFinishOne;
  auto finish = [&](uint32_t jd, const unsigned long long* stop, uint32_t epoch) -> int {
    const uint32_t ob = (jd - 1) & 1;
    HIPCHK(c, qmcs_finish(c->stream, seg_k + ob * P * segcap, seg_v + ob * P * segcap,
                          seg_n + ob * P, segcap, c->R, c->sk(0), c->sv(0),
                          &dcnt->n_store[c->cur], dcnt, dstats, (uint32_t)(jd * rows), stop,
                          epoch, one ? 1u : c->R,
                          one ? c->pinned_small_dev + c->pin_mirror : nullptr));
    return 0;
  };
  auto counters_after_finish = [&](qmc::Counters& out) -> int {
    return one ? read_mirror(c, out) : read_counters(c, out);
  };
  const bool prof = c->prof_whole();
  // One chain over steps [first, first + steps) with its gated gather and commit, then one
  // synchronization (with the counters); jd = the batches whose results are committed, done =
  // their steps, stop = the first step not taken, or ~0.  With hd, its batch is the chain's
  // first, already launched.
  auto run_chain = [&](uint32_t first, uint32_t steps, uint32_t& jd, uint32_t& done,
                       uint32_t& stop, const SmallHead* hd) -> int {
    std::vector<uint32_t> bnd(1, 0);  // batch boundaries, relative to `first`
    if (hd) bnd.push_back(std::min(hd->steps, steps));
    while (bnd.back() < steps) bnd.push_back(std::min(bnd.back() + kSmallBatch, steps));
    const uint32_t nb = (uint32_t)bnd.size() - 1;
    const uint32_t epoch = hd ? hd->epoch : ++c->small_epoch;
    const uint32_t j0 = hd ? 1u : 0u;  // the first batch launched here
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    if (prof && j0 < nb) {
      int rc = timing_pair(c, ev0, ev1);
      if (rc) return rc;
      HIPCHK(c, hipEventRecord(ev0, c->stream));
    }
    sl.epoch = epoch;
    for (uint32_t j = j0; j < nb; ++j) HIPCHK(c, batch(j, first + bnd[j], bnd[j + 1] - bnd[j]));
    if (ev1) HIPCHK(c, hipEventRecord(ev1, c->stream));
    int rc = finish(nb, dstop, epoch);  // also copies the stop word into the counters
    if (rc) return rc;
    rc = counters_after_finish(hc);  // synchronizes the stream
    if (rc) return rc;
    // the head batch and the rest are timed apart: the GPU may wait for the host between them
    if (hd && hd->ev0) defer_timing(c, 4, hd->ev0, hd->ev1, 1);
    if (ev0) defer_timing(c, 4, ev0, ev1, nb - j0);
    const uint64_t w = hc.small_stop;
    if ((uint32_t)(w >> 32) != epoch) {
      jd = nb;
      done = steps;
      stop = 0xFFFFFFFFu;
      return 0;
    }
    stop = 0xFFFFFFFFu - (uint32_t)w;
    const uint32_t s0 = step0 + first;
    if (stop < s0 || stop >= s0 + steps) {
      c->broken = true;
      return fail(c, QMC_ERR_HIP, "small step: stop outside the chain");
    }
    jd = 0;  // complete batches, not committed yet
    while (jd < nb && bnd[jd + 1] <= stop - s0) ++jd;
    done = bnd[jd];
    if (jd > 0) {
      rc = finish(jd, nullptr, 0);
      if (rc) return rc;
    }
    return 0;
  };
  kd = 0;
  uint32_t jd = 0, stop = 0;
  int rc = run_chain(0, nst, jd, kd, stop, head && head->steps ? head : nullptr);
  if (rc) return rc;
  if (stop != 0xFFFFFFFFu) {
    c->small_off = true;
    const uint32_t rest = stop - step0 - kd;  // steps of the stopped batch that every replica took
    if (rest > 0) {
      uint32_t jd2 = 0, done2 = 0, stop2 = 0;
      rc = run_chain(kd, rest, jd2, done2, stop2, nullptr);
      if (rc) return rc;
      if (stop2 != 0xFFFFFFFFu) {
        c->broken = true;
        return fail(c, QMC_ERR_HIP, "small step: inconsistent stop");
      }
      kd += rest;
    } else if (jd > 0) {
      rc = counters_after_finish(hc);  // the committed batches
      if (rc) return rc;
    }
  }
  if (kd == 0) return QMC_OK;  // not even the first step fits: nothing ran
  c->step = step0 + kd;
  c->n_occ = hc.n_store[c->cur];
  if (prof) add_cover(c, 4, before, hc, kd);
  return QMC_OK;
}

// Steps of the chunk as separate kernels per step: spawn (first step only, plus the second AB2
// term from N(s-1)), LSD radix sort of the children, and the merge, which also spawns the next
// step's children (both AB2 terms).  The store cycles through the canonical buffer and one (two
// for AB2) buffers of the segment area and ends in the canonical buffer; N(s-1) ends in its
// buffer.
int run_streamed(qmc_ctx* c, const Chunk& ch, uint32_t& kd, qmc::Counters& hc) {
  qmc::Counters* dcnt = c->counters();
  const qmc::Counters before = c->last_hc;
  const uint32_t nst = ch.nst;
  const uint32_t passes = qmck_sort_passes(c->kbits + c->rbits + (c->init_min ? 1u : 0u));
  const uint32_t step0 = c->step, cur0 = c->cur;
  const uint32_t nb = c->integrator == 1 ? 3u : 2u;
  uint64_t* bk[3] = {c->sk(0), c->alt_k(0), c->alt_k(1)};
  int2* bv[3] = {c->sv(0), c->alt_v(0), c->alt_v(1)};
  const int64_t* qshA = c->at<int64_t>(c->L.qshift);
  const int64_t* qshB = qshA + c->R;
  const uint8_t* dtab = ch.dtab;
  // Class 5 (the whole streamed step) is one interval per chunk, from before its first draws to
  // after its last merge, and times the merge class (2) beside it.
  const bool prof_step = c->prof_class == 5;
  const int32_t prof_k = prof_step ? 2 : c->prof_class;  // the class with per-step events
  const uint32_t nev = 2 * nst;
  hipEvent_t sev0 = nullptr, sev1 = nullptr;
  if (prof_step) {
    int rc = timing_pair(c, sev0, sev1);
    if (rc) return rc;
  }
  if (prof_k >= 0 && prof_k <= 2) {
    while (c->prof_ev.size() < nev) {
      hipEvent_t ev;
      HIPCHK(c, hipEventCreate(&ev));
      c->prof_ev.push_back(ev);
    }
  }
  // Every launch of the chunk, in stream order; with graphs on they are captured instead.
  auto enqueue = [&](hipStream_t st_q) -> hipError_t {
#define ENQ(x)                                   \
  do {                                           \
    const hipError_t e_ = (hipError_t)(x);       \
    if (e_ != hipSuccess) return e_;             \
  } while (0)
    // The merge class's tile counts and count adjustments start from zero (the adjustments are
    // left zero by every completed step, not by one an error stopped).  The step sort uses no
    // look-back words; the whole-store sort after a pulse clears its own.
    if (prof_step) ENQ(hipEventRecord(sev0, st_q));
    ENQ(qmck_batch_begin(st_q, dcnt, c->at<uint64_t>(c->L.status), c->L.status_words, nullptr,
                         0, c->ghist(0), 2 * qmc::kMaxPasses * qmc::kRadixBins));
    auto mark = [&](int32_t cls, uint32_t k, int which) -> hipError_t {
      if (prof_k != cls) return hipSuccess;
      return hipEventRecord(c->prof_ev[2 * k + which], st_q);
    };
    // the search index of the first step's parents (each merge writes the next one's)
    uint64_t* sidx = c->at<uint64_t>(c->L.sidx);
    ENQ(qmck_store_index(st_q, bk[0], &dcnt->n_store[cur0], sidx, c->L.cap_store));
    uint32_t cb = 0;  // child buffer pair holding the unsorted children of the current step
    ENQ(mark(0, 0, 0));
    // device table offsets of step k of the chunk: [circuit] (A), and the AB2 B term
    const uint32_t* dA = c->at<uint32_t>(c->L.tab_off) + (size_t)ch.first * c->C;
    const uint32_t* dB = c->at<uint32_t>(c->L.tabB_off) + ch.first;
    ENQ(qmck_spawn(st_q, bk[0], bv[0], dcnt, &dcnt->n_store[cur0], dtab, dA, c->Rc,
                         step0, c->cfg.seed, c->kbits, c->init_min, 0u, qshA, c->ck(cb), c->cv(cb),
                         c->L.cap_child, c->L.cap_store, c->ghist(step0 & 1), passes, &c->prop));
    if (ch.two)
      ENQ(qmck_spawn(st_q, c->pk(), c->pv(), dcnt, &dcnt->n_prev, dtab, dB, c->Rc,
                           step0, c->cfg.seed, c->kbits, c->init_min, 1u, qshB, c->ck(cb),
                           c->cv(cb),
                           c->L.cap_child, c->L.cap_store, c->ghist(step0 & 1), passes, nullptr));
    ENQ(mark(0, 0, 1));
    for (uint32_t k = 0; k < nst; ++k) {
      const uint32_t st = step0 + k, b = k % nb, cur = cur0 ^ (k & 1u);
      const bool more = k + 1 < nst;
      const uint32_t* toff_next = more ? dA + (size_t)(k + 1) * c->C : nullptr;
      const uint32_t* toffB_next = more && c->integrator == 1 ? dB + (k + 1) : nullptr;
      const uint32_t csel = st & 1;
      ENQ(mark(1, k, 0));
      ENQ(qmck_sort_step(st_q, c->ck(0), c->cv(0), c->ck(1), c->cv(1), dcnt, csel, passes,
                         c->ghist(csel), c->thist(0), c->thist(1), st, cb, c->L.cap_child));
      ENQ(mark(1, k, 1));
      const uint32_t cf = cb ^ (passes & 1);  // sorted children
      // With the Euler step and the comb, the merge also queues the records of N(st + 1) whose
      // combs can fire in step st + 1 (in the store buffer AB2 would use), and step st + 1 is
      // drawn from them alone; otherwise it is drawn from the whole of N(st + 1).
      const bool queue = more && nb == 2 && c->prop.kind == 0;
      ENQ(mark(2, k, 0));
      ENQ(qmck_merge(st_q, bk[b], bv[b], c->ck(cf), c->cv(cf), dcnt, cur, csel,
                     c->at<uint2>(c->L.splits), c->at<uint64_t>(c->L.status), st, c->kbits,
                     c->init_min, bk[(k + 1) % nb], bv[(k + 1) % nb], c->L.cap_store,
                     c->L.cap_store + c->L.cap_child, c->ghist(csel ^ 1), dtab,
                     queue ? toff_next : nullptr, c->Rc, qshA, c->cfg.seed, c->alt_k(1),
                     c->alt_v(1), c->at<uint32_t>(c->L.mpos), sidx));
      ENQ(mark(2, k, 1));
      cb = cf ^ 1;
      if (more) {
        // the records of step st + 1 into the other child buffers: from N(st + 1) (or its queued
        // records), and with AB2 the second term from N(st), this step's parents
        ENQ(mark(0, k + 1, 0));
        if (queue)
          ENQ(qmck_spawn(st_q, c->alt_k(1), c->alt_v(1), dcnt, &dcnt->n_active, dtab, toff_next,
                         c->Rc, st + 1, c->cfg.seed, c->kbits, c->init_min, 0u, qshA, c->ck(cb),
                         c->cv(cb), c->L.cap_child, c->L.cap_store, c->ghist(csel ^ 1), passes,
                         &c->prop));
        else
          ENQ(qmck_spawn(st_q, bk[(k + 1) % nb], bv[(k + 1) % nb], dcnt,
                         &dcnt->n_store[cur ^ 1u], dtab, toff_next, c->Rc, st + 1, c->cfg.seed,
                         c->kbits, c->init_min, 0u, qshA, c->ck(cb), c->cv(cb), c->L.cap_child,
                         c->L.cap_store, c->ghist(csel ^ 1), passes, &c->prop));
        if (toffB_next)
          ENQ(qmck_spawn(st_q, bk[b], bv[b], dcnt, &dcnt->n_store[cur], dtab, toffB_next, c->Rc,
                         st + 1, c->cfg.seed, c->kbits, c->init_min, 1u, qshB, c->ck(cb),
                         c->cv(cb), c->L.cap_child, c->L.cap_store, c->ghist(csel ^ 1), passes,
                         nullptr));
        ENQ(mark(0, k + 1, 1));
      }
    }
    if (prof_step) ENQ(hipEventRecord(sev1, st_q));
#undef ENQ
    return hipSuccess;
  };
  const bool graph = c->use_graph && c->prof_class < 0;
  if (!graph) {
    HIPCHK(c, enqueue(c->stream));
  } else {
    // Capture the chunk on a stream of its own (the context's stream may be the null stream,
    // which cannot be captured), update the executable graph of the previous chunk with it (same
    // launches, new arguments) or instantiate a new one, and launch it on the context's stream.
    if (!c->gstream) HIPCHK(c, hipStreamCreateWithFlags(&c->gstream, hipStreamNonBlocking));
    HIPCHK(c, hipStreamBeginCapture(c->gstream, hipStreamCaptureModeRelaxed));
    const hipError_t eq = enqueue(c->gstream);
    hipGraph_t g = nullptr;
    const hipError_t ec = hipStreamEndCapture(c->gstream, &g);
    if (eq != hipSuccess || ec != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      c->broken = true;
      return fail(c, QMC_ERR_HIP, std::string("graph capture: ") +
                                      hipGetErrorString(eq != hipSuccess ? eq : ec));
    }
    if (c->gexec) {
      hipGraphNode_t bad = nullptr;
      hipGraphExecUpdateResult res;
      if (hipGraphExecUpdate(c->gexec, g, &bad, &res) != hipSuccess ||
          res != hipGraphExecUpdateSuccess) {
        (void)hipGetLastError();
        (void)hipGraphExecDestroy(c->gexec);
        c->gexec = nullptr;
      }
    }
    hipError_t el = hipSuccess;
    if (!c->gexec) el = hipGraphInstantiate(&c->gexec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (el == hipSuccess) el = hipGraphLaunch(c->gexec, c->stream);
    if (el != hipSuccess) {
      c->broken = true;
      return fail(c, QMC_ERR_HIP, std::string("graph launch: ") + hipGetErrorString(el));
    }
  }
  int rc = read_counters(c, hc);
  if (rc) return rc;
  if (prof_k >= 0 && prof_k <= 2) {
    for (uint32_t k = 0; k < nst; ++k) {
      float ms = 0.f;
      HIPCHK(c, hipEventElapsedTime(&ms, c->prof_ev[2 * k], c->prof_ev[2 * k + 1]));
      c->prof_ms[prof_k] += ms;
      c->prof_launches[prof_k] += 1;
    }
  }
  if (prof_step) defer_timing(c, 5, sev0, sev1, 1);
  kd = nst;
  if (hc.err) {
    const uint32_t es = hc.err_step;
    if (es < step0 || es >= step0 + nst) {
      c->broken = true;
      return fail(c, QMC_ERR_HIP, "device error flag without a valid step");
    }
    kd = es - step0;
  }
  // N(step0 + j) is in bk[j mod nb] with count n_store[cur0 ^ (j & 1)].  N(s-1) first: it may
  // sit in the canonical buffer that N(s) then overwrites.
  const uint32_t cur = cur0 ^ (kd & 1u);
  if (c->integrator == 1 && kd > 0) {
    const uint32_t j = kd - 1;
    HIPCHK(c, qmck_copy_store(c->stream, bk[j % nb], bv[j % nb], c->pk(), c->pv(),
                              &dcnt->n_store[cur0 ^ (j & 1u)], c->L.cap_store));
    HIPCHK(c, hipMemcpyAsync(&dcnt->n_prev, &dcnt->n_store[cur0 ^ (j & 1u)], 8,
                             hipMemcpyDeviceToDevice, c->stream));
  }
  if (kd % nb != 0)
    HIPCHK(c, qmck_copy_store(c->stream, bk[kd % nb], bv[kd % nb], bk[0], bv[0],
                              &dcnt->n_store[cur], c->L.cap_store));
  if (kd > 0) {
    rc = read_counters(c, hc);
    if (rc) return rc;
  }
  c->cur = cur;
  c->step = step0 + kd;
  c->n_occ = hc.n_store[cur];
  if (prof_k == 1 || prof_k == 2) add_cover(c, prof_k, before, hc, kd);
  if (prof_step) add_cover(c, 5, before, hc, kd);
  return QMC_OK;
}

}  // namespace

namespace {

// Per-replica N^tot of the current store (the eq. (3) estimator pass with no observables),
// exact integers, synchronizing the stream.
int replica_ntot(qmc_ctx* c, std::vector<uint64_t>& nt) {
  const uint32_t R = c->R, stride = 5;
  unsigned long long* dout = c->at<unsigned long long>(c->L.obs_out);
  HIPCHK(c, hipMemsetAsync(dout, 0, (size_t)R * stride * 8, c->stream));
  HIPCHK(c, qmck_observe(c->stream, c->sk(c->cur), c->sv(c->cur), c->counters(), c->cur, c->n,
                         c->kbits, R, 0, c->at<uint64_t>(c->L.obs_in), 0, dout, stride,
                         c->cfg.store_capacity));
  std::vector<unsigned long long> acc((size_t)R * stride);
  HIPCHK(c, hipMemcpyAsync(acc.data(), dout, acc.size() * 8, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  nt.resize(R);
  for (uint32_t r = 0; r < R; ++r) nt[r] = acc[(size_t)r * stride];
  return QMC_OK;
}

// The variable-shift update after the step that brought the counter to a multiple of the
// period (qmc_config): a replica that reaches the target takes its N^tot as the reference, a
// started one updates S from ln(N^tot / reference) and takes a new reference.  The shifts are
// checked against the Q32 bound when the next step's tables are built.
int shift_update(qmc_ctx* c) {
  std::vector<uint64_t> nt;
  int rc = replica_ntot(c, nt);
  if (rc) return rc;
  const double rate = c->cfg.shift_zeta / ((double)c->cfg.shift_period * c->cfg.dt);
  for (uint32_t r = 0; r < c->R; ++r) {
    if (!c->shift_on[r]) {
      if (nt[r] >= c->cfg.shift_target) {
        c->shift_on[r] = 1;
        c->shift_ref[r] = nt[r];
      }
      continue;
    }
    if (nt[r] > 0 && c->shift_ref[r] > 0)
      c->shift[r] = c->shift[r] - rate * std::log((double)nt[r] / (double)c->shift_ref[r]);
    c->shift_ref[r] = nt[r];
  }
  return QMC_OK;
}

int step_impl(qmc_ctx* c, uint32_t nsteps, const double* s, const double* gamma);

}  // namespace

int qmc_step(qmc_ctx* c, uint32_t nsteps, const double* s, const double* gamma) {
  if (!c) return QMC_ERR_ARG;
  if (c->broken) return fail(c, QMC_ERR_STATE, "context unusable after a HIP error");
  if (nsteps == 0) return QMC_OK;
  if ((c->n_h && !s) || (c->n_l && !gamma)) return fail(c, QMC_ERR_ARG, "missing weights");
  if (c->cfg.shift_mode != 1) return step_impl(c, nsteps, s, gamma);
  // Variable shift: runs of steps up to the next multiple of the period, each followed by the
  // shift update.
  const uint32_t A = c->cfg.shift_period;
  uint32_t done = 0;
  while (done < nsteps) {
    const uint32_t k = std::min<uint32_t>(nsteps - done, A - c->step % A);
    int rc = step_impl(c, k, s + (size_t)done * c->n_h, gamma + (size_t)done * c->n_l);
    if (rc) return rc;
    done += k;
    if (c->step % A == 0) {
      rc = shift_update(c);
      if (rc) return rc;
    }
  }
  return QMC_OK;
}

namespace {

int step_impl(qmc_ctx* c, uint32_t nsteps, const double* s, const double* gamma) {
  const bool ab2 = c->integrator == 1;
  // AB2 without N(s-1): the first step of this call is an Euler step of its own.
  const uint32_t euler_first = ab2 && !c->have_prev ? 1u : 0u;
  auto wts = [&](uint32_t k, const double*& ws, const double*& wg) {
    ws = s + (size_t)k * c->n_h;
    wg = gamma + (size_t)k * c->n_l;
  };

  // Build and check every table of the call before launching anything: step k uses A(k) (the
  // only table for Euler) and, for AB2, B(k) from the weights of step k - 1.
  std::vector<int64_t> qsA, qsB, qs1;
  if (shifts_q32(c, 1.0, qs1) || (ab2 && (shifts_q32(c, 1.5, qsA) || shifts_q32(c, -0.5, qsB))))
    return fail(c, QMC_ERR_DT, "shift too large for Q32");
  uint64_t max_qa = 0, max_qb = 0;
  for (uint32_t r = 0; r < c->R; ++r) {
    max_qa = std::max(max_qa, uabs(ab2 ? qsA[r] : qs1[r]));
    if (ab2) max_qb = std::max(max_qb, uabs(qsB[r]));
    if (euler_first) max_qa = std::max(max_qa, uabs(qs1[r]));
  }
  // Tables of step k of circuit ci into (TA, TB); QMC_OK or the error with its message.  (AB2
  // runs with one circuit only.)
  const uint32_t NC = c->C;
  auto build_step = [&](uint32_t k, uint32_t ci, HostTable& TA, HostTable& TB,
                        std::string& why) -> int {
    const double *ws, *wg;
    wts(k, ws, wg);
    ws += c->wh_off[ci];
    wg += c->wl_off[ci];
    const bool two = ab2 && k >= euler_first;
    const uint32_t nh = (ci + 1 < NC ? c->wh_off[ci + 1] : c->n_h) - c->wh_off[ci];
    const uint32_t nl = (ci + 1 < NC ? c->wl_off[ci + 1] : c->n_l) - c->wl_off[ci];
    int rc = build_table_plan(c->plans[ci], c->cfg.dt, ws, wg, two ? 1.5 : 1.0, TA, why, nh, nl);
    if (!rc && two) {
      const double *ps, *pg;
      if (k > 0) {
        wts(k - 1, ps, pg);
      } else {
        ps = c->w_prev.data();
        pg = c->w_prev.data() + c->n_h;
      }
      rc = build_table_plan(c->plans[ci], c->cfg.dt, ps, pg, -0.5, TB, why);
      if (!rc && TB.q_diag + max_qb >= (1ull << 31)) {
        rc = QMC_ERR_DT;
        why = "diagonal group with shift violates the Q32 bound";
      }
      // A key receives at most one record per group of each table; the merges keep a key's
      // records together only up to kMergeSlack + 1 of them.
      if (!rc && TA.gx.size() + TB.gx.size() > (size_t)qmc::kMergeSlack + 1) {
        rc = QMC_ERR_ARG;
        why = "the two AB2 tables have more than 257 column groups between them";
      }
    }
    // A proposal puts up to k records of one parent on one key: every key's records from one
    // table must stay within the merge's run bound.
    if (!rc && c->prop.kind &&
        (uint64_t)c->prop.k * (TA.gx.size() - 1) + 1 > (uint64_t)qmc::kMergeSlack) {
      rc = QMC_ERR_ARG;
      why = "proposal samples times column groups exceed the merge's run bound (256)";
    }
    if (!rc && TA.q_diag + max_qa >= (1ull << 31)) {
      rc = QMC_ERR_DT;
      why = "diagonal group with shift violates the Q32 bound";
    }
    return rc;
  };
  // Table windows: steps [win0, win1) of this call have their packed tables (all circuits) in
  // the pinned staging area and their offsets ([step][circuit], and the AB2 B term's) staged
  // right after it; the LDS-resident step reads them there.  The fused and streamed kernels read
  // copies in the device table area (the same offsets) and tab_off / tabB_off, made when a chunk
  // on those paths first needs them; every launch of those steps reuses them.
  const uint32_t wmax = std::min<uint32_t>(nsteps, kMaxChunkSteps);
  std::vector<uint32_t> offA((size_t)wmax * NC, 0), offB(ab2 ? wmax : 0, 0);
  uint32_t win0 = 0, win1 = 0;
  size_t max_tbytes = 0;
  uint32_t* const po = reinterpret_cast<uint32_t*>(c->pinned + kTableArea);
  uint32_t* const pb = po + (size_t)kMaxChunkSteps * NC;
  std::vector<std::pair<size_t, size_t>> dev_spans;  // staged table bytes to copy to the device
  bool dev_ready = true;
  // offsets of steps [from, win1 - win0) of the window into pinned staging
  auto stage_window = [&](const std::vector<std::pair<size_t, size_t>>& spans, uint32_t from) {
    const size_t a = (size_t)from * NC, nw = (size_t)(win1 - win0) * NC;
    if (nw > a) std::memcpy(po + a, offA.data() + a, (nw - a) * 4);
    if (ab2) std::memcpy(pb, offB.data(), (size_t)(win1 - win0) * 4);
    dev_spans = spans;
    dev_ready = false;
  };
  auto ensure_device = [&]() -> int {
    if (dev_ready) return QMC_OK;
    for (const auto& sp : dev_spans)
      if (sp.second)
        HIPCHK(c, hipMemcpyAsync(c->at<uint8_t>(c->L.tab) + sp.first, c->pinned + sp.first,
                                 sp.second, hipMemcpyHostToDevice, c->stream));
    const size_t nw = (size_t)(win1 - win0) * NC;
    HIPCHK(c, hipMemcpyAsync(c->at<uint32_t>(c->L.tab_off), po, nw * 4, hipMemcpyHostToDevice,
                             c->stream));
    if (ab2)
      HIPCHK(c, hipMemcpyAsync(c->at<uint32_t>(c->L.tabB_off), pb, (size_t)(win1 - win0) * 4,
                               hipMemcpyHostToDevice, c->stream));
    dev_ready = true;
    return QMC_OK;
  };
  // Packs the tables of step k (all circuits, both AB2 terms) at `bytes` of the staging area
  // when they fit under `cap`; returns false otherwise.
  auto pack_step = [&](uint32_t k, uint32_t slot, std::vector<HostTable>& TA, HostTable& TB,
                       size_t base, size_t& used, size_t cap) -> bool {
    const bool two = ab2 && k >= euler_first;
    size_t need = two ? pack_table(TB, nullptr) : 0;
    for (uint32_t ci = 0; ci < NC; ++ci) need += pack_table(TA[ci], nullptr);
    if (used + need > cap) return false;
    for (uint32_t ci = 0; ci < NC; ++ci) {
      offA[(size_t)slot * NC + ci] = (uint32_t)(base + used);
      used += pack_table(TA[ci], c->pinned + base + used);
    }
    if (two) {
      offB[slot] = (uint32_t)(base + used);
      used += pack_table(TB, c->pinned + base + used);
    }
    return true;
  };
  const uint64_t fused_max_keys = (uint64_t)c->L.P * kFusedKeysPerSegment;
  // The LDS-resident step can start before every table of the call is built: its first batch
  // (steps [0, B0)) is launched as soon as their tables are packed, and the host builds the rest
  // while it runs.  A later table that fails, or that the step cannot take, only cancels that
  // batch: it writes scratch segments, never the store or the counters.
  SmallHead head;
  const uint32_t B0 = std::max<uint32_t>(2, std::min<uint32_t>(kHeadMax, nsteps / 4));
  const bool pipe = nsteps >= 8 && nsteps < 512 && !ab2 && !c->prop.kind && c->R <= c->L.P &&
                    (c->path == 3 ||
                     (c->path == 0 && !c->small_off && c->step >= c->streamed_until &&
                      c->n_occ <= fused_max_keys && c->small_limit > 0 &&
                      c->n_occ <= (uint64_t)c->R * c->small_limit));
  auto prelaunch = [&]() -> int {
    // the batch reads its tables from pinned staging and its offsets from a pinned area of their
    // own (pin_head), whose cache lines hold none of the offsets the host is about to write
    std::memcpy(c->pinned_small + c->pin_head, offA.data(), (size_t)B0 * NC * 4);
    std::vector<int64_t> q(2 * (size_t)c->R, 0);
    for (uint32_t r = 0; r < c->R; ++r) q[r] = qs1[r];
    int rc = upload_qshift(c, q);
    if (rc) return rc;
    SmallLaunch sl;
    small_setup(c, c->pinned_dev, sl);
    head.epoch = ++c->small_epoch;
    sl.epoch = head.epoch;
    if (c->prof_whole()) {
      rc = timing_pair(c, head.ev0, head.ev1);
      if (rc) return rc;
      HIPCHK(c, hipEventRecord(head.ev0, c->stream));
    }
    HIPCHK(c, small_batch(c, sl, 0, c->step, 0, 0, B0,
                          reinterpret_cast<const uint32_t*>(c->pinned_small_dev + c->pin_head)));
    if (head.ev1) HIPCHK(c, hipEventRecord(head.ev1, c->stream));
    head.steps = B0;
    return QMC_OK;
  };
  // A launched first batch that will not be continued: wait for it, return its events.
  auto drop_head = [&]() -> int {
    if (!head.steps) return QMC_OK;
    head.steps = 0;
    if (head.ev0) {
      c->ev_free.push_back(head.ev0);
      c->ev_free.push_back(head.ev1);
      head.ev0 = head.ev1 = nullptr;
    }
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return QMC_OK;
  };
  int pre_rc = QMC_OK;
  {
    // Long calls build on a few host threads (tables are independent), each packing its run of
    // steps into its own slice of the staging area while it fits (the first window); every
    // step is checked, and the first failing step in step order is reported.
    const uint32_t nth = nsteps >= 512 ? std::min<uint32_t>(kTableThreads, nsteps / 256) : 1u;
    struct Part {
      uint32_t a, b, stored, bad;
      size_t base, used;
      size_t max_bytes;
      int code;
      std::string why;
    };
    std::vector<Part> parts(nth);
    const size_t slice = (kTableArea / nth) & ~(size_t)255;  // slices stay 256-byte aligned
    for (uint32_t i = 0; i < nth; ++i) {
      Part& q = parts[i];
      q.a = (uint32_t)((uint64_t)nsteps * i / nth);
      q.b = (uint32_t)((uint64_t)nsteps * (i + 1) / nth);
      q.stored = q.a;
      q.bad = nsteps;
      q.base = slice * i;
      q.used = q.max_bytes = 0;
      q.code = QMC_OK;
    }
    auto part = [&](uint32_t i) {
      Part& q = parts[i];
      std::vector<HostTable> TA(NC);
      HostTable TB;
      for (uint32_t k = q.a; k < q.b; ++k) {
        for (uint32_t ci = 0; ci < NC; ++ci) {
          q.code = build_step(k, ci, TA[ci], TB, q.why);
          if (q.code) {
            q.bad = k;
            return;
          }
          q.max_bytes = std::max(q.max_bytes, pack_table(TA[ci], nullptr));
        }
        if (ab2 && k >= euler_first) q.max_bytes = std::max(q.max_bytes, pack_table(TB, nullptr));
        if (q.stored == k && k < wmax && pack_step(k, k, TA, TB, q.base, q.used, slice))
          q.stored = k + 1;
        if (pipe && nth == 1 && k + 1 == B0 && q.stored == B0 &&
            q.max_bytes <= kPersistTableBytes) {
          pre_rc = prelaunch();
          if (pre_rc) return;
          // The launched batch reads kPersistTableBytes from the start of each of its tables
          // while the host packs the later ones: those start past the last such read, on a cache
          // line of their own, so no line it brings into the caches holds bytes written later.
          q.used = (q.used + kPersistTableBytes + 255) & ~(size_t)255;
        }
      }
    };
    std::vector<std::thread> pool;
    for (uint32_t i = 1; i < nth; ++i) {
      try {
        pool.emplace_back(part, i);
      } catch (...) {  // no thread available: build that part here
        part(i);
      }
    }
    part(0);
    for (std::thread& th : pool) th.join();
    if (pre_rc) return pre_rc;
    for (const Part& q : parts)
      if (q.code) {
        int rc = drop_head();
        if (rc) return rc;
        return fail(c, q.code, "step " + std::to_string(c->step + q.bad) + ": " + q.why);
      }
    // the first window: every step up to the first part that could not store all of its steps
    std::vector<std::pair<size_t, size_t>> spans;
    win1 = 0;
    for (const Part& q : parts) {
      max_tbytes = std::max(max_tbytes, q.max_bytes);
      if (win1 == q.a) {
        spans.emplace_back(q.base, q.used);
        win1 = q.stored;
      }
    }
    if (win1 == 0) return fail(c, QMC_ERR_ARG, "step tables larger than the table area");
    // (the head batch reads its own copy of its offsets)
    stage_window(spans, 0u);
  }
  const uint32_t first_step = c->step;
  const bool fused_fits = max_tbytes <= kPersistTableBytes;
  if (c->path == 1 && !fused_fits)
    return fail(c, QMC_ERR_ARG, "step table larger than the fused kernel takes; use the "
                                "automatic or streamed path");
  if (c->path == 1 && c->prop.kind)
    return fail(c, QMC_ERR_ARG, "spawn proposals run on the streamed path");
  if (c->path == 3 && (ab2 || c->prop.kind || !fused_fits || c->R > c->L.P)) {
    int rc = drop_head();
    if (rc) return rc;
    return fail(c, QMC_ERR_ARG, "the LDS-resident step runs the Euler step and the comb with "
                                "step tables of at most 8 KB, one workgroup per segment");
  }
  uint32_t last_local_fail = 0xFFFFFFFFu;
  int32_t shift_mode = -1;  // shifts on the device: 0 single Euler term, 1 both AB2 terms
  while (c->step < first_step + nsteps) {
    const uint32_t k0 = c->step - first_step;
    const bool two = ab2 && k0 >= euler_first;
    const bool fused = c->path == 1 || (c->path == 0 && fused_fits && !c->prop.kind &&
                                        c->step >= c->streamed_until &&
                                        c->n_occ <= fused_max_keys);
    // the LDS-resident step: Euler, the comb, tables the fused kernel takes, every segment
    // small (tried while the whole store could fit; a segment that does not fit stops it)
    const bool small = c->path == 3 ||
                       (c->path == 0 && fused && !ab2 && !c->small_off && c->R <= c->L.P &&
                        c->small_limit > 0 && c->n_occ <= (uint64_t)c->R * c->small_limit);
    if (head.steps && !(small && k0 == 0)) {
      int rc = drop_head();
      if (rc) return rc;
    }
    if (shift_mode != (int32_t)two) {
      // shifts of this chunk's tables
      std::vector<int64_t> q(2 * (size_t)c->R, 0);
      for (uint32_t r = 0; r < c->R; ++r) {
        q[r] = two ? qsA[r] : qs1[r];
        if (two) q[c->R + r] = qsB[r];
      }
      int rc = upload_qshift(c, q);
      if (rc) return rc;
      shift_mode = (int32_t)two;
    }
    // One launch (fused) or one stream of launches: the remaining steps of the table window;
    // the Euler first step of AB2 runs alone; an automatic streamed run stops where the fused
    // kernel may be tried again.
    uint32_t kmax = two || !ab2 ? nsteps : k0 + 1;
    if (!fused && c->path == 0 && c->step < c->streamed_until)
      kmax = std::min<uint32_t>(kmax, c->streamed_until - first_step);
    if (k0 >= win1) {
      // the next window (calls longer than the first one): packed here, one step after another
      win0 = win1 = k0;
      size_t bytes = 0;
      std::vector<HostTable> TA(NC);
      HostTable TB;
      std::string why;
      while (win1 < nsteps && win1 - win0 < kMaxChunkSteps) {
        for (uint32_t ci = 0; ci < NC; ++ci)
          if (build_step(win1, ci, TA[ci], TB, why))
            return fail(c, QMC_ERR_STATE, "table changed: " + why);
        if (!pack_step(win1, win1 - win0, TA, TB, 0, bytes, kTableArea)) break;
        ++win1;
      }
      if (win1 == k0) return fail(c, QMC_ERR_ARG, "step tables larger than the table area");
      stage_window({{0, bytes}}, 0u);
    }
    Chunk ch;
    ch.dtab = c->at<uint8_t>(c->L.tab);
    ch.two = two;
    const uint32_t k1 = std::min<uint32_t>(kmax, win1);
    ch.nst = k1 - k0;
    ch.first = k0 - win0;
    qmc::Counters hc;
    uint32_t kd = 0, reason = 0;
    if (small) {
      const SmallHead hd = head;
      head = SmallHead{};
      int rc = run_small(c, ch, kd, hc, hd.steps ? &hd : nullptr);
      if (rc) return rc;
      if (kd == 0) {
        if (c->path == 3)
          return fail(c, QMC_ERR_STORE_CAP, "step " + std::to_string(c->step) +
                                                ": a replica outgrows the LDS-resident step");
        continue;  // the automatic mode takes this step with the fused kernel
      }
      continue;
    }
    int rc = ensure_device();
    if (rc) return rc;
    rc = fused ? run_fused(c, ch, kd, reason, hc) : run_streamed(c, ch, kd, hc);
    if (rc) return rc;
    if (ab2 && kd > 0) {
      // N(s-1) is now on the device; remember the weights of step s-1.
      const double *ws, *wg;
      wts(k0 + kd - 1, ws, wg);
      c->w_prev.assign(ws, ws + c->n_h);
      c->w_prev.insert(c->w_prev.end(), wg, wg + c->n_l);
      c->have_prev = true;
    }
    if (hc.err) {
      const uint32_t e = hc.err;
      const std::string at = "step " + std::to_string(c->step) + ": ";
      if (e & qmc::kErrLookback) {
        c->broken = true;
        return fail(c, QMC_ERR_HIP, at + "a bounded wait expired");
      }
      if (e & qmc::kErrOverflow) return fail(c, QMC_ERR_COUNT_OVERFLOW, at + "population outside int32");
      if (e & qmc::kErrStoreCap) return fail(c, QMC_ERR_STORE_CAP, at + "store capacity exceeded");
      if (e & qmc::kErrSpawnCap) return fail(c, QMC_ERR_SPAWN_CAP, at + "spawn capacity exceeded");
      // A key range outgrew its segment or inbox: rebalance once per step; then, in automatic
      // mode, run the next steps streamed.
      if (c->step == last_local_fail) {
        if (c->path == 0) {
          c->streamed_until = c->step + kStreamedWindow;
          continue;
        }
        if (e & qmc::kErrSegCap)
          return fail(c, QMC_ERR_STORE_CAP, at + "a key range exceeds one segment");
        return fail(c, QMC_ERR_SPAWN_CAP, at + "a key range receives more than one inbox");
      }
      last_local_fail = c->step;
    } else if (reason == 2) {
      c->broken = true;
      return fail(c, QMC_ERR_HIP, "fused step stopped without an error flag");
    }
  }
  return QMC_OK;
}

}  // namespace

int qmc_step_path(qmc_ctx* c, int32_t path) {
  if (!c || path < 0 || path > 3) return QMC_ERR_ARG;
  c->path = path;
  c->streamed_until = 0;
  c->small_off = false;
  return QMC_OK;
}

int qmc_small_limit(qmc_ctx* c, uint32_t keys) {
  if (!c || keys > (uint32_t)kSmallCap) return QMC_ERR_ARG;
  c->small_limit = keys;
  c->small_off = false;
  return QMC_OK;
}

int qmc_set_integrator(qmc_ctx* c, int32_t integrator) {
  if (!c || integrator < 0 || integrator > 1) return QMC_ERR_ARG;
  if (integrator == 1 && c->cfg.shift_mode == 1)
    return fail(c, QMC_ERR_ARG, "the variable shift runs with the Euler step");
  if (integrator == 1 && c->C > 1) return fail(c, QMC_ERR_ARG, "AB2 runs one circuit per context");
  if (integrator == 1 && c->prop.kind)
    return fail(c, QMC_ERR_ARG, "AB2 runs without spawn proposals");
  if (c->broken) return fail(c, QMC_ERR_STATE, "context unusable after a HIP error");
  c->integrator = integrator;
  c->have_prev = false;
  c->w_prev.clear();
  return QMC_OK;
}

int qmc_pulse_batch(qmc_ctx* c, const uint64_t* x, const uint64_t* z) {
  if (!c || !x || !z) return QMC_ERR_ARG;
  if (c->broken) return fail(c, QMC_ERR_STATE, "context unusable after a HIP error");
  const uint64_t qmask = c->n >= 32 ? 0xFFFFFFFFull : ((1ull << c->n) - 1);
  bool any_x = false;
  uint64_t* pin = reinterpret_cast<uint64_t*>(c->pinned_small);
  for (uint32_t ci = 0; ci < c->C; ++ci) {
    if ((x[ci] | z[ci]) & ~qmask) return fail(c, QMC_ERR_ARG, "pulse mask outside n bits");
    any_x = any_x || x[ci] != 0;
    pin[2 * ci] = x[ci];
    pin[2 * ci + 1] = z[ci];
  }
  qmc::Counters* dcnt = c->counters();
  HIPCHK(c, hipMemcpyAsync(c->at<uint64_t>(c->L.pulse), pin, (size_t)c->C * 16,
                           hipMemcpyHostToDevice, c->stream));
  // the look-back words are cleared only before the whole-store sort that a pulse with x != 0
  // needs (a diagonal pulse sorts nothing)
  HIPCHK(c, qmck_batch_begin(c->stream, dcnt, nullptr, 0,
                             any_x ? c->at<uint64_t>(c->L.sort_status) : nullptr,
                             any_x ? c->L.n_sort_status : 0, c->ghist(0),
                             2 * qmc::kMaxPasses * qmc::kRadixBins));
  HIPCHK(c, qmck_pulse(c->stream, c->sk(c->cur), c->sv(c->cur), dcnt, c->cur, c->n, c->kbits,
                       c->Rc, c->at<uint64_t>(c->L.pulse), any_x ? 1 : 0, c->ck(0), c->cv(0), 0,
                       c->L.cap_store));
  if (any_x) {
    const uint32_t passes = qmck_sort_passes(c->kbits + c->rbits);
    HIPCHK(c, qmck_digit_hist(c->stream, c->ck(0), dcnt, 0, passes, c->ghist(0), c->L.cap_store));
    HIPCHK(c, qmck_sort(c->stream, c->ck(0), c->cv(0), c->ck(1), c->cv(1), dcnt, 0, passes,
                        c->ghist(0), c->at<uint64_t>(c->L.sort_status), c->step, 0,
                        c->L.cap_sort, c->sort_ipt));
    const uint32_t out = passes & 1;
    HIPCHK(c, qmck_copy_store(c->stream, c->ck(out), c->cv(out), c->sk(c->cur), c->sv(c->cur),
                              &dcnt->n_child[0], c->L.cap_store));
  }
  qmc::Counters hc;
  int rc = read_counters(c, hc);  // also keeps the pinned masks alive until the copy is done
  if (rc) return rc;
  if (hc.err & qmc::kErrOverflow)
    return fail(c, QMC_ERR_COUNT_OVERFLOW, "pulse negated INT32_MIN");
  c->have_prev = false;  // AB2 restarts after a pulse (its next step is an Euler step)
  return QMC_OK;
}

int qmc_pulse(qmc_ctx* c, uint64_t x, uint64_t z) {
  if (!c) return QMC_ERR_ARG;
  std::vector<uint64_t> xs(c->C, x), zs(c->C, z);
  return qmc_pulse_batch(c, xs.data(), zs.data());
}

int qmc_set_proposal(qmc_ctx* c, int32_t kind, uint32_t samples, const int8_t* w1,
                     const int32_t* b1, const int8_t* w2, const int32_t* b2,
                     uint32_t hidden_shift) {
  if (!c || kind < 0 || kind > 3) return QMC_ERR_ARG;
  if (c->broken) return fail(c, QMC_ERR_STATE, "context unusable after a HIP error");
  if (kind == 0) {
    QmcProposal p{};
    p.log = c->prop.log;
    p.log_cap = c->prop.log_cap;
    p.log_count = c->prop.log_count;
    c->prop = p;
    return QMC_OK;
  }
  if (samples == 0 || samples > 64 || (samples & (samples - 1)))
    return fail(c, QMC_ERR_ARG, "proposal samples must be a power of two from 1 to 64");
  if (c->integrator != 0 || c->init_min != 0 || c->C != 1)
    return fail(c, QMC_ERR_ARG, "spawn proposals run with Euler, one circuit, no initiators");
  if (2 * c->n > (uint32_t)kPropIn) return fail(c, QMC_ERR_ARG, "key wider than the MLP input");
  QmcProposal p{};
  p.kind = (uint32_t)kind;
  p.k = samples;
  p.nbits = 2 * c->n;
  p.log = c->prop.log;
  p.log_cap = c->prop.log_cap;
  p.log_count = c->prop.log_count;
  if (kind == 3) {
    if (!w1 || !b1 || !w2 || !b2 || hidden_shift > 30)
      return fail(c, QMC_ERR_ARG, "the MLP proposal needs its weights and a shift <= 30");
    uint8_t* d = c->at<uint8_t>(c->L.mlp);
    HIPCHK(c, hipMemcpyAsync(d, w1, kMlpW1, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(d + kMlpW1, b1, kMlpB1, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(d + kMlpW1 + kMlpB1, w2, kMlpW2, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(d + kMlpW1 + kMlpB1 + kMlpW2, b2, kMlpB2, hipMemcpyHostToDevice,
                             c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));  // the caller's arrays may go away
    p.s1 = hidden_shift;
    p.w1 = reinterpret_cast<const int8_t*>(d);
    p.b1 = reinterpret_cast<const int32_t*>(d + kMlpW1);
    p.w2 = reinterpret_cast<const int8_t*>(d + kMlpW1 + kMlpB1);
    p.b2 = reinterpret_cast<const int32_t*>(d + kMlpW1 + kMlpB1 + kMlpW2);
  }
  c->prop = p;
  return QMC_OK;
}

int qmc_set_proposal_deep(qmc_ctx* c, uint32_t samples, const int8_t* w1, const int32_t* b1,
                          const int8_t* w2, const int32_t* b2, const int8_t* w3,
                          const int32_t* b3, uint32_t shift1, uint32_t shift2) {
  if (!c) return QMC_ERR_ARG;
  if (c->broken) return fail(c, QMC_ERR_STATE, "context unusable after a HIP error");
  if (samples == 0 || samples > 64 || (samples & (samples - 1)))
    return fail(c, QMC_ERR_ARG, "proposal samples must be a power of two from 1 to 64");
  if (c->integrator != 0 || c->init_min != 0 || c->C != 1)
    return fail(c, QMC_ERR_ARG, "spawn proposals run with Euler, one circuit, no initiators");
  if (2 * c->n > 64) return fail(c, QMC_ERR_ARG, "key wider than the network input");
  if (!w1 || !b1 || !w2 || !b2 || !w3 || !b3 || shift1 > 30 || shift2 > 30)
    return fail(c, QMC_ERR_ARG, "the network needs all its weights and shifts <= 30");
  uint8_t* d = c->at<uint8_t>(c->L.mlp) + kMlpBytes;
  const void* src[6] = {w1, b1, w2, b2, w3, b3};
  const size_t len[6] = {kDeepW1, kDeepB1, kDeepW2, kDeepB2, kDeepW3, kDeepB3};
  size_t off[6];
  size_t o = 0;
  for (int i = 0; i < 6; ++i) {
    off[i] = o;
    HIPCHK(c, hipMemcpyAsync(d + o, src[i], len[i], hipMemcpyHostToDevice, c->stream));
    o += len[i];
  }
  HIPCHK(c, hipStreamSynchronize(c->stream));  // the caller's arrays may go away
  QmcProposal p{};
  p.kind = 4;
  p.k = samples;
  p.log = c->prop.log;
  p.log_cap = c->prop.log_cap;
  p.log_count = c->prop.log_count;
  p.nbits = 2 * c->n;
  p.s1 = shift1;
  p.s2 = shift2;
  p.w1 = reinterpret_cast<const int8_t*>(d + off[0]);
  p.b1 = reinterpret_cast<const int32_t*>(d + off[1]);
  p.w2 = reinterpret_cast<const int8_t*>(d + off[2]);
  p.b2 = reinterpret_cast<const int32_t*>(d + off[3]);
  p.w3 = reinterpret_cast<const int8_t*>(d + off[4]);
  p.b3 = reinterpret_cast<const int32_t*>(d + off[5]);
  c->prop = p;
  return QMC_OK;
}

int qmc_log_spawns(qmc_ctx* c, void* d_events, uint64_t capacity, uint64_t* d_count) {
  if (!c || (d_events && !d_count)) return QMC_ERR_ARG;
  if (c->broken) return fail(c, QMC_ERR_STATE, "context unusable after a HIP error");
  c->prop.log = reinterpret_cast<SpawnEvent*>(d_events);
  c->prop.log_cap = d_events ? capacity : 0;
  c->prop.log_count = d_events ? reinterpret_cast<unsigned long long*>(d_count) : nullptr;
  return QMC_OK;
}

int qmc_use_graphs(qmc_ctx* c, int32_t on) {
  if (!c || (on != 0 && on != 1)) return QMC_ERR_ARG;
  if (c->broken) return fail(c, QMC_ERR_STATE, "context unusable after a HIP error");
  c->use_graph = on != 0;
  return QMC_OK;
}

int qmc_tune_sort(qmc_ctx* c, uint32_t records_per_thread, uint32_t* chosen) {
  if (!c) return QMC_ERR_ARG;
  if (c->broken) return fail(c, QMC_ERR_STATE, "context unusable after a HIP error");
  if (records_per_thread != 0) {
    if (!qmck_sort_tile_ok(records_per_thread))
      return fail(c, QMC_ERR_ARG, "sort tiles take 8, 12, 16 or 24 records per thread");
    c->sort_ipt = records_per_thread;
    if (chosen) *chosen = c->sort_ipt;
    return QMC_OK;
  }
  // Autotune: time every tile size on synthetic records of this context's key width and spawn
  // capacity (at most 4M records) in the child buffers, which hold nothing between calls, and
  // keep the fastest.  The sorted order does not depend on the tile size.
  qmc::Counters* dcnt = c->counters();
  const uint64_t n = std::min<uint64_t>(c->L.cap_child, 1ull << 22);
  const uint32_t bits = c->kbits + c->rbits + (c->init_min ? 1u : 0u);
  const uint64_t mask = bits >= 64 ? ~0ull : ((1ull << bits) - 1);
  const uint32_t passes = qmck_sort_passes(bits);
  uint64_t* pin_n = reinterpret_cast<uint64_t*>(c->pinned_small + 2048);
  *pin_n = n;
  hipEvent_t ev[2];
  HIPCHK(c, hipEventCreate(&ev[0]));
  HIPCHK(c, hipEventCreate(&ev[1]));
  uint32_t best = c->sort_ipt;
  float best_ms = 0.f;
  int rc = QMC_OK;
  for (uint32_t ipt : kSortIpts) {
    float fastest = 0.f;
    for (int rep = 0; rep < 3 && rc == QMC_OK; ++rep) {
      hipError_t e = (hipError_t)qmck_batch_begin(
          c->stream, dcnt, nullptr, 0, c->at<uint64_t>(c->L.sort_status), c->L.n_sort_status,
          c->ghist(0), 2 * qmc::kMaxPasses * qmc::kRadixBins);
      if (e == hipSuccess)
        e = (hipError_t)qmck_fill_sort_probe(c->stream, c->ck(0), c->cv(0), n, mask, 77 + rep);
      if (e == hipSuccess)
        e = hipMemcpyAsync(&dcnt->n_child[0], pin_n, 8, hipMemcpyHostToDevice, c->stream);
      if (e == hipSuccess)
        e = (hipError_t)qmck_digit_hist(c->stream, c->ck(0), dcnt, 0, passes, c->ghist(0), n);
      if (e == hipSuccess) e = hipEventRecord(ev[0], c->stream);
      if (e == hipSuccess)
        e = (hipError_t)qmck_sort(c->stream, c->ck(0), c->cv(0), c->ck(1), c->cv(1), dcnt, 0,
                                  passes, c->ghist(0), c->at<uint64_t>(c->L.sort_status), c->step,
                                  0, n, ipt);
      if (e == hipSuccess) e = hipEventRecord(ev[1], c->stream);
      if (e == hipSuccess) e = hipEventSynchronize(ev[1]);
      float ms = 0.f;
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, ev[0], ev[1]);
      if (e != hipSuccess) {
        c->broken = true;
        rc = fail(c, QMC_ERR_HIP, std::string("sort tuning: ") + hipGetErrorString(e));
        break;
      }
      if (rep == 0 || ms < fastest) fastest = ms;
    }
    if (rc) break;
    if (best_ms == 0.f || fastest < best_ms) {
      best_ms = fastest;
      best = ipt;
    }
  }
  (void)hipEventDestroy(ev[0]);
  (void)hipEventDestroy(ev[1]);
  if (rc) return rc;
  qmc::Counters hc;
  rc = read_counters(c, hc);
  if (rc) return rc;
  if (hc.err) {
    c->broken = true;
    return fail(c, QMC_ERR_HIP, "sort tuning raised a device error");
  }
  // leave the counters as a step expects them
  HIPCHK(c, qmck_batch_begin(c->stream, dcnt, nullptr, 0, c->at<uint64_t>(c->L.sort_status),
                             c->L.n_sort_status, c->ghist(0),
                             2 * qmc::kMaxPasses * qmc::kRadixBins));
  c->sort_ipt = best;
  if (chosen) *chosen = best;
  return QMC_OK;
}

int qmc_set_initiator(qmc_ctx* c, uint64_t min_walkers) {
  if (!c) return QMC_ERR_ARG;
  if (c->broken) return fail(c, QMC_ERR_STATE, "context unusable after a HIP error");
  if (min_walkers > 0 && c->prop.kind)
    return fail(c, QMC_ERR_ARG, "the initiator approximation runs without spawn proposals");
  if (min_walkers > 0 && c->C > 1)
    return fail(c, QMC_ERR_ARG, "the initiator approximation runs one circuit per context");
  if (min_walkers > 0 && c->kbits + c->rbits + 1 > 64)
    return fail(c, QMC_ERR_ARG, "no key bit left for the initiator flag");
  c->init_min = min_walkers;
  return QMC_OK;
}

int qmc_set_shift(qmc_ctx* c, uint32_t replica, double shift) {
  if (!c || replica >= c->R || !std::isfinite(shift)) return QMC_ERR_ARG;
  if (c->broken) return fail(c, QMC_ERR_STATE, "context unusable after a HIP error");
  std::vector<int64_t> qs;
  const double old = c->shift[replica];
  c->shift[replica] = shift;
  if (shifts_q32(c, 1.5, qs)) {  // the largest factor any table uses
    c->shift[replica] = old;
    return fail(c, QMC_ERR_DT, "shift too large for Q32");
  }
  return QMC_OK;  // uploaded with the tables of the next qmc_step
}

int qmc_observe(qmc_ctx* c, const qmc_obs_spec* spec, qmc_obs_out* out) {
  if (!c || !spec || !out) return QMC_ERR_ARG;
  if (c->broken) return fail(c, QMC_ERR_STATE, "context unusable after a HIP error");
  if (spec->n_pauli > kMaxPauli) return fail(c, QMC_ERR_ARG, "too many Pauli observables");
  const uint64_t nlook = (uint64_t)spec->n_psi * spec->n_psi;
  if (nlook > kMaxLookup) return fail(c, QMC_ERR_ARG, "|psi| support too large");
  const uint32_t R = c->R, NPl = spec->n_pauli;
  const uint32_t stride = 5 + 2 * NPl;
  std::vector<uint64_t> pxz(2 * (size_t)std::max<uint32_t>(NPl, 1), 0);
  for (uint32_t k = 0; k < NPl; ++k) {
    pxz[2 * k] = spec->px[k];
    pxz[2 * k + 1] = spec->pz[k];
  }
  unsigned long long* dout = c->at<unsigned long long>(c->L.obs_out);
  HIPCHK(c, hipMemsetAsync(dout, 0, (size_t)R * stride * 8, c->stream));
  HIPCHK(c, hipMemcpyAsync(c->at<uint64_t>(c->L.obs_in), pxz.data(), pxz.size() * 8,
                           hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, qmck_observe(c->stream, c->sk(c->cur), c->sv(c->cur), c->counters(), c->cur, c->n,
                         c->kbits, R, NPl, c->at<uint64_t>(c->L.obs_in), spec->want_eps ? 1 : 0,
                         dout, stride, c->cfg.store_capacity));
  std::vector<unsigned long long> acc((size_t)R * stride);
  HIPCHK(c, hipMemcpyAsync(acc.data(), dout, acc.size() * 8, hipMemcpyDeviceToHost, c->stream));
  std::vector<int64_t> look;
  std::vector<uint64_t> lk;
  if (nlook) {
    for (uint32_t u = 0; u < spec->n_psi; ++u)
      for (uint32_t v = 0; v < spec->n_psi; ++v)
        lk.push_back((spec->psi_index[v] << c->n) | spec->psi_index[u]);
    HIPCHK(c, hipMemcpyAsync(c->at<uint64_t>(c->L.look_keys), lk.data(), lk.size() * 8,
                             hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, qmck_lookup(c->stream, c->sk(c->cur), c->sv(c->cur), c->counters(), c->cur,
                          c->kbits, c->at<uint64_t>(c->L.look_keys), (uint32_t)nlook, R,
                          c->at<int64_t>(c->L.look_out)));
    look.resize((size_t)R * nlook * 2);
    HIPCHK(c, hipMemcpyAsync(look.data(), c->at<int64_t>(c->L.look_out), look.size() * 8,
                             hipMemcpyDeviceToHost, c->stream));
  }
  // per-replica occupied counts from the segment bounds
  std::vector<uint64_t> bounds(R + 1, 0);
  {
    std::vector<uint64_t> ck;
    std::vector<int2> cv;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    uint64_t n = 0;
    HIPCHK(c, hipMemcpy(&n, &c->counters()->n_store[c->cur], 8, hipMemcpyDeviceToHost));
    bounds[R] = n;
    // binary search of each replica's first key over device memory
    for (uint32_t r = 1; r < R; ++r) {
      const uint64_t target = (uint64_t)r << c->kbits;
      uint64_t lo = 0, hi = n;
      while (lo < hi) {
        uint64_t mid = (lo + hi) / 2, v = 0;
        HIPCHK(c, hipMemcpy(&v, c->sk(c->cur) + mid, 8, hipMemcpyDeviceToHost));
        if (v < target)
          lo = mid + 1;
        else
          hi = mid;
      }
      bounds[r] = lo;
    }
  }
  for (uint32_t r = 0; r < R; ++r) {
    const unsigned long long* a = acc.data() + (size_t)r * stride;
    const double nd0 = (double)c->nd0_re[r];
    if (out->n_occ) out->n_occ[r] = bounds[r + 1] - bounds[r];
    if (out->n_tot) out->n_tot[r] = a[0];
    if (out->shift) out->shift[r] = c->shift[r];
    const int64_t dre = (int64_t)a[1], dim = (int64_t)a[2];
    if (out->ndiag) {
      out->ndiag[2 * r] = dre;
      out->ndiag[2 * r + 1] = dim;
    }
    if (out->trace) out->trace[r] = (double)dre / nd0;
    if (out->theta) out->theta[r] = std::atan2((double)dim, (double)dre);
    for (uint32_t k = 0; k < NPl; ++k) {
      const int64_t pre = (int64_t)a[5 + 2 * k], pim = (int64_t)a[6 + 2 * k];
      if (out->pauli) {
        out->pauli[((size_t)r * NPl + k) * 2] = pre;
        out->pauli[((size_t)r * NPl + k) * 2 + 1] = pim;
      }
      if (out->pauli_val) {
        out->pauli_val[((size_t)r * NPl + k) * 2] = (double)pre / nd0;
        out->pauli_val[((size_t)r * NPl + k) * 2 + 1] = (double)pim / nd0;
      }
    }
    if (out->eps2) {
      out->eps2[2 * r] = a[3];
      out->eps2[2 * r + 1] = a[4];
    }
    if (out->eps)
      out->eps[r] = std::sqrt((double)a[4] * 18446744073709551616.0 + (double)a[3]) / nd0;
    if (out->fidelity) {
      double fre = 0.0, fim = 0.0;
      if (nlook) {
        size_t idx = 0;
        for (uint32_t u = 0; u < spec->n_psi; ++u)
          for (uint32_t v = 0; v < spec->n_psi; ++v, ++idx) {
            const double ur = spec->psi_re[u], ui = spec->psi_im[u];
            const double vr = spec->psi_re[v], vi = spec->psi_im[v];
            const double pr = ur * vr + ui * vi, pi = ur * vi - ui * vr;
            const double A = (double)look[((size_t)r * nlook + idx) * 2];
            const double B = (double)look[((size_t)r * nlook + idx) * 2 + 1];
            fre += pr * A - pi * B;
            fim += pr * B + pi * A;
          }
      }
      out->fidelity[2 * r] = fre / nd0;
      out->fidelity[2 * r + 1] = fim / nd0;
    }
  }
  return QMC_OK;
}

int qmc_export(qmc_ctx* c, uint32_t replica, uint64_t* keys, int32_t* re, int32_t* im,
               uint64_t cap, uint64_t* n) {
  if (!c || replica >= c->R || !n) return QMC_ERR_ARG;
  if (c->broken) return fail(c, QMC_ERR_STATE, "context unusable after a HIP error");
  // the replica's index range, found on the device, then only its records come over
  const uint64_t lo = c->kbits >= 64 ? 0 : (uint64_t)replica << c->kbits;
  const uint64_t hi = c->kbits >= 64 ? ~0ull : (((uint64_t)replica + 1) << c->kbits) - 1;
  uint64_t* dr = c->at<uint64_t>(c->L.look_out);  // scratch: two words
  HIPCHK(c, qmck_key_range(c->stream, c->sk(c->cur), &c->counters()->n_store[c->cur], lo, hi,
                           dr));
  uint64_t* pr = reinterpret_cast<uint64_t*>(c->pinned_small);
  HIPCHK(c, hipMemcpyAsync(pr, dr, 16, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  const uint64_t b = pr[0], m = pr[1] - pr[0];
  *n = m;
  if (m > cap) return fail(c, QMC_ERR_ARG, "export capacity too small");
  if (m == 0) return QMC_OK;
  std::vector<uint64_t> ck(m);
  std::vector<int2> cv(m);
  HIPCHK(c, hipMemcpyAsync(ck.data(), c->sk(c->cur) + b, m * 8, hipMemcpyDeviceToHost,
                           c->stream));
  HIPCHK(c, hipMemcpyAsync(cv.data(), c->sv(c->cur) + b, m * 8, hipMemcpyDeviceToHost,
                           c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  const uint64_t kmask = c->kbits >= 64 ? ~0ull : ((1ull << c->kbits) - 1);
  for (uint64_t i = 0; i < m; ++i) {
    keys[i] = ck[i] & kmask;
    re[i] = cv[i].x;
    im[i] = cv[i].y;
  }
  return QMC_OK;
}

int qmc_import(qmc_ctx* c, uint32_t replica, const uint64_t* keys, const int32_t* re,
               const int32_t* im, uint64_t n, uint32_t step) {
  if (!c || replica >= c->R) return QMC_ERR_ARG;
  if (c->broken) return fail(c, QMC_ERR_STATE, "context unusable after a HIP error");
  std::string why;
  int rc = check_records(c->n, keys, re, im, n, why);
  if (rc) return fail(c, rc, why);
  if (n > c->cfg.store_capacity) return fail(c, QMC_ERR_ARG, "more records than store capacity");
  std::vector<uint64_t> ck;
  std::vector<int2> cv;
  rc = download_store(c, ck, cv);
  if (rc) return rc;
  const uint64_t tag = c->kbits >= 64 ? 0 : (uint64_t)replica << c->kbits;
  const uint64_t lo = tag;
  const uint64_t hi = c->kbits >= 64 ? ~0ull : (((uint64_t)replica + 1) << c->kbits) - 1;
  const size_t b = (size_t)(std::lower_bound(ck.begin(), ck.end(), lo) - ck.begin());
  const size_t e = (size_t)(std::upper_bound(ck.begin(), ck.end(), hi) - ck.begin());
  std::vector<uint64_t> nk(ck.begin(), ck.begin() + b);
  std::vector<int2> nv(cv.begin(), cv.begin() + b);
  for (uint64_t i = 0; i < n; ++i) {
    nk.push_back(tag | keys[i]);
    nv.push_back(make_int2(re[i], im[i]));
  }
  nk.insert(nk.end(), ck.begin() + e, ck.end());
  nv.insert(nv.end(), cv.begin() + e, cv.end());
  rc = upload_store(c, c->cur, nk, nv);
  if (rc) return rc;
  c->step = step;
  c->small_off = false;  // a new state: the LDS-resident step may fit again
  return QMC_OK;
}

// N(s-1) of all replicas (AB2), sorted composite keys, from the device.
int download_prev(qmc_ctx* c, std::vector<uint64_t>& ck, std::vector<int2>& cv) {
  uint64_t n = 0;
  HIPCHK(c, hipMemcpyAsync(&n, &c->counters()->n_prev, 8, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  ck.resize(n);
  cv.resize(n);
  if (n) {
    HIPCHK(c, hipMemcpyAsync(ck.data(), c->pk(), n * 8, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(cv.data(), c->pv(), n * 8, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
  }
  return QMC_OK;
}

int qmc_set_prev(qmc_ctx* c, uint32_t replica, const uint64_t* keys, const int32_t* re,
                 const int32_t* im, uint64_t n, const double* s_prev, const double* gamma_prev) {
  if (!c || replica >= c->R) return QMC_ERR_ARG;
  if (c->broken) return fail(c, QMC_ERR_STATE, "context unusable after a HIP error");
  if (c->integrator != 1) return fail(c, QMC_ERR_ARG, "N(s-1) is only used by AB2");
  if ((c->n_h && !s_prev) || (c->n_l && !gamma_prev))
    return fail(c, QMC_ERR_ARG, "missing weights of step s-1");
  std::string why;
  int rc = check_records(c->n, keys, re, im, n, why);
  if (rc) return fail(c, rc, why);
  if (n > c->cfg.store_capacity) return fail(c, QMC_ERR_ARG, "more records than store capacity");
  std::vector<uint64_t> ck;
  std::vector<int2> cv;
  if (c->have_prev) {
    rc = download_prev(c, ck, cv);
    if (rc) return rc;
  }
  const uint64_t tag = c->kbits >= 64 ? 0 : (uint64_t)replica << c->kbits;
  const uint64_t hi = c->kbits >= 64 ? ~0ull : (((uint64_t)replica + 1) << c->kbits) - 1;
  const size_t b = (size_t)(std::lower_bound(ck.begin(), ck.end(), tag) - ck.begin());
  const size_t e = (size_t)(std::upper_bound(ck.begin(), ck.end(), hi) - ck.begin());
  std::vector<uint64_t> nk(ck.begin(), ck.begin() + b);
  std::vector<int2> nv(cv.begin(), cv.begin() + b);
  for (uint64_t i = 0; i < n; ++i) {
    nk.push_back(tag | keys[i]);
    nv.push_back(make_int2(re[i], im[i]));
  }
  nk.insert(nk.end(), ck.begin() + e, ck.end());
  nv.insert(nv.end(), cv.begin() + e, cv.end());
  const uint64_t m = nk.size();
  if (m) {
    HIPCHK(c, hipMemcpyAsync(c->pk(), nk.data(), m * 8, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->pv(), nv.data(), m * 8, hipMemcpyHostToDevice, c->stream));
  }
  HIPCHK(c, hipMemcpyAsync(&c->counters()->n_prev, &m, 8, hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  c->w_prev.assign(s_prev, s_prev + c->n_h);
  c->w_prev.insert(c->w_prev.end(), gamma_prev, gamma_prev + c->n_l);
  c->have_prev = true;
  return QMC_OK;
}

int qmc_export_prev(qmc_ctx* c, uint32_t replica, uint64_t* keys, int32_t* re, int32_t* im,
                    uint64_t cap, uint64_t* n) {
  if (!c || replica >= c->R || !n) return QMC_ERR_ARG;
  if (c->broken) return fail(c, QMC_ERR_STATE, "context unusable after a HIP error");
  if (c->integrator != 1 || !c->have_prev) return fail(c, QMC_ERR_ARG, "no N(s-1)");
  std::vector<uint64_t> ck;
  std::vector<int2> cv;
  int rc = download_prev(c, ck, cv);
  if (rc) return rc;
  const uint64_t lo = c->kbits >= 64 ? 0 : (uint64_t)replica << c->kbits;
  const uint64_t hi = c->kbits >= 64 ? ~0ull : (((uint64_t)replica + 1) << c->kbits) - 1;
  auto b = std::lower_bound(ck.begin(), ck.end(), lo);
  auto e = std::upper_bound(ck.begin(), ck.end(), hi);
  const uint64_t m = (uint64_t)(e - b);
  *n = m;
  if (m > cap) return fail(c, QMC_ERR_ARG, "export capacity too small");
  const uint64_t kmask = c->kbits >= 64 ? ~0ull : ((1ull << c->kbits) - 1);
  const size_t off = (size_t)(b - ck.begin());
  for (uint64_t i = 0; i < m; ++i) {
    keys[i] = ck[off + i] & kmask;
    re[i] = cv[off + i].x;
    im[i] = cv[off + i].y;
  }
  return QMC_OK;
}

int qmc_counters(qmc_ctx* c, qmc_stats* out) {
  if (!c || !out) return QMC_ERR_ARG;
  if (c->broken) return fail(c, QMC_ERR_STATE, "context unusable after a HIP error");
  qmc::Counters hc;
  int rc = read_counters(c, hc);
  if (rc) return rc;
  out->step = c->step;
  out->n_occ_total = hc.n_store[c->cur];
  out->walker_steps = hc.walker_steps;
  out->key_steps = hc.key_steps;
  out->child_steps = hc.child_steps;
  out->out_steps = hc.out_steps;
  out->spawn_steps = hc.child_steps - hc.death_steps;
  out->rebalances = hc.resplits + c->relaunches;
  return QMC_OK;
}

int qmc_profile(qmc_ctx* c, int32_t kernel_class) {
  if (!c || kernel_class < -1 || kernel_class >= kProfClasses) return QMC_ERR_ARG;
  int rc = settle_timings(c);  // (discarded below)
  if (rc) return rc;
  c->prof_class = kernel_class;
  for (int k = 0; k < kProfClasses; ++k) {
    c->prof_ms[k] = 0.0;
    c->prof_launches[k] = 0;
    c->prof_cover[k] = qmc_stats{};
  }
  return QMC_OK;
}

int qmc_profile_read_class(qmc_ctx* c, int32_t kernel_class, double* ms, uint64_t* launches,
                           qmc_stats* covered) {
  if (!c || kernel_class < 0 || kernel_class >= kProfClasses) return QMC_ERR_ARG;
  int rc = settle_timings(c);
  if (rc) return rc;
  if (ms) *ms = c->prof_ms[kernel_class];
  if (launches) *launches = c->prof_launches[kernel_class];
  if (covered) *covered = c->prof_cover[kernel_class];
  return QMC_OK;
}

int qmc_profile_read(qmc_ctx* c, double* ms, uint64_t* launches, qmc_stats* covered) {
  if (!c) return QMC_ERR_ARG;
  if (c->prof_class < 0) {
    if (ms) *ms = 0.0;
    if (launches) *launches = 0;
    if (covered) *covered = qmc_stats{};
    return QMC_OK;
  }
  return qmc_profile_read_class(c, c->prof_class, ms, launches, covered);
}

int qmc_coeff_table(const qmc_config* cfg, const qmc_model* model, const double* s,
                    const double* gamma, double scale, uint32_t cap_groups, uint32_t cap_terms,
                    uint32_t* n_groups, uint64_t* gxmask, uint32_t* gstart, uint32_t* n_terms,
                    uint64_t* tzmask, int64_t* tq) {
  std::string why;
  int rc = validate(cfg, model, why);
  if (rc) return rc;
  std::vector<SrcTerm> terms;
  compile_model(*model, cfg->n_qubits, terms);
  TermPlan P;
  make_plan(terms, model->n_h, P);
  HostTable T;
  if (!std::isfinite(scale)) return QMC_ERR_ARG;
  rc = build_table_plan(P, cfg->dt, s, gamma, scale, T, why);
  if (rc) return rc;
  *n_groups = (uint32_t)T.gx.size();
  *n_terms = (uint32_t)T.t.size();
  if (T.gx.size() > cap_groups || T.t.size() > cap_terms) return QMC_ERR_ARG;
  for (size_t g = 0; g < T.gx.size(); ++g) {
    gxmask[g] = T.gx[g];
    gstart[g] = T.gs[g];
  }
  gstart[T.gx.size()] = T.gs.back();
  for (size_t i = 0; i < T.t.size(); ++i) {
    tzmask[i] = T.t[i].zmask;
    tq[2 * i] = T.t[i].qre;
    tq[2 * i + 1] = T.t[i].qim;
  }
  return QMC_OK;
}

const char* qmc_last_error(const qmc_ctx* c) {
  if (!c) return "no context";
  return c->err.c_str();
}

void qmc_destroy(qmc_ctx* c) {
  if (!c) return;
  (void)hipStreamSynchronize(c->stream);
  for (hipEvent_t ev : c->prof_ev) (void)hipEventDestroy(ev);
  for (hipEvent_t ev : c->ev_free) (void)hipEventDestroy(ev);
  for (const qmc_ctx::PendingTime& t : c->ev_pending) {
    (void)hipEventDestroy(t.a);
    (void)hipEventDestroy(t.b);
  }
  if (c->pinned) (void)hipHostFree(c->pinned);
  if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
  if (c->gstream) (void)hipStreamDestroy(c->gstream);
  if (c->pinned_small) (void)hipHostFree(c->pinned_small);
  delete c;
}

}  // extern "C"
