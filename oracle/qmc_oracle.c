/*
 * qmc_oracle.c -- plain, slow CPU oracle for the real-time QMC population dynamics of
 * Shen & Lidar, arXiv:2502.18929 (main text eqs. (1)-(3) and the End Matter on spawn and
 * annihilation population dynamics).
 *
 * TEST INFRASTRUCTURE ONLY: loaded by tests/, by the package smoke check and by the CPU-baseline
 * leg of bench.py, never by the product path.  It shares no code with the HIP library.
 *
 * Where the paper is silent or its printed formula cannot be used as written, this file follows
 * these readings (each also listed in the design notes of the repository):
 *  R1  The dissipator is D[L]rho = 2 L rho L^dagger - {L^dagger L, rho} and the vectorized
 *      Liouvillian of eq. (2) is built from it with conj(L) (x) L, I (x) L^dagger L and
 *      (L^dagger L)^T (x) I; the printed forms drop a dagger / conjugate.
 *  R2  Key of |i><j| is (j << n) | i (column stacking; the printed vec(|i> (x) |j>) is garbled).
 *  R3  Spawning (End Matter, spawn step) draws a binomial count and a multinomial over the
 *      (target, Re/Im) channels of the column; here every channel amount dt * L_col * N is
 *      rounded stochastically with one systematic comb per parent, in Q32 fixed point.  The
 *      expectation is the one the paper states (E[children] = dt L N) and no p <= 1 is needed.
 *  R4  The diagonal entry of the column ("any state", including |i,j> itself) is applied as
 *      death/cloning to N(t) itself, with its own comb draw, before annihilation.
 *  R5  Coefficients are evaluated at the left end of the step (t_s = s * dt): the caller passes
 *      s_m(t_s) and gamma_k(t_s) per step.
 *  R6  No population control by default (the Liouvillian is trace preserving, so the paper uses
 *      none); an optional constant diagonal shift S per replica enters death as L_diag + S.
 *  R17 Initiator approximation (End Matter on simulation methodology, last paragraph): a parent
 *      is an initiator when its population |re| + |im| is at least a threshold (the caller's
 *      xi * N^diag, rounded up to whole walkers); every record a non-initiator spawns onto a key
 *      that is not occupied in N(s) is discarded.  "Occupied" means present in N(s), the vector
 *      being advanced, before annihilation; the rule covers the second AB2 term too (parents
 *      from N(s-1), targets checked against N(s)); death on the parent's own key in N(s) is
 *      never discarded.  Threshold 0 = off.
 *  R18 Spawn proposals (the End Matter's multinomial over the (target, Re/Im) channels of a
 *      column, with importance weights so that any proposal keeps the stated expectation):
 *      instead of the comb over every channel, a parent draws K (a power of two) channels
 *      ch = (group g >= 1, Re or Im) with probabilities P_ch / 2^32 and puts
 *      round(x_ch / (K P_ch)) walkers on each, x_ch being the channel's Q32 amount (the same
 *      integer the comb rounds).  The rounding is exact: the offset of the uniform inside its
 *      channel interval is uniform on [0, P_ch), and with K sub-draws it gives a uniform on
 *      [0, K P_ch).  The thresholds P_ch come from nonnegative integer weights W_ch: a floor
 *      F = floor(2^32 / (16 nch)) each, the rest shared in proportion to W_ch (all W = 0 counts
 *      as all W = 1), the rounding remainder to the last channel.  Weights: uniform (1 each),
 *      heat-bath (|x_ch| >> sh, sh = max(0, bitlen(|a| + |b|) + bitlen(q_off) - 24) with q_off
 *      the sum of the off-diagonal |q| of the table, so W < 2^24: the paper's |L|-proportional
 *      choice for this parent) or the scores of a small int8 MLP of the key bits (one score per group, both
 *      components).  Death keeps its comb.  Euler only, no initiator; 0 = the plain comb.
 *  R21 The learned proposal's inputs (2n key bits plus a one-hot over the model's terms, the
 *      learned-proposal configuration): weight W of both components of group g is
 *      min(2^24, max(0, score_{g-1})) of a network with inputs +1 / -1 for the 2n key bits,
 *      then 1 / 0 for every weight channel of the step (H monomials, then Lindblad operators)
 *      that is nonzero / zero -- on a gate circuit the one gate whose window holds the step over
 *      a constant background of noise channels -- two hidden layers of 128 units,
 *      h = min(127, max(0, b + w . x) >> s), and 64 group scores b3 + w3 . h2 (kind 4).
 *
 * Floating point: the only FP64 arithmetic is the coefficient quantization, done in a fixed
 * operation order (compile with -ffp-contract=off).  Everything the walkers touch is integer.
 */
#include "qmc_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------------------------ */
/* Philox4x32-10: Salmon, Moraes, Dror & Shaw, "Parallel random numbers: as easy as 1, 2, 3",  */
/* SC'11.  Ten rounds of the Philox S-box on a 4x32-bit counter, key bumped by the Weyl        */
/* constants between rounds.                                                                  */
/* ------------------------------------------------------------------------------------------ */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
  uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; ++round) {
    if (round > 0) {
      k0 += W0;
      k1 += W1;
    }
    uint64_t p0 = (uint64_t)M0 * (uint64_t)x0;
    uint64_t p1 = (uint64_t)M1 * (uint64_t)x2;
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t y0 = hi1 ^ x1 ^ k0;
    uint32_t y1 = lo1;
    uint32_t y2 = hi0 ^ x3 ^ k1;
    uint32_t y3 = lo0;
    x0 = y0; x1 = y1; x2 = y2; x3 = y3;
  }
  out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* Systematic comb rounding (reading R3).  E[out[k]] = x[k] / 2^32 exactly for U uniform. */
void orc_comb(uint32_t m, const int64_t* x, uint32_t U, int64_t* out) {
  uint64_t r = U;
  for (uint32_t k = 0; k < m; ++k) {
    uint64_t mag = x[k] < 0 ? (uint64_t)0 - (uint64_t)x[k] : (uint64_t)x[k];
    uint64_t t = r + mag;
    uint64_t cnt = t >> 32;
    r = t & 0xFFFFFFFFull;
    out[k] = x[k] < 0 ? -(int64_t)cnt : (int64_t)cnt;
  }
}

static int popc64(uint64_t v) { return __builtin_popcountll(v); }
static int parity64(uint64_t v) { return __builtin_parityll(v); }

/* ------------------------------------------------------------------------------------------ */
/* Context                                                                                     */
/* ------------------------------------------------------------------------------------------ */
typedef struct {
  uint64_t xmask, zmask; /* key-space masks of the map rho -> kappa A rho B */
  double kre, kim;       /* kappa0: coefficient before the time-dependent weight */
  uint32_t kind, index;  /* 0: weight s_m(t), m = index; 1: weight gamma_k(t), k = index */
} term_t;

typedef struct {
  uint64_t* key;
  int32_t* re;
  int32_t* im;
  uint64_t n;
} store_t;

struct orc_ctx {
  uint32_t n, R;
  uint64_t seed;
  double dt;
  uint32_t n_h, n_l;
  uint32_t n_terms;
  term_t* terms;
  store_t* st; /* [R] */
  double* shift; /* [R] */
  uint32_t step;
  uint64_t walker_steps; /* sum over steps and replicas of the parents' N^tot */
  uint64_t key_steps;    /* sum over steps and replicas of the parents' occupied keys */
  uint64_t child_steps;  /* sum over steps and replicas of emitted child records */
  uint64_t max_children; /* largest number of child records of one step (all replicas) */
  uint64_t* nchild;      /* [R] child records of the last step, per replica */
  /* AB2 (End Matter on simulation methodology): N(s-1) per replica and the weights of step
   * s-1, both needed by the second term of the two-step formula. */
  int ab2;
  store_t* prev;         /* [R] */
  double* w_prev;        /* [n_h + n_l] */
  int have_prev;         /* N(s-1) and w_prev are valid (false at step 0: Euler first step) */
  /* Initiator approximation (End Matter on simulation methodology, last paragraph): a parent
   * whose population |re| + |im| is below init_min is not an initiator, and the records it
   * spawns onto keys absent from N(s) are discarded.  0 = off (every parent spawns). */
  uint64_t init_min;
  /* Philox stream id of replica r is replica_base + r: a context that holds one circuit of a
   * batch draws what the batch draws for that circuit's replicas. */
  uint32_t replica_base;
  /* Spawn proposal (reading R18): kind 0 = the comb, 1 uniform, 2 heat-bath, 3 MLP scores;
   * prop_k samples per parent; the MLP's int8 weights, int32 biases and hidden shift. */
  uint32_t prop_kind, prop_k;
  /* Variable shift (population control of the FCIQMC background paragraph, the update rule of
   * Booth, Thom & Alavi 2009): mode 1 turns it on.  At every step s that is a multiple of
   * shift_period = A, a replica whose N^tot has reached shift_target starts to follow
   * S <- S - zeta / (A dt) * ln(N^tot(s) / N^tot(s - A)); shift_on marks the replicas that have
   * started, shift_ref holds their N^tot at the last update. */
  int shift_mode;
  double shift_zeta;
  uint32_t shift_period;
  uint64_t shift_target;
  uint8_t* shift_on;     /* [R] */
  uint64_t* shift_ref;   /* [R] */
  int8_t mlp_w1[ORC_MLP_HIDDEN][ORC_MLP_IN];
  int32_t mlp_b1[ORC_MLP_HIDDEN];
  int8_t mlp_w2[ORC_MLP_OUT][ORC_MLP_HIDDEN];
  int32_t mlp_b2[ORC_MLP_OUT];
  uint32_t mlp_s1;
  /* the deeper network (kind 4, reading R21) */
  int8_t deep_w1[ORC_DEEP_HIDDEN][ORC_DEEP_IN];
  int32_t deep_b1[ORC_DEEP_HIDDEN];
  int8_t deep_w2[ORC_DEEP_HIDDEN][ORC_DEEP_HIDDEN];
  int32_t deep_b2[ORC_DEEP_HIDDEN];
  int8_t deep_w3[ORC_DEEP_OUT][ORC_DEEP_HIDDEN];
  int32_t deep_b3[ORC_DEEP_OUT];
  uint32_t deep_s1, deep_s2;
};

/* Liouvillian source terms from eqs. (1)-(2) with reading R1.  Each term acts on a basis element
 * as rho -> kappa * A rho B with A = X^xa Z^za (left) and B = X^xb Z^zb (right).  On the key
 * (j << n) | i this gives the target key ^ ((xb << n) | xa) with sign
 * (-1)^{popc(za & i) + popc(zb & j)} * (-1)^{popc(zb & xb)}; the last, key-independent factor is
 * folded into kappa0 below. */
static int compile_terms(orc_ctx* c, const orc_monomial* h, const uint32_t* l_off,
                         const orc_monomial* l) {
  const uint32_t n = c->n;
  uint64_t cnt = 2ull * c->n_h;
  for (uint32_t k = 0; k < c->n_l; ++k) {
    uint64_t na = l_off[k + 1] - l_off[k];
    cnt += 3ull * na * na;
  }
  c->terms = (term_t*)calloc(cnt ? cnt : 1, sizeof(term_t));
  if (!c->terms) return ORC_ERR_NOMEM;
  uint32_t t = 0;
  /* -i[H, rho] = -i H rho + i rho H, eq. (1). */
  for (uint32_t m = 0; m < c->n_h; ++m) {
    uint64_t x = h[m].x, z = h[m].z;
    double hre = h[m].re, him = h[m].im;
    /* -i * H_m rho: A = P_m, B = I, kappa = -i h. */
    c->terms[t++] = (term_t){x, z, him, -hre, 0, m};
    /* +i * rho H_m: A = I, B = P_m, kappa = +i h, times the folded (-1)^{popc(x & z)}. */
    double f = (popc64(x & z) & 1) ? -1.0 : 1.0;
    c->terms[t++] = (term_t){x << n, z << n, f * -him, f * hre, 0, m};
  }
  /* (1/2) gamma D[L] rho = gamma L rho L^dagger - (gamma/2) {L^dagger L, rho}, L = sum_a c_a P_a. */
  for (uint32_t k = 0; k < c->n_l; ++k) {
    for (uint32_t a = l_off[k]; a < l_off[k + 1]; ++a) {
      for (uint32_t b = l_off[k]; b < l_off[k + 1]; ++b) {
        uint64_t xa = l[a].x, za = l[a].z, xb = l[b].x, zb = l[b].z;
        double ar = l[a].re, ai = l[a].im, br = l[b].re, bi = l[b].im;
        /* Jump term c_a conj(c_b) P_a rho P_b^dagger.  P_b^dagger = (-1)^{popc(xb&zb)} P_b, and
         * that sign cancels the folded constant of the right factor, so kappa0 = c_a conj(c_b). */
        c->terms[t++] = (term_t){(xb << n) | xa, (zb << n) | za, ar * br + ai * bi,
                                 ai * br - ar * bi, 1, k};
        /* conj(c_a) c_b P_a^dagger P_b = mu * X^{xa^xb} Z^{za^zb}, using
         * P_a^dagger = (-1)^{popc(xa&za)} P_a and Z^za X^xb = (-1)^{popc(za&xb)} X^xb Z^za. */
        double sg = ((popc64(xa & za) + popc64(za & xb)) & 1) ? -1.0 : 1.0;
        double mre = sg * (ar * br + ai * bi);
        double mim = sg * (ar * bi - ai * br);
        uint64_t x = xa ^ xb, z = za ^ zb;
        /* -(1/2) mu M rho */
        c->terms[t++] = (term_t){x, z, -0.5 * mre, -0.5 * mim, 1, k};
        /* -(1/2) mu rho M, with the folded (-1)^{popc(x & z)}. */
        double f = (popc64(x & z) & 1) ? -1.0 : 1.0;
        c->terms[t++] = (term_t){x << n, z << n, f * (-0.5 * mre), f * (-0.5 * mim), 1, k};
      }
    }
  }
  c->n_terms = t;
  return ORC_OK;
}

int orc_create(uint32_t n_qubits, uint32_t n_replicas, uint64_t seed, double dt, uint32_t n_h,
               const orc_monomial* h, uint32_t n_l, const uint32_t* l_off, const orc_monomial* l,
               const uint64_t* keys, const int32_t* re, const int32_t* im, uint64_t n0,
               orc_ctx** out) {
  if (!out || n_qubits < 1 || n_qubits > 32 || n_replicas < 1 || n_replicas >= (1u << 24))
    return ORC_ERR_ARG;
  if (!(dt > 0.0) || !isfinite(dt)) return ORC_ERR_ARG;
  uint64_t kmask = n_qubits == 32 ? ~0ull : ((1ull << (2 * n_qubits)) - 1);
  uint64_t qmask = n_qubits == 32 ? 0xFFFFFFFFull : ((1ull << n_qubits) - 1);
  for (uint32_t m = 0; m < n_h; ++m)
    if ((h[m].x & ~qmask) || (h[m].z & ~qmask)) return ORC_ERR_ARG;
  for (uint32_t k = 0; k < n_l; ++k)
    if (l_off[k + 1] < l_off[k]) return ORC_ERR_ARG;
  for (uint32_t a = 0; n_l && a < l_off[n_l]; ++a)
    if ((l[a].x & ~qmask) || (l[a].z & ~qmask)) return ORC_ERR_ARG;
  for (uint64_t i = 0; i < n0; ++i) {
    if (keys[i] & ~kmask) return ORC_ERR_ARG;
    if (i && keys[i] <= keys[i - 1]) return ORC_ERR_ARG;
    if (re[i] == 0 && im[i] == 0) return ORC_ERR_ARG;
  }
  orc_ctx* c = (orc_ctx*)calloc(1, sizeof(orc_ctx));
  if (!c) return ORC_ERR_NOMEM;
  c->n = n_qubits;
  c->R = n_replicas;
  c->seed = seed;
  c->dt = dt;
  c->n_h = n_h;
  c->n_l = n_l;
  int rc = compile_terms(c, h, l_off, l);
  if (rc) {
    orc_destroy(c);
    return rc;
  }
  c->st = (store_t*)calloc(n_replicas, sizeof(store_t));
  c->shift = (double*)calloc(n_replicas, sizeof(double));
  c->shift_on = (uint8_t*)calloc(n_replicas, 1);
  c->shift_ref = (uint64_t*)calloc(n_replicas, sizeof(uint64_t));
  c->nchild = (uint64_t*)calloc(n_replicas, sizeof(uint64_t));
  c->prev = (store_t*)calloc(n_replicas, sizeof(store_t));
  c->w_prev = (double*)calloc((size_t)n_h + n_l + 1, sizeof(double));
  if (!c->st || !c->shift || !c->shift_on || !c->shift_ref || !c->nchild || !c->prev ||
      !c->w_prev) {
    orc_destroy(c);
    return ORC_ERR_NOMEM;
  }
  for (uint32_t r = 0; r < n_replicas; ++r) {
    rc = orc_import(c, r, keys, re, im, n0, 0);
    if (rc) {
      orc_destroy(c);
      return rc;
    }
  }
  *out = c;
  return ORC_OK;
}

static void store_free(store_t* s) {
  free(s->key);
  free(s->re);
  free(s->im);
  s->key = NULL;
  s->re = s->im = NULL;
  s->n = 0;
}

void orc_destroy(orc_ctx* c) {
  if (!c) return;
  if (c->st)
    for (uint32_t r = 0; r < c->R; ++r) store_free(&c->st[r]);
  if (c->prev)
    for (uint32_t r = 0; r < c->R; ++r) store_free(&c->prev[r]);
  free(c->st);
  free(c->prev);
  free(c->w_prev);
  free(c->shift);
  free(c->shift_on);
  free(c->shift_ref);
  free(c->nchild);
  free(c->terms);
  free(c);
}

uint32_t orc_n_terms(const orc_ctx* c) { return c->n_terms; }

int orc_get_terms(const orc_ctx* c, uint64_t* xmask, uint64_t* zmask, double* kre, double* kim,
                  uint32_t* kind, uint32_t* index) {
  for (uint32_t t = 0; t < c->n_terms; ++t) {
    xmask[t] = c->terms[t].xmask;
    zmask[t] = c->terms[t].zmask;
    kre[t] = c->terms[t].kre;
    kim[t] = c->terms[t].kim;
    kind[t] = c->terms[t].kind;
    index[t] = c->terms[t].index;
  }
  return ORC_OK;
}

/* ------------------------------------------------------------------------------------------ */
/* Per-step coefficient table: quantize every source term to Q32, merge, group, check bound.  */
/* ------------------------------------------------------------------------------------------ */
typedef struct {
  uint64_t xmask, zmask;
  int64_t qre, qim;
} qterm_t;

typedef struct {
  uint32_t n_groups;   /* including the diagonal group 0 */
  uint64_t* gx;        /* [n_groups] */
  uint32_t* gs;        /* [n_groups + 1] */
  uint32_t n_terms;
  qterm_t* t;          /* [n_terms], grouped */
  uint64_t active[2];  /* bit m: weight channel m of the step is nonzero (H monomials, then
                          Lindblad operators; channels past 127 not kept) */
} table_t;

static int cmp_qterm(const void* a, const void* b) {
  const qterm_t* x = (const qterm_t*)a;
  const qterm_t* y = (const qterm_t*)b;
  if (x->xmask != y->xmask) return x->xmask < y->xmask ? -1 : 1;
  if (x->zmask != y->zmask) return x->zmask < y->zmask ? -1 : 1;
  return 0;
}

static void table_free(table_t* T) {
  free(T->gx);
  free(T->gs);
  free(T->t);
  memset(T, 0, sizeof(*T));
}

/* Q32 value of scale * dt * w * kappa0 for one component: the product w * kappa0 first, then dt,
 * then the integrator's factor (1 for Euler; 3/2 and -1/2 for the two AB2 terms), then an exact
 * scaling by 2^32 and round-half-even to an integer. */
static int q32(double dt, double w, double k, double scale, int64_t* out) {
  double v = ldexp(scale * (dt * (w * k)), 32);
  if (!isfinite(v) || fabs(v) >= 4611686018427387904.0 /* 2^62 */) return ORC_ERR_DT;
  *out = (int64_t)llrint(v);
  return ORC_OK;
}

static int build_table(const orc_ctx* c, const double* s, const double* gamma, double scale,
                       table_t* T) {
  memset(T, 0, sizeof(*T));
  for (uint32_t m = 0; m < c->n_h + c->n_l && m < 128; ++m) {
    const double w = m < c->n_h ? s[m] : gamma[m - c->n_h];
    if (w != 0.0) T->active[m >> 6] |= 1ull << (m & 63);
  }
  qterm_t* q = (qterm_t*)malloc((c->n_terms ? c->n_terms : 1) * sizeof(qterm_t));
  if (!q) return ORC_ERR_NOMEM;
  for (uint32_t i = 0; i < c->n_terms; ++i) {
    const term_t* tm = &c->terms[i];
    double w = tm->kind == 0 ? s[tm->index] : gamma[tm->index];
    if (!isfinite(w)) {
      free(q);
      return ORC_ERR_ARG;
    }
    q[i].xmask = tm->xmask;
    q[i].zmask = tm->zmask;
    if (q32(c->dt, w, tm->kre, scale, &q[i].qre) || q32(c->dt, w, tm->kim, scale, &q[i].qim)) {
      free(q);
      return ORC_ERR_DT;
    }
  }
  /* Merge terms with equal (xmask, zmask) by exact integer addition. */
  qsort(q, c->n_terms, sizeof(qterm_t), cmp_qterm);
  uint32_t m = 0;
  for (uint32_t i = 0; i < c->n_terms;) {
    qterm_t acc = q[i];
    uint32_t j = i + 1;
    while (j < c->n_terms && q[j].xmask == acc.xmask && q[j].zmask == acc.zmask) {
      acc.qre += q[j].qre;
      acc.qim += q[j].qim;
      ++j;
    }
    if (acc.qre != 0 || acc.qim != 0) q[m++] = acc;
    i = j;
  }
  /* Groups by xmask; group 0 is the diagonal one and always exists. */
  T->t = q;
  T->n_terms = m;
  T->gx = (uint64_t*)malloc((m + 1) * sizeof(uint64_t));
  T->gs = (uint32_t*)malloc((m + 2) * sizeof(uint32_t));
  if (!T->gx || !T->gs) {
    table_free(T);
    return ORC_ERR_NOMEM;
  }
  uint32_t g = 0;
  T->gx[0] = 0;
  T->gs[0] = 0;
  g = 1;
  for (uint32_t i = 0; i < m; ++i) {
    if (q[i].xmask == 0) continue;
    if (i == 0 || q[i].xmask != q[i - 1].xmask) {
      T->gs[g] = i;
      T->gx[g] = q[i].xmask;
      ++g;
    }
  }
  T->n_groups = g;
  T->gs[g] = m;
  /* Bound: per group sum of |q_re| + |q_im| < 2^31, so |c_re| + |c_im| < 2^31 for any key. */
  for (uint32_t gi = 0; gi < g; ++gi) {
    uint64_t sum = 0;
    for (uint32_t i = T->gs[gi]; i < T->gs[gi + 1]; ++i)
      sum += (uint64_t)llabs(q[i].qre) + (uint64_t)llabs(q[i].qim);
    if (sum >= (1ull << 31)) {
      table_free(T);
      return ORC_ERR_DT;
    }
  }
  return ORC_OK;
}

int orc_table(const orc_ctx* c, const double* s, const double* gamma, double scale,
              uint32_t cap_groups, uint32_t cap_terms, uint32_t* n_groups, uint64_t* gxmask,
              uint32_t* gstart, uint32_t* n_terms, uint64_t* tzmask, int64_t* tq) {
  table_t T;
  int rc = build_table(c, s, gamma, scale, &T);
  if (rc) return rc;
  *n_groups = T.n_groups;
  *n_terms = T.n_terms;
  if (T.n_groups > cap_groups || T.n_terms > cap_terms) {
    table_free(&T);
    return ORC_ERR_ARG;
  }
  for (uint32_t g = 0; g < T.n_groups; ++g) {
    gxmask[g] = T.gx[g];
    gstart[g] = T.gs[g];
  }
  gstart[T.n_groups] = T.gs[T.n_groups];
  for (uint32_t i = 0; i < T.n_terms; ++i) {
    tzmask[i] = T.t[i].zmask;
    tq[2 * i] = T.t[i].qre;
    tq[2 * i + 1] = T.t[i].qim;
  }
  table_free(&T);
  return ORC_OK;
}

/* Coefficient of group g at `key`: c = sum over the group's terms of (-1)^parity(zmask & key) q. */
static void group_coeff(const table_t* T, uint32_t g, uint64_t key, int64_t* cre, int64_t* cim) {
  int64_t re = 0, im = 0;
  for (uint32_t i = T->gs[g]; i < T->gs[g + 1]; ++i) {
    int neg = parity64(T->t[i].zmask & key);
    re += neg ? -T->t[i].qre : T->t[i].qre;
    im += neg ? -T->t[i].qim : T->t[i].qim;
  }
  *cre = re;
  *cim = im;
}

typedef struct {
  uint64_t key;
  double re, im;
} fent_t;

static int cmp_fent(const void* a, const void* b) {
  uint64_t x = ((const fent_t*)a)->key, y = ((const fent_t*)b)->key;
  return x < y ? -1 : (x > y ? 1 : 0);
}

int orc_column_fp(const orc_ctx* c, const double* s, const double* gamma, uint64_t key,
                  uint32_t cap, uint32_t* n, uint64_t* tkey, double* val) {
  fent_t* e = (fent_t*)malloc((c->n_terms ? c->n_terms : 1) * sizeof(fent_t));
  if (!e) return ORC_ERR_NOMEM;
  for (uint32_t i = 0; i < c->n_terms; ++i) {
    const term_t* tm = &c->terms[i];
    double w = tm->kind == 0 ? s[tm->index] : gamma[tm->index];
    double sg = parity64(tm->zmask & key) ? -1.0 : 1.0;
    e[i].key = key ^ tm->xmask;
    e[i].re = sg * c->dt * (w * tm->kre);
    e[i].im = sg * c->dt * (w * tm->kim);
  }
  qsort(e, c->n_terms, sizeof(fent_t), cmp_fent);
  uint32_t m = 0;
  for (uint32_t i = 0; i < c->n_terms;) {
    fent_t acc = e[i];
    uint32_t j = i + 1;
    while (j < c->n_terms && e[j].key == acc.key) {
      acc.re += e[j].re;
      acc.im += e[j].im;
      ++j;
    }
    if (m < cap) {
      tkey[m] = acc.key;
      val[2 * m] = acc.re;
      val[2 * m + 1] = acc.im;
    }
    ++m;
    i = j;
  }
  free(e);
  *n = m;
  return m > cap ? ORC_ERR_ARG : ORC_OK;
}

int orc_column_q(const orc_ctx* c, const double* s, const double* gamma, double scale,
                 uint64_t key, uint32_t cap, uint32_t* n, uint64_t* tkey, int64_t* val) {
  table_t T;
  int rc = build_table(c, s, gamma, scale, &T);
  if (rc) return rc;
  uint32_t m = 0;
  for (uint32_t g = 0; g < T.n_groups; ++g) {
    int64_t cre, cim;
    group_coeff(&T, g, key, &cre, &cim);
    if (cre == 0 && cim == 0) continue;
    if (m < cap) {
      tkey[m] = key ^ T.gx[g];
      val[2 * m] = cre;
      val[2 * m + 1] = cim;
    }
    ++m;
  }
  table_free(&T);
  *n = m;
  return m > cap ? ORC_ERR_ARG : ORC_OK;
}

/* ------------------------------------------------------------------------------------------ */
/* One step of the spawn / death / annihilation dynamics for one replica: Euler, or AB2.       */
/* ------------------------------------------------------------------------------------------ */
typedef struct {
  uint64_t key;
  int64_t re, im;
} rec_t;

static int cmp_rec(const void* a, const void* b) {
  uint64_t x = ((const rec_t*)a)->key, y = ((const rec_t*)b)->key;
  return x < y ? -1 : (x > y ? 1 : 0);
}

/* The records one population vector `in` contributes through one table T (the quantized
 * dt*L(t), scaled by the integrator's factor) and Philox stream `stream`, appended to rec[*nr]:
 *  - diagonal (death / cloning, reading R4): the comb of the diagonal group (plus the Q32 shift
 *    qs) applied to the parent with the uniform w1; with `keep_parent` the parent's own record
 *    carries it, (key, a + d_re, b + d_im), otherwise it is a record (key, d_re, d_im) of its own
 *    when nonzero (the second AB2 term adds to N(s+1), it does not carry N(s-1) over);
 *  - off-diagonal (spawn, reading R3): every group in table order, Re then Im, one comb with w0,
 *    a record (key ^ xmask, n_re, n_im) when nonzero. */
static int occupied(const store_t* st, uint64_t key) {
  uint64_t lo = 0, hi = st->n;
  while (lo < hi) {
    const uint64_t mid = lo + (hi - lo) / 2;
    if (st->key[mid] < key)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo < st->n && st->key[lo] == key;
}

/* ---- spawn proposals (reading R18) ---------------------------------------------------------- */

/* Scores of the groups 1..ORC_MLP_OUT for one key: input b is +1 where bit b of the key is set,
 * -1 where it is clear (b < 2n), 0 past 2n; hidden h_j = min(127, max(0, a_j) >> s1) with
 * a_j = sum_b w1[j][b] in_b + b1[j]; score_g = sum_j w2[g][j] h_j + b2[g] (int32, exact). */
static void mlp_scores(const orc_ctx* c, uint64_t key, int32_t* score) {
  int32_t h[ORC_MLP_HIDDEN];
  for (int j = 0; j < ORC_MLP_HIDDEN; ++j) {
    int32_t a = c->mlp_b1[j];
    for (uint32_t b = 0; b < 2 * c->n && b < ORC_MLP_IN; ++b)
      a += ((key >> b) & 1u) ? c->mlp_w1[j][b] : -(int32_t)c->mlp_w1[j][b];
    int32_t v = a > 0 ? (a >> c->mlp_s1) : 0;
    h[j] = v > 127 ? 127 : v;
  }
  for (int g = 0; g < ORC_MLP_OUT; ++g) {
    int32_t o = c->mlp_b2[g];
    for (int j = 0; j < ORC_MLP_HIDDEN; ++j) o += (int32_t)c->mlp_w2[g][j] * h[j];
    score[g] = o;
  }
}

int orc_mlp_scores(const orc_ctx* c, uint64_t key, int32_t* score) {
  if (!c || !score) return ORC_ERR_ARG;
  mlp_scores(c, key, score);
  return ORC_OK;
}

/* The deeper network (reading R21): input in_b = +1 / -1 where key bit b is set / clear for
 * b < 2n, in_{2n+m} = 1 where weight channel m of the step is nonzero and 0 where it is zero, 0
 * past; h1_j = min(127, max(0, b1_j + sum_i w1[j][i] in_i) >> s1), h2_j the same from h1 with
 * w2, b2, s2; score_g = b3_g + sum_j w3[g][j] h2_j (int32, exact: |sums| < 2^31). */
static void deep_scores(const orc_ctx* c, uint64_t key, const uint64_t* active, int32_t* score) {
  int32_t in[ORC_DEEP_IN], h1[ORC_DEEP_HIDDEN], h2[ORC_DEEP_HIDDEN];
  const uint32_t nb = 2 * c->n < ORC_DEEP_IN ? 2 * c->n : ORC_DEEP_IN;
  for (uint32_t i = 0; i < ORC_DEEP_IN; ++i) {
    if (i < nb) {
      in[i] = ((key >> i) & 1u) ? 1 : -1;
    } else {
      const uint32_t m = i - nb;
      in[i] = (active[m >> 6] >> (m & 63)) & 1u ? 1 : 0;
    }
  }
  for (int j = 0; j < ORC_DEEP_HIDDEN; ++j) {
    int32_t a = c->deep_b1[j];
    for (int i = 0; i < ORC_DEEP_IN; ++i) a += (int32_t)c->deep_w1[j][i] * in[i];
    const int32_t v = a > 0 ? (a >> c->deep_s1) : 0;
    h1[j] = v > 127 ? 127 : v;
  }
  for (int j = 0; j < ORC_DEEP_HIDDEN; ++j) {
    int32_t a = c->deep_b2[j];
    for (int i = 0; i < ORC_DEEP_HIDDEN; ++i) a += (int32_t)c->deep_w2[j][i] * h1[i];
    const int32_t v = a > 0 ? (a >> c->deep_s2) : 0;
    h2[j] = v > 127 ? 127 : v;
  }
  for (int g = 0; g < ORC_DEEP_OUT; ++g) {
    int32_t o = c->deep_b3[g];
    for (int j = 0; j < ORC_DEEP_HIDDEN; ++j) o += (int32_t)c->deep_w3[g][j] * h2[j];
    score[g] = o;
  }
}

int orc_step_active(const orc_ctx* c, const double* s, const double* gamma, uint64_t* active) {
  if (!c || !active) return ORC_ERR_ARG;
  table_t T;
  const int rc = build_table(c, s, gamma, 1.0, &T);
  if (rc) return rc;
  active[0] = T.active[0];
  active[1] = T.active[1];
  table_free(&T);
  return ORC_OK;
}

int orc_deep_scores(const orc_ctx* c, uint64_t key, const uint64_t* active, int32_t* score) {
  if (!c || !active || !score) return ORC_ERR_ARG;
  deep_scores(c, key, active, score);
  return ORC_OK;
}

/* Thresholds P[0..nch) (sum exactly 2^32, each >= 1) from weights W (each < 2^32). */
int orc_proposal_thresholds(uint32_t nch, const uint64_t* W, uint64_t* P) {
  if (nch == 0 || nch > 2 * 255 || !W || !P) return ORC_ERR_ARG;
  const uint64_t T = 1ull << 32;
  const uint64_t F = T / (16ull * nch), M = T - (uint64_t)nch * F;
  uint64_t S = 0;
  for (uint32_t i = 0; i < nch; ++i) {
    if (W[i] >= T) return ORC_ERR_ARG;
    S += W[i];
  }
  uint64_t used = 0;
  for (uint32_t i = 0; i + 1 < nch; ++i) {
    const uint64_t w = S ? W[i] : 1, tot = S ? S : nch;
    P[i] = F + (w * M) / tot;
    used += P[i];
  }
  P[nch - 1] = T - used;
  return ORC_OK;
}

/* One proposal draw: the channel whose interval [C_ch, C_ch + P_ch) holds u, o = u - C_ch, and
 * n = floor(|x| / (K P)) + [j P + o < |x| mod (K P)] with the sign of x_ch; j < K. */
int orc_proposal_draw(uint32_t nch, const int64_t* x, const uint64_t* P, uint32_t K, uint32_t u,
                      uint32_t j, uint32_t* ch_out, int64_t* n_out) {
  if (nch == 0 || !x || !P || K == 0 || (K & (K - 1)) || j >= K) return ORC_ERR_ARG;
  uint64_t C = 0;
  uint32_t ch = 0;
  while (ch + 1 < nch && (uint64_t)u >= C + P[ch]) C += P[ch++];
  const uint64_t o = (uint64_t)u - C, D = (uint64_t)K * P[ch], U = (uint64_t)j * P[ch] + o;
  const uint64_t a = x[ch] < 0 ? (uint64_t)(-x[ch]) : (uint64_t)x[ch];
  const uint64_t m = a / D + (U < a % D ? 1u : 0u);
  *ch_out = ch;
  *n_out = x[ch] < 0 ? -(int64_t)m : (int64_t)m;
  return ORC_OK;
}

static uint32_t bitlen64(uint64_t v) { return v ? 64u - (uint32_t)__builtin_clzll(v) : 0u; }

/* The proposal records of one parent (key, a + ib): xs[2(g-1) + comp] are its channel amounts. */
static int proposal_records(const orc_ctx* c, uint32_t r, const table_t* T, uint64_t key,
                            uint64_t sab, const int64_t* xs, uint64_t* W, uint64_t* P,
                            rec_t* rec, uint64_t* nr) {
  const uint32_t G = T->n_groups, nch = 2 * (G - 1);
  if (c->prop_kind == 1) {
    for (uint32_t i = 0; i < nch; ++i) W[i] = 1;
  } else if (c->prop_kind == 2) {
    /* |x_ch| <= sab * q_off < 2^(bitlen(sab) + bitlen(q_off)): shifted below 2^24 */
    uint64_t q_off = 0;
    for (uint32_t i = T->gs[1]; i < T->gs[G]; ++i)
      q_off += (uint64_t)llabs(T->t[i].qre) + (uint64_t)llabs(T->t[i].qim);
    const uint32_t bl = bitlen64(sab) + bitlen64(q_off);
    const uint32_t sh = bl > 24 ? bl - 24 : 0;
    for (uint32_t i = 0; i < nch; ++i)
      W[i] = (xs[i] < 0 ? (uint64_t)(-xs[i]) : (uint64_t)xs[i]) >> sh;
  } else {
    /* kinds 3 and 4: both components of group g weigh min(2^24, max(0, score_{g-1})) */
    int32_t score[ORC_MLP_OUT > ORC_DEEP_OUT ? ORC_MLP_OUT : ORC_DEEP_OUT];
    if (c->prop_kind == 3)
      mlp_scores(c, key, score);
    else
      deep_scores(c, key, T->active, score);
    const uint32_t nout = c->prop_kind == 3 ? ORC_MLP_OUT : ORC_DEEP_OUT;
    for (uint32_t g = 1; g < G; ++g) {
      const int32_t v = g - 1 < nout ? score[g - 1] : 0;
      const uint64_t w = v <= 0 ? 0 : (v > (1 << 24) ? (1u << 24) : (uint64_t)v);
      W[2 * (g - 1)] = W[2 * (g - 1) + 1] = w;
    }
  }
  int rc = orc_proposal_thresholds(nch, W, P);
  if (rc) return rc;
  const uint32_t pkey[2] = {(uint32_t)c->seed, (uint32_t)(c->seed >> 32)};
  for (uint32_t k = 0; k < c->prop_k; ++k) {
    /* sample k: Philox stream 0x40 + k of this walker and step */
    const uint32_t ctr[4] = {(uint32_t)key, (uint32_t)(key >> 32), c->step,
                             ((c->replica_base + r) << 8) | (0x40u + k)};
    uint32_t q[4];
    orc_philox4x32_10(ctr, pkey, q);
    uint32_t ch;
    int64_t m;
    orc_proposal_draw(nch, xs, P, c->prop_k, q[0], q[1] & (c->prop_k - 1), &ch, &m);
    if (m > INT32_MAX || m < -(int64_t)INT32_MAX) return ORC_ERR_COUNT_OVERFLOW;
    if (m != 0) {
      const uint32_t g = 1 + ch / 2;
      rec[(*nr)++] = (rec_t){key ^ T->gx[g], (ch & 1) ? 0 : m, (ch & 1) ? m : 0};
    }
  }
  return ORC_OK;
}

/* `occ` is N(s), the vector being advanced: with the initiator approximation a record from a
 * non-initiator parent survives only on a key occupied there. */
static int add_records(const orc_ctx* c, uint32_t r, const store_t* in, const table_t* T,
                       int64_t qs_re, uint32_t stream, int keep_parent, const store_t* occ,
                       rec_t* rec, uint64_t* nr) {
  const uint32_t G = T->n_groups;
  int64_t* xs = (int64_t*)malloc(2 * (size_t)(G ? G : 1) * sizeof(int64_t));
  int64_t* ns = (int64_t*)malloc(2 * (size_t)(G ? G : 1) * sizeof(int64_t));
  uint64_t* pw = (uint64_t*)malloc(4 * (size_t)(G ? G : 1) * sizeof(uint64_t));
  if (!xs || !ns || !pw) {
    free(xs);
    free(ns);
    free(pw);
    return ORC_ERR_NOMEM;
  }
  int rc = ORC_OK;
  const uint32_t pkey[2] = {(uint32_t)c->seed, (uint32_t)(c->seed >> 32)};
  for (uint64_t p = 0; p < in->n; ++p) {
    const uint64_t key = in->key[p];
    const int64_t a = in->re[p], b = in->im[p];
    /* Philox counter: the walker's key, the step, and (replica << 8) | stream. */
    const uint32_t ctr[4] = {(uint32_t)key, (uint32_t)(key >> 32), c->step,
                             ((c->replica_base + r) << 8) | stream};
    uint32_t w[4];
    orc_philox4x32_10(ctr, pkey, w);
    const int initiator =
        c->init_min == 0 || (uint64_t)(llabs(a) + llabs(b)) >= c->init_min;

    int64_t dre, dim;
    group_coeff(T, 0, key, &dre, &dim);
    dre += qs_re;
    int64_t x2[2] = {a * dre - b * dim, a * dim + b * dre};
    int64_t n2[2];
    orc_comb(2, x2, w[1], n2);
    if (keep_parent)
      rec[(*nr)++] = (rec_t){key, a + n2[0], b + n2[1]};
    else if ((n2[0] != 0 || n2[1] != 0) && (initiator || occupied(occ, key)))
      rec[(*nr)++] = (rec_t){key, n2[0], n2[1]};

    for (uint32_t g = 1; g < G; ++g) {
      int64_t cre, cim;
      group_coeff(T, g, key, &cre, &cim);
      xs[2 * (g - 1)] = a * cre - b * cim;
      xs[2 * (g - 1) + 1] = a * cim + b * cre;
    }
    if (c->prop_kind != 0) {
      if (G > 1)
        rc = proposal_records(c, r, T, key, (uint64_t)(llabs(a) + llabs(b)), xs, pw, pw + 2 * G,
                              rec, nr);
      if (rc) break;
      continue;
    }
    if (G > 1) orc_comb(2 * (G - 1), xs, w[0], ns);
    for (uint32_t g = 1; g < G; ++g) {
      int64_t cr = ns[2 * (g - 1)], ci = ns[2 * (g - 1) + 1];
      const uint64_t target = key ^ T->gx[g];
      if ((cr != 0 || ci != 0) && (initiator || occupied(occ, target)))
        rec[(*nr)++] = (rec_t){target, cr, ci};
    }
  }
  free(xs);
  free(ns);
  free(pw);
  return rc;
}

/* N(s+1) of replica r.  Euler (End Matter on simulation methodology):
 *   N(s+1) = N(s) + round(dt L(t_s) N(s)),
 * with table A = dt L(t_s).  AB2 (same paragraph), for s >= 1:
 *   N(s+1) = N(s) + round(3/2 dt L(t_s) N(s)) + round(-1/2 dt L(t_{s-1}) N(s-1)),
 * with table A = 3/2 dt L(t_s) on stream 0 and table B = -1/2 dt L(t_{s-1}) on N(s-1), stream 1.
 * Annihilation (End Matter): all records merged, summed by location, opposite signs cancel,
 * empty locations disappear. */
static int step_replica(const orc_ctx* c, uint32_t r, const table_t* A, int64_t qa,
                        const table_t* B, int64_t qb, store_t* out, uint64_t* nchild) {
  const store_t* in = &c->st[r];
  const store_t* pv = B ? &c->prev[r] : NULL;
  uint64_t per = A->n_groups > c->prop_k + 1 ? A->n_groups : c->prop_k + 1;
  uint64_t cap = in->n * per + 1;
  if (B) cap += pv->n * (uint64_t)B->n_groups;
  rec_t* rec = (rec_t*)malloc(cap * sizeof(rec_t));
  if (!rec) return ORC_ERR_NOMEM;
  uint64_t nr = 0;
  int rc = add_records(c, r, in, A, qa, 0u, 1, in, rec, &nr);
  if (!rc && B) rc = add_records(c, r, pv, B, qb, 1u, 0, in, rec, &nr);
  if (rc) {
    free(rec);
    return rc;
  }
  *nchild = nr - in->n;

  qsort(rec, nr, sizeof(rec_t), cmp_rec);
  uint64_t m = 0;
  for (uint64_t i = 0; i < nr;) {
    rec_t acc = rec[i];
    uint64_t j = i + 1;
    while (j < nr && rec[j].key == acc.key) {
      acc.re += rec[j].re;
      acc.im += rec[j].im;
      ++j;
    }
    if (acc.re < INT32_MIN || acc.re > INT32_MAX || acc.im < INT32_MIN || acc.im > INT32_MAX) {
      free(rec);
      return ORC_ERR_COUNT_OVERFLOW;
    }
    if (acc.re != 0 || acc.im != 0) rec[m++] = acc;
    i = j;
  }
  out->n = m;
  out->key = (uint64_t*)malloc((m ? m : 1) * sizeof(uint64_t));
  out->re = (int32_t*)malloc((m ? m : 1) * sizeof(int32_t));
  out->im = (int32_t*)malloc((m ? m : 1) * sizeof(int32_t));
  if (!out->key || !out->re || !out->im) {
    store_free(out);
    free(rec);
    return ORC_ERR_NOMEM;
  }
  for (uint64_t i = 0; i < m; ++i) {
    out->key[i] = rec[i].key;
    out->re[i] = (int32_t)rec[i].re;
    out->im[i] = (int32_t)rec[i].im;
  }
  free(rec);
  return ORC_OK;
}

static uint64_t diag_sum(const table_t* T) {
  uint64_t s = 0;
  for (uint32_t i = T->gs[0]; i < T->gs[1]; ++i)
    s += (uint64_t)llabs(T->t[i].qre) + (uint64_t)llabs(T->t[i].qim);
  return s;
}

/* The shifts of all replicas in Q32 for one table (factor `scale`), with the diagonal-group bound
 * including the shift. */
static int shifts_q32(const orc_ctx* c, const table_t* T, double scale, int64_t* qs) {
  const uint64_t dsum = diag_sum(T);
  for (uint32_t r = 0; r < c->R; ++r)
    if (q32(c->dt, 1.0, c->shift[r], scale, &qs[r]) ||
        dsum + (uint64_t)llabs(qs[r]) >= (1ull << 31))
      return ORC_ERR_DT;
  return ORC_OK;
}

static int one_step(orc_ctx* c, const double* s, const double* gamma, int threads) {
  const int two = c->ab2 && c->have_prev;
  table_t A, B;
  int rc = build_table(c, s, gamma, two ? 1.5 : 1.0, &A);
  if (rc) return rc;
  if (two) {
    rc = build_table(c, c->w_prev, c->w_prev + c->n_h, -0.5, &B);
    if (rc) {
      table_free(&A);
      return rc;
    }
  }
  store_t* nxt = (store_t*)calloc(c->R, sizeof(store_t));
  int* rcs = (int*)calloc(c->R, sizeof(int));
  int64_t* qa = (int64_t*)calloc(c->R, sizeof(int64_t));
  int64_t* qb = (int64_t*)calloc(c->R, sizeof(int64_t));
  if (!nxt || !rcs || !qa || !qb) rc = ORC_ERR_NOMEM;
  if (!rc) rc = shifts_q32(c, &A, two ? 1.5 : 1.0, qa);
  if (!rc && two) rc = shifts_q32(c, &B, -0.5, qb);
  if (rc == ORC_OK) {
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 1) num_threads(threads > 0 ? threads : 1)
#endif
    for (uint32_t r = 0; r < c->R; ++r)
      rcs[r] = step_replica(c, r, &A, qa[r], two ? &B : NULL, qb[r], &nxt[r], &c->nchild[r]);
    for (uint32_t r = 0; r < c->R; ++r)
      if (rcs[r] && !rc) rc = rcs[r];
  }
  (void)threads;
  if (rc == ORC_OK) {
    uint64_t tot_children = 0;
    for (uint32_t r = 0; r < c->R; ++r) tot_children += c->nchild[r];
    c->child_steps += tot_children;
    if (tot_children > c->max_children) c->max_children = tot_children;
    for (uint32_t r = 0; r < c->R; ++r) {
      for (uint64_t p = 0; p < c->st[r].n; ++p)
        c->walker_steps += (uint64_t)llabs((int64_t)c->st[r].re[p]) +
                           (uint64_t)llabs((int64_t)c->st[r].im[p]);
      c->key_steps += c->st[r].n;
      if (c->ab2) {
        store_free(&c->prev[r]);
        c->prev[r] = c->st[r];
      } else {
        store_free(&c->st[r]);
      }
      c->st[r] = nxt[r];
    }
    if (c->ab2) {
      memcpy(c->w_prev, s, c->n_h * sizeof(double));
      memcpy(c->w_prev + c->n_h, gamma, c->n_l * sizeof(double));
      c->have_prev = 1;
    }
    c->step += 1;
  } else if (nxt) {
    for (uint32_t r = 0; r < c->R; ++r) store_free(&nxt[r]);
  }
  free(qa);
  free(qb);
  free(nxt);
  free(rcs);
  table_free(&A);
  if (two) table_free(&B);
  return rc;
}

/* N^tot = sum |re| + |im| of one replica (eq. (3) paragraph). */
static uint64_t ntot_of(const store_t* st) {
  uint64_t t = 0;
  for (uint64_t p = 0; p < st->n; ++p)
    t += (uint64_t)llabs((int64_t)st->re[p]) + (uint64_t)llabs((int64_t)st->im[p]);
  return t;
}

/* The variable-shift update after a step (see shift_mode): at steps that are multiples of the
 * period, a replica that has reached the target starts (its N^tot becomes the reference), and
 * a started one takes S <- S - zeta / (A dt) * ln(N^tot / reference) and a new reference.  An
 * empty replica, or one whose reference is zero, keeps its shift. */
static void shift_update(orc_ctx* c) {
  if (c->shift_mode != 1 || c->step % c->shift_period != 0) return;
  for (uint32_t r = 0; r < c->R; ++r) {
    const uint64_t nt = ntot_of(&c->st[r]);
    if (!c->shift_on[r]) {
      if (nt >= c->shift_target) {
        c->shift_on[r] = 1;
        c->shift_ref[r] = nt;
      }
      continue;
    }
    if (nt > 0 && c->shift_ref[r] > 0)
      c->shift[r] = c->shift[r] - (c->shift_zeta / ((double)c->shift_period * c->dt)) *
                                      log((double)nt / (double)c->shift_ref[r]);
    c->shift_ref[r] = nt;
  }
}

int orc_set_shift_control(orc_ctx* c, int mode, double zeta, uint32_t period, uint64_t target) {
  if (mode != 0 && mode != 1) return ORC_ERR_ARG;
  if (mode == 1 && (period == 0 || !isfinite(zeta) || zeta < 0.0 || c->ab2)) return ORC_ERR_ARG;
  c->shift_mode = mode;
  c->shift_zeta = zeta;
  c->shift_period = period ? period : 1;
  c->shift_target = target;
  memset(c->shift_on, 0, c->R);
  memset(c->shift_ref, 0, c->R * sizeof(uint64_t));
  return ORC_OK;
}

int orc_step(orc_ctx* c, uint32_t nsteps, const double* s, const double* gamma) {
  for (uint32_t k = 0; k < nsteps; ++k) {
    int rc = one_step(c, s + (size_t)k * c->n_h, gamma + (size_t)k * c->n_l, 1);
    if (rc) return rc;
    shift_update(c);
  }
  return ORC_OK;
}

int orc_step_threads(orc_ctx* c, uint32_t nsteps, const double* s, const double* gamma,
                     int threads, int* threads_used) {
  int used = 1;
#ifdef _OPENMP
  if (threads <= 0) threads = omp_get_max_threads();
  used = threads < (int)c->R ? threads : (int)c->R;
#else
  threads = 1;
#endif
  if (threads_used) *threads_used = used;
  for (uint32_t k = 0; k < nsteps; ++k) {
    int rc = one_step(c, s + (size_t)k * c->n_h, gamma + (size_t)k * c->n_l, used);
    if (rc) return rc;
    shift_update(c);
  }
  return ORC_OK;
}

/* AB2 mode (End Matter on simulation methodology).  Switching it on or off clears N(s-1): the
 * next step is an Euler step unless orc_set_prev supplies N(s-1) and the weights of step s-1. */
int orc_set_integrator(orc_ctx* c, int ab2) {
  if (ab2 != 0 && ab2 != 1) return ORC_ERR_ARG;
  if (ab2 && c->shift_mode) return ORC_ERR_ARG;  /* the variable shift runs with Euler */
  if (ab2 && c->prop_kind) return ORC_ERR_ARG;
  c->ab2 = ab2;
  c->have_prev = 0;
  for (uint32_t r = 0; r < c->R; ++r) store_free(&c->prev[r]);
  return ORC_OK;
}

static int store_set(store_t* st, uint32_t n_qubits, const uint64_t* keys, const int32_t* re,
                     const int32_t* im, uint64_t n);

/* N(s-1) of one replica and the weights of step s-1 (s_prev[n_h], gamma_prev[n_l], shared by all
 * replicas) for an AB2 context resumed at step s >= 1; a replica whose N(s-1) is not set has an
 * empty one.  orc_import leaves N(s-1) alone. */
int orc_set_prev(orc_ctx* c, uint32_t replica, const uint64_t* keys, const int32_t* re,
                 const int32_t* im, uint64_t n, const double* s_prev, const double* gamma_prev) {
  if (!c->ab2 || replica >= c->R) return ORC_ERR_ARG;
  int rc = store_set(&c->prev[replica], c->n, keys, re, im, n);
  if (rc) return rc;
  memcpy(c->w_prev, s_prev, c->n_h * sizeof(double));
  memcpy(c->w_prev + c->n_h, gamma_prev, c->n_l * sizeof(double));
  c->have_prev = 1;
  return ORC_OK;
}

int orc_export_prev(const orc_ctx* c, uint32_t replica, uint64_t* keys, int32_t* re, int32_t* im,
                    uint64_t cap, uint64_t* n) {
  if (!c->ab2 || !c->have_prev || replica >= c->R) return ORC_ERR_ARG;
  const store_t* st = &c->prev[replica];
  *n = st->n;
  if (st->n > cap) return ORC_ERR_ARG;
  if (st->n) {
    memcpy(keys, st->key, st->n * sizeof(uint64_t));
    memcpy(re, st->re, st->n * sizeof(int32_t));
    memcpy(im, st->im, st->n * sizeof(int32_t));
  }
  return ORC_OK;
}

/* Ideal instantaneous Pauli pulse: P |i><j| P^dagger = (-1)^{popc(z&i) + popc(z&j)} |i^x><j^x|.
 * With AB2 the step after a pulse is an Euler step. */
int orc_pulse(orc_ctx* c, uint64_t x, uint64_t z) {
  const uint32_t n = c->n;
  const uint64_t qmask = n == 32 ? 0xFFFFFFFFull : ((1ull << n) - 1);
  if ((x & ~qmask) || (z & ~qmask)) return ORC_ERR_ARG;
  for (uint32_t r = 0; r < c->R; ++r) {
    store_t* st = &c->st[r];
    rec_t* rec = (rec_t*)malloc((st->n ? st->n : 1) * sizeof(rec_t));
    if (!rec) return ORC_ERR_NOMEM;
    for (uint64_t p = 0; p < st->n; ++p) {
      uint64_t i = st->key[p] & qmask, j = st->key[p] >> n;
      if (n == 32) j = st->key[p] >> 32;
      int neg = (popc64(z & i) + popc64(z & j)) & 1;
      uint64_t nk = ((j ^ x) << n) | (i ^ x);
      rec[p] = (rec_t){nk, neg ? -(int64_t)st->re[p] : st->re[p],
                       neg ? -(int64_t)st->im[p] : st->im[p]};
    }
    qsort(rec, st->n, sizeof(rec_t), cmp_rec);
    for (uint64_t p = 0; p < st->n; ++p) {
      if (rec[p].re > INT32_MAX || rec[p].im > INT32_MAX) {
        free(rec);
        return ORC_ERR_COUNT_OVERFLOW;
      }
    }
    for (uint64_t p = 0; p < st->n; ++p) {
      st->key[p] = rec[p].key;
      st->re[p] = (int32_t)rec[p].re;
      st->im[p] = (int32_t)rec[p].im;
    }
    free(rec);
  }
  /* AB2 (reading: a pulse restarts the two-step formula): the next step is an Euler step. */
  c->have_prev = 0;
  return ORC_OK;
}

int orc_set_replica_base(orc_ctx* c, uint32_t base) {
  if ((uint64_t)base + c->R > (1u << 24)) return ORC_ERR_ARG;
  c->replica_base = base;
  return ORC_OK;
}

int orc_set_initiator(orc_ctx* c, uint64_t min_walkers) {
  if (min_walkers && c->prop_kind) return ORC_ERR_ARG;
  c->init_min = min_walkers;
  return ORC_OK;
}

int orc_set_proposal(orc_ctx* c, uint32_t kind, uint32_t k, const int8_t* w1, const int32_t* b1,
                     const int8_t* w2, const int32_t* b2, uint32_t s1) {
  if (kind > 3) return ORC_ERR_ARG;
  if (kind && (k == 0 || k > 64 || (k & (k - 1)) || c->ab2 || c->init_min)) return ORC_ERR_ARG;
  if (kind == 3 && (!w1 || !b1 || !w2 || !b2 || s1 > 30)) return ORC_ERR_ARG;
  c->prop_kind = kind;
  c->prop_k = kind ? k : 0;
  if (kind == 3) {
    memcpy(c->mlp_w1, w1, sizeof(c->mlp_w1));
    memcpy(c->mlp_b1, b1, sizeof(c->mlp_b1));
    memcpy(c->mlp_w2, w2, sizeof(c->mlp_w2));
    memcpy(c->mlp_b2, b2, sizeof(c->mlp_b2));
    c->mlp_s1 = s1;
  }
  return ORC_OK;
}

int orc_set_proposal_deep(orc_ctx* c, uint32_t k, const int8_t* w1, const int32_t* b1,
                          const int8_t* w2, const int32_t* b2, const int8_t* w3,
                          const int32_t* b3, uint32_t s1, uint32_t s2) {
  if (k == 0 || k > 64 || (k & (k - 1)) || c->ab2 || c->init_min) return ORC_ERR_ARG;
  if (!w1 || !b1 || !w2 || !b2 || !w3 || !b3 || s1 > 30 || s2 > 30) return ORC_ERR_ARG;
  c->prop_kind = 4;
  c->prop_k = k;
  memcpy(c->deep_w1, w1, sizeof(c->deep_w1));
  memcpy(c->deep_b1, b1, sizeof(c->deep_b1));
  memcpy(c->deep_w2, w2, sizeof(c->deep_w2));
  memcpy(c->deep_b2, b2, sizeof(c->deep_b2));
  memcpy(c->deep_w3, w3, sizeof(c->deep_w3));
  memcpy(c->deep_b3, b3, sizeof(c->deep_b3));
  c->deep_s1 = s1;
  c->deep_s2 = s2;
  return ORC_OK;
}

int orc_set_shift(orc_ctx* c, uint32_t replica, double shift) {
  if (replica >= c->R || !isfinite(shift)) return ORC_ERR_ARG;
  c->shift[replica] = shift;
  return ORC_OK;
}

uint32_t orc_get_step(const orc_ctx* c) { return c->step; }

double orc_get_shift(const orc_ctx* c, uint32_t replica) {
  return replica < c->R ? c->shift[replica] : 0.0;
}

void orc_counters(const orc_ctx* c, uint64_t* walker_steps, uint64_t* key_steps,
                  uint64_t* child_steps, uint64_t* max_children) {
  *walker_steps = c->walker_steps;
  *key_steps = c->key_steps;
  *child_steps = c->child_steps;
  *max_children = c->max_children;
}

uint64_t orc_size(const orc_ctx* c, uint32_t replica) {
  return replica < c->R ? c->st[replica].n : 0;
}

int orc_export(const orc_ctx* c, uint32_t replica, uint64_t* keys, int32_t* re, int32_t* im,
               uint64_t cap, uint64_t* n) {
  if (replica >= c->R) return ORC_ERR_ARG;
  const store_t* st = &c->st[replica];
  *n = st->n;
  if (st->n > cap) return ORC_ERR_ARG;
  memcpy(keys, st->key, st->n * sizeof(uint64_t));
  memcpy(re, st->re, st->n * sizeof(int32_t));
  memcpy(im, st->im, st->n * sizeof(int32_t));
  return ORC_OK;
}

static int store_set(store_t* st, uint32_t n_qubits, const uint64_t* keys, const int32_t* re,
                     const int32_t* im, uint64_t n) {
  const uint64_t kmask = n_qubits == 32 ? ~0ull : ((1ull << (2 * n_qubits)) - 1);
  for (uint64_t i = 0; i < n; ++i) {
    if (keys[i] & ~kmask) return ORC_ERR_ARG;
    if (i && keys[i] <= keys[i - 1]) return ORC_ERR_ARG;
    if (re[i] == 0 && im[i] == 0) return ORC_ERR_ARG;
  }
  store_free(st);
  st->key = (uint64_t*)malloc((n ? n : 1) * sizeof(uint64_t));
  st->re = (int32_t*)malloc((n ? n : 1) * sizeof(int32_t));
  st->im = (int32_t*)malloc((n ? n : 1) * sizeof(int32_t));
  if (!st->key || !st->re || !st->im) return ORC_ERR_NOMEM;
  memcpy(st->key, keys, n * sizeof(uint64_t));
  memcpy(st->re, re, n * sizeof(int32_t));
  memcpy(st->im, im, n * sizeof(int32_t));
  st->n = n;
  return ORC_OK;
}

int orc_import(orc_ctx* c, uint32_t replica, const uint64_t* keys, const int32_t* re,
               const int32_t* im, uint64_t n, uint32_t step) {
  if (replica >= c->R) return ORC_ERR_ARG;
  int rc = store_set(&c->st[replica], c->n, keys, re, im, n);
  if (rc) return rc;
  c->step = step;
  return ORC_OK;
}

/* ------------------------------------------------------------------------------------------ */
/* Estimator numerators: eq. (3) normalization, trace (replica-aggregation paragraph),        */
/* sign angle and anti-Hermiticity (End Matter), all as exact integers.                        */
/* ------------------------------------------------------------------------------------------ */
static int64_t find_key(const store_t* st, uint64_t key, int64_t* re, int64_t* im) {
  uint64_t lo = 0, hi = st->n;
  while (lo < hi) {
    uint64_t mid = lo + (hi - lo) / 2;
    if (st->key[mid] < key)
      lo = mid + 1;
    else
      hi = mid;
  }
  if (lo < st->n && st->key[lo] == key) {
    *re = st->re[lo];
    *im = st->im[lo];
    return 1;
  }
  *re = 0;
  *im = 0;
  return 0;
}

/* v^2 for |v| < 2^32, exact in uint64. */
static uint64_t sq_abs(int64_t v) {
  uint64_t m = v < 0 ? (uint64_t)(-v) : (uint64_t)v;
  return m * m;
}

static void add128(uint64_t* lo, uint64_t* hi, uint64_t v) {
  uint64_t o = *lo;
  *lo = o + v;
  if (*lo < o) *hi += 1;
}

int orc_observe(const orc_ctx* c, uint32_t replica, uint32_t n_pauli, const uint64_t* px,
                const uint64_t* pz, uint32_t n_lookup, const uint64_t* lk, uint64_t* n_occ,
                uint64_t* n_tot, int64_t* ndiag, int64_t* pauli, int64_t* lookup,
                uint64_t* eps2) {
  if (replica >= c->R) return ORC_ERR_ARG;
  const store_t* st = &c->st[replica];
  const uint32_t n = c->n;
  const uint64_t qmask = n == 32 ? 0xFFFFFFFFull : ((1ull << n) - 1);
  uint64_t tot = 0;
  int64_t dre = 0, dim = 0;
  for (uint32_t k = 0; k < n_pauli; ++k) pauli[2 * k] = pauli[2 * k + 1] = 0;
  uint64_t elo = 0, ehi = 0;
  for (uint64_t p = 0; p < st->n; ++p) {
    const uint64_t key = st->key[p];
    const uint64_t i = key & qmask, j = n == 32 ? key >> 32 : key >> n;
    const int64_t a = st->re[p], b = st->im[p];
    tot += (uint64_t)(a < 0 ? -a : a) + (uint64_t)(b < 0 ? -b : b);
    if (i == j) {
      dre += a;
      dim += b;
    }
    /* Tr(P rho) with P = X^x Z^z: sum_i (-1)^{popc(z & i)} rho_{i, i^x}. */
    for (uint32_t k = 0; k < n_pauli; ++k) {
      if ((i ^ j) != px[k]) continue;
      int neg = popc64(pz[k] & i) & 1;
      pauli[2 * k] += neg ? -a : a;
      pauli[2 * k + 1] += neg ? -b : b;
    }
    /* |N_ij - conj(N_ji)|^2, and |N_ij|^2 for the (j,i) element when that one is empty. */
    const uint64_t kt = (i << n) | j;
    int64_t c2, d2;
    int64_t found = find_key(st, kt, &c2, &d2);
    add128(&elo, &ehi, sq_abs(a - c2));
    add128(&elo, &ehi, sq_abs(b + d2));
    if (!found) {
      add128(&elo, &ehi, sq_abs(a));
      add128(&elo, &ehi, sq_abs(b));
    }
  }
  for (uint32_t k = 0; k < n_lookup; ++k) find_key(st, lk[k], &lookup[2 * k], &lookup[2 * k + 1]);
  *n_occ = st->n;
  *n_tot = tot;
  ndiag[0] = dre;
  ndiag[1] = dim;
  eps2[0] = elo;
  eps2[1] = ehi;
  return ORC_OK;
}
