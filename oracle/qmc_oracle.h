/*
 * qmc_oracle.h -- CPU oracle for one population-dynamics time step of the real-time,
 * sign-problem-suppressed QMC of Shen & Lidar, arXiv:2502.18929.
 *
 * TEST INFRASTRUCTURE ONLY.  Only tests/, the package smoke check and the CPU-baseline leg of
 * bench.py may load this library.  It shares no code with the HIP path under
 * paper_2502_18929_amd/csrc: it has its own Philox, its own Liouvillian term compiler, its own
 * fixed-point quantizer, its own step and its own estimators, all written to be read against
 * the paper by eye, with no blocking or fusion.
 *
 * Conventions (the same contract the HIP library implements independently):
 *  - Qubit q of a basis state |i> is bit q of i.  The density-matrix element |i><j| (ket i,
 *    bra j) of an n-qubit system lives at key (j << n) | i: the column-stacking vec() of the
 *    paper's QMC-algorithm paragraph, eq. (2).
 *  - A Pauli monomial (x, z, c) is the operator c * X^x Z^z with
 *    X^x Z^z |i> = (-1)^popcount(z & i) |i ^ x>.
 *  - Walker populations are Gaussian integers re + i*im (signs {+-1, +-i}, End Matter on
 *    spawn and annihilation).
 */
#ifndef QMC_ORACLE_H
#define QMC_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct { uint64_t x, z; double re, im; } orc_monomial;

typedef struct orc_ctx orc_ctx;

/* Spawn-proposal MLP sizes (reading R18): key-bit inputs, hidden units, group scores. */
#define ORC_MLP_IN 64
#define ORC_MLP_HIDDEN 32
#define ORC_MLP_OUT 64
/* The deeper proposal network (reading R21): inputs (2n key bits, then one per weight channel of
 * the model), two hidden layers, group scores. */
#define ORC_DEEP_IN 128
#define ORC_DEEP_HIDDEN 128
#define ORC_DEEP_OUT 64

enum {
  ORC_OK = 0,
  ORC_ERR_ARG = -1,
  ORC_ERR_DT = -2,             /* a column group breaks the fixed-point bound (see orc_quantize) */
  ORC_ERR_COUNT_OVERFLOW = -5, /* an annihilated population left the int32 range */
  ORC_ERR_NOMEM = -7
};

/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): one block of four 32-bit words. */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

/* Systematic ("comb") stochastic rounding of m signed Q32 values with one 32-bit uniform U:
 * out[k] = sign(x[k]) * floor((r_k + |x[k]|) / 2^32), r_0 = U, r_{k+1} = (r_k + |x[k]|) mod 2^32.
 * Requires |x[k]| < 2^63. */
void orc_comb(uint32_t m, const int64_t* x, uint32_t U, int64_t* out);

/* Create a context: n qubits, R replicas, Philox seed, time step dt, the model of eq. (1)
 * (H(t) = sum_m s_m(t) h_m, L_k = sum_{a in [l_off[k], l_off[k+1])} l[a] with rates gamma_k(t))
 * and the initial population vector N(0) (same integer records for every replica, keys sorted
 * ascending and unique, no (0,0) entries). */
int orc_create(uint32_t n_qubits, uint32_t n_replicas, uint64_t seed, double dt,
               uint32_t n_h, const orc_monomial* h,
               uint32_t n_l, const uint32_t* l_off, const orc_monomial* l,
               const uint64_t* keys, const int32_t* re, const int32_t* im, uint64_t n0,
               orc_ctx** out);
void orc_destroy(orc_ctx* c);

/* Number of compiled source terms, and the terms themselves (unquantized kappa0, before the
 * time-dependent weight; kind 0 = H monomial `index`, kind 1 = Lindblad operator `index`). */
uint32_t orc_n_terms(const orc_ctx* c);
int orc_get_terms(const orc_ctx* c, uint64_t* xmask, uint64_t* zmask, double* kre, double* kim,
                  uint32_t* kind, uint32_t* index);

/* The quantized, merged, grouped coefficient table for one step with weights s[n_h], gamma[n_l]:
 * scale * dt * L(t) with scale 1 (Euler) or 3/2, -1/2 (the two AB2 terms).
 * Groups are ordered by xmask ascending; group 0 is always the diagonal (xmask 0, possibly empty).
 * gstart has n_groups+1 entries. Returns ORC_ERR_DT if the bound fails. */
int orc_table(const orc_ctx* c, const double* s, const double* gamma, double scale,
              uint32_t cap_groups, uint32_t cap_terms,
              uint32_t* n_groups, uint64_t* gxmask, uint32_t* gstart,
              uint32_t* n_terms, uint64_t* tzmask, int64_t* tq /* [n][2] */);

/* Column `key` of dt*L(t) (unquantized, FP64), merged by target key, targets ascending. */
int orc_column_fp(const orc_ctx* c, const double* s, const double* gamma, uint64_t key,
                  uint32_t cap, uint32_t* n, uint64_t* tkey, double* val /* [n][2] */);
/* Column `key` of the quantized table with factor `scale` (Q32 integers), merged by target key,
 * targets ascending. */
int orc_column_q(const orc_ctx* c, const double* s, const double* gamma, double scale,
                 uint64_t key, uint32_t cap, uint32_t* n, uint64_t* tkey,
                 int64_t* val /* [n][2] */);

/* Advance every replica by nsteps steps; s is [nsteps][n_h], gamma [nsteps][n_l].  Euler by
 * default; in AB2 mode every step after the first uses N(s-1) and the weights of step s-1. */
int orc_step(orc_ctx* c, uint32_t nsteps, const double* s, const double* gamma);
/* 0: Euler, 1: AB2 (End Matter on simulation methodology).  Clears N(s-1). */
int orc_set_integrator(orc_ctx* c, int ab2);
/* AB2: N(s-1) of one replica and the weights of step s-1 (shared by all replicas). */
int orc_set_prev(orc_ctx* c, uint32_t replica, const uint64_t* keys, const int32_t* re,
                 const int32_t* im, uint64_t n, const double* s_prev, const double* gamma_prev);
int orc_export_prev(const orc_ctx* c, uint32_t replica, uint64_t* keys, int32_t* re, int32_t* im,
                    uint64_t cap, uint64_t* n);
/* Apply the ideal instantaneous Pauli conjugation rho -> P rho P^dagger, P = X^x Z^z (with AB2,
 * the next step is an Euler step). */
int orc_pulse(orc_ctx* c, uint64_t x, uint64_t z);
/* Constant diagonal shift S added to the death coefficient (0 = none, the paper's setting). */
int orc_set_shift(orc_ctx* c, uint32_t replica, double shift);
/* The shift of one replica now. */
double orc_get_shift(const orc_ctx* c, uint32_t replica);
/* Variable shift (population control of the FCIQMC background paragraph; update rule of Booth,
 * Thom & Alavi 2009): mode 1 = on.  After every step whose index is a multiple of `period`
 * (A), a replica whose N^tot has reached `target` starts to follow
 * S <- S - zeta / (A dt) * ln(N^tot(s) / N^tot(s - A)).  Biased (the Liouvillian needs no shift);
 * Euler only.  Switching resets which replicas have started. */
int orc_set_shift_control(orc_ctx* c, int mode, double zeta, uint32_t period, uint64_t target);
/* Initiator approximation (End Matter on simulation methodology): parents with |re| + |im| below
 * min_walkers spawn only onto keys occupied in N(s) (reading R17).  0 = off. */
int orc_set_initiator(orc_ctx* c, uint64_t min_walkers);
/* Replica r draws Philox with stream id base + r (the counter's last word is
 * ((base + r) << 8) | stream): a context holding one circuit of a batch of circuits uses the ids
 * the batch gives that circuit's replicas.  Default 0. */
int orc_set_replica_base(orc_ctx* c, uint32_t base);
/* Spawn proposal (reading R18): kind 0 = the comb (default), 1 uniform, 2 heat-bath, 3 MLP
 * scores; k samples per parent (a power of two, <= 64); the MLP (kind 3) has int8 weights
 * w1[ORC_MLP_HIDDEN][ORC_MLP_IN], int32 b1[ORC_MLP_HIDDEN], int8 w2[ORC_MLP_OUT][ORC_MLP_HIDDEN],
 * int32 b2[ORC_MLP_OUT] and hidden shift s1 (copied).  Euler without initiators only. */
int orc_set_proposal(orc_ctx* c, uint32_t kind, uint32_t k, const int8_t* w1, const int32_t* b1,
                     const int8_t* w2, const int32_t* b2, uint32_t s1);
/* The MLP scores of groups 1..ORC_MLP_OUT for one key (the context's weights). */
int orc_mlp_scores(const orc_ctx* c, uint64_t key, int32_t* score);
/* Proposal kind 4 (reading R21): the deeper network, k samples per parent; int8 weights
 * w1[ORC_DEEP_HIDDEN][ORC_DEEP_IN], w2[ORC_DEEP_HIDDEN][ORC_DEEP_HIDDEN],
 * w3[ORC_DEEP_OUT][ORC_DEEP_HIDDEN], int32 biases b1, b2 [ORC_DEEP_HIDDEN], b3 [ORC_DEEP_OUT], hidden
 * shifts s1, s2 (copied).  Euler without initiators only. */
int orc_set_proposal_deep(orc_ctx* c, uint32_t k, const int8_t* w1, const int32_t* b1,
                          const int8_t* w2, const int32_t* b2, const int8_t* w3,
                          const int32_t* b3, uint32_t s1, uint32_t s2);
/* Its scores of groups 1..ORC_DEEP_OUT for one key, with the weight-channel indicators of a step
 * given as the bits of active[0..1] (bit m of the 128-bit mask: channel m nonzero). */
int orc_deep_scores(const orc_ctx* c, uint64_t key, const uint64_t* active, int32_t* score);
/* The weight-channel indicators of the step with weights s, gamma (the network input past the key
 * bits): bit m of active[0..1] set where channel m is nonzero. */
int orc_step_active(const orc_ctx* c, const double* s, const double* gamma, uint64_t* active);
/* Proposal thresholds (sum 2^32, each >= 1) from nch weights, and one draw from them. */
int orc_proposal_thresholds(uint32_t nch, const uint64_t* W, uint64_t* P);
int orc_proposal_draw(uint32_t nch, const int64_t* x, const uint64_t* P, uint32_t K, uint32_t u,
                      uint32_t j, uint32_t* ch, int64_t* n);

uint32_t orc_get_step(const orc_ctx* c);
/* Sums over all steps so far and all replicas of the parents' N^tot, of their occupied keys and
 * of the child records emitted, and the largest child-record count of one step. */
void orc_counters(const orc_ctx* c, uint64_t* walker_steps, uint64_t* key_steps,
                  uint64_t* child_steps, uint64_t* max_children);
uint64_t orc_size(const orc_ctx* c, uint32_t replica);
int orc_export(const orc_ctx* c, uint32_t replica, uint64_t* keys, int32_t* re, int32_t* im,
               uint64_t cap, uint64_t* n);
int orc_import(orc_ctx* c, uint32_t replica, const uint64_t* keys, const int32_t* re,
               const int32_t* im, uint64_t n, uint32_t step);

/* Estimator numerators for one replica (exact integers):
 *  n_occ, n_tot = sum(|re|+|im|), ndiag = sum over i==j of N (re, im),
 *  pauli[k] = sum over keys with ket^bra == px[k] of (-1)^popcount(pz[k] & ket) * N (re, im),
 *  lookup[k] = N at key lk[k] (0 if absent),
 *  eps2 = sum over all (i,j) of |N_ij - conj(N_ji)|^2 as a 128-bit (lo, hi) pair. */
int orc_observe(const orc_ctx* c, uint32_t replica,
                uint32_t n_pauli, const uint64_t* px, const uint64_t* pz,
                uint32_t n_lookup, const uint64_t* lk,
                uint64_t* n_occ, uint64_t* n_tot, int64_t* ndiag /* [2] */,
                int64_t* pauli /* [n_pauli][2] */, int64_t* lookup /* [n_lookup][2] */,
                uint64_t* eps2 /* [2] lo, hi */);

/* Wall-clock helper for the CPU baseline: runs orc_step with OpenMP across replicas when
 * threads > 1 and reports the threads used. */
int orc_step_threads(orc_ctx* c, uint32_t nsteps, const double* s, const double* gamma,
                     int threads, int* threads_used);

#ifdef __cplusplus
}
#endif
#endif
